"""Plain FP64 CPU oracle for the Kohn-Sham hot path (arXiv:2106.03872).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the CPU-baseline leg of the benchmark may import this module; the product
path never does.  It shares no code with the HIP library: its only inputs are
arrays (potential, projector tables, coefficients) drawn by the seeded
generator.

Every step follows the paper's definitions directly, without blocking, fusion
or reordering:

* Orbitals live in Fourier space as plane-wave coefficients on the full FFT
  box (the plane-wave basis of Section "DFT and TDDFT implementation"), with
  ``psi(r) = Omega^{-1/2} sum_G chi(G) c_G exp(+i G.r)`` so that
  ``int |psi|^2 = sum |c|^2``.
* The Hamiltonian (Eq. hamiltonian, static potential) is applied in operator
  form (Section "Implementation of the KS Hamiltonian"): kinetic energy
  ``|G|^2/2`` diagonal in Fourier space, the local potential multiplicative in
  real space, the Kleinman-Bylander non-local part (Eq. vnl) as sphere
  projections in real space, with two Fourier transforms in between.  The
  operator is restricted to the plane-wave sphere ``chi = [|G|^2/2 < E_cut]``:
  ``H = chi (K + F^-1 (V + V_nl) F) chi``.
* Time propagation: one step of the 4th-order truncated Taylor series of
  ``exp(-i H dt)`` (Section "Real-time propagation"), written as explicit
  powers ``sum_k (-i dt)^k / k! H^k c``.
* Density: ``n(r) = sum_k f_k |psi_k(r)|^2`` (Eq. density with occupations).
* Band energy ``sum_k f_k <psi_k|H|psi_k>`` and orbital norms.
* Orthonormalisation by Cholesky of the overlap (the orthogonalisation step of
  Section "Ground-state solution").
* Density-dependent local potential: the periodic Hartree potential solved in
  Fourier space (Section "Poisson solver"), ``V_H(G) = 4 pi n(G) / |G|^2``
  for ``G != 0`` and zero average, added to the static local potential.
* The optical-response probe of Section "Results" (the water-molecule
  spectrum): a field kick at t = 0, i.e. ``v_pert = -k.r delta(t)`` in
  Eq. hamiltonian, which multiplies every orbital by ``exp(i k.r)``; and the
  dipole moment, the first moment of the density.
* The ground-state eigensolver of Section "Ground-state solution":
  preconditioned steepest descent (Teter preconditioner in Fourier space)
  with subspace diagonalisation and Cholesky orthogonalisation, for a static
  Hamiltonian.
* The exchange-correlation potential ``v_xc[n]`` of Eq. hamiltonian in the
  local-density approximation (Slater exchange, Perdew-Zunger 1981
  correlation of the uniform gas), as an option of the density-dependent
  potential.
* The ETRS propagator (Eq. etrs, with the predictor of Eq. etrs0) whose two
  exponentials of ``H(t)`` share the powers ``H(t)^k c`` (the shared-lambda
  evaluation of the truncated Taylor series in Section "Real-time
  propagation").

Numerics: numpy FP64 / complex128; FFTs by ``scipy.fft`` (a library routine
standing in for the DFT sums) using all host cores.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft
import scipy.linalg

def _host_threads():
    # the host share this process may use: OMP_NUM_THREADS when set, else the
    # CPUs it is pinned to
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0)) or 1


WORKERS = _host_threads()


class Grid:
    """FFT box, reciprocal vectors and the plane-wave sphere (row O1).

    Box index ``j_a`` holds the integer frequency ``m_a = j_a`` for
    ``j_a < ceil(n_a/2)`` and ``j_a - n_a`` otherwise; ``G_a = 2 pi m_a / L_a``;
    ``K = |G|^2 / 2`` (kinetic term, diagonal in Fourier space);
    ``chi = K < E_cut`` (strict), or the whole box when ``E_cut <= 0``.
    """

    def __init__(self, n, L, ecut):
        self.n = tuple(int(x) for x in n)
        self.L = tuple(float(x) for x in L)
        self.ecut = float(ecut)
        self.N = int(np.prod(self.n))
        self.omega = float(np.prod(self.L))
        self.dV = self.omega / self.N
        self.m = []
        self.G = []
        for a in range(3):
            na = self.n[a]
            j = np.arange(na)
            ma = np.where(j < (na + 1) // 2, j, j - na)
            self.m.append(ma)
            self.G.append(2.0 * np.pi * ma / self.L[a])
        g0, g1, g2 = self.G
        self.K = 0.5 * (g0[:, None, None] ** 2 + g1[None, :, None] ** 2 + g2[None, None, :] ** 2)
        if self.ecut > 0:
            self.chi = self.K < self.ecut
        else:
            self.chi = np.ones(self.n, dtype=bool)
        self.npw = int(self.chi.sum())


class Hamiltonian:
    """Static Kohn-Sham Hamiltonian: grid, local potential, KB projectors.

    ``atoms`` is a list of ``(idx, beta)`` pairs: flat C-order grid indices of
    the sphere points of atom I and the projector values ``beta[j, p]`` there;
    ``d[I, p]`` are the KB coefficients (Eq. vnl).
    """

    def __init__(self, grid, vloc, atoms=(), d=None):
        self.grid = grid
        self.vloc = np.asarray(vloc, dtype=np.float64).reshape(grid.n)
        self.atoms = [(np.asarray(i, np.int64), np.asarray(b, np.float64)) for i, b in atoms]
        self.d = np.zeros((0, 0)) if d is None else np.asarray(d, np.float64)


def synthesize(grid, c):
    """Row O2: real-space orbitals ``Omega^{-1/2} sum_G chi c_G e^{+iG.r}``.

    ``c`` has shape ``[..., n0, n1, n2]``; coefficients outside the sphere are
    ignored.
    """
    u = scipy.fft.ifftn(np.where(grid.chi, c, 0.0), axes=(-3, -2, -1), norm="forward",
                        workers=WORKERS)
    return u / math.sqrt(grid.omega)


def analyze(grid, f):
    """Row O6: ``Omega^{1/2} N^{-1} sum_r f(r) e^{-iG.r}`` on the full box."""
    return scipy.fft.fftn(f, axes=(-3, -2, -1), norm="backward", workers=WORKERS) * (
        math.sqrt(grid.omega) / grid.N)


def projections(ham, psi_r):
    """Row O4: ``P[I, p, k] = dV sum_{j in S_I} beta_Ip(r_j) psi_k(r_j)``.

    The sphere integral of Eq. vnl becomes a grid sum with weight dV.
    """
    flat = psi_r.reshape(psi_r.shape[0], -1)
    out = []
    for idx, beta in ham.atoms:
        out.append(ham.grid.dV * (beta.T @ flat[:, idx].T))   # [nproj, norb]
    return out


def nonlocal_field(ham, P, norb):
    """Row O5: ``sum_I sum_p beta_Ip(r) d_Ip P[I, p, k]`` (overlapping spheres add)."""
    out = np.zeros((norb, ham.grid.N), np.complex128)
    for I, (idx, beta) in enumerate(ham.atoms):
        contrib = beta @ (ham.d[I][:, None] * P[I])           # [npts, norb]
        np.add.at(out, (slice(None), idx), contrib.T)
    return out.reshape((norb,) + ham.grid.n)


def ham_apply(ham, c):
    """Rows O2-O7: ``H c = chi (K c + analyze(V psi + v_nl psi))``."""
    c = np.asarray(c, np.complex128)
    single = c.ndim == 3
    if single:
        c = c[None]
    g = ham.grid
    psi_r = synthesize(g, c)
    phi = ham.vloc[None] * psi_r
    if ham.atoms:
        phi = phi + nonlocal_field(ham, projections(ham, psi_r), c.shape[0])
    hc = np.where(g.chi, g.K * c + analyze(g, phi), 0.0)
    return hc[0] if single else hc


def taylor4_coefficients(dt):
    """``(-i dt)^k / k!`` for k = 0..4 (truncated Taylor series of exp(-i H dt))."""
    return [(-1j * dt) ** k / math.factorial(k) for k in range(5)]


def taylor4_step(ham, c, dt, nsteps=1):
    """Row O8: ``nsteps`` applications of ``sum_{k=0}^{4} (-i dt)^k/k! H^k``."""
    a = taylor4_coefficients(dt)
    acc = np.where(ham.grid.chi, np.asarray(c, np.complex128), 0.0)
    for _ in range(nsteps):
        w = acc
        new = acc.copy()
        for k in range(1, 5):
            w = ham_apply(ham, w)
            new = new + a[k] * w
        acc = new
    return acc


def density(ham, c, occ):
    """Row O9: ``n(r) = sum_k f_k |psi_k(r)|^2`` (Eq. density with occupations)."""
    psi_r = synthesize(ham.grid, np.asarray(c, np.complex128))
    return np.einsum("k,kxyz->xyz", np.asarray(occ, np.float64), np.abs(psi_r) ** 2)


def norms(ham, c):
    """Row O10: ``||c_k||^2`` over the plane-wave sphere."""
    cc = np.where(ham.grid.chi, c, 0.0)
    return np.sum(np.abs(cc) ** 2, axis=(-3, -2, -1))


def band_energy(ham, c, occ):
    """Row O10: ``E = sum_k f_k Re <c_k|H c_k>`` (band energy of a static potential)."""
    c = np.where(ham.grid.chi, np.asarray(c, np.complex128), 0.0)
    hc = ham_apply(ham, c)
    e = np.sum(np.conj(c) * hc, axis=(-3, -2, -1))
    return float(np.sum(np.asarray(occ) * e.real)), e


def orthonormalize(ham, c):
    """Row O11: ``S = C^H C`` over the sphere, ``S = L L^H``, ``C <- C L^{-H}``.

    ``c`` is ``[norb, n0, n1, n2]``; the result is zero outside the sphere.
    """
    g = ham.grid
    C = np.where(g.chi, np.asarray(c, np.complex128), 0.0).reshape(c.shape[0], -1).T  # [N, norb]
    S = C.conj().T @ C
    Lc = np.linalg.cholesky(S)
    Cn = scipy.linalg.solve_triangular(Lc.conj(), C.T, lower=True)   # conj(L)^-1 C^T = (C L^-H)^T
    return Cn.reshape(c.shape)


def hartree(grid, n):
    """Periodic Hartree potential of the density ``n`` (Section "Poisson
    solver", periodic boundary conditions): the Poisson equation
    ``-lap V = 4 pi n`` becomes ``|G|^2 V(G) = 4 pi n(G)`` on the full box
    (not the orbital sphere); the ``G = 0`` term is set to zero (a neutralising
    background, so ``V_H`` has zero average).  ``n(G) = N^-1 sum_r n(r)
    e^{-iG.r}`` and ``V(r) = sum_G V(G) e^{+iG.r}``."""
    nG = scipy.fft.fftn(np.asarray(n, np.float64), norm="forward", workers=WORKERS)
    G2 = 2.0 * grid.K
    vG = np.zeros_like(nG)
    nz = G2 > 0
    vG[nz] = 4.0 * np.pi * nG[nz] / G2[nz]
    return scipy.fft.ifftn(vG, norm="forward", workers=WORKERS).real


# Perdew-Zunger (1981) parametrisation of the correlation energy per
# electron of the unpolarised uniform electron gas, eps_c(rs):
#   rs >= 1: gamma / (1 + beta1 sqrt(rs) + beta2 rs)
#   rs < 1:  A ln rs + B + C rs ln rs + D rs
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116


def _rs(n):
    """Wigner-Seitz radius ``rs = (3 / (4 pi n))^(1/3)`` (n > 0)."""
    return np.cbrt(3.0 / (4.0 * np.pi * n))


def lda_exchange(n):
    """Slater exchange of the uniform gas: ``eps_x = -(3/4) (3 n / pi)^(1/3)``
    per electron and ``v_x = d(n eps_x)/dn = (4/3) eps_x``; zero where
    ``n <= 0``.  Returns ``(v_x, eps_x)``."""
    n = np.asarray(n, np.float64)
    pos = n > 0
    e = np.zeros_like(n)
    e[pos] = -0.75 * np.cbrt(3.0 * n[pos] / np.pi)
    return 4.0 / 3.0 * e, e


def lda_correlation(n):
    """Perdew-Zunger correlation: ``eps_c(rs)`` from the two branches above
    and ``v_c = d(n eps_c)/dn = eps_c - (rs/3) d eps_c/d rs``, i.e.
      rs >= 1: eps_c (1 + 7/6 beta1 sqrt(rs) + 4/3 beta2 rs) / (1 + beta1 sqrt(rs) + beta2 rs)
      rs < 1:  A ln rs + (B - A/3) + 2/3 C rs ln rs + (2 D - C) rs / 3;
    zero where ``n <= 0``.  Returns ``(v_c, eps_c)``."""
    n = np.asarray(n, np.float64)
    v = np.zeros_like(n)
    e = np.zeros_like(n)
    pos = n > 0
    rs = _rs(n[pos])
    hi = rs >= 1.0
    ev = np.empty_like(rs)
    vv = np.empty_like(rs)
    s = np.sqrt(rs[hi])
    q = 1.0 + PZ_BETA1 * s + PZ_BETA2 * rs[hi]
    ev[hi] = PZ_GAMMA / q
    vv[hi] = ev[hi] * (1.0 + 7.0 / 6.0 * PZ_BETA1 * s + 4.0 / 3.0 * PZ_BETA2 * rs[hi]) / q
    r = rs[~hi]
    lr = np.log(r)
    ev[~hi] = PZ_A * lr + PZ_B + PZ_C * r * lr + PZ_D * r
    vv[~hi] = PZ_A * lr + (PZ_B - PZ_A / 3.0) + 2.0 / 3.0 * PZ_C * r * lr + (2.0 * PZ_D - PZ_C) * r / 3.0
    v[pos], e[pos] = vv, ev
    return v, e


def lda_xc(n):
    """Local-density exchange-correlation potential ``v_xc[n]`` of
    Eq. hamiltonian (Slater exchange + Perdew-Zunger correlation, spin
    unpolarised) and the energy per electron; returns ``(v_xc, eps_xc)``."""
    vx, ex = lda_exchange(n)
    vc, ec = lda_correlation(n)
    return vx + vc, ex + ec


def with_density(ham, n, xc=False):
    """The Hamiltonian of ``ham`` with local potential ``V_loc + V_H[n]``
    (``+ v_xc[n]`` in the local-density form when ``xc``)."""
    v = ham.vloc + hartree(ham.grid, n)
    if xc:
        v = v + lda_xc(n)[0]
    h = Hamiltonian(ham.grid, v)
    h.atoms, h.d = ham.atoms, ham.d
    return h


def etrs_step(ham, c, dt, occ, nsteps=1, xc=False):
    """``nsteps`` ETRS steps (Eq. etrs) of the orbitals ``c`` under
    ``H[n] = K + V_loc + V_H[n] + V_nl`` (``+ v_xc[n]`` when ``xc``; ``ham``
    holds ``V_loc``).

    One step from ``c(t)``:
      1. ``H(t) = H[n(c(t))]``;
      2. ``w_k = H(t)^k c`` for k = 1..4, shared by the two exponentials of
         ``H(t)``: ``half = sum_k (-i dt/2)^k/k! w_k`` and the predictor
         ``full = sum_k (-i dt)^k/k! w_k`` (Eq. etrs0);
      3. ``H(t+dt) = H[n(full)]``;
      4. ``c(t+dt) = sum_k (-i dt/2)^k/k! H(t+dt)^k half``.
    Returns the orbitals and the densities ``n(c(t+dt))`` after each step."""
    ah = taylor4_coefficients(0.5 * dt)
    af = taylor4_coefficients(dt)
    cur = np.where(ham.grid.chi, np.asarray(c, np.complex128), 0.0)
    dens = []
    for _ in range(nsteps):
        h_t = with_density(ham, density(ham, cur, occ), xc)
        w = cur
        half = cur.copy()
        full = cur.copy()
        for k in range(1, 5):
            w = ham_apply(h_t, w)
            half = half + ah[k] * w
            full = full + af[k] * w
        h_next = with_density(ham, density(ham, full, occ), xc)
        cur = taylor4_step(h_next, half, 0.5 * dt, 1)
        dens.append(density(ham, cur, occ))
    return cur, dens


def positions(grid):
    """Grid positions ``r_a = j_a L_a / n_a`` (cell origin at the corner)."""
    return [np.arange(grid.n[a]) * grid.L[a] / grid.n[a] for a in range(3)]


def kick(grid, c, k):
    """Field kick at t = 0: ``psi(r) -> exp(i k.r) psi(r)`` (the propagator of
    ``v_pert = -k.r delta(t)``), then projected on the plane-wave sphere."""
    x = positions(grid)
    phase = np.exp(1j * (k[0] * x[0][:, None, None] + k[1] * x[1][None, :, None] + k[2] * x[2][None, None, :]))
    psi = synthesize(grid, np.asarray(c, np.complex128))
    return np.where(grid.chi, analyze(grid, phase * psi), 0.0)


def dipole(grid, n):
    """Dipole moment, the first moment of the density: ``dV sum_r r n(r)``."""
    x = positions(grid)
    n = np.asarray(n, np.float64)
    return np.array([grid.dV * np.sum(n * x[0][:, None, None]),
                     grid.dV * np.sum(n * x[1][None, :, None]),
                     grid.dV * np.sum(n * x[2][None, None, :])])


def spectrum(dipoles, dt, k, omegas, damping):
    """Absorption of a kicked propagation (Section "Results": the spectrum is
    the Fourier transform of the dipole moments recorded after the kick).
    ``dipoles[n]`` is d(t_n), t_n = n dt, with d(0) right after the kick;
    x(t) = (d(t) - d(0)) . k/|k|; alpha(w) = |k|^-1 int x(t) e^{iwt - eta t} dt
    by the trapezoidal rule over the recorded times; S(w) = (2w/pi) Im alpha(w),
    whose integral over w is the number of electrons.  Returns (alpha, S)."""
    d = np.asarray(dipoles, np.float64)
    k = np.asarray(k, np.float64)
    kn = float(np.sqrt(np.sum(k * k)))
    x = (d - d[0]) @ (k / kn)
    t = dt * np.arange(len(x))
    w = np.asarray(omegas, np.float64)
    alpha = np.zeros(len(w), np.complex128)
    for i in range(len(w)):
        f = x * np.exp(1j * w[i] * t - damping * t)
        alpha[i] = dt * (np.sum(f) - 0.5 * (f[0] + f[-1])) / kn
    return alpha, 2.0 * w / np.pi * alpha.imag


# ------------------------------------------------- ground state (Section "Ground-state solution")

def teter(x):
    """Preconditioner factor of Teter, Payne and Allan (applied in Fourier
    space, Section "Ground-state solution"):
    ``K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4)``,
    ``x`` the kinetic energy of a plane wave over a reference kinetic energy."""
    x = np.asarray(x, np.float64)
    num = 27.0 + 18.0 * x + 12.0 * x ** 2 + 8.0 * x ** 3
    return num / (num + 16.0 * x ** 4)


def canonical_phases(Q):
    """Scale each column of ``Q`` by a unit phase so that its entry of largest
    modulus (the first one on ties) is real and positive."""
    Q = np.array(Q, np.complex128)
    for j in range(Q.shape[1]):
        k = int(np.argmax(np.abs(Q[:, j])))
        m = abs(Q[k, j])
        Q[:, j] *= np.conj(Q[k, j]) / m
        Q[k, j] = m
    return Q


def subspace_rotation(ham, c, w):
    """Subspace diagonalisation (Section "Ground-state solution"): the
    Rayleigh-Ritz matrix ``Hs = C^H (H C)`` of the orthonormal orbitals ``c``
    (``w = H c``), made exactly Hermitian, ``Hs = Q diag(e) Q^H`` with ``e``
    ascending and the phases of :func:`canonical_phases`; returns
    ``(C Q, W Q, e)``."""
    nb = c.shape[0]
    C = np.where(ham.grid.chi, c, 0.0).reshape(nb, -1)
    W = np.asarray(w, np.complex128).reshape(nb, -1)
    Hs = C.conj() @ W.T                       # Hs[i, j] = <c_i | H c_j>
    Hs = 0.5 * (Hs + Hs.conj().T)
    e, Q = np.linalg.eigh(Hs)
    Q = canonical_phases(Q)
    return (Q.T @ C).reshape(c.shape), (Q.T @ W).reshape(c.shape), e


def sd_direction(ham, c, w, e):
    """Preconditioned steepest-descent direction of each orbital:
    residual ``r = H c - e c``; reference kinetic energy
    ``T = sum K |r|^2 / sum |r|^2`` of the residual (``K = |G|^2/2``);
    ``p = teter(K / T) r`` (``p = r`` when ``T = 0``, ``p = 0`` when
    ``r = 0``); ``p <- p - <c|p> c``.  Returns ``(p, |r|)``."""
    g = ham.grid
    c = np.where(g.chi, c, 0.0)
    r = np.where(g.chi, w - e[:, None, None, None] * c, 0.0)
    ax = (-3, -2, -1)
    rr = np.sum(np.abs(r) ** 2, axis=ax)
    kr = np.sum(g.K * np.abs(r) ** 2, axis=ax)
    p = np.zeros_like(r)
    for i in range(c.shape[0]):
        if rr[i] == 0.0:
            continue
        T = kr[i] / rr[i]
        p[i] = r[i] if T <= 0.0 else teter(g.K / T) * r[i]
        p[i] = np.where(g.chi, p[i], 0.0)
        p[i] -= np.vdot(c[i], p[i]) * c[i]
    return p, np.sqrt(rr)


def sd_iteration(ham, c):
    """One iteration of the preconditioned steepest-descent eigensolver
    (Section "Ground-state solution") on orthonormal orbitals ``c``:

    1. ``W = H C``; subspace diagonalisation (:func:`subspace_rotation`)
       gives the Ritz values ``e``;
    2. per orbital the direction ``p`` of :func:`sd_direction`, normalised
       to ``q``;
    3. exact line minimisation of the Rayleigh quotient over the span of
       ``c`` and ``q``: the lowest eigenvector ``y`` (``|y| = 1``, ``y_0``
       real and non-negative; ``y_1`` real and positive when ``y_0 = 0``) of
       ``[[e, <c|Hq>], [<q|Hc>, <q|Hq>]]``, and ``c <- y_0 c + y_1 q``
       (unchanged when ``p = 0``);
    4. orthonormalisation (:func:`orthonormalize`).

    Returns ``(c, e, |r|)``."""
    g = ham.grid
    c = np.where(g.chi, np.asarray(c, np.complex128), 0.0)
    w = ham_apply(ham, c)
    c, w, e = subspace_rotation(ham, c, w)
    p, rn = sd_direction(ham, c, w, e)
    ax = (-3, -2, -1)
    u = np.sum(np.abs(p) ** 2, axis=ax)
    live = u > 0.0
    q = np.zeros_like(p)
    q[live] = p[live] / np.sqrt(u[live])[:, None, None, None]
    hq = ham_apply(ham, q)
    out = c.copy()
    for i in np.nonzero(live)[0]:
        b = np.vdot(c[i], hq[i])
        d = np.vdot(q[i], hq[i]).real
        lam, Y = np.linalg.eigh(np.array([[e[i], b], [np.conj(b), d]]))
        y = Y[:, 0]
        if abs(y[0]) > 0.0:
            y = y * np.conj(y[0]) / abs(y[0])
        else:
            y = y * np.conj(y[1]) / abs(y[1])
        out[i] = y[0] * c[i] + y[1] * q[i]
    return orthonormalize(ham, out), e, rn
