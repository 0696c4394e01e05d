"""Seeded synthetic inputs for the Kohn-Sham hot path.

This module only *draws inputs*: atom positions, a local potential field,
Kleinman-Bylander projector spheres and their radial forms, KB coefficients
and random plane-wave coefficients.  It performs none of the method's own
arithmetic (no FFT, no Hamiltonian, no cutoff mask, no normalisation of
orbitals) and it is the only code that both the oracle-side tests and the
GPU path consume.  The paper's systems (N2, Si, H2O, Al) need pseudopotential
files that are not available, so smooth Gaussian stand-ins of the same shape
are used (Section "Pseudopotentials": a multiplicative local part plus
sphere-localised projectors, Eq. vnl).

Recipe (all lengths in bohr, energies in Hartree, atomic units as in the
statement of the Hamiltonian, Eq. hamiltonian):

* grid ``n = (n0, n1, n2)`` on an orthorhombic cell ``L``; point ``j`` sits at
  ``r_j = (j0 L0/n0, j1 L1/n1, j2 L2/n2)``.
* atoms uniform in the cell.  Positions are redrawn whenever a grid point lies
  within a relative 1e-10 of a projector-sphere surface, so that sphere
  membership is never decided by rounding.
* local potential ``V(r) = sum_I sum_T -2 exp(-|r - R_I - T|^2 / 2)`` (depth
  2 Ha, width 1 bohr), summed over periodic images ``T`` until the Gaussian
  factor drops below 1e-20.
* projectors per atom, ordered ``[s, p_x, p_y, p_z]``:
  ``beta_s = exp(-r^2/(2 sigma^2))``, ``beta_pa = r_a exp(-r^2/(2 sigma^2))``
  with ``sigma = 0.8`` and ``r`` the minimum-image displacement, restricted to
  ``|r| < R_c = 2`` and scaled so that ``dV sum beta^2 = 1`` on the grid.
* KB coefficients ``d`` uniform in [0.5, 2], one value per (atom, l), shared by
  the three p components.
* orbital coefficients ``(a + i b) exp(-|G|^2/8)`` with ``a, b ~ N(0, 1)`` on all
  box points with ``|G|^2/2 < 1.1 E_cut`` (the whole box when ``E_cut <= 0``),
  zero elsewhere.  The 10 % margin is deliberate: coefficients just outside the
  plane-wave sphere are garbage that every consumer must ignore.

Random streams: ``numpy.random.default_rng`` (PCG64) children of
``SeedSequence(seed)``: child 0 draws positions, child 1 the KB coefficients,
child 2 the orbital coefficients.  Draws never depend on chunking or device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

R_CUT = 2.0          # projector sphere radius (bohr)
SIGMA_BETA = 0.8     # projector Gaussian width (bohr)
V_DEPTH = 2.0        # local Gaussian depth (Ha)
V_WIDTH = 1.0        # local Gaussian width (bohr)
NPROJ = 4            # s, px, py, pz
ORB_MARGIN = 1.1     # generate coefficients up to 1.1 * E_cut


@dataclass(frozen=True)
class Spec:
    """One synthetic Kohn-Sham system."""

    name: str
    n: tuple
    L: tuple
    ecut: float
    norb: int
    natoms: int
    seed: int
    occ: float = 1.0
    dt: float = 0.05
    nsteps: int = 1
    extra: dict = field(default_factory=dict, compare=False)

    @property
    def npoints(self) -> int:
        return int(np.prod(self.n))


def _cubic(name, n, L, norb, natoms, seed, **kw):
    return Spec(name=name, n=(n, n, n), L=(float(L),) * 3, ecut=10.0,
                norb=norb, natoms=natoms, seed=seed, **kw)


# The five workloads (sizes from the headline configuration list) plus small
# test systems that span several kernel tiles and leave ragged tails.
CONFIGS = {
    "cfg1_16": _cubic("cfg1_16", 16, 10.0, 8, 2, 1001, dt=0.05, nsteps=1),
    "cfg2_64": _cubic("cfg2_64", 64, 20.0, 128, 32, 1002),
    "cfg3_96": _cubic("cfg3_96", 96, 30.0, 512, 128, 1003, occ=2.0, dt=0.05, nsteps=20),
    "cfg4_96": _cubic("cfg4_96", 96, 30.0, 512, 128, 1004, occ=2.0, dt=0.05, nsteps=20),
    "cfg4_120": _cubic("cfg4_120", 120, 37.5, 1024, 256, 1005, occ=2.0, dt=0.05, nsteps=20),
    # small parity systems
    "t24": _cubic("t24", 24, 10.0, 10, 3, 7001, dt=0.05, nsteps=2),
    "t40": Spec(name="t40", n=(40, 40, 40), L=(13.2, 13.2, 13.2), ecut=10.0,
                norb=5, natoms=4, seed=7002, occ=2.0, dt=0.05, nsteps=1),
    "t32x": Spec(name="t32x", n=(32, 32, 32), L=(10.0, 11.0, 12.0), ecut=10.0,
                 norb=6, natoms=3, seed=7003, dt=0.04, nsteps=1),
    "t60": _cubic("t60", 60, 19.8, 3, 5, 7004, dt=0.05, nsteps=1),
    "t48": _cubic("t48", 48, 15.0, 33, 6, 7005, dt=0.05, nsteps=1),
}


def cubic_spec(name, n, L, norb, natoms, seed, **kw) -> Spec:
    return _cubic(name, n, L, norb, natoms, seed, **kw)


def _streams(seed):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(3)]


def _axis_coords(spec):
    return [np.arange(spec.n[a]) * (spec.L[a] / spec.n[a]) for a in range(3)]


def _min_image(x, R, L):
    return (x - R + 0.5 * L) % L - 0.5 * L


def _sphere_ties(spec, pos):
    """True when some grid point sits within 1e-10 (relative) of a sphere surface."""
    xs = _axis_coords(spec)
    rc2 = R_CUT * R_CUT
    for R in pos:
        d = [_min_image(xs[a], R[a], spec.L[a]) for a in range(3)]
        r2 = d[0][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[2][None, None, :] ** 2
        if np.any(np.abs(r2 - rc2) < 1e-10 * rc2):
            return True
    return False


def positions(spec) -> np.ndarray:
    rng = _streams(spec.seed)[0]
    L = np.asarray(spec.L)
    for _ in range(100):
        pos = rng.random((spec.natoms, 3)) * L
        if not _sphere_ties(spec, pos):
            return pos
    raise RuntimeError("could not draw tie-free atom positions")


def vloc(spec, pos=None) -> np.ndarray:
    """Sum of attractive periodic Gaussians on the grid, float64 [n0, n1, n2]."""
    if pos is None:
        pos = positions(spec)
    xs = _axis_coords(spec)
    rmax = math.sqrt(2.0 * V_WIDTH ** 2 * math.log(1e20))
    v = np.zeros(spec.n)
    for R in pos:
        g = []
        for a in range(3):
            La = spec.L[a]
            nimg = int(math.ceil(rmax / La)) + 1
            ga = np.zeros(spec.n[a])
            for t in range(-nimg, nimg + 1):
                ga += np.exp(-((xs[a] - R[a] - t * La) ** 2) / (2.0 * V_WIDTH ** 2))
            g.append(ga)
        v += -V_DEPTH * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
    return v


@dataclass
class Projectors:
    npts: np.ndarray   # int32 [natoms]
    idx: np.ndarray    # int32 [sum npts], flat C-order grid index
    beta: np.ndarray   # float64 [sum npts, NPROJ]
    d: np.ndarray      # float64 [natoms, NPROJ]

    def atom(self, i):
        off = int(self.npts[:i].sum())
        n = int(self.npts[i])
        return self.idx[off:off + n], self.beta[off:off + n]


def projectors(spec, pos=None) -> Projectors:
    if pos is None:
        pos = positions(spec)
    xs = _axis_coords(spec)
    dV = float(np.prod(spec.L)) / spec.npoints
    rc2 = R_CUT * R_CUT
    npts, idxs, betas = [], [], []
    for R in pos:
        d = [_min_image(xs[a], R[a], spec.L[a]) for a in range(3)]
        D0, D1, D2 = np.meshgrid(d[0], d[1], d[2], indexing="ij")
        r2 = D0 ** 2 + D1 ** 2 + D2 ** 2
        flat = np.flatnonzero(r2.ravel() < rc2)
        g = np.exp(-r2.ravel()[flat] / (2.0 * SIGMA_BETA ** 2))
        b = np.stack([g, D0.ravel()[flat] * g, D1.ravel()[flat] * g, D2.ravel()[flat] * g], axis=1)
        b /= np.sqrt(dV * np.sum(b * b, axis=0))[None, :]
        npts.append(len(flat))
        idxs.append(flat.astype(np.int32))
        betas.append(b)
    rng = _streams(spec.seed)[1]
    dl = rng.uniform(0.5, 2.0, size=(spec.natoms, 2))
    dcoef = np.stack([dl[:, 0], dl[:, 1], dl[:, 1], dl[:, 1]], axis=1)
    return Projectors(np.asarray(npts, np.int32), np.concatenate(idxs),
                      np.ascontiguousarray(np.concatenate(betas)), np.ascontiguousarray(dcoef))


def orbital_support(spec) -> np.ndarray:
    """Flat box indices that receive random coefficients (|G|^2/2 < 1.1 E_cut)."""
    g2 = np.zeros(spec.n)
    for a in range(3):
        na = spec.n[a]
        j = np.arange(na)
        ma = np.where(j < (na + 1) // 2, j, j - na)
        ga = 2.0 * np.pi * ma / spec.L[a]
        shape = [1, 1, 1]
        shape[a] = na
        g2 = g2 + (ga ** 2).reshape(shape)
    if spec.ecut <= 0:
        return np.arange(spec.npoints), g2.ravel()
    sel = np.flatnonzero(g2.ravel() < 2.0 * ORB_MARGIN * spec.ecut)
    return sel, g2.ravel()[sel]


def orbital_values(spec, norb=None) -> tuple:
    """(support indices int64, values complex128 [norb, nsupport])."""
    norb = spec.norb if norb is None else norb
    sel, g2 = orbital_support(spec)
    rng = _streams(spec.seed)[2]
    z = rng.standard_normal((norb, len(sel), 2))
    damp = np.exp(-g2 / 8.0)
    vals = (z[..., 0] + 1j * z[..., 1]) * damp[None, :]
    return sel, vals


def orbitals_box(spec, norb=None) -> np.ndarray:
    """Dense complex128 [norb, n0, n1, n2] coefficient boxes (small systems)."""
    sel, vals = orbital_values(spec, norb)
    out = np.zeros((vals.shape[0], spec.npoints), np.complex128)
    out[:, sel] = vals
    return out.reshape((vals.shape[0],) + tuple(spec.n))


def occupations(spec, norb=None) -> np.ndarray:
    norb = spec.norb if norb is None else norb
    return np.full(norb, float(spec.occ))


@dataclass
class System:
    spec: Spec
    pos: np.ndarray
    vloc: np.ndarray
    proj: Projectors


def system(spec) -> System:
    pos = positions(spec)
    return System(spec, pos, vloc(spec, pos), projectors(spec, pos))


def serving_trace(nreq=256, mean_rate=200.0, seed=2000):
    """Poisson arrival trace of independent small systems (mixed precision serving)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / mean_rate, size=nreq)
    t = np.cumsum(gaps)
    grids = rng.choice([24, 32, 40, 48, 60, 64], size=nreq)
    norbs = rng.integers(8, 257, size=nreq)
    nats = rng.integers(2, 33, size=nreq)
    reqs = []
    for r in range(nreq):
        n = int(grids[r])
        reqs.append((float(t[r]), cubic_spec(f"srv{r}", n, 0.33 * n, int(norbs[r]), int(nats[r]),
                                              3000 + r, dt=0.05, nsteps=50)))
    return reqs
