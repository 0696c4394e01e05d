/*
 * ks.h -- C ABI of libks: the data-parallel hot path of plane-wave real-time
 * TDDFT (Andrade et al., arXiv:2106.03872) on one AMD Instinct MI355X.
 *
 * Physics (atomic units throughout, as in the statement of the Hamiltonian,
 * Eq. hamiltonian):
 *   H = -1/2 nabla^2 + V_loc(r) + sum_I sum_p |beta_Ip> d_Ip <beta_Ip|
 * with a static multiplicative local potential (Section "Pseudopotentials":
 * local pseudopotential, Hartree and XC combine into one field) and
 * Kleinman-Bylander projectors localised in spheres (Eq. vnl).  H acts on the
 * plane-wave sphere chi(G) = [|G|^2/2 < E_cut] (H = chi H chi), kinetic term
 * in Fourier space, potential terms in real space, two FFTs per application
 * (Section "Implementation of the KS Hamiltonian").
 *
 * Conventions shared by every call:
 *  - Grid n = (n0, n1, n2), orthorhombic cell L = (L0, L1, L2) bohr, N = n0 n1 n2,
 *    Omega = L0 L1 L2, dV = Omega / N.  n1 must equal n2; every n_a must be one
 *    of 8 12 16 20 24 32 40 48 60 64 72 80 96 120 128.
 *  - Orbitals are plane-wave coefficients on the full FFT box, complex128
 *    interleaved (re, im), array [norb][n0][n1][n2] in C order (n2 fastest).
 *    Box index j_a holds m_a = j_a for j_a < ceil(n_a/2), else j_a - n_a;
 *    G_a = 2 pi m_a / L_a.  psi(r) = Omega^{-1/2} sum_G chi c_G exp(+i G.r),
 *    so int |psi|^2 = sum |c|^2.  Inputs outside chi are ignored; outputs are
 *    zero there.
 *  - Real-space fields (V_loc, density) are float64 [n0][n1][n2] with
 *    r_j = (j0 L0/n0, j1 L1/n1, j2 L2/n2).
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the system copies what it keeps.
 *  - stream is a hipStream_t (NULL = default stream).  Calls taking a stream
 *    are asynchronous with respect to the host and ordered on that stream.
 *    One ks_system must not be used from two threads or two streams at once
 *    (it owns one workspace); distinct systems are independent.
 *  - Errors: every call returns a ks_status and never aborts; ks_last_error()
 *    gives the message of the last failure on that system.
 */
#ifndef KS_H
#define KS_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KS_OK = 0,
  KS_EINVAL = 1,        /* bad argument: null pointer, size, aliasing, cutoff */
  KS_ENOMEM = 2,        /* device allocation failed */
  KS_EDEVICE = 3,       /* a HIP runtime error; see ks_last_error */
  KS_EUNSUPPORTED = 4   /* grid size or sphere without a kernel */
} ks_status;

typedef enum {
  KS_FP64 = 0,          /* all arithmetic in float64 / complex128 */
  KS_MIXED = 1          /* FP32 (complex64) transforms and pointwise work; orbital
                           state, Taylor sum, density, norms, energy in FP64 */
} ks_precision;

typedef struct ks_system ks_system;

/*
 * Create a system for grid n[3] (host), cell L[3] (host, bohr) and cutoff
 * ecut (Ha; ecut <= 0 means the whole FFT box, no sphere).  Builds the
 * plane-wave sphere tables (kinetic energies |G|^2/2 and the mask, from the
 * plane-wave basis of Section "DFT and TDDFT implementation") and allocates
 * the workspace of the H psi, propagation, density and reduction calls, so
 * that these allocate nothing.  Calls that do allocate device memory:
 * ks_system_set_projectors (its tables and projection workspace),
 * ks_system_set_chunk, the first ks_orthonormalize or ks_state_eigensolve of
 * a system (overlap matrices), ks_state_create, and the first
 * ks_state_propagate_etrs / ks_state_eigensolve of a state (extra orbital
 * blocks).  max_norb bounds norb in every later call.
 * Errors: KS_EINVAL (null, n < 1, L <= 0, max_norb < 1, n1 != n2, ecut > 0
 * with a sphere that contains a point of the Nyquist plane m_a = -n_a/2 of an
 * even n_a), KS_EUNSUPPORTED (size without a kernel, sphere too large for
 * LDS), KS_ENOMEM.  On error *out is NULL.
 */
ks_status ks_system_create(const int n[3], const double L[3], double ecut, int precision,
                           int max_norb, ks_system** out);

/*
 * Free the system and its device memory.  Waits for the work the system's
 * calls enqueued (on any stream, including replays of its states' captured
 * steps), not for the rest of the device.  With a pool the memory returns to
 * the pool and no HIP free is called.
 */
void ks_system_destroy(ks_system* sys);

/*
 * A non-blocking stream (hipStreamNonBlocking, default priority) on the
 * current device.  Work on it never waits for, and is never waited for by,
 * the legacy default stream, so a graph can be captured on it (ks_state_capture,
 * ks_batch_capture) while other threads use the default stream, as they do
 * for blocking host transfers.  KS_EINVAL on null, KS_EDEVICE.
 */
ks_status ks_stream_create(void** stream);
/* Destroy a stream from ks_stream_create (after its work has completed). */
void ks_stream_destroy(void* stream);

/*
 * Device memory pool for many short-lived systems (serving): one device
 * allocation of `bytes`, sub-allocated on the host, so that creating and
 * destroying pooled systems and their states calls no hipMalloc / hipFree
 * (which may synchronise the device).  A pool belongs to the device current
 * at its creation.  Errors: KS_EINVAL (null, bytes == 0), KS_ENOMEM.
 */
typedef struct ks_pool ks_pool;
ks_status ks_pool_create(unsigned long long bytes, ks_pool** out);
/* Free the pool's device memory; every system created in it must have been
 * destroyed. */
void ks_pool_destroy(ks_pool* pool);
/* Bytes in use, the most ever in use, and the largest free range (each
 * output nullable).  KS_EINVAL on a null pool. */
ks_status ks_pool_usage(ks_pool* pool, unsigned long long* used, unsigned long long* peak,
                        unsigned long long* largest_free);
/*
 * As ks_system_create, with every device buffer of the system and of its
 * states taken from `pool` (the pool's device must be current).  An
 * exhausted pool gives KS_ENOMEM, at creation or at the call that allocates
 * (see ks_system_create); the pool is not grown.  The message of a failed
 * creation is ks_last_error(NULL).
 */
ks_status ks_system_create_in(ks_pool* pool, const int n[3], const double L[3], double ecut, int precision,
                              int max_norb, ks_system** out);

/*
 * ks_system_create (pool == NULL) or ks_system_create_in with the orbitals
 * per pass set at creation: chunk > 0 sizes the workspace (plane
 * intermediates, packed pass buffers, projection partials) for
 * min(chunk, max_norb, 65535) orbitals, chunk == 0 takes the default (as
 * many orbitals as 16 GiB of plane intermediates hold, at most 65535: the
 * pass kernels put a pass's orbitals on the y extent of their launch grid).
 * Calls over more orbitals run in passes, with the same results.  A caller that holds many systems
 * (serving) trades passes for memory this way without the default
 * workspace ever being allocated.  KS_EINVAL for chunk < 0, otherwise as
 * ks_system_create / ks_system_create_in.
 */
ks_status ks_system_create_ex(ks_pool* pool, const int n[3], const double L[3], double ecut, int precision,
                              int max_norb, int chunk, ks_system** out);

/* Message of the last failing call on sys (or of the last failing create
 * when sys is NULL).  Valid until the next call on sys. */
const char* ks_last_error(const ks_system* sys);

/*
 * Set the local potential V_loc(r) (Eq. hamiltonian: ionic local part plus
 * any Hartree/XC/perturbation terms, combined as one multiplicative field).
 * v: device float64 [n0][n1][n2], copied on `stream`.  Default: V = 0.
 */
ks_status ks_system_set_vloc(ks_system* sys, const double* v, void* stream);

/*
 * Set the Kleinman-Bylander non-local term of Eq. vnl:
 *   v_nl psi(r) = sum_I sum_p beta_Ip(r) d_Ip dV sum_{j in S_I} beta_Ip(r_j) psi(r_j).
 * natoms >= 0, nproj >= 1 projectors per atom.  All arrays are host memory:
 *   npts [natoms]            number of grid points of sphere S_I
 *   idx  [sum npts]          flat C-order grid indices of the points of S_I,
 *                            atoms concatenated (duplicates count twice)
 *   beta [sum npts][nproj]   projector values at those points (row-major)
 *   d    [natoms][nproj]     KB coefficients
 * The library copies and regroups them (it keeps the host copies, so that a
 * change of x-tile shape can regroup them again); it synchronises `stream`
 * (pass the stream later calls use).  natoms = 0 removes the non-local term.
 * The new device tables are allocated and filled before the old ones are
 * freed: on KS_ENOMEM the system keeps its previous tables.
 * Errors: KS_EINVAL on null arrays or an index outside [0, N); KS_ENOMEM.
 */
ks_status ks_system_set_projectors(ks_system* sys, int natoms, int nproj, const int* npts,
                                   const int* idx, const double* beta, const double* d, void* stream);

/*
 * hpsi = H psi for norb orbitals (Section "Implementation of the KS
 * Hamiltonian").  psi, hpsi: device complex128 [norb][n0][n1][n2]; they must
 * not overlap.  Errors: KS_EINVAL (null, norb < 0 or > max_norb, psi == hpsi).
 */
ks_status ks_ham_apply(ks_system* sys, int norb, const void* psi, void* hpsi, void* stream);

/*
 * nsteps steps of the 4th-order truncated Taylor propagator (Section
 * "Real-time propagation"):
 *   psi <- sum_{k=0}^{4} (-i dt)^k / k!  H^k psi
 * applied in place to psi (device complex128 [norb][n0][n1][n2]).
 * rho: NULL, or device float64 [nsteps][n0][n1][n2] receiving the density
 * sum_i occ_i |psi_i(r)|^2 (Eq. density) after each step; occ: device
 * float64 [norb], required when rho is given.
 * Errors: KS_EINVAL (null psi, norb out of range, nsteps < 0, rho without occ).
 */
ks_status ks_propagate_step(ks_system* sys, int norb, void* psi, double dt, int nsteps,
                            const double* occ, double* rho, void* stream);

/*
 * rho(r) = sum_i occ_i |psi_i(r)|^2 (Eq. density with occupations).
 * psi: device complex128 [norb][n0][n1][n2]; occ: device float64 [norb];
 * rho: device float64 [n0][n1][n2] (overwritten).  Summation order over
 * orbitals is fixed, so the result is deterministic.
 */
ks_status ks_density(ks_system* sys, int norb, const void* psi, const double* occ, double* rho,
                     void* stream);

/*
 * Periodic Hartree potential (Section "Poisson solver", periodic boundary
 * conditions): v = V_H[rho] with V_H(G) = 4 pi rho(G) / |G|^2 for G != 0 and
 * V_H(G = 0) = 0 (a neutralising background: V_H has zero average),
 * rho(G) = N^-1 sum_r rho(r) e^{-iG.r}, V_H(r) = sum_G V_H(G) e^{+iG.r}, over
 * the whole box.  With add_vloc != 0 the system's static V_loc is added.
 * rho, v: device float64 [n0][n1][n2] (may be the same array).  KS_EINVAL on
 * null arguments.
 */
ks_status ks_hartree(ks_system* sys, const double* rho, double* v, int add_vloc, void* stream);

/* Exchange-correlation functionals of the density-dependent potential. */
typedef enum { KS_XC_NONE = 0, KS_XC_LDA = 1 } ks_xc;

/*
 * The exchange-correlation term v_xc[n] of Eq. hamiltonian that
 * ks_state_propagate_etrs adds to V_loc + V_H[n]: KS_XC_NONE (the default)
 * or KS_XC_LDA, the local-density form of the unpolarised electron gas
 * (see ks_lda_xc).  KS_EINVAL for a null system or another value.
 */
ks_status ks_system_set_xc(ks_system* sys, int functional);

/*
 * Local-density exchange-correlation potential of the density rho:
 * v (+)= v_xc(rho) pointwise (accumulate != 0 adds), with
 *   v_xc = v_x + v_c,  v_x = -(3 rho / pi)^(1/3) (Slater exchange),
 *   v_c = eps_c - (rs/3) d eps_c/d rs,  rs = (3 / (4 pi rho))^(1/3),
 *   eps_c = gamma / (1 + beta1 sqrt(rs) + beta2 rs)   (rs >= 1),
 *   eps_c = A ln rs + B + C rs ln rs + D rs           (rs < 1),
 * the Perdew-Zunger (1981) fit of the uniform gas's correlation energy
 * (gamma = -0.1423, beta1 = 1.0529, beta2 = 0.3334, A = 0.0311, B = -0.048,
 * C = 0.0020, D = -0.0116, Hartree atomic units); zero where rho <= 0.
 * rho, v: device float64 [n0][n1][n2] (may be the same array only without
 * accumulate).  KS_EINVAL on null arguments.
 */
ks_status ks_lda_xc(ks_system* sys, const double* rho, double* v, int accumulate, void* stream);

/*
 * Dipole moment, the first moment of the density (Section "Results", the
 * optical response of a kicked molecule): d_a = dV sum_r r_a rho(r) with grid
 * positions r_a = j_a L_a / n_a.  rho: device float64 [n0][n1][n2]; d: device
 * float64 [3].  Fixed summation order (deterministic).  KS_EINVAL on null
 * arguments.
 */
ks_status ks_dipole(ks_system* sys, const double* rho, double* d, void* stream);

/*
 * Allocation-free ks_dipole, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops): no ks_system is needed,
 * and the call makes no hipMalloc/hipFree or other allocating call.  Same
 * kernels and summation order as ks_dipole, so the results are identical.
 * n[3], L[3]: host; rho: device float64 [n0][n1][n2]; d: device float64 [3].
 * The partial sums live in a fixed 6 KiB array in the library's device image,
 * one per GPU, kept until the process ends; its device address is looked up
 * on the first call on each device.  Every call on one GPU uses that GPU's
 * array, so calls that overlap in time on one GPU (different streams or
 * threads) race: order them.  Errors: KS_EINVAL (null, n_a < 1, L_a <= 0, more
 * than KS_DIPOLE_NOALLOC_MAX_POINTS grid points), KS_EDEVICE; the message is
 * ks_last_error(NULL).
 */
#define KS_DIPOLE_NOALLOC_MAX_POINTS 2147483647LL
ks_status ks_dipole_noalloc(const int n[3], const double L[3], const double* rho, double* d, void* stream);

/*
 * Absorption spectrum of a kicked propagation (Section "Results": the
 * spectrum is the Fourier transform of the dipole moments after the kick):
 *   x(t_n) = (d(t_n) - d(0)) . k / |k|,  t_n = n dt,
 *   alpha(w) = |k|^-1 dt sum_{n=0}^{nt-1} c_n x(t_n) exp(i w t_n - damping t_n)
 *              (trapezoid weights: c_0 = c_{nt-1} = 1/2, else 1),
 *   S(w) = (2 w / pi) Im alpha(w)   (its integral over w is the number of
 *                                    electrons: the f-sum rule).
 * dipoles: device float64 [nt][3] with d(0), the dipole right after the kick,
 * first; k: host [3], the kick (bohr^-1); omegas: device float64 [nw] (Ha);
 * alpha: device float64 [nw][2] (re, im); strength: device float64 [nw].
 * Fixed summation order (deterministic).  No system needed.  KS_EINVAL:
 * null arguments, nt < 1, nw < 0, dt <= 0, non-finite damping, k zero or
 * non-finite; the message is ks_last_error(NULL).
 */
ks_status ks_spectrum(const double* dipoles, int nt, double dt, const double k[3], const double* omegas, int nw,
                      double damping, double* alpha, double* strength, void* stream);

/*
 * Orbital norms and band energy (energy expression of Section "DFT and TDDFT
 * implementation" reduced to sum_k f_k <psi_k|H|psi_k> for a static potential):
 *   norms[i] = sum_G |c_iG|^2 over the sphere           (device float64 [norb])
 *   energy[0] = sum_i occ_i Re <c_i|H c_i>               (device float64 [1])
 * Either output may be NULL; occ (device [norb]) is required for energy.
 */
ks_status ks_reduce(ks_system* sys, int norb, const void* psi, const double* occ, double* norms,
                    double* energy, void* stream);

/*
 * Orthonormalise the orbitals in place (orthogonalisation step of Section
 * "Ground-state solution"): S = C^H C over the sphere, S = L L^H (Cholesky,
 * positive diagonal), C <- C L^{-H}.  psi: device complex128
 * [norb][n0][n1][n2].  KS_EINVAL when a Cholesky pivot drops to 1e-12 of its
 * diagonal entry of S (numerically linearly dependent orbitals).  The first
 * call allocates a workspace for max_norb orbitals; the call synchronises
 * `stream` to read the pivot check.
 */
ks_status ks_orthonormalize(ks_system* sys, int norb, void* psi, void* stream);

/* ------------------------------------------------------------------------
 * Resident orbitals.  A ks_state holds norb orbitals of one system on the
 * device in the library's packed FP64 sphere layout, so that repeated steps
 * need no box conversion.  It belongs to its system (same stream rules) and
 * must be destroyed before the system.
 */
typedef struct ks_state ks_state;

/* Allocate the state (device memory for norb packed orbitals). */
ks_status ks_state_create(ks_system* sys, int norb, ks_state** out);
/* Free the state (waits for its system's enqueued work only). */
void ks_state_destroy(ks_state* state);
/* psi (device complex128 box [norb][n0][n1][n2]) -> state; outside chi ignored. */
ks_status ks_state_upload(ks_state* state, const void* psi, void* stream);
/* state -> psi (device complex128 box; zero outside chi). */
ks_status ks_state_download(ks_state* state, void* psi, void* stream);
/* As ks_propagate_step, on the resident orbitals; in addition, norms (NULL,
 * or device float64 [nsteps][norb]) receives ||c_i||^2 after each step.
 * Within one call the density of step s (s < nsteps-1) is taken from the
 * first H psi of step s+1, which synthesises the same orbitals. */
ks_status ks_state_propagate(ks_state* state, double dt, int nsteps, const double* occ, double* rho, double* norms,
                             void* stream);
/*
 * nsteps steps of the enforced-time-reversal-symmetry propagator (Eq. etrs)
 * under the density-dependent Hamiltonian H[n] = -1/2 lap + V_loc + V_H[n]
 * (+ v_xc[n] when ks_system_set_xc chose a functional) + V_nl, V_H the
 * periodic Hartree potential (see ks_hartree) and n = sum_i occ_i |psi_i|^2.
 * One step from psi(t):
 *   H(t) = H[n(psi(t))];
 *   w_k = H(t)^k psi for k = 1..4, shared by the two exponentials of H(t)
 *   (Section "Real-time propagation"): half = sum_k (-i dt/2)^k/k! w_k and the
 *   predictor full = sum_k (-i dt)^k/k! w_k (Eq. etrs0);
 *   H(t+dt) = H[n(full)];  psi(t+dt) = sum_k (-i dt/2)^k/k! H(t+dt)^k half.
 * That is 8 H psi and 2 densities per step.  occ is required; rho (NULL, or
 * float64 [nsteps][n0][n1][n2]) and norms (NULL, or float64 [nsteps][norb])
 * receive the density and ||c_i||^2 after each step.  The first call on a
 * state allocates its predictor buffer (norb packed orbitals).  The system's
 * potential is V_loc again when the call returns.  KS_EINVAL: null state or
 * occ, nsteps < 0, non-finite dt.
 */
ks_status ks_state_propagate_etrs(ks_state* state, double dt, int nsteps, const double* occ, double* rho,
                                  double* norms, void* stream);
/*
 * Field kick at t = 0 (the propagator of v_pert = -k.r delta(t) in Eq.
 * hamiltonian): every resident orbital becomes exp(i k.r) psi(r) with grid
 * positions r_a = j_a L_a / n_a, projected on the plane-wave sphere.  k: host
 * array of 3 (bohr^-1).  One orbital at a time through the system's work box
 * (a set-up operation, not the hot path).  KS_EINVAL: null state or k, or a
 * non-finite k.
 */
ks_status ks_state_kick(ks_state* state, const double k[3], void* stream);
/*
 * niter iterations of the preconditioned steepest-descent eigensolver
 * (Section "Ground-state solution") for the lowest norb eigenstates of the
 * system's static Hamiltonian, on the resident orbitals, which must be
 * orthonormal on entry (ks_orthonormalize) and are orthonormal on return.
 * One iteration:
 *   1. W = H C; subspace diagonalisation: the Rayleigh-Ritz matrix
 *      C^H W, made exactly Hermitian, = Q diag(e) Q^H with e ascending and
 *      each column of Q scaled so that its entry of largest modulus (the
 *      first on ties) is real and positive; C <- C Q, W <- W Q (the
 *      eigenproblem by blocked Jacobi sweeps until the off-diagonal
 *      Frobenius norm is at most 1e-14 of the matrix's, at most 60 sweeps);
 *   2. per orbital: residual r = w - e c; T = sum_G K|r|^2 / sum_G |r|^2
 *      with K = |G|^2/2; direction p = t(K/T) r with the Teter-Payne-Allan
 *      factor t(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4) (p = r
 *      when T = 0, p = 0 when r = 0); p <- p - <c|p> c; q = p/|p|;
 *   3. exact line minimisation of the Rayleigh quotient over span{c, q}:
 *      c <- y0 c + y1 q with y the lowest normalised eigenvector of
 *      [[e, <c|Hq>], [<q|Hc>, <q|Hq>]], y0 real >= 0 (c unchanged when p = 0);
 *   4. Cholesky orthonormalisation.
 * eig and resid (NULL, or device float64 [niter][norb]) receive e and |r|
 * of each iteration (the values at step 1-2, before the update).  FP64
 * systems only.  The first call on a state allocates three more orbital
 * blocks and about 6 norb^2 complex entries; every iteration synchronises the
 * stream (Jacobi convergence and the Cholesky status).  Errors: KS_EINVAL
 * (null state, niter < 0, linearly dependent orbitals), KS_EUNSUPPORTED
 * (mixed precision), KS_EDEVICE (Jacobi sweeps not converged, HIP errors).
 */
ks_status ks_state_eigensolve(ks_state* state, int niter, double* eig, double* resid, void* stream);
/* As ks_reduce, on the resident orbitals. */
ks_status ks_state_reduce(ks_state* state, const double* occ, double* norms, double* energy, void* stream);
/*
 * Capture one propagation step (ks_state_propagate with nsteps = 1 and the
 * given dt, occ, rho) into a HIP graph owned by the state; stream must not be
 * the default stream and kernel timing must be off.  Replaces an earlier
 * capture.  ks_state_replay launches the captured step on any stream.
 * The graph holds the system's workspace and tables and its launch shapes:
 * after ks_system_set_projectors, ks_system_set_chunk, ks_system_set_tuning
 * or ks_autotune on the system, ks_state_replay returns KS_EINVAL until the
 * step is captured again.  The occ and rho buffers given at capture must
 * stay allocated while the graph is replayed (ks_system_set_vloc is fine:
 * replays read the current potential).
 */
ks_status ks_state_capture(ks_state* state, double dt, const double* occ, double* rho, void* stream);
ks_status ks_state_replay(ks_state* state, void* stream);

/* ------------------------------------------------------------------------
 * Batched steps (serving): resident states of several distinct systems of
 * one grid (same n, L, ecut and precision, hence one plane-wave sphere) are
 * propagated together, one launch per kernel and H psi for all of them.
 * States are independent (Section "Real-time propagation"), and every
 * orbital goes through the same arithmetic as in its own ks_state_propagate,
 * so the results are bit-identical to stepping each state alone.
 *
 * ks_batch_create: states[nstates] (host array), distinct systems of one
 * x-tile shape.  A state with more orbitals than its system's pass (chunk)
 * is stepped in passes, as alone: pass p steps chunk p (orbitals
 * [p chunk, (p+1) chunk)) of every state that has one, so a system's
 * workspace need only hold one chunk.  A pass whose launch rows (orbital
 * groups, or orbitals for the projection sums) exceed a grid's y extent of
 * 65535 is launched in slices of rows.  Allocates a small device table (from
 * the first system's pool when it has one).  KS_EINVAL (null, empty, systems
 * that differ in grid / cell / cutoff / precision / x-tile shape, two states
 * of one system).
 * The batch holds the systems' buffers: after ks_system_set_projectors,
 * set_chunk, set_tuning or autotune on any of them, the batch calls return
 * KS_EINVAL (create it again).  Destroy the batch before its states.
 */
typedef struct ks_batch ks_batch;
ks_status ks_batch_create(ks_state* const* states, int nstates, ks_batch** out);
/* Waits for the work of the batch's systems, frees the table. */
void ks_batch_destroy(ks_batch* batch);
/* nsteps Taylor-4 steps (as ks_state_propagate without density or norms) of
 * every state of the batch, on `stream`. */
ks_status ks_batch_propagate(ks_batch* batch, double dt, int nsteps, void* stream);
/* Capture one batched step into a graph owned by the batch (non-default
 * stream, kernel timing off); ks_batch_replay launches it on any stream. */
ks_status ks_batch_capture(ks_batch* batch, double dt, void* stream);
ks_status ks_batch_replay(ks_batch* batch, void* stream);
/* Message of the last failing batch call (or of a failed ks_batch_create on
 * NULL). */
const char* ks_batch_last_error(const ks_batch* batch);
/* One-shot form: create a batch of the states, nsteps steps, destroy it
 * (waits for the steps).  Errors as ks_batch_create / ks_batch_propagate;
 * the message is ks_batch_last_error(NULL). */
ks_status ks_propagate_batch(ks_state* const* states, int nstates, double dt, int nsteps, void* stream);

/*
 * Device bytes a system of this shape plus a resident state of norb orbitals
 * will hold (host-only estimate for admission control; npoints = projector
 * points, chunk = 0 for the default chunk; a chunk is capped at 65535 as
 * ks_system_create_ex caps it).  Counts the real-space
 * projections (ks_tuning.projection = 0); projection 1 adds its table and
 * partials (see ks_tuning).
 */
ks_status ks_plan_footprint(const int n[3], const double L[3], double ecut, int precision, int norb, int npoints,
                            int nproj, int chunk, unsigned long long* bytes);

/* Number of plane waves in the sphere (packed coefficients per orbital). */
int ks_system_npw(const ks_system* sys);

/* Largest number of orbitals processed per pass (chunk size of the internal
 * pipeline).  The default is min(max_norb, 65535, the count whose plane
 * intermediate takes 16 GiB).  A call over norb orbitals runs
 * ceil(norb / chunk) passes of equal size (up to one orbital). */
int ks_system_chunk(const ks_system* sys);

/* Set the chunk size (1 <= chunk <= min(max_norb, 65535)); reallocates the
 * workspace, so call it at set-up time only.  KS_EINVAL when out of range. */
ks_status ks_system_set_chunk(ks_system* sys, int chunk);

/* ------------------------------------------------------------------------
 * Host-only planning calls (no device needed).  They expose the set-up
 * tables so that their construction can be checked on any machine.
 */

/*
 * The packed plane-wave sphere of grid n[3], cell L[3] and cutoff ecut (same
 * rules as ks_system_create; ecut <= 0 = full box): *npw receives the number
 * of plane waves; m_out (host int [npw][3], nullable) the integer frequencies
 * (m0, m1, m2) in the library's packed order (planes m0 ascending, then m1,
 * then a contiguous run of m2).  KS_EINVAL on bad arguments.
 */
ks_status ks_plan_sphere(const int n[3], const double L[3], double ecut, int* npw, int* m_out);

/*
 * The Kleinman-Bylander point tables that ks_system_set_projectors builds for
 * grid n[3] (same arguments, host memory).  counts[4] receives (slots, unique
 * points, entries, runs).  Optional outputs (host, nullable):
 *   point_flat    [unique points]     flat grid index of each unique point
 *   point_entries [unique points + 1] entry range of each unique point
 *   entry_atom    [entries]           atom of each entry
 *   entry_row     [entries]           input row (index into idx/beta) of each entry
 * Call once with NULL outputs to size them.  Errors as for
 * ks_system_set_projectors.
 */
ks_status ks_plan_projectors(const int n[3], int natoms, int nproj, const int* npts, const int* idx,
                             const double* beta, int* counts, int* point_flat, int* point_entries,
                             int* entry_atom, int* entry_row);

/* ------------------------------------------------------------------------
 * Introspection and kernel timing (instrumentation; not on the hot path).
 */
typedef struct {
  int npw;          /* plane waves in the sphere (packed coefficients per orbital) */
  int nplanes;      /* m0 planes touched by the sphere */
  int ncols;        /* (m0, m1) columns touched by the sphere */
  int chunk;        /* orbitals per internal pass */
  int natoms;       /* atoms with at least one projector point */
  int nproj;        /* projectors per atom */
  int nruns;        /* runs of consecutive x-points of the projector spheres */
  int nslots;       /* (x-tile, atom) pairs touched by the projector spheres */
  int npoints;      /* projector points (sum of npts) */
  int x_tile;       /* x-pencils per block in the x-pencil passes */
  int precision;    /* ks_precision */
  int x_half;       /* 1 if every sphere plane has |m0| < n0/4: the x-synthesis loads and
                       transforms only the nonzero half of its first-stage inputs */
  int x_group;      /* largest orbital group of an x-pencil block (tuning) */
  int plane_group;  /* largest orbital group of a plane block (tuning) */
  int x_shape;      /* tile shape of the x-pencil passes (see ks_tuning) */
  int x_threads;    /* threads per block in the x-pencil passes */
  int projection;   /* how the KB projections are formed (see ks_tuning) */
} ks_info;

/* Fill *info for sys.  KS_EINVAL on null arguments. */
ks_status ks_system_info(const ks_system* sys, ks_info* info);

/* ------------------------------------------------------------------------
 * Launch-schedule autotuning (set-up time; not on the hot path).
 *
 * Each plane and x-pencil block loops over a group of orbitals; the group
 * caps trade the per-block set-up (twiddles, potential, KB tables, column
 * tables, loaded once per block) against the number of blocks that fill the
 * chip.  The results of H psi do not depend on them (every orbital is
 * transformed by the same arithmetic in the same order).  The x-tile shape
 * trades LDS per block against blocks per compute unit; every transform is
 * computed the same way in either shape, but the projections are summed per
 * (tile, atom) before they are added across tiles, so results of the two
 * shapes differ by rounding only.
 */
typedef struct {
  int x_group;       /* cap on orbitals per x-pencil block, 1..64 */
  int plane_group;   /* cap on orbitals per plane block, 1..64 */
  double ms;         /* measured time of one H psi pass over the tuned orbital count (0 if not measured) */
  int from_cache;    /* 1 if the result came from the process-wide cache */
  int x_shape;       /* launch shape of the x-pencil passes (tile and x-transform factorisation):
                        0 = 64 pencils x 256 threads for n0 <= 32, 32 x 256 above; 1 = 16 pencils x
                        192 threads (n0 = 96 and 120 only; fewer LDS bytes per block, more blocks
                        resident per compute unit); 2 and 3 = the tiles of 0 and 1 with the second
                        radix plan of the x-transform (n0 = 96 only: 8 x 12 instead of 12 x 8); -1 in
                        ks_system_set_tuning keeps the current shape */
  int projection;    /* KB projections P_Ip (Eq. vnl): 0 = sphere sums of the synthesised orbitals in the
                        x-pass (real space; every precision); 1 = KS_MIXED only: the same sums taken in
                        reciprocal space, P_Ip = sum_G c_G w_Ip(G) with w_Ip(G) = (Omega^1/2 / N) sum_j
                        beta_Ip(r_j) e^{iG.r_j} tabulated once per set of projectors (d_Ip folded in),
                        as a split-BF16 product on the
                        matrix cores (x = hi + lo, a b = hi hi + hi lo + lo hi, FP32 accumulation; about
                        1e-7 relative on the projections).  Mode 1 holds the table (4 bytes per plane
                        wave and projector, and FP32 split-K partials of at most 64 MiB for passes of up to
                        8192 orbitals and 4096 projectors); the density-fused
                        first sub-step of a propagation with densities keeps the real-space sums.
                        ks_autotune does not change it; -1 in ks_system_set_tuning keeps it */
} ks_tuning;

/* Time one H psi pass over min(norb, chunk) orbitals (zero coefficients; the
 * kernels' timing does not depend on the values) for each candidate of
 * x-pass shape (tile and radix plan) and group caps on `stream`, keep the
 * fastest (a shape later in the order 0..3 only when it is at least 1 % faster
 * than the best earlier one, so that near-ties do not flip between runs), and
 * return it in *out
 * (nullable).  A change of tile shape rebuilds the per-tile projector tables
 * from the inputs of the last ks_system_set_projectors.
 * Results are cached per process by (grid, precision, number of sphere
 * planes, orbitals per pass rounded up to a power of two): a later system of
 * the same shape takes the cached caps without timing.  Synchronises `stream`; overwrites the
 * system's internal workspace.  KS_EINVAL for norb outside [1, max_norb]. */
ks_status ks_autotune(ks_system* sys, int norb, void* stream, ks_tuning* out);

/* Set the group caps (x_group, plane_group in [1, 64]) and the tile shape
 * (x_shape: -1 keeps it; a shape the grid lacks is KS_EINVAL); ms and
 * from_cache are ignored.  A change of shape waits for the system's work and
 * rebuilds the projector tables (as ks_system_set_projectors does).  KS_EINVAL
 * otherwise. */
ks_status ks_system_set_tuning(ks_system* sys, const ks_tuning* t);

/* Kernel classes reported by ks_kernel_time. */
typedef enum {
  KS_K_PACK = 0, KS_K_UNPACK, KS_K_PLANE_INV, KS_K_XPROJ, KS_K_PROJ_REDUCE, KS_K_XAPPLY,
  KS_K_PLANE_FWD, KS_K_XDENS, KS_K_DOTS, KS_K_GEMM, KS_K_EIG, KS_K_SD, KS_K_GPROJ, KS_K_COUNT
} ks_kernel_id;

/*
 * enable != 0: record a HIP event pair around every kernel launch of sys on
 * the stream it is launched on, and reset the accumulated times; enable == 0:
 * stop recording.  Costs two event records per launch while on.
 */
ks_status ks_set_kernel_timing(ks_system* sys, int enable);

/*
 * Accumulated device time (ms) and launch count of one kernel class since
 * timing was enabled.  Synchronises the recorded events.  Either output may
 * be NULL.  KS_EINVAL for an unknown id.
 */
ks_status ks_kernel_time(ks_system* sys, int kernel_id, double* total_ms, long long* launches);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */
