// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ks.h"

struct ks_batch;

namespace ks {

// Plane-wave sphere in packed order: planes m0 = m0lo .. m0lo+nplanes-1, in
// each plane the columns m1 = m1lo(plane) .. , in each column the run of m2
// values m2lo(col) .. m2lo(col)+len-1 stored contiguously.
struct SphereTab {
  const int* plane_col0;  // [nplanes+1] first column id of each plane
  const int* plane_m1lo;  // [nplanes]
  const int* col_off;     // [ncols+1] packed offset of each column (col_off[ncols] = npw)
  const int* col_m2lo;    // [ncols]
  int nplanes, m0lo;
  int n0, n1, n2;
};

// Kleinman-Bylander projector tables, grouped per x-tile (NB consecutive
// x-pencils p = j1*n2 + j2).  Positions are LDS offsets w*(n0+1) + j0 in the
// tile's pencil buffer (w = p - tile*NB).
//  - slot:  one (tile, atom) pair; the points of a slot are contiguous rows
//           of beta, ordered (tile, atom, pencil, j0)
//  - unique point: one grid point of the tile touched by any sphere; its
//           entries (slot, beta row), ordered by atom, are the primary entry
//           (the first atom) stored with the point, and the extra entries of
//           points where spheres overlap, stored apart (scatter side)
struct ProjTab {
  const int* pt_lds;         // [npoints] LDS offset of each beta row's point
  const int* slot_off;       // [ntiles+1] slot range of each tile
  const int* slot_atom;      // [nslots]
  const int* slot_pt;        // [nslots+1] beta-row range of each slot
  const int* atom_slot_off;  // [natoms+1]
  const int* atom_slots;     // slots of each atom, ascending
  const int* up_off;         // [ntiles+1] unique-point range of each tile
  const int* up_key;         // [nunique] LDS offset | primary slot << 16 | extra entries << 24
  const int* up_x;           // [nunique] first extra entry of the point
  const double* up_beta;     // [nunique][nproj] beta row of the primary entry
  const int* x_slot;         // [nextra] tile-local slot of each extra entry
  const double* x_beta;      // [nextra][nproj]
  const double* beta;        // [npoints][nproj], rows in slot order
  const double* d;           // [natoms][nproj]
  const int4* item;          // [ntiles][threads per x-block] projection work of each lane (see build_proj)
  int natoms, nproj, nslots;
};

// One system of a batched launch (several systems of one grid, hence one
// sphere and one tiling, in one launch of each H psi kernel): its buffers
// and projector tables.  Block row y of a batched launch belongs to job
// rows[y].x, orbital group rows[y].y of rows[y].z (proj_reduce: orbital
// rows[y].y).
struct BatchJob {
  const void* win;    // packed input orbitals of the H psi (plane synthesis; kinetic term)
  void* wout;         // packed H psi (working precision), or null
  double2* acc;       // Taylor accumulator (the FP64 state)
  void* T;            // plane intermediates
  void* U;
  void* partial;      // projection partial sums
  double2* DP;        // KB coefficients times projections
  const double* V;    // local potential
  ProjTab pt;
  int nb;             // orbitals
};

// Reciprocal-space projection table of the mixed-precision path (k_gproj.hip):
// W_Ip(G) of the P = natoms * nproj projectors in real form, split into BF16
// hi and lo parts, [ncol][kpad / 8][16] (per column and group of 8 k: 8 hi,
// then 8 lo), ncol = 2 * P rounded up to a multiple of 128 columns, kpad =
// 2 * npw rounded up to a multiple of 32; and the split-K partial products.
struct GTab {
  __bf16* w = nullptr;
  float* part = nullptr;
  size_t part_bytes = 0;
  int ncol = 0, kpad = 0, P = 0;
};

// up_key fields
constexpr int UP_POS_BITS = 16, UP_SLOT_BITS = 8;
constexpr int UP_MAX_SLOT = (1 << UP_SLOT_BITS) - 1, UP_MAX_EXTRA = 127;

constexpr int KB_MAX_NPROJ = 8;        // projectors per atom
constexpr size_t GEMM_PART_MAX = 256ull << 20;    // largest split-K partial buffer of the n x n products
constexpr int KB_TILE_DP = 128;        // (slot, projector) pairs staged per x-tile
constexpr int KB_CACHED_POINTS = 16;   // points of an item held in registers across orbitals
constexpr int KB_MAX_GROUP_LOG = 4;    // at most 16 lanes per (slot, projector) pair
// Largest y extent of a launch grid.  The pass kernels put the orbitals of a
// pass (or their groups, or the rows of a batch) on it, so a pass holds at
// most this many orbitals and batched launches are issued in slices of rows.
constexpr int KS_MAX_GRID_Y = 65535;

enum HMode { H_OUT = 0, H_TAYLOR = 1 };

struct Taylor {
  double2 coef;   // (-i dt)^k / k!
  int write_w;    // store w_k = H w_{k-1}
  double2 coef2;  // coefficient of the second accumulator (when one is given)
};

}  // namespace ks

// Device memory pool (ks_pool_create): one device allocation, sub-allocated
// on the host (first fit, 256-byte aligned, neighbouring free ranges merged).
struct ks_pool {
  char* base = nullptr;
  size_t bytes = 0, used = 0, peak = 0;
  int device = 0;
  std::map<size_t, size_t> free_ranges;   // offset -> size
  std::map<size_t, size_t> live;          // offset -> size
  std::vector<ks_system*> systems;        // systems created in the pool (released if the pool goes first)
  std::mutex mu;
};

struct ks_system {
  int n[3];
  double L[3];
  double ecut;
  int prec;
  int max_norb;
  long long N;
  int npl;  // n1*n2
  double omega, dV;

  // sphere
  int nplanes = 0, m0lo = 0, ncols = 0, npw = 0, npw_stride = 0, ncol_max = 0;
  int npp_max = 0;   // largest number of packed coefficients in one m0 plane
  int* d_plane_col0 = nullptr;
  int* d_plane_m1lo = nullptr;
  int* d_col_off = nullptr;
  int* d_col_m2lo = nullptr;
  double2* d_tw0 = nullptr;
  double2* d_tw1 = nullptr;
  float2* d_tw0f = nullptr;
  float2* d_tw1f = nullptr;

  // local potential: d_v is the potential the Hamiltonian applies (V_loc,
  // or V_loc + V_H[n] inside a density-dependent propagation), d_vloc the
  // static V_loc
  double* d_v = nullptr;
  double* d_vloc = nullptr;
  double* d_kin = nullptr;   // |G|^2/2 of each packed coefficient [npw]
  bool have_v = false;
  // Hartree solve: complex work box [n0][n1][n2] and a density [n0][n1][n2]
  double2* d_hbox = nullptr;
  double* d_rho_w = nullptr;

  // projectors
  int natoms = 0, nproj = 0, nslots = 0, nruns = 0, npoints = 0, nuniq = 0;
  // x-tile shape (see x_shape_nb / x_shape_threads): pencils per tile and
  // threads per block of the x-pencil passes
  int xshape = 0, xnb = 32, xnt = 256, ntiles = 0;
  bool x_half = false;   // every sphere plane has |m0| < n0/4 (band-limited x-synthesis input)
  bool yz_half = false;  // every sphere point has |m1| < n1/4 and |m2| < n2/4 (band-limited y, z transforms)
  int xg_max = 8, pg_max = 8;   // orbital-group caps of the x-pencil and plane passes (tunable)
  int xc = 0;                   // exchange-correlation term of the density-dependent potential (ks_xc)
  // projections: 0 = summed in the x-pass from the synthesised orbitals
  // (real space), 1 = the reciprocal-space split-BF16 product with the table
  // gp (mixed precision; ks_tuning.projection)
  int proj_mode = 0;
  int *d_pt_lds = nullptr, *d_slot_off = nullptr, *d_slot_atom = nullptr, *d_slot_pt = nullptr,
      *d_atom_slot_off = nullptr, *d_atom_slots = nullptr, *d_up_off = nullptr, *d_up_key = nullptr,
      *d_up_x = nullptr, *d_x_slot = nullptr;
  double *d_beta = nullptr, *d_up_beta = nullptr, *d_x_beta = nullptr, *d_kb = nullptr;
  int4* d_item = nullptr;
  ks::GTab gp;
  // the projector inputs as last set, kept so the per-tile tables can be
  // rebuilt for another tile shape
  struct {
    int natoms = 0, nproj = 0;
    std::vector<int> npts, idx;
    std::vector<double> beta, d;
  } proj_in;

  // workspace (one chunk of cb orbitals)
  int cb = 1;
  void* pk[3] = {nullptr, nullptr, nullptr};  // packed chunk buffers
  void* T = nullptr;                          // [cb][nplanes][n1*n2]
  void* U = nullptr;
  void* partial = nullptr;                    // [cb][nslots][nproj]
  double2* DP = nullptr;                      // [cb][natoms][nproj]
  double* red = nullptr;                      // [2*max_norb]
  double* dens_part = nullptr;                // [ceil(cb/8)][N] partial densities
  size_t partial_cap = 0, dp_cap = 0;

  // orthonormalisation workspace (allocated on first use)
  void* ortho_pk = nullptr;
  double2* ortho_S = nullptr;
  double2* ortho_W = nullptr;
  int* ortho_info = nullptr;
  double* ortho_diag = nullptr;
  double2* gemm_part = nullptr;   // split-K partials of the n x n products (gemm_part_bytes)
  size_t gemm_part_bytes = 0;
  int ortho_cap = 0;

  // kernel timing (ks_set_kernel_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev;       // pairs
  std::vector<int> ev_kid;          // kernel class of each pair
  int ev_used = 0;
  double kt_ms[16] = {0};
  long long kt_n[16] = {0};

  std::string err;

  // device memory source (nullptr: hipMalloc / hipFree per buffer)
  ks_pool* pool = nullptr;
  bool pool_lost = false;   // the pool was destroyed first: buffers are gone, frees do nothing
  // recorded on the stream of every call that enqueues work (outside stream
  // capture): destroying the system or one of its states waits for it
  // instead of the whole device
  hipEvent_t done = nullptr;
  // bumped whenever buffers or launch shapes that a captured graph holds change
  unsigned long long gen = 0;
  // live states and batches of the system: destroying the system releases
  // their device memory and leaves them as empty handles, so handles may be
  // destroyed in any order
  std::vector<ks_state*> states;
  std::vector<ks_batch*> batches;
};

// Orbitals kept resident on the device in the packed FP64 layout.
struct ks_state {
  ks_system* sys = nullptr;
  int norb = 0;
  double2* data = nullptr;     // [norb][npw_stride]
  double2* aux = nullptr;      // [norb][npw_stride] ETRS predictor / eigensolver work (allocated on first use)
  // eigensolver work (allocated on first use): two more orbital blocks, the
  // Rayleigh-Ritz matrix, its eigenvectors and the Jacobi work (2 norb^2 +
  // bj_work_elems(norb) entries), and [2*norb + 2 + 2*bj_order(norb)]
  // doubles (Ritz values, residual norms, off-diagonal norm, its row partials)
  double2* gs_buf[2] = {nullptr, nullptr};
  double2* gs_mat = nullptr;
  double* gs_vec = nullptr;
  hipGraph_t graph = nullptr;  // one captured propagation step
  hipGraphExec_t exec = nullptr;
  unsigned long long graph_gen = 0;   // system generation at capture
};

// One pass of a batch: the chunk p (orbitals [p cb, (p+1) cb)) of every
// state that has one, stepped by one launch per kernel.
struct ks_batch_pass {
  ks::BatchJob* jobs[4] = {nullptr, nullptr, nullptr, nullptr};   // the 4 Taylor sub-steps
  int4* rows_x = nullptr;                 // x-pass rows (job, group, groups)
  int4* rows_p = nullptr;                 // plane-pass rows
  int4* rows_r = nullptr;                 // projection-reduce rows (job, orbital)
  int nrows_x = 0, nrows_p = 0, nrows_r = 0, max_natoms = 0;
};

// Several resident states of distinct systems of one grid, stepped together
// by one launch per H psi kernel and pass (ks_batch_create).
struct ks_batch {
  std::vector<ks_state*> states;
  std::vector<unsigned long long> gens;   // each system's generation at creation
  ks_system* s0 = nullptr;                // the first system: sphere, twiddles, precision, caps
  char* dev = nullptr;                    // device tables (jobs and rows of every pass)
  size_t dev_bytes = 0;
  std::vector<ks_batch_pass> passes;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace ks {

// launchers (ks_kernels.hip); return false when the size has no kernel
bool launch_pack(const ks_system* s, int nb, const double2* box, long long box_stride, void* pk,
                 hipStream_t st);
bool launch_unpack(const ks_system* s, int nb, const void* pk, bool pk_fp64, double2* box, long long box_stride,
                   hipStream_t st);
bool launch_plane_inv(const ks_system* s, int nb, const void* pk, bool in_fp64, void* T, hipStream_t st);
// with rho: also the density of the synthesised orbitals (occ), written or
// added (accumulate) to rho
bool launch_xproj(const ks_system* s, int nb, const void* T, void* partial, const double* occ, double* rho,
                  int accumulate, hipStream_t st);
bool launch_proj_reduce(const ks_system* s, int nb, const void* partial, double2* DP, hipStream_t st);
bool launch_xapply(const ks_system* s, int nb, const void* T, const double2* DP, void* U, hipStream_t st);
bool launch_plane_fwd(const ks_system* s, int nb, const void* U, const void* win, bool win_fp64, void* wout,
                      void* acc, void* acc2, HMode mode, Taylor tay, hipStream_t st);
bool launch_xdens(const ks_system* s, int nb, const void* T, const double* occ, double* rho, int accumulate,
                  hipStream_t st);
// Batched launches over several systems of s's grid (s supplies the sphere,
// twiddles, precision and launch caps); jobs and rows in device memory, see
// BatchJob.  x-passes: rows of orbital groups (apply = false: projections,
// true: local potential, scatter and analysis); proj_reduce: one row per
// (job, orbital) and max_natoms blocks per row; plane passes: rows of orbital
// groups, Taylor mode with the jobs' acc and wout.
bool launch_plane_inv_batch(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, bool in_fp64,
                            hipStream_t st);
bool launch_x_batch(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, bool apply, hipStream_t st);
bool launch_proj_reduce_batch(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, int max_natoms,
                              hipStream_t st);
bool launch_plane_fwd_batch(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, bool win_fp64,
                            Taylor tay, hipStream_t st);
// orbitals per block of the x-pencil and plane passes for a launch over
// total_orbitals orbitals (the same rule as the single-system launches)
int x_group_size(const ks_system* s, long long total_orbitals);
int plane_group_size(const ks_system* s, long long total_orbitals);
bool launch_dots(const ks_system* s, int nb, const void* a, const void* b, double* out, hipStream_t st);
bool launch_energy_sum(int norb, const double* occ, const double* red, double* energy, hipStream_t st);
// part: split-K partial products (part_bytes of them; NULL: no split)
bool launch_overlap(int norb, int npw, const double2* P, int ldp, double2* S, double2* part, size_t part_bytes,
                    hipStream_t st);
// bytes of split-K partials the products of up to n orbitals over K use
size_t gemm_part_bytes(int n, int K);
// S = L L^H in place (lower); the inverses of L's diagonal blocks go to the
// same blocks of X
bool launch_cholesky(int n, double2* S, double2* X, double* diag0, int* info, hipStream_t st);
// X = L^-1 (lower, upper triangle zero), given the diagonal blocks from launch_cholesky
bool launch_trtri(int n, const double2* L, double2* X, hipStream_t st);
bool launch_apply_lower(int norb, int npw, const double2* X, const double2* P, int ldp, double2* Y, hipStream_t st);

// reciprocal-space projections (k_gproj.hip): k-chunks of a product over nb
// orbitals, the partial-product bytes of passes of up to cb orbitals, the
// table W (zeroed by the caller) from the projector inputs (pt_off
// [natoms+1] point offsets, idx, beta [points][np], d [natoms][np], all in
// device memory), and DP [nb][natoms][nproj] from the packed orbitals win
bool launch_gproj_table(const ks_system* s, const int* pt_off, const int* idx, const double* beta, const double* d,
                        int natoms, int np, __bf16* W, int kpad, hipStream_t st);
int gproj_splits(int nb, int ncol, int ksteps);
size_t gproj_part_bytes(int cb, int ncol, int ksteps);
bool launch_gproj(const ks_system* s, int nb, const void* win, bool win_fp64, double2* DP, hipStream_t st);

// v = V_H[rho] (+ vloc when not null); uses the system's work box
bool launch_hartree(const ks_system* s, const double* rho, double* v, const double* vloc, hipStream_t st);
// v (+)= v_xc[rho] in the local-density form (N points of the system's box)
void launch_lda_xc(const ks_system* s, const double* rho, double* v, int accumulate, hipStream_t st);

// psi <- chi exp(i k.r) psi for one orbital held on the complex box W (in place)
bool launch_kick(const ks_system* s, double2* W, const double k[3], hipStream_t st);
// absorption spectrum of a dipole series (see k_response.hip); k: host, |k| > 0
void launch_spectrum(const double* d, int nt, double dt, const double k[3], const double* omegas, int nw,
                     double eta, double2* alpha, double* strength, hipStream_t st);
// d[0..2] = dV sum_r r rho(r) (device output; uses the work box for partial sums)
bool launch_dipole(const ks_system* s, const double* rho, double* d, hipStream_t st);
// the same on grid n, cell L, with the partial sums in part (DIPOLE_SCRATCH_DOUBLES)
void launch_dipole_grid(const int n[3], const double L[3], const double* rho, double* part, double* d,
                        hipStream_t st);
// doubles of the static scratch of the allocation-free dipole
constexpr int DIPOLE_SCRATCH_DOUBLES = 3 * 256;
// device address of the static dipole scratch on the current device (looked
// up once per device)
hipError_t dipole_scratch(double** out);

// dense complex products for the eigensolver (MFMA FP64):
// S[i][j] = sum_e conj(A[i][e]) B[j][e]   (norb x norb, rows of length npw)
bool launch_gemm_ch(int norb, int npw, const double2* A, int lda, const double2* B, int ldb, double2* S, double2* part,
                    size_t part_bytes, hipStream_t st);
// Y[i][e] = sum_j Q[i][j] X[j][e]   (Q row-major norb x norb)
bool launch_rotate(int norb, int npw, const double2* Q, const double2* X, int ldx, double2* Y, int ldy, hipStream_t st);

// subspace eigenproblem (k_ground.hip), blocked Jacobi on the matrix padded
// to order bj_order(n): A = (H + H^H)/2 (padded with zeros) and Vt = I; one
// round t (An, Vn from A, Vt; Ublk: the round's block unitaries); out =
// {off-diagonal |A|^2, |A|^2} over the padded order (per-row partials in
// part, 2 per row); eigenvalues ascending
// and eigenvectors as the rows of Q (n x n), phase-fixed.  Work elements:
// bj_work_elems(n) (A, An, Vt, Vn, Ublk).
int bj_order(int n);
size_t bj_work_elems(int n);
int bj_rounds(int n);
void launch_hermitize(int n, const double2* H, double2* A, double2* Vt, hipStream_t st);
void launch_bj_round(int n, const double2* A, double2* An, const double2* Vt, double2* Vn, double2* Ublk, int t,
                     hipStream_t st);
void launch_offdiag(int n, const double2* A, double* part /*2n*/, double* out, hipStream_t st);
void launch_eig_finish(int n, const double2* A, const double2* Vt, double* eig, double2* Q, hipStream_t st);
// steepest-descent steps over norb packed orbitals (one block per orbital)
void launch_sd_direction(int norb, int npw, int stride, const double2* C, const double2* W, const double* e,
                         const double* kin, double2* Qd, double* resid, hipStream_t st);
void launch_sd_update(int norb, int npw, int stride, double2* C, const double2* Qd, const double2* HQ, const double* e,
                      hipStream_t st);

bool supported_size(int n);
int x_tile_nb(int n0);
bool x_shape_available(int n0, int shape);
int x_shape_nb(int n0, int shape);
int x_shape_threads(int shape);
size_t plane_lds_bytes(const ks_system* s);

// kernel-side views of a system's sphere and projector tables
inline SphereTab sphere_tab(const ks_system* s) {

  SphereTab t;
  t.plane_col0 = s->d_plane_col0;
  t.plane_m1lo = s->d_plane_m1lo;
  t.col_off = s->d_col_off;
  t.col_m2lo = s->d_col_m2lo;
  t.nplanes = s->nplanes;
  t.m0lo = s->m0lo;
  t.n0 = s->n[0];
  t.n1 = s->n[1];
  t.n2 = s->n[2];
  return t;
}

inline ProjTab proj_tab(const ks_system* s) {
  ProjTab c;
  c.pt_lds = s->d_pt_lds;
  c.slot_off = s->d_slot_off;
  c.slot_atom = s->d_slot_atom;
  c.slot_pt = s->d_slot_pt;
  c.atom_slot_off = s->d_atom_slot_off;
  c.atom_slots = s->d_atom_slots;
  c.up_off = s->d_up_off;
  c.up_key = s->d_up_key;
  c.up_x = s->d_up_x;
  c.up_beta = s->d_up_beta;
  c.x_slot = s->d_x_slot;
  c.x_beta = s->d_x_beta;
  c.beta = s->d_beta;
  c.d = s->d_kb;
  c.item = s->d_item;
  c.natoms = s->natoms;
  c.nproj = s->nproj;
  c.nslots = s->nslots;
  return c;
}

}  // namespace ks
