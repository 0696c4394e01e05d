// Full-box transforms (HIP, gfx950): the periodic Hartree potential of a
// density, the field kick of the orbitals, and the dipole moment.
//
// Periodic Hartree potential of a density on the full FFT box:
// V_H(G) = 4 pi n(G) / |G|^2 for G != 0 and 0 at G = 0 (Section "Poisson
// solver", periodic boundary conditions), with n(G) = N^-1 sum_r n(r)
// e^{-iG.r} and V_H(r) = sum_G V_H(G) e^{+iG.r}.
//
// Five launches over a complex work box W [n0][n1][n2]:
//   z analysis (rows; the real density in), y analysis, x analysis + Poisson
//   kernel + x synthesis, y synthesis, z synthesis (real part out, plus V_loc
//   when given).  Nothing is pruned: the density fills the box.
#include <mutex>

#include "ks_common.hpp"

namespace ks {

constexpr int HNB = 32;   // transforms per block

// z (contiguous rows): block = HNB consecutive rows (j0, j1), staged in LDS
// with coalesced loads and stores.  SIGN -1: real density in, W out;
// SIGN +1: W in, Re(W) (+ vloc) out.
template <int N2, int SIGN>
__global__ __launch_bounds__(NT) void hz_kernel(const double* __restrict__ rho, double2* __restrict__ W,
                                                double* __restrict__ vout, const double* __restrict__ vloc,
                                                const double2* __restrict__ tw0, long long nrows) {
  __shared__ double2 X[HNB * (N2 + 1)];
  __shared__ double2 tw[N2];
  const int tid = threadIdx.x;
  for (int i = tid; i < N2; i += NT) tw[i] = tw0[i];
  const long long row0 = (long long)blockIdx.x * HNB;
  const int nr = (nrows - row0) < HNB ? (int)(nrows - row0) : HNB;
  const long long base = row0 * N2;
  for (int i = tid; i < nr * N2; i += NT) {
    const int r = i / N2, e = i - r * N2;
    X[r * (N2 + 1) + e] = (SIGN < 0) ? double2{rho[base + i], 0.0} : W[base + i];
  }
  __syncthreads();
  fft_batch<N2, SIGN, HNB, NT, double2>(X, N2 + 1, nr, tw);
  for (int i = tid; i < nr * N2; i += NT) {
    const int r = i / N2, e = i - r * N2;
    const double2 v = X[r * (N2 + 1) + e];
    if (SIGN < 0) W[base + i] = v;
    else vout[base + i] = v.x + (vloc ? vloc[base + i] : 0.0);
  }
}

// y: block = HNB consecutive j2 of one j0 plane; element (t, e) of the tile
// is W[(j0*N1 + e)*n2 + j2_0 + t] (coalesced over t); in place (every
// element is loaded in the first stage and stored in the last).
template <int N1, int SIGN>
__global__ __launch_bounds__(NT) void hy_kernel(double2* __restrict__ W, int n2, const double2* __restrict__ tw0) {
  __shared__ double2 X[HNB * (N1 + 1)];
  __shared__ double2 tw[N1];
  const int tid = threadIdx.x;
  for (int i = tid; i < N1; i += NT) tw[i] = tw0[i];
  const int tiles = (n2 + HNB - 1) / HNB;
  const int j0 = blockIdx.x / tiles, t0 = (blockIdx.x - j0 * tiles) * HNB;
  const int nt = n2 - t0 < HNB ? n2 - t0 : HNB;
  double2* base = W + (long long)j0 * N1 * n2 + t0;
  __syncthreads();
  fft_io<N1, SIGN, HNB, NT, SRC_FN, DST_FN, double2>(
      X, N1 + 1, nt, tw, [&](int t, int e) -> double2 { return base[(long long)e * n2 + t]; },
      [&](int t, int e, double2 v, int, int) { base[(long long)e * n2 + t] = v; });
}

// x: block = HNB consecutive pencils p = j1*n2 + j2; analysis, the Poisson
// kernel scale/|G|^2 (0 at G = 0) in LDS, synthesis; in place.
template <int N0>
__global__ __launch_bounds__(NT) void hx_kernel(double2* __restrict__ W, int n1, int n2, double g0, double g1,
                                                double g2, double scale, const double2* __restrict__ tw0) {
  __shared__ double2 X[HNB * (N0 + 1)];
  __shared__ double2 tw[N0];
  const int tid = threadIdx.x;
  for (int i = tid; i < N0; i += NT) tw[i] = tw0[i];
  const int npl = n1 * n2;
  const int p0 = blockIdx.x * HNB;
  const int nt = npl - p0 < HNB ? npl - p0 : HNB;
  double2* base = W + p0;
  __syncthreads();
  fft_io<N0, -1, HNB, NT, SRC_FN, DST_LDS, double2>(
      X, N0 + 1, nt, tw, [&](int t, int e) -> double2 { return base[(long long)e * npl + t]; }, no_store{});
  for (int i = tid; i < nt * N0; i += NT) {
    const int t = i / N0, e = i - t * N0;
    const int p = p0 + t, j1 = p / n2, j2 = p - j1 * n2;
    const double k0 = g0 * fold(e, N0), k1 = g1 * fold(j1, n1), k2 = g2 * fold(j2, n2);
    const double G2 = k0 * k0 + k1 * k1 + k2 * k2;
    const double f = G2 > 0.0 ? scale / G2 : 0.0;
    double2& x = X[t * (N0 + 1) + e];
    x = double2{x.x * f, x.y * f};
  }
  __syncthreads();
  fft_io<N0, +1, HNB, NT, SRC_LDS, DST_FN, double2>(
      X, N0 + 1, nt, tw, no_load{}, [&](int t, int e, double2 v, int, int) { base[(long long)e * npl + t] = v; });
}

// z rows of a complex box in place (rows staged in LDS, coalesced).
template <int N2, int SIGN>
__global__ __launch_bounds__(NT) void hzc_kernel(double2* __restrict__ W, const double2* __restrict__ tw0,
                                                 long long nrows) {
  __shared__ double2 X[HNB * (N2 + 1)];
  __shared__ double2 tw[N2];
  const int tid = threadIdx.x;
  for (int i = tid; i < N2; i += NT) tw[i] = tw0[i];
  const long long row0 = (long long)blockIdx.x * HNB;
  const int nr = (nrows - row0) < HNB ? (int)(nrows - row0) : HNB;
  double2* base = W + row0 * N2;
  for (int i = tid; i < nr * N2; i += NT) {
    const int r = i / N2, e = i - r * N2;
    X[r * (N2 + 1) + e] = base[i];
  }
  __syncthreads();
  fft_batch<N2, SIGN, HNB, NT, double2>(X, N2 + 1, nr, tw);
  for (int i = tid; i < nr * N2; i += NT) {
    const int r = i / N2, e = i - r * N2;
    base[i] = X[r * (N2 + 1) + e];
  }
}

// Field kick, x part: synthesis along x, then psi(r) *= exp(i k.r) / N with
// r = (j0 h0, j1 h1, j2 h2), then analysis along x; in place.  The y and z
// transforms around it complete the 3-D synthesis and analysis.
template <int N0>
__global__ __launch_bounds__(NT) void hx_kick_kernel(double2* __restrict__ W, int n1, int n2, double k0, double k1,
                                                     double k2, double h0, double h1, double h2, double scale,
                                                     const double2* __restrict__ tw0) {
  __shared__ double2 X[HNB * (N0 + 1)];
  __shared__ double2 tw[N0];
  const int tid = threadIdx.x;
  for (int i = tid; i < N0; i += NT) tw[i] = tw0[i];
  const int npl = n1 * n2;
  const int p0 = blockIdx.x * HNB;
  const int nt = npl - p0 < HNB ? npl - p0 : HNB;
  double2* base = W + p0;
  __syncthreads();
  fft_io<N0, +1, HNB, NT, SRC_FN, DST_LDS, double2>(
      X, N0 + 1, nt, tw, [&](int t, int e) -> double2 { return base[(long long)e * npl + t]; }, no_store{});
  for (int i = tid; i < nt * N0; i += NT) {
    const int t = i / N0, e = i - t * N0;
    const int p = p0 + t, j1 = p / n2, j2 = p - j1 * n2;
    const double th = k0 * (e * h0) + k1 * (j1 * h1) + k2 * (j2 * h2);
    double sn, cs;
    sincos(th, &sn, &cs);
    double2& x = X[t * (N0 + 1) + e];
    x = double2{scale * (x.x * cs - x.y * sn), scale * (x.x * sn + x.y * cs)};
  }
  __syncthreads();
  fft_io<N0, -1, HNB, NT, SRC_LDS, DST_FN, double2>(
      X, N0 + 1, nt, tw, no_load{}, [&](int t, int e, double2 v, int, int) { base[(long long)e * npl + t] = v; });
}

// Dipole moment: dV sum_r r_a rho(r).  Each block sums a contiguous range of
// points (fixed order within the block: per-thread strided sums, then a tree
// over the threads); dipole_sum adds the block partials in order.
constexpr int DIP_BLOCKS = 256;

__global__ __launch_bounds__(NT) void dipole_part_kernel(const double* __restrict__ rho, int n0, int n1, int n2,
                                                         double h0, double h1, double h2,
                                                         double* __restrict__ part) {
  __shared__ double red[3][NT];
  const long long N = (long long)n0 * n1 * n2;
  const long long per = (N + DIP_BLOCKS - 1) / DIP_BLOCKS;
  const long long a = blockIdx.x * per, b = a + per < N ? a + per : N;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (long long i = a + threadIdx.x; i < b; i += NT) {
    const long long j12 = i % ((long long)n1 * n2);
    const int j0 = (int)(i / ((long long)n1 * n2)), j1 = (int)(j12 / n2), j2 = (int)(j12 % n2);
    const double v = rho[i];
    sx += v * (j0 * h0);
    sy += v * (j1 * h1);
    sz += v * (j2 * h2);
  }
  red[0][threadIdx.x] = sx;
  red[1][threadIdx.x] = sy;
  red[2][threadIdx.x] = sz;
  __syncthreads();
  for (int m = NT / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void dipole_sum_kernel(const double* __restrict__ part, double dV, double* __restrict__ d) {
  const int c = threadIdx.x;
  if (c >= 3) return;
  double s = 0.0;
  for (int b = 0; b < DIP_BLOCKS; ++b) s += part[b * 3 + c];
  d[c] = dV * s;
}

// ------------------------------------------------------------------ launchers

template <int N1>
static void hartree_yz(const ks_system* s, const double* rho, double2* W, double* v, const double* vloc, int sign,
                       hipStream_t st) {
  const long long nrows = (long long)s->n[0] * s->n[1];
  const unsigned zblocks = (unsigned)((nrows + HNB - 1) / HNB);
  const unsigned yblocks = (unsigned)(s->n[0] * ((s->n[2] + HNB - 1) / HNB));
  if (sign < 0) {
    hz_kernel<N1, -1><<<zblocks, NT, 0, st>>>(rho, W, nullptr, nullptr, s->d_tw1, nrows);
    hy_kernel<N1, -1><<<yblocks, NT, 0, st>>>(W, s->n[2], s->d_tw1);
  } else {
    hy_kernel<N1, +1><<<yblocks, NT, 0, st>>>(W, s->n[2], s->d_tw1);
    hz_kernel<N1, +1><<<zblocks, NT, 0, st>>>(nullptr, W, v, vloc, s->d_tw1, nrows);
  }
}

template <int N0>
static void hartree_x(const ks_system* s, double2* W, hipStream_t st) {
  const int npl = s->n[1] * s->n[2];
  const double g0 = 2.0 * M_PI / s->L[0], g1 = 2.0 * M_PI / s->L[1], g2 = 2.0 * M_PI / s->L[2];
  hx_kernel<N0><<<(unsigned)((npl + HNB - 1) / HNB), NT, 0, st>>>(W, s->n[1], s->n[2], g0, g1, g2,
                                                                 4.0 * M_PI / (double)s->N, s->d_tw0);
}

static bool yz_pass(const ks_system* s, const double* rho, double2* W, double* v, const double* vloc, int sign,
                    hipStream_t st) {
  switch (s->n[1]) {
#define KS_CASE(c) case c: hartree_yz<c>(s, rho, W, v, vloc, sign, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

// ------------------------------------------ local-density exchange-correlation
// v_xc[n] of Eq. hamiltonian for the unpolarised gas: Slater exchange
// eps_x = -(3/4) (3 n / pi)^(1/3), v_x = (4/3) eps_x, and the Perdew-Zunger
// (1981) correlation fit in rs = (3 / (4 pi n))^(1/3),
//   rs >= 1: eps_c = gamma / q,  q = 1 + beta1 sqrt(rs) + beta2 rs,
//            v_c = eps_c (1 + 7/6 beta1 sqrt(rs) + 4/3 beta2 rs) / q
//   rs < 1:  v_c = A ln rs + (B - A/3) + 2/3 C rs ln rs + (2 D - C) rs / 3
// (v_c = eps_c - rs/3 d eps_c / d rs); zero where n <= 0.
__device__ __forceinline__ double lda_vxc(double n) {
  if (!(n > 0.0)) return 0.0;
  constexpr double GAMMA = -0.1423, BETA1 = 1.0529, BETA2 = 0.3334;
  constexpr double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
  const double ex = -0.75 * cbrt(3.0 * n / M_PI);
  const double vx = 4.0 / 3.0 * ex;
  const double rs = cbrt(3.0 / (4.0 * M_PI * n));
  double vc;
  if (rs >= 1.0) {
    const double sq = sqrt(rs);
    const double q = 1.0 + BETA1 * sq + BETA2 * rs;
    vc = GAMMA / q * (1.0 + 7.0 / 6.0 * BETA1 * sq + 4.0 / 3.0 * BETA2 * rs) / q;
  } else {
    const double lr = log(rs);
    vc = A * lr + (B - A / 3.0) + 2.0 / 3.0 * C * rs * lr + (2.0 * D - C) * rs / 3.0;
  }
  return vx + vc;
}

// v[i] (+)= v_xc(rho[i])
__global__ __launch_bounds__(NT) void lda_xc_kernel(const double* __restrict__ rho, double* __restrict__ v,
                                                    long long N, int accumulate) {
  const long long i = (long long)blockIdx.x * NT + threadIdx.x;
  if (i >= N) return;
  const double x = lda_vxc(rho[i]);
  v[i] = accumulate ? v[i] + x : x;
}

void launch_lda_xc(const ks_system* s, const double* rho, double* v, int accumulate, hipStream_t st) {
  lda_xc_kernel<<<(unsigned)((s->N + NT - 1) / NT), NT, 0, st>>>(rho, v, s->N, accumulate);
}

bool launch_hartree(const ks_system* s, const double* rho, double* v, const double* vloc, hipStream_t st) {
  double2* W = s->d_hbox;
  if (!yz_pass(s, rho, W, nullptr, nullptr, -1, st)) return false;
  switch (s->n[0]) {
#define KS_CASE(c) case c: hartree_x<c>(s, W, st); break;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
  return yz_pass(s, nullptr, W, v, vloc, +1, st);
}

}  // namespace ks

namespace ks {

template <int N1>
static void kick_yz(const ks_system* s, double2* W, int sign, hipStream_t st) {
  const long long nrows = (long long)s->n[0] * s->n[1];
  const unsigned zblocks = (unsigned)((nrows + HNB - 1) / HNB);
  const unsigned yblocks = (unsigned)(s->n[0] * ((s->n[2] + HNB - 1) / HNB));
  if (sign > 0) {
    hzc_kernel<N1, +1><<<zblocks, NT, 0, st>>>(W, s->d_tw1, nrows);
    hy_kernel<N1, +1><<<yblocks, NT, 0, st>>>(W, s->n[2], s->d_tw1);
  } else {
    hy_kernel<N1, -1><<<yblocks, NT, 0, st>>>(W, s->n[2], s->d_tw1);
    hzc_kernel<N1, -1><<<zblocks, NT, 0, st>>>(W, s->d_tw1, nrows);
  }
}

template <int N0>
static void kick_x(const ks_system* s, double2* W, const double k[3], hipStream_t st) {
  const int npl = s->n[1] * s->n[2];
  hx_kick_kernel<N0><<<(unsigned)((npl + HNB - 1) / HNB), NT, 0, st>>>(
      W, s->n[1], s->n[2], k[0], k[1], k[2], s->L[0] / s->n[0], s->L[1] / s->n[1], s->L[2] / s->n[2],
      1.0 / (double)s->N, s->d_tw0);
}

static bool kick_yz_pass(const ks_system* s, double2* W, int sign, hipStream_t st) {
  switch (s->n[1]) {
#define KS_CASE(c) case c: kick_yz<c>(s, W, sign, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

bool launch_kick(const ks_system* s, double2* W, const double k[3], hipStream_t st) {
  if (!kick_yz_pass(s, W, +1, st)) return false;
  switch (s->n[0]) {
#define KS_CASE(c) case c: kick_x<c>(s, W, k, st); break;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
  return kick_yz_pass(s, W, -1, st);
}

void launch_dipole_grid(const int n[3], const double L[3], const double* rho, double* part, double* d,
                        hipStream_t st) {
  const double dV = (L[0] * L[1] * L[2]) / ((double)n[0] * n[1] * n[2]);
  dipole_part_kernel<<<DIP_BLOCKS, NT, 0, st>>>(rho, n[0], n[1], n[2], L[0] / n[0], L[1] / n[1], L[2] / n[2], part);
  dipole_sum_kernel<<<1, 64, 0, st>>>(part, dV, d);
}

bool launch_dipole(const ks_system* s, const double* rho, double* d, hipStream_t st) {
  double* part = reinterpret_cast<double*>(s->d_hbox);   // 3 * DIP_BLOCKS doubles of the work box
  launch_dipole_grid(s->n, s->L, rho, part, d, st);
  return true;
}

// Partial sums of the allocation-free dipole (ks_dipole_noalloc): a fixed
// array in the library's device image, one copy per device, held until the
// process ends.  Host code never passes the array's name to a kernel: it
// takes the array's device address from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[DIPOLE_SCRATCH_DOUBLES];
static_assert(DIPOLE_SCRATCH_DOUBLES >= 3 * DIP_BLOCKS, "dipole partials exceed the static scratch");

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t dipole_scratch(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace ks
