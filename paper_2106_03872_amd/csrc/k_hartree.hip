// Periodic Hartree potential of a density on the full FFT box (HIP, gfx950):
// V_H(G) = 4 pi n(G) / |G|^2 for G != 0 and 0 at G = 0 (Section "Poisson
// solver", periodic boundary conditions), with n(G) = N^-1 sum_r n(r)
// e^{-iG.r} and V_H(r) = sum_G V_H(G) e^{+iG.r}.
//
// Five launches over a complex work box W [n0][n1][n2]:
//   z analysis (rows; the real density in), y analysis, x analysis + Poisson
//   kernel + x synthesis, y synthesis, z synthesis (real part out, plus V_loc
//   when given).  Nothing is pruned: the density fills the box.
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

// ------------------------------------------------------------------ launcher

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
