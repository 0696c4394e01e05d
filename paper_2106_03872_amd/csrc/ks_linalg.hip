// Dense complex FP64 linear algebra for the orthonormalisation of the
// orbitals (orthogonalisation step of Section "Ground-state solution"):
//   S = C^H C  (overlap over the packed plane-wave sphere, MFMA FP64)
//   S = L L^H  (blocked right-looking Cholesky)
//   X = L^-1   (blocked triangular inverse)
//   C <- conj(X) C  (rows = orbitals), i.e. Psi <- Psi L^-H  (MFMA FP64)
// The matrices are small (n = orbitals <= a few thousand); the two GEMMs are
// the only large contractions and run on the matrix cores.
#include <algorithm>

#include "ks_internal.h"

namespace ks {

typedef double dvec4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ MFMA GEMM
// Cout[m][n] = sum_k op(A)[m][k] * B(k, n) for complex FP64, op = conj when
// CONJ_A.  A is row-major [M][lda] (k contiguous).  B is either [N][ldb] with
// k contiguous (B_KN = false: B(k, n) = Bm[n][k]) or [K][ldb] with n
// contiguous (B_KN = true).  LOWER_A: A is lower triangular (k <= m), so
// k-tiles above the diagonal are skipped.  LOWER_OUT: only tiles with
// m-tile >= n-tile are produced.
//
// Split K: chunk z sums k in [z kchunk, (z+1) kchunk) (kchunk a multiple of
// GBK) into Cout + z * cstride; a fixed-order sum over z
// (sum_partials_kernel) completes the product.
//
// Block order (one-dimensional grid of mt * nt * nz tiles, rounded up to a
// multiple of XCDS): the hardware hands workgroup w to XCD w mod XCDS, so
// logical tile l = (w mod XCDS) * G/XCDS + w / XCDS gives each XCD a
// contiguous run of logical tiles, and the logical order puts tiles that
// read the same operand next to each other, so that its L2 serves the
// repeats: with B_KN, the m-tiles of one n-tile (which share B's column
// block); otherwise the tiles of one K chunk (which share that chunk of A
// and B).
//
// v_mfma_f64_16x16x4_f64 operand layout on gfx950 (64 lanes, measured):
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane
// j + 16 (i mod 4), element i div 4 of the 4-double accumulator.
constexpr int GBM = 64, GBN = 64, GBK = 16;
constexpr int XCDS = 8;   // accelerator dies (each with its own L2)

template <bool CONJ_A, bool B_KN, bool LOWER_A, bool LOWER_OUT>
__global__ __launch_bounds__(256) void zgemm_mfma_kernel(int M, int N, int K, const double2* __restrict__ A, long long lda,
                                                         const double2* __restrict__ Bm, long long ldb,
                                                         double2* __restrict__ Cout, long long ldc, int kchunk,
                                                         long long cstride) {
  __shared__ double2 As[GBK][GBM + 1];
  __shared__ double2 Bs[GBK][GBN + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int mt = (M + GBM - 1) / GBM, nt = (N + GBN - 1) / GBN;
  const int nz = (K + kchunk - 1) / kchunk;
  const long long tiles = (long long)mt * nt * nz;
  const long long per = gridDim.x / XCDS;
  const long long l = (long long)(blockIdx.x % XCDS) * per + blockIdx.x / XCDS;
  if (l >= tiles) return;
  int mi, ni, z;
  if (B_KN) {
    mi = (int)(l % mt);
    ni = (int)((l / mt) % nt);
    z = (int)(l / ((long long)mt * nt));
  } else {
    ni = (int)(l % nt);
    mi = (int)((l / nt) % mt);
    z = (int)(l / ((long long)mt * nt));
  }
  const int m0 = mi * GBM, n0 = ni * GBN;
  if (LOWER_OUT && n0 > m0) return;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  dvec4 re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = dvec4{0.0, 0.0, 0.0, 0.0};
  const int kbeg = z * kchunk;
  const int kend = LOWER_A ? min(min(K, kbeg + kchunk), m0 + GBM) : min(K, kbeg + kchunk);
  Cout += z * cstride;
  const double sa = CONJ_A ? -1.0 : 1.0;
  // The next k-tile is loaded into registers while the current one is
  // multiplied from LDS.  A tile: 64 rows x 16 k, k fastest across threads.
  constexpr int PT = GBM * GBK / 256;
  static_assert(GBN * GBK / 256 == PT, "equal A and B tile shares");
  double2 ra[PT], rb[PT];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int i = tid + j * 256;
      {
        const int kk = i % GBK, mm = i / GBK;
        const int m = m0 + mm, k = k0 + kk;
        ra[j] = (m < M && k < K) ? A[(long long)m * lda + k] : double2{0.0, 0.0};
      }
      if (B_KN) {
        const int nn = i % GBN, kk = i / GBN;
        const int n = n0 + nn, k = k0 + kk;
        rb[j] = (n < N && k < K) ? Bm[(long long)k * ldb + n] : double2{0.0, 0.0};
      } else {
        const int kk = i % GBK, nn = i / GBK;
        const int n = n0 + nn, k = k0 + kk;
        rb[j] = (n < N && k < K) ? Bm[(long long)n * ldb + k] : double2{0.0, 0.0};
      }
    }
  };
  if (kbeg < kend) load_tile(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int i = tid + j * 256;
      As[i % GBK][i / GBK] = ra[j];
      if (B_KN) Bs[i / GBN][i % GBN] = rb[j];
      else Bs[i % GBK][i / GBK] = rb[j];
    }
    __syncthreads();
    if (k0 + GBK < kend) load_tile(k0 + GBK);
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 4) {
      const int kr = ks + (lane >> 4), c = lane & 15;
      double2 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[kr][wm + t * 16 + c];
        b[t] = Bs[kr][wn + t * 16 + c];
      }
#pragma unroll
      for (int ta = 0; ta < 2; ++ta) {
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
          re[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, b[tb].x, re[ta][tb], 0, 0, 0);
          re[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-sa * a[ta].y, b[tb].y, re[ta][tb], 0, 0, 0);
          im[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, b[tb].y, im[ta][tb], 0, 0, 0);
          im[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa * a[ta].y, b[tb].x, im[ta][tb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int ta = 0; ta < 2; ++ta) {
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + ta * 16 + 4 * r + (lane >> 4);
        const int n = n0 + wn + tb * 16 + (lane & 15);
        if (m < M && n < N) Cout[(long long)m * ldc + n] = double2{re[ta][tb][r], im[ta][tb][r]};
      }
    }
  }
}

// ------------------------------------------------------------ blocked Cholesky
constexpr int CB = 32;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ double2 zmulc(double2 a, double2 b) { return double2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }

constexpr int CH_NT = 256;

// Factor the diagonal block at k0 in place (lower, upper part zeroed) and
// write the inverse of the factor into the same block of X; a pivot at or
// below 1e-12 of the original diagonal entry sets *info (the orbitals are
// numerically linearly dependent).
__global__ __launch_bounds__(CH_NT) void potrf_diag_kernel(double2* S, double2* X, int n, int k0,
                                                           const double* __restrict__ diag0, int* info) {
  __shared__ double2 a[CB][CB + 1];
  __shared__ double2 x[CB][CB + 1];
  __shared__ double rd[CB];
  const int tid = threadIdx.x;
  const int nb = min(CB, n - k0);
  for (int i = tid; i < CB * CB; i += CH_NT) {
    const int r = i / CB, c = i % CB;
    a[r][c] = (r < nb && c < nb && c <= r) ? S[(long long)(k0 + r) * n + k0 + c] : double2{0.0, 0.0};
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      double d = a[j][j].x;
      if (!(d > 1e-12 * diag0[k0 + j])) {
        info[0] = 1;
        d = 1.0;
      }
      const double sd = sqrt(d);
      a[j][j] = double2{sd, 0.0};
      rd[j] = 1.0 / sd;
    }
    __syncthreads();
    const double inv = rd[j];
    for (int i = j + 1 + tid; i < nb; i += CH_NT) a[i][j] = double2{a[i][j].x * inv, a[i][j].y * inv};
    __syncthreads();
    for (int t = tid; t < CB * CB; t += CH_NT) {
      const int r = t / CB, c = t % CB;
      if (c > j && r >= c && r < nb) {
        const double2 u = zmulc(a[r][j], a[c][j]);
        a[r][c] = double2{a[r][c].x - u.x, a[r][c].y - u.y};
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < nb * nb; i += CH_NT) {
    const int r = i / nb, c = i % nb;
    S[(long long)(k0 + r) * n + k0 + c] = c <= r ? a[r][c] : double2{0.0, 0.0};
  }
  // inverse of the factor by forward substitution, column c by the eight
  // lanes 8c .. 8c+7 of one wave: row r of column c is
  //   x[r][c] = (delta_rc - sum_{c <= q < r} a[r][q] x[q][c]) / a[r][r],
  // the sum split over the lanes by q mod 8 and added by a fixed butterfly
  const int c = tid >> 3, part = tid & 7;
  for (int r = 0; r < nb; ++r) {
    double sx = 0.0, sy = 0.0;
    for (int q = c + part; q < r; q += 8) {
      const double2 u = zmul(a[r][q], x[q][c]);
      sx += u.x;
      sy += u.y;
    }
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
      sx += __shfl_xor(sx, m, 64);
      sy += __shfl_xor(sy, m, 64);
    }
    if (part == 0 && c < nb)
      x[r][c] = r < c ? double2{0.0, 0.0} : double2{((r == c ? 1.0 : 0.0) - sx) * rd[r], -sy * rd[r]};
  }
  __syncthreads();
  for (int i = tid; i < nb * nb; i += CH_NT) {
    const int r = i / nb, cc = i % nb;
    X[(long long)(k0 + r) * n + k0 + cc] = x[r][cc];
  }
}

// Rows below the diagonal block: L_rk = A_rk L_kk^-H, a product with the
// inverted diagonal block (Xkk = L_kk^-1, lower):
//   L_rk[r][c] = sum_{q <= c} A_rk[r][q] conj(Xkk[c][q]).
// Block of 64 rows; thread (column c, rows r0 + 8 s).
__global__ __launch_bounds__(256) void trsm_panel_kernel(double2* S, const double2* __restrict__ X, int n, int k0) {
  __shared__ double2 xk[CB][CB + 1];
  __shared__ double2 ar[64][CB + 1];
  const int nb = min(CB, n - k0);
  const int tid = threadIdx.x;
  const int rb = k0 + nb + blockIdx.x * 64;
  for (int i = tid; i < CB * CB; i += 256) {
    const int r = i / CB, c = i % CB;
    xk[r][c] = (r < nb && c < nb) ? X[(long long)(k0 + r) * n + k0 + c] : double2{0.0, 0.0};
  }
  for (int i = tid; i < 64 * CB; i += 256) {
    const int r = i / CB, c = i % CB;
    ar[r][c] = (rb + r < n && c < nb) ? S[(long long)(rb + r) * n + k0 + c] : double2{0.0, 0.0};
  }
  __syncthreads();
  const int c = tid % CB, r0 = tid / CB;
  double2 acc[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) acc[s] = double2{0.0, 0.0};
  for (int q = 0; q <= c; ++q) {
    const double2 xv = xk[c][q];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const double2 u = zmulc(ar[r0 + 8 * s][q], xv);
      acc[s].x += u.x;
      acc[s].y += u.y;
    }
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int r = r0 + 8 * s;
    if (rb + r < n && c < nb) S[(long long)(rb + r) * n + k0 + c] = acc[s];
  }
}

// trailing update of the lower triangle: A_ij -= L_ik L_jk^H for tiles i >= j > k
__global__ __launch_bounds__(256) void herk_update_kernel(double2* S, int n, int k0) {
  __shared__ double2 li[CB][CB + 1], lj[CB][CB + 1];
  const int nb = min(CB, n - k0);
  const int r0 = k0 + nb + blockIdx.y * CB, c0 = k0 + nb + blockIdx.x * CB;
  if (c0 > r0 || r0 >= n) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < CB * CB; i += 256) {
    const int r = i / CB, c = i % CB;
    li[r][c] = (r0 + r < n && c < nb) ? S[(long long)(r0 + r) * n + k0 + c] : double2{0.0, 0.0};
    lj[r][c] = (c0 + r < n && c < nb) ? S[(long long)(c0 + r) * n + k0 + c] : double2{0.0, 0.0};
  }
  __syncthreads();
  for (int t = tid; t < CB * CB; t += 256) {
    const int r = t / CB, c = t % CB;
    const int gr = r0 + r, gc = c0 + c;
    if (gr < n && gc < n && gc <= gr) {
      double sx = 0.0, sy = 0.0;
      for (int m = 0; m < nb; ++m) {
        const double2 u = zmulc(li[r][m], lj[c][m]);
        sx += u.x;
        sy += u.y;
      }
      double2* p = S + (long long)gr * n + gc;
      *p = double2{p->x - sx, p->y - sy};
    }
  }
}

// ------------------------------------------------------- blocked lower inverse
// X = L^-1 from the inverses of L's diagonal blocks (written by the
// factorisation) by merging groups of w blocks pairwise, w = 1, 2, 4, ...:
// for the top group t and the bottom group b of a pair,
//   X_bt = -X_bb L_bt X_tt,
// in two stages through T = L_bt X_tt, which is kept transposed in the
// pair's strict upper block of X (cleared at the end).  Block (tile (ti, tj)
// of the pair's w x w tiles, pair); X_tt and X_bb are read as lower
// triangular, so the scratch in the upper triangle is never read as X.
template <int STAGE>
__global__ __launch_bounds__(256) void trinv_level_kernel(const double2* __restrict__ L, double2* __restrict__ X, int n,
                                                          int w) {
  __shared__ double2 ta[CB][CB + 1], tb[CB][CB + 1];
  const int nbk = (n + CB - 1) / CB;
  const int top0 = blockIdx.y * 2 * w, bot0 = top0 + w;
  const int wb = min(w, nbk - bot0);
  const int ti = blockIdx.x / w, tj = blockIdx.x % w;
  if (wb <= 0 || ti >= wb) return;
  const int tid = threadIdx.x, c = tid % CB, r0 = tid / CB;
  double2 acc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) acc[s] = double2{0.0, 0.0};
  const int kbeg = STAGE == 0 ? tj : 0, kend = STAGE == 0 ? w : ti + 1;
  for (int kk = kbeg; kk < kend; ++kk) {
    __syncthreads();
    for (int e = tid; e < CB * CB; e += 256) {
      const int r = e / CB, q = e % CB;
      if (STAGE == 0) {
        // T(ti, tj) = sum_kk L(b_ti, t_kk) X(t_kk, t_tj)
        const int lr = (bot0 + ti) * CB + r, lc = (top0 + kk) * CB + q;
        ta[r][q] = (lr < n && lc < n) ? L[(long long)lr * n + lc] : double2{0.0, 0.0};
        const int xr = (top0 + kk) * CB + r, xc = (top0 + tj) * CB + q;
        tb[r][q] = (xr < n && xc < n && xc <= xr) ? X[(long long)xr * n + xc] : double2{0.0, 0.0};
      } else {
        // X(b_ti, t_tj) = - sum_kk X(b_ti, b_kk) T(kk, tj); T[i][j] sits at X[j][i]
        const int xr = (bot0 + ti) * CB + r, xc = (bot0 + kk) * CB + q;
        ta[r][q] = (xr < n && xc < n && xc <= xr) ? X[(long long)xr * n + xc] : double2{0.0, 0.0};
        const int tr = (bot0 + kk) * CB + q, tc = (top0 + tj) * CB + r;   // tb[q][r] = T[tr][tc]
        tb[q][r] = (tr < n && tc < n) ? X[(long long)tc * n + tr] : double2{0.0, 0.0};
      }
    }
    __syncthreads();
    for (int m = 0; m < CB; ++m) {
      const double2 bv = tb[m][c];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double2 u = zmul(ta[r0 + 8 * s][m], bv);
        acc[s].x += u.x;
        acc[s].y += u.y;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int r = r0 + 8 * s;
    const int gi = (bot0 + ti) * CB + r, gj = (top0 + tj) * CB + c;
    if (gi >= n || gj >= n) continue;
    if (STAGE == 0) X[(long long)gj * n + gi] = acc[s];
    else X[(long long)gi * n + gj] = double2{-acc[s].x, -acc[s].y};
  }
}

__global__ void zero_upper_kernel(double2* X, int n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long long)n * n) return;
  const int r = i / n, c = i % n;
  if (c > r) X[i] = double2{0.0, 0.0};
}

// ------------------------------------------------------------------ launchers

// one-dimensional grid of the mt * nt * nz tiles, a multiple of XCDS
unsigned gemm_grid(int M, int N, int nz) {
  const long long t = (long long)((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN) * nz;
  return (unsigned)((t + XCDS - 1) / XCDS * XCDS);
}

// Fixed-order sum of nz partial products [nz][n][n] (only tiles on or below
// the diagonal when lower)
__global__ __launch_bounds__(256) void sum_partials_kernel(const double2* __restrict__ part, int nz, int n, bool lower,
                                                           double2* __restrict__ out) {
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  if (g >= (long long)n * n) return;
  const int i = (int)(g / n), j = (int)(g % n);
  if (lower && j / GBN > i / GBM) return;
  double2 s = part[g];
  for (int z = 1; z < nz; ++z) {
    const double2 v = part[(long long)z * n * n + g];
    s.x += v.x;
    s.y += v.y;
  }
  out[g] = s;
}

// Split of the K = npw contraction for an n x n product: enough blocks to
// fill the chip (about 2048 working blocks), chunks of at least 256,
// partials within part_bytes.
struct KSplit {
  int nz, kchunk;
};

KSplit ksplit(int n, int K, bool lower, size_t part_bytes) {
  const long long t = (long long)((n + GBN - 1) / GBN) * ((n + GBM - 1) / GBM);
  const long long tiles = lower ? (t + (n + GBM - 1) / GBM) / 2 : t;
  long long nz = (2048 + tiles - 1) / tiles;
  nz = std::min<long long>(nz, (long long)(part_bytes / ((size_t)n * n * sizeof(double2))));
  nz = std::min<long long>(nz, (K + 255) / 256);
  nz = std::max<long long>(nz, 1);
  int kchunk = (int)((K + nz - 1) / nz);
  kchunk = (kchunk + GBK - 1) / GBK * GBK;
  return KSplit{(K + kchunk - 1) / kchunk, kchunk};
}

size_t gemm_part_bytes(int n, int K) {
  size_t b = 0;
  for (bool lower : {true, false}) {
    const KSplit sp = ksplit(n, K, lower, GEMM_PART_MAX);
    if (sp.nz > 1) b = std::max(b, (size_t)sp.nz * n * n * sizeof(double2));
  }
  return b;
}

bool launch_overlap(int norb, int npw, const double2* P, int ldp, double2* S, double2* part, size_t part_bytes,
                    hipStream_t st) {
  // S[i][j] = sum_e conj(P[i][e]) P[j][e], tiles on and below the diagonal
  const KSplit sp = ksplit(norb, npw, true, part ? part_bytes : 0);
  const unsigned grid = gemm_grid(norb, norb, sp.nz);
  if (sp.nz == 1) {
    zgemm_mfma_kernel<true, false, false, true><<<grid, 256, 0, st>>>(norb, norb, npw, P, ldp, P, ldp, S, norb, sp.kchunk, 0);
    return true;
  }
  zgemm_mfma_kernel<true, false, false, true><<<grid, 256, 0, st>>>(norb, norb, npw, P, ldp, P, ldp, part, norb, sp.kchunk,
                                                                    (long long)norb * norb);
  sum_partials_kernel<<<(unsigned)(((long long)norb * norb + 255) / 256), 256, 0, st>>>(part, sp.nz, norb, true, S);
  return true;
}

__global__ void save_diag_kernel(const double2* __restrict__ S, int n, double* __restrict__ d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = S[(long long)i * n + i].x;
}

bool launch_cholesky(int n, double2* S, double2* X, double* diag0, int* info, hipStream_t st) {
  save_diag_kernel<<<(n + 255) / 256, 256, 0, st>>>(S, n, diag0);
  for (int k0 = 0; k0 < n; k0 += CB) {
    potrf_diag_kernel<<<1, CH_NT, 0, st>>>(S, X, n, k0, diag0, info);
    const int rest = n - k0 - min(CB, n - k0);
    if (rest > 0) {
      trsm_panel_kernel<<<(rest + 63) / 64, 256, 0, st>>>(S, X, n, k0);
      const int nt = (rest + CB - 1) / CB;
      herk_update_kernel<<<dim3(nt, nt), 256, 0, st>>>(S, n, k0);
    }
  }
  return true;
}

bool launch_trtri(int n, const double2* L, double2* X, hipStream_t st) {
  const int nbk = (n + CB - 1) / CB;
  for (int w = 1; w < nbk; w *= 2) {
    const dim3 grid(w * w, (nbk + 2 * w - 1) / (2 * w));
    trinv_level_kernel<0><<<grid, 256, 0, st>>>(L, X, n, w);
    trinv_level_kernel<1><<<grid, 256, 0, st>>>(L, X, n, w);
  }
  zero_upper_kernel<<<(unsigned)(((long long)n * n + 255) / 256), 256, 0, st>>>(X, n);
  return true;
}

bool launch_apply_lower(int norb, int npw, const double2* X, const double2* P, int ldp, double2* Y, hipStream_t st) {
  const unsigned grid = gemm_grid(norb, npw, 1);
  // Y[i][e] = sum_{j <= i} conj(X[i][j]) P[j][e]
  zgemm_mfma_kernel<true, true, true, false><<<grid, 256, 0, st>>>(norb, npw, norb, X, norb, P, ldp, Y, ldp, norb, 0);
  return true;
}

bool launch_gemm_ch(int norb, int npw, const double2* A, int lda, const double2* B, int ldb, double2* S, double2* part,
                    size_t part_bytes, hipStream_t st) {
  const KSplit sp = ksplit(norb, npw, false, part ? part_bytes : 0);
  const unsigned grid = gemm_grid(norb, norb, sp.nz);
  if (sp.nz == 1) {
    zgemm_mfma_kernel<true, false, false, false><<<grid, 256, 0, st>>>(norb, norb, npw, A, lda, B, ldb, S, norb, sp.kchunk, 0);
    return true;
  }
  zgemm_mfma_kernel<true, false, false, false><<<grid, 256, 0, st>>>(norb, norb, npw, A, lda, B, ldb, part, norb, sp.kchunk,
                                                                     (long long)norb * norb);
  sum_partials_kernel<<<(unsigned)(((long long)norb * norb + 255) / 256), 256, 0, st>>>(part, sp.nz, norb, false, S);
  return true;
}

bool launch_rotate(int norb, int npw, const double2* Q, const double2* X, int ldx, double2* Y, int ldy, hipStream_t st) {
  const unsigned grid = gemm_grid(norb, npw, 1);
  zgemm_mfma_kernel<false, true, false, false><<<grid, 256, 0, st>>>(norb, npw, norb, Q, norb, X, ldx, Y, ldy, norb, 0);
  return true;
}

}  // namespace ks
