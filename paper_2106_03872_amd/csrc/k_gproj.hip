// Kleinman-Bylander projections in reciprocal space for the mixed-precision
// path: the sphere sums of Eq. vnl written as one dense product over the
// packed plane waves and evaluated on the matrix cores as split-BF16 (three
// terms, FP32 accumulation).
//
// With psi(r) = Omega^-1/2 sum_G c_G e^{iG.r} and r_j = j L / n, the
// projection P_Ip = dV sum_{j in S_I} beta_Ip(r_j) psi(r_j) equals
// (Omega^1/2 / N) sum_G c_G sum_j beta_Ip(r_j) e^{iG.r_j}.  The x-pass that
// applies the nonlocal term takes DP = (Omega^1/2 / N) d_Ip P_Ip (the
// analysis scale of its output folded in), so
//   DP_Ip = sum_G c_G W_Ip(G),  W_Ip(G) = d_Ip (Omega / N^2) sum_j beta_Ip(r_j) e^{iG.r_j},
// a product of the packed orbitals [nb][npw] with a table W [npw][P]
// (P = natoms * nproj) built once per set of projectors.  In real arithmetic
// (k = 2g + r runs over the real and imaginary parts of c_g, column
// c = 2q + t gives the real (t = 0) or imaginary (t = 1) part of entry q):
//   B[2g][2q] = Re W, B[2g+1][2q] = -Im W, B[2g][2q+1] = Im W, B[2g+1][2q+1] = Re W,
// so DP = A B with A[o][k] the interleaved coefficients as stored.
//
// Split-BF16: x = hi(x) + lo(x) + O(2^-18 |x|) with hi = bf16(x) and
// lo = bf16(x - hi) (|lo| <= 2^-9 |x|); a b is taken as hi hi + hi lo + lo hi
// (the dropped lo lo term is at most 2^-18 |a b|), each on
// v_mfma_f32_16x16x32_bf16.
// B is stored split; A is split as it is staged.
#include "ks_common.hpp"

namespace ks {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int GP_MAXN = 128;   // largest grid size along an axis
constexpr int GP_BT = 128;     // block tile (orbitals x table columns)
constexpr int GP_LROW = 72;    // bf16 per staged row: 4 k-groups x (8 hi + 8 lo) + 8 padding

// Table W in the layout the product reads: column c holds, per group of 8
// consecutive k, the 8 hi parts and then the 8 lo parts ([c][k/8][16]).
__device__ __forceinline__ long long w_at(int c, int k, int kpad) {
  return (long long)c * (2 * kpad) + 16 * (k >> 3) + (k & 7);
}

__device__ __forceinline__ void split_store(__bf16* W, long long at, double x0, double x1) {
  const float f0 = (float)x0, f1 = (float)x1;
  const __bf16 h0 = (__bf16)f0, h1 = (__bf16)f1;
  const __bf16 l0 = (__bf16)(float)(x0 - (double)(float)h0), l1 = (__bf16)(float)(x1 - (double)(float)h1);
  W[at] = h0;
  W[at + 1] = h1;
  W[at + 8] = l0;
  W[at + 9] = l1;
}

// One thread per packed plane wave g, block row y for the atoms I = y, y +
// gridDim.y, ...: the sum over the atom's sphere points of
// beta_Ip(r_j) e^{iG.r_j} in FP64, the phase taken from per-axis tables of
// unit roots (exact integer residues).
__global__ __launch_bounds__(256) void gproj_table_kernel(SphereTab sp, int ncols, int npw, int kpad, int natoms,
                                                          const int* __restrict__ pt_off, const int* __restrict__ idx,
                                                          const double* __restrict__ beta,
                                                          const double* __restrict__ d, int np, double scale,
                                                          __bf16* __restrict__ W) {
  __shared__ double2 u[3][GP_MAXN];
  __shared__ int sj[256][3];
  __shared__ double sb[256 * KB_MAX_NPROJ];
  const int t = threadIdx.x;
  const int g = blockIdx.x * 256 + t;
  const int n[3] = {sp.n0, sp.n1, sp.n2};
  for (int a = 0; a < 3; ++a)
    for (int k = t; k < n[a]; k += 256) {
      double sn, cs;
      sincospi(2.0 * k / n[a], &sn, &cs);
      u[a][k] = double2{cs, sn};
    }
  int m[3] = {0, 0, 0};
  if (g < npw) {
    const int cc = find_col(sp.col_off, ncols, g);
    const int pi = find_col(sp.plane_col0, sp.nplanes, cc);
    m[0] = sp.m0lo + pi;
    m[1] = sp.plane_m1lo[pi] + (cc - sp.plane_col0[pi]);
    m[2] = sp.col_m2lo[cc] + (g - sp.col_off[cc]);
  }
  for (int a = 0; a < 3; ++a) m[a] = ((m[a] % n[a]) + n[a]) % n[a];
  for (int I = blockIdx.y; I < natoms; I += gridDim.y) {   // uniform per block
    double2 acc[KB_MAX_NPROJ];
#pragma unroll
    for (int p = 0; p < KB_MAX_NPROJ; ++p) acc[p] = double2{0.0, 0.0};
    const int j1 = pt_off[I + 1];
    for (int j0 = pt_off[I]; j0 < j1; j0 += 256) {
      const int nj = min(256, j1 - j0);
      __syncthreads();
      if (t < nj) {
        const int f = idx[j0 + t];
        sj[t][0] = f / (sp.n1 * sp.n2);
        sj[t][1] = (f / sp.n2) % sp.n1;
        sj[t][2] = f % sp.n2;
        for (int p = 0; p < np; ++p) sb[t * KB_MAX_NPROJ + p] = beta[(long long)(j0 + t) * np + p];
      }
      __syncthreads();
      for (int j = 0; j < nj; ++j) {
        const double2 a0 = u[0][(m[0] * sj[j][0]) % sp.n0];
        const double2 a1 = u[1][(m[1] * sj[j][1]) % sp.n1];
        const double2 a2 = u[2][(m[2] * sj[j][2]) % sp.n2];
        const double2 b01{a0.x * a1.x - a0.y * a1.y, a0.x * a1.y + a0.y * a1.x};
        const double2 ph{b01.x * a2.x - b01.y * a2.y, b01.x * a2.y + b01.y * a2.x};
#pragma unroll
        for (int p = 0; p < KB_MAX_NPROJ; ++p)
          if (p < np) {
            const double bv = sb[j * KB_MAX_NPROJ + p];
            acc[p].x += bv * ph.x;
            acc[p].y += bv * ph.y;
          }
      }
    }
    if (g < npw) {
#pragma unroll
      for (int p = 0; p < KB_MAX_NPROJ; ++p)
        if (p < np) {
          const int q = I * np + p;
          const double f = d[q] * scale;
          const double wr = f * acc[p].x, wi = f * acc[p].y;
          split_store(W, w_at(2 * q, 2 * g, kpad), wr, -wi);
          split_store(W, w_at(2 * q + 1, 2 * g, kpad), wi, wr);
        }
    }
  }
}

__device__ __forceinline__ void ld4(const float* p, float v[4]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ __forceinline__ void ld4(const double* p, float v[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  v[0] = (float)a.x; v[1] = (float)a.y; v[2] = (float)b.x; v[3] = (float)b.y;
}

// Global loads of k-step ks for one thread: four pieces of 4 consecutive k
// of A (zero beyond k2 = 2 npw) and four 16-byte pieces of the table.
template <typename TA>
__device__ __forceinline__ void gp_load(const TA* const (&ag)[4], const __bf16* const (&bg)[4],
                                        const int (&akoff)[4], int ks, int k2, float (&ra)[4][4],
                                        u32x4 (&rb)[4]) {
  const int k = ks * 32;
  if (k + 32 <= k2) {
#pragma unroll
    for (int v = 0; v < 4; ++v) ld4(ag[v] + k, ra[v]);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) ra[v][e] = (k + akoff[v] + e < k2) ? (float)ag[v][k + e] : 0.0f;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) rb[v] = *reinterpret_cast<const u32x4*>(bg[v] + 2 * k);
}

// part[s][o][c] = sum over k-chunk s of A[o][k] B[k][c].  Block: a 128 x 128
// output tile over one k-chunk, four waves of 64 x 64 (4 x 4 MFMA tiles of
// 16 x 16).  Per k-step of 32 the block stages A (split to hi/lo once) and
// the table slice in LDS, double-buffered with one barrier per step, while
// the next step's global loads are in flight.  With S a multiple of 8 the
// blocks of one k-chunk share an XCD (blocks are dealt to the 8 XCDs in
// turn), so the A and table slices of a chunk are read from HBM once per XCD.
// MFMA lane layout (16x16x32 bf16): A[i][k] in lane i + 16 (k / 8), element
// k % 8; B[k][j] in lane j + 16 (k / 8); D[i][j] in lane j + 16 (i / 4),
// element i % 4.
template <typename TA>
__global__ __launch_bounds__(256) void gproj_gemm_kernel(const TA* __restrict__ A, long long lda2, int nb, int k2,
                                                         const __bf16* __restrict__ W, int kpad, int ncol, int ntc,
                                                         int tiles, int splits, int kpc, int ksteps,
                                                         float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) __bf16 sA[2][GP_BT * GP_LROW];
  __shared__ __attribute__((aligned(16))) __bf16 sB[2][GP_BT * GP_LROW];
  const int b = blockIdx.x;
  int chunk, tile;
  if (splits % 8 == 0) {
    const int xcd = b & 7, local = b >> 3;
    chunk = xcd + 8 * (local / tiles);
    tile = local % tiles;
  } else {
    chunk = b / tiles;
    tile = b % tiles;
  }
  const int rt = tile / ntc, ct = tile % ntc;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const TA* ag[4];
  const __bf16* bg[4];
  int apos[4], bpos[4], akoff[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int e = v * 256 + t, rc = e >> 3, pc = e & 7;
    const int r = min(rt * GP_BT + rc, nb - 1);    // rows past nb: valid data, results not stored
    ag[v] = A + (long long)r * lda2 + 4 * pc;
    akoff[v] = 4 * pc;
    apos[v] = rc * GP_LROW + (pc >> 1) * 16 + (pc & 1) * 4;   // hi at +0, lo at +8
    bg[v] = W + (long long)(ct * GP_BT + rc) * (2 * kpad) + 8 * pc;
    bpos[v] = rc * GP_LROW + 8 * pc;
  }
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ks0 = chunk * kpc, ks1 = min(ks0 + kpc, ksteps);
  float ra[4][4];
  u32x4 rb[4];
  if (ks0 < ks1) gp_load<TA>(ag, bg, akoff, ks0, k2, ra, rb);
  const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
  for (int ks = ks0; ks < ks1; ++ks) {
    const int buf = (ks - ks0) & 1;
    __bf16* a_s = sA[buf];
    __bf16* b_s = sB[buf];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      bf16x4 h, l;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const __bf16 hh = (__bf16)ra[v][e];
        h[e] = hh;
        l[e] = (__bf16)(ra[v][e] - (float)hh);
      }
      *reinterpret_cast<bf16x4*>(a_s + apos[v]) = h;
      *reinterpret_cast<bf16x4*>(a_s + apos[v] + 8) = l;
      *reinterpret_cast<u32x4*>(b_s + bpos[v]) = rb[v];
    }
    __syncthreads();
    if (ks + 1 < ks1) gp_load<TA>(ag, bg, akoff, ks + 1, k2, ra, rb);
    bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const __bf16* pa = a_s + (wr + 16 * i + l16) * GP_LROW + 16 * kq;
      ah[i] = *reinterpret_cast<const bf16x8*>(pa);
      al[i] = *reinterpret_cast<const bf16x8*>(pa + 8);
      const __bf16* pb = b_s + (wc + 16 * i + l16) * GP_LROW + 16 * kq;
      bh[i] = *reinterpret_cast<const bf16x8*>(pb);
      bl[i] = *reinterpret_cast<const bf16x8*>(pb + 8);
    }
    // term-major: each accumulator is updated once every 16 MFMAs
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
  }
  float* out = part + (long long)chunk * nb * ncol;
  const int row0 = rt * GP_BT + wr, col0 = ct * GP_BT + wc;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = row0 + 16 * i + 4 * kq + e;
        if (r < nb) out[(long long)r * ncol + col0 + 16 * j + l16] = acc[i][j][e];
      }
}

// DP[o][q] = (sum_s part[s][o][2q], sum_s part[s][o][2q+1]) in FP64, the
// k-chunks added in ascending order.
__global__ __launch_bounds__(128) void gproj_reduce_kernel(const float* __restrict__ part, int splits, int nb,
                                                           int ncol, int P, double2* __restrict__ DP) {
  const int q = blockIdx.x * 128 + threadIdx.x, o = blockIdx.y;
  if (q >= P) return;
  double x = 0.0, y = 0.0;
  for (int s = 0; s < splits; ++s) {
    const float2 v = *reinterpret_cast<const float2*>(part + ((long long)s * nb + o) * ncol + 2 * q);
    x += (double)v.x;
    y += (double)v.y;
  }
  DP[(long long)o * P + q] = double2{x, y};
}

}  // namespace

int gproj_splits(int nb, int ncol, int ksteps) {
  const int tiles = ((nb + GP_BT - 1) / GP_BT) * (ncol / GP_BT);
  int s = std::max(1, 1024 / tiles);           // about four blocks per compute unit, <= 64 MiB of partials
  s = std::min(s, 64);
  s = std::min(s, std::max(1, ksteps / 8));    // at least 8 k-steps per block
  if (s >= 8) s = s / 8 * 8;
  return std::max(s, 1);
}

size_t gproj_part_bytes(int cb, int ncol, int ksteps) {
  size_t most = 0;
  for (int nb = 1; nb <= cb; ++nb)
    most = std::max(most, (size_t)gproj_splits(nb, ncol, ksteps) * nb * ncol * sizeof(float));
  return most;
}

bool launch_gproj_table(const ks_system* s, const int* pt_off, const int* idx, const double* beta, const double* d,
                        int natoms, int np, __bf16* W, int kpad, hipStream_t st) {
  if (natoms == 0) return true;
  if (np > KB_MAX_NPROJ || s->n[0] > GP_MAXN || s->n[1] > GP_MAXN || s->n[2] > GP_MAXN) return false;
  const double scale = s->omega / ((double)s->N * (double)s->N);
  const dim3 grid((s->npw + 255) / 256, std::min(natoms, KS_MAX_GRID_Y));
  gproj_table_kernel<<<grid, 256, 0, st>>>(sphere_tab(s), s->ncols, s->npw, kpad, natoms, pt_off, idx, beta, d, np,
                                           scale, W);
  return true;
}

bool launch_gproj(const ks_system* s, int nb, const void* win, bool win_fp64, double2* DP, hipStream_t st) {
  const GTab& g = s->gp;
  if (nb == 0 || g.P == 0) return true;
  const int ksteps = g.kpad / 32;
  const int splits = gproj_splits(nb, g.ncol, ksteps);
  if ((size_t)splits * nb * g.ncol * sizeof(float) > g.part_bytes) return false;
  const int ntc = g.ncol / GP_BT, tiles = ((nb + GP_BT - 1) / GP_BT) * ntc;
  const int kpc = (ksteps + splits - 1) / splits;
  const long long lda2 = 2LL * s->npw_stride;
  const int k2 = 2 * s->npw;
  if (win_fp64)
    gproj_gemm_kernel<double><<<tiles * splits, 256, 0, st>>>(static_cast<const double*>(win), lda2, nb, k2, g.w,
                                                               g.kpad, g.ncol, ntc, tiles, splits, kpc, ksteps, g.part);
  else
    gproj_gemm_kernel<float><<<tiles * splits, 256, 0, st>>>(static_cast<const float*>(win), lda2, nb, k2, g.w,
                                                              g.kpad, g.ncol, ntc, tiles, splits, kpc, ksteps, g.part);
  gproj_reduce_kernel<<<dim3((g.P + 127) / 128, nb), 128, 0, st>>>(g.part, splits, nb, g.ncol, g.P, DP);
  return true;
}

}  // namespace ks
