// HIP kernels of the Kohn-Sham Hamiltonian application for gfx950.
//
// One application H c on a chunk of orbitals runs five passes:
//   plane_inv : sphere-packed c -> per m0 plane, z- then y-synthesis (pruned)
//               -> T[o][m0 plane][j1][j2]
//   xproj     : x-synthesis of each x-pencil in LDS, then the KB projections
//               dV sum beta psi over each pencil's runs of sphere points
//   proj_red  : per atom and projector, sum the runs (fixed order) and scale
//               by d_Ip (Eq. vnl)
//   xapply    : x-synthesis again, V psi + sum_p beta_Ip d_Ip P_Ip on the
//               sphere points, x-analysis, keep the m0 planes -> U
//   plane_fwd : y- then z-analysis (pruned to the sphere) + kinetic |G|^2/2 c,
//               with the Taylor-4 epilogue when propagating.
// The orbitals never exist on the full real-space box in HBM: the x-pencil
// passes hold them in LDS only.
#include "fft_device.hpp"
#include "ks_internal.h"

namespace ks {

constexpr int NT = 256;

#define KS_SIZES(X) X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(60) X(64) X(72) X(80) X(96) X(120) X(128)

bool supported_size(int n) {
  switch (n) {
#define KS_CASE(v) case v:
    KS_SIZES(KS_CASE)
#undef KS_CASE
    return true;
    default:
      return false;
  }
}

// pencils per x-tile
int x_tile_nb(int n0) { return n0 <= 32 ? 64 : 32; }
template <int N> struct xnb { static constexpr int value = N <= 32 ? 64 : 32; };
constexpr int PNB = 32;  // transforms per batch in the plane passes

template <typename T> __device__ __forceinline__ T czero() { return T{0, 0}; }

template <typename T> __device__ __forceinline__ T to_c(double2 a) {
  return T{static_cast<decltype(T{}.x)>(a.x), static_cast<decltype(T{}.x)>(a.y)};
}
template <typename T> __device__ __forceinline__ double2 to_d(T a) { return double2{double(a.x), double(a.y)}; }

// largest c in [0, nc) with off[c] <= e (off ascending)
__device__ __forceinline__ int find_col(const int* off, int nc, int e) {
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ pack / unpack

template <typename T>
__global__ __launch_bounds__(NT) void pack_kernel(const double2* __restrict__ box, long long box_stride,
                                                  T* __restrict__ pk, int pk_stride, SphereTab tab) {
  __shared__ int s_off[130];
  __shared__ int s_m2lo[129];
  const int pi = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int c0 = tab.plane_col0[pi], nc = tab.plane_col0[pi + 1] - c0;
  for (int i = tid; i <= nc; i += NT) s_off[i] = tab.col_off[c0 + i];
  for (int i = tid; i < nc; i += NT) s_m2lo[i] = tab.col_m2lo[c0 + i];
  __syncthreads();
  const int j0 = wrap(tab.m0lo + pi, tab.n0);
  const int m1lo = tab.plane_m1lo[pi];
  const double2* b = box + (long long)o * box_stride + (long long)j0 * tab.n1 * tab.n2;
  T* out = pk + (long long)o * pk_stride;
  for (int e = s_off[0] + tid; e < s_off[nc]; e += NT) {
    const int c = find_col(s_off, nc, e);
    const int m1 = m1lo + c, m2 = s_m2lo[c] + (e - s_off[c]);
    out[e] = to_c<T>(b[(long long)wrap(m1, tab.n1) * tab.n2 + wrap(m2, tab.n2)]);
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void unpack_kernel(const T* __restrict__ pk, int pk_stride,
                                                    double2* __restrict__ box, long long box_stride,
                                                    SphereTab tab) {
  const long long N = (long long)tab.n0 * tab.n1 * tab.n2;
  const long long bi = (long long)blockIdx.x * NT + threadIdx.x;
  if (bi >= N) return;
  const int o = blockIdx.y;
  const int j2 = bi % tab.n2;
  const int j1 = (bi / tab.n2) % tab.n1;
  const int j0 = bi / ((long long)tab.n1 * tab.n2);
  double2 v{0.0, 0.0};
  const int pi = fold(j0, tab.n0) - tab.m0lo;
  if (pi >= 0 && pi < tab.nplanes) {
    const int c = fold(j1, tab.n1) - tab.plane_m1lo[pi];
    const int c0 = tab.plane_col0[pi];
    if (c >= 0 && c < tab.plane_col0[pi + 1] - c0) {
      const int cc = c0 + c;
      const int t = fold(j2, tab.n2) - tab.col_m2lo[cc];
      const int off = tab.col_off[cc];
      if (t >= 0 && t < tab.col_off[cc + 1] - off) v = to_d(pk[(long long)o * pk_stride + off + t]);
    }
  }
  box[(long long)o * box_stride + bi] = v;
}

// ----------------------------------------------------------- plane synthesis
// Block (plane pi, orbital o).  LDS: twiddles [N] | Z [ncol][N+1] | Y [PNB][N+1].

template <int N, typename R>
__global__ __launch_bounds__(NT) void plane_inv_kernel(const cplx<R>* __restrict__ pk, int pk_stride,
                                                       cplx<R>* __restrict__ Tout, SphereTab tab,
                                                       const cplx<R>* __restrict__ twN, int ncol_max) {
  using C = cplx<R>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  C* Z = tw + N;
  C* Y = Z + ncol_max * (N + 1);
  const int pi = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int c0 = tab.plane_col0[pi], nc = tab.plane_col0[pi + 1] - c0;
  const int m1lo = tab.plane_m1lo[pi];
  for (int i = tid; i < N; i += NT) tw[i] = twN[i];
  const C* in = pk + (long long)o * pk_stride;
  for (int i = tid; i < nc * N; i += NT) {
    const int c = i / N, j2 = i - c * N;
    const int off = tab.col_off[c0 + c], len = tab.col_off[c0 + c + 1] - off;
    const int t = fold(j2, N) - tab.col_m2lo[c0 + c];
    Z[c * (N + 1) + j2] = (t >= 0 && t < len) ? in[off + t] : czero<C>();
  }
  __syncthreads();
  for (int cb = 0; cb < nc; cb += PNB) fft_batch<N, +1, PNB, NT>(Z + cb * (N + 1), N + 1, nc - cb, tw);
  C* out = Tout + ((long long)o * tab.nplanes + pi) * N * N;
  for (int w0 = 0; w0 < N; w0 += PNB) {
    for (int i = tid; i < PNB * N; i += NT) {
      const int w = i % PNB, j1 = i / PNB;
      const int c = fold(j1, N) - m1lo;
      Y[w * (N + 1) + j1] = (c >= 0 && c < nc && w0 + w < N) ? Z[c * (N + 1) + w0 + w] : czero<C>();
    }
    __syncthreads();
    fft_batch<N, +1, PNB, NT>(Y, N + 1, N - w0, tw);
    for (int i = tid; i < PNB * N; i += NT) {
      const int w = i % PNB, r1 = i / PNB;
      if (w0 + w < N) out[r1 * N + w0 + w] = Y[w * (N + 1) + r1];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ plane analysis
// Block (plane pi, orbital o): y-analysis of U's plane, keep the disk columns,
// z-analysis of each column, keep its m2 run, then the kinetic term and the
// output mode.

template <int N, typename R>
__global__ __launch_bounds__(NT) void plane_fwd_kernel(const cplx<R>* __restrict__ Uin,
                                                       const cplx<R>* win,
                                                       cplx<R>* __restrict__ wout, double2* acc,
                                                       int pk_stride, int acc_stride, SphereTab tab,
                                                       const cplx<R>* __restrict__ twN, int ncol_max, int mode,
                                                       Taylor tay, double g0, double g1, double g2) {
  using C = cplx<R>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  C* Z = tw + N;
  C* Y = Z + ncol_max * (N + 1);
  __shared__ int s_off[130];
  __shared__ int s_m2lo[129];
  const int pi = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int c0 = tab.plane_col0[pi], nc = tab.plane_col0[pi + 1] - c0;
  const int m1lo = tab.plane_m1lo[pi];
  for (int i = tid; i < N; i += NT) tw[i] = twN[i];
  for (int i = tid; i <= nc; i += NT) s_off[i] = tab.col_off[c0 + i];
  for (int i = tid; i < nc; i += NT) s_m2lo[i] = tab.col_m2lo[c0 + i];
  const C* u = Uin + ((long long)o * tab.nplanes + pi) * N * N;
  for (int w0 = 0; w0 < N; w0 += PNB) {
    for (int i = tid; i < PNB * N; i += NT) {
      const int w = i % PNB, r1 = i / PNB;
      Y[w * (N + 1) + r1] = (w0 + w < N) ? u[r1 * N + w0 + w] : czero<C>();
    }
    __syncthreads();
    fft_batch<N, -1, PNB, NT>(Y, N + 1, N - w0, tw);
    for (int i = tid; i < PNB * nc; i += NT) {
      const int w = i % PNB, c = i / PNB;
      if (w0 + w < N) Z[c * (N + 1) + w0 + w] = Y[w * (N + 1) + wrap(m1lo + c, N)];
    }
    __syncthreads();
  }
  for (int cb = 0; cb < nc; cb += PNB) fft_batch<N, -1, PNB, NT>(Z + cb * (N + 1), N + 1, nc - cb, tw);
  // epilogue over the packed elements of this plane
  const int m0 = tab.m0lo + pi;
  const double k0 = g0 * m0;
  const long long ob = (long long)o * pk_stride;
  for (int e = s_off[0] + tid; e < s_off[nc]; e += NT) {
    const int c = find_col(s_off, nc, e);
    const int m1 = m1lo + c, m2 = s_m2lo[c] + (e - s_off[c]);
    const double k1 = g1 * m1, k2 = g2 * m2;
    const double K = 0.5 * (k0 * k0 + k1 * k1 + k2 * k2);
    const C ph = Z[c * (N + 1) + wrap(m2, N)];
    const C w = win[ob + e];
    const double2 hw{K * double(w.x) + double(ph.x), K * double(w.y) + double(ph.y)};
    if (mode == H_OUT) {
      wout[ob + e] = to_c<C>(hw);
    } else {
      if (tay.write_w) wout[ob + e] = to_c<C>(hw);
      double2* a = acc + (long long)o * acc_stride + e;
      double2 av = *a;
      av.x += tay.coef.x * hw.x - tay.coef.y * hw.y;
      av.y += tay.coef.x * hw.y + tay.coef.y * hw.x;
      *a = av;
    }
  }
}

// -------------------------------------------------------------- x-pencil passes
// Block (tile of NB consecutive pencils p = j1*n2 + j2, orbital o).
// LDS: twiddles [N0] | X [NB][N0+1], X[w][j0].

template <int N0, int NB, typename C>
__device__ __forceinline__ void x_load(C* X, const C* __restrict__ Tin, long long plane_stride, int nplanes,
                                       int m0lo, int p0, int npencils) {
  const int tid = threadIdx.x;
  for (int i = tid; i < nplanes * NB; i += NT) {
    const int w = i % NB, pi = i / NB;
    const int p = p0 + w;
    X[w * (N0 + 1) + wrap(m0lo + pi, N0)] = (p < npencils) ? Tin[pi * plane_stride + p] : czero<C>();
  }
  for (int i = tid; i < (N0 - nplanes) * NB; i += NT) {
    const int w = i % NB, jj = i / NB;
    int j0 = m0lo + nplanes + jj;
    j0 = ((j0 % N0) + N0) % N0;
    X[w * (N0 + 1) + j0] = czero<C>();
  }
}

template <int N0, typename R>
__global__ __launch_bounds__(NT) void xproj_kernel(const cplx<R>* __restrict__ Tin, cplx<R>* __restrict__ partial,
                                                   SphereTab tab, ChordTab ct, const cplx<R>* __restrict__ tw0,
                                                   double scale) {
  using C = cplx<R>;
  constexpr int NB = xnb<N0>::value;
  __shared__ C tw[N0];
  __shared__ C X[NB * (N0 + 1)];
  const int tile = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int npl = tab.n1 * tab.n2;
  const int p0 = tile * NB;
  const int chA = ct.tile_off[tile], chB = ct.tile_off[tile + 1];
  if (chA == chB) return;  // no sphere point in this tile (uniform per block)
  for (int i = tid; i < N0; i += NT) tw[i] = tw0[i];
  x_load<N0, NB>(X, Tin + (long long)o * tab.nplanes * npl, npl, tab.nplanes, tab.m0lo, p0, npl);
  __syncthreads();
  fft_batch<N0, +1, NB, NT>(X, N0 + 1, NB, tw);
  const int np = ct.nproj;
  for (int i = tid; i < (chB - chA) * np; i += NT) {
    const int ch = chA + i / np, q = i % np;
    const int w = ct.ch_pencil[ch] - p0, r0 = ct.ch_r0[ch], len = ct.ch_len[ch], bo = ct.ch_boff[ch];
    double sx = 0.0, sy = 0.0;
    for (int l = 0; l < len; ++l) {
      const double b = ct.beta[(long long)(bo + l) * np + q];
      const C x = X[w * (N0 + 1) + r0 + l];
      sx += b * double(x.x);
      sy += b * double(x.y);
    }
    partial[((long long)o * ct.nchords + ch) * np + q] = C{R(sx * scale), R(sy * scale)};
  }
}

template <int N0, typename R>
__global__ __launch_bounds__(NT) void xapply_kernel(const cplx<R>* __restrict__ Tin, cplx<R>* __restrict__ Uout,
                                                    const double* __restrict__ V, const double2* __restrict__ DP,
                                                    SphereTab tab, ChordTab ct, const cplx<R>* __restrict__ tw0,
                                                    double sc_in, double sc_out) {
  using C = cplx<R>;
  constexpr int NB = xnb<N0>::value;
  __shared__ C tw[N0];
  __shared__ C X[NB * (N0 + 1)];
  const int tile = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int npl = tab.n1 * tab.n2;
  const int p0 = tile * NB;
  for (int i = tid; i < N0; i += NT) tw[i] = tw0[i];
  x_load<N0, NB>(X, Tin + (long long)o * tab.nplanes * npl, npl, tab.nplanes, tab.m0lo, p0, npl);
  __syncthreads();
  fft_batch<N0, +1, NB, NT>(X, N0 + 1, NB, tw);
  const int np = ct.nproj;
  for (int i = tid; i < N0 * NB; i += NT) {
    const int w = i % NB, r0 = i / NB;
    const int p = p0 + w;
    if (p >= npl) continue;
    const C x = X[w * (N0 + 1) + r0];
    const double v = V[(long long)r0 * npl + p] * sc_in;
    double fx = v * double(x.x), fy = v * double(x.y);
    if (ct.natoms > 0) {
      const int cA = ct.pen_off[p], cB = ct.pen_off[p + 1];
      for (int ch = cA; ch < cB; ++ch) {
        const int t = r0 - ct.ch_r0[ch];
        if (t < 0 || t >= ct.ch_len[ch]) continue;
        const double* b = ct.beta + (long long)(ct.ch_boff[ch] + t) * np;
        const double2* dp = DP + ((long long)o * ct.natoms + ct.ch_atom[ch]) * np;
        for (int q = 0; q < np; ++q) {
          fx += b[q] * dp[q].x;
          fy += b[q] * dp[q].y;
        }
      }
    }
    X[w * (N0 + 1) + r0] = C{R(fx), R(fy)};
  }
  __syncthreads();
  fft_batch<N0, -1, NB, NT>(X, N0 + 1, NB, tw);
  C* out = Uout + (long long)o * tab.nplanes * npl;
  for (int i = tid; i < tab.nplanes * NB; i += NT) {
    const int w = i % NB, pi = i / NB;
    const int p = p0 + w;
    if (p < npl) {
      const C x = X[w * (N0 + 1) + wrap(tab.m0lo + pi, N0)];
      out[(long long)pi * npl + p] = C{R(double(x.x) * sc_out), R(double(x.y) * sc_out)};
    }
  }
}

// density: block = tile, loops over the nb orbitals of the chunk in order
template <int N0, typename R>
__global__ __launch_bounds__(NT) void xdens_kernel(const cplx<R>* __restrict__ Tin, int nb,
                                                   const double* __restrict__ occ, double* __restrict__ rho,
                                                   int accumulate, SphereTab tab, const cplx<R>* __restrict__ tw0,
                                                   double inv_omega) {
  using C = cplx<R>;
  constexpr int NB = xnb<N0>::value;
  constexpr int IT = (N0 * NB + NT - 1) / NT;
  __shared__ C tw[N0];
  __shared__ C X[NB * (N0 + 1)];
  const int tile = blockIdx.x, tid = threadIdx.x;
  const int npl = tab.n1 * tab.n2;
  const int p0 = tile * NB;
  for (int i = tid; i < N0; i += NT) tw[i] = tw0[i];
  double a[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) a[k] = 0.0;
  for (int o = 0; o < nb; ++o) {
    x_load<N0, NB>(X, Tin + (long long)o * tab.nplanes * npl, npl, tab.nplanes, tab.m0lo, p0, npl);
    __syncthreads();
    fft_batch<N0, +1, NB, NT>(X, N0 + 1, NB, tw);
    const double f = occ[o] * inv_omega;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int i = tid + k * NT;
      if (i < N0 * NB) {
        const int w = i % NB, r0 = i / NB;
        const C x = X[w * (N0 + 1) + r0];
        a[k] += f * (double(x.x) * double(x.x) + double(x.y) * double(x.y));
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int i = tid + k * NT;
    if (i < N0 * NB) {
      const int w = i % NB, r0 = i / NB;
      const int p = p0 + w;
      if (p < npl) {
        double* r = rho + (long long)r0 * npl + p;
        *r = accumulate ? *r + a[k] : a[k];
      }
    }
  }
}

// KB projections: P_Ip = sum of the runs of atom I (ascending chord order),
// DP = d_Ip P_Ip.  One thread per (orbital, atom, projector).
template <typename C>
__global__ __launch_bounds__(NT) void proj_reduce_kernel(const C* __restrict__ partial, double2* __restrict__ DP,
                                                         ChordTab ct, int nb) {
  const long long i = (long long)blockIdx.x * NT + threadIdx.x;
  const long long tot = (long long)nb * ct.natoms * ct.nproj;
  if (i >= tot) return;
  const int q = i % ct.nproj;
  const int I = (i / ct.nproj) % ct.natoms;
  const int o = i / ((long long)ct.nproj * ct.natoms);
  double sx = 0.0, sy = 0.0;
  for (int k = ct.atom_off[I]; k < ct.atom_off[I + 1]; ++k) {
    const C v = partial[((long long)o * ct.nchords + ct.atom_list[k]) * ct.nproj + q];
    sx += double(v.x);
    sy += double(v.y);
  }
  const double dd = ct.d[I * ct.nproj + q];
  DP[i] = double2{dd * sx, dd * sy};
}

// per-orbital sums over the packed sphere: out[2o] = sum |a|^2, out[2o+1] = sum Re conj(a) b
template <typename C>
__global__ __launch_bounds__(NT) void dots_kernel(const C* __restrict__ a, const C* __restrict__ b, int stride,
                                                  int npw, double* __restrict__ out) {
  __shared__ double s0[NT], s1[NT];
  const int o = blockIdx.x, tid = threadIdx.x;
  const C* pa = a + (long long)o * stride;
  const C* pb = b ? b + (long long)o * stride : nullptr;
  double x0 = 0.0, x1 = 0.0;
  for (int e = tid; e < npw; e += NT) {
    const C u = pa[e];
    x0 += double(u.x) * double(u.x) + double(u.y) * double(u.y);
    if (pb) {
      const C v = pb[e];
      x1 += double(u.x) * double(v.x) + double(u.y) * double(v.y);
    }
  }
  s0[tid] = x0;
  s1[tid] = x1;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      s0[tid] += s0[tid + h];
      s1[tid] += s1[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[2 * o] = s0[0];
    out[2 * o + 1] = s1[0];
  }
}

__global__ void energy_sum_kernel(int norb, const double* __restrict__ occ, const double* __restrict__ red,
                                  double* __restrict__ energy) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double e = 0.0;
    for (int o = 0; o < norb; ++o) e += occ[o] * red[2 * o + 1];
    energy[0] = e;
  }
}

// ------------------------------------------------------------------ launchers

static SphereTab sphere_tab(const ks_system* s) {
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

static ChordTab chord_tab(const ks_system* s) {
  ChordTab c;
  c.ch_pencil = s->d_ch_pencil;
  c.ch_atom = s->d_ch_atom;
  c.ch_r0 = s->d_ch_r0;
  c.ch_len = s->d_ch_len;
  c.ch_boff = s->d_ch_boff;
  c.beta = s->d_beta;
  c.tile_off = s->d_tile_off;
  c.pen_off = s->d_pen_off;
  c.atom_off = s->d_atom_off;
  c.atom_list = s->d_atom_list;
  c.d = s->d_kb;
  c.nchords = s->nchords;
  c.natoms = s->natoms;
  c.nproj = s->nproj;
  return c;
}

size_t plane_lds_bytes(const ks_system* s) {
  const int N = s->n[1];
  return sizeof(double2) * ((size_t)N + (size_t)s->ncol_max * (N + 1) + (size_t)PNB * (N + 1));
}

bool launch_pack(const ks_system* s, int nb, const double2* box, long long box_stride, void* pk, hipStream_t st) {
  pack_kernel<double2><<<dim3(s->nplanes, nb), NT, 0, st>>>(box, box_stride, (double2*)pk, s->npw_stride,
                                                             sphere_tab(s));
  return true;
}

bool launch_unpack(const ks_system* s, int nb, const void* pk, double2* box, long long box_stride, hipStream_t st) {
  const unsigned gx = (unsigned)((s->N + NT - 1) / NT);
  unpack_kernel<double2><<<dim3(gx, nb), NT, 0, st>>>((const double2*)pk, s->npw_stride, box, box_stride,
                                                       sphere_tab(s));
  return true;
}

template <int N>
static void plane_inv_n(const ks_system* s, int nb, const void* pk, void* T, hipStream_t st) {
  const size_t lds = plane_lds_bytes(s);
  plane_inv_kernel<N, double><<<dim3(s->nplanes, nb), NT, lds, st>>>(
      (const double2*)pk, s->npw_stride, (double2*)T, sphere_tab(s), s->d_tw1, s->ncol_max);
}

bool launch_plane_inv(const ks_system* s, int nb, const void* pk, void* T, hipStream_t st) {
  switch (s->n[1]) {
#define KS_CASE(v) case v: plane_inv_n<v>(s, nb, pk, T, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

template <int N>
static void plane_fwd_n(const ks_system* s, int nb, const void* U, const void* win, void* wout, void* acc,
                        HMode mode, Taylor tay, hipStream_t st) {
  const size_t lds = plane_lds_bytes(s);
  const double g0 = 2.0 * M_PI / s->L[0], g1 = 2.0 * M_PI / s->L[1], g2 = 2.0 * M_PI / s->L[2];
  plane_fwd_kernel<N, double><<<dim3(s->nplanes, nb), NT, lds, st>>>(
      (const double2*)U, (const double2*)win, (double2*)wout, (double2*)acc, s->npw_stride, s->npw_stride,
      sphere_tab(s), s->d_tw1, s->ncol_max, (int)mode, tay, g0, g1, g2);
}

bool launch_plane_fwd(const ks_system* s, int nb, const void* U, const void* win, void* wout, void* acc,
                      HMode mode, Taylor tay, hipStream_t st) {
  switch (s->n[1]) {
#define KS_CASE(v) case v: plane_fwd_n<v>(s, nb, U, win, wout, acc, mode, tay, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

template <int N0>
static void xproj_n(const ks_system* s, int nb, const void* T, void* partial, hipStream_t st) {
  const double scale = s->dV / sqrt(s->omega);
  xproj_kernel<N0, double><<<dim3(s->ntiles, nb), NT, 0, st>>>((const double2*)T, (double2*)partial,
                                                                sphere_tab(s), chord_tab(s), s->d_tw0, scale);
}

bool launch_xproj(const ks_system* s, int nb, const void* T, void* partial, hipStream_t st) {
  switch (s->n[0]) {
#define KS_CASE(v) case v: xproj_n<v>(s, nb, T, partial, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

bool launch_proj_reduce(const ks_system* s, int nb, const void* partial, double2* DP, hipStream_t st) {
  const long long tot = (long long)nb * s->natoms * s->nproj;
  if (tot == 0) return true;
  proj_reduce_kernel<double2><<<(unsigned)((tot + NT - 1) / NT), NT, 0, st>>>((const double2*)partial, DP,
                                                                             chord_tab(s), nb);
  return true;
}

template <int N0>
static void xapply_n(const ks_system* s, int nb, const void* T, const double2* DP, void* U, hipStream_t st) {
  const double sc_in = 1.0 / sqrt(s->omega);
  const double sc_out = sqrt(s->omega) / (double)s->N;
  xapply_kernel<N0, double><<<dim3(s->ntiles, nb), NT, 0, st>>>((const double2*)T, (double2*)U, s->d_v, DP,
                                                                 sphere_tab(s), chord_tab(s), s->d_tw0, sc_in,
                                                                 sc_out);
}

bool launch_xapply(const ks_system* s, int nb, const void* T, const double2* DP, void* U, hipStream_t st) {
  switch (s->n[0]) {
#define KS_CASE(v) case v: xapply_n<v>(s, nb, T, DP, U, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

template <int N0>
static void xdens_n(const ks_system* s, int nb, const void* T, const double* occ, double* rho, int accumulate,
                    hipStream_t st) {
  xdens_kernel<N0, double><<<dim3(s->ntiles), NT, 0, st>>>((const double2*)T, nb, occ, rho, accumulate,
                                                            sphere_tab(s), s->d_tw0, 1.0 / s->omega);
}

bool launch_xdens(const ks_system* s, int nb, const void* T, const double* occ, double* rho, int accumulate,
                  hipStream_t st) {
  switch (s->n[0]) {
#define KS_CASE(v) case v: xdens_n<v>(s, nb, T, occ, rho, accumulate, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

bool launch_dots(const ks_system* s, int nb, const void* a, const void* b, double* out, hipStream_t st) {
  dots_kernel<double2><<<nb, NT, 0, st>>>((const double2*)a, (const double2*)b, s->npw_stride, s->npw, out);
  return true;
}

bool launch_energy_sum(int norb, const double* occ, const double* red, double* energy, hipStream_t st) {
  energy_sum_kernel<<<1, 64, 0, st>>>(norb, occ, red, energy);
  return true;
}

}  // namespace ks
