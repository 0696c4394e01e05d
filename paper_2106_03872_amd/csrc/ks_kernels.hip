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
constexpr int NTP = 384; // threads per plane-pass block

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
// Block (plane pi, orbital o).  LDS: twiddles [N] | Z [ncol][N+1] | Y [YB][N+1].
// z-synthesis of each disk column straight from the packed coefficients into
// Z; y-synthesis of YB r2-columns at a time straight from Z into T.

template <int N> struct pnb { static constexpr int value = N <= 64 ? 64 : (N <= 96 ? 48 : (N <= 120 ? 24 : 16)); };

template <int N, typename R>
__global__ __launch_bounds__(NTP) void plane_inv_kernel(const cplx<R>* __restrict__ pk, int pk_stride,
                                                        cplx<R>* __restrict__ Tout, SphereTab tab,
                                                        const cplx<R>* __restrict__ twN, int ncol_max) {
  using C = cplx<R>;
  constexpr int YB = pnb<N>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  C* Z = tw + N;
  C* Y = Z + ncol_max * (N + 1);
  __shared__ int s_off[130];
  __shared__ int s_m2lo[129];
  const int pi = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int c0 = tab.plane_col0[pi], nc = tab.plane_col0[pi + 1] - c0;
  const int m1lo = tab.plane_m1lo[pi];
  for (int i = tid; i < N; i += NTP) tw[i] = twN[i];
  for (int i = tid; i <= nc; i += NTP) s_off[i] = tab.col_off[c0 + i];
  for (int i = tid; i < nc; i += NTP) s_m2lo[i] = tab.col_m2lo[c0 + i];
  __syncthreads();
  const C* in = pk + (long long)o * pk_stride;
  for (int cb = 0; cb < nc; cb += YB) {
    fft_io<N, +1, YB, NTP, SRC_FN, DST_LDS, C>(
        Z + cb * (N + 1), N + 1, nc - cb, tw,
        [&](int t, int e) -> C {
          const int c = cb + t;
          const int idx = fold(e, N) - s_m2lo[c];
          return (idx >= 0 && idx < s_off[c + 1] - s_off[c]) ? in[s_off[c] + idx] : czero<C>();
        },
        no_store{});
  }
  C* out = Tout + ((long long)o * tab.nplanes + pi) * N * N;
  for (int w0 = 0; w0 < N; w0 += YB) {
    fft_io<N, +1, YB, NTP, SRC_FN, DST_FN, C>(
        Y, N + 1, N - w0, tw,
        [&](int t, int e) -> C {
          const int c = fold(e, N) - m1lo;
          return (c >= 0 && c < nc) ? Z[c * (N + 1) + w0 + t] : czero<C>();
        },
        [&](int t, int e, C v, int, int) { out[e * N + w0 + t] = v; });
    __syncthreads();
  }
}

// ------------------------------------------------------------ plane analysis
// Block (plane pi, orbital o): y-analysis of YB r2-columns of U at a time,
// keeping the disk columns in Z; z-analysis of each column with the kinetic
// term and the output mode applied to the outputs inside the sphere.

template <int N, typename R>
__global__ __launch_bounds__(NTP) void plane_fwd_kernel(const cplx<R>* __restrict__ Uin, const cplx<R>* win,
                                                        cplx<R>* __restrict__ wout, double2* acc, int pk_stride,
                                                        int acc_stride, SphereTab tab,
                                                        const cplx<R>* __restrict__ twN, int ncol_max, int mode,
                                                        Taylor tay, double g0, double g1, double g2) {
  using C = cplx<R>;
  constexpr int YB = pnb<N>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  C* Z = tw + N;
  C* Y = Z + ncol_max * (N + 1);
  __shared__ int s_off[130];
  __shared__ int s_m2lo[129];
  const int pi = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int c0 = tab.plane_col0[pi], nc = tab.plane_col0[pi + 1] - c0;
  const int m1lo = tab.plane_m1lo[pi];
  for (int i = tid; i < N; i += NTP) tw[i] = twN[i];
  for (int i = tid; i <= nc; i += NTP) s_off[i] = tab.col_off[c0 + i];
  for (int i = tid; i < nc; i += NTP) s_m2lo[i] = tab.col_m2lo[c0 + i];
  __syncthreads();
  const C* u = Uin + ((long long)o * tab.nplanes + pi) * N * N;
  for (int w0 = 0; w0 < N; w0 += YB) {
    fft_io<N, -1, YB, NTP, SRC_FN, DST_FN, C>(
        Y, N + 1, N - w0, tw, [&](int t, int e) -> C { return u[e * N + w0 + t]; },
        [&](int t, int e, C v, int, int) {
          const int c = fold(e, N) - m1lo;
          if (c >= 0 && c < nc) Z[c * (N + 1) + w0 + t] = v;
        });
    __syncthreads();
  }
  const double k0 = g0 * (tab.m0lo + pi);
  const long long ob = (long long)o * pk_stride;
  double2* accp = acc ? acc + (long long)o * acc_stride : nullptr;
  for (int cb = 0; cb < nc; cb += YB) {
    fft_io<N, -1, YB, NTP, SRC_LDS, DST_FN, C>(
        Z + cb * (N + 1), N + 1, nc - cb, tw, no_load{}, [&](int t, int e, C ph, int, int) {
          const int c = cb + t;
          const int m2 = fold(e, N);
          const int idx = m2 - s_m2lo[c];
          if (idx < 0 || idx >= s_off[c + 1] - s_off[c]) return;
          const int ep = s_off[c] + idx;
          const double k1 = g1 * (m1lo + c), k2 = g2 * m2;
          const double K = 0.5 * (k0 * k0 + k1 * k1 + k2 * k2);
          const C w = win[ob + ep];
          const double2 hw{K * double(w.x) + double(ph.x), K * double(w.y) + double(ph.y)};
          if (mode == H_OUT) {
            wout[ob + ep] = to_c<C>(hw);
          } else {
            if (tay.write_w) wout[ob + ep] = to_c<C>(hw);
            double2 av = accp[ep];
            av.x += tay.coef.x * hw.x - tay.coef.y * hw.y;
            av.y += tay.coef.x * hw.y + tay.coef.y * hw.x;
            accp[ep] = av;
          }
        });
  }
}

// -------------------------------------------------------------- x-pencil passes
// Block (tile of NB consecutive pencils p = j1*n2 + j2, orbital o).  The
// x-synthesis reads T (planes m0 of each pencil) straight into its first
// stage; LDS X[w][j0] holds one exchange buffer of the tile.

template <int N0, int NB, typename C>
struct TLoader {
  const C* Tin;
  int npl, nplanes, m0lo, p0;
  __device__ C operator()(int t, int e) const {
    const int pi = fold(e, N0) - m0lo;
    const int p = p0 + t;
    return (pi >= 0 && pi < nplanes && p < npl) ? Tin[(long long)pi * npl + p] : czero<C>();
  }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

template <int N0, typename R>
__global__ __launch_bounds__(NT) void xproj_kernel(const cplx<R>* __restrict__ Tin, cplx<R>* __restrict__ partial,
                                                   SphereTab tab, ProjTab pt, const cplx<R>* __restrict__ tw0,
                                                   double scale) {
  using C = cplx<R>;
  constexpr int NB = xnb<N0>::value;
  __shared__ C X[NB * (N0 + 1)];
  const int tile = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int npl = tab.n1 * tab.n2;
  const int sA = pt.slot_off[tile], ns = pt.slot_off[tile + 1] - sA;
  if (ns == 0) return;  // no sphere point in this tile (uniform per block)
  const TLoader<N0, NB, C> ld{Tin + (long long)o * tab.nplanes * npl, npl, tab.nplanes, tab.m0lo, tile * NB};
  fft_io<N0, +1, NB, NT, SRC_FN, DST_LDS, C>(X, N0 + 1, NB, tw0, ld, no_store{});
  const int np = pt.nproj;
  const int wave = tid >> 6, lane = tid & 63;
  for (int sl = wave; sl < ns; sl += NT / 64) {
    const int k0 = pt.slot_pt[sA + sl], k1 = pt.slot_pt[sA + sl + 1];
    double ax[KB_MAX_NPROJ], ay[KB_MAX_NPROJ];
#pragma unroll
    for (int q = 0; q < KB_MAX_NPROJ; ++q) ax[q] = ay[q] = 0.0;
    for (int base = k0; base < k1; base += 64) {
      const int k = base + lane;
      C x = czero<C>();
      if (k < k1) x = X[pt.pt_lds[k]];
      const double* b = pt.beta + (long long)k * np;
#pragma unroll
      for (int q = 0; q < KB_MAX_NPROJ; ++q) {
        if (q < np) {
          const double bv = k < k1 ? b[q] : 0.0;
          ax[q] += wave_sum(bv * double(x.x));
          ay[q] += wave_sum(bv * double(x.y));
        }
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < KB_MAX_NPROJ; ++q)
        if (q < np) partial[((long long)o * pt.nslots + sA + sl) * np + q] = C{R(ax[q] * scale), R(ay[q] * scale)};
    }
  }
}

template <int N0, typename R>
__global__ __launch_bounds__(NT) void xapply_kernel(const cplx<R>* __restrict__ Tin, cplx<R>* __restrict__ Uout,
                                                    const double* __restrict__ V, const double2* __restrict__ DP,
                                                    SphereTab tab, ProjTab pt, const cplx<R>* __restrict__ tw0,
                                                    double sc_in, double sc_out) {
  using C = cplx<R>;
  constexpr int NB = xnb<N0>::value;
  using LS = last_shape<N0, NB, NT>;
  __shared__ C X[NB * (N0 + 1)];
  __shared__ double2 dps[KB_TILE_DP];
  const int tile = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
  const int npl = tab.n1 * tab.n2;
  const int p0 = tile * NB;
  // potential at the outputs of this thread's last synthesis stage (times Omega^-1/2)
  double vr[LS::items][LS::radix];
  last_stage_positions<N0, NB, NT>(NB, [&](int it, int q, int t, int e) {
    vr[it][q] = (p0 + t < npl) ? V[(long long)e * npl + p0 + t] * sc_in : 0.0;
  });
  const int np = pt.nproj;
  const int sA = pt.slot_off[tile], ns = pt.slot_off[tile + 1] - sA;
  for (int i = tid; i < ns * np; i += NT) {
    const int sl = i / np, q = i - sl * np;
    dps[i] = DP[((long long)o * pt.natoms + pt.slot_atom[sA + sl]) * np + q];
  }
  const TLoader<N0, NB, C> ld{Tin + (long long)o * tab.nplanes * npl, npl, tab.nplanes, tab.m0lo, p0};
  // synthesis, then psi <- V psi as the outputs are written
  fft_io<N0, +1, NB, NT, SRC_FN, DST_FN_LDS, C>(X, N0 + 1, NB, tw0, ld, [&](int t, int e, C v, int it, int q) {
    X[t * (N0 + 1) + e] = C{R(vr[it][q] * double(v.x)), R(vr[it][q] * double(v.y))};
  });
  if (ns > 0) {
    const int uA = pt.up_off[tile], uB = pt.up_off[tile + 1];
    for (int u = uA + tid; u < uB; u += NT) {
      double fx = 0.0, fy = 0.0;
      for (int e = pt.up_ent[u]; e < pt.up_ent[u + 1]; ++e) {
        const double* b = pt.beta + (long long)pt.ent_brow[e] * np;
        const double2* dp = dps + pt.ent_slot[e] * np;
        for (int q = 0; q < np; ++q) {
          fx += b[q] * dp[q].x;
          fy += b[q] * dp[q].y;
        }
      }
      C& x = X[pt.up_lds[u]];
      x = C{R(double(x.x) + fx), R(double(x.y) + fy)};
    }
    __syncthreads();
  }
  C* out = Uout + (long long)o * tab.nplanes * npl;
  const int nplanes = tab.nplanes, m0lo = tab.m0lo;
  fft_io<N0, -1, NB, NT, SRC_LDS, DST_FN, C>(X, N0 + 1, NB, tw0, no_load{}, [&](int t, int e, C v, int, int) {
    const int pi = fold(e, N0) - m0lo;
    const int p = p0 + t;
    if (pi >= 0 && pi < nplanes && p < npl)
      out[(long long)pi * npl + p] = C{R(double(v.x) * sc_out), R(double(v.y) * sc_out)};
  });
}

// density: block = tile, loops over the nb orbitals of the chunk in order;
// |psi|^2 is accumulated straight from the last synthesis stage.
template <int N0, typename R>
__global__ __launch_bounds__(NT) void xdens_kernel(const cplx<R>* __restrict__ Tin, int nb,
                                                   const double* __restrict__ occ, double* __restrict__ rho,
                                                   int accumulate, SphereTab tab, const cplx<R>* __restrict__ tw0,
                                                   double inv_omega) {
  using C = cplx<R>;
  constexpr int NB = xnb<N0>::value;
  using LS = last_shape<N0, NB, NT>;
  __shared__ C X[NB * (N0 + 1)];
  const int tile = blockIdx.x;
  const int npl = tab.n1 * tab.n2;
  const int p0 = tile * NB;
  double a[LS::items][LS::radix];
#pragma unroll
  for (int it = 0; it < LS::items; ++it)
#pragma unroll
    for (int q = 0; q < LS::radix; ++q) a[it][q] = 0.0;
  for (int o = 0; o < nb; ++o) {
    const TLoader<N0, NB, C> ld{Tin + (long long)o * tab.nplanes * npl, npl, tab.nplanes, tab.m0lo, p0};
    const double f = occ[o] * inv_omega;
    fft_io<N0, +1, NB, NT, SRC_FN, DST_FN, C>(X, N0 + 1, NB, tw0, ld, [&](int, int, C v, int it, int q) {
      a[it][q] += f * (double(v.x) * double(v.x) + double(v.y) * double(v.y));
    });
    __syncthreads();
  }
  last_stage_positions<N0, NB, NT>(NB, [&](int it, int q, int t, int e) {
    const int p = p0 + t;
    if (p < npl) {
      double* r = rho + (long long)e * npl + p;
      *r = accumulate ? *r + a[it][q] : a[it][q];
    }
  });
}

// KB projections: P_Ip = sum over the (tile, atom) slots of atom I in
// ascending order, DP = d_Ip P_Ip (Eq. vnl).  One wavefront per (atom, orbital):
// lane = 8 * slot-lane + q; slot-lanes are combined in a fixed order.
template <typename C>
__global__ __launch_bounds__(64) void proj_reduce_kernel(const C* __restrict__ partial, double2* __restrict__ DP,
                                                         ProjTab pt) {
  __shared__ double2 red[64];
  const int I = blockIdx.x, o = blockIdx.y, lane = threadIdx.x;
  const int q = lane & 7, sl = lane >> 3;
  const int np = pt.nproj;
  double sx = 0.0, sy = 0.0;
  if (q < np) {
    for (int k = pt.atom_slot_off[I] + sl; k < pt.atom_slot_off[I + 1]; k += 8) {
      const C v = partial[((long long)o * pt.nslots + pt.atom_slots[k]) * np + q];
      sx += double(v.x);
      sy += double(v.y);
    }
  }
  red[lane] = double2{sx, sy};
  __syncthreads();
  if (lane < 8 && q < np) {
    double tx = 0.0, ty = 0.0;
    for (int j = 0; j < 8; ++j) {
      tx += red[j * 8 + lane].x;
      ty += red[j * 8 + lane].y;
    }
    const double dd = pt.d[I * np + q];
    DP[((long long)o * pt.natoms + I) * np + q] = double2{dd * tx, dd * ty};
  }
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

static ProjTab proj_tab(const ks_system* s) {
  ProjTab c;
  c.pt_lds = s->d_pt_lds;
  c.slot_off = s->d_slot_off;
  c.slot_atom = s->d_slot_atom;
  c.slot_pt = s->d_slot_pt;
  c.atom_slot_off = s->d_atom_slot_off;
  c.atom_slots = s->d_atom_slots;
  c.up_off = s->d_up_off;
  c.up_lds = s->d_up_lds;
  c.up_ent = s->d_up_ent;
  c.ent_slot = s->d_ent_slot;
  c.ent_brow = s->d_ent_brow;
  c.beta = s->d_beta;
  c.d = s->d_kb;
  c.natoms = s->natoms;
  c.nproj = s->nproj;
  c.nslots = s->nslots;
  return c;
}

size_t plane_lds_bytes(const ks_system* s) {
  const int N = s->n[1];
  const int yb = N <= 64 ? 64 : (N <= 96 ? 48 : (N <= 120 ? 24 : 16));   // pnb<N>
  return sizeof(double2) * ((size_t)N + (size_t)s->ncol_max * (N + 1) + (size_t)yb * (N + 1));
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
  plane_inv_kernel<N, double><<<dim3(s->nplanes, nb), NTP, lds, st>>>(
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
  plane_fwd_kernel<N, double><<<dim3(s->nplanes, nb), NTP, lds, st>>>(
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
                                                                sphere_tab(s), proj_tab(s), s->d_tw0, scale);
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
  if (s->natoms == 0 || nb == 0) return true;
  proj_reduce_kernel<double2><<<dim3(s->natoms, nb), 64, 0, st>>>((const double2*)partial, DP, proj_tab(s));
  return true;
}

template <int N0>
static void xapply_n(const ks_system* s, int nb, const void* T, const double2* DP, void* U, hipStream_t st) {
  const double sc_in = 1.0 / sqrt(s->omega);
  const double sc_out = sqrt(s->omega) / (double)s->N;
  xapply_kernel<N0, double><<<dim3(s->ntiles, nb), NT, 0, st>>>((const double2*)T, (double2*)U, s->d_v, DP,
                                                                 sphere_tab(s), proj_tab(s), s->d_tw0, sc_in,
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
