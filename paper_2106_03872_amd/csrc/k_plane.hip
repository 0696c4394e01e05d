// Plane passes of the Kohn-Sham Hamiltonian (HIP, gfx950): per m0 plane of
// the plane-wave sphere, z- and y-synthesis into T, and y- and z-analysis of
// U with the kinetic term and the Taylor-4 epilogue (Section
// "Implementation of the KS Hamiltonian"; Section "Real-time propagation").
#include "ks_common.hpp"

namespace ks {

constexpr int EP_PRE = 4;   // packed coefficients per thread whose loads are issued ahead

// ----------------------------------------------------------- plane synthesis
// Block (plane pi, orbital group).  For each orbital of the group in order:
// its packed coefficients of the plane (contiguous, so the loads coalesce;
// fetched into registers one orbital ahead) are staged in LDS; z-synthesis of
// each disk column from the staging area into Z; y-synthesis of YB
// r2-columns at a time from Z straight into T.
// LDS: twiddles [N] | Z [ncol][N+1] | Y [YB][N+1] (the staging area of the
// packed coefficients, consumed before the y-synthesis, shares Y) | [npp_max]
// bytes (unused here).  `stage` = 0 when a plane's coefficients do not fit in
// Y: the z-synthesis then reads them from HBM directly.

// BATCH: one launch over several systems of the grid; the block's system
// (its input, T and orbital count) comes from jobs[rows[blockIdx.y].x].
template <int N, typename R, typename TIN, bool HB, bool BATCH = false>
__global__ __launch_bounds__(NTP) void plane_inv_kernel(const TIN* __restrict__ pk, int nb, int pk_stride,
                                                        cplx<R>* __restrict__ Tout, SphereTab tab,
                                                        const cplx<R>* __restrict__ twN, int ncol_max, int stage,
                                                        const BatchJob* __restrict__ jobs = nullptr,
                                                        const int4* __restrict__ rows = nullptr) {
  using C = cplx<R>;
  constexpr int YB = pnb<N>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  C* Z = tw + N;
  C* Y = Z + ncol_max * (N + 1);
  C* S = Y;
  __shared__ int s_off[130];
  __shared__ int s_m2lo[129];
  const int pi = blockIdx.x, tid = threadIdx.x;
  int oa, ob;
  if constexpr (BATCH) {
    const int4 r = rows[blockIdx.y];
    pk = static_cast<const TIN*>(jobs[r.x].win);
    Tout = static_cast<cplx<R>*>(jobs[r.x].T);
    nb = jobs[r.x].nb;
    group_range(nb, r.y, r.z, oa, ob);
  } else {
    orbital_range(nb, oa, ob);
  }
  const int c0 = tab.plane_col0[pi], nc = tab.plane_col0[pi + 1] - c0;
  const int m1lo = tab.plane_m1lo[pi];
  for (int i = tid; i < N; i += NTP) tw[i] = twN[i];
  for (int i = tid; i <= nc; i += NTP) s_off[i] = tab.col_off[c0 + i];
  for (int i = tid; i < nc; i += NTP) s_m2lo[i] = tab.col_m2lo[c0 + i];
  const int e0 = tab.col_off[c0], npp = tab.col_off[c0 + nc] - e0;
  // this thread's first EP_PRE coefficients of the next orbital
  TIN cin[EP_PRE];
  auto fetch = [&](int o) {
    const TIN* in = pk + (long long)o * pk_stride + e0;
#pragma unroll
    for (int j = 0; j < EP_PRE; ++j) {
      const int k = tid + j * NTP;
      if (k < npp) cin[j] = in[k];
    }
  };
  if (stage && oa < ob) fetch(oa);
  __syncthreads();
  for (int o = oa; o < ob; ++o) {
    const TIN* in = pk + (long long)o * pk_stride;
    if (stage) {
#pragma unroll
      for (int j = 0; j < EP_PRE; ++j) {
        const int k = tid + j * NTP;
        if (k < npp) S[k] = cvt<C>(cin[j]);
      }
      for (int k = tid + EP_PRE * NTP; k < npp; k += NTP) S[k] = cvt<C>(in[e0 + k]);
      if (o + 1 < ob) fetch(o + 1);
      __syncthreads();
      for (int cb = 0; cb < nc; cb += YB) {
        auto load = [&](int t, int e) -> C {
          const int c = cb + t;
          const int idx = fold(e, N) - s_m2lo[c];
          return (idx >= 0 && idx < s_off[c + 1] - s_off[c]) ? S[s_off[c] - e0 + idx] : czero<C>();
        };
        if constexpr (HB) fft_io<N, +1, YB, NTP, SRC_FN, DST_LDS, C>(Z + cb * (N + 1), N + 1, nc - cb, tw, banded(load), no_store{});
        else fft_io<N, +1, YB, NTP, SRC_FN, DST_LDS, C>(Z + cb * (N + 1), N + 1, nc - cb, tw, load, no_store{});
      }
    } else {
      for (int cb = 0; cb < nc; cb += YB) {
        auto load = [&](int t, int e) -> C {
          const int c = cb + t;
          const int idx = fold(e, N) - s_m2lo[c];
          return (idx >= 0 && idx < s_off[c + 1] - s_off[c]) ? cvt<C>(in[s_off[c] + idx]) : czero<C>();
        };
        if constexpr (HB) fft_io<N, +1, YB, NTP, SRC_FN, DST_LDS, C>(Z + cb * (N + 1), N + 1, nc - cb, tw, banded(load), no_store{});
        else fft_io<N, +1, YB, NTP, SRC_FN, DST_LDS, C>(Z + cb * (N + 1), N + 1, nc - cb, tw, load, no_store{});
      }
    }
    C* out = Tout + ((long long)o * tab.nplanes + pi) * N * N;
    for (int w0 = 0; w0 < N; w0 += YB) {
      auto load = [&](int t, int e) -> C {
        const int c = fold(e, N) - m1lo;
        return (c >= 0 && c < nc) ? Z[c * (N + 1) + w0 + t] : czero<C>();
      };
      auto store = [&](int t, int e, C v, int, int) { st_stream(out + e * N + w0 + t, v); };
      if constexpr (HB) fft_io<N, +1, YB, NTP, SRC_FN, DST_FN, C>(Y, N + 1, N - w0, tw, banded(load), store);
      else fft_io<N, +1, YB, NTP, SRC_FN, DST_FN, C>(Y, N + 1, N - w0, tw, load, store);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ plane analysis
// Block (plane pi, orbital group).  For each orbital of the group in order:
// y-analysis of YB r2-columns of U at a time into the disk columns Z; the
// z-analysis of every column in place; then the epilogue over the plane's
// packed coefficients, which are contiguous, so its loads and stores
// coalesce: + 1/2|G|^2 c and the output mode.  The next U chunk (also across
// orbitals) is loaded while the current one is transformed, and an orbital's
// epilogue operands are loaded before its transforms.
// LDS: twiddles [N] | Z [ncol][N+1] | Y [YB][N+1] | column of each packed
// coefficient of the plane [npp_max] (bytes).

// BATCH: as plane_inv_kernel; U, win, wout, acc and the orbital count come
// from the block's job (no second accumulator).
template <int N, typename R, typename TW, bool HB, bool BATCH = false>
__global__ __launch_bounds__(NTP) void plane_fwd_kernel(const cplx<R>* __restrict__ Uin, int nb, const TW* win,
                                                        cplx<R>* __restrict__ wout, double2* acc, double2* acc2,
                                                        int pk_stride,
                                                        int acc_stride, SphereTab tab,
                                                        const cplx<R>* __restrict__ twN, int ncol_max, int mode,
                                                        Taylor tay, double g0, double g1, double g2,
                                                        const BatchJob* __restrict__ jobs = nullptr,
                                                        const int4* __restrict__ rows = nullptr) {
  using C = cplx<R>;
  constexpr int YB = pnb<N>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  C* Z = tw + N;
  C* Y = Z + ncol_max * (N + 1);
  unsigned char* s_col = reinterpret_cast<unsigned char*>(Y + YB * (N + 1));
  __shared__ int s_off[130];
  __shared__ int s_m2lo[129];
  const int pi = blockIdx.x, tid = threadIdx.x;
  int oa, ob;
  if constexpr (BATCH) {
    const int4 r = rows[blockIdx.y];
    Uin = static_cast<const cplx<R>*>(jobs[r.x].U);
    win = static_cast<const TW*>(jobs[r.x].win);
    wout = static_cast<cplx<R>*>(jobs[r.x].wout);
    acc = jobs[r.x].acc;
    acc2 = nullptr;
    nb = jobs[r.x].nb;
    group_range(nb, r.y, r.z, oa, ob);
  } else {
    orbital_range(nb, oa, ob);
  }
  const int c0 = tab.plane_col0[pi], nc = tab.plane_col0[pi + 1] - c0;
  const int m1lo = tab.plane_m1lo[pi];
  for (int i = tid; i < N; i += NTP) tw[i] = twN[i];
  for (int i = tid; i <= nc; i += NTP) s_off[i] = tab.col_off[c0 + i];
  for (int i = tid; i < nc; i += NTP) s_m2lo[i] = tab.col_m2lo[c0 + i];
  __syncthreads();
  const int e0 = s_off[0], npp = s_off[nc] - e0;
  for (int c = tid; c < nc; c += NTP)
    for (int k = s_off[c]; k < s_off[c + 1]; ++k) s_col[k - e0] = (unsigned char)c;
  const double k0 = g0 * (tab.m0lo + pi);
  const long long uplane = (long long)tab.nplanes * N * N;
  using FR = fft_regs<N, YB, NTP, C>;
  FR pre;
  if (oa < ob) {
    const C* u = Uin + ((long long)oa * tab.nplanes + pi) * N * N;
    fft_preload<N, YB, NTP, C>(pre, N, [&](int t, int e) -> C { return ld_stream(u + e * N + t); });
  }
  __syncthreads();
  for (int o = oa; o < ob; ++o) {
    const C* u = Uin + ((long long)o * tab.nplanes + pi) * N * N;
    const long long obase = (long long)o * pk_stride + e0;
    double2* accp = acc ? acc + (long long)o * acc_stride + e0 : nullptr;
    double2* acc2p = acc2 ? acc2 + (long long)o * acc_stride + e0 : nullptr;
    // epilogue operands of this orbital
    TW wv[EP_PRE];
    double2 av[EP_PRE];
#pragma unroll
    for (int j = 0; j < EP_PRE; ++j) {
      const int k = tid + j * NTP;
      if (k < npp) {
        wv[j] = win[obase + k];
        if (mode != H_OUT) av[j] = accp[k];
      }
    }
    for (int w0 = 0; w0 < N; w0 += YB) {
      const int w1 = w0 + YB;
      auto next = [&] {
        if (w1 < N) {
          fft_preload<N, YB, NTP, C>(pre, N - w1, [&](int t, int e) -> C { return ld_stream(u + e * N + w1 + t); });
        } else if (o + 1 < ob) {
          const C* un = u + uplane;
          fft_preload<N, YB, NTP, C>(pre, N, [&](int t, int e) -> C { return ld_stream(un + e * N + t); });
        }
      };
      auto store = [&](int t, int e, C v, int, int) {
        const int c = fold(e, N) - m1lo;
        if (c >= 0 && c < nc) Z[c * (N + 1) + w0 + t] = v;
      };
      if constexpr (HB) fft_io<N, -1, YB, NTP, SRC_PRE, DST_FN, C>(Y, N + 1, N - w0, tw, preloaded(pre, next), banded(store));
      else fft_io<N, -1, YB, NTP, SRC_PRE, DST_FN, C>(Y, N + 1, N - w0, tw, preloaded(pre, next), store);
      __syncthreads();
    }
    // z-analysis in place; with HB only the band |m2| < n2/4, which holds every column's run, is written
    for (int cb = 0; cb < nc; cb += YB) {
      C* zb = Z + cb * (N + 1);
      if constexpr (HB)
        fft_io<N, -1, YB, NTP, SRC_LDS, DST_FN_LDS, C>(zb, N + 1, nc - cb, tw, no_load{},
                                                     banded([&](int t, int e, C v, int, int) { zb[t * (N + 1) + e] = v; }));
      else
        fft_batch<N, -1, YB, NTP, C>(zb, N + 1, nc - cb, tw);
    }
    // the second accumulator (ETRS predictor) is read where it is updated,
    // so the common single-accumulator path keeps its registers
    auto epilogue = [&](int k, TW w, double2 av_in) {
      const int c = s_col[k];
      const int m2 = s_m2lo[c] + (k + e0 - s_off[c]);
      const C ph = Z[c * (N + 1) + wrap(m2, N)];
      const double k1 = g1 * (m1lo + c), k2 = g2 * m2;
      const double K = 0.5 * (k0 * k0 + k1 * k1 + k2 * k2);
      const double2 hw{K * double(w.x) + double(ph.x), K * double(w.y) + double(ph.y)};
      if (mode == H_OUT) {
        wout[obase + k] = to_c<C>(hw);
      } else {
        if (tay.write_w) wout[obase + k] = to_c<C>(hw);
        double2 a = av_in;
        a.x += tay.coef.x * hw.x - tay.coef.y * hw.y;
        a.y += tay.coef.x * hw.y + tay.coef.y * hw.x;
        accp[k] = a;
        if (acc2p) {
          double2 b = acc2p[k];
          b.x += tay.coef2.x * hw.x - tay.coef2.y * hw.y;
          b.y += tay.coef2.x * hw.y + tay.coef2.y * hw.x;
          acc2p[k] = b;
        }
      }
    };
#pragma unroll
    for (int j = 0; j < EP_PRE; ++j) {
      const int k = tid + j * NTP;
      if (k < npp) epilogue(k, wv[j], mode != H_OUT ? av[j] : double2{0.0, 0.0});
    }
    for (int k = tid + EP_PRE * NTP; k < npp; k += NTP)
      epilogue(k, win[obase + k], mode != H_OUT ? accp[k] : double2{0.0, 0.0});
    __syncthreads();   // Z is rewritten by the next orbital
  }
}

// ------------------------------------------------------------------ launchers

size_t plane_lds_bytes(const ks_system* s) {
  const int N = s->n[1];
  const int yb = N <= 64 ? 64 : (N <= 96 ? 48 : (N <= 120 ? 24 : 16));   // pnb<N>
  const size_t es = s->prec == KS_FP64 ? sizeof(double2) : sizeof(float2);
  return es * ((size_t)N + (size_t)s->ncol_max * (N + 1) + (size_t)yb * (N + 1)) + ((size_t)s->npp_max + 15) / 16 * 16;
}

// Orbital groups per plane-pass launch: up to pg_max orbitals per block,
// fewer when the launch would have fewer than about 4 blocks per CU.
static int plane_groups(const ks_system* s, int nb) {
  long long g = (long long)s->nplanes * nb / (256 * 4);
  g = g < 1 ? 1 : (g > s->pg_max ? s->pg_max : g);
  return (int)((nb + g - 1) / g);
}

// Batched launches pass (rows, jobs, nrows): the grid's y extent is nrows
// and every per-system argument comes from the jobs; nb and the pointers
// below are then unused.
struct BatchRef {
  const BatchJob* jobs = nullptr;
  const int4* rows = nullptr;
  int nrows = 0;
};

template <int N, typename R, typename TIN, bool B>
static void plane_inv_t(const ks_system* s, int nb, const void* pk, void* T, const void* tw, const BatchRef& b,
                        hipStream_t st) {
  constexpr int YB = pnb<N>::value;
  const int stage = s->npp_max <= YB * (N + 1) ? 1 : 0;
  const dim3 grid(s->nplanes, B ? b.nrows : plane_groups(s, nb));
  if (s->yz_half)
    plane_inv_kernel<N, R, TIN, true, B><<<grid, NTP, plane_lds_bytes(s), st>>>(
        (const TIN*)pk, nb, s->npw_stride, (cplx<R>*)T, sphere_tab(s), (const cplx<R>*)tw, s->ncol_max, stage, b.jobs,
        b.rows);
  else
    plane_inv_kernel<N, R, TIN, false, B><<<grid, NTP, plane_lds_bytes(s), st>>>(
        (const TIN*)pk, nb, s->npw_stride, (cplx<R>*)T, sphere_tab(s), (const cplx<R>*)tw, s->ncol_max, stage, b.jobs,
        b.rows);
}

template <int N, bool B>
static void plane_inv_n(const ks_system* s, int nb, const void* pk, bool in_fp64, void* T, const BatchRef& b,
                        hipStream_t st) {
  if (!mixed(s)) plane_inv_t<N, double, double2, B>(s, nb, pk, T, s->d_tw1, b, st);
  else if (in_fp64) plane_inv_t<N, float, double2, B>(s, nb, pk, T, s->d_tw1f, b, st);
  else plane_inv_t<N, float, float2, B>(s, nb, pk, T, s->d_tw1f, b, st);
}

bool launch_plane_inv(const ks_system* s, int nb, const void* pk, bool in_fp64, void* T, hipStream_t st) {
  switch (s->n[1]) {
#define KS_CASE(v) case v: plane_inv_n<v, false>(s, nb, pk, in_fp64, T, BatchRef{}, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

bool launch_plane_inv_batch(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, bool in_fp64,
                            hipStream_t st) {
  const BatchRef b{jobs, rows, nrows};
  switch (s->n[1]) {
#define KS_CASE(v) case v: plane_inv_n<v, true>(s, 0, nullptr, in_fp64, nullptr, b, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

template <int N, typename R, typename TW, bool B>
static void plane_fwd_t(const ks_system* s, int nb, const void* U, const void* win, void* wout, void* acc, void* acc2,
                        HMode mode, Taylor tay, const void* tw, const BatchRef& b, hipStream_t st) {
  const double g0 = 2.0 * M_PI / s->L[0], g1 = 2.0 * M_PI / s->L[1], g2 = 2.0 * M_PI / s->L[2];
  const dim3 grid(s->nplanes, B ? b.nrows : plane_groups(s, nb));
  if (s->yz_half)
    plane_fwd_kernel<N, R, TW, true, B><<<grid, NTP, plane_lds_bytes(s), st>>>(
        (const cplx<R>*)U, nb, (const TW*)win, (cplx<R>*)wout, (double2*)acc, (double2*)acc2, s->npw_stride, s->npw_stride,
        sphere_tab(s), (const cplx<R>*)tw, s->ncol_max, (int)mode, tay, g0, g1, g2, b.jobs, b.rows);
  else
    plane_fwd_kernel<N, R, TW, false, B><<<grid, NTP, plane_lds_bytes(s), st>>>(
        (const cplx<R>*)U, nb, (const TW*)win, (cplx<R>*)wout, (double2*)acc, (double2*)acc2, s->npw_stride, s->npw_stride,
        sphere_tab(s), (const cplx<R>*)tw, s->ncol_max, (int)mode, tay, g0, g1, g2, b.jobs, b.rows);
}

template <int N, bool B>
static void plane_fwd_n(const ks_system* s, int nb, const void* U, const void* win, bool win_fp64, void* wout,
                        void* acc, void* acc2, HMode mode, Taylor tay, const BatchRef& b, hipStream_t st) {
  if (!mixed(s)) plane_fwd_t<N, double, double2, B>(s, nb, U, win, wout, acc, acc2, mode, tay, s->d_tw1, b, st);
  else if (win_fp64) plane_fwd_t<N, float, double2, B>(s, nb, U, win, wout, acc, acc2, mode, tay, s->d_tw1f, b, st);
  else plane_fwd_t<N, float, float2, B>(s, nb, U, win, wout, acc, acc2, mode, tay, s->d_tw1f, b, st);
}

bool launch_plane_fwd(const ks_system* s, int nb, const void* U, const void* win, bool win_fp64, void* wout,
                      void* acc, void* acc2, HMode mode, Taylor tay, hipStream_t st) {
  switch (s->n[1]) {
#define KS_CASE(v) case v: plane_fwd_n<v, false>(s, nb, U, win, win_fp64, wout, acc, acc2, mode, tay, BatchRef{}, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

bool launch_plane_fwd_batch(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, bool win_fp64,
                            Taylor tay, hipStream_t st) {
  const BatchRef b{jobs, rows, nrows};
  switch (s->n[1]) {
#define KS_CASE(v) case v: plane_fwd_n<v, true>(s, 0, nullptr, nullptr, win_fp64, nullptr, nullptr, nullptr, H_TAYLOR, tay, b, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

int plane_group_size(const ks_system* s, long long total_orbitals) {
  long long g = (long long)s->nplanes * total_orbitals / (256 * 4);
  return (int)(g < 1 ? 1 : (g > s->pg_max ? s->pg_max : g));
}

}  // namespace ks
