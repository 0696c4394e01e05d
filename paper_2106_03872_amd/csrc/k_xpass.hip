// x-pencil passes of the Kohn-Sham Hamiltonian (HIP, gfx950): x-synthesis
// in LDS, Kleinman-Bylander projections (Eq. vnl), local potential and KB
// scatter, x-analysis; the density sum (Eq. density).
#include "ks_common.hpp"

namespace ks {

// -------------------------------------------------------------- x-pencil passes
// Block (tile of NB consecutive pencils p = j1*n2 + j2, orbital o).  The
// x-synthesis reads T (planes m0 of each pencil) straight into its first
// stage; LDS X[w][j0] holds one exchange buffer of the tile.

template <int N0, int NB, typename C>
struct TLoader {
  const C* base;   // T of this orbital at the tile's first pencil
  int npl, nplanes, m0lo, tvalid;
  __device__ TLoader(const C* Tin, int o, int npl_, int nplanes_, int m0lo_, int p0)
      : base(Tin + ((long long)o * nplanes_ * npl_ + p0)), npl(npl_), nplanes(nplanes_), m0lo(m0lo_),
        tvalid(npl_ - p0) {}
  __device__ C operator()(int t, int e) const {
    const int pi = fold(e, N0) - m0lo;
    return (pi >= 0 && pi < nplanes && t < tvalid) ? ld_stream(base + (unsigned)(pi * npl + t)) : czero<C>();
  }
};

// x from another lane of the same row of 16 by the DPP permutation CTRL
// (quad_perm, row_half_mirror, row_mirror: every source lane is in the row)
template <int CTRL>
__device__ __forceinline__ double dpp_lane(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
constexpr int DPP_QUAD_XOR1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_XOR2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;

// Orbital groups: block (tile, y) handles the orbitals [y*nb/ng, (y+1)*nb/ng)
// of its tile in order (ng = gridDim.y).  The next orbital's T is loaded into
// registers while the current one is transformed, and the per-tile data
// (twiddles, potential, KB tables) is fetched once per block.

// DENS: the block also accumulates the density sum_o occ_o |psi_o|^2 / Omega
// of its orbitals from the synthesis outputs and writes its group's partial
// density (as xdens does), so a propagation step gets the density of its
// input orbitals from its first H psi.
// BATCH: one launch over several systems of the grid (no density); the
// block's system (T, partial sums, projector tables, orbital count) comes
// from jobs[rows[blockIdx.y].x].
template <int N0, class SH, typename R, bool HB, bool DENS, bool BATCH = false>
__global__ __launch_bounds__(SH::XT) void xproj_kernel(const cplx<R>* __restrict__ Tin, int nb,
                                                   cplx<R>* __restrict__ partial, SphereTab tab, ProjTab pt,
                                                   const cplx<R>* __restrict__ tw0, double scale,
                                                   const double* __restrict__ occ, double* __restrict__ dpart,
                                                   double inv_omega, const BatchJob* __restrict__ jobs = nullptr,
                                                   const int4* __restrict__ rows = nullptr) {
  using C = cplx<R>;
  static_assert(!(BATCH && DENS), "batched launches carry no density");
  constexpr int NB = SH::NB, XT = SH::XT;
  using FR = fft_regs<N0, NB, XT, C, HB, SH::V>;
  using LS = last_shape<N0, NB, XT, SH::V>;
  __shared__ C X[NB * (N0 + 1)];
  __shared__ C tw[N0];
  const int tile = blockIdx.x, tid = threadIdx.x;
  int oa, ob;
  if constexpr (BATCH) {
    const int4 r = rows[blockIdx.y];
    Tin = static_cast<const C*>(jobs[r.x].T);
    partial = static_cast<C*>(jobs[r.x].partial);
    pt = jobs[r.x].pt;
    nb = jobs[r.x].nb;
    group_range(nb, r.y, r.z, oa, ob);
  } else {
    orbital_range(nb, oa, ob);
  }
  const int npl = tab.n1 * tab.n2;
  const int p0 = tile * NB;
  const int sA = pt.slot_off[tile], ns = pt.slot_off[tile + 1] - sA;
  if (!DENS && ns == 0) return;  // no sphere point in this tile (uniform per block)
  for (int i = tid; i < N0; i += XT) tw[i] = tw0[i];
  double a[DENS ? LS::items : 1][DENS ? LS::radix : 1];
  if constexpr (DENS) {
#pragma unroll
    for (int it = 0; it < LS::items; ++it)
#pragma unroll
      for (int q = 0; q < LS::radix; ++q) a[it][q] = 0.0;
  }
  // Projections: each lane sums beta * psi over its rows [ka, kb) of one
  // (slot, projector) pair of the tile (in point order); the 2^g lanes of a
  // pair, adjacent and aligned, are then added by a fixed butterfly and the
  // group's first lane writes the pair (work planned per tile on the host).
  // (the host plans XT projection lanes per tile)
  const int np = pt.nproj;
  const int4 item = pt.item[(long long)tile * XT + tid];
  const int ka = item.x, kb = item.y;
  const int sl = item.z / np, kq = item.z - sl * np;
  const int glanes = 1 << (item.w & 0xff);
  const bool writer = (item.w & 256) != 0;
  // The first KP points of the item (LDS position, beta) are the same for
  // all orbitals of the block and stay in registers.
  constexpr int KP = KB_CACHED_POINTS;
  int cpos[KP];
  double cbeta[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) {
    const int k = ka + c;
    const bool in = k < kb;
    cpos[c] = in ? pt.pt_lds[k] : 0;
    cbeta[c] = in ? pt.beta[(long long)k * np + kq] : 0.0;
  }
  C* pout = partial + (long long)(sA + sl) * np + kq;
  const long long pstride = (long long)pt.nslots * np;
  FR pre;
  if (oa < ob) fft_preload_regs(pre, NB, TLoader<N0, NB, C>(Tin, oa, npl, tab.nplanes, tab.m0lo, p0));
  for (int o = oa; o < ob; ++o) {
    auto next = [&] {
      if (o + 1 < ob)
        fft_preload_regs(pre, NB, TLoader<N0, NB, C>(Tin, o + 1, npl, tab.nplanes, tab.m0lo, p0));
    };
    if constexpr (DENS) {
      const double f = occ[o] * inv_omega;
      fft_io<N0, +1, NB, XT, SRC_PRE, DST_FN_LDS, C, SH::V>(X, N0 + 1, NB, tw, preloaded(pre, next),
                                                   [&](int t, int e, C v, int it, int q) {
                                                     X[t * (N0 + 1) + e] = v;
                                                     a[it][q] += f * (double(v.x) * double(v.x) + double(v.y) * double(v.y));
                                                   });
      if (ns == 0) {
        __syncthreads();   // X is rewritten by the next orbital's first stage
        continue;
      }
    } else {
      fft_io<N0, +1, NB, XT, SRC_PRE, DST_LDS, C, SH::V>(X, N0 + 1, NB, tw, preloaded(pre, next), no_store{});
    }
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int c = 0; c < KP; ++c) {
      if (ka + c < kb) {
        const C x = X[cpos[c]];
        sx += cbeta[c] * double(x.x);
        sy += cbeta[c] * double(x.y);
      }
    }
    for (int k = ka + KP; k < kb; ++k) {
      const double bv = pt.beta[(long long)k * np + kq];
      const C x = X[pt.pt_lds[k]];
      sx += bv * double(x.x);
      sy += bv * double(x.y);
    }
    // the group's lanes add their sums by a fixed butterfly (the partners of
    // stage m: lane pairs of a quad, then quads, then mirrored halves of 8 and
    // of 16 lanes; after stage m every lane of an aligned 2m-lane block holds
    // the block's sum, as with lane index xor m)
    static_assert(KB_MAX_GROUP_LOG == 4, "four butterfly stages");
    {
      double vx = dpp_lane<DPP_QUAD_XOR1>(sx), vy = dpp_lane<DPP_QUAD_XOR1>(sy);
      if (glanes > 1) {
        sx += vx;
        sy += vy;
      }
      vx = dpp_lane<DPP_QUAD_XOR2>(sx);
      vy = dpp_lane<DPP_QUAD_XOR2>(sy);
      if (glanes > 2) {
        sx += vx;
        sy += vy;
      }
      vx = dpp_lane<DPP_HALF_MIRROR>(sx);
      vy = dpp_lane<DPP_HALF_MIRROR>(sy);
      if (glanes > 4) {
        sx += vx;
        sy += vy;
      }
      vx = dpp_lane<DPP_MIRROR>(sx);
      vy = dpp_lane<DPP_MIRROR>(sy);
      if (glanes > 8) {
        sx += vx;
        sy += vy;
      }
    }
    if (writer) pout[o * pstride] = C{R(sx * scale), R(sy * scale)};
    __syncthreads();   // X is rewritten by the next orbital's first stage
  }
  if constexpr (DENS) {
    double* pb = dpart + (long long)blockIdx.y * tab.n0 * npl + p0;
    last_stage_positions<N0, NB, XT, SH::V>(NB, [&](int it, int q, int t, int e) {
      if (p0 + t < npl) pb[e * npl + t] = a[it][q];
    });
  }
}

// KB scatter (Eq. vnl): X[point] += sum over the point's entries (in atom
// order) of beta_entry . dP[slot].
template <typename C>
__device__ __forceinline__ void kb_add(C* X, int key, double fx, double fy) {
  C& x = X[key & ((1 << UP_POS_BITS) - 1)];
  x = C{decltype(x.x)(double(x.x) + fx), decltype(x.x)(double(x.y) + fy)};
}

// extra entries of a point where spheres overlap (rare)
__device__ __forceinline__ void kb_extra(const double2* dps, const ProjTab& pt, int np, int u, int key, double& fx,
                                         double& fy) {
  const int nx = key >> (UP_POS_BITS + UP_SLOT_BITS);
  if (nx == 0) return;
  const int x0 = pt.up_x[u];
  for (int e = x0; e < x0 + nx; ++e) {
    const double* b = pt.x_beta + (long long)e * np;
    const double2* dp = dps + pt.x_slot[e] * np;
    for (int q = 0; q < np; ++q) {
      fx += b[q] * dp[q].x;
      fy += b[q] * dp[q].y;
    }
  }
}

// NP projectors per atom fixed at compile time: two unique points per thread
// and pass, u and u + XT, with the table loads of both issued before either
// is used.
template <int NP, int XT, typename C>
__device__ __forceinline__ void kb_scatter_fixed(C* X, const double2* dps, const ProjTab& pt, int uA, int uB) {
  const int tid = threadIdx.x;
  for (int u = uA + tid; u < uB; u += 2 * XT) {
    const int ub = u + XT;
    const bool two = ub < uB;
    const int ka = pt.up_key[u];
    const int kb = two ? pt.up_key[ub] : 0;
    double ba[NP], bb[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      ba[q] = pt.up_beta[(long long)u * NP + q];
      bb[q] = two ? pt.up_beta[(long long)ub * NP + q] : 0.0;
    }
    const double2* da = dps + ((ka >> UP_POS_BITS) & UP_MAX_SLOT) * NP;
    const double2* db = dps + ((kb >> UP_POS_BITS) & UP_MAX_SLOT) * NP;
    double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const double2 pa = da[q], pb = db[q];
      ax += ba[q] * pa.x;
      ay += ba[q] * pa.y;
      bx += bb[q] * pb.x;
      by += bb[q] * pb.y;
    }
    kb_extra(dps, pt, NP, u, ka, ax, ay);
    kb_add(X, ka, ax, ay);
    if (two) {
      kb_extra(dps, pt, NP, ub, kb, bx, by);
      kb_add(X, kb, bx, by);
    }
  }
}

// any number of projectors per atom: one point at a time
template <int XT, typename C>
__device__ __forceinline__ void kb_scatter_any(C* X, const double2* dps, const ProjTab& pt, int uA, int uB) {
  const int np = pt.nproj, tid = threadIdx.x;
  for (int u = uA + tid; u < uB; u += XT) {
    const int key = pt.up_key[u];
    const double* b = pt.up_beta + (long long)u * np;
    const double2* dp = dps + ((key >> UP_POS_BITS) & UP_MAX_SLOT) * np;
    double fx = 0.0, fy = 0.0;
    for (int q = 0; q < np; ++q) {
      fx += b[q] * dp[q].x;
      fy += b[q] * dp[q].y;
    }
    kb_extra(dps, pt, np, u, key, fx, fy);
    kb_add(X, key, fx, fy);
  }
}

// BATCH: as xproj_kernel (T, U, V, d P, projector tables and orbital count
// from the block's job).
template <int N0, class SH, typename R, bool HB, bool BATCH = false>
__global__ __launch_bounds__(SH::XT) void xapply_kernel(const cplx<R>* __restrict__ Tin, int nb,
                                                    cplx<R>* __restrict__ Uout, const double* __restrict__ V,
                                                    const double2* __restrict__ DP, SphereTab tab, ProjTab pt,
                                                    const cplx<R>* __restrict__ tw0, double sc_v,
                                                    const BatchJob* __restrict__ jobs = nullptr,
                                                    const int4* __restrict__ rows = nullptr) {
  using C = cplx<R>;
  constexpr int NB = SH::NB, XT = SH::XT;
  using LS = last_shape<N0, NB, XT, SH::V>;
  using FR = fft_regs<N0, NB, XT, C, HB, SH::V>;
  __shared__ C X[NB * (N0 + 1)];
  __shared__ double2 dps[KB_TILE_DP];
  __shared__ C tw[N0];
  const int tile = blockIdx.x, tid = threadIdx.x;
  int oa, ob;
  if constexpr (BATCH) {
    const int4 r = rows[blockIdx.y];
    Tin = static_cast<const C*>(jobs[r.x].T);
    Uout = static_cast<C*>(jobs[r.x].U);
    V = jobs[r.x].V;
    DP = jobs[r.x].DP;
    pt = jobs[r.x].pt;
    nb = jobs[r.x].nb;
    group_range(nb, r.y, r.z, oa, ob);
  } else {
    orbital_range(nb, oa, ob);
  }
  for (int i = tid; i < N0; i += XT) tw[i] = tw0[i];
  const int npl = tab.n1 * tab.n2;
  const int p0 = tile * NB;
  // potential at the outputs of this thread's last synthesis stage, times the
  // synthesis and analysis scales Omega^-1/2 Omega^1/2 / N = 1/N
  double vr[LS::items][LS::radix];
  const double* vbase = V + p0;
  last_stage_positions<N0, NB, XT, SH::V>(NB, [&](int it, int q, int t, int e) {
    vr[it][q] = (p0 + t < npl) ? vbase[e * npl + t] * sc_v : 0.0;
  });
  // KB coefficients d*P of this tile's slots: thread tid < ns*np stages one
  // (slot, projector) value per orbital.
  const int np = pt.nproj;
  const int sA = pt.slot_off[tile], ns = pt.slot_off[tile + 1] - sA;
  const int ndp = ns * np;   // <= KB_TILE_DP <= XT
  const long long dp_stride = (long long)pt.natoms * np;
  long long dp_off = 0;
  if (tid < ndp) {
    const int sl = tid / np, q = tid - sl * np;
    dp_off = (long long)pt.slot_atom[sA + sl] * np + q;
  }
  const int uA = pt.up_off[tile], uB = pt.up_off[tile + 1];
  const int nplanes = tab.nplanes, m0lo = tab.m0lo;
  const int tvalid = npl - p0;
  FR pre;
  if (oa < ob) fft_preload_regs(pre, NB, TLoader<N0, NB, C>(Tin, oa, npl, nplanes, m0lo, p0));
  double2 dnext = {0.0, 0.0};
  if (tid < ndp && oa < ob) dnext = DP[oa * dp_stride + dp_off];
  for (int o = oa; o < ob; ++o) {
    // this orbital's d*P (fetched one orbital ahead); the previous orbital's
    // scatter has finished reading dps, and the stage barriers publish it
    if (tid < ndp) dps[tid] = dnext;
    auto next = [&] {
      if (o + 1 < ob) {
        fft_preload_regs(pre, NB, TLoader<N0, NB, C>(Tin, o + 1, npl, nplanes, m0lo, p0));
        if (tid < ndp) dnext = DP[(o + 1) * dp_stride + dp_off];
      }
    };
    // synthesis, then psi <- V psi as the outputs are written
    fft_io<N0, +1, NB, XT, SRC_PRE, DST_FN_LDS, C, SH::V>(X, N0 + 1, NB, tw, preloaded(pre, next), [&](int t, int e, C v, int it, int q) {
      X[t * (N0 + 1) + e] = C{R(vr[it][q] * double(v.x)), R(vr[it][q] * double(v.y))};
    });
    if (ns > 0) {
      if (np == 4) kb_scatter_fixed<4, XT>(X, dps, pt, uA, uB);
      else kb_scatter_any<XT>(X, dps, pt, uA, uB);
      __syncthreads();
    }
    C* obase = Uout + (long long)o * nplanes * npl + p0;
    auto store = [&](int t, int e, C v, int, int) {
      const int pi = fold(e, N0) - m0lo;
      if (pi >= 0 && pi < nplanes && t < tvalid) st_stream(obase + (unsigned)(pi * npl + t), v);
    };
    // only the sphere's planes are stored; with HB they all lie in the band |m0| < n0/4
    if constexpr (HB) fft_io<N0, -1, NB, XT, SRC_LDS, DST_FN, C, SH::V>(X, N0 + 1, NB, tw, no_load{}, banded(store));
    else fft_io<N0, -1, NB, XT, SRC_LDS, DST_FN, C, SH::V>(X, N0 + 1, NB, tw, no_load{}, store);
    __syncthreads();   // X and dps are rewritten for the next orbital
  }
}

// density: block (tile, orbital group); |psi|^2 is accumulated
// straight from the last synthesis stage over the group's orbitals in order
// and written to the group's partial density; dens_sum adds the groups in
// order.
template <int N0, class SH, typename R, bool HB>
__global__ __launch_bounds__(SH::XT) void xdens_kernel(const cplx<R>* __restrict__ Tin, int nb,
                                                   const double* __restrict__ occ, double* __restrict__ part,
                                                   SphereTab tab, const cplx<R>* __restrict__ tw0,
                                                   double inv_omega) {
  using C = cplx<R>;
  constexpr int NB = SH::NB, XT = SH::XT;
  using LS = last_shape<N0, NB, XT, SH::V>;
  __shared__ C X[NB * (N0 + 1)];
  __shared__ C tw[N0];
  const int tile = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
  const int npl = tab.n1 * tab.n2;
  const int p0 = tile * NB;
  for (int i = tid; i < N0; i += XT) tw[i] = tw0[i];
  double a[LS::items][LS::radix];
#pragma unroll
  for (int it = 0; it < LS::items; ++it)
#pragma unroll
    for (int q = 0; q < LS::radix; ++q) a[it][q] = 0.0;
  int oa, ob;
  orbital_range(nb, oa, ob);
  // the next orbital's T is loaded once the first stage has consumed the current one
  using FR = fft_regs<N0, NB, XT, C, HB, SH::V>;
  FR pre;
  if (oa < ob) fft_preload_regs(pre, NB, TLoader<N0, NB, C>(Tin, oa, npl, tab.nplanes, tab.m0lo, p0));
  for (int o = oa; o < ob; ++o) {
    auto next = [&] {
      if (o + 1 < ob)
        fft_preload_regs(pre, NB, TLoader<N0, NB, C>(Tin, o + 1, npl, tab.nplanes, tab.m0lo, p0));
    };
    const double f = occ[o] * inv_omega;
    fft_io<N0, +1, NB, XT, SRC_PRE, DST_FN, C, SH::V>(X, N0 + 1, NB, tw, preloaded(pre, next), [&](int, int, C v, int it, int q) {
      a[it][q] += f * (double(v.x) * double(v.x) + double(v.y) * double(v.y));
    });
    __syncthreads();
  }
  double* pb = part + (long long)g * tab.n0 * npl + p0;
  last_stage_positions<N0, NB, XT, SH::V>(NB, [&](int it, int q, int t, int e) {
    if (p0 + t < npl) pb[e * npl + t] = a[it][q];
  });
}

// rho (+)= sum over groups g = 0..ng-1 of part[g] (in order)
__global__ __launch_bounds__(NT) void dens_sum_kernel(const double* __restrict__ part, int ng, long long N,
                                                      double* __restrict__ rho, int accumulate) {
  const long long i = (long long)blockIdx.x * NT + threadIdx.x;
  if (i >= N) return;
  double s = accumulate ? rho[i] : 0.0;
  for (int g = 0; g < ng; ++g) s += part[g * N + i];
  rho[i] = s;
}

// ------------------------------------------------------------------ launchers

// Orbital groups per x-pass launch: groups of at most xg_max orbitals (sizes
// differing by at most one), fewer orbitals per group when the launch would
// otherwise have too few blocks to fill the chip (about 12 per CU).
static int x_groups(const ks_system* s, int nb) {
  const long long blocks = (long long)s->ntiles * nb;
  long long g = blocks / (256 * 12);
  g = g < 1 ? 1 : (g > s->xg_max ? s->xg_max : g);
  return (int)((nb + g - 1) / g);
}

// Launch shapes of the x-pencil blocks: a tile (pencils NB x threads XT)
// and the factorisation of the x-transform (plan variant V, fft_device.hpp).
// Shape 0 is xnb<N0> pencils x NT threads; shape 1 is 16 pencils x 192
// threads, for the largest grids only (smaller LDS buffers, more blocks
// resident per CU); shapes 2 and 3 are shapes 0 and 1 with the second
// factorisation of n0 (n0 = 96: 8 x 12 instead of 12 x 8).  The autotuner
// picks the shape per grid and precision.
template <int NB_, int XT_>
struct XShape {
  static constexpr int NB = NB_, XT = XT_, V = 0;
};
template <int NB_, int XT_>
struct XShapeAlt {
  static constexpr int NB = NB_, XT = XT_, V = 1;
};
template <int N0> constexpr bool has_shape1 = N0 == 96 || N0 == 120;
template <int N0> constexpr bool has_alt_plan = N0 == 96;

template <int N0, class F>
static void with_shape(const ks_system* s, F&& f) {
  if constexpr (has_alt_plan<N0>) {
    if (s->xshape == 2) {
      f(XShapeAlt<xnb<N0>::value, NT>{});
      return;
    }
    if (s->xshape == 3) {
      f(XShapeAlt<16, 192>{});
      return;
    }
  }
  if constexpr (has_shape1<N0>) {
    if (s->xshape == 1) {
      f(XShape<16, 192>{});
      return;
    }
  }
  f(XShape<xnb<N0>::value, NT>{});
}

bool x_shape_available(int n0, int shape) {
  if (shape == 0) return true;
  if (shape < 1 || shape > 3) return false;
  switch (n0) {
#define KS_CASE(v) case v: return (shape == 1 || shape == 3 ? has_shape1<v> : true) && (shape < 2 || has_alt_plan<v>);
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

int x_shape_nb(int n0, int shape) { return shape == 1 || shape == 3 ? 16 : x_tile_nb(n0); }
int x_shape_threads(int shape) { return shape == 1 || shape == 3 ? 192 : NT; }

template <int N0, bool HB>
static void xproj_n(const ks_system* s, int nb, const void* T, void* partial, const double* occ, double* rho,
                    int accumulate, hipStream_t st) {
  const double scale = s->dV / sqrt(s->omega);
  const double inv_omega = 1.0 / s->omega;
  const bool dens = rho != nullptr;
  // with the density: groups of at least DENS_GROUP orbitals, so the partial
  // densities fit their buffer
  const int ng = dens ? std::min(x_groups(s, nb), (nb + DENS_GROUP - 1) / DENS_GROUP) : x_groups(s, nb);
  with_shape<N0>(s, [&](auto sh) {
    using SH = decltype(sh);
    const dim3 grid(s->ntiles, ng);
    if (!dens) {
      if (!mixed(s))
        xproj_kernel<N0, SH, double, HB, false><<<grid, SH::XT, 0, st>>>(
            (const double2*)T, nb, (double2*)partial, sphere_tab(s), proj_tab(s), s->d_tw0, scale, nullptr, nullptr,
            inv_omega);
      else
        xproj_kernel<N0, SH, float, HB, false><<<grid, SH::XT, 0, st>>>(
            (const float2*)T, nb, (float2*)partial, sphere_tab(s), proj_tab(s), s->d_tw0f, scale, nullptr, nullptr,
            inv_omega);
    } else if (!mixed(s)) {
      xproj_kernel<N0, SH, double, HB, true><<<grid, SH::XT, 0, st>>>(
          (const double2*)T, nb, (double2*)partial, sphere_tab(s), proj_tab(s), s->d_tw0, scale, occ, s->dens_part,
          inv_omega);
    } else {
      xproj_kernel<N0, SH, float, HB, true><<<grid, SH::XT, 0, st>>>(
          (const float2*)T, nb, (float2*)partial, sphere_tab(s), proj_tab(s), s->d_tw0f, scale, occ, s->dens_part,
          inv_omega);
    }
  });
  if (dens)
    dens_sum_kernel<<<(unsigned)((s->N + NT - 1) / NT), NT, 0, st>>>(s->dens_part, ng, s->N, rho, accumulate);
}

bool launch_xproj(const ks_system* s, int nb, const void* T, void* partial, const double* occ, double* rho,
                  int accumulate, hipStream_t st) {
  switch (s->n[0]) {
#define KS_CASE(v) \
  case v: s->x_half ? xproj_n<v, true>(s, nb, T, partial, occ, rho, accumulate, st) \
                    : xproj_n<v, false>(s, nb, T, partial, occ, rho, accumulate, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

template <int N0, bool HB>
static void xapply_n(const ks_system* s, int nb, const void* T, const double2* DP, void* U, hipStream_t st) {
  // synthesis scale Omega^-1/2 and analysis scale Omega^1/2/N folded into V
  // (the KB coefficients carry the analysis scale from proj_reduce)
  const double sc_v = 1.0 / (double)s->N;
  const int ng = x_groups(s, nb);
  with_shape<N0>(s, [&](auto sh) {
    using SH = decltype(sh);
    const dim3 grid(s->ntiles, ng);
    if (!mixed(s))
      xapply_kernel<N0, SH, double, HB><<<grid, SH::XT, 0, st>>>((const double2*)T, nb, (double2*)U, s->d_v, DP,
                                                                sphere_tab(s), proj_tab(s), s->d_tw0, sc_v);
    else
      xapply_kernel<N0, SH, float, HB><<<grid, SH::XT, 0, st>>>((const float2*)T, nb, (float2*)U, s->d_v, DP,
                                                               sphere_tab(s), proj_tab(s), s->d_tw0f, sc_v);
  });
}

bool launch_xapply(const ks_system* s, int nb, const void* T, const double2* DP, void* U, hipStream_t st) {
  switch (s->n[0]) {
#define KS_CASE(v) \
  case v: s->x_half ? xapply_n<v, true>(s, nb, T, DP, U, st) : xapply_n<v, false>(s, nb, T, DP, U, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

// Batched launches: one x-pass launch over several systems of the grid (all
// of one tile shape, that of s).
template <int N0, bool HB>
static void x_batch_n(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, bool apply,
                      hipStream_t st) {
  const dim3 grid(s->ntiles, nrows);
  const double scale = s->dV / sqrt(s->omega);
  const double sc_v = 1.0 / (double)s->N;
  with_shape<N0>(s, [&](auto sh) {
    using SH = decltype(sh);
    if (!apply) {
      if (!mixed(s))
        xproj_kernel<N0, SH, double, HB, false, true><<<grid, SH::XT, 0, st>>>(
            nullptr, 0, nullptr, sphere_tab(s), ProjTab{}, s->d_tw0, scale, nullptr, nullptr, 0.0, jobs, rows);
      else
        xproj_kernel<N0, SH, float, HB, false, true><<<grid, SH::XT, 0, st>>>(
            nullptr, 0, nullptr, sphere_tab(s), ProjTab{}, s->d_tw0f, scale, nullptr, nullptr, 0.0, jobs, rows);
    } else if (!mixed(s)) {
      xapply_kernel<N0, SH, double, HB, true><<<grid, SH::XT, 0, st>>>(
          nullptr, 0, nullptr, nullptr, nullptr, sphere_tab(s), ProjTab{}, s->d_tw0, sc_v, jobs, rows);
    } else {
      xapply_kernel<N0, SH, float, HB, true><<<grid, SH::XT, 0, st>>>(
          nullptr, 0, nullptr, nullptr, nullptr, sphere_tab(s), ProjTab{}, s->d_tw0f, sc_v, jobs, rows);
    }
  });
}

bool launch_x_batch(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, bool apply,
                    hipStream_t st) {
  switch (s->n[0]) {
#define KS_CASE(v) \
  case v: s->x_half ? x_batch_n<v, true>(s, jobs, rows, nrows, apply, st) \
                    : x_batch_n<v, false>(s, jobs, rows, nrows, apply, st); return true;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
}

int x_group_size(const ks_system* s, long long total_orbitals) {
  long long g = (long long)s->ntiles * total_orbitals / (256 * 12);
  return (int)(g < 1 ? 1 : (g > s->xg_max ? s->xg_max : g));
}

// Orbital groups of the density pass: each group writes one partial density
// that dens_sum adds in order, so the groups are as large as keeps about 12
// blocks per CU busy, and hold at least DENS_GROUP orbitals.
static int dens_groups(const ks_system* s, int nb) {
  const int by_size = (nb + DENS_GROUP - 1) / DENS_GROUP;
  const int by_fill = (256 * 12 + s->ntiles - 1) / s->ntiles;
  return std::max(1, std::min(by_size, by_fill));
}

template <int N0, bool HB>
static void xdens_n(const ks_system* s, int nb, const void* T, const double* occ, double* part, hipStream_t st) {
  const int ng = dens_groups(s, nb);
  with_shape<N0>(s, [&](auto sh) {
    using SH = decltype(sh);
    const dim3 grid(s->ntiles, ng);
    if (!mixed(s))
      xdens_kernel<N0, SH, double, HB><<<grid, SH::XT, 0, st>>>((const double2*)T, nb, occ, part, sphere_tab(s),
                                                               s->d_tw0, 1.0 / s->omega);
    else
      xdens_kernel<N0, SH, float, HB><<<grid, SH::XT, 0, st>>>((const float2*)T, nb, occ, part, sphere_tab(s),
                                                              s->d_tw0f, 1.0 / s->omega);
  });
}

bool launch_xdens(const ks_system* s, int nb, const void* T, const double* occ, double* rho, int accumulate,
                  hipStream_t st) {
  switch (s->n[0]) {
#define KS_CASE(v) \
  case v: s->x_half ? xdens_n<v, true>(s, nb, T, occ, s->dens_part, st) : xdens_n<v, false>(s, nb, T, occ, s->dens_part, st); break;
    KS_SIZES(KS_CASE)
#undef KS_CASE
    default:
      return false;
  }
  const int ng = dens_groups(s, nb);
  dens_sum_kernel<<<(unsigned)((s->N + NT - 1) / NT), NT, 0, st>>>(s->dens_part, ng, s->N, rho, accumulate);
  return true;
}

}  // namespace ks
