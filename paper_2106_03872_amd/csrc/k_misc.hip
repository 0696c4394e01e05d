// Small kernels of the hot path (HIP, gfx950): box <-> packed sphere
// conversion at the boundary, the per-atom KB projection sums (Eq. vnl),
// norms and band energy reductions.
#include "ks_common.hpp"

namespace ks {

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

int x_tile_nb(int n0) { return n0 <= 32 ? 64 : 32; }

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

// KB projections: P_Ip = sum over the (tile, atom) slots of atom I in
// ascending order, DP = scale d_Ip P_Ip (Eq. vnl; scale is the analysis
// normalisation that the x-analysis leaves out).  One wavefront per (atom,
// orbital): lane = 8 * slot-lane + q; slot-lanes are combined in a fixed order.
// BATCH: block (I, y) reduces orbital rows[y].y of job rows[y].x (its
// partial sums, coefficients and tables); atoms beyond the job's count exit.
template <typename C, bool BATCH = false>
__global__ __launch_bounds__(64) void proj_reduce_kernel(const C* __restrict__ partial, double2* __restrict__ DP,
                                                         ProjTab pt, double scale,
                                                         const BatchJob* __restrict__ jobs = nullptr,
                                                         const int4* __restrict__ rows = nullptr) {
  __shared__ double2 red[64];
  const int I = blockIdx.x, lane = threadIdx.x;
  int o = blockIdx.y;
  if constexpr (BATCH) {
    const int4 r = rows[blockIdx.y];
    partial = static_cast<const C*>(jobs[r.x].partial);
    DP = jobs[r.x].DP;
    pt = jobs[r.x].pt;
    o = r.y;
    if (I >= pt.natoms) return;   // uniform per block
  }
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
    const double dd = pt.d[I * np + q] * scale;
    DP[((long long)o * pt.natoms + I) * np + q] = double2{dd * tx, dd * ty};
  }
}

// per-orbital sums over the packed sphere: out[2o] = sum |a|^2, out[2o+1] = sum Re conj(a) b
template <typename CA, typename CB_>
__global__ __launch_bounds__(NT) void dots_kernel(const CA* __restrict__ a, const CB_* __restrict__ b, int stride,
                                                  int npw, double* __restrict__ out) {
  __shared__ double s0[NT], s1[NT];
  const int o = blockIdx.x, tid = threadIdx.x;
  const CA* pa = a + (long long)o * stride;
  const CB_* pb = b ? b + (long long)o * stride : nullptr;
  double x0 = 0.0, x1 = 0.0;
  for (int e = tid; e < npw; e += NT) {
    const CA u = pa[e];
    x0 += double(u.x) * double(u.x) + double(u.y) * double(u.y);
    if (pb) {
      const CB_ v = pb[e];
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

bool launch_pack(const ks_system* s, int nb, const double2* box, long long box_stride, void* pk, hipStream_t st) {
  pack_kernel<double2><<<dim3(s->nplanes, nb), NT, 0, st>>>(box, box_stride, (double2*)pk, s->npw_stride,
                                                             sphere_tab(s));
  return true;
}

bool launch_unpack(const ks_system* s, int nb, const void* pk, bool pk_fp64, double2* box, long long box_stride,
                   hipStream_t st) {
  const unsigned gx = (unsigned)((s->N + NT - 1) / NT);
  if (pk_fp64)
    unpack_kernel<double2><<<dim3(gx, nb), NT, 0, st>>>((const double2*)pk, s->npw_stride, box, box_stride,
                                                         sphere_tab(s));
  else
    unpack_kernel<float2><<<dim3(gx, nb), NT, 0, st>>>((const float2*)pk, s->npw_stride, box, box_stride,
                                                        sphere_tab(s));
  return true;
}

bool launch_proj_reduce(const ks_system* s, int nb, const void* partial, double2* DP, hipStream_t st) {
  if (s->natoms == 0 || nb == 0) return true;
  const double scale = sqrt(s->omega) / (double)s->N;
  if (!mixed(s))
    proj_reduce_kernel<double2><<<dim3(s->natoms, nb), 64, 0, st>>>((const double2*)partial, DP, proj_tab(s), scale);
  else
    proj_reduce_kernel<float2><<<dim3(s->natoms, nb), 64, 0, st>>>((const float2*)partial, DP, proj_tab(s), scale);
  return true;
}

bool launch_proj_reduce_batch(const ks_system* s, const BatchJob* jobs, const int4* rows, int nrows, int max_natoms,
                              hipStream_t st) {
  if (max_natoms == 0 || nrows == 0) return true;
  const double scale = sqrt(s->omega) / (double)s->N;
  if (!mixed(s))
    proj_reduce_kernel<double2, true><<<dim3(max_natoms, nrows), 64, 0, st>>>(nullptr, nullptr, ProjTab{}, scale, jobs,
                                                                             rows);
  else
    proj_reduce_kernel<float2, true><<<dim3(max_natoms, nrows), 64, 0, st>>>(nullptr, nullptr, ProjTab{}, scale, jobs,
                                                                            rows);
  return true;
}

// a: the FP64 state; b: H applied to it in the working precision (or null)
bool launch_dots(const ks_system* s, int nb, const void* a, const void* b, double* out, hipStream_t st) {
  if (!mixed(s))
    dots_kernel<double2, double2><<<nb, NT, 0, st>>>((const double2*)a, (const double2*)b, s->npw_stride, s->npw,
                                                     out);
  else
    dots_kernel<double2, float2><<<nb, NT, 0, st>>>((const double2*)a, (const float2*)b, s->npw_stride, s->npw,
                                                    out);
  return true;
}

bool launch_energy_sum(int norb, const double* occ, const double* red, double* energy, hipStream_t st) {
  energy_sum_kernel<<<1, 64, 0, st>>>(norb, occ, red, energy);
  return true;
}

}  // namespace ks
