// Optical absorption of a kicked propagation (HIP, gfx950): the Fourier
// transform of the dipole moments recorded after the kick (Section
// "Results", the water-molecule spectrum).
//
//   x(t_n)  = (d(t_n) - d(0)) . k / |k|,   t_n = n dt, n = 0 .. nt-1
//   alpha(w) = |k|^-1 dt sum_n c_n x(t_n) e^{i w t_n - eta t_n}
//              (trapezoid weights c_0 = c_{nt-1} = 1/2, else 1)
//   S(w)    = (2 w / pi) Im alpha(w)
#include <cmath>

#include "ks_internal.h"

namespace ks {

constexpr int SPEC_NT = 256;

// Block iw: thread j sums the terms n = j, j + SPEC_NT, ... in order; the
// per-thread sums are added by a fixed tree (deterministic).
__global__ __launch_bounds__(SPEC_NT) void spectrum_kernel(const double* __restrict__ d, int nt, double dt,
                                                           double ux, double uy, double uz, double inv_k,
                                                           const double* __restrict__ omegas, int nw, double eta,
                                                           double2* __restrict__ alpha, double* __restrict__ strength) {
  __shared__ double sr[SPEC_NT], si[SPEC_NT];
  const int iw = blockIdx.x, tid = threadIdx.x;
  if (iw >= nw) return;
  const double om = omegas[iw];
  double ar = 0.0, ai = 0.0;
  for (int n = tid; n < nt; n += SPEC_NT) {
    const double x = (d[3 * n] - d[0]) * ux + (d[3 * n + 1] - d[1]) * uy + (d[3 * n + 2] - d[2]) * uz;
    const double t = dt * n;
    double s, c;
    sincos(om * t, &s, &c);
    const double f = ((n == 0 || n == nt - 1) ? 0.5 : 1.0) * x * exp(-eta * t);
    ar += f * c;
    ai += f * s;
  }
  sr[tid] = ar;
  si[tid] = ai;
  __syncthreads();
  for (int h = SPEC_NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      sr[tid] += sr[tid + h];
      si[tid] += si[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double2 a{dt * sr[0] * inv_k, dt * si[0] * inv_k};
    alpha[iw] = a;
    strength[iw] = 2.0 * om / M_PI * a.y;
  }
}

void launch_spectrum(const double* d, int nt, double dt, const double k[3], const double* omegas, int nw,
                     double eta, double2* alpha, double* strength, hipStream_t st) {
  const double kn = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  if (nw > 0)
    spectrum_kernel<<<nw, SPEC_NT, 0, st>>>(d, nt, dt, k[0] / kn, k[1] / kn, k[2] / kn, 1.0 / kn, omegas, nw, eta,
                                            alpha, strength);
}

}  // namespace ks
