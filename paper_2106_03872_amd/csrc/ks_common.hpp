// Device helpers and launch constants shared by the kernel translation units.
#pragma once
#include "fft_device.hpp"
#include "ks_internal.h"

namespace ks {

constexpr int NT = 256;   // threads per x-pencil block
constexpr int DENS_GROUP = 8;   // smallest orbital group of a density block

#define KS_SIZES(X) X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(60) X(64) X(72) X(80) X(96) X(120) X(128)

// pencils per x-tile (host side: x_tile_nb)
template <int N> struct xnb { static constexpr int value = N <= 32 ? 64 : 32; };
constexpr int NTP = 384; // threads per plane-pass block

template <typename T> __device__ __forceinline__ T czero() { return T{0, 0}; }

template <typename T> __device__ __forceinline__ T to_c(double2 a) {
  return T{static_cast<decltype(T{}.x)>(a.x), static_cast<decltype(T{}.x)>(a.y)};
}
template <typename T> __device__ __forceinline__ double2 to_d(T a) { return double2{double(a.x), double(a.y)}; }
template <typename C, typename T> __device__ __forceinline__ C cvt(T a) {
  using E = decltype(C{}.x);
  return C{E(a.x), E(a.y)};
}

// largest c in [0, nc) with off[c] <= e (off ascending)
__device__ __forceinline__ int find_col(const int* off, int nc, int e) {
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}


template <int N> struct pnb { static constexpr int value = N <= 64 ? 64 : (N <= 96 ? 48 : (N <= 120 ? 24 : 16)); };

inline bool mixed(const ks_system* s) { return s->prec == KS_MIXED; }

// Orbital group of a block: the orbitals [y*nb/ng, (y+1)*nb/ng) with
// y = blockIdx.y and ng = gridDim.y (group sizes differ by at most one).
__device__ __forceinline__ void orbital_range(int nb, int& oa, int& ob) {
  oa = (int)((long long)blockIdx.y * nb / gridDim.y);
  ob = (int)((long long)(blockIdx.y + 1) * nb / gridDim.y);
}

// The same for group g of ng over nb orbitals (a batched launch's row).
__device__ __forceinline__ void group_range(int nb, int g, int ng, int& oa, int& ob) {
  oa = (int)((long long)g * nb / ng);
  ob = (int)((long long)(g + 1) * nb / ng);
}

}  // namespace ks
