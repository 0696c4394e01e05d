// Batched mixed-radix (2/3/4/5/6/8) complex FFTs on LDS-resident data for
// gfx950.  Used by the real<->Fourier space passes of the Kohn-Sham
// Hamiltonian ("two Fourier transforms" per application, Section
// "Implementation of the KS Hamiltonian").
//
// Formulation: Stockham autosort.  For a length-N transform factored as
// N = R_1 R_2 ... R_s, stage t (radix R, Ns = R_1...R_{t-1}) maps butterfly
// b = 0..N/R-1 as
//     v_q   = x[b + q N/R] * W^{q (b mod Ns) N/(Ns R)}        (q = 0..R-1)
//     v     = DFT_R(v)
//     y[(b div Ns) Ns R + (b mod Ns) + q Ns] = v_q
// and leaves the result in natural order.  W = exp(sign * 2 pi i / N).
// Each stage reads every input of the batch into registers, synchronises the
// block, then writes in place, so one LDS buffer per batch suffices.
//
// The whole block (NT threads) cooperates on NB transforms; work item
// i -> (transform i mod NB, butterfly i div NB), so neighbouring lanes touch
// neighbouring transforms at the same butterfly (uniform twiddle index, and a
// transform stride of N+1 elements keeps 16-byte accesses spread over banks).
// Every thread must call the batch routine the same number of times (it
// contains block barriers).
#pragma once
#include <hip/hip_runtime.h>

namespace ks {

template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename R> using cplx = typename cvec<R>::type;

template <typename T> __device__ __forceinline__ T cadd(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ T csub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
  return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ T cmulc(T a, T b) {
  return T{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T, typename S> __device__ __forceinline__ T cscale(T a, S s) { return T{a.x * s, a.y * s}; }
// multiply by sign*i
template <int SIGN, typename T> __device__ __forceinline__ T cmul_i(T a) {
  return SIGN > 0 ? T{-a.y, a.x} : T{a.y, -a.x};
}

// ---------------------------------------------------------------- codelets
// y_k = sum_q v_q exp(SIGN 2 pi i q k / R), in place.

template <int R, int SIGN, typename T> struct dft;

template <int SIGN, typename T> struct dft<2, SIGN, T> {
  __device__ __forceinline__ static void run(T* v) {
    T a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int SIGN, typename T> struct dft<3, SIGN, T> {
  __device__ __forceinline__ static void run(T* v) {
    using R = decltype(v[0].x);
    const R c = R(-0.5), s = R(0.86602540378443864676372317075293618);  // cos, sin of 2pi/3
    T a = cadd(v[1], v[2]);
    T d = csub(v[1], v[2]);
    T t1 = T{v[0].x + c * a.x, v[0].y + c * a.y};
    T t2 = cmul_i<SIGN>(cscale(d, s));
    v[0] = cadd(v[0], a);
    v[1] = cadd(t1, t2);
    v[2] = csub(t1, t2);
  }
};

template <int SIGN, typename T> struct dft<4, SIGN, T> {
  __device__ __forceinline__ static void run(T* v) {
    T a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    T c = cadd(v[1], v[3]), d = cmul_i<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

template <int SIGN, typename T> struct dft<5, SIGN, T> {
  __device__ __forceinline__ static void run(T* v) {
    using R = decltype(v[0].x);
    // cos/sin of 2pi/5 and 4pi/5
    const R c1 = R(0.30901699437494742410229341718281906);
    const R c2 = R(-0.80901699437494742410229341718281906);
    const R s1 = R(0.95105651629515357211643933337938214);
    const R s2 = R(0.58778525229247312916870595463907277);
    T a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    T a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    T r1 = T{v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    T r2 = T{v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    T i1 = cmul_i<SIGN>(T{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    T i2 = cmul_i<SIGN>(T{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(r1, i1);
    v[4] = csub(r1, i1);
    v[2] = cadd(r2, i2);
    v[3] = csub(r2, i2);
  }
};

// radix 6 = two radix-3 DFTs (even / odd inputs) combined by a radix-2 step
template <int SIGN, typename T> struct dft<6, SIGN, T> {
  __device__ __forceinline__ static void run(T* v) {
    using R = decltype(v[0].x);
    T e[3] = {v[0], v[2], v[4]};
    T o[3] = {v[1], v[3], v[5]};
    dft<3, SIGN, T>::run(e);
    dft<3, SIGN, T>::run(o);
    const R h = R(0.5), s = R(0.86602540378443864676372317075293618);
    // w^1 = exp(SIGN i pi/3), w^2 = exp(SIGN 2 i pi/3)
    T o1 = T{h * o[1].x - SIGN * s * o[1].y, h * o[1].y + SIGN * s * o[1].x};
    T o2 = T{-h * o[2].x - SIGN * s * o[2].y, -h * o[2].y + SIGN * s * o[2].x};
    v[0] = cadd(e[0], o[0]);
    v[3] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[4] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[5] = csub(e[2], o2);
  }
};

// radix 8 = radix-2 on (even, odd) radix-4 halves
template <int SIGN, typename T> struct dft<8, SIGN, T> {
  __device__ __forceinline__ static void run(T* v) {
    using R = decltype(v[0].x);
    T e[4] = {v[0], v[2], v[4], v[6]};
    T o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, SIGN, T>::run(e);
    dft<4, SIGN, T>::run(o);
    const R r = R(0.70710678118654752440084436210484904);
    // o[k] *= exp(SIGN 2 pi i k / 8)
    T o1 = T{r * (o[1].x - SIGN * o[1].y), r * (o[1].y + SIGN * o[1].x)};
    T o2 = cmul_i<SIGN>(o[2]);
    T o3 = T{-r * (o[3].x + SIGN * o[3].y), r * (SIGN * o[3].x - o[3].y)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// ------------------------------------------------------------- radix plans

template <int... Rs> struct radix_list {};

template <int N> struct plan;   // factorisation used for length N
template <> struct plan<8> { using list = radix_list<8>; };
template <> struct plan<12> { using list = radix_list<4, 3>; };
template <> struct plan<16> { using list = radix_list<4, 4>; };
template <> struct plan<20> { using list = radix_list<4, 5>; };
template <> struct plan<24> { using list = radix_list<4, 6>; };
template <> struct plan<30> { using list = radix_list<6, 5>; };
template <> struct plan<32> { using list = radix_list<4, 8>; };
template <> struct plan<36> { using list = radix_list<6, 6>; };
template <> struct plan<40> { using list = radix_list<8, 5>; };
template <> struct plan<48> { using list = radix_list<8, 6>; };
template <> struct plan<60> { using list = radix_list<4, 3, 5>; };
template <> struct plan<64> { using list = radix_list<8, 8>; };
template <> struct plan<72> { using list = radix_list<8, 3, 3>; };
template <> struct plan<80> { using list = radix_list<4, 4, 5>; };
template <> struct plan<96> { using list = radix_list<6, 4, 4>; };
template <> struct plan<100> { using list = radix_list<4, 5, 5>; };
template <> struct plan<120> { using list = radix_list<8, 5, 3>; };
template <> struct plan<128> { using list = radix_list<8, 4, 4>; };

// One Stockham stage over a batch of NB transforms laid out at
// buf[t * ts + e] (element stride 1).  tw[j] = exp(-2 pi i j / N).
template <int N, int R, int NS, int SIGN, int NB, int NT, typename T>
__device__ __forceinline__ void stockham_stage(T* buf, int ts, int ntrans, const T* tw) {
  constexpr int NBF = N / R;
  constexpr int TOT = NB * NBF;
  constexpr int ITEMS = (TOT + NT - 1) / NT;
  const int tid = threadIdx.x;
  T v[ITEMS][R];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int i = tid + it * NT;
    const int t = i % NB, b = i / NB;
    if ((TOT % NT == 0 || i < TOT) && t < ntrans) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[it][q] = buf[t * ts + b + q * NBF];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int i = tid + it * NT;
    const int t = i % NB, b = i / NB;
    if ((TOT % NT == 0 || i < TOT) && t < ntrans) {
      const int k = b % NS;
      if (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          const T w = tw[q * k * (N / (NS * R))];
          v[it][q] = SIGN < 0 ? cmul(v[it][q], w) : cmulc(v[it][q], w);
        }
      }
      dft<R, SIGN, T>::run(v[it]);
      const int o = (b / NS) * NS * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[t * ts + o + q * NS] = v[it][q];
    }
  }
  __syncthreads();
}

template <int N, int NS, int SIGN, int NB, int NT, typename T, int R, int... Rest>
__device__ __forceinline__ void stockham_run(T* buf, int ts, int ntrans, const T* tw) {
  stockham_stage<N, R, NS, SIGN, NB, NT, T>(buf, ts, ntrans, tw);
  if constexpr (sizeof...(Rest) > 0) stockham_run<N, NS * R, SIGN, NB, NT, T, Rest...>(buf, ts, ntrans, tw);
}

template <int N, int SIGN, int NB, int NT, typename T, int... Rs>
__device__ __forceinline__ void fft_batch_impl(radix_list<Rs...>, T* buf, int ts, int ntrans, const T* tw) {
  stockham_run<N, 1, SIGN, NB, NT, T, Rs...>(buf, ts, ntrans, tw);
}

// In-place DFT  x_k <- sum_j x_j exp(SIGN 2 pi i j k / N)  of transforms
// t < ntrans (t < NB) stored at buf[t * ts + 0 .. N-1].  Block-collective.
template <int N, int SIGN, int NB, int NT, typename T>
__device__ __forceinline__ void fft_batch(T* buf, int ts, int ntrans, const T* tw) {
  fft_batch_impl<N, SIGN, NB, NT, T>(typename plan<N>::list{}, buf, ts, ntrans, tw);
}

__device__ __forceinline__ int fold(int j, int n) { return 2 * j < n ? j : j - n; }
__device__ __forceinline__ int wrap(int m, int n) { return m < 0 ? m + n : m; }

}  // namespace ks
