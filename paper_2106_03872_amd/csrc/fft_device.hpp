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

#include <type_traits>

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

// Prime-factor (Good-Thomas) codelets for N = N1 N2 with gcd(N1, N2) = 1:
// input n = (N2 n1 + N1 n2) mod N, output k = (A k1 + B k2) mod N with
// A = N2 (N2^-1 mod N1), B = N1 (N1^-1 mod N2); no twiddle factors.
constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

template <int N1, int N2, int SIGN, typename T> struct dft_pfa {
  static constexpr int N = N1 * N2;
  static constexpr int A = N2 * inv_mod(N2 % N1, N1);
  static constexpr int B = N1 * inv_mod(N1 % N2, N2);
  __device__ __forceinline__ static void run(T* v) {
    T a[N1][N2];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1)
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) a[n1][n2] = v[(N2 * n1 + N1 * n2) % N];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) dft<N2, SIGN, T>::run(a[n1]);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      T c[N1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) c[n1] = a[n1][k2];
      dft<N1, SIGN, T>::run(c);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) v[(A * k1 + B * k2) % N] = c[k1];
    }
  }
};

template <int SIGN, typename T> struct dft<10, SIGN, T> : dft_pfa<2, 5, SIGN, T> {};
template <int SIGN, typename T> struct dft<12, SIGN, T> : dft_pfa<3, 4, SIGN, T> {};
template <int SIGN, typename T> struct dft<15, SIGN, T> : dft_pfa<3, 5, SIGN, T> {};

// ------------------------------------------------------------- radix plans

template <int... Rs> struct radix_list {};

template <int N> struct plan;   // factorisation used for length N (first radix first)
template <> struct plan<8> { using list = radix_list<8>; };
template <> struct plan<12> { using list = radix_list<12>; };
template <> struct plan<16> { using list = radix_list<4, 4>; };
template <> struct plan<20> { using list = radix_list<4, 5>; };
template <> struct plan<24> { using list = radix_list<4, 6>; };
template <> struct plan<30> { using list = radix_list<6, 5>; };
template <> struct plan<32> { using list = radix_list<4, 8>; };
template <> struct plan<36> { using list = radix_list<6, 6>; };
template <> struct plan<40> { using list = radix_list<8, 5>; };
template <> struct plan<48> { using list = radix_list<8, 6>; };
template <> struct plan<60> { using list = radix_list<12, 5>; };
template <> struct plan<64> { using list = radix_list<8, 8>; };
template <> struct plan<72> { using list = radix_list<12, 6>; };
template <> struct plan<80> { using list = radix_list<8, 10>; };
template <> struct plan<96> { using list = radix_list<12, 8>; };
template <> struct plan<100> { using list = radix_list<10, 10>; };
template <> struct plan<120> { using list = radix_list<12, 10>; };
template <> struct plan<128> { using list = radix_list<8, 4, 4>; };

// A second factorisation for the x-pencil transforms of some lengths (the
// launch-schedule autotuner times both): variant 0 is plan<N>, variant 1
// alt_plan<N>.  A band-limited first stage needs a first radix divisible by 4.
template <int N> struct alt_plan;
template <> struct alt_plan<96> { using list = radix_list<8, 12>; };
template <int N, int V> struct plan_v { using list = typename plan<N>::list; };
template <int N> struct plan_v<N, 1> { using list = typename alt_plan<N>::list; };

// Where a stage reads from / writes to.  LDS stages work in place on the
// batch buffer; the first stage may instead pull its inputs from a loader
// functor and the last stage may push its outputs to a store functor.
enum { SRC_LDS = 0, SRC_FN = 1, SRC_PRE = 2 };   // SRC_PRE: inputs already in a register array (fft_preload)
enum { DST_LDS = 0, DST_FN = 1, DST_FN_LDS = 2 };   // DST_FN_LDS: the functor writes the batch buffer

// Streaming (non-temporal) global loads and stores for the plane
// intermediates, which are written once and read once or twice per pass:
// they then do not evict the small per-block tables (potential, projector and
// scatter tables) that every orbital of a block re-reads from L2.
template <typename T> struct native2;
template <> struct native2<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct native2<float2> { typedef float type __attribute__((ext_vector_type(2))); };
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  using V = typename native2<T>::type;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return T{v[0], v[1]};
}
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T x) {
  using V = typename native2<T>::type;
  const V v = {x.x, x.y};
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}

// Band-limited operands.  A load or store functor derived from `band`
// declares that the elements outside e < N/4 or e >= 3N/4 are zero (loads,
// first stage) or not wanted (stores, last stage).  With a radix R divisible
// by 4 those are the butterfly elements R/4 <= q < 3R/4 (first stage:
// e = b + q N/R; last stage: e = k + q N/R); the stage then neither loads nor
// stores them, and what only feeds the skipped stores is never computed.  For
// other radices the declaration changes nothing.
struct band {};
template <class F>
constexpr bool is_band = std::is_base_of<band, std::remove_cv_t<std::remove_reference_t<F>>>::value;
template <int R>
__device__ constexpr bool in_band(int q) {
  return R % 4 != 0 || q < R / 4 || q >= 3 * R / 4;
}
template <class F>
struct band_fn : band {
  F f;
  __device__ explicit band_fn(F g) : f(g) {}
  template <class... A>
  __device__ auto operator()(A... a) const {
    return f(a...);
  }
};
template <class F>
__device__ band_fn<F> banded(F f) {
  return band_fn<F>(f);
}

struct no_load {
  template <typename T> __device__ T operator()(int, int) const { return T{}; }
};
struct no_store {
  template <typename T> __device__ void operator()(int, int, T, int, int) const {}
};

// threadIdx.x behind an empty volatile asm: the per-thread index arithmetic of
// each stage is then computed where it is used instead of being hoisted out
// of a caller's loop and kept live across it (which costs more registers
// than the few integer operations it saves).
template <int NT>
__device__ __forceinline__ int fresh_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  __builtin_assume(t >= 0 && t < NT);
  return t;
}

// One Stockham stage over a batch of NB transforms laid out at buf[t*ts + e].
// tw[j] = exp(-2 pi i j / N) (global or LDS).
//   load(t, e)             -> element e of transform t        (SRC_FN)
//   store(t, e, v, it, q)  <- output element e of transform t (DST_FN*); it and q
//                             index the caller's per-thread register arrays
template <int N, int R, int NS, int SIGN, int NB, int NT, int SRC, int DST, typename T, class Load, class Store>
__device__ __forceinline__ void stockham_stage(T* buf, int ts, int ntrans, const T* __restrict__ tw, Load& load,
                                               Store& store) {
  constexpr int NBF = N / R;
  constexpr int TOT = NB * NBF;
  constexpr int ITEMS = (TOT + NT - 1) / NT;
  const int tid = fresh_tid<NT>();
  T v[ITEMS][R];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int i = tid + it * NT;
    const int t = i % NB, b = i / NB;
    if ((TOT % NT == 0 || i < TOT) && t < ntrans) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if constexpr (SRC == SRC_FN) {
          if (!is_band<Load> || in_band<R>(q)) v[it][q] = load(t, b + q * NBF);
          else v[it][q] = T{0, 0};
        } else if constexpr (SRC == SRC_PRE) {
          v[it][q] = load.r.get(it, q);
        } else {
          v[it][q] = buf[t * ts + b + q * NBF];
        }
      }
    }
  }
  if constexpr (SRC == SRC_LDS && DST != DST_FN) __syncthreads();   // in place: all reads before writes
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int i = tid + it * NT;
    const int t = i % NB, b = i / NB;
    if ((TOT % NT == 0 || i < TOT) && t < ntrans) {
      const int k = b % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          const T w = tw[q * k * (N / (NS * R))];
          v[it][q] = SIGN < 0 ? cmul(v[it][q], w) : cmulc(v[it][q], w);
        }
      }
      dft<R, SIGN, T>::run(v[it]);
      const int o = (b / NS) * NS * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if constexpr (DST == DST_LDS) buf[t * ts + o + q * NS] = v[it][q];
        else if (!is_band<Store> || in_band<R>(q)) store(t, o + q * NS, v[it][q], it, q);
      }
    }
  }
  if constexpr (SRC == SRC_PRE) load.refill();
  if constexpr (DST != DST_FN) __syncthreads();
}

template <int N, int NS, int SIGN, int NB, int NT, int SRC, int DST, typename T, class Load, class Store, int R,
          int... Rest>
__device__ __forceinline__ void stockham_run(T* buf, int ts, int ntrans, const T* tw, Load& load, Store& store) {
  constexpr bool last = sizeof...(Rest) == 0;
  stockham_stage<N, R, NS, SIGN, NB, NT, SRC, (last ? DST : DST_LDS), T>(buf, ts, ntrans, tw, load, store);
  if constexpr (!last)
    stockham_run<N, NS * R, SIGN, NB, NT, SRC_LDS, DST, T, Load, Store, Rest...>(buf, ts, ntrans, tw, load, store);
}

template <int N, int SIGN, int NB, int NT, int SRC, int DST, typename T, class Load, class Store, int... Rs>
__device__ __forceinline__ void fft_io_impl(radix_list<Rs...>, T* buf, int ts, int ntrans, const T* tw, Load& load,
                                            Store& store) {
  stockham_run<N, 1, SIGN, NB, NT, SRC, DST, T, Load, Store, Rs...>(buf, ts, ntrans, tw, load, store);
}

// DFT  x_k = sum_j x_j exp(SIGN 2 pi i j k / N)  of transforms t < ntrans
// (t < NB) of a batch, block-collective.  buf[t*ts + 0..N-1] is the exchange
// buffer; inputs come from buf (SRC_LDS) or load (SRC_FN), outputs go to buf
// (DST_LDS) or store (DST_FN, DST_FN_LDS).  The caller must synchronise the
// block before a SRC_FN call whose first stage overwrites buf, and after a
// DST_FN call before buf is overwritten.
template <int N, int SIGN, int NB, int NT, int SRC, int DST, typename T, int V = 0, class Load, class Store>
__device__ __forceinline__ void fft_io(T* buf, int ts, int ntrans, const T* tw, Load&& load, Store&& store) {
  fft_io_impl<N, SIGN, NB, NT, SRC, DST, T>(typename plan_v<N, V>::list{}, buf, ts, ntrans, tw, load, store);
}

// First-stage inputs of one batch held in registers, so that the loads of the
// next batch can be issued before the current one is transformed.  HALF: the
// inputs are known to vanish outside the band e < N/4 or e >= 3N/4 (a sphere
// of planes |m| < N/4); the first-stage element q of a butterfly reads
// e = b + q*N/R, so only q < R/4 and q >= 3R/4 are held and loaded.
template <int N, int NB, int NT, typename T, typename L, bool HALF> struct first_stage_regs;
template <int N, int NB, int NT, typename T, int R, int... Rest, bool HALF>
struct first_stage_regs<N, NB, NT, T, radix_list<R, Rest...>, HALF> {
  static_assert(!HALF || R % 4 == 0, "band-limited input needs a first radix divisible by 4");
  static constexpr int radix = R;
  static constexpr int nb = NB, nt = NT;
  static constexpr int NBF = N / R;
  static constexpr int TOT = NB * NBF;
  static constexpr int items = (TOT + NT - 1) / NT;
  static constexpr int nq = HALF ? R / 2 : R;
  static constexpr bool held(int q) { return !HALF || q < R / 4 || q >= 3 * R / 4; }
  static constexpr int slot(int q) { return (!HALF || q < R / 4) ? q : q - R / 2; }
  T v[items][nq];
  __device__ __forceinline__ T get(int it, int q) const { return held(q) ? v[it][slot(q)] : T{0, 0}; }
};
template <int N, int NB, int NT, typename T, bool HALF = false, int V = 0>
using fft_regs = first_stage_regs<N, NB, NT, T, typename plan_v<N, V>::list, HALF>;

// SRC_PRE source: r holds the first-stage inputs; refill() is called once the
// first stage has consumed them and written its outputs, so that the loads it
// issues (typically the next batch into r) overlap the rest of the transform.
template <class FR, class F>
struct pre_src {
  FR& r;
  F refill;
};
template <class FR, class F>
__device__ __forceinline__ pre_src<FR, F> preloaded(FR& r, F refill) {
  return pre_src<FR, F>{r, refill};
}

// Load the first-stage inputs of transforms t < ntrans into the register
// set r (an fft_regs): load(t, e) as in fft_io.
template <class FR, class Load>
__device__ __forceinline__ void fft_preload_regs(FR& r, int ntrans, Load&& load) {
  constexpr int NB = FR::nb, NT = FR::nt;
  const int tid = fresh_tid<NT>();
#pragma unroll
  for (int it = 0; it < FR::items; ++it) {
    const int i = tid + it * NT;
    const int t = i % NB, b = i / NB;
    if ((FR::TOT % NT == 0 || i < FR::TOT) && t < ntrans) {
#pragma unroll
      for (int q = 0; q < FR::radix; ++q)
        if (FR::held(q)) r.v[it][FR::slot(q)] = load(t, b + q * FR::NBF);
    }
  }
}
template <int N, int NB, int NT, typename T, bool HALF, class Load>
__device__ __forceinline__ void fft_preload(fft_regs<N, NB, NT, T, HALF>& r, int ntrans, Load&& load) {
  fft_preload_regs(r, ntrans, load);
}

// In-place DFT of transforms in buf (natural order in and out).
template <int N, int SIGN, int NB, int NT, typename T>
__device__ __forceinline__ void fft_batch(T* buf, int ts, int ntrans, const T* tw) {
  fft_io<N, SIGN, NB, NT, SRC_LDS, DST_LDS, T>(buf, ts, ntrans, tw, no_load{}, no_store{});
}

// Output positions of the last stage: f(it, q, t, e) for every (item, q) the
// calling thread will produce (used to prefetch per-element data).
template <int N, int NB, int NT, int R, int NS, class F>
__device__ __forceinline__ void last_stage_positions_impl(int ntrans, F& f) {
  constexpr int NBF = N / R;
  constexpr int TOT = NB * NBF;
  constexpr int ITEMS = (TOT + NT - 1) / NT;
  const int tid = fresh_tid<NT>();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int i = tid + it * NT;
    const int t = i % NB, b = i / NB;
    if ((TOT % NT == 0 || i < TOT) && t < ntrans) {
      const int o = (b / NS) * NS * R + b % NS;
#pragma unroll
      for (int q = 0; q < R; ++q) f(it, q, t, o + q * NS);
    }
  }
}

template <int N, int NB, int NT, int NSacc, int R, int... Rest, class F>
__device__ __forceinline__ void last_positions_run(radix_list<R, Rest...>, int ntrans, F& f) {
  if constexpr (sizeof...(Rest) == 0) last_stage_positions_impl<N, NB, NT, R, NSacc>(ntrans, f);
  else last_positions_run<N, NB, NT, NSacc * R>(radix_list<Rest...>{}, ntrans, f);
}

template <int N, int NB, int NT, int V = 0, class F>
__device__ __forceinline__ void last_stage_positions(int ntrans, F&& f) {
  last_positions_run<N, NB, NT, 1>(typename plan_v<N, V>::list{}, ntrans, f);
}

// number of (item, q) slots per thread in the last stage
template <int N, int NB, int NT, typename L> struct last_stage_shape;
template <int N, int NB, int NT, int R> struct last_stage_shape<N, NB, NT, radix_list<R>> {
  static constexpr int radix = R;
  static constexpr int items = (NB * (N / R) + NT - 1) / NT;
};
template <int N, int NB, int NT, int R, int R2, int... Rest>
struct last_stage_shape<N, NB, NT, radix_list<R, R2, Rest...>> : last_stage_shape<N, NB, NT, radix_list<R2, Rest...>> {};
template <int N, int NB, int NT, int V = 0>
using last_shape = last_stage_shape<N, NB, NT, typename plan_v<N, V>::list>;

__device__ __forceinline__ int fold(int j, int n) { return 2 * j < n ? j : j - n; }
__device__ __forceinline__ int wrap(int m, int n) { return m < 0 ? m + n : m; }

}  // namespace ks
