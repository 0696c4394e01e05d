// Ground-state eigensolver kernels (Section "Ground-state solution"): the
// subspace diagonalisation (a Hermitian eigenproblem of the orbitals'
// Rayleigh-Ritz matrix, solved by parallel cyclic Jacobi rotations) and the
// per-orbital steps of the preconditioned steepest descent (residual, Teter
// preconditioner, exact line minimisation over the orbital and its
// direction).  All reductions run in a fixed order.
#include "ks_internal.h"

namespace ks {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ double2 cconj(double2 a) { return double2{a.x, -a.y}; }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return double2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return double2{a.x * s, a.y * s}; }

// ---------------------------------------------------------- Jacobi rotations
//
// Blocked cyclic Jacobi.  The (zero-padded) matrix of order N2 = a multiple
// of 2 BJ_B is cut into nblk = N2 / BJ_B index blocks.  Round t of a sweep
// pairs the blocks by the round-robin tournament (pair 0 is (m-1, t), pair
// k > 0 is ((t+k) mod (m-1), (t-k) mod (m-1)), m = nblk): over the m-1
// rounds every block meets every other once.  Each pair's 2 BJ_B x 2 BJ_B
// sub-problem gets one cyclic sweep of 2x2 rotations (same tournament inside)
// giving a unitary U; then A <- U^H A U and V <- V U with U block diagonal
// over the round's pairs.  Padding rows and columns are zero, so they are
// never rotated and stay decoupled.

__device__ __forceinline__ void round_pair(int t, int k, int m, int& p, int& q) {
  int a, b;
  if (k == 0) {
    a = m - 1;
    b = t;
  } else {
    a = (t + k) % (m - 1);
    b = (t - k + m - 1) % (m - 1);
  }
  p = min(a, b);
  q = max(a, b);
}

constexpr int BJ_B = 16;            // index block
constexpr int BJ_M = 2 * BJ_B;      // sub-problem order
constexpr int BJ_NT = 256;
static_assert(BJ_B * BJ_B == BJ_NT, "one thread per 2x2 block of a sub-problem");

// Rotation J (2x2, acting on indices p < q) with (J^H A J)_pq = 0 for the
// Hermitian block [[a, b], [conj(b), c]]: with b = |b| e^{i phi}, the phase
// D = diag(1, e^{-i phi}) makes the block real, and the real symmetric
// rotation [[cs, sn], [-sn, cs]] with t = tan(theta) the smaller root of
// t^2 + 2 tau t - 1 = 0, tau = (c - a) / (2|b|), zeroes it; J = D R, i.e.
//   J = [[cs, sn], [-f, g]],  f = sn e, g = cs e,  e = e^{-i phi}.
// With h = |tau| + sqrt(1 + tau^2) = 1/|t|: cs = h / sqrt(1 + h^2) and
// sn = sign(tau) / sqrt(1 + h^2), so the chain has two reciprocal square
// roots and one square root and no division.  An element so small against
// the diagonal gap that h^2 would overflow is left alone (the rotation angle
// would be below 1e-150).
struct Rot {
  double cs, sn;
  double2 f, g;
};

__device__ __forceinline__ Rot make_rot(double a, double c, double2 b) {
  Rot r{1.0, 0.0, double2{0.0, 0.0}, double2{1.0, 0.0}};
  const double b2 = b.x * b.x + b.y * b.y;
  if (b2 == 0.0) return r;
  const double rb = rsqrt(b2);   // 1 / |b|
  const double tau = 0.5 * (c - a) * rb;
  const double at = fabs(tau);
  if (!(at < 1e150)) return r;
  const double h = at + sqrt(fma(tau, tau, 1.0));
  const double rh = rsqrt(fma(h, h, 1.0));
  r.cs = h * rh;
  r.sn = tau >= 0.0 ? rh : -rh;
  const double2 e{b.x * rb, -b.y * rb};
  r.f = cscale(e, r.sn);
  r.g = cscale(e, r.cs);
  return r;
}

// (x0, x1) J: the row vector (x0, x1) times the rotation
__device__ __forceinline__ void rot_right(const Rot& r, double2 x0, double2 x1, double2& y0, double2& y1) {
  const double2 a = cmul(x1, r.f), b = cmul(x1, r.g);
  y0 = double2{r.cs * x0.x - a.x, r.cs * x0.y - a.y};
  y1 = double2{r.sn * x0.x + b.x, r.sn * x0.y + b.y};
}

// J^H (x0, x1)^T: the rotation's adjoint times the column vector (x0, x1)
__device__ __forceinline__ void rot_left_adj(const Rot& r, double2 x0, double2 x1, double2& y0, double2& y1) {
  const double2 a = cmul(cconj(r.f), x1), b = cmul(cconj(r.g), x1);
  y0 = double2{r.cs * x0.x - a.x, r.cs * x0.y - a.y};
  y1 = double2{r.sn * x0.x + b.x, r.sn * x0.y + b.y};
}

// global index of local index l of block pair (I, J)
__device__ __forceinline__ int bj_index(int I, int J, int l) { return l < BJ_B ? I * BJ_B + l : J * BJ_B + (l - BJ_B); }

// Block k of round t: one cyclic sweep on the sub-problem of block pair k;
// its unitary goes to Ublk[k] (row-major BJ_M x BJ_M).  S and U are kept in
// two LDS copies: inner round r reads one and writes the other (every entry
// is rewritten), so a round needs one barrier.
__global__ __launch_bounds__(BJ_NT) void bj_solve_kernel(const double2* __restrict__ A, int N2, int t,
                                                         double2* __restrict__ Ublk) {
  __shared__ double2 S[2][BJ_M][BJ_M + 1];
  __shared__ double2 U[2][BJ_M][BJ_M + 1];
  const int k = blockIdx.x, tid = threadIdx.x;
  int I, J;
  round_pair(t, k, N2 / BJ_B, I, J);
  for (int e = tid; e < BJ_M * BJ_M; e += BJ_NT) {
    const int r = e / BJ_M, c = e % BJ_M;
    S[0][r][c] = A[(long long)bj_index(I, J, r) * N2 + bj_index(I, J, c)];
    U[0][r][c] = double2{r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  const int P2 = tid / BJ_B, Q2 = tid % BJ_B;
  int cur = 0;
  for (int r = 0; r < BJ_M - 1; ++r) {
    // 2x2 block (P2, Q2) of S <- J^H S J, and columns pk of rows P2, P2 +
    // BJ_B of U <- U J (each entry has one owner); the block's entries are
    // read before the rotations are formed, so their LDS latency overlaps it
    int pi[2], pk[2];
    round_pair(r, P2, BJ_M, pi[0], pi[1]);
    round_pair(r, Q2, BJ_M, pk[0], pk[1]);
    double2 sv[2][2], uv[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        sv[a][b] = S[cur][pi[a]][pk[b]];
        uv[a][b] = U[cur][P2 + a * BJ_B][pk[b]];
      }
    // every thread forms the two rotations it applies (of its row pair and
    // its column pair) from the current copy, so no barrier publishes them
    const Rot ri = make_rot(S[cur][pi[0]][pi[0]].x, S[cur][pi[1]][pi[1]].x, S[cur][pi[0]][pi[1]]);
    const Rot rk = make_rot(S[cur][pk[0]][pk[0]].x, S[cur][pk[1]][pk[1]].x, S[cur][pk[0]][pk[1]]);
    double2 tr[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a) rot_right(rk, sv[a][0], sv[a][1], tr[a][0], tr[a][1]);
    const int nx = cur ^ 1;
#pragma unroll
    for (int j = 0; j < 2; ++j) rot_left_adj(ri, tr[0][j], tr[1][j], S[nx][pi[0]][pk[j]], S[nx][pi[1]][pk[j]]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = P2 + h * BJ_B;
      rot_right(rk, uv[h][0], uv[h][1], U[nx][row][pk[0]], U[nx][row][pk[1]]);
    }
    __syncthreads();
    cur = nx;
  }
  double2* out = Ublk + (long long)k * BJ_M * BJ_M;
  for (int e = tid; e < BJ_M * BJ_M; e += BJ_NT) out[e] = U[cur][e / BJ_M][e % BJ_M];
}

constexpr int BJ_VCOLS = 64;   // columns of V per block of the V update
constexpr int BJ_LD = BJ_M + 1;

// Round t: blocks [0, P^2) form An[rows of pair a][columns of pair b] =
// U_a^H A U_b; the remaining blocks form the rows of pair a of Vn = (V U)^T
// over BJ_VCOLS columns: Vn[g(i)][c] = sum_k U_a[k][i] Vt[g(k)][c] (the
// BJ_M rows of Vt staged in LDS first).
__global__ __launch_bounds__(BJ_NT) void bj_apply_kernel(const double2* __restrict__ A, double2* __restrict__ An,
                                                         const double2* __restrict__ Vt, double2* __restrict__ Vn,
                                                         int N2, int t, const double2* __restrict__ Ublk) {
  // A blocks: Ua, Ub, X (BJ_M x BJ_LD each); V blocks: Ua, then the staged
  // rows of Vt (BJ_M x (BJ_VCOLS + 1))
  __shared__ double2 sm[3 * BJ_M * BJ_LD];
  static_assert(BJ_M * (BJ_VCOLS + 1) <= 2 * BJ_M * BJ_LD, "staged V rows fit the A-block buffers");
  double2* Ua = sm;
  double2* Ub = sm + BJ_M * BJ_LD;
  double2* X = sm + 2 * BJ_M * BJ_LD;
  const int tid = threadIdx.x, nblk = N2 / BJ_B, P = nblk / 2;
  constexpr int PER = BJ_M * BJ_M / BJ_NT;
  if ((int)blockIdx.x < P * P) {
    const int ka = blockIdx.x / P, kb = blockIdx.x % P;
    int Ia, Ja, Ib, Jb;
    round_pair(t, ka, nblk, Ia, Ja);
    round_pair(t, kb, nblk, Ib, Jb);
    const double2* ua = Ublk + (long long)ka * BJ_M * BJ_M;
    const double2* ub = Ublk + (long long)kb * BJ_M * BJ_M;
    for (int e = tid; e < BJ_M * BJ_M; e += BJ_NT) {
      const int r = e / BJ_M, c = e % BJ_M;
      Ua[r * BJ_LD + c] = ua[e];
      Ub[r * BJ_LD + c] = ub[e];
      X[r * BJ_LD + c] = A[(long long)bj_index(Ia, Ja, r) * N2 + bj_index(Ib, Jb, c)];
    }
    __syncthreads();
    double2 tmp[PER];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int e = tid + s * BJ_NT, r = e / BJ_M, c = e % BJ_M;
      double2 acc{0.0, 0.0};
      #pragma unroll 4
      for (int l = 0; l < BJ_M; ++l) acc = cadd(acc, cmul(X[r * BJ_LD + l], Ub[l * BJ_LD + c]));
      tmp[s] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int e = tid + s * BJ_NT;
      X[(e / BJ_M) * BJ_LD + e % BJ_M] = tmp[s];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int e = tid + s * BJ_NT, r = e / BJ_M, c = e % BJ_M;
      double2 acc{0.0, 0.0};
      #pragma unroll 4
      for (int l = 0; l < BJ_M; ++l) acc = cadd(acc, cmul(cconj(Ua[l * BJ_LD + r]), X[l * BJ_LD + c]));
      An[(long long)bj_index(Ia, Ja, r) * N2 + bj_index(Ib, Jb, c)] = acc;
    }
    return;
  }
  const int nch = (N2 + BJ_VCOLS - 1) / BJ_VCOLS;
  const int w = blockIdx.x - P * P, ka = w / nch, c0 = (w % nch) * BJ_VCOLS;
  if (ka >= P) return;
  int Ia, Ja;
  round_pair(t, ka, nblk, Ia, Ja);
  constexpr int VLD = BJ_VCOLS + 1;
  double2* Vs = sm + BJ_M * BJ_LD;
  const double2* ua = Ublk + (long long)ka * BJ_M * BJ_M;
  for (int e = tid; e < BJ_M * BJ_M; e += BJ_NT) Ua[(e / BJ_M) * BJ_LD + e % BJ_M] = ua[e];
  for (int e = tid; e < BJ_M * BJ_VCOLS; e += BJ_NT) {
    const int l = e / BJ_VCOLS, cc = e % BJ_VCOLS, c = c0 + cc;
    Vs[l * VLD + cc] = c < N2 ? Vt[(long long)bj_index(Ia, Ja, l) * N2 + c] : double2{0.0, 0.0};
  }
  __syncthreads();
  for (int e = tid; e < BJ_M * BJ_VCOLS; e += BJ_NT) {
    const int i = e / BJ_VCOLS, cc = e % BJ_VCOLS, c = c0 + cc;
    double2 acc{0.0, 0.0};
    #pragma unroll 4
    for (int l = 0; l < BJ_M; ++l) acc = cadd(acc, cmul(Ua[l * BJ_LD + i], Vs[l * VLD + cc]));
    if (c < N2) Vn[(long long)bj_index(Ia, Ja, i) * N2 + c] = acc;
  }
}

// A = (H + H^H) / 2 padded with zeros to order N2, Vt = I (order N2)
__global__ __launch_bounds__(256) void hermitize_kernel(const double2* __restrict__ H, int n, double2* __restrict__ A,
                                                        double2* __restrict__ Vt, int N2) {
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  if (g >= (long long)N2 * N2) return;
  const int i = (int)(g / N2), j = (int)(g % N2);
  double2 a{0.0, 0.0};
  if (i < n && j < n) {
    const double2 x = H[(long long)i * n + j], y = H[(long long)j * n + i];
    a = double2{0.5 * (x.x + y.x), 0.5 * (x.y - y.y)};
  }
  A[g] = a;
  Vt[g] = double2{i == j ? 1.0 : 0.0, 0.0};
}

constexpr int RED_NT = 256;

// Row i: part[2i] = sum_{j != i} |A_ij|^2, part[2i+1] = sum_j |A_ij|^2
// (fixed order); offdiag_sum_kernel adds the rows in order into out[0..1].
__global__ __launch_bounds__(RED_NT) void offdiag_rows_kernel(const double2* __restrict__ A, int n,
                                                              double* __restrict__ part) {
  __shared__ double s0[RED_NT], s1[RED_NT];
  const int i = blockIdx.x, tid = threadIdx.x;
  const double2* row = A + (long long)i * n;
  double off = 0.0, all = 0.0;
  for (int j = tid; j < n; j += RED_NT) {
    const double2 a = row[j];
    const double v = a.x * a.x + a.y * a.y;
    all += v;
    if (j != i) off += v;
  }
  s0[tid] = off;
  s1[tid] = all;
  __syncthreads();
  for (int h = RED_NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      s0[tid] += s0[tid + h];
      s1[tid] += s1[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[2 * i] = s0[0];
    part[2 * i + 1] = s1[0];
  }
}

__global__ __launch_bounds__(RED_NT) void offdiag_sum_kernel(const double* __restrict__ part, int n,
                                                             double* __restrict__ out) {
  __shared__ double s0[RED_NT], s1[RED_NT];
  const int tid = threadIdx.x;
  double off = 0.0, all = 0.0;
  for (int i = tid; i < n; i += RED_NT) {
    off += part[2 * i];
    all += part[2 * i + 1];
  }
  s0[tid] = off;
  s1[tid] = all;
  __syncthreads();
  for (int h = RED_NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      s0[tid] += s0[tid + h];
      s1[tid] += s1[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

// Block i: eigenvalue lambda_i = A_ii goes to rank r_i (ascending; equal
// values by index); row r_i of Q receives eigenvector i scaled by the unit
// phase that makes its entry of largest modulus (the first on ties) real and
// positive.
__global__ __launch_bounds__(RED_NT) void eig_finish_kernel(const double2* __restrict__ A,
                                                            const double2* __restrict__ Vt, int n, int ld,
                                                            double* __restrict__ eig, double2* __restrict__ Q) {
  __shared__ double sm[RED_NT];
  __shared__ int si[RED_NT], sc[RED_NT];
  const int i = blockIdx.x, tid = threadIdx.x;
  const double li = A[(long long)i * ld + i].x;
  const double2* v = Vt + (long long)i * ld;
  double best = -1.0;
  int bi = n, cnt = 0;
  for (int j = tid; j < n; j += RED_NT) {
    const double2 x = v[j];
    const double mg = x.x * x.x + x.y * x.y;
    if (mg > best) {
      best = mg;
      bi = j;
    }
    const double lj = A[(long long)j * ld + j].x;
    cnt += (lj < li || (lj == li && j < i)) ? 1 : 0;
  }
  sm[tid] = best;
  si[tid] = bi;
  sc[tid] = cnt;
  __syncthreads();
  for (int h = RED_NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      const double mo = sm[tid + h];
      const int io = si[tid + h];
      if (mo > sm[tid] || (mo == sm[tid] && io < si[tid])) {
        sm[tid] = mo;
        si[tid] = io;
      }
      sc[tid] += sc[tid + h];
    }
    __syncthreads();
  }
  const int k = si[0], r = sc[0];
  const double2 vk = v[k];
  const double mk = sqrt(vk.x * vk.x + vk.y * vk.y);
  const double2 ph{vk.x / mk, -vk.y / mk};
  double2* out = Q + (long long)r * n;
  for (int j = tid; j < n; j += RED_NT) out[j] = (j == k) ? double2{mk, 0.0} : cmul(v[j], ph);
  if (tid == 0) eig[r] = li;
}

// ------------------------------------------------------ steepest descent

constexpr int SD_NT = 512;

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[SD_NT]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int a = 0; a < NV; ++a) sh[a][tid] = v[a];
  __syncthreads();
  for (int h = SD_NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int a = 0; a < NV; ++a) sh[a][tid] += sh[a][tid + h];
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = sh[a][0];
  __syncthreads();
}

// Teter-Payne-Allan factor (27 + 18x + 12x^2 + 8x^3) / (same + 16x^4)
__device__ __forceinline__ double teter(double x) {
  const double x2 = x * x, x3 = x2 * x;
  const double num = 27.0 + 18.0 * x + 12.0 * x2 + 8.0 * x3;
  return num / (num + 16.0 * x2 * x2);
}

// Block o (one orbital): r = w - e c, T = sum K|r|^2 / sum |r|^2,
// p = teter(K/T) r (p = r when T = 0, p = 0 when r = 0), p <- p - <c|p> c,
// q = p / |p| (q = 0 when p = 0).  resid[o] = |r|.
__global__ __launch_bounds__(SD_NT) void sd_direction_kernel(const double2* __restrict__ C, const double2* __restrict__ W,
                                                             const double* __restrict__ e, const double* __restrict__ kin,
                                                             double2* __restrict__ Qd, double* __restrict__ resid,
                                                             int npw, int stride) {
  __shared__ double sh[2][SD_NT];
  const int o = blockIdx.x, tid = threadIdx.x;
  const double2* c = C + (long long)o * stride;
  const double2* w = W + (long long)o * stride;
  double2* q = Qd + (long long)o * stride;
  const double eo = e[o];
  double v[2] = {0.0, 0.0};
  for (int g = tid; g < npw; g += SD_NT) {
    const double2 cg = c[g], wg = w[g];
    const double2 r{wg.x - eo * cg.x, wg.y - eo * cg.y};
    const double rr = r.x * r.x + r.y * r.y;
    v[0] += rr;
    v[1] += kin[g] * rr;
  }
  block_sum<2>(v, sh);
  const double rr = v[0], kr = v[1];
  if (tid == 0) resid[o] = sqrt(rr);
  if (rr == 0.0) {
    for (int g = tid; g < npw; g += SD_NT) q[g] = double2{0.0, 0.0};
    return;
  }
  const double T = kr / rr;
  const bool flat = !(T > 0.0);
  const double invT = flat ? 0.0 : 1.0 / T;
  double u[2] = {0.0, 0.0};
  for (int g = tid; g < npw; g += SD_NT) {
    const double2 cg = c[g], wg = w[g];
    const double f = flat ? 1.0 : teter(kin[g] * invT);
    const double2 p{f * (wg.x - eo * cg.x), f * (wg.y - eo * cg.y)};
    u[0] += cg.x * p.x + cg.y * p.y;   // <c|p>
    u[1] += cg.x * p.y - cg.y * p.x;
  }
  block_sum<2>(u, sh);
  const double2 cp{u[0], u[1]};
  double nn[1] = {0.0};
  for (int g = tid; g < npw; g += SD_NT) {
    const double2 cg = c[g], wg = w[g];
    const double f = flat ? 1.0 : teter(kin[g] * invT);
    const double2 p{f * (wg.x - eo * cg.x) - (cp.x * cg.x - cp.y * cg.y),
                    f * (wg.y - eo * cg.y) - (cp.x * cg.y + cp.y * cg.x)};
    nn[0] += p.x * p.x + p.y * p.y;
  }
  block_sum<1>(nn, sh);
  const double s = nn[0] > 0.0 ? 1.0 / sqrt(nn[0]) : 0.0;
  for (int g = tid; g < npw; g += SD_NT) {
    const double2 cg = c[g], wg = w[g];
    const double f = flat ? 1.0 : teter(kin[g] * invT);
    const double2 p{f * (wg.x - eo * cg.x) - (cp.x * cg.x - cp.y * cg.y),
                    f * (wg.y - eo * cg.y) - (cp.x * cg.y + cp.y * cg.x)};
    q[g] = double2{p.x * s, p.y * s};
  }
}

// Block o: beta = <c|Hq>, d = <q|Hq>; the lowest eigenvector y of
// [[e, beta], [conj(beta), d]] (|y| = 1, y0 real >= 0; y1 real > 0 when
// y0 = 0) replaces c by y0 c + y1 q.  Nothing changes when q = 0.
__global__ __launch_bounds__(SD_NT) void sd_update_kernel(double2* __restrict__ C, const double2* __restrict__ Qd,
                                                          const double2* __restrict__ HQ, const double* __restrict__ e,
                                                          int npw, int stride) {
  __shared__ double sh[4][SD_NT];
  const int o = blockIdx.x, tid = threadIdx.x;
  double2* c = C + (long long)o * stride;
  const double2* q = Qd + (long long)o * stride;
  const double2* hq = HQ + (long long)o * stride;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = tid; g < npw; g += SD_NT) {
    const double2 cg = c[g], qg = q[g], hg = hq[g];
    v[0] += cg.x * hg.x + cg.y * hg.y;   // <c|Hq>
    v[1] += cg.x * hg.y - cg.y * hg.x;
    v[2] += qg.x * hg.x + qg.y * hg.y;   // Re <q|Hq>
    v[3] += qg.x * qg.x + qg.y * qg.y;   // |q|^2
  }
  block_sum<4>(v, sh);
  if (v[3] == 0.0) return;
  const double a = e[o], d = v[2];
  const double2 b{v[0], v[1]};
  const double bb = sqrt(b.x * b.x + b.y * b.y);
  const double h = 0.5 * (a - d), rad = sqrt(h * h + bb * bb);
  double y0;
  double2 y1;
  if (bb == 0.0) {
    y0 = a <= d ? 1.0 : 0.0;
    y1 = double2{a <= d ? 0.0 : 1.0, 0.0};
  } else if (h <= 0.0) {
    // a <= d: y = (d - lambda, -conj(b)), d - lambda = rad - h >= 0
    y0 = rad - h;
    y1 = double2{-b.x, b.y};
  } else {
    // a > d: y = (|b|, -(a - lambda) conj(b) / |b|), a - lambda = h + rad
    y0 = bb;
    const double s = -(h + rad) / bb;
    y1 = double2{s * b.x, -s * b.y};
  }
  const double nrm = sqrt(y0 * y0 + y1.x * y1.x + y1.y * y1.y);
  y0 /= nrm;
  y1 = double2{y1.x / nrm, y1.y / nrm};
  for (int g = tid; g < npw; g += SD_NT) {
    const double2 cg = c[g], qg = q[g];
    c[g] = double2{y0 * cg.x + (y1.x * qg.x - y1.y * qg.y), y0 * cg.y + (y1.x * qg.y + y1.y * qg.x)};
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

int bj_order(int n) { return (n + BJ_M - 1) / BJ_M * BJ_M; }

int bj_rounds(int n) { return bj_order(n) / BJ_B - 1; }

size_t bj_work_elems(int n) {
  const size_t N2 = (size_t)bj_order(n);
  return 4 * N2 * N2 + (N2 / BJ_M) * BJ_M * BJ_M;
}

void launch_hermitize(int n, const double2* H, double2* A, double2* Vt, hipStream_t st) {
  const int N2 = bj_order(n);
  hermitize_kernel<<<(unsigned)(((long long)N2 * N2 + 255) / 256), 256, 0, st>>>(H, n, A, Vt, N2);
}

void launch_bj_round(int n, const double2* A, double2* An, const double2* Vt, double2* Vn, double2* Ublk, int t,
                     hipStream_t st) {
  const int N2 = bj_order(n), P = N2 / BJ_M, nch = (N2 + BJ_VCOLS - 1) / BJ_VCOLS;
  bj_solve_kernel<<<P, BJ_NT, 0, st>>>(A, N2, t, Ublk);
  bj_apply_kernel<<<P * P + P * nch, BJ_NT, 0, st>>>(A, An, Vt, Vn, N2, t, Ublk);
}

void launch_offdiag(int n, const double2* A, double* part, double* out, hipStream_t st) {
  offdiag_rows_kernel<<<n, RED_NT, 0, st>>>(A, n, part);
  offdiag_sum_kernel<<<1, RED_NT, 0, st>>>(part, n, out);
}

void launch_eig_finish(int n, const double2* A, const double2* Vt, double* eig, double2* Q, hipStream_t st) {
  eig_finish_kernel<<<n, RED_NT, 0, st>>>(A, Vt, n, bj_order(n), eig, Q);
}

void launch_sd_direction(int norb, int npw, int stride, const double2* C, const double2* W, const double* e,
                         const double* kin, double2* Qd, double* resid, hipStream_t st) {
  sd_direction_kernel<<<norb, SD_NT, 0, st>>>(C, W, e, kin, Qd, resid, npw, stride);
}

void launch_sd_update(int norb, int npw, int stride, double2* C, const double2* Qd, const double2* HQ, const double* e,
                      hipStream_t st) {
  sd_update_kernel<<<norb, SD_NT, 0, st>>>(C, Qd, HQ, e, npw, stride);
}

}  // namespace ks
