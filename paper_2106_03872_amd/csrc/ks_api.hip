// Host runtime of libks: system set-up (plane-wave sphere tables, twiddles,
// projector runs), workspace ownership and the C ABI entry points declared in
// include/ks.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ks_internal.h"

using namespace ks;

namespace {

thread_local std::string g_create_err;

ks_status fail(ks_system* s, ks_status st, const std::string& msg) {
  if (s) s->err = msg; else g_create_err = msg;
  return st;
}

#define KS_HIP(s, call)                                                                        \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail((s), e_ == hipErrorOutOfMemory ? KS_ENOMEM : KS_EDEVICE,                     \
                  std::string(#call) + ": " + hipGetErrorString(e_));                          \
  } while (0)

// ------------------------------------------------------------ device pool

constexpr size_t POOL_ALIGN = 256;

void* pool_alloc(ks_pool* p, size_t bytes) {
  bytes = (bytes + POOL_ALIGN - 1) / POOL_ALIGN * POOL_ALIGN;
  std::lock_guard<std::mutex> lk(p->mu);
  for (auto it = p->free_ranges.begin(); it != p->free_ranges.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t off = it->first, rest = it->second - bytes;
    p->free_ranges.erase(it);
    if (rest) p->free_ranges[off + bytes] = rest;
    p->live[off] = bytes;
    p->used += bytes;
    p->peak = std::max(p->peak, p->used);
    return p->base + off;
  }
  return nullptr;
}

void pool_free(ks_pool* p, void* ptr) {
  std::lock_guard<std::mutex> lk(p->mu);
  const size_t off = (size_t)((char*)ptr - p->base);
  auto it = p->live.find(off);
  if (it == p->live.end()) return;
  size_t start = off, len = it->second;
  p->used -= len;
  p->live.erase(it);
  auto nx = p->free_ranges.lower_bound(start);
  if (nx != p->free_ranges.end() && nx->first == start + len) {   // merge with the next free range
    len += nx->second;
    nx = p->free_ranges.erase(nx);
  }
  if (nx != p->free_ranges.begin()) {                               // and with the previous one
    auto pv = std::prev(nx);
    if (pv->first + pv->second == start) {
      start = pv->first;
      len += pv->second;
      p->free_ranges.erase(pv);
    }
  }
  p->free_ranges[start] = len;
}

ks_status dalloc(ks_system* s, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (s && s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (s && s->pool) {
    *p = pool_alloc(s->pool, bytes);
    if (!*p) return fail(s, KS_ENOMEM, "device pool exhausted (" + std::to_string(bytes) + " B requested)");
    return KS_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(s, KS_ENOMEM, "hipMalloc(" + std::to_string(bytes) + " B): " + hipGetErrorString(e));
  }
  return KS_OK;
}

// The caller makes sure no enqueued work still uses p.
void dfree(ks_system* s, void*& p) {
  if (p) {
    if (s && s->pool) pool_free(s->pool, p);
    else if (!(s && s->pool_lost)) (void)hipFree(p);
  }
  p = nullptr;
}

// Record the system's completion event on st after the work a call enqueued
// (not while st is being captured into a graph: the capture's replays
// record it instead).
void track(ks_system* s, hipStream_t st) {
  if (!s || !s->done) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
    (void)hipEventRecord(s->done, st);
}

// Records the completion event when the enclosing call returns.
struct Track {
  ks_system* s;
  hipStream_t st;
  Track(ks_system* s_, void* stream) : s(s_), st((hipStream_t)stream) {}
  ~Track() { track(s, st); }
};

// Wait until the work the system enqueued has finished (its own work only).
void wait_own(ks_system* s) {
  if (s && s->done) (void)hipEventSynchronize(s->done);
}

template <typename T> ks_status upload(ks_system* s, T** dst, const std::vector<T>& v) {
  dfree(s, reinterpret_cast<void*&>(*dst));
  ks_status st = dalloc(s, reinterpret_cast<void**>(dst), v.size() * sizeof(T));
  if (st != KS_OK) return st;
  if (!v.empty()) KS_HIP(s, hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return KS_OK;
}

ks_status launch_ok(ks_system* s, bool ok, const char* what) {
  if (!ok) return fail(s, KS_EUNSUPPORTED, std::string("no kernel for this size: ") + what);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(s, KS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return KS_OK;
}

// ---------------------------------------------------------------- timing
constexpr int EV_PAIRS = 16384;

void timing_flush(ks_system* s) {
  for (int i = 0; i < s->ev_used; ++i) {
    float ms = 0.0f;
    if (hipEventSynchronize(s->ev[2 * i + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, s->ev[2 * i], s->ev[2 * i + 1]) == hipSuccess) {
      s->kt_ms[s->ev_kid[i]] += ms;
      s->kt_n[s->ev_kid[i]] += 1;
    }
  }
  s->ev_used = 0;
}

void timing_free(ks_system* s) {
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  s->ev.clear();
  s->ev_kid.clear();
  s->ev_used = 0;
  s->timing = false;
}

// Launch one kernel (f returns false when the size has no kernel); with
// timing on, bracket it by an event pair on its stream.
template <typename F> ks_status kcall(ks_system* s, int kid, hipStream_t st, const char* what, F&& f) {
  int slot = -1;
  if (s->timing) {
    if (s->ev_used == EV_PAIRS) timing_flush(s);
    slot = s->ev_used++;
    s->ev_kid[slot] = kid;
    (void)hipEventRecord(s->ev[2 * slot], st);
  }
  const bool ok = f();
  if (slot >= 0) (void)hipEventRecord(s->ev[2 * slot + 1], st);
  return launch_ok(s, ok, what);
}

// exp(-2 pi i j / n), computed in long double and rounded
std::vector<double2> twiddles(int n) {
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<double2> t(n);
  for (int j = 0; j < n; ++j) {
    const long double a = 2.0L * pi * (long double)j / (long double)n;
    t[j] = double2{(double)cosl(a), (double)(-sinl(a))};
  }
  return t;
}

std::vector<float2> twiddles_f(int n) {
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<float2> t(n);
  for (int j = 0; j < n; ++j) {
    const long double a = 2.0L * pi * (long double)j / (long double)n;
    t[j] = float2{(float)cosl(a), (float)(-sinl(a))};
  }
  return t;
}

// |G|^2/2 for integer frequencies (same operation order as the definition
// K = ((g0^2 + g1^2) + g2^2) / 2 with g_a = (2 pi m_a) / L_a)
double kin(const double L[3], int m0, int m1, int m2) {
  const double g0 = 2.0 * M_PI * m0 / L[0];
  const double g1 = 2.0 * M_PI * m1 / L[1];
  const double g2 = 2.0 * M_PI * m2 / L[2];
  return 0.5 * (g0 * g0 + g1 * g1 + g2 * g2);
}

// Packed plane-wave sphere (row a0): planes m0, columns m1, runs of m2.
struct SphereHost {
  std::vector<int> plane_col0, plane_m1lo, col_off, col_m2lo;
  int m0lo = 0, npw = 0, ncol_max = 0;
};

ks_status build_sphere(const int n[3], const double L[3], double ecut, SphereHost& h, std::string& err) {
  int prev_m0 = 0;
  bool any_plane = false;
  auto mlo = [&](int a) { return -(n[a] / 2); };
  auto mhi = [&](int a) { return (n[a] - 1) / 2; };
  for (int m0 = mlo(0); m0 <= mhi(0); ++m0) {
    int first_col = 0, prev_m1 = 0, ncol = 0;
    bool have_col = false;
    std::vector<int> coff, cm2;
    for (int m1 = mlo(1); m1 <= mhi(1); ++m1) {
      int lo = 1 << 30, hi = -(1 << 30), cnt = 0;
      for (int m2 = mlo(2); m2 <= mhi(2); ++m2) {
        if (ecut <= 0.0 || kin(L, m0, m1, m2) < ecut) {
          lo = std::min(lo, m2);
          hi = std::max(hi, m2);
          ++cnt;
        }
      }
      if (cnt == 0) continue;
      if (cnt != hi - lo + 1) { err = "sphere column is not contiguous"; return KS_EUNSUPPORTED; }
      // a sphere (not the whole box) must stay clear of the Nyquist planes
      // m_a = -n_a/2 of even sizes, where G and -G fold onto one box index
      if (ecut > 0.0 && ((n[0] % 2 == 0 && m0 == mlo(0)) || (n[1] % 2 == 0 && m1 == mlo(1)) ||
                         (n[2] % 2 == 0 && lo == mlo(2)))) {
        err = "the plane-wave sphere reaches a Nyquist plane of the grid";
        return KS_EINVAL;
      }
      if (have_col && m1 != prev_m1 + 1) { err = "sphere plane is not contiguous"; return KS_EUNSUPPORTED; }
      if (!have_col) first_col = m1;
      have_col = true;
      prev_m1 = m1;
      coff.push_back(h.npw);
      cm2.push_back(lo);
      h.npw += cnt;
      ++ncol;
    }
    if (ncol == 0) continue;
    if (any_plane && m0 != prev_m0 + 1) { err = "sphere planes are not contiguous"; return KS_EUNSUPPORTED; }
    if (!any_plane) h.m0lo = m0;
    any_plane = true;
    prev_m0 = m0;
    h.plane_col0.push_back((int)h.col_off.size());
    h.plane_m1lo.push_back(first_col);
    h.col_off.insert(h.col_off.end(), coff.begin(), coff.end());
    h.col_m2lo.insert(h.col_m2lo.end(), cm2.begin(), cm2.end());
    h.ncol_max = std::max(h.ncol_max, ncol);
  }
  if (!any_plane) { err = "the plane-wave sphere is empty"; return KS_EINVAL; }
  h.plane_col0.push_back((int)h.col_off.size());
  h.col_off.push_back(h.npw);
  return KS_OK;
}

// Kleinman-Bylander tables per x-tile (row a0 for Eq. vnl): slots (tile,
// atom) with their beta rows ordered (tile, atom, pencil, j0), and the unique
// grid points of each tile with their (slot, beta row) entries ordered by
// atom.  LDS positions are w*(n0+1) + j0 within the tile's pencil buffer.
struct ProjHost {
  int nproj = 1, npoints = 0, nruns = 0, ntiles = 0, xnb = 32, lanes = 256;
  std::vector<double> brows;
  std::vector<int> brow_input;   // input row of each beta row
  std::vector<int> pt_lds, slot_off, slot_atom, slot_pt, atom_slot_off, atom_slots;
  std::vector<int> up_off, up_lds, up_ent, ent_slot, ent_brow;
  std::vector<int4> item;
};

ks_status build_proj(const int n[3], int xnb, int lanes, int natoms, int nproj, const int* npts, const int* idx,
                     const double* beta, ProjHost& h, std::string& err) {
  if (natoms < 0) { err = "natoms < 0"; return KS_EINVAL; }
  if (natoms > 0 && (nproj < 1 || !npts)) { err = "nproj < 1 or npts is null"; return KS_EINVAL; }
  if (lanes < KB_TILE_DP) { err = "x-block narrower than the staged KB pairs"; return KS_EINVAL; }
  if (nproj > KB_MAX_NPROJ) {
    err = "more than " + std::to_string(KB_MAX_NPROJ) + " projectors per atom";
    return KS_EUNSUPPORTED;
  }
  const long long N = (long long)n[0] * n[1] * n[2];
  const int npl = n[1] * n[2];
  long long total = 0;
  for (int I = 0; I < natoms; ++I) {
    if (npts[I] < 0) { err = "negative npts"; return KS_EINVAL; }
    total += npts[I];
  }
  if (total > 0 && (!idx || !beta)) { err = "idx or beta is null"; return KS_EINVAL; }
  if (total > (1LL << 30)) { err = "too many projector points"; return KS_EINVAL; }
  const int np = std::max(1, nproj);
  const int NB = xnb, W = n[0] + 1;
  const int nt = (npl + NB - 1) / NB;
  h.nproj = np;
  h.npoints = (int)total;
  h.ntiles = nt;
  h.xnb = xnb;
  h.lanes = lanes;
  struct Pt { int tile, p, atom, j0, row; };
  std::vector<Pt> pts;
  pts.reserve(total);
  long long off = 0;
  for (int I = 0; I < natoms; ++I) {
    for (int j = 0; j < npts[I]; ++j, ++off) {
      const long long f = idx[off];
      if (f < 0 || f >= N) { err = "projector index outside the grid"; return KS_EINVAL; }
      const int p = (int)(f % npl);
      pts.push_back(Pt{p / NB, p, I, (int)(f / npl), (int)off});
    }
  }
  // projection side: order (tile, atom, pencil, j0)
  std::stable_sort(pts.begin(), pts.end(), [](const Pt& a, const Pt& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.atom != b.atom) return a.atom < b.atom;
    if (a.p != b.p) return a.p < b.p;
    return a.j0 < b.j0;
  });
  h.brows.assign((size_t)total * np, 0.0);
  h.brow_input.assign(total, 0);
  h.pt_lds.assign(total, 0);
  h.slot_off.assign(nt + 1, 0);
  std::vector<int> slot_of(pts.size());   // tile-local slot index of each beta row
  int local = -1;
  for (size_t k = 0; k < pts.size(); ++k) {
    const Pt& q = pts[k];
    const bool new_slot = k == 0 || q.tile != pts[k - 1].tile || q.atom != pts[k - 1].atom;
    const bool extend = !new_slot && q.p == pts[k - 1].p && q.j0 == pts[k - 1].j0 + 1;
    if (k == 0 || q.tile != pts[k - 1].tile) local = -1;
    if (new_slot) {
      h.slot_atom.push_back(q.atom);
      h.slot_pt.push_back((int)k);
      h.slot_off[q.tile + 1]++;
      ++local;
    }
    slot_of[k] = local;
    if (!extend) ++h.nruns;
    h.pt_lds[k] = (q.p - q.tile * NB) * W + q.j0;
    h.brow_input[k] = q.row;
    for (int c = 0; c < np; ++c) h.brows[k * np + c] = beta[(size_t)q.row * np + c];
  }
  const int nslots = (int)h.slot_atom.size();
  h.slot_pt.push_back((int)total);
  for (int t = 0; t < nt; ++t) {
    h.slot_off[t + 1] += h.slot_off[t];
    if ((h.slot_off[t + 1] - h.slot_off[t]) * np > KB_TILE_DP) {
      err = "too many atoms touch one x-tile (" + std::to_string(h.slot_off[t + 1] - h.slot_off[t]) + " x " +
            std::to_string(np) + " projectors > " + std::to_string(KB_TILE_DP) + ")";
      return KS_EUNSUPPORTED;
    }
  }
  // Projection work of each lane of a tile's block: every (slot, projector)
  // pair gets 2^g adjacent lanes (g = 0..4, aligned to 2^g), enough that each
  // lane's share of the slot's beta rows fits the registers cached across
  // orbitals; when a tile would need more lanes than the block has, the
  // largest groups are halved (their lanes then loop over extra rows).
  // item = (first row, end row, local slot * nproj + projector, g | 256 for
  // the group's first lane).
  h.item.assign((size_t)nt * lanes, make_int4(0, 0, 0, 0));
  for (int t = 0; t < nt; ++t) {
    const int s0 = h.slot_off[t], ns = h.slot_off[t + 1] - s0;
    std::vector<int> lg(ns, 0);
    for (int j = 0; j < ns; ++j) {
      const int len = h.slot_pt[s0 + j + 1] - h.slot_pt[s0 + j];
      const int need = (len + KB_CACHED_POINTS - 1) / KB_CACHED_POINTS;
      while ((1 << lg[j]) < need && lg[j] < KB_MAX_GROUP_LOG) ++lg[j];
    }
    for (;;) {
      long long used = 0;
      for (int j = 0; j < ns; ++j) used += (long long)np << lg[j];
      if (used <= lanes) break;
      int jm = 0;
      for (int j = 1; j < ns; ++j)
        if (lg[j] > lg[jm]) jm = j;
      --lg[jm];
    }
    std::vector<int> order(ns);
    for (int j = 0; j < ns; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lg[a] > lg[b]; });
    int base = 0;
    for (int j : order) {
      const int k0 = h.slot_pt[s0 + j], len = h.slot_pt[s0 + j + 1] - k0, g = 1 << lg[j];
      for (int q = 0; q < np; ++q, base += g)
        for (int sg = 0; sg < g; ++sg)
          h.item[(size_t)t * lanes + base + sg] =
              make_int4(k0 + (int)((long long)len * sg / g), k0 + (int)((long long)len * (sg + 1) / g), j * np + q,
                        lg[j] | (sg == 0 ? 256 : 0));
    }
  }
  h.atom_slot_off.assign(natoms + 1, 0);
  h.atom_slots.assign(nslots, 0);
  for (int k = 0; k < nslots; ++k) h.atom_slot_off[h.slot_atom[k] + 1]++;
  for (int I = 0; I < natoms; ++I) h.atom_slot_off[I + 1] += h.atom_slot_off[I];
  {
    std::vector<int> fill(h.atom_slot_off.begin(), h.atom_slot_off.end() - 1);
    for (int k = 0; k < nslots; ++k) h.atom_slots[fill[h.slot_atom[k]]++] = k;
  }
  // scatter side: order (tile, pencil, j0, atom); one entry per (point, atom)
  std::vector<int> order(pts.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const Pt& x = pts[a];
    const Pt& y = pts[b];
    if (x.tile != y.tile) return x.tile < y.tile;
    if (x.p != y.p) return x.p < y.p;
    if (x.j0 != y.j0) return x.j0 < y.j0;
    return x.atom < y.atom;
  });
  h.up_off.assign(nt + 1, 0);
  for (size_t i = 0; i < order.size(); ++i) {
    const Pt& q = pts[order[i]];
    const bool new_pt = i == 0 || q.tile != pts[order[i - 1]].tile || q.p != pts[order[i - 1]].p ||
                        q.j0 != pts[order[i - 1]].j0;
    if (new_pt) {
      h.up_lds.push_back((q.p - q.tile * NB) * W + q.j0);
      h.up_ent.push_back((int)h.ent_slot.size());
      h.up_off[q.tile + 1]++;
    }
    h.ent_slot.push_back(slot_of[order[i]]);
    h.ent_brow.push_back(order[i]);
  }
  h.up_ent.push_back((int)h.ent_slot.size());
  for (int t = 0; t < nt; ++t) h.up_off[t + 1] += h.up_off[t];
  return KS_OK;
}

void free_workspace(ks_system* s) {
  for (auto& p : s->pk) dfree(s, p);
  dfree(s, s->T);
  dfree(s, s->U);
  dfree(s, s->partial);
  dfree(s, reinterpret_cast<void*&>(s->DP));
  dfree(s, reinterpret_cast<void*&>(s->dens_part));
  s->partial_cap = s->dp_cap = 0;
}

void free_gtab(ks_system* s, GTab& g) {
  void* w = g.w;
  void* part = g.part;
  dfree(s, w);
  dfree(s, part);
  g = GTab{};
}

ks_status alloc_proj_workspace(ks_system* s) {
  dfree(s, s->partial);
  dfree(s, reinterpret_cast<void*&>(s->DP));
  if (s->gp.P > 0) {   // the reciprocal-space product's partials follow the pass size
    void* part = s->gp.part;
    dfree(s, part);
    s->gp.part = nullptr;
    s->gp.part_bytes = 0;
    const size_t bytes = gproj_part_bytes(s->cb, s->gp.ncol, s->gp.kpad / 32);
    ks_status st = dalloc(s, &part, bytes);
    if (st != KS_OK) return st;
    s->gp.part = static_cast<float*>(part);
    s->gp.part_bytes = bytes;
  }
  const size_t pbytes = (size_t)s->cb * std::max(1, s->nslots) * std::max(1, s->nproj) * sizeof(double2);
  const size_t dbytes = (size_t)s->cb * std::max(1, s->natoms) * std::max(1, s->nproj) * sizeof(double2);
  ks_status st = dalloc(s, &s->partial, pbytes);
  if (st != KS_OK) return st;
  st = dalloc(s, reinterpret_cast<void**>(&s->DP), dbytes);
  if (st != KS_OK) return st;
  s->partial_cap = pbytes;
  s->dp_cap = dbytes;
  return KS_OK;
}

ks_status alloc_workspace(ks_system* s) {
  free_workspace(s);
  const size_t es = s->prec == KS_FP64 ? sizeof(double2) : sizeof(float2);   // working precision
  for (int i = 0; i < 3; ++i) {
    // pk[0] holds the FP64 orbital state / Taylor accumulator
    ks_status st = dalloc(s, &s->pk[i], (size_t)s->cb * s->npw_stride * (i == 0 ? sizeof(double2) : es));
    if (st != KS_OK) return st;
  }
  {
    ks_status st = dalloc(s, reinterpret_cast<void**>(&s->dens_part),
                          (size_t)((s->cb + 7) / 8) * s->N * sizeof(double));
    if (st != KS_OK) return st;
  }
  const size_t tb = (size_t)s->cb * s->nplanes * s->npl * es;
  ks_status st = dalloc(s, &s->T, tb);
  if (st != KS_OK) return st;
  st = dalloc(s, &s->U, tb);
  if (st != KS_OK) return st;
  return alloc_proj_workspace(s);
}

// Default orbitals per pass: as many as give KS_CHUNK_BYTES of plane
// intermediate T (larger passes mean fewer, fuller launches; 1024 orbitals
// of a 120^3 grid in one pass: 12.5 GB each for T and U in FP64).
constexpr double KS_CHUNK_BYTES = 16.0 * 1024 * 1024 * 1024;

int default_chunk(const ks_system* s) {
  const double per = (double)s->nplanes * s->npl * (s->prec == KS_FP64 ? sizeof(double2) : sizeof(float2));
  int cb = (int)std::max(1.0, std::floor(KS_CHUNK_BYTES / per));
  return std::max(1, std::min({cb, s->max_norb, KS_MAX_GRID_Y}));
}

// Orbitals per pass for a call over norb orbitals: the passes are balanced
// (ceil(norb / cb) passes of equal size up to one), so no pass is a small
// remainder that leaves most of the chip idle.
int chunk_len(const ks_system* s, int norb) {
  const int passes = (norb + s->cb - 1) / s->cb;
  return passes > 0 ? (norb + passes - 1) / passes : s->cb;
}

ks_status check_common(ks_system* s, int norb) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (norb < 0 || norb > s->max_norb)
    return fail(s, KS_EINVAL, "norb " + std::to_string(norb) + " outside [0, " + std::to_string(s->max_norb) + "]");
  return KS_OK;
}

// H applied to nb packed orbitals win; result per mode (see plane_fwd_kernel)
// win_fp64: the input is the FP64 orbital state (else the working precision)
// H applied to nb packed orbitals win.  With rho (only when natoms > 0), the
// x-projection pass also writes (or adds, accumulate) the density
// sum occ |win|^2 to rho.
ks_status hpsi_packed(ks_system* s, int nb, const void* win, bool win_fp64, void* wout, void* acc, HMode mode, Taylor tay,
                      hipStream_t st, const double* occ = nullptr, double* rho = nullptr, int accumulate = 0,
                      void* acc2 = nullptr) {
  ks_status r = kcall(s, KS_K_PLANE_INV, st, "plane_inv", [&] { return launch_plane_inv(s, nb, win, win_fp64, s->T, st); });
  if (r != KS_OK) return r;
  if (s->natoms > 0 && s->proj_mode == 1 && !rho) {
    r = kcall(s, KS_K_GPROJ, st, "gproj", [&] { return launch_gproj(s, nb, win, win_fp64, s->DP, st); });
    if (r != KS_OK) return r;
  } else if (s->natoms > 0) {
    r = kcall(s, KS_K_XPROJ, st, "xproj", [&] { return launch_xproj(s, nb, s->T, s->partial, occ, rho, accumulate, st); });
    if (r != KS_OK) return r;
    r = kcall(s, KS_K_PROJ_REDUCE, st, "proj_reduce", [&] { return launch_proj_reduce(s, nb, s->partial, s->DP, st); });
    if (r != KS_OK) return r;
  }
  r = kcall(s, KS_K_XAPPLY, st, "xapply", [&] { return launch_xapply(s, nb, s->T, s->DP, s->U, st); });
  if (r != KS_OK) return r;
  return kcall(s, KS_K_PLANE_FWD, st, "plane_fwd",
               [&] { return launch_plane_fwd(s, nb, s->U, win, win_fp64, wout, acc, acc2, mode, tay, st); });
}

ks_status density_packed(ks_system* s, int nb, const void* pk, const double* occ, double* rho, int accumulate,
                         hipStream_t st) {
  ks_status r = kcall(s, KS_K_PLANE_INV, st, "plane_inv", [&] { return launch_plane_inv(s, nb, pk, true, s->T, st); });
  if (r != KS_OK) return r;
  return kcall(s, KS_K_XDENS, st, "xdens", [&] { return launch_xdens(s, nb, s->T, occ, rho, accumulate, st); });
}

// (-i dt)^k / k!, k = 0..4 (truncated Taylor series of exp(-i H dt))
void taylor_coefficients(double dt, double2 coef[5]) {
  double re = 1.0, im = 0.0;
  coef[0] = double2{1.0, 0.0};
  for (int k = 1; k <= 4; ++k) {
    const double nr = im * dt, ni = -re * dt;  // multiply by -i dt
    re = nr / k;
    im = ni / k;
    coef[k] = double2{re, im};
  }
}

// nsteps Taylor-4 steps on nb packed FP64 orbitals `state` (stride npw_stride),
// in place.  With rho, the density after step s is written (accumulate = 0) or
// added (accumulate = 1) to rho + s*N: for s < nsteps-1 by the first H psi of
// step s+1, whose x-projection pass synthesises exactly those orbitals (when
// there are projectors), for the last step by a density pass.  With norms,
// ||c_o||^2 after step s goes to norms[s*norms_stride + o].
ks_status taylor_packed(ks_system* s, int nb, double2* state, double dt, int nsteps, const double* occ, double* rho,
                        int accumulate, double* norms, int norms_stride, hipStream_t st) {
  double2 coef[5];
  taylor_coefficients(dt, coef);
  ks_status r;
  const bool fuse = rho && s->natoms > 0;
  for (int step = 0; step < nsteps; ++step) {
    // w1 = H psi -> pk1, w2 -> pk2, w3 -> pk1, w4 not stored; state += a_k w_k
    void* src[4] = {state, s->pk[1], s->pk[2], s->pk[1]};
    void* dst[4] = {s->pk[1], s->pk[2], s->pk[1], nullptr};
    for (int k = 1; k <= 4; ++k) {
      Taylor tay{coef[k], k < 4 ? 1 : 0, {0.0, 0.0}};
      const bool in64 = k == 1 || s->prec == KS_FP64;
      double* rho_prev = (fuse && k == 1 && step > 0) ? rho + (size_t)(step - 1) * s->N : nullptr;
      if ((r = hpsi_packed(s, nb, src[k - 1], in64, dst[k - 1], state, H_TAYLOR, tay, st, occ, rho_prev,
                           accumulate)) != KS_OK)
        return r;
    }
    if (rho && (!fuse || step == nsteps - 1) &&
        (r = density_packed(s, nb, state, occ, rho + (size_t)step * s->N, accumulate, st)) != KS_OK)
      return r;
    if (norms) {
      if ((r = kcall(s, KS_K_DOTS, st, "dots", [&] { return launch_dots(s, nb, state, nullptr, s->red, st); })) != KS_OK)
        return r;
      KS_HIP(s, hipMemcpy2DAsync(norms + (size_t)step * norms_stride, sizeof(double), s->red, 2 * sizeof(double),
                                 sizeof(double), nb, hipMemcpyDeviceToDevice, st));
    }
  }
  return KS_OK;
}

// process-wide autotuning results: (grid, precision, sphere planes, orbitals
// per pass rounded up to a power of two) -> (group caps, x-tile shape)
using TuneKey = std::tuple<int, int, int, int, int, int>;
std::mutex g_tune_mu;
struct TuneResult {
  int xg = 0, pg = 0, shape = 0;   // group caps and x-tile shape (xg == 0: none)
};
std::map<TuneKey, TuneResult> g_tune_cache;

// Density of the nb-orbital passes of a resident state (all passes, in
// order) into rho.
ks_status state_density(ks_system* s, ks_state* t, const double2* orbitals, const double* occ, double* rho,
                        hipStream_t st) {
  const int cl = chunk_len(s, t->norb);
  for (int o0 = 0; o0 < t->norb; o0 += cl) {
    const int nb = std::min(cl, t->norb - o0);
    const ks_status r = density_packed(s, nb, orbitals + (size_t)o0 * s->npw_stride, occ + o0, rho, o0 > 0, st);
    if (r != KS_OK) return r;
  }
  return KS_OK;
}

// d_v = V_loc + V_H[d_rho_w] (+ v_xc[d_rho_w])
ks_status update_potential(ks_system* s, hipStream_t st) {
  if (!launch_hartree(s, s->d_rho_w, s->d_v, s->d_vloc, st)) return fail(s, KS_EUNSUPPORTED, "no Hartree kernel");
  if (s->xc == KS_XC_LDA) launch_lda_xc(s, s->d_rho_w, s->d_v, 1, st);
  return launch_ok(s, true, "hartree");
}

// nsteps ETRS steps (Eq. etrs) of the resident orbitals under the
// density-dependent H[n] = K + V_loc + V_H[n] + V_nl; see ks_state_propagate_etrs.
ks_status etrs_packed(ks_system* s, ks_state* t, double dt, int nsteps, const double* occ, double* rho, double* norms,
                      hipStream_t st) {
  double2 ch[5], cf[5];
  taylor_coefficients(0.5 * dt, ch);
  taylor_coefficients(dt, cf);
  const int cl = chunk_len(s, t->norb);
  const size_t row = (size_t)s->npw_stride * sizeof(double2);
  ks_status r;
  // H(t): the potential of the current orbitals
  if ((r = state_density(s, t, t->data, occ, s->d_rho_w, st)) != KS_OK) return r;
  if ((r = update_potential(s, st)) != KS_OK) return r;
  for (int step = 0; step < nsteps; ++step) {
    // w_k = H(t)^k c, shared: c <- sum_k (-i dt/2)^k/k! w_k (in place), predictor <- sum_k (-i dt)^k/k! w_k
    for (int o0 = 0; o0 < t->norb; o0 += cl) {
      const int nb = std::min(cl, t->norb - o0);
      double2* slice = t->data + (size_t)o0 * s->npw_stride;
      double2* pred = t->aux + (size_t)o0 * s->npw_stride;
      KS_HIP(s, hipMemcpyAsync(pred, slice, nb * row, hipMemcpyDeviceToDevice, st));
      void* src[4] = {slice, s->pk[1], s->pk[2], s->pk[1]};
      void* dst[4] = {s->pk[1], s->pk[2], s->pk[1], nullptr};
      for (int k = 1; k <= 4; ++k) {
        Taylor tay{ch[k], k < 4 ? 1 : 0, cf[k]};
        const bool in64 = k == 1 || s->prec == KS_FP64;
        if ((r = hpsi_packed(s, nb, src[k - 1], in64, dst[k - 1], slice, H_TAYLOR, tay, st, nullptr, nullptr, 0,
                             pred)) != KS_OK)
          return r;
      }
    }
    // H(t + dt) from the predictor's density (Eq. etrs0)
    if ((r = state_density(s, t, t->aux, occ, s->d_rho_w, st)) != KS_OK) return r;
    if ((r = update_potential(s, st)) != KS_OK) return r;
    // second half-step with H(t + dt)
    for (int o0 = 0; o0 < t->norb; o0 += cl) {
      const int nb = std::min(cl, t->norb - o0);
      if ((r = taylor_packed(s, nb, t->data + (size_t)o0 * s->npw_stride, 0.5 * dt, 1, nullptr, nullptr, 0, nullptr, 0,
                             st)) != KS_OK)
        return r;
    }
    // density (and potential) of the new orbitals
    if ((r = state_density(s, t, t->data, occ, s->d_rho_w, st)) != KS_OK) return r;
    if (rho)
      KS_HIP(s, hipMemcpyAsync(rho + (size_t)step * s->N, s->d_rho_w, s->N * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (norms) {
      for (int o0 = 0; o0 < t->norb; o0 += cl) {
        const int nb = std::min(cl, t->norb - o0);
        const double2* slice = t->data + (size_t)o0 * s->npw_stride;
        if ((r = kcall(s, KS_K_DOTS, st, "dots", [&] { return launch_dots(s, nb, slice, nullptr, s->red, st); })) != KS_OK)
          return r;
        KS_HIP(s, hipMemcpy2DAsync(norms + (size_t)step * t->norb + o0, sizeof(double), s->red, 2 * sizeof(double),
                                   sizeof(double), nb, hipMemcpyDeviceToDevice, st));
      }
    }
    if (step + 1 < nsteps && (r = update_potential(s, st)) != KS_OK) return r;
  }
  return KS_OK;
}

// Small matrices of the Cholesky orthonormalisation (max_norb^2), allocated
// on first use.
ks_status ensure_ortho_mats(ks_system* s) {
  if (s->ortho_S) return KS_OK;
  const size_t n = (size_t)s->max_norb;
  ks_status r;
  if ((r = dalloc(s, reinterpret_cast<void**>(&s->ortho_S), n * n * sizeof(double2))) != KS_OK ||
      (r = dalloc(s, reinterpret_cast<void**>(&s->ortho_W), n * n * sizeof(double2))) != KS_OK ||
      (r = dalloc(s, reinterpret_cast<void**>(&s->ortho_info), sizeof(int))) != KS_OK ||
      (r = dalloc(s, reinterpret_cast<void**>(&s->ortho_diag), n * sizeof(double))) != KS_OK ||
      ((s->gemm_part_bytes = gemm_part_bytes(s->max_norb, s->npw)) > 0 &&
       (r = dalloc(s, reinterpret_cast<void**>(&s->gemm_part), s->gemm_part_bytes)) != KS_OK)) {
    void* p[] = {s->ortho_S, s->ortho_W, s->ortho_info, s->ortho_diag, s->gemm_part};
    for (void* q : p) dfree(s, q);
    s->ortho_S = s->ortho_W = s->gemm_part = nullptr;
    s->gemm_part_bytes = 0;
    s->ortho_info = nullptr;
    s->ortho_diag = nullptr;
    return r;
  }
  return KS_OK;
}

// Cholesky orthonormalisation of n packed FP64 orbitals C (stride npw_stride)
// in place, through Y (n orbitals of scratch).  Synchronises the stream to
// read the factorisation's status.
ks_status orthonormalize_packed(ks_system* s, int n, double2* C, double2* Y, hipStream_t st) {
  ks_status r;
  const size_t ld = s->npw_stride;
  KS_HIP(s, hipMemsetAsync(s->ortho_info, 0, sizeof(int), st));
  if ((r = kcall(s, KS_K_GEMM, st, "overlap", [&] { return launch_overlap(n, s->npw, C, ld, s->ortho_S, s->gemm_part, s->gemm_part_bytes, st); })) != KS_OK)
    return r;
  if ((r = launch_ok(s, launch_cholesky(n, s->ortho_S, s->ortho_W, s->ortho_diag, s->ortho_info, st), "cholesky")) != KS_OK) return r;
  if ((r = launch_ok(s, launch_trtri(n, s->ortho_S, s->ortho_W, st), "trtri")) != KS_OK) return r;
  if ((r = kcall(s, KS_K_GEMM, st, "apply", [&] { return launch_apply_lower(n, s->npw, s->ortho_W, C, ld, Y, st); })) !=
      KS_OK)
    return r;
  int info = 0;
  KS_HIP(s, hipMemcpyAsync(&info, s->ortho_info, sizeof(int), hipMemcpyDeviceToHost, st));
  KS_HIP(s, hipStreamSynchronize(st));
  if (info) return fail(s, KS_EINVAL, "overlap matrix is not positive definite (orbitals linearly dependent)");
  KS_HIP(s, hipMemcpy2DAsync(C, ld * sizeof(double2), Y, ld * sizeof(double2), s->npw * sizeof(double2), n,
                             hipMemcpyDeviceToDevice, st));
  return KS_OK;
}

// Jacobi sweeps stop once the off-diagonal Frobenius norm is at most
// JACOBI_TOL of the whole matrix's.
constexpr double JACOBI_TOL = 1e-14;
constexpr int JACOBI_MAX_SWEEPS = 60;

// Eigenvalues (ascending, into eig) and eigenvectors (rows of Q, the phase
// of each fixed so that its largest entry is real and positive) of the
// Hermitian part of the n x n matrix H, by blocked Jacobi sweeps.  work:
// bj_work_elems(n); off: 2 + 2 bj_order(n) doubles.  Synchronises the stream
// once per sweep.
ks_status subspace_eigh(ks_system* s, int n, const double2* H, double2* work, double* off, double* eig, double2* Q,
                        hipStream_t st) {
  const int N2 = bj_order(n);
  const size_t nn = (size_t)N2 * N2;
  double2 *A = work, *An = work + nn, *V = work + 2 * nn, *Vn = work + 3 * nn, *Ublk = work + 4 * nn;
  ks_status r;
  if ((r = kcall(s, KS_K_EIG, st, "hermitize", [&] { launch_hermitize(n, H, A, V, st); return true; })) != KS_OK)
    return r;
  bool done = n < 2;
  for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS && !done; ++sweep) {
    for (int t = 0; t < bj_rounds(n); ++t) {
      if ((r = kcall(s, KS_K_EIG, st, "jacobi", [&] { launch_bj_round(n, A, An, V, Vn, Ublk, t, st); return true; })) !=
          KS_OK)
        return r;
      std::swap(A, An);
      std::swap(V, Vn);
    }
    if ((r = kcall(s, KS_K_EIG, st, "offdiag", [&] { launch_offdiag(N2, A, off + 2, off, st); return true; })) != KS_OK)
      return r;
    double h[2] = {0.0, 0.0};
    KS_HIP(s, hipMemcpyAsync(h, off, sizeof(h), hipMemcpyDeviceToHost, st));
    KS_HIP(s, hipStreamSynchronize(st));
    done = h[0] <= JACOBI_TOL * JACOBI_TOL * h[1];
  }
  if (!done) return fail(s, KS_EDEVICE, "subspace eigensolver: Jacobi sweeps did not converge");
  return kcall(s, KS_K_EIG, st, "eig_finish", [&] { launch_eig_finish(n, A, V, eig, Q, st); return true; });
}

}  // namespace

extern "C" {

static ks_status system_create(ks_pool* pool, const int n[3], const double L[3], double ecut, int precision,
                               int max_norb, int chunk, ks_system** out);

ks_status ks_system_create(const int n[3], const double L[3], double ecut, int precision, int max_norb,
                           ks_system** out) {
  return system_create(nullptr, n, L, ecut, precision, max_norb, 0, out);
}

static ks_status check_pool(ks_pool* pool, ks_system** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pool->device) {
    if (out) *out = nullptr;
    return fail(nullptr, KS_EINVAL, "the pool belongs to another device");
  }
  return KS_OK;
}

ks_status ks_system_create_in(ks_pool* pool, const int n[3], const double L[3], double ecut, int precision,
                              int max_norb, ks_system** out) {
  if (!pool) {
    if (out) *out = nullptr;
    return fail(nullptr, KS_EINVAL, "pool is null");
  }
  const ks_status r = check_pool(pool, out);
  return r != KS_OK ? r : system_create(pool, n, L, ecut, precision, max_norb, 0, out);
}

ks_status ks_system_create_ex(ks_pool* pool, const int n[3], const double L[3], double ecut, int precision,
                              int max_norb, int chunk, ks_system** out) {
  if (chunk < 0) {
    if (out) *out = nullptr;
    return fail(nullptr, KS_EINVAL, "chunk must be >= 0");
  }
  if (pool) {
    const ks_status r = check_pool(pool, out);
    if (r != KS_OK) return r;
  }
  return system_create(pool, n, L, ecut, precision, max_norb, chunk, out);
}

ks_status ks_stream_create(void** out) {
  if (!out) return fail(nullptr, KS_EINVAL, "out is null");
  *out = nullptr;
  hipStream_t st = nullptr;
  const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(nullptr, KS_EDEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
  *out = st;
  return KS_OK;
}

void ks_stream_destroy(void* stream) {
  if (stream) (void)hipStreamDestroy((hipStream_t)stream);
}

ks_status ks_pool_create(unsigned long long bytes, ks_pool** out) {
  if (!out) return fail(nullptr, KS_EINVAL, "out is null");
  *out = nullptr;
  if (bytes == 0) return fail(nullptr, KS_EINVAL, "pool size must be positive");
  ks_pool* p = new ks_pool();
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(nullptr, KS_EDEVICE, "hipGetDevice failed");
  }
  p->bytes = (size_t)(bytes + POOL_ALIGN - 1) / POOL_ALIGN * POOL_ALIGN;
  void* b = nullptr;
  const hipError_t e = hipMalloc(&b, p->bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return fail(nullptr, KS_ENOMEM, "hipMalloc(" + std::to_string(bytes) + " B): " + hipGetErrorString(e));
  }
  p->base = (char*)b;
  p->free_ranges[0] = p->bytes;
  *out = p;
  return KS_OK;
}

void ks_pool_destroy(ks_pool* p) {
  if (!p) return;
  // systems still alive lose their pool: their buffers go with it, and their
  // later frees do nothing
  for (ks_system* s : p->systems) {
    wait_own(s);
    s->pool = nullptr;
    s->pool_lost = true;
  }
  (void)hipFree(p->base);
  delete p;
}

ks_status ks_pool_usage(ks_pool* p, unsigned long long* used, unsigned long long* peak, unsigned long long* largest_free) {
  if (!p) return fail(nullptr, KS_EINVAL, "pool is null");
  std::lock_guard<std::mutex> lk(p->mu);
  if (used) *used = p->used;
  if (peak) *peak = p->peak;
  if (largest_free) {
    size_t m = 0;
    for (const auto& f : p->free_ranges) m = std::max(m, f.second);
    *largest_free = m;
  }
  return KS_OK;
}

static ks_status system_create(ks_pool* pool, const int n[3], const double L[3], double ecut, int precision,
                               int max_norb, int chunk, ks_system** out) {
  if (!out) return fail(nullptr, KS_EINVAL, "out is null");
  *out = nullptr;
  if (!n || !L) return fail(nullptr, KS_EINVAL, "n or L is null");
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return fail(nullptr, KS_EINVAL, "grid size must be positive");
    if (!(L[a] > 0.0) || !std::isfinite(L[a])) return fail(nullptr, KS_EINVAL, "cell lengths must be positive");
    if (!supported_size(n[a]))
      return fail(nullptr, KS_EUNSUPPORTED, "grid size " + std::to_string(n[a]) + " has no FFT kernel");
  }
  if (n[1] != n[2]) return fail(nullptr, KS_EINVAL, "n1 must equal n2");
  if (max_norb < 1) return fail(nullptr, KS_EINVAL, "max_norb must be >= 1");
  if (precision != KS_FP64 && precision != KS_MIXED) return fail(nullptr, KS_EUNSUPPORTED, "unknown precision");
  if (!std::isfinite(ecut)) return fail(nullptr, KS_EINVAL, "ecut must be finite");

  ks_system* s = new ks_system();
  s->pool = pool;
  if (pool) {
    std::lock_guard<std::mutex> lk(pool->mu);
    pool->systems.push_back(s);
  }
  if (hipEventCreateWithFlags(&s->done, hipEventDisableTiming) != hipSuccess) {
    s->done = nullptr;
    delete s;
    return fail(nullptr, KS_EDEVICE, "hipEventCreateWithFlags failed");
  }
  for (int a = 0; a < 3; ++a) {
    s->n[a] = n[a];
    s->L[a] = L[a];
  }
  s->ecut = ecut;
  s->prec = precision;
  s->max_norb = max_norb;
  s->N = (long long)n[0] * n[1] * n[2];
  s->npl = n[1] * n[2];
  s->omega = L[0] * L[1] * L[2];
  s->dV = s->omega / (double)s->N;

  SphereHost sh;
  {
    std::string msg;
    const ks_status r = build_sphere(n, L, ecut, sh, msg);
    if (r != KS_OK) {
      ks_system_destroy(s);
      return fail(nullptr, r, msg);
    }
  }
  std::vector<int>& plane_col0 = sh.plane_col0;
  std::vector<int>& plane_m1lo = sh.plane_m1lo;
  std::vector<int>& col_off = sh.col_off;
  std::vector<int>& col_m2lo = sh.col_m2lo;
  const int npw = sh.npw;
  s->m0lo = sh.m0lo;
  s->ncol_max = sh.ncol_max;
  for (size_t pi = 0; pi + 1 < sh.plane_col0.size(); ++pi)
    s->npp_max = std::max(s->npp_max, sh.col_off[sh.plane_col0[pi + 1]] - sh.col_off[sh.plane_col0[pi]]);
  s->nplanes = (int)plane_m1lo.size();
  s->ncols = (int)col_m2lo.size();
  s->npw = npw;
  s->npw_stride = (npw + 63) / 64 * 64;
  s->xshape = 0;
  s->xnb = x_shape_nb(n[0], 0);
  s->xnt = x_shape_threads(0);
  s->ntiles = (s->npl + s->xnb - 1) / s->xnb;
  s->x_half = s->m0lo >= -(n[0] / 4) && s->m0lo + s->nplanes - 1 < n[0] / 4;
  s->yz_half = true;
  for (int pi = 0; pi < s->nplanes; ++pi) {
    const int nc = plane_col0[pi + 1] - plane_col0[pi];
    if (plane_m1lo[pi] < -(n[1] / 4) || plane_m1lo[pi] + nc - 1 >= n[1] / 4) s->yz_half = false;
    for (int c = plane_col0[pi]; c < plane_col0[pi + 1]; ++c)
      if (col_m2lo[c] < -(n[2] / 4) || col_m2lo[c] + (col_off[c + 1] - col_off[c]) - 1 >= n[2] / 4) s->yz_half = false;
  }

  if (plane_lds_bytes(s) > 160 * 1024) {
    ks_system_destroy(s);
    return fail(nullptr, KS_EUNSUPPORTED, "plane-wave sphere too large for the plane pass LDS budget");
  }

  ks_status st;
  if ((st = upload(s, &s->d_plane_col0, plane_col0)) != KS_OK ||
      (st = upload(s, &s->d_plane_m1lo, plane_m1lo)) != KS_OK ||
      (st = upload(s, &s->d_col_off, col_off)) != KS_OK || (st = upload(s, &s->d_col_m2lo, col_m2lo)) != KS_OK ||
      (st = upload(s, &s->d_tw0, twiddles(n[0]))) != KS_OK || (st = upload(s, &s->d_tw1, twiddles(n[1]))) != KS_OK ||
      (st = upload(s, &s->d_tw0f, twiddles_f(n[0]))) != KS_OK || (st = upload(s, &s->d_tw1f, twiddles_f(n[1]))) != KS_OK) {
    g_create_err = s->err;
    ks_system_destroy(s);
    return st;
  }
  {
    // |G|^2/2 of each packed coefficient (preconditioner of the eigensolver)
    std::vector<double> kp((size_t)npw);
    for (int pi = 0; pi < s->nplanes; ++pi)
      for (int c = plane_col0[pi]; c < plane_col0[pi + 1]; ++c)
        for (int e = col_off[c]; e < col_off[c + 1]; ++e)
          kp[e] = kin(L, s->m0lo + pi, plane_m1lo[pi] + (c - plane_col0[pi]), col_m2lo[c] + (e - col_off[c]));
    if ((st = upload(s, &s->d_kin, kp)) != KS_OK) {
      g_create_err = s->err;
      ks_system_destroy(s);
      return st;
    }
  }
  if ((st = dalloc(s, reinterpret_cast<void**>(&s->d_v), s->N * sizeof(double))) != KS_OK ||
      (st = dalloc(s, reinterpret_cast<void**>(&s->d_vloc), s->N * sizeof(double))) != KS_OK ||
      (st = dalloc(s, reinterpret_cast<void**>(&s->d_hbox), s->N * sizeof(double2))) != KS_OK ||
      (st = dalloc(s, reinterpret_cast<void**>(&s->d_rho_w), s->N * sizeof(double))) != KS_OK ||
      (st = dalloc(s, reinterpret_cast<void**>(&s->red), 2 * (size_t)max_norb * sizeof(double))) != KS_OK) {
    g_create_err = s->err;
    ks_system_destroy(s);
    return st;
  }
  if (hipMemset(s->d_v, 0, s->N * sizeof(double)) != hipSuccess ||
      hipMemset(s->d_vloc, 0, s->N * sizeof(double)) != hipSuccess) {
    g_create_err = "hipMemset failed";
    ks_system_destroy(s);
    return KS_EDEVICE;
  }
  std::vector<int> zero_tiles(s->ntiles + 1, 0), zero1(1, 0);
  if ((st = upload(s, &s->d_slot_off, zero_tiles)) != KS_OK ||
      (st = upload(s, &s->d_up_off, zero_tiles)) != KS_OK || (st = upload(s, &s->d_atom_slot_off, zero1)) != KS_OK) {
    g_create_err = s->err;
    ks_system_destroy(s);
    return st;
  }
  s->cb = chunk > 0 ? std::min({chunk, max_norb, KS_MAX_GRID_Y}) : default_chunk(s);
  if ((st = alloc_workspace(s)) != KS_OK) {
    g_create_err = s->err;
    ks_system_destroy(s);
    return st;
  }
  *out = s;
  return KS_OK;
}

static void batch_release(ks_batch* b);
static void state_release(ks_state* t);

void ks_system_destroy(ks_system* s) {
  if (!s) return;
  wait_own(s);
  while (!s->batches.empty()) batch_release(s->batches.back());
  while (!s->states.empty()) state_release(s->states.back());
  if (s->pool) {
    std::lock_guard<std::mutex> lk(s->pool->mu);
    auto& v = s->pool->systems;
    v.erase(std::remove(v.begin(), v.end(), s), v.end());
  }
  timing_free(s);
  free_workspace(s);
  free_gtab(s, s->gp);
  void* ptrs[] = {s->d_plane_col0, s->d_plane_m1lo, s->d_col_off, s->d_col_m2lo, s->d_tw0, s->d_tw1,
                  s->d_tw0f, s->d_tw1f, s->d_v, s->d_vloc, s->d_kin, s->d_hbox, s->d_rho_w, s->d_pt_lds, s->d_slot_off, s->d_slot_atom, s->d_slot_pt,
                  s->d_atom_slot_off, s->d_atom_slots,
                  s->d_up_off, s->d_up_key, s->d_up_x, s->d_x_slot, s->d_beta, s->d_up_beta, s->d_x_beta, s->d_item,
                  s->d_kb, s->red, s->ortho_pk, s->ortho_S, s->ortho_W, s->ortho_info, s->ortho_diag, s->gemm_part};
  for (void* p : ptrs) dfree(s, p);
  if (s->done) (void)hipEventDestroy(s->done);
  delete s;
}

const char* ks_last_error(const ks_system* s) { return s ? s->err.c_str() : g_create_err.c_str(); }

int ks_system_npw(const ks_system* s) { return s ? s->npw : 0; }
int ks_system_chunk(const ks_system* s) { return s ? s->cb : 0; }

ks_status ks_system_set_chunk(ks_system* s, int chunk) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (chunk < 1 || chunk > s->max_norb || chunk > KS_MAX_GRID_Y)
    return fail(s, KS_EINVAL, "chunk outside [1, min(max_norb, " + std::to_string(KS_MAX_GRID_Y) + ")]");
  wait_own(s);
  s->cb = chunk;
  ++s->gen;
  return alloc_workspace(s);
}

ks_status ks_system_set_vloc(ks_system* s, const double* v, void* stream) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!v) return fail(s, KS_EINVAL, "v is null");
  Track tk(s, stream);
  KS_HIP(s, hipMemcpyAsync(s->d_v, v, s->N * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  KS_HIP(s, hipMemcpyAsync(s->d_vloc, v, s->N * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  s->have_v = true;
  return KS_OK;
}

// Uploads the per-tile projector tables ph (built for the system's current
// tile shape) and the KB energies d [natoms][nproj]; the caller has waited
// for the system's work.
static ks_status install_proj(ks_system* s, const ProjHost& ph, int natoms, const double* d) {
  const int np = ph.nproj;
  std::vector<double> kb((size_t)natoms * np);
  for (size_t k = 0; k < kb.size(); ++k) kb[k] = d[k];
  // scatter tables: the primary entry of each unique point stored with it
  const int nuniq = (int)ph.up_lds.size();
  std::vector<int> up_key(nuniq), up_x(nuniq), x_slot;
  std::vector<double> up_beta((size_t)nuniq * np), x_beta;
  for (int u = 0; u < nuniq; ++u) {
    const int e0 = ph.up_ent[u], e1 = ph.up_ent[u + 1];
    const int nx = e1 - e0 - 1, slot = ph.ent_slot[e0];
    if (ph.up_lds[u] >= (1 << UP_POS_BITS) || slot > UP_MAX_SLOT || nx > UP_MAX_EXTRA)
      return fail(s, KS_EUNSUPPORTED, "projector sphere overlap or x-tile too large for the scatter tables");
    up_key[u] = ph.up_lds[u] | slot << UP_POS_BITS | nx << (UP_POS_BITS + UP_SLOT_BITS);
    up_x[u] = (int)x_slot.size();
    for (int c = 0; c < np; ++c) up_beta[(size_t)u * np + c] = ph.brows[(size_t)ph.ent_brow[e0] * np + c];
    for (int e = e0 + 1; e < e1; ++e) {
      x_slot.push_back(ph.ent_slot[e]);
      for (int c = 0; c < np; ++c) x_beta.push_back(ph.brows[(size_t)ph.ent_brow[e] * np + c]);
    }
  }
  // New device copies first; the system's tables are replaced only when
  // every one of them was allocated and filled, so a failure (KS_ENOMEM)
  // leaves the old tables, shape and workspace in place.
  std::vector<void*> fresh;
  auto put = [&](auto& vec, auto** dst) -> ks_status {
    using T = typename std::decay_t<decltype(vec)>::value_type;
    *dst = nullptr;
    ks_status st = dalloc(s, reinterpret_cast<void**>(dst), vec.size() * sizeof(T));
    if (st != KS_OK) return st;
    fresh.push_back(*dst);
    if (!vec.empty())
      KS_HIP(s, hipMemcpy(*dst, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice));
    return KS_OK;
  };
  int *pt_lds, *slot_off, *slot_atom, *slot_pt, *atom_slot_off, *atom_slots, *up_off, *up_key2, *up_x2, *x_slot2;
  double *brows, *up_beta2, *x_beta2, *kb2;
  int4* item;
  void* partial = nullptr;
  double2* DP = nullptr;
  const int na = (natoms > 0 && ph.npoints > 0) ? natoms : 0;
  const size_t pbytes = (size_t)s->cb * std::max<size_t>(1, ph.slot_atom.size()) * std::max(1, np) * sizeof(double2);
  const size_t dbytes = (size_t)s->cb * std::max(1, na) * std::max(1, np) * sizeof(double2);
  ks_status st;
  if ((st = put(ph.pt_lds, &pt_lds)) != KS_OK || (st = put(ph.slot_off, &slot_off)) != KS_OK ||
      (st = put(ph.slot_atom, &slot_atom)) != KS_OK || (st = put(ph.slot_pt, &slot_pt)) != KS_OK ||
      (st = put(ph.atom_slot_off, &atom_slot_off)) != KS_OK || (st = put(ph.atom_slots, &atom_slots)) != KS_OK ||
      (st = put(ph.up_off, &up_off)) != KS_OK || (st = put(up_key, &up_key2)) != KS_OK ||
      (st = put(up_x, &up_x2)) != KS_OK || (st = put(x_slot, &x_slot2)) != KS_OK ||
      (st = put(ph.brows, &brows)) != KS_OK || (st = put(up_beta, &up_beta2)) != KS_OK ||
      (st = put(x_beta, &x_beta2)) != KS_OK || (st = put(kb, &kb2)) != KS_OK || (st = put(ph.item, &item)) != KS_OK ||
      (st = dalloc(s, &partial, pbytes)) != KS_OK ||
      (fresh.push_back(partial), st = dalloc(s, reinterpret_cast<void**>(&DP), dbytes)) != KS_OK) {
    for (void*& q : fresh) dfree(s, q);
    return st;
  }
  auto swap_in = [&](auto*& field, auto* v) {
    void* old = field;
    dfree(s, old);
    field = v;
  };
  swap_in(s->d_pt_lds, pt_lds);
  swap_in(s->d_slot_off, slot_off);
  swap_in(s->d_slot_atom, slot_atom);
  swap_in(s->d_slot_pt, slot_pt);
  swap_in(s->d_atom_slot_off, atom_slot_off);
  swap_in(s->d_atom_slots, atom_slots);
  swap_in(s->d_up_off, up_off);
  swap_in(s->d_up_key, up_key2);
  swap_in(s->d_up_x, up_x2);
  swap_in(s->d_x_slot, x_slot2);
  swap_in(s->d_beta, brows);
  swap_in(s->d_up_beta, up_beta2);
  swap_in(s->d_x_beta, x_beta2);
  swap_in(s->d_kb, kb2);
  swap_in(s->d_item, item);
  swap_in(s->partial, partial);
  swap_in(s->DP, DP);
  s->partial_cap = pbytes;
  s->dp_cap = dbytes;
  s->natoms = na;
  s->nproj = np;
  s->nslots = (int)ph.slot_atom.size();
  s->nruns = ph.nruns;
  s->npoints = ph.npoints;
  s->nuniq = (int)ph.up_lds.size();
  return KS_OK;
}

// The reciprocal-space projection table of the projector inputs (natoms
// atoms of np projectors; npts, idx, beta, d as ks_system_set_projectors
// takes them) in fresh device buffers; the caller swaps them in (or frees
// them).  Synchronous; the caller has waited for the system's work.
static ks_status build_gtab(ks_system* s, int natoms, int np, const int* npts, const int* idx, const double* beta,
                            const double* d, GTab& out) {
  out = GTab{};
  const int P = natoms * np;
  if (P == 0) return KS_OK;   // nothing to project
  std::vector<int> off((size_t)natoms + 1, 0);
  for (int I = 0; I < natoms; ++I) off[I + 1] = off[I] + npts[I];
  const size_t npoints = (size_t)off[natoms];
  GTab g;
  g.P = P;
  g.ncol = 2 * ((P + 63) / 64 * 64);
  g.kpad = (2 * s->npw + 31) / 32 * 32;
  g.part_bytes = gproj_part_bytes(s->cb, g.ncol, g.kpad / 32);
  const size_t wbytes = (size_t)g.ncol * 2 * g.kpad * sizeof(__bf16);
  void *w = nullptr, *part = nullptr, *t_off = nullptr, *t_idx = nullptr, *t_beta = nullptr, *t_d = nullptr;
  auto release = [&](bool keep) {
    dfree(s, t_off);
    dfree(s, t_idx);
    dfree(s, t_beta);
    dfree(s, t_d);
    if (!keep) {
      dfree(s, w);
      dfree(s, part);
    }
  };
  ks_status st;
  if ((st = dalloc(s, &w, wbytes)) != KS_OK || (st = dalloc(s, &part, g.part_bytes)) != KS_OK ||
      (st = dalloc(s, &t_off, off.size() * sizeof(int))) != KS_OK ||
      (st = dalloc(s, &t_idx, npoints * sizeof(int))) != KS_OK ||
      (st = dalloc(s, &t_beta, npoints * np * sizeof(double))) != KS_OK ||
      (st = dalloc(s, &t_d, (size_t)P * sizeof(double))) != KS_OK) {
    release(false);
    return st;
  }
  hipError_t e = hipMemcpy(t_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess && npoints) e = hipMemcpy(t_idx, idx, npoints * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess && npoints) e = hipMemcpy(t_beta, beta, npoints * np * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(t_d, d, (size_t)P * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(w, 0, wbytes, nullptr);
  if (e == hipSuccess && !launch_gproj_table(s, static_cast<const int*>(t_off), static_cast<const int*>(t_idx),
                                             static_cast<const double*>(t_beta), static_cast<const double*>(t_d),
                                             natoms, np, static_cast<__bf16*>(w), g.kpad, nullptr)) {
    release(false);
    return fail(s, KS_EUNSUPPORTED, "no reciprocal-space projection table for this grid or projector count");
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    release(false);
    return fail(s, KS_EDEVICE, std::string("projection table: ") + hipGetErrorString(e));
  }
  release(true);
  g.w = static_cast<__bf16*>(w);
  g.part = static_cast<float*>(part);
  out = g;
  return KS_OK;
}

ks_status ks_system_set_projectors(ks_system* s, int natoms, int nproj, const int* npts, const int* idx,
                                   const double* beta, const double* d, void* stream) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (natoms > 0 && !d) return fail(s, KS_EINVAL, "d is null");
  ProjHost ph;
  {
    std::string msg;
    const ks_status r = build_proj(s->n, s->xnb, s->xnt, natoms, nproj, npts, idx, beta, ph, msg);
    if (r != KS_OK) return fail(s, r, msg);
  }
  KS_HIP(s, hipStreamSynchronize((hipStream_t)stream));
  wait_own(s);   // the old tables may still be read by work on another stream
  ++s->gen;
  const int na = std::max(0, natoms), np = ph.nproj;
  std::vector<double> dcopy(d, d + (size_t)na * np);
  GTab fresh;
  if (s->proj_mode == 1 && ph.npoints > 0) {
    const ks_status r = build_gtab(s, na, np, npts, idx, beta, dcopy.data(), fresh);
    if (r != KS_OK) return r;
  }
  const ks_status r = install_proj(s, ph, na, dcopy.data());
  if (r != KS_OK) {
    free_gtab(s, fresh);
    return r;   // the previous tables (and inputs) stay
  }
  free_gtab(s, s->gp);
  s->gp = fresh;
  // keep the inputs: another tile shape rebuilds the tables from them
  auto& in = s->proj_in;
  in.natoms = na;
  in.nproj = nproj;
  in.npts.assign(npts, npts + na);
  in.idx.assign(idx, idx + ph.npoints);
  in.beta.assign(beta, beta + (size_t)ph.npoints * np);
  in.d = std::move(dcopy);
  return KS_OK;
}

// Switch the x-pencil passes to tile shape `shape`: the per-tile projector
// tables are rebuilt for the new tiles from the stored inputs.
static ks_status set_x_shape(ks_system* s, int shape) {
  if (shape == s->xshape) return KS_OK;
  if (!x_shape_available(s->n[0], shape)) return fail(s, KS_EINVAL, "x-tile shape not available for this grid");
  const int nb = x_shape_nb(s->n[0], shape), nt = x_shape_threads(shape);
  const auto& in = s->proj_in;
  ProjHost ph;
  {
    std::string msg;
    const ks_status r = build_proj(s->n, nb, nt, in.natoms, in.nproj, in.npts.data(), in.idx.data(),
                                   in.beta.data(), ph, msg);
    if (r != KS_OK) return fail(s, r, msg);
  }
  wait_own(s);
  ++s->gen;
  const ks_status r = install_proj(s, ph, in.natoms, in.d.data());
  if (r != KS_OK) return r;   // tables, shape and workspace unchanged
  s->xshape = shape;
  s->xnb = nb;
  s->xnt = nt;
  s->ntiles = (s->npl + nb - 1) / nb;
  return KS_OK;
}

// Form the KB projections in real space (mode 0) or as the reciprocal-space
// split-BF16 product (mode 1, mixed precision; the table is built from the
// stored projector inputs).  A failure leaves the mode and table as they were.
static ks_status set_projection(ks_system* s, int mode) {
  if (mode == s->proj_mode) return KS_OK;
  if (mode != 0 && mode != 1) return fail(s, KS_EINVAL, "projection must be 0 or 1");
  if (mode == 1 && s->prec != KS_MIXED)
    return fail(s, KS_EINVAL, "the split-BF16 projection (1) is for mixed-precision systems only");
  wait_own(s);
  ++s->gen;
  GTab fresh;
  if (mode == 1 && s->natoms > 0) {
    const auto& in = s->proj_in;
    const ks_status r = build_gtab(s, in.natoms, in.nproj, in.npts.data(), in.idx.data(), in.beta.data(),
                                   in.d.data(), fresh);
    if (r != KS_OK) return r;
  }
  free_gtab(s, s->gp);
  s->gp = fresh;
  s->proj_mode = mode;
  return KS_OK;
}

ks_status ks_ham_apply(ks_system* s, int norb, const void* psi, void* hpsi, void* stream) {
  ks_status r = check_common(s, norb);
  if (r != KS_OK) return r;
  if (norb == 0) return KS_OK;
  if (!psi || !hpsi) return fail(s, KS_EINVAL, "psi or hpsi is null");
  const size_t bytes = (size_t)norb * s->N * sizeof(double2);
  const char* a = (const char*)psi;
  const char* b = (const char*)hpsi;
  if (a < b + bytes && b < a + bytes) return fail(s, KS_EINVAL, "psi and hpsi overlap");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  Taylor none{{0.0, 0.0}, 0, {0.0, 0.0}};
  const int cl = chunk_len(s, norb);
  for (int o0 = 0; o0 < norb; o0 += cl) {
    const int nb = std::min(cl, norb - o0);
    const double2* in = (const double2*)psi + (size_t)o0 * s->N;
    double2* out = (double2*)hpsi + (size_t)o0 * s->N;
    if ((r = kcall(s, KS_K_PACK, st, "pack", [&] { return launch_pack(s, nb, in, s->N, s->pk[0], st); })) != KS_OK) return r;
    if ((r = hpsi_packed(s, nb, s->pk[0], true, s->pk[1], nullptr, H_OUT, none, st)) != KS_OK) return r;
    const bool fp64 = s->prec == KS_FP64;
    if ((r = kcall(s, KS_K_UNPACK, st, "unpack", [&] { return launch_unpack(s, nb, s->pk[1], fp64, out, s->N, st); })) != KS_OK) return r;
  }
  return KS_OK;
}

ks_status ks_propagate_step(ks_system* s, int norb, void* psi, double dt, int nsteps, const double* occ,
                            double* rho, void* stream) {
  ks_status r = check_common(s, norb);
  if (r != KS_OK) return r;
  if (nsteps < 0) return fail(s, KS_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt)) return fail(s, KS_EINVAL, "dt must be finite");
  if (norb == 0 || nsteps == 0) return KS_OK;
  if (!psi) return fail(s, KS_EINVAL, "psi is null");
  if (rho && !occ) return fail(s, KS_EINVAL, "rho requires occ");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  const int cl = chunk_len(s, norb);
  for (int o0 = 0; o0 < norb; o0 += cl) {
    const int nb = std::min(cl, norb - o0);
    double2* box = (double2*)psi + (size_t)o0 * s->N;
    if ((r = kcall(s, KS_K_PACK, st, "pack", [&] { return launch_pack(s, nb, box, s->N, s->pk[0], st); })) != KS_OK) return r;
    if ((r = taylor_packed(s, nb, (double2*)s->pk[0], dt, nsteps, occ ? occ + o0 : nullptr, rho, o0 > 0, nullptr, 0,
                           st)) != KS_OK)
      return r;
    if ((r = kcall(s, KS_K_UNPACK, st, "unpack", [&] { return launch_unpack(s, nb, s->pk[0], true, box, s->N, st); })) != KS_OK) return r;
  }
  return KS_OK;
}

ks_status ks_density(ks_system* s, int norb, const void* psi, const double* occ, double* rho, void* stream) {
  ks_status r = check_common(s, norb);
  if (r != KS_OK) return r;
  if (!rho) return fail(s, KS_EINVAL, "rho is null");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  if (norb == 0) {
    KS_HIP(s, hipMemsetAsync(rho, 0, s->N * sizeof(double), st));
    return KS_OK;
  }
  if (!psi || !occ) return fail(s, KS_EINVAL, "psi or occ is null");
  const int cl = chunk_len(s, norb);
  for (int o0 = 0; o0 < norb; o0 += cl) {
    const int nb = std::min(cl, norb - o0);
    const double2* box = (const double2*)psi + (size_t)o0 * s->N;
    if ((r = kcall(s, KS_K_PACK, st, "pack", [&] { return launch_pack(s, nb, box, s->N, s->pk[0], st); })) != KS_OK) return r;
    if ((r = density_packed(s, nb, s->pk[0], occ + o0, rho, o0 > 0, st)) != KS_OK) return r;
  }
  return KS_OK;
}

ks_status ks_system_set_xc(ks_system* s, int functional) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (functional != KS_XC_NONE && functional != KS_XC_LDA) return fail(s, KS_EINVAL, "unknown exchange-correlation functional");
  s->xc = functional;
  return KS_OK;
}

ks_status ks_lda_xc(ks_system* s, const double* rho, double* v, int accumulate, void* stream) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!rho || !v) return fail(s, KS_EINVAL, "rho or v is null");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  launch_lda_xc(s, rho, v, accumulate, st);
  return launch_ok(s, true, "lda_xc");
}

ks_status ks_hartree(ks_system* s, const double* rho, double* v, int add_vloc, void* stream) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!rho || !v) return fail(s, KS_EINVAL, "rho or v is null");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  if (!launch_hartree(s, rho, v, add_vloc ? s->d_vloc : nullptr, st))
    return fail(s, KS_EUNSUPPORTED, "no Hartree kernel for this grid");
  return launch_ok(s, true, "hartree");
}

ks_status ks_dipole(ks_system* s, const double* rho, double* d, void* stream) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!rho || !d) return fail(s, KS_EINVAL, "rho or d is null");
  Track tk(s, stream);
  return launch_ok(s, launch_dipole(s, rho, d, (hipStream_t)stream), "dipole");
}

ks_status ks_dipole_noalloc(const int n[3], const double L[3], const double* rho, double* d, void* stream) {
  if (!n || !L || !rho || !d) return fail(nullptr, KS_EINVAL, "null argument");
  long long N = 1;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return fail(nullptr, KS_EINVAL, "grid size must be positive");
    if (!(L[a] > 0.0) || !std::isfinite(L[a])) return fail(nullptr, KS_EINVAL, "cell lengths must be positive");
    N *= n[a];
  }
  if (N > KS_DIPOLE_NOALLOC_MAX_POINTS)
    return fail(nullptr, KS_EINVAL,
                "grid of " + std::to_string(N) + " points exceeds the allocation-free dipole's limit of " +
                    std::to_string(KS_DIPOLE_NOALLOC_MAX_POINTS));
  double* part = nullptr;
  const hipError_t e = dipole_scratch(&part);
  if (e != hipSuccess) return fail(nullptr, KS_EDEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
  const hipStream_t st = (hipStream_t)stream;
  launch_dipole_grid(n, L, rho, part, d, st);
  const hipError_t e2 = hipGetLastError();
  if (e2 != hipSuccess) return fail(nullptr, KS_EDEVICE, std::string("dipole: ") + hipGetErrorString(e2));
  return KS_OK;
}

ks_status ks_spectrum(const double* dipoles, int nt, double dt, const double k[3], const double* omegas, int nw,
                      double damping, double* alpha, double* strength, void* stream) {
  if (!dipoles || !k || (nw > 0 && (!omegas || !alpha || !strength))) return fail(nullptr, KS_EINVAL, "null argument");
  if (nt < 1 || nw < 0) return fail(nullptr, KS_EINVAL, "nt must be >= 1 and nw >= 0");
  if (!std::isfinite(dt) || !(dt > 0.0) || !std::isfinite(damping))
    return fail(nullptr, KS_EINVAL, "dt must be positive and damping finite");
  if (!std::isfinite(k[0]) || !std::isfinite(k[1]) || !std::isfinite(k[2]) ||
      k[0] * k[0] + k[1] * k[1] + k[2] * k[2] == 0.0)
    return fail(nullptr, KS_EINVAL, "the kick must be finite and non-zero");
  launch_spectrum(dipoles, nt, dt, k, omegas, nw, damping, reinterpret_cast<double2*>(alpha), strength,
                  (hipStream_t)stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, KS_EDEVICE, std::string("spectrum: ") + hipGetErrorString(e));
  return KS_OK;
}

ks_status ks_reduce(ks_system* s, int norb, const void* psi, const double* occ, double* norms, double* energy,
                    void* stream) {
  ks_status r = check_common(s, norb);
  if (r != KS_OK) return r;
  if (energy && !occ) return fail(s, KS_EINVAL, "energy requires occ");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  if (norb == 0) {
    if (energy) KS_HIP(s, hipMemsetAsync(energy, 0, sizeof(double), st));
    return KS_OK;
  }
  if (!psi) return fail(s, KS_EINVAL, "psi is null");
  Taylor none{{0.0, 0.0}, 0, {0.0, 0.0}};
  const int cl = chunk_len(s, norb);
  for (int o0 = 0; o0 < norb; o0 += cl) {
    const int nb = std::min(cl, norb - o0);
    const double2* box = (const double2*)psi + (size_t)o0 * s->N;
    if ((r = kcall(s, KS_K_PACK, st, "pack", [&] { return launch_pack(s, nb, box, s->N, s->pk[0], st); })) != KS_OK) return r;
    if (energy && (r = hpsi_packed(s, nb, s->pk[0], true, s->pk[1], nullptr, H_OUT, none, st)) != KS_OK) return r;
    const void* hp = energy ? s->pk[1] : nullptr;
    double* red = s->red + 2 * (size_t)o0;
    if ((r = kcall(s, KS_K_DOTS, st, "dots", [&] { return launch_dots(s, nb, s->pk[0], hp, red, st); })) != KS_OK)
      return r;
  }
  if (norms)
    KS_HIP(s, hipMemcpy2DAsync(norms, sizeof(double), s->red, 2 * sizeof(double), sizeof(double), norb,
                               hipMemcpyDeviceToDevice, st));
  if (energy) return kcall(s, KS_K_DOTS, st, "energy_sum", [&] { return launch_energy_sum(norb, occ, s->red, energy, st); });
  return KS_OK;
}

ks_status ks_orthonormalize(ks_system* s, int norb, void* psi, void* stream) {
  ks_status r = check_common(s, norb);
  if (r != KS_OK) return r;
  if (norb == 0) return KS_OK;
  if (!psi) return fail(s, KS_EINVAL, "psi is null");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  if ((r = ensure_ortho_mats(s)) != KS_OK) return r;
  if (!s->ortho_pk &&
      (r = dalloc(s, &s->ortho_pk, 2 * (size_t)s->max_norb * s->npw_stride * sizeof(double2))) != KS_OK)
    return r;
  double2* P = (double2*)s->ortho_pk;
  double2* Y = P + (size_t)s->max_norb * s->npw_stride;
  KS_HIP(s, hipMemsetAsync(s->ortho_info, 0, sizeof(int), st));
  double2* box = (double2*)psi;
  if ((r = kcall(s, KS_K_PACK, st, "pack", [&] { return launch_pack(s, norb, box, s->N, P, st); })) != KS_OK) return r;
  if ((r = kcall(s, KS_K_GEMM, st, "overlap",
                 [&] { return launch_overlap(norb, s->npw, P, s->npw_stride, s->ortho_S, s->gemm_part, s->gemm_part_bytes, st); })) != KS_OK)
    return r;
  if ((r = launch_ok(s, launch_cholesky(norb, s->ortho_S, s->ortho_W, s->ortho_diag, s->ortho_info, st), "cholesky")) != KS_OK) return r;
  if ((r = launch_ok(s, launch_trtri(norb, s->ortho_S, s->ortho_W, st), "trtri")) != KS_OK) return r;
  if ((r = kcall(s, KS_K_GEMM, st, "apply",
                 [&] { return launch_apply_lower(norb, s->npw, s->ortho_W, P, s->npw_stride, Y, st); })) != KS_OK)
    return r;
  int info = 0;
  KS_HIP(s, hipMemcpyAsync(&info, s->ortho_info, sizeof(int), hipMemcpyDeviceToHost, st));
  KS_HIP(s, hipStreamSynchronize(st));
  if (info) return fail(s, KS_EINVAL, "overlap matrix is not positive definite (orbitals linearly dependent)");
  return kcall(s, KS_K_UNPACK, st, "unpack", [&] { return launch_unpack(s, norb, Y, true, box, s->N, st); });
}

ks_status ks_plan_sphere(const int n[3], const double L[3], double ecut, int* npw, int* m_out) {
  if (!n || !L || !npw) return fail(nullptr, KS_EINVAL, "null argument");
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1 || !(L[a] > 0.0)) return fail(nullptr, KS_EINVAL, "bad grid or cell");
  SphereHost h;
  std::string msg;
  const ks_status r = build_sphere(n, L, ecut, h, msg);
  if (r != KS_OK) return fail(nullptr, r, msg);
  *npw = h.npw;
  if (m_out) {
    const int nplanes = (int)h.plane_m1lo.size();
    for (int pi = 0; pi < nplanes; ++pi) {
      for (int c = h.plane_col0[pi]; c < h.plane_col0[pi + 1]; ++c) {
        const int m1 = h.plane_m1lo[pi] + (c - h.plane_col0[pi]);
        for (int e = h.col_off[c]; e < h.col_off[c + 1]; ++e) {
          m_out[3 * e] = h.m0lo + pi;
          m_out[3 * e + 1] = m1;
          m_out[3 * e + 2] = h.col_m2lo[c] + (e - h.col_off[c]);
        }
      }
    }
  }
  return KS_OK;
}

ks_status ks_plan_projectors(const int n[3], int natoms, int nproj, const int* npts, const int* idx,
                             const double* beta, int* counts, int* point_flat, int* point_entries,
                             int* entry_atom, int* entry_row) {
  if (!n || !counts) return fail(nullptr, KS_EINVAL, "null argument");
  ProjHost h;
  std::string msg;
  const int xnb = x_tile_nb(n[0]);
  const ks_status r = build_proj(n, xnb, x_shape_threads(0), natoms, nproj, npts, idx, beta, h, msg);
  if (r != KS_OK) return fail(nullptr, r, msg);
  const int nuniq = (int)h.up_lds.size(), nent = (int)h.ent_slot.size();
  counts[0] = (int)h.slot_atom.size();
  counts[1] = nuniq;
  counts[2] = nent;
  counts[3] = h.nruns;
  const int W = n[0] + 1, npl = n[1] * n[2];
  for (int t = 0; t < h.ntiles; ++t) {
    for (int u = h.up_off[t]; u < h.up_off[t + 1]; ++u) {
      if (point_flat) {
        const int w = h.up_lds[u] / W, j0 = h.up_lds[u] % W;
        point_flat[u] = j0 * npl + t * xnb + w;
      }
      if (point_entries) point_entries[u] = h.up_ent[u];
      for (int e = h.up_ent[u]; e < h.up_ent[u + 1]; ++e) {
        const int slot = h.slot_off[t] + h.ent_slot[e];
        if (entry_atom) entry_atom[e] = h.slot_atom[slot];
        if (entry_row) entry_row[e] = h.brow_input[h.ent_brow[e]];
        // projection side consistency: the entry's beta row lies in its slot
        if (h.ent_brow[e] < h.slot_pt[slot] || h.ent_brow[e] >= h.slot_pt[slot + 1])
          return fail(nullptr, KS_EDEVICE, "inconsistent projector tables");
      }
    }
  }
  if (point_entries) point_entries[nuniq] = nent;
  return KS_OK;
}

// ------------------------------------------------------------ resident state

ks_status ks_state_create(ks_system* s, int norb, ks_state** out) {
  if (!out) return fail(s, KS_EINVAL, "out is null");
  *out = nullptr;
  ks_status r = check_common(s, norb);
  if (r != KS_OK) return r;
  if (norb < 1) return fail(s, KS_EINVAL, "norb must be >= 1");
  ks_state* t = new ks_state();
  t->sys = s;
  t->norb = norb;
  if ((r = dalloc(s, reinterpret_cast<void**>(&t->data), (size_t)norb * s->npw_stride * sizeof(double2))) != KS_OK) {
    delete t;
    return r;
  }
  s->states.push_back(t);
  *out = t;
  return KS_OK;
}

static void state_drop_graph(ks_state* t) {
  if (t->exec) (void)hipGraphExecDestroy(t->exec);
  if (t->graph) (void)hipGraphDestroy(t->graph);
  t->exec = nullptr;
  t->graph = nullptr;
}

// Free a state's device memory and graph and detach it from its system
// (after its system's enqueued work); the handle stays valid but empty.
static void state_release(ks_state* t) {
  ks_system* s = t->sys;
  if (!s) return;
  wait_own(s);
  // batches holding this state hold freed buffers from now on
  for (size_t i = s->batches.size(); i-- > 0;) {
    ks_batch* b = s->batches[i];
    if (std::find(b->states.begin(), b->states.end(), t) != b->states.end()) batch_release(b);
  }
  state_drop_graph(t);
  void* p = t->data;
  dfree(s, p);
  void* bufs[] = {t->aux, t->gs_buf[0], t->gs_buf[1], t->gs_mat, t->gs_vec};
  for (void* q : bufs) dfree(s, q);
  t->data = t->aux = t->gs_buf[0] = t->gs_buf[1] = t->gs_mat = nullptr;
  t->gs_vec = nullptr;
  s->states.erase(std::remove(s->states.begin(), s->states.end(), t), s->states.end());
  t->sys = nullptr;
}

void ks_state_destroy(ks_state* t) {
  if (!t) return;
  state_release(t);
  delete t;
}

ks_status ks_state_upload(ks_state* t, const void* psi, void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!psi) return fail(s, KS_EINVAL, "psi is null");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  const double2* box = (const double2*)psi;
  return kcall(s, KS_K_PACK, st, "pack", [&] { return launch_pack(s, t->norb, box, s->N, t->data, st); });
}

ks_status ks_state_download(ks_state* t, void* psi, void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!psi) return fail(s, KS_EINVAL, "psi is null");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  double2* box = (double2*)psi;
  return kcall(s, KS_K_UNPACK, st, "unpack", [&] { return launch_unpack(s, t->norb, t->data, true, box, s->N, st); });
}

ks_status ks_state_propagate(ks_state* t, double dt, int nsteps, const double* occ, double* rho, double* norms,
                             void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (nsteps < 0) return fail(s, KS_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt)) return fail(s, KS_EINVAL, "dt must be finite");
  if (rho && !occ) return fail(s, KS_EINVAL, "rho requires occ");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  ks_status r;
  const int cl = chunk_len(s, t->norb);
  for (int o0 = 0; o0 < t->norb; o0 += cl) {
    const int nb = std::min(cl, t->norb - o0);
    double2* slice = t->data + (size_t)o0 * s->npw_stride;
    if ((r = taylor_packed(s, nb, slice, dt, nsteps, occ ? occ + o0 : nullptr, rho, o0 > 0,
                           norms ? norms + o0 : nullptr, t->norb, st)) != KS_OK)
      return r;
  }
  return KS_OK;
}

ks_status ks_state_propagate_etrs(ks_state* t, double dt, int nsteps, const double* occ, double* rho, double* norms,
                                  void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (nsteps < 0) return fail(s, KS_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt)) return fail(s, KS_EINVAL, "dt must be finite");
  if (!occ) return fail(s, KS_EINVAL, "occ is required (the Hamiltonian depends on the density)");
  if (nsteps == 0) return KS_OK;
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  if (!t->aux) {
    ks_status r = dalloc(s, reinterpret_cast<void**>(&t->aux), (size_t)t->norb * s->npw_stride * sizeof(double2));
    if (r != KS_OK) return r;
  }
  const ks_status r = etrs_packed(s, t, dt, nsteps, occ, rho, norms, st);
  // the system's Hamiltonian is the static one again between calls
  const hipError_t e =
      hipMemcpyAsync(s->d_v, s->d_vloc, s->N * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (r != KS_OK) return r;
  if (e != hipSuccess) return fail(s, KS_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
  return KS_OK;
}

ks_status ks_state_kick(ks_state* t, const double k[3], void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!k || !std::isfinite(k[0]) || !std::isfinite(k[1]) || !std::isfinite(k[2]))
    return fail(s, KS_EINVAL, "k must be three finite numbers");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  ks_status r;
  for (int o = 0; o < t->norb; ++o) {
    double2* c = t->data + (size_t)o * s->npw_stride;
    if ((r = launch_ok(s, launch_unpack(s, 1, c, true, s->d_hbox, s->N, st), "unpack")) != KS_OK) return r;
    if ((r = launch_ok(s, launch_kick(s, s->d_hbox, k, st), "kick")) != KS_OK) return r;
    if ((r = launch_ok(s, launch_pack(s, 1, s->d_hbox, s->N, c, st), "pack")) != KS_OK) return r;
  }
  return KS_OK;
}

ks_status ks_state_eigensolve(ks_state* t, int niter, double* eig, double* resid, void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (niter < 0) return fail(s, KS_EINVAL, "niter < 0");
  if (s->prec != KS_FP64) return fail(s, KS_EUNSUPPORTED, "the eigensolver runs on FP64 systems");
  if (niter == 0) return KS_OK;
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  const int n = t->norb;
  const size_t ld = s->npw_stride, nn = (size_t)n * n, blk = (size_t)n * ld * sizeof(double2);
  ks_status r;
  if ((!t->aux && (r = dalloc(s, reinterpret_cast<void**>(&t->aux), blk)) != KS_OK) ||
      (!t->gs_buf[0] && (r = dalloc(s, reinterpret_cast<void**>(&t->gs_buf[0]), blk)) != KS_OK) ||
      (!t->gs_buf[1] && (r = dalloc(s, reinterpret_cast<void**>(&t->gs_buf[1]), blk)) != KS_OK) ||
      (!t->gs_mat &&
       (r = dalloc(s, reinterpret_cast<void**>(&t->gs_mat), (2 * nn + bj_work_elems(n)) * sizeof(double2))) != KS_OK) ||
      (!t->gs_vec && (r = dalloc(s, reinterpret_cast<void**>(&t->gs_vec),
                                 (2 * (size_t)n + 2 + 2 * (size_t)bj_order(n)) * sizeof(double))) != KS_OK) ||
      (r = ensure_ortho_mats(s)) != KS_OK)
    return r;
  double2 *C = t->data, *B1 = t->aux, *B2 = t->gs_buf[0], *B3 = t->gs_buf[1];
  double2 *Hs = t->gs_mat, *Qm = t->gs_mat + nn, *work = t->gs_mat + 2 * nn;
  double *e = t->gs_vec, *rn = t->gs_vec + n, *off = t->gs_vec + 2 * n;
  const int cl = chunk_len(s, n);
  const Taylor none{{0.0, 0.0}, 0, {0.0, 0.0}};
  const size_t row = ld * sizeof(double2), used = s->npw * sizeof(double2);
  for (int it = 0; it < niter; ++it) {
    // W = H C
    for (int o0 = 0; o0 < n; o0 += cl)
      if ((r = hpsi_packed(s, std::min(cl, n - o0), C + o0 * ld, true, B1 + o0 * ld, nullptr, H_OUT, none, st)) != KS_OK)
        return r;
    // subspace diagonalisation: Hs = C^H W = Q diag(e) Q^H; C <- Q^T C, W <- Q^T W
    if ((r = kcall(s, KS_K_GEMM, st, "rayleigh_ritz", [&] { return launch_gemm_ch(n, s->npw, C, ld, B1, ld, Hs, s->gemm_part, s->gemm_part_bytes, st); })) !=
        KS_OK)
      return r;
    if ((r = subspace_eigh(s, n, Hs, work, off, e, Qm, st)) != KS_OK) return r;
    if ((r = kcall(s, KS_K_GEMM, st, "rotate", [&] { return launch_rotate(n, s->npw, Qm, C, ld, B3, ld, st); })) != KS_OK ||
        (r = kcall(s, KS_K_GEMM, st, "rotate", [&] { return launch_rotate(n, s->npw, Qm, B1, ld, B2, ld, st); })) != KS_OK)
      return r;
    KS_HIP(s, hipMemcpy2DAsync(C, row, B3, row, used, n, hipMemcpyDeviceToDevice, st));
    // preconditioned directions q (B1) from the residuals of C, W (B2)
    if ((r = kcall(s, KS_K_SD, st, "sd_direction", [&] {
           launch_sd_direction(n, s->npw, (int)ld, C, B2, e, s->d_kin, B1, rn, st);
           return true;
         })) != KS_OK)
      return r;
    // H q (B3), line minimisation, orthonormalisation
    for (int o0 = 0; o0 < n; o0 += cl)
      if ((r = hpsi_packed(s, std::min(cl, n - o0), B1 + o0 * ld, true, B3 + o0 * ld, nullptr, H_OUT, none, st)) != KS_OK)
        return r;
    if ((r = kcall(s, KS_K_SD, st, "sd_update", [&] {
           launch_sd_update(n, s->npw, (int)ld, C, B1, B3, e, st);
           return true;
         })) != KS_OK)
      return r;
    if ((r = orthonormalize_packed(s, n, C, B2, st)) != KS_OK) return r;
    if (eig) KS_HIP(s, hipMemcpyAsync(eig + (size_t)it * n, e, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (resid) KS_HIP(s, hipMemcpyAsync(resid + (size_t)it * n, rn, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  return KS_OK;
}

ks_status ks_state_reduce(ks_state* t, const double* occ, double* norms, double* energy, void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (energy && !occ) return fail(s, KS_EINVAL, "energy requires occ");
  hipStream_t st = (hipStream_t)stream;
  Track tk(s, st);
  Taylor none{{0.0, 0.0}, 0, {0.0, 0.0}};
  ks_status r;
  // norms only: one launch over every resident orbital
  const int step = energy ? chunk_len(s, t->norb) : t->norb;
  for (int o0 = 0; o0 < t->norb; o0 += step) {
    const int nb = std::min(step, t->norb - o0);
    const double2* slice = t->data + (size_t)o0 * s->npw_stride;
    if (energy && (r = hpsi_packed(s, nb, slice, true, s->pk[1], nullptr, H_OUT, none, st)) != KS_OK) return r;
    const void* hp = energy ? s->pk[1] : nullptr;
    double* red = s->red + 2 * (size_t)o0;
    if ((r = kcall(s, KS_K_DOTS, st, "dots", [&] { return launch_dots(s, nb, slice, hp, red, st); })) != KS_OK)
      return r;
  }
  if (norms)
    KS_HIP(s, hipMemcpy2DAsync(norms, sizeof(double), s->red, 2 * sizeof(double), sizeof(double), t->norb,
                               hipMemcpyDeviceToDevice, st));
  if (energy)
    return kcall(s, KS_K_DOTS, st, "energy_sum", [&] { return launch_energy_sum(t->norb, occ, s->red, energy, st); });
  return KS_OK;
}

ks_status ks_state_capture(ks_state* t, double dt, const double* occ, double* rho, void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!stream) return fail(s, KS_EINVAL, "capture needs a non-default stream");
  if (s->timing) return fail(s, KS_EINVAL, "kernel timing must be off while capturing");
  if (rho && !occ) return fail(s, KS_EINVAL, "rho requires occ");
  hipStream_t st = (hipStream_t)stream;
  state_drop_graph(t);
  KS_HIP(s, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const ks_status r = ks_state_propagate(t, dt, 1, occ, rho, nullptr, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (r != KS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return fail(s, KS_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  t->graph = g;
  const hipError_t e2 = hipGraphInstantiate(&t->exec, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    state_drop_graph(t);
    return fail(s, KS_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
  }
  t->graph_gen = s->gen;
  return KS_OK;
}

ks_status ks_state_replay(ks_state* t, void* stream) {
  if (!t) return fail(nullptr, KS_EINVAL, "null state");
  ks_system* s = t->sys;
  if (!s) return fail(nullptr, KS_EINVAL, "the state's system was destroyed");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (!t->exec) return fail(s, KS_EINVAL, "no captured step");
  if (t->graph_gen != s->gen)
    return fail(s, KS_EINVAL, "the system's buffers or launch shapes changed since the capture; capture again");
  Track tk(s, stream);
  KS_HIP(s, hipGraphLaunch(t->exec, (hipStream_t)stream));
  return KS_OK;
}

// ------------------------------------------------------------ batched steps

static void batch_drop_graph(ks_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

static bool same_grid(const ks_system* a, const ks_system* b) {
  for (int i = 0; i < 3; ++i)
    if (a->n[i] != b->n[i] || a->L[i] != b->L[i]) return false;
  return a->ecut == b->ecut && a->prec == b->prec;
}

static ks_status batch_check(ks_batch* b) {
  for (size_t j = 0; j < b->states.size(); ++j)
    if (b->states[j]->sys->pool_lost) return fail(b->s0, KS_EINVAL, "a system's pool was destroyed");
  for (size_t j = 0; j < b->states.size(); ++j)
    if (b->states[j]->sys->gen != b->gens[j])
      return fail(b->s0, KS_EINVAL, "a system of the batch changed its buffers or launch shapes; create the batch again");
  return KS_OK;
}

ks_status ks_batch_create(ks_state* const* states, int nstates, ks_batch** out) {
  if (!out) return fail(nullptr, KS_EINVAL, "out is null");
  *out = nullptr;
  if (!states || nstates < 1) return fail(nullptr, KS_EINVAL, "a batch needs at least one state");
  ks_system* s0 = states[0] ? states[0]->sys : nullptr;
  if (!s0) return fail(nullptr, KS_EINVAL, "null state");
  int npass = 0;
  for (int j = 0; j < nstates; ++j) {
    const ks_state* t = states[j];
    if (!t) return fail(nullptr, KS_EINVAL, "null state");
    if (!same_grid(t->sys, s0))
      return fail(nullptr, KS_EINVAL, "the states' systems differ in grid, cell, cutoff or precision");
    if (t->sys->xshape != s0->xshape)
      return fail(nullptr, KS_EINVAL, "the states' systems differ in x-tile shape (tuning)");
    if (t->sys->proj_mode != 0)
      return fail(nullptr, KS_EINVAL, "batches form the projections in real space (projection 0)");
    for (int i = 0; i < j; ++i)
      if (states[i]->sys == t->sys) return fail(nullptr, KS_EINVAL, "two states of one system (they share its workspace)");
    const int cl = chunk_len(t->sys, t->norb);
    npass = std::max(npass, (t->norb + cl - 1) / cl);
  }
  // Pass p holds chunk p of every state with more than p chunks; each pass's
  // tables: jobs of the 4 Taylor sub-steps, then the x, plane and reduce rows.
  struct Host {
    std::vector<BatchJob> jobs;
    std::vector<int4> rx, rp, rr;
    int njobs = 0, max_natoms = 0;
  };
  std::vector<Host> hp(npass);
  size_t total_bytes = 0;
  for (int p = 0; p < npass; ++p) {
    Host& h = hp[p];
    std::vector<int> js, nbs, o0s;
    long long total = 0;
    for (int j = 0; j < nstates; ++j) {
      const ks_state* t = states[j];
      const int cl = chunk_len(t->sys, t->norb), o0 = p * cl;
      if (o0 >= t->norb) continue;
      js.push_back(j);
      o0s.push_back(o0);
      nbs.push_back(std::min(cl, t->norb - o0));
      total += nbs.back();
      h.max_natoms = std::max(h.max_natoms, t->sys->natoms);
    }
    h.njobs = (int)js.size();
    const int gx = x_group_size(s0, total), gp = plane_group_size(s0, total);
    for (int q = 0; q < h.njobs; ++q) {
      const int nb = nbs[q];
      const int ngx = (nb + gx - 1) / gx, ngp = (nb + gp - 1) / gp;
      for (int g = 0; g < ngx; ++g) h.rx.push_back(make_int4(q, g, ngx, 0));
      for (int g = 0; g < ngp; ++g) h.rp.push_back(make_int4(q, g, ngp, 0));
      if (states[js[q]]->sys->natoms > 0)
        for (int o = 0; o < nb; ++o) h.rr.push_back(make_int4(q, o, 0, 0));
    }
    // jobs of the four Taylor sub-steps: w1 = H c -> pk1, w2 -> pk2, w3 -> pk1, w4 not stored
    h.jobs.resize((size_t)4 * h.njobs);
    for (int k = 0; k < 4; ++k) {
      for (int q = 0; q < h.njobs; ++q) {
        ks_state* t = states[js[q]];
        ks_system* s = t->sys;
        double2* c = t->data + (size_t)o0s[q] * s->npw_stride;
        BatchJob& x = h.jobs[(size_t)k * h.njobs + q];
        const void* src[4] = {c, s->pk[1], s->pk[2], s->pk[1]};
        void* dst[4] = {s->pk[1], s->pk[2], s->pk[1], nullptr};
        x.win = src[k];
        x.wout = dst[k];
        x.acc = c;
        x.T = s->T;
        x.U = s->U;
        x.partial = s->partial;
        x.DP = s->DP;
        x.V = s->d_v;
        x.pt = proj_tab(s);
        x.nb = nbs[q];
      }
    }
    total_bytes += h.jobs.size() * sizeof(BatchJob) +
                   (h.rx.size() + h.rp.size() + std::max<size_t>(h.rr.size(), 1)) * sizeof(int4);
  }
  ks_batch* b = new ks_batch();
  b->s0 = s0;
  for (int j = 0; j < nstates; ++j) {
    b->states.push_back(states[j]);
    b->gens.push_back(states[j]->sys->gen);
  }
  b->dev_bytes = total_bytes;
  void* dev = nullptr;
  ks_status r = dalloc(s0, &dev, b->dev_bytes);
  if (r != KS_OK) {
    delete b;
    return fail(nullptr, r, s0->err);
  }
  b->dev = (char*)dev;
  std::vector<char> host(b->dev_bytes, 0);
  size_t off = 0;
  b->passes.resize(npass);
  for (int p = 0; p < npass; ++p) {
    Host& h = hp[p];
    ks_batch_pass& bp = b->passes[p];
    const size_t jb = h.jobs.size() * sizeof(BatchJob);
    memcpy(host.data() + off, h.jobs.data(), jb);
    for (int k = 0; k < 4; ++k) bp.jobs[k] = reinterpret_cast<BatchJob*>(b->dev + off) + (size_t)k * h.njobs;
    off += jb;
    auto put = [&](const std::vector<int4>& v, int4*& dst, size_t n) {
      if (!v.empty()) memcpy(host.data() + off, v.data(), v.size() * sizeof(int4));
      dst = reinterpret_cast<int4*>(b->dev + off);
      off += n * sizeof(int4);
    };
    put(h.rx, bp.rows_x, h.rx.size());
    put(h.rp, bp.rows_p, h.rp.size());
    put(h.rr, bp.rows_r, std::max<size_t>(h.rr.size(), 1));
    bp.nrows_x = (int)h.rx.size();
    bp.nrows_p = (int)h.rp.size();
    bp.nrows_r = (int)h.rr.size();
    bp.max_natoms = h.max_natoms;
  }
  const hipError_t e = hipMemcpy(b->dev, host.data(), b->dev_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    ks_batch_destroy(b);
    return fail(nullptr, KS_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  for (ks_state* t : b->states) t->sys->batches.push_back(b);
  *out = b;
  return KS_OK;
}

// Free a batch's table and graph and detach it from its systems (after their
// enqueued work); the handle stays valid but empty.
static void batch_release(ks_batch* b) {
  if (!b->s0) return;
  for (ks_state* t : b->states) wait_own(t->sys);
  batch_drop_graph(b);
  void* p = b->dev;
  dfree(b->s0, p);
  b->dev = nullptr;
  for (ks_state* t : b->states) {
    auto& v = t->sys->batches;
    v.erase(std::remove(v.begin(), v.end(), b), v.end());
  }
  b->states.clear();
  b->gens.clear();
  b->s0 = nullptr;
}

void ks_batch_destroy(ks_batch* b) {
  if (!b) return;
  batch_release(b);
  delete b;
}

// f(rows + r0, n) over consecutive slices of at most KS_MAX_GRID_Y rows (each
// batched kernel reads its row as rows[blockIdx.y]).
extern "C++" {
template <class F>
static bool row_slices(const int4* rows, int nrows, F&& f) {
  for (int r0 = 0; r0 < nrows; r0 += KS_MAX_GRID_Y)
    if (!f(rows + r0, std::min(KS_MAX_GRID_Y, nrows - r0))) return false;
  return true;
}
}

// nsteps Taylor-4 steps of every state of the batch, one launch per kernel
// (per slice of rows) and H psi for all of them.
static ks_status batch_taylor(ks_batch* b, double dt, int nsteps, hipStream_t st) {
  ks_system* s0 = b->s0;
  double2 coef[5];
  taylor_coefficients(dt, coef);
  ks_status r;
  // chunk-outer, step-inner, as a state stepped alone
  for (const ks_batch_pass& bp : b->passes) {
    for (int step = 0; step < nsteps; ++step) {
      for (int k = 1; k <= 4; ++k) {
        const BatchJob* jobs = bp.jobs[k - 1];
        const bool in64 = k == 1 || s0->prec == KS_FP64;
        const Taylor tay{coef[k], k < 4 ? 1 : 0, {0.0, 0.0}};
        if ((r = kcall(s0, KS_K_PLANE_INV, st, "plane_inv",
                       [&] {
                         return row_slices(bp.rows_p, bp.nrows_p, [&](const int4* rs, int n) {
                           return launch_plane_inv_batch(s0, jobs, rs, n, in64, st);
                         });
                       })) != KS_OK)
          return r;
        if (bp.max_natoms > 0) {
          if ((r = kcall(s0, KS_K_XPROJ, st, "xproj",
                         [&] {
                           return row_slices(bp.rows_x, bp.nrows_x, [&](const int4* rs, int n) {
                             return launch_x_batch(s0, jobs, rs, n, false, st);
                           });
                         })) != KS_OK)
            return r;
          if ((r = kcall(s0, KS_K_PROJ_REDUCE, st, "proj_reduce", [&] {
                 return row_slices(bp.rows_r, bp.nrows_r, [&](const int4* rs, int n) {
                   return launch_proj_reduce_batch(s0, jobs, rs, n, bp.max_natoms, st);
                 });
               })) != KS_OK)
            return r;
        }
        if ((r = kcall(s0, KS_K_XAPPLY, st, "xapply",
                       [&] {
                         return row_slices(bp.rows_x, bp.nrows_x, [&](const int4* rs, int n) {
                           return launch_x_batch(s0, jobs, rs, n, true, st);
                         });
                       })) != KS_OK)
          return r;
        if ((r = kcall(s0, KS_K_PLANE_FWD, st, "plane_fwd",
                       [&] {
                         return row_slices(bp.rows_p, bp.nrows_p, [&](const int4* rs, int n) {
                           return launch_plane_fwd_batch(s0, jobs, rs, n, in64, tay, st);
                         });
                       })) !=
            KS_OK)
          return r;
      }
    }
  }
  return KS_OK;
}

static void batch_track(ks_batch* b, hipStream_t st) {
  for (ks_state* t : b->states) track(t->sys, st);
}

ks_status ks_batch_propagate(ks_batch* b, double dt, int nsteps, void* stream) {
  if (!b) return fail(nullptr, KS_EINVAL, "null batch");
  if (!b->s0) return fail(nullptr, KS_EINVAL, "a state or system of the batch was destroyed");
  if (nsteps < 0) return fail(b->s0, KS_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt)) return fail(b->s0, KS_EINVAL, "dt must be finite");
  ks_status r = batch_check(b);
  if (r != KS_OK) return r;
  const hipStream_t st = (hipStream_t)stream;
  r = batch_taylor(b, dt, nsteps, st);
  batch_track(b, st);
  return r;
}

ks_status ks_batch_capture(ks_batch* b, double dt, void* stream) {
  if (!b) return fail(nullptr, KS_EINVAL, "null batch");
  if (!b->s0) return fail(nullptr, KS_EINVAL, "a state or system of the batch was destroyed");
  ks_system* s0 = b->s0;
  if (!stream) return fail(s0, KS_EINVAL, "capture needs a non-default stream");
  if (!std::isfinite(dt)) return fail(s0, KS_EINVAL, "dt must be finite");
  if (s0->timing) return fail(s0, KS_EINVAL, "kernel timing must be off while capturing");
  ks_status r = batch_check(b);
  if (r != KS_OK) return r;
  const hipStream_t st = (hipStream_t)stream;
  batch_drop_graph(b);
  KS_HIP(s0, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  r = batch_taylor(b, dt, 1, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (r != KS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return fail(s0, KS_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  b->graph = g;
  const hipError_t e2 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    batch_drop_graph(b);
    return fail(s0, KS_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
  }
  return KS_OK;
}

ks_status ks_batch_replay(ks_batch* b, void* stream) {
  if (!b) return fail(nullptr, KS_EINVAL, "null batch");
  if (!b->s0) return fail(nullptr, KS_EINVAL, "a state or system of the batch was destroyed");
  if (!b->exec) return fail(b->s0, KS_EINVAL, "no captured step");
  ks_status r = batch_check(b);
  if (r != KS_OK) return r;
  const hipStream_t st = (hipStream_t)stream;
  KS_HIP(b->s0, hipGraphLaunch(b->exec, st));
  batch_track(b, st);
  return KS_OK;
}

const char* ks_batch_last_error(const ks_batch* b) {
  return (b && b->s0) ? b->s0->err.c_str() : ks_last_error(nullptr);
}

ks_status ks_propagate_batch(ks_state* const* states, int nstates, double dt, int nsteps, void* stream) {
  ks_batch* b = nullptr;
  ks_status r = ks_batch_create(states, nstates, &b);
  if (r != KS_OK) return r;
  r = ks_batch_propagate(b, dt, nsteps, stream);
  if (r != KS_OK) g_create_err = b->s0->err;
  ks_batch_destroy(b);   // waits for the systems' own work, which includes these steps
  return r;
}

ks_status ks_plan_footprint(const int n[3], const double L[3], double ecut, int precision, int norb, int npoints,
                            int nproj, int chunk, unsigned long long* bytes) {
  if (!n || !L || !bytes || norb < 1 || npoints < 0) return fail(nullptr, KS_EINVAL, "bad argument");
  SphereHost h;
  std::string msg;
  const ks_status r = build_sphere(n, L, ecut, h, msg);
  if (r != KS_OK) return fail(nullptr, r, msg);
  const double es = precision == KS_FP64 ? 16.0 : 8.0;
  const double npl = (double)n[1] * n[2], N = (double)n[0] * npl;
  const double nplanes = (double)h.plane_m1lo.size();
  const double stride = (double)((h.npw + 63) / 64 * 64);
  int cb = chunk;
  if (cb <= 0) cb = std::max(1, std::min(norb, (int)std::floor(KS_CHUNK_BYTES / (nplanes * npl * es))));
  cb = std::min(cb, KS_MAX_GRID_Y);
  const double np = std::max(1, nproj);
  double b = 0.0;
  b += (double)cb * stride * (16.0 + 2.0 * es);         // packed chunk buffers
  b += 2.0 * cb * nplanes * npl * es;                   // plane intermediates
  b += N * 40.0 + 2.0 * norb * 8.0;                     // potential, static potential, density and complex
                                                        // work box of the Hartree solve; reductions
  b += (double)((cb + 7) / 8) * N * 8.0;                // partial densities
  b += npoints * (np * 8.0 + 4 * 4.0) + 64.0 * 1024;    // KB tables
  b += (double)cb * npoints * np * 16.0 / 8.0;          // projection partials (upper bound)
  b += (double)norb * stride * 16.0;                    // resident state
  b += 2.0 * norb * norb * 16.0 + (double)gemm_part_bytes(norb, h.npw);   // orthonormalisation
  *bytes = (unsigned long long)b;
  return KS_OK;
}

ks_status ks_system_info(const ks_system* s, ks_info* info) {
  if (!s || !info) return KS_EINVAL;
  info->npw = s->npw;
  info->nplanes = s->nplanes;
  info->ncols = s->ncols;
  info->chunk = s->cb;
  info->natoms = s->natoms;
  info->nproj = s->nproj;
  info->nruns = s->nruns;
  info->nslots = s->nslots;
  info->npoints = s->npoints;
  info->x_tile = s->xnb;
  info->precision = s->prec;
  info->x_half = s->x_half ? 1 : 0;
  info->x_group = s->xg_max;
  info->plane_group = s->pg_max;
  info->x_shape = s->xshape;
  info->x_threads = s->xnt;
  info->projection = s->proj_mode;
  return KS_OK;
}

// ------------------------------------------------------------------ tuning

ks_status ks_system_set_tuning(ks_system* s, const ks_tuning* t) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (!t || t->x_group < 1 || t->x_group > 64 || t->plane_group < 1 || t->plane_group > 64)
    return fail(s, KS_EINVAL, "group caps must lie in [1, 64]");
  if (s->pool_lost) return fail(s, KS_EINVAL, "the system's pool was destroyed");
  if (t->projection != -1 && t->projection != 0 && t->projection != 1)
    return fail(s, KS_EINVAL, "projection must be -1, 0 or 1");
  if (t->projection == 1 && s->prec != KS_MIXED)
    return fail(s, KS_EINVAL, "the split-BF16 projection (1) is for mixed-precision systems only");
  if (t->x_shape != -1) {
    const ks_status r = set_x_shape(s, t->x_shape);
    if (r != KS_OK) return r;
  }
  s->xg_max = t->x_group;
  s->pg_max = t->plane_group;
  ++s->gen;
  if (t->projection != -1) return set_projection(s, t->projection);
  return KS_OK;
}

ks_status ks_autotune(ks_system* s, int norb, void* stream, ks_tuning* out) {
  ks_status r = check_common(s, norb);
  if (r != KS_OK) return r;
  if (norb < 1) return fail(s, KS_EINVAL, "norb must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  const int nb = chunk_len(s, norb);
  int nb2 = 1;
  while (nb2 < nb) nb2 *= 2;
  const TuneKey key{s->n[0], s->n[1], s->n[2], s->prec, s->nplanes, nb2};
  TuneResult found;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) found = it->second;
  }
  if (found.xg > 0) {
    if ((r = set_x_shape(s, found.shape)) != KS_OK) return r;
    s->xg_max = found.xg;
    s->pg_max = found.pg;
    ++s->gen;
    if (out) *out = ks_tuning{s->xg_max, s->pg_max, 0.0, 1, s->xshape, s->proj_mode};
    return KS_OK;
  }
  const bool timing = s->timing;
  s->timing = false;   // keep the search out of the kernel-time counters
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto done = [&](ks_status v) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    s->timing = timing;
    return v;
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return done(fail(s, KS_EDEVICE, "hipEventCreate failed"));
  if (hipMemsetAsync(s->pk[0], 0, (size_t)nb * s->npw_stride * sizeof(double2), st) != hipSuccess)
    return done(fail(s, KS_EDEVICE, "hipMemsetAsync failed"));
  Taylor none{{0.0, 0.0}, 0, {0.0, 0.0}};
  const int xgs[] = {2, 4, 8, 16, 32, 64};
  const int pgs[] = {1, 2, 4, 8, 16};
  // Within a shape the fastest caps win; a later shape (in the order 0..3)
  // replaces an earlier one only when it is at least SHAPE_MARGIN faster, so
  // shapes that time within noise of each other do not flip between runs.
  constexpr float SHAPE_MARGIN = 0.01f;
  TuneResult best{s->xg_max, s->pg_max, s->xshape};
  float best_ms = -1.0f;
  for (int shape = 0; shape < 4; ++shape) {
    if (!x_shape_available(s->n[0], shape)) continue;
    if ((r = set_x_shape(s, shape)) != KS_OK) return done(r);
    TuneResult sbest{s->xg_max, s->pg_max, shape};
    float sbest_ms = -1.0f;
    for (int xg : xgs) {
      for (int pg : pgs) {
        s->xg_max = xg;
        s->pg_max = pg;
        if ((r = hpsi_packed(s, nb, s->pk[0], true, s->pk[1], nullptr, H_OUT, none, st)) != KS_OK) return done(r);
        if (hipEventRecord(e0, st) != hipSuccess) return done(fail(s, KS_EDEVICE, "hipEventRecord failed"));
        for (int rep = 0; rep < 2; ++rep)
          if ((r = hpsi_packed(s, nb, s->pk[0], true, s->pk[1], nullptr, H_OUT, none, st)) != KS_OK) return done(r);
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
          return done(fail(s, KS_EDEVICE, "event timing failed"));
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          return done(fail(s, KS_EDEVICE, "hipEventElapsedTime failed"));
        ms *= 0.5f;
        if (sbest_ms < 0.0f || ms < sbest_ms) {
          sbest_ms = ms;
          sbest = TuneResult{xg, pg, shape};
        }
      }
    }
    if (best_ms < 0.0f || sbest_ms < (1.0f - SHAPE_MARGIN) * best_ms) {
      best_ms = sbest_ms;
      best = sbest;
    }
  }
  if ((r = set_x_shape(s, best.shape)) != KS_OK) return done(r);
  s->xg_max = best.xg;
  s->pg_max = best.pg;
  ++s->gen;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  if (out) *out = ks_tuning{best.xg, best.pg, (double)best_ms, 0, best.shape, s->proj_mode};
  return done(KS_OK);
}

ks_status ks_set_kernel_timing(ks_system* s, int enable) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  timing_free(s);
  for (int k = 0; k < 16; ++k) {
    s->kt_ms[k] = 0.0;
    s->kt_n[k] = 0;
  }
  if (!enable) return KS_OK;
  s->ev.resize(2 * EV_PAIRS);
  s->ev_kid.assign(EV_PAIRS, 0);
  for (auto& e : s->ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      e = nullptr;
      timing_free(s);
      return fail(s, KS_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(r));
    }
  }
  s->timing = true;
  return KS_OK;
}

ks_status ks_kernel_time(ks_system* s, int kernel_id, double* total_ms, long long* launches) {
  if (!s) return fail(nullptr, KS_EINVAL, "null system");
  if (kernel_id < 0 || kernel_id >= KS_K_COUNT) return fail(s, KS_EINVAL, "unknown kernel id");
  timing_flush(s);
  if (total_ms) *total_ms = s->kt_ms[kernel_id];
  if (launches) *launches = s->kt_n[kernel_id];
  return KS_OK;
}

}  // extern "C"
