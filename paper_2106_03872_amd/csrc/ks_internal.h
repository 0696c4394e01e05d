// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/ks.h"

namespace ks {

// Plane-wave sphere in packed order: planes m0 = m0lo .. m0lo+nplanes-1, in
// each plane the columns m1 = m1lo(plane) .. , in each column the run of m2
// values m2lo(col) .. m2lo(col)+len-1 stored contiguously.
struct SphereTab {
  const int* plane_col0;  // [nplanes+1] first column id of each plane
  const int* plane_m1lo;  // [nplanes]
  const int* col_off;     // [ncols+1] packed offset of each column (col_off[ncols] = npw)
  const int* col_m2lo;    // [ncols]
  int nplanes, m0lo;
  int n0, n1, n2;
};

// Kleinman-Bylander projector points regrouped into runs ("chords") of
// consecutive j0 along x-pencils (fixed j1, j2).
struct ChordTab {
  const int* ch_pencil;    // [nchords] pencil index j1*n2+j2
  const int* ch_atom;      // [nchords]
  const int* ch_r0;        // [nchords] first j0 of the run
  const int* ch_len;       // [nchords]
  const int* ch_boff;      // [nchords] first row of the run in beta
  const double* beta;      // [npoints][nproj] reordered projector values
  const int* tile_off;     // [ntiles+1] chord range of each x-tile
  const int* pen_off;      // [npencils+1] chord range of each pencil
  const int* atom_off;     // [natoms+1]
  const int* atom_list;    // chords of each atom, ascending
  const double* d;         // [natoms][nproj]
  int nchords, natoms, nproj;
};

enum HMode { H_OUT = 0, H_TAYLOR = 1 };

struct Taylor {
  double2 coef;  // (-i dt)^k / k!
  int write_w;   // store w_k = H w_{k-1}
};

}  // namespace ks

struct ks_system {
  int n[3];
  double L[3];
  double ecut;
  int prec;
  int max_norb;
  long long N;
  int npl;  // n1*n2
  double omega, dV;

  // sphere
  int nplanes = 0, m0lo = 0, ncols = 0, npw = 0, npw_stride = 0, ncol_max = 0;
  int* d_plane_col0 = nullptr;
  int* d_plane_m1lo = nullptr;
  int* d_col_off = nullptr;
  int* d_col_m2lo = nullptr;
  double2* d_tw0 = nullptr;
  double2* d_tw1 = nullptr;
  float2* d_tw0f = nullptr;
  float2* d_tw1f = nullptr;

  // local potential
  double* d_v = nullptr;
  bool have_v = false;

  // projectors
  int natoms = 0, nproj = 0, nchords = 0, npoints = 0;
  int xnb = 32, ntiles = 0;
  int *d_ch_pencil = nullptr, *d_ch_atom = nullptr, *d_ch_r0 = nullptr, *d_ch_len = nullptr,
      *d_ch_boff = nullptr, *d_tile_off = nullptr, *d_pen_off = nullptr, *d_atom_off = nullptr,
      *d_atom_list = nullptr;
  double *d_beta = nullptr, *d_kb = nullptr;

  // workspace (one chunk of cb orbitals)
  int cb = 1;
  void* pk[3] = {nullptr, nullptr, nullptr};  // packed chunk buffers
  void* T = nullptr;                          // [cb][nplanes][n1*n2]
  void* U = nullptr;
  void* partial = nullptr;                    // [cb][nchords][nproj]
  double2* DP = nullptr;                      // [cb][natoms][nproj]
  double* red = nullptr;                      // [2*max_norb]
  size_t partial_cap = 0, dp_cap = 0;

  // orthonormalisation workspace (allocated on first use)
  void* ortho_pk = nullptr;
  double2* ortho_S = nullptr;
  double2* ortho_W = nullptr;
  int* ortho_info = nullptr;
  int ortho_cap = 0;

  // kernel timing (ks_set_kernel_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev;       // pairs
  std::vector<int> ev_kid;          // kernel class of each pair
  int ev_used = 0;
  double kt_ms[16] = {0};
  long long kt_n[16] = {0};

  std::string err;
};

namespace ks {

// launchers (ks_kernels.hip); return false when the size has no kernel
bool launch_pack(const ks_system* s, int nb, const double2* box, long long box_stride, void* pk,
                 hipStream_t st);
bool launch_unpack(const ks_system* s, int nb, const void* pk, double2* box, long long box_stride,
                   hipStream_t st);
bool launch_plane_inv(const ks_system* s, int nb, const void* pk, void* T, hipStream_t st);
bool launch_xproj(const ks_system* s, int nb, const void* T, void* partial, hipStream_t st);
bool launch_proj_reduce(const ks_system* s, int nb, const void* partial, double2* DP, hipStream_t st);
bool launch_xapply(const ks_system* s, int nb, const void* T, const double2* DP, void* U, hipStream_t st);
bool launch_plane_fwd(const ks_system* s, int nb, const void* U, const void* win, void* wout, void* acc,
                      HMode mode, Taylor tay, hipStream_t st);
bool launch_xdens(const ks_system* s, int nb, const void* T, const double* occ, double* rho, int accumulate,
                  hipStream_t st);
bool launch_dots(const ks_system* s, int nb, const void* a, const void* b, double* out, hipStream_t st);
bool launch_energy_sum(int norb, const double* occ, const double* red, double* energy, hipStream_t st);

bool supported_size(int n);
int x_tile_nb(int n0);
size_t plane_lds_bytes(const ks_system* s);

}  // namespace ks
