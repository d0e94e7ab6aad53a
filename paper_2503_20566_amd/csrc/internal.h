// Internal declarations shared by the host API (api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/gipeps.h"

namespace gipeps {

// Largest boundary-MPS bond after the row application (chi * Dk) the LDS-resident kernels hold,
// and largest physical (vertical-bond) dimension.
constexpr int kMaxN = 72;
constexpr int kMaxDk = 2;
constexpr int kMaxM = kMaxN * kMaxDk;  // rows of the QR working matrix (left bond * physical)

// Static shape tables of one problem, copied to the device once per handle.
struct Dims {
  int L, N, Dk, chi;
  int n_sites;
  int P4;          // Dk^4: row stride of a projected tensor
  int site_stride; // chi * Dk * chi: doubles per stored boundary site
  int row_stride;  // L * site_stride
  int maxN;        // largest fused bond chi*Dk actually reached (<= kMaxN)
};

struct DeviceTables {
  int64_t* site_offset;  // [L*L+1]
  int8_t* Q;             // [L*L]
  int* bond;             // [(L-1)][L+1]  bond[y][c] of boundary row y (cut c); bond[y][0]=bond[y][L]=1
  int* qrk;              // [(L-1)][L]    qrk[y][c] = columns of Q_c / rows of R_c in row y's QR sweep
};

}  // namespace gipeps

struct peps_handle {
  gipeps::Dims d;
  int dtype;
  int ckpt_every;
  int device;
  double plaq_coef[8];
  double elec[8];
  int64_t n_params;
  std::vector<int64_t> site_offset;
  std::vector<int8_t> Q;
  std::vector<int> bond;  // host copy of DeviceTables::bond
  std::vector<int> qrk;
  gipeps::DeviceTables t;
};

namespace gipeps {

// Workspace map for a batch of B samples (byte offsets into ws; 256-byte aligned).
struct WsLayout {
  size_t down;      // double [L-1][B][row_stride]    boundary rows D_0..D_{L-2}
  size_t lognu;     // double [B][L]                  ln nu_y (index y), slot 0 unused
  size_t qscr;      // double [B][L][kMaxM*kMaxN]     per-site Q factors of the row being swept
  size_t up;        // double [L-1][B][row_stride]    up boundaries U_1..U_{L-1} (mirrored sweep)
  size_t uplognu;   // double [B][L]
  size_t fproj;     // double [B][L*L][P4]            mirrored projected tensors (d <-> u)
  size_t flag;      // uint32 [4]                     state flags written by the host
  size_t total;
};
WsLayout ws_layout(const peps_handle* h, int B, uint32_t what);

// Kernel launchers (one per .hip file family); each returns a hipError_t.
hipError_t launch_links_from_powers(const Dims& d, const uint8_t* powers, int B, uint8_t* links,
                                    hipStream_t s);
hipError_t launch_project(const Dims& d, const DeviceTables& t, const double* theta,
                          const uint8_t* links, int B, double* proj, int32_t* block_id,
                          uint8_t* valid, hipStream_t s);
hipError_t launch_row0_to_mps(const Dims& d, const double* proj, const uint8_t* valid, int B,
                              double* out_row, hipStream_t s);
hipError_t launch_row_sweep(const Dims& d, const DeviceTables& t, int y, const double* proj,
                            const uint8_t* valid, int B, const double* prev_row, double* out_row,
                            double* qscr, double* lognu, hipStream_t s);
hipError_t launch_close(const Dims& d, const int* bond_last, const double* proj,
                        const uint8_t* valid, int B, const double* last_row, const double* lognu,
                        double* log_abs, double* sign, hipStream_t s);

}  // namespace gipeps
