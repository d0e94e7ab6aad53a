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
// Largest fused bond of the large-bond row sweep (working matrices in global memory; D_k = 2,
// chi <= 64) and its per-sample slot of working matrices: X | A J (2 (n+1) n), R | G ((n+1) n)
// and Y (2n x n), n = kMaxNBig.
constexpr int kMaxNBig = 128;
constexpr int kBigSlot = 2 * (kMaxNBig + 1) * kMaxNBig + (kMaxNBig + 1) * kMaxNBig + 2 * kMaxNBig * kMaxNBig;
// Largest working state Dk^(L+1) of the complex exact-contraction path held in LDS (3^7: 6 x 6 at
// Dk = 3); above it, up to kCxMaxWorkGlobal (3^11: 10 x 10 at Dk = 3), the two working states of a
// sample live in a global slot.
constexpr int kCxMaxWork = 2187;
constexpr int kCxMaxWorkGlobal = 177147;

// Static shape tables of one problem, copied to the device once per handle.
struct Dims {
  int L, N, Dk, chi;
  int n_sites;
  int P4;          // Dk^4: row stride of a projected tensor
  int site_stride; // chi * Dk * chi: doubles per stored boundary site
  int row_stride;  // L * site_stride
  int maxN;        // largest fused bond chi*Dk actually reached (<= kMaxN; <= kMaxNBig for the
                   // amplitude alone)
  int mixed;       // 1: contractions in FP32 (factorisations, logs and sums stay FP64)
  int max_sweeps;  // Jacobi sweep limit per SVD
  // tuning of the row sweep (peps_tuning): Jacobi lanes per column pair, preconditioning of the
  // down (reversible) and up sweeps' large SVDs, smallest cut dimension that is preconditioned
  int jacobi_lanes, down_precond, up_precond, precond_min;
  int small_waves;  // waves per SIMD of the chi*Dk <= 32 row-sweep kernels: 2 or 4
  int var_sweeps;   // variational compression: fitting sweeps after each row's SVD truncation (0: none)
  int matter;       // 1: hard-core bosons on the vertices (occupation plane in the configuration)
  int planes;       // planes of a configuration: 2 (links) or 3 (links + occupations)
  int cx32;         // complex handles: 1 when the exact contractions run in complex64
  // measurement support: the row-sweep kernels add each workgroup's shader-clock cycles per phase
  // of the row step into phase_clk[PEPS_PH_COUNT] (device) when it is not null
  unsigned long long* phase_clk = nullptr;
};

struct DeviceTables {
  int64_t* site_offset;  // [L*L+1]
  int8_t* Q;             // [L*L]
  int* bond;             // [(L-1)][L+1]  bond[y][c] of boundary row y (cut c); bond[y][0]=bond[y][L]=1
  int* qrk;              // [(L-1)][L]    qrk[y][c] = columns of Q_c / rows of R_c in row y's QR sweep
  double* plaq;          // [8] c[t]
  double* elec;          // [8] e[n]
};

}  // namespace gipeps

struct peps_handle {
  gipeps::Dims d;
  int dtype;
  int ckpt_every;
  bool keep_tape;  // amplitude stores every row's factorisations; logderiv reverses them
  int device;
  double plaq_coef[8];
  double elec[8];
  double hop, mass;  // eq. matter: hopping coupling J and chemical potential m (matter only)
  int64_t n_params;
  std::vector<int64_t> site_offset;
  std::vector<int8_t> Q;
  std::vector<int> bond;  // host copy of DeviceTables::bond
  std::vector<int> qrk;
  gipeps::DeviceTables t;
  // per-kernel timing: (family, start, stop) event triples, recorded while profiling is on
  const void* last_amp_ws = nullptr;  // workspace and batch of the last peps_amplitude
  int last_amp_B = -1;
  const void* last_energy_ws = nullptr;  // workspace and batch of the last peps_local_energy
  int last_energy_B = -1;
  bool profiling = false;
  struct Rec { int family; hipEvent_t a, b; };
  std::vector<Rec> recs;
};

namespace gipeps {

// Workspace map for a batch of B samples (byte offsets into ws; 256-byte aligned).
struct WsLayout {
  size_t down;      // double [L-1][B][row_stride]    boundary rows D_0..D_{L-2}
  size_t lognu;     // double [B][L]                  ln nu_y (index y), slot 0 unused
  size_t qscr;      // double [B][L][qslot]           per-site Q factors of the row being swept
  size_t wbig;      // double [B][kBigSlot]           working matrices of the large-bond row sweep
  size_t qall;      // double [L-2][B][L][qslot]      keep_tape: Q factors of rows 1..L-2
  size_t tall;      // double [L-2][B][L][tape slot]  keep_tape: factorisation tapes of rows 1..L-2
  size_t up;        // double [L-1][B][row_stride]    up boundaries U_1..U_{L-1} (mirrored sweep)
  size_t uplognu;   // double [B][L]
  size_t fproj;     // double [B][L*L][P4]            mirrored projected tensors (d <-> u)
  size_t strip;     // double [B][strip_scratch]      per-sample strip halves X1_c, Y1_c
  size_t part;      // double [B][L-1]                per-strip plaquette sums
  size_t pabs;      // double [B][L-1]                per-strip sums of |c[t] ratio|
  size_t tape;      // double [B][L][tape slot]       factorisations of the row being reversed
  size_t qbar;      // double [B][L][qslot]           adjoints of the row's Q factors
  size_t xbar;      // double [B][2 * bond]           adjoint of the last X of the row (bond: 72 or 128)
  size_t psibar;    // double [2][B][row_stride]      adjoint boundary rows (double buffer)
  size_t rowtmp;    // double [B][row_stride]         recomputed boundary row
  size_t lognu2;    // double [B][L]                  ln nu of recomputed rows (unused values)
  size_t seg;       // double [ckpt][B][row_stride]   rows recomputed from a checkpoint
  size_t sr;        // double [B + 8]                 sr_build: (O v)_b and <O>.v
  size_t cg;        // double [3 n_params + 2 (kMaxCgIter + 2)]  sr_solve: r, p, q and CG scalars
  size_t flag;      // uint32 [4]                     state flags written by the host
  size_t status;    // uint32 [B]                     per-sample PEPS_FLAG_* bits
  size_t escale;    // double [B]                     magnitude of E_loc's terms (last local energy)
  size_t venv;      // double [B][2(L+1)+2][site]     variational compression: environments, Q, R
  size_t lprop;     // uint8 [B][2][L][L]             Metropolis proposals
  size_t laprop;    // double [B]                     ln|Psi| of the proposals
  size_t sgprop;    // double [B]                     sign of the proposals (unused)
  size_t moved;     // uint8 [B]                      link moves: chains whose proposal differs
  size_t amp_end, energy_end, logderiv_end, sample_end;
  size_t total;
};
WsLayout ws_layout(const peps_handle* h, int B, uint32_t what);
size_t qslot_doubles(const Dims& d);  // doubles per (sample, site) Q-factor slot of the row sweep

// Kernel launchers (one per .hip file family); each returns a hipError_t.
hipError_t launch_sample_powers(const Dims& d, uint64_t seed, uint64_t stream, int B, uint8_t* powers,
                                hipStream_t s);
hipError_t launch_propose(const Dims& d, int p, int sweep, uint64_t seed, uint64_t stream, int B,
                          const uint8_t* cur, uint8_t* prop, hipStream_t s);
hipError_t launch_propose_hop(const Dims& d, int dir, int x, int y, int B, const uint8_t* cur,
                              uint8_t* prop, uint8_t* moved, hipStream_t s);
// moved (uint8 [B], or null when every chain moved): 0 marks a chain whose proposal is its state
hipError_t launch_accept(const Dims& d, int p, int sweep, uint64_t seed, uint64_t stream, int B,
                         const uint8_t* moved, const double* la_prop, const uint8_t* valid_prop,
                         const uint8_t* prop, double* la_cur, uint8_t* cur, int32_t* accepted,
                         hipStream_t s);
hipError_t launch_links_from_powers(const Dims& d, const uint8_t* powers, int B, uint8_t* links,
                                    hipStream_t s);
hipError_t launch_matter_links(const Dims& d, const DeviceTables& t, const uint8_t* powers,
                               const uint8_t* occ, int B, uint8_t* links, hipStream_t s);
hipError_t launch_project(const Dims& d, const DeviceTables& t, const double* theta,
                          const uint8_t* links, int B, double* proj, int32_t* block_id,
                          uint8_t* valid, hipStream_t s);
hipError_t launch_row0_to_mps(const Dims& d, const double* proj, const uint8_t* valid, int B,
                              double* out_row, hipStream_t s);
// up: an up sweep (mirrored lattice; its factorisations are never reversed), preconditioned with
// d.up_precond, else d.down_precond (see peps_tuning)
// status (uint32 [B] or null): bit PEPS_FLAG_SVD_NOCONV is OR-ed in for a sample whose Jacobi
// stopped at the sweep limit without converging
hipError_t launch_row_sweep(const Dims& d, const DeviceTables& t, int y, const double* proj,
                            const uint8_t* valid, int B, const double* prev_row, double* out_row,
                            double* qscr, double* lognu, double* tape, hipStream_t s,
                            bool up = false, uint32_t* status = nullptr, double* wbig = nullptr);
// wbig: per-sample working slots (double [B][kBigSlot]) of the large-bond kernel, required when
// d.maxN > kMaxN
// Ragged batch: row y of up to kMaxRagged lattices in one launch (passed by value as a kernel
// argument, so the launch needs no device memory of its own).
constexpr int kMaxRagged = 8;
struct RaggedRow {
  Dims d;
  const int* bond;
  const int* qrk;
  const double* proj;
  const uint8_t* valid;
  const double* prev_row;
  double* out_row;
  double* qscr;
  size_t qslot;  // doubles per (sample, site) Q-factor slot (qslot_doubles of the group's shapes)
  double* lognu;
  uint32_t* status;
  double* wbig;
  int first_block;  // first workgroup of the group; B samples follow
};
struct RaggedRows {
  int n;
  RaggedRow g[kMaxRagged];
};
// maxN: largest fused bond over the groups (selects the instantiation); mixed, lanes, waves,
// precondition settings: taken from `tune` (the first group's handle)
hipError_t launch_row_sweep_ragged(const RaggedRows& r, int total_blocks, int y, int Dk, int maxN,
                                   const Dims& tune, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
// variational compression of row y's boundary (out_row, in place) against the exact product of row
// y with prev_row; a no-op when d.var_sweeps == 0
hipError_t launch_var_refine(const Dims& d, const DeviceTables& t, int y, const double* proj, const uint8_t* valid,
                             int B, const double* prev_row, double* out_row, double* venv, double* lognu,
                             hipStream_t s);
size_t tape_slot_doubles(const Dims& d);  // doubles per (sample, site) of the row-sweep tape
size_t strip_scratch_doubles(const Dims& d);
hipError_t launch_mirror_proj(const Dims& d, const double* proj, const uint8_t* valid, int B,
                              double* fproj, hipStream_t s);
hipError_t launch_strip(const Dims& d, int py, const DeviceTables& t, const double* proj,
                        const double* theta, const uint8_t* links, const uint8_t* valid, int B,
                        const double* down, const double* up, const double* plaq, double hop,
                        double* scratch, double* part, double* pabs, hipStream_t s, double* wbig = nullptr);
// links_pass 0: the strip's plaquette moves; 1 (matter): its link moves
hipError_t launch_strip_mc(const Dims& d, int py, int sweep, uint64_t seed, uint64_t stream,
                           const DeviceTables& t, const double* theta, uint8_t* links,
                           const uint8_t* valid, int B, const double* down, const double* up,
                           double* scratch, int32_t* accepted, int links_pass, hipStream_t s,
                           double* wbig = nullptr);
hipError_t launch_eloc_final(const Dims& d, const uint8_t* links, const uint8_t* valid, int B,
                             const double* elec, double mass, const double* part, const double* pabs,
                             double* e_loc, double* scale, hipStream_t s);
hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s);
hipError_t launch_adj_close(const Dims& d, const int* bond_last, const double* proj,
                            const uint8_t* valid, int B, const double* last_row, double* psibar,
                            double* O, hipStream_t s);
hipError_t launch_adj_row0(const Dims& d, const uint8_t* valid, int B, const double* psibar,
                           double* O, hipStream_t s);
hipError_t launch_adj_row(const Dims& d, const DeviceTables& t, int y, const double* proj,
                          const uint8_t* valid, int B, const double* prev_row,
                          const double* cur_row, const double* tape, const double* qscr,
                          const double* psibar_in, double* qbar, double* xbar, double* psibar_out,
                          double* O, hipStream_t s, double* wbig = nullptr);
hipError_t launch_vjp(const Dims& d, const DeviceTables& t, const int32_t* block_id,
                      const uint8_t* valid, const double* w, const double* O, int B, double* vjp,
                      hipStream_t s);
// Conjugate-gradient pieces of sr_solve: vector steps and the fixed-order dot products (r.r into
// sc[2k], p.q into sc[2k+1]).
enum { kCgInit = 0, kCgShift = 1, kCgStep = 2, kCgDir = 3, kCgDotRR = 4, kCgDotPQ = 5 };
constexpr int kMaxCgIter = 10000;
hipError_t launch_sr_rows(const Dims& d, const DeviceTables& t, int64_t n_params, const int32_t* block_id,
                          const uint8_t* valid, const double* O, const double* omean, int B, int64_t row0,
                          int64_t nrows, double* S, hipStream_t s);
hipError_t launch_cg(int op, int64_t n, double* x, double* r, double* p, double* q, const double* F,
                     double* sc, int k, double shift, hipStream_t s);
hipError_t launch_sr(const Dims& d, const DeviceTables& t, int64_t n_params, const int32_t* block_id,
                     const uint8_t* valid, const double* O, const double* e_loc, int B, int mode,
                     const double* v, double* F, double* omean, double* S_or_Sv, double* ov,
                     double* omv, hipStream_t s);
hipError_t launch_close(const Dims& d, const int* bond_last, const double* proj,
                        const uint8_t* valid, int B, const double* last_row, const double* lognu,
                        double* log_abs, double* sign, hipStream_t s);

// Complex exact-contraction path (k_complex.hip); complex vectors are interleaved (re, im) doubles.
size_t cx_lds_bytes(const Dims& d, int which);  // 0: states / logderiv kernels, 1: local energy
size_t cx_work(const Dims& d);         // Dk^(L+1): entries of one working state
// bytes of one complex entry of the contractions' states: 8 (complex64) or 16 (complex128)
inline size_t cx_elem_bytes(const Dims& d) { return d.cx32 ? 2 * sizeof(float) : 2 * sizeof(double); }
bool cx_work_global(const Dims& d);    // working states above kCxMaxWork live in a global slot (wscr)
hipError_t launch_cx_project(const Dims& d, const DeviceTables& t, const double* theta, const uint8_t* links,
                             int B, double* proj, int32_t* block_id, uint8_t* valid, hipStream_t s);
hipError_t launch_cx_states(const Dims& d, const double* proj, const uint8_t* valid, int B, double* states,
                            double* expo, double* log_abs, double* phase, double* wscr, hipStream_t s);
hipError_t launch_cx_eloc(const Dims& d, const DeviceTables& t, const double* theta, const uint8_t* links,
                          const double* proj, const uint8_t* valid, int B, const double* states, double* e_loc,
                          double* gscr, double* wscr, hipStream_t s);
// one strip-ratio Metropolis sweep of complex chains (links updated in place, accepted added to)
hipError_t launch_cx_strip_mc(const Dims& d, const DeviceTables& t, const double* theta, uint8_t* links,
                              const uint8_t* valid, int B, double* states, double* gscr, double* wscr,
                              uint64_t seed, uint64_t stream, int sweep, int32_t* accepted, hipStream_t s);
hipError_t launch_cx_logderiv(const Dims& d, const double* proj, const uint8_t* valid, int B, const double* states,
                              double* gscr, double* O, double* wscr, hipStream_t s);
hipError_t launch_cx_weights(int B, int mode, const double* log_abs, const uint8_t* valid, double* w,
                             hipStream_t s);
int cx_blocks_per_site(const Dims& d);
// per site, the weighted samples of each block (off: int32 [L*L][N^3+1], list: int32 [L*L][B])
hipError_t launch_cx_index(const Dims& d, int B, const int32_t* bid, const double* w, int32_t* off, int32_t* list,
                           hipStream_t s);
hipError_t launch_cx_force(const Dims& d, const DeviceTables& t, int64_t n, int B, const int32_t* off,
                           const int32_t* list, const double* w, const double* O, const double* e_loc, double* sc,
                           double* omean, double* g, hipStream_t s);
hipError_t launch_cx_matvec(const Dims& d, const DeviceTables& t, int64_t n, int B, const int32_t* bid,
                            const int32_t* off, const int32_t* list, const double* w, const double* O,
                            const double* omean, double shift, const double* v, double* ov, double* sc, double* out,
                            hipStream_t s);
hipError_t launch_cx_dot(int64_t n, const double* a, const double* b, double* out, hipStream_t s);
hipError_t launch_cx_axpy(int64_t n, double ar, double ai, const double* z, const double* x, double* y,
                          hipStream_t s);

// Workspace of a complex (PEPS_C128_EXACT) handle: row states and their exponents, the backward
// states of the log-derivatives, and (PEPS_WS_TVMC) the tVMC buffers.
struct CxWs {
  size_t states;   // double [B][2(L+1)][Dk^L][2]   V_0..V_L, Top_0..Top_L
  size_t expo;     // double [B][2(L+1)]            their power-of-two exponents
  size_t gscr;     // double [B][L][Dk^(L+1)][2]    backward states of one row
  size_t wscr;     // double [B][2][Dk^(L+1)][2]    working states (only above kCxMaxWork entries)
  size_t w;        // double [B]                     sample weights
  size_t ov;       // double [B][2]                  O_b . v
  size_t sc;       // double [64]                    <E>, <w O.v>, CG scalars
  size_t ioff;     // int32 [L*L][N^3+1]             per site: first index of each block's samples
  size_t ilist;    // int32 [L*L][B]                 per site: the weighted samples, by block
  size_t omean;    // double [n][2]
  size_t g;        // double [n][2]                  force (right side of eq. tVMC)
  size_t y, r, p, q;  // double [n][2]             CG vectors
  size_t proj;     // double [B][L*L][P4][2]         tvmc_step's own buffers
  size_t bid;      // int32 [B][L*L]
  size_t valid;    // uint8 [B]
  size_t la;       // double [B]
  size_t phase;    // double [B][2]
  size_t O;        // double [B][L*L][P4][2]
  size_t eloc;     // double [B][2]
  size_t xdot;     // double [n][2]
  size_t theta1;   // double [n][2]
  size_t lprop;    // uint8 [B][2][L][L]             (PEPS_WS_SAMPLE) Metropolis proposals
  size_t laprop;   // double [B]                     their ln|Psi|
  size_t phprop;   // double [B][2]                  their phase
  size_t moved;    // uint8 [B]
  size_t base_end, total;
};
CxWs cx_ws_layout(const peps_handle* h, int B, uint32_t what);

}  // namespace gipeps
