// peps_amplitude_noalloc: the amplitude (SM S-2 eq. project with the canonical boundary sweep) for
// callers that cannot allocate device memory -- code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc.  The same kernels as peps_amplitude (row 0 as an MPS, one
// k_row_sweep launch per row, k_close) run on a fixed scratch array that lives in this file instead
// of on a caller workspace: two boundary rows used alternately (only the last one is needed), the
// ln nu_y, the per-site Q factors of the row being swept and the per-sample flag words.
//
// The array is a file-scope __device__ object, so each GPU that loads the library holds one copy for
// the life of the process.  Host code never passes its name to a kernel: the device address of the
// copy on each GPU is taken once per device with hipGetSymbolAddress (with that device current) and
// every kernel argument and offset is derived from that address.
#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;  // 128 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* g_scratch_ptr[kMaxDevices] = {};
std::once_flag g_scratch_once[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of this GPU's scratch copy (looked up on the first call per device).
hipError_t scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    if (e == hipSuccess) g_scratch_ptr[dev] = p;
  });
  *out = g_scratch_ptr[dev];
  return g_scratch_err[dev];
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the scratch parts for a batch of B (256-byte aligned).
struct NoAllocLayout {
  size_t row[2], lognu, qscr, status, total;
};

NoAllocLayout layout_for(const gipeps::Dims& d, int B) {
  NoAllocLayout w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t Bz = (size_t)B;
  w.row[0] = take(sizeof(double) * Bz * d.row_stride);
  w.row[1] = take(sizeof(double) * Bz * d.row_stride);
  w.lognu = take(sizeof(double) * Bz * d.L);
  w.qscr = take(sizeof(double) * Bz * d.L * gipeps::qslot_doubles(d));
  w.status = take(sizeof(uint32_t) * Bz);
  w.total = off;
  return w;
}

}  // namespace

extern "C" int peps_amplitude_noalloc(peps_handle* h, const double* proj, const uint8_t* valid,
                                      int32_t B, double* log_abs, double* sign, void* stream) {
  using namespace gipeps;
  if (h && h->dtype == PEPS_C128_EXACT) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || (B > 0 && (!proj || !valid || !log_abs || !sign))) return PEPS_ERR_ARG;
  if (h->d.var_sweeps > 0) return PEPS_ERR_UNSUPPORTED;  // the fixed scratch holds no fitting environments
  if (h->d.maxN > kMaxN) return PEPS_ERR_UNSUPPORTED;    // nor the large-bond working matrices
  if (B == 0) return PEPS_OK;
  const Dims& d = h->d;
  const NoAllocLayout w = layout_for(d, B);
  if (w.total > kScratchBytes) return PEPS_ERR_WORKSPACE;
  // the handle's shape tables must already be on this device (peps_create puts them there when a
  // GPU is present); this entry point uploads nothing
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return PEPS_ERR_HIP;
  if (h->device < 0) return PEPS_ERR_STATE;
  if (h->device != dev) return PEPS_ERR_ARG;
  void* base = nullptr;
  if (scratch_on(dev, &base) != hipSuccess || !base) return PEPS_ERR_HIP;
  char* b = static_cast<char*>(base);
  double* rows[2] = {reinterpret_cast<double*>(b + w.row[0]), reinterpret_cast<double*>(b + w.row[1])};
  double* lognu = reinterpret_cast<double*>(b + w.lognu);
  double* qscr = reinterpret_cast<double*>(b + w.qscr);
  uint32_t* status = reinterpret_cast<uint32_t*>(b + w.status);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the flag words start at zero on every call (a fill kernel: the array keeps the last call's bits)
  hipError_t e = launch_fill_u32(status, (size_t)B, 0u, s);
  if (e == hipSuccess) e = launch_row0_to_mps(d, proj, valid, B, rows[0], s);
  for (int y = 1; y <= d.L - 2 && e == hipSuccess; ++y)
    e = launch_row_sweep(d, h->t, y, proj, valid, B, rows[(y - 1) & 1], rows[y & 1], qscr, lognu,
                         nullptr, s, /*precond=*/false, status);
  if (e == hipSuccess)
    e = launch_close(d, h->t.bond + (size_t)(d.L - 2) * (d.L + 1), proj, valid, B,
                     rows[(d.L - 2) & 1], lognu, log_abs, sign, s);
  return e == hipSuccess ? PEPS_OK : PEPS_ERR_HIP;
}
