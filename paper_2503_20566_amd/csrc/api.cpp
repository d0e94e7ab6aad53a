// Host side of the C ABI declared in include/gipeps.h: argument checks, static shape tables,
// workspace map and kernel sequencing.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

using namespace gipeps;

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? PEPS_OK : PEPS_ERR_HIP; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// complex handles: exact contraction in complex128 or complex64
bool is_cx(int dtype) { return dtype == PEPS_C128_EXACT || dtype == PEPS_C64_EXACT; }

// Bond tables of the canonical sweep (identical for the down and the mirrored up sweep).
//   bond[0][c]: row 0 as an MPS (1 at the ends, Dk inside);
//   row y >= 1: fused bonds m_c = bond[y-1][c] * (Dk inside, 1 at the ends); QR left to right
//   gives qrk[y][c] = min(qrk[y][c-1] * Dk, m_{c+1}) (qrk[y][-1] = 1); truncation right to left
//   gives bond[y][c] = min(chi, qrk[y][c-1], Dk * bond[y][c+1]) (bond[y][L] = 1, bond[y][0] = 1).
void build_bonds(peps_handle* h) {
  const int L = h->d.L, Dk = h->d.Dk, chi = h->d.chi;
  h->bond.assign((size_t)(L - 1) * (L + 1), 1);
  h->qrk.assign((size_t)(L - 1) * L, 1);
  int maxN = 1;
  for (int c = 0; c <= L; ++c) h->bond[c] = (c == 0 || c == L) ? 1 : Dk;
  for (int y = 1; y <= L - 2; ++y) {
    const int* bp = &h->bond[(size_t)(y - 1) * (L + 1)];
    int* bn = &h->bond[(size_t)y * (L + 1)];
    int* q = &h->qrk[(size_t)y * L];
    std::vector<int> m(L + 1);
    for (int c = 0; c <= L; ++c) {
      m[c] = bp[c] * ((c == 0 || c == L) ? 1 : Dk);
      maxN = std::max(maxN, m[c]);
    }
    int r = 1;
    for (int c = 0; c < L - 1; ++c) {
      q[c] = std::min(r * Dk, m[c + 1]);
      r = q[c];
      maxN = std::max(maxN, r);
    }
    q[L - 1] = 1;
    int cn = 1;
    bn[L] = 1;
    for (int c = L - 1; c >= 1; --c) {
      bn[c] = std::min(std::min(chi, q[c - 1]), Dk * cn);
      cn = bn[c];
      maxN = std::max(maxN, Dk * cn);
    }
    bn[0] = 1;
  }
  h->d.maxN = maxN;
}

void free_tables(peps_handle* h) {
  if (h->t.site_offset) (void)hipFree(h->t.site_offset);
  if (h->t.Q) (void)hipFree(h->t.Q);
  if (h->t.bond) (void)hipFree(h->t.bond);
  if (h->t.qrk) (void)hipFree(h->t.qrk);
  if (h->t.plaq) (void)hipFree(h->t.plaq);
  if (h->t.elec) (void)hipFree(h->t.elec);
  h->t = DeviceTables{};
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  hipError_t e = hipMalloc((void**)dst, std::max<size_t>(1, src.size()) * sizeof(T));
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

bool ws_ok(const void* ws, size_t have, size_t need) { return need == 0 || (ws && have >= need); }

// Bracket one launch with events when profiling (events on the launch's own stream).
template <class F>
hipError_t timed(peps_handle* h, int family, hipStream_t s, F&& launch) {
  if (!h->profiling) return launch();
  peps_handle::Rec r{family, nullptr, nullptr};
  hipError_t e = hipEventCreate(&r.a);
  if (e == hipSuccess) e = hipEventCreate(&r.b);
  if (e == hipSuccess) e = hipEventRecord(r.a, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(r.b, s);
  if (e == hipSuccess) {
    h->recs.push_back(r);
  } else {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  return e;
}

// Upload the static tables to the current device on first use (so a handle can be created and
// queried on a host without a GPU).  A handle is bound to the device of its first launch.
int ensure_device(peps_handle* h) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return PEPS_ERR_HIP;
  if (h->device >= 0) return dev == h->device ? PEPS_OK : PEPS_ERR_ARG;
  if (upload(&h->t.site_offset, h->site_offset) != hipSuccess ||
      upload(&h->t.Q, h->Q) != hipSuccess || upload(&h->t.bond, h->bond) != hipSuccess ||
      upload(&h->t.qrk, h->qrk) != hipSuccess ||
      upload(&h->t.plaq, std::vector<double>(h->plaq_coef, h->plaq_coef + 8)) != hipSuccess ||
      upload(&h->t.elec, std::vector<double>(h->elec, h->elec + 8)) != hipSuccess) {
    free_tables(h);
    return PEPS_ERR_HIP;
  }
  h->device = dev;
  return PEPS_OK;
}

}  // namespace

namespace gipeps {

// Q-factor slot of one site in the row sweep (the kernel instantiation's MAXM * MAXN).
size_t qslot_doubles(const Dims& d) {
  const int mn = (d.Dk == 1 || d.maxN <= 32) ? 32 : (d.maxN <= kMaxN ? kMaxN : kMaxNBig);
  return (size_t)mn * d.Dk * mn;
}


CxWs cx_ws_layout(const peps_handle* h, int B, uint32_t what) {
  const Dims& d = h->d;
  const size_t Bz = (size_t)B, L = d.L, n = (size_t)h->n_params, P4 = d.P4, ns = d.n_sites;
  size_t S = 1;
  for (int i = 0; i < d.L; ++i) S *= d.Dk;
  const size_t W = S * d.Dk, cxb = 2 * sizeof(double), cxs = cx_elem_bytes(d);  // cxs: the contractions' states
  CxWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  w.states = take(cxs * Bz * 2 * (L + 1) * S);
  w.expo = take(sizeof(double) * Bz * 2 * (L + 1));
  w.gscr = take(cxs * Bz * L * W);
  w.wscr = take(cx_work_global(d) ? cxs * Bz * 2 * W : 0);
  w.base_end = off;
  if (what & PEPS_WS_SAMPLE) {
    w.lprop = take((size_t)d.planes * L * L * Bz);
    w.laprop = take(sizeof(double) * Bz);
    w.phprop = take(cxb * Bz);
    w.moved = take(Bz);
  }
  if (what & PEPS_WS_TVMC) {
    w.w = take(sizeof(double) * Bz);
    w.ov = take(cxb * Bz);
    w.sc = take(sizeof(double) * 64);
    w.ioff = take(sizeof(int32_t) * ns * (size_t)(d.N * d.N * d.N + 1));
    w.ilist = take(sizeof(int32_t) * ns * Bz);
    w.omean = take(cxb * n);
    w.g = take(cxb * n);
    w.y = take(cxb * n);
    w.r = take(cxb * n);
    w.p = take(cxb * n);
    w.q = take(cxb * n);
    w.proj = take(cxb * Bz * ns * P4);
    w.bid = take(sizeof(int32_t) * Bz * ns);
    w.valid = take(Bz);
    w.la = take(sizeof(double) * Bz);
    w.phase = take(cxb * Bz);
    w.O = take(cxb * Bz * ns * P4);
    w.eloc = take(cxb * Bz);
    w.xdot = take(cxb * n);
    w.theta1 = take(cxb * n);
  }
  w.total = off;
  return w;
}

WsLayout ws_layout(const peps_handle* h, int B, uint32_t what) {
  const Dims& d = h->d;
  const size_t Bz = (size_t)B;
  WsLayout w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  w.down = take(sizeof(double) * (size_t)(d.L - 1) * Bz * d.row_stride);
  w.lognu = take(sizeof(double) * Bz * d.L);
  w.qscr = take(sizeof(double) * Bz * d.L * qslot_doubles(d));
  w.wbig = take(d.maxN > kMaxN ? sizeof(double) * Bz * kBigSlot : 0);
  const size_t kept_rows = h->keep_tape ? (size_t)std::max(0, d.L - 2) : 0;
  w.qall = take(sizeof(double) * kept_rows * Bz * d.L * qslot_doubles(d));
  w.tall = take(sizeof(double) * kept_rows * Bz * d.L * tape_slot_doubles(d));
  w.venv = take(d.var_sweeps > 0 ? sizeof(double) * Bz * (size_t)(2 * (d.L + 1) + 2) * d.site_stride : 0);
  w.flag = take(64);
  w.status = take(sizeof(uint32_t) * Bz);
  w.escale = take(sizeof(double) * Bz);
  w.amp_end = off;
  w.up = take(sizeof(double) * (size_t)(d.L - 1) * Bz * d.row_stride);
  w.uplognu = take(sizeof(double) * Bz * d.L);
  w.fproj = take(sizeof(double) * Bz * d.n_sites * d.P4);
  w.strip = take(sizeof(double) * Bz * strip_scratch_doubles(d));
  w.part = take(sizeof(double) * Bz * (d.L - 1));
  w.pabs = take(sizeof(double) * Bz * (d.L - 1));
  w.energy_end = off;
  off = w.amp_end;  // the logderiv parts reuse the energy region
  w.tape = take(sizeof(double) * Bz * d.L * tape_slot_doubles(d));
  w.qbar = take(sizeof(double) * Bz * d.L * qslot_doubles(d));
  w.xbar = take(sizeof(double) * Bz * (d.maxN > kMaxN ? 2 * kMaxNBig : kMaxM));
  w.psibar = take(sizeof(double) * 2 * Bz * d.row_stride);
  w.rowtmp = take(sizeof(double) * Bz * d.row_stride);
  w.lognu2 = take(sizeof(double) * Bz * d.L);
  w.seg = take(sizeof(double) * (size_t)std::max(1, h->ckpt_every) * Bz * d.row_stride);
  w.sr = take(sizeof(double) * (Bz + 8));
  w.cg = take(sizeof(double) * (3 * (size_t)h->n_params + 2 * (size_t)(kMaxCgIter + 2)));
  w.logderiv_end = off;
  off = w.amp_end;  // the sampler's parts reuse the energy region too
  w.lprop = take((size_t)d.planes * d.L * d.L * Bz);
  w.laprop = take(sizeof(double) * Bz);
  w.sgprop = take(sizeof(double) * Bz);
  w.moved = take(Bz);
  w.sample_end = off;
  w.total = w.amp_end;
  if (what & PEPS_WS_ENERGY) w.total = std::max(w.total, w.energy_end);
  if (what & PEPS_WS_LOGDERIV) w.total = std::max(w.total, w.logderiv_end);
  if (what & PEPS_WS_SAMPLE) w.total = std::max(w.total, w.sample_end);
  return w;
}

}  // namespace gipeps

extern "C" {

const char* peps_status_string(int status) {
  switch (status) {
    case PEPS_OK: return "ok";
    case PEPS_ERR_ARG: return "invalid argument (null pointer, negative size or value out of range)";
    case PEPS_ERR_UNSUPPORTED: return "problem outside the shapes the library supports";
    case PEPS_ERR_WORKSPACE: return "workspace missing or too small";
    case PEPS_ERR_HIP: return "HIP runtime error or kernel launch failure";
    case PEPS_ERR_STATE: return "call order: run peps_amplitude on this batch and workspace first";
    default: return "unknown status";
  }
}

int peps_create(const peps_problem* p, peps_handle** out) {
  if (!p || !out) return PEPS_ERR_ARG;
  *out = nullptr;
  if (p->L < 2 || p->N < 2 || p->N > 8 || p->chi < 1) return PEPS_ERR_ARG;
  if (p->dtype != PEPS_F64 && p->dtype != PEPS_F32_MIXED && p->dtype != PEPS_C128_EXACT && p->dtype != PEPS_C64_EXACT)
    return PEPS_ERR_ARG;
  const bool cplx = is_cx(p->dtype);
  if (p->ckpt_every < 0 || (p->keep_tape != 0 && p->keep_tape != 1)) return PEPS_ERR_ARG;
  if (p->keep_tape && p->ckpt_every > 1) return PEPS_ERR_ARG;
  if (p->max_sweeps < 0 || p->max_sweeps > 1000) return PEPS_ERR_ARG;
  for (int k = 0; k < p->N; ++k)
    if (p->deg[k] < 1) return PEPS_ERR_ARG;
  for (int k = 1; k < p->N; ++k) {
    if (!std::isfinite(p->plaq_coef[k])) return PEPS_ERR_ARG;
    if (p->plaq_coef[k] != p->plaq_coef[p->N - k]) return PEPS_ERR_ARG;  // Hermitian H_B
  }
  for (int n = 0; n < p->N; ++n)
    if (!std::isfinite(p->elec[n])) return PEPS_ERR_ARG;
  if (p->matter != 0 && p->matter != 1) return PEPS_ERR_ARG;
  if (p->var_sweeps < 0 || p->var_sweeps > 100) return PEPS_ERR_ARG;
  if (p->var_sweeps > 0 && (p->keep_tape || is_cx(p->dtype))) return PEPS_ERR_UNSUPPORTED;
  if (!std::isfinite(p->hop) || !std::isfinite(p->mass)) return PEPS_ERR_ARG;
  if (!p->matter && (p->hop != 0.0 || p->mass != 0.0)) return PEPS_ERR_ARG;  // no matter to act on
  if (p->L > 64) return PEPS_ERR_UNSUPPORTED;
  for (int k = 1; k < p->N; ++k)
    if (p->deg[k] != p->deg[0]) return PEPS_ERR_UNSUPPORTED;
  if (!cplx && p->deg[0] > kMaxDk) return PEPS_ERR_UNSUPPORTED;
  if (cplx) {  // exact contraction in the full row space: Dk^(L+1) working entries per sample
    int64_t w = 1;
    for (int i = 0; i <= p->L && w <= kCxMaxWorkGlobal; ++i) w *= p->deg[0];
    if (p->deg[0] > 3 || w > kCxMaxWorkGlobal || p->matter || p->keep_tape) return PEPS_ERR_UNSUPPORTED;
  }

  peps_handle* h = new (std::nothrow) peps_handle();
  if (!h) return PEPS_ERR_ARG;
  h->d.L = p->L;
  h->d.N = p->N;
  h->d.Dk = p->deg[0];
  h->d.chi = p->chi;
  h->d.n_sites = p->L * p->L;
  h->d.P4 = h->d.Dk * h->d.Dk * h->d.Dk * h->d.Dk;
  h->dtype = p->dtype;
  h->d.mixed = p->dtype == PEPS_F32_MIXED ? 1 : 0;
  h->d.cx32 = p->dtype == PEPS_C64_EXACT ? 1 : 0;
  h->d.max_sweeps = p->max_sweeps > 0 ? p->max_sweeps : 40;
  // default tuning (measured fastest at Z3 16x16, chi = 36; peps_autotune / peps_set_tuning change it)
  h->d.jacobi_lanes = 8;
  h->d.down_precond = PEPS_PRECOND_SORTED_QR;
  h->d.up_precond = PEPS_PRECOND_QR_T;
  h->d.precond_min = 16;
  h->d.small_waves = 2;
  h->d.matter = p->matter;
  h->d.var_sweeps = p->var_sweeps;
  h->d.planes = p->matter ? 3 : 2;
  h->hop = p->hop;
  h->mass = p->mass;
  h->ckpt_every = p->ckpt_every;
  h->keep_tape = p->keep_tape != 0;
  for (int i = 0; i < 8; ++i) {
    h->plaq_coef[i] = (i < p->N) ? p->plaq_coef[i] : 0.0;
    h->elec[i] = (i < p->N) ? p->elec[i] : 0.0;
  }
  build_bonds(h);
  const int bmax = *std::max_element(h->bond.begin(), h->bond.end());
  h->d.site_stride = bmax * h->d.Dk * bmax;
  h->d.row_stride = p->L * h->d.site_stride;
  // fused bonds up to kMaxN on every path; up to kMaxNBig (D_k = 2) for the amplitude alone,
  // without a stored tape or variational compression
  if (!cplx && h->d.maxN > kMaxN &&
      (h->d.maxN > kMaxNBig || h->d.Dk != 2 || p->keep_tape || p->var_sweeps > 0)) {
    delete h;
    return PEPS_ERR_UNSUPPORTED;
  }
  // layout: a site with n present legs holds N^(n-1) blocks of Dk^n entries per occupation p
  // (eq. A): p = 0 only, or p = 0 then p = 1 with matter
  const int L = p->L, N = p->N, Dk = h->d.Dk;
  h->site_offset.assign((size_t)L * L + 1, 0);
  h->Q.assign((size_t)L * L, 0);
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      const int n = (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1);
      int64_t blocks = p->matter ? 2 : 1, size = 1;
      for (int i = 0; i < n - 1; ++i) blocks *= N;
      for (int i = 0; i < n; ++i) size *= Dk;
      const int s = y * L + x;
      h->site_offset[s + 1] = h->site_offset[s] + blocks * size;
      int q = p->Q ? (int)p->Q[s] : 0;
      q %= N;
      if (q < 0) q += N;
      h->Q[s] = (int8_t)q;
    }
  h->n_params = h->site_offset.back();
  h->device = -1;
  // With a GPU present the tables go to the current device now, so that no later call has to
  // allocate (peps_amplitude_noalloc relies on it); on a host without one they are built by the
  // first call that launches work.
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    if (int st = ensure_device(h)) {
      delete h;
      return st;
    }
  } else {
    (void)hipGetLastError();  // clear the no-device status
  }
  *out = h;
  return PEPS_OK;
}

int peps_destroy(peps_handle* h) {
  if (!h) return PEPS_ERR_ARG;
  for (auto& r : h->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  free_tables(h);
  delete h;
  return PEPS_OK;
}

int peps_param_layout(const peps_handle* h, int64_t* n_params, int64_t* site_offset) {
  if (!h || !n_params) return PEPS_ERR_ARG;
  *n_params = h->n_params;
  if (site_offset) std::memcpy(site_offset, h->site_offset.data(), h->site_offset.size() * sizeof(int64_t));
  return PEPS_OK;
}

int peps_workspace_bytes(const peps_handle* h, int32_t B, uint32_t what, size_t* bytes) {
  if (!h || !bytes || B < 0) return PEPS_ERR_ARG;
  if (what & ~uint32_t(PEPS_WS_AMPLITUDE | PEPS_WS_ENERGY | PEPS_WS_LOGDERIV | PEPS_WS_SAMPLE | PEPS_WS_TVMC))
    return PEPS_ERR_ARG;
  if (is_cx(h->dtype)) {
    *bytes = (B == 0 || what == 0) ? 0 : cx_ws_layout(h, B, what).total;
    return PEPS_OK;
  }
  if (what & PEPS_WS_TVMC) return PEPS_ERR_ARG;  // the tVMC buffers belong to complex handles
  *bytes = (B == 0 || what == 0) ? 0 : ws_layout(h, B, what).total;
  return PEPS_OK;
}

int peps_links_from_powers(peps_handle* h, const uint8_t* powers, int32_t B, uint8_t* links,
                           void* stream) {
  if (!h || B < 0 || (B > 0 && (!powers || !links))) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  if (int st = ensure_device(h)) return st;
  return hip_status(launch_links_from_powers(h->d, powers, B, links, (hipStream_t)stream));
}

int peps_matter_links(peps_handle* h, const uint8_t* powers, const uint8_t* occupations, int32_t B,
                      uint8_t* links, void* stream) {
  if (!h || B < 0 || (B > 0 && (!powers || !occupations || !links))) return PEPS_ERR_ARG;
  if (!h->d.matter) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  if (int st = ensure_device(h)) return st;
  return hip_status(launch_matter_links(h->d, h->t, powers, occupations, B, links, (hipStream_t)stream));
}

int peps_sample_init(peps_handle* h, uint64_t seed, uint64_t stream_id, int32_t B, uint8_t* powers,
                     uint8_t* links, void* stream) {
  if (!h || B < 0 || (B > 0 && (!powers || !links))) return PEPS_ERR_ARG;
  if (h->d.matter) return PEPS_ERR_UNSUPPORTED;  // matter chains start from peps_matter_links
  if (B == 0) return PEPS_OK;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_sample_powers(h->d, seed, stream_id, B, powers, s);
  if (e == hipSuccess) e = launch_links_from_powers(h->d, powers, B, links, s);
  return hip_status(e);
}

int peps_project(peps_handle* h, const double* theta, const uint8_t* links, int32_t B,
                 double* proj, int32_t* block_id, uint8_t* valid, void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || (B > 0 && (!theta || !links || !proj || !block_id || !valid)))
    return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  return hip_status(timed(h, PEPS_K_PROJECT, s, [&] {
    return launch_project(h->d, h->t, theta, links, B, proj, block_id, valid, s);
  }));
}

int peps_amplitude(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B,
                   double* log_abs, double* sign, void* ws, size_t ws_bytes, void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || (B > 0 && (!proj || !valid || !log_abs || !sign))) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const WsLayout w = ws_layout(h, B, PEPS_WS_AMPLITUDE);
  if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  const Dims& d = h->d;
  char* base = (char*)ws;
  double* down = (double*)(base + w.down);
  double* lognu = (double*)(base + w.lognu);
  double* qscr = (double*)(base + w.qscr);
  const size_t rs = (size_t)B * d.row_stride;
  // keep_tape: row y's Q factors and tape go to slot y-1 of the kept region
  const size_t qrow = (size_t)B * d.L * qslot_doubles(d), trow = (size_t)B * d.L * tape_slot_doubles(d);
  double* qall = (double*)(base + w.qall);
  double* tall = (double*)(base + w.tall);
  uint32_t* status = (uint32_t*)(base + w.status);
  hipError_t e = launch_fill_u32(status, (size_t)B, 0u, s);
  if (e == hipSuccess) e = launch_row0_to_mps(d, proj, valid, B, down, s);
  for (int y = 1; y <= d.L - 2 && e == hipSuccess; ++y)
    e = timed(h, PEPS_K_ROW_SWEEP, s, [&] {
      hipError_t r = launch_row_sweep(d, h->t, y, proj, valid, B, down + (size_t)(y - 1) * rs,
                                      down + (size_t)y * rs,
                                      h->keep_tape ? qall + (size_t)(y - 1) * qrow : qscr, lognu,
                                      h->keep_tape ? tall + (size_t)(y - 1) * trow : nullptr, s,
                                      /*up=*/false, status, (double*)(base + w.wbig));
      if (r == hipSuccess)
        r = launch_var_refine(d, h->t, y, proj, valid, B, down + (size_t)(y - 1) * rs, down + (size_t)y * rs,
                              (double*)(base + w.venv), lognu, s);
      return r;
    });
  if (e == hipSuccess)
    e = timed(h, PEPS_K_CLOSE, s, [&] {
      return launch_close(d, h->t.bond + (size_t)(d.L - 2) * (d.L + 1), proj, valid, B,
                          down + (size_t)(d.L - 2) * rs, lognu, log_abs, sign, s);
    });
  if (e == hipSuccess) {
    h->last_amp_ws = ws;
    h->last_amp_B = B;
  }
  h->last_energy_ws = nullptr;  // a new batch's boundaries: the stored E_loc scales are stale
  h->last_energy_B = -1;
  return hip_status(e);
}

int peps_amplitude_ragged(int32_t n, peps_handle* const* hs, const double* const* proj,
                          const uint8_t* const* valid, const int32_t* B, double* const* log_abs,
                          double* const* sign, void* const* ws, const size_t* ws_bytes, void* stream) {
  if (n < 1 || n > kMaxRagged || !hs || !proj || !valid || !B || !log_abs || !sign || !ws || !ws_bytes)
    return PEPS_ERR_ARG;
  int max_n = 1, max_L = 0;
  bool any_big = false, all_big = true;
  for (int i = 0; i < n; ++i) {
    peps_handle* h = hs[i];
    if (!h || B[i] < 0 || is_cx(h->dtype)) return PEPS_ERR_ARG;
    if (B[i] > 0 && (!proj[i] || !valid[i] || !log_abs[i] || !sign[i])) return PEPS_ERR_ARG;
    if (h->dtype != hs[0]->dtype) return PEPS_ERR_ARG;  // one arithmetic per launch
    // one instantiation for every group: D_k = 2, no stored tape or fitting sweeps, and the
    // large-bond slots either in every workspace or in none
    if (h->d.Dk != 2 || h->keep_tape || h->d.var_sweeps > 0) return PEPS_ERR_UNSUPPORTED;
    const bool big = h->d.maxN > kMaxN;
    any_big |= big;
    all_big &= big;
    max_n = std::max(max_n, h->d.maxN);
    max_L = std::max(max_L, h->d.L);
  }
  if (any_big && !all_big) return PEPS_ERR_UNSUPPORTED;
  for (int i = 0; i < n; ++i) {
    if (B[i] == 0) continue;
    const WsLayout w = ws_layout(hs[i], B[i], PEPS_WS_AMPLITUDE);
    if (!ws_ok(ws[i], ws_bytes[i], w.total)) return PEPS_ERR_WORKSPACE;
    if (int st = ensure_device(hs[i])) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    if (B[i] == 0) continue;
    const WsLayout w = ws_layout(hs[i], B[i], PEPS_WS_AMPLITUDE);
    char* base = (char*)ws[i];
    e = launch_fill_u32((uint32_t*)(base + w.status), (size_t)B[i], 0u, s);
    if (e == hipSuccess) e = launch_row0_to_mps(hs[i]->d, proj[i], valid[i], B[i], (double*)(base + w.down), s);
  }
  // row y of every lattice that has it, in one launch
  for (int y = 1; y <= max_L - 2 && e == hipSuccess; ++y) {
    RaggedRows r{};
    int blocks = 0;
    for (int i = 0; i < n; ++i) {
      const peps_handle* h = hs[i];
      if (B[i] == 0 || y > h->d.L - 2) continue;
      const WsLayout w = ws_layout(h, B[i], PEPS_WS_AMPLITUDE);
      char* base = (char*)ws[i];
      double* down = (double*)(base + w.down);
      const size_t rs = (size_t)B[i] * h->d.row_stride;
      RaggedRow& g = r.g[r.n++];
      g.d = h->d;
      g.bond = h->t.bond;
      g.qrk = h->t.qrk;
      g.proj = proj[i];
      g.valid = valid[i];
      g.prev_row = down + (size_t)(y - 1) * rs;
      g.out_row = down + (size_t)y * rs;
      g.qscr = (double*)(base + w.qscr);
      g.qslot = qslot_doubles(h->d);
      g.lognu = (double*)(base + w.lognu);
      g.status = (uint32_t*)(base + w.status);
      g.wbig = (double*)(base + w.wbig);
      g.first_block = blocks;
      blocks += B[i];
    }
    e = timed(hs[0], PEPS_K_ROW_SWEEP, s,
              [&] { return launch_row_sweep_ragged(r, blocks, y, 2, max_n, hs[0]->d, s); });
  }
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    if (B[i] == 0) continue;
    peps_handle* h = hs[i];
    const WsLayout w = ws_layout(h, B[i], PEPS_WS_AMPLITUDE);
    char* base = (char*)ws[i];
    const size_t rs = (size_t)B[i] * h->d.row_stride;
    e = launch_close(h->d, h->t.bond + (size_t)(h->d.L - 2) * (h->d.L + 1), proj[i], valid[i], B[i],
                     (double*)(base + w.down) + (size_t)(h->d.L - 2) * rs, (double*)(base + w.lognu), log_abs[i],
                     sign[i], s);
  }
  // each workspace now holds its lattice's rows, as after peps_amplitude on it (a handle listed
  // more than once keeps its last non-empty group)
  for (int i = 0; i < n; ++i) {
    hs[i]->last_amp_ws = nullptr;
    hs[i]->last_amp_B = -1;
    hs[i]->last_energy_ws = nullptr;
    hs[i]->last_energy_B = -1;
  }
  for (int i = 0; i < n && e == hipSuccess; ++i)
    if (B[i] > 0) {
      hs[i]->last_amp_ws = ws[i];
      hs[i]->last_amp_B = B[i];
    }
  return hip_status(e);
}

int peps_metropolis(peps_handle* h, const double* theta, uint64_t seed, uint64_t stream_id,
                    int32_t first_sweep, int32_t n_sweeps, int32_t B, uint8_t* links, double* log_abs,
                    int32_t* accepted, double* proj, int32_t* block_id, uint8_t* valid, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!h || B < 0 || n_sweeps < 0 || first_sweep < 0 ||
      (B > 0 && (!theta || !links || !log_abs || !proj || !block_id || !valid)))
    return PEPS_ERR_ARG;
  if (h->d.N < 2) return PEPS_ERR_UNSUPPORTED;
  if (B == 0) return PEPS_OK;
  // complex handles: the same chains with ln|Psi| of the exact complex amplitude
  const bool cplx = is_cx(h->dtype);
  size_t need = 0, o_lprop = 0, o_laprop = 0, o_sgprop = 0, o_moved = 0;
  if (cplx) {
    const CxWs w = cx_ws_layout(h, B, PEPS_WS_AMPLITUDE | PEPS_WS_SAMPLE);
    need = w.total;
    o_lprop = w.lprop;
    o_laprop = w.laprop;
    o_sgprop = w.phprop;
    o_moved = w.moved;
  } else {
    const WsLayout w = ws_layout(h, B, PEPS_WS_AMPLITUDE | PEPS_WS_SAMPLE);
    need = w.total;
    o_lprop = w.lprop;
    o_laprop = w.laprop;
    o_sgprop = w.sgprop;
    o_moved = w.moved;
  }
  if (!ws_ok(ws, ws_bytes, need)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  uint8_t* lprop = (uint8_t*)(base + o_lprop);
  double* laprop = (double*)(base + o_laprop);
  double* sgprop = (double*)(base + o_sgprop);  // sign (real) or phase (complex) of a proposal
  uint8_t* moved = (uint8_t*)(base + o_moved);
  int sw_cur = first_sweep;
  auto amplitude = [&](const uint8_t* lk, double* la) {
    if (cplx) {
      int r = peps_cx_project(h, theta, lk, B, proj, block_id, valid, stream);
      return r == PEPS_OK ? peps_cx_amplitude(h, proj, valid, B, la, sgprop, ws, ws_bytes, stream) : r;
    }
    int r = peps_project(h, theta, lk, B, proj, block_id, valid, stream);
    return r == PEPS_OK ? peps_amplitude(h, proj, valid, B, la, sgprop, ws, ws_bytes, stream) : r;
  };
  // ln|Psi| of the starting states, then one proposal per plaquette and sweep for every chain; with
  // matter each plaquette row is followed by the link moves of its strip, by window column
  int st = amplitude(links, log_abs);
  const int L = h->d.L;
  auto decide = [&](int p, const uint8_t* mv) {
    int r = amplitude(lprop, laprop);
    if (r == PEPS_OK)
      r = hip_status(launch_accept(h->d, p, sw_cur, seed, stream_id, B, mv, laprop, valid, lprop, log_abs,
                                   links, accepted, s));
    return r;
  };
  for (int sw = first_sweep; sw < first_sweep + n_sweeps && st == PEPS_OK; ++sw) {
    sw_cur = sw;
    for (int py = 0; py < L - 1 && st == PEPS_OK; ++py) {
      for (int px = 0; px < L - 1 && st == PEPS_OK; ++px) {
        const int p = py * (L - 1) + px;
        st = hip_status(launch_propose(h->d, p, sw, seed, stream_id, B, links, lprop, s));
        if (st == PEPS_OK) st = decide(p, nullptr);
      }
      for (int px = 0; px < L - 1 && h->d.matter && st == PEPS_OK; ++px)
        for (int m = 0; m < 4 && st == PEPS_OK; ++m) {
          int dir, x, y;
          if (m == 0) { dir = 1; x = px; y = py; }
          else if (m == 1) { dir = 0; x = px; y = py; }
          else if (m == 2) { if (py != L - 2) continue; dir = 0; x = px; y = L - 1; }
          else { if (px != L - 2) continue; dir = 1; x = L - 1; y = py; }
          const int link = dir == 0 ? y * (L - 1) + x : L * (L - 1) + y * L + x;
          st = hip_status(launch_propose_hop(h->d, dir, x, y, B, links, lprop, moved, s));
          if (st == PEPS_OK) st = decide((L - 1) * (L - 1) + link, moved);
        }
    }
  }
  // the boundary rows in ws belong to the last proposal, not to the returned states
  h->last_amp_ws = nullptr;
  h->last_amp_B = -1;
  return st;
}

int peps_metropolis_strip(peps_handle* h, const double* theta, uint64_t seed, uint64_t stream_id,
                          int32_t first_sweep, int32_t n_sweeps, int32_t B, uint8_t* links,
                          double* log_abs, int32_t* accepted, double* proj, int32_t* block_id,
                          uint8_t* valid, void* ws, size_t ws_bytes, void* stream) {
  if (!h || B < 0 || n_sweeps < 0 || first_sweep < 0 ||
      (B > 0 && (!theta || !links || !log_abs || !proj || !block_id || !valid)))
    return PEPS_ERR_ARG;
  if (is_cx(h->dtype)) {
    // complex handles: per sweep the row states of the current chains, then one strip-ratio sweep;
    // finally ln|Psi| (and the row states) of the final chains
    if (h->d.N < 2) return PEPS_ERR_UNSUPPORTED;
    if (B == 0) return PEPS_OK;
    const CxWs w = cx_ws_layout(h, B, PEPS_WS_AMPLITUDE | PEPS_WS_SAMPLE);
    if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
    if (int st = ensure_device(h)) return st;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    double* phase = (double*)(base + w.phprop);  // scratch for the states kernel's phases
    int st = PEPS_OK;
    for (int sw = first_sweep; sw < first_sweep + n_sweeps && st == PEPS_OK; ++sw) {
      st = peps_cx_project(h, theta, links, B, proj, block_id, valid, stream);
      if (st == PEPS_OK) st = peps_cx_amplitude(h, proj, valid, B, log_abs, phase, ws, ws_bytes, stream);
      if (st == PEPS_OK)
        st = hip_status(timed(h, PEPS_K_STRIP, s, [&] {
          return launch_cx_strip_mc(h->d, h->t, theta, links, valid, B, (double*)(base + w.states),
                                    (double*)(base + w.gscr), (double*)(base + w.wscr), seed, stream_id, sw,
                                    accepted, s);
        }));
    }
    if (st == PEPS_OK) st = peps_cx_project(h, theta, links, B, proj, block_id, valid, stream);
    if (st == PEPS_OK) st = peps_cx_amplitude(h, proj, valid, B, log_abs, phase, ws, ws_bytes, stream);
    return st;
  }
  if (B == 0) return PEPS_OK;
  const WsLayout w = ws_layout(h, B, PEPS_WS_AMPLITUDE | PEPS_WS_ENERGY);
  if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  const Dims& d = h->d;
  char* base = (char*)ws;
  double* down = (double*)(base + w.down);
  double* lognu = (double*)(base + w.lognu);
  double* up = (double*)(base + w.up);
  double* uplognu = (double*)(base + w.uplognu);
  double* fproj = (double*)(base + w.fproj);
  double* qscr = (double*)(base + w.qscr);
  double* strip = (double*)(base + w.strip);
  uint32_t* status = (uint32_t*)(base + w.status);
  double* wbig = (double*)(base + w.wbig);  // large bonds: working slots of the row sweeps and strips
  const size_t rs = (size_t)B * d.row_stride;
  const int L = d.L;
  // up boundary U_y lives in slot L-1-y of `up` (mirrored down boundary), D_y in slot y of `down`
  auto down_row = [&](int y) {  // D_y of the current configuration from D_{y-1}
    hipError_t r = launch_project(d, h->t, theta, links, B, proj, block_id, valid, s);
    if (r != hipSuccess) return r;
    if (y == 0) return launch_row0_to_mps(d, proj, valid, B, down, s);
    r = launch_row_sweep(d, h->t, y, proj, valid, B, down + (size_t)(y - 1) * rs, down + (size_t)y * rs, qscr,
                         lognu, nullptr, s, /*up=*/false, status, wbig);
    return r == hipSuccess ? launch_var_refine(d, h->t, y, proj, valid, B, down + (size_t)(y - 1) * rs,
                                               down + (size_t)y * rs, (double*)(base + w.venv), lognu, s)
                           : r;
  };
  auto up_row = [&](int y) {  // U_y of the current configuration from U_{y+1}
    const int yp = L - 1 - y;
    hipError_t r = launch_project(d, h->t, theta, links, B, proj, block_id, valid, s);
    if (r == hipSuccess) r = launch_mirror_proj(d, proj, valid, B, fproj, s);
    if (r != hipSuccess) return r;
    if (yp == 0) return launch_row0_to_mps(d, fproj, valid, B, up, s);
    r = launch_row_sweep(d, h->t, yp, fproj, valid, B, up + (size_t)(yp - 1) * rs, up + (size_t)yp * rs, qscr,
                         uplognu, nullptr, s, /*up=*/true, status, wbig);
    return r == hipSuccess ? launch_var_refine(d, h->t, yp, fproj, valid, B, up + (size_t)(yp - 1) * rs,
                                               up + (size_t)yp * rs, (double*)(base + w.venv), uplognu, s)
                           : r;
  };
  // the strip's plaquette moves, then (matter) its link moves against the updated strip
  auto strip_moves = [&](int py, int sw) {
    hipError_t r = launch_strip_mc(d, py, sw, seed, stream_id, h->t, theta, links, valid, B, down, up,
                                   strip, accepted, 0, s, wbig);
    if (r == hipSuccess && d.matter)
      r = launch_strip_mc(d, py, sw, seed, stream_id, h->t, theta, links, valid, B, down, up, strip,
                          accepted, 1, s, wbig);
    return r;
  };
  hipError_t e = launch_fill_u32(status, (size_t)B, 0u, s);
  // valid flags of the starting states (the strips skip invalid chains), also when no boundary row
  // is built before the first strip (L = 2)
  if (e == hipSuccess) e = launch_project(d, h->t, theta, links, B, proj, block_id, valid, s);
  // the boundaries on the far side of the first sweep's direction (odd sweeps go up)
  if (n_sweeps > 0 && e == hipSuccess) {
    if (first_sweep % 2 == 1)
      for (int y = L - 1; y >= 2 && e == hipSuccess; --y) e = up_row(y);
    else
      for (int y = 0; y <= L - 3 && e == hipSuccess; ++y) e = down_row(y);
  }
  for (int sw = first_sweep; sw < first_sweep + n_sweeps && e == hipSuccess; ++sw) {
    if (sw % 2 == 1) {
      // upwards: strip py between D_{py-1} (built in this pass) and U_{py+2} (rows not yet visited)
      for (int py = 0; py <= L - 2 && e == hipSuccess; ++py) {
        e = strip_moves(py, sw);
        if (e == hipSuccess && py <= L - 3) e = down_row(py);
      }
    } else {
      // downwards: strip py between U_{py+2} (built in this pass) and D_{py-1} (rows not yet visited)
      for (int py = L - 2; py >= 0 && e == hipSuccess; --py) {
        e = strip_moves(py, sw);
        if (e == hipSuccess && py >= 1) e = up_row(py + 1);
      }
    }
  }
  if (e != hipSuccess) return hip_status(e);
  // ln|Psi| of the final states; leaves the workspace in the state peps_amplitude leaves
  int st = peps_project(h, theta, links, B, proj, block_id, valid, stream);
  double* sg = (double*)(base + w.part);  // sign output parked in the energy region (unused here)
  if (st == PEPS_OK) st = peps_amplitude(h, proj, valid, B, log_abs, sg, ws, ws_bytes, stream);
  return st;
}

int peps_local_energy(peps_handle* h, const double* theta, const uint8_t* links,
                      const double* proj, const uint8_t* valid, int32_t B, double* e_loc,
                      void* ws, size_t ws_bytes, void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || (B > 0 && (!theta || !links || !proj || !valid || !e_loc))) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const WsLayout w = ws_layout(h, B, PEPS_WS_AMPLITUDE | PEPS_WS_ENERGY);
  if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
  if (h->last_amp_ws != ws || h->last_amp_B != B) return PEPS_ERR_STATE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  const Dims& d = h->d;
  char* base = (char*)ws;
  double* down = (double*)(base + w.down);
  double* up = (double*)(base + w.up);
  double* uplognu = (double*)(base + w.uplognu);
  double* fproj = (double*)(base + w.fproj);
  double* qscr = (double*)(base + w.qscr);
  double* strip = (double*)(base + w.strip);
  double* part = (double*)(base + w.part);
  double* pabs = (double*)(base + w.pabs);
  double* escale = (double*)(base + w.escale);
  double* wbig = (double*)(base + w.wbig);  // large bonds: working slots of the row sweep and strips
  const size_t rs = (size_t)B * d.row_stride;
  // up boundaries U_{L-1} .. U_2 = mirrored down boundaries D'_0 .. D'_{L-3}
  hipError_t e = launch_mirror_proj(d, proj, valid, B, fproj, s);
  if (e == hipSuccess && d.L >= 3) e = launch_row0_to_mps(d, fproj, valid, B, up, s);
  for (int yp = 1; yp <= d.L - 3 && e == hipSuccess; ++yp)
    e = timed(h, PEPS_K_ROW_SWEEP, s, [&] {
      hipError_t r = launch_row_sweep(d, h->t, yp, fproj, valid, B, up + (size_t)(yp - 1) * rs,
                                      up + (size_t)yp * rs, qscr, uplognu, nullptr, s, /*up=*/true,
                                      (uint32_t*)(base + w.status), wbig);
      if (r == hipSuccess)
        r = launch_var_refine(d, h->t, yp, fproj, valid, B, up + (size_t)(yp - 1) * rs, up + (size_t)yp * rs,
                              (double*)(base + w.venv), uplognu, s);
      return r;
    });
  for (int py = 0; py <= d.L - 2 && e == hipSuccess; ++py)
    e = timed(h, PEPS_K_STRIP, s, [&] {
      return launch_strip(d, py, h->t, proj, theta, links, valid, B, down, up, h->t.plaq, h->hop, strip,
                          part, pabs, s, wbig);
    });
  if (e == hipSuccess)
    e = launch_eloc_final(d, links, valid, B, h->t.elec, h->mass, part, pabs, e_loc, escale, s);
  if (e == hipSuccess) {
    h->last_energy_ws = ws;
    h->last_energy_B = B;
  }
  return hip_status(e);
}

int peps_eloc_scale(peps_handle* h, int32_t B, const void* ws, size_t ws_bytes, double* scale,
                    void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || (B > 0 && !scale)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const WsLayout w = ws_layout(h, B, PEPS_WS_AMPLITUDE);
  if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
  if (h->last_energy_ws != ws || h->last_energy_B != B) return PEPS_ERR_STATE;
  if (int st = ensure_device(h)) return st;
  return hip_status(hipMemcpyAsync(scale, (const char*)ws + w.escale, sizeof(double) * (size_t)B,
                                   hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

int peps_logderiv(peps_handle* h, const double* proj, const int32_t* block_id,
                  const uint8_t* valid, int32_t B, const double* w, double* O, double* vjp,
                  void* ws, size_t ws_bytes, void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || (B > 0 && (!proj || !block_id || !valid))) return PEPS_ERR_ARG;
  if (B > 0 && !O) return PEPS_ERR_ARG;  // O is the kernels' output buffer, also when only vjp is wanted
  if (h->d.var_sweeps > 0) return PEPS_ERR_UNSUPPORTED;  // no adjoint of the fitting sweeps
  if (B == 0) return PEPS_OK;
  const WsLayout wl = ws_layout(h, B, PEPS_WS_AMPLITUDE | PEPS_WS_LOGDERIV);
  if (!ws_ok(ws, ws_bytes, wl.total)) return PEPS_ERR_WORKSPACE;
  if (h->last_amp_ws != ws || h->last_amp_B != B) return PEPS_ERR_STATE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  const Dims& d = h->d;
  char* base = (char*)ws;
  uint32_t* status = (uint32_t*)(base + wl.status);
  double* down = (double*)(base + wl.down);
  double* qscr = (double*)(base + wl.qscr);
  double* tape = (double*)(base + wl.tape);
  double* qbar = (double*)(base + wl.qbar);
  double* xbar = (double*)(base + wl.xbar);
  double* psibar = (double*)(base + wl.psibar);
  double* rowtmp = (double*)(base + wl.rowtmp);
  double* lognu2 = (double*)(base + wl.lognu2);
  double* seg = (double*)(base + wl.seg);
  double* wbig = (double*)(base + wl.wbig);  // large bonds: working slots, shared by the kernels in turn
  const size_t rs = (size_t)B * d.row_stride;
  // O doubles as the per-sample output; without a caller buffer it lives behind the tape
  double* Ob = O;
  if (!Ob) return PEPS_ERR_ARG;  // vjp is formed from O, so O is required
  const int L = d.L, k = h->ckpt_every;
  hipError_t e = launch_fill(Ob, (size_t)B * d.n_sites * d.P4, 0.0, s);
  int cur = 0;
  if (e == hipSuccess)
    e = timed(h, PEPS_K_ADJOINT, s, [&] {
      return launch_adj_close(d, h->t.bond + (size_t)(L - 2) * (L + 1), proj, valid, B,
                              down + (size_t)(L - 2) * rs, psibar, Ob, s);
    });
  // boundary row y-1 for the reverse step of row y: stored (k = 0) or recomputed from the
  // checkpoint at the start of its segment (rows c0 = multiple of k are the checkpoints)
  int seg_base = -1;
  auto row_in = [&](int r) -> double* {
    if (k <= 1 || r % k == 0) return down + (size_t)r * rs;
    const int c0 = (r / k) * k;
    if (seg_base != c0) {
      for (int q = c0 + 1; q < std::min(c0 + k, L - 1) && e == hipSuccess; ++q) {
        const double* prev = (q - 1 == c0) ? down + (size_t)c0 * rs : seg + (size_t)(q - 1 - c0) * rs;
        e = launch_row_sweep(d, h->t, q, proj, valid, B, prev, seg + (size_t)(q - c0) * rs, qscr,
                             lognu2, nullptr, s, /*up=*/false, status, wbig);
      }
      seg_base = c0;
    }
    return seg + (size_t)(r - c0) * rs;
  };
  const size_t qrow = (size_t)B * L * qslot_doubles(d), trow = (size_t)B * L * tape_slot_doubles(d);
  for (int y = L - 2; y >= 1 && e == hipSuccess; --y) {
    double* prev = row_in(y - 1);
    if (e != hipSuccess) break;
    // the row's factorisations: stored by peps_amplitude (keep_tape), else recomputed here
    double* rowout = rowtmp;
    double* rq = qscr;
    double* rt = tape;
    if (h->keep_tape) {
      rowout = down + (size_t)y * rs;
      rq = (double*)(base + wl.qall) + (size_t)(y - 1) * qrow;
      rt = (double*)(base + wl.tall) + (size_t)(y - 1) * trow;
    } else {
      e = timed(h, PEPS_K_ROW_SWEEP, s, [&] {
        return launch_row_sweep(d, h->t, y, proj, valid, B, prev, rowtmp, qscr, lognu2, tape, s,
                                /*up=*/false, status, wbig);
      });
    }
    if (e == hipSuccess)
      e = timed(h, PEPS_K_ADJOINT, s, [&] {
        return launch_adj_row(d, h->t, y, proj, valid, B, prev, rowout, rt, rq,
                              psibar + (size_t)cur * rs, qbar, xbar,
                              psibar + (size_t)(1 - cur) * rs, Ob, s, wbig);
      });
    cur = 1 - cur;
  }
  if (e == hipSuccess) e = launch_adj_row0(d, valid, B, psibar + (size_t)cur * rs, Ob, s);
  if (e == hipSuccess && vjp) e = launch_vjp(d, h->t, block_id, valid, w, Ob, B, vjp, s);
  return hip_status(e);
}

int sr_build(peps_handle* h, const double* O, const int32_t* block_id, const uint8_t* valid,
             const double* e_loc, int32_t B, int32_t mode, const double* v, double* F,
             double* O_mean, double* S_or_Sv, void* ws, size_t ws_bytes, void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || (mode != SR_MATVEC && mode != SR_DENSE)) return PEPS_ERR_ARG;
  if (B > 0 && (!O || !block_id || !valid || !e_loc || !F || !O_mean || !S_or_Sv)) return PEPS_ERR_ARG;
  if (B > 0 && mode == SR_MATVEC && !v) return PEPS_ERR_ARG;
  if (mode == SR_DENSE && h->n_params > 8192) return PEPS_ERR_UNSUPPORTED;
  if (B == 0) return PEPS_OK;
  const WsLayout wl = ws_layout(h, B, PEPS_WS_LOGDERIV);
  if (!ws_ok(ws, ws_bytes, wl.sr + sizeof(double) * ((size_t)B + 8))) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  double* ov = (double*)((char*)ws + wl.sr);
  double* omv = ov + B;
  return hip_status(timed(h, PEPS_K_SR, s, [&] {
    return launch_sr(h->d, h->t, h->n_params, block_id, valid, O, e_loc, B, mode, v, F, O_mean,
                     S_or_Sv, ov, omv, s);
  }));
}

int sr_dense_rows(peps_handle* h, const double* O, const int32_t* block_id, const uint8_t* valid,
                  int32_t B, const double* O_mean, int64_t row0, int64_t nrows, double* S_rows,
                  void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || row0 < 0 || nrows < 0 || row0 + nrows > h->n_params) return PEPS_ERR_ARG;
  if (nrows > 0x7fffffff) return PEPS_ERR_ARG;
  if (B > 0 && nrows > 0 && (!O || !block_id || !valid || !O_mean || !S_rows)) return PEPS_ERR_ARG;
  if (B == 0 || nrows == 0) return PEPS_OK;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  return hip_status(timed(h, PEPS_K_SR, s, [&] {
    return launch_sr_rows(h->d, h->t, h->n_params, block_id, valid, O, O_mean, B, row0, nrows, S_rows, s);
  }));
}

int peps_flags(peps_handle* h, int32_t B, const void* ws, size_t ws_bytes, uint32_t* flags,
               void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || (B > 0 && !flags)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const WsLayout w = ws_layout(h, B, PEPS_WS_AMPLITUDE);
  if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  return hip_status(hipMemcpyAsync(flags, (const char*)ws + w.status, sizeof(uint32_t) * (size_t)B,
                                   hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

int sr_solve(peps_handle* h, const double* O, const int32_t* block_id, const uint8_t* valid,
             const double* e_loc, int32_t B, double shift, int32_t max_iter, double rtol, double* x,
             double* F, double* O_mean, int32_t* iterations, double* rel_residual, void* ws,
             size_t ws_bytes, void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || B < 0 || max_iter < 0 || max_iter > kMaxCgIter || !(shift >= 0.0) || !(rtol >= 0.0))
    return PEPS_ERR_ARG;
  if (B > 0 && (!O || !block_id || !valid || !e_loc || !x || !F || !O_mean)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const WsLayout wl = ws_layout(h, B, PEPS_WS_LOGDERIV);
  if (!ws_ok(ws, ws_bytes, wl.logderiv_end)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = h->n_params;
  double* ov = (double*)((char*)ws + wl.sr);
  double* omv = ov + B;
  double* r = (double*)((char*)ws + wl.cg);
  double* p = r + n;
  double* q = p + n;
  double* sc = q + n;
  auto matvec = [&](const double* v, double* out) {  // S v (F and <O> rewritten, same values)
    return timed(h, PEPS_K_SR, s, [&] {
      return launch_sr(h->d, h->t, n, block_id, valid, O, e_loc, B, SR_MATVEC, v, F, O_mean, out, ov,
                       omv, s);
    });
  };
  auto host = [&](const double* src, double* dst, int cnt) {
    hipError_t e = hipMemcpyAsync(dst, src, sizeof(double) * cnt, hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
  };
  // F and <O>: written by every S v pass (here with v = 0 into the scratch p)
  hipError_t e = launch_fill(q, (size_t)n, 0.0, s);
  if (e == hipSuccess) e = matvec(q, p);
  if (e == hipSuccess) e = launch_cg(kCgInit, n, x, r, p, q, F, sc, 0, shift, s);
  if (e == hipSuccess) e = launch_cg(kCgDotRR, n, x, r, p, q, F, sc, 0, shift, s);
  double f2 = 0.0, rr = 0.0;
  if (e == hipSuccess) e = host(sc, &f2, 1);
  rr = f2;
  int k = 0;
  while (e == hipSuccess && f2 > 0.0 && k < max_iter && rr > rtol * rtol * f2) {
    e = matvec(p, q);
    if (e == hipSuccess) e = launch_cg(kCgShift, n, x, r, p, q, F, sc, k, shift, s);
    if (e == hipSuccess) e = launch_cg(kCgDotPQ, n, x, r, p, q, F, sc, k, shift, s);
    if (e == hipSuccess) e = launch_cg(kCgStep, n, x, r, p, q, F, sc, k, shift, s);
    if (e == hipSuccess) e = launch_cg(kCgDotRR, n, x, r, p, q, F, sc, k + 1, shift, s);
    double two[2] = {0.0, 0.0};  // p.q, then r.r after the step
    if (e == hipSuccess) e = host(sc + 2 * k + 1, two, 2);
    if (e != hipSuccess || !(two[0] > 0.0)) break;  // breakdown: x and r were left unchanged
    rr = two[1];
    ++k;
    if (rr <= rtol * rtol * f2) break;
    e = launch_cg(kCgDir, n, x, r, p, q, F, sc, k - 1, shift, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (iterations) *iterations = k;
  if (rel_residual) *rel_residual = f2 > 0.0 ? std::sqrt(rr / f2) : 0.0;
  return hip_status(e);
}

// ---------------------------------------------------------------------------------------------
// Complex exact-contraction path and tVMC (k_complex.hip)

int peps_cx_project(peps_handle* h, const double* theta, const uint8_t* links, int32_t B, double* proj,
                    int32_t* block_id, uint8_t* valid, void* stream) {
  if (!h || B < 0 || (B > 0 && (!theta || !links || !proj || !block_id || !valid))) return PEPS_ERR_ARG;
  if (!is_cx(h->dtype)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  return hip_status(timed(h, PEPS_K_PROJECT, s, [&] {
    return launch_cx_project(h->d, h->t, theta, links, B, proj, block_id, valid, s);
  }));
}

int peps_cx_amplitude(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B, double* log_abs,
                      double* phase, void* ws, size_t ws_bytes, void* stream) {
  if (!h || B < 0 || (B > 0 && (!proj || !valid || !log_abs || !phase))) return PEPS_ERR_ARG;
  if (!is_cx(h->dtype)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const CxWs w = cx_ws_layout(h, B, PEPS_WS_AMPLITUDE);
  if (!ws_ok(ws, ws_bytes, w.base_end)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  hipError_t e = timed(h, PEPS_K_ROW_SWEEP, s, [&] {
    return launch_cx_states(h->d, proj, valid, B, (double*)(base + w.states), (double*)(base + w.expo), log_abs,
                            phase, (double*)(base + w.wscr), s);
  });
  h->last_amp_ws = e == hipSuccess ? ws : nullptr;
  h->last_amp_B = e == hipSuccess ? B : -1;
  return hip_status(e);
}

int peps_cx_local_energy(peps_handle* h, const double* theta, const uint8_t* links, const double* proj,
                         const uint8_t* valid, int32_t B, double* e_loc, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!h || B < 0 || (B > 0 && (!theta || !links || !proj || !valid || !e_loc))) return PEPS_ERR_ARG;
  if (!is_cx(h->dtype)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const CxWs w = cx_ws_layout(h, B, PEPS_WS_AMPLITUDE);
  if (!ws_ok(ws, ws_bytes, w.base_end)) return PEPS_ERR_WORKSPACE;
  if (h->last_amp_ws != ws || h->last_amp_B != B) return PEPS_ERR_STATE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  return hip_status(timed(h, PEPS_K_STRIP, s, [&] {
    return launch_cx_eloc(h->d, h->t, theta, links, proj, valid, B, (const double*)((char*)ws + w.states), e_loc,
                          (double*)((char*)ws + w.gscr), (double*)((char*)ws + w.wscr), s);
  }));
}

int peps_cx_logderiv(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B, double* O, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!h || B < 0 || (B > 0 && (!proj || !valid || !O))) return PEPS_ERR_ARG;
  if (!is_cx(h->dtype)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const CxWs w = cx_ws_layout(h, B, PEPS_WS_AMPLITUDE);
  if (!ws_ok(ws, ws_bytes, w.base_end)) return PEPS_ERR_WORKSPACE;
  if (h->last_amp_ws != ws || h->last_amp_B != B) return PEPS_ERR_STATE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  return hip_status(timed(h, PEPS_K_ADJOINT, s, [&] {
    return launch_cx_logderiv(h->d, proj, valid, B, (const double*)(base + w.states), (double*)(base + w.gscr), O,
                              (double*)(base + w.wscr), s);
  }));
}

namespace {
// tvmc_rhs on validated arguments (ws sized for PEPS_WS_TVMC)
int cx_rhs(peps_handle* h, const gipeps::CxWs& w, char* base, const double* O, const int32_t* bid,
           const uint8_t* valid, const double* e_loc, const double* log_abs, int B, int weights, double shift,
           int max_iter, double rtol, double* xdot, double* energy, int* iterations, double* rel_residual,
           hipStream_t s) {
  using namespace gipeps;
  const int64_t n = h->n_params;
  double* wt = (double*)(base + w.w);
  double* ov = (double*)(base + w.ov);
  double* sc = (double*)(base + w.sc);
  double* omean = (double*)(base + w.omean);
  double* g = (double*)(base + w.g);
  double* y = (double*)(base + w.y);
  double* r = (double*)(base + w.r);
  double* p = (double*)(base + w.p);
  double* q = (double*)(base + w.q);
  auto host = [&](const double* src, double* dst, int cnt) {
    hipError_t e = hipMemcpyAsync(dst, src, sizeof(double) * cnt, hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
  };
  int32_t* ioff = (int32_t*)(base + w.ioff);
  int32_t* ilist = (int32_t*)(base + w.ilist);
  hipError_t e = launch_cx_weights(B, weights, log_abs, valid, wt, s);
  if (e == hipSuccess) e = launch_cx_index(h->d, B, bid, wt, ioff, ilist, s);
  if (e == hipSuccess)
    e = timed(h, PEPS_K_SR, s, [&] {
      return launch_cx_force(h->d, h->t, n, B, ioff, ilist, wt, O, e_loc, sc, omean, g, s);
    });
  double em[2] = {0.0, 0.0};
  if (e == hipSuccess) e = host(sc, em, 2);
  if (energy) {
    energy[0] = em[0];
    energy[1] = em[1];
  }
  // conjugate gradients for (S + shift I) y = g from y = 0 (Hermitian inner products)
  if (e == hipSuccess) e = launch_fill(y, 2 * (size_t)n, 0.0, s);
  if (e == hipSuccess) e = hipMemcpyAsync(r, g, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p, g, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, s);
  double two[2] = {0.0, 0.0};
  if (e == hipSuccess) e = launch_cx_dot(n, r, r, sc + 4, s);
  if (e == hipSuccess) e = host(sc + 4, two, 2);
  const double f2 = two[0];
  double rr = f2;
  int k = 0;
  while (e == hipSuccess && f2 > 0.0 && k < max_iter && rr > rtol * rtol * f2) {
    e = timed(h, PEPS_K_SR, s, [&] {
      return launch_cx_matvec(h->d, h->t, n, B, bid, ioff, ilist, wt, O, omean, shift, p, ov, sc, q, s);
    });
    if (e == hipSuccess) e = launch_cx_dot(n, p, q, sc + 6, s);
    if (e == hipSuccess) e = host(sc + 6, two, 2);
    if (e != hipSuccess || !(two[0] > 0.0)) break;  // breakdown: y and r left unchanged
    const double alpha = rr / two[0];
    e = launch_cx_axpy(n, alpha, 0.0, p, y, y, s);
    if (e == hipSuccess) e = launch_cx_axpy(n, -alpha, 0.0, q, r, r, s);
    if (e == hipSuccess) e = launch_cx_dot(n, r, r, sc + 8, s);
    if (e == hipSuccess) e = host(sc + 8, two, 2);
    if (e != hipSuccess) break;
    const double rr_new = two[0];
    ++k;
    if (rr_new <= rtol * rtol * f2) {
      rr = rr_new;
      break;
    }
    e = launch_cx_axpy(n, rr_new / rr, 0.0, p, r, p, s);  // p = r + beta p
    rr = rr_new;
  }
  // alphadot = -i y
  if (e == hipSuccess) e = launch_fill(xdot, 2 * (size_t)n, 0.0, s);
  if (e == hipSuccess) e = launch_cx_axpy(n, 0.0, -1.0, y, xdot, xdot, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (iterations) *iterations = k;
  if (rel_residual) *rel_residual = f2 > 0.0 ? std::sqrt(rr / f2) : 0.0;
  return hip_status(e);
}
}  // namespace

int tvmc_rhs(peps_handle* h, const double* O, const int32_t* block_id, const uint8_t* valid, const double* e_loc,
             const double* log_abs, int32_t B, int32_t weights, double shift, int32_t max_iter, double rtol,
             double* xdot, double* energy, int32_t* iterations, double* rel_residual, void* ws, size_t ws_bytes,
             void* stream) {
  if (!h || B < 0 || max_iter < 0 || max_iter > kMaxCgIter || !(shift >= 0.0) || !(rtol >= 0.0)) return PEPS_ERR_ARG;
  if (weights != TVMC_WEIGHT_UNIFORM && weights != TVMC_WEIGHT_PSI2) return PEPS_ERR_ARG;
  if (B > 0 && (!O || !block_id || !valid || !e_loc || !log_abs || !xdot)) return PEPS_ERR_ARG;
  if (!is_cx(h->dtype)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const CxWs w = cx_ws_layout(h, B, PEPS_WS_TVMC);
  if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  int it = 0;
  const int st = cx_rhs(h, w, (char*)ws, O, block_id, valid, e_loc, log_abs, B, weights, shift, max_iter, rtol, xdot,
                        energy, &it, rel_residual, (hipStream_t)stream);
  if (iterations) *iterations = it;
  return st;
}

int tvmc_step(peps_handle* h, double* theta, const uint8_t* links, int32_t B, int32_t weights, int32_t order,
              double dt, double shift, int32_t max_iter, double rtol, double* energy, int32_t* iterations,
              void* ws, size_t ws_bytes, void* stream) {
  if (!h || B < 0 || max_iter < 0 || max_iter > kMaxCgIter || !(shift >= 0.0) || !(rtol >= 0.0) ||
      !std::isfinite(dt) || (order != 1 && order != 2))
    return PEPS_ERR_ARG;
  if (weights != TVMC_WEIGHT_UNIFORM && weights != TVMC_WEIGHT_PSI2) return PEPS_ERR_ARG;
  if (B > 0 && (!theta || !links)) return PEPS_ERR_ARG;
  if (!is_cx(h->dtype)) return PEPS_ERR_ARG;
  if (B == 0) return PEPS_OK;
  const CxWs w = cx_ws_layout(h, B, PEPS_WS_TVMC);
  if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  double* proj = (double*)(base + w.proj);
  int32_t* bid = (int32_t*)(base + w.bid);
  uint8_t* valid = (uint8_t*)(base + w.valid);
  double* la = (double*)(base + w.la);
  double* phase = (double*)(base + w.phase);
  double* O = (double*)(base + w.O);
  double* eloc = (double*)(base + w.eloc);
  double* xdot = (double*)(base + w.xdot);
  double* theta1 = (double*)(base + w.theta1);
  const int64_t n = h->n_params;
  // alphadot at parameters th: projection, amplitude, O, E_loc, then the linear system
  auto velocity = [&](const double* th, double* en, int* it) {
    int st = peps_cx_project(h, th, links, B, proj, bid, valid, s);
    if (st == PEPS_OK) st = peps_cx_amplitude(h, proj, valid, B, la, phase, ws, ws_bytes, s);
    if (st == PEPS_OK) st = peps_cx_logderiv(h, proj, valid, B, O, ws, ws_bytes, s);
    if (st == PEPS_OK) st = peps_cx_local_energy(h, th, links, proj, valid, B, eloc, ws, ws_bytes, s);
    if (st == PEPS_OK)
      st = cx_rhs(h, w, base, O, bid, valid, eloc, la, B, weights, shift, max_iter, rtol, xdot, en, it, nullptr, s);
    return st;
  };
  int it[2] = {0, 0};
  double e0[2] = {0.0, 0.0};
  int st = velocity(theta, e0, &it[0]);
  if (order == 1) {
    if (st == PEPS_OK) st = hip_status(launch_cx_axpy(n, dt, 0.0, xdot, theta, theta, s));
  } else {
    // alpha_1 = alpha + c_1 dt alphadot, c_1 = (1 + i)/2; alpha <- alpha_1 + c_2 dt alphadot(alpha_1)
    if (st == PEPS_OK) st = hip_status(launch_cx_axpy(n, 0.5 * dt, 0.5 * dt, xdot, theta, theta1, s));
    if (st == PEPS_OK) st = velocity(theta1, nullptr, &it[1]);
    if (st == PEPS_OK) st = hip_status(launch_cx_axpy(n, 0.5 * dt, -0.5 * dt, xdot, theta1, theta, s));
  }
  if (st == PEPS_OK) st = hip_status(hipStreamSynchronize(s));
  if (energy) {
    energy[0] = e0[0];
    energy[1] = e0[1];
  }
  if (iterations) {
    iterations[0] = it[0];
    iterations[1] = it[1];
  }
  // the states in ws belong to alpha_1 (order 2) or to the old alpha: not to the new parameters
  h->last_amp_ws = nullptr;
  h->last_amp_B = -1;
  return st;
}

int peps_get_tuning(const peps_handle* h, peps_tuning* t) {
  if (!h || !t) return PEPS_ERR_ARG;
  t->jacobi_lanes = h->d.jacobi_lanes;
  t->down_precond = h->d.down_precond;
  t->up_precond = h->d.up_precond;
  t->precond_min = h->d.precond_min;
  t->small_waves = h->d.small_waves;
  return PEPS_OK;
}

namespace {
bool tuning_ok(const peps_tuning& t) {
  return (t.jacobi_lanes == 4 || t.jacobi_lanes == 8) &&
         (t.down_precond == PEPS_PRECOND_NONE || t.down_precond == PEPS_PRECOND_SORTED_QR) &&
         (t.up_precond == PEPS_PRECOND_NONE || t.up_precond == PEPS_PRECOND_QR_T ||
          t.up_precond == PEPS_PRECOND_SORTED_QR) &&
         t.precond_min >= 2 && t.precond_min <= 1024 && (t.small_waves == 2 || t.small_waves == 4);
}
void apply_tuning(peps_handle* h, const peps_tuning& t) {
  h->d.jacobi_lanes = t.jacobi_lanes;
  h->d.down_precond = t.down_precond;
  h->d.up_precond = t.up_precond;
  h->d.precond_min = t.precond_min;
  h->d.small_waves = t.small_waves;
  // boundary rows and tapes left in a workspace came from the previous tuning
  h->last_amp_ws = nullptr;
  h->last_amp_B = -1;
  h->last_energy_ws = nullptr;
  h->last_energy_B = -1;
}
}  // namespace

int peps_set_tuning(peps_handle* h, const peps_tuning* t) {
  if (!h || !t || !tuning_ok(*t)) return PEPS_ERR_ARG;
  apply_tuning(h, *t);
  return PEPS_OK;
}

int peps_autotune(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B, void* ws,
                  size_t ws_bytes, peps_tuning* best, peps_tune_result* results, int32_t capacity,
                  int32_t* count, void* stream) {
  if (h && is_cx(h->dtype)) return PEPS_ERR_ARG;  // complex handles: peps_cx_* / tvmc_*
  if (!h || !best || B <= 0 || !proj || !valid || capacity < 0 || (capacity > 0 && !results))
    return PEPS_ERR_ARG;
  const WsLayout w = ws_layout(h, B, PEPS_WS_AMPLITUDE | PEPS_WS_ENERGY);
  if (!ws_ok(ws, ws_bytes, w.total)) return PEPS_ERR_WORKSPACE;
  if (int st = ensure_device(h)) return st;
  hipStream_t s = (hipStream_t)stream;
  Dims& d = h->d;
  char* base = (char*)ws;
  double* wbig = (double*)(base + w.wbig);
  double* down = (double*)(base + w.down);
  double* lognu = (double*)(base + w.lognu);
  double* qscr = (double*)(base + w.qscr);
  double* up = (double*)(base + w.up);
  double* uplognu = (double*)(base + w.uplognu);
  double* fproj = (double*)(base + w.fproj);
  uint32_t* status = (uint32_t*)(base + w.status);
  const size_t rs = (size_t)B * d.row_stride;
  const size_t qrow = (size_t)B * d.L * qslot_doubles(d), trow = (size_t)B * d.L * tape_slot_doubles(d);
  // one down sweep as peps_amplitude runs it (taped when the handle keeps the tape), or the up
  // sweep of peps_local_energy
  auto sweep = [&](bool upward) {
    hipError_t e = hipSuccess;
    if (!upward) {
      e = launch_row0_to_mps(d, proj, valid, B, down, s);
      for (int y = 1; y <= d.L - 2 && e == hipSuccess; ++y)
        e = launch_row_sweep(d, h->t, y, proj, valid, B, down + (size_t)(y - 1) * rs, down + (size_t)y * rs,
                             h->keep_tape ? (double*)(base + w.qall) + (size_t)(y - 1) * qrow : qscr, lognu,
                             h->keep_tape ? (double*)(base + w.tall) + (size_t)(y - 1) * trow : nullptr, s,
                             /*up=*/false, status, wbig);
    } else {
      e = launch_mirror_proj(d, proj, valid, B, fproj, s);
      if (e == hipSuccess) e = launch_row0_to_mps(d, fproj, valid, B, up, s);
      for (int yp = 1; yp <= d.L - 3 && e == hipSuccess; ++yp)
        e = launch_row_sweep(d, h->t, yp, fproj, valid, B, up + (size_t)(yp - 1) * rs, up + (size_t)yp * rs,
                             qscr, uplognu, nullptr, s, /*up=*/true, status, wbig);
    }
    return e;
  };
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  auto timed_sweep = [&](bool upward, double* ms) {
    hipError_t r = hipEventRecord(ev[0], s);
    if (r == hipSuccess) r = sweep(upward);
    if (r == hipSuccess) r = hipEventRecord(ev[1], s);
    if (r == hipSuccess) r = hipEventSynchronize(ev[1]);
    float f = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&f, ev[0], ev[1]);
    *ms = f;
    return r;
  };
  const peps_tuning saved{d.jacobi_lanes, d.down_precond, d.up_precond, d.precond_min, d.small_waves};
  // warm-up of both directions (first launches of each kernel instantiation load it)
  double dummy = 0.0;
  if (e == hipSuccess) e = timed_sweep(false, &dummy);
  if (e == hipSuccess) e = timed_sweep(true, &dummy);
  // candidates: lanes {8, 4} x threshold {16, 32} (x waves per SIMD {2, 4} where the chi*Dk <= 32
  // kernels run); per combination the fastest down and up modes.  The large-bond kernel always runs
  // four lanes per column pair: there only the thresholds and modes are tried.
  const int lanes[2] = {8, 4}, thrs[2] = {16, 32}, waves[2] = {2, 4};
  const int nwaves = (d.Dk == 1 || d.maxN <= 32) ? 2 : 1;
  const int a0 = d.maxN > kMaxN ? 1 : 0;
  const int dmodes[2] = {PEPS_PRECOND_SORTED_QR, PEPS_PRECOND_NONE};
  const int umodes[3] = {PEPS_PRECOND_QR_T, PEPS_PRECOND_SORTED_QR, PEPS_PRECOND_NONE};
  int n = 0;
  double best_ms = 0.0;
  bool have_best = false;
  peps_tuning bt = saved;
  auto record = [&](int mode, int upward, double ms) {
    if (n < capacity)
      results[n] = peps_tune_result{d.jacobi_lanes, mode, d.precond_min, d.small_waves, upward, ms};
    ++n;
  };
  for (int a = a0; a < 2 && e == hipSuccess; ++a)
    for (int b = 0; b < 2 && e == hipSuccess; ++b)
      for (int c = 0; c < nwaves && e == hipSuccess; ++c) {
        d.jacobi_lanes = lanes[a];
        d.precond_min = thrs[b];
        d.small_waves = waves[c];
        double bd = 0.0, bu = 0.0;
        int md = dmodes[0], mu = umodes[0];
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
          d.down_precond = dmodes[i];
          double ms = 0.0;
          e = timed_sweep(false, &ms);
          record(dmodes[i], 0, ms);
          if (i == 0 || ms < bd) {
            bd = ms;
            md = dmodes[i];
          }
        }
        for (int i = 0; i < 3 && e == hipSuccess; ++i) {
          d.up_precond = umodes[i];
          double ms = 0.0;
          e = timed_sweep(true, &ms);
          record(umodes[i], 1, ms);
          if (i == 0 || ms < bu) {
            bu = ms;
            mu = umodes[i];
          }
        }
        if (e == hipSuccess && (!have_best || bd + bu < best_ms)) {
          have_best = true;
          best_ms = bd + bu;
          bt = peps_tuning{lanes[a], md, mu, thrs[b], waves[c]};
        }
      }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  apply_tuning(h, e == hipSuccess ? bt : saved);
  if (count) *count = n;
  if (e != hipSuccess) return PEPS_ERR_HIP;
  *best = bt;
  return PEPS_OK;
}

int peps_profile_enable(peps_handle* h, int32_t on) {
  if (!h) return PEPS_ERR_ARG;
  h->profiling = on != 0;
  return PEPS_OK;
}

int peps_profile_phases(peps_handle* h, uint64_t* counters) {
  if (!h) return PEPS_ERR_ARG;
  h->d.phase_clk = reinterpret_cast<unsigned long long*>(counters);
  return PEPS_OK;
}

int peps_profile_read(peps_handle* h, int32_t family, int64_t* launches, double* total_ms) {
  if (!h || !launches || !total_ms || family < 0 || family >= PEPS_K_COUNT) return PEPS_ERR_ARG;
  *launches = 0;
  *total_ms = 0.0;
  int st = PEPS_OK;
  std::vector<peps_handle::Rec> keep;
  for (auto& r : h->recs) {
    if (r.family != family) {
      keep.push_back(r);
      continue;
    }
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      st = PEPS_ERR_HIP;
    *launches += 1;
    *total_ms += ms;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  h->recs.swap(keep);
  return st;
}

}  // extern "C"
