// Stochastic-reconfiguration build over a batch (SM S-1 eq. gradient, read as the covariance
// <O E> - <O><E>; SM S-3 S_mn = <O_m O_n> - <O_m><O_n>; plain means over the valid samples).
//
// O arrives block-sparse: per sample and site only the selected block is nonzero, stored in the
// projected layout with its block index.  Every kernel here reduces over samples in index order
// (no atomics), so results are bitwise reproducible.
//   k_sr_site   : one workgroup per site: <O>, F, and (matvec mode) S v = <O (O v)> - <O> (<O> . v)
//   k_sr_ov     : (O v)_b per sample (gathers v through the block index)
//   k_sr_dot    : <O> . v (single workgroup)
//   k_sr_dense  : dense S for small parameter counts
//   k_sr_rows   : rows of the dense S for any parameter count (block-sparse scatter per sample)
#include "dev_common.h"
#include "internal.h"

namespace gipeps {

namespace {

struct SiteShape {
  int nb, bs;  // blocks and block size of the site
};

__device__ SiteShape site_shape(const Dims& d, int s) {
  const int x = s % d.L, y = s / d.L;
  const int np = (x > 0) + (x < d.L - 1) + (y > 0) + (y < d.L - 1);
  SiteShape r{1, 1};
  for (int i = 0; i < np; ++i) r.bs *= d.Dk;
  for (int i = 0; i < np - 1; ++i) r.nb *= d.N;
  return r;
}

// Number of valid samples and the mean local energy over them (every thread gets both).
__device__ void valid_stats(const uint8_t* valid, const double* e, int B, double* red, double* nv,
                            double* emean) {
  double c = 0.0, s = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x)
    if (valid[b]) {
      c += 1.0;
      s += e ? e[b] : 0.0;
    }
  *nv = block_sum(c, red);
  const double tot = block_sum(s, red);
  *emean = (*nv > 0.0) ? tot / *nv : 0.0;
}

}  // namespace

__global__ void k_sr_site(Dims d, const int64_t* __restrict__ site_offset,
                          const int32_t* __restrict__ block_id, const uint8_t* __restrict__ valid,
                          const double* __restrict__ O, const double* __restrict__ e_loc,
                          const double* __restrict__ ov, const double* __restrict__ omv, int B,
                          double* __restrict__ F, double* __restrict__ omean, double* __restrict__ Sv) {
  __shared__ double red[16];
  const int s = blockIdx.x;
  double nv, em;
  valid_stats(valid, e_loc, B, red, &nv, &em);
  const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
  const SiteShape sh = site_shape(d, s);
  for (int ent = threadIdx.x; ent < sh.nb * sh.bs; ent += blockDim.x) {
    const int blk = ent / sh.bs, e = ent % sh.bs;
    double so = 0.0, soe = 0.0, sov = 0.0;
    for (int b = 0; b < B; ++b) {
      if (!valid[b] || block_id[(size_t)b * d.n_sites + s] != blk) continue;
      const double o = O[((size_t)b * d.n_sites + s) * d.P4 + e];
      so += o;
      soe += o * e_loc[b];
      if (ov) sov += o * ov[b];
    }
    const double om = so * inv;
    const int64_t m = site_offset[s] + ent;
    omean[m] = om;
    F[m] = soe * inv - om * em;
    if (ov) Sv[m] = sov * inv - om * omv[0];
  }
}

__global__ void k_sr_ov(Dims d, const int64_t* __restrict__ site_offset,
                        const int32_t* __restrict__ block_id, const uint8_t* __restrict__ valid,
                        const double* __restrict__ O, const double* __restrict__ v,
                        double* __restrict__ ov) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  double acc = 0.0;
  if (valid[b]) {
    for (int idx = threadIdx.x; idx < d.n_sites * d.P4; idx += blockDim.x) {
      const int s = idx / d.P4, e = idx % d.P4;
      const SiteShape sh = site_shape(d, s);
      if (e >= sh.bs) continue;
      const int blk = block_id[(size_t)b * d.n_sites + s];
      acc += O[(size_t)b * d.n_sites * d.P4 + idx] * v[site_offset[s] + (int64_t)blk * sh.bs + e];
    }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) ov[b] = acc;
}

__global__ void k_sr_dot(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                         double* __restrict__ out) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += a[i] * b[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = acc;
}

// Dense S (row m per workgroup): S_mn = <O_m O_n> - <O_m><O_n>.
__global__ void k_sr_dense(Dims d, const int64_t* __restrict__ site_offset,
                           const int32_t* __restrict__ block_id, const uint8_t* __restrict__ valid,
                           const double* __restrict__ O, const double* __restrict__ omean, int B,
                           int64_t n_params, double* __restrict__ S) {
  __shared__ double red[16];
  __shared__ int sm_site, sm_blk, sm_e;
  const int64_t m = blockIdx.x;
  if (threadIdx.x == 0) {
    int s = 0;
    while (site_offset[s + 1] <= m) ++s;
    const SiteShape sh = site_shape(d, s);
    const int64_t r = m - site_offset[s];
    sm_site = s;
    sm_blk = (int)(r / sh.bs);
    sm_e = (int)(r % sh.bs);
  }
  double nv, em;
  valid_stats(valid, nullptr, B, red, &nv, &em);
  const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
  const int s1 = sm_site, b1 = sm_blk, e1 = sm_e;
  for (int64_t n = threadIdx.x; n < n_params; n += blockDim.x) {
    int s2 = 0;
    while (site_offset[s2 + 1] <= n) ++s2;
    const SiteShape sh = site_shape(d, s2);
    const int64_t r = n - site_offset[s2];
    const int b2 = (int)(r / sh.bs), e2 = (int)(r % sh.bs);
    double acc = 0.0;
    for (int b = 0; b < B; ++b) {
      if (!valid[b]) continue;
      if (block_id[(size_t)b * d.n_sites + s1] != b1 || block_id[(size_t)b * d.n_sites + s2] != b2) continue;
      acc += O[((size_t)b * d.n_sites + s1) * d.P4 + e1] * O[((size_t)b * d.n_sites + s2) * d.P4 + e2];
    }
    S[m * n_params + n] = acc * inv - omean[m] * omean[n];
  }
}

// Rows row0 .. row0 + gridDim.x - 1 of S (one workgroup per row m): the row is cleared, then every
// valid sample whose selected block holds m adds O_bm times its own nonzeros (one block per site);
// an entry n is always updated by the thread that owns its (site, entry) pair, so the samples are
// added in index order without atomics, as k_sr_dense adds them.
__global__ void k_sr_rows(Dims d, const int64_t* __restrict__ site_offset,
                          const int32_t* __restrict__ block_id, const uint8_t* __restrict__ valid,
                          const double* __restrict__ O, const double* __restrict__ omean, int B,
                          int64_t n_params, int64_t row0, double* __restrict__ S) {
  __shared__ double red[16];
  __shared__ int sm_site, sm_blk, sm_e;
  const int64_t m = row0 + blockIdx.x;
  double* row = S + (size_t)blockIdx.x * (size_t)n_params;
  if (threadIdx.x == 0) {
    int s = 0;
    while (site_offset[s + 1] <= m) ++s;
    const SiteShape sh = site_shape(d, s);
    const int64_t r = m - site_offset[s];
    sm_site = s;
    sm_blk = (int)(r / sh.bs);
    sm_e = (int)(r % sh.bs);
  }
  double nv, em;
  valid_stats(valid, nullptr, B, red, &nv, &em);  // its barriers also publish sm_*
  const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
  const int s1 = sm_site, b1 = sm_blk, e1 = sm_e;
  for (int64_t n = threadIdx.x; n < n_params; n += blockDim.x) row[n] = 0.0;
  __syncthreads();
  const int nse = d.n_sites * d.P4;
  for (int b = 0; b < B; ++b) {
    if (!valid[b] || block_id[(size_t)b * d.n_sites + s1] != b1) continue;  // same in every thread
    const double w = O[((size_t)b * d.n_sites + s1) * d.P4 + e1];
    for (int idx = threadIdx.x; idx < nse; idx += blockDim.x) {
      const int s = idx / d.P4, e = idx % d.P4;
      const SiteShape sh = site_shape(d, s);
      if (e >= sh.bs) continue;
      const int64_t n = site_offset[s] + (int64_t)block_id[(size_t)b * d.n_sites + s] * sh.bs + e;
      row[n] += w * O[((size_t)b * d.n_sites + s) * d.P4 + e];
    }
  }
  __syncthreads();
  for (int64_t n = threadIdx.x; n < n_params; n += blockDim.x) row[n] = row[n] * inv - omean[m] * omean[n];
}

// Conjugate-gradient vector steps of sr_solve ((S + shift I) x = F).  The scalars of iteration k
// live at sc[2k] = r.r and sc[2k+1] = p.q (sc[2k+2] = the next r.r), written by k_sr_dot.
__global__ void k_cg_init(const double* __restrict__ F, double* __restrict__ x, double* __restrict__ r,
                          double* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    x[i] = 0.0;
    r[i] = F[i];
    p[i] = F[i];
  }
}

__global__ void k_cg_shift(double* __restrict__ q, const double* __restrict__ p, double shift, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] += shift * p[i];
}

// x += alpha p, r -= alpha q with alpha = sc[2k] / sc[2k+1]; nothing when p.q <= 0 (breakdown)
__global__ void k_cg_step(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                          const double* __restrict__ q, const double* __restrict__ sc, int k, int64_t n) {
  const double pq = sc[2 * k + 1];
  if (!(pq > 0.0)) return;
  const double alpha = sc[2 * k] / pq;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
  }
}

// p = r + beta p with beta = sc[2k+2] / sc[2k]
__global__ void k_cg_dir(double* __restrict__ p, const double* __restrict__ r, const double* __restrict__ sc,
                         int k, int64_t n) {
  const double beta = sc[2 * k + 2] / sc[2 * k];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = r[i] + beta * p[i];
}

hipError_t launch_cg(int op, int64_t n, double* x, double* r, double* p, double* q, const double* F,
                     double* sc, int k, double shift, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
  switch (op) {
    case kCgInit: hipLaunchKernelGGL(k_cg_init, grid, blk, 0, s, F, x, r, p, n); break;
    case kCgShift: hipLaunchKernelGGL(k_cg_shift, grid, blk, 0, s, q, p, shift, n); break;
    case kCgStep: hipLaunchKernelGGL(k_cg_step, grid, blk, 0, s, x, r, p, q, sc, k, n); break;
    case kCgDir: hipLaunchKernelGGL(k_cg_dir, grid, blk, 0, s, p, r, sc, k, n); break;
    case kCgDotRR: hipLaunchKernelGGL(k_sr_dot, dim3(1), dim3(1024), 0, s, r, r, n, sc + 2 * k); break;
    case kCgDotPQ: hipLaunchKernelGGL(k_sr_dot, dim3(1), dim3(1024), 0, s, p, q, n, sc + 2 * k + 1); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sr(const Dims& d, const DeviceTables& t, int64_t n_params, const int32_t* block_id,
                     const uint8_t* valid, const double* O, const double* e_loc, int B, int mode,
                     const double* v, double* F, double* omean, double* S_or_Sv, double* ov,
                     double* omv, hipStream_t s) {
  // <O> and F first (the matvec needs <O> . v)
  hipLaunchKernelGGL(k_sr_site, dim3(d.n_sites), dim3(256), 0, s, d, t.site_offset, block_id, valid,
                     O, e_loc, (const double*)nullptr, (const double*)nullptr, B, F, omean,
                     (double*)nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == SR_MATVEC) {
    hipLaunchKernelGGL(k_sr_ov, dim3(B), dim3(256), 0, s, d, t.site_offset, block_id, valid, O, v, ov);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sr_dot, dim3(1), dim3(1024), 0, s, omean, v, n_params, omv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sr_site, dim3(d.n_sites), dim3(256), 0, s, d, t.site_offset, block_id, valid,
                       O, e_loc, (const double*)ov, (const double*)omv, B, F, omean, S_or_Sv);
  } else {
    hipLaunchKernelGGL(k_sr_dense, dim3((unsigned)n_params), dim3(256), 0, s, d, t.site_offset,
                       block_id, valid, O, omean, B, n_params, S_or_Sv);
  }
  return hipGetLastError();
}

hipError_t launch_sr_rows(const Dims& d, const DeviceTables& t, int64_t n_params, const int32_t* block_id,
                          const uint8_t* valid, const double* O, const double* omean, int B, int64_t row0,
                          int64_t nrows, double* S, hipStream_t s) {
  if (nrows == 0 || B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sr_rows, dim3((unsigned)nrows), dim3(256), 0, s, d, t.site_offset, block_id, valid,
                     O, omean, B, n_params, row0, S);
  return hipGetLastError();
}

}  // namespace gipeps
