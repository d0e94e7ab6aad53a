// Input support and projection kernels.
//
//  * k_links_from_powers: closed form of prod_p P_p^{k_p}|0> (plaquette operator of eq. H_b):
//    h(x,y) = k(x,y) - k(x,y-1), v(x,y) = k(x-1,y) - k(x,y) (mod N), k outside the grid = 0; an
//    occupation plane, when the problem has matter, is all empty.
//  * k_matter_links: a Gauss-law configuration around given hard-core boson occupations p (eq.
//    gauss_N with matter): the charge Q - p of each vertex is carried along its row to column 0
//    and down column 0, h(x,y) = sum_{x'>x} (Q-p)(x',y), v(0,y) = sum_{y'>y, all x'} (Q-p),
//    other vertical links 0, plus the closed form of the plaquette powers above.
//  * k_project: eq. A / eq. gcf / SM S-2.  One workgroup per sample, one thread per vertex: the
//    leg charges are the labels of the four links (GCF), the Gauss law is checked (with the
//    vertex's occupation p when the problem has matter), the block index is the mixed-radix value
//    of the first (#legs - 1) present charges (lexicographic order of the allowed tuples, the last
//    charge being fixed by the Gauss law), offset by p times the blocks per occupation, and the
//    block is gathered.  The per-sample valid flag is a workgroup AND-reduction.
//  * k_row0_to_mps: row 0 as the first boundary MPS, site [l][u][r].
#include "internal.h"

namespace gipeps {

// label change of link (dir, x, y) under prod_p P_p^{k_p}
__device__ __forceinline__ int plaquette_flux(const uint8_t* k, int L, int dir, int x, int y) {
  const int Lp = L - 1;
  auto kk = [&](int xx, int yy) -> int {
    return (xx >= 0 && xx < Lp && yy >= 0 && yy < Lp) ? (int)k[yy * Lp + xx] : 0;
  };
  if (dir == 0 && x < L - 1) return kk(x, y) - kk(x, y - 1);
  if (dir == 1 && y < L - 1) return kk(x - 1, y) - kk(x, y);
  return 0;
}

__device__ __forceinline__ uint8_t mod_label(int n, int N) {
  n %= N;
  return (uint8_t)(n < 0 ? n + N : n);
}

__global__ void k_links_from_powers(int L, int N, int planes, const uint8_t* __restrict__ powers,
                                    uint8_t* __restrict__ links) {
  const int b = blockIdx.x;
  const uint8_t* k = powers + (size_t)b * (L - 1) * (L - 1);
  uint8_t* out = links + (size_t)b * planes * L * L;
  for (int i = threadIdx.x; i < planes * L * L; i += blockDim.x) {
    const int dir = i / (L * L), y = (i / L) % L, x = i % L;
    out[i] = dir < 2 ? mod_label(plaquette_flux(k, L, dir, x, y), N) : (uint8_t)0;
  }
}

__global__ void k_matter_links(int L, int N, const int8_t* __restrict__ Q, const uint8_t* __restrict__ powers,
                               const uint8_t* __restrict__ occ, uint8_t* __restrict__ links) {
  const int b = blockIdx.x;
  const uint8_t* k = powers + (size_t)b * (L - 1) * (L - 1);
  const uint8_t* p = occ + (size_t)b * L * L;
  uint8_t* out = links + (size_t)b * 3 * L * L;
  for (int i = threadIdx.x; i < 3 * L * L; i += blockDim.x) {
    const int dir = i / (L * L), y = (i / L) % L, x = i % L;
    int n = 0;
    if (dir == 0 && x < L - 1) {
      for (int xx = x + 1; xx < L; ++xx) n += (int)Q[y * L + xx] - (int)p[y * L + xx];
    } else if (dir == 1 && x == 0 && y < L - 1) {
      for (int v = (y + 1) * L; v < L * L; ++v) n += (int)Q[v] - (int)p[v];
    }
    out[i] = dir < 2 ? mod_label(n + plaquette_flux(k, L, dir, x, y), N) : p[y * L + x];
  }
}

__global__ void k_project(Dims d, const int64_t* __restrict__ site_offset,
                          const int8_t* __restrict__ Q, const double* __restrict__ theta,
                          const uint8_t* __restrict__ links, double* __restrict__ proj,
                          int32_t* __restrict__ block_id, uint8_t* __restrict__ valid) {
  const int b = blockIdx.x;
  const int L = d.L, N = d.N, Dk = d.Dk;
  const uint8_t* lk = links + (size_t)b * d.planes * L * L;
  double* pb = proj + (size_t)b * d.n_sites * d.P4;
  int ok = 1;
  for (int s = threadIdx.x; s < d.n_sites; s += blockDim.x) {
    const int x = s % L, y = s / L;
    const bool pres[4] = {x > 0, x < L - 1, y > 0, y < L - 1};
    const int q[4] = {pres[0] ? (int)lk[y * L + x - 1] : 0, pres[1] ? (int)lk[y * L + x] : 0,
                      pres[2] ? (int)lk[L * L + (y - 1) * L + x] : 0,
                      pres[3] ? (int)lk[L * L + y * L + x] : 0};
    const int occ = d.matter ? (int)lk[2 * L * L + s] : 0;
    int div = occ + q[0] + q[2] - q[1] - q[3] - (int)Q[s];
    div %= N;
    if (div < 0) div += N;
    bool good = occ <= 1;  // hard-core bosons
    for (int i = 0; i < 4; ++i) good = good && (q[i] < N);
    good = good && (div == 0);
    int npres = 0;
    for (int i = 0; i < 4; ++i) npres += pres[i];
    int bsize = 1;
    for (int i = 0; i < npres; ++i) bsize *= Dk;
    double* dst = pb + (size_t)s * d.P4;
    if (!good) {
      ok = 0;
      block_id[(size_t)b * d.n_sites + s] = -1;
      for (int i = 0; i < d.P4; ++i) dst[i] = 0.0;
      continue;
    }
    int idx = 0, seen = 0, per_occ = 1;
    for (int i = 0; i < 4; ++i) {
      if (!pres[i]) continue;
      if (seen < npres - 1) {
        idx = idx * N + q[i];
        per_occ *= N;
      }
      ++seen;
    }
    idx += occ * per_occ;
    block_id[(size_t)b * d.n_sites + s] = idx;
    const double* src = theta + site_offset[s] + (int64_t)idx * bsize;
    for (int i = 0; i < bsize; ++i) dst[i] = src[i];
    for (int i = bsize; i < d.P4; ++i) dst[i] = 0.0;
  }
  ok = __syncthreads_and(ok);
  if (threadIdx.x == 0) valid[b] = (uint8_t)ok;
}

__global__ void k_row0_to_mps(Dims d, const double* __restrict__ proj,
                              const uint8_t* __restrict__ valid, double* __restrict__ out_row) {
  const int b = blockIdx.x;
  if (!valid[b]) return;
  const int L = d.L, Dk = d.Dk;
  const double* pb = proj + (size_t)b * d.n_sites * d.P4;
  double* ob = out_row + (size_t)b * d.row_stride;
  for (int c = 0; c < L; ++c) {
    const int dl = c > 0 ? Dk : 1, dr = c < L - 1 ? Dk : 1, du = Dk;  // dd = 1 on row 0
    const double* T = pb + (size_t)c * d.P4;                            // T[l][r][0][u]
    double* S = ob + (size_t)c * d.site_stride;                         // S[l][u][r]
    for (int i = threadIdx.x; i < dl * du * dr; i += blockDim.x) {
      const int l = i / (du * dr), u = (i / dr) % du, r = i % dr;
      S[i] = T[(l * dr + r) * du + u];
    }
  }
}

hipError_t launch_links_from_powers(const Dims& d, const uint8_t* powers, int B, uint8_t* links,
                                    hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_links_from_powers, dim3(B), dim3(256), 0, s, d.L, d.N, d.planes, powers, links);
  return hipGetLastError();
}

hipError_t launch_matter_links(const Dims& d, const DeviceTables& t, const uint8_t* powers,
                               const uint8_t* occ, int B, uint8_t* links, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_matter_links, dim3(B), dim3(256), 0, s, d.L, d.N, t.Q, powers, occ, links);
  return hipGetLastError();
}

hipError_t launch_project(const Dims& d, const DeviceTables& t, const double* theta,
                          const uint8_t* links, int B, double* proj, int32_t* block_id,
                          uint8_t* valid, hipStream_t s) {
  if (B == 0) return hipSuccess;
  const int threads = d.n_sites <= 256 ? 256 : 1024;
  hipLaunchKernelGGL(k_project, dim3(B), dim3(threads), 0, s, d, t.site_offset, t.Q, theta, links,
                     proj, block_id, valid);
  return hipGetLastError();
}

hipError_t launch_row0_to_mps(const Dims& d, const double* proj, const uint8_t* valid, int B,
                              double* out_row, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row0_to_mps, dim3(B), dim3(64), 0, s, d, proj, valid, out_row);
  return hipGetLastError();
}

}  // namespace gipeps
