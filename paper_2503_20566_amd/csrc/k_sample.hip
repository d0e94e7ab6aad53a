// Metropolis sampling of link configurations (SM S-2, configuration sampling): input support that
// generates Metropolis-sampled workloads on the device.
//
// Generator: Philox4x64-10 (philox.h), key = (seed, stream), counter = (chain, sweep, plaquette,
// purpose).  Purposes: 0 initial power k_p = x mod N (sweep 0), 1 proposal power
// t = 1 + x mod (N - 1), 2 acceptance uniform.  Plaquettes p = py (L - 1) + px in that order.
//
//  * k_sample_powers: one workgroup per chain, the initial plaquette powers (the links follow
//    from k_links_from_powers).
//  * k_propose: one workgroup per chain, s' = P_p^t s (raise h(px,py) and v(px+1,py), lower
//    h(px,py+1) and v(px,py) by t, mod N; the plaquette operator of eq. H_b).
//  * k_propose_hop (matter): one workgroup per chain, s' = s with the boson moved across link
//    (d, x, y) when exactly one end is occupied (the link raised when it moves towards -x / -y,
//    lowered otherwise; eq. matter's hopping), else s' = s and the chain is marked as not moved.
//    Link moves draw their uniform from counter (chain, sweep, (L-1)^2 + link index, 2), link index
//    y (L-1) + x (horizontal) or L (L-1) + y L + x (vertical).
//  * k_accept: one workgroup per chain, accept iff the chain moved and u < exp(2 (ln|Psi(s')| -
//    ln|Psi(s)|)) in float64, and copy the proposal over the state.
#include "internal.h"
#include "philox.h"

namespace gipeps {

__global__ void k_sample_powers(int L, int N, uint64_t seed, uint64_t stream,
                                uint8_t* __restrict__ powers) {
  const int b = blockIdx.x;
  const int np = (L - 1) * (L - 1);
  for (int p = threadIdx.x; p < np; p += blockDim.x)
    powers[(size_t)b * np + p] = (uint8_t)(philox_draw((uint64_t)b, 0, (uint64_t)p, 0, seed, stream) % (uint64_t)N);
}

__global__ void k_propose(int L, int N, int planes, int p, int sweep, uint64_t seed, uint64_t stream,
                          const uint8_t* __restrict__ cur, uint8_t* __restrict__ prop) {
  const int b = blockIdx.x;
  const int n = planes * L * L;
  const int px = p % (L - 1), py = p / (L - 1);
  const int t = 1 + (int)(philox_draw((uint64_t)b, (uint64_t)sweep, (uint64_t)p, 1, seed, stream) %
                          (uint64_t)(N - 1));
  const uint8_t* s = cur + (size_t)b * n;
  uint8_t* d = prop + (size_t)b * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int v = s[i];
    // links[0][y][x] = h(x, y) at y*L + x, links[1][y][x] = v(x, y) at L*L + y*L + x
    if (i == py * L + px) v += t;                    // h(px, py)
    if (i == L * L + py * L + px + 1) v += t;        // v(px+1, py)
    if (i == (py + 1) * L + px) v += N - t;          // h(px, py+1)
    if (i == L * L + py * L + px) v += N - t;        // v(px, py)
    d[i] = i < 2 * L * L ? (uint8_t)(v % N) : (uint8_t)v;  // occupations (plane 2) unchanged
  }
}

__global__ void k_propose_hop(int L, int N, int dir, int x, int y, const uint8_t* __restrict__ cur,
                              uint8_t* __restrict__ prop, uint8_t* __restrict__ moved) {
  const int b = blockIdx.x;
  const int n = 3 * L * L;
  const uint8_t* s = cur + (size_t)b * n;
  uint8_t* d = prop + (size_t)b * n;
  const int ia = 2 * L * L + y * L + x;                                  // occupation of (x, y)
  const int ib = 2 * L * L + (y + (dir == 1)) * L + x + (dir == 0);       // of its neighbour
  const int il = dir * L * L + y * L + x;                                // the link between them
  const int pa = s[ia], pb = s[ib];
  const bool mv = pa != pb;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int v = s[i];
    if (mv && i == il) v = (v + (pb ? 1 : N - 1)) % N;
    if (mv && i == ia) v = pb;
    if (mv && i == ib) v = pa;
    d[i] = (uint8_t)v;
  }
  if (threadIdx.x == 0) moved[b] = mv ? 1 : 0;
}

__global__ void k_accept(int L, int planes, int p, int sweep, uint64_t seed, uint64_t stream,
                         const uint8_t* __restrict__ moved, const double* __restrict__ la_prop,
                         const uint8_t* __restrict__ valid_prop, const uint8_t* __restrict__ prop,
                         double* __restrict__ la_cur, uint8_t* __restrict__ cur,
                         int32_t* __restrict__ accepted) {
  const int b = blockIdx.x;
  const int n = planes * L * L;
  const double u = philox_uniform(philox_draw((uint64_t)b, (uint64_t)sweep, (uint64_t)p, 2, seed, stream));
  const double lp = la_prop[b], lc = la_cur[b];
  const bool acc = (!moved || moved[b]) && valid_prop[b] && u < exp(2.0 * (lp - lc));
  if (!acc) return;  // uniform over the workgroup
  const uint8_t* s = prop + (size_t)b * n;
  uint8_t* d = cur + (size_t)b * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
  if (threadIdx.x == 0) {
    la_cur[b] = lp;
    if (accepted) accepted[b] += 1;
  }
}

hipError_t launch_sample_powers(const Dims& d, uint64_t seed, uint64_t stream, int B, uint8_t* powers,
                                hipStream_t s) {
  if (B == 0 || d.L < 2) return hipSuccess;
  hipLaunchKernelGGL(k_sample_powers, dim3(B), dim3(64), 0, s, d.L, d.N, seed, stream, powers);
  return hipGetLastError();
}

hipError_t launch_propose(const Dims& d, int p, int sweep, uint64_t seed, uint64_t stream, int B,
                          const uint8_t* cur, uint8_t* prop, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_propose, dim3(B), dim3(64), 0, s, d.L, d.N, d.planes, p, sweep, seed, stream, cur,
                     prop);
  return hipGetLastError();
}

hipError_t launch_propose_hop(const Dims& d, int dir, int x, int y, int B, const uint8_t* cur,
                              uint8_t* prop, uint8_t* moved, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_propose_hop, dim3(B), dim3(64), 0, s, d.L, d.N, dir, x, y, cur, prop, moved);
  return hipGetLastError();
}

hipError_t launch_accept(const Dims& d, int p, int sweep, uint64_t seed, uint64_t stream, int B,
                         const uint8_t* moved, const double* la_prop, const uint8_t* valid_prop,
                         const uint8_t* prop, double* la_cur, uint8_t* cur, int32_t* accepted,
                         hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_accept, dim3(B), dim3(64), 0, s, d.L, d.planes, p, sweep, seed, stream, moved,
                     la_prop, valid_prop, prop, la_cur, cur, accepted);
  return hipGetLastError();
}

}  // namespace gipeps
