// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11): the counter-based generator of the Metropolis samplers.  Key = (seed, stream), counter =
// (chain, sweep, plaquette, purpose); a draw is the first 64-bit output word x, and
// u = (x >> 11) * 2^-53 is a uniform double in [0, 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gipeps {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// First output word at counter (c0, c1, c2, c3) and key (k0, k1).  A round maps the counter to
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped by (W0, W1)
// between rounds.
__device__ inline uint64_t philox_draw(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                       uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t h0 = __umul64hi(kPhiloxM0, c0), l0 = kPhiloxM0 * c0;
    const uint64_t h1 = __umul64hi(kPhiloxM1, c2), l1 = kPhiloxM1 * c2;
    const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = l1;
    c2 = n2;
    c3 = l0;
  }
  return c0;
}

__device__ inline double philox_uniform(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

}  // namespace gipeps
