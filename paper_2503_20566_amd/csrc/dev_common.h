// Device helpers shared by the kernel files: deterministic wave64 / lane-group reductions and the
// row-sweep tape layout.
#pragma once

#include <hip/hip_runtime.h>

namespace gipeps {

// Butterfly sum over the 64 lanes of a wave: every lane obtains the same bits.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 8 consecutive lanes of a lane group (xor shuffles stay inside the group).
__device__ __forceinline__ double group8_sum(double v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  return v;
}

// Block sum in a fixed order (waves in index order); every thread receives the result.
// red: LDS scratch of at least blockDim.x / 64 doubles.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (int)(blockDim.x >> 6);
  for (int w = 0; w < nw; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Tape of one row sweep, one slot per (sample, site) (doubles):
//   R   : R_c of the QR at site c, column-major with leading dimension MAXN
//   A, J: final Jacobi matrix (nr x nc, ld nr) and accumulated rotations (nc x nc, ld nc) of the
//         SVD at site c >= 1
//   S, P: column norms and descending permutation (as doubles) of that SVD
//   F   : [0] orientation (1 = Jacobi on Theta^T), [1] nu of the row (slot 0 only)
template <int MAXN>
struct TapeSlot {
  static constexpr int R = 0;
  static constexpr int A = MAXN * MAXN;
  static constexpr int J = 2 * MAXN * MAXN;
  static constexpr int S = 3 * MAXN * MAXN;
  static constexpr int P = 3 * MAXN * MAXN + MAXN;
  static constexpr int F = 3 * MAXN * MAXN + 2 * MAXN;
  static constexpr int size = 3 * MAXN * MAXN + 2 * MAXN + 8;
};

}  // namespace gipeps
