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

// Lane permutation of a double through DPP (VALU lane moves, no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 8 consecutive lanes of a lane group: quad xor 1, quad xor 2, then the mirror inside
// each half row pairs the two quads.  Every lane of the group obtains the same bits (each step adds
// the same two values, in either order).
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  return v;
}

// Wave sum through DPP inside each 16-lane row, then the four row sums read in a fixed order.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = group8_sum(v);
  v += dpp_d<0x140>(v);  // row_mirror: pairs the two half rows
  const long long bits = __double_as_longlong(v);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), 16 * r);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 16 * r);
    s += __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  return s;
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

// Register-tiled product over a workgroup: out(i, j) = sum_{k<K} a(i, k) b(k, j) for i < M, j < N.
// Each thread owns TM x TN output tiles (round-robin over the threads, consecutive threads along j),
// so an operand element fetched once feeds TM or TN multiply-adds.  The k sum runs in ascending
// order for every output (deterministic).  sink(i, j, v) receives each output once.  No barrier
// inside: the caller synchronises before reading the outputs.
template <int TM, int TN, class FA, class FB, class FS>
__device__ __forceinline__ void tile_gemm(int M, int N, int K, FA a, FB b, FS sink) {
  const int tn = (N + TN - 1) / TN, tiles = ((M + TM - 1) / TM) * tn;
  for (int t = threadIdx.x; t < tiles; t += blockDim.x) {
    const int i0 = (t / tn) * TM, j0 = (t % tn) * TN;
    double acc[TM][TN];
#pragma unroll
    for (int ii = 0; ii < TM; ++ii)
#pragma unroll
      for (int jj = 0; jj < TN; ++jj) acc[ii][jj] = 0.0;
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
      double av[TM], bv[TN];
#pragma unroll
      for (int ii = 0; ii < TM; ++ii) av[ii] = (i0 + ii < M) ? a(i0 + ii, k) : 0.0;
#pragma unroll
      for (int jj = 0; jj < TN; ++jj) bv[jj] = (j0 + jj < N) ? b(k, j0 + jj) : 0.0;
#pragma unroll
      for (int ii = 0; ii < TM; ++ii)
#pragma unroll
        for (int jj = 0; jj < TN; ++jj) acc[ii][jj] += av[ii] * bv[jj];
    }
#pragma unroll
    for (int ii = 0; ii < TM; ++ii)
#pragma unroll
      for (int jj = 0; jj < TN; ++jj)
        if (i0 + ii < M && j0 + jj < N) sink(i0 + ii, j0 + jj, acc[ii][jj]);
  }
}

// As tile_gemm, but the outputs are held in registers until every thread of the workgroup has
// read its operands (one barrier, reached by all threads), so sink may overwrite an operand.
// Requires ceil(M/TM) * ceil(N/TN) <= ROUNDS * blockDim.x.
template <int TM, int TN, int ROUNDS, class FA, class FB, class FS>
__device__ __forceinline__ void tile_gemm_sync(int M, int N, int K, FA a, FB b, FS sink) {
  const int tn = (N + TN - 1) / TN, tiles = ((M + TM - 1) / TM) * tn;
  double acc[ROUNDS][TM][TN];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int t = threadIdx.x + r * blockDim.x;
    const int i0 = (t / tn) * TM, j0 = (t % tn) * TN;
#pragma unroll
    for (int ii = 0; ii < TM; ++ii)
#pragma unroll
      for (int jj = 0; jj < TN; ++jj) acc[r][ii][jj] = 0.0;
    if (t < tiles) {
#pragma unroll 4
      for (int k = 0; k < K; ++k) {
        double av[TM], bv[TN];
#pragma unroll
        for (int ii = 0; ii < TM; ++ii) av[ii] = (i0 + ii < M) ? a(i0 + ii, k) : 0.0;
#pragma unroll
        for (int jj = 0; jj < TN; ++jj) bv[jj] = (j0 + jj < N) ? b(k, j0 + jj) : 0.0;
#pragma unroll
        for (int ii = 0; ii < TM; ++ii)
#pragma unroll
          for (int jj = 0; jj < TN; ++jj) acc[r][ii][jj] += av[ii] * bv[jj];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int t = threadIdx.x + r * blockDim.x;
    if (t >= tiles) continue;
    const int i0 = (t / tn) * TM, j0 = (t % tn) * TN;
#pragma unroll
    for (int ii = 0; ii < TM; ++ii)
#pragma unroll
      for (int jj = 0; jj < TN; ++jj)
        if (i0 + ii < M && j0 + jj < N) sink(i0 + ii, j0 + jj, acc[r][ii][jj]);
  }
}

typedef double dvec4 __attribute__((ext_vector_type(4)));

// FP64 product on the matrix cores (v_mfma_f64_16x16x4f64): out(i, j) = sum_k a(i, k) b(k, j).
// Each wave takes 16 x 16 output tiles, two at a time (two independent accumulation chains).  Per
// 4-deep k step lane l supplies A[i0 + l%16][k0 + l/16] and B[k0 + l/16][j0 + l%16] and afterwards
// holds D[i0 + l/16 + 4v][j0 + l%16] for v < 4 (lane layout checked on the device).  A lane reads
// one A and one B element per 1024 multiply-adds of the wave, a quarter of what the 4 x 4
// register tiles of tile_gemm read.  The k steps run in ascending order for every output
// (deterministic).  sink(i, j, v) receives each output once; no barrier inside.
template <class FA, class FB, class FS>
__device__ __forceinline__ void mfma_gemm(int M, int N, int K, FA a, FB b, FS sink) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int tn = (N + 15) / 16, tiles = ((M + 15) / 16) * tn;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < tiles; t += 2 * nw) {
    const int t2 = t + nw;
    const bool two = t2 < tiles;  // wave-uniform
    const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
    const int i1 = two ? (t2 / tn) * 16 : i0, j1 = two ? (t2 % tn) * 16 : j0;
    dvec4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + lk;
      const bool kin = k < K;
      const double a0 = (kin && i0 + li < M) ? a(i0 + li, k) : 0.0;
      const double b0 = (kin && j0 + li < N) ? b(k, j0 + li) : 0.0;
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c0, 0, 0, 0);
      if (two) {
        const double a1 = (kin && i1 + li < M) ? a(i1 + li, k) : 0.0;
        const double b1 = (kin && j1 + li < N) ? b(k, j1 + li) : 0.0;
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + lk + 4 * v, col = j0 + li;
      if (row < M && col < N) sink(row, col, c0[v]);
    }
    if (two) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i1 + lk + 4 * v, col = j1 + li;
        if (row < M && col < N) sink(row, col, c1[v]);
      }
    }
  }
}

// As mfma_gemm, but a wave holds the accumulators of all its tiles (at most MAXT) until every
// thread of the workgroup has read its operands (one barrier), so sink may overwrite an operand.
// Requires ceil(M/16) * ceil(N/16) <= MAXT * (blockDim.x / 64).  Every thread must call it.
template <int MAXT, class FA, class FB, class FS>
__device__ __forceinline__ void mfma_gemm_sync(int M, int N, int K, FA a, FB b, FS sink) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int tn = (N + 15) / 16, tiles = ((M + 15) / 16) * tn;
  const int li = lane & 15, lk = lane >> 4;
  dvec4 c[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    c[q] = dvec4{0.0, 0.0, 0.0, 0.0};
    const int t = wave + q * nw;
    if (t < tiles) {
      const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
      for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + lk;
        const double av = (k < K && i0 + li < M) ? a(i0 + li, k) : 0.0;
        const double bv = (k < K && j0 + li < N) ? b(k, j0 + li) : 0.0;
        c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c[q], 0, 0, 0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = wave + q * nw;
    if (t >= tiles) continue;
    const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + lk + 4 * v, col = j0 + li;
      if (row < M && col < N) sink(row, col, c[q][v]);
    }
  }
}

// As tile_gemm_staged (one operand from global memory, copied K-chunk by K-chunk into buf by all
// threads, the next chunk's loads issued before the current one is used), with the products on the
// matrix cores as in mfma_gemm_sync (at most MAXT tiles per wave).  KC is a multiple of 4.
template <int MAXT, int KC, int SPT, bool STAGE_A, class FG, class FL, class FS>
__device__ __forceinline__ void mfma_gemm_staged(int M, int N, int K, FG gload, FL lop, double* buf, FS sink) {
  static_assert(KC % 4 == 0, "chunks of whole k steps");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int R = STAGE_A ? M : N;
  const int tn = (N + 15) / 16, tiles = ((M + 15) / 16) * tn;
  const int li = lane & 15, lk = lane >> 4;
  const int nch = (K + KC - 1) / KC;
  dvec4 c[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; ++q) c[q] = dvec4{0.0, 0.0, 0.0, 0.0};
  double pf[SPT];
  auto load_chunk = [&](int k0) {
    const int kc = (K - k0 < KC) ? K - k0 : KC;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = threadIdx.x + q * blockDim.x;
      const int kk = e / R, rr = e % R;
      pf[q] = (kk < kc) ? gload(rr, k0 + kk) : 0.0;
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = threadIdx.x + q * blockDim.x;
      if (e < R * KC) buf[e] = pf[q];
    }
  };
  if (nch > 0) {
    load_chunk(0);
    store_chunk();
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int k0 = ch * KC;
    const int kc = (K - k0 < KC) ? K - k0 : KC;
    if (ch + 1 < nch) load_chunk(k0 + KC);
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
      const int t = wave + q * nw;
      if (t < tiles) {
        const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
        for (int kk0 = 0; kk0 < kc; kk0 += 4) {
          const int kk = kk0 + lk;
          const bool kin = kk < kc;
          double av, bv;
          if (STAGE_A) {
            av = (kin && i0 + li < M) ? buf[kk * R + i0 + li] : 0.0;
            bv = (kin && j0 + li < N) ? lop(k0 + kk, j0 + li) : 0.0;
          } else {
            av = (kin && i0 + li < M) ? lop(i0 + li, k0 + kk) : 0.0;
            bv = (kin && j0 + li < N) ? buf[kk * R + j0 + li] : 0.0;
          }
          c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c[q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (ch + 1 < nch) {
      store_chunk();
      __syncthreads();
    }
  }
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = wave + q * nw;
    if (t >= tiles) continue;
    const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + lk + 4 * v, col = j0 + li;
      if (row < M && col < N) sink(row, col, c[q][v]);
    }
  }
}

// As tile_gemm_sync, with one operand read from global memory: it is copied K-chunk by K-chunk
// (KC values of k) into the LDS buffer buf by all threads together, so that every load of a chunk
// is in flight at once, and the next chunk's loads are issued before the current chunk is used.
// STAGE_A: the staged operand is A, gload(i, k) = A(i, k); else it is B, gload(j, k) = B(k, j).
// lop is the other operand's accessor, (i, k) for A resp. (k, j) for B.  buf holds
// (STAGE_A ? M : N) * KC doubles; R * KC <= SPT * blockDim.x.  Outputs reach sink(i, j, v) after the
// last barrier, so sink may overwrite either operand.  Every thread must call it.
template <int TM, int TN, int ROUNDS, int KC, int SPT, bool STAGE_A, class FG, class FL, class FS>
__device__ __forceinline__ void tile_gemm_staged(int M, int N, int K, FG gload, FL lop, double* buf, FS sink) {
  const int R = STAGE_A ? M : N;
  const int tn = (N + TN - 1) / TN, tiles = ((M + TM - 1) / TM) * tn;
  const int nch = (K + KC - 1) / KC;
  double acc[ROUNDS][TM][TN];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r)
#pragma unroll
    for (int ii = 0; ii < TM; ++ii)
#pragma unroll
      for (int jj = 0; jj < TN; ++jj) acc[r][ii][jj] = 0.0;
  double pf[SPT];
  auto load_chunk = [&](int k0) {
    const int kc = (K - k0 < KC) ? K - k0 : KC;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = threadIdx.x + q * blockDim.x;
      const int kk = e / R, rr = e % R;
      pf[q] = (kk < kc) ? gload(rr, k0 + kk) : 0.0;
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = threadIdx.x + q * blockDim.x;
      if (e < R * KC) buf[e] = pf[q];
    }
  };
  if (nch > 0) {
    load_chunk(0);
    store_chunk();
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int k0 = ch * KC;
    const int kc = (K - k0 < KC) ? K - k0 : KC;
    if (ch + 1 < nch) load_chunk(k0 + KC);
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const int t = threadIdx.x + r * blockDim.x;
      if (t < tiles) {
        const int i0 = (t / tn) * TM, j0 = (t % tn) * TN;
        for (int kk = 0; kk < kc; ++kk) {
          double av[TM], bv[TN];
#pragma unroll
          for (int ii = 0; ii < TM; ++ii)
            av[ii] = (i0 + ii < M) ? (STAGE_A ? buf[kk * R + i0 + ii] : lop(i0 + ii, k0 + kk)) : 0.0;
#pragma unroll
          for (int jj = 0; jj < TN; ++jj)
            bv[jj] = (j0 + jj < N) ? (STAGE_A ? lop(k0 + kk, j0 + jj) : buf[kk * R + j0 + jj]) : 0.0;
#pragma unroll
          for (int ii = 0; ii < TM; ++ii)
#pragma unroll
            for (int jj = 0; jj < TN; ++jj) acc[r][ii][jj] += av[ii] * bv[jj];
        }
      }
    }
    __syncthreads();
    if (ch + 1 < nch) {
      store_chunk();
      __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int t = threadIdx.x + r * blockDim.x;
    if (t >= tiles) continue;
    const int i0 = (t / tn) * TM, j0 = (t % tn) * TN;
#pragma unroll
    for (int ii = 0; ii < TM; ++ii)
#pragma unroll
      for (int jj = 0; jj < TN; ++jj)
        if (i0 + ii < M && j0 + jj < N) sink(i0 + ii, j0 + jj, acc[r][ii][jj]);
  }
}

// Tape of one row sweep, one slot per (sample, site) (doubles):
//   R   : R_c of the QR at site c, column-major with leading dimension MAXN
//   U, V: the p = min(m, n) left and right singular vectors of Theta_c (site c >= 1), in
//         descending singular-value order, column a at U + a*MAXN (rows < m) resp. V + a*MAXN
//         (rows < n); a vector whose singular value is 0 is stored as 0
//   S   : the p singular values, descending
//   F   : [0] orientation of the Jacobi (1 = run on Theta^T), [1] nu of the row (slot 0 only)
template <int MAXN>
struct TapeSlot {
  static constexpr int R = 0;
  static constexpr int U = MAXN * MAXN;
  static constexpr int V = 2 * MAXN * MAXN;
  static constexpr int S = 3 * MAXN * MAXN;
  static constexpr int F = 3 * MAXN * MAXN + MAXN;
  static constexpr int size = 3 * MAXN * MAXN + MAXN + 8;
};

}  // namespace gipeps
