// Complex tensors and real-time evolution (SM S-3): exact contraction on small lattices.
//
// A truncated SVD is not a holomorphic function of the tensors, so the derivative
// O_m = d ln Psi / d alpha_m of eq. tVMC is taken here on the exact amplitude: the network is
// contracted row by row in the full space of the vertical bonds of a row cut (dimension Dk^L),
// where Psi is multilinear in the site tensors and d Psi / dT_x is the network with site x open.
//
// Row states.  V_y (bonds below row y, indexed by the d legs of row y, leg x most significant)
// is the contraction of rows 0..y-1 with V_0 = e_0; Top_y (the same bonds, from above) contracts
// rows y..L-1 with Top_L = e_0.  A row is absorbed one site at a time: the working state holds the
// legs already passed, one horizontal bond h and the legs still to pass, [p_0..p_{x-1}, h,
// p_x..p_{L-1}] (Dk^{L+1} entries), and site x trades (h, its absorbed leg) for (its new leg, h').
// Absent legs (lattice edge) are padded to Dk with the block at index 0, so every site is a
// Dk^4 tensor [l][r][d][u] and the edges are selected by e_0 boundary states.  After each row the
// state is rescaled by an exact power of two (no rounding), its exponent kept.
//
//  * k_cx_project: Gauss law, block selection (as the real projection) and complex gather.
//  * k_cx_states: V_0..V_L and Top_0..Top_L of a sample; Psi = V_L[0] 2^{s}.
//  * k_cx_eloc: E_loc (SM S-1 eq. Es) with exact ratios: <V_py R'_py R'_py+1, Top_py+2> over the
//    same with the sample's rows, the primed rows holding the blocks of P_p^{-t} s at columns
//    px, px+1.
//  * k_cx_logderiv: per row y, forward states F_x (V_y with sites < x absorbed) and backward
//    states G_x (Top_{y+1} with sites > x absorbed downwards); the environment of site x is
//    sum F_x G_x over the legs they share, divided by the row's <V_y R_y, Top_{y+1}>.
//  * tVMC linear algebra: sample weights (uniform, or |Psi|^2 normalised over the batch for exact
//    enumeration), <O>, <E>, the force g_m = <O*_m E> - <O*_m><E> (the covariance reading of eq.
//    gradient, also the right side of eq. tVMC), S v = <O* (O.v)> - <O*> (<O>.v) without forming
//    S, Hermitian conjugate gradients for (S + shift) y = g, and the update alpha += c dt alphadot
//    of eq. secondorder.
#include "dev_common.h"
#include "internal.h"
#include "philox.h"

namespace gipeps {

namespace {

constexpr int kCT = 256;  // threads per workgroup of the complex kernels

// complex numbers of the contractions: cxt<double> (complex128) or cxt<float> (complex64); the tVMC
// linear algebra, the ratios and every output stay complex128 (cx)
template <typename RT>
struct cxt {
  RT re, im;
};
using cx = cxt<double>;
template <typename RT>
__device__ __forceinline__ cxt<RT> cadd(cxt<RT> a, cxt<RT> b) { return cxt<RT>{a.re + b.re, a.im + b.im}; }
template <typename RT>
__device__ __forceinline__ cxt<RT> cmul(cxt<RT> a, cxt<RT> b) {
  return cxt<RT>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename RT>
__device__ __forceinline__ cxt<RT> cfma(cxt<RT> a, cxt<RT> b, cxt<RT> c) {  // a b + c
  return cxt<RT>{fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
template <typename RT>
__device__ __forceinline__ cxt<RT> cconj(cxt<RT> a) { return cxt<RT>{a.re, -a.im}; }
template <typename RT>
__device__ __forceinline__ cx to_d(cxt<RT> a) { return cx{(double)a.re, (double)a.im}; }
template <typename RT>
__device__ __forceinline__ cxt<RT> from_d(cx a) { return cxt<RT>{(RT)a.re, (RT)a.im}; }
__device__ __forceinline__ cx cdiv(cx a, cx b) {  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, den = b.re + b.im * r;
    return cx{(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  const double r = b.re / b.im, den = b.im + b.re * r;
  return cx{(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}

__device__ __forceinline__ int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Complex block sum in a fixed order; every thread receives the result.
__device__ cx block_sum_cx(cx v, double* red) { return cx{block_sum(v.re, red), block_sum(v.im, red)}; }

// Largest |re|, |im| over n entries (every thread receives it).
template <typename RT>
__device__ double block_absmax(const cxt<RT>* v, int n, double* red) {
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    m = fmax(m, fmax(fabs((double)v[i].re), fabs((double)v[i].im)));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// Selected block of site (x, y) for the labels lab(dir, x, y): block index as the projection's,
// written padded to Dk^4 complex entries [l][r][d][u] (absent legs at index 0).  Returns false if
// the site violates the Gauss law.
template <typename RT, class LAB>
__device__ bool gather_padded(const double* theta, const int64_t* site_offset, const int8_t* Q, int L, int N,
                              int Dk, int x, int y, LAB lab, cxt<RT>* dst) {
  const bool pres[4] = {x > 0, x < L - 1, y > 0, y < L - 1};
  const int q[4] = {pres[0] ? lab(0, x - 1, y) : 0, pres[1] ? lab(0, x, y) : 0,
                    pres[2] ? lab(1, x, y - 1) : 0, pres[3] ? lab(1, x, y) : 0};
  int div = (q[0] + q[2] - q[1] - q[3] - (int)Q[y * L + x]) % N;
  if (div < 0) div += N;
  const int P4 = Dk * Dk * Dk * Dk;
  for (int i = threadIdx.x; i < P4; i += blockDim.x) dst[i] = cxt<RT>{0, 0};
  if (div != 0) return false;
  int npres = 0, idx = 0, seen = 0;
  for (int i = 0; i < 4; ++i) npres += pres[i];
  for (int i = 0; i < 4; ++i) {
    if (!pres[i]) continue;
    if (seen < npres - 1) idx = idx * N + q[i];
    ++seen;
  }
  const int dl = pres[0] ? Dk : 1, dr = pres[1] ? Dk : 1, dd = pres[2] ? Dk : 1, du = pres[3] ? Dk : 1;
  const int bsize = dl * dr * dd * du;
  const double* src = theta + 2 * (site_offset[y * L + x] + (int64_t)idx * bsize);
  __syncthreads();  // zero fill before the scatter
  for (int i = threadIdx.x; i < bsize; i += blockDim.x) {
    int t = i;
    const int u = t % du; t /= du;
    const int d = t % dd; t /= dd;
    const int r = t % dr; t /= dr;
    const int l = t;
    dst[((l * Dk + r) * Dk + d) * Dk + u] = cxt<RT>{(RT)src[2 * i], (RT)src[2 * i + 1]};
  }
  return true;
}

// Compact projected block (first Dk^#present entries, row-major over the present legs) of site
// (x, y) into the padded [l][r][d][u] layout.
template <typename RT>
__device__ void load_padded(const cx* comp, int L, int Dk, int x, int y, cxt<RT>* dst) {
  const int dl = x > 0 ? Dk : 1, dr = x < L - 1 ? Dk : 1, dd = y > 0 ? Dk : 1, du = y < L - 1 ? Dk : 1;
  const int P4 = Dk * Dk * Dk * Dk;
  for (int i = threadIdx.x; i < P4; i += blockDim.x) {
    int t = i;
    const int u = t % Dk; t /= Dk;
    const int d = t % Dk; t /= Dk;
    const int r = t % Dk; t /= Dk;
    const int l = t;
    cx v{0.0, 0.0};
    if (l < dl && r < dr && d < dd && u < du) v = comp[((l * dr + r) * dd + d) * du + u];
    dst[i] = from_d<RT>(v);
  }
}

// One site of a row: W_{x+1} = W_x contracted with T over (h, absorbed leg).  down = true absorbs
// d (a row applied from below: new leg u); down = false absorbs u (from above: new leg d).
// The input entry ((A Dk + h) Dk + a) tail + R and the output entry ((A Dk + b) Dk + hp) tail + R
// share the column (A, R) (A: the legs left of x, R: the legs right of it, tail = Dk^(L-x-1)), so
// one thread takes a column: it reads the column's Dk^2 inputs once and writes its Dk^2 outputs,
// with the site tensor held in registers at Dk <= 2.  Win may equal Wout (in place): the columns
// of different threads are disjoint and each thread reads its column before writing it.
template <int Dk, typename RT, int U = 1>
__device__ void absorb_site(const cxt<RT>* Win, cxt<RT>* Wout, const cxt<RT>* T, int L, int x, bool down) {
  using C = cxt<RT>;
  constexpr int D2 = Dk * Dk;
  const unsigned tail = (unsigned)ipow(Dk, L - x - 1), ncol = (unsigned)ipow(Dk, L - 1);
  constexpr bool kTreg = Dk <= 2;
  C Tr[kTreg ? D2 * D2 : 1];
  // Tr[(h Dk + a) D2 + (b Dk + hp)] = the factor of input (h, a) in output (b, hp)
  auto tf = [&](int h, int a, int b, int hp) -> C {
    return down ? T[((h * Dk + hp) * Dk + a) * Dk + b] : T[((h * Dk + hp) * Dk + b) * Dk + a];
  };
  if constexpr (kTreg) {
#pragma unroll
    for (int h = 0; h < Dk; ++h)
#pragma unroll
      for (int a = 0; a < Dk; ++a)
#pragma unroll
        for (int b = 0; b < Dk; ++b)
#pragma unroll
          for (int hp = 0; hp < Dk; ++hp) Tr[(h * Dk + a) * D2 + b * Dk + hp] = tf(h, a, b, hp);
  }
  // U columns per iteration: their loads are issued before any of their arithmetic, so a thread
  // has U columns' loads in flight (the local energy's partial rows take U = 2)
  for (unsigned c0 = threadIdx.x; c0 < ncol; c0 += U * blockDim.x) {
    C w[U][D2];
    size_t base[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned c = c0 + u * blockDim.x;
      const unsigned A = c / tail, R = c - A * tail;
      base[u] = (size_t)A * D2 * tail + R;
#pragma unroll
      for (int q = 0; q < D2; ++q) w[u][q] = c < ncol ? Win[base[u] + (size_t)q * tail] : C{0, 0};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (c0 + u * blockDim.x >= ncol) break;
#pragma unroll
      for (int b = 0; b < Dk; ++b)
#pragma unroll
        for (int hp = 0; hp < Dk; ++hp) {
          C acc{0, 0};
#pragma unroll
          for (int h = 0; h < Dk; ++h)
#pragma unroll
            for (int a = 0; a < Dk; ++a) {
              C f;
              if constexpr (kTreg)
                f = Tr[(h * Dk + a) * D2 + b * Dk + hp];
              else
                f = tf(h, a, b, hp);
              acc = cfma(w[u][h * Dk + a], f, acc);
            }
          Wout[base[u] + (size_t)(b * Dk + hp) * tail] = acc;
        }
    }
  }
}

// As absorb_site (U = 1), with the Dk outputs (b, .) of a column on lane group b of one wave: Dk
// groups of 64 / Dk lanes (the lanes beyond Dk (64 / Dk) idle), each holding the D2 Dk factors of
// its outputs in registers instead of all D2 D2, for a lower register count and more waves per
// SIMD.  Every lane of a column reads the column's D2 inputs; the in-place update stays safe because
// a column's lanes share one wave and every output depends on all of its inputs, so each wave's
// loads of a column complete before any of its stores.  Each output sums in absorb_site's order.
template <int Dk, typename RT>
__device__ void absorb_site_split(const cxt<RT>* Win, cxt<RT>* Wout, const cxt<RT>* T, int L, int x, bool down) {
  using C = cxt<RT>;
  constexpr int D2 = Dk * Dk;
  constexpr int CPW = 64 / Dk;  // columns per wave and iteration
  const unsigned tail = (unsigned)ipow(Dk, L - x - 1), ncol = (unsigned)ipow(Dk, L - 1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int b = lane / CPW, cl = lane - b * CPW;
  if (b >= Dk) return;  // idle lanes (no barrier below)
  // Tb[(h Dk + a) Dk + hp] = the factor of input (h, a) in output (b, hp)
  C Tb[D2 * Dk];
#pragma unroll
  for (int h = 0; h < Dk; ++h)
#pragma unroll
    for (int a = 0; a < Dk; ++a)
#pragma unroll
      for (int hp = 0; hp < Dk; ++hp)
        Tb[(h * Dk + a) * Dk + hp] = down ? T[((h * Dk + hp) * Dk + a) * Dk + b] : T[((h * Dk + hp) * Dk + b) * Dk + a];
  for (unsigned c = (unsigned)(wave * CPW + cl); c < ncol; c += (unsigned)(nwave * CPW)) {
    const unsigned A = c / tail, R = c - A * tail;
    const size_t base = (size_t)A * D2 * tail + R;
    C w[D2];
#pragma unroll
    for (int q = 0; q < D2; ++q) w[q] = Win[base + (size_t)q * tail];
    C acc[Dk];
#pragma unroll
    for (int hp = 0; hp < Dk; ++hp) {
      acc[hp] = C{0, 0};
#pragma unroll
      for (int h = 0; h < Dk; ++h)
#pragma unroll
        for (int a = 0; a < Dk; ++a) acc[hp] = cfma(w[h * Dk + a], Tb[(h * Dk + a) * Dk + hp], acc[hp]);
    }
#pragma unroll
    for (int hp = 0; hp < Dk; ++hp) Wout[base + (size_t)(b * Dk + hp) * tail] = acc[hp];
  }
}

// state (Dk^L, leg 0 most significant) -> the row's working layout with h = 0 in front
template <typename RT>
__device__ void state_to_work(const cxt<RT>* V, cxt<RT>* W, int S, int Dk) {
  for (int i = threadIdx.x; i < S * Dk; i += blockDim.x) W[i] = i < S ? V[i] : cxt<RT>{0, 0};
}

// Absorb a whole row (tensors T[x], padded) into the state in w (working layout, h in front), in
// place: afterwards w holds W_L = [p_0..p_{L-1}, h].
template <int Dk, typename RT>
__device__ void absorb_row(cxt<RT>* w, const cxt<RT>* T, int L, bool down) {
  const int P4 = Dk * Dk * Dk * Dk;
  for (int x = 0; x < L; ++x) {
    absorb_site<Dk, RT>(w, w, T + (size_t)x * P4, L, x, down);
    __syncthreads();
  }
}

// Bilinear <W_L (h = 0 slots), Top>, summed in FP64
template <typename RT>
__device__ cx overlap(const cxt<RT>* WL, const cxt<RT>* Top, int S, int Dk, double* red) {
  cx acc{0.0, 0.0};
  for (int p = threadIdx.x; p < S; p += blockDim.x) acc = cfma(to_d(WL[(size_t)p * Dk]), to_d(Top[p]), acc);
  return block_sum_cx(acc, red);
}

// Backward states of a row with tensors T (padded): G_{L-1}[p, h] = Top[p] delta(h, 0), and G_{x-1}
// from G_x through site x, absorbing its u leg (from above), for x = L-1 down to xmin + 1.  G_x
// (W entries at G + x W) has the legs [p_0..p_x, h, p_{x+1}..p_{L-1}]: p_0..p_x face the row's u
// legs, h is the bond right of site x, p_{x+1}.. are the d legs of the sites already absorbed --
// the layout of a forward state after sites 0..x, so that the two meet by a plain bilinear sum.
template <int Dk, typename RT>
__device__ void backward_states(const cxt<RT>* top, const cxt<RT>* T, cxt<RT>* G, int L, int xmin) {
  using C = cxt<RT>;
  constexpr int D2 = Dk * Dk;
  const int W = ipow(Dk, L + 1);
  const unsigned ncol = (unsigned)ipow(Dk, L - 1);
  for (int i = threadIdx.x; i < W; i += blockDim.x)
    G[(size_t)(L - 1) * W + i] = (i % Dk == 0) ? top[i / Dk] : C{0, 0};
  __syncthreads();
  // input ((A Dk + u) Dk + hp) tail + R of G_x, output ((A Dk + h) Dk + dd) tail + R of G_{x-1}: one
  // column (A, R) per thread, as in absorb_site
  for (int x = L - 1; x > xmin; --x) {
    const unsigned tail = (unsigned)ipow(Dk, L - x - 1);
    const C* Gx = G + (size_t)x * W;
    C* Gm = G + (size_t)(x - 1) * W;
    const C* Tx = T + (size_t)x * D2 * D2;
    for (unsigned c = threadIdx.x; c < ncol; c += blockDim.x) {
      const unsigned A = c / tail, R = c - A * tail;
      const size_t base = (size_t)A * D2 * tail + R;
      C g[D2];
#pragma unroll
      for (int q = 0; q < D2; ++q) g[q] = Gx[base + (size_t)q * tail];
#pragma unroll
      for (int h = 0; h < Dk; ++h)
#pragma unroll
        for (int dd = 0; dd < Dk; ++dd) {
          C acc{0, 0};
#pragma unroll
          for (int u = 0; u < Dk; ++u)
#pragma unroll
            for (int hp = 0; hp < Dk; ++hp)
              acc = cfma(g[u * Dk + hp], Tx[((h * Dk + hp) * Dk + dd) * Dk + u], acc);
          Gm[base + (size_t)(h * Dk + dd) * tail] = acc;
        }
    }
    __syncthreads();
  }
}

// Plain bilinear sum over n entries, in FP64 (every thread receives it)
template <typename RT>
__device__ cx dot_cx(const cxt<RT>* a, const cxt<RT>* b, int n, double* red) {
  cx acc{0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc = cfma(to_d(a[i]), to_d(b[i]), acc);
  return block_sum_cx(acc, red);
}

struct CxShape {
  int L, N, Dk, S, W, P4;
};
__device__ CxShape cx_shape(const Dims& d) {
  CxShape c;
  c.L = d.L; c.N = d.N; c.Dk = d.Dk;
  c.S = ipow(d.Dk, d.L);
  c.W = c.S * d.Dk;
  c.P4 = d.P4;
  return c;
}

// The working state of a sample (W complex): in the dynamic LDS (one state: every absorption runs
// in place), or, when it exceeds kCxMaxWork entries (wscr != null), in the sample's slot of wscr,
// which holds two states (2 W complex per sample); the row tensors follow the state in LDS, or
// start the LDS.
template <typename RT>
__device__ __forceinline__ cxt<RT>* work_state(double* smem, double* wscr, int b, int W) {
  return wscr ? reinterpret_cast<cxt<RT>*>(wscr) + (size_t)b * 2 * W : reinterpret_cast<cxt<RT>*>(smem);
}
template <typename RT>
__device__ __forceinline__ cxt<RT>* row_tensors(double* smem, double* wscr, int W) {
  return wscr ? reinterpret_cast<cxt<RT>*>(smem) : reinterpret_cast<cxt<RT>*>(smem) + (size_t)W;
}

// W_L[p, h] -> the working layout of the next row, h = 0 in front: w[i] = W_L[i Dk] for i < S, zero
// for S <= i < W.  In LDS (W <= kCxMaxWork) in place through registers; with the state in global
// memory through the sample's second slot spare, the returned buffer holding the result.
constexpr int kXR = (kCxMaxWork + kCT - 1) / kCT;  // entries per thread of an LDS state
// (not inlined: its staging registers would otherwise add to the E_loc kernel's peak register use)
template <int Dk, typename RT>
__device__ __attribute__((noinline)) cxt<RT>* next_row_layout(cxt<RT>* w, cxt<RT>* spare, int S, int W) {
  using C = cxt<RT>;
  if (!spare) {
    C v[kXR];
#pragma unroll
    for (int r = 0; r < kXR; ++r) {
      const int i = threadIdx.x + r * kCT;
      v[r] = i < S ? w[(size_t)i * Dk] : C{0, 0};
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kXR; ++r) {
      const int i = threadIdx.x + r * kCT;
      if (i < W) w[i] = v[r];
    }
    __syncthreads();
    return w;
  }
  for (int i = threadIdx.x; i < W; i += blockDim.x) spare[i] = i < S ? w[(size_t)i * Dk] : C{0, 0};
  __syncthreads();
  return spare;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kCT)
k_cx_project(Dims d, const int64_t* __restrict__ site_offset, const int8_t* __restrict__ Q,
             const double* __restrict__ theta, const uint8_t* __restrict__ links, double* __restrict__ proj,
             int32_t* __restrict__ block_id, uint8_t* __restrict__ valid) {
  const int b = blockIdx.x;
  const int L = d.L, N = d.N, Dk = d.Dk;
  const uint8_t* lk = links + (size_t)b * d.planes * L * L;
  double* pb = proj + (size_t)b * d.n_sites * d.P4 * 2;
  int ok = 1;
  for (int s = threadIdx.x; s < d.n_sites; s += blockDim.x) {
    const int x = s % L, y = s / L;
    const bool pres[4] = {x > 0, x < L - 1, y > 0, y < L - 1};
    const int q[4] = {pres[0] ? (int)lk[y * L + x - 1] : 0, pres[1] ? (int)lk[y * L + x] : 0,
                      pres[2] ? (int)lk[L * L + (y - 1) * L + x] : 0, pres[3] ? (int)lk[L * L + y * L + x] : 0};
    int div = (q[0] + q[2] - q[1] - q[3] - (int)Q[s]) % N;
    if (div < 0) div += N;
    bool good = div == 0;
    for (int i = 0; i < 4; ++i) good = good && q[i] < N;
    int npres = 0, idx = 0, seen = 0, bsize = 1;
    for (int i = 0; i < 4; ++i) npres += pres[i];
    for (int i = 0; i < npres; ++i) bsize *= Dk;
    double* dst = pb + (size_t)s * d.P4 * 2;
    if (!good) {
      ok = 0;
      block_id[(size_t)b * d.n_sites + s] = -1;
      for (int i = 0; i < 2 * d.P4; ++i) dst[i] = 0.0;
      continue;
    }
    for (int i = 0; i < 4; ++i) {
      if (!pres[i]) continue;
      if (seen < npres - 1) idx = idx * N + q[i];
      ++seen;
    }
    block_id[(size_t)b * d.n_sites + s] = idx;
    const double* src = theta + 2 * (site_offset[s] + (int64_t)idx * bsize);
    for (int i = 0; i < 2 * bsize; ++i) dst[i] = src[i];
    for (int i = 2 * bsize; i < 2 * d.P4; ++i) dst[i] = 0.0;
  }
  ok = __syncthreads_and(ok);
  if (threadIdx.x == 0) valid[b] = (uint8_t)ok;
}

// states: per sample V_0..V_L then Top_0..Top_L (S complex each); expo: per sample the 2(L+1)
// power-of-two exponents.
template <int Dk, typename RT>
__global__ void __launch_bounds__(kCT) __attribute__((amdgpu_waves_per_eu(4)))
k_cx_states(Dims d, const double* __restrict__ proj, const uint8_t* __restrict__ valid, double* __restrict__ states,
            double* __restrict__ expo, double* __restrict__ log_abs, double* __restrict__ phase,
            double* __restrict__ wscr) {
  extern __shared__ double smem[];
  __shared__ double red[kCT / 64];
  const int b = blockIdx.x;
  const CxShape c = cx_shape(d);
  const int L = c.L, S = c.S, W = c.W, P4 = c.P4;
  if (!valid[b]) {
    if (threadIdx.x == 0) {
      log_abs[b] = -INFINITY;
      phase[2 * b] = 0.0;
      phase[2 * b + 1] = 0.0;
    }
    return;
  }
  using C = cxt<RT>;
  C* w0 = work_state<RT>(smem, wscr, b, W);
  C* T = row_tensors<RT>(smem, wscr, W);  // one row, L x P4
  const cx* pb = reinterpret_cast<const cx*>(proj) + (size_t)b * d.n_sites * P4;
  C* st = reinterpret_cast<C*>(states) + (size_t)b * 2 * (L + 1) * S;
  double* ex = expo + (size_t)b * 2 * (L + 1);
  for (int pass = 0; pass < 2; ++pass) {  // 0: from below (V), 1: from above (Top)
    const bool down = pass == 0;
    C* out = st + (size_t)pass * (L + 1) * S;
    double e = 0.0;
    const int first = down ? 0 : L;
    for (int i = threadIdx.x; i < S; i += blockDim.x) out[(size_t)first * S + i] = C{(RT)(i == 0 ? 1 : 0), 0};
    if (threadIdx.x == 0) ex[pass * (L + 1) + first] = 0.0;
    __syncthreads();
    for (int k = 0; k < L; ++k) {
      const int y = down ? k : L - 1 - k;
      const int from = down ? y : y + 1, to = down ? y + 1 : y;
      for (int x = 0; x < L; ++x) load_padded(pb + (size_t)(y * L + x) * P4, L, Dk, x, y, T + (size_t)x * P4);
      state_to_work(out + (size_t)from * S, w0, S, Dk);
      __syncthreads();
      absorb_row<Dk, RT>(w0, T, L, down);
      const C* WL = w0;
      // the new state, rescaled by an exact power of two
      const double m = block_absmax(WL, W, red);
      int sh = 0;
      if (m > 0.0) (void)frexp(m, &sh);
      for (int p = threadIdx.x; p < S; p += blockDim.x) {
        const C v = WL[(size_t)p * Dk];
        out[(size_t)to * S + p] = C{ldexp(v.re, -sh), ldexp(v.im, -sh)};
      }
      e += (double)sh;
      if (threadIdx.x == 0) ex[pass * (L + 1) + to] = e;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const cx psi = to_d(st[(size_t)L * S]);  // V_L[0]
    const double a = hypot(psi.re, psi.im);
    log_abs[b] = a > 0.0 ? log(a) + ex[L] * 0.6931471805599453 : -INFINITY;
    phase[2 * b] = a > 0.0 ? psi.re / a : 0.0;
    phase[2 * b + 1] = a > 0.0 ? psi.im / a : 0.0;
  }
}

// Columns per iteration of the local energy's and the strip sampler's partial-row absorptions:
// two for complex128 at Dk <= 2 (measured at 10 x 10, D = 4: E_loc 91 -> 78 ms per tVMC step),
// one elsewhere (at D = 6 the second column's registers cost more: E_loc 569 -> 756 ms at B = 256).
template <int Dk, typename RT>
constexpr int eloc_cols() { return (Dk <= 2 && sizeof(RT) == sizeof(double)) ? 2 : 1; }

// The local energy's absorptions (all of them down, by the sample's row tensors or the primed
// ones): lane-split at Dk = 3, where the unsplit loop holds all D2 D2 factors of a site in
// registers and the kernel runs one wave per SIMD (three when split; 10 x 10, D = 6, 8192 samples,
// complex64: 8.89 -> 7.42 s per E_loc); eloc_cols columns per thread and iteration elsewhere.  The
// strip sampler keeps the unsplit loop (two waves per SIMD there; split, a sweep took 7.52 -> 7.95 s).
template <int Dk, typename RT>
__device__ __forceinline__ void eloc_absorb(const cxt<RT>* Win, cxt<RT>* Wout, const cxt<RT>* T, int L, int x) {
  if constexpr (Dk == 3)
    absorb_site_split<Dk, RT>(Win, Wout, T, L, x, true);
  else
    absorb_site<Dk, RT, eloc_cols<Dk, RT>()>(Win, Wout, T, L, x, true);
}

// <F R0[px..L-1] R1[0..px+1], G_px+1> for the strip sampler (the local energy keeps the same steps
// in a lambda of its own, which the compiler allocates more tightly): F the forward state of row
// py after px sites (R0: the row's tensors), R1 row py+1, G_x its backward states from the
// boundary above (backward_states); w0 the working state, w1 its second slot when the state lives
// in global memory (else null).
template <int Dk, typename RT>
__device__ cx strip_meet(const cxt<RT>* F, cxt<RT>* w0, cxt<RT>* w1, const cxt<RT>* T0, const cxt<RT>* T1,
                         const cxt<RT>* G, int L, int S, int W, int px, double* red) {
  constexpr int P4 = Dk * Dk * Dk * Dk;
  cxt<RT>* a = w0;
  absorb_site<Dk, RT, eloc_cols<Dk, RT>()>(F, a, T0 + (size_t)px * P4, L, px, true);
  __syncthreads();
  for (int x = px + 1; x < L; ++x) {
    absorb_site<Dk, RT, eloc_cols<Dk, RT>()>(a, a, T0 + (size_t)x * P4, L, x, true);
    __syncthreads();
  }
  a = next_row_layout<Dk, RT>(a, w1, S, W);
  for (int x = 0; x <= px + 1; ++x) {
    absorb_site<Dk, RT, eloc_cols<Dk, RT>()>(a, a, T1 + (size_t)x * P4, L, x, true);
    __syncthreads();
  }
  return dot_cx(a, G + (size_t)(px + 1) * W, W, red);
}

// E_loc (complex) of every valid sample; NaN where a strip's denominator vanishes.
//
// The ratio of plaquette p = (px, py) is <V_py R'_py R'_py+1, Top_py+2> over the same with the
// sample's rows; only the sites px, px+1 of the two rows differ.  Per pair of rows the backward
// states G_x of row py+1 (Top_py+2 with the sites right of x absorbed from above) are formed once,
// and the forward state F of row py (V_py with the sites left of px absorbed) is carried from one
// px to the next; a plaquette then absorbs the sites px..L-1 of row py from F, the sites 0..px+1
// of row py+1, and meets G_px+1: L + 2 site absorptions instead of the 2 L of a whole strip.  The
// denominator is the same contraction with the sample's own blocks.  gscr holds G_1..G_L-1 in the
// sample's slots 1..L-1 and F in slot 0.
template <int Dk, typename RT>
__global__ void __launch_bounds__(kCT)
k_cx_eloc(Dims d, const int64_t* __restrict__ site_offset, const int8_t* __restrict__ Q,
          const double* __restrict__ plaq, const double* __restrict__ elec, const double* __restrict__ theta,
          const uint8_t* __restrict__ links, const double* __restrict__ proj, const uint8_t* __restrict__ valid,
          const double* __restrict__ states, double* __restrict__ e_loc, double* __restrict__ gscr,
          double* __restrict__ wscr) {
  extern __shared__ double smem[];
  __shared__ double red[kCT / 64];
  const int b = blockIdx.x;
  const CxShape c = cx_shape(d);
  const int L = c.L, N = c.N, S = c.S, W = c.W, P4 = c.P4;
  if (!valid[b]) {
    if (threadIdx.x == 0) {
      e_loc[2 * b] = NAN;
      e_loc[2 * b + 1] = NAN;
    }
    return;
  }
  using C = cxt<RT>;
  C* w0 = work_state<RT>(smem, wscr, b, W);
  C* w1 = wscr ? w0 + W : nullptr;      // second slot of a state in global memory
  C* T0 = row_tensors<RT>(smem, wscr, W);  // row py
  C* T1 = T0 + L * P4;     // row py + 1
  C* M = T1 + L * P4;      // the four modified blocks
  const cx* pb = reinterpret_cast<const cx*>(proj) + (size_t)b * d.n_sites * P4;
  const C* st = reinterpret_cast<const C*>(states) + (size_t)b * 2 * (L + 1) * S;
  const uint8_t* lk = links + (size_t)b * d.planes * L * L;
  C* G = reinterpret_cast<C*>(gscr) + (size_t)b * L * W;  // G_x at slot x (x >= 1)
  C* F = G;                                                // forward state of row py, slot 0
  // electric part
  double el = 0.0;
  for (int i = threadIdx.x; i < 2 * L * L; i += blockDim.x) {
    const int dir = i / (L * L), y = (i / L) % L, x = i % L;
    if ((dir == 0 && x < L - 1) || (dir == 1 && y < L - 1)) el += elec[lk[i]];
  }
  el = block_sum(el, red);
  cx off{0.0, 0.0};
  bool finite = true;
  // <F R0[px..L-1] R1[0..px+1], G_px+1> with F the forward state after px sites of row py
  auto meet = [&](int px) -> cx {
    C* a = w0;
    eloc_absorb<Dk, RT>(F, a, T0 + (size_t)px * P4, L, px);
    __syncthreads();
    for (int x = px + 1; x < L; ++x) {
      eloc_absorb<Dk, RT>(a, a, T0 + (size_t)x * P4, L, x);
      __syncthreads();
    }
    a = next_row_layout<Dk, RT>(a, w1, S, W);
    for (int x = 0; x <= px + 1; ++x) {
      eloc_absorb<Dk, RT>(a, a, T1 + (size_t)x * P4, L, x);
      __syncthreads();
    }
    const cx r = dot_cx(a, G + (size_t)(px + 1) * W, W, red);
    return r;
  };
  for (int py = 0; py < L - 1; ++py) {
    for (int x = 0; x < L; ++x) {
      load_padded(pb + (size_t)(py * L + x) * P4, L, Dk, x, py, T0 + (size_t)x * P4);
      load_padded(pb + (size_t)((py + 1) * L + x) * P4, L, Dk, x, py + 1, T1 + (size_t)x * P4);
    }
    __syncthreads();
    backward_states<Dk, RT>(st + (size_t)(L + 1 + py + 2) * S, T1, G, L, 1);
    state_to_work(st + (size_t)py * S, F, S, Dk);
    __syncthreads();
    const cx den = meet(0);
    if (den.re == 0.0 && den.im == 0.0) finite = false;
    for (int px = 0; px < L - 1; ++px) {
      for (int t = 1; t < N; ++t) {
        const double ct = plaq[t];
        if (ct == 0.0) continue;
        // labels of P_p^{-t} s (p = (px, py)): h(px,py) and v(px+1,py) lowered by t, h(px,py+1) and
        // v(px,py) raised
        auto lab = [&](int dir, int x, int y) -> int {
          int n = lk[(size_t)dir * L * L + y * L + x];
          if (dir == 0 && y == py && x == px) n -= t;
          if (dir == 1 && y == py && x == px + 1) n -= t;
          if (dir == 0 && y == py + 1 && x == px) n += t;
          if (dir == 1 && y == py && x == px) n += t;
          n %= N;
          return n < 0 ? n + N : n;
        };
        for (int k = 0; k < 4; ++k)
          (void)gather_padded<RT>(theta, site_offset, Q, L, N, Dk, px + (k >> 1), py + (k & 1), lab, M + (size_t)k * P4);
        __syncthreads();
        // swap the modified blocks into the rows, contract, swap back
        for (int i = threadIdx.x; i < P4; i += blockDim.x)
          for (int k = 0; k < 4; ++k) {
            C* slot = ((k & 1) ? T1 : T0) + (size_t)(px + (k >> 1)) * P4 + i;
            const C tmp = *slot;
            *slot = M[(size_t)k * P4 + i];
            M[(size_t)k * P4 + i] = tmp;
          }
        __syncthreads();
        const cx num = meet(px);
        for (int i = threadIdx.x; i < P4; i += blockDim.x)
          for (int k = 0; k < 4; ++k) {
            C* slot = ((k & 1) ? T1 : T0) + (size_t)(px + (k >> 1)) * P4 + i;
            const C tmp = *slot;
            *slot = M[(size_t)k * P4 + i];
            M[(size_t)k * P4 + i] = tmp;
          }
        __syncthreads();
        const cx r = cdiv(num, den);
        off = cadd(off, cx{ct * r.re, ct * r.im});
      }
      // F: absorb the sample's site px of row py
      if (px + 1 < L - 1) {
        if constexpr (Dk == 3)
          absorb_site_split<Dk, RT>(F, F, T0 + (size_t)px * P4, L, px, true);
        else
          absorb_site<Dk, RT>(F, F, T0 + (size_t)px * P4, L, px, true);
        __syncthreads();
      }
    }
  }
  if (threadIdx.x == 0) {
    e_loc[2 * b] = finite ? el + off.re : NAN;
    e_loc[2 * b + 1] = finite ? off.im : NAN;
  }
}

// One Metropolis sweep of complex chains with strip ratios (SM S-2 configuration sampling; the
// proposals, order and acceptance rule of peps_metropolis: plaquettes p = py (L-1) + px in
// increasing order, power t = 1 + x mod (N-1) from counter (chain, sweep, p, 1), accepted iff
// u < |Psi(s') / Psi(s)|^2 with u from counter (chain, sweep, p, 2)).  The ratio is that of the
// local energy, <V_py R'_py R'_py+1, Top_py+2> over the current configuration's, with the forward
// state carried across the row pair and the backward states of its upper row; the rows below py
// are re-contracted as the chain moves (V_py+1 from V_py and the updated row py, stored over the
// states' V slot), the rows above py+1 are those of the configuration at the sweep's start (Top
// from k_cx_states), untouched before their strip.  The chain's links are kept in LDS and written
// back at the end.  states, gscr, wscr: as for k_cx_eloc.
constexpr int kCxMaxLinks = 2 * 64 * 64;
template <int Dk, typename RT>
__global__ void __launch_bounds__(kCT)
k_cx_strip_mc(Dims d, const int64_t* __restrict__ site_offset, const int8_t* __restrict__ Q,
              const double* __restrict__ theta, uint8_t* __restrict__ links, const uint8_t* __restrict__ valid,
              double* __restrict__ states, double* __restrict__ gscr, double* __restrict__ wscr, uint64_t seed,
              uint64_t stream, int sweep, int32_t* __restrict__ accepted) {
  extern __shared__ double smem[];
  __shared__ double red[kCT / 64];
  __shared__ uint8_t slk[kCxMaxLinks];
  __shared__ int sacc;
  const int b = blockIdx.x;
  if (!valid[b]) return;
  using C = cxt<RT>;
  const CxShape c = cx_shape(d);
  const int L = c.L, N = c.N, S = c.S, W = c.W, P4 = c.P4;
  C* w0 = work_state<RT>(smem, wscr, b, W);
  C* w1 = wscr ? w0 + W : nullptr;
  C* T0 = row_tensors<RT>(smem, wscr, W);  // row py, current configuration
  C* T1 = T0 + L * P4;                      // row py + 1
  C* M = T1 + L * P4;                       // the four blocks of the proposal
  C* st = reinterpret_cast<C*>(states) + (size_t)b * 2 * (L + 1) * S;
  C* G = reinterpret_cast<C*>(gscr) + (size_t)b * L * W;
  C* F = G;
  uint8_t* lk = links + (size_t)b * d.planes * L * L;
  for (int i = threadIdx.x; i < 2 * L * L; i += blockDim.x) slk[i] = lk[i];
  if (threadIdx.x == 0) sacc = 0;
  __syncthreads();
  auto cur = [&](int dir, int x, int y) -> int { return slk[(size_t)dir * L * L + y * L + x]; };
  auto meet = [&](int px) -> cx { return strip_meet<Dk, RT>(F, w0, w1, T0, T1, G, L, S, W, px, red); };
  for (int py = 0; py < L - 1; ++py) {
    for (int x = 0; x < L; ++x) {
      (void)gather_padded<RT>(theta, site_offset, Q, L, N, Dk, x, py, cur, T0 + (size_t)x * P4);
      (void)gather_padded<RT>(theta, site_offset, Q, L, N, Dk, x, py + 1, cur, T1 + (size_t)x * P4);
    }
    __syncthreads();
    backward_states<Dk, RT>(st + (size_t)(L + 1 + py + 2) * S, T1, G, L, 1);
    state_to_work<RT>(st + (size_t)py * S, F, S, Dk);
    __syncthreads();
    cx den = meet(0);
    for (int px = 0; px < L - 1; ++px) {
      const int p = py * (L - 1) + px;
      const int t = 1 + (int)(philox_draw((uint64_t)b, (uint64_t)sweep, (uint64_t)p, 1, seed, stream) %
                              (uint64_t)(N - 1));
      // labels of P_p^t s: h(px,py) and v(px+1,py) raised by t, h(px,py+1) and v(px,py) lowered
      auto lab = [&](int dir, int x, int y) -> int {
        int n = cur(dir, x, y);
        if (dir == 0 && y == py && x == px) n += t;
        if (dir == 1 && y == py && x == px + 1) n += t;
        if (dir == 0 && y == py + 1 && x == px) n -= t;
        if (dir == 1 && y == py && x == px) n -= t;
        n %= N;
        return n < 0 ? n + N : n;
      };
      bool ok = true;
      for (int k = 0; k < 4; ++k)
        ok &= gather_padded<RT>(theta, site_offset, Q, L, N, Dk, px + (k >> 1), py + (k & 1), lab,
                                M + (size_t)k * P4);
      __syncthreads();
      for (int i = threadIdx.x; i < P4; i += blockDim.x)
        for (int k = 0; k < 4; ++k) {
          C* slot = ((k & 1) ? T1 : T0) + (size_t)(px + (k >> 1)) * P4 + i;
          const C tmp = *slot;
          *slot = M[(size_t)k * P4 + i];
          M[(size_t)k * P4 + i] = tmp;
        }
      __syncthreads();
      const cx num = meet(px);
      const double u = philox_uniform(philox_draw((uint64_t)b, (uint64_t)sweep, (uint64_t)p, 2, seed, stream));
      // u < |num / den|^2 as u |den|^2 < |num|^2: a chain whose amplitude vanishes accepts any
      // proposal of nonzero amplitude, as the amplitude rule does (the same on every thread)
      const bool acc = ok && u * (den.re * den.re + den.im * den.im) < num.re * num.re + num.im * num.im;
      if (acc) {
        den = num;
        if (threadIdx.x == 0) {
          const int n = L * L;
          slk[py * L + px] = (uint8_t)lab(0, px, py);
          slk[n + py * L + px + 1] = (uint8_t)lab(1, px + 1, py);
          slk[(py + 1) * L + px] = (uint8_t)lab(0, px, py + 1);
          slk[n + py * L + px] = (uint8_t)lab(1, px, py);
          ++sacc;
        }
      } else {
        for (int i = threadIdx.x; i < P4; i += blockDim.x)
          for (int k = 0; k < 4; ++k) {
            C* slot = ((k & 1) ? T1 : T0) + (size_t)(px + (k >> 1)) * P4 + i;
            const C tmp = *slot;
            *slot = M[(size_t)k * P4 + i];
            M[(size_t)k * P4 + i] = tmp;
          }
      }
      __syncthreads();
      if (px + 1 < L - 1) {  // F through the current site px of row py
        absorb_site<Dk, RT>(F, F, T0 + (size_t)px * P4, L, px, true);
        __syncthreads();
      }
    }
    // V_py+1 of the current configuration, rescaled by an exact power of two (ratios only)
    state_to_work<RT>(st + (size_t)py * S, w0, S, Dk);
    __syncthreads();
    absorb_row<Dk, RT>(w0, T0, L, true);
    const double m = block_absmax(w0, W, red);
    int sh = 0;
    if (m > 0.0) (void)frexp(m, &sh);
    for (int q = threadIdx.x; q < S; q += blockDim.x) {
      const C v = w0[(size_t)q * Dk];
      st[(size_t)(py + 1) * S + q] = C{ldexp(v.re, -sh), ldexp(v.im, -sh)};
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < 2 * L * L; i += blockDim.x) lk[i] = slk[i];
  if (threadIdx.x == 0 && accepted) accepted[b] += sacc;
}

// O (complex, projected layout) of every valid sample; zero for invalid ones.  gscr: per sample
// L working states G_0..G_{L-1} (Dk^{L+1} complex each).
template <int Dk, typename RT>
__global__ void __launch_bounds__(kCT) __attribute__((amdgpu_waves_per_eu(4)))
k_cx_logderiv(Dims d, const double* __restrict__ proj, const uint8_t* __restrict__ valid,
              const double* __restrict__ states, double* __restrict__ gscr, double* __restrict__ O,
              double* __restrict__ wscr) {
  extern __shared__ double smem[];
  __shared__ double red[kCT / 64];
  __shared__ cx part[kCT];
  const int b = blockIdx.x;
  const CxShape c = cx_shape(d);
  const int L = c.L, S = c.S, W = c.W, P4 = c.P4;
  cx* Ob = reinterpret_cast<cx*>(O) + (size_t)b * d.n_sites * P4;
  if (!valid[b]) {
    for (int i = threadIdx.x; i < d.n_sites * P4; i += blockDim.x) Ob[i] = cx{0.0, 0.0};
    return;
  }
  using C = cxt<RT>;
  C* w0 = work_state<RT>(smem, wscr, b, W);
  C* T = row_tensors<RT>(smem, wscr, W);
  const cx* pb = reinterpret_cast<const cx*>(proj) + (size_t)b * d.n_sites * P4;
  const C* st = reinterpret_cast<const C*>(states) + (size_t)b * 2 * (L + 1) * S;
  C* G = reinterpret_cast<C*>(gscr) + (size_t)b * L * W;
  const int chunks = kCT / P4;  // threads per environment entry
  for (int y = 0; y < L; ++y) {
    for (int x = 0; x < L; ++x) load_padded(pb + (size_t)(y * L + x) * P4, L, Dk, x, y, T + (size_t)x * P4);
    const C* top = st + (size_t)(L + 1 + y + 1) * S;  // Top_{y+1}
    __syncthreads();  // the row's tensors are in LDS
    backward_states<Dk, RT>(top, T, G, L, 0);
    // forward states and the environments; the row's amplitude from the last forward state
    state_to_work(st + (size_t)y * S, w0, S, Dk);
    __syncthreads();
    C* F = w0;
    // first the row amplitude <V_y R_y, Top_{y+1}> (the environments' common denominator)
    absorb_row<Dk, RT>(F, T, L, true);
    const cx psi = overlap(F, top, S, Dk, red);
    state_to_work(st + (size_t)y * S, w0, S, Dk);
    __syncthreads();
    for (int x = 0; x < L; ++x) {
      const int tail = ipow(Dk, L - x - 1), nA = ipow(Dk, x), nterm = nA * tail;
      const C* Gx = G + (size_t)x * W;
      const int e = threadIdx.x / chunks, ch = threadIdx.x % chunks;
      // the environment's Dk^(L-1) terms summed in FP64 (each product formed from the stored
      // states, whose precision is the handle's)
      cx acc{0.0, 0.0};
      if (e < P4) {
        const int h = e / (Dk * Dk * Dk), hp = (e / (Dk * Dk)) % Dk, dd = (e / Dk) % Dk, u = e % Dk;
        for (int k = ch; k < nterm; k += chunks) {
          const unsigned A = (unsigned)k / (unsigned)tail, R = (unsigned)k - A * (unsigned)tail;
          acc = cfma(to_d(F[((A * Dk + h) * Dk + dd) * tail + R]), to_d(Gx[((A * Dk + u) * Dk + hp) * tail + R]),
                     acc);
        }
      }
      part[threadIdx.x] = acc;
      __syncthreads();
      // environment entry e in padded [l][r][d][u] order -> O entry of the compact block
      if (threadIdx.x < P4) {
        const int ee = threadIdx.x;
        cx env{0.0, 0.0};
        for (int k = 0; k < chunks; ++k) env = cadd(env, part[ee * chunks + k]);
        const int l = ee / (Dk * Dk * Dk), r = (ee / (Dk * Dk)) % Dk, dd = (ee / Dk) % Dk, u = ee % Dk;
        const int dl = x > 0 ? Dk : 1, dr = x < L - 1 ? Dk : 1, ddm = y > 0 ? Dk : 1, du = y < L - 1 ? Dk : 1;
        cx* Os = Ob + (size_t)(y * L + x) * P4;
        if (l < dl && r < dr && dd < ddm && u < du) Os[((l * dr + r) * ddm + dd) * du + u] = cdiv(env, psi);
        // entries beyond the block stay zero
        const int bsize = dl * dr * ddm * du;
        if (ee >= bsize) Os[ee] = cx{0.0, 0.0};
      }
      absorb_site<Dk, RT>(F, F, T + (size_t)x * P4, L, x, true);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------------------
// tVMC linear algebra.  w: double [B]; O: complex [B][n_sites][P4] (projected); vectors complex [n].

// Sample weights: uniform over the valid samples, or |Psi|^2 normalised over them.
__global__ void __launch_bounds__(kCT)
k_cx_weights(int B, int mode, const double* __restrict__ log_abs, const uint8_t* __restrict__ valid,
             double* __restrict__ w) {
  __shared__ double red[kCT / 64];
  double m = -INFINITY, cnt = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x)
    if (valid[b]) {
      m = fmax(m, log_abs[b]);
      cnt += 1.0;
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  double mx = -INFINITY;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) mx = fmax(mx, red[i]);
  __syncthreads();
  cnt = block_sum(cnt, red);
  double tot = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x)
    if (valid[b]) tot += mode == 0 ? 1.0 : exp(2.0 * (log_abs[b] - mx));
  tot = block_sum(tot, red);
  for (int b = threadIdx.x; b < B; b += blockDim.x)
    w[b] = (!valid[b] || cnt == 0.0) ? 0.0 : (mode == 0 ? 1.0 : exp(2.0 * (log_abs[b] - mx))) / tot;
}

// <E> = sum_b w_b E_b into sc[0..1]
__global__ void __launch_bounds__(kCT)
k_cx_emean(int B, const double* __restrict__ w, const double* __restrict__ e_loc, double* __restrict__ sc) {
  __shared__ double red[kCT / 64];
  cx acc{0.0, 0.0};
  for (int b = threadIdx.x; b < B; b += blockDim.x)
    if (w[b] != 0.0) acc = cadd(acc, cx{w[b] * e_loc[2 * b], w[b] * e_loc[2 * b + 1]});
  acc = block_sum_cx(acc, red);
  if (threadIdx.x == 0) {
    sc[0] = acc.re;
    sc[1] = acc.im;
  }
}

// Per site, the samples of nonzero weight that select each block, in ascending sample order:
// list[s][off[s][j] .. off[s][j+1]) (a stable counting sort of the block ids of site s).  The
// parameter loops below then visit only the samples whose O has the parameter's block, in the
// same order as a scan over every sample would.  One workgroup per site: thread t counts the
// blocks of the samples [t c, (t + 1) c) (c = ceil(B / kCT)), an exclusive scan over (block,
// thread) gives each thread its first slot per block, and each thread writes its samples in
// order.  With more than kIndexBlocks blocks per site one thread does the same serially.
constexpr int kIndexBlocks = 16;
__global__ void __launch_bounds__(kCT)
k_cx_index(Dims d, int B, int nblk, const int32_t* __restrict__ bid, const double* __restrict__ w,
           int32_t* __restrict__ off, int32_t* __restrict__ list) {
  __shared__ int32_t cnt[kIndexBlocks][kCT + 1];
  const int s = blockIdx.x;
  int32_t* o = off + (size_t)s * (nblk + 1);
  int32_t* li = list + (size_t)s * B;
  if (nblk > kIndexBlocks) {
    if (threadIdx.x != 0) return;
    for (int j = 0; j <= nblk; ++j) o[j] = 0;
    for (int b = 0; b < B; ++b)
      if (w[b] != 0.0) ++o[bid[(size_t)b * d.n_sites + s] + 1];
    for (int j = 0; j < nblk; ++j) o[j + 1] += o[j];
    // fill in order: o[j] advances as block j receives its samples, then shifts back
    for (int b = 0; b < B; ++b)
      if (w[b] != 0.0) li[o[bid[(size_t)b * d.n_sites + s]]++] = b;
    for (int j = nblk; j > 0; --j) o[j] = o[j - 1];
    o[0] = 0;
    return;
  }
  const int t = threadIdx.x, c = (B + kCT - 1) / kCT;
  const int b0 = t * c, b1 = min(B, b0 + c);
  for (int j = 0; j < nblk; ++j) cnt[j][t] = 0;
  for (int b = b0; b < b1; ++b)
    if (w[b] != 0.0) ++cnt[bid[(size_t)b * d.n_sites + s]][t];
  __syncthreads();
  if (t == 0) {  // exclusive scan in (block, thread) order; cnt[j][kCT] keeps block j's total
    int run = 0;
    for (int j = 0; j < nblk; ++j) {
      o[j] = run;
      for (int u = 0; u < kCT; ++u) {
        const int v = cnt[j][u];
        cnt[j][u] = run;
        run += v;
      }
    }
    o[nblk] = run;
  }
  __syncthreads();
  for (int b = b0; b < b1; ++b)
    if (w[b] != 0.0) li[cnt[bid[(size_t)b * d.n_sites + s]][t]++] = b;
}

// The parameter-side sums run one workgroup per (site s, block j): the block's bsize entries k
// across the threads, each entry's samples (the list of block j at site s, ascending) split over
// kCT / bsize lanes that each walk every lanes-th sample in order; the lanes' partial sums are then
// added in lane order.  Blocks j beyond the site's count hold no parameters and return at once.
struct CxParamBlock {
  int64_t base;  // parameter index of entry 0 of the block
  int bsize, lanes, k, lane, first, last;
  bool exists;
};
__device__ __forceinline__ CxParamBlock param_block(const Dims& d, int nblk, const int64_t* site_offset,
                                                    const int32_t* off) {
  CxParamBlock p;
  const int s = blockIdx.x / nblk, j = blockIdx.x % nblk;
  const int L = d.L, x = s % L, y = s / L;
  p.bsize = ipow(d.Dk, (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1));
  p.base = site_offset[s] + (int64_t)j * p.bsize;
  p.exists = p.base < site_offset[s + 1];
  p.lanes = kCT / p.bsize;
  p.k = threadIdx.x % p.bsize;
  p.lane = threadIdx.x / p.bsize;
  const int32_t* o = off + (size_t)s * (nblk + 1);
  p.first = o[j];
  p.last = o[j + 1];
  return p;
}

// omean_m = sum_b w_b O_bm;  g_m = sum_b w_b conj(O_bm) E_b - conj(omean_m) <E>
__global__ void __launch_bounds__(kCT)
k_cx_force(Dims d, int B, int nblk, const int64_t* __restrict__ site_offset, const int32_t* __restrict__ off,
           const int32_t* __restrict__ list, const double* __restrict__ w, const double* __restrict__ O,
           const double* __restrict__ e_loc, const double* __restrict__ sc, double* __restrict__ omean,
           double* __restrict__ g) {
  __shared__ cx part_m[kCT], part_e[kCT];
  const CxParamBlock p = param_block(d, nblk, site_offset, off);
  if (!p.exists) return;
  const int s = blockIdx.x / nblk;
  const cx* Oc = reinterpret_cast<const cx*>(O);
  const int32_t* li = list + (size_t)s * B;
  cx om{0.0, 0.0}, oe{0.0, 0.0};
  if (p.lane < p.lanes) {
    for (int i = p.first + p.lane; i < p.last; i += p.lanes) {
      const int b = li[i];
      const cx o = Oc[((size_t)b * d.n_sites + s) * d.P4 + p.k];
      om = cadd(om, cx{w[b] * o.re, w[b] * o.im});
      const cx t = cmul(cconj(o), cx{e_loc[2 * b], e_loc[2 * b + 1]});
      oe = cadd(oe, cx{w[b] * t.re, w[b] * t.im});
    }
  }
  part_m[threadIdx.x] = om;
  part_e[threadIdx.x] = oe;
  __syncthreads();
  if ((int)threadIdx.x < p.bsize) {
    cx m{0.0, 0.0}, e{0.0, 0.0};
    for (int l = 0; l < p.lanes; ++l) {
      m = cadd(m, part_m[l * p.bsize + p.k]);
      e = cadd(e, part_e[l * p.bsize + p.k]);
    }
    const cx em{sc[0], sc[1]};
    const cx gm = cadd(e, cmul(cx{-m.re, m.im}, em));  // - conj(om) <E>
    const int64_t q = p.base + p.k;
    omean[2 * q] = m.re;
    omean[2 * q + 1] = m.im;
    g[2 * q] = gm.re;
    g[2 * q + 1] = gm.im;
  }
}

// ov_b = sum_m O_bm v_m (per sample); the valid-weighted <O>.v into sc[2..3]
__global__ void __launch_bounds__(kCT)
k_cx_ov(Dims d, int B, const int64_t* __restrict__ site_offset, const int32_t* __restrict__ bid,
        const double* __restrict__ w, const double* __restrict__ O, const double* __restrict__ v,
        double* __restrict__ ov) {
  __shared__ double red[kCT / 64];
  const int b = blockIdx.x;
  if (w[b] == 0.0) {
    if (threadIdx.x == 0) {
      ov[2 * b] = 0.0;
      ov[2 * b + 1] = 0.0;
    }
    return;
  }
  const int L = d.L, Dk = d.Dk;
  const cx* Oc = reinterpret_cast<const cx*>(O) + (size_t)b * d.n_sites * d.P4;
  const cx* vc = reinterpret_cast<const cx*>(v);
  cx acc{0.0, 0.0};
  for (int i = threadIdx.x; i < d.n_sites * d.P4; i += blockDim.x) {
    const int s = i / d.P4, k = i % d.P4;
    const int x = s % L, y = s / L;
    const int bsize = ipow(Dk, (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1));
    if (k >= bsize) continue;
    const int64_t m = site_offset[s] + (int64_t)bid[(size_t)b * d.n_sites + s] * bsize + k;
    acc = cfma(Oc[i], vc[m], acc);
  }
  acc = block_sum_cx(acc, red);
  if (threadIdx.x == 0) {
    ov[2 * b] = acc.re;
    ov[2 * b + 1] = acc.im;
  }
}

// out_m = sum_b w_b conj(O_bm) ov_b - conj(omean_m) (sum_b w_b ov_b) + shift v_m
__global__ void __launch_bounds__(kCT)
k_cx_sv(Dims d, int B, int nblk, const int64_t* __restrict__ site_offset, const int32_t* __restrict__ off,
        const int32_t* __restrict__ list, const double* __restrict__ w, const double* __restrict__ O,
        const double* __restrict__ ov, const double* __restrict__ omean, const double* __restrict__ sc, double shift,
        const double* __restrict__ v, double* __restrict__ out) {
  __shared__ cx part[kCT];
  const CxParamBlock p = param_block(d, nblk, site_offset, off);
  if (!p.exists) return;
  const int s = blockIdx.x / nblk;
  const cx* Oc = reinterpret_cast<const cx*>(O);
  const int32_t* li = list + (size_t)s * B;
  cx acc{0.0, 0.0};
  if (p.lane < p.lanes) {
    for (int i = p.first + p.lane; i < p.last; i += p.lanes) {
      const int b = li[i];
      const cx t = cmul(cconj(Oc[((size_t)b * d.n_sites + s) * d.P4 + p.k]), cx{ov[2 * b], ov[2 * b + 1]});
      acc = cadd(acc, cx{w[b] * t.re, w[b] * t.im});
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < p.bsize) {
    cx a{0.0, 0.0};
    for (int l = 0; l < p.lanes; ++l) a = cadd(a, part[l * p.bsize + p.k]);
    const int64_t q = p.base + p.k;
    const cx wov{sc[2], sc[3]};
    const cx om{omean[2 * q], omean[2 * q + 1]};
    a = cadd(a, cmul(cx{-om.re, om.im}, wov));
    out[2 * q] = a.re + shift * v[2 * q];
    out[2 * q + 1] = a.im + shift * v[2 * q + 1];
  }
}

// sc[2..3] = sum_b w_b ov_b
__global__ void __launch_bounds__(kCT)
k_cx_wov(int B, const double* __restrict__ w, const double* __restrict__ ov, double* __restrict__ sc) {
  __shared__ double red[kCT / 64];
  cx acc{0.0, 0.0};
  for (int b = threadIdx.x; b < B; b += blockDim.x)
    if (w[b] != 0.0) acc = cadd(acc, cx{w[b] * ov[2 * b], w[b] * ov[2 * b + 1]});
  acc = block_sum_cx(acc, red);
  if (threadIdx.x == 0) {
    sc[2] = acc.re;
    sc[3] = acc.im;
  }
}

// Hermitian dot <a, b> = sum conj(a_m) b_m in a fixed order into out[0..1]
__global__ void __launch_bounds__(kCT)
k_cx_dot(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out) {
  __shared__ double red[kCT / 64];
  cx acc{0.0, 0.0};
  for (int64_t m = threadIdx.x; m < n; m += blockDim.x)
    acc = cadd(acc, cmul(cx{a[2 * m], -a[2 * m + 1]}, cx{b[2 * m], b[2 * m + 1]}));
  acc = block_sum_cx(acc, red);
  if (threadIdx.x == 0) {
    out[0] = acc.re;
    out[1] = acc.im;
  }
}

// y = x + (ar + i ai) z   (y may alias x)
__global__ void __launch_bounds__(kCT)
k_cx_axpy(int64_t n, double ar, double ai, const double* __restrict__ z, const double* x, double* y) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const cx r = cfma(cx{ar, ai}, cx{z[2 * m], z[2 * m + 1]}, cx{x[2 * m], x[2 * m + 1]});
  y[2 * m] = r.re;
  y[2 * m + 1] = r.im;
}

// ---------------------------------------------------------------------------------------------
size_t cx_work(const Dims& d) {
  size_t W = d.Dk;
  for (int i = 0; i < d.L; ++i) W *= d.Dk;
  return W;
}

bool cx_work_global(const Dims& d) { return cx_work(d) > (size_t)kCxMaxWork; }

size_t cx_lds_bytes(const Dims& d, int which) {
  const size_t W = cx_work(d), P4 = d.P4, L = d.L;
  const size_t cxb = cx_elem_bytes(d);
  const size_t work = cx_work_global(d) ? 0 : W;  // the working state in LDS unless too large
  if (which == 0) return cxb * (work + L * P4);                   // states, logderiv
  return cxb * (work + 2 * L * P4 + 4 * P4);                      // eloc
}

// dynamic LDS above the default per-workgroup limit must be allowed per kernel
template <class K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_cx_project(const Dims& d, const DeviceTables& t, const double* theta, const uint8_t* links,
                             int B, double* proj, int32_t* block_id, uint8_t* valid, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cx_project, dim3(B), dim3(kCT), 0, s, d, t.site_offset, t.Q, theta, links, proj, block_id,
                     valid);
  return hipGetLastError();
}

template <int Dk, typename RT>
hipError_t launch_cx_states_t(const Dims& d, const double* proj, const uint8_t* valid, int B, double* states,
                              double* expo, double* log_abs, double* phase, double* wscr, hipStream_t s) {
  if (hipError_t e = allow_lds(k_cx_states<Dk, RT>, cx_lds_bytes(d, 0))) return e;
  hipLaunchKernelGGL((k_cx_states<Dk, RT>), dim3(B), dim3(kCT), cx_lds_bytes(d, 0), s, d, proj, valid, states, expo,
                     log_abs, phase, cx_work_global(d) ? wscr : nullptr);
  return hipGetLastError();
}

// instantiation of a complex kernel launcher for the handle's Dk (1..3) and contraction type
#define GIPEPS_CX_DISPATCH(F, ...)                              \
  switch (d.Dk * 2 + (d.cx32 ? 1 : 0)) {                        \
    case 2: return F<1, double>(__VA_ARGS__);                   \
    case 3: return F<1, float>(__VA_ARGS__);                    \
    case 4: return F<2, double>(__VA_ARGS__);                   \
    case 5: return F<2, float>(__VA_ARGS__);                    \
    case 6: return F<3, double>(__VA_ARGS__);                   \
    case 7: return F<3, float>(__VA_ARGS__);                    \
    default: return hipErrorInvalidValue;                       \
  }

hipError_t launch_cx_states(const Dims& d, const double* proj, const uint8_t* valid, int B, double* states,
                            double* expo, double* log_abs, double* phase, double* wscr, hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (cx_work_global(d) && !wscr) return hipErrorInvalidValue;
  GIPEPS_CX_DISPATCH(launch_cx_states_t, d, proj, valid, B, states, expo, log_abs, phase, wscr, s)
}

template <int Dk, typename RT>
hipError_t launch_cx_eloc_t(const Dims& d, const DeviceTables& t, const double* theta, const uint8_t* links,
                            const double* proj, const uint8_t* valid, int B, const double* states, double* e_loc,
                            double* gscr, double* wscr, hipStream_t s) {
  if (hipError_t e = allow_lds(k_cx_eloc<Dk, RT>, cx_lds_bytes(d, 1))) return e;
  hipLaunchKernelGGL((k_cx_eloc<Dk, RT>), dim3(B), dim3(kCT), cx_lds_bytes(d, 1), s, d, t.site_offset, t.Q, t.plaq,
                     t.elec, theta, links, proj, valid, states, e_loc, gscr, cx_work_global(d) ? wscr : nullptr);
  return hipGetLastError();
}

hipError_t launch_cx_eloc(const Dims& d, const DeviceTables& t, const double* theta, const uint8_t* links,
                          const double* proj, const uint8_t* valid, int B, const double* states, double* e_loc,
                          double* gscr, double* wscr, hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (!gscr || (cx_work_global(d) && !wscr)) return hipErrorInvalidValue;
  GIPEPS_CX_DISPATCH(launch_cx_eloc_t, d, t, theta, links, proj, valid, B, states, e_loc, gscr, wscr, s)
}

template <int Dk, typename RT>
hipError_t launch_cx_strip_mc_t(const Dims& d, const DeviceTables& t, const double* theta, uint8_t* links,
                                const uint8_t* valid, int B, double* states, double* gscr, double* wscr,
                                uint64_t seed, uint64_t stream, int sweep, int32_t* accepted, hipStream_t s) {
  if (hipError_t e = allow_lds(k_cx_strip_mc<Dk, RT>, cx_lds_bytes(d, 1))) return e;
  hipLaunchKernelGGL((k_cx_strip_mc<Dk, RT>), dim3(B), dim3(kCT), cx_lds_bytes(d, 1), s, d, t.site_offset, t.Q,
                     theta, links, valid, states, gscr, cx_work_global(d) ? wscr : nullptr, seed, stream, sweep,
                     accepted);
  return hipGetLastError();
}

hipError_t launch_cx_strip_mc(const Dims& d, const DeviceTables& t, const double* theta, uint8_t* links,
                              const uint8_t* valid, int B, double* states, double* gscr, double* wscr,
                              uint64_t seed, uint64_t stream, int sweep, int32_t* accepted, hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (!gscr || d.L * d.L * 2 > kCxMaxLinks || (cx_work_global(d) && !wscr)) return hipErrorInvalidValue;
  GIPEPS_CX_DISPATCH(launch_cx_strip_mc_t, d, t, theta, links, valid, B, states, gscr, wscr, seed, stream, sweep,
                     accepted, s)
}

template <int Dk, typename RT>
hipError_t launch_cx_logderiv_t(const Dims& d, const double* proj, const uint8_t* valid, int B,
                                const double* states, double* gscr, double* O, double* wscr, hipStream_t s) {
  if (hipError_t e = allow_lds(k_cx_logderiv<Dk, RT>, cx_lds_bytes(d, 0))) return e;
  hipLaunchKernelGGL((k_cx_logderiv<Dk, RT>), dim3(B), dim3(kCT), cx_lds_bytes(d, 0), s, d, proj, valid, states, gscr,
                     O, cx_work_global(d) ? wscr : nullptr);
  return hipGetLastError();
}

hipError_t launch_cx_logderiv(const Dims& d, const double* proj, const uint8_t* valid, int B, const double* states,
                              double* gscr, double* O, double* wscr, hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (cx_work_global(d) && !wscr) return hipErrorInvalidValue;
  GIPEPS_CX_DISPATCH(launch_cx_logderiv_t, d, proj, valid, B, states, gscr, O, wscr, s)
}
#undef GIPEPS_CX_DISPATCH

hipError_t launch_cx_weights(int B, int mode, const double* log_abs, const uint8_t* valid, double* w,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_cx_weights, dim3(1), dim3(kCT), 0, s, B, mode, log_abs, valid, w);
  return hipGetLastError();
}

int cx_blocks_per_site(const Dims& d) {  // largest number of blocks of a site: N^3
  return d.N * d.N * d.N;
}

hipError_t launch_cx_index(const Dims& d, int B, const int32_t* bid, const double* w, int32_t* off, int32_t* list,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_cx_index, dim3(d.n_sites), dim3(kCT), 0, s, d, B, cx_blocks_per_site(d), bid, w, off, list);
  return hipGetLastError();
}

hipError_t launch_cx_force(const Dims& d, const DeviceTables& t, int64_t n, int B, const int32_t* off,
                           const int32_t* list, const double* w, const double* O, const double* e_loc, double* sc,
                           double* omean, double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_emean, dim3(1), dim3(kCT), 0, s, B, w, e_loc, sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  const int nblk = cx_blocks_per_site(d);
  hipLaunchKernelGGL(k_cx_force, dim3((unsigned)(d.n_sites * nblk)), dim3(kCT), 0, s, d, B, nblk, t.site_offset,
                     off, list, w, O, e_loc, sc, omean, g);
  return hipGetLastError();
}

hipError_t launch_cx_matvec(const Dims& d, const DeviceTables& t, int64_t n, int B, const int32_t* bid,
                            const int32_t* off, const int32_t* list, const double* w, const double* O,
                            const double* omean, double shift, const double* v, double* ov, double* sc, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_cx_ov, dim3(B), dim3(kCT), 0, s, d, B, t.site_offset, bid, w, O, v, ov);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_cx_wov, dim3(1), dim3(kCT), 0, s, B, w, ov, sc);
    e = hipGetLastError();
  }
  if (e == hipSuccess && n > 0) {
    const int nblk = cx_blocks_per_site(d);
    hipLaunchKernelGGL(k_cx_sv, dim3((unsigned)(d.n_sites * nblk)), dim3(kCT), 0, s, d, B, nblk, t.site_offset,
                       off, list, w, O, ov, omean, sc, shift, v, out);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_cx_dot(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_dot, dim3(1), dim3(kCT), 0, s, n, a, b, out);
  return hipGetLastError();
}

hipError_t launch_cx_axpy(int64_t n, double ar, double ai, const double* z, const double* x, double* y,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cx_axpy, dim3((unsigned)((n + kCT - 1) / kCT)), dim3(kCT), 0, s, n, ar, ai, z, x, y);
  return hipGetLastError();
}

}  // namespace gipeps
