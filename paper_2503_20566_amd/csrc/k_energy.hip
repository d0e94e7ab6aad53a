// Local energy (SM S-1 eq. Es) of the boundary-MPS amplitude.
//
//   E_loc(s) = sum_l e[n_l] + sum_p sum_{t=1}^{N-1} c[t] Psi(P_p^-t s) / Psi(s)
//              [+ m sum_x p_x + J sum_links Psi(s_hop) / Psi(s)   with matter, eq. matter],
//
// the ratio of plaquette p = (px, py) taken on the two-row strip (py, py+1) contracted exactly
// between s's down boundary D_{py-1} and up boundary U_{py+2} (a plaquette move only changes links
// inside that strip, so both configurations share the environments).  With hard-core bosons, a
// link whose ends differ in occupation connects s to the configuration s_hop in which the boson
// crossed it (the link raised when it moved towards -x / -y, lowered otherwise); its ratio is taken
// the same way on the strip and two-column window that hold both ends: a horizontal link of row y
// in strip min(y, L-2) at its own column, a vertical link (x, y)-(x, y+1) in strip y at window
// column min(x, L-2).
//
//  * k_mirror_proj: rows reversed and d <-> u swapped, so the row-sweep kernel run on the mirrored
//    tensors yields the up boundaries (U_y = D'_{L-1-y}).
//  * k_strip: one workgroup per sample for one strip.  Left environments E_c and right environments
//    F_c of the strip are built column by column; the t-independent halves X1_c = E_c D_c and
//    Y1_c = F_{c+1} U_c are kept (per-sample scratch), so a plaquette window costs one U and one D
//    absorption per power t.  The strip's sum_{px,t} c[t] ratio is written per (sample, strip),
//    and beside it sum_{px,t} |c[t] ratio|.
//  * k_eloc_final: electric (and mass) term plus the strip sums, in a fixed order; the same for the
//    magnitudes |e[n_l]|, |m p_x| and |coefficient * ratio| (the per-sample scale of E_loc's terms).
//
// Index conventions (all row-major, leftmost slowest):
//   E_c[a][l][l'][b]    a: down-boundary bond, l / l': lower / upper row bond, b: up-boundary bond
//   X1_c[l][l'][b][d][a'],  W_c[l][l'][d][r][r'][u'] = sum_u T_lo[l][r][d][u] T_hi[l'][r'][u][u'],
//   X3_c[b][a'][r][r'][u'], Y1_c[a'][r][r'][b][u'], Y3_c[a'][l][l'][b][d].
#include "dev_common.h"
#include "internal.h"
#include "philox.h"

namespace gipeps {

namespace {

constexpr int kT = 512;
constexpr int kW = kT / 64;
constexpr int kEnv = kMaxN / kMaxDk * kMaxDk * kMaxDk * (kMaxN / kMaxDk);  // chi*2*2*chi = 5184
constexpr int kX = kEnv * kMaxDk;                                         // 10368
constexpr int kSite = kEnv / kMaxDk;                 // chi*2*chi = 2592: one boundary site
constexpr int kPPT = (kX / 8 + kT - 1) / kT;          // (b, a') pairs per thread in the W contractions
// large bonds (chi <= 64 at D_k = 2): the same quantities, held in the sample's global slot
constexpr int kEnvBig = (kMaxNBig / kMaxDk) * kMaxDk * kMaxDk * (kMaxNBig / kMaxDk);  // 16384
constexpr int kXBig = kEnvBig * kMaxDk;                                               // 32768

struct Strip {
  int L, N, Dk, py, dD, dU, B;
  const int* bD;        // bond table of D_{py-1} (null: trivial boundary)
  const int* bU;        // bond table of U_{py+2} (null: trivial boundary)
  const double* Drow;   // this sample's D_{py-1} row
  const double* Urow;   // this sample's U_{py+2} row
  int site_stride;
  __device__ int chiD(int c) const { return bD ? bD[c] : 1; }
  __device__ int chiU(int c) const { return bU ? bU[c] : 1; }
  __device__ int hl(int c) const { return (c > 0 && c < L) ? Dk : 1; }
};

// W[l][l'][d][r][r'][u'] of column c from the lower (lo) and upper (hi) row blocks.
__device__ void build_w(const Strip& S, int c, const double* lo, const double* hi, double* W) {
  const int hl = S.hl(c), hr = S.hl(c + 1), Dk = S.Dk, dD = S.dD, dU = S.dU;
  const int n = hl * hl * dD * hr * hr * dU;
  for (int idx = threadIdx.x; idx < n; idx += kT) {
    int t = idx;
    const int up = t % dU; t /= dU;
    const int rp = t % hr; t /= hr;
    const int r = t % hr; t /= hr;
    const int d = t % dD; t /= dD;
    const int lp = t % hl; t /= hl;
    const int l = t;
    double acc = 0.0;
    for (int u = 0; u < Dk; ++u)
      acc += lo[((l * hr + r) * dD + d) * Dk + u] * hi[((lp * hr + rp) * Dk + u) * dU + up];
    W[idx] = acc;
  }
}

// A configuration next to s: a plaquette move P_p^-t (p = (px, py)), a boson hop across link
// (hd, hx, hy) changing its label by hstep (the two ends' occupations exchanged), or s itself.
struct Move {
  int px, py, t;           // plaquette move (t = 0: none)
  int hd, hx, hy, hstep;   // hop (hstep = 0: none)
};
__device__ __forceinline__ Move plaquette_move(int px, int py, int t) { return Move{px, py, t, 0, 0, 0, 0}; }
__device__ __forceinline__ Move hop_move(int d, int x, int y, int step) { return Move{0, 0, 0, d, x, y, step}; }

// Label of link (dir, x, y) in the configuration mv leads to.
__device__ int mlabel(const uint8_t* lk, int L, int N, int dir, int x, int y, const Move& mv) {
  int n = lk[(size_t)dir * L * L + y * L + x];
  const int px = mv.px, py = mv.py, t = mv.t;
  if (dir == 0 && y == py && x == px) n -= t;
  if (dir == 1 && y == py && x == px + 1) n -= t;
  if (dir == 0 && y == py + 1 && x == px) n += t;
  if (dir == 1 && y == py && x == px) n += t;
  if (dir == mv.hd && x == mv.hx && y == mv.hy) n += mv.hstep;
  n %= N;
  return n < 0 ? n + N : n;
}

// Occupation of vertex (x, y) in the configuration mv leads to (0 without matter): a hop
// exchanges the occupations of the link's two ends.
__device__ int mocc(const uint8_t* lk, int L, bool matter, int x, int y, const Move& mv) {
  if (!matter) return 0;
  if (mv.hstep != 0) {
    const int bx = mv.hx + (mv.hd == 0), by = mv.hy + (mv.hd == 1);
    if (x == mv.hx && y == mv.hy) return lk[(size_t)2 * L * L + by * L + bx];
    if (x == bx && y == by) return lk[(size_t)2 * L * L + mv.hy * L + mv.hx];
  }
  return lk[(size_t)2 * L * L + y * L + x];
}

// Gather the block of site (x, y) selected by the configuration mv leads to into dst
// (Dk^#legs entries): p-major block index, as in the projection.
__device__ void gather_block(const double* theta, const int64_t* site_offset, const uint8_t* lk,
                             int L, int N, int Dk, bool matter, int x, int y, const Move& mv, double* dst) {
  const bool pres[4] = {x > 0, x < L - 1, y > 0, y < L - 1};
  int q[4];
  q[0] = pres[0] ? mlabel(lk, L, N, 0, x - 1, y, mv) : 0;
  q[1] = pres[1] ? mlabel(lk, L, N, 0, x, y, mv) : 0;
  q[2] = pres[2] ? mlabel(lk, L, N, 1, x, y - 1, mv) : 0;
  q[3] = pres[3] ? mlabel(lk, L, N, 1, x, y, mv) : 0;
  int npres = 0;
  for (int i = 0; i < 4; ++i) npres += pres[i];
  int idx = 0, seen = 0, per_occ = 1;
  for (int i = 0; i < 4; ++i) {
    if (!pres[i]) continue;
    if (seen < npres - 1) {
      idx = idx * N + q[i];
      per_occ *= N;
    }
    ++seen;
  }
  idx += mocc(lk, L, matter, x, y, mv) * per_occ;
  int bsize = 1;
  for (int i = 0; i < npres; ++i) bsize *= Dk;
  const double* src = theta + site_offset[y * L + x] + (int64_t)idx * bsize;
  for (int i = threadIdx.x; i < bsize; i += kT) dst[i] = src[i];
}

// Boundary site (rows x cols, row-major, n <= SITE entries) from global memory into LDS (or the
// sample's global slot); a trivial boundary (src == nullptr) is the 1 x 1 tensor 1.  All loads of
// a thread precede its stores.
template <int SITE = kSite>
__device__ void stage_site(double* dst, const double* src, int n) {
  constexpr int SPT = (SITE + kT - 1) / kT;
  if (!src) {
    if (threadIdx.x == 0) dst[0] = 1.0;
    return;
  }
  double v[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int i = threadIdx.x + q * kT;
    v[q] = (i < n) ? src[i] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int i = threadIdx.x + q * kT;
    if (i < n) dst[i] = v[q];
  }
}

// X3[(b,a')][o] = sum_i X1[(l,l',b,d,a')] W[i][o] over the cU*cDn pairs (b, a'), i = (l,l',d) < ni,
// o = (r,r',u') < no (both <= 8).  Each pair's inputs are read once and give all its outputs.
// In place (src == dst) every thread reads before the barrier and writes after it.
template <bool INPLACE, int PPT = kPPT>
__device__ void contract_left(const double* X1, double* dst, const double* W, int cU, int cDn, int dD,
                              int ni, int no) {
  double out[PPT][8];
  const int np = cU * cDn;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pr = threadIdx.x + q * kT;
#pragma unroll
    for (int o = 0; o < 8; ++o) out[q][o] = 0.0;
    if (pr < np) {
      const int bb = pr / cDn, ap = pr % cDn;
      double x[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        x[i] = (i < ni) ? X1[((size_t)((i / dD) * cU + bb) * dD + i % dD) * cDn + ap] : 0.0;
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        if (o >= no) break;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (i < ni) acc += x[i] * W[i * no + o];
        out[q][o] = acc;
      }
    }
  }
  if (INPLACE) __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pr = threadIdx.x + q * kT;
    if (pr < np)
#pragma unroll
      for (int o = 0; o < 8; ++o)
        if (o < no) dst[(size_t)pr * no + o] = out[q][o];
  }
}

// Y3[(a',l,l',b,d)] = sum_o Y1[(a',r,r',b,u')] W[i][o] over the cDn*cU pairs (a', b), same index
// conventions as contract_left.
template <bool INPLACE, int PPT = kPPT>
__device__ void contract_right(const double* Y1, double* dst, const double* W, int cU, int cDn, int dU,
                               int dD, int ni, int no) {
  double out[PPT][8];
  const int np = cDn * cU;
  const int nop = no / dU, nip = ni / dD;  // (r,r') and (l,l') counts
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pr = threadIdx.x + q * kT;
#pragma unroll
    for (int i = 0; i < 8; ++i) out[q][i] = 0.0;
    if (pr < np) {
      const int ap = pr / cU, bb = pr % cU;
      double y[8];
#pragma unroll
      for (int o = 0; o < 8; ++o)
        y[o] = (o < no) ? Y1[((size_t)(ap * nop + o / dU) * cU + bb) * dU + o % dU] : 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (i >= ni) break;
        double acc = 0.0;
#pragma unroll
        for (int o = 0; o < 8; ++o)
          if (o < no) acc += y[o] * W[i * no + o];
        out[q][i] = acc;
      }
    }
  }
  if (INPLACE) __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pr = threadIdx.x + q * kT;
    if (pr < np) {
      const int ap = pr / cU, bb = pr % cU;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < ni) dst[((size_t)(ap * nip + i / dD) * cU + bb) * dD + i % dD] = out[q][i];
    }
  }
}

}  // namespace

__global__ void k_mirror_proj(Dims d, const double* __restrict__ proj,
                              const uint8_t* __restrict__ valid, double* __restrict__ fproj) {
  const int b = blockIdx.x;
  if (!valid[b]) return;
  const int L = d.L, Dk = d.Dk;
  for (int idx = threadIdx.x; idx < d.n_sites * d.P4; idx += blockDim.x) {
    const int s = idx / d.P4, e = idx % d.P4;
    const int x = s % L, yp = s / L, y = L - 1 - yp;  // mirrored row yp holds original row y
    const int dl = x > 0 ? Dk : 1, dr = x < L - 1 ? Dk : 1;
    const int dd = y > 0 ? Dk : 1, du = y < L - 1 ? Dk : 1;  // original d / u dims
    double v = 0.0;
    if (e < dl * dr * dd * du) {
      // mirrored block [l][r][u][d] (dims dl, dr, du, dd) from original [l][r][d][u]
      int t = e;
      const int dm = t % dd; t /= dd;
      const int um = t % du; t /= du;
      const int r = t % dr; t /= dr;
      const int l = t;
      v = proj[((size_t)b * d.n_sites + (size_t)y * L + x) * d.P4 + ((l * dr + r) * dd + dm) * du + um];
    }
    fproj[((size_t)b * d.n_sites + s) * d.P4 + e] = v;
  }
}

// BIG: fused bonds above 72 (chi <= 64): X and the staged site in the sample's global slot (wbig)
// instead of LDS, the environment E still in LDS, X1 / Y1 slots of kXBig doubles
template <bool BIG>
__global__ void __launch_bounds__(kT)
k_strip(Dims d, int py, const int* __restrict__ bond_all, const double* __restrict__ proj,
        const double* __restrict__ theta, const int64_t* __restrict__ site_offset,
        const uint8_t* __restrict__ links, const uint8_t* __restrict__ valid,
        const double* __restrict__ down, const double* __restrict__ up,
        const double* __restrict__ plaq, double hop, double* __restrict__ scratch,
        double* __restrict__ part, double* __restrict__ pabs, double* __restrict__ wbig) {
  constexpr int ENV = BIG ? kEnvBig : kEnv;
  constexpr int XS = BIG ? kXBig : kX;
  constexpr int SITE = ENV / kMaxDk;
  constexpr int PPT = (XS / 8 + kT - 1) / kT;
  static_assert(!BIG || XS + SITE <= kBigSlot, "large-bond slot");
  __shared__ double lE[ENV];  // the environment stays in LDS (128 KB at the large size)
  __shared__ double lX[BIG ? 1 : XS];
  __shared__ double sW[64];
  __shared__ double sW2[64];
  __shared__ double lS[BIG ? 1 : SITE];  // staged boundary site (D or U) of the product at hand
  __shared__ double sTb[4][16];
  __shared__ double sRed[kW];
  const int b = blockIdx.x;
  if (!valid[b]) return;
  double* const sE = lE;
  double* const sX = BIG ? wbig + (size_t)b * kBigSlot : lX;
  double* const sS = BIG ? sX + XS : lS;
  const int L = d.L, Dk = d.Dk, N = d.N;
  Strip S;
  S.L = L; S.N = N; S.Dk = Dk; S.py = py; S.B = gridDim.x;
  S.dD = py > 0 ? Dk : 1;
  S.dU = (py + 1 < L - 1) ? Dk : 1;
  S.site_stride = d.site_stride;
  S.bD = py >= 1 ? bond_all + (size_t)(py - 1) * (L + 1) : nullptr;
  S.bU = (py + 2 <= L - 1) ? bond_all + (size_t)(L - 3 - py) * (L + 1) : nullptr;
  const size_t rs = (size_t)gridDim.x * d.row_stride;
  S.Drow = S.bD ? down + (size_t)(py - 1) * rs + (size_t)b * d.row_stride : nullptr;
  S.Urow = S.bU ? up + (size_t)(L - 3 - py) * rs + (size_t)b * d.row_stride : nullptr;
  const double* plo = proj + ((size_t)b * d.n_sites + (size_t)py * L) * d.P4;
  const double* phi = proj + ((size_t)b * d.n_sites + (size_t)(py + 1) * L) * d.P4;
  const uint8_t* lk = links + (size_t)b * d.planes * L * L;
  const bool matter = d.matter != 0;
  // per-sample scratch: X1_c and Y1_c, L slots of XS each
  double* gX1 = scratch + (size_t)b * ((size_t)2 * L * XS);
  double* gY1 = gX1 + (size_t)L * XS;
  const int dD = S.dD, dU = S.dU;

  // ---------------- left environments ----------------
  if (threadIdx.x == 0) sE[0] = 1.0;
  __syncthreads();
  for (int c = 0; c < L; ++c) {
    const int hl = S.hl(c), hr = S.hl(c + 1);
    const int cD = S.chiD(c), cDn = S.chiD(c + 1), cU = S.chiU(c), cUn = S.chiU(c + 1);
    build_w(S, c, plo + (size_t)c * d.P4, phi + (size_t)c * d.P4, sW);
    // X1[(l,l',b)][(d,a')] = sum_a E[a][(l,l',b)] D[a][(d,a')]
    stage_site<SITE>(sS, S.Drow ? S.Drow + (size_t)c * S.site_stride : nullptr, cD * dD * cDn);
    __syncthreads();
    {
      const int rows = hl * hl * cU, cols = dD * cDn;
      double* gx = gX1 + (size_t)c * XS;
      mfma_gemm(rows, cols, cD, [&](int row, int a) { return sE[(size_t)a * rows + row]; },
                      [&](int a, int col) { return sS[(size_t)a * cols + col]; },
                      [&](int row, int col, double v) {
                        sX[(size_t)row * cols + col] = v;
                        gx[(size_t)row * cols + col] = v;
                      });
    }
    __syncthreads();
    // X3[b][a'][r][r'][u'] = sum_{l,l',d} X1[l][l'][b][d][a'] W[l][l'][d][r][r'][u'] (in place)
    contract_left<true, PPT>(sX, sX, sW, cU, cDn, dD, hl * hl * dD, hr * hr * dU);
    stage_site<SITE>(sS, S.Urow ? S.Urow + (size_t)c * S.site_stride : nullptr, cU * dU * cUn);
    __syncthreads();
    // E'[(a',r,r')][b'] = sum_{(b,u')} X3[b][(a',r,r')][u'] U[(b,u')][b']
    {
      const int rows = cDn * hr * hr, K = cU * dU;
      mfma_gemm(rows, cUn, K,
                      [&](int row, int k) { return sX[((size_t)(k / dU) * rows + row) * dU + k % dU]; },
                      [&](int k, int bp) { return sS[(size_t)k * cUn + bp]; },
                      [&](int row, int bp, double v) { sE[(size_t)row * cUn + bp] = v; });
    }
    __syncthreads();
  }
  const double psi_strip = sE[0];
  __syncthreads();

  // ---------------- right environments ----------------
  if (threadIdx.x == 0) sE[0] = 1.0;
  __syncthreads();
  for (int c = L - 1; c >= 0; --c) {
    const int hl = S.hl(c), hr = S.hl(c + 1);
    const int cD = S.chiD(c), cDn = S.chiD(c + 1), cU = S.chiU(c), cUn = S.chiU(c + 1);
    build_w(S, c, plo + (size_t)c * d.P4, phi + (size_t)c * d.P4, sW);
    // Y1[(a',r,r')][(b,u')] = sum_{b'} F[(a',r,r')][b'] U[(b,u')][b']
    stage_site<SITE>(sS, S.Urow ? S.Urow + (size_t)c * S.site_stride : nullptr, cU * dU * cUn);
    __syncthreads();
    {
      const int rows = cDn * hr * hr, cols = cU * dU;
      double* gy = gY1 + (size_t)c * XS;
      mfma_gemm(rows, cols, cUn, [&](int row, int bp) { return sE[(size_t)row * cUn + bp]; },
                      [&](int bp, int col) { return sS[(size_t)col * cUn + bp]; },
                      [&](int row, int col, double v) {
                        sX[(size_t)row * cols + col] = v;
                        gy[(size_t)row * cols + col] = v;
                      });
    }
    __syncthreads();
    // Y3[a'][l][l'][b][d] = sum_{r,r',u'} Y1[a'][r][r'][b][u'] W[l][l'][d][r][r'][u'] (in place)
    contract_right<true, PPT>(sX, sX, sW, cU, cDn, dU, dD, hl * hl * dD, hr * hr * dU);
    stage_site<SITE>(sS, S.Drow ? S.Drow + (size_t)c * S.site_stride : nullptr, cD * dD * cDn);
    __syncthreads();
    // F[a][(l,l',b)] = sum_{(a',d)} D[a][d][a'] Y3[a'][(l,l',b)][d]
    {
      const int cols = hl * hl * cU, K = cDn * dD;
      mfma_gemm(cD, cols, K,
                      [&](int a, int k) { return sS[((size_t)a * dD + k % dD) * cDn + k / dD]; },
                      [&](int k, int col) { return sX[((size_t)(k / dD) * cols + col) * dD + k % dD]; },
                      [&](int a, int col, double v) { sE[(size_t)a * cols + col] = v; });
    }
    __syncthreads();
  }

  // ---------------- plaquette and hop windows ----------------
  // strip amplitude of the configuration mv leads to, which differs from s only inside the window
  // of columns (px, px+1): the left half at cut px+1, G_L = (X1_px . W'_px) . U_px, dotted with
  // the right half G_R = (Y1_{px+1} . W'_{px+1}) . D_{px+1}
  auto window_num = [&](const Move& mv, int px) -> double {
    const int c0 = px, c1 = px + 1;
    gather_block(theta, site_offset, lk, L, N, Dk, matter, c0, py, mv, sTb[0]);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, c0, py + 1, mv, sTb[1]);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, c1, py, mv, sTb[2]);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, c1, py + 1, mv, sTb[3]);
    __syncthreads();
    build_w(S, c0, sTb[0], sTb[1], sW);
    build_w(S, c1, sTb[2], sTb[3], sW2);
    __syncthreads();
    {
      const int hl = S.hl(c0), hr = S.hl(c0 + 1);
      const int cU = S.chiU(c0), cDn = S.chiD(c0 + 1), cUn = S.chiU(c0 + 1);
      const double* X1 = gX1 + (size_t)c0 * XS;
      contract_left<false, PPT>(X1, sX, sW, cU, cDn, dD, hl * hl * dD, hr * hr * dU);
      stage_site<SITE>(sS, S.Urow ? S.Urow + (size_t)c0 * S.site_stride : nullptr, cU * dU * cUn);
      __syncthreads();
      const int rows = cDn * hr * hr, K = cU * dU;
      mfma_gemm(rows, cUn, K,
                      [&](int row, int k) { return sX[((size_t)(k / dU) * rows + row) * dU + k % dU]; },
                      [&](int k, int bp) { return sS[(size_t)k * cUn + bp]; },
                      [&](int row, int bp, double v) { sE[(size_t)row * cUn + bp] = v; });
      __syncthreads();
    }
    double part_num = 0.0;
    {
      const int hl = S.hl(c1), hr = S.hl(c1 + 1);
      const int cD = S.chiD(c1), cDn = S.chiD(c1 + 1), cU = S.chiU(c1);
      const double* Y1 = gY1 + (size_t)c1 * XS;
      contract_right<false, PPT>(Y1, sX, sW2, cU, cDn, dU, dD, hl * hl * dD, hr * hr * dU);
      stage_site<SITE>(sS, S.Drow ? S.Drow + (size_t)c1 * S.site_stride : nullptr, cD * dD * cDn);
      __syncthreads();
      const int cols = hl * hl * cU, K = cDn * dD;
      mfma_gemm(cD, cols, K,
                      [&](int a, int k) { return sS[((size_t)a * dD + k % dD) * cDn + k / dD]; },
                      [&](int k, int col) { return sX[((size_t)(k / dD) * cols + col) * dD + k % dD]; },
                      [&](int a, int col, double v) { part_num += v * sE[(size_t)a * cols + col]; });
    }
    const double num = block_sum(part_num, sRed);
    __syncthreads();
    return num;
  };
  double esum = 0.0;  // kept identical in every thread
  double eabs = 0.0;  // sum of |coefficient * ratio|: the magnitude the cancellation in esum is measured against
  for (int px = 0; px < L - 1; ++px) {
    for (int t = 1; t < N; ++t) {
      const double ct = plaq[t];
      if (ct == 0.0) continue;
      const double term = ct * window_num(plaquette_move(px, py, t), px) / psi_strip;
      esum += term;
      eabs += fabs(term);
    }
  }
  if (matter && hop != 0.0) {
    // links of this strip whose two ends differ in occupation (the same in every thread): the
    // horizontal links of row py (and of row L-1 in the last strip), then the vertical links of
    // row py; the hop raises the link when the boson moves towards -x / -y
    const uint8_t* occ = lk + (size_t)2 * L * L;
    const int y_last = (py == L - 2) ? L - 1 : py;
    for (int yy = py; yy <= y_last; ++yy)
      for (int x = 0; x < L - 1; ++x) {
        const int pa = occ[yy * L + x], pb = occ[yy * L + x + 1];
        if (pa == pb) continue;
        const double term = hop * window_num(hop_move(0, x, yy, pb ? 1 : -1), x) / psi_strip;
        esum += term;
        eabs += fabs(term);
      }
    for (int x = 0; x < L; ++x) {
      const int pa = occ[py * L + x], pb = occ[(py + 1) * L + x];
      if (pa == pb) continue;
      const double term = hop * window_num(hop_move(1, x, py, pb ? 1 : -1), x < L - 1 ? x : L - 2) / psi_strip;
      esum += term;
      eabs += fabs(term);
    }
  }
  if (threadIdx.x == 0) {
    part[(size_t)b * (L - 1) + py] = esum;
    pabs[(size_t)b * (L - 1) + py] = eabs;
  }
}

// Metropolis proposals of one strip with strip ratios (SM S-2 configuration sampling in its
// finite-PEPS form; the strip contraction is that of the local energy): one workgroup per chain.
// The right environments of the strip's current configuration are built first (keeping Y1_c);
// then for px = 0 .. L-2 the proposal s' = P_p^t s, p = (px, py), is contracted as a window
// between the left environment E_px and Y1_{px+1}, accepted iff u < (Psi_py(s') / Psi_py(s))^2,
// and E_{px+1} = (E_px D_px) W_px U_px is formed for the configuration after the decision (the
// proposal's left half when accepted).  Blocks are gathered from theta and the chain's links, which
// are updated in place; t and u are the Philox draws of counter (chain, sweep, p, 1 / 2).
// links_pass = 1 (matter): the strip's link moves instead, by window column (see the loop), each
// decided against E_px and u of counter (chain, sweep, (L-1)^2 + link index, 2); E_{px+1} is formed
// after the window's last decision.
// BIG: fused bonds above 72, X and the staged site in the sample's global slot, as in k_strip.
template <bool BIG>
__global__ void __launch_bounds__(kT)
k_strip_mc(Dims d, int py, int sweep, uint64_t seed, uint64_t stream,
           const int* __restrict__ bond_all, const double* __restrict__ theta,
           const int64_t* __restrict__ site_offset, uint8_t* __restrict__ links,
           const uint8_t* __restrict__ valid, const double* __restrict__ down,
           const double* __restrict__ up, double* __restrict__ scratch, int32_t* __restrict__ accepted,
           int links_pass, double* __restrict__ wbig) {
  constexpr int ENV = BIG ? kEnvBig : kEnv;
  constexpr int XS = BIG ? kXBig : kX;
  constexpr int SITE = ENV / kMaxDk;
  constexpr int PPT = (XS / 8 + kT - 1) / kT;
  static_assert(!BIG || XS + SITE <= kBigSlot, "large-bond slot");
  __shared__ double lE[ENV];  // the environment stays in LDS (128 KB at the large size)
  __shared__ double lX[BIG ? 1 : XS];
  __shared__ double sW[64];
  __shared__ double sW2[64];
  __shared__ double lS[BIG ? 1 : SITE];
  __shared__ double sTb[4][16];
  __shared__ double sRed[kW];
  const int b = blockIdx.x;
  if (!valid[b]) return;
  double* const sE = lE;
  double* const sX = BIG ? wbig + (size_t)b * kBigSlot : lX;
  double* const sS = BIG ? sX + XS : lS;
  const int L = d.L, Dk = d.Dk, N = d.N;
  Strip S;
  S.L = L; S.N = N; S.Dk = Dk; S.py = py; S.B = gridDim.x;
  S.dD = py > 0 ? Dk : 1;
  S.dU = (py + 1 < L - 1) ? Dk : 1;
  S.site_stride = d.site_stride;
  S.bD = py >= 1 ? bond_all + (size_t)(py - 1) * (L + 1) : nullptr;
  S.bU = (py + 2 <= L - 1) ? bond_all + (size_t)(L - 3 - py) * (L + 1) : nullptr;
  const size_t rs = (size_t)gridDim.x * d.row_stride;
  S.Drow = S.bD ? down + (size_t)(py - 1) * rs + (size_t)b * d.row_stride : nullptr;
  S.Urow = S.bU ? up + (size_t)(L - 3 - py) * rs + (size_t)b * d.row_stride : nullptr;
  uint8_t* lk = links + (size_t)b * d.planes * L * L;
  const bool matter = d.matter != 0;
  double* gX1 = scratch + (size_t)b * ((size_t)2 * L * XS);
  double* gY1 = gX1 + (size_t)L * XS;
  const int dD = S.dD, dU = S.dU;

  // ---------------- right environments of the current strip ----------------
  if (threadIdx.x == 0) sE[0] = 1.0;
  __syncthreads();
  for (int c = L - 1; c >= 0; --c) {
    const int hl = S.hl(c), hr = S.hl(c + 1);
    const int cD = S.chiD(c), cDn = S.chiD(c + 1), cU = S.chiU(c), cUn = S.chiU(c + 1);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, c, py, plaquette_move(0, py, 0), sTb[0]);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, c, py + 1, plaquette_move(0, py, 0), sTb[1]);
    stage_site<SITE>(sS, S.Urow ? S.Urow + (size_t)c * S.site_stride : nullptr, cU * dU * cUn);
    __syncthreads();
    build_w(S, c, sTb[0], sTb[1], sW);
    {
      const int rows = cDn * hr * hr, cols = cU * dU;
      double* gy = gY1 + (size_t)c * XS;
      mfma_gemm(rows, cols, cUn, [&](int row, int bp) { return sE[(size_t)row * cUn + bp]; },
                [&](int bp, int col) { return sS[(size_t)col * cUn + bp]; },
                [&](int row, int col, double v) {
                  sX[(size_t)row * cols + col] = v;
                  gy[(size_t)row * cols + col] = v;
                });
    }
    __syncthreads();
    contract_right<true, PPT>(sX, sX, sW, cU, cDn, dU, dD, hl * hl * dD, hr * hr * dU);
    stage_site<SITE>(sS, S.Drow ? S.Drow + (size_t)c * S.site_stride : nullptr, cD * dD * cDn);
    __syncthreads();
    {
      const int cols = hl * hl * cU, K = cDn * dD;
      mfma_gemm(cD, cols, K,
                [&](int a, int k) { return sS[((size_t)a * dD + k % dD) * cDn + k / dD]; },
                [&](int k, int col) { return sX[((size_t)(k / dD) * cols + col) * dD + k % dD]; },
                [&](int a, int col, double v) { sE[(size_t)a * cols + col] = v; });
    }
    __syncthreads();
  }
  double psi = sE[0];  // the strip amplitude of the current configuration
  __syncthreads();

  // ---------------- left pass: proposals, decisions, left environments ----------------
  // X1_px = E_px D_px into its global slot (every left half of window px reads it)
  auto form_x1 = [&](int px) {
    const int c0 = px;
    const int hl = S.hl(c0), cD = S.chiD(c0), cDn = S.chiD(c0 + 1), cU = S.chiU(c0);
    double* gx = gX1 + (size_t)c0 * XS;
    stage_site<SITE>(sS, S.Drow ? S.Drow + (size_t)c0 * S.site_stride : nullptr, cD * dD * cDn);
    __syncthreads();
    const int rows = hl * hl * cU, cols = dD * cDn;
    mfma_gemm(rows, cols, cD, [&](int row, int a) { return sE[(size_t)a * rows + row]; },
              [&](int a, int col) { return sS[(size_t)a * cols + col]; },
              [&](int row, int col, double v) { gx[(size_t)row * cols + col] = v; });
  };
  // (X1_px W) U_px -> sE: the left half at cut px+1 for the column-px tensors in W
  auto left_half = [&](int px, const double* W) {
    const int c0 = px;
    const int hl = S.hl(c0), hr = S.hl(c0 + 1);
    const int cDn = S.chiD(c0 + 1), cU = S.chiU(c0), cUn = S.chiU(c0 + 1);
    contract_left<false, PPT>(gX1 + (size_t)c0 * XS, sX, W, cU, cDn, dD, hl * hl * dD, hr * hr * dU);
    stage_site<SITE>(sS, S.Urow ? S.Urow + (size_t)c0 * S.site_stride : nullptr, cU * dU * cUn);
    __syncthreads();
    const int rows = cDn * hr * hr, K = cU * dU;
    mfma_gemm(rows, cUn, K,
              [&](int row, int k) { return sX[((size_t)(k / dU) * rows + row) * dU + k % dU]; },
              [&](int k, int bp) { return sS[(size_t)k * cUn + bp]; },
              [&](int row, int bp, double v) { sE[(size_t)row * cUn + bp] = v; });
    __syncthreads();
  };
  // the window's strip amplitude: (Y1_{px+1} W2) D_{px+1} dotted with the left half in sE
  auto right_dot = [&](int px, const double* W2) -> double {
    const int c1 = px + 1;
    const int hl1 = S.hl(c1), hr1 = S.hl(c1 + 1);
    const int cD1 = S.chiD(c1), cDn1 = S.chiD(c1 + 1), cU1 = S.chiU(c1);
    contract_right<false, PPT>(gY1 + (size_t)c1 * XS, sX, W2, cU1, cDn1, dU, dD, hl1 * hl1 * dD,
                          hr1 * hr1 * dU);
    stage_site<SITE>(sS, S.Drow ? S.Drow + (size_t)c1 * S.site_stride : nullptr, cD1 * dD * cDn1);
    __syncthreads();
    const int cols = hl1 * hl1 * cU1, K = cDn1 * dD;
    double part_num = 0.0;
    mfma_gemm(cD1, cols, K,
              [&](int a, int k) { return sS[((size_t)a * dD + k % dD) * cDn1 + k / dD]; },
              [&](int k, int col) { return sX[((size_t)(k / dD) * cols + col) * dD + k % dD]; },
              [&](int a, int col, double v) { part_num += v * sE[(size_t)a * cols + col]; });
    return block_sum(part_num, sRed);  // same value in every thread
  };
  // W of columns px (sW) and px+1 (sW2) in the configuration mv leads to
  auto window_w = [&](int px, const Move& mv) {
    gather_block(theta, site_offset, lk, L, N, Dk, matter, px, py, mv, sTb[0]);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, px, py + 1, mv, sTb[1]);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, px + 1, py, mv, sTb[2]);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, px + 1, py + 1, mv, sTb[3]);
    __syncthreads();
    build_w(S, px, sTb[0], sTb[1], sW);
    build_w(S, px + 1, sTb[2], sTb[3], sW2);
    __syncthreads();
  };
  // E_{px+1} of the current configuration: (X1_px W_px) U_px
  auto advance = [&](int px) {
    gather_block(theta, site_offset, lk, L, N, Dk, matter, px, py, plaquette_move(0, py, 0), sTb[0]);
    gather_block(theta, site_offset, lk, L, N, Dk, matter, px, py + 1, plaquette_move(0, py, 0), sTb[1]);
    __syncthreads();
    build_w(S, px, sTb[0], sTb[1], sW);
    __syncthreads();
    left_half(px, sW);
  };
  int nacc = 0;
  if (threadIdx.x == 0) sE[0] = 1.0;
  __syncthreads();
  for (int px = 0; px < L - 1; ++px) {
    form_x1(px);
    if (links_pass == 0) {
      const int p = py * (L - 1) + px;
      const int t = 1 + (int)(philox_draw((uint64_t)b, (uint64_t)sweep, (uint64_t)p, 1, seed, stream) %
                              (uint64_t)(N - 1));
      const double u = philox_uniform(philox_draw((uint64_t)b, (uint64_t)sweep, (uint64_t)p, 2, seed, stream));
      // the proposal s' = P_p^t s = P_p^-(N-t) s: its left half into sE, then its ratio
      window_w(px, plaquette_move(px, py, N - t));
      left_half(px, sW);
      const double num = right_dot(px, sW2);
      const double ratio = num / psi;
      if (psi != 0.0 && u < ratio * ratio) {
        // s <- P_p^t s; sE already holds E_{px+1} of the new configuration
        if (threadIdx.x == 0) {
          uint8_t* h0 = lk + (size_t)py * L + px;             // h(px, py)
          uint8_t* h1 = lk + (size_t)(py + 1) * L + px;       // h(px, py+1)
          uint8_t* v0 = lk + (size_t)L * L + py * L + px;     // v(px, py)
          uint8_t* v1 = v0 + 1;                               // v(px+1, py)
          *h0 = (uint8_t)((*h0 + t) % N);
          *v1 = (uint8_t)((*v1 + t) % N);
          *h1 = (uint8_t)((*h1 + N - t) % N);
          *v0 = (uint8_t)((*v0 + N - t) % N);
        }
        psi = num;
        ++nacc;
        __syncthreads();
      } else {
        advance(px);
      }
    } else {
      // the link moves of window px (vertical (px, py), horizontal (px, py), in the last strip the
      // horizontal (px, L-1), and at px = L-2 the vertical (L-1, py)), each against E_px through
      // X1_px; a link whose ends hold equal occupations has no move
      for (int m = 0; m < 4; ++m) {
        int dir, x, y;
        if (m == 0) { dir = 1; x = px; y = py; }
        else if (m == 1) { dir = 0; x = px; y = py; }
        else if (m == 2) { if (py != L - 2) continue; dir = 0; x = px; y = L - 1; }
        else { if (px != L - 2) continue; dir = 1; x = L - 1; y = py; }
        uint8_t* occ = lk + (size_t)2 * L * L;
        const int ia = y * L + x, ib = (y + (dir == 1)) * L + x + (dir == 0);
        const int pa = occ[ia], pb = occ[ib];
        if (pa == pb) continue;  // same in every thread
        const int link = dir == 0 ? y * (L - 1) + x : L * (L - 1) + y * L + x;
        const uint64_t cnt = (uint64_t)((L - 1) * (L - 1) + link);
        const double u = philox_uniform(philox_draw((uint64_t)b, (uint64_t)sweep, cnt, 2, seed, stream));
        const int step = pb ? 1 : -1;
        window_w(px, hop_move(dir, x, y, step));
        left_half(px, sW);
        const double num = right_dot(px, sW2);
        const double ratio = num / psi;
        if (psi != 0.0 && u < ratio * ratio) {
          if (threadIdx.x == 0) {
            uint8_t* l = lk + (size_t)dir * L * L + y * L + x;
            *l = (uint8_t)((*l + (step > 0 ? 1 : N - 1)) % N);
            occ[ia] = (uint8_t)pb;
            occ[ib] = (uint8_t)pa;
          }
          psi = num;
          ++nacc;
        }
        __syncthreads();  // the chain's configuration as decided, before the next move reads it
      }
      advance(px);
    }
  }
  if (threadIdx.x == 0 && accepted) accepted[b] += nacc;
}

// E_loc = electric (+ mass) term + strip sums, and its magnitude M = sum_l |e[n_l]| (+ sum_x |m p_x|)
// + the strips' sums of |coefficient * ratio| (the size of the terms that E_loc adds up, against
// which its rounding and the mixed path's error are measured; NaN where E_loc is).
__global__ void k_eloc_final(Dims d, const uint8_t* __restrict__ links,
                             const uint8_t* __restrict__ valid, const double* __restrict__ elec,
                             double mass, const double* __restrict__ part, const double* __restrict__ pabs,
                             double* __restrict__ e_loc, double* __restrict__ scale) {
  __shared__ double red[4];
  __shared__ double reda[4];
  const int b = blockIdx.x;
  const int L = d.L;
  if (!valid[b]) {
    if (threadIdx.x == 0) {
      e_loc[b] = NAN;
      scale[b] = NAN;
    }
    return;
  }
  const uint8_t* lk = links + (size_t)b * d.planes * L * L;
  double acc = 0.0, aacc = 0.0;
  for (int i = threadIdx.x; i < 2 * L * L; i += blockDim.x) {
    const int dir = i / (L * L), y = (i / L) % L, x = i % L;
    if ((dir == 0 && x < L - 1) || (dir == 1 && y < L - 1)) {
      acc += elec[lk[i]];
      aacc += fabs(elec[lk[i]]);
    }
  }
  if (d.matter)  // mass term: m times the occupation of each vertex
    for (int i = threadIdx.x; i < L * L; i += blockDim.x) {
      const double v = mass * (double)lk[2 * L * L + i];
      acc += v;
      aacc += fabs(v);
    }
  acc = wave_sum(acc);
  aacc = wave_sum(aacc);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = acc;
    reda[threadIdx.x >> 6] = aacc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, sa = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      s += red[w];
      sa += reda[w];
    }
    for (int py = 0; py < L - 1; ++py) {
      s += part[(size_t)b * (L - 1) + py];
      sa += pabs[(size_t)b * (L - 1) + py];
    }
    e_loc[b] = s;
    scale[b] = sa;
  }
}

size_t strip_scratch_doubles(const Dims& d) { return (size_t)2 * d.L * (d.maxN > kMaxN ? kXBig : kX); }

hipError_t launch_mirror_proj(const Dims& d, const double* proj, const uint8_t* valid, int B,
                              double* fproj, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mirror_proj, dim3(B), dim3(256), 0, s, d, proj, valid, fproj);
  return hipGetLastError();
}

hipError_t launch_strip(const Dims& d, int py, const DeviceTables& t, const double* proj,
                        const double* theta, const uint8_t* links, const uint8_t* valid, int B,
                        const double* down, const double* up, const double* plaq, double hop,
                        double* scratch, double* part, double* pabs, hipStream_t s, double* wbig) {
  if (B == 0) return hipSuccess;
  // The strip contractions stay FP64 in the mixed path too: with FP32 arithmetic the strip
  // amplitudes of random-sign tensors cancel enough to move E/site by ~4e-2 relative.
  if (d.maxN > kMaxN) {
    if (d.Dk != 2 || d.maxN > kMaxNBig || !wbig) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_strip<true>, dim3(B), dim3(kT), 0, s, d, py, t.bond, proj, theta,
                       t.site_offset, links, valid, down, up, plaq, hop, scratch, part, pabs, wbig);
  } else {
    hipLaunchKernelGGL(k_strip<false>, dim3(B), dim3(kT), 0, s, d, py, t.bond, proj, theta,
                       t.site_offset, links, valid, down, up, plaq, hop, scratch, part, pabs, wbig);
  }
  return hipGetLastError();
}

hipError_t launch_strip_mc(const Dims& d, int py, int sweep, uint64_t seed, uint64_t stream,
                           const DeviceTables& t, const double* theta, uint8_t* links,
                           const uint8_t* valid, int B, const double* down, const double* up,
                           double* scratch, int32_t* accepted, int links_pass, hipStream_t s,
                           double* wbig) {
  if (B == 0 || d.N < 2) return hipSuccess;
  if (d.maxN > kMaxN) {
    if (d.Dk != 2 || d.maxN > kMaxNBig || !wbig) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_strip_mc<true>, dim3(B), dim3(kT), 0, s, d, py, sweep, seed, stream, t.bond, theta,
                       t.site_offset, links, valid, down, up, scratch, accepted, links_pass, wbig);
  } else {
    hipLaunchKernelGGL(k_strip_mc<false>, dim3(B), dim3(kT), 0, s, d, py, sweep, seed, stream, t.bond, theta,
                       t.site_offset, links, valid, down, up, scratch, accepted, links_pass, wbig);
  }
  return hipGetLastError();
}

hipError_t launch_eloc_final(const Dims& d, const uint8_t* links, const uint8_t* valid, int B,
                             const double* elec, double mass, const double* part, const double* pabs,
                             double* e_loc, double* scale, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eloc_final, dim3(B), dim3(256), 0, s, d, links, valid, elec, mass, part, pabs,
                     e_loc, scale);
  return hipGetLastError();
}

}  // namespace gipeps
