// Hand-written adjoint of the boundary-MPS amplitude: O_k(s) = d ln|Psi(s)| / d theta_k (SM S-1,
// definition of O_m, for real tensors), the exact derivative of every step of the contraction as
// it is defined (row application, QR sweep, truncated SVD sweep, normalisation, close).
//
// Reverse order, per sample (one workgroup per sample):
//   k_adj_close : c = <row_{L-1}|D_{L-2}>; seeds dlnPsi/dD_{L-2} = (dc/dD)/c and the top row's O.
//   per row y = L-2 .. 1, after the row has been recomputed with its factorisations taped:
//     k_adj_svd : normalisation and right-to-left SVD sweep in reverse (sites 0 .. L-1), giving
//                 Qbar_c of every QR factor and Xbar_{L-1};
//     k_adj_qr  : left-to-right QR sweep in reverse (sites L-1 .. 0): QR backward and the row
//                 application backward, giving dlnPsi/dD_{y-1} and row y's O.
//   k_adj_row0  : row 0 is D_0 itself.
//   k_vjp       : sum_b w_b O_b scattered into the parameter layout, per site in a fixed sample
//                 order (deterministic, no atomics).
//
// Backward formulas used (derived from the first-order perturbation of each factorisation):
//   * truncated SVD Theta = U S V^T (thin, p = min(m, n) triplets, the first k kept; gU, gS, gV
//     zero outside the kept ones):
//       Thetabar = U [ (skew(U^T gU) o F) S + S (skew(V^T gV) o F) + diag(gS) ] V^T
//                  + (I - U U^T) gU S^-1 V^T + U S^-1 gV^T (I - V V^T),
//     skew(X) = X - X^T, F_jk = 1 / (s_k^2 - s_j^2) (j != k; taken as 0 where s_k = s_j), the
//     kept-discarded pairs included.  One of the two projector terms vanishes because one factor
//     is square.  Requires the kept singular values to be nonzero.
//   * QR X = Q R (Householder branch), k = min(m, n), R = [R1 | R2] with R1 k x k:
//       Qbar' = Qbar + Q R2 R2bar^T,  M = R1 R1bar^T - Qbar'^T Q,
//       Xbar[:, :k] = (Qbar' + Q sym(M)) R1^-T,  Xbar[:, k:] = Q R2bar,
//     sym(M) = the symmetric matrix whose lower triangle is that of M.  Requires R1 invertible.
//   * normalisation psi_0 = Theta_0 / nu, ln nu added to ln|Psi|:
//       Thetabar_0 = (psibar_0 + psi_0 (1 - <psi_0, psibar_0>)) / nu.
#include <algorithm>

#include "dev_common.h"
#include "internal.h"

namespace gipeps {

namespace {

constexpr int kT = 512;

// Accessors of one taped SVD (site c >= 1): U (m x p), V (n x p), sorted singular values.
template <int MAXN>
struct SvdTape {
  using TS = TapeSlot<MAXN>;
  const double* slot;
  const double* sig;  // LDS copy, descending
  int nc, trans;      // p = nc = min(m, n)
  __device__ double U(int i, int a) const { return slot[TS::U + (size_t)a * MAXN + i]; }
  __device__ double V(int col, int a) const { return slot[TS::V + (size_t)a * MAXN + col]; }
  __device__ double G(int i, int a) const { return U(i, a) * sig[a]; }  // G = U S
};

// Stage the singular values of a taped SVD into LDS.
template <int MAXN>
__device__ SvdTape<MAXN> load_svd(const double* slot, int m, int n, double* sSig) {
  using TS = TapeSlot<MAXN>;
  SvdTape<MAXN> t;
  t.slot = slot;
  t.trans = slot[TS::F] != 0.0;
  t.nc = m < n ? m : n;
  for (int a = threadIdx.x; a < t.nc; a += kT) sSig[a] = slot[TS::S + a];
  __syncthreads();
  t.sig = sSig;
  return t;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Close in reverse: psibar_{L-2} = (dc/dD_{L-2}) / c and O of row L-1 = (dc/dT) / c.
// ---------------------------------------------------------------------------------------------
// E: environment entries per cut (bond * horizontal dimension), 72 or 128 (large bonds)
template <int E>
__global__ void k_adj_close(Dims d, const int* __restrict__ bond_last, const double* __restrict__ proj,
                            const uint8_t* __restrict__ valid, const double* __restrict__ last_row,
                            double* __restrict__ psibar, double* __restrict__ O) {
  __shared__ double e[65 * E];     // left environments e_0 .. e_L (L <= 64)
  __shared__ double f0[E], f1[E];  // right environment at the current cut
  const int b = blockIdx.x;
  if (!valid[b]) return;
  const int L = d.L, Dk = d.Dk;
  const double* pb = proj + ((size_t)b * d.n_sites + (size_t)(L - 1) * L) * d.P4;
  const double* mp = last_row + (size_t)b * d.row_stride;
  auto hl = [&](int c) { return (c > 0 && c < L) ? Dk : 1; };
  if (threadIdx.x == 0) {
    e[0] = 1.0;
    f1[0] = 1.0;
  }
  __syncthreads();
  for (int c = 0; c < L; ++c) {
    const int dl = hl(c), dr = hl(c + 1), bc = bond_last[c], bn = bond_last[c + 1];
    const double* Bs = mp + (size_t)c * d.site_stride;
    const double* T = pb + (size_t)c * d.P4;  // T[l][rr][dd], du = 1
    for (int idx = threadIdx.x; idx < bn * dr; idx += blockDim.x) {
      const int ap = idx / dr, rr = idx % dr;
      double acc = 0.0;
      for (int a = 0; a < bc; ++a)
        for (int l = 0; l < dl; ++l)
          for (int dd = 0; dd < Dk; ++dd)
            acc += e[(size_t)c * E + a * dl + l] * Bs[(a * Dk + dd) * bn + ap] * T[(l * dr + rr) * Dk + dd];
      e[(size_t)(c + 1) * E + idx] = acc;
    }
    __syncthreads();
  }
  const double inv = 1.0 / e[(size_t)L * E];
  double* pbar = psibar + (size_t)b * d.row_stride;
  double* Ob = O + ((size_t)b * d.n_sites + (size_t)(L - 1) * L) * d.P4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* fin = f1;   // f_{c+1}
  double* fout = f0;  // f_c
  for (int c = L - 1; c >= 0; --c) {
    const int dl = hl(c), dr = hl(c + 1), bc = bond_last[c], bn = bond_last[c + 1];
    const double* Bs = mp + (size_t)c * d.site_stride;
    const double* T = pb + (size_t)c * d.P4;
    const double* ec = e + (size_t)c * E;
    double* Pb = pbar + (size_t)c * d.site_stride;
    for (int idx = threadIdx.x; idx < bc * Dk * bn; idx += blockDim.x) {
      const int a = idx / (Dk * bn), dd = (idx / bn) % Dk, ap = idx % bn;
      double acc = 0.0;
      for (int l = 0; l < dl; ++l)
        for (int rr = 0; rr < dr; ++rr)
          acc += ec[a * dl + l] * T[(l * dr + rr) * Dk + dd] * fin[ap * dr + rr];
      Pb[idx] = acc * inv;
    }
    const int nent = dl * dr * Dk;  // O of the top-row block T[l][rr][dd]: one wave per entry
    for (int ent = wave; ent < nent; ent += nw) {
      const int l = ent / (dr * Dk), rr = (ent / Dk) % dr, dd = ent % Dk;
      double acc = 0.0;
      for (int idx = lane; idx < bc * bn; idx += 64) {
        const int a = idx / bn, ap = idx % bn;
        acc += ec[a * dl + l] * Bs[(a * Dk + dd) * bn + ap] * fin[ap * dr + rr];
      }
      acc = wave_sum(acc);
      if (lane == 0) Ob[(size_t)c * d.P4 + ent] = acc * inv;
    }
    for (int idx = threadIdx.x; idx < bc * dl; idx += blockDim.x) {
      const int a = idx / dl, l = idx % dl;
      double acc = 0.0;
      for (int ap = 0; ap < bn; ++ap)
        for (int rr = 0; rr < dr; ++rr)
          for (int dd = 0; dd < Dk; ++dd)
            acc += Bs[(a * Dk + dd) * bn + ap] * T[(l * dr + rr) * Dk + dd] * fin[ap * dr + rr];
      fout[idx] = acc;
    }
    __syncthreads();
    double* tmp = fin;
    fin = fout;
    fout = tmp;
  }
}

// Row 0 is D_0 itself (site [l][u][r] from T[l][r][0][u]).
__global__ void k_adj_row0(Dims d, const uint8_t* __restrict__ valid, const double* __restrict__ psibar,
                           double* __restrict__ O) {
  const int b = blockIdx.x;
  if (!valid[b]) return;
  const int L = d.L, Dk = d.Dk;
  const double* pbar = psibar + (size_t)b * d.row_stride;
  double* Ob = O + (size_t)b * d.n_sites * d.P4;
  for (int c = 0; c < L; ++c) {
    const int dl = c > 0 ? Dk : 1, dr = c < L - 1 ? Dk : 1, du = Dk;
    for (int i = threadIdx.x; i < dl * du * dr; i += blockDim.x) {
      const int l = i / (du * dr), u = (i / dr) % du, r = i % dr;
      Ob[(size_t)c * d.P4 + (l * dr + r) * du + u] = pbar[(size_t)c * d.site_stride + i];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Normalisation and SVD sweep in reverse for row y.
// ---------------------------------------------------------------------------------------------
template <int MAXN, int DK>
__global__ void __launch_bounds__(kT)
k_adj_svd(Dims d, const int* __restrict__ bond_all, const int* __restrict__ qrk_all, int y,
          const uint8_t* __restrict__ valid, const double* __restrict__ cur_row,
          const double* __restrict__ tape, const double* __restrict__ qscr,
          const double* __restrict__ psibar_in, double* __restrict__ qbar, double* __restrict__ xbar,
          double* __restrict__ wbig) {
  constexpr int MAXM = MAXN * DK;
  constexpr int KD = MAXN / DK;  // largest kept bond
  // large bonds: three of the working matrices in the sample's global slot (wbig), the core /
  // Theta-bar and the staging in LDS
  constexpr bool BIG = MAXN > kMaxN;
  using TS = TapeSlot<MAXN>;
  constexpr int MSZ = (2 * MAXN * KD > MAXN * MAXN) ? 2 * MAXN * KD : MAXN * MAXN;
  static_assert(!BIG || 2 * MAXN * KD + MSZ <= kBigSlot, "large-bond slot");
  __shared__ double lGb[BIG ? 1 : MAXN * KD];   // Gbar_c [i][a], ld KD
  __shared__ double lGV[BIG ? 1 : MAXN * KD];   // gV [col][a], ld KD
  __shared__ double lM[BIG ? 1 : MSZ];          // M1 | M2 (p x KD each), later T1 / T2
  __shared__ double lC[MAXN * MAXN];            // core C' / C'', later Thetabar (m x n, ld n): LDS at every size
  __shared__ double sSig[MAXN];
  __shared__ double sGS[MAXN];
  __shared__ double sRed[kT / 64];
  // products with the tape (U, V) and Q: K-chunks staged through sBuf, on the matrix cores
  constexpr int KCH = 16, SPT = (MAXN * KCH + kT - 1) / kT;
  constexpr int QT = ((MAXM + 15) / 16 * ((MAXN + 15) / 16) + kT / 64 - 1) / (kT / 64);
  __shared__ double sBuf[MAXN * KCH];
  const int b = blockIdx.x;
  if (!valid[b]) return;
  double* const slot = BIG ? wbig + (size_t)b * kBigSlot : nullptr;
  double* const sGb = BIG ? slot : lGb;
  double* const sGV = BIG ? slot + MAXN * KD : lGV;
  double* const sM = BIG ? slot + 2 * MAXN * KD : lM;
  double* const sC = lC;
  const int L = d.L, Dk = DK;
  const int* bnew = bond_all + (size_t)y * (L + 1);
  const int* qrk = qrk_all + (size_t)y * L;
  const double* tp = tape + (size_t)b * L * TS::size;
  const double* qs = qscr + (size_t)b * L * (MAXM * MAXN);
  double* qb = qbar + (size_t)b * L * (MAXM * MAXN);
  const double* psi = cur_row + (size_t)b * d.row_stride;
  const double* pbar = psibar_in + (size_t)b * d.row_stride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // ---- site 0: normalisation, Theta_0 = Q_0 G_1 ----
  {
    const int chi1 = bnew[1], n0 = Dk * chi1, r0 = qrk[0];
    const double nu = tp[TS::F + 1];
    double part = 0.0;
    for (int i = threadIdx.x; i < n0; i += kT) part += psi[i] * pbar[i];
    const double dot = block_sum(part, sRed);
    for (int i = threadIdx.x; i < n0; i += kT) sC[i] = (pbar[i] + psi[i] * (1.0 - dot)) / nu;
    const int m1 = qrk[0], n1 = Dk * ((L - 1 == 1) ? 1 : bnew[2]);
    SvdTape<MAXN> t1 = load_svd<MAXN>(tp + (size_t)1 * TS::size, m1, n1, sSig);
    // Qbar_0[(u)][t] = sum_j Thetabar_0[u][j] G_1[t][j];  Gbar_1[t][j] = sum_u Q_0[u][t] Thetabar_0[u][j]
    for (int idx = threadIdx.x; idx < Dk * r0; idx += kT) {
      const int t = idx / Dk, u = idx % Dk;
      double acc = 0.0;
      for (int j = 0; j < chi1; ++j) acc += sC[u * chi1 + j] * t1.G(t, j);
      qb[idx] = acc;
    }
    for (int idx = threadIdx.x; idx < r0 * chi1; idx += kT) {
      const int t = idx / chi1, j = idx % chi1;
      double acc = 0.0;
      for (int u = 0; u < Dk; ++u) acc += qs[(size_t)t * Dk + u] * sC[u * chi1 + j];
      sGb[t * KD + j] = acc;
    }
    __syncthreads();
  }

  // ---- sites 1 .. L-1: truncated SVD backward ----
  for (int c = 1; c < L; ++c) {
    const int m = qrk[c - 1];
    const int chin = (c == L - 1) ? 1 : bnew[c + 1];
    const int n = Dk * chin;
    const int kk = bnew[c];
    SvdTape<MAXN> t = load_svd<MAXN>(tp + (size_t)c * TS::size, m, n, sSig);
    const int p = t.nc;  // = min(m, n)
    // gS[a] = sum_i U[i][a] Gbar[i][a];  gV[col][a] = psibar_c[a][col]
    for (int a = wave; a < kk; a += kT / 64) {
      double acc = 0.0;
      for (int i = lane; i < m; i += 64) acc += t.U(i, a) * sGb[i * KD + a];
      acc = wave_sum(acc);
      if (lane == 0) sGS[a] = acc;
    }
    const double* pbc = pbar + (size_t)c * d.site_stride;
    for (int idx = threadIdx.x; idx < kk * n; idx += kT) {
      const int a = idx / n, col = idx % n;
      sGV[col * KD + a] = pbc[idx];
    }
    __syncthreads();
    // M1[j][a] = s_a sum_i U[i][j] Gbar[i][a];  M2[j][a] = sum_col V[col][j] gV[col][a]
    double* M1 = sM;
    double* M2 = sM + p * KD;
    mfma_gemm_staged<QT, KCH, SPT, true>(
        p, kk, m, [&](int j, int i) { return t.U(i, j); }, [&](int i, int a) { return sGb[i * KD + a]; }, sBuf,
        [&](int j, int a, double v) { M1[j * KD + a] = v * t.sig[a]; });
    mfma_gemm_staged<QT, KCH, SPT, true>(
        p, kk, n, [&](int j, int col) { return t.V(col, j); }, [&](int col, int a) { return sGV[col * KD + a]; },
        sBuf, [&](int j, int a, double v) { M2[j * KD + a] = v; });
    __syncthreads();
    // core C (p x p), with the projector term folded in (C' or C'')
    for (int idx = threadIdx.x; idx < p * p; idx += kT) {
      const int j = idx / p, k = idx % p;
      const double sj = t.sig[j], sk = t.sig[k];
      double v;
      if (j == k) {
        v = (j < kk) ? sGS[j] : 0.0;
      } else {
        const double m1jk = (k < kk) ? M1[j * KD + k] : 0.0, m1kj = (j < kk) ? M1[k * KD + j] : 0.0;
        const double m2jk = (k < kk) ? M2[j * KD + k] : 0.0, m2kj = (j < kk) ? M2[k * KD + j] : 0.0;
        const double den = sk * sk - sj * sj;
        const double num = (m1jk - m1kj) * sk + sj * (m2jk - m2kj);
        v = (den != 0.0) ? num / den : 0.0;
      }
      if (!t.trans && k < kk && sk > 0.0) v -= M1[j * KD + k] / sk;
      if (t.trans && j < kk && sj > 0.0) v -= M2[k * KD + j] / sj;
      sC[idx] = v;
    }
    __syncthreads();
    if (!t.trans) {
      // T1 (m x p) = U C' + [Gbar | 0];  Thetabar = T1 V^T
      mfma_gemm_staged<QT, KCH, SPT, true>(
          m, p, p, [&](int i, int j) { return t.U(i, j); }, [&](int j, int a) { return sC[j * p + a]; }, sBuf,
          [&](int i, int a, double v) { sM[i * p + a] = v + ((a < kk) ? sGb[i * KD + a] : 0.0); });
      __syncthreads();
      mfma_gemm_staged<QT, KCH, SPT, false>(
          m, n, p, [&](int col, int a) { return t.V(col, a); }, [&](int i, int a) { return sM[i * p + a]; }, sBuf,
          [&](int i, int col, double v) { sC[i * n + col] = v; });
    } else {
      // T2 (p x n) = C'' V^T + S^-1 gV^T;  Thetabar = U T2
      mfma_gemm_staged<QT, KCH, SPT, false>(
          p, n, p, [&](int col, int k) { return t.V(col, k); }, [&](int a, int k) { return sC[a * p + k]; }, sBuf,
          [&](int a, int col, double v) {
            const double sa = t.sig[a];
            sM[a * n + col] = v + ((a < kk && sa > 0.0) ? sGV[col * KD + a] / sa : 0.0);
          });
      __syncthreads();
      mfma_gemm_staged<QT, KCH, SPT, true>(
          m, n, p, [&](int i, int a) { return t.U(i, a); }, [&](int a, int col) { return sM[a * n + col]; }, sBuf,
          [&](int i, int col, double v) { sC[i * n + col] = v; });
    }
    __syncthreads();
    if (c < L - 1) {
      // Theta_c[i][(u,j)] = sum_t Q_c[(i,u)][t] G_{c+1}[t][j]
      const int rc = qrk[c], mq = m * Dk;
      const int m2 = rc, n2 = Dk * ((c + 1 == L - 1) ? 1 : bnew[c + 2]);
      SvdTape<MAXN> t2 = load_svd<MAXN>(tp + (size_t)(c + 1) * TS::size, m2, n2, sSig);
      const double* Qc = qs + (size_t)c * (MAXM * MAXN);
      double* Qb = qb + (size_t)c * (MAXM * MAXN);
      auto th = [&](int row, int j) { return sC[(row / Dk) * n + (row % Dk) * chin + j]; };
      mfma_gemm_staged<QT, KCH, SPT, false>(
          mq, rc, chin, [&](int tt, int j) { return t2.G(tt, j); }, th, sBuf,
          [&](int row, int tt, double v) { Qb[(size_t)tt * mq + row] = v; });  // ld mq
      mfma_gemm_staged<QT, KCH, SPT, true>(
          rc, chin, mq, [&](int tt, int row) { return Qc[(size_t)tt * mq + row]; }, th, sBuf,
          [&](int tt, int j, double v) { sGb[tt * KD + j] = v; });
    } else {
      double* xb = xbar + (size_t)b * MAXM;
      for (int idx = threadIdx.x; idx < m * Dk; idx += kT) xb[idx] = sC[(idx / Dk) * n + idx % Dk];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// QR sweep and row application in reverse for row y: psibar_{y-1} and O of row y.
// ---------------------------------------------------------------------------------------------
template <int MAXN, int DK>
__global__ void __launch_bounds__(kT)
k_adj_qr(Dims d, const int* __restrict__ bond_all, const int* __restrict__ qrk_all, int y,
         const double* __restrict__ proj, const uint8_t* __restrict__ valid,
         const double* __restrict__ prev_row, const double* __restrict__ qscr,
         const double* __restrict__ tape, const double* __restrict__ qbar,
         const double* __restrict__ xbar, double* __restrict__ psibar_out, double* __restrict__ O,
         double* __restrict__ wbig) {
  constexpr int MAXM = MAXN * DK;
  // 16 x 16 matrix-core tiles per wave of the products with up to MAXM x MAXN outputs
  constexpr int QT = ((MAXM + 15) / 16 * ((MAXN + 15) / 16) + kT / 64 - 1) / (kT / 64);
  // large bonds: Xbar and Z in the sample's global slot (wbig), Rbar in LDS, B read from the
  // boundary row, sB only stages the factors of the products
  constexpr bool BIG = MAXN > kMaxN;
  // chunks of up to MAXM rows of the global factors staged through sB (8 rows at the large size,
  // where R-bar takes most of the LDS)
  constexpr int KCH = BIG ? 8 : ((MAXN / (DK * DK)) / 4 * 4 < 16 ? (MAXN / (DK * DK)) / 4 * 4 : 16);
  constexpr int SPT = (MAXM * KCH + kT - 1) / kT;
  constexpr int SBSZ = BIG ? MAXM * KCH : MAXN * MAXN / DK;
  static_assert(KCH >= 4 && MAXM * KCH <= SBSZ, "staging chunk fits sB");
  static_assert(!BIG || 2 * MAXM * MAXN <= kBigSlot, "large-bond slot");
  using TS = TapeSlot<MAXN>;
  __shared__ double lXb[BIG ? 1 : MAXM * MAXN];  // Xbar_c (m x n, column-major ld m)
  __shared__ double lRb[MAXN * MAXN];  // Rbar_{c-1} (column-major ld MAXN), later M (ld MAXN): LDS at every size
  __shared__ double sB[SBSZ];
  __shared__ double sT[DK * DK * DK * DK];
  __shared__ double sRed[16 * (kT / 64)];
  const int b = blockIdx.x;
  if (!valid[b]) return;
  double* const slot = BIG ? wbig + (size_t)b * kBigSlot : nullptr;
  double* const sXb = BIG ? slot : lXb;
  double* const sRb = lRb;
  double* const sZ = BIG ? slot + MAXM * MAXN : lXb;  // Z (over Xbar when in LDS)
  const int L = d.L, Dk = DK;
  const int* bprev = bond_all + (size_t)(y - 1) * (L + 1);
  const int* qrk = qrk_all + (size_t)y * L;
  const double* tp = tape + (size_t)b * L * TS::size;
  const double* qs = qscr + (size_t)b * L * (MAXM * MAXN);
  const double* qb = qbar + (size_t)b * L * (MAXM * MAXN);
  const double* prev = prev_row + (size_t)b * d.row_stride;
  double* pout = psibar_out + (size_t)b * d.row_stride;
  const double* pb = proj + ((size_t)b * d.n_sites + (size_t)y * L) * d.P4;
  double* Ob = O + ((size_t)b * d.n_sites + (size_t)y * L) * d.P4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  {
    const int m = qrk[L - 2] * Dk;
    const double* xb = xbar + (size_t)b * MAXM;
    for (int i = threadIdx.x; i < m; i += kT) sXb[i] = xb[i];
  }
  __syncthreads();
  for (int c = L - 1; c >= 0; --c) {
    const int dl = c > 0 ? Dk : 1, dr = c < L - 1 ? Dk : 1;
    const int bc = bprev[c], bn = bprev[c + 1];
    const int r = (c == 0) ? 1 : qrk[c - 1];
    const int m = r * Dk, n = bn * dr;
    const int mc = bc * dl;  // columns of R_{c-1}
    const double* Bs = prev + (size_t)c * d.site_stride;
    if constexpr (!BIG)
      for (int i = threadIdx.x; i < bc * Dk * bn; i += kT) sB[i] = Bs[i];
    auto Bv = [&](int idx) -> double { return BIG ? Bs[idx] : sB[idx]; };  // B[a][dd][a'] flat
    for (int i = threadIdx.x; i < dl * dr * Dk * Dk; i += kT) sT[i] = pb[(size_t)c * d.P4 + i];
    // R_{c-1} (r x mc, ld MAXN) staged in sRb until the products that read it are done
    if (c >= 1) {
      const double* Rt = tp + (size_t)(c - 1) * TS::size + TS::R;
      if constexpr (BIG) {
        for (int idx = threadIdx.x; idx < mc * MAXN; idx += kT) sRb[idx] = (idx % MAXN < r) ? Rt[idx] : 0.0;
      } else {
        constexpr int RPT = (MAXN * MAXN + kT - 1) / kT;
        double st[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int idx = threadIdx.x + q * kT;
          st[q] = (idx < mc * MAXN && idx % MAXN < r) ? Rt[idx] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int idx = threadIdx.x + q * kT;
          if (idx < mc * MAXN) sRb[idx] = st[q];
        }
      }
    } else if (threadIdx.x == 0) {
      sRb[0] = 1.0;
    }
    __syncthreads();
    auto R = [&](int i, int j) -> double { return sRb[(size_t)j * MAXN + i]; };
    // ---- O of row y, site c: Tbar[l][rr][dd][u] = sum_{i,a,a'} Xbar[(i,u),(a',rr)] R[i][a dl+l] B[a][dd][a']
    {
      // 2 x 2 tiles of (i, a'): Y[i][l][dd][a'] = sum_a R[i][a dl+l] B[a][dd][a'] kept in registers
      // (half an LDS load per multiply-add), then contracted with the four Xbar entries of each
      // (i, a') into the 16 Tbar partial sums
      double acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0;
      const int ti = (r + 1) / 2, ta = (bn + 1) / 2;
      for (int t = threadIdx.x; t < ti * ta; t += kT) {
        const int i0 = (t / ta) * 2, a0 = (t % ta) * 2;
        double pv[2][2][2][DK];
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int l = 0; l < 2; ++l)
#pragma unroll
              for (int dd = 0; dd < DK; ++dd) pv[ii][jj][l][dd] = 0.0;
        for (int a = 0; a < bc; ++a) {
          double rv[2][2], bv[2][DK];
#pragma unroll
          for (int ii = 0; ii < 2; ++ii)
#pragma unroll
            for (int l = 0; l < 2; ++l)
              rv[ii][l] = (i0 + ii < r && l < dl) ? R(i0 + ii, a * dl + l) : 0.0;
#pragma unroll
          for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int dd = 0; dd < DK; ++dd)
              bv[jj][dd] = (a0 + jj < bn) ? Bv((a * DK + dd) * bn + a0 + jj) : 0.0;
#pragma unroll
          for (int ii = 0; ii < 2; ++ii)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
#pragma unroll
              for (int l = 0; l < 2; ++l)
#pragma unroll
                for (int dd = 0; dd < DK; ++dd) pv[ii][jj][l][dd] += rv[ii][l] * bv[jj][dd];
        }
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const int i = i0 + ii, ap = a0 + jj;
            if (i >= r || ap >= bn) continue;
#pragma unroll
            for (int l = 0; l < 2; ++l)
#pragma unroll
              for (int rr = 0; rr < 2; ++rr) {
                if (l >= dl || rr >= dr) continue;
#pragma unroll
                for (int dd = 0; dd < DK; ++dd)
#pragma unroll
                  for (int u = 0; u < DK; ++u)
                    acc[((l * dr + rr) * DK + dd) * DK + u] +=
                        sXb[(size_t)(ap * dr + rr) * m + i * DK + u] * pv[ii][jj][l][dd];
              }
          }
      }
      const int nent = dl * dr * Dk * Dk;
      for (int q = 0; q < nent; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) sRed[q * (kT / 64) + wave] = v;
      }
      __syncthreads();
      for (int q = threadIdx.x; q < nent; q += kT) {
        double s = 0.0;
        for (int w = 0; w < kT / 64; ++w) s += sRed[q * (kT / 64) + w];
        Ob[(size_t)c * d.P4 + q] = s;
      }
    }
    // ---- Z[(i,l)][(dd,a')] = sum_{u,rr} Xbar[(i,u),(a',rr)] T[l][rr][dd][u], into sZ (in place
    // over Xbar when both are in LDS)
    const int nz = Dk * bn;  // row length of Z
    {
      auto z_entry = [&](int idx) -> double {
        const int il = idx / nz, col = idx % nz;
        const int i = il / dl, l = il % dl, dd = col / bn, ap = col % bn;
        double z = 0.0;
        for (int u = 0; u < Dk; ++u)
          for (int rr = 0; rr < dr; ++rr)
            z += sXb[(size_t)(ap * dr + rr) * m + i * Dk + u] * sT[((l * dr + rr) * Dk + dd) * Dk + u];
        return z;
      };
      if constexpr (BIG) {
        for (int idx = threadIdx.x; idx < r * dl * nz; idx += kT) sZ[idx] = z_entry(idx);
      } else {
        constexpr int ZPT = (MAXM * MAXN + kT - 1) / kT;
        double zr[ZPT];
#pragma unroll
        for (int q = 0; q < ZPT; ++q) {
          const int idx = threadIdx.x + q * kT;
          zr[q] = (idx < r * dl * nz) ? z_entry(idx) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < ZPT; ++q) {
          const int idx = threadIdx.x + q * kT;
          if (idx < r * dl * nz) sZ[idx] = zr[q];
        }
      }
      __syncthreads();
    }
    // ---- Bbar[a][(dd,a')] = sum_{(i,l)} R[i][a dl+l] Z[(i,l)][(dd,a')]
    double* Pb = pout + (size_t)c * d.site_stride;
    mfma_gemm(bc, nz, r * dl, [&](int a, int k) { return R(k / dl, a * dl + k % dl); },
                    [&](int k, int col) { return sZ[(size_t)k * nz + col]; },
                    [&](int a, int col, double v) { Pb[(size_t)a * nz + col] = v; });
    if (c == 0) break;
    __syncthreads();  // R no longer read: sRb takes Rbar
    // ---- Rbar[i][a dl+l] = sum_{(dd,a')} Z[(i,l)][(dd,a')] B[a][(dd,a')]
    mfma_gemm(r * dl, bc, nz, [&](int il, int k) { return sZ[(size_t)il * nz + k]; },
                    [&](int k, int a) { return Bv(a * nz + k); },
                    [&](int il, int a, double v) { sRb[(size_t)(a * dl + il % dl) * MAXN + il / dl] = v; });
    __syncthreads();
    // ---- QR backward of X_{c-1} = Q R (m2 x n2, k2 = min) -> Xbar_{c-1} in sXb (ld m2)
    const int r2 = (c - 1 == 0) ? 1 : qrk[c - 2];
    const int m2 = r2 * Dk, n2 = mc, k2 = qrk[c - 1];
    const double* Q = qs + (size_t)(c - 1) * (MAXM * MAXN);    // m2 x k2, ld m2
    const double* Qb = qb + (size_t)(c - 1) * (MAXM * MAXN);   // m2 x k2, ld m2
    const double* Rq = tp + (size_t)(c - 1) * TS::size + TS::R;  // k2 x n2, ld MAXN
    auto RQ = [&](int i, int j) -> double { return Rq[(size_t)j * MAXN + i]; };
    // Qbar' = Qbar + Q R2 R2bar^T (cols < k2) and Xbar[:, k2:] = Q R2bar; all loads of a thread
    // are issued before its stores
    if constexpr (BIG) {  // Qbar (m2 x k2) into sXb[:, :k2]
      for (int idx = threadIdx.x; idx < m2 * k2; idx += kT) sXb[idx] = Qb[idx];
    } else {  // Qbar (m2 x k2) into sXb[:, :k2]; loads at clamped addresses, all in flight at once
      constexpr int QPT = (MAXM * MAXN + kT - 1) / kT;
      double st[QPT];
      const int tot = m2 * k2;
#pragma unroll
      for (int q = 0; q < QPT; ++q) {
        const int idx = threadIdx.x + q * kT;
        st[q] = Qb[idx < tot ? idx : tot - 1];
      }
#pragma unroll
      for (int q = 0; q < QPT; ++q) {
        const int idx = threadIdx.x + q * kT;
        if (idx < tot) sXb[idx] = st[q];
      }
    }
    if (n2 > k2) {
      // wide X (m2 = k2 < n2): R = [R1 | R2].  Qbar' = Qbar + Q (R2 R2bar^T), Xbar[:, k2:] = Q R2bar,
      // with T = R2 R2bar^T (k2 x k2) parked behind Xbar in sXb (m2 n2 + k2^2 <= 2 n2^2 fits)
      const int w2 = n2 - k2;
      double* T = sXb + (size_t)m2 * n2;
      tile_gemm<4, 4>(k2, k2, w2, [&](int a, int kk) { return RQ(a, k2 + kk); },
                      [&](int kk, int bb) { return sRb[(size_t)(k2 + kk) * MAXN + bb]; },
                      [&](int a, int bb, double v) { T[(size_t)bb * k2 + a] = v; });
      __syncthreads();
      mfma_gemm_staged<QT, KCH, SPT, true>(
          m2, k2, k2, [&](int i, int t) { return Q[(size_t)t * m2 + i]; },
          [&](int t, int j) { return T[(size_t)j * k2 + t]; }, sB,
          [&](int i, int j, double v) { sXb[(size_t)j * m2 + i] += v; });
      mfma_gemm_staged<QT, KCH, SPT, true>(
          m2, w2, k2, [&](int i, int t) { return Q[(size_t)t * m2 + i]; },
          [&](int t, int jj) { return sRb[(size_t)(k2 + jj) * MAXN + t]; }, sB,
          [&](int i, int jj, double v) { sXb[(size_t)(k2 + jj) * m2 + i] = v; });
    }
    __syncthreads();
    // M = R1 R1bar^T - Qbar'^T Q  (k2 x k2), the global factors R1 and Q staged through sB (B is
    // no longer needed): first R1 R1bar^T into registers, then the second product subtracts
    mfma_gemm_staged<QT, KCH, SPT, true>(
        k2, k2, k2, [&](int a, int kk) { return RQ(a, kk); },
        [&](int kk, int bb) { return sRb[(size_t)kk * MAXN + bb]; }, sB,
        [&](int a, int bb, double v) { sRb[(size_t)a * MAXN + bb] = v; });
    __syncthreads();
    mfma_gemm_staged<QT, KCH, SPT, false>(
        k2, k2, m2, [&](int bb, int kk) { return Q[(size_t)bb * m2 + kk]; },
        [&](int a, int kk) { return sXb[(size_t)a * m2 + kk]; }, sB,
        [&](int a, int bb, double v) { sRb[(size_t)a * MAXN + bb] -= v; });
    __syncthreads();
    // Bm = Qbar' + Q sym(M)  (m2 x k2), into sXb[:, :k2]
    mfma_gemm_staged<QT, KCH, SPT, true>(
        m2, k2, k2, [&](int i, int a) { return Q[(size_t)a * m2 + i]; },
        [&](int a, int j) { return (a >= j) ? sRb[(size_t)a * MAXN + j] : sRb[(size_t)j * MAXN + a]; }, sB,
        [&](int i, int j, double v) { sXb[(size_t)j * m2 + i] += v; });
    // R1 into sRb for the triangular solve (M is no longer read)
    if constexpr (BIG) {
      for (int idx = threadIdx.x; idx < k2 * MAXN; idx += kT) {
        const int i = idx % MAXN, j = idx / MAXN;
        sRb[idx] = (i < k2) ? RQ(i, j) : 0.0;
      }
    } else {
      constexpr int RPT = (MAXN * MAXN + kT - 1) / kT;
      double st[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int idx = threadIdx.x + q * kT;
        const int i = idx % MAXN, j = idx / MAXN;
        st[q] = (j < k2 && i < k2) ? RQ(i, j) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int idx = threadIdx.x + q * kT;
        const int j = idx / MAXN;
        if (j < k2) sRb[idx] = st[q];
      }
    }
    __syncthreads();
    // Xbar[:, :k2] = Bm R1^-T in blocks of 8 columns from the right: rows are independent, so
    // inside a block each row solves its 8 unknowns alone; one product then removes the block
    // from every column to its left (two barriers per block)
    for (int j1 = k2; j1 > 0; j1 -= 8) {
      const int j0 = j1 - 8 > 0 ? j1 - 8 : 0;
      for (int i = threadIdx.x; i < m2; i += kT) {
        for (int j = j1 - 1; j >= j0; --j) {
          double acc = sXb[(size_t)j * m2 + i];
          for (int l = j + 1; l < j1; ++l) acc -= sRb[(size_t)l * MAXN + j] * sXb[(size_t)l * m2 + i];
          sXb[(size_t)j * m2 + i] = acc / sRb[(size_t)j * MAXN + j];
        }
      }
      __syncthreads();
      if (j0 > 0) {
        mfma_gemm(m2, j0, j1 - j0, [&](int i, int l) { return sXb[(size_t)(j0 + l) * m2 + i]; },
                        [&](int l, int jp) { return sRb[(size_t)(j0 + l) * MAXN + jp]; },
                        [&](int i, int jp, double v) { sXb[(size_t)jp * m2 + i] -= v; });
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// vjp[theta] = sum_b w_b O_b: one workgroup per site, samples summed in index order.
// ---------------------------------------------------------------------------------------------
__global__ void k_vjp(Dims d, const int64_t* __restrict__ site_offset, const int32_t* __restrict__ block_id,
                      const uint8_t* __restrict__ valid, const double* __restrict__ w,
                      const double* __restrict__ O, int B, double* __restrict__ vjp) {
  const int s = blockIdx.x;
  const int L = d.L, Dk = d.Dk, N = d.N;
  const int x = s % L, y = s / L;
  const int np = (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1);
  int bs = 1, nb = 1;
  for (int i = 0; i < np; ++i) bs *= Dk;
  for (int i = 0; i < np - 1; ++i) nb *= N;
  for (int ent = threadIdx.x; ent < nb * bs; ent += blockDim.x) {
    const int blk = ent / bs, e = ent % bs;
    double acc = 0.0;
    for (int bb = 0; bb < B; ++bb) {
      if (!valid[bb] || block_id[(size_t)bb * d.n_sites + s] != blk) continue;
      acc += (w ? w[bb] : 1.0) * O[((size_t)bb * d.n_sites + s) * d.P4 + e];
    }
    vjp[site_offset[s] + ent] = acc;
  }
}

__global__ void k_fill(double* __restrict__ p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_adj_close(const Dims& d, const int* bond_last, const double* proj,
                            const uint8_t* valid, int B, const double* last_row, double* psibar,
                            double* O, hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (d.maxN > kMaxN)
    hipLaunchKernelGGL(k_adj_close<kMaxNBig>, dim3(B), dim3(256), 0, s, d, bond_last, proj, valid, last_row,
                       psibar, O);
  else
    hipLaunchKernelGGL(k_adj_close<kMaxN>, dim3(B), dim3(256), 0, s, d, bond_last, proj, valid, last_row,
                       psibar, O);
  return hipGetLastError();
}

hipError_t launch_adj_row0(const Dims& d, const uint8_t* valid, int B, const double* psibar,
                           double* O, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_row0, dim3(B), dim3(64), 0, s, d, valid, psibar, O);
  return hipGetLastError();
}

hipError_t launch_adj_row(const Dims& d, const DeviceTables& t, int y, const double* proj,
                          const uint8_t* valid, int B, const double* prev_row,
                          const double* cur_row, const double* tape, const double* qscr,
                          const double* psibar_in, double* qbar, double* xbar, double* psibar_out,
                          double* O, hipStream_t s, double* wbig) {
  if (B == 0) return hipSuccess;
  if (d.maxN > kMaxN && (d.Dk != 2 || d.maxN > kMaxNBig || !wbig)) return hipErrorInvalidValue;
#define GIPEPS_ADJ(MN, DKV)                                                                          \
  hipLaunchKernelGGL((k_adj_svd<MN, DKV>), dim3(B), dim3(kT), 0, s, d, t.bond, t.qrk, y, valid,      \
                     cur_row, tape, qscr, psibar_in, qbar, xbar, wbig);                              \
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;                                 \
  hipLaunchKernelGGL((k_adj_qr<MN, DKV>), dim3(B), dim3(kT), 0, s, d, t.bond, t.qrk, y, proj, valid, \
                     prev_row, qscr, tape, qbar, xbar, psibar_out, O, wbig);
  if (d.Dk == 2 && d.maxN <= 32) {
    GIPEPS_ADJ(32, 2)
  } else if (d.Dk == 2 && d.maxN <= kMaxN) {
    GIPEPS_ADJ(72, 2)
  } else if (d.Dk == 2) {
    GIPEPS_ADJ(kMaxNBig, 2)
  } else {
    GIPEPS_ADJ(32, 1)
  }
#undef GIPEPS_ADJ
  return hipGetLastError();
}

hipError_t launch_vjp(const Dims& d, const DeviceTables& t, const int32_t* block_id,
                      const uint8_t* valid, const double* w, const double* O, int B, double* vjp,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_vjp, dim3(d.n_sites), dim3(256), 0, s, d, t.site_offset, block_id, valid, w, O,
                     B, vjp);
  return hipGetLastError();
}

}  // namespace gipeps
