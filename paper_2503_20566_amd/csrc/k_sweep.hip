// One boundary-MPS row step: apply row y to the boundary D_{y-1}, left-canonicalise with
// Householder QR, truncate right to left with one-sided Jacobi SVDs, normalise (SM S-2 eq. project;
// VMC section, cutoff chi).  The state after the step depends only on the state before it, so the
// factorisation routines here need not be LAPACK's: the QR is unblocked Householder (reflectors as
// in LAPACK's dgeqr2/dorg2r, written from their definition) and the SVD is Hestenes' one-sided
// Jacobi method with round-robin pair ordering, sorted descending afterwards.
//
// Mapping: one workgroup (512 threads = 8 wave64) per sample, the whole row in one launch.  The
// working matrices live in LDS (145 KB at chi*Dk = 72); the Q factors of the row are parked in a
// per-sample global slot between the two sweeps.  Column work inside a factorisation is spread over
// the 8 waves (one column or one column pair per wave), lanes run over rows, dot products are
// wave64 butterfly reductions (all lanes obtain the same bits, so the result is deterministic).
#include "internal.h"

namespace gipeps {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxSweeps = 40;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------------------------
// Householder QR of the m x n column-major matrix X (ld = m), k = min(m, n) reflectors.
// On return: R (k x n, row i starting at the diagonal) copied to sR with ld = ldr (R[i][j] at
// sR[j*ldr + i], zeros below the diagonal), and X overwritten by the explicit m x k factor Q.
// ---------------------------------------------------------------------------------------------
__device__ void householder_qr(double* X, int m, int n, double* sR, int ldr, double* sTau) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = m < n ? m : n;
  for (int j = 0; j < k; ++j) {
    if (wave == 0) {
      double* col = X + (size_t)j * m;
      double s2 = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) s2 += col[i] * col[i];
      s2 = wave_sum(s2);
      const double alpha = col[j];
      double tau = 0.0;
      if (s2 != 0.0) {
        const double beta = -copysign(sqrt(alpha * alpha + s2), alpha);
        tau = (beta - alpha) / beta;
        const double scal = 1.0 / (alpha - beta);
        for (int i = j + 1 + lane; i < m; i += 64) col[i] *= scal;
        if (lane == 0) col[j] = beta;
      }
      if (lane == 0) sTau[j] = tau;
    }
    __syncthreads();
    const double tau = sTau[j];
    if (tau != 0.0) {
      const double* v = X + (size_t)j * m;
      for (int jj = j + 1 + wave; jj < n; jj += kWaves) {
        double* c = X + (size_t)jj * m;
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) w += v[i] * c[i];
        w = wave_sum(w) + c[j];
        w *= tau;
        if (lane == 0) c[j] -= w;
        for (int i = j + 1 + lane; i < m; i += 64) c[i] -= v[i] * w;
      }
    }
    __syncthreads();
  }
  // R out
  for (int idx = threadIdx.x; idx < k * n; idx += kThreads) {
    const int i = idx % k, j = idx / k;
    sR[(size_t)j * ldr + i] = (i <= j) ? X[(size_t)j * m + i] : 0.0;
  }
  __syncthreads();
  // explicit Q (backward accumulation of the reflectors, in place)
  for (int j = k - 1; j >= 0; --j) {
    const double tau = sTau[j];
    const double* v = X + (size_t)j * m;
    if (j < k - 1 && tau != 0.0) {
      for (int jj = j + 1 + wave; jj < k; jj += kWaves) {
        double* c = X + (size_t)jj * m;
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) w += v[i] * c[i];
        w = wave_sum(w) + c[j];
        w *= tau;
        if (lane == 0) c[j] -= w;
        for (int i = j + 1 + lane; i < m; i += 64) c[i] -= v[i] * w;
      }
    }
    __syncthreads();
    double* col = X + (size_t)j * m;
    for (int i = threadIdx.x; i < m; i += kThreads) {
      if (i > j) col[i] *= -tau;
      else if (i == j) col[i] = 1.0 - tau;
      else col[i] = 0.0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// One-sided Jacobi on the column-major nA x mA matrix A (ld = nA): orthogonalise its columns,
// accumulating the rotations in J (mA x mA, column-major, starts as identity).  On return
// sSig[i] = ||A[:, i]|| and sPerm[a] = index of the a-th largest (ties by index).
// A = Theta^T, so J holds Theta's left singular vectors and A's columns are s_i v_i.
// ---------------------------------------------------------------------------------------------
__device__ void jacobi_svd(double* A, int nA, int mA, double* J, double* sSig, int* sPerm,
                           int* sFlag) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int idx = threadIdx.x; idx < mA * mA; idx += kThreads)
    J[idx] = (idx % mA == idx / mA) ? 1.0 : 0.0;
  if (threadIdx.x == 0) *sFlag = 0;
  __syncthreads();
  const double tol = fmax(1e-15, 2.220446049250313e-16 * (double)nA);
  const int ncp = mA + (mA & 1);
  if (mA > 1) {
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
      for (int s = 0; s < ncp - 1; ++s) {
        for (int kp = wave; kp < ncp / 2; kp += kWaves) {
          const int p = (kp == 0) ? 0 : ((kp - 1 + s) % (ncp - 1)) + 1;
          const int q = ((ncp - 2 - kp + s) % (ncp - 1)) + 1;
          if (p >= mA || q >= mA) continue;
          const int i = p < q ? p : q, j = p < q ? q : p;
          double* ai = A + (size_t)i * nA;
          double* aj = A + (size_t)j * nA;
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int r = lane; r < nA; r += 64) {
            const double x = ai[r], y = aj[r];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
          al = wave_sum(al);
          be = wave_sum(be);
          ga = wave_sum(ga);
          if (ga == 0.0 || fabs(ga) <= tol * sqrt(al * be)) continue;
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (fabs(zeta) > 1e150) ? 0.5 / zeta
                                                 : copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int r = lane; r < nA; r += 64) {
            const double x = ai[r], y = aj[r];
            ai[r] = cs * x - sn * y;
            aj[r] = sn * x + cs * y;
          }
          double* ji = J + (size_t)i * mA;
          double* jj = J + (size_t)j * mA;
          for (int r = lane; r < mA; r += 64) {
            const double x = ji[r], y = jj[r];
            ji[r] = cs * x - sn * y;
            jj[r] = sn * x + cs * y;
          }
          if (lane == 0) *sFlag = 1;
        }
        __syncthreads();
      }
      const int rotated = *sFlag;
      __syncthreads();
      if (threadIdx.x == 0) *sFlag = 0;
      __syncthreads();
      if (!rotated) break;
    }
  }
  for (int i = wave; i < mA; i += kWaves) {
    const double* ai = A + (size_t)i * nA;
    double s2 = 0.0;
    for (int r = lane; r < nA; r += 64) s2 += ai[r] * ai[r];
    s2 = wave_sum(s2);
    if (lane == 0) sSig[i] = sqrt(s2);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < mA; i += kThreads) {
    const double si = sSig[i];
    int rank = 0;
    for (int j = 0; j < mA; ++j) {
      const double sj = sSig[j];
      rank += (sj > si) || (sj == si && j < i);
    }
    sPerm[rank] = i;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// The row step.  LDS: sX (QR matrix, later A | J of the Jacobi), sR (R, later G = U_k S_k),
// sB (boundary site cache), sT (row tensor).
// ---------------------------------------------------------------------------------------------
template <int MAXN, int DK>
__global__ void __launch_bounds__(kThreads)
k_row_sweep(Dims d, const int* __restrict__ bond_all, const int* __restrict__ qrk_all, int y,
            const double* __restrict__ proj, const uint8_t* __restrict__ valid,
            const double* __restrict__ prev_row, double* __restrict__ out_row,
            double* __restrict__ qscr, double* __restrict__ lognu) {
  constexpr int MAXM = MAXN * DK;
  // sX holds the QR matrix (MAXM x MAXN) and later A and J of the Jacobi (2 x MAXN^2)
  constexpr int XSIZE = (MAXM * MAXN > 2 * MAXN * MAXN) ? MAXM * MAXN : 2 * MAXN * MAXN;
  __shared__ double sX[XSIZE];
  __shared__ double sR[MAXN * MAXN];
  __shared__ double sB[MAXN * MAXN / DK];
  __shared__ double sT[DK * DK * DK * DK];
  __shared__ double sTau[MAXN];
  __shared__ double sSig[MAXN];
  __shared__ int sPerm[MAXN];
  __shared__ int sFlag;

  const int b = blockIdx.x;
  if (!valid[b]) return;
  const int L = d.L, Dk = d.Dk, chi = d.chi;
  const int* bprev = bond_all + (size_t)(y - 1) * (L + 1);
  const int* bnew = bond_all + (size_t)y * (L + 1);
  const int* qrk = qrk_all + (size_t)y * L;
  const double* pb = proj + ((size_t)b * d.n_sites + (size_t)y * L) * d.P4;
  const double* prev = prev_row + (size_t)b * d.row_stride;
  double* outp = out_row + (size_t)b * d.row_stride;
  double* qs = qscr + (size_t)b * L * (MAXM * MAXN);
  (void)chi;

  // ---------------- left-to-right: X_c = R_{c-1} M_c, QR ----------------
  int r_prev = 1;
  if (threadIdx.x == 0) sR[0] = 1.0;
  __syncthreads();
  int m_last = 0;
  for (int c = 0; c < L; ++c) {
    const int dl = c > 0 ? Dk : 1, dr = c < L - 1 ? Dk : 1;
    const int bc = bprev[c], bn = bprev[c + 1];
    const double* Bs = prev + (size_t)c * d.site_stride;  // [a][dd][a']
    for (int i = threadIdx.x; i < bc * Dk * bn; i += kThreads) sB[i] = Bs[i];
    for (int i = threadIdx.x; i < dl * dr * Dk * Dk; i += kThreads) sT[i] = pb[(size_t)c * d.P4 + i];
    __syncthreads();
    const int m = r_prev * Dk, n = bn * dr;
    // X[(i,u),(a',rr)] = sum_{a,l,dd} R[i][a*dl+l] B[a][dd][a'] T[l][rr][dd][u]
    for (int idx = threadIdx.x; idx < m * n; idx += kThreads) {
      const int row = idx % m, col = idx / m;
      const int i = row / Dk, u = row % Dk, ap = col / dr, rr = col % dr;
      double acc = 0.0;
      for (int a = 0; a < bc; ++a) {
        for (int l = 0; l < dl; ++l) {
          const double rv = sR[(size_t)(a * dl + l) * MAXN + i];
          double inner = 0.0;
          for (int dd = 0; dd < Dk; ++dd)
            inner += sB[(a * Dk + dd) * bn + ap] * sT[((l * dr + rr) * Dk + dd) * Dk + u];
          acc += rv * inner;
        }
      }
      sX[idx] = acc;
    }
    __syncthreads();
    if (c == L - 1) {
      m_last = m;
      break;
    }
    householder_qr(sX, m, n, sR, MAXN, sTau);
    const int k = qrk[c];
    double* qdst = qs + (size_t)c * (MAXM * MAXN);
    for (int i = threadIdx.x; i < m * k; i += kThreads) qdst[i] = sX[i];
    r_prev = k;
    __syncthreads();
  }

  // ---------------- right-to-left: Theta_c, Jacobi SVD, truncate ----------------
  // Theta_{L-1}: r_prev x (Dk * 1), entries X[(i,u), 0].  A = Theta^T, nA = Dk*chi', mA = rows.
  double* A = sX;            // nA x mA
  double* Jm = sX + MAXN * MAXN;
  double* G = sR;            // G[i][a] at G[i*MAXN + a]
  int chi_next = 1;
  {
    // stage Theta_{L-1}^T into a temporary in sB (<= MAXM doubles), then into A
    const int m = m_last;
    for (int i = threadIdx.x; i < m; i += kThreads) sB[i] = sX[i];
    __syncthreads();
    const int mA = m / Dk, nA = Dk;
    for (int idx = threadIdx.x; idx < mA * nA; idx += kThreads) {
      const int i = idx / nA, u = idx % nA;
      A[idx] = sB[i * Dk + u];
    }
    __syncthreads();
  }
  for (int c = L - 1; c >= 1; --c) {
    const int mA = qrk[c - 1];           // rows of Theta_c
    const int nA = Dk * chi_next;        // cols of Theta_c
    if (c < L - 1) {
      const int kc = qrk[c];             // inner dimension (cols of Q_c)
      const double* Qc = qs + (size_t)c * (MAXM * MAXN);
      const int mq = mA * Dk;            // rows of Q_c
      for (int idx = threadIdx.x; idx < mA * nA; idx += kThreads) {
        const int i = idx / nA, col = idx % nA, u = col / chi_next, j = col % chi_next;
        double acc = 0.0;
        for (int t = 0; t < kc; ++t) acc += Qc[(size_t)t * mq + i * Dk + u] * G[t * MAXN + j];
        A[idx] = acc;
      }
      __syncthreads();
    }
    jacobi_svd(A, nA, mA, Jm, sSig, sPerm, &sFlag);
    const int kk = bnew[c];
    double* S = outp + (size_t)c * d.site_stride;  // [a][u][j], a < kk
    for (int idx = threadIdx.x; idx < kk * nA; idx += kThreads) {
      const int a = idx / nA, col = idx % nA;
      const int p = sPerm[a];
      const double sg = sSig[p];
      S[idx] = (sg > 0.0) ? A[(size_t)p * nA + col] / sg : 0.0;
    }
    for (int idx = threadIdx.x; idx < mA * kk; idx += kThreads) {
      const int i = idx / kk, a = idx % kk;
      const int p = sPerm[a];
      G[i * MAXN + a] = Jm[(size_t)p * mA + i] * sSig[p];
    }
    __syncthreads();
    chi_next = kk;
  }
  // site 0: Theta_0 = Q_0 G_1 (Dk x chi_1), normalise
  {
    const int k0 = qrk[0];
    const double* Q0 = qs;
    const int n0 = Dk * chi_next;
    for (int idx = threadIdx.x; idx < n0; idx += kThreads) {
      const int u = idx / chi_next, j = idx % chi_next;
      double acc = 0.0;
      for (int t = 0; t < k0; ++t) acc += Q0[(size_t)t * Dk + u] * G[t * MAXN + j];
      sB[idx] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s2 = 0.0;
      for (int i = 0; i < n0; ++i) s2 += sB[i] * sB[i];
      sSig[0] = sqrt(s2);
      lognu[(size_t)b * L + y] = log(sSig[0]);
    }
    __syncthreads();
    const double nu = sSig[0];
    double* S0 = outp;
    for (int idx = threadIdx.x; idx < n0; idx += kThreads) S0[idx] = sB[idx] / nu;
  }
}

// ---------------------------------------------------------------------------------------------
// Close: c = <row_{L-1} | D_{L-2}>, ln|Psi| = sum_y ln nu_y + ln|c|.  One workgroup per sample.
// ---------------------------------------------------------------------------------------------
__global__ void k_close(Dims d, const int* __restrict__ bond_last, const double* __restrict__ proj,
                        const uint8_t* __restrict__ valid, const double* __restrict__ last_row,
                        const double* __restrict__ lognu, double* __restrict__ log_abs,
                        double* __restrict__ sign) {
  __shared__ double e0[kMaxN * kMaxDk];
  __shared__ double e1[kMaxN * kMaxDk];
  const int b = blockIdx.x;
  const int L = d.L, Dk = d.Dk;
  if (!valid[b]) {
    if (threadIdx.x == 0) {
      log_abs[b] = -HUGE_VAL;
      sign[b] = 0.0;
    }
    return;
  }
  const double* pb = proj + ((size_t)b * d.n_sites + (size_t)(L - 1) * L) * d.P4;
  const double* mp = last_row + (size_t)b * d.row_stride;
  if (threadIdx.x == 0) e0[0] = 1.0;
  __syncthreads();
  double* ein = e0;
  double* eout = e1;
  for (int c = 0; c < L; ++c) {
    const int dl = c > 0 ? Dk : 1, dr = c < L - 1 ? Dk : 1;
    const int bc = bond_last[c], bn = bond_last[c + 1];
    const double* Bs = mp + (size_t)c * d.site_stride;
    const double* T = pb + (size_t)c * d.P4;  // T[l][r][dd][0], du = 1
    for (int idx = threadIdx.x; idx < bn * dr; idx += blockDim.x) {
      const int ap = idx / dr, rr = idx % dr;
      double acc = 0.0;
      for (int a = 0; a < bc; ++a)
        for (int l = 0; l < dl; ++l)
          for (int dd = 0; dd < Dk; ++dd)
            acc += ein[a * dl + l] * Bs[(a * Dk + dd) * bn + ap] * T[(l * dr + rr) * Dk + dd];
      eout[idx] = acc;
    }
    __syncthreads();
    double* tmp = ein;
    ein = eout;
    eout = tmp;
  }
  if (threadIdx.x == 0) {
    const double c = ein[0];
    double s = 0.0;
    for (int yy = 1; yy <= L - 2; ++yy) s += lognu[(size_t)b * L + yy];
    if (c == 0.0 || !isfinite(c)) {
      log_abs[b] = (c == 0.0) ? -HUGE_VAL : NAN;
      sign[b] = 0.0;
    } else {
      log_abs[b] = s + log(fabs(c));
      sign[b] = c > 0.0 ? 1.0 : -1.0;
    }
  }
}

hipError_t launch_row_sweep(const Dims& d, const DeviceTables& t, int y, const double* proj,
                            const uint8_t* valid, int B, const double* prev_row, double* out_row,
                            double* qscr, double* lognu, hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (d.Dk == 2 && d.maxN <= 32)
    hipLaunchKernelGGL((k_row_sweep<32, 2>), dim3(B), dim3(kThreads), 0, s, d, t.bond, t.qrk, y,
                       proj, valid, prev_row, out_row, qscr, lognu);
  else if (d.Dk == 2)
    hipLaunchKernelGGL((k_row_sweep<72, 2>), dim3(B), dim3(kThreads), 0, s, d, t.bond, t.qrk, y,
                       proj, valid, prev_row, out_row, qscr, lognu);
  else  // Dk == 1: every bond has dimension 1
    hipLaunchKernelGGL((k_row_sweep<32, 1>), dim3(B), dim3(kThreads), 0, s, d, t.bond, t.qrk, y,
                       proj, valid, prev_row, out_row, qscr, lognu);
  return hipGetLastError();
}

hipError_t launch_close(const Dims& d, const int* bond_last, const double* proj,
                        const uint8_t* valid, int B, const double* last_row, const double* lognu,
                        double* log_abs, double* sign, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_close, dim3(B), dim3(128), 0, s, d, bond_last, proj, valid, last_row, lognu,
                     log_abs, sign);
  return hipGetLastError();
}

}  // namespace gipeps
