// Precision: CT is the arithmetic of the contraction with the row tensor (FP32 on the mixed path);
// every product with a QR or SVD factor (R_{c-1} B_c, Q_c G_{c+1}) and the factorisations stay FP64,
// because those factors carry the Schmidt weights that decide the truncation.
//
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
#include "dev_common.h"
#include "internal.h"

namespace gipeps {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;

constexpr int kGroups = kThreads / 8;  // 64 groups of 8 lanes
// Lanes per column pair in the Jacobi (GW, 4 or 8) is a template parameter chosen per handle (the
// autotuner times both): eight measured fastest at chi*Dk = 72, where four lanes double each
// lane's dependent chains and the step is latency-bound (one or two waves per SIMD).
// First lane of the Jacobi's J rows (two lanes per row): above the column groups, wave aligned.
constexpr int kJLane0 = 320;

// ---------------------------------------------------------------------------------------------
// Householder QR of the m x n column-major matrix X (ld = m, in LDS), k = min(m, n) reflectors
// (H_j = I - tau_j v_j v_j^T, v_j[j] = 1, zero above j; as LAPACK's dgeqr2/dorg2r define them).
// On return R (k x n) is in sR (R[i][j] at sR[j*ldr + i], zeros below the diagonal, rows >= k
// untouched), the explicit m x k factor Q is in qdst (global, ld m), and X holds the reflectors.
//
// Column jj belongs to 8-lane group jj mod 64 for the whole factorisation and stays in its
// registers (RPL rows per lane, row = lane + 8t).  Step j: every group applies H_j (read from a
// double-buffered LDS copy of v_j) to its columns right of j; the group owning column j+1 then
// forms H_{j+1} at once from the updated column and publishes it -- one barrier per reflector, and
// per step one column is written to LDS instead of the whole trailing matrix being read and
// rewritten.  Q = H_0 ... H_{k-1} [I; 0] is then accumulated column by column in registers
// (column jj needs H_jj .. H_0 only), reading the reflectors from X, with no barrier at all.
// vbuf: 2 * MAXM doubles of LDS.  qdst may point to LDS.
// ---------------------------------------------------------------------------------------------
template <int MAXM, int NMAX>
__device__ __forceinline__ void householder_qr(double* X, int m, int n, double* sR, int ldr, double* sTau,
                                               double* vbuf, double* qdst) {
  constexpr int RPL = MAXM / 8;                           // m <= MAXM
  constexpr int CPG = (NMAX + kGroups - 1) / kGroups;     // columns per group (n <= NMAX)
  static_assert(MAXM % 8 == 0, "rows per lane");
  // independent partial sums in the per-lane dot products (shorter dependent chains on the
  // reflector's critical path)
  constexpr int kAcc = RPL >= 12 ? 3 : (RPL >= 6 ? 2 : 1);
  const int g = threadIdx.x >> 3, gl = threadIdx.x & 7;
  const int k = m < n ? m : n;
  double c[CPG][RPL];
#pragma unroll
  for (int q = 0; q < CPG; ++q) {
    const int jj = g + q * kGroups;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = gl + 8 * t;
      c[q][t] = (jj < n && row < m) ? X[(size_t)jj * m + row] : 0.0;
    }
  }
  // H_j from the current column col (rows >= j): scale it into v_j in place, publish v_j and tau_j
  auto make_reflector = [&](double (&col)[RPL], int j) {
    double s2p[kAcc] = {}, alpha = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = gl + 8 * t;
      s2p[t % kAcc] += (row > j) ? col[t] * col[t] : 0.0;
      alpha += (row == j) ? col[t] : 0.0;
    }
    double s2 = s2p[0];
#pragma unroll
    for (int a = 1; a < kAcc; ++a) s2 += s2p[a];
    s2 = group8_sum(s2);
    alpha = group8_sum(alpha);
    double tau = 0.0, beta = alpha, scal = 1.0;
    if (s2 != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + s2), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    double* v = vbuf + (j & 1) * MAXM;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = gl + 8 * t;
      if (row > j) col[t] *= scal;
      if (row == j) col[t] = beta;
      v[row] = (row > j) ? col[t] : (row == j ? 1.0 : 0.0);
    }
    if (gl == 0) sTau[j] = tau;
  };
  if (g == 0 && k > 0) make_reflector(c[0], 0);
  __syncthreads();
  // the reflector's rows are cached in registers, except at the large-bond size (32 rows per lane)
  // where they are read from LDS where used
  constexpr bool VCACHE = RPL <= 18;
  for (int j = 0; j < k; ++j) {
    const double tau = sTau[j];
    const double* v = vbuf + (j & 1) * MAXM;
    double vr[VCACHE ? RPL : 1];
    if constexpr (VCACHE) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) vr[t] = v[gl + 8 * t];
    }
    auto V = [&](int t) -> double { if constexpr (VCACHE) return vr[t]; else return v[gl + 8 * t]; };
#pragma unroll
    for (int q = 0; q < CPG; ++q) {
      const int jj = g + q * kGroups;
      if (jj > j && jj < n) {
        if (tau != 0.0) {
          double wp[kAcc] = {};
#pragma unroll
          for (int t = 0; t < RPL; ++t) wp[t % kAcc] += V(t) * c[q][t];
          double w = wp[0];
#pragma unroll
          for (int a = 1; a < kAcc; ++a) w += wp[a];
          w = group8_sum(w) * tau;
#pragma unroll
          for (int t = 0; t < RPL; ++t) c[q][t] -= V(t) * w;
        }
        if (jj == j + 1 && jj < k) make_reflector(c[q], jj);
      }
    }
    __syncthreads();
  }
  // R into sR; reflectors (with the unit diagonal) back into X for the accumulation of Q
#pragma unroll
  for (int q = 0; q < CPG; ++q) {
    const int jj = g + q * kGroups;
    if (jj < n) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = gl + 8 * t;
        if (row < k) sR[(size_t)jj * ldr + row] = (row <= jj) ? c[q][t] : 0.0;
        if (jj < k && row < m) X[(size_t)jj * m + row] = (row > jj) ? c[q][t] : (row == jj ? 1.0 : 0.0);
      }
    }
  }
  __syncthreads();
  // Q columns: every group walks the same j sequence, so the eight groups of a wave read the same
  // reflector (LDS broadcast) and each v_j is loaded once per step
#pragma unroll
  for (int q = 0; q < CPG; ++q) {
    const int jj = g + q * kGroups;
#pragma unroll
    for (int t = 0; t < RPL; ++t) c[q][t] = (gl + 8 * t == jj) ? 1.0 : 0.0;
  }
  const int jtop = (k - 1 < kGroups * CPG - 1) ? k - 1 : kGroups * CPG - 1;
  for (int j = jtop; j >= 0; --j) {
    const double tau = sTau[j];
    if (tau == 0.0) continue;
    const double* vj = X + (size_t)j * m;
    double vr[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = gl + 8 * t;
      vr[t] = (row < m) ? vj[row] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < CPG; ++q) {
      const int jj = g + q * kGroups;
      if (jj >= j && jj < k) {
        double wp[kAcc] = {};
#pragma unroll
        for (int t = 0; t < RPL; ++t) wp[t % kAcc] += vr[t] * c[q][t];
        double w = wp[0];
#pragma unroll
        for (int a = 1; a < kAcc; ++a) w += wp[a];
        w = group8_sum(w) * tau;
#pragma unroll
        for (int t = 0; t < RPL; ++t) c[q][t] -= vr[t] * w;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CPG; ++q) {
    const int jj = g + q * kGroups;
    if (jj < k) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = gl + 8 * t;
        if (row < m) qdst[(size_t)jj * m + row] = c[q][t];
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// Rotation arithmetic of the Jacobi step.  The Jacobi scales its matrix by a power of two so that
// ||A||_F^2 is of order one, which keeps every argument below a normal number far from the
// exponent limits; the square root and reciprocal therefore use the hardware estimates refined by
// Newton steps, without the rescaling and special-value handling of the library routines.
// ---------------------------------------------------------------------------------------------
// t = tan(theta) of the smaller rotation angle annihilating a_i.a_j, from dd = |a_j|^2 - |a_i|^2
// and g2 = 2 a_i.a_j (g2 != 0): t = sign(dd) g2 / (|dd| + sqrt(dd^2 + g2^2)).  The square root
// takes one Goldschmidt iteration and one correction, the quotient one Newton step and one
// correction; the angle need not be exact to the last bit (the next sweep removes any residue),
// only cos and sin must be consistent, which rsqrt_1to2 ensures.
__device__ __forceinline__ double rotation_tangent(double dd, double g2) {
  const double x = dd * dd + g2 * g2;
  const double y0 = __builtin_amdgcn_rsq(x);
  double g = x * y0, h = 0.5 * y0;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double rr = fma(fma(-g, g, x), h, g);  // sqrt(x)
  const double den = fabs(dd) + rr;
  double y = __builtin_amdgcn_rcp(den);
  y = fma(y, fma(-den, y, 1.0), y);
  const double q = g2 * y;
  return copysign(1.0, dd) * fma(fma(-den, q, g2), y, q);
}

// 1 / sqrt(a) for a in [1, 2]
__device__ __forceinline__ double rsqrt_1to2(double a) {
  double y = __builtin_amdgcn_rsq(a);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double hy = 0.5 * y;
    y = fma(hy, fma(-a * y, y, 1.0), y);
  }
  return y;
}

// ---------------------------------------------------------------------------------------------
// One-sided Jacobi (Hestenes) on the nr x nc matrix A (nr >= nc), column j at A + j*ld: rotate
// column pairs until all are mutually orthogonal, accumulating the rotations in J (nc x nc, column
// j at J + j*ld, starts as identity), so A_in J = A_out with orthogonal columns.  A pair is left
// alone when (a_i.a_j)^2 <= tol^2 |a_i|^2 |a_j|^2 or when either column is numerically zero (norm
// below 64 eps ||A||_F), which keeps rank-deficient inputs from rotating rounding noise forever.
// The sweeps stop after one without rotations, or after one in which every pair's relative
// off-diagonal |a_i.a_j| / (|a_i| |a_j|) was at most 1e-6 before its rotation: convergence is
// quadratic there, and on the boundary matrices of this method the sweep that follows such a
// sweep never rotates (same final orthogonality, ~1 sweep in 11 saved).
//
// Ordering: odd-even transposition over ncp = nc rounded up to even slots (a zero dummy column
// fills the last slot when nc is odd).  Rounds alternate between the pairs (2k, 2k+1) and
// (2k+1, 2k+2); after each rotation the two columns exchange slots, so in ncp rounds every pair
// meets once.  Group k (8 lanes, 9 rows per lane at MAXN = 72) keeps the A columns of slots 2k and
// 2k+1 in registers for the whole factorisation, with their squared norms (exact at the start of
// each sweep, then updated from the rotation: |a_i'|^2 = |a_i|^2 - t a_i.a_j, |a_j'|^2 =
// |a_j|^2 + t a_i.a_j with t = s / c), so a round computes one dot product, not three.  The
// (2k, 2k+1) rounds need no communication; in the (2k+1, 2k+2) rounds group k fetches slot 2k+2
// from group k+1 through LDS, rotates the pair, keeps the partner's rotated column and hands its
// own rotated column back.
// J is not carried with the columns: the groups occupy the first 4.5 waves, and the lanes from
// kJLane0 up (idle otherwise) hold J by rows, a lane pair per row (slots [0, MAXN/2) and
// [MAXN/2, ncp)).  Each group publishes its round's (c, s) in a four-round ring; the J lanes
// apply an inner and a boundary round after the boundary round's second barrier, which halves
// the LDS traffic of the hand-over and takes the J update off the groups' path.
// On return A and J hold the columns (stride ld = MAXN + 1, zero rows from nr resp. nc up to
// MAXN), sSig[i] = ||A[:, i]|| and sPerm[a] = index of the a-th largest (ties by index).
// ---------------------------------------------------------------------------------------------
template <int GW>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(GW == 4 || GW == 8, "group reductions over 4 or 8 lanes");
  v += dpp_d<0xB1>(v);  // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);  // quad_perm [2,3,0,1]
  if (GW == 8) v += dpp_d<0x141>(v);  // row_half_mirror
  return v;
}

// Rotation of the pair (u, v) from their squared norms nu, nv (carried, not recomputed) and the
// dot product; dn = (s / c) (u . v) gives the squared norms after it: nu - dn and nv + dn.
struct PairRot {
  double c, s, dn;
  bool on;
};
template <int GW, int RPL>
__device__ __forceinline__ PairRot pair_rotation(const double (&u)[RPL], const double (&v)[RPL], double nu,
                                                    double nv, bool u_first, double zero2, double tol2,
                                                    bool& big_any) {
  constexpr double kQuadratic2 = 1e-12;  // (1e-6)^2
  double g = 0.0;
#pragma unroll
  for (int t = 0; t < RPL; ++t) g += u[t] * v[t];
  g = group_sum<GW>(g);
  const double al = u_first ? nu : nv, be = u_first ? nv : nu;
  big_any |= al > zero2 && be > zero2 && g * g > kQuadratic2 * al * be;
  PairRot r{1.0, 0.0, 0.0, false};
  if (!(g == 0.0 || al <= zero2 || be <= zero2 || g * g <= tol2 * al * be)) {
    const double dd = be - al, g2 = 2.0 * g;
    const double tn = rotation_tangent(dd, g2);
    const double cs = rsqrt_1to2(1.0 + tn * tn), sn = cs * tn;
    r = PairRot{cs, u_first ? sn : -sn, (u_first ? tn : -tn) * g, true};
  }
  return r;
}

// As pair_rotation with the second column v read through an accessor (from LDS) instead of registers.
template <int GW, int RPL, class FV>
__device__ __forceinline__ PairRot pair_rotation_lds(const double (&u)[RPL], FV v, double nu, double nv, bool u_first,
                                                        double zero2, double tol2, bool& big_any) {
  constexpr double kQuadratic2 = 1e-12;  // (1e-6)^2
  double g = 0.0;
#pragma unroll
  for (int t = 0; t < RPL; ++t) g += u[t] * v(t);
  g = group_sum<GW>(g);
  const double al = u_first ? nu : nv, be = u_first ? nv : nu;
  big_any |= al > zero2 && be > zero2 && g * g > kQuadratic2 * al * be;
  PairRot r{1.0, 0.0, 0.0, false};
  if (!(g == 0.0 || al <= zero2 || be <= zero2 || g * g <= tol2 * al * be)) {
    const double dd = be - al, g2 = 2.0 * g;
    const double tn = rotation_tangent(dd, g2);
    const double cs = rsqrt_1to2(1.0 + tn * tn), sn = cs * tn;
    r = PairRot{cs, u_first ? sn : -sn, (u_first ? tn : -tn) * g, true};
  }
  return r;
}

// hb: the hand-over buffers (2 ceil(nc/2) columns of MAXN doubles, of MAXN + 8 at the large-bond size) and ring: the rotation ring (4
// rounds of MAXN/2 (c, s) pairs); both in LDS.  With A and J themselves in LDS they overlay them
// (hb = A, ring = J: both are dead while the sweeps run); with A and J in global memory (the
// large-bond kernel) they are separate LDS buffers.  JL0: first lane of the J rows.
template <int MAXN, int GW, int JL0 = kJLane0>
__device__ __forceinline__ bool jacobi_svd(double* A, int nr, int nc, double* J, double* sSig,
                                           int* sPerm, int* sFlag, double* sScal, int max_sweeps,
                                           double* hb, double2* ring) {
  constexpr int RPL = MAXN / GW;  // rows per lane of a column group
  constexpr int HS = MAXN / 2;    // slots per J half row
  constexpr int ld = MAXN + 1;
  constexpr int SLOT = MAXN;      // one A column handed over
  // bank offset of hand-over slot q: consecutive groups' 8-lane stores start 16 banks apart.  The
  // large-bond size pads the slot stride by 8 doubles instead of rotating inside the slot, so that
  // every hand-over address is the slot's base plus a constant (no per-row address registers).
  constexpr bool PADSLOT = MAXN > kMaxN;
  constexpr int SLOTP = PADSLOT ? SLOT + 8 : SLOT;
  constexpr int kRot = (!PADSLOT && (2 * SLOT) % 64 == 0) ? 8 : 0;
  static_assert(MAXN % GW == 0 && (MAXN / 2) * GW <= JL0, "column groups below the J lanes");
  static_assert(JL0 % 64 == 0 && JL0 + 2 * MAXN <= kThreads && MAXN % 4 == 0, "J rows fit");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = threadIdx.x / GW, gl = threadIdx.x % GW;
  {
    double s2 = 0.0;
    for (int idx = threadIdx.x; idx < nr * nc; idx += kThreads) {
      const double v = A[(size_t)(idx / nr) * ld + idx % nr];
      s2 += v * v;
    }
    s2 = wave_sum_dpp(s2);
    if (lane == 0) sScal[wave] = s2;
  }
  if (threadIdx.x < 2) sFlag[threadIdx.x] = 0;
  const int ncp = nc + (nc & 1), np = ncp / 2;
  const bool active = nc > 1 && k < np;
  // J lanes: lane pair (2r, 2r+1) holds row r of J, slots [0, HS) and [HS, ncp)
  const int jl = (int)threadIdx.x - JL0;
  const int jr = jl >> 1, jh = jl & 1;
  const bool jact = nc > 1 && jl >= 0 && jr < nc;
  const int jb = jh * HS;  // first slot of this half row
  // one register array serves both roles (a lane is either a column-group lane or a J lane), so
  // that the compiler does not keep both sets live: X | Y for the groups, the J half row else
  static_assert(2 * RPL <= HS, "X and Y fit in the J half row");
  double Jr[HS];
  double (&X)[RPL] = *reinterpret_cast<double (*)[RPL]>(&Jr[0]);
  double (&Y)[RPL] = *reinterpret_cast<double (*)[RPL]>(&Jr[RPL]);
  int idX = 2 * k, idY = 2 * k + 1;
  double nX = 0.0, nY = 0.0;  // |X|^2, |Y|^2: exact at each sweep's start, updated per rotation
  if (active) {
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = gl + GW * t;
      X[t] = (idX < nc && r < nr) ? A[(size_t)idX * ld + r] : 0.0;
      Y[t] = (idY < nc && r < nr) ? A[(size_t)idY * ld + r] : 0.0;
    }
  }
  if (jact) {
#pragma unroll
    for (int q = 0; q < HS; ++q) Jr[q] = (jb + q == jr) ? 1.0 : 0.0;
  }
  __syncthreads();  // A read into registers: the hand-over buffers below overlay it
  double fro2 = 0.0;
  for (int w = 0; w < kWaves; ++w) fro2 += sScal[w];
  // exact power-of-two scaling to ||A||_F ~ 1 (undone on write-back)
  int fexp = 0;
  (void)frexp(fro2, &fexp);
  const int shift = (fro2 > 0.0) ? -(fexp / 2) : 0;
  if (active) {
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      X[t] = ldexp(X[t], shift);
      Y[t] = ldexp(Y[t], shift);
    }
  }
  fro2 = ldexp(fro2, 2 * shift);
  const double zero2 = fro2 * (64.0 * 2.220446049250313e-16) * (64.0 * 2.220446049250313e-16);
  const double tol = fmax(1e-15, 2.220446049250313e-16 * (double)nr);
  const double tol2 = tol * tol;
  // hand-over buffers: slot q of buffer 1 at hb + q*SLOTP, of buffer 2 at hb + (np + q)*SLOTP
  auto at = [&](int q, int e) -> double& {
    if constexpr (PADSLOT)
      return hb[(size_t)q * SLOTP + e];
    else
      return hb[(size_t)q * SLOT + (e + kRot * (q & 3)) % SLOT];
  };
  int* id1 = sPerm;
  int* id2 = sPerm + np;
  double* nrm1 = sSig;  // norms travelling with the handed-over columns
  double* nrm2 = sSig + np;
  // rotations of the last four rounds, (c, s) per pair, in the (idle) J area.  Every group below
  // HS writes its entry each round; (0, 1) marks a pair that does not exist: applied to the J rows
  // it keeps the left slot and only flips the sign of a slot beyond ncp, so the J lanes apply all
  // entries without tests (all stay finite: the J rows start finite and so do all entries).
  const bool ring_writer = k < HS && gl == 0;
  int rnd = 0;  // round counter (all threads)

  // round (2k, 2k+1) with slot 2k in u and slot 2k+1 in v; afterwards the slots are exchanged,
  // i.e. the caller swaps the roles of the two register sets
  auto inner = [&](double (&u)[RPL], double (&v)[RPL], double& nu, double& nv, int iu, int iv, bool& rot_any,
                   bool& big_any) {
    if (ring_writer && !active) ring[(rnd & 3) * HS + k] = make_double2(0.0, 1.0);
    if (active) {
      const PairRot r = pair_rotation<GW, RPL>(u, v, nu, nv, iu < iv, zero2, tol2, big_any);
      nu -= r.dn;
      nv += r.dn;
      if (gl == 0) ring[(rnd & 3) * HS + k] = make_double2(r.c, r.s);
      if (r.on) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const double a = u[t], b = v[t];
          u[t] = r.c * a - r.s * b;
          v[t] = r.c * b + r.s * a;
        }
        rot_any = true;
      }
    }
    ++rnd;
  };
  // J rows: apply the rotations of the inner round t0 and the boundary round t0 + 1.  A pair
  // (left, right) with rotation (c, s) maps to left' = c right + s left, right' = c left - s right
  // (the rotated pair also exchanges its slots, as the columns do).
  // (c, s) are read in chunks of kJC pairs (a scheduling barrier after each) so that the J lanes'
  // live registers stay near one half row plus a chunk
  constexpr int kJC = ((MAXN / 4) % 6 == 0) ? 6 : 4;
  static_assert((HS / 2) % kJC == 0, "whole chunks of pairs per half row");
  auto japply = [&](int t0) {
    if (!jact) return;
    const double2* ri = ring + (t0 & 3) * HS + jb / 2;  // inner pairs (2k, 2k+1), k = jb/2 + q/2
#pragma unroll
    for (int q0 = 0; q0 < HS / 2; q0 += kJC) {
      double2 cs[kJC];
#pragma unroll
      for (int e = 0; e < kJC; ++e) cs[e] = ri[q0 + e];
#pragma unroll
      for (int e = 0; e < kJC; ++e) {
        const int q = 2 * (q0 + e);
        const double u = Jr[q], v = Jr[q + 1];
        Jr[q] = cs[e].x * v + cs[e].y * u;
        Jr[q + 1] = cs[e].x * u - cs[e].y * v;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // boundary pairs (2k+1, 2k+2): (HS - 1, HS) across the lane pair, then inside the half row
    const double2* rb = ring + ((t0 + 1) & 3) * HS;
    {
      const double2 c = rb[HS / 2 - 1];
      const double mine = jh ? Jr[0] : Jr[HS - 1];
      const double other = dpp_d<0xB1>(mine);  // quad_perm [1,0,3,2]: the other half row
      if (jh == 0)
        Jr[HS - 1] = c.x * other + c.y * mine;
      else
        Jr[0] = c.x * other - c.y * mine;
    }
#pragma unroll
    for (int q0 = 0; q0 < HS / 2; q0 += kJC) {
      double2 cs[kJC];
#pragma unroll
      for (int e = 0; e < kJC; ++e)
        if (q0 + e + 1 < HS / 2) cs[e] = rb[jb / 2 + q0 + e];
#pragma unroll
      for (int e = 0; e < kJC; ++e) {
        if (q0 + e + 1 < HS / 2) {  // local pair (q, q + 1), q = 2 (q0 + e) + 1
          const int q = 2 * (q0 + e) + 1;
          const double u = Jr[q], v = Jr[q + 1];
          Jr[q] = cs[e].x * v + cs[e].y * u;
          Jr[q + 1] = cs[e].x * u - cs[e].y * v;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  // round (2k+1, 2k+2) with slot 2k in lo and slot 2k+1 in hi; the J rows then catch up on this
  // round and the inner round before it
  auto boundary = [&](double (&lo)[RPL], double (&hi)[RPL], double& nlo, double& nhi, int& ilo, int& ihi,
                      bool& rot_any, bool& big_any) {
    if (active) {  // slot 2k goes to group k-1
#pragma unroll
      for (int t = 0; t < RPL; ++t) at(k, gl + GW * t) = lo[t];
      if (gl == 0) {
        id1[k] = ilo;
        nrm1[k] = nlo;
      }
    }
    if (ring_writer && !(active && k + 1 < np)) ring[(rnd & 3) * HS + k] = make_double2(0.0, 1.0);
    __syncthreads();
    if (active && k + 1 < np) {  // pair (slot 2k+1, slot 2k+2): keep the rotated partner
      const int ip = id1[k + 1];
      const double nP = nrm1[k + 1];
      PairRot r;
      if constexpr (!PADSLOT) {
        double P[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) P[t] = at(k + 1, gl + GW * t);
        r = pair_rotation<GW, RPL>(hi, P, nhi, nP, ihi < ip, zero2, tol2, big_any);
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const double a = hi[t], b = P[t];
          at(np + k, gl + GW * t) = r.c * a - r.s * b;
          hi[t] = r.c * b + r.s * a;
        }
      } else {
        // long columns (large bonds): the partner is read from LDS twice, for the dot product and
        // for the rotation, instead of being held in registers beside the lane's own pair
        r = pair_rotation_lds<GW, RPL>(hi, [&](int t) { return at(k + 1, gl + GW * t); }, nhi, nP, ihi < ip,
                                       zero2, tol2, big_any);
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const double a = hi[t], b = at(k + 1, gl + GW * t);
          at(np + k, gl + GW * t) = r.c * a - r.s * b;
          hi[t] = r.c * b + r.s * a;
        }
      }
      if (gl == 0) ring[(rnd & 3) * HS + k] = make_double2(r.c, r.s);
      rot_any |= r.on;
      if (gl == 0) {
        id2[k] = ihi;
        nrm2[k] = nhi - r.dn;
      }
      ihi = ip;
      nhi = nP + r.dn;
    }
    __syncthreads();
    if (active && k >= 1) {  // slot 2k receives the rotated slot 2k-1 of group k-1
#pragma unroll
      for (int t = 0; t < RPL; ++t) lo[t] = at(np + k - 1, gl + GW * t);
      ilo = id2[k - 1];
      nlo = nrm2[k - 1];
    }
    japply(rnd - 1);
    ++rnd;
  };

  bool more = false;  // still rotating after the last sweep run: not converged
  if (nc > 1) {
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      bool rot_any = false, big_any = false;
      if (active) {
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          sx += X[t] * X[t];
          sy += Y[t] * Y[t];
        }
        nX = group_sum<GW>(sx);
        nY = group_sum<GW>(sy);
      }
      // two round pairs per iteration so that the register roles return: (X, Y) = (2k, 2k+1)
      for (int h = 0; h + 2 <= np; h += 2) {
        inner(X, Y, nX, nY, idX, idY, rot_any, big_any);  // now Y = 2k, X = 2k+1
        boundary(Y, X, nY, nX, idY, idX, rot_any, big_any);
        inner(Y, X, nY, nX, idY, idX, rot_any, big_any);  // now X = 2k, Y = 2k+1
        boundary(X, Y, nX, nY, idX, idY, rot_any, big_any);
      }
      if (np & 1) {
        inner(X, Y, nX, nY, idX, idY, rot_any, big_any);
        boundary(Y, X, nY, nX, idY, idX, rot_any, big_any);
        // restore the roles (X, Y) = (2k, 2k+1); only on the groups' lanes, since X and Y share
        // their registers with the J rows
        if (active) {
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            const double a = X[t];
            X[t] = Y[t];
            Y[t] = a;
          }
        }
        const int ti = idX;
        idX = idY;
        idY = ti;
        const double tnrm = nX;
        nX = nY;
        nY = tnrm;
      }
      if (rot_any) sFlag[0] = 1;
      if (big_any) sFlag[1] = 1;
      __syncthreads();
      more = sFlag[0] != 0 && sFlag[1] != 0;
      __syncthreads();
      if (threadIdx.x < 2) sFlag[threadIdx.x] = 0;
      __syncthreads();
      if (!more) break;
    }
  }
  // hand-over buffers and rotation ring dead: column ids of the slots for the J rows
  if (active && gl == 0) {
    sPerm[2 * k] = idX;
    sPerm[2 * k + 1] = idY;
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = gl + GW * t;
      if (idX < nc) A[(size_t)idX * ld + r] = ldexp(X[t], -shift);
      if (idY < nc) A[(size_t)idY * ld + r] = ldexp(Y[t], -shift);
    }
  } else if (nc == 1 && k == 0) {
    for (int t = 0; t < RPL; ++t) {
      const int r = gl + GW * t;
      if (r >= nr) A[r] = 0.0;
      J[r] = (r == 0) ? 1.0 : 0.0;
    }
  }
  if (jact) {
#pragma unroll
    for (int q = 0; q < HS; ++q) {
      if (jb + q < ncp) {
        const int id = sPerm[jb + q];
        if (id < nc) J[(size_t)id * ld + jr] = Jr[q];
      }
    }
  }
  __syncthreads();
  {
    const int g8 = threadIdx.x >> 3, l8 = threadIdx.x & 7;
    for (int i = g8; i < nc; i += kThreads / 8) {
      const double* ai = A + (size_t)i * ld;
      double s2 = 0.0;
      for (int r = l8; r < nr; r += 8) s2 += ai[r] * ai[r];
      s2 = group8_sum(s2);
      if (l8 == 0) sSig[i] = sqrt(s2);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nc; i += kThreads) {
    const double si = sSig[i];
    int rank = 0;
    for (int j = 0; j < nc; ++j) {
      const double sj = sSig[j];
      rank += (sj > si) || (sj == si && j < i);
    }
    sPerm[rank] = i;
  }
  __syncthreads();
  return !more;
}

// ---------------------------------------------------------------------------------------------
// The row step.  LDS: sX (QR matrix, later A | J of the Jacobi), sR (R, later G = U_k S_k),
// sB (boundary site cache), sT (row tensor).  With a tape pointer the factorisations are recorded
// (TapeSlot layout) for the adjoint.
// ---------------------------------------------------------------------------------------------
// pmode: preconditioning of the large truncated SVDs (cuts whose smaller dimension is at least
// pthr and where Theta is wide or square): PEPS_PRECOND_NONE, PEPS_PRECOND_QR_T (QR of Theta^T,
// Jacobi on R_x^T; only for sweeps that are never reversed) or PEPS_PRECOND_SORTED_QR (columns
// sorted by norm, QR, Jacobi on R^T).
// The row step of sample b, shared by the batch kernel (one lattice) and the ragged kernel (several
// lattices in one launch).  qslot: doubles per (sample, site) Q-factor slot of qscr.
template <int MAXN, int DK, typename CT, int GW>
__device__ __forceinline__ void row_sweep_body(const Dims& d, const int* __restrict__ bond_all,
                                               const int* __restrict__ qrk_all, int y,
                                               const double* __restrict__ proj, const uint8_t* __restrict__ valid,
                                               const double* __restrict__ prev_row, double* __restrict__ out_row,
                                               double* __restrict__ qscr, size_t qslot, double* __restrict__ lognu,
                                               double* __restrict__ tape, int pmode, int pthr,
                                               uint32_t* __restrict__ status, double* __restrict__ wbig, int b) {
  constexpr int MAXM = MAXN * DK;
  // Large bonds (chi * Dk above the LDS-resident limit): the working matrices X, A | J and R | G
  // live in a per-sample slot of global memory (wbig, kBigSlot doubles; the working set stays in
  // the L2 and last-level caches), the Jacobi's hand-over buffers and rotation ring in LDS.
  constexpr bool BIG = MAXN > kMaxN;
  static_assert(!BIG || MAXN == kMaxNBig, "one large-bond instantiation");
  // sX holds the QR matrix (MAXM x MAXN) and later A and J of the Jacobi (2 x MAXN^2)
  constexpr int XSIZE = (MAXM * MAXN > 2 * (MAXN + 1) * MAXN) ? MAXM * MAXN : 2 * (MAXN + 1) * MAXN;
  constexpr int XPT = (MAXM * MAXN + kThreads - 1) / kThreads;  // X entries per thread
  // staging chunk of Q in the Theta product (KCH rows of Q^T) and the LDS buffer sB that holds it,
  // the Householder vector pair and (LDS-resident case) the boundary site
  constexpr int KCH = BIG ? 8 : ((MAXN / (DK * DK)) / 4 * 4 < 16 ? (MAXN / (DK * DK)) / 4 * 4 : 16);
  constexpr int SBSIZE = BIG ? (MAXM * KCH > 2 * MAXM ? MAXM * KCH : 2 * MAXM) : MAXN * MAXN / DK;
  static_assert(!BIG || XSIZE + (MAXN + 1) * MAXN + MAXM * MAXN <= kBigSlot, "large-bond slot");
  using TS = TapeSlot<MAXN>;
  __shared__ double sXl[BIG ? 1 : XSIZE];
  __shared__ double sRl[BIG ? 1 : (MAXN + 1) * MAXN];
  __shared__ double sB[SBSIZE];
  __shared__ double sHB[BIG ? 2 * (MAXN / 2) * (MAXN + 8) : 1];  // Jacobi hand-over buffers (padded slots)
  __shared__ double2 sRing[BIG ? 4 * (MAXN / 2) : 1];      // Jacobi rotation ring
  __shared__ double sT[DK * DK * DK * DK];
  __shared__ double sTau[MAXN];
  __shared__ double sSig[MAXN];
  __shared__ double sScal[kWaves];
  __shared__ int sPerm[MAXN];
  __shared__ int sCol[MAXN];  // sorted-column QR: rank of each Theta column by norm
  __shared__ int sFlag[2];
  // phase clocks (d.phase_clk set): cycles per phase and the last mark, kept by thread 0 in LDS
  __shared__ unsigned long long sPh[PEPS_PH_COUNT + 1];

  if (!valid[b]) return;
  const bool phon = d.phase_clk != nullptr;
  if (phon && threadIdx.x == 0) {
    for (int p = 0; p < PEPS_PH_COUNT; ++p) sPh[p] = 0;
    sPh[PEPS_PH_COUNT] = __builtin_readcyclecounter();
  }
  // thread 0 books the cycles since the previous mark to phase p (called right after a barrier)
  auto mark = [&](int p) {
    if (phon && threadIdx.x == 0) {
      const unsigned long long t = __builtin_readcyclecounter();
      sPh[p] += t - sPh[PEPS_PH_COUNT];
      sPh[PEPS_PH_COUNT] = t;
    }
  };
  double* const sX = BIG ? wbig + (size_t)b * kBigSlot : sXl;
  double* const sR = BIG ? sX + XSIZE : sRl;
  double* const sY = BIG ? sR + (MAXN + 1) * MAXN : sXl;  // Y = R_{c-1} B_c (in place in sX when LDS)
  const int L = d.L, Dk = DK;
  const int* bprev = bond_all + (size_t)(y - 1) * (L + 1);
  const int* bnew = bond_all + (size_t)y * (L + 1);
  const int* qrk = qrk_all + (size_t)y * L;
  const double* pb = proj + ((size_t)b * d.n_sites + (size_t)y * L) * d.P4;
  const double* prev = prev_row + (size_t)b * d.row_stride;
  double* outp = out_row + (size_t)b * d.row_stride;
  double* qs = qscr + (size_t)b * L * qslot;
  double* tp = tape ? tape + (size_t)b * L * TS::size : nullptr;

  // ---------------- left to right: X_c = R_{c-1} M_c, QR ----------------
  int r_prev = 1;
  if (threadIdx.x == 0) sR[0] = 1.0;
  __syncthreads();
  int m_last = 0;
  for (int c = 0; c < L; ++c) {
    const int dl = c > 0 ? Dk : 1, dr = c < L - 1 ? Dk : 1;
    const int bc = bprev[c], bn = bprev[c + 1];
    const double* Bs = prev + (size_t)c * d.site_stride;  // [a][dd][a']
    if constexpr (!BIG)
      for (int i = threadIdx.x; i < bc * Dk * bn; i += kThreads) sB[i] = Bs[i];
    for (int i = threadIdx.x; i < dl * dr * Dk * Dk; i += kThreads) sT[i] = pb[(size_t)c * d.P4 + i];
    __syncthreads();
    // Y[(i,l)][(dd,a')] = sum_a R[i][a*dl+l] B[a][(dd,a')]   (into sY; R carries the Schmidt
    // weights: kept in FP64 on both paths)
    {
      const int ncol = Dk * bn;
      mfma_gemm(r_prev * dl, ncol, bc,
                      [&](int il, int a) { return sR[(size_t)(a * dl + il % dl) * MAXN + il / dl]; },
                      [&](int a, int col) { return BIG ? Bs[a * ncol + col] : sB[a * ncol + col]; },
                      [&](int il, int col, double v) { sY[(size_t)il * ncol + col] = v; });
    }
    __syncthreads();
    // X[(i,u),(a',rr)] = sum_{l,dd} Y[i][l][dd][a'] T[l][rr][dd][u]   (registers, then sX)
    const int m = r_prev * Dk, n = bn * dr;
    // FP32 arithmetic sees Y scaled by an exact power of two that brings its largest entry into
    // [1/2, 1): Y follows the partial norms of the row, which leave FP32's exponent range on large
    // lattices (Z4 32 x 32: about e^-50 per row on average); the scale is undone in FP64.
    double ysc = 1.0, yun = 1.0;
    if constexpr (sizeof(CT) < sizeof(double)) {
      double mx = 0.0;
      for (int idx = threadIdx.x; idx < r_prev * dl * Dk * bn; idx += kThreads) mx = fmax(mx, fabs(sY[idx]));
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
      if ((threadIdx.x & 63) == 0) sScal[threadIdx.x >> 6] = mx;
      __syncthreads();
      mx = 0.0;
      for (int w = 0; w < kWaves; ++w) mx = fmax(mx, sScal[w]);
      if (mx > 0.0 && mx <= 1.7976931348623157e308) {
        int e = 0;
        (void)frexp(mx, &e);
        ysc = ldexp(1.0, -e);
        yun = ldexp(1.0, e);
      }
    }
    auto x_entry = [&](int idx) -> double {
      const int row = idx % m, col = idx / m;
      const int i = row / DK, u = row % DK, ap = col / dr, rr = col % dr;
      CT acc = 0;
#pragma unroll
      for (int l = 0; l < DK; ++l)
#pragma unroll
        for (int dd = 0; dd < DK; ++dd)
          if (l < dl) {
            if constexpr (sizeof(CT) < sizeof(double))
              acc += (CT)(sY[((i * dl + l) * DK + dd) * bn + ap] * ysc) *
                     (CT)sT[((l * dr + rr) * DK + dd) * DK + u];
            else
              acc += sY[((i * dl + l) * DK + dd) * bn + ap] * sT[((l * dr + rr) * DK + dd) * DK + u];
          }
      if constexpr (sizeof(CT) < sizeof(double))
        return (double)acc * yun;
      else
        return acc;
    };
    if constexpr (BIG) {
      // Y and X in separate global buffers: no staging
      for (int idx = threadIdx.x; idx < m * n; idx += kThreads) sX[idx] = x_entry(idx);
    } else {
      // in place in LDS: every thread's entries read before any is written
      double xr[XPT];
#pragma unroll
      for (int q = 0; q < XPT; ++q) {
        const int idx = threadIdx.x + q * kThreads;
        xr[q] = (idx < m * n) ? x_entry(idx) : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < XPT; ++q) {
        const int idx = threadIdx.x + q * kThreads;
        if (idx < m * n) sX[idx] = xr[q];
      }
    }
    __syncthreads();
    mark(PEPS_PH_X);
    if (c == L - 1) {
      m_last = m;
      break;
    }
    const int k = qrk[c];
    double* qdst = qs + (size_t)c * qslot;
    householder_qr<MAXM, MAXN>(sX, m, n, sR, MAXN, sTau, sB, qdst);
    if (tp) {
      double* tr = tp + (size_t)c * TS::size + TS::R;
      for (int i = threadIdx.x; i < MAXN * n; i += kThreads) tr[i] = sR[i];
    }
    r_prev = k;
    __syncthreads();
    mark(PEPS_PH_QR);
  }

  // ---------------- right to left: Theta_c, Jacobi SVD, truncate ----------------
  // Jacobi storage: columns padded to an odd stride (ld = rows + 1) against LDS bank conflicts
  double* A = sX;
  double* Jm = sX + (MAXN + 1) * MAXN;
  double* G = sR;  // G[i][a] at G[i*MAXN + a]
  double* const hb = BIG ? sHB : A;
  double2* const ring = BIG ? sRing : reinterpret_cast<double2*>(Jm);
  // J lanes above the column groups: (MAXN / 2) * GW lanes, rounded up to whole waves
  constexpr int JL0 = BIG ? ((MAXN / 2) * GW + 63) / 64 * 64 : kJLane0;
  int chi_next = 1;
  bool converged = true;  // every SVD of the row (same value on every thread)
  for (int i = threadIdx.x; i < m_last; i += kThreads) sB[i] = sX[i];  // Theta_{L-1}
  __syncthreads();
  for (int c = L - 1; c >= 1; --c) {
    const int mA = qrk[c - 1];     // rows of Theta_c
    const int nA = Dk * chi_next;  // cols of Theta_c, index (u, j)
    // Jacobi on Theta^T unless Theta is tall: Theta's columns (u, j) carry the previous cut's
    // singular values, and on the square case the graded orientation needs ~1.7x more sweeps
    const bool trans = mA <= nA;
    const int nr = trans ? nA : mA, nc = trans ? mA : nA;
    constexpr int lda = MAXN + 1, ldj = MAXN + 1;  // the Jacobi's padded column stride
    // PEPS_PRECOND_QR_T: large Theta^T = Q_x R_x first (Householder), then the Jacobi on R_x^T:
    // on the boundary matrices of this method that takes 6.5 instead of 11.5 sweeps (CPU
    // experiment on captured 72 x 72 Theta).  Theta = (R_x^T W Sigma^-1) Sigma (Q_x W)^T, so the
    // left vectors are the normalised Jacobi columns and the right vectors Q_x W.  Only for sweeps
    // that are never reversed (the up sweeps): a left vector of singular value s then carries an
    // error ~ eps ||Theta|| / s, which the truncated-SVD backward would amplify by 1 / s_kept
    // through the kept-discarded terms (Euler identity off by 4e-9 instead of ~1e-13), and a
    // reversed sweep must repeat the forward arithmetic exactly; the kept vectors are unaffected.
    const bool pre = pmode == PEPS_PRECOND_QR_T && trans && mA >= pthr;
    // PEPS_PRECOND_SORTED_QR preconditions from the other side: Theta's columns sorted by norm
    // (P), Theta P = Q_1 R (Householder), and the Jacobi on R^T: R^T W = Y Sigma gives
    // Theta = (Q_1 W) Sigma (P Y)^T, so the left vectors are accumulated (Q_1 W, orthogonal to
    // rounding) and the right vectors are the normalised Jacobi columns, the same split as the
    // Jacobi on Theta^T itself; 8.0 instead of 11.5 sweeps on the captured 72 x 72 Theta.
    const bool sq = pmode == PEPS_PRECOND_SORTED_QR && trans && mA >= pthr;
    const bool jt = trans && !pre;  // left vectors accumulated, right vectors from the columns
    if (c == L - 1) {
      for (int idx = threadIdx.x; idx < mA * nA; idx += kThreads) {
        const int i = idx / nA, col = idx % nA;
        const double v = sB[i * Dk + col];  // chi_next = 1: col = u
        (sq ? Jm[(size_t)col * mA + i]
            : A[pre ? (size_t)i * nA + col : trans ? (size_t)i * lda + col : (size_t)col * lda + i]) = v;
      }
    } else {
      const int kc = qrk[c];
      const double* Qc = qs + (size_t)c * qslot;
      const int mq = mA * Dk;
      // Theta[i][(u,j)] = sum_t Q[(i,u)][t] G[t][j]   (G = U_k S_k spans the kept singular
      // values: FP64 on both paths)
      // chunks of Q (MAXM rows) staged through sB
      constexpr int SPT = (MAXM * KCH + kThreads - 1) / kThreads;
      // tiles per wave: G has chi_next <= MAXN / DK columns (counted as MAXN in the LDS kernels)
      constexpr int QT = ((MAXM + 15) / 16 * (((BIG ? MAXN / DK : MAXN) + 15) / 16) + kWaves - 1) / kWaves;
      static_assert(KCH >= 4 && MAXM * KCH <= SBSIZE, "staging chunk fits sB");
      mfma_gemm_staged<QT, KCH, SPT, true>(
          mq, chi_next, kc, [&](int iu, int t) { return Qc[(size_t)t * mq + iu]; },
          [&](int t, int j) { return G[t * MAXN + j]; }, sB, [&](int iu, int j, double v) {
            const int i = iu / Dk, col = (iu % Dk) * chi_next + j;
            (sq ? Jm[(size_t)col * mA + i]
                : A[pre ? (size_t)i * nA + col : trans ? (size_t)i * lda + col : (size_t)col * lda + i]) = v;
          });
    }
    __syncthreads();
    mark(PEPS_PH_THETA);
    if (pre) {
      // Theta^T (nA x mA, ld nA) = Q_x R_x: R_x into the J area, Q_x into sR (G is consumed)
      householder_qr<MAXN, MAXN>(A, nA, mA, Jm, MAXN, sTau, sB, sR);
      // B = R_x^T (mA x mA, lower triangular) into the Jacobi's A area
      for (int idx = threadIdx.x; idx < mA * mA; idx += kThreads) {
        const int i = idx / mA, r = idx % mA;  // column i of B, row r
        A[(size_t)i * lda + r] = (r >= i) ? Jm[(size_t)r * MAXN + i] : 0.0;
      }
      __syncthreads();
      mark(PEPS_PH_PRECOND);
      converged &= jacobi_svd<MAXN, GW, JL0>(A, mA, mA, Jm, sSig, sPerm, sFlag, sScal, d.max_sweeps, hb, ring);
      mark(PEPS_PH_JACOBI);
      // V = Q_x W (nA x mA) over W in the J area
      mfma_gemm_sync<((MAXN + 15) / 16) * ((MAXN + 15) / 16) / kWaves + 1>(
          nA, mA, mA, [&](int i, int t) { return sR[(size_t)t * nA + i]; },
          [&](int t, int pp) { return Jm[(size_t)pp * ldj + t]; },
          [&](int i, int pp, double v) { Jm[(size_t)pp * ldj + i] = v; });
      __syncthreads();
    } else if (sq) {
      // Theta (mA x nA, ld mA) is in the J area: column norms, ranks (descending, ties by index)
      {
        const int g8 = threadIdx.x >> 3, l8 = threadIdx.x & 7;
        for (int col = g8; col < nA; col += kThreads / 8) {
          double s2 = 0.0;
          for (int i = l8; i < mA; i += 8) s2 += Jm[(size_t)col * mA + i] * Jm[(size_t)col * mA + i];
          s2 = group8_sum(s2);
          if (l8 == 0) sSig[col] = s2;
        }
      }
      __syncthreads();
      for (int col = threadIdx.x; col < nA; col += kThreads) {
        const double sc = sSig[col];
        int rank = 0;
        for (int j = 0; j < nA; ++j) rank += (sSig[j] > sc) || (sSig[j] == sc && j < col);
        sCol[col] = rank;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < mA * nA; idx += kThreads) {
        const int col = idx / mA, i = idx % mA;
        A[(size_t)sCol[col] * mA + i] = Jm[idx];
      }
      __syncthreads();
      // Theta P = Q_1 R: R (mA x nA) into the J area, Q_1 (mA x mA, ld mA) into sR (G is consumed)
      householder_qr<MAXN, MAXN>(A, mA, nA, Jm, MAXN, sTau, sB, sR);
      // B = R^T (nA x mA): column i is row i of R
      for (int idx = threadIdx.x; idx < mA * nA; idx += kThreads) {
        const int i = idx / nA, r = idx % nA;
        A[(size_t)i * lda + r] = (r >= i) ? Jm[(size_t)r * MAXN + i] : 0.0;
      }
      __syncthreads();
      mark(PEPS_PH_PRECOND);
      converged &= jacobi_svd<MAXN, GW, JL0>(A, nA, mA, Jm, sSig, sPerm, sFlag, sScal, d.max_sweeps, hb, ring);
      mark(PEPS_PH_JACOBI);
      // U = Q_1 W (mA x mA) over W in the J area
      mfma_gemm_sync<((MAXN + 15) / 16) * ((MAXN + 15) / 16) / kWaves + 1>(
          mA, mA, mA, [&](int i, int t) { return sR[(size_t)t * mA + i]; },
          [&](int t, int pp) { return Jm[(size_t)pp * ldj + t]; },
          [&](int i, int pp, double v) { Jm[(size_t)pp * ldj + i] = v; });
      __syncthreads();
    } else {
      converged &= jacobi_svd<MAXN, GW, JL0>(A, nr, nc, Jm, sSig, sPerm, sFlag, sScal, d.max_sweeps, hb, ring);
      mark(PEPS_PH_JACOBI);
    }
    // row of the Jacobi's columns that holds Theta column col (the sorted-column QR permutes them)
    auto vrow = [&](int col) { return sq ? sCol[col] : col; };
    const int kk = bnew[c];
    double* S = outp + (size_t)c * d.site_stride;  // [a][u][j], a < kk
    for (int idx = threadIdx.x; idx < kk * nA; idx += kThreads) {
      const int a = idx / nA, col = idx % nA;
      const int p = sPerm[a];
      if (!jt) {
        S[idx] = Jm[(size_t)p * ldj + col];
      } else {
        const double sg = sSig[p];
        S[idx] = (sg > 0.0) ? A[(size_t)p * lda + vrow(col)] / sg : 0.0;
      }
    }
    if (tp) {
      // singular vectors in descending order: the normalised Jacobi columns on one side, the
      // accumulated rotations on the other
      double* ts = tp + (size_t)c * TS::size;
      const int np = pre ? mA : nc;  // triplets
      for (int idx = threadIdx.x; idx < np * MAXN; idx += kThreads) {
        const int a = idx / MAXN, row = idx % MAXN;
        const int p = sPerm[a];
        const double sg = sSig[p];
        // left vectors (rows < mA) and right vectors (rows < nA)
        const double an_u = (row < mA && sg > 0.0) ? A[(size_t)p * lda + row] / sg : 0.0;
        const double an_v = (row < nA && sg > 0.0) ? A[(size_t)p * lda + vrow(row)] / sg : 0.0;
        const double j_u = (row < mA) ? Jm[(size_t)p * ldj + row] : 0.0;
        const double j_v = (row < nA) ? Jm[(size_t)p * ldj + row] : 0.0;
        ts[TS::U + idx] = jt ? j_u : an_u;
        ts[TS::V + idx] = jt ? an_v : j_v;
      }
      for (int a = threadIdx.x; a < np; a += kThreads) ts[TS::S + a] = sSig[sPerm[a]];
      if (threadIdx.x == 0) ts[TS::F] = trans ? 1.0 : 0.0;
    }
    __syncthreads();  // G_{c+1} fully consumed before it is overwritten
    for (int idx = threadIdx.x; idx < mA * kk; idx += kThreads) {
      const int i = idx / kk, a = idx % kk;
      const int p = sPerm[a];
      G[i * MAXN + a] = jt ? Jm[(size_t)p * ldj + i] * sSig[p] : A[(size_t)p * lda + i];
    }
    __syncthreads();
    mark(PEPS_PH_REST);
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
      if (tp) tp[TS::F + 1] = sSig[0];
    }
    __syncthreads();
    const double nu = sSig[0];
    double* S0 = outp;
    for (int idx = threadIdx.x; idx < n0; idx += kThreads) S0[idx] = sB[idx] / nu;
  }
  if (status && !converged && threadIdx.x == 0) atomicOr(status + b, (uint32_t)PEPS_FLAG_SVD_NOCONV);
  if (phon && threadIdx.x == 0) {
    mark(PEPS_PH_REST);
    for (int p = 0; p < PEPS_PH_COUNT; ++p) atomicAdd(d.phase_clk + p, sPh[p]);
  }
}

// One boundary row for a whole batch of one lattice: one workgroup per sample.
// MINW: waves per SIMD the kernel is compiled for (2: up to 256 VGPRs, one workgroup per CU; 4:
// at most 128 VGPRs, so two workgroups share a CU when their LDS fits, as the chi*Dk <= 32 ones do)
template <int MAXN, int DK, typename CT, int GW, int MINW>
__global__ void __launch_bounds__(kThreads, MINW)
k_row_sweep(Dims d, const int* __restrict__ bond_all, const int* __restrict__ qrk_all, int y,
            const double* __restrict__ proj, const uint8_t* __restrict__ valid,
            const double* __restrict__ prev_row, double* __restrict__ out_row,
            double* __restrict__ qscr, double* __restrict__ lognu, double* __restrict__ tape,
            int pmode, int pthr, uint32_t* __restrict__ status, double* __restrict__ wbig) {
  row_sweep_body<MAXN, DK, CT, GW>(d, bond_all, qrk_all, y, proj, valid, prev_row, out_row, qscr,
                                   (size_t)(MAXN * DK) * MAXN, lognu, tape, pmode, pthr, status, wbig,
                                   (int)blockIdx.x);
}

// Row y of several lattices in one launch (ragged batch): group i owns workgroups
// [first_block_i, first_block_i + B_i); each group brings its own shape tables, tensors, rows and
// scratch (its Q-factor slot stride from its own shapes).
template <int MAXN, int DK, typename CT, int GW, int MINW>
__global__ void __launch_bounds__(kThreads, MINW)
k_row_sweep_ragged(RaggedRows r, int y, int pmode, int pthr) {
  int i = 0;
  while (i + 1 < r.n && (int)blockIdx.x >= r.g[i + 1].first_block) ++i;
  const RaggedRow& g = r.g[i];
  row_sweep_body<MAXN, DK, CT, GW>(g.d, g.bond, g.qrk, y, g.proj, g.valid, g.prev_row, g.out_row, g.qscr,
                                   g.qslot, g.lognu, nullptr, pmode, pthr, g.status, g.wbig,
                                   (int)blockIdx.x - g.first_block);
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

size_t tape_slot_doubles(const Dims& d) {
  return (d.Dk == 2 && d.maxN > kMaxN) ? TapeSlot<kMaxNBig>::size
         : (d.Dk == 2 && d.maxN > 32) ? TapeSlot<72>::size : TapeSlot<32>::size;
}

hipError_t launch_row_sweep(const Dims& d, const DeviceTables& t, int y, const double* proj,
                            const uint8_t* valid, int B, const double* prev_row, double* out_row,
                            double* qscr, double* lognu, double* tape, hipStream_t s, bool up,
                            uint32_t* status, double* wbig) {
  if (B == 0) return hipSuccess;
  if (d.maxN > kMaxN && (d.Dk != 2 || d.maxN > kMaxNBig || !wbig)) return hipErrorInvalidValue;
  const int pmode = up ? d.up_precond : d.down_precond;
  const int pthr = d.precond_min;
#define GIPEPS_ROW(MN, DKV, CTV, GWV, MW)                                                                   \
  hipLaunchKernelGGL((k_row_sweep<MN, DKV, CTV, GWV, MW>), dim3(B), dim3(kThreads), 0, s, d, t.bond, t.qrk, \
                     y, proj, valid, prev_row, out_row, qscr, lognu, tape, pmode, pthr, status, wbig);
#define GIPEPS_ROW_MW(MN, DKV, CTV, GWV)        \
  if (MN <= 32 && d.small_waves == 4) {         \
    GIPEPS_ROW(MN, DKV, CTV, GWV, (MN <= 32 ? 4 : 2)) \
  } else {                                      \
    GIPEPS_ROW(MN, DKV, CTV, GWV, 2)            \
  }
#define GIPEPS_ROW_GW(MN, DKV, CTV)  \
  if (d.jacobi_lanes == 4) {         \
    GIPEPS_ROW_MW(MN, DKV, CTV, 4)   \
  } else {                           \
    GIPEPS_ROW_MW(MN, DKV, CTV, 8)   \
  }
#define GIPEPS_ROW_CT(MN, DKV)     \
  if (d.mixed) {                   \
    GIPEPS_ROW_GW(MN, DKV, float)  \
  } else {                         \
    GIPEPS_ROW_GW(MN, DKV, double) \
  }
  if (d.Dk == 2 && d.maxN <= 32) {
    GIPEPS_ROW_CT(32, 2)
  } else if (d.Dk == 2 && d.maxN <= kMaxN) {
    GIPEPS_ROW_CT(72, 2)
  } else if (d.Dk == 2) {  // large bonds: four Jacobi lanes per column pair (the J rows need the rest)
    if (d.mixed) {
      GIPEPS_ROW(kMaxNBig, 2, float, 4, 2)
    } else {
      GIPEPS_ROW(kMaxNBig, 2, double, 4, 2)
    }
  } else {  // Dk == 1: every bond has dimension 1
    GIPEPS_ROW_CT(32, 1)
  }
#undef GIPEPS_ROW_CT
#undef GIPEPS_ROW_GW
#undef GIPEPS_ROW_MW
#undef GIPEPS_ROW
  return hipGetLastError();
}

hipError_t launch_row_sweep_ragged(const RaggedRows& r, int total_blocks, int y, int Dk, int maxN,
                                   const Dims& tune, hipStream_t s) {
  if (total_blocks == 0) return hipSuccess;
  if (r.n < 1 || r.n > kMaxRagged || Dk != 2 || maxN > kMaxNBig) return hipErrorInvalidValue;
  const int pmode = tune.down_precond, pthr = tune.precond_min;
#define GIPEPS_RAG(MN, CTV, GWV, MW)                                                                         \
  hipLaunchKernelGGL((k_row_sweep_ragged<MN, 2, CTV, GWV, MW>), dim3(total_blocks), dim3(kThreads), 0, s, r, y, \
                     pmode, pthr);
#define GIPEPS_RAG_GW(MN, CTV, MW)    \
  if (tune.jacobi_lanes == 4) {       \
    GIPEPS_RAG(MN, CTV, 4, MW)        \
  } else {                            \
    GIPEPS_RAG(MN, CTV, 8, MW)        \
  }
#define GIPEPS_RAG_CT(MN, MW)         \
  if (tune.mixed) {                   \
    GIPEPS_RAG_GW(MN, float, MW)      \
  } else {                            \
    GIPEPS_RAG_GW(MN, double, MW)     \
  }
  if (maxN <= 32) {
    if (tune.small_waves == 4) {
      GIPEPS_RAG_CT(32, 4)
    } else {
      GIPEPS_RAG_CT(32, 2)
    }
  } else if (maxN <= kMaxN) {
    GIPEPS_RAG_CT(72, 2)
  } else if (tune.mixed) {  // large bonds: four Jacobi lanes per column pair
    GIPEPS_RAG(kMaxNBig, float, 4, 2)
  } else {
    GIPEPS_RAG(kMaxNBig, double, 4, 2)
  }
#undef GIPEPS_RAG_CT
#undef GIPEPS_RAG_GW
#undef GIPEPS_RAG
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Variational compression of one boundary row (the fitting algorithm; SM S-2 "SVD or variational
// compression"): the row's truncated MPS G (k_row_sweep's output: bonds bond[y][c], right-canonical)
// is refined by `sweeps` sweeps of single-site updates that maximise |<G|M>| / ||G|| for the exact
// product M_c[(a,l), u, (b,r)] = sum_d D_c[a, d, b] T_c[l, r, d, u] of row y with D = D_{y-1}
// (never formed).  At site c the optimal tensor is C = L_c M_c R_{c+1} (L, R: overlaps of G's
// canonical sites with M), computed as
//   X1[g, l, d, b]   = sum_a L_c[(a,l), g] D_c[a, d, b]          (matrix cores, one product per l)
//   X2[(g,u),(b,r)]  = sum_{l,d} X1[g, l, d, b] T_c[l, r, d, u]  (per (g, b) pair)
//   C[(g,u), q]      = sum_{(b,r)} X2[(g,u),(b,r)] R_{c+1}[(b,r), q]   (matrix cores)
// Left to right C = Q R (Householder) gives the left-canonical site Q and L_{c+1} = X2^T Q; right to
// left C^T = Q R gives the right-canonical site Q^T and R_c from G_c through
//   Y[(g,u),(b,r)] = sum_q G_c[g, u, q] R_{c+1}[(b,r), q],  W[g, l, d, b] = sum_{u,r} T Y,
//   R_c[(a,l), g] = sum_{d,b} D_c[a, d, b] W[g, l, d, b].
// The last site of a pass keeps C; after the last sweep G_0 = C / ||C|| and ln nu_y = ln ||C||.
// One workgroup per sample; environments (L+1 each) and the Q and R factors in a per-sample global
// scratch (venv), the working products in LDS.
// ---------------------------------------------------------------------------------------------
namespace {
constexpr int kVX = kMaxN * kMaxN;  // (chi Dk) x (chi Dk) doubles: the largest X1 / X2 / C
}

__global__ void __launch_bounds__(kThreads)
k_var_refine(Dims d, const int* __restrict__ bond_all, int y, const double* __restrict__ proj,
             const uint8_t* __restrict__ valid, const double* __restrict__ prev_row, double* __restrict__ out_row,
             double* __restrict__ venv, double* __restrict__ lognu, int sweeps) {
  __shared__ double sX[kVX];
  __shared__ double sC[kVX];
  __shared__ double sTau[kMaxN];
  __shared__ double sV[2 * kMaxN];
  __shared__ double sRed[kWaves];
  const int b = blockIdx.x;
  if (!valid[b]) return;
  const int L = d.L, Dk = d.Dk;
  const int* bP = bond_all + (size_t)(y - 1) * (L + 1);  // bonds of D_{y-1}
  const int* bG = bond_all + (size_t)y * (L + 1);        // bonds of the refined row
  auto hl = [&](int c) { return (c > 0 && c < L) ? Dk : 1; };
  const double* D = prev_row + (size_t)b * d.row_stride;
  double* G = out_row + (size_t)b * d.row_stride;
  const double* T = proj + (size_t)b * d.n_sites * d.P4 + (size_t)y * L * d.P4;
  const size_t slot = (size_t)d.site_stride;
  double* Lenv = venv + (size_t)b * (2 * (L + 1) + 2) * slot;
  double* Renv = Lenv + (size_t)(L + 1) * slot;
  double* qbuf = Renv + (size_t)(L + 1) * slot;   // Q factor (column-major)
  double* rbuf = qbuf + slot;                     // R factor (unused)

  // C = L_c M_c R_{c+1} into sC as column-major [(g,u) + m q] (m = bG[c] Dk); X2 stays in sX
  auto center = [&](int c) {
    const int a0 = bP[c], a1 = bP[c + 1], g0 = bG[c], g1 = bG[c + 1], h0 = hl(c), h1 = hl(c + 1);
    const double* Dc = D + (size_t)c * slot;
    const double* Lc = Lenv + (size_t)c * slot;
    const double* Rn = Renv + (size_t)(c + 1) * slot;
    const double* Tc = T + (size_t)c * d.P4;  // [l][r][d][u], dims h0, h1, Dk, Dk
    for (int l = 0; l < h0; ++l)
      mfma_gemm(g0, Dk * a1, a0, [&](int i, int k) { return Lc[(size_t)(k * h0 + l) * g0 + i]; },
                [&](int k, int j) { return Dc[(size_t)k * Dk * a1 + j]; },
                [&](int i, int j, double v) { sX[((size_t)(i * h0 + l) * Dk) * a1 + j] = v; });
    __syncthreads();
    // X1[g][l][d][b] -> X2[(g,u)][(b,r)] per (g, b) pair, all reads before the barrier
    const int np = g0 * a1;
    constexpr int PPT = (kMaxN * kMaxN / 2 + kThreads - 1) / kThreads + 1;
    double out[PPT][4];
    for (int q = 0; q < PPT; ++q) {
      const int pr = threadIdx.x + q * kThreads;
      if (pr >= np) continue;
      const int g = pr / a1, bb = pr % a1;
      double in[4];
      for (int l = 0; l < h0; ++l)
        for (int dd = 0; dd < Dk; ++dd) in[l * Dk + dd] = sX[((size_t)(g * h0 + l) * Dk + dd) * a1 + bb];
      for (int u = 0; u < Dk; ++u)
        for (int r = 0; r < h1; ++r) {
          double acc = 0.0;
          for (int l = 0; l < h0; ++l)
            for (int dd = 0; dd < Dk; ++dd) acc += in[l * Dk + dd] * Tc[((l * h1 + r) * Dk + dd) * Dk + u];
          out[q][u * h1 + r] = acc;
        }
    }
    __syncthreads();
    for (int q = 0; q < PPT; ++q) {
      const int pr = threadIdx.x + q * kThreads;
      if (pr >= np) continue;
      const int g = pr / a1, bb = pr % a1;
      for (int u = 0; u < Dk; ++u)
        for (int r = 0; r < h1; ++r) sX[(size_t)(g * Dk + u) * (a1 * h1) + bb * h1 + r] = out[q][u * h1 + r];
    }
    __syncthreads();
    const int m = g0 * Dk;
    mfma_gemm(m, g1, a1 * h1, [&](int i, int k) { return sX[(size_t)i * (a1 * h1) + k]; },
              [&](int k, int j) { return Rn[(size_t)k * g1 + j]; },
              [&](int i, int j, double v) { sC[(size_t)i + (size_t)m * j] = v; });
    __syncthreads();
  };
  // R_c[(a,l), g] from the site G_c (row-major [g][u][q]) and R_{c+1}
  auto env_right = [&](int c) {
    const int a0 = bP[c], a1 = bP[c + 1], g0 = bG[c], g1 = bG[c + 1], h0 = hl(c), h1 = hl(c + 1);
    const double* Dc = D + (size_t)c * slot;
    const double* Gc = G + (size_t)c * slot;
    const double* Rn = Renv + (size_t)(c + 1) * slot;
    const double* Tc = T + (size_t)c * d.P4;
    double* Rc = Renv + (size_t)c * slot;
    mfma_gemm(g0 * Dk, a1 * h1, g1, [&](int i, int k) { return Gc[(size_t)i * g1 + k]; },
              [&](int k, int j) { return Rn[(size_t)j * g1 + k]; },
              [&](int i, int j, double v) { sX[(size_t)i * (a1 * h1) + j] = v; });
    __syncthreads();
    const int np = g0 * a1;
    constexpr int PPT = (kMaxN * kMaxN / 2 + kThreads - 1) / kThreads + 1;
    double out[PPT][4];
    for (int q = 0; q < PPT; ++q) {
      const int pr = threadIdx.x + q * kThreads;
      if (pr >= np) continue;
      const int g = pr / a1, bb = pr % a1;
      double in[4];
      for (int u = 0; u < Dk; ++u)
        for (int r = 0; r < h1; ++r) in[u * h1 + r] = sX[(size_t)(g * Dk + u) * (a1 * h1) + bb * h1 + r];
      for (int l = 0; l < h0; ++l)
        for (int dd = 0; dd < Dk; ++dd) {
          double acc = 0.0;
          for (int u = 0; u < Dk; ++u)
            for (int r = 0; r < h1; ++r) acc += Tc[((l * h1 + r) * Dk + dd) * Dk + u] * in[u * h1 + r];
          out[q][l * Dk + dd] = acc;
        }
    }
    __syncthreads();
    for (int q = 0; q < PPT; ++q) {
      const int pr = threadIdx.x + q * kThreads;
      if (pr >= np) continue;
      const int g = pr / a1, bb = pr % a1;
      for (int l = 0; l < h0; ++l)
        for (int dd = 0; dd < Dk; ++dd) sX[((size_t)(g * h0 + l) * Dk + dd) * a1 + bb] = out[q][l * Dk + dd];
    }
    __syncthreads();
    for (int l = 0; l < h0; ++l)
      mfma_gemm(a0, g0, Dk * a1, [&](int i, int k) { return Dc[(size_t)i * Dk * a1 + k]; },
                [&](int k, int j) { return sX[((size_t)(j * h0 + l) * Dk) * a1 + k]; },
                [&](int i, int j, double v) { Rc[(size_t)(i * h0 + l) * g0 + j] = v; });
    __syncthreads();
  };

  if (threadIdx.x == 0) {
    Renv[(size_t)L * slot] = 1.0;
    Lenv[0] = 1.0;
  }
  __syncthreads();
  for (int c = L - 1; c >= 1; --c) env_right(c);
  double nu = 1.0;
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int c = 0; c < L; ++c) {  // left to right
      center(c);
      const int g0 = bG[c], g1 = bG[c + 1], m = g0 * Dk;
      double* Gc = G + (size_t)c * slot;
      if (c == L - 1) {
        for (int i = threadIdx.x; i < m * g1; i += blockDim.x) Gc[(i % m) * g1 + i / m] = sC[i];
        __syncthreads();
        break;
      }
      householder_qr<kMaxN, kMaxN>(sC, m, g1, rbuf, g1, sTau, sV, qbuf);
      __syncthreads();
      for (int i = threadIdx.x; i < m * g1; i += blockDim.x) Gc[(i % m) * g1 + i / m] = qbuf[i];
      // L_{c+1}[(b,r), q] = sum_{(g,u)} X2[(g,u),(b,r)] Q[(g,u), q]
      const int a1 = bP[c + 1], h1 = hl(c + 1);
      double* Ln = Lenv + (size_t)(c + 1) * slot;
      mfma_gemm(a1 * h1, g1, m, [&](int i, int k) { return sX[(size_t)k * (a1 * h1) + i]; },
                [&](int k, int j) { return qbuf[(size_t)k + (size_t)m * j]; },
                [&](int i, int j, double v) { Ln[(size_t)i * g1 + j] = v; });
      __syncthreads();
    }
    for (int c = L - 1; c >= 0; --c) {  // right to left
      center(c);
      const int g0 = bG[c], g1 = bG[c + 1], m = g0 * Dk;
      double* Gc = G + (size_t)c * slot;
      if (c == 0) {
        double ss = 0.0;
        for (int i = threadIdx.x; i < m * g1; i += blockDim.x) ss += sC[i] * sC[i];
        nu = sqrt(block_sum(ss, sRed));
        const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
        for (int i = threadIdx.x; i < m * g1; i += blockDim.x) Gc[(i % m) * g1 + i / m] = sC[i] * inv;
        __syncthreads();
        break;
      }
      // C^T as column-major [(u,q) + (Dk g1) g]: C^T[(u,q)][g] = C[(g,u)][q]
      const int mt = Dk * g1;
      for (int i = threadIdx.x; i < m * g1; i += blockDim.x) {
        const int gu = i % m, q = i / m, g = gu / Dk, u = gu % Dk;
        sX[(size_t)(u * g1 + q) + (size_t)mt * g] = sC[i];
      }
      __syncthreads();
      householder_qr<kMaxN, kMaxN>(sX, mt, g0, rbuf, g0, sTau, sV, qbuf);
      __syncthreads();
      // G_c[g][u][q] = Q[(u,q)][g]
      for (int i = threadIdx.x; i < g0 * Dk * g1; i += blockDim.x) {
        const int g = i / (Dk * g1), uq = i % (Dk * g1);
        Gc[i] = qbuf[(size_t)uq + (size_t)mt * g];
      }
      __syncthreads();
      env_right(c);
    }
  }
  if (threadIdx.x == 0 && sweeps > 0) lognu[(size_t)b * L + y] = log(nu);
}

hipError_t launch_var_refine(const Dims& d, const DeviceTables& t, int y, const double* proj, const uint8_t* valid,
                             int B, const double* prev_row, double* out_row, double* venv, double* lognu,
                             hipStream_t s) {
  if (B == 0 || d.var_sweeps <= 0 || y < 1) return hipSuccess;
  hipLaunchKernelGGL(k_var_refine, dim3(B), dim3(kThreads), 0, s, d, t.bond, y, proj, valid, prev_row, out_row, venv,
                     lognu, d.var_sweeps);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
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
