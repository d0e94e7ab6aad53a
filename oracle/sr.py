"""Stochastic-reconfiguration force and overlap matrix (oracle; test infrastructure only).

Paper passages followed:
  * SM S-1 eq. gradient, which is printed with both terms identical (a typesetting slip); it is
    read as the covariance g_m = <O*_m E_loc> - <O*_m><E_loc>;
  * SM S-3: S_mn = <O*_m O_n> - <O*_m><O_n>;
  * SM S-1 / VMC section: the SR parameter update solves (S + shift I) x = F; at scale S is never
    formed and the solve is conjugate gradients over S v products (Hestenes-Stiefel CG, written
    from its textbook definition).
<...> is the plain sample mean over the batch (weight 1/B each).  Real O here.
"""
import numpy as np


def sr_force_and_mean(O, e_loc):
    """O: [B, n_params] dense log-derivatives, e_loc: [B].  Returns (F, O_mean)."""
    O = np.asarray(O, dtype=np.float64)
    e = np.asarray(e_loc, dtype=np.float64)
    B = O.shape[0]
    o_mean = O.sum(axis=0) / B
    F = (O * e[:, None]).sum(axis=0) / B - o_mean * (e.sum() / B)
    return F, o_mean


def sr_matrix(O):
    """Dense S = <O^T O> - <O>^T <O>."""
    O = np.asarray(O, dtype=np.float64)
    B = O.shape[0]
    o_mean = O.sum(axis=0) / B
    return O.T @ O / B - np.outer(o_mean, o_mean)


def sr_matrix_rows(O, rows):
    """Rows `rows` of S = <O^T O> - <O>^T <O> without forming the rest of S."""
    O = np.asarray(O, dtype=np.float64)
    B = O.shape[0]
    o_mean = O.sum(axis=0) / B
    return O[:, rows].T @ O / B - np.outer(o_mean[rows], o_mean)


def sr_matvec(O, v):
    """S v without forming S: O^T (O v) / B - <O> (<O> . v)."""
    O = np.asarray(O, dtype=np.float64)
    B = O.shape[0]
    o_mean = O.sum(axis=0) / B
    return O.T @ (O @ v) / B - o_mean * float(o_mean @ v)


def sr_solve_cg(O, e_loc, shift, max_iter, rtol):
    """Conjugate gradients for (S + shift I) x = F from x0 = 0, with S v = sr_matvec(O, v).

    Iteration k: q = (S + shift I) p, alpha = r.r / p.q, x += alpha p, r -= alpha q,
    beta = r'.r' / r.r, p = r' + beta p.  Stops when ||r|| <= rtol ||F|| or after max_iter steps.
    Returns (x, iterations, ||r|| / ||F||).
    """
    F, _ = sr_force_and_mean(O, e_loc)
    x = np.zeros_like(F)
    r = F.copy()
    p = r.copy()
    rr = float(r @ r)
    f2 = rr
    if f2 == 0.0:
        return x, 0, 0.0
    k = 0
    while k < max_iter and rr > rtol * rtol * f2:
        q = sr_matvec(O, p) + shift * p
        pq = float(p @ q)
        if pq <= 0.0:
            break
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
    return x, k, float(np.sqrt(rr / f2))
