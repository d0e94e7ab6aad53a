"""Stochastic-reconfiguration force and overlap matrix (oracle; test infrastructure only).

Paper passages followed:
  * SM S-1 eq. gradient, which is printed with both terms identical (a typesetting slip); it is
    read as the covariance g_m = <O*_m E_loc> - <O*_m><E_loc>;
  * SM S-3: S_mn = <O*_m O_n> - <O*_m><O_n>.
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


def sr_matvec(O, v):
    """S v without forming S: O^T (O v) / B - <O> (<O> . v)."""
    O = np.asarray(O, dtype=np.float64)
    B = O.shape[0]
    o_mean = O.sum(axis=0) / B
    return O.T @ (O @ v) / B - o_mean * float(o_mean @ v)
