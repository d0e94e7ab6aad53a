"""Log-derivatives O_k(s) = d ln|Psi(s)| / d theta_k (oracle; test infrastructure only).

Paper passage: SM S-1 defines O_m = (1/Psi*) dPsi*/d alpha*_m for the amplitude; for real
tensors this is d ln|Psi| / d theta_k.  The amplitude differentiated here is the canonical
truncated boundary-MPS amplitude of `contract.amplitude` (every step of it, including the QR and
truncated-SVD factorisations), re-expressed with CPU PyTorch float64 operations so that reverse-
mode autodiff supplies the derivative.  Slicing the thin SVD to the kept singular values makes
the backward pass include the kept-discarded coupling terms 1/(s_i^2 - s_j^2).

Per configuration only the selected blocks of every site have a nonzero derivative, so the result
is returned in the projected layout: one array per site with the shape of its selected block.
"""
import numpy as np
import torch


def _row_as_mps(row):
    return [T[:, :, 0, :].permute(0, 2, 1) for T in row]


def _mpo_apply(mps, row):
    out = []
    for B, T in zip(mps, row):
        M = torch.einsum("apb,lrpu->alubr", B, T)
        a, l, u, b, r = M.shape
        out.append(M.reshape(a * l, u, b * r))
    return out


def _compress(mps, chi):
    L = len(mps)
    R = torch.ones((1, 1), dtype=torch.float64)
    qs = []
    for c in range(L - 1):
        X = torch.einsum("ij,jpk->ipk", R, mps[c])
        r, p, n = X.shape
        Q, R = torch.linalg.qr(X.reshape(r * p, n), mode="reduced")
        qs.append(Q.reshape(r, p, Q.shape[1]))
    theta = torch.einsum("ij,jpk->ipk", R, mps[L - 1])
    out = [None] * L
    for c in range(L - 1, 0, -1):
        r, p, n = theta.shape
        U, S, Vh = torch.linalg.svd(theta.reshape(r, p * n), full_matrices=False)
        k = min(chi, S.shape[0])
        out[c] = Vh[:k].reshape(k, p, n)
        theta = torch.einsum("ipj,jk->ipk", qs[c - 1], U[:, :k] * S[:k])
    nu = torch.linalg.norm(theta)
    out[0] = theta / nu
    return out, torch.log(nu)


def _close(mps, row):
    env = torch.ones((1, 1), dtype=torch.float64)
    for B, T in zip(mps, row):
        env = torch.einsum("al,apb,lrp->br", env, B, T[:, :, :, 0])
    return env[0, 0]


def log_abs_amplitude_torch(tensors, chi):
    """ln|Psi| of the canonical truncated contraction as a differentiable torch scalar."""
    L = len(tensors)
    mps = _row_as_mps(tensors[0])
    total = torch.zeros((), dtype=torch.float64)
    for y in range(1, L - 1):
        mps, ln_nu = _compress(_mpo_apply(mps, tensors[y]), chi)
        total = total + ln_nu
    c = _close(mps, tensors[L - 1])
    return total + torch.log(torch.abs(c))


def log_derivatives(tensors, chi):
    """(ln|Psi|, grads) with grads[y][x] = d ln|Psi| / d (selected block of site (x, y))."""
    L = len(tensors)
    leaves = [[torch.tensor(np.asarray(tensors[y][x], dtype=np.float64), requires_grad=True)
               for x in range(L)] for y in range(L)]
    val = log_abs_amplitude_torch(leaves, chi)
    val.backward()
    grads = [[leaves[y][x].grad.numpy().copy() for x in range(L)] for y in range(L)]
    return float(val.item()), grads


def grads_to_theta(layout, block_ids, grads):
    """Scatter per-site block gradients into a dense vector over the parameter layout."""
    out = np.zeros(layout.n_params)
    L = layout.L
    for y in range(L):
        for x in range(L):
            _, shape, off = layout.blocks[layout.site(x, y)][int(block_ids[y, x])]
            out[off: off + int(np.prod(shape))] = grads[y][x].reshape(-1)
    return out


def finite_difference(f, theta, k, step=1e-6):
    """Central difference (f(theta + h e_k) - f(theta - h e_k)) / 2h of a scalar function."""
    tp = np.array(theta, dtype=np.float64, copy=True)
    tm = np.array(theta, dtype=np.float64, copy=True)
    tp[k] += step
    tm[k] -= step
    return (f(tp) - f(tm)) / (2.0 * step)

