"""CPU emulation of where FP32 arithmetic can enter the canonical boundary sweep and the strip
ratios (test infrastructure: evidence for the mixed path's choice of FP32 products).

The canonical sweep of the oracle (VMC section; SM S-2 eq. project) is re-expressed with the row
application factored as the kernels factor it: for site c, Y = R_{c-1} B_c (the QR factor times the
boundary site) and X = Y T_c (the contraction with the row tensor), then QR; right to left,
Theta_c = Q_c G_{c+1} and the truncated SVD.  Each product can be rounded to FP32 (operands and
arithmetic in float32, result widened back):
    "xt"    X = Y T             (the library's PEPS_F32_MIXED product)
    "rb"    Y = R B
    "qg"    Theta = Q G
    "strip" every product of the strip contractions that give the local-energy ratios (SM S-1
            eq. Es), and the ratios themselves
QR and SVD stay FP64 (numpy/LAPACK), as do logs and sums.  With no placement the functions equal
the oracle's (checked in the test).
"""
import math

import numpy as np

from oracle.contract import close, flip_vertical, row_as_mps
from oracle.energy import _absorb_left, _absorb_right, _trivial_mps, electric_energy
from oracle.lattice import apply_plaquette
from oracle.layout import project


def _prod(place, key, subscripts, *ops):
    if key in place:
        return np.einsum(subscripts, *[np.asarray(o, dtype=np.float32) for o in ops]).astype(np.float64)
    return np.einsum(subscripts, *ops)


def compress_row(Bmps, row, chi, place):
    """Apply one row to the boundary and compress it (oracle.contract.mpo_apply + compress with
    the kernels' factorisation of the row application).  Returns (new boundary, ln nu)."""
    L = len(row)
    R = np.ones((1, 1))
    qs = []
    X = None
    for c in range(L):
        B, T = Bmps[c], row[c]                    # B[a, d, b], T[l, r, d, u]
        a, dl = B.shape[0], T.shape[0]
        Rr = R.reshape(R.shape[0], a, dl)           # fused left bond (a, l), boundary bond major
        Y = _prod(place, "rb", "ial,adb->ildb", Rr, B)
        X = _prod(place, "xt", "ildb,lrdu->iubr", Y, T)
        i, u, b, r = X.shape
        X = X.reshape(i, u, b * r)
        if c == L - 1:
            break
        Q, R = np.linalg.qr(X.reshape(i * u, b * r), mode="reduced")
        qs.append(Q.reshape(i, u, Q.shape[1]))
    theta = X
    out = [None] * L
    for c in range(L - 1, 0, -1):
        r, p, n = theta.shape
        U, S, Vh = np.linalg.svd(theta.reshape(r, p * n), full_matrices=False)
        k = min(chi, S.shape[0])
        out[c] = Vh[:k].reshape(k, p, n)
        theta = _prod(place, "qg", "ipj,jk->ipk", qs[c - 1], U[:, :k] * S[:k])
    nu = float(np.linalg.norm(theta))
    out[0] = theta / nu
    return out, math.log(nu)


def down_boundaries(tensors, chi, place):
    L = len(tensors)
    D = [row_as_mps(tensors[0])]
    lognu = [0.0]
    for y in range(1, L - 1):
        mps, ln_nu = compress_row(D[-1], tensors[y], chi, place)
        D.append(mps)
        lognu.append(ln_nu)
    return D, lognu


def amplitude(tensors, chi, place):
    L = len(tensors)
    D, lognu = down_boundaries(tensors, chi, place)
    c = close(D[L - 2], tensors[L - 1])
    return sum(lognu) + math.log(abs(c)), math.copysign(1.0, c)


def local_energy(layout, theta, links, chi, c_tab, e_tab, place):
    """E_loc of SM S-1 eq. Es as oracle.energy.local_energy, with the chosen FP32 products."""
    L, N = layout.L, layout.N
    ok, T, _ = project(layout, theta, links)
    assert ok
    D, _ = down_boundaries(T, chi, place)
    Dp, _ = down_boundaries(flip_vertical(T), chi, place)
    U = {L - 1 - yp: m for yp, m in enumerate(Dp)}
    cast = (lambda x: np.asarray(x, dtype=np.float32)) if "strip" in place else (lambda x: x)
    e_off = 0.0
    for py in range(L - 1):
        Dm = D[py - 1] if py >= 1 else _trivial_mps(L)
        Up = U[py + 2] if py + 2 <= L - 1 else _trivial_mps(L)
        E = [cast(np.ones((1, 1, 1, 1)))]
        for c in range(L):
            E.append(_absorb_left(E[-1], cast(Dm[c]), cast(T[py][c]), cast(T[py + 1][c]), cast(Up[c])))
        F = [None] * (L + 1)
        F[L] = cast(np.ones((1, 1, 1, 1)))
        for c in range(L - 1, -1, -1):
            F[c] = _absorb_right(F[c + 1], cast(Dm[c]), cast(T[py][c]), cast(T[py + 1][c]), cast(Up[c]))
        denom = E[L].reshape(())
        for px in range(L - 1):
            for t in range(1, N):
                if c_tab[t] == 0.0:
                    continue
                s2 = apply_plaquette(links, px, py, (N - t) % N, N)
                _, T2, _ = project(layout, theta, s2)
                X = _absorb_left(E[px], cast(Dm[px]), cast(T2[py][px]), cast(T2[py + 1][px]), cast(Up[px]))
                X = _absorb_left(X, cast(Dm[px + 1]), cast(T2[py][px + 1]), cast(T2[py + 1][px + 1]),
                                 cast(Up[px + 1]))
                num = np.einsum("abcd,abcd->", X, F[px + 2])
                e_off += c_tab[t] * float(num / denom)
    return electric_energy(links, e_tab) + e_off
