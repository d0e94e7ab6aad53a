"""Amplitude of a projected GCF PEPS: exact contraction and the canonical boundary MPS (oracle).

Paper passages followed:
  * SM S-2 eq. project: for a physical configuration the amplitude is the single-layer network
    of the selected blocks (bond dimension D_k); it is contracted with standard boundary methods,
    "SVD or variational compression".
  * VMC section: the boundary MPS has cutoff chi (chi = 3 D_k suffices); cost is dominated by the
    boundary compression and the plaquette terms.

The paper does not fix which compression is meant, and different compressions differ at the
truncation-error level, so the amplitude is *defined* here by one algorithm (the reading stated in
the design notes):

  1. B_0 = row 0 as an MPS; site c has indices [left bond l, physical u, right bond r].
  2. for y = 1 .. L-2:
       a. M = row_y applied to B_{y-1}: the boundary's physical leg is summed with the row's d leg,
          the row's u leg becomes the new physical leg, bonds fuse as (boundary bond, row bond),
          boundary bond major.  Exact.
       b. left-to-right sweep of reduced QR factorisations (left-canonical form);
       c. right-to-left sweep of SVDs; at each cut keep k = min(chi, rows, cols) singular values
          (largest first) and absorb U_k S_k into the site on the left;
       d. divide the leftmost site by the 2-norm nu_y of the state; accumulate ln nu_y.
  3. close: c = <row_{L-1} | B_{L-2}> contracted exactly;
  4. ln|Psi| = sum_y ln nu_y + ln|c|, sign(Psi) = sign(c).

The truncated state produced by b-c depends only on the state M (not on the QR/SVD gauge) as long
as singular values at each cut are not degenerate across the cut-off, which is why a GPU path may
reach the same state with different factorisation routines.

Variational compression (the other method the paper names; the fitting algorithm of Verstraete,
Murg and Cirac, Adv. Phys. 57, 143 (2008)), optional: after step 2c the truncated MPS G (bond
dimensions kept) is refined by `var_sweeps` sweeps of single-site updates that maximise the overlap
|<G|M>| / ||G|| with the exact product M, and ln nu_y becomes ln ||G||.  A sweep runs left to right
then right to left; G starts right-canonical (step 2c leaves it so); at site c the optimal tensor
for fixed canonical neighbours is C = L_c M_c R_{c+1}, L and R the overlaps of G's canonical sites
with M's; C is then split by a reduced QR (left to right: G_c = Q, left-canonical; right to left:
G_c = Q^T of the QR of C^T, right-canonical) and the environment advances.  The last site of a
pass keeps C.  Only the span of each Q enters the state, so any QR routine gives the same state
when C has full column rank.
"""
import math

import numpy as np


# ----------------------------------------------------------------------------------------------
# exact contraction (textbook einsum over the whole network; small lattices only)
# ----------------------------------------------------------------------------------------------
def exact_amplitude(tensors):
    """Contract the projected network exactly with numpy.einsum.

    tensors[y][x] is a (l, r, d, u) array; absent legs have dimension 1.  Bond labels: one label
    per horizontal link h(x, y) and per vertical link v(x, y).  Limited by einsum to lattices with
    at most 52 links (L <= 5).
    """
    L = len(tensors)
    lab = {}

    def label(key):
        if key not in lab:
            lab[key] = len(lab)
        return lab[key]

    operands = []
    for y in range(L):
        for x in range(L):
            T = tensors[y][x]
            keep, subs = [], []
            for leg, key in enumerate((("h", x - 1, y), ("h", x, y), ("v", x, y - 1), ("v", x, y))):
                present = (x > 0, x < L - 1, y > 0, y < L - 1)[leg]
                if present:
                    keep.append(leg)
                    subs.append(label(key))
            idx = tuple(slice(None) if leg in keep else 0 for leg in range(4))
            operands.append(T[idx])
            operands.append(subs)
    if len(lab) > 52:
        raise ValueError("exact_amplitude: too many links for einsum")
    return float(np.einsum(*operands, [], optimize="greedy"))


# ----------------------------------------------------------------------------------------------
# boundary MPS pieces
# ----------------------------------------------------------------------------------------------
def row_as_mps(row):
    """Bottom row (d legs of dimension 1) as an MPS with sites [l, u, r]."""
    return [np.ascontiguousarray(T[:, :, 0, :].transpose(0, 2, 1)) for T in row]


def mpo_apply(mps, row):
    """Step 2a: exact application of a row to the boundary MPS.

    B[a, p, a'] with the row tensor T[l, r, d, u]: sum over p = d; result site
    M[(a, l), u, (a', r)] with the boundary bond index major in each fused bond.
    """
    out = []
    for B, T in zip(mps, row):
        M = np.einsum("apb,lrpu->alubr", B, T)
        a, l, u, b, r = M.shape
        out.append(M.reshape(a * l, u, b * r))
    return out


def compress(mps, chi):
    """Steps 2b-2d: QR sweep left to right, truncating SVD sweep right to left, normalisation.

    Returns (new_mps, ln_nu, bond_dims).  Factorisations are LAPACK's (numpy.linalg.qr in reduced
    mode, numpy.linalg.svd with singular values in descending order).
    """
    L = len(mps)
    R = np.ones((1, 1))
    qs = []
    for c in range(L - 1):
        X = np.einsum("ij,jpk->ipk", R, mps[c])
        r, p, n = X.shape
        Q, R = np.linalg.qr(X.reshape(r * p, n), mode="reduced")
        qs.append(Q.reshape(r, p, Q.shape[1]))
    theta = np.einsum("ij,jpk->ipk", R, mps[L - 1])
    out = [None] * L
    for c in range(L - 1, 0, -1):
        r, p, n = theta.shape
        U, S, Vh = np.linalg.svd(theta.reshape(r, p * n), full_matrices=False)
        k = min(chi, S.shape[0])
        out[c] = Vh[:k].reshape(k, p, n)
        theta = np.einsum("ipj,jk->ipk", qs[c - 1], U[:, :k] * S[:k])
    nu = float(np.linalg.norm(theta))
    out[0] = theta / nu
    return out, math.log(nu), [s.shape[0] for s in out] + [1]


def _qr_positive(A):
    """Reduced QR with a nonnegative diagonal of R (a fixed gauge)."""
    Q, R = np.linalg.qr(A, mode="reduced")
    sg = np.where(np.diagonal(R) < 0, -1.0, 1.0)
    return Q * sg


def variational_refine(target, guess, sweeps):
    """Variational compression of the exact product `target` (sites [a, p, b]) into an MPS with the
    bond dimensions of `guess` (right-canonical), by `sweeps` left-right sweeps of single-site
    updates (module docstring).  Returns (normalised MPS, ln ||G||)."""
    L = len(target)
    G = [np.array(g, dtype=np.result_type(g, target[0]), copy=True) for g in guess]
    R = [None] * (L + 1)
    R[L] = np.ones((1, 1))
    for c in range(L - 1, 0, -1):
        R[c] = np.einsum("apb,gpq,bq->ag", target[c], G[c], R[c + 1])
    Lenv = [None] * (L + 1)
    Lenv[0] = np.ones((1, 1))
    for _ in range(sweeps):
        for c in range(L):                                   # left to right
            C = np.einsum("ag,apb,bq->gpq", Lenv[c], target[c], R[c + 1])
            if c == L - 1:
                G[c] = C
                break
            g, p, q = C.shape
            G[c] = _qr_positive(C.reshape(g * p, q)).reshape(g, p, q)
            Lenv[c + 1] = np.einsum("ag,apb,gpq->bq", Lenv[c], target[c], G[c])
        for c in range(L - 1, -1, -1):                       # right to left
            C = np.einsum("ag,apb,bq->gpq", Lenv[c], target[c], R[c + 1])
            if c == 0:
                G[c] = C
                break
            g, p, q = C.shape
            G[c] = _qr_positive(C.reshape(g, p * q).T).T.reshape(g, p, q)
            R[c] = np.einsum("apb,gpq,bq->ag", target[c], G[c], R[c + 1])
    nu = float(np.linalg.norm(G[0]))
    G[0] = G[0] / nu
    return G, math.log(nu)


def close(mps, row):
    """Step 3: exact overlap of the top row (u legs of dimension 1) with the boundary MPS."""
    env = np.ones((1, 1))
    for B, T in zip(mps, row):
        env = np.einsum("al,apb,lrp->br", env, B, T[:, :, :, 0])
    return float(env[0, 0])


def down_boundaries(tensors, chi, var_sweeps=0):
    """Boundary MPSs D_0 .. D_{L-2} and their ln nu (D_0 = row 0, unnormalised, ln nu_0 = 0);
    var_sweeps > 0: each truncated row refined by that many variational sweeps."""
    L = len(tensors)
    D = [row_as_mps(tensors[0])]
    lognu = [0.0]
    for y in range(1, L - 1):
        M = mpo_apply(D[-1], tensors[y])
        mps, ln_nu = compress(M, chi)[:2]
        if var_sweeps > 0:
            mps, ln_nu = variational_refine(M, mps, var_sweeps)
        D.append(mps)
        lognu.append(ln_nu)
    return D, lognu


def amplitude(tensors, chi, var_sweeps=0):
    """Canonical truncated amplitude: returns (ln|Psi|, sign).  Zero amplitude gives (-inf, 0)."""
    L = len(tensors)
    D, lognu = down_boundaries(tensors, chi, var_sweeps)
    c = close(D[L - 2], tensors[L - 1])
    if c == 0.0:
        return -math.inf, 0.0
    return sum(lognu) + math.log(abs(c)), math.copysign(1.0, c)


def flip_vertical(tensors):
    """Mirror the lattice top-to-bottom: row y -> row L-1-y, legs d <-> u."""
    L = len(tensors)
    return [[np.ascontiguousarray(tensors[L - 1 - y][x].transpose(0, 1, 3, 2)) for x in range(L)]
            for y in range(L)]


def up_boundaries(tensors, chi, var_sweeps=0):
    """Up environments U_y for y = L-1 .. 1 (dict y -> MPS with physical legs = row y's d legs).

    Built by the same algorithm on the mirrored lattice: U_y = D'_{L-1-y}.
    """
    L = len(tensors)
    Dp, _ = down_boundaries(flip_vertical(tensors), chi, var_sweeps)
    return {L - 1 - yp: m for yp, m in enumerate(Dp)}
