"""Exact diagonalisation of pure Z_N gauge theory in the link basis (oracle; pins only).

Built independently of `lattice.apply_plaquette` and `energy`: the Hamiltonian of eq. H_b and
eq. electric is assembled on the full tensor-product link space from single-link operators
(U |n> = |n+1 mod N>, the electric term diagonal in |n>) with Kronecker products, then restricted
to the configurations that obey the Gauss law (eq. gauss_N).  Used to pin the local energy:
for any wavefunction, the |Psi|^2-weighted mean of E_loc equals <Psi|H|Psi>/<Psi|Psi>.
"""
import numpy as np
import scipy.sparse as sp


def _link_list(L):
    """Real links in a fixed order; key (dir, y, x) -> position."""
    keys = [(0, y, x) for y in range(L) for x in range(L - 1)] + \
           [(1, y, x) for y in range(L - 1) for x in range(L)]
    return keys, {k: i for i, k in enumerate(keys)}


def _single(op, pos, nl, N):
    mats = [sp.identity(N, format="csr")] * nl
    mats = list(mats)
    mats[pos] = sp.csr_matrix(op)
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(out, m, format="csr")
    return out


def hamiltonian_full(L, N, c_tab, e_tab):
    """Sparse H on the whole link space (dimension N^{#links}); basis index = digits of the link
    labels in `_link_list` order, first link most significant."""
    keys, pos = _link_list(L)
    nl = len(keys)
    Uop = np.zeros((N, N))
    for n in range(N):
        Uop[(n + 1) % N, n] = 1.0
    Eop = np.diag(np.asarray(e_tab, dtype=float))
    dim = N ** nl
    H = sp.csr_matrix((dim, dim))
    for k in keys:
        H = H + _single(Eop, pos[k], nl, N)
    for py in range(L - 1):
        for px in range(L - 1):
            P = _single(Uop, pos[(0, py, px)], nl, N) @ _single(Uop, pos[(1, py, px + 1)], nl, N) \
                @ _single(Uop.T, pos[(0, py + 1, px)], nl, N) @ _single(Uop.T, pos[(1, py, px)], nl, N)
            Pt = sp.identity(dim, format="csr")
            for t in range(1, N):
                Pt = Pt @ P
                if c_tab[t] != 0.0:
                    H = H + c_tab[t] * Pt
    return H


def physical_basis(L, N, Q=None):
    """Indices (in the full link basis) and link arrays [n, 2, L, L] of the Gauss-law states."""
    keys, _ = _link_list(L)
    nl = len(keys)
    dim = N ** nl
    digits = np.zeros((dim, nl), dtype=np.int64)
    rem = np.arange(dim)
    for i in range(nl - 1, -1, -1):
        digits[:, i] = rem % N
        rem //= N
    links = np.zeros((dim, 2, L, L), dtype=np.int64)
    for i, (d, y, x) in enumerate(keys):
        links[:, d, y, x] = digits[:, i]
    ok = np.ones(dim, dtype=bool)
    for y in range(L):
        for x in range(L):
            div = np.zeros(dim, dtype=np.int64)
            if x > 0:
                div += links[:, 0, y, x - 1]
            if y > 0:
                div += links[:, 1, y - 1, x]
            if x < L - 1:
                div -= links[:, 0, y, x]
            if y < L - 1:
                div -= links[:, 1, y, x]
            q = 0 if Q is None else int(Q[y, x])
            ok &= (div - q) % N == 0
    idx = np.nonzero(ok)[0]
    return idx, links[idx].astype(np.uint8)


def physical_hamiltonian(L, N, c_tab, e_tab, Q=None):
    """Dense H restricted to the physical subspace, with that subspace's link configurations."""
    idx, links = physical_basis(L, N, Q)
    H = hamiltonian_full(L, N, c_tab, e_tab)
    return H[idx][:, idx].toarray(), links


def ground_energy(L, N, c_tab, e_tab, Q=None):
    H, _ = physical_hamiltonian(L, N, c_tab, e_tab, Q)
    return float(np.linalg.eigvalsh(H)[0])
