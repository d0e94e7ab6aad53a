"""Exact diagonalisation of Z_N gauge theory in the electric basis (oracle; pins only).

Built independently of `lattice.apply_plaquette`, `lattice.apply_hop` and `energy`: the
Hamiltonian of eq. H_b and eq. electric (and, with hard-core bosons, eq. matter) is assembled on
the full tensor-product space from single-link operators (U |n> = |n+1 mod N>, the electric term
diagonal in |n>) and single-site boson operators (c |1> = |0>, c |0> = 0) with Kronecker products,
then restricted to the configurations that obey the Gauss law (eq. gauss_N) and, with matter, hold
a given number of bosons.  Used to pin the local energy: for any wavefunction, the
|Psi|^2-weighted mean of E_loc equals <Psi|H|Psi>/<Psi|Psi>.
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


def _factor_at(op, pos, dims):
    """op acting on factor `pos` of the tensor product with factor dimensions `dims`."""
    left = int(np.prod(dims[:pos], dtype=np.int64))
    right = int(np.prod(dims[pos + 1:], dtype=np.int64))
    return sp.kron(sp.kron(sp.identity(left, format="csr"), sp.csr_matrix(op)),
                   sp.identity(right, format="csr"), format="csr")


def _matter_space(L, N):
    """Factors of the link (x) matter space: the real links in `_link_list` order, then the vertices
    row-major (dimension 2 each); first factor most significant."""
    keys, lpos = _link_list(L)
    sites = [(x, y) for y in range(L) for x in range(L)]
    spos = {v: len(keys) + i for i, v in enumerate(sites)}
    return keys, lpos, sites, spos, [N] * len(keys) + [2] * len(sites)


def hamiltonian_full_matter(L, N, c_tab, e_tab, hop, mass):
    """Sparse H of eq. H_b + eq. electric + eq. matter (hard-core bosons, uniform m_x = mass,
    coupling J = hop) on the whole link (x) matter space."""
    keys, lpos, sites, spos, dims = _matter_space(L, N)
    dim = int(np.prod(dims, dtype=np.int64))
    Uop = np.zeros((N, N))
    for n in range(N):
        Uop[(n + 1) % N, n] = 1.0
    cop = np.array([[0.0, 1.0], [0.0, 0.0]])   # c |1> = |0>
    H = sp.csr_matrix((dim, dim))
    for k in keys:
        H = H + _factor_at(np.diag(np.asarray(e_tab, dtype=float)), lpos[k], dims)
    for py in range(L - 1):
        for px in range(L - 1):
            P = _factor_at(Uop, lpos[(0, py, px)], dims) @ _factor_at(Uop, lpos[(1, py, px + 1)], dims) \
                @ _factor_at(Uop.T, lpos[(0, py + 1, px)], dims) @ _factor_at(Uop.T, lpos[(1, py, px)], dims)
            Pt = sp.identity(dim, format="csr")
            for t in range(1, N):
                Pt = Pt @ P
                if c_tab[t] != 0.0:
                    H = H + c_tab[t] * Pt
    for d, y, x in keys:
        a, b = (x, y), ((x + 1, y) if d == 0 else (x, y + 1))
        Tm = _factor_at(cop.T, spos[a], dims) @ _factor_at(Uop, lpos[(d, y, x)], dims) @ _factor_at(cop, spos[b], dims)
        H = H + hop * (Tm + Tm.T)
    for v in sites:
        H = H + mass * _factor_at(np.diag([0.0, 1.0]), spos[v], dims)
    return H


def physical_basis_matter(L, N, n_bosons, Q=None):
    """Indices (in the link (x) matter basis) and configurations [n, 3, L, L] (plane 2 = p) of the
    states that obey the Gauss law with matter and hold n_bosons bosons."""
    keys, lpos, sites, spos, dims = _matter_space(L, N)
    dim = int(np.prod(dims, dtype=np.int64))
    digits = np.zeros((dim, len(dims)), dtype=np.int64)
    rem = np.arange(dim)
    for i in range(len(dims) - 1, -1, -1):
        digits[:, i] = rem % dims[i]
        rem //= dims[i]
    ok = np.sum(digits[:, len(keys):], axis=1) == n_bosons
    for (x, y) in sites:
        div = digits[:, spos[(x, y)]].copy()
        if x > 0:
            div += digits[:, lpos[(0, y, x - 1)]]
        if y > 0:
            div += digits[:, lpos[(1, y - 1, x)]]
        if x < L - 1:
            div -= digits[:, lpos[(0, y, x)]]
        if y < L - 1:
            div -= digits[:, lpos[(1, y, x)]]
        q = 0 if Q is None else int(Q[y, x])
        ok &= (div - q) % N == 0
    idx = np.nonzero(ok)[0]
    conf = np.zeros((idx.size, 3, L, L), dtype=np.uint8)
    for i, (d, y, x) in enumerate(keys):
        conf[:, d, y, x] = digits[idx, i]
    for (x, y) in sites:
        conf[:, 2, y, x] = digits[idx, spos[(x, y)]]
    return idx, conf


def physical_hamiltonian(L, N, c_tab, e_tab, Q=None, n_bosons=None, hop=0.0, mass=0.0):
    """Dense H restricted to the physical subspace, with that subspace's configurations.  Pure
    gauge (n_bosons None): link arrays [n, 2, L, L]; with hard-core bosons: [n, 3, L, L]."""
    if n_bosons is None:
        idx, links = physical_basis(L, N, Q)
        H = hamiltonian_full(L, N, c_tab, e_tab)
    else:
        idx, links = physical_basis_matter(L, N, n_bosons, Q)
        H = hamiltonian_full_matter(L, N, c_tab, e_tab, hop, mass)
    return H[idx][:, idx].toarray(), links


def ground_energy(L, N, c_tab, e_tab, Q=None, n_bosons=None, hop=0.0, mass=0.0):
    H, _ = physical_hamiltonian(L, N, c_tab, e_tab, Q, n_bosons, hop, mass)
    return float(np.linalg.eigvalsh(H)[0])
