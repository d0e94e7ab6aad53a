"""Lattice, link labels, Gauss law and plaquette moves (oracle; test infrastructure only).

Paper passages followed:
  * Hamiltonian section: link space spanned by electric eigenstates |n>, n in Z_N; the raising
    operator U maps |n> to |n+1 mod N>.
  * eq. gauss_N and SM S-2 (Gauss law for the gauge canonical form): at every vertex
    (p + n_l + n_d - n_u - n_r) mod N = Q_x, with p the matter occupation.
  * eq. matter and SM S-2 (configuration sampling with matter): the hopping c^dag_x U_(x,a) c_(x+e_a)
    moves a hard-core boson from x + e_a to x and raises the link between them; its conjugate moves
    it back and lowers the link.  Both keep the Gauss law.
  * eq. H_b / SM S-2 (configuration sampling): the plaquette operator
    P_x = U_{x,1} U_{x+e1,2} U^dag_{x+e2,1} U^dag_{x,2} raises the bottom and right links of the
    plaquette and lowers its top and left links, so it preserves the Gauss law.

Conventions (stated once, used everywhere):
  * vertices (x, y), 0 <= x, y < L, open boundary;
  * links[0, y, x] = h(x, y), the link from (x, y) to (x+1, y), defined for x < L-1;
  * links[1, y, x] = v(x, y), the link from (x, y) to (x, y+1), defined for y < L-1;
  * unused slots (x = L-1 in links[0], y = L-1 in links[1]) hold 0;
  * with matter (hard-core bosons) a configuration has a third plane: links[2, y, x] = p(x, y) in
    {0, 1}, the occupation of vertex (x, y); without it p = 0 everywhere;
  * a missing link at the lattice edge counts as label 0 in the Gauss law;
  * plaquette p = (px, py), 0 <= px, py < L-1, has lower-left vertex (px, py).
"""
import itertools

import numpy as np


def n_links(L):
    return 2 * L * (L - 1)


def n_plaquettes(L):
    return (L - 1) * (L - 1)


def link_mask(L):
    """Boolean mask [2, L, L] of the slots that hold real links."""
    m = np.zeros((2, L, L), dtype=bool)
    m[0, :, : L - 1] = True
    m[1, : L - 1, :] = True
    return m


def vertex_legs(links, x, y):
    """Labels (n_l, n_r, n_d, n_u) on the four links meeting at vertex (x, y).

    Absent links (lattice edge) are returned as None.
    """
    L = links.shape[-1]
    n_l = int(links[0, y, x - 1]) if x > 0 else None
    n_r = int(links[0, y, x]) if x < L - 1 else None
    n_d = int(links[1, y - 1, x]) if y > 0 else None
    n_u = int(links[1, y, x]) if y < L - 1 else None
    return n_l, n_r, n_d, n_u


def occupation(links, x, y):
    """Matter occupation p at vertex (x, y): plane 2 of a configuration with matter, else 0."""
    return int(links[2, y, x]) if links.shape[0] == 3 else 0


def gauss_residual(links, N, Q=None):
    """Per-vertex (p + n_l + n_d - n_r - n_u - Q_x) mod N, an int array [L, L] (0 = satisfied).

    Follows eq. gauss_N; absent links count as 0, p = 0 without a matter plane.
    """
    L = links.shape[-1]
    out = np.zeros((L, L), dtype=np.int64)
    for y in range(L):
        for x in range(L):
            n_l, n_r, n_d, n_u = (0 if n is None else n for n in vertex_legs(links, x, y))
            q = 0 if Q is None else int(Q[y, x])
            out[y, x] = (occupation(links, x, y) + n_l + n_d - n_r - n_u - q) % N
    return out


def is_physical(links, N, Q=None):
    return bool(np.all(gauss_residual(links, N, Q) == 0))


def apply_plaquette(links, px, py, t, N):
    """Return P_p^t applied to a configuration: h(px,py) += t, v(px+1,py) += t,
    h(px,py+1) -= t, v(px,py) -= t, all mod N (operator order of eq. H_b)."""
    out = np.array(links, dtype=np.int64, copy=True)
    out[0, py, px] = (out[0, py, px] + t) % N
    out[1, py, px + 1] = (out[1, py, px + 1] + t) % N
    out[0, py + 1, px] = (out[0, py + 1, px] - t) % N
    out[1, py, px] = (out[1, py, px] - t) % N
    return out.astype(np.uint8)


def hop_endpoints(d, x, y):
    """Vertices joined by link (d, x, y): (x, y) and its neighbour along +x (d = 0) or +y (d = 1)."""
    return (x, y), ((x + 1, y) if d == 0 else (x, y + 1))


def apply_hop(links, d, x, y, N):
    """The configuration that the hopping term of link (d, x, y) connects to s, or None.

    With a = (x, y) and b its neighbour: if b holds the boson and a is empty, c^dag_a U c_b moves
    it to a and raises the link; if a holds it and b is empty, the conjugate c^dag_b U^dag c_a moves
    it to b and lowers the link.  Equal occupations (hard-core bosons): no term, None.
    """
    (ax, ay), (bx, by) = hop_endpoints(d, x, y)
    pa, pb = int(links[2, ay, ax]), int(links[2, by, bx])
    if pa == pb:
        return None
    out = np.array(links, dtype=np.int64, copy=True)
    step = 1 if pb == 1 else -1
    out[d, y, x] = (out[d, y, x] + step) % N
    out[2, ay, ax], out[2, by, bx] = pb, pa
    return out.astype(np.uint8)


def links_from_powers(k, N):
    """Configuration prod_p P_p^{k_p} |0>, built by applying the plaquette moves one by one.

    k: int array [L-1, L-1] indexed [py, px].  Starting from the all-zero (physical) field and
    applying only plaquette moves keeps every vertex on the Gauss law (SM S-2).
    """
    L = k.shape[0] + 1
    links = np.zeros((2, L, L), dtype=np.uint8)
    for py in range(L - 1):
        for px in range(L - 1):
            if k[py, px] % N:
                links = apply_plaquette(links, px, py, int(k[py, px]), N)
    return links


def matter_links(k, occ, N, Q=None):
    """A configuration with occupations occ (uint8 [L, L], indexed [y, x]) that obeys the Gauss
    law, times prod_p P_p^{k_p}.

    The flux carries each vertex's charge Q_x - p_x along its row to column 0 and down column 0:
    h(x, y) = sum_{x' > x} (Q - p)(x', y), v(0, y) = sum_{y' > y} sum_x' (Q - p)(x', y'), every
    other vertical link 0 (mod N); vertex (0, 0) then obeys the Gauss law exactly when
    sum_x p_x = sum_x Q_x (mod N).  The plaquette moves are applied on top (SM S-2).
    """
    occ = np.asarray(occ, dtype=np.int64)
    L = occ.shape[0]
    q = (np.zeros((L, L), dtype=np.int64) if Q is None else np.asarray(Q, dtype=np.int64)) - occ
    links = np.zeros((3, L, L), dtype=np.int64)
    for y in range(L):
        for x in range(L - 1):
            links[0, y, x] = np.sum(q[y, x + 1:]) % N
    for y in range(L - 1):
        links[1, y, 0] = np.sum(q[y + 1:, :]) % N
    links[2] = occ
    links = links.astype(np.uint8)
    for py in range(L - 1):
        for px in range(L - 1):
            if k[py, px] % N:
                links = apply_plaquette(links, px, py, int(k[py, px]), N)
    return links


def enumerate_physical(L, N, Q=None):
    """All physical link configurations by brute force over every labelling of every link.

    Exponential in the number of links: only for the smallest lattices (2x2, 3x3).
    Returns an array [n_phys, 2, L, L] in lexicographic order of the flattened real links.
    """
    mask = link_mask(L)
    idx = np.argwhere(mask)
    out = []
    for labels in itertools.product(range(N), repeat=len(idx)):
        links = np.zeros((2, L, L), dtype=np.uint8)
        for (d, y, x), n in zip(idx, labels):
            links[d, y, x] = n
        if is_physical(links, N, Q):
            out.append(links)
    return np.array(out, dtype=np.uint8)
