"""Block-sparse gauge-invariant site tensors, parameter layout and projection (oracle).

Paper passages followed:
  * eq. A: the vertex tensor A^p_{lrdu} is nonzero only on blocks whose leg charges obey
    p + q(l) + q(d) - q(r) - q(u) = Q_x (mod N); the bond dimension is D = sum_k D_k, D_k the
    degeneracy of charge k.
  * eq. gcf (gauge canonical form): B^n_{lr} = delta_{lr} delta_{n,q(l)} delta_{n,q(r)}, so the
    link tensors carry no parameters and a link label n fixes the charge sector of the virtual
    bond on that link.
  * SM S-2 eq. project and the VMC section: a physical configuration selects exactly one block
    of every vertex tensor; a Gauss-law-violating configuration has amplitude exactly zero.

Layout (the parameter vector theta):
  * sites in row-major order, site index y*L + x;
  * inside a site, the legs present at that vertex in the order (l, r, d, u) (Fig. 1: d is the
    down leg); a leg missing at the lattice edge has dimension 1 and charge 0;
  * blocks = charge tuples of the present legs, in lexicographic order, that obey eq. A with
    p = 0; a block has shape prod(deg[q]) over present legs, stored row-major in (l, r, d, u);
  * with matter (hard-core bosons, p in {0, 1}): all p = 0 blocks of a site, then all p = 1 blocks
    (eq. A with that p), each group ordered as above;
  * offsets are prefix sums over sites and blocks.
"""
import itertools

import numpy as np

from .lattice import occupation, vertex_legs

LEG_NAMES = ("l", "r", "d", "u")


def present_legs(x, y, L):
    """Which of (l, r, d, u) exist at vertex (x, y)."""
    return (x > 0, x < L - 1, y > 0, y < L - 1)


def site_blocks(x, y, L, N, deg, Q=0, p=0):
    """Allowed blocks of the tensor at (x, y) for matter occupation p: list of
    (charges(ql,qr,qd,qu), shape(dl,dr,dd,du)).

    Charges of absent legs are 0 and their dimensions 1.  Order: lexicographic over the
    present legs' charges in (l, r, d, u) order (eq. A).
    """
    pres = present_legs(x, y, L)
    ranges = [range(N) if q else range(1) for q in pres]
    blocks = []
    for ql, qr, qd, qu in itertools.product(*ranges):
        if (p + ql + qd - qr - qu - Q) % N != 0:
            continue
        shape = tuple(deg[q] if p else 1 for q, p in zip((ql, qr, qd, qu), pres))
        blocks.append(((ql, qr, qd, qu), shape))
    return blocks


class Layout:
    """Parameter layout of a GCF gauge-invariant PEPS on an open L x L lattice."""

    def __init__(self, L, N, deg, Q=None, matter=False):
        self.L, self.N = L, N
        self.deg = tuple(int(d) for d in deg)
        assert len(self.deg) == N
        self.Q = np.zeros((L, L), dtype=np.int64) if Q is None else np.asarray(Q, dtype=np.int64)
        self.matter = bool(matter)
        self.blocks = []          # per site: list of (charges, shape, offset), p-major with matter
        self.n_blocks_p = []      # per site: number of blocks of one occupation p
        self.site_offset = [0]
        off = 0
        for y in range(L):
            for x in range(L):
                lst = []
                for p in ((0, 1) if self.matter else (0,)):
                    for ch, shape in site_blocks(x, y, L, N, self.deg, int(self.Q[y, x]) % N, p):
                        lst.append((ch, shape, off))
                        off += int(np.prod(shape))
                    if p == 0:
                        self.n_blocks_p.append(len(lst))
                self.blocks.append(lst)
                self.site_offset.append(off)
        self.n_params = off

    def site(self, x, y):
        return y * self.L + x

    def block_index(self, x, y, charges, p=0):
        s = self.site(x, y)
        lo = p * self.n_blocks_p[s]
        for i, (ch, _, _) in enumerate(self.blocks[s][lo: lo + self.n_blocks_p[s]]):
            if ch == tuple(charges):
                return lo + i
        raise KeyError((x, y, charges, p))


def site_charges(links, x, y):
    """Charges (ql, qr, qd, qu) selected at (x, y): in GCF each virtual charge equals the
    label of its link (eq. gcf); absent legs carry charge 0."""
    return tuple(0 if n is None else n for n in vertex_legs(links, x, y))


def project(layout, theta, links):
    """Projected single-sector tensors of one configuration (SM S-2 eq. project).

    Returns (valid, tensors, block_ids): tensors[y][x] is the selected block of A_(x,y) as a
    4-index array (l, r, d, u) with the block's shape, block_ids[y, x] its index in the site's
    block list.  If any vertex violates the Gauss law the amplitude is exactly zero: valid is
    False and tensors is None.  With matter the occupation p of each vertex (plane 2) takes part
    in the Gauss law and selects the p group of blocks; a layout without matter takes p = 0.
    """
    L = layout.L
    # float64, or complex128 for the complex tensors of real-time evolution (SM S-3)
    dtype = np.complex128 if np.iscomplexobj(theta) else np.float64
    block_ids = np.full((L, L), -1, dtype=np.int64)
    tensors = [[None] * L for _ in range(L)]
    valid = True
    for y in range(L):
        for x in range(L):
            ch = site_charges(links, x, y)
            p = occupation(links, x, y) if layout.matter else 0
            if p not in (0, 1) or (p + ch[0] + ch[2] - ch[1] - ch[3] - int(layout.Q[y, x])) % layout.N != 0:
                valid = False
                continue
            i = layout.block_index(x, y, ch, p)
            _, shape, off = layout.blocks[layout.site(x, y)][i]
            block_ids[y, x] = i
            tensors[y][x] = np.asarray(theta[off: off + int(np.prod(shape))], dtype=dtype).reshape(shape)
    if not valid:
        return False, None, block_ids
    return True, tensors, block_ids
