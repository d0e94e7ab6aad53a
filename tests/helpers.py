"""Shared test helpers: build oracle layouts, random tensors and configurations."""
import numpy as np

from oracle.layout import Layout, project
from oracle.lattice import links_from_powers
from paper_2503_20566_amd import synth


def make_problem(L, N, Dk, seed=1234, scale=None):
    lay = Layout(L, N, [Dk] * N)
    D = N * Dk
    theta = synth.theta_normals(lay.n_params, D if scale is None else scale, seed=seed)
    return lay, theta


def configs(batch, L, N, seed=5678):
    k = synth.plaquette_powers(batch, L, N, seed=seed)
    return np.stack([links_from_powers(k[b], N) for b in range(batch)])


def tensors_of(lay, theta, links):
    ok, T, bid = project(lay, theta, links)
    assert ok
    return T, bid


def toric_theta(lay, Dk_pad):
    """Toric-code tensors in GCF: every allowed block has a single nonzero entry 1 at index
    (0, 0, 0, 0) (for D_k = 1 that is the whole block), so every physical configuration has
    amplitude exactly 1."""
    theta = np.zeros(lay.n_params)
    for site_blocks in lay.blocks:
        for _, shape, off in site_blocks:
            theta[off] = 1.0
    return theta


def gauge_transform(lay, theta, seed, horizontal_general=True, vertical_general=False):
    """Apply random block-diagonal gauge matrices on every bond (eq. gcf's X -> A X, X^-1 B
    with B absorbed into the vertex tensors): invertible on horizontal bonds, orthogonal on
    vertical bonds (invertible there too with vertical_general).  Returns the new vector."""
    L, N, deg = lay.L, lay.N, lay.deg
    Dk = deg[0]
    nh, nv = (L - 1) * L * N, L * (L - 1) * N
    Xh = synth.gauge_matrices(nh, Dk, orthogonal=not horizontal_general, seed=seed)
    Xv = synth.gauge_matrices(nv, Dk, orthogonal=not vertical_general, seed=seed + 1)

    def hmat(x, y, q):
        return Xh[(y * (L - 1) + x) * N + q]

    def vmat(x, y, q):
        return Xv[(y * L + x) * N + q]

    out = np.array(theta, copy=True)
    for y in range(L):
        for x in range(L):
            for (ql, qr, qd, qu), shape, off in lay.blocks[lay.site(x, y)]:
                A = out[off: off + int(np.prod(shape))].reshape(shape)
                if x > 0:      # left leg: X^-1 of the bond shared with the left neighbour
                    A = np.einsum("ij,jrdu->irdu", np.linalg.inv(hmat(x - 1, y, ql)), A)
                if x < L - 1:  # right leg: X
                    A = np.einsum("lrdu,rj->ljdu", A, hmat(x, y, qr))
                if y > 0:
                    A = np.einsum("ij,lrju->lriu", np.linalg.inv(vmat(x, y - 1, qd)), A)
                if y < L - 1:
                    A = np.einsum("lrdu,uj->lrdj", A, vmat(x, y, qu))
                out[off: off + int(np.prod(shape))] = A.reshape(-1)
    return out


def charged_sector(L, N, seed, odd_z2=False):
    """A reference configuration and its background charges Q = its Gauss residual (eq. gauss_N
    with Q_x on the right-hand side).  odd_z2: Z2 strings on the horizontal links (2j, y) -> (2j+1, y)
    (L even), one odd link at every vertex, so Q = 1 everywhere; otherwise uniform random labels."""
    from oracle.lattice import gauss_residual, link_mask
    if odd_z2:
        assert N == 2 and L % 2 == 0
        base = np.zeros((2, L, L), dtype=np.uint8)
        base[0, :, 0::2] = 1
    else:
        base = synth.link_labels(L, N, seed) * link_mask(L).astype(np.uint8)
    return base, gauss_residual(base, N).astype(np.int8)


def sector_configs(base, powers, N):
    """prod_p P_p^{k_p} applied to the reference configuration, one per grid of powers; plaquette
    moves keep every vertex's residual, so all stay in the reference's sector."""
    from oracle.lattice import apply_plaquette
    out = []
    for k in powers:
        s = base.copy()
        for py in range(k.shape[0]):
            for px in range(k.shape[1]):
                if k[py, px]:
                    s = apply_plaquette(s, px, py, int(k[py, px]), N)
        out.append(s)
    return np.stack(out)
