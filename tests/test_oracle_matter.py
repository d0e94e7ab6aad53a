"""Pins of the matter extension of the oracle (Z_N gauge field coupled to hard-core bosons).

Paper passages: eq. gauss_N and eq. A with the matter occupation p; eq. matter (mass and
gauge-covariant hopping); SM S-2 (Gauss law with matter, hopping moves c^dag_x U c_(x+e)).

  * the exact diagonalisation (oracle/ed.py, Kronecker products of single-link and single-site
    operators) reproduces the paper's printed ED energy of the 3 x 3 lattice with 2 bosons
    (tests/golden/ed_z2_boson_3x3.json): this fixes the Hamiltonian's conventions;
  * every hopping move of oracle/lattice.py is an off-diagonal element of that ED Hamiltonian with
    the coupling J, keeps the Gauss law and undoes itself;
  * the local energy with mass and hopping terms obeys the ED identity
    sum |Psi|^2 E_loc / sum |Psi|^2 = <Psi|H|Psi> / <Psi|Psi> at exact chi;
  * the matter layout's projection equals the pure-gauge projection with background charges
    Q - p on the p group of blocks (same tensors, same truncated amplitude, bit for bit);
  * occupations that break the Gauss law give amplitude zero; random block-diagonal gauge
    transformations leave the amplitude unchanged;
  * the configuration builder obeys the Gauss law exactly when the total charge allows it.
"""
import json
import math
import pathlib

import numpy as np
import pytest

from oracle import ed
from oracle.contract import amplitude
from oracle.energy import local_energy, paper_tables
from oracle.lattice import apply_hop, is_physical, link_mask, links_from_powers, matter_links
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth
from tests.helpers import gauge_transform

GOLDEN = json.loads((pathlib.Path(__file__).parent / "golden" / "ed_z2_boson_3x3.json").read_text())
_ED = {}


def ed_3x3():
    """The golden case's physical Hamiltonian (built once: ~10 s)."""
    if "h" not in _ED:
        g = GOLDEN
        c, e = paper_tables(g["N"], g["h"], g["g"])
        _ED["h"] = ed.physical_hamiltonian(g["L"], g["N"], c, e, n_bosons=g["n_bosons"], hop=g["J"], mass=g["mass"])
    return _ED["h"]


def state(lay, theta, cfg, chi):
    psi = []
    for s in cfg:
        ok, T, _ = project(lay, theta, s)
        assert ok
        la, sg = amplitude(T, chi)
        psi.append(sg * math.exp(la))
    return np.array(psi)


def test_ed_reproduces_the_papers_3x3_boson_energy():
    H, cfg = ed_3x3()
    g = GOLDEN
    e0 = np.linalg.eigvalsh(H)[0] / g["L"] ** 2
    print("ED 3x3, 2 bosons: %.12f per site (paper %.10f), %d physical states" % (e0, g["e_site"], len(cfg)))
    assert abs(e0 - g["e_site"]) <= 0.6 * 10.0 ** -g["digits"]


def test_hop_moves_are_the_ed_off_diagonal_elements():
    H, cfg = ed_3x3()
    L, N, J = GOLDEN["L"], GOLDEN["N"], GOLDEN["J"]
    index = {s.tobytes(): i for i, s in enumerate(cfg)}
    rng = np.random.default_rng(3)
    for i in rng.choice(len(cfg), 40, replace=False):
        s = cfg[i]
        hops = set()
        for d, y, x in zip(*np.nonzero(link_mask(L))):
            s2 = apply_hop(s, int(d), int(x), int(y), N)
            if s2 is None:
                continue
            assert is_physical(s2, N) and int(s2[2].sum()) == int(s[2].sum())
            back = apply_hop(s2, int(d), int(x), int(y), N)
            assert back is not None and np.array_equal(back, s)
            j = index[s2.tobytes()]
            assert H[i, j] == J
            hops.add(j)
        # every other off-diagonal element of row i is a plaquette term (coefficient -2h for Z2)
        for j in np.nonzero(H[i])[0]:
            if j != i and j not in hops:
                assert H[i, j] == -2.0 * GOLDEN["h"]


@pytest.mark.parametrize("L,N,Dk,nb,hop,mass", [(2, 2, 2, 2, 0.5, 0.3), (2, 3, 1, 3, -0.7, -0.2), (3, 2, 2, 2, None, None)])
def test_matter_local_energy_ed_identity(L, N, Dk, nb, hop, mass):
    if hop is None:                        # the golden case's Hamiltonian
        (H, cfg), g = ed_3x3(), GOLDEN
        c, e = paper_tables(N, g["h"], g["g"])
        hop, mass = g["J"], g["mass"]
    else:
        c, e = paper_tables(N, 1.0, 0.33)
        H, cfg = ed.physical_hamiltonian(L, N, c, e, n_bosons=nb, hop=hop, mass=mass)
    lay = Layout(L, N, [Dk] * N, matter=True)
    theta = synth.theta_normals(lay.n_params, N * Dk, seed=9)
    chi = Dk ** L * 4
    psi = state(lay, theta, cfg, chi)
    el = np.array([local_energy(lay, theta, s, chi, c, e, hop=hop, mass=mass) for s in cfg])
    lhs = np.sum(psi ** 2 * el) / np.sum(psi ** 2)
    rhs = psi @ H @ psi / (psi @ psi)
    print("L=%d N=%d: <E_loc> %.15f, <H> %.15f over %d states" % (L, N, lhs, rhs, len(cfg)))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    # the scale bounds each E_loc and holds its diagonal part
    for s in cfg[:6]:
        v, m = local_energy(lay, theta, s, chi, c, e, with_scale=True, hop=hop, mass=mass)
        assert abs(v) <= m * (1 + 1e-12) and m >= abs(mass) * int(s[2].sum())


def test_matter_projection_is_background_charge_projection():
    L, N, Dk, chi = 6, 3, 2, 4
    lay = Layout(L, N, [Dk] * N, matter=True)
    theta = synth.theta_normals(lay.n_params, N * Dk, seed=11)
    occ = synth.occupations(3, L, 6)
    k = synth.plaquette_powers(3, L, N)
    for b in range(3):
        s = matter_links(k[b], occ[b], N)
        ok, T, bid = project(lay, theta, s)
        assert ok
        q = (-occ[b].astype(np.int64)) % N
        lay_q = Layout(L, N, [Dk] * N, Q=q)
        th_q = np.zeros(lay_q.n_params)
        for y in range(L):
            for x in range(L):
                st = lay.site(x, y)
                p = int(occ[b, y, x])
                group = lay.blocks[st][p * lay.n_blocks_p[st]: (p + 1) * lay.n_blocks_p[st]]
                assert len(group) == len(lay_q.blocks[st])
                for (ch, shape, off), (ch_q, shape_q, off_q) in zip(group, lay_q.blocks[st]):
                    assert ch == ch_q and shape == shape_q
                    th_q[off_q: off_q + int(np.prod(shape))] = theta[off: off + int(np.prod(shape))]
        ok_q, T_q, bid_q = project(lay_q, th_q, s[:2])
        assert ok_q
        # block id with matter = p * (blocks per occupation) + the background-charge block id
        assert np.array_equal(bid - occ[b] * np.array(lay.n_blocks_p).reshape(L, L), bid_q)
        assert amplitude(T, chi) == amplitude(T_q, chi)


def test_matter_gauss_law_and_gauge_invariance():
    L, N, Dk, chi = 4, 2, 2, 16
    lay = Layout(L, N, [Dk] * N, matter=True)
    theta = synth.theta_normals(lay.n_params, N * Dk, seed=13)
    occ = synth.occupations(4, L, 4)
    k = synth.plaquette_powers(4, L, N)
    th_g = gauge_transform(lay, theta, seed=17)
    for b in range(4):
        s = matter_links(k[b], occ[b], N)
        ok, T, _ = project(lay, theta, s)
        ok_g, T_g, _ = project(lay, th_g, s)
        la, sg = amplitude(T, chi)
        la_g, sg_g = amplitude(T_g, chi)
        assert ok and ok_g and sg == sg_g and abs(la - la_g) <= 1e-11 * abs(la)
        # moving one boson without its flux breaks the Gauss law at two vertices
        s_bad = s.copy()
        y, x = np.argwhere(s[2] == 1)[0]
        y2, x2 = np.argwhere(s[2] == 0)[0]
        s_bad[2, y, x], s_bad[2, y2, x2] = 0, 1
        assert not is_physical(s_bad, N)
        assert not project(lay, theta, s_bad)[0]
        # an occupation outside {0, 1} is not a hard-core boson state
        s_two = s.copy()
        s_two[2, y2, x2] = 2
        assert not project(lay, theta, s_two)[0]


@pytest.mark.parametrize("N", [2, 3, 4])
def test_matter_links_builder(N):
    L = 5
    k = synth.plaquette_powers(6, L, N)
    for nb in range(0, 9):
        occ = synth.occupations(6, L, nb, seed=40 + nb)
        for b in range(6):
            s = matter_links(k[b], occ[b], N)
            assert np.array_equal(s[2], occ[b]) and not s[:2][~link_mask(L)].any()
            assert is_physical(s, N) == (nb % N == 0)
    zero = np.zeros((L, L), dtype=np.uint8)
    assert np.array_equal(matter_links(k[0], zero, N)[:2], links_from_powers(k[0], N))
