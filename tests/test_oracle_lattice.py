"""Pins of the oracle's lattice and layout code against counting, brute force and closed forms."""
import numpy as np
import pytest

from oracle import ed
from oracle.lattice import (apply_plaquette, enumerate_physical, gauss_residual, is_physical,
                            links_from_powers, n_plaquettes)
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth


@pytest.mark.parametrize("L,N", [(2, 2), (2, 3), (2, 4), (3, 2)])
def test_physical_space_dimension_bruteforce(L, N):
    # Open lattice, Q = 0: the physical space is spanned by plaquette powers, N^{N_plaq} states.
    phys = enumerate_physical(L, N)
    assert len(phys) == N ** n_plaquettes(L)


def test_two_enumerations_agree_and_match_plaquette_powers():
    # brute force over labellings (lattice.py) vs vectorised basis filter (ed.py) vs the image of
    # all plaquette-power grids: three independent constructions of the same set (Z2, 3x3).
    L, N = 3, 2
    a = {p.tobytes() for p in enumerate_physical(L, N)}
    b = {p.tobytes() for p in ed.physical_basis(L, N)[1]}
    grids = np.array(np.meshgrid(*[range(N)] * 4, indexing="ij")).reshape(4, -1).T
    c = {links_from_powers(g.reshape(2, 2), N).tobytes() for g in grids}
    assert a == b == c


def test_z3_3x3_dimension():
    idx, links = ed.physical_basis(3, 3)
    assert len(idx) == 3 ** 4


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_plaquette_moves_preserve_gauss_law(N):
    rng = np.random.default_rng(N)
    L = 5
    links = links_from_powers(rng.integers(0, N, (L - 1, L - 1)), N)
    assert is_physical(links, N)
    for _ in range(30):
        px, py, t = rng.integers(0, L - 1), rng.integers(0, L - 1), rng.integers(1, N)
        links = apply_plaquette(links, px, py, t, N)
        assert np.all(gauss_residual(links, N) == 0)


def test_plaquette_move_touches_exactly_four_links_and_inverts():
    N, L = 3, 4
    z = np.zeros((2, L, L), dtype=np.uint8)
    s = apply_plaquette(z, 1, 1, 1, N)
    assert int((s != 0).sum()) == 4
    assert s[0, 1, 1] == 1 and s[1, 1, 2] == 1 and s[0, 2, 1] == 2 and s[1, 1, 1] == 2
    assert np.array_equal(apply_plaquette(s, 1, 1, N - 1, N), z)


def test_violating_configuration_detected():
    N, L = 3, 3
    s = np.zeros((2, L, L), dtype=np.uint8)
    s[0, 1, 0] = 1                      # a single raised link breaks two vertices
    r = gauss_residual(s, N)
    assert int((r != 0).sum()) == 2


@pytest.mark.parametrize("L,N,Dk", [(4, 2, 1), (16, 2, 2), (16, 3, 2), (32, 4, 2), (8, 4, 2),
                                    (12, 4, 2), (24, 4, 2), (10, 2, 3), (5, 5, 3)])
def test_parameter_count_closed_form(L, N, Dk):
    # eq. A with p = 0: for n present legs one charge is fixed by the others, so a site holds
    # N^{n-1} blocks of D_k^n entries each.
    lay = Layout(L, N, [Dk] * N)
    closed = 0
    for y in range(L):
        for x in range(L):
            n = (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1)
            closed += N ** (n - 1) * Dk ** n
    assert lay.n_params == closed


def test_parameter_counts_of_the_workloads():
    want = {"z2_4x4_d2": 72, "z2_16x16_d4": 26912, "z3_16x16_d6": 88752, "z4_32x32_d8": 937024,
            "z4_32x32_d8_chi36": 937024}
    for name, w in synth.WORKLOADS.items():
        assert Layout(w["L"], w["N"], [w["Dk"]] * w["N"]).n_params == want[name]


def test_blocks_lexicographic_and_gauss_allowed():
    lay = Layout(3, 3, [2, 1, 3])
    for site in lay.blocks:
        chs = [b[0] for b in site]
        assert chs == sorted(chs)
        for (ql, qr, qd, qu), shape, _ in site:
            assert (ql + qd - qr - qu) % 3 == 0


def test_projection_selects_link_sectors_and_zero_for_unphysical():
    L, N, Dk = 4, 3, 2
    lay = Layout(L, N, [Dk] * N)
    theta = np.arange(lay.n_params, dtype=float)
    s = links_from_powers(np.array([[1, 2, 0], [0, 1, 1], [2, 2, 1]]), N)
    ok, T, bid = project(lay, theta, s)
    assert ok
    for y in range(L):
        for x in range(L):
            ch, shape, off = lay.blocks[lay.site(x, y)][bid[y, x]]
            ql = s[0, y, x - 1] if x > 0 else 0
            qr = s[0, y, x] if x < L - 1 else 0
            qd = s[1, y - 1, x] if y > 0 else 0
            qu = s[1, y, x] if y < L - 1 else 0
            assert ch == (ql, qr, qd, qu)
            assert T[y][x].reshape(-1)[0] == off
    bad = s.copy()
    bad[1, 0, 0] = (bad[1, 0, 0] + 1) % N
    assert project(lay, theta, bad)[0] is False
