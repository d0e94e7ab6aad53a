"""Oracle pins for sectors with background charges Q_x (eq. gauss_N with no matter field; the odd-Z2
theory is Q_x = 1 at every vertex).

* sector sizes: on an open L x L lattice the 2L(L-1) link labels obey L^2 vertex conditions of
  rank L^2 - 1 (their sum is an identity), so a sector with sum_x Q_x = 0 (mod N) holds
  N^{(L-1)^2} = N^{N_plaq} states and any other holds none;
* odd Z2 on 2 x 2: the two physical states (both horizontal or both vertical links odd) each carry
  two odd and two even links, so zero electric energy, and the plaquette swaps them: E_0 = -J for
  every h;
* h = 0: the plaquette moves act freely and transitively on a sector, so the uniform superposition
  has every P_p = 1 and E_0 = -J N_plaq (Z2), -2 J N_plaq (Z_N >= 3) in every sector;
* the layout: every site keeps N^{n-1} blocks of D_k^n entries in any sector, and a configuration
  projects to a valid tensor network exactly when it obeys the charged Gauss law;
* E_loc in a charged sector: sum |Psi|^2 E_loc / sum |Psi|^2 = <Psi|H|Psi> / <Psi|Psi> with H from
  Kronecker products restricted to the sector (independent of the plaquette-move code), and the
  truncated amplitude equals the exact contraction when chi is exact.
"""
import math

import numpy as np
import pytest

from oracle import ed
from oracle.contract import amplitude, exact_amplitude
from oracle.energy import config_tables, local_energy
from oracle.lattice import gauss_residual, is_physical, link_mask, n_plaquettes
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth
from tests.helpers import charged_sector, sector_configs


def _q_with_sum(L, N, seed, total):
    rng = np.random.Generator(np.random.PCG64(seed))
    Q = rng.integers(0, N, size=(L, L))
    Q[-1, -1] = (Q[-1, -1] - Q.sum() + total) % N
    return Q


@pytest.mark.parametrize("L,N", [(2, 2), (2, 3), (3, 2), (2, 4), (3, 3)])
def test_sector_sizes(L, N):
    for seed in range(3):
        Q = _q_with_sum(L, N, seed, 0)
        idx, _ = ed.physical_basis(L, N, Q)
        assert len(idx) == N ** n_plaquettes(L), (Q, len(idx))
        Qbad = _q_with_sum(L, N, seed, 1)
        idx, _ = ed.physical_basis(L, N, Qbad)
        assert len(idx) == 0


@pytest.mark.parametrize("h", [0.0, 0.3, 0.5, 2.0])
def test_odd_z2_2x2_closed_form(h):
    c, e = config_tables(2, 1.0, h)
    Q = np.ones((2, 2), dtype=np.int64)
    H, links = ed.physical_hamiltonian(2, 2, c, e, Q)
    assert len(links) == 2
    assert math.isclose(float(np.linalg.eigvalsh(H)[0]), -1.0, abs_tol=1e-12)


@pytest.mark.parametrize("L,N,odd", [(2, 2, True), (3, 2, False), (2, 3, False), (3, 3, False)])
def test_zero_field_point_in_charged_sectors(L, N, odd):
    c, e = config_tables(N, 1.0, 0.0)
    Q = np.ones((L, L), dtype=np.int64) if odd else _q_with_sum(L, N, 7, 0)
    E0 = ed.ground_energy(L, N, c, e, Q)
    assert math.isclose(E0, -n_plaquettes(L) * (1 if N == 2 else 2), abs_tol=1e-10)


@pytest.mark.parametrize("L,N,Dk", [(4, 2, 2), (5, 3, 1), (4, 4, 2)])
def test_layout_and_projection_in_charged_sectors(L, N, Dk):
    Q = _q_with_sum(L, N, 11, 0)
    lay0, lay = Layout(L, N, [Dk] * N), Layout(L, N, [Dk] * N, Q)
    assert lay.n_params == lay0.n_params
    for y in range(L):
        for x in range(L):
            nb = len(lay.blocks[lay.site(x, y)])
            n = (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1)
            assert nb == N ** (n - 1)
            for (ql, qr, qd, qu), shape, off in lay.blocks[lay.site(x, y)]:
                assert (ql + qd - qr - qu - Q[y, x]) % N == 0
    theta = synth.theta_normals(lay.n_params, N * Dk, seed=3)
    mask = link_mask(L)
    for seed in range(20):
        s = synth.link_labels(L, N, seed) * mask.astype(np.uint8)
        ok, T, bid = project(lay, theta, s)
        assert ok == is_physical(s, N, Q)
        # a configuration in the reference's own sector (Q := its residual) is always valid
        lay_s = Layout(L, N, [Dk] * N, gauss_residual(s, N))
        assert project(lay_s, theta, s)[0]


@pytest.mark.parametrize("L,N,Dk,chi,h,odd", [(2, 2, 1, 4, 0.5, True), (2, 2, 2, 4, 0.5, True),
                                              (3, 2, 2, 4, 0.3, False), (2, 3, 2, 4, 0.4, False),
                                              (3, 3, 1, 4, 0.4, False)])
def test_ed_identity_local_energy_charged(L, N, Dk, chi, h, odd):
    Q = np.ones((L, L), dtype=np.int64) if odd else _q_with_sum(L, N, 5, 0)
    lay = Layout(L, N, [Dk] * N, Q)
    theta = synth.theta_normals(lay.n_params, N * Dk, seed=41)
    c, e = config_tables(N, 1.0, h)
    Hp, links = ed.physical_hamiltonian(L, N, c, e, Q)
    amp = []
    for s in links:
        ok, T, _ = project(lay, theta, s)
        assert ok
        ex = exact_amplitude(T)
        la, sg = amplitude(T, chi)
        assert math.isclose(la, math.log(abs(ex)), rel_tol=1e-11, abs_tol=1e-11)
        assert sg == math.copysign(1.0, ex)
        amp.append(ex)
    psi = np.array(amp)
    eloc = np.array([local_energy(lay, theta, s, chi, c, e) for s in links])
    lhs = float(np.sum(psi ** 2 * eloc) / np.sum(psi ** 2))
    rhs = float(psi @ Hp @ psi / (psi @ psi))
    assert math.isclose(lhs, rhs, rel_tol=1e-10, abs_tol=1e-10)
    assert lhs >= np.linalg.eigvalsh(Hp)[0] - 1e-10


@pytest.mark.parametrize("L,N,odd", [(4, 2, True), (6, 3, False), (5, 4, False)])
def test_sector_helpers_stay_in_sector(L, N, odd):
    base, Q = charged_sector(L, N, 9, odd_z2=odd)
    if odd:
        assert (Q == 1).all()
    configs = sector_configs(base, synth.plaquette_powers(8, L, N, seed=2), N)
    for s in configs:
        assert is_physical(s, N, Q)
        assert not s[~link_mask(L)].any()
