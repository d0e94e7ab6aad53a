"""Pins of the oracle local energy: ED in an independently built link basis, closed forms,
zero variance, toric code."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ed
from oracle.contract import amplitude, exact_amplitude
from oracle.energy import config_tables, electric_energy, local_energy, local_energy_exact, paper_tables
from oracle.layout import Layout, project
from oracle.lattice import n_plaquettes
from tests.helpers import configs, gauge_transform, make_problem, tensors_of, toric_theta

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _amp_exact(lay, theta):
    def f(links):
        ok, T, _ = project(lay, theta, links)
        return exact_amplitude(T) if ok else 0.0
    return f


def test_ed_closed_forms_2x2():
    # One plaquette, four links: the physical space is the N plaquette powers k, with every link
    # label +-k; the Hamiltonian is an N x N matrix whose ground energy has a closed form.
    with open(os.path.join(GOLDEN, "ed_2x2_closed_forms.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        c, e = config_tables(case["N"], case["J"], case["h"])
        E0 = ed.ground_energy(2, case["N"], c, e)
        assert math.isclose(E0, eval(case["closed_form"], {"sqrt": math.sqrt}), abs_tol=1e-12)


@pytest.mark.parametrize("L,N", [(2, 2), (3, 2), (2, 3), (3, 3)])
def test_ed_zero_field_point(L, N):
    # h = 0: every plaquette operator commutes and has eigenvalue 1 on the uniform superposition,
    # so E_0 = sum_p sum_t c[t] = -J N_plaq (Z2) or -2 J N_plaq (Z_N, N >= 3).
    c, e = config_tables(N, 1.0, 0.0)
    E0 = ed.ground_energy(L, N, c, e)
    want = -n_plaquettes(L) * (1 if N == 2 else 2)
    assert math.isclose(E0, want, abs_tol=1e-10)


def test_paper_and_config_conventions_differ_by_constant_and_factor():
    # With J = h_p and h = g: Z_N>=3: H_paper = H_cfg + 2 g N_links; Z2: H_paper = 2 H_cfg + 2 g N_links.
    for N, L in [(2, 2), (3, 2), (2, 3)]:
        g, hp = 0.37, 1.0
        cc, ec = config_tables(N, hp, g)
        cp, ep = paper_tables(N, hp, g)
        Ec = ed.ground_energy(L, N, cc, ec)
        Ep = ed.ground_energy(L, N, cp, ep)
        nl = 2 * L * (L - 1)
        f = 2.0 if N == 2 else 1.0
        assert math.isclose(Ep, f * Ec + 2 * g * nl, abs_tol=1e-10)


@pytest.mark.parametrize("L,N,Dk,chi,h", [(2, 2, 1, 4, 0.5), (2, 3, 2, 4, 0.4), (2, 4, 2, 4, 0.5),
                                          (3, 2, 2, 4, 0.5), (3, 3, 1, 4, 0.4), (3, 2, 1, 4, 0.3)])
def test_ed_identity_local_energy(L, N, Dk, chi, h):
    # sum_s |Psi(s)|^2 E_loc(s) / sum_s |Psi(s)|^2 = <Psi|H|Psi> / <Psi|Psi> for ANY Psi, with H
    # built from Kronecker products in the link basis (independent of the plaquette-move code).
    lay, theta = make_problem(L, N, Dk, seed=31)
    c, e = config_tables(N, 1.0, h)
    Hp, links = ed.physical_hamiltonian(L, N, c, e)
    psi = np.array([_amp_exact(lay, theta)(s) for s in links])
    eloc = np.array([local_energy(lay, theta, s, chi, c, e) for s in links])
    lhs = float(np.sum(psi ** 2 * eloc) / np.sum(psi ** 2))
    rhs = float(psi @ Hp @ psi / (psi @ psi))
    assert math.isclose(lhs, rhs, rel_tol=1e-10, abs_tol=1e-10)
    assert lhs >= np.linalg.eigvalsh(Hp)[0] - 1e-10


def test_zero_variance_for_exact_ground_state_2x2():
    # SM S-1: for an eigenstate E_loc(s) = E_g for every s.  With D_k = 1 on 2x2, setting the
    # corner (0,0) block scalars to the ground-state amplitudes (the corner's block is selected by
    # the plaquette power alone) and every other entry to 1 represents the ground state exactly.
    for N, h in [(2, 0.5), (3, 0.4), (4, 0.5)]:
        c, e = config_tables(N, 1.0, h)
        Hp, links = ed.physical_hamiltonian(2, N, c, e)
        w, v = np.linalg.eigh(Hp)
        g = v[:, 0] * np.sign(v[np.argmax(np.abs(v[:, 0])), 0])
        lay = Layout(2, N, [1] * N)
        theta = np.ones(lay.n_params)
        for i, s in enumerate(links):
            _, _, bid = project(lay, theta, s)
            ch, shape, off = lay.blocks[0][bid[0, 0]]
            theta[off] = g[i]
        for s in links:
            assert math.isclose(local_energy(lay, theta, s, 4, c, e), w[0], abs_tol=1e-12)


@pytest.mark.parametrize("L,N,Dk,chi", [(4, 2, 1, 4), (4, 3, 2, 4), (16, 2, 2, 4), (16, 3, 2, 6)])
def test_toric_code_local_energy_closed_form(L, N, Dk, chi):
    # Psi = 1 for every physical s, so E_loc(s) = N_plaq * sum_t c[t] + sum_l e[n_l(s)]; at h = 0
    # that is -J N_plaq (Z2) and -2 J N_plaq (Z_N).  Padded to D_k = 2 and gauge-transformed the
    # state is unchanged.
    lay = Layout(L, N, [Dk] * N)
    theta = toric_theta(lay, Dk)
    if Dk > 1:
        theta = gauge_transform(lay, theta, seed=77)
    for h in (0.0, 0.4):
        c, e = config_tables(N, 1.0, h)
        for s in configs(2, L, N, seed=3):
            want = n_plaquettes(L) * float(np.sum(c[1:])) + electric_energy(s, e)
            assert math.isclose(local_energy(lay, theta, s, chi, c, e), want, abs_tol=1e-9)
    c, e = config_tables(N, 1.0, 0.0)
    s = configs(1, L, N, seed=8)[0]
    assert math.isclose(local_energy(lay, theta, s, chi, c, e),
                        -n_plaquettes(L) * (1 if N == 2 else 2), abs_tol=1e-9)


@pytest.mark.parametrize("L,N,Dk", [(4, 2, 2), (4, 3, 2)])
def test_strip_ratios_equal_exact_ratios_when_chi_is_exact(L, N, Dk):
    lay, theta = make_problem(L, N, Dk, seed=41)
    c, e = config_tables(N, 1.0, 0.4)
    for s in configs(3, L, N, seed=42):
        a = local_energy(lay, theta, s, 4, c, e)
        b = local_energy_exact(lay, theta, s, c, e, _amp_exact(lay, theta))
        assert math.isclose(a, b, rel_tol=1e-10, abs_tol=1e-10)


def test_strip_local_energy_under_truncation_is_gauge_invariant():
    L, N, Dk, chi = 6, 3, 2, 3
    lay, theta = make_problem(L, N, Dk, seed=51)
    theta2 = gauge_transform(lay, theta, seed=52)
    c, e = config_tables(N, 1.0, 0.4)
    s = configs(1, L, N, seed=53)[0]
    assert math.isclose(local_energy(lay, theta, s, chi, c, e),
                        local_energy(lay, theta2, s, chi, c, e), rel_tol=1e-9)
    T, _ = tensors_of(lay, theta, s)
    assert amplitude(T, chi)[0] != amplitude(T, 8)[0]


# ---- the local-energy scale M(s) = sum_l |e[n_l]| + sum_{p,t} |c[t] ratio_{p,t}| ----

@pytest.mark.parametrize("L,N,Dk,chi", [(4, 2, 1, 4), (4, 3, 2, 4), (6, 3, 2, 6)])
def test_scale_toric_code_closed_form(L, N, Dk, chi):
    # every ratio is 1 for the (padded, gauged) toric code, so M(s) = N_plaq sum_t |c[t]| +
    # sum_l |e[n_l(s)]| exactly; with h = 0.4 the electric terms have both signs, so M > |E_loc|
    lay = Layout(L, N, [Dk] * N)
    theta = toric_theta(lay, Dk)
    if Dk > 1:
        theta = gauge_transform(lay, theta, seed=79)
    c, e = config_tables(N, 1.0, 0.4)
    for s in configs(3, L, N, seed=4):
        el, m = local_energy(lay, theta, s, chi, c, e, with_scale=True)
        mask = np.ones_like(s, dtype=bool)
        mask[0, :, L - 1] = False
        mask[1, L - 1, :] = False
        want = n_plaquettes(L) * float(np.sum(np.abs(c[1:]))) + float(np.sum(np.abs(e)[s[mask]]))
        assert math.isclose(m, want, rel_tol=1e-12)
        assert m > abs(el) + 1e-6


@pytest.mark.parametrize("L,N,Dk", [(3, 2, 2), (4, 3, 2)])
def test_scale_equals_exact_ratio_magnitudes_when_chi_is_exact(L, N, Dk):
    # with chi exact the strip ratios are amplitude ratios, so M(s) must equal the magnitudes of
    # the exact-amplitude terms (numpy.einsum contraction of the whole network, no boundary code)
    lay, theta = make_problem(L, N, Dk, seed=43)
    c, e = config_tables(N, 1.0, 0.4)
    amp = _amp_exact(lay, theta)
    from oracle.lattice import apply_plaquette
    for s in configs(3, L, N, seed=44):
        el, m = local_energy(lay, theta, s, 4, c, e, with_scale=True)
        psi = amp(s)
        mag = 0.0
        for py in range(L - 1):
            for px in range(L - 1):
                for t in range(1, N):
                    mag += abs(c[t] * amp(apply_plaquette(s, px, py, (N - t) % N, N)) / psi)
        mask = np.ones_like(s, dtype=bool)
        mask[0, :, L - 1] = False
        mask[1, L - 1, :] = False
        mag += float(np.sum(np.abs(e)[s[mask]]))
        assert math.isclose(m, mag, rel_tol=1e-10)
        assert abs(el) <= m * (1 + 1e-12)


def test_scale_bounds_local_energy_under_truncation():
    # |E_loc| <= M for truncated strips too, and the scale is NaN exactly where E_loc is
    L, N, Dk, chi = 6, 3, 2, 3
    lay, theta = make_problem(L, N, Dk, seed=55)
    c, e = config_tables(N, 1.0, 0.4)
    for s in configs(4, L, N, seed=56):
        el, m = local_energy(lay, theta, s, chi, c, e, with_scale=True)
        assert el == local_energy(lay, theta, s, chi, c, e)
        assert abs(el) <= m
    bad = configs(1, L, N, seed=57)[0].copy()
    bad[0, 0, 0] = (bad[0, 0, 0] + 1) % N   # breaks the Gauss law at two vertices
    el, m = local_energy(lay, theta, bad, chi, c, e, with_scale=True)
    assert math.isnan(el) and math.isnan(m)
