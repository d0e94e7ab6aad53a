"""Pins of the oracle amplitude: exact einsum, closed forms, homogeneity, gauge invariance."""
import math

import numpy as np
import pytest

from oracle.contract import amplitude, exact_amplitude
from oracle.layout import Layout, project
from oracle.lattice import links_from_powers
from tests.helpers import configs, gauge_transform, make_problem, tensors_of, toric_theta


def test_dk1_amplitude_is_product_of_block_scalars():
    # D_k = 1 (the z2_4x4_d2 shape): every bond is one-dimensional, the network is a product of
    # scalars.
    lay, theta = make_problem(4, 2, 1)
    for s in configs(16, 4, 2):
        T, _ = tensors_of(lay, theta, s)
        prod = np.prod([T[y][x].item() for y in range(4) for x in range(4)])
        la, sg = amplitude(T, 16)
        assert math.isclose(la, math.log(abs(prod)), rel_tol=0, abs_tol=1e-12)
        assert sg == math.copysign(1.0, prod)


@pytest.mark.parametrize("L,N,Dk,chi", [(2, 2, 2, 4), (3, 2, 2, 4), (3, 3, 2, 4), (4, 2, 2, 4),
                                        (4, 3, 2, 4), (4, 4, 3, 9)])
def test_boundary_mps_equals_exact_contraction_when_chi_is_exact(L, N, Dk, chi):
    # chi >= D_k^{floor(L/2)} means no truncation happens: the canonical algorithm must then
    # reproduce the textbook einsum contraction.
    lay, theta = make_problem(L, N, Dk, seed=7)
    for s in configs(6, L, N, seed=11):
        T, _ = tensors_of(lay, theta, s)
        ex = exact_amplitude(T)
        la, sg = amplitude(T, chi)
        assert math.isclose(la, math.log(abs(ex)), abs_tol=1e-11)
        assert sg == math.copysign(1.0, ex)


def test_truncation_is_active_and_changes_the_value():
    # Guard against a vacuous test suite: at chi = 2 on 4x4 D_k = 2 the truncated amplitude
    # differs from the exact one.
    lay, theta = make_problem(4, 2, 2, seed=3)
    s = configs(1, 4, 2, seed=4)[0]
    T, _ = tensors_of(lay, theta, s)
    assert abs(amplitude(T, 2)[0] - math.log(abs(exact_amplitude(T)))) > 1e-6


@pytest.mark.parametrize("scale", [3.7, -0.25])
def test_homogeneity_under_truncation(scale):
    # Scaling one site tensor by c scales Psi by c exactly, truncation included (SVD truncation
    # commutes with scalars).
    L, N, Dk, chi = 8, 3, 2, 4
    lay, theta = make_problem(L, N, Dk, seed=21)
    s = configs(1, L, N, seed=22)[0]
    T, _ = tensors_of(lay, theta, s)
    la0, sg0 = amplitude(T, chi)
    for (x, y) in [(0, 0), (3, 4), (7, 7), (5, 0), (0, 6)]:
        T2 = [[t.copy() for t in row] for row in T]
        T2[y][x] = T2[y][x] * scale
        la, sg = amplitude(T2, chi)
        assert math.isclose(la, la0 + math.log(abs(scale)), abs_tol=1e-10)
        assert sg == sg0 * math.copysign(1.0, scale)


def test_gauge_invariance_with_truncation():
    # eq. gcf: A -> A X, B -> X^-1 B leaves the state unchanged.  The truncated amplitude is
    # invariant under invertible X on horizontal bonds (MPS gauge) and orthogonal X on vertical
    # bonds (physical legs of the boundary MPS), even while truncating.
    L, N, Dk, chi = 8, 2, 2, 4
    lay, theta = make_problem(L, N, Dk, seed=5)
    theta2 = gauge_transform(lay, theta, seed=99)
    for s in configs(4, L, N, seed=6):
        T1, _ = tensors_of(lay, theta, s)
        T2, _ = tensors_of(lay, theta2, s)
        a1, s1 = amplitude(T1, chi)
        a2, s2 = amplitude(T2, chi)
        assert math.isclose(a1, a2, abs_tol=1e-10) and s1 == s2


def test_general_vertical_gauge_invariant_only_when_exact():
    # General invertible X on the vertical bonds changes the boundary MPS's physical legs, so
    # only the exact contraction is invariant; the truncated one moves.
    L, N, Dk = 4, 2, 2
    lay, theta = make_problem(L, N, Dk, seed=8)
    theta2 = gauge_transform(lay, theta, seed=5, vertical_general=True)
    s = configs(1, L, N, seed=9)[0]
    T1, _ = tensors_of(lay, theta, s)
    T2, _ = tensors_of(lay, theta2, s)
    assert math.isclose(exact_amplitude(T1), exact_amplitude(T2), rel_tol=1e-10)
    assert math.isclose(amplitude(T1, 4)[0], amplitude(T2, 4)[0], abs_tol=1e-10)
    assert abs(amplitude(T1, 2)[0] - amplitude(T2, 2)[0]) > 1e-8


@pytest.mark.parametrize("L,N,Dk,chi", [(6, 2, 2, 4), (6, 3, 2, 6), (16, 3, 2, 6)])
def test_padded_toric_code_with_gauges_has_unit_amplitude(L, N, Dk, chi):
    lay = Layout(L, N, [Dk] * N)
    theta = gauge_transform(lay, toric_theta(lay, Dk), seed=123)
    for s in configs(3, L, N, seed=4):
        T, _ = tensors_of(lay, theta, s)
        la, sg = amplitude(T, chi)
        assert abs(la) < 1e-10 and sg == 1.0


def test_unphysical_configuration_has_zero_amplitude():
    lay, theta = make_problem(4, 3, 2)
    s = links_from_powers(np.ones((3, 3), dtype=int), 3)
    s[0, 2, 1] = (s[0, 2, 1] + 1) % 3
    assert project(lay, theta, s)[0] is False


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_single_cut_truncation_keeps_the_largest_schmidt_values(k):
    # Two-site MPS psi = U diag(s) V^T with known, unsorted Schmidt values s.  The truncated state
    # must be the Eckart-Young best rank-k approximation: ln nu = ln sqrt(sum of the k largest
    # s^2), and ||psi - nu * psi_k||^2 = sum of the discarded s^2.  Keeping the first k columns of
    # an unsorted SVD, or the smallest ones, fails both.
    from oracle.contract import compress
    rng = np.random.Generator(np.random.PCG64(1000 + k))
    n = 6
    s = np.array([0.3, 2.0, 0.05, 1.1, 0.7, 0.01])
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    mps = [(U * s).reshape(1, n, n), V.T.reshape(n, n, 1)]
    out, ln_nu, bonds = compress(mps, k)
    top = np.argsort(-s)[:k]
    assert bonds[1] == k
    assert math.isclose(ln_nu, 0.5 * math.log(float(np.sum(s[top] ** 2))), rel_tol=1e-12, abs_tol=1e-14)
    psi = (U * s) @ V.T
    psi_k = math.exp(ln_nu) * np.einsum("xia,ajy->ij", out[0], out[1])
    best = (U[:, top] * s[top]) @ V[:, top].T
    assert np.allclose(psi_k, best, atol=1e-12)
    discarded = float(np.sum(s ** 2) - np.sum(s[top] ** 2))
    assert math.isclose(float(np.sum((psi - psi_k) ** 2)), discarded, rel_tol=1e-9, abs_tol=1e-15)
