"""Pins of the oracle log-derivatives (finite differences, Euler identity, exact case) and of the
SR build (library covariance)."""
import math

import numpy as np
import pytest
import torch

from oracle.contract import amplitude, exact_amplitude
from oracle.layout import project
from oracle.logderiv import finite_difference, grads_to_theta, log_derivatives
from oracle.sr import sr_force_and_mean, sr_matrix, sr_matvec, sr_solve_cg
from tests.helpers import configs, make_problem, tensors_of


def _lnpsi(lay, s, chi):
    def f(th):
        ok, T, _ = project(lay, th, s)
        return amplitude(T, chi)[0]
    return f


@pytest.mark.parametrize("L,N,Dk,chi", [(5, 2, 2, 3), (6, 3, 2, 3)])
def test_logderiv_matches_central_differences_under_truncation(L, N, Dk, chi):
    lay, theta = make_problem(L, N, Dk, seed=61)
    s = configs(1, L, N, seed=62)[0]
    T, bid = tensors_of(lay, theta, s)
    val, grads = log_derivatives(T, chi)
    assert math.isclose(val, amplitude(T, chi)[0], abs_tol=1e-12)
    g = grads_to_theta(lay, bid, grads)
    rng = np.random.default_rng(63)
    sel = np.nonzero(g)[0]                      # coordinates inside the selected blocks
    for k in rng.choice(sel, size=12, replace=False):
        fd = finite_difference(_lnpsi(lay, s, chi), theta, k, step=1e-6)
        assert math.isclose(g[k], fd, rel_tol=1e-6, abs_tol=1e-8), (k, g[k], fd)


def test_euler_identity_per_site():
    # Psi is homogeneous of degree 1 in every site tensor (truncation included), so
    # sum_{k in site x} theta_k O_k = 1 for every site and sample.
    L, N, Dk, chi = 6, 3, 2, 3
    lay, theta = make_problem(L, N, Dk, seed=71)
    for s in configs(2, L, N, seed=72):
        T, _ = tensors_of(lay, theta, s)
        _, grads = log_derivatives(T, chi)
        for y in range(L):
            for x in range(L):
                assert math.isclose(float(np.sum(grads[y][x] * T[y][x])), 1.0, abs_tol=1e-10)


def test_logderiv_equals_exact_gradient_when_chi_is_exact():
    # With no truncation the derivative must equal that of the textbook einsum contraction.
    L, N, Dk = 4, 3, 2
    lay, theta = make_problem(L, N, Dk, seed=81)
    s = configs(1, L, N, seed=82)[0]
    T, _ = tensors_of(lay, theta, s)
    _, grads = log_derivatives(T, 4)
    leaves = [[torch.tensor(T[y][x], requires_grad=True) for x in range(L)] for y in range(L)]
    # exact amplitude as a torch einsum over the whole network
    ops, subs = [], []
    lab = {}
    for y in range(L):
        for x in range(L):
            keep, sub = [], []
            for leg, key in enumerate((("h", x - 1, y), ("h", x, y), ("v", x, y - 1), ("v", x, y))):
                if (x > 0, x < L - 1, y > 0, y < L - 1)[leg]:
                    keep.append(leg)
                    sub.append(lab.setdefault(key, len(lab)))
            idx = tuple(slice(None) if leg in keep else 0 for leg in range(4))
            ops.append(leaves[y][x][idx])
            subs.append(sub)
    args = []
    for o, sb in zip(ops, subs):
        args += [o, sb]
    psi = torch.einsum(*args, [])
    torch.log(torch.abs(psi)).backward()
    assert math.isclose(float(psi.detach()), exact_amplitude(T), rel_tol=1e-12)
    for y in range(L):
        for x in range(L):
            assert np.allclose(grads[y][x], leaves[y][x].grad.numpy(), rtol=1e-9, atol=1e-11)


def test_sr_build_matches_library_covariance():
    rng = np.random.default_rng(5)
    B, P = 64, 23
    O = rng.standard_normal((B, P)) * rng.uniform(0.1, 2.0, P)
    e = rng.standard_normal(B) - 3.0
    F, om = sr_force_and_mean(O, e)
    S = sr_matrix(O)
    C = np.cov(np.concatenate([O, e[:, None]], axis=1).T, bias=True)
    assert np.allclose(S, np.cov(O.T, bias=True), atol=1e-12)
    assert np.allclose(F, C[:P, P], atol=1e-12)
    assert np.allclose(om, O.mean(axis=0), atol=1e-14)
    assert np.allclose(S, S.T) and np.linalg.eigvalsh(S)[0] > -1e-12
    v = rng.standard_normal(P)
    assert np.allclose(sr_matvec(O, v), S @ v, atol=1e-12)


def test_sr_matrix_rows_are_rows_of_the_library_covariance():
    from oracle.sr import sr_matrix_rows
    rng = np.random.default_rng(8)
    B, P = 50, 31
    O = rng.standard_normal((B, P)) * rng.uniform(0.1, 2.0, P)
    C = np.cov(O.T, bias=True)
    for rows in (np.arange(0, 5), np.arange(17, 31), np.array([3, 29, 11])):
        assert np.allclose(sr_matrix_rows(O, rows), C[rows], atol=1e-12)


@pytest.mark.parametrize("B,P,shift", [(64, 23, 1e-3), (16, 40, 1e-2), (200, 60, 1e-4)])
def test_sr_cg_solves_the_shifted_system(B, P, shift):
    # CG against a dense solve (library routine) of (S + shift I) x = F, rank-deficient S included
    # (B < P); in exact arithmetic CG ends within P steps, here it reaches the tolerance
    rng = np.random.default_rng(B + P)
    O = rng.standard_normal((B, P)) * rng.uniform(0.1, 2.0, P)
    e = rng.standard_normal(B) - 3.0
    F, _ = sr_force_and_mean(O, e)
    want = np.linalg.solve(sr_matrix(O) + shift * np.eye(P), F)
    x, it, rel = sr_solve_cg(O, e, shift, 10 * P, 1e-12)
    assert rel <= 1e-12 and it <= 10 * P
    assert np.allclose(x, want, rtol=1e-8, atol=1e-10 * np.abs(want).max())
    r = F - (sr_matvec(O, x) + shift * x)
    assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(F)


def test_sr_cg_stops_at_max_iter_and_zero_force():
    rng = np.random.default_rng(3)
    O = rng.standard_normal((32, 20))
    e = rng.standard_normal(32)
    x, it, rel = sr_solve_cg(O, e, 1e-3, 2, 1e-14)
    assert it == 2 and rel > 1e-14
    x0, it0, rel0 = sr_solve_cg(O, np.zeros(32), 1e-3, 50, 1e-10)  # E = 0: F = 0 exactly
    assert it0 == 0 and rel0 == 0.0 and not x0.any()
