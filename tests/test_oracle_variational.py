"""Pins of the oracle's variational boundary compression (oracle/contract.py: variational_refine;
SM S-2 "SVD or variational compression", VMC section).

Fidelities are computed from full state vectors (brute force over every physical index), not from
the routine's environments:
  * two sites: the best approximation of given rank is the truncated SVD (Eckart-Young), so the
    refinement must return the SVD truncation's state;
  * the fidelity |<G|M>| / (||G|| ||M||) never decreases from sweep to sweep and starts at the SVD
    truncation's; the sweeps reach a fixed point (one more sweep changes nothing);
  * when chi holds every bond the compression is exact: the amplitude equals the exact contraction;
  * every boundary row of a truncating sweep is fitted at least as well as by the SVD truncation.
(Better row fidelities do not make the final overlap closer to the exact amplitude on most samples:
on 12 samples of a 5 x 5 Z3 lattice at chi = 2 it was closer on 6.)
"""
import math

import numpy as np

from oracle.contract import amplitude, compress, exact_amplitude, mpo_apply, variational_refine
from oracle.layout import project
from tests.helpers import configs, make_problem


def full_state(mps):
    """Dense state vector of an open MPS (sites [a, p, b], edge bonds 1)."""
    v = mps[0]
    for s in mps[1:]:
        v = np.einsum("...a,apb->...pb", v, s)
    return v.reshape(-1)


def fidelity(G, M):
    g, m = full_state(G), full_state(M)
    return abs(np.vdot(g, m)) / (np.linalg.norm(g) * np.linalg.norm(m))


def random_mps(dims, p, rng):
    return [rng.standard_normal((dims[c], p, dims[c + 1])) for c in range(len(dims) - 1)]


def test_two_sites_give_the_truncated_svd():
    rng = np.random.default_rng(1)
    M = random_mps([1, 6, 1], 4, rng)
    for k in (1, 2, 3):
        guess, _, _ = compress(M, k)
        G, ln_nu = variational_refine(M, guess, 3)
        a, b = full_state(guess), full_state(G)
        assert abs(abs(np.vdot(a, b)) - 1.0) <= 1e-12
        # the norm of the truncation: its singular values' 2-norm
        sv = np.linalg.svd(full_state(M).reshape(4, 4), compute_uv=False)
        assert abs(ln_nu - math.log(np.linalg.norm(sv[:k]))) <= 1e-12


def test_fidelity_monotone_and_fixed_point():
    rng = np.random.default_rng(2)
    M = random_mps([1, 4, 8, 8, 4, 1], 2, rng)
    guess, _, dims = compress(M, 3)
    f = [fidelity(guess, M)]
    G = guess
    for _ in range(6):
        G, _ = variational_refine(M, G, 1)
        f.append(fidelity(G, M))
    print("fidelity by sweep:", ["%.10f" % x for x in f])
    assert all(b >= a - 1e-13 for a, b in zip(f, f[1:]))
    assert f[-1] > f[0] + 1e-6                      # the refinement improves on the SVD truncation
    G2, _ = variational_refine(M, G, 30)
    G3, _ = variational_refine(M, G2, 1)
    assert abs(abs(np.vdot(full_state(G2), full_state(G3))) / (np.linalg.norm(full_state(G2)) *
               np.linalg.norm(full_state(G3))) - 1.0) <= 1e-12
    # ln nu is the norm of the fitted state
    G4, ln_nu = variational_refine(M, guess, 2)
    assert abs(np.linalg.norm(full_state(G4)) - 1.0) <= 1e-12
    # nu is the norm of the fitted (unnormalised) state, |<G|M>| / ||G|| at the optimum of the last site
    g4 = full_state(G4)
    assert abs(math.log(abs(np.vdot(g4, full_state(M)))) - ln_nu) <= 1e-10


def test_exact_chi_gives_the_exact_amplitude():
    L, N, Dk = 4, 3, 2
    lay, theta = make_problem(L, N, Dk, seed=3)
    for s in configs(3, L, N, seed=4):
        ok, T, _ = project(lay, theta, s)
        la, sg = amplitude(T, 16, var_sweeps=2)
        ex = exact_amplitude(T)
        assert abs(la - math.log(abs(ex))) <= 1e-12 * abs(la) and sg == math.copysign(1.0, ex)


def test_rows_of_the_sweep_are_fitted_better():
    # the fidelity of each boundary row with its exact product, brute force, on a truncating lattice
    L, N, Dk, chi = 6, 3, 2, 3
    lay, theta = make_problem(L, N, Dk, seed=7)
    ok, T, _ = project(lay, theta, configs(1, L, N, seed=8)[0])
    from oracle.contract import row_as_mps
    D = row_as_mps(T[0])
    for y in range(1, 4):
        M = mpo_apply(D, T[y])
        g_svd, _, _ = compress(M, chi)
        g_var, _ = variational_refine(M, g_svd, 3)
        f_svd, f_var = fidelity(g_svd, M), fidelity(g_var, M)
        assert f_var >= f_svd - 1e-13
        D = g_var
