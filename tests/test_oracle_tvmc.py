"""Pins of the real-time (tVMC) oracle, oracle/tvmc.py (SM S-3 eq. tVMC, eq. secondorder):

* the complex amplitude of the exact contraction equals the canonical boundary-MPS contraction
  when chi is exact (two independent contraction orders);
* O_k = d ln Psi / d theta_k against central finite differences along the real AND the imaginary
  axis of theta_k (both equal the holomorphic derivative only if the amplitude is holomorphic and
  O_k is right);
* the complex local energy obeys the ED identity sum |Psi|^2 E_loc / sum |Psi|^2 = <Psi|H|Psi> /
  <Psi|Psi> with H built from Kronecker products (oracle/ed.py, independent code);
* the evolution against exp(-i H t) of exact diagonalisation on lattices where the ansatz can
  represent every state: the two-stage update of eq. secondorder has amplitude error O(dt^2)
  (infidelity falls ~16x when dt halves), a single Euler stage O(dt) (~4x), and the direction of
  time is the physical one;
* a charged sector in the style of the real-time workload (toric-code state with a string of
  flipped links, Gauss-law defects at its ends, complex perturbation), 3 x 3, D_k = 2: the
  evolved state follows exact diagonalisation in that sector and <H> is conserved to O(dt^2).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import ed, tvmc
from oracle.contract import down_boundaries
from oracle.energy import config_tables
from oracle.lattice import gauss_residual
from oracle.layout import Layout, project
from tests.helpers import configs, toric_theta


def complex_theta(lay, seed, scale=0.5, shift=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal(lay.n_params) + 1j * rng.standard_normal(lay.n_params)) * scale + shift


def test_complex_exact_contraction_equals_boundary_mps_at_exact_chi():
    L, N, Dk = 4, 2, 2
    lay = Layout(L, N, [Dk] * N)
    theta = complex_theta(lay, 5, shift=0.0)
    for s in configs(3, L, N, seed=6):
        ok, T, _ = project(lay, theta, s)
        D, lognu = down_boundaries(T, 4)
        env = np.ones((1, 1), dtype=complex)
        for B, Tt in zip(D[L - 2], T[L - 1]):
            env = np.einsum("al,apb,lrp->br", env, B, Tt[:, :, :, 0])
        psi_mps = math.exp(sum(lognu)) * env[0, 0]
        psi = tvmc.exact_amplitude(T)
        assert abs(psi_mps - psi) <= 1e-12 * abs(psi)


def test_log_derivatives_are_holomorphic_and_match_finite_differences():
    L, N, Dk = 3, 2, 2
    lay = Layout(L, N, [Dk] * N)
    theta = complex_theta(lay, 7, shift=0.0)
    s = configs(1, L, N, seed=8)[0]
    O = tvmc.log_derivatives(lay, theta, s)
    ok, _, bid = project(lay, theta, s)
    f = tvmc.amplitude_of(lay, theta)
    psi = f(s)
    rng = np.random.default_rng(9)
    nz = np.nonzero(O)[0]
    assert nz.size > 0 and np.count_nonzero(O) < lay.n_params   # only the selected blocks
    h = 1e-6
    for k in rng.choice(nz, 12, replace=False):
        for step in (h, 1j * h):                     # real and imaginary directions
            tp, tm = theta.copy(), theta.copy()
            tp[k] += step
            tm[k] -= step
            fd = (np.log(tvmc.amplitude_of(lay, tp)(s)) - np.log(tvmc.amplitude_of(lay, tm)(s))) / (2 * step)
            assert abs(fd - O[k]) <= 1e-6 * max(1.0, abs(O[k])), (k, step, fd, O[k])
    # homogeneity (Euler identity): sum over a site's selected entries of theta_k O_k = 1
    for y in range(L):
        for x in range(L):
            _, shape, off = lay.blocks[lay.site(x, y)][bid[y, x]]
            sl_ = slice(off, off + int(np.prod(shape)))
            assert abs(np.sum(theta[sl_] * O[sl_]) - 1.0) <= 1e-12
    assert psi != 0


@pytest.mark.parametrize("L,N,Dk,h", [(2, 3, 2, 0.4), (3, 2, 2, 0.3)])
def test_complex_local_energy_ed_identity(L, N, Dk, h):
    c, e = config_tables(N, 1.0, h)
    lay = Layout(L, N, [Dk] * N)
    theta = complex_theta(lay, 11, shift=0.0)
    Hp, cfg = ed.physical_hamiltonian(L, N, c, e)
    psi = tvmc.state_vector(lay, theta, cfg)
    eloc = np.array([tvmc.local_energy(lay, theta, s, c, e) for s in cfg])
    lhs = np.sum(np.abs(psi) ** 2 * eloc) / np.sum(np.abs(psi) ** 2)
    rhs = np.vdot(psi, Hp @ psi) / np.vdot(psi, psi)
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs) and abs(rhs.imag) <= 1e-12 * abs(rhs)


def _infidelity(L, N, Dk, dt, T, order, h=0.5):
    c, e = config_tables(N, 1.0, h)
    lay = Layout(L, N, [Dk] * N)
    theta = complex_theta(lay, 3)
    Hp, cfg = ed.physical_hamiltonian(L, N, c, e)
    psi0 = tvmc.state_vector(lay, theta, cfg)
    psi0 /= np.linalg.norm(psi0)
    thetas, energies = tvmc.evolve(lay, theta, cfg, c, e, dt, int(round(T / dt)), order=order)
    psi = tvmc.state_vector(lay, thetas[-1], cfg)
    psi /= np.linalg.norm(psi)
    exact = sl.expm(-1j * Hp * T) @ psi0
    return 1.0 - abs(np.vdot(exact, psi)) ** 2


@pytest.mark.parametrize("N", [2, 3])
def test_second_order_update_follows_exact_evolution(N):
    # 2 x 2, D_k = 1: the corner tensors' block scalars reach every state of the N-dimensional
    # physical space, so the variational evolution is exact up to the integrator's error
    a = _infidelity(2, N, 1, 0.04, 1.0, order=2)
    b = _infidelity(2, N, 1, 0.02, 1.0, order=2)
    print("N=%d second order: 1 - fidelity %.2e (dt 0.04), %.2e (dt 0.02), ratio %.1f" % (N, a, b, a / b))
    assert a <= 1e-5 and 10.0 < a / b < 25.0
    a1 = _infidelity(2, N, 1, 0.04, 1.0, order=1)
    b1 = _infidelity(2, N, 1, 0.02, 1.0, order=1)
    print("N=%d first order: 1 - fidelity %.2e, %.2e, ratio %.1f" % (N, a1, b1, a1 / b1))
    assert 2.5 < a1 / b1 < 5.0 and a1 > 30 * a


def test_charged_string_state_follows_exact_evolution_and_conserves_energy():
    # a horizontal string across the middle row (its two links at L = 3) flipped on the toric-code
    # state: Gauss-law defects (background charges) at its ends; D_k = 2 with a complex perturbation
    L, N, Dk, h = 3, 2, 2, 0.2
    s0 = np.zeros((2, L, L), dtype=np.uint8)
    s0[0, 1, 0] = 1                      # h(0,1): from (0,1) to (1,1)
    s0[0, 1, 1] = 1                      # h(1,1): on to (2,1)
    Q = gauss_residual(s0, N)
    assert np.count_nonzero(Q) == 2      # the defects sit at the string's ends
    c, e = config_tables(N, 1.0, h)
    lay = Layout(L, N, [Dk] * N, Q=Q)
    theta = toric_theta(lay, Dk).astype(complex)
    rng = np.random.Generator(np.random.PCG64(21))
    theta = theta + 1e-1 * (rng.standard_normal(lay.n_params) + 1j * rng.standard_normal(lay.n_params))
    Hp, cfg = ed.physical_hamiltonian(L, N, c, e, Q=Q)
    psi0 = tvmc.state_vector(lay, theta, cfg)
    psi0 /= np.linalg.norm(psi0)
    e_exact = float(np.vdot(psi0, Hp @ psi0).real)
    T, out = 0.6, {}
    for dt in (0.06, 0.03):
        thetas, energies = tvmc.evolve(lay, theta, cfg, c, e, dt, int(round(T / dt)))
        psi = tvmc.state_vector(lay, thetas[-1], cfg)
        psi /= np.linalg.norm(psi)
        exact = sl.expm(-1j * Hp * T) @ psi0
        out[dt] = (1.0 - abs(np.vdot(exact, psi)) ** 2, abs(energies[-1] - energies[0]))
        assert abs(energies[0] - e_exact) <= 1e-10 * abs(e_exact)
    print("charged string: (1 - fidelity, |<H>(T) - <H>(0)|) per dt:", out)
    # second order: infidelity ~ dt^4 (amplitude error ~ dt^2) and <H> drift ~ dt^2
    assert out[0.03][0] <= 1e-5 and 10.0 < out[0.06][0] / out[0.03][0] < 25.0
    assert out[0.03][1] <= 1e-3 * abs(e_exact) and out[0.06][1] / out[0.03][1] > 3.0
