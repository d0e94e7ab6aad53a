"""GPU parity of the complex exact-contraction path and the tVMC step (SM S-3: eq. tVMC, S_mn,
eq. secondorder) against the real-time oracle (oracle/tvmc.py).

* ln|Psi|, the phase of Psi, E_loc and every element of O = d ln Psi / d theta (complex, holomorphic)
  against the oracle's exact einsum contraction, on Z2/Z3 lattices with D_k = 1, 2, 3 (the D_k of the
  real-time workload) and a charged sector; at 5 x 5 and the largest supported shape (6 x 6, D_k = 3)
  against exact boundary-MPS amplitudes of the oracle and central differences of them;
* the velocity of eq. tVMC with |Psi|^2 weights over every configuration of a sector, and with plain
  means over a set of configurations, against the oracle's dense solve;
* time steps of eq. secondorder (and single Euler stages) against the oracle's evolution, step by
  step, on the toric-code state with a string of flipped links (Gauss-law defects at its ends);
* the per-site Euler identity sum_k theta_k O_k = 1 over a whole batch;
* Metropolis chains of |Psi|^2 for complex tensors (peps_metropolis on a complex handle): the
  oracle's chains decision for decision, and a chi-square test against the exact distribution;
* the sampled real-time loop (chains, then tvmc_step with plain means) against the exactly
  weighted evolution: <H> and the electric-field profile after eight steps.
"""
import math

import numpy as np
import pytest
import torch

from oracle import tvmc
from oracle.contract import down_boundaries
from oracle.energy import config_tables
from oracle.lattice import gauss_residual, links_from_powers
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth
from tests.helpers import toric_theta

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def complex_theta(n, seed, scale=0.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * scale


def handle(lib, L, N, Dk, h=0.4, Q=None):
    c, e = config_tables(N, 1.0, h)
    P = lib.Peps(L, N, Dk, 4, c, e, Q=Q, dtype=lib.PEPS_C128_EXACT)
    lay = Layout(L, N, [Dk] * N, Q)
    assert P.n_params == lay.n_params and P.site_offset == lay.site_offset
    return P, lay, (c, e)


def dense_O(P, lay, O, bid):
    """GPU O (projected layout) -> dense [B][n_params] (each block at its parameter offset)."""
    B, L = O.shape[0], P.L
    out = np.zeros((B, P.n_params), dtype=complex)
    for b in range(B):
        for s in range(L * L):
            x, y = s % L, s // L
            npres = (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1)
            bs = P.Dk ** npres
            off = P.site_offset[s] + int(bid[b, s]) * bs
            out[b, off: off + bs] = O[b, s, :bs]
            assert not O[b, s, bs:].any()
    return out


def evaluate(P, theta, links):
    from paper_2503_20566_amd import gipeps
    th = torch.from_numpy(theta).cuda()
    lk = torch.from_numpy(links).cuda()
    B = links.shape[0]
    proj, bid, valid = P.cx_project(th, lk)
    ws = P.workspace(B, gipeps.PEPS_WS_AMPLITUDE)
    la, ph = P.cx_amplitude(proj, valid, ws)
    O = P.cx_logderiv(proj, valid, ws)
    el = P.cx_local_energy(th, lk, proj, valid, ws)
    torch.cuda.synchronize()
    return dict(la=la.cpu().numpy(), ph=ph.cpu().numpy(), O=O.cpu().numpy(), el=el.cpu().numpy(),
                bid=bid.cpu().numpy(), valid=valid.cpu().numpy())


@pytest.mark.parametrize("L,N,Dk,B", [(3, 2, 2, 6), (4, 3, 1, 6), (4, 2, 2, 5), (3, 2, 3, 4)])
def test_cx_amplitude_eloc_O_against_oracle(lib, L, N, Dk, B):
    say("complex parity", L, N, Dk, B)
    P, lay, (c, e) = handle(lib, L, N, Dk)
    theta = complex_theta(P.n_params, 100 + L + N + Dk)
    powers = synth.plaquette_powers(B, L, N, seed=7)
    links = np.stack([links_from_powers(powers[b], N) for b in range(B)])
    r = evaluate(P, theta, links)
    assert r["valid"].all()
    Od = dense_O(P, lay, r["O"], r["bid"])
    for b in range(B):
        ok, T, bid = project(lay, theta, links[b])
        assert ok and np.array_equal(bid.reshape(-1), r["bid"][b])
        psi = tvmc.exact_amplitude(T)
        assert abs(r["la"][b] - np.log(abs(psi))) <= 1e-10 * max(1.0, abs(np.log(abs(psi)))), b
        assert abs(r["ph"][b] - psi / abs(psi)) <= 1e-10, b
        el = tvmc.local_energy(lay, theta, links[b], c, e)
        assert abs(r["el"][b] - el) <= 1e-10 * max(1.0, abs(el)), (b, r["el"][b], el)
        O = tvmc.log_derivatives(lay, theta, links[b])
        assert np.max(np.abs(Od[b] - O)) <= 1e-10 * np.max(np.abs(O)), b


def bmps_amplitude(T):
    """Psi by the oracle's canonical boundary-MPS contraction at a cutoff above every bond (exact;
    pinned against the exact einsum contraction for complex tensors); einsum's own contraction
    is too slow from 5 x 5 on and runs out of index labels at 6 x 6."""
    L = len(T)
    D, lognu = down_boundaries(T, 10 ** 6)
    env = np.ones((1, 1), dtype=complex)
    for Bm, Tt in zip(D[L - 2], T[L - 1]):
        env = np.einsum("al,apb,lrp->br", env, Bm, Tt[:, :, :, 0])
    return math.exp(sum(lognu)) * env[0, 0]


# (7, 2, 3) and (11, 2, 2): Dk^(L+1) = 6561 and 4096, above the LDS limit of 2187: the working
# states in the workspace
@pytest.mark.parametrize("L,N,Dk,B", [(5, 3, 2, 2), (6, 2, 3, 2), (7, 2, 3, 2), (11, 2, 2, 1)])
def test_cx_larger_shapes_against_oracle(lib, L, N, Dk, B):
    # ln|Psi|, phase and E_loc against exact amplitudes from the oracle's boundary MPS; O by central
    # differences of that amplitude along the real and the imaginary axis of sampled coordinates
    say("complex parity, larger", L, N, Dk, B)
    P, lay, (c, e) = handle(lib, L, N, Dk)
    theta = complex_theta(P.n_params, 200 + L + N + Dk)
    powers = synth.plaquette_powers(B, L, N, seed=9)
    links = np.stack([links_from_powers(powers[b], N) for b in range(B)])
    r = evaluate(P, theta, links)
    assert r["valid"].all()
    Od = dense_O(P, lay, r["O"], r["bid"])

    def amp(th, s):
        ok, T, _ = project(lay, th, s)
        return bmps_amplitude(T) if ok else 0.0

    rng = np.random.default_rng(L + Dk)
    for b in range(B):
        psi = amp(theta, links[b])
        assert abs(r["la"][b] - np.log(abs(psi))) <= 1e-10 * abs(np.log(abs(psi))), b
        assert abs(r["ph"][b] - psi / abs(psi)) <= 1e-10, b
        el = tvmc.local_energy(lay, theta, links[b], c, e, amp=lambda s: amp(theta, s))
        assert abs(r["el"][b] - el) <= 1e-10 * max(1.0, abs(el)), (b, r["el"][b], el)
        nz = np.nonzero(Od[b])[0]
        for k in rng.choice(nz, 6, replace=False):
            for step in (1e-6, 1e-6j):
                tp, tm = theta.copy(), theta.copy()
                tp[k] += step
                tm[k] -= step
                fd = (np.log(amp(tp, links[b])) - np.log(amp(tm, links[b]))) / (2 * step)
                assert abs(fd - Od[b, k]) <= 1e-6 * max(1.0, abs(Od[b, k])), (b, k, step, fd, Od[b, k])


@pytest.mark.parametrize("c64", [False, True])
def test_cx_charged_string_and_invalid_samples(lib, c64):
    # complex128: 1e-10 against the oracle; complex64 (PEPS_C64_EXACT): the 1e-5 criteria of the
    # complex64 tests below; invalid samples give -inf, zero phase, NaN E_loc and zero O either way
    say("complex charged string", "complex64" if c64 else "complex128")
    L, N, Dk = 3, 2, 2
    s0 = np.zeros((2, L, L), dtype=np.uint8)
    s0[0, 1, 0] = s0[0, 1, 1] = 1          # a string across the middle row: defects at its ends
    Q = gauss_residual(s0, N)
    P, lay, (c, e) = (handle64 if c64 else handle)(lib, L, N, Dk, h=0.2, Q=Q)
    tol = 1e-5 if c64 else 1e-10
    theta = toric_theta(lay, Dk).astype(complex) + 0.1 * complex_theta(P.n_params, 21, scale=1.0)
    powers = synth.plaquette_powers(4, L, N, seed=3)
    good = np.stack([(links_from_powers(powers[b], N) + s0) % N for b in range(4)]).astype(np.uint8)
    bad = np.stack([links_from_powers(powers[b], N) for b in range(2)])   # the Q = 0 sector: unphysical here
    links = np.concatenate([good, bad])
    r = evaluate(P, theta, links)
    assert r["valid"].tolist() == [1, 1, 1, 1, 0, 0]
    assert np.all(np.isneginf(r["la"][4:])) and np.all(r["ph"][4:] == 0) and np.all(np.isnan(r["el"][4:]))
    assert not r["O"][4:].any()
    Od = dense_O(P, lay, r["O"][:4], r["bid"][:4])
    for b in range(4):
        ok, T, _ = project(lay, theta, links[b])
        psi = tvmc.exact_amplitude(T)
        assert abs(r["la"][b] - np.log(abs(psi))) <= tol and abs(r["ph"][b] - psi / abs(psi)) <= tol
        el = tvmc.local_energy(lay, theta, links[b], c, e)
        assert abs(r["el"][b] - el) <= (tol * max(1.0, abs(el)) if c64 else tol)
        O = tvmc.log_derivatives(lay, theta, links[b])
        assert np.max(np.abs(Od[b] - O)) <= tol * np.max(np.abs(O))


def _sector(L, N, Q_links=None):
    """Every configuration of the sector of Q_links (or Q = 0): the plaquette powers of Z_N."""
    import itertools
    out = []
    for k in itertools.product(range(N), repeat=(L - 1) ** 2):
        s = links_from_powers(np.array(k).reshape(L - 1, L - 1), N)
        out.append(s if Q_links is None else ((s + Q_links) % N).astype(np.uint8))
    return np.stack(out)


def _string_problem(lib):
    L, N, Dk, h = 3, 2, 2, 0.2
    s0 = np.zeros((2, L, L), dtype=np.uint8)
    s0[0, 1, 0] = s0[0, 1, 1] = 1
    Q = gauss_residual(s0, N)
    P, lay, tabs = handle(lib, L, N, Dk, h=h, Q=Q)
    theta = toric_theta(lay, Dk).astype(complex)
    rng = np.random.Generator(np.random.PCG64(21))
    theta = theta + 1e-1 * (rng.standard_normal(lay.n_params) + 1j * rng.standard_normal(lay.n_params))
    return P, lay, tabs, theta, _sector(L, N, s0)


@pytest.mark.parametrize("weights", ["psi2", "uniform"])
def test_tvmc_velocity_against_oracle(lib, weights):
    say("tvmc velocity", weights)
    P, lay, (c, e), theta, cfg = _string_problem(lib)
    shift = 1e-3
    want, eh, _, _ = tvmc.tdvp_rhs(lay, theta, cfg, c, e, shift=shift, weights=weights)
    th = torch.from_numpy(theta).cuda()
    lk = torch.from_numpy(cfg).cuda()
    B = cfg.shape[0]
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_TVMC)
    proj, bid, valid = P.cx_project(th, lk)
    la, _ = P.cx_amplitude(proj, valid, ws)
    O = P.cx_logderiv(proj, valid, ws)
    el = P.cx_local_energy(th, lk, proj, valid, ws)
    mode = lib.TVMC_WEIGHT_PSI2 if weights == "psi2" else lib.TVMC_WEIGHT_UNIFORM
    x, en, it, rel = P.tvmc_rhs(O, bid, valid, el, la, ws, weights=mode, shift=shift, max_iter=5000, rtol=1e-14)
    x = x.cpu().numpy()
    say("CG iterations %d, relative residual %.1e, |x| %.3e, <H> %.12f (oracle %.12f)"
        % (it, rel, np.linalg.norm(want), en.real, eh))
    assert rel <= 1e-13
    assert abs(en.real - eh) <= 1e-11 * abs(eh)
    assert np.linalg.norm(x - want) <= 1e-9 * np.linalg.norm(want)


@pytest.mark.parametrize("order", [2, 1])
def test_tvmc_steps_follow_oracle_evolution(lib, order):
    say("tvmc steps, order", order)
    P, lay, (c, e), theta, cfg = _string_problem(lib)
    shift, dt, steps = 1e-3, 0.05, 4
    thetas, energies = tvmc.evolve(lay, theta, cfg, c, e, dt, steps, order=order, shift=shift)
    th = torch.from_numpy(theta.copy()).cuda()
    lk = torch.from_numpy(cfg).cuda()
    ws = P.workspace(cfg.shape[0], lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_TVMC)
    for k in range(steps):
        en, its = P.tvmc_step(th, lk, ws, dt, weights=lib.TVMC_WEIGHT_PSI2, order=order, shift=shift,
                              max_iter=5000, rtol=1e-14)
        got = th.cpu().numpy()
        err = np.linalg.norm(got - thetas[k + 1]) / np.linalg.norm(thetas[k + 1])
        say("step %d: <H> %.12f (oracle %.12f), CG %s, |theta - oracle| / |theta| %.1e"
            % (k, en.real, energies[k], its, err))
        assert abs(en.real - energies[k]) <= 1e-10 * abs(energies[k])
        assert err <= 1e-9


@pytest.mark.parametrize("strip", [False, True])
def test_complex_chains_match_oracle(lib, strip):
    # peps_metropolis (and, strip, peps_metropolis_strip) on a complex handle: the chains of
    # |Psi|^2 of the exact complex amplitude, decision for decision the oracle's sampler fed with the
    # oracle's exact amplitudes
    from oracle.sampler import metropolis
    say("complex metropolis parity", "strip ratios" if strip else "amplitudes")
    L, N, Dk, B, sweeps = 4, 2, 2, 6, 2
    P, lay, _ = handle(lib, L, N, Dk)
    theta = complex_theta(P.n_params, 17)
    seed, stream = 55, 4
    _, links = P.sample_init(B, seed, stream)
    start = links.cpu().numpy()
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_SAMPLE)
    run = P.metropolis_strip if strip else P.metropolis
    la, acc = run(torch.from_numpy(theta).cuda(), links, seed, 1, sweeps, ws, stream_id=stream)
    torch.cuda.synchronize()
    got, la, acc = links.cpu().numpy(), la.cpu().numpy(), acc.cpu().numpy()

    def log_abs(s):
        ok, T, _ = project(lay, theta, s)
        return float(np.log(abs(tvmc.exact_amplitude(T)))) if ok else -np.inf

    for b in range(B):
        s, lf, a = metropolis(start[b], log_abs, N, seed, stream, b, 1, sweeps)
        assert np.array_equal(got[b], s) and a == acc[b], b
        assert abs(la[b] - lf) <= 1e-10 * max(1.0, abs(lf))
    assert acc.sum() > 0


def test_complex_chains_sample_psi_squared(lib):
    # chi-square of the chains' end states against |Psi|^2 / sum |Psi|^2 over the 16 states of the
    # 3 x 3 Z2 string sector, random complex tensors (a far from uniform |Psi|^2: with a nearly flat
    # target most proposals are accepted and a fixed sweep order is close to periodic), chains
    # started at uniformly drawn states; cells merged to an expectation of at least 10
    from scipy import stats
    say("complex metropolis chi-square")
    P, lay, tabs, _, cfg = _string_problem(lib)
    theta = complex_theta(P.n_params, 31)
    th = torch.from_numpy(theta).cuda()
    ws = P.workspace(cfg.shape[0], lib.PEPS_WS_AMPLITUDE)
    proj, _, valid = P.cx_project(th, torch.from_numpy(cfg).cuda())
    la_all, _ = P.cx_amplitude(proj, valid, ws)
    p = np.exp(2 * (la_all.cpu().numpy() - la_all.max().item()))
    p /= p.sum()
    B, sweeps = 8192, 20
    start = np.random.default_rng(5).integers(0, len(cfg), B)
    links = torch.from_numpy(cfg[start]).cuda()
    ws2 = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_SAMPLE)
    _, acc = P.metropolis(th, links, 8, 1, sweeps, ws2, stream_id=0)
    torch.cuda.synchronize()
    end = links.cpu().numpy()
    index = {s.tobytes(): i for i, s in enumerate(cfg)}
    counts = np.bincount([index[s.tobytes()] for s in end], minlength=len(cfg)).astype(float)
    exp = p * B
    o2, e2, ob, eb = [], [], 0.0, 0.0
    for i in np.argsort(exp):
        ob += counts[i]
        eb += exp[i]
        if eb >= 10:
            o2.append(ob)
            e2.append(eb)
            ob = eb = 0.0
    if eb > 0:
        o2[-1] += ob
        e2[-1] += eb
    chi2 = float(np.sum((np.array(o2) - np.array(e2)) ** 2 / np.array(e2)))
    pval = 1.0 - stats.chi2.cdf(chi2, len(o2) - 1)
    say("chi2 %.1f over %d cells (%d states), p %.3f, acceptance %.3f, largest p %.3f"
        % (chi2, len(o2), len(cfg), pval, acc.sum().item() / (B * sweeps * 4), p.max()))
    assert pval > 1e-3 and len(o2) >= 4


def test_sampled_evolution_follows_exact_dynamics(lib):
    # the whole real-time loop on the GPU: Metropolis chains of the complex |Psi|^2 (continued for
    # two sweeps before each step), tvmc_step with plain means over them, against the same steps
    # with exact |Psi|^2 weights over all 16 configurations of the 3 x 3 string sector (equal to the
    # oracle's evolution, tested above); observables from the exact distribution of each state:
    # <H> and the electric-field profile <n_l> (the links of the string start near 1)
    say("sampled real-time evolution")
    P, lay, (c, e), theta, cfg = _string_problem(lib)
    B, dt, steps, shift = 8192, 0.05, 8, 1e-3
    lk_all = torch.from_numpy(cfg).cuda()
    th_ex = torch.from_numpy(theta.copy()).cuda()
    th_mc = th_ex.clone()
    ws_ex = P.workspace(cfg.shape[0], lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_TVMC)
    ws_mc = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_TVMC | lib.PEPS_WS_SAMPLE)
    chains = torch.from_numpy(cfg[np.random.default_rng(3).integers(0, len(cfg), B)]).cuda()
    P.metropolis(th_mc, chains, 5, 1, 10, ws_mc)                  # burn-in

    def observables(th):
        proj, bid, valid = P.cx_project(th, lk_all)
        la, _ = P.cx_amplitude(proj, valid, ws_ex)
        el = P.cx_local_energy(th, lk_all, proj, valid, ws_ex)
        p = torch.exp(2.0 * (la - la.max()))
        p = (p / p.sum()).cpu().numpy()
        return float(np.sum(p * el.cpu().numpy().real)), np.tensordot(p, cfg[:, :2].astype(float), axes=1)

    e0, prof0 = observables(th_ex)
    for k in range(steps):
        P.tvmc_step(th_ex, lk_all, ws_ex, dt, weights=lib.TVMC_WEIGHT_PSI2, shift=shift, rtol=1e-12)
        P.metropolis(th_mc, chains, 5, 11 + 2 * k, 2, ws_mc)
        P.tvmc_step(th_mc, chains, ws_mc, dt, weights=lib.TVMC_WEIGHT_UNIFORM, shift=shift, rtol=1e-12)
    e_ex, prof_ex = observables(th_ex)
    e_mc, prof_mc = observables(th_mc)
    moved = np.max(np.abs(prof_ex - prof0))
    diff = np.max(np.abs(prof_mc - prof_ex))
    say("T = %.2f: <H> exact %.6f sampled %.6f (start %.6f); profile moved %.3f, sampled - exact %.3f"
        % (dt * steps, e_ex, e_mc, e0, moved, diff))
    # statistical error of the sampled averages ~ 1 / sqrt(8192) per step; <H> is conserved up to the
    # integrator's O(dt^2) drift (pinned against exact evolution in the oracle's tests): within 1%
    assert abs(e_mc - e_ex) <= 2e-2 * abs(e_ex) and abs(e_ex - e0) <= 1e-2 * abs(e0)
    assert diff <= 5e-2 and moved >= 3 * diff


def test_euler_identity_on_a_batch(lib):
    # Psi is homogeneous of degree one in each site's selected block: sum_k theta_k O_k = 1 per site
    say("complex Euler identity")
    L, N, Dk, B = 6, 3, 2, 256
    P, lay, _ = handle(lib, L, N, Dk)
    theta = complex_theta(P.n_params, 5)
    th = torch.from_numpy(theta).cuda()
    lk = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda())
    proj, bid, valid = P.cx_project(th, lk)
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE)
    la, ph = P.cx_amplitude(proj, valid, ws)
    O = P.cx_logderiv(proj, valid, ws)
    s = (O * proj).sum(dim=2)
    torch.cuda.synchronize()
    assert bool(valid.all()) and bool(torch.isfinite(la).all())
    assert torch.max(torch.abs(s - 1.0)).item() < 1e-9


def test_cx_real_time_workload_shape(lib):
    # the real-time workload's tensors, D = 6 (D_k = 3) on 10 x 10, contracted exactly (working states
    # of 3^11 entries in the workspace): ln|Psi| and phase against the oracle's exact boundary MPS, the
    # Euler identity of O on every site, E_loc finite
    L, N, Dk, B = 10, 2, 3, 2
    say("complex 10x10 D=6")
    P, lay, (c, e) = handle(lib, L, N, Dk)
    theta = complex_theta(P.n_params, 31)
    powers = synth.plaquette_powers(B, L, N, seed=13)
    links = np.stack([links_from_powers(powers[b], N) for b in range(B)])
    r = evaluate(P, theta, links)
    assert r["valid"].all() and np.all(np.isfinite(r["el"]))
    ok, T, _ = project(lay, theta, links[0])
    psi = bmps_amplitude(T)
    assert abs(r["la"][0] - np.log(abs(psi))) <= 1e-10 * abs(np.log(abs(psi)))
    assert abs(r["ph"][0] - psi / abs(psi)) <= 1e-10
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.cx_project(th, torch.from_numpy(links).cuda())
    O = torch.from_numpy(r["O"]).cuda()
    s = (O * proj).sum(dim=2)
    assert torch.max(torch.abs(s - 1.0)).item() < 1e-9


# ---------------- complex64 contractions (PEPS_C64_EXACT) ----------------
# Criteria fixed from the arithmetic before the first run: the row states, site absorptions and
# environments round to complex64 (unit roundoff 6e-8) over at most Dk^(L+1) terms per entry, with
# the overlaps, ratios and logs in FP64; ln|Psi| and the phase to 1e-5, E_loc to 1e-5 of
# max(1, |E_loc|) and O to 1e-5 of the sample's largest |O| against the FP64 oracle.

def handle64(lib, L, N, Dk, h=0.4, Q=None):
    c, e = config_tables(N, 1.0, h)
    P = lib.Peps(L, N, Dk, 4, c, e, Q=Q, dtype=lib.PEPS_C64_EXACT)
    lay = Layout(L, N, [Dk] * N, Q)
    return P, lay, (c, e)


@pytest.mark.parametrize("L,N,Dk,B", [(3, 2, 2, 6), (4, 3, 1, 6), (4, 2, 2, 5), (3, 2, 3, 4)])
def test_c64_amplitude_eloc_O_against_oracle(lib, L, N, Dk, B):
    say("complex64 parity", L, N, Dk, B)
    P, lay, (c, e) = handle64(lib, L, N, Dk)
    theta = complex_theta(P.n_params, 100 + L + N + Dk)
    powers = synth.plaquette_powers(B, L, N, seed=7)
    links = np.stack([links_from_powers(powers[b], N) for b in range(B)])
    r = evaluate(P, theta, links)
    assert r["valid"].all()
    Od = dense_O(P, lay, r["O"], r["bid"])
    worst = [0.0, 0.0, 0.0, 0.0]
    for b in range(B):
        ok, T, _ = project(lay, theta, links[b])
        psi = tvmc.exact_amplitude(T)
        el = tvmc.local_energy(lay, theta, links[b], c, e)
        O = tvmc.log_derivatives(lay, theta, links[b])
        errs = (abs(r["la"][b] - np.log(abs(psi))), abs(r["ph"][b] - psi / abs(psi)),
                abs(r["el"][b] - el) / max(1.0, abs(el)), np.max(np.abs(Od[b] - O)) / np.max(np.abs(O)))
        worst = [max(w, x) for w, x in zip(worst, errs)]
    say("worst: ln|Psi| %.1e, phase %.1e, E_loc %.1e, O %.1e" % tuple(worst))
    assert worst[0] <= 1e-5 and worst[1] <= 1e-5 and worst[2] <= 1e-5 and worst[3] <= 1e-5


def test_c64_beyond_lds_against_c128(lib):
    # working states in the workspace (7 x 7, Dk = 3: 3^8 entries) on both paths, the same criteria
    # against the complex128 path (itself pinned to the oracle at this shape)
    L, N, Dk, B = 7, 2, 3, 2
    say("complex64 beyond LDS", L, N, Dk, B)
    P, lay, _ = handle(lib, L, N, Dk)
    P64, _, _ = handle64(lib, L, N, Dk)
    theta = complex_theta(P.n_params, 57)
    powers = synth.plaquette_powers(B, L, N, seed=3)
    links = np.stack([links_from_powers(powers[b], N) for b in range(B)])
    r, q = evaluate(P, theta, links), evaluate(P64, theta, links)
    la = np.max(np.abs(q["la"] - r["la"]))
    ph = np.max(np.abs(q["ph"] - r["ph"]))
    el = np.max(np.abs(q["el"] - r["el"]) / np.maximum(1.0, np.abs(r["el"])))
    O = max(np.max(np.abs(q["O"][b] - r["O"][b])) / np.max(np.abs(r["O"][b])) for b in range(B))
    say("complex64 vs complex128: ln|Psi| %.1e, phase %.1e, E_loc %.1e, O %.1e" % (la, ph, el, O))
    assert la <= 1e-5 and ph <= 1e-5 and el <= 1e-5 and O <= 1e-5


def test_c64_tvmc_steps_follow_oracle_evolution(lib):
    # eq. secondorder with complex64 contractions and the FP64 solve against the oracle's evolution:
    # <H> to 1e-6 relative and theta to 1e-4 relative after each of four steps (the solve amplifies
    # the contractions' rounding by up to |S| / shift)
    say("complex64 tvmc steps")
    _, lay, (c, e), theta, cfg = _string_problem(lib)
    P = lib.Peps(3, 2, 2, 4, c, e, Q=lay.Q.astype(np.int8), dtype=lib.PEPS_C64_EXACT)
    shift, dt, steps = 1e-3, 0.05, 4
    thetas, energies = tvmc.evolve(lay, theta, cfg, c, e, dt, steps, order=2, shift=shift)
    th = torch.from_numpy(theta.copy()).cuda()
    lk = torch.from_numpy(cfg).cuda()
    ws = P.workspace(cfg.shape[0], lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_TVMC)
    for k in range(steps):
        en, its = P.tvmc_step(th, lk, ws, dt, weights=lib.TVMC_WEIGHT_PSI2, order=2, shift=shift,
                              max_iter=5000, rtol=1e-14)
        got = th.cpu().numpy()
        err = np.linalg.norm(got - thetas[k + 1]) / np.linalg.norm(thetas[k + 1])
        say("step %d: <H> %.12f (oracle %.12f), CG %s, |theta - oracle| / |theta| %.1e"
            % (k, en.real, energies[k], its, err))
        assert abs(en.real - energies[k]) <= 1e-6 * abs(energies[k])
        assert err <= 1e-4


def test_c64_chains_sample_psi_squared(lib):
    # peps_metropolis on a complex64 handle: chi-square of the chains' end states against |Psi|^2 of
    # the complex128 path over the 16 states of the 3 x 3 Z2 string sector (acceptance decided in
    # FP64 from the complex64 contraction's ln|Psi|)
    from scipy import stats
    say("complex64 metropolis chi-square")
    P, lay, (c, e), _, cfg = _string_problem(lib)
    P64 = lib.Peps(3, 2, 2, 4, c, e, Q=lay.Q.astype(np.int8), dtype=lib.PEPS_C64_EXACT)
    theta = complex_theta(P.n_params, 31)
    th = torch.from_numpy(theta).cuda()
    ws = P.workspace(cfg.shape[0], lib.PEPS_WS_AMPLITUDE)
    proj, _, valid = P.cx_project(th, torch.from_numpy(cfg).cuda())
    la_all, _ = P.cx_amplitude(proj, valid, ws)
    p = np.exp(2 * (la_all.cpu().numpy() - la_all.max().item()))
    p /= p.sum()
    B, sweeps = 8192, 20
    start = np.random.default_rng(6).integers(0, len(cfg), B)
    links = torch.from_numpy(cfg[start]).cuda()
    ws2 = P64.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_SAMPLE)
    _, acc = P64.metropolis(th, links, 9, 1, sweeps, ws2, stream_id=0)
    torch.cuda.synchronize()
    end = links.cpu().numpy()
    index = {s.tobytes(): i for i, s in enumerate(cfg)}
    counts = np.bincount([index[s.tobytes()] for s in end], minlength=len(cfg)).astype(float)
    exp = p * B
    o2, e2, ob, eb = [], [], 0.0, 0.0
    for i in np.argsort(exp):
        ob += counts[i]
        eb += exp[i]
        if eb >= 10:
            o2.append(ob)
            e2.append(eb)
            ob = eb = 0.0
    if eb > 0:
        o2[-1] += ob
        e2[-1] += eb
    chi2 = float(np.sum((np.array(o2) - np.array(e2)) ** 2 / np.array(e2)))
    pval = 1.0 - stats.chi2.cdf(chi2, len(o2) - 1)
    say("chi2 %.1f over %d cells, p %.3f, acceptance %.3f" % (chi2, len(o2), pval, acc.sum().item() / (B * sweeps * 4)))
    assert pval > 1e-3 and len(o2) >= 4


def _c64_euler_10x10_d6(lib, theta_kind):
    L, N, Dk, B = 10, 2, 3, 2
    P, lay, _ = handle(lib, L, N, Dk)
    P64, _, _ = handle64(lib, L, N, Dk)
    if theta_kind == "random":
        theta = complex_theta(P.n_params, 31)
    else:  # the real-time workload's tensors: the toric code padded to D = 6 with 1e-3 complex noise
        theta = toric_theta(lay, Dk).astype(complex) + 1e-3 * complex_theta(P.n_params, 32, scale=1.0)
    th = torch.from_numpy(theta).cuda()
    powers = synth.plaquette_powers(B, L, N, seed=13)
    lk = torch.from_numpy(np.stack([links_from_powers(powers[b], N) for b in range(B)])).cuda()
    proj, _, valid = P64.cx_project(th, lk)
    ws = P64.workspace(B, lib.PEPS_WS_AMPLITUDE)
    la64, _ = P64.cx_amplitude(proj, valid, ws)
    O = P64.cx_logderiv(proj, valid, ws)
    ws2 = P.workspace(B, lib.PEPS_WS_AMPLITUDE)
    la128, _ = P.cx_amplitude(proj, valid, ws2)
    s = (O * proj).sum(dim=2)
    torch.cuda.synchronize()
    eul = torch.max(torch.abs(s - 1.0)).item()
    dla = torch.max(torch.abs(la64 - la128)).item()
    say("complex64 10x10 D=6, %s tensors: Euler identity %.1e, ln|Psi| vs complex128 %.1e" % (theta_kind, eul, dla))
    assert bool(valid.all())
    return eul, dla


def test_c64_euler_identity_at_the_real_time_shape(lib):
    # the real-time workload's tensors (10 x 10, D = 6) in complex64: sum_k theta_k O_k = 1 on every
    # site and ln|Psi| against the complex128 path, both to 1e-5
    eul, dla = _c64_euler_10x10_d6(lib, "toric")
    assert eul < 1e-5 and dla < 1e-5


@pytest.mark.xfail(strict=True, reason="complex64 environments of random complex tensors at 10 x 10, D = 6 "
                                       "cancel: the Euler identity holds to 5e-5, not 1e-5")
def test_c64_euler_identity_random_tensors_10x10_d6(lib):
    # measured miss, kept strict: the states' complex64 rounding (about a hundred absorptions each)
    # amplified by the cancellation of the environment sums of random complex tensors
    eul, dla = _c64_euler_10x10_d6(lib, "random")
    assert dla < 1e-5
    assert eul < 1e-5


@pytest.mark.parametrize("L,N,Dk,B,sweeps,c64", [(3, 2, 2, 64, 3, False), (4, 3, 2, 24, 2, False),
                                                 (3, 2, 3, 16, 2, False), (4, 2, 2, 32, 2, True),
                                                 (7, 2, 3, 4, 1, False)])
def test_complex_strip_chains_equal_plain_chains(lib, L, N, Dk, B, sweeps, c64):
    # peps_metropolis_strip on a complex handle makes the decisions of peps_metropolis (same
    # proposals, order and uniforms; the exact strip ratio in place of the amplitude ratio): the
    # same chains and accept counts, and ln|Psi| of the final states; (7, 2, 3): working states in
    # the workspace
    say("complex strip chains", L, N, Dk, B, sweeps, "complex64" if c64 else "complex128")
    P, lay, _ = (handle64 if c64 else handle)(lib, L, N, Dk)
    theta = complex_theta(P.n_params, 40 + L + Dk)
    th = torch.from_numpy(theta).cuda()
    _, a = P.sample_init(B, 11, 2)
    b = a.clone()
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_SAMPLE)
    la_a, acc_a = P.metropolis(th, a, 11, 1, sweeps, ws, stream_id=2)
    la_b, acc_b = P.metropolis_strip(th, b, 11, 1, sweeps, ws, stream_id=2)
    torch.cuda.synchronize()
    say("accepted %d of %d proposals" % (int(acc_a.sum()), B * sweeps * (L - 1) ** 2))
    assert torch.equal(a, b) and torch.equal(acc_a, acc_b)
    assert acc_a.sum().item() > 0
    tol = 1e-5 if c64 else 1e-10
    assert torch.max(torch.abs(la_a - la_b)).item() <= tol * max(1.0, torch.max(torch.abs(la_a)).item())
