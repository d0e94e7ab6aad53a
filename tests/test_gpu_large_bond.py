"""GPU parity of the large-bond amplitude and its adjoint (fused bond chi * D_k from 73 up to 128,
working matrices in global memory) against the FP64 oracle: every element on lattices large
enough for the cutoff to truncate, sampled outputs at the Z4 32 x 32, D = 8, chi = 64 shape, the
padded toric code (exact zero singular values), the mixed path against the FP64 one, and for O_k
the Euler identity on a whole batch, central differences and checkpointed recompute.
"""
import math

import numpy as np
import pytest
import torch

from oracle.contract import amplitude
from oracle.energy import config_tables
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth
from tests.helpers import gauge_transform, toric_theta

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _setup(lib, L, N, chi, B, seed=5678, theta=None, dtype=0):
    c, e = config_tables(N, 1.0, 0.5)
    P = lib.Peps(L, N, 2, chi, c, e, dtype=dtype)
    lay = Layout(L, N, [2] * N)
    assert P.n_params == lay.n_params
    if theta is None:
        theta = synth.theta_normals(P.n_params, N * 2)
    links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N, seed=seed)).cuda())
    return P, lay, theta, links


def _run(lib, P, theta, links):
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(links.shape[0], lib.PEPS_WS_AMPLITUDE)
    la, sg = P.amplitude(proj, valid, ws)
    flags = P.flags(links.shape[0], ws)
    torch.cuda.synchronize()
    return la.cpu().numpy(), sg.cpu().numpy(), valid.cpu().numpy(), flags.cpu().numpy()


def _oracle(lay, theta, links, chi):
    ok, T, _ = project(lay, theta, links)
    return amplitude(T, chi) if ok else (-math.inf, 0.0)


def _compare(lay, theta, host, la, sg, chi, idx, rtol):
    worst = 0.0
    for b in idx:
        o_la, o_sg = _oracle(lay, theta, host[b], chi)
        err = abs(la[b] - o_la)
        worst = max(worst, err / abs(o_la))
        assert err <= rtol * abs(o_la), (b, la[b], o_la)
        assert sg[b] == o_sg, b
    return worst


@pytest.mark.parametrize("L,N,chi,B", [(14, 2, 64, 6), (12, 3, 40, 5), (15, 2, 48, 4)])
def test_large_bond_amplitude_every_element(lib, L, N, chi, B):
    # fused bonds 128, 80 and 96: the large-bond kernel; the cutoff truncates the central cuts
    say("large bond every element", L, N, chi, B)
    P, lay, theta, links = _setup(lib, L, N, chi, B, seed=L * 7 + chi)
    assert 2 * min(chi, 2 ** (L // 2)) > 72
    la, sg, valid, flags = _run(lib, P, theta, links)
    assert valid.all() and not flags.any()
    worst = _compare(lay, theta, links.cpu().numpy(), la, sg, chi, range(B), rtol=1e-10)
    say("max rel |d ln Psi| =", worst)


def test_large_bond_z4_32x32_chi64_sampled(lib):
    # the Z4 32 x 32, D = 8, chi = 64 lattice; oracle on sampled outputs of a 64-sample batch
    L, N, chi, B = 32, 4, 64, 64
    say("large bond Z4 32x32 chi=64", B)
    P, lay, theta, links = _setup(lib, L, N, chi, B)
    la, sg, valid, flags = _run(lib, P, theta, links)
    assert valid.all() and np.all(np.isfinite(la)) and not flags.any()
    worst = _compare(lay, theta, links.cpu().numpy(), la, sg, chi, [0, B // 2, B - 1], rtol=1e-10)
    say("max rel |d ln Psi| =", worst)


def test_large_bond_padded_toric_code_is_one(lib):
    # Psi = 1 for every physical configuration; random gauges on every bond, exact zero singular
    # values at chi = 64 (fused bond 128)
    L, N, chi, B = 14, 2, 64, 8
    say("large bond toric", L, chi)
    lay = Layout(L, N, [2] * N)
    theta = gauge_transform(lay, toric_theta(lay, 2), seed=9)
    P, _, _, links = _setup(lib, L, N, chi, B, theta=theta)
    la, sg, valid, flags = _run(lib, P, theta, links)
    assert valid.all() and not flags.any()
    assert np.max(np.abs(la)) < 1e-9 and np.all(sg == 1.0)


def test_large_bond_mixed_matches_fp64(lib):
    # the mixed path's criterion (ln|Psi| within 1e-4 relative per sample) on the large-bond kernel
    L, N, chi, B = 16, 4, 64, 32
    say("large bond mixed vs fp64", L, N, chi, B)
    out = {}
    for dtype in (lib.PEPS_F64, lib.PEPS_F32_MIXED):
        P, lay, theta, links = _setup(lib, L, N, chi, B, dtype=dtype)
        out[dtype] = _run(lib, P, theta, links)
        assert out[dtype][2].all() and not out[dtype][3].any()
    a, m = out[lib.PEPS_F64][0], out[lib.PEPS_F32_MIXED][0]
    rel = np.abs(a - m) / np.abs(a)
    say("mixed rel max", rel.max())
    assert rel.max() <= 1e-4
    assert np.array_equal(out[lib.PEPS_F64][1], out[lib.PEPS_F32_MIXED][1])


def test_large_bond_deterministic_and_ragged(lib):
    L, N, chi = 14, 2, 64
    say("large bond determinism")
    P, lay, theta, links = _setup(lib, L, N, chi, 3, seed=3)
    a = _run(lib, P, theta, links)
    b = _run(lib, P, theta, links)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # a batch of one: the same first sample
    c = _run(lib, P, theta, links[:1].contiguous())
    assert c[0][0] == a[0][0]


# ---- the adjoint at fused bonds above 72 ----

def _run_O(lib, P, theta, links):
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(links.shape[0], lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_LOGDERIV)
    la, sg = P.amplitude(proj, valid, ws)
    O, _ = P.logderiv(proj, bid, valid, ws)
    torch.cuda.synchronize()
    return proj, bid, valid, la, O, ws


def _compare_O(lay, theta, links_b, O_b, chi, rtol):
    from oracle.logderiv import log_derivatives
    ok, T, _ = project(lay, theta, links_b)
    _, grads = log_derivatives(T, chi)
    L = lay.L
    scale = max(np.max(np.abs(g)) for row in grads for g in row)
    worst = 0.0
    for y in range(L):
        for x in range(L):
            g = grads[y][x].reshape(-1)
            got = O_b[y * L + x, : g.size]
            err = np.max(np.abs(got - g))
            worst = max(worst, err / scale)
            assert err <= rtol * scale, (y, x, got, g)
            assert not O_b[y * L + x, g.size:].any()
    return worst


@pytest.mark.parametrize("L,N,chi,B", [(12, 3, 40, 3), (14, 2, 64, 3), (15, 2, 48, 2)])
def test_large_bond_logderiv_every_element(lib, L, N, chi, B):
    say("large bond logderiv every element", L, N, chi, B)
    P, lay, theta, links = _setup(lib, L, N, chi, B, seed=L * 13 + N)
    proj, bid, valid, la, O, ws = _run_O(lib, P, theta, links)
    assert valid.all()
    O, lh = O.cpu().numpy(), links.cpu().numpy()
    worst = max(_compare_O(lay, theta, lh[b], O[b], chi, 1e-9) for b in range(B))
    say("worst rel", worst)


def test_large_bond_logderiv_z4_32x32_chi64(lib):
    # the Z4 32 x 32, chi = 64 shape: the Euler identity (sum over a site's selected entries of
    # proj * O = 1, truncation included) on the whole batch, the oracle on sampled outputs
    L, N, chi, B = 32, 4, 64, 64
    say("large bond logderiv Z4 32x32", B)
    P, lay, theta, links = _setup(lib, L, N, chi, B)
    proj, bid, valid, la, O, ws = _run_O(lib, P, theta, links)
    s = (proj * O).sum(dim=2)
    say("euler max", torch.max(torch.abs(s - 1.0)).item())
    assert torch.max(torch.abs(s - 1.0)).item() < 1e-9
    O, lh = O.cpu().numpy(), links.cpu().numpy()
    for b in (0, B - 1):
        say("sample", b, "worst rel", _compare_O(lay, theta, lh[b], O[b], chi, 1e-8))


def test_large_bond_logderiv_checkpoints_bitwise(lib):
    # recomputing every row (ckpt 0) and recomputing from checkpoints every 3 rows: same bits
    L, N, chi, B = 14, 2, 64, 4
    say("large bond logderiv checkpoints")
    outs = []
    for ckpt in (0, 3):
        c, e = config_tables(N, 1.0, 0.5)
        P = lib.Peps(L, N, 2, chi, c, e, ckpt_every=ckpt)
        theta = synth.theta_normals(P.n_params, N * 2)
        links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N, seed=11)).cuda())
        outs.append(_run_O(lib, P, theta, links)[4].cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_large_bond_logderiv_finite_differences(lib):
    # central differences (step 1e-6) of the GPU amplitude on 16 parameters of one sample
    L, N, chi = 14, 2, 64
    say("large bond logderiv FD")
    P, lay, theta, links = _setup(lib, L, N, chi, 1, seed=21)
    proj, bid, valid, la, O, ws = _run_O(lib, P, theta, links)
    th = torch.from_numpy(theta).cuda()
    bidh, Oh = bid.cpu().numpy()[0], O.cpu().numpy()[0]
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(16):
        s = int(rng.integers(0, L * L))
        x, y = s % L, s // L
        bs = 2 ** ((x > 0) + (x < L - 1) + (y > 0) + (y < L - 1))
        e = int(rng.integers(0, bs))
        k = P.site_offset[s] + int(bidh[s]) * bs + e
        vals = []
        for sgn in (1.0, -1.0):
            t2 = th.clone()
            t2[k] += sgn * h
            p2, _, v2 = P.project(t2, links)
            l2, _ = P.amplitude(p2, v2, ws)
            vals.append(l2.item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - Oh[s, e]) <= 1e-6 * max(1.0, abs(Oh[s, e])), (s, e, fd, Oh[s, e])


# ---- the local energy at fused bonds above 72 ----

def _run_E(lib, P, theta, links):
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(links.shape[0], lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_ENERGY)
    P.amplitude(proj, valid, ws)
    el = P.local_energy(th, links, proj, valid, ws)
    flags = P.flags(links.shape[0], ws)
    torch.cuda.synchronize()
    return el.cpu().numpy(), valid.cpu().numpy(), flags.cpu().numpy()


def _check_E(lay, theta, links, el, chi, N, idx, rtol):
    from oracle.energy import local_energy
    c, e = config_tables(N, 1.0, 0.5)
    worst = 0.0
    for b in idx:
        ref = local_energy(lay, theta, links[b], chi, c, e)
        err = abs(el[b] - ref)
        worst = max(worst, err / max(1.0, abs(ref)))
        assert err <= rtol * max(1.0, abs(ref)), (b, el[b], ref)
    return worst


@pytest.mark.parametrize("L,N,chi,B", [(12, 3, 40, 3), (14, 2, 64, 3), (15, 2, 48, 2)])
def test_large_bond_local_energy_every_element(lib, L, N, chi, B):
    say("large bond E_loc every element", L, N, chi, B)
    P, lay, theta, links = _setup(lib, L, N, chi, B, seed=L * 17 + N)
    el, valid, flags = _run_E(lib, P, theta, links)
    assert valid.all() and not flags.any()
    say("worst rel", _check_E(lay, theta, links.cpu().numpy(), el, chi, N, range(B), 1e-10))


def test_large_bond_local_energy_z4_32x32_chi64_sampled(lib):
    L, N, chi, B = 32, 4, 64, 32
    say("large bond E_loc Z4 32x32 chi=64", B)
    P, lay, theta, links = _setup(lib, L, N, chi, B)
    el, valid, flags = _run_E(lib, P, theta, links)
    assert valid.all() and np.all(np.isfinite(el)) and not flags.any()
    say("worst rel", _check_E(lay, theta, links.cpu().numpy(), el, chi, N, [0, B - 1], 1e-9))


def test_large_bond_local_energy_toric_closed_form(lib):
    # Psi = 1 for every physical configuration: E_loc = N_plaq sum_t c[t] + sum_l e[n_l]
    from oracle.energy import electric_energy
    L, N, chi, B = 14, 2, 64, 6
    say("large bond E_loc toric", L, chi)
    lay = Layout(L, N, [2] * N)
    theta = gauge_transform(lay, toric_theta(lay, 2), seed=4)
    P, _, _, links = _setup(lib, L, N, chi, B, theta=theta)
    el, valid, flags = _run_E(lib, P, theta, links)
    c, e = config_tables(N, 1.0, 0.5)
    lh = links.cpu().numpy()
    for b in range(B):
        exact = (L - 1) ** 2 * sum(c[1:]) + electric_energy(lh[b], e)
        assert abs(el[b] - exact) <= 1e-9 * max(1.0, abs(exact)), (b, el[b], exact)


# ---- the samplers at fused bonds above 72 ----

def _log_abs_fn(lay, theta, chi):
    def f(s):
        ok, T, _ = project(lay, theta, s)
        return amplitude(T, chi)[0] if ok else -np.inf
    return f


@pytest.mark.parametrize("L,N,chi,B,sweeps", [(12, 3, 40, 3, 2), (14, 2, 64, 2, 2)])
def test_large_bond_strip_chains_match_oracle(lib, L, N, chi, B, sweeps):
    # strip-ratio chains (one pass in each direction) bit-identical to the oracle's, accept counts
    # and ln|Psi| of the final states included
    from oracle.sampler import metropolis_strip
    say("large bond strip chains", L, N, chi, B, sweeps)
    c, e = config_tables(N, 1.0, 0.5)
    P = lib.Peps(L, N, 2, chi, c, e)
    lay = Layout(L, N, [2] * N)
    theta = synth.theta_normals(P.n_params, N * 2, seed=L * 7 + N)
    seed, stream = 4242, 3
    _, links = P.sample_init(B, seed, stream)
    start = links.cpu().numpy()
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_ENERGY)
    la, acc = P.metropolis_strip(torch.from_numpy(theta).cuda(), links, seed, 1, sweeps, ws, stream_id=stream)
    torch.cuda.synchronize()
    got, la, acc = links.cpu().numpy(), la.cpu().numpy(), acc.cpu().numpy()
    f = _log_abs_fn(lay, theta, chi)
    for b in range(B):
        s, a = metropolis_strip(start[b], lay, theta, chi, seed, stream, b, 1, sweeps)
        assert np.array_equal(got[b], s), b
        assert a == acc[b], (b, a, acc[b])
        lf = f(s)
        assert abs(la[b] - lf) <= 1e-10 * max(1.0, abs(lf)), (b, la[b], lf)
    assert acc.sum() > 0


def test_large_bond_plain_chains_match_oracle(lib):
    # one amplitude per proposal and chain (the large-bond amplitude), chains bit-identical
    from oracle.sampler import metropolis
    L, N, chi, B = 12, 3, 40, 2
    say("large bond plain chains", L, N, chi, B)
    c, e = config_tables(N, 1.0, 0.5)
    P = lib.Peps(L, N, 2, chi, c, e)
    lay = Layout(L, N, [2] * N)
    theta = synth.theta_normals(P.n_params, N * 2, seed=5)
    seed, stream = 2024, 1
    _, links = P.sample_init(B, seed, stream)
    start = links.cpu().numpy()
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_SAMPLE)
    la, acc = P.metropolis(torch.from_numpy(theta).cuda(), links, seed, 1, 1, ws, stream_id=stream)
    torch.cuda.synchronize()
    got, la, acc = links.cpu().numpy(), la.cpu().numpy(), acc.cpu().numpy()
    f = _log_abs_fn(lay, theta, chi)
    for b in range(B):
        s, lf, a = metropolis(start[b], f, N, seed, stream, b, 1, 1)
        assert np.array_equal(got[b], s), b
        assert a == acc[b], (b, a, acc[b])
        assert abs(la[b] - lf) <= 1e-10 * max(1.0, abs(lf)), (b, la[b], lf)
