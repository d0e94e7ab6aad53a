"""GPU parity of link generation, projection and the boundary-MPS amplitude against the oracle.

Integer work (links, block ids, valid flags) and the gather are compared bit for bit; ln|Psi| is
compared element by element against the FP64 oracle (relative 1e-10 on small lattices, sampled
outputs at the full 16 x 16 shapes), and the sign exactly.
"""
import math

import numpy as np
import pytest
import torch

from oracle.contract import amplitude
from oracle.energy import config_tables
from oracle.lattice import gauss_residual, links_from_powers
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth
from tests.helpers import gauge_transform, toric_theta

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def make(lib, L, N, Dk, chi, B, seed=5678, theta=None, dtype=0):
    c, e = config_tables(N, 1.0, 0.4)
    P = lib.Peps(L, N, Dk, chi, c, e, dtype=dtype)
    lay = Layout(L, N, [Dk] * N)
    assert P.n_params == lay.n_params
    if theta is None:
        theta = synth.theta_normals(P.n_params, N * Dk)
    powers = synth.plaquette_powers(B, L, N, seed=seed)
    return P, lay, theta, powers


def gpu_links(P, powers):
    return P.links_from_powers(torch.from_numpy(powers).cuda())


def oracle_amp(lay, theta, links, chi):
    ok, T, _ = project(lay, theta, links)
    return amplitude(T, chi) if ok else (-math.inf, 0.0)


@pytest.mark.parametrize("L,N", [(16, 3), (8, 4), (4, 2), (2, 5)])
def test_links_from_powers_bit_exact(lib, L, N):
    say("links_from_powers", L, N)
    P, lay, theta, powers = make(lib, L, N, 1, 4, 37, seed=L * 10 + N)
    g = gpu_links(P, powers).cpu().numpy()
    for b in range(powers.shape[0]):
        assert np.array_equal(g[b], links_from_powers(powers[b], N)), b


@pytest.mark.parametrize("L,N,Dk", [(16, 3, 2), (5, 4, 2), (4, 2, 1)])
def test_project_bit_exact_including_violations(lib, L, N, Dk):
    say("project", L, N, Dk)
    B = 23
    P, lay, theta, powers = make(lib, L, N, Dk, 4, B)
    links = gpu_links(P, powers)
    rng = np.random.default_rng(1)
    host = links.cpu().numpy()
    for b in range(0, B, 3):       # break the Gauss law in every third sample
        d, y, x = rng.integers(0, 2), rng.integers(0, L - 1), rng.integers(0, L - 1)
        host[b, d, y, x] = (host[b, d, y, x] + 1) % N
    links = torch.from_numpy(host).cuda()
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    torch.cuda.synchronize()
    proj, bid, valid = proj.cpu().numpy(), bid.cpu().numpy(), valid.cpu().numpy()
    for b in range(B):
        ok, T, obid = project(lay, theta, host[b])
        assert bool(valid[b]) == ok == (np.all(gauss_residual(host[b], N) == 0))
        assert np.array_equal(bid[b].reshape(L, L), obid)
        if ok:
            for y in range(L):
                for x in range(L):
                    blk = T[y][x].reshape(-1)
                    row = proj[b, y * L + x]
                    assert np.array_equal(row[: blk.size], blk) and not row[blk.size:].any()


def _run_amp(P, theta, links):
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(links.shape[0])
    la, sg = P.amplitude(proj, valid, ws)
    torch.cuda.synchronize()
    return la.cpu().numpy(), sg.cpu().numpy(), valid.cpu().numpy()


def _compare(lay, theta, links_host, la, sg, chi, idx, rtol, atol=1e-12):
    worst = 0.0
    for b in idx:
        o_la, o_sg = oracle_amp(lay, theta, links_host[b], chi)
        err = abs(la[b] - o_la)
        worst = max(worst, err)
        assert err <= max(atol, rtol * abs(o_la)), (b, la[b], o_la)
        assert sg[b] == o_sg, b
    return worst


def test_amplitude_config1_all_samples(lib):
    # Z2 4x4, D_k = 1 (D = 2), chi = 16 exact, 256 samples: every output element.
    say("amplitude config1")
    P, lay, theta, powers = make(lib, 4, 2, 1, 16, 256)
    links = gpu_links(P, powers)
    la, sg, valid = _run_amp(P, theta, links)
    assert valid.all()
    worst = _compare(lay, theta, links.cpu().numpy(), la, sg, 16, range(256), rtol=0, atol=1e-12)
    say("config1 max |d ln Psi| =", worst)


@pytest.mark.parametrize("L,N,Dk,chi,B", [(4, 3, 2, 4, 40), (6, 3, 2, 3, 33), (7, 2, 2, 5, 29),
                                          (6, 4, 2, 6, 17), (3, 2, 2, 1, 9), (9, 3, 2, 7, 5)])
def test_amplitude_small_lattices_every_element(lib, L, N, Dk, chi, B):
    say("amplitude small", L, N, Dk, chi, B)
    P, lay, theta, powers = make(lib, L, N, Dk, chi, B, seed=L + 100 * chi)
    links = gpu_links(P, powers)
    la, sg, valid = _run_amp(P, theta, links)
    assert valid.all()
    _compare(lay, theta, links.cpu().numpy(), la, sg, chi, range(B), rtol=1e-10)


@pytest.mark.parametrize("L,N,Dk,chi,B", [(16, 3, 2, 36, 2048), (16, 2, 2, 16, 4096)])
def test_amplitude_full_shape_sampled(lib, L, N, Dk, chi, B):
    # the batch and launch configuration the benchmark times; oracle on sampled outputs
    say("amplitude full shape", L, N, Dk, chi, B)
    P, lay, theta, powers = make(lib, L, N, Dk, chi, B)
    links = gpu_links(P, powers)
    la, sg, valid = _run_amp(P, theta, links)
    assert valid.all() and np.all(np.isfinite(la))
    idx = [0, 1, B // 3, B // 2, B - 2, B - 1]
    worst = _compare(lay, theta, links.cpu().numpy(), la, sg, chi, idx, rtol=1e-10)
    say("full shape max |d ln Psi| =", worst)


def test_invalid_samples_give_zero_amplitude(lib):
    say("amplitude invalid")
    P, lay, theta, powers = make(lib, 6, 3, 2, 4, 8)
    host = gpu_links(P, powers).cpu().numpy()
    host[2, 0, 3, 1] = (host[2, 0, 3, 1] + 1) % 3
    host[5, 1, 0, 0] = (host[5, 1, 0, 0] + 2) % 3
    la, sg, valid = _run_amp(P, theta, torch.from_numpy(host).cuda())
    assert list(valid) == [1, 1, 0, 1, 1, 0, 1, 1]
    for b in (2, 5):
        assert la[b] == -math.inf and sg[b] == 0.0
    _compare(lay, theta, host, la, sg, 4, [0, 1, 3, 4, 6, 7], rtol=1e-10)


def test_padded_toric_code_full_shape_is_one(lib):
    # Psi = 1 for every physical configuration, at the full 16x16 Z3 D_k = 2 chi = 36 shape, with
    # random gauges on every bond (exact rank-deficient inputs exercise zero singular values).
    say("amplitude toric 16x16")
    L, N, Dk, chi, B = 16, 3, 2, 36, 64
    lay = Layout(L, N, [Dk] * N)
    theta = gauge_transform(lay, toric_theta(lay, Dk), seed=5)
    P, _, _, powers = make(lib, L, N, Dk, chi, B, theta=theta)
    la, sg, valid = _run_amp(P, theta, gpu_links(P, powers))
    assert valid.all()
    assert np.max(np.abs(la)) < 1e-9 and np.all(sg == 1.0)


def test_amplitude_is_deterministic(lib):
    say("amplitude determinism")
    P, lay, theta, powers = make(lib, 10, 3, 2, 12, 64)
    links = gpu_links(P, powers)
    a = _run_amp(P, theta, links)
    b = _run_amp(P, theta, links)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_batch_of_one_and_ragged(lib):
    say("amplitude B=1,3")
    for B in (1, 3):
        P, lay, theta, powers = make(lib, 5, 2, 2, 3, B, seed=B)
        links = gpu_links(P, powers)
        la, sg, valid = _run_amp(P, theta, links)
        _compare(lay, theta, links.cpu().numpy(), la, sg, 3, range(B), rtol=1e-10)


@pytest.mark.parametrize("L,N,Dk,chi,B", [(6, 3, 2, 4, 16), (10, 3, 2, 20, 16)])
def test_phase_clocks_leave_results_unchanged(lib, L, N, Dk, chi, B):
    # peps_profile_phases only reads the shader clock: ln|Psi| bit-identical with and without it,
    # every phase that runs at this shape booked, nothing negative
    say("phase clocks", L, N, Dk, chi, B)
    c, e = config_tables(N, 1.0, 0.4)
    P = lib.Peps(L, N, Dk, chi, c, e)
    theta = torch.from_numpy(synth.theta_normals(P.n_params, N * Dk)).cuda()
    links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda())
    proj, _, valid = P.project(theta, links)
    ws = P.workspace(B)
    la0, sg0 = P.amplitude(proj, valid, ws)
    cnt = torch.zeros(len(lib.PHASES), dtype=torch.int64, device="cuda")
    P.profile_phases(cnt)
    la1, sg1 = P.amplitude(proj, valid, ws)
    P.profile_phases(None)
    torch.cuda.synchronize()
    cyc = dict(zip(lib.PHASES, cnt.cpu().tolist()))
    say("cycles", cyc)
    assert torch.equal(la0, la1) and torch.equal(sg0, sg1)
    assert all(v >= 0 for v in cyc.values())
    for ph in ("X", "QR", "Theta", "Jacobi", "rest"):
        assert cyc[ph] > 0, ph
