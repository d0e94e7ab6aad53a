"""GPU parity of the variational boundary compression (var_sweeps > 0; SM S-2 "SVD or variational
compression", the fitting sweeps after each row's SVD truncation) against the oracle's
variational_refine.

* ln|Psi|, sign and E_loc (its down and up boundaries refined) of every sample on lattices that
  truncate at several cuts, on both kernel sizes (chi*Dk <= 32 and the chi*Dk = 72 instantiation),
  1 to 3 sweeps, the refined amplitude differing from the SVD truncation's;
* at exact chi the refinement leaves the amplitude exact (equal to the SVD path's);
* strip-sampler chains with refined boundaries equal the oracle's, decision for decision;
* Z3 16 x 16, D = 6, chi = 36 (the benchmark lattice), one sweep: sampled ln|Psi| and E_loc
  against the oracle, and the refined path's cost beside the SVD path's.
"""
import time

import numpy as np
import pytest
import torch

from oracle.contract import amplitude
from oracle.energy import config_tables, local_energy
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def make(lib, L, N, Dk, chi, k, h=0.4):
    c, e = config_tables(N, 1.0, h)
    P = lib.Peps(L, N, Dk, chi, c, e, var_sweeps=k)
    lay = Layout(L, N, [Dk] * N)
    theta = synth.theta_normals(P.n_params, N * Dk, seed=50 + L + N + chi)
    return P, lay, theta, (c, e)


def run(P, theta, powers):
    th = torch.from_numpy(theta).cuda()
    links = P.links_from_powers(torch.from_numpy(powers).cuda())
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(powers.shape[0], 1 | 2)
    la, sg = P.amplitude(proj, valid, ws)
    el = P.local_energy(th, links, proj, valid, ws)
    torch.cuda.synchronize()
    return links.cpu().numpy(), la.cpu().numpy(), sg.cpu().numpy(), el.cpu().numpy()


# every shape truncates at two or more cuts (with one truncated cut the SVD truncation is already the
# optimal fit and the sweeps change nothing); (12, 3, 2, 20, ...) runs the chi*Dk = 72 kernels
@pytest.mark.parametrize("L,N,Dk,chi,B,k", [(5, 3, 2, 3, 5, 1), (6, 2, 2, 3, 4, 3), (6, 3, 2, 3, 4, 2),
                                            (8, 3, 2, 5, 3, 2), (10, 2, 2, 6, 2, 1), (12, 3, 2, 20, 2, 1)])
def test_variational_every_sample_against_oracle(lib, L, N, Dk, chi, B, k):
    say("variational parity", L, N, Dk, chi, B, k)
    P, lay, theta, (c, e) = make(lib, L, N, Dk, chi, k)
    powers = synth.plaquette_powers(B, L, N, seed=11)
    links, la, sg, el = run(P, theta, powers)
    changed = False
    for b in range(B):
        ok, T, _ = project(lay, theta, links[b])
        o_la, o_sg = amplitude(T, chi, var_sweeps=k)
        s_la, _ = amplitude(T, chi)
        o_el, o_m = local_energy(lay, theta, links[b], chi, c, e, with_scale=True, var_sweeps=k)
        say("sample %d: ln|Psi| GPU %.12f oracle %.12f (SVD alone %.12f); E_loc rel %.1e"
            % (b, la[b], o_la, s_la, abs(el[b] - o_el) / o_m))
        assert abs(la[b] - o_la) <= 1e-10 * abs(o_la) and sg[b] == o_sg, b
        assert abs(el[b] - o_el) <= 1e-9 * o_m, (b, el[b], o_el)
        changed = changed or abs(o_la - s_la) > 1e-9 * abs(s_la)
    assert changed                       # the sweeps moved the amplitude off the SVD truncation's


def test_variational_at_exact_chi_is_exact(lib):
    L, N, Dk, chi, B = 5, 3, 2, 16, 4
    P, lay, theta, _ = make(lib, L, N, Dk, chi, 2)
    P0, _, _, _ = make(lib, L, N, Dk, chi, 0)
    powers = synth.plaquette_powers(B, L, N, seed=12)
    _, la, sg, el = run(P, theta, powers)
    _, la0, sg0, el0 = run(P0, theta, powers)
    assert np.max(np.abs(la - la0)) <= 1e-11 * np.max(np.abs(la0)) and np.array_equal(sg, sg0)
    assert np.max(np.abs(el - el0)) <= 1e-9 * np.max(np.abs(el0))


def test_variational_strip_chains_match_oracle(lib):
    from oracle.sampler import metropolis_strip
    say("variational strip metropolis")
    L, N, Dk, chi, B, k, sweeps = 5, 3, 2, 3, 4, 2, 2
    P, lay, theta, _ = make(lib, L, N, Dk, chi, k)
    _, links = P.sample_init(B, 77, 1)
    start = links.cpu().numpy()
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_ENERGY)
    la, acc = P.metropolis_strip(torch.from_numpy(theta).cuda(), links, 77, 1, sweeps, ws, stream_id=1)
    torch.cuda.synchronize()
    got, acc = links.cpu().numpy(), acc.cpu().numpy()
    for b in range(B):
        s, a = metropolis_strip(start[b], lay, theta, chi, 77, 1, b, 1, sweeps, var_sweeps=k)
        assert np.array_equal(got[b], s) and a == acc[b], b
    assert acc.sum() > 0


def test_variational_logderiv_is_refused(lib):
    P, lay, theta, _ = make(lib, 4, 2, 2, 2, 1)
    th = torch.from_numpy(theta).cuda()
    links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(2, 4, 2)).cuda())
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(2)
    P.amplitude(proj, valid, ws)
    with pytest.raises(lib.PepsError) as err:
        P.logderiv(proj, bid, valid, ws)
    assert err.value.status == lib.PEPS_ERR_UNSUPPORTED


def test_variational_benchmark_lattice(lib):
    L, N, Dk, chi, B = 16, 3, 2, 36, 256
    say("variational z3 16x16 chi 36, B", B)
    P, lay, theta, (c, e) = make(lib, L, N, Dk, chi, 1)
    P0, _, _, _ = make(lib, L, N, Dk, chi, 0)
    powers = synth.plaquette_powers(B, L, N)
    times = {}
    for name, H in (("svd", P0), ("variational", P)):
        th = torch.from_numpy(theta).cuda()
        links = H.links_from_powers(torch.from_numpy(powers).cuda())
        proj, bid, valid = H.project(th, links)
        ws = H.workspace(B, 1)
        H.amplitude(proj, valid, ws)
        torch.cuda.synchronize()
        t0 = time.time()
        la, sg = H.amplitude(proj, valid, ws)
        torch.cuda.synchronize()
        times[name] = time.time() - t0
        if name == "variational":
            la_v, sg_v, lh = la.cpu().numpy(), sg.cpu().numpy(), links.cpu().numpy()
    say("amplitude of %d samples: SVD %.3f s, SVD + 1 sweep %.3f s" % (B, times["svd"], times["variational"]))
    for b in (0, B - 1):
        ok, T, _ = project(lay, theta, lh[b])
        o_la, o_sg = amplitude(T, chi, var_sweeps=1)
        assert abs(la_v[b] - o_la) <= 1e-10 * abs(o_la) and sg_v[b] == o_sg, b
