"""GPU parity of the local energy against the oracle (FP64 path): every element on small
lattices, sampled outputs at the full 16 x 16 shapes, closed forms at full shape (toric code),
zero-amplitude configurations."""
import math

import numpy as np
import pytest
import torch

from oracle.energy import config_tables, electric_energy, local_energy
from oracle.lattice import n_plaquettes
from oracle.layout import Layout
from paper_2503_20566_amd import synth
from tests.helpers import gauge_transform, toric_theta

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def run(lib, L, N, Dk, chi, B, h=0.4, theta=None, seed=5678, links_host=None):
    c, e = config_tables(N, 1.0, h)
    P = lib.Peps(L, N, Dk, chi, c, e)
    lay = Layout(L, N, [Dk] * N)
    if theta is None:
        theta = synth.theta_normals(P.n_params, N * Dk)
    if links_host is None:
        powers = synth.plaquette_powers(B, L, N, seed=seed)
        links = P.links_from_powers(torch.from_numpy(powers).cuda())
    else:
        links = torch.from_numpy(links_host).cuda()
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B)
    P.amplitude(proj, valid, ws)
    el = P.local_energy(th, links, proj, valid, ws)
    torch.cuda.synchronize()
    return lay, theta, links.cpu().numpy(), el.cpu().numpy(), valid.cpu().numpy(), (c, e)


def check(lay, theta, links, el, chi, tabs, idx, rtol):
    worst = 0.0
    for b in idx:
        ref = local_energy(lay, theta, links[b], chi, *tabs)
        err = abs(el[b] - ref)
        worst = max(worst, err / max(1.0, abs(ref)))
        assert err <= rtol * max(1.0, abs(ref)), (b, el[b], ref)
    return worst


def test_eloc_config1_all_samples(lib):
    say("eloc config1")
    L, N, Dk, chi, B = 4, 2, 1, 16, 256
    lay, theta, links, el, valid, tabs = run(lib, L, N, Dk, chi, B, h=0.5)
    assert valid.all()
    say("worst rel", check(lay, theta, links, el, chi, tabs, range(B), 1e-11))


@pytest.mark.parametrize("L,N,Dk,chi,B", [(2, 3, 2, 4, 7), (3, 2, 2, 4, 9), (4, 3, 2, 4, 12),
                                          (6, 3, 2, 3, 10), (5, 4, 2, 5, 6), (7, 2, 2, 6, 5)])
def test_eloc_small_lattices_every_element(lib, L, N, Dk, chi, B):
    say("eloc small", L, N, Dk, chi, B)
    lay, theta, links, el, valid, tabs = run(lib, L, N, Dk, chi, B, seed=L * 7 + N)
    assert valid.all()
    check(lay, theta, links, el, chi, tabs, range(B), 1e-10)


@pytest.mark.parametrize("L,N,Dk,chi,B,h", [(16, 3, 2, 36, 2048, 0.4), (16, 2, 2, 16, 4096, 0.3)])
def test_eloc_full_shape_sampled(lib, L, N, Dk, chi, B, h):
    say("eloc full shape", L, N, Dk, chi, B)
    lay, theta, links, el, valid, tabs = run(lib, L, N, Dk, chi, B, h=h)
    assert valid.all() and np.all(np.isfinite(el))
    say("worst rel", check(lay, theta, links, el, chi, tabs, [0, B // 2, B - 1], 1e-9))


def test_eloc_toric_full_shape_closed_form(lib):
    # Psi = 1: E_loc = N_plaq * sum_t c[t] + sum_l e[n_l] for every sample, at 16x16 Z3 chi = 36
    say("eloc toric 16x16")
    L, N, Dk, chi, B = 16, 3, 2, 36, 128
    lay = Layout(L, N, [Dk] * N)
    theta = gauge_transform(lay, toric_theta(lay, Dk), seed=9)
    lay, theta, links, el, valid, (c, e) = run(lib, L, N, Dk, chi, B, theta=theta)
    want = np.array([n_plaquettes(L) * float(np.sum(c[1:])) + electric_energy(links[b], e) for b in range(B)])
    assert np.max(np.abs(el - want)) < 1e-8


def test_eloc_zero_amplitude_is_nan(lib):
    say("eloc invalid")
    L, N, Dk, chi, B = 5, 3, 2, 4, 4
    powers = synth.plaquette_powers(B, L, N, seed=3)
    from oracle.lattice import links_from_powers
    host = np.stack([links_from_powers(powers[b], N) for b in range(B)])
    host[1, 0, 2, 2] = (host[1, 0, 2, 2] + 1) % N
    lay, theta, links, el, valid, tabs = run(lib, L, N, Dk, chi, B, links_host=host)
    assert list(valid) == [1, 0, 1, 1]
    assert math.isnan(el[1])
    check(lay, theta, links, el, chi, tabs, [0, 2, 3], 1e-10)


def test_eloc_requires_matching_amplitude_call(lib):
    say("eloc state check")
    c, e = config_tables(3, 1.0, 0.4)
    P = lib.Peps(4, 3, 2, 4, c, e)
    theta = torch.from_numpy(synth.theta_normals(P.n_params, 6)).cuda()
    links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(4, 4, 3)).cuda())
    proj, bid, valid = P.project(theta, links)
    ws = P.workspace(4)
    with pytest.raises(lib.PepsError) as err:
        P.local_energy(theta, links, proj, valid, ws)
    assert err.value.status == lib.PEPS_ERR_STATE
