"""Every row-sweep tuning choice against the oracle, and the autotuner.

The truncated boundary depends only on the state, so each choice of Jacobi lanes, preconditioning
of the down and up sweeps, preconditioning threshold and waves per SIMD must give the oracle's
ln|Psi|, E_loc and O_k to rounding.  Shapes: one on the chi*Dk = 72 kernels (Z3 8x8, chi = 20:
fused bonds up to 40, truncating), one on the chi*Dk <= 32 kernels (Z2 8x8, chi = 12) and one on
the large-bond kernels (Z2 14x14, chi = 64: fused bond 128, truncating; there the Jacobi lanes and
waves are fixed and only the preconditioning choices act).
"""
import numpy as np
import pytest
import torch

from oracle.contract import amplitude
from oracle.energy import config_tables, local_energy
from oracle.layout import Layout, project
from oracle.logderiv import log_derivatives
from paper_2503_20566_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def choices(g):
    base = {"jacobi_lanes": 8, "down_precond": g.PEPS_PRECOND_SORTED_QR, "up_precond": g.PEPS_PRECOND_QR_T,
            "precond_min": 16, "small_waves": 2}
    out = [base]
    for k, v in (("jacobi_lanes", 4), ("down_precond", g.PEPS_PRECOND_NONE), ("up_precond", g.PEPS_PRECOND_NONE),
                 ("up_precond", g.PEPS_PRECOND_SORTED_QR), ("precond_min", 4), ("precond_min", 32),
                 ("small_waves", 4)):
        out.append(dict(base, **{k: v}))
    out.append({"jacobi_lanes": 4, "down_precond": g.PEPS_PRECOND_NONE, "up_precond": g.PEPS_PRECOND_SORTED_QR,
                "precond_min": 4, "small_waves": 4})
    return out


@pytest.mark.parametrize("L,N,Dk,chi,B", [(8, 3, 2, 20, 4), (8, 2, 2, 12, 4), (14, 2, 2, 64, 2)])
def test_every_tuning_choice_matches_oracle(lib, L, N, Dk, chi, B):
    c, e = config_tables(N, 1.0, 0.4)
    lay = Layout(L, N, [Dk] * N)
    theta = synth.theta_normals(lay.n_params, N * Dk, seed=300 + L + N)
    powers = synth.plaquette_powers(B, L, N, seed=301)
    P = lib.Peps(L, N, Dk, chi, c, e)
    th = torch.from_numpy(theta).cuda()
    links = P.links_from_powers(torch.from_numpy(powers).cuda())
    lh = links.cpu().numpy()
    ref = []
    for b in range(B):
        ok, T, _ = project(lay, theta, lh[b])
        la, sg = amplitude(T, chi)
        el, m = local_energy(lay, theta, lh[b], chi, c, e, with_scale=True)
        _, grads = log_derivatives(T, chi)
        ref.append((la, sg, el, m, grads))
    for t in choices(lib):
        say("tuning", L, N, Dk, chi, t)
        P.set_tuning(t)
        assert P.get_tuning() == t
        proj, bid, valid = P.project(th, links)
        ws = P.workspace(B)
        la, sg = P.amplitude(proj, valid, ws)
        O, _ = P.logderiv(proj, bid, valid, ws)
        el = P.local_energy(th, links, proj, valid, ws)
        torch.cuda.synchronize()
        la, sg, O, el = la.cpu().numpy(), sg.cpu().numpy(), O.cpu().numpy(), el.cpu().numpy()
        for b, (o_la, o_sg, o_el, o_m, grads) in enumerate(ref):
            assert abs(la[b] - o_la) <= 1e-10 * abs(o_la) and sg[b] == o_sg, (t, b)
            assert abs(el[b] - o_el) <= 1e-10 * o_m, (t, b, el[b], o_el)
            scale = max(np.max(np.abs(gr)) for row in grads for gr in row)
            for y in range(L):
                for x in range(L):
                    gr = grads[y][x].reshape(-1)
                    assert np.max(np.abs(O[b, y * L + x, : gr.size] - gr)) <= 1e-9 * scale, (t, b, y, x)
        del ws


def test_autotune_sets_a_valid_tuning_and_keeps_results(lib, tmp_path):
    L, N, Dk, chi, B = 10, 3, 2, 16, 64
    c, e = config_tables(N, 1.0, 0.4)
    P = lib.Peps(L, N, Dk, chi, c, e)
    th = torch.from_numpy(synth.theta_normals(P.n_params, N * Dk)).cuda()
    links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda())
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_ENERGY)
    la0, _ = P.amplitude(proj, valid, ws)
    torch.cuda.synchronize()
    la0 = la0.clone()
    cache = str(tmp_path / "tuning.json")
    r = P.autotune(proj, valid, ws, cache=cache)
    say("autotune", r["tuning"], "candidates", len(r["candidates"]))
    assert r["source"] == "measured" and len(r["candidates"]) == 40   # chi*Dk = 32: the waves knob too
    assert P.get_tuning() == r["tuning"]
    assert all(x["ms"] > 0.0 for x in r["candidates"])
    # the tuning invalidated the workspace state; a fresh amplitude agrees to rounding
    with pytest.raises(lib.PepsError) as err:
        P.local_energy(th, links, proj, valid, ws)
    assert err.value.status == lib.PEPS_ERR_STATE
    la1, _ = P.amplitude(proj, valid, ws)
    torch.cuda.synchronize()
    assert torch.max(torch.abs(la1 - la0)).item() <= 1e-11 * torch.max(torch.abs(la0)).item()
    # a second handle of the same problem takes the cached choice without timing anything
    P2 = lib.Peps(L, N, Dk, chi, c, e)
    r2 = P2.autotune(proj, valid, ws, cache=cache)
    assert r2["source"].startswith("cache") and P2.get_tuning() == r["tuning"]
