"""The ragged batch (several lattices, one launch per boundary row) against each lattice's own
peps_amplitude and the oracle.

Groups whose lattice selects the same row-sweep instantiation as the ragged launch give the same
bits; a smaller lattice whose own kernel is the chi * D_k <= 32 one agrees to rounding.  The
workspaces are left as peps_amplitude leaves them, so O_k and E_loc may follow on each.
"""
import math

import numpy as np
import pytest
import torch

from oracle.contract import amplitude
from oracle.energy import config_tables
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _group(lib, L, N, chi, B, seed):
    c, e = config_tables(N, 1.0, 0.5)
    P = lib.Peps(L, N, 2, chi, c, e)
    theta = synth.theta_normals(P.n_params, N * 2, seed=seed)
    th = torch.from_numpy(theta).cuda()
    links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N, seed=seed + 1)).cuda())
    proj, bid, valid = P.project(th, links)
    return dict(P=P, L=L, N=N, chi=chi, theta=theta, th=th, links=links, proj=proj, bid=bid, valid=valid)


def _alone(lib, g, what):
    ws = g["P"].workspace(g["proj"].shape[0], what)
    la, sg = g["P"].amplitude(g["proj"], g["valid"], ws)
    return la, sg, ws


def _oracle(g, b):
    ok, T, _ = project(Layout(g["L"], g["N"], [2] * g["N"]), g["theta"], g["links"][b].cpu().numpy())
    return amplitude(T, g["chi"]) if ok else (-math.inf, 0.0)


def test_ragged_matches_each_lattice_alone(lib):
    # the Z4 lattices of the 32 x 32 study at chi = 36 (8 x 8 alone runs the chi * D_k <= 32 kernel)
    say("ragged Z4 8/12/24 chi=36")
    groups = [_group(lib, L, 4, 36, B, seed) for L, B, seed in ((8, 24, 1), (12, 16, 2), (24, 8, 3))]
    amp = lib.PEPS_WS_AMPLITUDE
    alone = [_alone(lib, g, amp)[:2] for g in groups]
    wss = [g["P"].workspace(g["proj"].shape[0], amp) for g in groups]
    out = lib.amplitude_ragged([(g["P"], g["proj"], g["valid"], ws) for g, ws in zip(groups, wss)])
    torch.cuda.synchronize()
    for g, (la_a, sg_a), (la_r, sg_r) in zip(groups, alone, out):
        assert torch.equal(sg_a, sg_r), g["L"]
        if g["L"] == 8:
            rel = ((la_a - la_r).abs() / la_a.abs()).max().item()
            say("L 8 rel", rel)
            assert rel <= 1e-12
        else:
            assert torch.equal(la_a, la_r), g["L"]
        la = la_r.cpu().numpy()
        for b in (0, la.shape[0] - 1):
            o_la, o_sg = _oracle(g, b)
            assert abs(la[b] - o_la) <= 1e-10 * abs(o_la), (g["L"], b, la[b], o_la)
            assert sg_r[b].item() == o_sg


def test_ragged_workspace_serves_logderiv_and_energy(lib):
    say("ragged then O and E_loc")
    groups = [_group(lib, L, 3, 12, B, seed) for L, B, seed in ((10, 12, 4), (12, 8, 5))]
    res = []
    for mode in ("alone", "ragged"):
        wss = [g["P"].workspace(g["proj"].shape[0]) for g in groups]
        if mode == "alone":
            for g, ws in zip(groups, wss):
                g["P"].amplitude(g["proj"], g["valid"], ws)
        else:
            lib.amplitude_ragged([(g["P"], g["proj"], g["valid"], ws) for g, ws in zip(groups, wss)])
        out = []
        for g, ws in zip(groups, wss):
            O, _ = g["P"].logderiv(g["proj"], g["bid"], g["valid"], ws)
            el = g["P"].local_energy(g["th"], g["links"], g["proj"], g["valid"], ws)
            out.append((O.clone(), el.clone()))
        torch.cuda.synchronize()
        res.append(out)
    for (Oa, ea), (Or, er) in zip(*res):
        assert torch.equal(Oa, Or) and torch.equal(ea, er)


def test_ragged_large_bonds_and_edge_groups(lib):
    # two large-bond lattices in one launch, bit-identical to each alone; then groups with one row
    # (L = 3), none (L = 2) and an empty batch beside a full one
    say("ragged large bonds")
    amp = lib.PEPS_WS_AMPLITUDE
    groups = [_group(lib, 14, 2, 64, 3, 6), _group(lib, 16, 2, 64, 2, 7)]
    alone = [_alone(lib, g, amp)[:2] for g in groups]
    wss = [g["P"].workspace(g["proj"].shape[0], amp) for g in groups]
    out = lib.amplitude_ragged([(g["P"], g["proj"], g["valid"], ws) for g, ws in zip(groups, wss)])
    torch.cuda.synchronize()
    for (la_a, sg_a), (la_r, sg_r) in zip(alone, out):
        assert torch.equal(la_a, la_r) and torch.equal(sg_a, sg_r)
    say("ragged edge groups")
    groups = [_group(lib, 3, 3, 4, 5, 8), _group(lib, 2, 3, 4, 4, 9), _group(lib, 9, 3, 4, 6, 10)]
    empty = groups[2]["proj"][:0], groups[2]["valid"][:0]
    alone = [_alone(lib, g, amp)[:2] for g in groups]
    wss = [g["P"].workspace(g["proj"].shape[0], amp) for g in groups]
    items = [(g["P"], g["proj"], g["valid"], ws) for g, ws in zip(groups, wss)]
    items.append((groups[2]["P"], empty[0], empty[1], wss[2]))
    out = lib.amplitude_ragged(items)
    torch.cuda.synchronize()
    for g, (la_a, sg_a), (la_r, sg_r) in zip(groups, alone, out):
        assert torch.equal(sg_a, sg_r), g["L"]
        rel = ((la_a - la_r).abs() / la_a.abs().clamp_min(1e-300)).max().item()
        assert rel <= 1e-12, (g["L"], rel)
    assert out[3][0].numel() == 0
