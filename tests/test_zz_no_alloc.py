"""peps_amplitude_noalloc (fixed in-library scratch, no allocation) against peps_amplitude.

Both run the same kernels on the same inputs, so ln|Psi| and sign must be bit-identical.  Two calls
in a row on each shape, the second with a smaller, different batch (the scratch keeps the first
call's contents); a batch beyond the fixed scratch is refused before anything runs.
"""
import numpy as np
import pytest
import torch

from oracle.contract import amplitude
from oracle.energy import config_tables
from oracle.lattice import links_from_powers
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("L,N,Dk,chi,B1,B2", [(16, 3, 2, 36, 60, 23), (4, 2, 1, 16, 256, 7),
                                              (10, 2, 2, 16, 40, 9)])
def test_noalloc_amplitude_equals_workspace_amplitude(lib, L, N, Dk, chi, B1, B2):
    say("noalloc amplitude", L, N, Dk, chi, B1, B2)
    c, e = config_tables(N, 1.0, 0.4)
    P = lib.Peps(L, N, Dk, chi, c, e)
    theta = synth.theta_normals(P.n_params, N * Dk)
    th = torch.from_numpy(theta).cuda()
    lay = Layout(L, N, [Dk] * N)
    for call, (B, seed) in enumerate(((B1, 901), (B2, 902))):
        powers = synth.plaquette_powers(B, L, N, seed=seed)
        links = P.links_from_powers(torch.from_numpy(powers).cuda())
        proj, bid, valid = P.project(th, links)
        la, sg = P.amplitude_noalloc(proj, valid)
        ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE)
        la_ref, sg_ref = P.amplitude(proj, valid, ws)
        torch.cuda.synchronize()
        say("call %d: B = %d, max |difference| %.1e" % (call, B, (la - la_ref).abs().max().item()))
        assert torch.equal(la, la_ref) and torch.equal(sg, sg_ref)
        # one sample against the oracle as well
        ok, T, _ = project(lay, theta, links_from_powers(powers[B - 1], N))
        o_la, o_sg = amplitude(T, chi)
        assert abs(la[B - 1].item() - o_la) <= 1e-10 * abs(o_la) and sg[B - 1].item() == o_sg
        del ws


def test_noalloc_refuses_batches_beyond_the_scratch(lib):
    # 68 samples at L = 16, chi = 36, Dk = 2 need more than the 128 MiB scratch (67 fit); the
    # buffers are sized for the batch (all samples invalid) so nothing could read out of bounds
    L, B = 16, 68
    c, e = config_tables(3, 1.0, 0.4)
    P = lib.Peps(L, 3, 2, 36, c, e)
    proj = torch.zeros((B, L * L, 16), dtype=torch.float64, device="cuda")
    valid = torch.zeros((B,), dtype=torch.uint8, device="cuda")
    la = torch.zeros((B,), dtype=torch.float64, device="cuda")
    sg = torch.zeros((B,), dtype=torch.float64, device="cuda")
    st = lib.lib().peps_amplitude_noalloc(P._h, lib._ptr(proj), lib._ptr(valid), B, lib._ptr(la),
                                          lib._ptr(sg), lib._stream())
    assert st == lib.PEPS_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert not la.any()
