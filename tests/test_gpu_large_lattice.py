"""Z4 lattices of the 32 x 32 study (8 x 8, 12 x 12, 24 x 24, 32 x 32; D_k = 2, D = 8) at chi = 36,
the largest cutoff the kernels hold with D_k = 2 (chi * D_k = 72; the study's chi = 64 needs 128).

* ln|Psi|, sign and every log-derivative element of sampled configurations against the oracle,
  FP64 path; the mixed path's ln|Psi| within 1e-4 relative of the FP64 oracle on the same samples;
* the per-site Euler identity sum_k theta_k O_k = 1 on the whole batch (any size, truncation on);
* E_loc at 32 x 32 against the closed form of the gauged, padded toric code (Psi = 1 on every
  physical configuration: E_loc = N_plaq sum_t c[t] + sum_l e[n_l]).

Each lattice size is its own handle and launch sequence (the ragged variant that mixes sizes in
one launch is not built).
"""
import numpy as np
import pytest
import torch

from oracle.contract import amplitude
from oracle.energy import config_tables, electric_energy
from oracle.lattice import n_plaquettes
from oracle.layout import Layout, project
from oracle.logderiv import log_derivatives
from paper_2503_20566_amd import synth
from tests.helpers import gauge_transform, toric_theta

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def run(lib, L, N, Dk, chi, B, dtype, theta=None, energy=False, grads=True):
    c, e = config_tables(N, 1.0, 0.5)
    P = lib.Peps(L, N, Dk, chi, c, e, dtype=dtype)
    if theta is None:
        theta = synth.theta_normals(P.n_params, N * Dk)
    links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda())
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B)
    la, sg = P.amplitude(proj, valid, ws)
    el = P.local_energy(th, links, proj, valid, ws) if energy else None
    O, euler = None, None
    if grads:
        O, _ = P.logderiv(proj, bid, valid, ws)
        euler = (O * proj).sum(dim=2)
    torch.cuda.synchronize()
    assert bool(valid.all())
    host = lambda t: None if t is None else t.cpu().numpy()
    return theta, host(links), host(la), host(sg), host(el), host(O), host(euler), (c, e)


@pytest.mark.parametrize("L,B,idx", [(8, 64, [0, 63]), (12, 64, [0, 63]), (24, 32, [0, 31]),
                                     (32, 32, [0, 31])])
def test_z4_lattices_against_oracle(lib, L, B, idx):
    N, Dk, chi = 4, 2, 36
    say("z4 large lattice fp64", L, B)
    theta, lh, la, sg, _, O, euler, _ = run(lib, L, N, Dk, chi, B, lib.PEPS_F64)
    assert np.max(np.abs(euler - 1.0)) < 1e-9
    say("mixed", L, B)
    _, _, la_m, _, _, _, euler_m, _ = run(lib, L, N, Dk, chi, B, lib.PEPS_F32_MIXED)
    lay = Layout(L, N, [Dk] * N)
    for b in idx:
        ok, T, _ = project(lay, theta, lh[b])
        ola, osg = amplitude(T, chi)
        assert abs(la[b] - ola) <= 1e-10 * abs(ola), (b, la[b], ola)
        assert sg[b] == osg
        assert abs(la_m[b] - ola) <= 1e-4 * abs(ola), (b, la_m[b], ola)
        _, grads = log_derivatives(T, chi)
        scale = max(np.max(np.abs(g)) for row in grads for g in row)
        worst = 0.0
        for y in range(L):
            for x in range(L):
                g = grads[y][x].reshape(-1)
                err = np.max(np.abs(O[b, y * L + x, : g.size] - g))
                worst = max(worst, err / scale)
        say("sample", b, "ln|Psi| rel fp64 %.1e mixed %.1e, O rel %.1e" %
            (abs(la[b] - ola) / abs(ola), abs(la_m[b] - ola) / abs(ola), worst))
        assert worst <= 1e-8


def test_z4_32x32_toric_code_energy(lib):
    L, N, Dk, chi, B = 32, 4, 2, 36, 32
    say("z4 32x32 toric energy")
    lay = Layout(L, N, [Dk] * N)
    theta = gauge_transform(lay, toric_theta(lay, Dk), seed=13)
    _, lh, la, _, el, _, euler, (c, e) = run(lib, L, N, Dk, chi, B, lib.PEPS_F64, theta=theta, energy=True,
                                              grads=False)
    want = np.array([n_plaquettes(L) * float(np.sum(c[1:])) + electric_energy(lh[b], e) for b in range(B)])
    say("max |E_loc - closed form| %.2e, max |ln Psi| %.2e" % (np.max(np.abs(el - want)), np.max(np.abs(la))))
    assert np.max(np.abs(el - want)) < 1e-8
    assert np.max(np.abs(la)) < 1e-8


def test_z4_32x32_mixed_whole_batch(lib):
    # The whole 1024-sample batch of the Z4 32 x 32 study at chi = 36: the mixed path's FP32 row
    # products stay inside FP32's exponent range (exact power-of-two prescale), so every E_loc is
    # finite, ln|Psi| is within 1e-5 relative of the FP64 path for every sample and the
    # |Psi|^2-weighted E/site within 1e-5; the worst sample is checked against the oracle.
    L, N, Dk, chi, B = 32, 4, 2, 36, 1024
    say("z4 32x32 mixed whole batch")
    c, e = config_tables(N, 1.0, 0.5)
    out = {}
    for dt in (lib.PEPS_F64, lib.PEPS_F32_MIXED):
        P = lib.Peps(L, N, Dk, chi, c, e, dtype=dt, ckpt_every=1)
        theta = synth.theta_normals(P.n_params, N * Dk)
        links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda())
        th = torch.from_numpy(theta).cuda()
        proj, bid, valid = P.project(th, links)
        ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_ENERGY)
        la, _ = P.amplitude(proj, valid, ws)
        el = P.local_energy(th, links, proj, valid, ws)
        torch.cuda.synchronize()
        out[dt] = (la.cpu().numpy(), el.cpu().numpy(), links.cpu().numpy(), theta)
        del ws, proj
    la_d, el_d, lh, theta = out[lib.PEPS_F64]
    la_m, el_m, _, _ = out[lib.PEPS_F32_MIXED]
    assert np.isfinite(el_d).all() and np.isfinite(el_m).all()
    rel = np.abs(la_m - la_d) / np.abs(la_d)
    w = np.exp(2.0 * (la_d - la_d.max()))
    es_d, es_m = np.sum(w * el_d) / np.sum(w), np.sum(w * el_m) / np.sum(w)
    say("ln|Psi| rel p50 %.1e p99 %.1e max %.1e; E/site rel %.1e" %
        (np.percentile(rel, 50), np.percentile(rel, 99), rel.max(), abs(es_m - es_d) / abs(es_d)))
    assert rel.max() <= 1e-5
    assert abs(es_m - es_d) <= 1e-5 * abs(es_d)
    b = int(np.argmax(rel))
    ok, T, _ = project(Layout(L, N, [Dk] * N), theta, lh[b])
    ola, _ = amplitude(T, chi)
    assert abs(la_d[b] - ola) <= 1e-10 * abs(ola)
    assert abs(la_m[b] - ola) <= 1e-5 * abs(ola)


def test_z4_32x32_checkpoints_and_tape_bitwise_and_their_memory(lib):
    # the log-derivatives at the 32 x 32 shape from the stored tape, from every row recomputed and
    # from checkpoints every 8 rows: the same arithmetic, so the same bits; the workspace each mode
    # needs per sample (the tape is the HBM-for-compute trade: about 0.2 GB per sample here)
    from tests.test_gpu_logderiv import run_O, setup
    L, N, Dk, chi, B = 32, 4, 2, 36, 4
    outs, sizes = [], {}
    for ckpt, keep in ((0, False), (8, False), (1, True)):
        P, theta, th, links = setup(lib, L, N, Dk, chi, B, ckpt=ckpt, keep_tape=keep)
        sizes[(ckpt, keep)] = P.workspace_bytes(B) / B
        proj, bid, valid, la, O, _, ws = run_O(P, th, links)
        outs.append(O.cpu().numpy())
        s = (proj * O).sum(dim=2)
        assert torch.max(torch.abs(s - 1.0)).item() < 1e-9   # Euler identity, every site
        del ws
    say("workspace bytes per sample (ckpt, keep_tape):", {k: "%.3g" % v for k, v in sizes.items()})
    assert sizes[(1, True)] > 5 * sizes[(0, False)]
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_z4_32x32_s_row_blocks(lib):
    # S streamed by row blocks at the 32 x 32 shape (937,024 parameters): rows against the
    # oracle's covariance rows on seeded synthetic O (no oracle input from the GPU path)
    from oracle.sr import sr_matrix_rows
    from tests.test_gpu_logderiv import setup, synthetic_sr_inputs
    L, N, Dk, chi, B = 32, 4, 2, 36, 24
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    assert P.n_params == 937024
    lay = Layout(L, N, [Dk] * N)
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B, lib.PEPS_WS_LOGDERIV)
    O, e, Od, eh = synthetic_sr_inputs(P, lay, links.cpu().numpy(), seed=41)
    _, om, _ = P.sr_build(O, bid, valid, e, ws, mode=lib.SR_MATVEC, v=th)
    rows = [(0, 16), (468000, 16), (P.n_params - 8, 8)]
    got = [P.sr_dense_rows(O, bid, valid, om, a, k) for a, k in rows]
    torch.cuda.synchronize()
    for (a, k), g in zip(rows, got):
        want = sr_matrix_rows(Od, np.arange(a, a + k))
        g = g.cpu().numpy()
        assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want)), (a, k)
