"""GPU parity of the hand-written adjoint (O_k = d ln|Psi| / d theta_k) and of the SR build.

* every element against the oracle's reverse-mode autodiff on small lattices (exact and
  truncating boundary MPS);
* central finite differences (step 1e-6, FP64) of the GPU amplitude on 32 parameters inside the
  selected blocks at the 16 x 16 Z3 chi = 36 shape;
* the Euler identity sum_{k in site} theta_k O_k = 1 (any size, truncation included) on the
  whole 2048-sample batch;
* checkpointed recompute gives the same bits as stored rows;
* sr_build, sr_solve and sr_dense_rows against the oracle's covariances and CG on the same seeded
  synthetic O and E_loc (4 x 4 and the Z3 16 x 16 shape).
"""
import numpy as np
import pytest
import torch

from oracle.energy import config_tables
from oracle.layout import Layout, project
from oracle.logderiv import log_derivatives
from oracle.sr import sr_force_and_mean, sr_matrix, sr_matvec, sr_solve_cg
from paper_2503_20566_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def setup(lib, L, N, Dk, chi, B, seed=5678, ckpt=0, theta=None, keep_tape=False):
    c, e = config_tables(N, 1.0, 0.4)
    P = lib.Peps(L, N, Dk, chi, c, e, ckpt_every=ckpt, keep_tape=keep_tape)
    if theta is None:
        theta = synth.theta_normals(P.n_params, N * Dk)
    powers = synth.plaquette_powers(B, L, N, seed=seed)
    links = P.links_from_powers(torch.from_numpy(powers).cuda())
    th = torch.from_numpy(theta).cuda()
    return P, theta, th, links


def run_O(P, th, links, w=None, want_vjp=False):
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(links.shape[0])
    la, sg = P.amplitude(proj, valid, ws)
    O, vjp = P.logderiv(proj, bid, valid, ws, w=w, want_vjp=want_vjp)
    torch.cuda.synchronize()
    return proj, bid, valid, la, O, vjp, ws


def oracle_O(lay, theta, links, chi):
    ok, T, bid = project(lay, theta, links)
    _, grads = log_derivatives(T, chi)
    return grads


def compare_sample(lay, theta, links_b, O_b, chi, rtol):
    L = lay.L
    grads = oracle_O(lay, theta, links_b, chi)
    worst = 0.0
    scale = max(np.max(np.abs(g)) for row in grads for g in row)
    for y in range(L):
        for x in range(L):
            g = grads[y][x].reshape(-1)
            got = O_b[y * L + x, : g.size]
            err = np.max(np.abs(got - g))
            worst = max(worst, err / scale)
            assert err <= rtol * scale, (y, x, got, g)
            assert not O_b[y * L + x, g.size:].any()
    return worst


# (8, 2, 2, 16) and (10, 2, 2, 16) reach fused bonds of 32 with the full row width of the chi*Dk = 32
# kernels (the staging chunks of their products are sized for it)
@pytest.mark.parametrize("L,N,Dk,chi,B", [(4, 2, 1, 16, 6), (2, 3, 2, 4, 5), (3, 2, 2, 4, 5),
                                          (4, 3, 2, 4, 6), (5, 2, 2, 3, 6), (6, 3, 2, 3, 5),
                                          (6, 4, 2, 5, 4), (7, 2, 2, 6, 3), (8, 2, 2, 16, 3),
                                          (10, 2, 2, 16, 2)])
def test_logderiv_small_every_element(lib, L, N, Dk, chi, B):
    say("logderiv small", L, N, Dk, chi, B)
    P, theta, th, links = setup(lib, L, N, Dk, chi, B, seed=L * 13 + N)
    proj, bid, valid, la, O, _, _ = run_O(P, th, links)
    lay = Layout(L, N, [Dk] * N)
    O, lh = O.cpu().numpy(), links.cpu().numpy()
    worst = max(compare_sample(lay, theta, lh[b], O[b], chi, 1e-9) for b in range(B))
    say("worst rel", worst)


def test_logderiv_full_shape_oracle_sampled(lib):
    say("logderiv 16x16 oracle sample")
    L, N, Dk, chi, B = 16, 3, 2, 36, 2048
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    proj, bid, valid, la, O, _, _ = run_O(P, th, links)
    lay = Layout(L, N, [Dk] * N)
    O, lh = O.cpu().numpy(), links.cpu().numpy()
    for b in (0, 1, 255, 511, 1023, 1024, 2046, B - 1):
        say("sample", b, "worst rel", compare_sample(lay, theta, lh[b], O[b], chi, 1e-8))


@pytest.mark.parametrize("L,N,Dk,chi,B", [(16, 3, 2, 36, 2048), (16, 2, 2, 16, 4096)])
def test_logderiv_full_shape_euler_identity(lib, L, N, Dk, chi, B):
    # Psi is homogeneous of degree one in every site tensor, truncation included:
    # sum over a site's selected entries of proj * O = 1 for every sample and site.
    say("logderiv euler", L, N, Dk, chi, B)
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    proj, bid, valid, la, O, _, _ = run_O(P, th, links)
    s = (proj * O).sum(dim=2)
    assert torch.max(torch.abs(s - 1.0)).item() < 1e-9


def test_logderiv_finite_differences_full_shape(lib):
    # central differences of the GPU amplitude itself, step 1e-6, on 32 parameters of sample 0
    say("logderiv FD 16x16")
    L, N, Dk, chi = 16, 3, 2, 36
    P, theta, th, links = setup(lib, L, N, Dk, chi, 1)
    proj, bid, valid, la, O, _, ws = run_O(P, th, links)
    site_off = P.site_offset
    bidh, Oh = bid.cpu().numpy()[0], O.cpu().numpy()[0]
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(32):
        s = int(rng.integers(0, L * L))
        x, y = s % L, s // L
        npres = (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1)
        bs = Dk ** npres
        e = int(rng.integers(0, bs))
        k = site_off[s] + int(bidh[s]) * bs + e
        vals = []
        for sgn in (1.0, -1.0):
            t2 = th.clone()
            t2[k] += sgn * h
            p2, _, v2 = P.project(t2, links)
            l2, _ = P.amplitude(p2, v2, ws)
            vals.append(l2.item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - Oh[s, e]) <= 1e-6 * max(1.0, abs(Oh[s, e])), (s, e, fd, Oh[s, e])


@pytest.mark.parametrize("L,N,Dk,chi,B", [(10, 3, 2, 8, 64), (16, 3, 2, 36, 64)])
def test_checkpointed_recompute_and_stored_tape_are_bitwise_identical(lib, L, N, Dk, chi, B):
    # recomputing every row (ckpt 0), recomputing from checkpoints (3, 4) and reversing the
    # factorisations the amplitude stored (keep_tape) run the same arithmetic
    say("logderiv checkpoints / stored tape", L, N, Dk, chi, B)
    outs = []
    for ckpt, keep in ((0, False), (3, False), (4, False), (1, True), (0, True)):
        P, theta, th, links = setup(lib, L, N, Dk, chi, B, ckpt=ckpt, keep_tape=keep)
        proj, bid, valid, la, O, _, ws = run_O(P, th, links)
        outs.append(O.cpu().numpy())
        if keep:  # the boundary rows the energy reads are untouched by the reverse sweep
            e_keep = P.local_energy(th, links, proj, valid, ws).cpu().numpy()
            P0, _, _, _ = setup(lib, L, N, Dk, chi, B)
            p0, b0, v0, _, _, _, ws0 = run_O(P0, th, links)
            assert np.array_equal(e_keep, P0.local_energy(th, links, p0, v0, ws0).cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_vjp_and_invalid_samples(lib):
    say("logderiv vjp")
    L, N, Dk, chi, B = 6, 3, 2, 4, 12
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    host = links.cpu().numpy()
    host[4, 0, 2, 2] = (host[4, 0, 2, 2] + 1) % N
    links = torch.from_numpy(host).cuda()
    w = torch.linspace(-1.0, 2.0, B, dtype=torch.float64).cuda()
    proj, bid, valid, la, O, vjp, _ = run_O(P, th, links, w=w, want_vjp=True)
    O, bid, valid, vjp, w = (t.cpu().numpy() for t in (O, bid, valid, vjp, w))
    assert valid[4] == 0 and not O[4].any()
    ref = np.zeros(P.n_params)
    for b in range(B):
        if not valid[b]:
            continue
        for s in range(L * L):
            x, y = s % L, s // L
            bs = Dk ** ((x > 0) + (x < L - 1) + (y > 0) + (y < L - 1))
            off = P.site_offset[s] + bid[b, s] * bs
            ref[off: off + bs] += w[b] * O[b, s, :bs]
    assert np.allclose(vjp, ref, rtol=1e-13, atol=1e-13)


def synthetic_sr_inputs(P, lay, links_host, seed):
    """Seeded synthetic log-derivatives and local energies for the SR parity tests (neither side
    computes them, so the oracle's inputs do not come from the GPU path).  Returns the GPU's
    projected-layout O [B][L*L][Dk^4] and e_loc [B], and the oracle's dense O rows [B][n_params]
    placed through the oracle's own block selection."""
    L, Dk = P.L, P.Dk
    B = links_host.shape[0]
    vals = synth.normals((B, L * L, Dk ** 4), seed)
    e = 10.0 * synth.normals((B,), seed + 1)
    O = np.zeros_like(vals)
    dense = np.zeros((B, lay.n_params))
    for b in range(B):
        ok, _, bid = project(lay, np.zeros(lay.n_params), links_host[b])
        assert ok
        for s in range(L * L):
            x, y = s % L, s // L
            _, shape, off = lay.blocks[s][bid[y, x]]
            bs = int(np.prod(shape))
            O[b, s, :bs] = vals[b, s, :bs]
            dense[b, off: off + bs] = vals[b, s, :bs]
    return torch.from_numpy(O).cuda(), torch.from_numpy(e).cuda(), dense, e


@pytest.mark.parametrize("L,N,Dk,chi,B,dense", [(4, 3, 2, 4, 96, True), (16, 3, 2, 36, 256, False)])
def test_sr_build_matches_oracle(lib, L, N, Dk, chi, B, dense):
    # F, <O> and S v (and the dense S where it fits) against the oracle's covariances on the same
    # seeded synthetic O and E_loc; the Z3 16 x 16 case has 88,752 parameters
    say("sr_build", L, N, Dk, B)
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    lay = Layout(L, N, [Dk] * N)
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B, lib.PEPS_WS_LOGDERIV)
    O, e, Od, eh = synthetic_sr_inputs(P, lay, links.cpu().numpy(), seed=L * 100 + B)
    vh = synth.normals((P.n_params,), 3)
    v = torch.from_numpy(vh).cuda()
    F, om, Sv = P.sr_build(O, bid, valid, e, ws, mode=lib.SR_MATVEC, v=v)
    torch.cuda.synchronize()
    Fr, omr = sr_force_and_mean(Od, eh)
    Svr = sr_matvec(Od, vh)
    for name, got, want in (("F", F, Fr), ("<O>", om, omr), ("S v", Sv, Svr)):
        err = np.max(np.abs(got.cpu().numpy() - want)) / np.max(np.abs(want))
        say("%s max error / max |value| %.2e" % (name, err))
        assert err <= 1e-12, name
    if dense:
        F2, _, S = P.sr_build(O, bid, valid, e, ws, mode=lib.SR_DENSE)
        torch.cuda.synchronize()
        assert np.allclose(S.cpu().numpy(), sr_matrix(Od), rtol=1e-11, atol=1e-12)
        assert np.array_equal(F.cpu().numpy(), F2.cpu().numpy())


def test_autograd_function_is_project_amplitude_and_the_vjp(lib):
    # gipeps.Amplitude: forward = peps_project + peps_amplitude, backward = peps_logderiv's vjp
    # with w = grad_output (the vjp itself is pinned to the oracle above)
    say("autograd Amplitude")
    L, N, Dk, chi, B = 6, 3, 2, 4, 5
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    ws = P.workspace(B)
    t = th.clone().requires_grad_(True)
    la = lib.Amplitude.apply(t, P, links, ws)
    w = torch.linspace(0.5, 2.0, B, dtype=torch.float64, device="cuda")
    (la * w).sum().backward()
    proj, bid, valid = P.project(th, links)
    la2, _ = P.amplitude(proj, valid, ws)
    _, vjp = P.logderiv(proj, bid, valid, ws, w=w, want_vjp=True)
    torch.cuda.synchronize()
    assert torch.equal(la.detach(), la2)
    assert torch.equal(t.grad, vjp)


def test_sr_solve_matches_oracle(lib):
    # CG on (S + shift I) x = F: against the oracle's CG and a dense library solve on the same
    # seeded synthetic O and E_loc
    say("sr_solve small")
    L, N, Dk, chi, B = 4, 3, 2, 4, 96
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    lay = Layout(L, N, [Dk] * N)
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B, lib.PEPS_WS_LOGDERIV)
    O, e, Od, eh = synthetic_sr_inputs(P, lay, links.cpu().numpy(), seed=11)
    shift = 1e-2
    x, F, om, it, rel = P.sr_solve(O, bid, valid, e, ws, shift, 2000, 1e-12)
    x2, _, _, it2, rel2 = P.sr_solve(O, bid, valid, e, ws, shift, 2000, 1e-12)
    torch.cuda.synchronize()
    assert torch.equal(x, x2) and it == it2 and rel == rel2  # fixed-order reductions
    Fr, _ = sr_force_and_mean(Od, eh)
    xo, ito, relo = sr_solve_cg(Od, eh, shift, 2000, 1e-12)
    want = np.linalg.solve(sr_matrix(Od) + shift * np.eye(P.n_params), Fr)
    xh = x.cpu().numpy()
    say("iterations gpu", it, "oracle", ito, "rel", rel, relo)
    assert rel <= 1e-12 and 0 < it < 2000 and relo <= 1e-12  # both converge (paths differ by rounding)
    assert np.allclose(xh, xo, rtol=1e-7, atol=1e-9 * np.abs(xo).max())
    assert np.allclose(xh, want, rtol=1e-7, atol=1e-9 * np.abs(want).max())
    assert np.allclose(F.cpu().numpy(), Fr, rtol=1e-12, atol=1e-12)


def test_sr_solve_full_shape_residual(lib):
    # Z3 16x16 chi = 36: the reported relative residual equals the one recomputed from an
    # independent S v call (sr_build), and the stopping rule holds
    say("sr_solve 16x16")
    L, N, Dk, chi, B = 16, 3, 2, 36, 2048
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    proj, bid, valid, la, O, _, ws = run_O(P, th, links)
    e = P.local_energy(th, links, proj, valid, ws)
    shift, rtol, max_iter = 1e-3, 1e-5, 400
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    x, F, om, it, rel = P.sr_solve(O, bid, valid, e, ws, shift, max_iter, rtol)
    t1.record()
    torch.cuda.synchronize()
    say("iterations", it, "rel", rel, "ms per iteration %.2f" % (t0.elapsed_time(t1) / max(it, 1)))
    _, _, Sx = P.sr_build(O, bid, valid, e, ws, mode=lib.SR_MATVEC, v=x)
    r = F - (Sx + shift * x)
    rel2 = float(torch.linalg.norm(r) / torch.linalg.norm(F))
    say("recomputed", rel2)
    assert rel <= rtol or it == max_iter
    assert abs(rel2 - rel) <= 1e-6 * max(rel, 1e-12) + 1e-13


def test_sr_dense_rows_are_the_dense_mode_rows(lib):
    # row blocks of S (any parameter count): bitwise the rows of sr_build's dense mode, in ragged
    # blocks that cover every row
    say("sr_dense_rows small")
    L, N, Dk, chi, B = 4, 3, 2, 4, 80
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    proj, bid, valid, la, O, _, ws = run_O(P, th, links)
    e = P.local_energy(th, links, proj, valid, ws)
    _, om, S = P.sr_build(O, bid, valid, e, ws, mode=lib.SR_DENSE)
    n = P.n_params
    cuts = [0, 7, 100, n // 2, n - 3, n]
    blocks = [P.sr_dense_rows(O, bid, valid, om, a, b - a) for a, b in zip(cuts[:-1], cuts[1:])]
    torch.cuda.synchronize()
    assert torch.equal(torch.cat(blocks), S)


def test_sr_dense_rows_full_shape(lib):
    # the Z3 16 x 16 chi = 36 shape (88,752 parameters, beyond the dense mode): rows against the
    # oracle's covariance rows on seeded synthetic O
    from oracle.sr import sr_matrix_rows
    say("sr_dense_rows full shape")
    L, N, Dk, chi, B = 16, 3, 2, 36, 48
    P, theta, th, links = setup(lib, L, N, Dk, chi, B)
    lay = Layout(L, N, [Dk] * N)
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B, lib.PEPS_WS_LOGDERIV)
    O, e, Od, eh = synthetic_sr_inputs(P, lay, links.cpu().numpy(), seed=21)
    _, om, _ = P.sr_build(O, bid, valid, e, ws, mode=lib.SR_MATVEC, v=th)
    rows = [(0, 40), (44000, 64), (P.n_params - 24, 24)]
    got = [P.sr_dense_rows(O, bid, valid, om, a, k) for a, k in rows]
    torch.cuda.synchronize()
    for (a, k), g in zip(rows, got):
        want = sr_matrix_rows(Od, np.arange(a, a + k))
        g = g.cpu().numpy()
        scale = np.max(np.abs(want))
        assert np.max(np.abs(g - want)) <= 1e-12 * scale, (a, k)
