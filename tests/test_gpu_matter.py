"""GPU parity with hard-core bosons on the vertices (eq. matter, eq. gauss_N and eq. A with p).

Matter enters the configuration (an occupation plane), the block tables (a p = 1 group of blocks
per site), the projection's Gauss check and block choice, and the local energy (mass term and one
hopping ratio per link whose ends differ in occupation); the contraction and the adjoint work on
the selected blocks unchanged.

* configurations built around seeded occupations: bit-exact against the oracle's builder;
* small lattices, every sample: block ids, valid flags, ln|Psi| and sign, E_loc (with its scale
  M) and every log-derivative element against the oracle, exact and truncating boundary MPS;
* unphysical occupations (a boson moved without its flux, an occupation of 2, a boson count the
  charges forbid) are zero-amplitude data;
* Z2 16 x 16 at half filling (128 bosons), D_k = 2, chi = 24: sampled ln|Psi|, E_loc and O against
  the oracle, the per-site Euler identity on the whole batch;
* Metropolis chains with plaquette and link moves (full-recompute and strip samplers, the latter
  also on the chi * Dk = 72 kernels) are the oracle's chains move for move, conserve the boson
  number, and agree with each other at exact chi.
"""
import numpy as np
import pytest
import torch

from oracle.contract import amplitude
from oracle.energy import local_energy, paper_tables
from oracle.lattice import is_physical, matter_links
from oracle.layout import Layout, project
from oracle.logderiv import log_derivatives
from paper_2503_20566_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def setup(lib, L, N, Dk, chi, B, nb, hop=0.5, mass=0.3, h_p=1.0, g=0.33, seed=31):
    c, e = paper_tables(N, h_p, g)
    P = lib.Peps(L, N, Dk, chi, c, e, matter=True, hop=hop, mass=mass)
    lay = Layout(L, N, [Dk] * N, matter=True)
    assert P.n_params == lay.n_params and P.site_offset == lay.site_offset
    theta = synth.theta_normals(P.n_params, N * Dk, seed=L * 5 + N)
    powers = synth.plaquette_powers(B, L, N, seed=seed)
    occ = synth.occupations(B, L, nb, seed=seed + 1)
    links = P.matter_links(torch.from_numpy(powers).cuda(), torch.from_numpy(occ).cuda())
    torch.cuda.synchronize()
    return P, lay, theta, links, (powers, occ), dict(c_tab=c, e_tab=e, hop=hop, mass=mass)


def run(P, theta, links, want_O=True):
    B = links.shape[0]
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B)
    la, sg = P.amplitude(proj, valid, ws)
    el = P.local_energy(th, links, proj, valid, ws)
    m = P.eloc_scale(B, ws)
    O = P.logderiv(proj, bid, valid, ws)[0] if want_O else None
    torch.cuda.synchronize()
    host = lambda t: None if t is None else t.cpu().numpy()  # noqa: E731
    return dict(bid=host(bid), valid=host(valid), la=host(la), sg=host(sg), el=host(el), m=host(m), O=host(O))


def check_sample(lay, theta, s, chi, ham, r, b, rtol=1e-10):
    L = lay.L
    ok, T, obid = project(lay, theta, s)
    assert ok and r["valid"][b] == 1
    assert np.array_equal(r["bid"][b].reshape(L, L), obid)
    ola, osg = amplitude(T, chi)
    assert abs(r["la"][b] - ola) <= rtol * max(1.0, abs(ola)) and r["sg"][b] == osg, (b, r["la"][b], ola)
    oel, om = local_energy(lay, theta, s, chi, ham["c_tab"], ham["e_tab"], with_scale=True,
                           hop=ham["hop"], mass=ham["mass"])
    assert abs(r["el"][b] - oel) <= rtol * om and abs(r["m"][b] - om) <= rtol * om, (b, r["el"][b], oel)
    if r["O"] is None:
        return
    _, grads = log_derivatives(T, chi)
    scale = max(np.max(np.abs(gr)) for row in grads for gr in row)
    for y in range(L):
        for x in range(L):
            gr = grads[y][x].reshape(-1)
            got = r["O"][b, y * L + x]
            assert np.max(np.abs(got[: gr.size] - gr)) <= 10 * rtol * scale and not got[gr.size:].any(), (b, y, x)


@pytest.mark.parametrize("L,N,nb", [(5, 2, 6), (6, 3, 9), (4, 4, 8), (7, 2, 0)])
def test_matter_links_bit_exact(lib, L, N, nb):
    say("matter links", L, N, nb)
    B = 16
    P, lay, theta, links, (powers, occ), _ = setup(lib, L, N, 1, 4, B, nb)
    got = links.cpu().numpy()
    for b in range(B):
        want = matter_links(powers[b], occ[b], N)
        assert np.array_equal(got[b], want), b
        assert is_physical(want, N)


@pytest.mark.parametrize("L,N,Dk,chi,B,nb,hop,mass", [
    (4, 2, 2, 16, 8, 4, 0.5, 0.3),      # exact chi
    (6, 2, 2, 4, 6, 8, 0.5, 0.0),       # truncating
    (5, 3, 2, 6, 5, 6, -0.7, 0.2),      # Z3, negative hopping
    (4, 4, 1, 8, 6, 4, 0.9, -1.1),      # Z4, D_k = 1
    (6, 2, 1, 4, 4, 18, 0.5, 0.3)])     # half filling
def test_matter_small_every_element(lib, L, N, Dk, chi, B, nb, hop, mass):
    say("matter small", L, N, Dk, chi, B, nb, hop, mass)
    P, lay, theta, links, _, ham = setup(lib, L, N, Dk, chi, B, nb, hop=hop, mass=mass)
    r = run(P, theta, links)
    lh = links.cpu().numpy()
    assert r["valid"].all()
    for b in range(B):
        check_sample(lay, theta, lh[b], chi, ham, r, b)


def test_unphysical_occupations_are_zero_amplitude(lib):
    say("matter unphysical")
    L, N, Dk, chi, B = 4, 3, 2, 6, 6
    P, lay, theta, links, _, ham = setup(lib, L, N, Dk, chi, B, 3)
    lh = links.cpu().numpy().copy()
    lh[3, 2] = 0
    lh[3, 2, 1, 1] = 1                 # one boson where the flux expects none (and none elsewhere)
    lh[4, 2, 0, 0] = 2                 # not a hard-core occupation
    occ5 = np.zeros((1, L, L), dtype=np.uint8)
    occ5[0, 0, :2] = 1                 # two bosons: the Z3 charge sum forbids it
    lh[5] = P.matter_links(torch.from_numpy(synth.plaquette_powers(1, L, N)).cuda(),
                           torch.from_numpy(occ5).cuda()).cpu().numpy()[0]
    r = run(P, theta, torch.from_numpy(lh).cuda(), want_O=False)
    assert r["valid"].tolist() == [1, 1, 1, 0, 0, 0]
    assert np.all(np.isneginf(r["la"][3:])) and np.all(r["sg"][3:] == 0) and np.all(np.isnan(r["el"][3:]))
    for b in range(3, 6):
        assert not project(lay, theta, lh[b])[0]
    for b in range(3):
        check_sample(lay, theta, lh[b], chi, ham, r, b)


def test_z2_16x16_half_filling(lib):
    say("matter z2 16x16 half filling")
    L, N, Dk, chi, B = 16, 2, 2, 24, 64
    P, lay, theta, links, _, ham = setup(lib, L, N, Dk, chi, B, L * L // 2, hop=0.5, mass=0.0)
    th = torch.from_numpy(theta).cuda()
    proj, bid, valid = P.project(th, links)
    ws = P.workspace(B)
    la, sg = P.amplitude(proj, valid, ws)
    el = P.local_energy(th, links, proj, valid, ws)
    m = P.eloc_scale(B, ws)
    O, _ = P.logderiv(proj, bid, valid, ws)
    euler = (O * proj).sum(dim=2)  # sum over one site's selected block of theta_k O_k
    torch.cuda.synchronize()
    assert bool(valid.all())
    assert torch.max(torch.abs(euler - 1.0)).item() < 1e-9
    r = dict(bid=bid.cpu().numpy(), valid=valid.cpu().numpy(), la=la.cpu().numpy(), sg=sg.cpu().numpy(),
             el=el.cpu().numpy(), m=m.cpu().numpy(), O=O.cpu().numpy())
    lh = links.cpu().numpy()
    for b in (0, B // 2, B - 1):
        say("sample", b)
        check_sample(lay, theta, lh[b], chi, ham, r, b, rtol=1e-9)


def _oracle_log_abs(lay, theta, chi):
    def f(s):
        ok, T, _ = project(lay, theta, s)
        return amplitude(T, chi)[0] if ok else -np.inf
    return f


def _chains(lib, L, N, Dk, chi, B, nb, seed=41):
    P, lay, theta, links, _, _ = setup(lib, L, N, Dk, chi, B, nb, seed=seed)
    return P, lay, theta, links


@pytest.mark.parametrize("L,N,Dk,chi,B,nb,sweeps", [(4, 2, 1, 16, 8, 4, 2), (4, 3, 2, 3, 6, 3, 1),
                                                    (5, 2, 2, 3, 5, 6, 1)])
def test_matter_chains_match_oracle(lib, L, N, Dk, chi, B, nb, sweeps):
    # full-recompute sampler: plaquette rows, each followed by its strip's link moves
    from oracle.sampler import metropolis
    say("matter metropolis parity", L, N, Dk, chi, B, nb, sweeps)
    P, lay, theta, links = _chains(lib, L, N, Dk, chi, B, nb)
    start = links.cpu().numpy()
    seed, stream = 77, 5
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_SAMPLE)
    la, acc = P.metropolis(torch.from_numpy(theta).cuda(), links, seed, 1, sweeps, ws, stream_id=stream)
    torch.cuda.synchronize()
    got, la, acc = links.cpu().numpy(), la.cpu().numpy(), acc.cpu().numpy()
    f = _oracle_log_abs(lay, theta, chi)
    for b in range(B):
        s, lf, a = metropolis(start[b], f, N, seed, stream, b, 1, sweeps)
        assert np.array_equal(got[b], s), b
        assert a == acc[b] and int(got[b, 2].sum()) == nb
        assert abs(la[b] - lf) <= 1e-10 * max(1.0, abs(lf))
    assert acc.sum() > 0


# (10, 3, 2, 20, 3, 48, 2): fused bonds up to chi * Dk = 40 on the kernels built for 72 (the
# benchmark's), one pass in each direction
@pytest.mark.parametrize("L,N,Dk,chi,B,nb,sweeps", [(4, 2, 2, 4, 8, 4, 2), (5, 3, 2, 3, 6, 6, 2),
                                                    (6, 2, 1, 4, 6, 18, 2), (10, 3, 2, 20, 3, 48, 2)])
def test_matter_strip_chains_match_oracle(lib, L, N, Dk, chi, B, nb, sweeps):
    from oracle.sampler import metropolis_strip
    say("matter strip metropolis parity", L, N, Dk, chi, B, nb, sweeps)
    P, lay, theta, links = _chains(lib, L, N, Dk, chi, B, nb)
    start = links.cpu().numpy()
    seed, stream = 4243, 1
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_ENERGY)
    la, acc = P.metropolis_strip(torch.from_numpy(theta).cuda(), links, seed, 1, sweeps, ws, stream_id=stream)
    torch.cuda.synchronize()
    got, la, acc = links.cpu().numpy(), la.cpu().numpy(), acc.cpu().numpy()
    f = _oracle_log_abs(lay, theta, chi)
    for b in range(B):
        s, a = metropolis_strip(start[b], lay, theta, chi, seed, stream, b, 1, sweeps)
        assert np.array_equal(got[b], s), b
        assert a == acc[b], (b, a, acc[b])
        assert int(got[b, 2].sum()) == nb and is_physical(got[b], N)
        lf = f(s)
        assert abs(la[b] - lf) <= 1e-10 * max(1.0, abs(lf)), (b, la[b], lf)
    assert acc.sum() > 0


def test_matter_strip_chains_equal_plain_chains_when_chi_is_exact(lib):
    say("matter strip vs plain sampler, exact chi")
    L, N, Dk, chi, B = 4, 2, 2, 16, 10
    P, lay, theta, a = _chains(lib, L, N, Dk, chi, B, 6)
    th = torch.from_numpy(theta).cuda()
    b = a.clone()
    ws = P.workspace(B, lib.PEPS_WS_AMPLITUDE | lib.PEPS_WS_ENERGY | lib.PEPS_WS_SAMPLE)
    la_a, acc_a = P.metropolis(th, a, 9, 1, 1, ws, stream_id=1)   # sweep 1: strips upwards, as plain
    la_b, acc_b = P.metropolis_strip(th, b, 9, 1, 1, ws, stream_id=1)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(acc_a, acc_b) and acc_a.sum().item() > 0
    assert torch.max(torch.abs(la_a - la_b)).item() <= 1e-10 * torch.max(torch.abs(la_a)).item()


def test_matter_sample_init_is_refused(lib):
    P, lay, theta, links, _, _ = setup(lib, 4, 2, 1, 4, 2, 2)
    with pytest.raises(lib.PepsError) as err:
        P.sample_init(2, 1)
    assert err.value.status == lib.PEPS_ERR_UNSUPPORTED
