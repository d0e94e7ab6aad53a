"""Pins of the oracle's Metropolis sampling with hard-core bosons (SM S-2: plaquette and link
moves; eq. matter: the hopping that a link move proposes).

  * chains of plaquette and link moves are distributed as |Psi|^2 over the whole physical sector
    of 2 bosons on the 3 x 3 Z2 lattice (every state from the exact diagonalisation's basis,
    exact amplitudes), by a chi-square test; the boson number is conserved;
  * with matter, the strip sampler at exact chi is the full-recompute sampler with the same
    counters, move for move (a stale environment or tensor after an accepted hop breaks it).
"""
import numpy as np
import pytest
from scipy import stats

from oracle import ed
from oracle.contract import amplitude
from oracle.energy import paper_tables
from oracle.lattice import is_physical, matter_links
from oracle.layout import Layout, project
from oracle.sampler import link_counter, link_moves, metropolis, metropolis_strip
from paper_2503_20566_amd import synth


def test_link_moves_cover_every_link_once_per_sweep():
    L = 5
    seen = []
    for py in range(L - 1):
        for px, d, x, y in link_moves(L, py):
            assert (d == 0 and x == px) or (d == 1 and x in (px, px + 1))
            seen.append((d, x, y))
    assert len(seen) == len(set(seen)) == 2 * L * (L - 1)
    idx = {link_counter(L, d, x, y) for d, x, y in seen}
    assert idx == set(range((L - 1) ** 2, (L - 1) ** 2 + 2 * L * (L - 1)))


def test_matter_chains_sample_psi_squared():
    L, N, Dk, nb, chains, sweeps = 3, 2, 1, 2, 800, 40   # 10 sweeps do not burn in (p ~ 1e-6)
    c, e = paper_tables(N, 1.0, 0.33)
    _, cfg = ed.physical_basis_matter(L, N, nb)
    lay = Layout(L, N, [Dk] * N, matter=True)
    theta = synth.theta_normals(lay.n_params, N * Dk, seed=19)
    tab = {}
    for s in cfg:
        ok, T, _ = project(lay, theta, s)
        tab[s.tobytes()] = amplitude(T, 64)[0]
    keys = sorted(tab)
    la = np.array([tab[k] for k in keys])
    p = np.exp(2 * (la - la.max()))
    p /= p.sum()
    counts = dict.fromkeys(keys, 0)
    occ = synth.occupations(chains, L, nb, seed=3)
    k = synth.plaquette_powers(chains, L, N, seed=4)
    accepted = 0
    for ch in range(chains):
        s0 = matter_links(k[ch], occ[ch], N)
        s, lf, acc = metropolis(s0, lambda x: tab[x.tobytes()], N, 7, 0, ch, 1, sweeps)
        assert is_physical(s, N) and int(s[2].sum()) == nb and lf == tab[s.tobytes()]
        counts[s.tobytes()] += 1
        accepted += acc
    obs = np.array([counts[kk] for kk in keys], dtype=float)
    exp = p * chains
    order = np.argsort(exp)
    o2, e2, ob, eb = [], [], 0.0, 0.0
    for i in order:                      # cells merged to an expectation of at least 10
        ob += obs[i]
        eb += exp[i]
        if eb >= 10:
            o2.append(ob)
            e2.append(eb)
            ob = eb = 0.0
    if eb > 0:
        o2[-1] += ob
        e2[-1] += eb
    chi2 = float(np.sum((np.array(o2) - np.array(e2)) ** 2 / np.array(e2)))
    pval = 1.0 - stats.chi2.cdf(chi2, len(o2) - 1)
    print("3x3 Z2, 2 bosons: %d states, %d cells, chi2 %.1f, p %.3f, accepted %d" % (len(keys), len(o2), chi2, pval, accepted))
    assert accepted > 0 and pval > 1e-3


@pytest.mark.parametrize("L,N,Dk,nb,chains,sweeps", [(4, 2, 2, 4, 3, 2), (4, 3, 1, 3, 3, 2)])
def test_matter_strip_chain_equals_full_chain_at_exact_chi(L, N, Dk, nb, chains, sweeps):
    lay = Layout(L, N, [Dk] * N, matter=True)
    theta = synth.theta_normals(lay.n_params, N * Dk, seed=23)
    chi = 64

    def log_abs(s):
        ok, T, _ = project(lay, theta, s)
        return amplitude(T, chi)[0] if ok else -np.inf

    occ = synth.occupations(chains, L, nb, seed=5)
    k = synth.plaquette_powers(chains, L, N, seed=6)
    total = 0
    for ch in range(chains):
        s0 = matter_links(k[ch], occ[ch], N)
        want, _, acc_w = metropolis(s0, log_abs, N, 31, 2, ch, 1, sweeps, zigzag=True)
        got, acc_g = metropolis_strip(s0, lay, theta, chi, 31, 2, ch, 1, sweeps)
        assert np.array_equal(got, want), ch
        assert acc_g == acc_w and int(got[2].sum()) == nb
        total += acc_g
    assert total > 0
