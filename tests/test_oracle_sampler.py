"""Pins of the oracle's Metropolis sampler (SM S-2 configuration sampling) and of its counter-based
generator: the generator against numpy's Philox4x64-10 bit generator (a library routine), the
chain's stationary distribution against the exact |Psi|^2 / sum |Psi|^2 on lattices small enough to
enumerate (chi-square test), plus structural properties."""
import numpy as np
import pytest
from scipy import stats

from oracle.contract import amplitude
from oracle.lattice import apply_plaquette, enumerate_physical, is_physical
from oracle.layout import project
from oracle.sampler import (draw, initial_links, initial_powers, metropolis, philox4x64_10,
                            uniform)
from tests.helpers import make_problem


def test_philox_matches_numpy_bit_generator():
    # numpy's Philox increments its 256-bit counter before generating, so its first four raw
    # outputs for counter c are philox4x64_10(c + 1); the cases include carries between words
    rng = np.random.default_rng(7)
    cases = [((0, 0, 0, 0), (5, 7)), ((2**64 - 1, 5, 0, 9), (2**64 - 1, 3)),
             ((2**64 - 1, 2**64 - 1, 3, 0), (0, 0))]
    for _ in range(20):
        cases.append((tuple(int(v) for v in rng.integers(0, 2**63, 4, dtype=np.int64)),
                      tuple(int(v) for v in rng.integers(0, 2**63, 2, dtype=np.int64))))
    for ctr, key in cases:
        bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
        want = [int(v) for v in bg.random_raw(4)]
        c = sum(int(v) << (64 * i) for i, v in enumerate(ctr)) + 1
        nxt = tuple((c >> (64 * i)) & (2**64 - 1) for i in range(4))
        assert list(philox4x64_10(nxt, key)) == want, (ctr, key)


def test_uniform_range():
    assert uniform(0) == 0.0
    assert uniform(2**64 - 1) == 1.0 - 2.0**-53
    assert uniform(1 << 11) == 2.0**-53


@pytest.mark.parametrize("N", [2, 3, 4])
def test_initial_state_physical_and_powers_in_range(N):
    L = 5
    for chain in range(6):
        k = initial_powers(L, N, 5678, 0, chain)
        assert k.min() >= 0 and k.max() < N
        assert is_physical(initial_links(L, N, 5678, 0, chain), N)
    # draws depend on every counter word and on the key
    base = draw(5678, 0, 3, 2, 1, 1)
    assert len({base, draw(5678, 0, 4, 2, 1, 1), draw(5678, 0, 3, 3, 1, 1), draw(5678, 0, 3, 2, 2, 1),
                draw(5678, 0, 3, 2, 1, 2), draw(5679, 0, 3, 2, 1, 1), draw(5678, 1, 3, 2, 1, 1)}) == 7


def _table(L, N, Dk, chi):
    """Exact ln|Psi| of every physical configuration (oracle amplitude; chi exact here)."""
    lay, theta = make_problem(L, N, Dk, seed=11)
    tab = {}
    for s in enumerate_physical(L, N):
        ok, T, _ = project(lay, theta, s)
        tab[s.tobytes()] = amplitude(T, chi)[0]
    return tab


def _chi2_pvalue(L, N, Dk, chains, sweeps):
    tab = _table(L, N, Dk, 64)
    keys = sorted(tab)
    la = np.array([tab[k] for k in keys])
    p = np.exp(2 * (la - la.max()))
    p /= p.sum()
    counts = dict.fromkeys(keys, 0)
    accepted = 0
    for c in range(chains):
        s0 = initial_links(L, N, 99, 0, c)
        s, lf, acc = metropolis(s0, lambda x: tab[x.tobytes()], N, 99, 0, c, 1, sweeps)
        assert is_physical(s, N) and lf == tab[s.tobytes()]
        counts[s.tobytes()] += 1
        accepted += acc
    obs = np.array([counts[k] for k in keys], dtype=float)
    exp = p * chains
    # merge cells with small expectation so the chi-square approximation holds
    order = np.argsort(exp)
    o2, e2, ob, eb = [], [], 0.0, 0.0
    for i in order:
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
    return 1.0 - stats.chi2.cdf(chi2, len(o2) - 1), accepted


@pytest.mark.parametrize("L,N,Dk,chains,sweeps", [(2, 3, 2, 1500, 12), (3, 2, 1, 1500, 15)])
def test_chain_samples_psi_squared(L, N, Dk, chains, sweeps):
    # SM S-2 / VMC section: the chain's states are distributed as |Psi|^2 (exact amplitudes of every
    # physical state on an enumerable lattice); fixed seeds, so the test is deterministic
    pval, accepted = _chi2_pvalue(L, N, Dk, chains, sweeps)
    assert accepted > 0
    assert pval > 1e-3, pval


def test_chain_detects_a_wrong_target():
    # the chi-square test has power: sampling |Psi|^4 instead of |Psi|^2 fails it
    L, N, Dk, chains, sweeps = 3, 2, 1, 1500, 15
    tab = _table(L, N, Dk, 64)
    keys = sorted(tab)
    la = np.array([tab[k] for k in keys])
    p = np.exp(2 * (la - la.max()))
    p /= p.sum()
    counts = dict.fromkeys(keys, 0)
    for c in range(chains):
        s, _, _ = metropolis(initial_links(L, N, 99, 0, c), lambda x: 2 * tab[x.tobytes()], N, 99, 0, c,
                             1, sweeps)
        counts[s.tobytes()] += 1
    obs = np.array([counts[k] for k in keys], dtype=float)
    chi2 = float(np.sum((obs - p * chains) ** 2 / (p * chains)))
    assert 1.0 - stats.chi2.cdf(chi2, len(keys) - 1) < 1e-6


def test_metropolis_keeps_state_on_rejection_and_is_deterministic():
    L, N = 3, 3
    s0 = initial_links(L, N, 5, 1, 2)
    # target with Psi(s') = 0 for every s' != s0: nothing is ever accepted
    never = metropolis(s0, lambda x: 0.0 if np.array_equal(x, s0) else -np.inf, N, 5, 1, 2, 1, 3)
    assert np.array_equal(never[0], s0) and never[2] == 0
    # flat target: every proposal is accepted (u < 1), so the state is the product of all moves
    s, _, acc = metropolis(s0, lambda x: 0.0, N, 5, 1, 2, 1, 2)
    assert acc == 2 * (L - 1) ** 2
    want = s0
    for w in (1, 2):
        for py in range(L - 1):
            for px in range(L - 1):
                t = 1 + draw(5, 1, 2, w, py * (L - 1) + px, 1) % (N - 1)
                want = apply_plaquette(want, px, py, t, N)
    assert np.array_equal(s, want)
    again = metropolis(s0, lambda x: float(x.sum()) * 0.1, N, 5, 1, 2, 1, 2)
    once = metropolis(s0, lambda x: float(x.sum()) * 0.1, N, 5, 1, 2, 1, 2)
    assert np.array_equal(again[0], once[0]) and again[2] == once[2]


@pytest.mark.parametrize("L,N,Dk,chains,sweeps", [(3, 2, 1, 6, 3), (3, 3, 2, 4, 2), (4, 2, 2, 3, 2),
                                                  (5, 2, 2, 2, 2), (4, 3, 2, 3, 2), (2, 4, 2, 5, 3)])
def test_strip_chain_equals_exact_chain_when_chi_is_exact(L, N, Dk, chains, sweeps):
    # With chi exact the strip ratio Psi_py(s')/Psi_py(s) is the amplitude ratio, so the strip
    # sampler must take every decision of the plain sampler (same zig-zag order) fed with exact
    # amplitudes (the
    # boundary-MPS amplitude at a chi above every bond, itself pinned to the plain contraction).
    # D_k = 2 with L >= 4 makes the boundaries carry information: a wrong boundary row, stale
    # tensors after an acceptance or a stale strip amplitude each break the chains; two or more
    # sweeps cover both directions.
    from oracle.sampler import metropolis_strip
    lay, theta = make_problem(L, N, Dk, seed=17)
    chi = 64

    def log_abs(s):
        ok, T, _ = project(lay, theta, s)
        return amplitude(T, chi)[0] if ok else -np.inf

    total = 0
    for c in range(chains):
        s0 = initial_links(L, N, 31, 2, c)
        want, _, acc_w = metropolis(s0, log_abs, N, 31, 2, c, 1, sweeps, zigzag=True)
        got, acc_g = metropolis_strip(s0, lay, theta, chi, 31, 2, c, 1, sweeps)
        assert np.array_equal(got, want), c
        assert acc_g == acc_w
        total += acc_g
    assert total > 0


def test_strip_chain_truncating_stays_physical_and_depends_on_chi():
    # under truncation the strip chain is its own sampler: physical states, deterministic, and
    # (for this seed) a different path from the exact-chi chain of the same counters
    from oracle.sampler import metropolis_strip
    L, N, Dk = 5, 3, 2
    lay, theta = make_problem(L, N, Dk, seed=23)
    s0 = initial_links(L, N, 77, 0, 1)
    a, na = metropolis_strip(s0, lay, theta, 2, 77, 0, 1, 1, 2)
    b, nb = metropolis_strip(s0, lay, theta, 2, 77, 0, 1, 1, 2)
    c, nc = metropolis_strip(s0, lay, theta, 64, 77, 0, 1, 1, 2)
    assert np.array_equal(a, b) and na == nb
    assert is_physical(a, N) and na > 0
    assert not np.array_equal(a, c)
