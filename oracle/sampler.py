"""Metropolis sampling of link configurations (oracle; test infrastructure only).

Paper passages followed:
  * SM S-2, configuration sampling: a new configuration is proposed by acting with a plaquette
    operator on the current one (which keeps the Gauss law), the plaquettes are visited one after
    the other, and a proposal is accepted when a uniform number falls below |Psi(s')/Psi(s)|^2.
  * VMC section: samples are drawn from |Psi(s)|^2.

The paper fixes neither the random-number generator nor the visiting order.  Reading used here and
by the GPU (stated once):
  * generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
    1, 2, 3", SC'11), key = (seed, stream), counter = (chain, sweep, plaquette, purpose); the first
    64-bit output word x of a counter is the draw; u = (x >> 11) * 2^-53 is a uniform double in
    [0, 1);
  * purposes: 0 = initial plaquette power k_p = x mod N (sweep index 0), 1 = proposal power
    t = 1 + x mod (N - 1), 2 = acceptance uniform;
  * plaquettes p = py * (L - 1) + px visited in that order (row-major from the bottom row);
  * acceptance iff u < exp(2 (ln|Psi(s')| - ln|Psi(s)|)), evaluated in float64.

With matter (SM S-2: links are visited as well, to move the bosons; eq. matter's hopping), a
link move proposes s' = the configuration in which the boson crossed the link (`apply_hop`); a
link whose ends hold equal occupations has no move and draws nothing.  Reading of the order: the
links are grouped by the strip of their ratio window (horizontal links of row py, and of row L-1 in
the last strip; vertical links of row py), and each strip's links are visited right after its
plaquette row, by window column px: the vertical link (px, py), the horizontal link (px, py), the
horizontal link (px, L-1) in the last strip, and at px = L-2 also the vertical link (L-1, py).  This
keeps every move's ratio window to the right of the ones already decided, which is what the strip
sampler's environment reuse needs.  Counter of a link move: (chain, sweep, P + index, 2) with
P = (L-1)^2 plaquettes, index y (L-1) + x for horizontal link (x, y) and L (L-1) + y L + x for
vertical link (x, y).
"""
import numpy as np

from oracle.lattice import apply_hop, apply_plaquette, links_from_powers

_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def philox4x64_10(counter, key):
    """Philox4x64 with 10 rounds, from its published definition.

    One round maps the counter (c0, c1, c2, c3) with key (k0, k1) to
    (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)), where hi/lo are the upper and
    lower 64 bits of the 128-bit product; the key is bumped by the Weyl constants (W0, W1) between
    rounds.  counter: four ints < 2^64; key: two ints < 2^64.  Returns four ints.
    """
    c0, c1, c2, c3 = (int(v) & _MASK for v in counter)
    k0, k1 = (int(v) & _MASK for v in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0) & _MASK, p1 & _MASK, ((p0 >> 64) ^ c3 ^ k1) & _MASK, p0 & _MASK
    return c0, c1, c2, c3


def draw(seed, stream, chain, sweep, plaquette, purpose):
    """The 64-bit draw of one (chain, sweep, plaquette, purpose) counter."""
    return philox4x64_10((chain, sweep, plaquette, purpose), (seed, stream))[0]


def uniform(x):
    """Uniform double in [0, 1) from the top 53 bits of a 64-bit draw."""
    return float(x >> 11) * 2.0 ** -53


def initial_powers(L, N, seed, stream, chain):
    """Initial plaquette powers k_p = x mod N, x the draw of counter (chain, 0, p, 0)."""
    k = np.zeros((L - 1, L - 1), dtype=np.int64)
    for py in range(L - 1):
        for px in range(L - 1):
            k[py, px] = draw(seed, stream, chain, 0, py * (L - 1) + px, 0) % N
    return k


def initial_links(L, N, seed, stream, chain):
    """Initial configuration prod_p P_p^{k_p} |0> of one chain."""
    return links_from_powers(initial_powers(L, N, seed, stream, chain), N)


def strip_order(L, sweep, zigzag):
    """Plaquette rows py in visiting order: ascending, or with zigzag ascending on odd sweep indices
    and descending on even ones."""
    rows = list(range(L - 1))
    return rows if (not zigzag or sweep % 2 == 1) else rows[::-1]


def link_moves(L, py):
    """(window column px, direction d, x, y) of the link moves of strip py, in visiting order."""
    out = []
    for px in range(L - 1):
        out.append((px, 1, px, py))
        out.append((px, 0, px, py))
        if py == L - 2:
            out.append((px, 0, px, L - 1))
        if px == L - 2:
            out.append((px, 1, L - 1, py))
    return out


def link_counter(L, d, x, y):
    """Counter index of the move of link (d, x, y)."""
    P = (L - 1) * (L - 1)
    return P + (y * (L - 1) + x if d == 0 else L * (L - 1) + y * L + x)


def metropolis(links, log_abs, N, seed, stream, chain, first_sweep, n_sweeps, zigzag=False):
    """Metropolis sweeps of one chain (SM S-2 configuration sampling).

    links: uint8 [2, L, L] physical start ([3, L, L] with matter); log_abs: callable mapping a
    configuration to ln|Psi| (float, -inf for Psi = 0).  Sweep w = first_sweep .. first_sweep +
    n_sweeps - 1 visits every plaquette once in row-major order (with zigzag, the plaquette rows in
    the order of `strip_order`), proposes s' = P_p^t s with t = 1 + x mod (N - 1) (purpose 1) and
    accepts iff u < exp(2 (ln|Psi(s')| - ln|Psi(s)|)) with u from purpose 2; with matter, each
    plaquette row is followed by the link moves of its strip (`link_moves`).
    Returns (final links, its ln|Psi|, number of accepted proposals).
    """
    L = links.shape[1]
    matter = links.shape[0] == 3
    s = np.array(links, dtype=np.uint8, copy=True)
    la = log_abs(s)
    accepted = 0
    for w in range(first_sweep, first_sweep + n_sweeps):
        for py in strip_order(L, w, zigzag):
            for px in range(L - 1):
                p = py * (L - 1) + px
                t = 1 + draw(seed, stream, chain, w, p, 1) % (N - 1)
                sp = apply_plaquette(s, px, py, t, N)
                lap = log_abs(sp)
                u = uniform(draw(seed, stream, chain, w, p, 2))
                with np.errstate(invalid="ignore", over="ignore"):
                    ratio = np.exp(2.0 * (lap - la))
                if u < ratio:
                    s, la = sp, lap
                    accepted += 1
            for _, d, x, y in (link_moves(L, py) if matter else []):
                sp = apply_hop(s, d, x, y, N)
                if sp is None:
                    continue
                lap = log_abs(sp)
                u = uniform(draw(seed, stream, chain, w, link_counter(L, d, x, y), 2))
                with np.errstate(invalid="ignore", over="ignore"):
                    ratio = np.exp(2.0 * (lap - la))
                if u < ratio:
                    s, la = sp, lap
                    accepted += 1
    return s, la, accepted


def metropolis_strip(links, layout, theta, chi, seed, stream, chain, first_sweep, n_sweeps, var_sweeps=0):
    """Metropolis sweeps that take each acceptance ratio on the two-row strip of the plaquette,
    reusing the strip's environments (SM S-2 configuration sampling in its finite-PEPS form; the
    strip contraction is that of the local energy, eq. Es).

    Same generator, counters and acceptance rule as `metropolis`, with |Psi(s')/Psi(s)| replaced by
    |Psi_py(s') / Psi_py(s)|, Psi_py the strip amplitude <U_{py+2}| row py+1, row py |D_{py-1}> of
    plaquette p = (px, py), D and U the canonical down and up boundaries of the current
    configuration.  Plaquette rows are visited upwards on odd sweep indices and downwards on even
    ones (`strip_order` with zigzag), px = 0 .. L-2 within a row.  Per strip: the right
    environments F of the current configuration; per plaquette the proposal's ratio from the left
    environment E_px, the proposal's columns px, px+1 (a move changes those two only) and F_{px+2},
    the decision, and E_{px+1} = E_px absorbed through column px after the decision.
    (Here the boundaries are recomputed before every strip; a pass that builds them as it goes
    obtains the same ones, since the rows they cover have not changed since.)
    With matter, the strip's link moves (`link_moves`) follow in a second left-to-right pass: the
    right environments of the configuration after the plaquette pass, then per window column px
    every link move of that window against E_px, and E_{px+1} after the window's decisions.
    When chi is exact the strip ratio is the amplitude ratio and the chain is that of
    `metropolis(..., zigzag=True)` with exact amplitudes.  var_sweeps: boundaries by variational
    compression (oracle/contract.py).  Returns (final links, accepted count).
    """
    from oracle.contract import down_boundaries, up_boundaries
    from oracle.energy import _absorb_left, _absorb_right, _trivial_mps
    from oracle.layout import project

    L, N = layout.L, layout.N
    s = np.array(links, dtype=np.uint8, copy=True)
    accepted = 0

    def tensors(cfg):
        ok, T, _ = project(layout, theta, cfg)
        assert ok
        return T

    for w in range(first_sweep, first_sweep + n_sweeps):
        for py in strip_order(L, w, True):
            T = tensors(s)
            Dm = down_boundaries(T, chi, var_sweeps)[0][py - 1] if py >= 1 else _trivial_mps(L)
            Up = up_boundaries(T, chi, var_sweeps)[py + 2] if py + 2 <= L - 1 else _trivial_mps(L)
            F = [None] * (L + 1)
            F[L] = np.ones((1, 1, 1, 1))
            for c in range(L - 1, -1, -1):
                F[c] = _absorb_right(F[c + 1], Dm[c], T[py][c], T[py + 1][c], Up[c])
            psi = float(F[0].reshape(()))
            E = np.ones((1, 1, 1, 1))
            for px in range(L - 1):
                p = py * (L - 1) + px
                t = 1 + draw(seed, stream, chain, w, p, 1) % (N - 1)
                sp = apply_plaquette(s, px, py, t, N)
                Tp = tensors(sp)
                X = _absorb_left(E, Dm[px], Tp[py][px], Tp[py + 1][px], Up[px])
                X2 = _absorb_left(X, Dm[px + 1], Tp[py][px + 1], Tp[py + 1][px + 1], Up[px + 1])
                num = float(np.einsum("abcd,abcd->", X2, F[px + 2]))
                u = uniform(draw(seed, stream, chain, w, p, 2))
                if psi != 0.0 and u < (num / psi) ** 2:
                    s, T, psi = sp, Tp, num
                    E = X
                    accepted += 1
                else:
                    E = _absorb_left(E, Dm[px], T[py][px], T[py + 1][px], Up[px])
            if s.shape[0] != 3:
                continue
            # link moves of the strip: a second pass against the updated configuration
            for c in range(L - 1, -1, -1):
                F[c] = _absorb_right(F[c + 1], Dm[c], T[py][c], T[py + 1][c], Up[c])
            psi = float(F[0].reshape(()))
            E = np.ones((1, 1, 1, 1))
            moves = link_moves(L, py)
            for px in range(L - 1):
                for wx, d, x, y in moves:
                    if wx != px:
                        continue
                    sp = apply_hop(s, d, x, y, N)
                    if sp is None:
                        continue
                    Tp = tensors(sp)
                    X = _absorb_left(E, Dm[px], Tp[py][px], Tp[py + 1][px], Up[px])
                    X2 = _absorb_left(X, Dm[px + 1], Tp[py][px + 1], Tp[py + 1][px + 1], Up[px + 1])
                    num = float(np.einsum("abcd,abcd->", X2, F[px + 2]))
                    u = uniform(draw(seed, stream, chain, w, link_counter(L, d, x, y), 2))
                    if psi != 0.0 and u < (num / psi) ** 2:
                        s, T, psi = sp, Tp, num
                        accepted += 1
                E = _absorb_left(E, Dm[px], T[py][px], T[py + 1][px], Up[px])
    return s, accepted
