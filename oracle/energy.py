"""Hamiltonian tables and the local energy (oracle; test infrastructure only).

Paper passages followed:
  * eq. H_b: the magnetic term is a sum over plaquettes of the plaquette operator plus its
    Hermitian conjugate; eq. electric: H_E = g sum_l (2 - 2 cos(2 pi E_l / N)) for Z_N.
  * SM S-1 eq. Es: E_loc(s) = sum_{s'} <s|H|s'> Psi(s') / Psi(s).
  * SM S-2: plaquette moves P_p^t keep a configuration physical.
  * eq. matter: with hard-core bosons, sum_x m_x p_x plus the hopping c^dag_x U c_(x+e) + h.c. with
    coupling J (uniform m_x here); each hopping term connects s to at most one s' (apply_hop).

Tables.  H = sum_p sum_{t=1}^{N-1} c[t] P_p^t + sum_l e[n_l], with c real and c[t] = c[N-t]
(Hermitian) and e diagonal in the electric basis.  Two presets:
  * config convention "-J sum_p plaquette - h sum_l electric":
      Z2:  c[1] = -J,               e[n] = -h (-1)^n
      ZN:  c[1] = c[N-1] = -J,      e[n] = -2 h cos(2 pi n / N)
  * paper convention (eq. H_b and eq. electric, plaquette coupling h_p, electric coupling g):
      Z2:  c[1] = -2 h_p,           e[n] = g (2 - 2 cos(pi n))
      ZN:  c[1] = c[N-1] = -h_p,    e[n] = g (2 - 2 cos(2 pi n / N))
(For Z2, P_p = P_p^dag, so "P + h.c." doubles the single term.)

Local energy.  <s|P_p^t|s'> = 1 exactly when s' = P_p^{-t} s, so
    E_loc(s) = sum_l e[n_l(s)] + sum_p sum_t c[t] Psi(P_p^{-t} s) / Psi(s).
For the boundary-MPS amplitude the ratio of plaquette p = (px, py) is taken, as in finite-PEPS
VMC, over the two-row strip (py, py+1) contracted exactly between the configuration's own down
environment D_{py-1} and up environment U_{py+2}; both configurations share these environments
because a plaquette move only changes links inside the strip.
"""
import math

import numpy as np

from .contract import down_boundaries, up_boundaries
from .lattice import apply_hop, apply_plaquette, link_mask
from .layout import project


def config_tables(N, J, h):
    c = np.zeros(N)
    e = np.zeros(N)
    if N == 2:
        c[1] = -J
        e[:] = [-h, h]
    else:
        c[1] = c[N - 1] = -J
        e[:] = [-2.0 * h * math.cos(2.0 * math.pi * n / N) for n in range(N)]
    return c, e


def paper_tables(N, h_p, g):
    c = np.zeros(N)
    if N == 2:
        c[1] = -2.0 * h_p
    else:
        c[1] = c[N - 1] = -h_p
    e = np.array([g * (2.0 - 2.0 * math.cos(2.0 * math.pi * n / N)) for n in range(N)])
    return c, e


def electric_energy(links, e):
    """Diagonal part sum_l e[n_l] over the real links only."""
    m = link_mask(links.shape[-1])
    return float(np.sum(np.asarray(e)[links[:2][m].astype(np.int64)]))


def electric_magnitude(links, e):
    """sum_l |e[n_l]| over the real links (the electric part of the local-energy scale)."""
    m = link_mask(links.shape[-1])
    return float(np.sum(np.abs(np.asarray(e))[links[:2][m].astype(np.int64)]))


def _trivial_mps(L):
    return [np.ones((1, 1, 1)) for _ in range(L)]


def _absorb_left(E, D, T, Tp, U):
    """E[a,l,l',b] -> E[a',r,r',b'] through one column: boundary D below, rows T (lower) and
    Tp (upper) sharing the vertical bond u, boundary U above.  Pairwise contractions in a fixed
    order (the value is that of the five-tensor contraction)."""
    X = np.einsum("aklb,adc->klbdc", E, D)
    X = np.einsum("klbdc,kmdu->lbcmu", X, T)
    X = np.einsum("lbcmu,lnuv->bcmnv", X, Tp)
    return np.einsum("bcmnv,bve->cmne", X, U)


def _absorb_right(F, D, T, Tp, U):
    X = np.einsum("cmne,bve->cmnbv", F, U)
    X = np.einsum("cmnbv,lnuv->cmblu", X, Tp)
    X = np.einsum("cmblu,kmdu->cblkd", X, T)
    return np.einsum("cblkd,adc->aklb", X, D)


def strip_environments(Dm, row_lo, row_hi, Up):
    """Left and right environments of a two-row strip; E[0] and F[L] are trivial.

    Dm: boundary MPS below the strip (physical legs = row_lo's d legs), Up: boundary MPS above it
    (physical legs = row_hi's u legs).  Returns (E, F) with E[c] covering columns < c and F[c]
    columns >= c.
    """
    L = len(row_lo)
    E = [np.ones((1, 1, 1, 1))]
    for c in range(L):
        E.append(_absorb_left(E[-1], Dm[c], row_lo[c], row_hi[c], Up[c]))
    F = [None] * (L + 1)
    F[L] = np.ones((1, 1, 1, 1))
    for c in range(L - 1, -1, -1):
        F[c] = _absorb_right(F[c + 1], Dm[c], row_lo[c], row_hi[c], Up[c])
    return E, F


def hop_window(L, d, x, y):
    """Strip py and window px (columns px, px+1 of rows py, py+1) that hold both ends of link
    (d, x, y): a horizontal link of row y sits in strip min(y, L-2), a vertical link (x, y)-(x, y+1)
    in strip y with window min(x, L-2)."""
    if d == 0:
        return min(y, L - 2), x
    return y, min(x, L - 2)


def local_energy(layout, theta, links, chi, c_tab, e_tab, with_scale=False, hop=0.0, mass=0.0, var_sweeps=0):
    """E_loc(s) of SM S-1 eq. Es with the strip amplitude ratios described above.

    With matter (layout.matter; eq. matter with uniform m_x = mass and coupling J = hop): the
    diagonal mass * sum_x p_x, and for every link whose two ends differ in occupation the term
    hop * Psi(s') / Psi(s), s' = apply_hop(s), the ratio taken on the strip and window of
    hop_window (both ends lie inside them, so s and s' share that strip's environments).

    var_sweeps > 0: boundaries by variational compression (oracle/contract.py).
    Returns NaN for a configuration with zero amplitude.  with_scale: return (E_loc, M) where
    M = sum of the magnitudes of the terms that E_loc adds up (|e[n_l]|, |mass p_x|, each
    |coefficient * ratio|; |E_loc| <= M); (NaN, NaN) for a zero amplitude.
    """
    L, N = layout.L, layout.N
    valid, T, _ = project(layout, theta, links)
    if not valid:
        return (math.nan, math.nan) if with_scale else math.nan
    D, _ = down_boundaries(T, chi, var_sweeps)
    Uenv = up_boundaries(T, chi, var_sweeps)
    hops = {py: [] for py in range(L - 1)}
    if layout.matter and hop != 0.0:
        for d, y, x in zip(*np.nonzero(link_mask(L))):
            s2 = apply_hop(links, int(d), int(x), int(y), N)
            if s2 is not None:
                py, px = hop_window(L, int(d), int(x), int(y))
                hops[py].append((px, s2))
    e_off = 0.0
    e_mag = 0.0
    for py in range(L - 1):
        Dm = D[py - 1] if py >= 1 else _trivial_mps(L)
        Up = Uenv[py + 2] if py + 2 <= L - 1 else _trivial_mps(L)
        E, F = strip_environments(Dm, T[py], T[py + 1], Up)
        denom = float(E[L].reshape(()))
        if denom == 0.0:
            return (math.nan, math.nan) if with_scale else math.nan

        def window_num(px, s2):  # strip amplitude of s2 (the ratio's numerator)
            ok, T2, _ = project(layout, theta, s2)
            assert ok
            X = _absorb_left(E[px], Dm[px], T2[py][px], T2[py + 1][px], Up[px])
            X = _absorb_left(X, Dm[px + 1], T2[py][px + 1], T2[py + 1][px + 1], Up[px + 1])
            return float(np.einsum("abcd,abcd->", X, F[px + 2]))

        for px in range(L - 1):
            for t in range(1, N):
                if c_tab[t] == 0.0:
                    continue
                term = c_tab[t] * window_num(px, apply_plaquette(links, px, py, (N - t) % N, N)) / denom  # P_p^{-t} s
                e_off += term
                e_mag += abs(term)
        for px, s2 in hops[py]:
            term = hop * window_num(px, s2) / denom
            e_off += term
            e_mag += abs(term)
    n_occ = int(np.sum(links[2])) if layout.matter else 0
    e_loc = electric_energy(links, e_tab) + mass * n_occ + e_off
    if with_scale:
        return e_loc, electric_magnitude(links, e_tab) + abs(mass) * n_occ + e_mag
    return e_loc


def local_energy_exact(layout, theta, links, c_tab, e_tab, amp):
    """E_loc with exact amplitudes supplied by `amp(links) -> Psi` (small lattices)."""
    L, N = layout.L, layout.N
    psi = amp(links)
    if psi == 0.0:
        return math.nan
    tot = electric_energy(links, e_tab)
    for py in range(L - 1):
        for px in range(L - 1):
            for t in range(1, N):
                if c_tab[t] != 0.0:
                    tot += c_tab[t] * amp(apply_plaquette(links, px, py, (N - t) % N, N)) / psi
    return tot
