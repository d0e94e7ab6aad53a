"""Where FP32 products may enter the mixed path: CPU emulation (tests/precision_emulation.py) of
the canonical sweep and the strip ratios with chosen products rounded to FP32, measured with the
per-sample criterion C1, delta(s) = |E_fp32(s) - E_fp64(s)| / M(s), M the magnitude of E_loc's terms.

Placements: "xt" (X = Y T, the product the library runs in FP32), "rb" + "qg" (the products with
the QR and SVD factors), "strip" (the strip contractions behind the local-energy ratios).  Findings
asserted here:
  * with no FP32 product the emulation is the oracle (it re-expresses the same algorithm);
  * on typical configurations every placement keeps delta below 1e-5 and ln|Psi| within 1e-6;
  * on the near-node configuration that is the mixed path's worst at the benchmark shape (Z3 16x16,
    chi = 36, uniform sample 1309, whose E_loc ~ -4.5e5 is a sum of terms of magnitude ~1e6), every
    placement misses 1e-5 by two orders and the placements differ by less than a factor 3: the
    error there is set by the cancellation, not by which products are FP32.
"""
import math

import numpy as np
import pytest

from oracle.contract import amplitude
from oracle.energy import config_tables, local_energy
from oracle.lattice import links_from_powers
from oracle.layout import Layout, project
from paper_2503_20566_amd import synth
from tests import precision_emulation as pe
from tests.helpers import configs

PLACEMENTS = [{"xt"}, {"xt", "rb"}, {"xt", "qg"}, {"xt", "rb", "qg"}, {"xt", "strip"}]


def _measure(lay, theta, s, chi, c, e, placements):
    ok, T, _ = project(lay, theta, s)
    la = amplitude(T, chi)[0]
    el, m = local_energy(lay, theta, s, chi, c, e, with_scale=True)
    la0 = pe.amplitude(T, chi, set())[0]
    el0 = pe.local_energy(lay, theta, s, chi, c, e, set())
    # the oracle itself, to rounding (the factored row application rounds in another order, which
    # the cancellation at near-node configurations amplifies; the FP64 bar of the GPU tests)
    assert abs(la0 - la) <= 1e-12 * abs(la) and abs(el0 - el) <= 1e-9 * m
    out = {}
    for place in placements:
        lp = pe.amplitude(T, chi, place)[0]
        ep = pe.local_energy(lay, theta, s, chi, c, e, place)
        out["+".join(sorted(place))] = (abs(ep - el) / m, abs(lp - la) / abs(la))
    return m, out


def test_placements_on_a_uniform_z3_8x8_batch():
    L, N, Dk, chi = 8, 3, 2, 12
    lay = Layout(L, N, [Dk] * N)
    theta = synth.theta_normals(lay.n_params, N * Dk)
    c, e = config_tables(N, 1.0, 0.4)
    rows = [_measure(lay, theta, s, chi, c, e, PLACEMENTS)[1] for s in configs(12, L, N, seed=77)]
    for key in rows[0]:
        d = max(r[key][0] for r in rows)
        lr = max(r[key][1] for r in rows)
        print("Z3 8x8 chi=12, 12 uniform samples, FP32 %-12s: delta max %.2e, ln|Psi| rel max %.2e"
              % (key, d, lr))
        assert d <= 1e-5 and lr <= 1e-6


@pytest.mark.parametrize("b,near_node", [(0, False), (1309, True)])
def test_placements_at_the_benchmark_shape(b, near_node):
    L, N, Dk, chi, B = 16, 3, 2, 36, 2048
    lay = Layout(L, N, [Dk] * N)
    theta = synth.theta_normals(lay.n_params, N * Dk)
    c, e = config_tables(N, 1.0, 0.4)
    s = links_from_powers(synth.plaquette_powers(B, L, N)[b], N)
    m, res = _measure(lay, theta, s, chi, c, e, [{"xt"}, {"xt", "rb", "qg"}, {"xt", "strip"}])
    for key, (d, lr) in res.items():
        print("Z3 16x16 chi=36 sample %d (M = %.3g), FP32 %-9s: delta %.2e, ln|Psi| rel %.2e" % (b, m, key, d, lr))
    deltas = [d for d, _ in res.values()]
    if near_node:
        assert min(deltas) > 1e-4 and max(deltas) < 3 * min(deltas)
    else:
        assert max(deltas) <= 1e-5 and max(lr for _, lr in res.values()) <= 1e-6
    assert math.isfinite(m)
