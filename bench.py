"""Throughput of the GCF-PEPS VMC hot path on one MI355X.

One step = one pass of the hot path over one batch of synthetic configurations already resident
in HBM: projection, amplitude (down boundary sweep + close), log-derivatives, local energy and
the SR build (force, mean and one S*v product), each through the C ABI.

Prints ONE JSON line.  `value` is the metric's rate, amplitude + dlnPsi samples/s: B / the time of the
project + amplitude + logderiv part of each timed step, of the headline path (mixed: FP32 product
of boundary and row tensor, FP64 factorisations); `step_samples_per_s` is the whole step's rate.
`other_path` times the other precision on the same batch and `mixed_vs_f64` states the differences
between the two against the criteria of the design notes (per-sample E_loc error against the
magnitude of its terms; E/site over chains drawn from |Psi|^2).  `roofline` is computed for the dominant kernel
family from its HIP-event durations measured inside the timed region; `cpu_baseline` times the plain
CPU oracle on a bounded sample of the same workload (run before the GPU is touched).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload z3_16x16_d6] [--dtype mixed|f64]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk/CU
                                 # (FP64 matrix-core dense peak is the same 78.6 TFLOP/s)

# HBM bytes per k_row_sweep launch at z3_16x16_d6 (mean over the step's 27 launches: 14 taped
# down-sweep rows, 13 up-sweep rows) from rocprofv3 FETCH_SIZE / WRITE_SIZE runs, scaled by a
# plain-copy calibration (FETCH x2.00, WRITE x1.00); valid only for the kernel source and build
# flags they were measured with (sha256 prefixes of k_sweep.hip, dev_common.h and build.py),
# reported as null otherwise.
ROW_SWEEP_TRAFFIC = {"sources": {"csrc/k_sweep.hip": "8bf47d09c6b23d74", "csrc/dev_common.h": "dc494028c62ca1a2",
                                 "build.py": "f7ebea33db24a875"},
                     "workload": "z3_16x16_d6", "bytes": 1058784 * 1024 * 2.00 + 2021970 * 1024 * 1.00}


# Executed FP64 work per k_row_sweep launch at z3_16x16_d6 from rocprofv3 counters
# (profiles/pmc_fp64_mfma_z3_16x16_d6.md): 64 x SQ_INSTS_VALU_FLOPS_FP64(+_TRANS) (per-wave counts,
# FMA = 2) + 512 x SQ_INSTS_VALU_MFMA_MOPS_F64, and the MfmaUtil / VALUBusy / LdsUtil percentages;
# valid only for the kernel source and build flags they were measured with.
ROW_SWEEP_EXECUTED = {"sources": {"csrc/k_sweep.hip": "8bf47d09c6b23d74", "csrc/dev_common.h": "dc494028c62ca1a2",
                                  "build.py": "f7ebea33db24a875"},
                      "workload": "z3_16x16_d6",
                      "flops": 64 * (4.7527e9 + 5.9116e7) + 512 * 3.7085e7,
                      "mfma_util_pct": 0.64, "valu_busy_pct": 29.0, "lds_util_pct": 21.9}


def _sources_match(sources):
    import hashlib
    pkg = os.path.join(ROOT, "paper_2503_20566_amd")
    for name, want in sources.items():
        with open(os.path.join(pkg, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != want:
                return False
    return True


def _row_sweep_traffic(workload):
    if not _sources_match(ROW_SWEEP_TRAFFIC["sources"]):
        return None
    return ROW_SWEEP_TRAFFIC["bytes"] if workload == ROW_SWEEP_TRAFFIC["workload"] else None


def _row_sweep_executed(workload, avg_ms):
    e = ROW_SWEEP_EXECUTED
    if workload != e["workload"] or not avg_ms or not _sources_match(e["sources"]):
        return None
    tf = e["flops"] / (avg_ms * 1e-3) / 1e12
    return {"flops_per_launch": e["flops"], "tflops": tf, "frac": tf / FP64_VECTOR_PEAK_TFLOPS,
            "mfma_util_pct": e["mfma_util_pct"], "valu_busy_pct": e["valu_busy_pct"],
            "lds_util_pct": e["lds_util_pct"], "source": "rocprofv3 counters, profiles/pmc_fp64_mfma_z3_16x16_d6.md"}


def _fused_bond(wl):
    """Largest fused bond chi * D_k the row sweeps reach (the library's maxN)."""
    bond, qrk = bond_tables(wl["L"], wl["Dk"], wl["chi"])
    return max(max(wl["Dk"] * x for row in bond for x in row), max(x for row in qrk for x in row))


def _large_bond(wl):
    """Fused bonds above 72 (up to 128) run on the large-bond kernels, which offer no stored tape."""
    return _fused_bond(wl) > 72


def bond_tables(L, Dk, chi):
    """Bond dimensions of the canonical sweep (same recurrence as the library's tables)."""
    bond = [[(1 if c in (0, L) else Dk) for c in range(L + 1)]]
    qrk = [[1] * L]
    for y in range(1, L - 1):
        bp = bond[-1]
        m = [bp[c] * (1 if c in (0, L) else Dk) for c in range(L + 1)]
        q = [1] * L
        r = 1
        for c in range(L - 1):
            q[c] = min(r * Dk, m[c + 1])
            r = q[c]
        bn = [1] * (L + 1)
        cn = 1
        for c in range(L - 1, 0, -1):
            bn[c] = min(chi, q[c - 1], Dk * cn)
            cn = bn[c]
        bond.append(bn)
        qrk.append(q)
    return bond, qrk


def _qr_flops(m, n):
    k = min(m, n)
    r = 2.0 * m * n * k - (m + n) * k * k + 2.0 * k ** 3 / 3.0      # Householder R
    q = 4.0 * m * k * k - 2.0 * (m + k) * k * k + 4.0 * k ** 3 / 3.0  # explicit Q (m x k)
    return r + q


def _svd_flops(m, n):
    m, n = max(m, n), min(m, n)
    return 6.0 * m * n * n + 20.0 * n ** 3                             # R-SVD with U1, V (GVL)


def row_sweep_flops(L, Dk, chi, matrix_core_only=False):
    """Algorithmic FP64 flops of one sample's down sweep (all rows y = 1..L-2): the row
    application as the factored contraction R (B T), Householder QR with explicit Q, the thin
    SVD at every cut (dense-LAPACK op counts), and Theta = Q G. With matrix_core_only, only the
    products the kernel runs on the matrix cores (R B and Q G)."""
    bond, qrk = bond_tables(L, Dk, chi)
    total = 0.0
    mc = 0.0
    for y in range(1, L - 1):
        bp, bn, q = bond[y - 1], bond[y], qrk[y]
        r = 1
        for c in range(L):
            dl = Dk if c > 0 else 1
            dr = Dk if c < L - 1 else 1
            total += 2.0 * r * dl * Dk * bp[c + 1] * bp[c]            # Y = R B
            mc += 2.0 * r * dl * Dk * bp[c + 1] * bp[c]
            total += 2.0 * (r * Dk) * (bp[c + 1] * dr) * (dl * Dk)    # X = Y T
            if c < L - 1:
                total += _qr_flops(r * Dk, bp[c + 1] * dr)
                r = q[c]
        for c in range(L - 1, 0, -1):
            mA, nA = q[c - 1], Dk * bn[c + 1]
            total += _svd_flops(mA, nA)
            if c < L - 1:
                total += 2.0 * (mA * Dk) * q[c] * bn[c + 1]
                mc += 2.0 * (mA * Dk) * q[c] * bn[c + 1]
    return mc if matrix_core_only else total


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo; lscpu reports the same field)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# host cores a one-GPU share of the measurement machine provides: worker pools are sized to this
# share, whatever the affinity mask shows
HOST_CORES_PER_GPU = 16


def cpu_baseline(wl, seconds=15.0):
    """Time the oracle (never tuned) on host cores over a bounded sample of the workload."""
    import concurrent.futures as cf
    import numpy as np  # noqa: F401
    available = len(os.sched_getaffinity(0))
    cores = max(1, min(available, HOST_CORES_PER_GPU))
    n = 0
    t0 = time.time()
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=cores, initializer=_pool_init,
                                mp_context=mp.get_context("fork")) as ex:
        batch = cores
        start = 0
        while time.time() - t0 < seconds:
            list(ex.map(_oracle_one, [(wl, i) for i in range(start, start + batch)]))
            start += batch
            n += batch
    dt = time.time() - t0
    return {"value": n / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "cores_available": available, "cpu_model": cpu_model(),
            "sample": "%d configurations of %s through the oracle's step (projection, ln|Psi|, O_k "
                      "by CPU autodiff, E_loc), one process per core, one BLAS thread each; "
                      "%d of the %d cores in the affinity mask (a one-GPU share is %d host cores)%s"
                      % (n, wl["name"], cores, available, HOST_CORES_PER_GPU,
                                      "; uniform plaquette-power configurations of the workload's "
                                      "shape (the oracle's cost per configuration does not depend "
                                      "on which one)" if wl.get("sweeps") else "")}


def _pool_init():
    import numpy  # noqa: F401  (load the BLAS before limiting it)
    import torch
    from threadpoolctl import threadpool_limits
    torch.set_num_threads(1)          # one compute thread per worker process
    threadpool_limits(limits=1)


_ORACLE_CACHE = {}


def _oracle_one(arg):
    """One sample of the step through the oracle: projection, ln|Psi|, O_k (autodiff), E_loc."""
    wl, i = arg
    from oracle.contract import amplitude
    from oracle.energy import config_tables, local_energy
    from oracle.lattice import links_from_powers
    from oracle.layout import Layout, project
    from oracle.logderiv import log_derivatives
    from paper_2503_20566_amd import synth
    key = wl["name"]
    if key not in _ORACLE_CACHE:
        lay = Layout(wl["L"], wl["N"], [wl["Dk"]] * wl["N"])
        theta = synth.theta_normals(lay.n_params, wl["N"] * wl["Dk"])
        powers = synth.plaquette_powers(wl["batch"], wl["L"], wl["N"])
        _ORACLE_CACHE[key] = (lay, theta, powers)
    lay, theta, powers = _ORACLE_CACHE[key]
    s = links_from_powers(powers[i % wl["batch"]], wl["N"])
    ok, T, _ = project(lay, theta, s)
    la = amplitude(T, wl["chi"])
    log_derivatives(T, wl["chi"])
    c, e = config_tables(wl["N"], wl["J"], wl["h"])
    return la, local_energy(lay, theta, s, wl["chi"], c, e)


def precision_figures(L, mix, f64, chains=False):
    """Mixed vs FP64 on one batch: the per-sample criteria and the reported-only figures.  A batch
    of uniformly drawn configurations also gets its |Psi|^2-reweighted mean; a batch of Metropolis
    chains is already |Psi|^2-distributed, so its plain mean is the VMC estimate."""
    import numpy as np
    la_rel = np.abs(mix["la"] - f64["la"]) / np.abs(f64["la"])
    de = np.abs(mix["el"] - f64["el"])
    delta = de / f64["m"]
    rel_e = de / np.abs(f64["el"])
    w = np.exp(2.0 * (f64["la"] - f64["la"].max()))   # |Psi|^2 weights of uniformly drawn samples
    ess = float(w.sum() ** 2 / np.sum(w * w))
    wd = float(np.sum(w * f64["el"]) / np.sum(w))
    wm = float(np.sum(w * mix["el"]) / np.sum(w))
    plain = abs(float(mix["el"].mean()) - float(f64["el"].mean())) / abs(float(f64["el"].mean()))
    if chains:
        return {"ln_psi_rel_max": float(la_rel.max()),
                "ln_psi_abs_max": float(np.max(np.abs(mix["la"] - f64["la"]))),
                "c1_delta_max": float(delta.max()),
                "c1_delta_p50_p90_p99": [float(v) for v in np.percentile(delta, [50, 90, 99])],
                "e_loc_rel_p50_p90_p99_max": [float(v) for v in np.percentile(rel_e, [50, 90, 99, 100])],
                "chain_plain_mean_e_site_rel": plain}
    return {"ln_psi_rel_max": float(la_rel.max()),
            "ln_psi_abs_max": float(np.max(np.abs(mix["la"] - f64["la"]))),
            "c1_delta_max": float(delta.max()),
            "c1_delta_p50_p90_p99": [float(v) for v in np.percentile(delta, [50, 90, 99])],
            "e_loc_rel_p50_p90_p99_max": [float(v) for v in np.percentile(rel_e, [50, 90, 99, 100])],
            "uniform_weighted_e_site_rel": abs(wm - wd) / abs(wd), "uniform_weighted_ess": ess,
            "uniform_plain_mean_e_site_rel": plain}


def sampled_chain_e_site(wl, c, e, sweeps=10):
    """E/site as VMC measures it (plain mean over configurations drawn from |Psi|^2): chains from
    Philox initial states and `sweeps` strip-sampler sweeps of the FP64 path, then E_loc of the
    final configurations through both paths (outside the timed region)."""
    import numpy as np
    import torch
    from paper_2503_20566_amd import gipeps, synth
    L, N, Dk, chi, B = wl["L"], wl["N"], wl["Dk"], wl["chi"], wl["batch"]
    Pd = gipeps.Peps(L, N, Dk, chi, c, e, dtype=gipeps.PEPS_F64)
    Pm = gipeps.Peps(L, N, Dk, chi, c, e, dtype=gipeps.PEPS_F32_MIXED)
    th = torch.from_numpy(synth.theta_normals(Pd.n_params, N * Dk)).cuda()
    _, links = Pd.sample_init(B, synth.SAMPLE_SEED, 0)
    ws = Pd.workspace(B, gipeps.PEPS_WS_AMPLITUDE | gipeps.PEPS_WS_ENERGY)
    _, acc = Pd.metropolis_strip(th, links, synth.SAMPLE_SEED, 1, sweeps, ws)
    out = {}
    for name, P in (("f64", Pd), ("mixed", Pm)):
        proj, bid, valid = P.project(th, links)
        la, _ = P.amplitude(proj, valid, ws)
        el = P.local_energy(th, links, proj, valid, ws)
        m = P.eloc_scale(B, ws)
        out[name] = {"la": la.cpu().numpy(), "el": el.cpu().numpy(), "m": m.cpu().numpy()}
    torch.cuda.synchronize()
    del ws
    Pd.close()
    Pm.close()
    torch.cuda.empty_cache()
    fig = precision_figures(L, out["mixed"], out["f64"])
    ed = float(out["f64"]["el"].mean()) / L ** 2
    em = float(out["mixed"]["el"].mean()) / L ** 2
    return {"chains": B, "sweeps": sweeps, "acceptance": acc.sum().item() / (B * sweeps * (L - 1) ** 2),
            "e_site_f64": ed, "e_site_mixed": em, "e_site_rel": abs(em - ed) / abs(ed),
            "c1_delta_max": fig["c1_delta_max"], "ln_psi_rel_max": fig["ln_psi_rel_max"]}


def sample_chains(sweeps, plain_sweeps):
    """Chain generation of the Z2 16x16 workload (4096 chains, chi = 16): sweeps per second of the
    strip-ratio sampler and of the plain one, each timed after one untimed sweep."""
    import time
    import torch
    from paper_2503_20566_amd import gipeps, synth
    wl = synth.WORKLOADS["z2_16x16_d4"]
    L, N, Dk, chi, B = wl["L"], wl["N"], wl["Dk"], wl["chi"], wl["batch"]
    c = [0.0, -wl["J"]]
    e = [-wl["h"], wl["h"]]
    torch.cuda.set_device(0)
    P = gipeps.Peps(L, N, Dk, chi, c, e)
    theta = torch.from_numpy(synth.theta_normals(P.n_params, N * Dk)).cuda()
    ws = P.workspace(B, gipeps.PEPS_WS_AMPLITUDE | gipeps.PEPS_WS_ENERGY | gipeps.PEPS_WS_SAMPLE)
    out = {"workload": "z2_16x16_d4", "chains": B, "proposals_per_sweep": (L - 1) ** 2}
    for name, fn, n in (("strip", P.metropolis_strip, sweeps), ("plain", P.metropolis, plain_sweeps)):
        if n <= 0:
            continue
        _, links = P.sample_init(B, synth.SAMPLE_SEED, 0)
        fn(theta, links.clone(), synth.SAMPLE_SEED, 1, 1, ws)
        torch.cuda.synchronize()
        t0 = time.time()
        _, acc = fn(theta, links, synth.SAMPLE_SEED, 1, n, ws)
        torch.cuda.synchronize()
        dt = time.time() - t0
        out[name] = {"sweeps": n, "s_per_sweep": dt / n, "chain_sweeps_per_s": B * n / dt,
                     "acceptance": acc.sum().item() / (B * n * (L - 1) ** 2)}
    if "strip" in out and "plain" in out:
        out["speedup"] = out["plain"]["s_per_sweep"] / out["strip"]["s_per_sweep"]
    print(json.dumps(out), flush=True)


def tvmc_run(steps, sweeps, B=8192, L=10, Dk=2, dt=0.01, shift=1e-4, c64=False, resample=0):
    """Real-time steps (SM S-3) on the 10 x 10 Z2 lattice at h = 0.2, J = 1 with a pair of Gauss-law
    defects at the ends of a 3-link string in the middle row; the toric-code state padded to
    D = 2 Dk with complex noise of 1e-3 on the added entries (D = 4 by default, where 8192 samples
    fit: at D = 6 the exact contraction needs 55 MB of workspace per sample).  B chains of the
    sector are drawn from |Psi|^2 by the complex Metropolis sampler, then each timed step is one
    tvmc_step (eq. secondorder, plain sample means, CG to 1e-8).  c64: the contractions in complex64
    (PEPS_C64_EXACT), which halves the row states' workspace.  resample: strip-sampler sweeps of the
    chains before every timed step (inside the timed loop), as a sampled real-time loop runs."""
    import time
    import torch
    from paper_2503_20566_amd import gipeps, synth
    N, h = 2, 0.2
    c, e = [0.0, -1.0], [-h, h]
    s0 = torch.zeros((2, L, L), dtype=torch.uint8)
    y0 = L // 2
    for x in range(L // 2 - 2, L // 2 + 1):          # 3 horizontal links in the middle row
        s0[0, y0, x] = 1
    Q = torch.zeros((L, L), dtype=torch.int64)
    for x in range(L):                               # Gauss residual of the string: its two ends
        for y in range(L):
            nl = int(s0[0, y, x - 1]) if x > 0 else 0
            nr = int(s0[0, y, x]) if x < L - 1 else 0
            nd = int(s0[1, y - 1, x]) if y > 0 else 0
            nu = int(s0[1, y, x]) if y < L - 1 else 0
            Q[y, x] = (nl + nd - nr - nu) % N
    torch.cuda.set_device(0)
    P = gipeps.Peps(L, N, Dk, 4, c, e, Q=Q.numpy().astype("int8"),
                    dtype=gipeps.PEPS_C64_EXACT if c64 else gipeps.PEPS_C128_EXACT)
    # toric code: the entry (0,0,0,0) of every block is 1; the other entries complex noise 1e-3
    rng = torch.Generator().manual_seed(synth.THETA_SEED)
    theta = (torch.randn(P.n_params, generator=rng, dtype=torch.float64)
             + 1j * torch.randn(P.n_params, generator=rng, dtype=torch.float64)) * 1e-3
    for s in range(L * L):
        x, y = s % L, s // L
        npres = (x > 0) + (x < L - 1) + (y > 0) + (y < L - 1)
        bs = Dk ** npres
        for off in range(P.site_offset[s], P.site_offset[s + 1], bs):
            theta[off] = 1.0
    theta = theta.cuda()
    _, links = P.sample_init(B, synth.SAMPLE_SEED, 0)
    links = (links + s0.cuda()) % N                  # the string's sector
    ws = P.workspace(B, gipeps.PEPS_WS_AMPLITUDE | gipeps.PEPS_WS_TVMC | gipeps.PEPS_WS_SAMPLE)
    t0 = time.time()
    acc = torch.zeros((B,), dtype=torch.int32, device="cuda")
    for k in range(sweeps):                          # one call per sweep: a progress line each
        P.metropolis_strip(theta, links, synth.SAMPLE_SEED, 1 + k, 1, ws, accepted=acc)
        torch.cuda.synchronize()
        print("tvmc: sweep %d of %d done (%.1f s)" % (k + 1, sweeps, time.time() - t0), file=sys.stderr, flush=True)
    t_sample = time.time() - t0
    print("tvmc: %d chains sampled (%d sweeps) in %.1f s" % (B, sweeps, t_sample), file=sys.stderr, flush=True)
    _, its = P.tvmc_step(theta.clone(), links, ws, dt, shift=shift, rtol=1e-8, max_iter=500)   # warm-up
    torch.cuda.synchronize()
    print("tvmc: warm-up step done, CG iterations %s" % (its,), file=sys.stderr, flush=True)
    # kernel families of the step; the sampler's sweeps are read apart (its strip kernel shares the
    # E_loc family's counters, its row states the states family's)
    fams = (("project", gipeps.PEPS_K_PROJECT), ("states", gipeps.PEPS_K_ROW_SWEEP),
            ("e_loc", gipeps.PEPS_K_STRIP), ("logderiv", gipeps.PEPS_K_ADJOINT), ("sr", gipeps.PEPS_K_SR))

    def read_parts(acc):
        for name, fam in fams:
            n, ms = P.profile_read(fam)
            a = acc.setdefault(name, [0, 0.0])
            a[0] += n
            a[1] += ms

    P.profile(True)
    energies, iters = [], []
    step_acc, sample_acc = {}, {}
    t0 = time.time()
    for k in range(steps):
        if resample:
            P.metropolis_strip(theta, links, synth.SAMPLE_SEED, 1 + sweeps + k * resample, resample, ws)
            read_parts(sample_acc)
        en, its = P.tvmc_step(theta, links, ws, dt, shift=shift, rtol=1e-8, max_iter=500)
        read_parts(step_acc)
        energies.append(en.real)
        iters.append(its)
        print("tvmc: step %d <H> %.10f, CG %s" % (k, en.real, its), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_steps = time.time() - t0
    parts = {name: {"launches": n, "ms_per_step": ms / max(1, steps)} for name, (n, ms) in step_acc.items()}
    sample_names = {"project": "project", "states": "states", "e_loc": "strip_sweeps"}
    sample_parts = {sample_names.get(name, name): {"launches": n, "ms_per_step": ms / max(1, steps)}
                    for name, (n, ms) in sample_acc.items() if n}
    out = {"metric": "tVMC steps/s", "value": steps / t_steps, "unit": "steps/s", "ms_per_step": 1e3 * t_steps / steps,
           "samples_per_s": 2 * B * steps / t_steps, "dtype": "c64+f64" if c64 else "c128", "data": "synthetic",
           "config": {"workload": "tvmc_z2_10x10_d%d_string" % (2 * Dk), "L": L, "D": 2 * Dk, "samples": B, "dt": dt,
                      "shift": shift, "cg_rtol": 1e-8, "cg_max_iter": 500, "contraction": "exact"},
           "n_params": P.n_params, "energies": energies, "drift_rel": abs(energies[-1] - energies[0]) / abs(energies[0]),
           "cg_iterations": iters, "parts_ms_per_step": parts, "resample_parts_ms_per_step": sample_parts,
           "sampling": {"sweeps": sweeps, "seconds": t_sample, "sampler": "strip ratios (peps_metropolis_strip)",
                        "resample_sweeps_per_step": resample,
                        "acceptance": acc.sum().item() / (B * sweeps * (L - 1) ** 2) if sweeps else None}}
    print(json.dumps(out), flush=True)


def ragged_run(steps):
    """Several lattices of the Z4 32 x 32 study together: the amplitude of 1024 samples of each,
    timed three ways on the same inputs: one lattice after the other on one stream, each on its own
    stream, and as one ragged batch (peps_amplitude_ragged: one launch per boundary row for all
    lattices).  Two sets: 8 x 8, 12 x 12, 24 x 24 at chi = 36 and 12 x 12, 24 x 24, 32 x 32 at
    chi = 64 (the large-bond kernels; the 8 x 8 lattice never reaches their bond and cannot join)."""
    import torch
    from paper_2503_20566_amd import gipeps, synth
    N, Dk, B = 4, 2, 1024
    c = [0.0, -1.0, 0.0, -1.0]
    e = [-2.0 * 0.5 * math.cos(2.0 * math.pi * n / N) for n in range(N)]
    sets = []
    for chi, Ls in ((36, (8, 12, 24)), (64, (12, 24, 32))):
        groups = []
        for L in Ls:
            P = gipeps.Peps(L, N, Dk, chi, c, e, dtype=gipeps.PEPS_F32_MIXED)
            th = torch.from_numpy(synth.theta_normals(P.n_params, N * Dk)).cuda()
            links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda())
            proj, _, valid = P.project(th, links)
            groups.append((P, proj, valid, P.workspace(B, gipeps.PEPS_WS_AMPLITUDE)))
        streams = [torch.cuda.Stream() for _ in groups]

        def sequential():
            for P, proj, valid, ws in groups:
                P.amplitude(proj, valid, ws)

        def concurrent():
            for st in streams:
                st.wait_stream(torch.cuda.current_stream())
            for (P, proj, valid, ws), st in zip(groups, streams):
                with torch.cuda.stream(st):
                    P.amplitude(proj, valid, ws)
            for st in streams:
                torch.cuda.current_stream().wait_stream(st)

        def ragged():
            gipeps.amplitude_ragged(groups)

        res = {"chi": chi, "lattices": list(Ls), "batch_each": B}
        for name, fn in (("sequential", sequential), ("streams", concurrent), ("ragged", ragged)):
            fn()
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(steps):
                fn()
            t1.record()
            torch.cuda.synchronize()
            res[name + "_ms"] = t0.elapsed_time(t1) / steps
            print("chi %d %s: %.1f ms" % (chi, name, res[name + "_ms"]), file=sys.stderr, flush=True)
        res["samples_per_s_ragged"] = len(Ls) * B / (res["ragged_ms"] * 1e-3)
        sets.append(res)
        del groups
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "ragged", "what": "amplitude (project excluded) of 1024 samples per lattice, "
                      "mixed path, Z4 D = 8", "steps": steps, "sets": sets}), flush=True)


def matter_run(steps, warmup, sweeps, B=2048, L=16, Dk=2, chi=36):
    """Z2 gauge field with hard-core bosons at half filling (L^2/2 bosons), (h, g, J) = (1, 0.33,
    0.5) of the paper's boson study, D = 4, chi = 36, FP64: the step project + amplitude + logderiv
    + local_energy (hopping windows included) timed over `steps` batches, then `sweeps` strip-sampler
    sweeps (plaquette and link moves) of the same chains.  The amplitude stores its factorisations
    for the reverse sweep (keep_tape), as the headline step does."""
    import time
    import torch
    from paper_2503_20566_amd import gipeps, synth
    N, hp, g, J = 2, 1.0, 0.33, 0.5
    c = [0.0, -2.0 * hp]                                   # H_B = -h (P + P^dag), P = P^dag for Z2
    e = [g * (2.0 - 2.0 * math.cos(math.pi * n)) for n in range(N)]
    torch.cuda.set_device(0)
    P = gipeps.Peps(L, N, Dk, chi, c, e, matter=True, hop=J, mass=0.0, ckpt_every=1, keep_tape=True)
    theta = torch.from_numpy(synth.theta_normals(P.n_params, N * Dk)).cuda()
    occ = torch.from_numpy(synth.occupations(B, L, L * L // 2)).cuda()
    links = P.matter_links(torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda(), occ)
    ws = P.workspace(B)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    parts = {"amplitude_dlnpsi": 0.0, "local_energy": 0.0}
    for k in range(warmup + steps):
        ev[0].record()
        proj, bid, valid = P.project(theta, links)
        P.amplitude(proj, valid, ws)
        P.logderiv(proj, bid, valid, ws)
        ev[1].record()
        P.local_energy(theta, links, proj, valid, ws)
        ev[2].record()
        torch.cuda.synchronize()
        if k >= warmup:
            parts["amplitude_dlnpsi"] += ev[0].elapsed_time(ev[1]) / steps
            parts["local_energy"] += ev[1].elapsed_time(ev[2]) / steps
    print("matter: %d steps timed" % steps, file=sys.stderr, flush=True)
    ws2 = P.workspace(B, gipeps.PEPS_WS_AMPLITUDE | gipeps.PEPS_WS_ENERGY)
    P.metropolis_strip(theta, links, synth.SAMPLE_SEED, 1, 1, ws2)   # warm-up sweep
    torch.cuda.synchronize()
    t0 = time.time()
    _, acc = P.metropolis_strip(theta, links, synth.SAMPLE_SEED, 2, sweeps, ws2)
    torch.cuda.synchronize()
    t_sw = (time.time() - t0) / max(1, sweeps)
    nb = torch.sum(links[:, 2].to(torch.int64), dim=(1, 2))
    out = {"metric": "amplitude+dlnPsi samples/s (Z2 + hard-core bosons)",
           "value": B / (parts["amplitude_dlnpsi"] * 1e-3), "unit": "samples/s",
           "step_samples_per_s": B / ((parts["amplitude_dlnpsi"] + parts["local_energy"]) * 1e-3),
           "parts_ms_per_step": parts, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "z2_boson_16x16_d4_half_filling", "L": L, "D": N * Dk, "chi": chi, "batch": B,
                      "bosons": L * L // 2, "h": hp, "g": g, "J": J},
           "chains": {"sweeps": sweeps, "s_per_sweep": t_sw,
                      "moves_accepted_per_chain_sweep": acc.sum().item() / (B * (sweeps + 1)),
                      "boson_number_conserved": bool(torch.all(nb == L * L // 2).item())}}
    print(json.dumps(out), flush=True)


def hamiltonian_tables(wl):
    """Plaquette coefficients c[t] and electric energies e[n] of a workload: -J on the powers 1 and
    N-1 (one power for Z2), e[n] = -2 h cos(2 pi n / N) (Z2: -h, h)."""
    N, J, h = wl["N"], wl["J"], wl["h"]
    c = [0.0] * N
    if N == 2:
        c[1] = -J
        return c, [-h, h]
    c[1] = c[N - 1] = -J
    return c, [-2.0 * h * math.cos(2.0 * math.pi * n / N) for n in range(N)]


def phase_split(workload, dtype_name, tuning_cache, verbose=True):
    """Shader-clock cycles per phase of the row-sweep kernel (peps_profile_phases) on one workload's
    uniform batch: the down sweep of the amplitude (taped rows) and the mirrored up sweep of the
    local energy, each as the share of every phase and the cycles per workgroup and row."""
    import torch
    from paper_2503_20566_amd import gipeps, synth
    wl = dict(synth.WORKLOADS[workload])
    L, N, Dk, chi, B = wl["L"], wl["N"], wl["Dk"], wl["chi"], wl["batch"]
    c, e = hamiltonian_tables(wl)
    torch.cuda.set_device(0)
    dtype = gipeps.PEPS_F32_MIXED if dtype_name == "mixed" else gipeps.PEPS_F64
    big = _large_bond(wl)
    P = gipeps.Peps(L, N, Dk, chi, c, e, dtype=dtype, ckpt_every=1, keep_tape=not big)
    theta = torch.from_numpy(synth.theta_normals(P.n_params, N * Dk)).cuda()
    links = P.links_from_powers(torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda())
    ws = P.workspace(B)
    proj, _, valid = P.project(theta, links)
    tuned = P.autotune(proj, valid, ws, cache=tuning_cache) if not big else None
    P.amplitude(proj, valid, ws)                        # warm-up
    torch.cuda.synchronize()
    counters = torch.zeros(len(gipeps.PHASES), dtype=torch.int64, device="cuda")
    P.profile_phases(counters)
    out = {"workload": workload, "dtype": dtype_name, "batch": B,
           "tuning": tuned["tuning"] if tuned else None, "clock": "shader clock cycles of the first thread"}
    for name, run, rows in (("down", lambda: P.amplitude(proj, valid, ws), L - 2),
                            ("up", lambda: P.local_energy(theta, links, proj, valid, ws), L - 3)):
        counters.zero_()
        run()
        torch.cuda.synchronize()
        cyc = counters.cpu().tolist()
        tot = float(sum(cyc))
        out[name] = {"rows": rows, "cycles_per_workgroup_row": tot / (B * rows),
                     "share": {ph: cyc[i] / tot for i, ph in enumerate(gipeps.PHASES)}}
        if verbose:
            print("%s sweep: %s" % (name, ", ".join("%s %.1f%%" % (ph, 100 * cyc[i] / tot)
                                                   for i, ph in enumerate(gipeps.PHASES))),
                  file=sys.stderr, flush=True)
    P.profile_phases(None)
    del P, ws
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="z3_16x16_d6")
    ap.add_argument("--dtype", default="mixed", choices=["f64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--keep-tape", type=int, default=-1, choices=[-1, 0, 1],
                    help="1: the amplitude stores every row's factorisations for the reverse sweep; "
                         "0: the reverse sweep recomputes them; -1 (default): 1 when it fits in "
                         "70%% of free device memory")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--sample-chains", action="store_true",
                    help="only time the chain generation of the Z2 16x16 workload: Philox initial "
                         "states, then --sweeps strip-ratio Metropolis sweeps and --plain-sweeps "
                         "sweeps of the plain sampler (one amplitude per proposal)")
    ap.add_argument("--sweeps", type=int, default=10)
    ap.add_argument("--tuning-cache", default=os.path.join(ROOT, "paper_2503_20566_amd", "tuning.json"),
                    help="JSON cache of peps_autotune results (read; a new key is measured and written)")
    ap.add_argument("--no-tune", action="store_true", help="keep the handle's default tuning")
    ap.add_argument("--no-chains", action="store_true",
                    help="skip the E/site check on |Psi|^2-sampled chains (an untimed strip-sampler "
                         "run; for profiling runs)")
    ap.add_argument("--plain-sweeps", type=int, default=1)
    ap.add_argument("--matter", action="store_true",
                    help="only time the Z2 + hard-core boson workload (16x16, half filling, D = 4, chi = 36): "
                         "--steps batches of amplitude + logderiv + local energy, then --sweeps strip-sampler "
                         "sweeps with plaquette and link moves")
    ap.add_argument("--ragged", action="store_true",
                    help="only time the Z4 study lattices together: one after the other, on concurrent "
                         "streams, and as one ragged batch (--steps repetitions)")
    ap.add_argument("--tvmc", action="store_true",
                    help="only time real-time steps (complex tensors, exact contraction) on the 10x10 "
                         "Z2 string-defect state, 8192 Metropolis-sampled configurations, --steps steps")
    ap.add_argument("--tvmc-d", type=int, default=4, choices=(4, 6),
                    help="bond dimension of the --tvmc state: 4 (default), or 6, the real-time workload's "
                         "tensors, where one sample holds 55 MB of workspace (use --tvmc-batch)")
    ap.add_argument("--tvmc-batch", type=int, default=8192, help="samples of the --tvmc run")
    ap.add_argument("--tvmc-dtype", default="c128", choices=("c128", "c64"),
                    help="contractions of the --tvmc run in complex128 or complex64 (the solve in FP64)")
    ap.add_argument("--tvmc-sweeps", type=int, default=2, help="Metropolis sweeps before the --tvmc steps")
    ap.add_argument("--tvmc-resample", type=int, default=0,
                    help="strip-sampler sweeps of the chains before every timed --tvmc step (timed with it)")
    ap.add_argument("--phase-split", action="store_true",
                    help="only measure the row-sweep kernel's phases (shader clocks per phase) on "
                         "--workload's uniform batch, --dtype path: the amplitude's down sweep and "
                         "the local energy's up sweep")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = 1 << 27                                   # 2^27 doubles = 1 GiB
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 3}))
        return
    if args.sample_chains:
        sample_chains(args.sweeps, args.plain_sweeps)
        return
    if args.tvmc:
        tvmc_run(args.steps, args.tvmc_sweeps, B=args.tvmc_batch, Dk=args.tvmc_d // 2, c64=args.tvmc_dtype == "c64",
                 resample=args.tvmc_resample)
        return
    if args.phase_split:
        print(json.dumps(phase_split(args.workload, args.dtype, args.tuning_cache)), flush=True)
        return
    if args.matter:
        matter_run(args.steps, args.warmup, args.sweeps)
        return
    if args.ragged:
        ragged_run(args.steps)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: every box here has a single MI355X and this "
              "path shards by samples (see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2503_20566_amd import synth

    wl = dict(synth.WORKLOADS[args.workload])
    wl["name"] = args.workload
    # the CPU leg runs first, before this process touches the GPU (its workers are forked)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl)

    import torch
    from paper_2503_20566_amd import gipeps
    L, N, Dk, chi, B = wl["L"], wl["N"], wl["Dk"], wl["chi"], wl["batch"]
    J, h = wl["J"], wl["h"]
    c, e = hamiltonian_tables(wl)
    torch.cuda.set_device(0)
    powers = torch.from_numpy(synth.plaquette_powers(B, L, N)).cuda()

    # fused bonds above 72 (Z4 32 x 32 at chi = 64): the large-bond kernels, with the reverse sweep
    # recomputing each row (no stored tape)
    big = _large_bond(wl)
    keep = 0 if big else args.keep_tape
    if keep < 0:
        probe = gipeps.Peps(L, N, Dk, chi, c, e, ckpt_every=1, keep_tape=True)
        free, _ = torch.cuda.mem_get_info()
        keep = 1 if probe.workspace_bytes(B) < 0.7 * free else 0
        probe.close()

    tuned = {}

    chain_links = None
    if wl.get("sweeps"):
        # the batch as the workload defines it: chains from Philox-drawn plaquette powers after
        # `sweeps` strip-sampler sweeps of the FP64 path (input generation, not timed)
        Pc = gipeps.Peps(L, N, Dk, chi, c, e)
        th_c = torch.from_numpy(synth.theta_normals(Pc.n_params, N * Dk)).cuda()
        _, chain_links = Pc.sample_init(B, synth.SAMPLE_SEED, 0)
        wsc = Pc.workspace(B, gipeps.PEPS_WS_AMPLITUDE | gipeps.PEPS_WS_ENERGY)
        Pc.metropolis_strip(th_c, chain_links, synth.SAMPLE_SEED, 1, wl["sweeps"], wsc)
        torch.cuda.synchronize()
        del wsc, Pc
        print("batch: %d chains after %d strip-sampler sweeps" % (B, wl["sweeps"]), file=sys.stderr, flush=True)

    def make(dtype):
        P = gipeps.Peps(L, N, Dk, chi, c, e, dtype=dtype, ckpt_every=1, keep_tape=bool(keep))
        theta = torch.from_numpy(synth.theta_normals(P.n_params, N * Dk)).cuda()
        links = P.links_from_powers(powers) if chain_links is None else chain_links.clone()
        ws = P.workspace(B)
        if not args.no_tune:
            # row-sweep tuning for this shape and batch (cached, else timed here; not part of a step)
            proj, _, valid = P.project(theta, links)
            r = P.autotune(proj, valid, ws, cache=args.tuning_cache)
            tuned["mixed" if dtype == gipeps.PEPS_F32_MIXED else "f64"] = r
            print("tuning (%s): %s" % (r["source"], r["tuning"]), file=sys.stderr, flush=True)
        return P, theta, links, ws

    def step(P, theta, links, ws, out, marks=None):
        # marks: events recorded between the parts (same stream, no synchronisation)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if marks is not None else None
        if ev:
            ev[0].record()
        proj, bid, valid = P.project(theta, links)
        la, sg = P.amplitude(proj, valid, ws)
        O, _ = P.logderiv(proj, bid, valid, ws)
        if ev:
            ev[1].record()
        el = P.local_energy(theta, links, proj, valid, ws)
        if ev:
            ev[2].record()
        P.sr_build(O, bid, valid, el, ws, mode=gipeps.SR_MATVEC, v=theta)
        if ev:
            ev[3].record()
            marks.append(ev)
        out.update(la=la, el=el, O=O)

    def graph_ms(P, theta, links, ws, steps):
        # the same step captured once as a HIP graph and replayed: no host work per step
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step(P, theta, links, ws, {})
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step(P, theta, links, ws, {})
        g.replay()
        torch.cuda.synchronize()
        print("graph captured and replayed once", file=sys.stderr, flush=True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            g.replay()
        t1.record()
        torch.cuda.synchronize()
        del g
        return t0.elapsed_time(t1) / steps

    def timed(dtype, steps, warmup, profile):
        P, theta, links, ws = make(dtype)
        tag = "mixed" if dtype == gipeps.PEPS_F32_MIXED else "f64"
        out = {}
        for _ in range(warmup):
            step(P, theta, links, ws, out)
        torch.cuda.synchronize()
        print("%s: %d warmup steps done" % (tag, warmup), file=sys.stderr, flush=True)
        for fam in range(6):
            P.profile_read(fam)
        if profile:
            P.profile(True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        marks = []
        t0.record()
        for _ in range(steps):
            step(P, theta, links, ws, out, marks)
        t1.record()
        torch.cuda.synchronize()
        P.profile(False)
        ms = t0.elapsed_time(t1) / steps
        print("%s: %d timed steps, %.1f ms per step" % (tag, steps, ms), file=sys.stderr, flush=True)
        per_step = sorted(m[0].elapsed_time(m[3]) for m in marks)
        parts = {name: sum(m[i].elapsed_time(m[i + 1]) for m in marks) / steps
                 for i, name in enumerate(("project+amplitude+logderiv", "local_energy", "sr_build"))}
        kern = {}
        names = ["project", "row_sweep", "close", "strip", "adjoint", "sr"]
        for fam, name in enumerate(names):
            n, tot = P.profile_read(fam)
            if n:
                kern[name] = {"launches": n, "avg_ms": tot / n, "ms_per_step": tot / steps}
        res = {k: v.double().cpu().numpy() for k, v in out.items() if k in ("la", "el")}
        res["m"] = P.eloc_scale(B, ws).cpu().numpy()
        res["O_max"] = float(out["O"].abs().max().item())
        res["O"] = out["O"]
        if profile:
            res["graph_ms"] = graph_ms(P, theta, links, ws, steps)
            print("%s: graph replay %.1f ms per step" % (tag, res["graph_ms"]), file=sys.stderr, flush=True)
        del P, ws
        torch.cuda.empty_cache()
        res["parts"] = parts
        res["per_step"] = {"median": per_step[len(per_step) // 2] if len(per_step) % 2 else
                           0.5 * (per_step[len(per_step) // 2 - 1] + per_step[len(per_step) // 2]),
                           "min": per_step[0], "max": per_step[-1]}
        return ms, kern, res

    main_dtype = gipeps.PEPS_F32_MIXED if args.dtype == "mixed" else gipeps.PEPS_F64
    other_dtype = gipeps.PEPS_F64 if main_dtype == gipeps.PEPS_F32_MIXED else gipeps.PEPS_F32_MIXED
    ms, kern, res = timed(main_dtype, args.steps, args.warmup, True)
    ms2, _, res2 = timed(other_dtype, max(1, args.steps // 2), 1, False)
    import numpy as np
    mixed_res, f64_res = (res, res2) if main_dtype == gipeps.PEPS_F32_MIXED else (res2, res)
    O_rel = float((mixed_res["O"] - f64_res["O"]).abs().max().item() / f64_res["O_max"])
    errs = precision_figures(L, mixed_res, f64_res, chains=chain_links is not None)
    errs["O_rel_max"] = O_rel
    if big:
        # 10 strip-sampler sweeps of the 1024 chains would add minutes to the run: not drawn here
        errs["sampled_chains"] = None
    elif chain_links is not None:
        # the timed batch is itself the chains: C2 is its plain mean
        ed = float(f64_res["el"].mean()) / L ** 2
        em = float(mixed_res["el"].mean()) / L ** 2
        errs["sampled_chains"] = {"chains": B, "sweeps": wl["sweeps"], "e_site_f64": ed,
                                  "e_site_mixed": em, "e_site_rel": abs(em - ed) / abs(ed),
                                  "c1_delta_max": errs["c1_delta_max"],
                                  "ln_psi_rel_max": errs["ln_psi_rel_max"], "batch": "the timed batch"}
    else:
        errs["sampled_chains"] = None if args.no_chains else sampled_chain_e_site(wl, c, e)
    errs["criteria"] = ("C1: max over the batch of |dE_loc| / M <= 1e-5, M = sum |e[n_l]| + "
                        "sum |c[t] ratio| (FP64 path); C2: |dE/site| / |E/site| <= 1e-5 for the plain "
                        "mean over chains drawn from |Psi|^2; ln|Psi| rel <= 1e-4 per sample")
    errs["met"] = {"ln_psi": errs["ln_psi_rel_max"] <= 1e-4, "C1": errs["c1_delta_max"] <= 1e-5,
                   "C2": None if errs["sampled_chains"] is None else errs["sampled_chains"]["e_site_rel"] <= 1e-5}
    errs["against"] = "FP64 GPU path on the same configurations (itself within 1e-9 of the FP64 oracle in the tests)"

    # roofline of the dominant family: the boundary row sweep (FP64 ALU bound)
    rs = kern.get("row_sweep")
    flops_sample = row_sweep_flops(L, Dk, chi)
    per_launch = flops_sample * B / max(1, L - 2)      # one launch = one row for the whole batch
    achieved = per_launch / (rs["avg_ms"] * 1e-3) / 1e12 if rs else None
    roof = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": (achieved / FP64_VECTOR_PEAK_TFLOPS) if achieved else None,
            "traffic": _row_sweep_traffic(args.workload),
            "kernel": "k_row_sweep (one boundary row for the whole batch per launch)",
            "flops_per_launch": per_launch,
            "matrix_core_flop_share": row_sweep_flops(L, Dk, chi, matrix_core_only=True) / flops_sample,
            "executed": _row_sweep_executed(args.workload, rs["avg_ms"] if rs else None)}
    if not big:
        # where the row sweep's cycles go, from the kernel's own clocks (an untimed extra pass)
        ps = phase_split(args.workload, args.dtype, args.tuning_cache, verbose=False)
        roof["phase_split"] = {"source": "peps_profile_phases, shader clock of each workgroup's first thread",
                               "down_sweep_share": ps["down"]["share"], "up_sweep_share": ps["up"]["share"],
                               "cycles_per_workgroup_row": ps["down"]["cycles_per_workgroup_row"]}

    amp_ms = res["parts"]["project+amplitude+logderiv"]
    out = {
        "metric": "amplitude+dlnPsi samples/s, Z%d %dx%d D=%d chi=%d: FP32 vs FP64 at stated rel err"
                  % (N, L, L, N * Dk, chi),
        "value": B / (amp_ms * 1e-3),
        "value_basis": "B / the project + amplitude + logderiv part of each timed step (HIP events "
                       "between the calls, on their stream); the whole step's rate is step_samples_per_s",
        "step_samples_per_s": B / (ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "step_ms_median_min_max": [res["per_step"]["median"], res["per_step"]["min"], res["per_step"]["max"]],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_dtype == gipeps.PEPS_F32_MIXED else "f64",
        "data": ("synthetic: i.i.d. N(0,1)/D tensor entries (seed %d), uniform plaquette powers (seed %d)"
                 % (synth.THETA_SEED, synth.SAMPLE_SEED)) if chain_links is None else
                ("synthetic: i.i.d. N(0,1)/D tensor entries (seed %d); chains from Philox plaquette powers "
                 "(seed %d) after %d strip-sampler sweeps" % (synth.THETA_SEED, synth.SAMPLE_SEED, wl["sweeps"])),
        "config": {"workload": args.workload, "L": L, "N": N, "D": N * Dk, "Dk": Dk, "chi": chi,
                   "batch": B, "J": J, "h": h, "ckpt_every": 1, "keep_tape": bool(keep),
                   "step": "project + amplitude + logderiv + local_energy + sr_build(S*v)"},
        "other_path": {"dtype": "f64" if other_dtype == gipeps.PEPS_F64 else "f32+f64",
                       "value": B / (res2["parts"]["project+amplitude+logderiv"] * 1e-3),
                       "step_samples_per_s": B / (ms2 * 1e-3), "ms_per_step": ms2},
        # the step's parts (events between the calls inside the timed steps): amplitude + dlnPsi
        # alone (project, amplitude, logderiv) and the local energy and SR build beside it
        "parts_ms_per_step": res["parts"],
        "graph_replay": {"ms_per_step": res["graph_ms"], "samples_per_s": B / (res["graph_ms"] * 1e-3),
                         "note": "the same step captured once as a HIP graph, replayed after the timed steps"},
        "mixed_vs_f64": errs,
        "kernels": kern,
        "tuning": {k: {"chosen": v["tuning"], "source": v["source"],
                       "candidates_ms": [[x["jacobi_lanes"], x["precond"], x["precond_min"], x["small_waves"],
                                          "up" if x["up"] else "down", round(x["ms"], 2)]
                                         for x in v["candidates"]]} for k, v in tuned.items()},
        "roofline": roof,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
