"""Thin ctypes binding of libgipeps.so (the C ABI in include/gipeps.h).

Argument marshalling only: every step of the hot path runs in the library's HIP kernels.  Device
buffers are torch tensors on the current CUDA (HIP) device; calls are enqueued on torch's
current stream.  The binding raises if the library is missing: there is no CPU fallback.
"""
import ctypes
import json
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgipeps.so")

PEPS_OK, PEPS_ERR_ARG, PEPS_ERR_UNSUPPORTED, PEPS_ERR_WORKSPACE, PEPS_ERR_HIP, PEPS_ERR_STATE = range(6)
PEPS_F64, PEPS_F32_MIXED, PEPS_C128_EXACT, PEPS_C64_EXACT = 0, 1, 2, 3
PEPS_WS_AMPLITUDE, PEPS_WS_ENERGY, PEPS_WS_LOGDERIV, PEPS_WS_SAMPLE, PEPS_WS_TVMC = 1, 2, 4, 8, 16
TVMC_WEIGHT_UNIFORM, TVMC_WEIGHT_PSI2 = 0, 1
PEPS_FLAG_SVD_NOCONV = 1
SR_MATVEC, SR_DENSE = 0, 1

EXPORTED = ("peps_create", "peps_destroy", "peps_status_string", "peps_param_layout",
            "peps_workspace_bytes", "peps_links_from_powers", "peps_project", "peps_amplitude",
            "peps_local_energy", "peps_logderiv", "sr_build", "peps_profile_enable",
            "peps_profile_read", "peps_sample_init", "peps_metropolis", "peps_metropolis_strip",
            "peps_flags", "sr_solve", "sr_dense_rows", "peps_eloc_scale", "peps_amplitude_noalloc",
            "peps_get_tuning", "peps_set_tuning", "peps_autotune", "peps_matter_links",
            "peps_cx_project", "peps_cx_amplitude", "peps_cx_local_energy", "peps_cx_logderiv",
            "tvmc_rhs", "tvmc_step", "peps_amplitude_ragged", "peps_profile_phases")
PEPS_PRECOND_NONE, PEPS_PRECOND_QR_T, PEPS_PRECOND_SORTED_QR = 0, 1, 2
PEPS_K_PROJECT, PEPS_K_ROW_SWEEP, PEPS_K_CLOSE, PEPS_K_STRIP, PEPS_K_ADJOINT, PEPS_K_SR = range(6)
# phases of the row-sweep kernel (peps_profile_phases)
PHASES = ("X", "QR", "Theta", "precond", "Jacobi", "rest")


class PepsProblem(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("N", ctypes.c_int32), ("deg", ctypes.c_int32 * 8),
                ("chi", ctypes.c_int32), ("Q", ctypes.POINTER(ctypes.c_int8)),
                ("plaq_coef", ctypes.c_double * 8), ("elec", ctypes.c_double * 8),
                ("dtype", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
                ("keep_tape", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("matter", ctypes.c_int32), ("hop", ctypes.c_double), ("mass", ctypes.c_double),
                ("var_sweeps", ctypes.c_int32)]


class PepsTuning(ctypes.Structure):
    _fields_ = [("jacobi_lanes", ctypes.c_int32), ("down_precond", ctypes.c_int32),
                ("up_precond", ctypes.c_int32), ("precond_min", ctypes.c_int32),
                ("small_waves", ctypes.c_int32)]


class PepsTuneResult(ctypes.Structure):
    _fields_ = [("jacobi_lanes", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("precond_min", ctypes.c_int32), ("small_waves", ctypes.c_int32),
                ("up", ctypes.c_int32), ("ms", ctypes.c_double)]


TUNING_FIELDS = [f for f, _ in PepsTuning._fields_]


class PepsError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__("%s failed: status %d (%s)" % (fn, status, msg))
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgipeps.so is not built (run __graft_entry__.build()); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64p, szp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), \
            ctypes.POINTER(ctypes.c_size_t)
        L.peps_status_string.restype = ctypes.c_char_p
        L.peps_status_string.argtypes = [ctypes.c_int]
        L.peps_create.argtypes = [ctypes.POINTER(PepsProblem), ctypes.POINTER(vp)]
        L.peps_destroy.argtypes = [vp]
        L.peps_param_layout.argtypes = [vp, i64p, i64p]
        L.peps_workspace_bytes.argtypes = [vp, i32, ctypes.c_uint32, szp]
        L.peps_links_from_powers.argtypes = [vp, vp, i32, vp, vp]
        L.peps_matter_links.argtypes = [vp, vp, vp, i32, vp, vp]
        L.peps_cx_project.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
        L.peps_cx_amplitude.argtypes = [vp, vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]
        L.peps_cx_local_energy.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, ctypes.c_size_t, vp]
        L.peps_cx_logderiv.argtypes = [vp, vp, vp, i32, vp, vp, ctypes.c_size_t, vp]
        L.tvmc_rhs.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, ctypes.c_double, i32, ctypes.c_double, vp,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_double), vp, ctypes.c_size_t, vp]
        L.tvmc_step.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.c_double, ctypes.c_double, i32, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), vp,
                                ctypes.c_size_t, vp]
        L.peps_project.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
        u64 = ctypes.c_uint64
        L.peps_sample_init.argtypes = [vp, u64, u64, i32, vp, vp, vp]
        L.peps_flags.argtypes = [vp, i32, vp, ctypes.c_size_t, vp, vp]
        L.peps_eloc_scale.argtypes = [vp, i32, vp, ctypes.c_size_t, vp, vp]
        L.peps_get_tuning.argtypes = [vp, ctypes.POINTER(PepsTuning)]
        L.peps_set_tuning.argtypes = [vp, ctypes.POINTER(PepsTuning)]
        L.peps_autotune.argtypes = [vp, vp, vp, i32, vp, ctypes.c_size_t, ctypes.POINTER(PepsTuning),
                                    ctypes.POINTER(PepsTuneResult), i32, ctypes.POINTER(ctypes.c_int32), vp]
        dbl = ctypes.c_double
        L.sr_solve.argtypes = [vp, vp, vp, vp, vp, i32, dbl, i32, dbl, vp, vp, vp,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(dbl), vp,
                               ctypes.c_size_t, vp]
        L.peps_metropolis.argtypes = [vp, vp, u64, u64, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp,
                                      ctypes.c_size_t, vp]
        L.peps_metropolis_strip.argtypes = [vp, vp, u64, u64, i32, i32, i32, vp, vp, vp, vp, vp, vp,
                                            vp, ctypes.c_size_t, vp]
        L.sr_dense_rows.argtypes = [vp, vp, vp, vp, i32, vp, ctypes.c_int64, ctypes.c_int64, vp, vp]
        L.peps_amplitude.argtypes = [vp, vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]
        L.peps_amplitude_noalloc.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.peps_amplitude_ragged.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.peps_local_energy.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, ctypes.c_size_t, vp]
        L.peps_logderiv.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.sr_build.argtypes = [vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.peps_profile_enable.argtypes = [vp, i32]
        L.peps_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]
        L.peps_profile_phases.argtypes = [vp, vp]
        for name in EXPORTED:
            getattr(L, name).restype = ctypes.c_int if name != "peps_status_string" else ctypes.c_char_p
        _lib = L
    return _lib


def _check(fn, status):
    if status != PEPS_OK:
        raise PepsError(fn, status, lib().peps_status_string(status).decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Peps:
    """One problem (lattice, group, sectors, cutoff, Hamiltonian tables) bound to a handle."""

    def __init__(self, L, N, Dk, chi, plaq_coef, elec, Q=None, dtype=PEPS_F64, ckpt_every=0,
                 keep_tape=False, max_sweeps=0, matter=False, hop=0.0, mass=0.0, var_sweeps=0):
        p = PepsProblem()
        p.L, p.N, p.chi, p.dtype, p.ckpt_every = L, N, chi, dtype, ckpt_every
        p.keep_tape = 1 if keep_tape else 0
        p.max_sweeps = max_sweeps
        p.matter, p.hop, p.mass = (1 if matter else 0), float(hop), float(mass)
        p.var_sweeps = var_sweeps
        for k in range(8):
            p.deg[k] = Dk if k < N else 0
            p.plaq_coef[k] = float(plaq_coef[k]) if k < N else 0.0
            p.elec[k] = float(elec[k]) if k < N else 0.0
        self._Q = None
        if Q is not None:
            self._Q = (ctypes.c_int8 * (L * L))(*[int(q) for q in Q.reshape(-1)])
            p.Q = ctypes.cast(self._Q, ctypes.POINTER(ctypes.c_int8))
        self.L, self.N, self.Dk, self.chi = L, N, Dk, chi
        self.dtype, self.keep_tape = dtype, bool(keep_tape)
        self.matter = bool(matter)
        self.planes = 3 if matter else 2   # planes of a configuration (links [, occupations])
        self._h = ctypes.c_void_p()
        _check("peps_create", lib().peps_create(ctypes.byref(p), ctypes.byref(self._h)))
        n = ctypes.c_int64()
        offs = (ctypes.c_int64 * (L * L + 1))()
        _check("peps_param_layout", lib().peps_param_layout(self._h, ctypes.byref(n), offs))
        self.n_params = n.value
        self.site_offset = list(offs)
        self.P4 = Dk ** 4

    def close(self):
        if self._h:
            lib().peps_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- row-sweep tuning ----------------------------------------------------------------------
    def get_tuning(self):
        t = PepsTuning()
        _check("peps_get_tuning", lib().peps_get_tuning(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f in TUNING_FIELDS}

    def set_tuning(self, tuning):
        t = PepsTuning(*[int(tuning[f]) for f in TUNING_FIELDS])
        _check("peps_set_tuning", lib().peps_set_tuning(self._h, ctypes.byref(t)))

    def tuning_key(self, B):
        return "L%d_N%d_Dk%d_chi%d_%s_B%d_tape%d" % (self.L, self.N, self.Dk, self.chi,
                                                    "mixed" if self.dtype == PEPS_F32_MIXED else "f64",
                                                    B, int(self.keep_tape))

    def autotune(self, proj, valid, ws, cache=None):
        """peps_autotune on this batch, or the cached result for the same key (the JSON file at
        `cache`, written here when the key is new).  Returns {"tuning", "candidates", "source"}."""
        B = proj.shape[0]
        key = self.tuning_key(B)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table and set(table[key]["tuning"]) == set(TUNING_FIELDS):
            self.set_tuning(table[key]["tuning"])
            return dict(table[key], source="cache " + os.path.basename(cache))
        best = PepsTuning()
        cap = 64
        res = (PepsTuneResult * cap)()
        n = ctypes.c_int32()
        _check("peps_autotune", lib().peps_autotune(self._h, _ptr(proj), _ptr(valid), B, _ptr(ws), ws.numel(),
                                                    ctypes.byref(best), res, cap, ctypes.byref(n), _stream()))
        entry = {"tuning": {f: getattr(best, f) for f in TUNING_FIELDS},
                 "candidates": [{f: getattr(r, f) for f, _ in PepsTuneResult._fields_}
                                for r in res[:min(n.value, cap)]]}
        if cache:
            table[key] = entry
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(entry, source="measured")

    # -- per-kernel timing -------------------------------------------------------------------
    def profile(self, on=True):
        _check("peps_profile_enable", lib().peps_profile_enable(self._h, 1 if on else 0))

    def profile_phases(self, counters):
        """Row-sweep phase clocks into counters (int64 cuda tensor [len(PHASES)], zeroed by the
        caller; accumulated by every later row-sweep launch), or None to switch them off."""
        if counters is not None:
            assert counters.dtype == torch.int64 and counters.is_cuda and counters.numel() == len(PHASES)
        self._phases = counters  # keep the buffer alive while the library holds its address
        _check("peps_profile_phases", lib().peps_profile_phases(self._h, _ptr(counters) if counters is not None
                                                                else None))

    def profile_read(self, family):
        """(launches, total_ms) of one kernel family since the last read."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check("peps_profile_read", lib().peps_profile_read(self._h, family, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    # -- workspace ------------------------------------------------------------------------
    def workspace_bytes(self, B, what=PEPS_WS_AMPLITUDE | PEPS_WS_ENERGY | PEPS_WS_LOGDERIV):
        n = ctypes.c_size_t()
        _check("peps_workspace_bytes", lib().peps_workspace_bytes(self._h, B, what, ctypes.byref(n)))
        return n.value

    def workspace(self, B, what=PEPS_WS_AMPLITUDE | PEPS_WS_ENERGY | PEPS_WS_LOGDERIV, device="cuda"):
        return torch.empty(max(1, self.workspace_bytes(B, what)), dtype=torch.uint8, device=device)

    # -- hot path ---------------------------------------------------------------------------
    def links_from_powers(self, powers):
        B = powers.shape[0]
        links = torch.empty((B, self.planes, self.L, self.L), dtype=torch.uint8, device=powers.device)
        _check("peps_links_from_powers",
               lib().peps_links_from_powers(self._h, _ptr(powers), B, _ptr(links), _stream()))
        return links

    # -- complex tensors, exact contraction, tVMC (dtype PEPS_C128_EXACT / PEPS_C64_EXACT) ------
    def cx_project(self, theta, links):
        """theta: complex128 [n_params]; returns (proj complex128 [B][L*L][Dk^4], block_id, valid)."""
        assert theta.dtype == torch.complex128
        B = links.shape[0]
        dev = links.device
        proj = torch.empty((B, self.L * self.L, self.P4), dtype=torch.complex128, device=dev)
        bid = torch.empty((B, self.L * self.L), dtype=torch.int32, device=dev)
        valid = torch.empty((B,), dtype=torch.uint8, device=dev)
        _check("peps_cx_project", lib().peps_cx_project(self._h, _ptr(theta), _ptr(links), B, _ptr(proj), _ptr(bid),
                                                        _ptr(valid), _stream()))
        return proj, bid, valid

    def cx_amplitude(self, proj, valid, ws):
        """(ln|Psi| float64 [B], phase Psi/|Psi| complex128 [B]); leaves the row states in ws."""
        B = proj.shape[0]
        la = torch.empty((B,), dtype=torch.float64, device=proj.device)
        ph = torch.empty((B,), dtype=torch.complex128, device=proj.device)
        _check("peps_cx_amplitude", lib().peps_cx_amplitude(self._h, _ptr(proj), _ptr(valid), B, _ptr(la), _ptr(ph),
                                                            _ptr(ws), ws.numel(), _stream()))
        return la, ph

    def cx_local_energy(self, theta, links, proj, valid, ws):
        B = proj.shape[0]
        el = torch.empty((B,), dtype=torch.complex128, device=proj.device)
        _check("peps_cx_local_energy",
               lib().peps_cx_local_energy(self._h, _ptr(theta), _ptr(links), _ptr(proj), _ptr(valid), B, _ptr(el),
                                          _ptr(ws), ws.numel(), _stream()))
        return el

    def cx_logderiv(self, proj, valid, ws):
        B = proj.shape[0]
        O = torch.empty((B, self.L * self.L, self.P4), dtype=torch.complex128, device=proj.device)
        _check("peps_cx_logderiv", lib().peps_cx_logderiv(self._h, _ptr(proj), _ptr(valid), B, _ptr(O), _ptr(ws),
                                                          ws.numel(), _stream()))
        return O

    def tvmc_rhs(self, O, bid, valid, e_loc, log_abs, ws, weights=TVMC_WEIGHT_UNIFORM, shift=1e-4, max_iter=2000,
                 rtol=1e-12):
        """(alphadot complex128 [n_params], <E_loc> complex, CG iterations, relative residual)."""
        B = O.shape[0]
        x = torch.empty((self.n_params,), dtype=torch.complex128, device=O.device)
        en = (ctypes.c_double * 2)()
        it, rel = ctypes.c_int32(), ctypes.c_double()
        _check("tvmc_rhs", lib().tvmc_rhs(self._h, _ptr(O), _ptr(bid), _ptr(valid), _ptr(e_loc), _ptr(log_abs), B,
                                          weights, shift, max_iter, rtol, _ptr(x), en, ctypes.byref(it),
                                          ctypes.byref(rel), _ptr(ws), ws.numel(), _stream()))
        return x, complex(en[0], en[1]), it.value, rel.value

    def tvmc_step(self, theta, links, ws, dt, weights=TVMC_WEIGHT_UNIFORM, order=2, shift=1e-4, max_iter=2000,
                  rtol=1e-12):
        """One step of eq. secondorder, theta (complex128 [n_params]) updated in place; returns
        (<H> at the start of the step, CG iterations of the two stages)."""
        B = links.shape[0]
        en = (ctypes.c_double * 2)()
        its = (ctypes.c_int32 * 2)()
        _check("tvmc_step", lib().tvmc_step(self._h, _ptr(theta), _ptr(links), B, weights, order, dt, shift, max_iter,
                                            rtol, en, its, _ptr(ws), ws.numel(), _stream()))
        return complex(en[0], en[1]), (its[0], its[1])

    def matter_links(self, powers, occupations):
        """Configurations uint8 [B][3][L][L] around the given occupations (uint8 [B][L][L])."""
        B = powers.shape[0]
        assert occupations.shape == (B, self.L, self.L) and occupations.dtype == torch.uint8
        links = torch.empty((B, 3, self.L, self.L), dtype=torch.uint8, device=powers.device)
        _check("peps_matter_links",
               lib().peps_matter_links(self._h, _ptr(powers), _ptr(occupations), B, _ptr(links),
                                       _stream()))
        return links

    def sample_init(self, B, seed, stream_id=0, device="cuda"):
        """Philox-seeded initial chains: (powers uint8 [B][L-1][L-1], links uint8 [B][2][L][L])."""
        powers = torch.empty((B, self.L - 1, self.L - 1), dtype=torch.uint8, device=device)
        links = torch.empty((B, 2, self.L, self.L), dtype=torch.uint8, device=device)
        _check("peps_sample_init", lib().peps_sample_init(self._h, seed, stream_id, B, _ptr(powers),
                                                          _ptr(links), _stream()))
        return powers, links

    def metropolis(self, theta, links, seed, first_sweep, n_sweeps, ws, stream_id=0, accepted=None):
        """Metropolis sweeps of the chains in links (updated in place); returns (log_abs, accepted)."""
        B = links.shape[0]
        dev = links.device
        la = torch.empty((B,), dtype=torch.float64, device=dev)
        if accepted is None:
            accepted = torch.zeros((B,), dtype=torch.int32, device=dev)
        cplx = self.dtype in (PEPS_C128_EXACT, PEPS_C64_EXACT)
        proj = torch.empty((B, self.L * self.L, self.P4), dtype=torch.complex128 if cplx else torch.float64,
                           device=dev)
        bid = torch.empty((B, self.L * self.L), dtype=torch.int32, device=dev)
        valid = torch.empty((B,), dtype=torch.uint8, device=dev)
        _check("peps_metropolis",
               lib().peps_metropolis(self._h, _ptr(theta), seed, stream_id, first_sweep, n_sweeps, B,
                                     _ptr(links), _ptr(la), _ptr(accepted), _ptr(proj), _ptr(bid),
                                     _ptr(valid), _ptr(ws), ws.numel(), _stream()))
        return la, accepted

    def metropolis_strip(self, theta, links, seed, first_sweep, n_sweeps, ws, stream_id=0,
                         accepted=None):
        """The same sweeps with strip ratios and environment reuse (ws sized for PEPS_WS_AMPLITUDE |
        PEPS_WS_ENERGY, or PEPS_WS_AMPLITUDE | PEPS_WS_SAMPLE for a complex handle); links updated in
        place; returns (log_abs of the final states, accepted)."""
        B = links.shape[0]
        dev = links.device
        la = torch.empty((B,), dtype=torch.float64, device=dev)
        if accepted is None:
            accepted = torch.zeros((B,), dtype=torch.int32, device=dev)
        cplx = self.dtype in (PEPS_C128_EXACT, PEPS_C64_EXACT)
        proj = torch.empty((B, self.L * self.L, self.P4), dtype=torch.complex128 if cplx else torch.float64,
                           device=dev)
        bid = torch.empty((B, self.L * self.L), dtype=torch.int32, device=dev)
        valid = torch.empty((B,), dtype=torch.uint8, device=dev)
        _check("peps_metropolis_strip",
               lib().peps_metropolis_strip(self._h, _ptr(theta), seed, stream_id, first_sweep, n_sweeps,
                                           B, _ptr(links), _ptr(la), _ptr(accepted), _ptr(proj),
                                           _ptr(bid), _ptr(valid), _ptr(ws), ws.numel(), _stream()))
        return la, accepted

    def sr_dense_rows(self, O, block_id, valid, O_mean, row0, nrows):
        """Rows [row0, row0 + nrows) of the dense S (float64 [nrows][n_params])."""
        B = O.shape[0]
        S = torch.empty((nrows, self.n_params), dtype=torch.float64, device=O.device)
        _check("sr_dense_rows", lib().sr_dense_rows(self._h, _ptr(O), _ptr(block_id), _ptr(valid), B,
                                                    _ptr(O_mean), row0, nrows, _ptr(S), _stream()))
        return S

    def sr_solve(self, O, block_id, valid, e_loc, ws, shift, max_iter, rtol):
        """(S + shift I) x = F by CG: returns (x, F, O_mean, iterations, relative residual)."""
        B = O.shape[0]
        dev = O.device
        x = torch.empty((self.n_params,), dtype=torch.float64, device=dev)
        F = torch.empty_like(x)
        om = torch.empty_like(x)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        _check("sr_solve", lib().sr_solve(self._h, _ptr(O), _ptr(block_id), _ptr(valid), _ptr(e_loc), B,
                                          float(shift), int(max_iter), float(rtol), _ptr(x), _ptr(F),
                                          _ptr(om), ctypes.byref(it), ctypes.byref(rel), _ptr(ws),
                                          ws.numel(), _stream()))
        return x, F, om, it.value, rel.value

    def flags(self, B, ws):
        """Per-sample PEPS_FLAG_* bits of the sweeps since the last amplitude on ws (uint32 [B])."""
        out = torch.empty((B,), dtype=torch.int32, device=ws.device)
        _check("peps_flags", lib().peps_flags(self._h, B, _ptr(ws), ws.numel(), _ptr(out), _stream()))
        return out

    def eloc_scale(self, B, ws):
        """sum |e[n_l]| + sum |c[t] ratio| of each E_loc of the last local_energy on ws (float64 [B])."""
        out = torch.empty((B,), dtype=torch.float64, device=ws.device)
        _check("peps_eloc_scale", lib().peps_eloc_scale(self._h, B, _ptr(ws), ws.numel(), _ptr(out),
                                                        _stream()))
        return out

    def project(self, theta, links):
        B = links.shape[0]
        dev = links.device
        proj = torch.empty((B, self.L * self.L, self.P4), dtype=torch.float64, device=dev)
        bid = torch.empty((B, self.L * self.L), dtype=torch.int32, device=dev)
        valid = torch.empty((B,), dtype=torch.uint8, device=dev)
        _check("peps_project", lib().peps_project(self._h, _ptr(theta), _ptr(links), B, _ptr(proj),
                                                  _ptr(bid), _ptr(valid), _stream()))
        return proj, bid, valid

    def amplitude(self, proj, valid, ws):
        B = proj.shape[0]
        la = torch.empty((B,), dtype=torch.float64, device=proj.device)
        sg = torch.empty((B,), dtype=torch.float64, device=proj.device)
        _check("peps_amplitude", lib().peps_amplitude(self._h, _ptr(proj), _ptr(valid), B, _ptr(la),
                                                      _ptr(sg), _ptr(ws), ws.numel(), _stream()))
        return la, sg

    def amplitude_noalloc(self, proj, valid, log_abs=None, sign=None):
        """peps_amplitude_noalloc: ln|Psi|, sign without a workspace (outputs may be passed in)."""
        B = proj.shape[0]
        if log_abs is None:
            log_abs = torch.empty((B,), dtype=torch.float64, device=proj.device)
        if sign is None:
            sign = torch.empty((B,), dtype=torch.float64, device=proj.device)
        _check("peps_amplitude_noalloc",
               lib().peps_amplitude_noalloc(self._h, _ptr(proj), _ptr(valid), B, _ptr(log_abs),
                                            _ptr(sign), _stream()))
        return log_abs, sign

    def local_energy(self, theta, links, proj, valid, ws):
        B = proj.shape[0]
        e = torch.empty((B,), dtype=torch.float64, device=proj.device)
        _check("peps_local_energy", lib().peps_local_energy(self._h, _ptr(theta), _ptr(links), _ptr(proj),
                                                            _ptr(valid), B, _ptr(e), _ptr(ws), ws.numel(),
                                                            _stream()))
        return e

    def logderiv(self, proj, block_id, valid, ws, w=None, want_O=True, want_vjp=False):
        B = proj.shape[0]
        dev = proj.device
        O = torch.empty_like(proj) if want_O else None
        vjp = torch.empty((self.n_params,), dtype=torch.float64, device=dev) if want_vjp else None
        _check("peps_logderiv", lib().peps_logderiv(self._h, _ptr(proj), _ptr(block_id), _ptr(valid), B,
                                                    _ptr(w), _ptr(O), _ptr(vjp), _ptr(ws), ws.numel(),
                                                    _stream()))
        return O, vjp

    def sr_build(self, O, block_id, valid, e_loc, ws, mode=SR_MATVEC, v=None):
        B = O.shape[0]
        dev = O.device
        F = torch.empty((self.n_params,), dtype=torch.float64, device=dev)
        om = torch.empty((self.n_params,), dtype=torch.float64, device=dev)
        if mode == SR_DENSE:
            S = torch.empty((self.n_params, self.n_params), dtype=torch.float64, device=dev)
        else:
            S = torch.empty((self.n_params,), dtype=torch.float64, device=dev)
        _check("sr_build", lib().sr_build(self._h, _ptr(O), _ptr(block_id), _ptr(valid), _ptr(e_loc), B,
                                          mode, _ptr(v), _ptr(F), _ptr(om), _ptr(S), _ptr(ws), ws.numel(),
                                          _stream()))
        return F, om, S


def amplitude_ragged(groups):
    """peps_amplitude_ragged over groups [(peps, proj, valid, ws), ...]: ln|Psi| and sign of each
    group's batch, one launch per boundary row for all lattices."""
    n = len(groups)
    vp = ctypes.c_void_p
    hs = (vp * n)(*[g[0]._h.value for g in groups])
    outs = []
    for P, proj, valid, ws in groups:
        B = proj.shape[0]
        outs.append((torch.empty((B,), dtype=torch.float64, device=proj.device),
                     torch.empty((B,), dtype=torch.float64, device=proj.device)))
    arr = lambda xs: (vp * n)(*xs)
    _check("peps_amplitude_ragged", lib().peps_amplitude_ragged(
        n, hs, arr([_ptr(g[1]) for g in groups]), arr([_ptr(g[2]) for g in groups]),
        (ctypes.c_int32 * n)(*[g[1].shape[0] for g in groups]), arr([_ptr(o[0]) for o in outs]),
        arr([_ptr(o[1]) for o in outs]), arr([_ptr(g[3]) for g in groups]),
        (ctypes.c_size_t * n)(*[g[3].numel() for g in groups]), _stream()))
    return outs


class Amplitude(torch.autograd.Function):
    """ln|Psi(s)| of a batch as a differentiable function of theta.

    forward(theta, peps, links, ws) = peps_project + peps_amplitude -> log_abs [B];
    backward(grad) = peps_logderiv with w = grad: theta.grad = sum_b grad_b d ln|Psi_b| / d theta
    (the vjp output).  ws must not be used by another peps_amplitude between the two.
    """

    @staticmethod
    def forward(ctx, theta, peps, links, ws):
        proj, bid, valid = peps.project(theta, links)
        la, _ = peps.amplitude(proj, valid, ws)
        ctx.peps, ctx.ws = peps, ws
        ctx.save_for_backward(proj, bid, valid)
        return la

    @staticmethod
    def backward(ctx, grad):
        proj, bid, valid = ctx.saved_tensors
        w = grad.to(torch.float64).contiguous()
        _, vjp = ctx.peps.logderiv(proj, bid, valid, ctx.ws, w=w, want_O=True, want_vjp=True)
        return vjp, None, None, None
