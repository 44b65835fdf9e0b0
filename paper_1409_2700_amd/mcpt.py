"""Thin ctypes binding of libmcpt (include/mcpt.h): argument marshalling only.

Every step of the solve runs inside the HIP library; this module only lays out
the arguments.  Importing it fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MCPT_LIBRARY", os.path.join(_HERE, "libmcpt.so"))

MCPT_OK = 0
MCPT_PENDING = 1
MCPT_ERR_INVALID = -1
MCPT_ERR_NOMEM = -2
MCPT_ERR_DEVICE = -3
MCPT_ERR_NOT_CONVERGED = -4
MCPT_ERR_DIVERGED = -5
MCPT_ERR_NONFINITE = -6
MCPT_ERR_ADMISSION = -7
MCPT_ERR_UNKNOWN_ID = -8

MCPT_FP64, MCPT_FP32, MCPT_BF16 = 0, 1, 2
MCPT_HOST, MCPT_DEVICE = 0, 1
MCPT_SERVE_BATCH_END, MCPT_SERVE_RETIRE_AT_TICKS, MCPT_SERVE_JOIN_AT_TICKS = 0, 1, 2

STATUS_NAMES = {
    0: "MCPT_OK", 1: "MCPT_PENDING", -1: "MCPT_ERR_INVALID", -2: "MCPT_ERR_NOMEM",
    -3: "MCPT_ERR_DEVICE", -4: "MCPT_ERR_NOT_CONVERGED", -5: "MCPT_ERR_DIVERGED",
    -6: "MCPT_ERR_NONFINITE", -7: "MCPT_ERR_ADMISSION", -8: "MCPT_ERR_UNKNOWN_ID",
}

# every symbol include/mcpt.h declares
EXPORTS = [
    "mcpt_create", "mcpt_destroy", "mcpt_last_error", "mcpt_set_stream", "mcpt_upload", "mcpt_run",
    "mcpt_solve", "mcpt_energy", "mcpt_release", "mcpt_set_timing", "mcpt_timing_read",
    "mcpt_upload_batch", "mcpt_solve_batch", "mcpt_cluster_results",
    "mcpt_serve_config", "mcpt_submit", "mcpt_poll", "mcpt_wait", "mcpt_serve_stats",
    "mcpt_autotune", "mcpt_tune_export", "mcpt_tune_import", "mcpt_singles", "mcpt_singles_result",
    "mcpt_lccd_attach", "mcpt_upload_scaled", "mcpt_fd_stencil", "mcpt_dimer_attach",
    "mcpt_run_static", "mcpt_dimer_tau", "mcpt_device_rates", "mcpt_serve_staging",
    "mcpt_serve_tick_mode",
]


class mcpt_problem(C.Structure):
    _fields_ = [
        ("n_mono", C.c_int32), ("n_occ", C.c_void_p), ("n_vir", C.c_void_p), ("eps", C.c_void_p),
        ("k_intra", C.c_void_p), ("n_pair", C.c_int64), ("pair", C.c_void_p), ("v_dimer", C.c_void_p),
        ("memory", C.c_int32),
    ]


class mcpt_options(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_sweeps", C.c_int32), ("precision", C.c_int32),
        ("polish", C.c_int32), ("deterministic", C.c_int32), ("check_every", C.c_int32),
        ("inner_sweeps", C.c_int32), ("warm_t", C.c_void_p), ("graph", C.c_int32), ("autotune", C.c_int32),
    ]


class mcpt_summary(C.Structure):
    _fields_ = [
        ("e_total", C.c_double), ("e_mono", C.c_double), ("e_dimer", C.c_double),
        ("e_mono0", C.c_double), ("residual", C.c_double), ("seconds", C.c_double),
        ("sweeps", C.c_int32), ("polish_sweeps", C.c_int32), ("status", C.c_int32),
        ("iso_sweeps", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class mcpt_timing(C.Structure):
    _fields_ = [
        ("pair_ms", C.c_double), ("mono_ms", C.c_double), ("pair_launches", C.c_int64),
        ("mono_launches", C.c_int64), ("pair_flops", C.c_double), ("pair_v_bytes", C.c_double),
        ("lowp_ms", C.c_double), ("lowp_launches", C.c_int64), ("lowp_flops", C.c_double),
        ("lowp_v_bytes", C.c_double), ("singles_ms", C.c_double), ("singles_launches", C.c_int64),
        ("singles_v_bytes", C.c_double), ("lccd_ring_ms", C.c_double), ("lccd_ladder_ms", C.c_double),
        ("lccd_launches", C.c_int64), ("lccd_w_bytes", C.c_double), ("lccd_ladder_flops", C.c_double),
        ("dimer_ladder_ms", C.c_double), ("dimer_ring_ms", C.c_double), ("dimer_launches", C.c_int64),
        ("dimer_w_bytes", C.c_double), ("dimer_ladder_flops", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class mcpt_rates(C.Structure):
    _fields_ = [("mfma_f64_tflops", C.c_double), ("valu_f64_tflops", C.c_double), ("clock_ghz", C.c_double),
                ("compute_units", C.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def device_rates(device: int = 0) -> dict:
    """mcpt_device_rates: sustained FP64 MFMA and VALU rates and the shader clock."""
    r = mcpt_rates()
    _check(lib().mcpt_device_rates(device, C.byref(r)))
    return r.as_dict()


class mcpt_lccd_integrals(C.Structure):
    _fields_ = [("w_vvvv", C.c_void_p), ("q_oooo", C.c_void_p), ("j_oovv", C.c_void_p), ("memory", C.c_int32)]


class mcpt_dimer_integrals(C.Structure):
    _fields_ = [("w_vvvv", C.c_void_p), ("q_oooo", C.c_void_p), ("c_x", C.c_void_p), ("c_y", C.c_void_p),
                ("memory", C.c_int32)]


class mcpt_fd_mode(C.Structure):
    _fields_ = [("n_pair", C.c_int64), ("pair", C.c_void_p), ("scale", C.c_void_p)]


class mcpt_fd_result(C.Structure):
    _fields_ = [("e", C.c_double * 5), ("d2e", C.c_double), ("sweeps", C.c_int32 * 5), ("status", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {"e": list(self.e), "d2e": self.d2e, "sweeps": list(self.sweeps), "status": self.status}


class mcpt_singles_summary(C.Structure):
    _fields_ = [
        ("e_m1", C.c_double), ("e_m1_0", C.c_double), ("residual", C.c_double), ("seconds", C.c_double),
        ("sweeps", C.c_int32), ("status", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class mcpt_serve_counters(C.Structure):
    _fields_ = [
        ("completed", C.c_uint64), ("batches", C.c_uint64), ("budget", C.c_uint64),
        ("bytes_in_use", C.c_uint64), ("bytes_reserved", C.c_uint64), ("queued", C.c_int32),
        ("running_batches", C.c_int32), ("workers", C.c_int32), ("tickets", C.c_int32),
        ("staging_pinned_bytes", C.c_uint64), ("staged_pageable", C.c_uint64),
        ("joined_at_ticks", C.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class mcpt_tune_result(C.Structure):
    _fields_ = [
        ("n_variants", C.c_int32), ("best", C.c_int32), ("sb", C.c_int32 * 16), ("nw", C.c_int32 * 16),
        ("pd", C.c_int32 * 16), ("reserved", C.c_int32), ("ms", C.c_double * 16),
    ]

    def as_dict(self) -> dict:
        n = self.n_variants
        return {"best": self.best, "variants": [{"sb": self.sb[k], "nw": self.nw[k], "pd": self.pd[k],
                                                 "ms": self.ms[k]} for k in range(n)]}


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libmcpt.so is not built ({path}); run __graft_entry__.build() first")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.mcpt_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(P)]
    lib.mcpt_destroy.argtypes = [P]
    lib.mcpt_destroy.restype = None
    lib.mcpt_last_error.restype = C.c_char_p
    lib.mcpt_set_stream.argtypes = [P, P]
    lib.mcpt_upload.argtypes = [P, C.POINTER(mcpt_problem), C.POINTER(C.c_uint64)]
    lib.mcpt_run.argtypes = [P, C.c_uint64, C.POINTER(mcpt_options), C.POINTER(mcpt_summary)]
    lib.mcpt_run_static.argtypes = [P, C.c_uint64, C.POINTER(mcpt_options), C.POINTER(mcpt_summary)]
    lib.mcpt_dimer_tau.argtypes = [P, C.c_uint64, P]
    lib.mcpt_device_rates.argtypes = [C.c_int, C.POINTER(mcpt_rates)]
    lib.mcpt_solve.argtypes = [P, C.POINTER(mcpt_problem), C.POINTER(mcpt_options),
                               C.POINTER(C.c_uint64), C.POINTER(mcpt_summary)]
    lib.mcpt_energy.argtypes = [P, C.c_uint64, P, P, P, P]
    lib.mcpt_release.argtypes = [P, C.c_uint64]
    lib.mcpt_set_timing.argtypes = [P, C.c_int]
    lib.mcpt_timing_read.argtypes = [P, C.POINTER(mcpt_timing)]
    lib.mcpt_upload_batch.argtypes = [P, C.POINTER(mcpt_problem), C.c_int32, C.POINTER(C.c_uint64)]
    lib.mcpt_solve_batch.argtypes = [P, C.POINTER(mcpt_problem), C.c_int32, C.POINTER(mcpt_options),
                                     C.POINTER(C.c_uint64), C.POINTER(mcpt_summary)]
    lib.mcpt_cluster_results.argtypes = [P, C.c_uint64, C.c_int32, C.POINTER(mcpt_summary)]
    lib.mcpt_serve_config.argtypes = [P, C.c_int32, C.c_int32, C.c_int64]
    lib.mcpt_serve_staging.argtypes = [P, C.c_uint64]
    lib.mcpt_serve_tick_mode.argtypes = [P, C.c_int32]
    lib.mcpt_submit.argtypes = [P, C.POINTER(mcpt_problem), C.POINTER(mcpt_options), C.POINTER(C.c_uint64)]
    lib.mcpt_poll.argtypes = [P, C.c_uint64, C.POINTER(mcpt_summary)]
    lib.mcpt_wait.argtypes = [P, C.c_uint64, C.c_int32, C.POINTER(mcpt_summary)]
    lib.mcpt_serve_stats.argtypes = [P, C.POINTER(mcpt_serve_counters)]
    lib.mcpt_autotune.argtypes = [P, C.c_uint64, C.c_int32, C.POINTER(mcpt_tune_result)]
    lib.mcpt_tune_export.argtypes = [P, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.mcpt_tune_import.argtypes = [P, C.c_char_p]
    lib.mcpt_singles.argtypes = [P, C.c_uint64, P, C.c_int32, C.POINTER(mcpt_options),
                                 C.POINTER(mcpt_singles_summary)]
    lib.mcpt_singles_result.argtypes = [P, C.c_uint64, P, P]
    lib.mcpt_lccd_attach.argtypes = [P, C.c_uint64, C.POINTER(mcpt_lccd_integrals)]
    lib.mcpt_dimer_attach.argtypes = [P, C.c_uint64, C.POINTER(mcpt_dimer_integrals)]
    lib.mcpt_upload_scaled.argtypes = [P, C.c_uint64, C.c_int64, P, P, C.POINTER(C.c_uint64)]
    lib.mcpt_fd_stencil.argtypes = [P, C.c_uint64, C.c_int32, C.POINTER(mcpt_fd_mode), C.c_int32, P, C.c_double, P,
                                    C.POINTER(mcpt_options), C.POINTER(mcpt_fd_result)]
    for name in EXPORTS:
        fn = getattr(lib, name)
        if name not in ("mcpt_destroy", "mcpt_last_error"):
            fn.restype = C.c_int
    return lib


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


class MCPTError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(status: int, allow=()) -> int:
    if status != MCPT_OK and status not in allow:
        raise MCPTError(status, lib().mcpt_last_error().decode())
    return status


def last_error() -> str:
    return lib().mcpt_last_error().decode()


class HostProblem:
    """Keeps the host arrays of a problem alive and exposes an mcpt_problem."""

    def __init__(self, prob):
        self.n_occ = np.ascontiguousarray(prob.n_occ, dtype=np.int32)
        self.n_vir = np.ascontiguousarray(prob.n_vir, dtype=np.int32)
        self.eps = np.ascontiguousarray(prob.eps, dtype=np.float64)
        self.k = np.ascontiguousarray(prob.k, dtype=np.float64)
        self.pairs = np.ascontiguousarray(prob.pairs, dtype=np.int32).reshape(-1, 2)
        self.v = np.ascontiguousarray(prob.v, dtype=np.float64)
        self.c = mcpt_problem(
            n_mono=len(self.n_occ), n_occ=_ptr(self.n_occ), n_vir=_ptr(self.n_vir), eps=_ptr(self.eps),
            k_intra=_ptr(self.k), n_pair=len(self.pairs), pair=_ptr(self.pairs), v_dimer=_ptr(self.v),
            memory=MCPT_HOST)


def make_options(tol=1e-10, max_sweeps=200, precision=MCPT_FP64, polish=1, deterministic=0,
                 check_every=1, inner_sweeps=0, warm_t: np.ndarray | None = None, graph=0, autotune=0):
    o = mcpt_options(tol=tol, max_sweeps=max_sweeps, precision=precision, polish=polish,
                     deterministic=deterministic, check_every=check_every, inner_sweeps=inner_sweeps,
                     warm_t=_ptr(warm_t), graph=graph, autotune=autotune)
    o._keep = warm_t
    return o


class Context:
    """One device context (mcpt_create / mcpt_destroy)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = C.c_void_p()
        _check(lib().mcpt_create(device, hbm_budget, C.byref(h)))
        self.h = h
        self._sizes = {}
        self._clusters = {}
        self._pairs = {}      # pair list (monomer indices) of each resident problem

    def close(self):
        if self.h:
            lib().mcpt_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_handle: int | None):
        _check(lib().mcpt_set_stream(self.h, stream_handle))

    def upload(self, prob) -> int:
        hp = prob if isinstance(prob, HostProblem) else HostProblem(prob)
        pid = C.c_uint64()
        _check(lib().mcpt_upload(self.h, C.byref(hp.c), C.byref(pid)))
        self._sizes[pid.value] = (hp.n_occ.copy(), hp.n_vir.copy(), len(hp.pairs))
        self._pairs[pid.value] = np.asarray(hp.pairs).reshape(-1, 2).copy()
        return pid.value

    def upload_batch(self, probs) -> int:
        """Several independent clusters as one resident batch (mcpt_upload_batch)."""
        hps = [p if isinstance(p, HostProblem) else HostProblem(p) for p in probs]
        arr = (mcpt_problem * len(hps))(*[hp.c for hp in hps])
        pid = C.c_uint64()
        _check(lib().mcpt_upload_batch(self.h, arr, len(hps), C.byref(pid)))
        n_occ = np.concatenate([hp.n_occ for hp in hps])
        n_vir = np.concatenate([hp.n_vir for hp in hps])
        self._sizes[pid.value] = (n_occ, n_vir, int(sum(len(hp.pairs) for hp in hps)))
        self._clusters[pid.value] = [(len(hp.n_occ), len(hp.pairs)) for hp in hps]
        offs = np.concatenate([[0], np.cumsum([len(hp.n_occ) for hp in hps])])
        self._pairs[pid.value] = np.concatenate([np.asarray(hp.pairs).reshape(-1, 2) + offs[q]
                                                 for q, hp in enumerate(hps)] or [np.zeros((0, 2), np.int32)])
        return pid.value

    def cluster_results(self, pid: int) -> list:
        n = len(self._clusters.get(pid, [None]))
        out = (mcpt_summary * n)()
        _check(lib().mcpt_cluster_results(self.h, pid, n, out))
        return [s.as_dict() for s in out]

    def cluster_slices(self, pid: int):
        """(monomer slice, pair slice) of each cluster in the concatenated arrays."""
        out, m0, p0 = [], 0, 0
        for nm, np_ in self._clusters.get(pid, [(len(self._sizes[pid][0]), self._sizes[pid][2])]):
            out.append((slice(m0, m0 + nm), slice(p0, p0 + np_)))
            m0 += nm
            p0 += np_
        return out

    def upload_device(self, n_occ, n_vir, pairs, eps_ptr: int, k_ptr: int, v_ptr: int) -> int:
        """Upload from device buffers (e.g. torch tensors' data_ptr()); sizes and pairs on the host."""
        n_occ = np.ascontiguousarray(n_occ, dtype=np.int32)
        n_vir = np.ascontiguousarray(n_vir, dtype=np.int32)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        c = mcpt_problem(n_mono=len(n_occ), n_occ=_ptr(n_occ), n_vir=_ptr(n_vir), eps=eps_ptr,
                         k_intra=k_ptr, n_pair=len(pairs), pair=_ptr(pairs), v_dimer=v_ptr,
                         memory=MCPT_DEVICE)
        pid = C.c_uint64()
        _check(lib().mcpt_upload(self.h, C.byref(c), C.byref(pid)))
        self._sizes[pid.value] = (n_occ.copy(), n_vir.copy(), len(pairs))
        self._pairs[pid.value] = pairs.copy()
        return pid.value

    def run(self, pid: int, raise_on_error: bool = True, **opts) -> dict:
        o = make_options(**opts)
        s = mcpt_summary()
        st = lib().mcpt_run(self.h, pid, C.byref(o), C.byref(s))
        if raise_on_error:
            _check(st)
        d = s.as_dict()
        d["return"] = st
        return d

    def run_static(self, pid: int, raise_on_error: bool = True, **opts) -> dict:
        """mcpt_run_static: the FP64 eager solve with the library's fixed Tau scratch."""
        o = make_options(**opts)
        s = mcpt_summary()
        st = lib().mcpt_run_static(self.h, pid, C.byref(o), C.byref(s))
        if raise_on_error:
            _check(st)
        d = s.as_dict()
        d["return"] = st
        return d

    def solve(self, prob, raise_on_error: bool = True, **opts):
        pid = self.upload(prob)
        return pid, self.run(pid, raise_on_error=raise_on_error, **opts)

    def energy(self, pid: int, want_t: bool = True) -> dict:
        if pid not in self._sizes:
            raise MCPTError(MCPT_ERR_UNKNOWN_ID, f"unknown problem id or ticket {pid}")
        n_occ, n_vir, n_pair = self._sizes[pid]
        N = len(n_occ)
        e_m2 = np.empty(N)
        de_m2 = np.empty(N)
        e_d2 = np.empty(max(n_pair, 1))
        nt = int(np.sum((n_occ.astype(np.int64) * n_vir) ** 2))
        t = np.empty(nt) if want_t else None
        _check(lib().mcpt_energy(self.h, pid, _ptr(e_m2), _ptr(de_m2), _ptr(e_d2), _ptr(t)))
        out = {"e_m2": e_m2, "de_m2": de_m2, "e_d2": e_d2[:n_pair]}
        if want_t:
            out["t"] = t
        return out

    # ---- singles (mcpt_singles / mcpt_singles_result) ----
    def singles(self, pid: int, w, raise_on_error: bool = True, tol=1e-10, max_sweeps=500, check_every=1,
                device_ptr: int | None = None) -> dict:
        """Singles of a resident problem from the source w (host array of
        sum_X o_X v_X values, or device_ptr of such a device buffer)."""
        o = make_options(tol=tol, max_sweeps=max_sweeps, check_every=check_every)
        s = mcpt_singles_summary()
        if device_ptr is not None:
            st = lib().mcpt_singles(self.h, pid, device_ptr, MCPT_DEVICE, C.byref(o), C.byref(s))
        else:
            wa = np.ascontiguousarray(w, dtype=np.float64)
            st = lib().mcpt_singles(self.h, pid, _ptr(wa), MCPT_HOST, C.byref(o), C.byref(s))
        if raise_on_error:
            _check(st)
        d = s.as_dict()
        d["return"] = st
        return d

    def singles_result(self, pid: int) -> dict:
        if pid not in self._sizes:
            raise MCPTError(MCPT_ERR_UNKNOWN_ID, f"unknown problem id {pid}")
        n_occ, n_vir, _ = self._sizes[pid]
        e = np.empty(len(n_occ))
        t = np.empty(int(np.sum(n_occ.astype(np.int64) * n_vir)))
        _check(lib().mcpt_singles_result(self.h, pid, _ptr(e), _ptr(t)))
        return {"e_m1": e, "t1": t}

    # ---- full monomer equation (mcpt_lccd_attach) ----
    def lccd_attach(self, pid: int, ints, device_ptrs: tuple | None = None):
        """Attach the intramonomer integrals (an object with flat w, q, j arrays,
        or device_ptrs = (w, q, j) of device buffers); ints None detaches."""
        if ints is None and device_ptrs is None:
            _check(lib().mcpt_lccd_attach(self.h, pid, None))
            return
        if device_ptrs is not None:
            li = mcpt_lccd_integrals(device_ptrs[0], device_ptrs[1], device_ptrs[2], MCPT_DEVICE)
            _check(lib().mcpt_lccd_attach(self.h, pid, C.byref(li)))
            return
        w = np.ascontiguousarray(ints.w, dtype=np.float64)
        q = np.ascontiguousarray(ints.q, dtype=np.float64)
        j = np.ascontiguousarray(ints.j, dtype=np.float64)
        li = mcpt_lccd_integrals(_ptr(w), _ptr(q), _ptr(j), MCPT_HOST)
        _check(lib().mcpt_lccd_attach(self.h, pid, C.byref(li)))

    # ---- dimer-internal terms (mcpt_dimer_attach) ----
    def dimer_attach(self, pid: int, dints, device_ptrs: tuple | None = None):
        """Attach the dimer classes of Eq. 59 (an object with flat w, q, cx, cy
        arrays, or device_ptrs = (w, q, cx, cy) of device buffers); dints None detaches."""
        if dints is None and device_ptrs is None:
            _check(lib().mcpt_dimer_attach(self.h, pid, None))
            return
        if device_ptrs is not None:
            di = mcpt_dimer_integrals(*device_ptrs, MCPT_DEVICE)
            _check(lib().mcpt_dimer_attach(self.h, pid, C.byref(di)))
            return
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (dints.w, dints.q, dints.cx, dints.cy)]
        di = mcpt_dimer_integrals(*[_ptr(a) for a in arrs], MCPT_HOST)
        _check(lib().mcpt_dimer_attach(self.h, pid, C.byref(di)))

    def dimer_tau(self, pid: int) -> np.ndarray:
        """Tau of every pair (mcpt_dimer_tau), flat in the caller's pair order: pair p
        contributes Tau_XY[i][a][j][b], oX vX oY vY values."""
        n_occ, n_vir, _ = self._sizes[pid]
        pairs = self._pairs[pid]
        nx = np.asarray(n_occ, dtype=np.int64) * np.asarray(n_vir, dtype=np.int64)
        tau = np.empty(int(np.sum(nx[pairs[:, 0]] * nx[pairs[:, 1]])) if len(pairs) else 0)
        _check(lib().mcpt_dimer_tau(self.h, pid, _ptr(tau)))
        return tau

    # ---- finite-displacement geometries (mcpt_upload_scaled / mcpt_fd_stencil) ----
    def upload_scaled(self, base: int, pairs, scale) -> int:
        """Resident copy of `base` with the listed pair blocks scaled."""
        pa = np.ascontiguousarray(pairs, dtype=np.int64)
        sa = np.ascontiguousarray(scale, dtype=np.float64)
        pid = C.c_uint64()
        _check(lib().mcpt_upload_scaled(self.h, base, len(pa), _ptr(pa), _ptr(sa), C.byref(pid)))
        self._sizes[pid.value] = self._sizes[base]
        if base in self._pairs:
            self._pairs[pid.value] = self._pairs[base]
        if base in self._clusters:
            self._clusters[pid.value] = self._clusters[base]
        return pid.value

    def fd_stencil(self, base: int, modes, cell, step: float, w=None, **opts) -> list:
        """modes: list of (pair indices, scale array [4][n]) for -2h, -h, +h, +2h;
        cell: unit-cell monomer indices.  Returns one result dict per mode."""
        keep = []
        arr = (mcpt_fd_mode * len(modes))()
        for m, (pairs, scale) in enumerate(modes):
            pa = np.ascontiguousarray(pairs, dtype=np.int64)
            sa = np.ascontiguousarray(scale, dtype=np.float64).reshape(4, len(pa))
            keep += [pa, sa]
            arr[m] = mcpt_fd_mode(len(pa), _ptr(pa), _ptr(sa))
        ca = np.ascontiguousarray(cell, dtype=np.int32)
        wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        o = make_options(**opts)
        res = (mcpt_fd_result * len(modes))()
        _check(lib().mcpt_fd_stencil(self.h, base, len(modes), arr, len(ca), _ptr(ca), float(step), _ptr(wa),
                                     C.byref(o), res))
        return [r.as_dict() for r in res]

    def release(self, pid: int):
        _check(lib().mcpt_release(self.h, pid))
        self._sizes.pop(pid, None)
        self._pairs.pop(pid, None)

    def set_timing(self, on: bool):
        _check(lib().mcpt_set_timing(self.h, 1 if on else 0))

    def timing(self) -> dict:
        t = mcpt_timing()
        _check(lib().mcpt_timing_read(self.h, C.byref(t)))
        return t.as_dict()

    # ---- tile autotuner ----
    def autotune(self, pid: int, precision: int) -> dict:
        r = mcpt_tune_result()
        _check(lib().mcpt_autotune(self.h, pid, precision, C.byref(r)))
        return r.as_dict()

    def tune_table(self) -> str:
        n = C.c_size_t()
        _check(lib().mcpt_tune_export(self.h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().mcpt_tune_export(self.h, buf, n.value, C.byref(n)))
        return buf.value.decode()

    def load_tune_table(self, text: str):
        _check(lib().mcpt_tune_import(self.h, text.encode()))

    # ---- serving (mcpt_submit / mcpt_poll) ----
    def serve_config(self, workers: int = 4, max_batch: int = 32, max_batch_pairs: int = 1 << 20):
        _check(lib().mcpt_serve_config(self.h, workers, max_batch, max_batch_pairs))

    def serve_staging(self, nbytes: int):
        """mcpt_serve_staging: cap of the pinned host staging of submitted requests."""
        _check(lib().mcpt_serve_staging(self.h, nbytes))

    def serve_tick_mode(self, mode: int):
        """mcpt_serve_tick_mode: MCPT_SERVE_BATCH_END, MCPT_SERVE_RETIRE_AT_TICKS (default) or
        MCPT_SERVE_JOIN_AT_TICKS."""
        _check(lib().mcpt_serve_tick_mode(self.h, mode))

    def submit(self, prob, **opts) -> int:
        """Queue one solve; returns its ticket (usable with energy / release once done)."""
        hp = prob if isinstance(prob, HostProblem) else HostProblem(prob)
        o = make_options(**opts)
        t = C.c_uint64()
        _check(lib().mcpt_submit(self.h, C.byref(hp.c), C.byref(o), C.byref(t)))
        self._sizes[t.value] = (hp.n_occ.copy(), hp.n_vir.copy(), len(hp.pairs))
        return t.value

    def _finished(self, st: int, s: mcpt_summary):
        if st == MCPT_PENDING:
            return None
        _check(st)
        d = s.as_dict()
        d["error"] = last_error() if d["status"] != MCPT_OK else ""
        return d

    def poll(self, ticket: int):
        """None while queued or running, else the request's summary (seconds = latency)."""
        s = mcpt_summary()
        return self._finished(lib().mcpt_poll(self.h, ticket, C.byref(s)), s)

    def wait(self, ticket: int, timeout_ms: int = -1):
        s = mcpt_summary()
        return self._finished(lib().mcpt_wait(self.h, ticket, timeout_ms, C.byref(s)), s)

    def serve_stats(self) -> dict:
        s = mcpt_serve_counters()
        _check(lib().mcpt_serve_stats(self.h, C.byref(s)))
        return s.as_dict()


def split_t(t_flat: np.ndarray, n_occ, n_vir):
    """Per-monomer views T_X[i, j, a, b] of the t_amp array of mcpt_energy."""
    out, off = [], 0
    for o, v in zip(n_occ, n_vir):
        o, v = int(o), int(v)
        sz = o * o * v * v
        out.append(t_flat[off:off + sz].reshape(o, o, v, v))
        off += sz
    return out
