"""Python binding of the C ABI in include/ldopf.h, with the same call names.

Every function marshals numpy arrays into the C structures and returns the
library's outputs; no step of the method runs in Python. Errors raise
``LdopfError`` carrying the library's code and detail text.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N
from ._native import (LDOPF_BUFFER_TOO_SMALL, LDOPF_DEVICE_ERROR, LDOPF_INCONSISTENT_SUBSYSTEM,  # noqa: F401
                      LDOPF_INVALID_ARGUMENT, LDOPF_NUMERICAL, LDOPF_OUT_OF_MEMORY, LDOPF_UNSUPPORTED,
                      LDOPF_FP32_MIXED, LDOPF_FP64, LDOPF_NOT_CONVERGED, LDOPF_OK,
                      LDOPF_REQ_DONE, LDOPF_REQ_FAILED, LDOPF_REQ_QUEUED, LDOPF_REQ_RUNNING,
                      LDOPF_PATH_AUTO, LDOPF_PATH_PERSISTENT, LDOPF_PATH_STREAMED,
                      LDOPF_RESIDUAL_AGGREGATED, LDOPF_RESIDUAL_PAPER, LDOPF_RHO_BALANCE, LDOPF_RHO_FIXED,
                      ldopf_batch_sizes, ldopf_batch_status,
                      ldopf_options, ldopf_server_stats, ldopf_sizes, ldopf_status)


class LdopfError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = N.lib()
        self.code = code
        self.detail = lib.ldopf_last_error_detail().decode()
        super().__init__(f"{where}: {lib.ldopf_error_string(code).decode()} ({code}): {self.detail}")


def _check(code: int, where: str, allow=(LDOPF_OK,)) -> int:
    if code not in allow:
        raise LdopfError(code, where)
    return code


def _ptr(a, ctype):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


_NET_FIELDS = {
    "bus_phases": np.uint8, "bus_wlo": np.float64, "bus_whi": np.float64, "bus_gsh": np.float64,
    "bus_bsh": np.float64, "line_from": np.int32, "line_to": np.int32, "line_phases": np.uint8,
    "line_r": np.float64, "line_x": np.float64, "line_gs_from": np.float64, "line_bs_from": np.float64,
    "line_gs_to": np.float64, "line_bs_to": np.float64, "line_tau": np.float64, "line_plo": np.float64,
    "line_phi": np.float64, "line_qlo": np.float64, "line_qhi": np.float64, "load_bus": np.int32,
    "load_phases": np.uint8, "load_conn": np.uint8, "load_a": np.float64, "load_b": np.float64,
    "load_alpha": np.float64, "load_beta": np.float64, "gen_bus": np.int32, "gen_phases": np.uint8,
    "gen_plo": np.float64, "gen_phi": np.float64, "gen_qlo": np.float64, "gen_qhi": np.float64,
    "gen_cost_p": np.float64, "gen_cost_q": np.float64,
}
_CT = {np.uint8: C.c_uint8, np.int32: C.c_int32, np.float64: C.c_double}


class Network:
    """ldopf_network over contiguous copies of a network dict (kept alive here)."""

    def __init__(self, net: dict):
        self.keep = {}
        s = N.ldopf_network()
        for k in ("n_bus", "n_line", "n_load", "n_gen", "root"):
            setattr(s, k, int(net[k]))
        for k, dt in _NET_FIELDS.items():
            v = net.get(k)
            if v is None:
                continue
            arr = np.ascontiguousarray(v, dtype=dt)
            self.keep[k] = arr
            setattr(s, k, arr.ctypes.data_as(C.POINTER(_CT[dt])))
        self.struct = s


def ldopf_default_options(**kw) -> ldopf_options:
    o = ldopf_options()
    N.lib().ldopf_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def ldopf_describe_network(net: dict) -> dict:
    """Host-only assembly + decomposition; returns the consensus LP arrays."""
    lib = N.lib()
    nw = Network(net)
    sz = np.zeros(5, dtype=np.int64)
    _check(lib.ldopf_describe_network(C.byref(nw.struct), _ptr(sz, C.c_int64), *([None] * 9)), "ldopf_describe_network")
    n, S, nloc, aw, rows = (int(v) for v in sz)
    out = {"c": np.empty(n), "lo": np.empty(n), "hi": np.empty(n), "x_init": np.empty(n),
           "n_s": np.empty(S, np.int32), "m_s": np.empty(S, np.int32), "A": np.empty(aw), "b": np.empty(rows),
           "gidx": np.empty(nloc, np.int64)}
    _check(lib.ldopf_describe_network(
        C.byref(nw.struct), _ptr(sz, C.c_int64), _ptr(out["c"], C.c_double), _ptr(out["lo"], C.c_double),
        _ptr(out["hi"], C.c_double), _ptr(out["x_init"], C.c_double), _ptr(out["n_s"], C.c_int32),
        _ptr(out["m_s"], C.c_int32), _ptr(out["A"], C.c_double), _ptr(out["b"], C.c_double),
        _ptr(out["gidx"], C.c_int64)), "ldopf_describe_network")
    out["n"] = n
    out["S"] = S
    return out


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(int(stream.cuda_stream))  # a torch.cuda.Stream


class Problem:
    """Owner of one ldopf_problem handle."""

    def __init__(self, handle: C.c_void_p):
        self.h = handle

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may be gone already
            pass

    def close(self):
        if getattr(self, "h", None):
            N.lib().ldopf_destroy(self.h)
            self.h = None

    # -- the calls of the C ABI, same names without the prefix
    def sizes(self) -> ldopf_sizes:
        s = ldopf_sizes()
        _check(N.lib().ldopf_get_sizes(self.h, C.byref(s)), "ldopf_get_sizes")
        return s

    def set_options(self, opts: ldopf_options):
        _check(N.lib().ldopf_set_options(self.h, C.byref(opts)), "ldopf_set_options")

    def solve(self) -> ldopf_status:
        st = ldopf_status()
        code = N.lib().ldopf_solve(self.h, C.byref(st))
        _check(code, "ldopf_solve", allow=(LDOPF_OK, LDOPF_NOT_CONVERGED))
        return st

    def solve_noalloc(self) -> ldopf_status:
        st = ldopf_status()
        code = N.lib().ldopf_solve_noalloc(self.h, C.byref(st))
        _check(code, "ldopf_solve_noalloc", allow=(LDOPF_OK, LDOPF_NOT_CONVERGED))
        return st

    def reset(self):
        _check(N.lib().ldopf_reset(self.h), "ldopf_reset")

    def warm_start(self, xs: np.ndarray, lam: np.ndarray):
        xs = np.ascontiguousarray(xs, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        _check(N.lib().ldopf_warm_start(self.h, _ptr(xs, C.c_double), _ptr(lam, C.c_double), xs.shape[0]),
               "ldopf_warm_start")

    def get_global(self) -> np.ndarray:
        x = np.empty(self.sizes().n)
        _check(N.lib().ldopf_get_global(self.h, _ptr(x, C.c_double), x.shape[0]), "ldopf_get_global")
        return x

    def get_local(self):
        nl = self.sizes().n_local
        xs, lam = np.empty(nl), np.empty(nl)
        _check(N.lib().ldopf_get_local(self.h, _ptr(xs, C.c_double), _ptr(lam, C.c_double), nl), "ldopf_get_local")
        return xs, lam

    def get_structure(self):
        s = self.sizes()
        g = np.empty(s.n_local, np.int64)
        off = np.empty(s.n_sub + 1, np.int64)
        _check(N.lib().ldopf_get_structure(self.h, _ptr(g, C.c_int64), g.shape[0], _ptr(off, C.c_int64), off.shape[0]),
               "ldopf_get_structure")
        return g, off

    def get_history(self) -> np.ndarray:
        ln = C.c_int64(0)
        _check(N.lib().ldopf_get_history(self.h, None, 0, C.byref(ln)), "ldopf_get_history")
        H = np.empty((ln.value, 4))
        _check(N.lib().ldopf_get_history(self.h, _ptr(H, C.c_double), ln.value, C.byref(ln)), "ldopf_get_history")
        return H

    def get_operators(self):
        s = self.sizes()
        ab = np.empty(s.op_words)
        bb = np.empty(s.n_local)
        rk = np.empty(s.n_sub, np.int32)
        _check(N.lib().ldopf_get_operators(self.h, _ptr(ab, C.c_double), ab.shape[0], _ptr(bb, C.c_double),
                                           bb.shape[0], _ptr(rk, C.c_int32), rk.shape[0]), "ldopf_get_operators")
        return ab, bb, rk

    def get_rho_log(self):
        """[(first sweep, rho)] of every change residual balancing made in the last solve."""
        ln = C.c_int64(0)
        _check(N.lib().ldopf_get_rho_log(self.h, None, None, 0, C.byref(ln)), "ldopf_get_rho_log")
        sw = np.empty(ln.value, np.int64)
        rh = np.empty(ln.value)
        _check(N.lib().ldopf_get_rho_log(self.h, _ptr(sw, C.c_int64), _ptr(rh, C.c_double), ln.value, C.byref(ln)),
               "ldopf_get_rho_log")
        return [(int(a), float(b)) for a, b in zip(sw, rh)]

    def get_phase_times(self, part: int = 0) -> np.ndarray:
        """Per-phase ms of workgroup `part` in the last profiled solve."""
        ms = np.zeros(8)
        _check(N.lib().ldopf_get_phase_times_part(self.h, int(part), _ptr(ms, C.c_double)),
               "ldopf_get_phase_times_part")
        return ms

    def objective(self) -> float:
        f = C.c_double(0.0)
        _check(N.lib().ldopf_objective(self.h, C.byref(f)), "ldopf_objective")
        return f.value

    def get_global_device(self, x_device_ptr: int, cap: int):
        _check(N.lib().ldopf_get_global_device(self.h, C.c_void_p(x_device_ptr), cap), "ldopf_get_global_device")

    def get_local_device(self, xs_ptr: int, lam_ptr: int, cap: int):
        _check(N.lib().ldopf_get_local_device(self.h, C.c_void_p(xs_ptr), C.c_void_p(lam_ptr), cap),
               "ldopf_get_local_device")


def ldopf_create(net: dict, opts: ldopf_options | None = None, stream=None) -> Problem:
    """Assemble, decompose, upload and precompute on the GPU."""
    nw = Network(net)
    h = C.c_void_p()
    _check(N.lib().ldopf_create(C.byref(nw.struct), C.byref(opts) if opts is not None else None,
                                _stream_handle(stream), C.byref(h)), "ldopf_create")
    return Problem(h)


def ldopf_solve_many(problems, allow=(LDOPF_OK, LDOPF_NOT_CONVERGED)):
    """Solve several problems together in one launch; returns their statuses."""
    n = len(problems)
    hs = (C.c_void_p * n)(*[p.h for p in problems])
    st = (ldopf_status * n)()
    _check(N.lib().ldopf_solve_many(hs, n, st), "ldopf_solve_many", allow=allow)
    return list(st)


def ldopf_create_lp(n, c, lo, hi, x_init, n_s, m_s, A, b, gidx, opts: ldopf_options | None = None,
                    stream=None) -> Problem:
    """Create from the consensus LP directly (see include/ldopf.h)."""
    c = np.ascontiguousarray(c, np.float64)
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    xi = None if x_init is None else np.ascontiguousarray(x_init, np.float64)
    n_s = np.ascontiguousarray(n_s, np.int32)
    m_s = np.ascontiguousarray(m_s, np.int32)
    A = np.ascontiguousarray(A, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    gidx = np.ascontiguousarray(gidx, np.int64)
    h = C.c_void_p()
    _check(N.lib().ldopf_create_lp(int(n), _ptr(c, C.c_double), _ptr(lo, C.c_double), _ptr(hi, C.c_double),
                                   _ptr(xi, C.c_double), int(n_s.shape[0]), _ptr(n_s, C.c_int32),
                                   _ptr(m_s, C.c_int32), _ptr(A, C.c_double) if A.size else None,
                                   _ptr(b, C.c_double) if b.size else None, _ptr(gidx, C.c_int64),
                                   C.byref(opts) if opts is not None else None, _stream_handle(stream),
                                   C.byref(h)), "ldopf_create_lp")
    return Problem(h)


class Batch:
    """Owner of one ldopf_batch handle (batched load scenarios)."""

    def __init__(self, handle: C.c_void_p):
        self.h = handle

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may be gone already
            pass

    def close(self):
        if getattr(self, "h", None):
            N.lib().ldopf_batch_destroy(self.h)
            self.h = None

    def sizes(self) -> ldopf_batch_sizes:
        s = ldopf_batch_sizes()
        _check(N.lib().ldopf_batch_get_sizes(self.h, C.byref(s)), "ldopf_batch_get_sizes")
        return s

    def set_options(self, opts: ldopf_options):
        _check(N.lib().ldopf_batch_set_options(self.h, C.byref(opts)), "ldopf_batch_set_options")

    def reset(self):
        _check(N.lib().ldopf_batch_reset(self.h), "ldopf_batch_reset")

    def solve(self) -> ldopf_batch_status:
        st = ldopf_batch_status()
        _check(N.lib().ldopf_batch_solve(self.h, C.byref(st)), "ldopf_batch_solve")
        return st

    def scenario(self, k: int) -> ldopf_status:
        st = ldopf_status()
        _check(N.lib().ldopf_batch_get_scenario(self.h, int(k), C.byref(st)), "ldopf_batch_get_scenario")
        return st

    def get_global(self, k: int) -> np.ndarray:
        x = np.empty(self.sizes().n)
        _check(N.lib().ldopf_batch_get_global(self.h, int(k), _ptr(x, C.c_double), x.shape[0]), "ldopf_batch_get_global")
        return x

    def get_local(self, k: int):
        nl = self.sizes().n_local
        xs, lam = np.empty(nl), np.empty(nl)
        _check(N.lib().ldopf_batch_get_local(self.h, int(k), _ptr(xs, C.c_double), _ptr(lam, C.c_double), nl),
               "ldopf_batch_get_local")
        return xs, lam

    def tune(self, cache_path: str | None = None):
        r, w = C.c_int32(0), C.c_int32(0)
        _check(N.lib().ldopf_batch_tune(self.h, cache_path.encode() if cache_path else None, C.byref(r), C.byref(w)),
               "ldopf_batch_tune")
        return r.value, w.value


def ldopf_batch_create(net: dict, load_scale: np.ndarray, opts: ldopf_options | None = None, stream=None) -> Batch:
    """Batched scenarios: load_scale is [n_scen, n_load]; scenario k multiplies
    every load's reference powers by load_scale[k, load]."""
    nw = Network(net)
    sc = np.ascontiguousarray(load_scale, dtype=np.float64)
    if sc.ndim != 2 or sc.shape[1] != int(net["n_load"]):
        raise ValueError("load_scale must be [n_scen, n_load]")
    if opts is None:
        opts = ldopf_default_options(precision=LDOPF_FP32_MIXED)
    h = C.c_void_p()
    _check(N.lib().ldopf_batch_create(C.byref(nw.struct), int(sc.shape[0]), _ptr(sc, C.c_double), C.byref(opts),
                                      _stream_handle(stream), C.byref(h)), "ldopf_batch_create")
    return Batch(h)


def ldopf_request_estimate(net: dict, opts: ldopf_options | None = None):
    """(device bytes, workgroups) the server's admission counts for a request."""
    nw = Network(net)
    b, w = C.c_int64(0), C.c_int32(0)
    _check(N.lib().ldopf_request_estimate(C.byref(nw.struct), C.byref(opts) if opts is not None else None,
                                          C.byref(b), C.byref(w)), "ldopf_request_estimate")
    return b.value, w.value


class Server:
    """Owner of one ldopf_server (the serving request loop)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 8):
        h = C.c_void_p()
        _check(N.lib().ldopf_server_create(int(hbm_budget_bytes), int(max_slots), C.byref(h)), "ldopf_server_create")
        self.h = h

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may be gone already
            pass

    def close(self):
        if getattr(self, "h", None):
            N.lib().ldopf_server_destroy(self.h)
            self.h = None

    def submit(self, net: dict, opts: ldopf_options | None = None) -> int:
        nw = Network(net)
        rid = C.c_int64(0)
        _check(N.lib().ldopf_server_submit(self.h, C.byref(nw.struct), C.byref(opts) if opts is not None else None,
                                           C.byref(rid)), "ldopf_server_submit")
        return rid.value

    def poll(self, rid: int):
        state = C.c_int32(0)
        st = ldopf_status()
        _check(N.lib().ldopf_server_poll(self.h, int(rid), C.byref(state), C.byref(st)), "ldopf_server_poll")
        return state.value, st

    def wait(self, rid: int, timeout_s: float = -1.0):
        state = C.c_int32(0)
        st = ldopf_status()
        _check(N.lib().ldopf_server_wait(self.h, int(rid), float(timeout_s), C.byref(state), C.byref(st)),
               "ldopf_server_wait")
        return state.value, st

    def cancel(self, rid: int):
        _check(N.lib().ldopf_server_cancel(self.h, int(rid)), "ldopf_server_cancel")

    def fetch(self, rid: int):
        sz = np.zeros(2, np.int64)
        _check(N.lib().ldopf_server_fetch(self.h, int(rid), None, 0, None, None, 0, _ptr(sz, C.c_int64)),
               "ldopf_server_fetch")
        x, xs, lam = np.empty(sz[0]), np.empty(sz[1]), np.empty(sz[1])
        _check(N.lib().ldopf_server_fetch(self.h, int(rid), _ptr(x, C.c_double), x.shape[0], _ptr(xs, C.c_double),
                                          _ptr(lam, C.c_double), xs.shape[0], None), "ldopf_server_fetch")
        return x, xs, lam

    def release(self, rid: int):
        _check(N.lib().ldopf_server_release(self.h, int(rid)), "ldopf_server_release")

    def stats(self) -> ldopf_server_stats:
        st = ldopf_server_stats()
        _check(N.lib().ldopf_server_get_stats(self.h, C.byref(st)), "ldopf_server_get_stats")
        return st
