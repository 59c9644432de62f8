"""Thin ctypes binding of libipi.so (C ABI in include/ipi.h).

Functions keep the C names (``ipi_mdp_create_csr``, ``ipi_bellman``,
``ipi_solve``, ...) and only marshal arguments: torch CUDA tensors are passed
by ``data_ptr()`` and the stream by ``torch.cuda.current_stream().cuda_stream``.
Every step of the computation runs in the library's HIP kernels; there is no
fallback.  If the library is not built, loading raises ``RuntimeError``.

``MDP`` is a small convenience wrapper over a handle.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_int32, c_int64, c_uint32, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libipi.so")

IPI_OK = 0
IPI_E_INVALID_ARG = 1
IPI_E_NOT_STOCHASTIC = 2
IPI_E_OOM = 3
IPI_E_DEVICE = 4
IPI_E_NOT_CONVERGED = 5
IPI_E_NUMERICAL = 6
IPI_E_TOO_LARGE = 7
IPI_E_CANCELLED = 8
IPI_E_NOT_FOUND = 9
IPI_E_PENDING = 10

IPI_DEVICE_PTRS = 0x1
IPI_VAL_FP32 = 0x2
IPI_FP32_ORIGIN = 0x4
IPI_BORROW = 0x8
IPI_NO_VALIDATE = 0x10
IPI_VAL_FP32_ONLY = 0x20
IPI_VAL_SPLIT = 0x40

IPI_FP64 = 0
IPI_FP32_MIXED = 1
IPI_FP32_INNER = 2
INNER = {"gmres": 0, "richardson": 1, "tfqmr": 2, "bicgstab": 3}
PC = {"none": 0, "jacobi": 1}


class IPIError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ipi status {status}: {msg}")
        self.status = status


class ipi_solve_opts(Structure):
    _fields_ = [("atol", c_double), ("rtol_cert", c_double), ("alpha", c_double),
                ("max_outer", c_int32), ("max_inner", c_int32), ("inner", c_int32), ("pc", c_int32),
                ("richardson_scale", c_double), ("gmres_restart", c_int32), ("precision", c_int32),
                ("reorth", c_int32), ("mode", c_int32), ("profile", c_int32), ("v0", c_void_p),
                ("richardson_block", c_int32)]


class ipi_solve_info(Structure):
    _fields_ = [("outer_iters", c_int32), ("converged", c_int32), ("inner_iters", c_int64),
                ("final_rho", c_double), ("device_ms", c_double), ("alg_bytes", c_double),
                ("precision", c_int32), ("inner", c_int32), ("bellman_calls", c_int32), ("ppi_cached", c_int32),
                ("bellman_ms", c_double), ("bellman_bytes", c_double), ("inner_ms", c_double),
                ("inner_resid", c_double), ("product_calls", c_int64), ("product_ms", c_double),
                ("product_bytes", c_double), ("fp64_rho", c_double), ("err_bound", c_double),
                ("block_launches", c_int64), ("block_sweeps", c_int32), ("block_calls", c_int64),
                ("block_ms", c_double), ("block_bytes", c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ipi_mdp_desc(Structure):
    _fields_ = [("S", c_int64), ("A", c_int32), ("nnz", c_int64), ("k_min", c_int32), ("k_max", c_int32),
                ("uniform_k", c_int32), ("row_ptr_bytes", c_int32), ("has_fp32", c_int32), ("band", c_int32),
                ("gamma", c_double), ("device_bytes", c_int64), ("has_fp64", c_int32),
                ("fp32_row_perturbation", c_double), ("stencil_patterns", c_int32),
                ("stencil_pairs", c_int32), ("has_split", c_int32), ("split_row_perturbation", c_double)]


class ipi_tuning(Structure):
    _fields_ = [("bellman_lanes", c_int32), ("bellman_states_per_tile", c_int32),
                ("spmv_lanes", c_int32), ("spmv_states_per_tile", c_int32),
                ("bellman_chunk", c_int32), ("spmv_chunk", c_int32), ("spmv_schedule", c_int32),
                ("spmv_workgroups", c_int32), ("band_rows", c_int32), ("ppi_cached", c_int32),
                ("blocked_prefetch", c_int32)]


_lib = None


def lib():
    """Load libipi.so (raises RuntimeError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: the HIP library is required (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    st = c_int32
    L.ipi_mdp_create_csr.restype = st
    L.ipi_mdp_create_csr.argtypes = [c_int64, c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_double, c_uint32, c_void_p, POINTER(c_void_p)]
    L.ipi_mdp_destroy.restype = st
    L.ipi_mdp_destroy.argtypes = [c_void_p]
    L.ipi_mdp_describe.restype = st
    L.ipi_mdp_describe.argtypes = [c_void_p, POINTER(ipi_mdp_desc)]
    L.ipi_opts_default.restype = None
    L.ipi_opts_default.argtypes = [POINTER(ipi_solve_opts)]
    L.ipi_opts_set.restype = st
    L.ipi_opts_set.argtypes = [POINTER(ipi_solve_opts), c_char_p, c_char_p]
    L.ipi_bellman.restype = st
    L.ipi_bellman.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
    L.ipi_solve.restype = st
    L.ipi_solve.argtypes = [c_void_p, POINTER(ipi_solve_opts), c_void_p, c_void_p, POINTER(ipi_solve_info),
                            c_void_p]
    L.ipi_solve_noalloc.restype = st
    L.ipi_solve_noalloc.argtypes = [c_void_p, POINTER(ipi_solve_opts), c_void_p, c_void_p,
                                    POINTER(ipi_solve_info), c_void_p]
    L.ipi_solve_batch.restype = st
    L.ipi_solve_batch.argtypes = [c_int32, POINTER(c_void_p), POINTER(ipi_solve_opts), POINTER(c_void_p),
                                  POINTER(c_void_p), POINTER(ipi_solve_info), POINTER(c_int32), c_void_p]
    L.ipi_get_tuning.restype = st
    L.ipi_get_tuning.argtypes = [c_void_p, POINTER(ipi_tuning)]
    L.ipi_set_tuning.restype = st
    L.ipi_set_tuning.argtypes = [c_void_p, POINTER(ipi_tuning)]
    L.ipi_autotune.restype = st
    L.ipi_autotune.argtypes = [c_void_p, c_int32, c_char_p, c_void_p]
    L.ipi_footprint_bytes.restype = c_int64
    L.ipi_footprint_bytes.argtypes = [c_int64, c_int32, c_int64, c_int32, POINTER(ipi_solve_opts)]
    L.ipi_stream_read.restype = st
    L.ipi_stream_read.argtypes = [c_void_p, c_int64, c_void_p, c_void_p]
    L.ipi_last_error.restype = c_char_p
    L.ipi_last_error.argtypes = []
    L.ipi_version.restype = c_char_p
    L.ipi_version.argtypes = []
    _lib = L
    return L


def _check(status, allow=(IPI_OK,)):
    if status not in allow:
        raise IPIError(status, lib().ipi_last_error().decode())
    return status


def _ptr(x):
    """Device pointer of a torch tensor, or the data pointer of a numpy array."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError(f"unsupported buffer type {type(x)}")


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ---------------------------------------------------------------------------
# C-named wrappers
# ---------------------------------------------------------------------------

def ipi_mdp_create_csr(S, A, nnz, row_ptr, col, val, g, gamma, flags=0, stream=None):
    h = c_void_p()
    st = lib().ipi_mdp_create_csr(int(S), int(A), int(nnz), _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(g),
                                  float(gamma), int(flags), _stream(stream), ctypes.byref(h))
    _check(st)
    return h.value


def ipi_mdp_destroy(handle):
    _check(lib().ipi_mdp_destroy(handle))


def ipi_mdp_describe(handle):
    d = ipi_mdp_desc()
    _check(lib().ipi_mdp_describe(handle, ctypes.byref(d)))
    return {k: getattr(d, k) for k, _ in d._fields_}


def ipi_opts_default():
    o = ipi_solve_opts()
    lib().ipi_opts_default(ctypes.byref(o))
    return o


def ipi_opts_set(opts, name, value):
    _check(lib().ipi_opts_set(ctypes.byref(opts), str(name).encode(), str(value).encode()))


def ipi_bellman(handle, V, TV, pi, resid=None, rho=None, precision=IPI_FP64, stream=None):
    _check(lib().ipi_bellman(handle, _ptr(V), _ptr(TV), _ptr(pi), _ptr(resid), _ptr(rho), int(precision),
                             _stream(stream)))


def ipi_solve(handle, opts, V_out, pi_out, stream=None):
    info = ipi_solve_info()
    st = lib().ipi_solve(handle, ctypes.byref(opts), _ptr(V_out), _ptr(pi_out), ctypes.byref(info),
                         _stream(stream))
    _check(st, allow=(IPI_OK, IPI_E_NOT_CONVERGED))
    return st, info.to_dict()


def ipi_solve_noalloc(handle, opts, V_out, pi_out, stream=None):
    info = ipi_solve_info()
    st = lib().ipi_solve_noalloc(handle, ctypes.byref(opts), _ptr(V_out), _ptr(pi_out), ctypes.byref(info),
                                 _stream(stream))
    _check(st, allow=(IPI_OK, IPI_E_NOT_CONVERGED))
    return st, info.to_dict()


def ipi_solve_batch(handles, opts_list, V_outs, pi_outs, stream=None):
    n = len(handles)
    H = (c_void_p * n)(*handles)
    O = (ipi_solve_opts * n)(*opts_list)
    Vp = (c_void_p * n)(*[_ptr(v) for v in V_outs])
    Pp = (c_void_p * n)(*[_ptr(p) for p in pi_outs])
    infos = (ipi_solve_info * n)()
    sts = (c_int32 * n)()
    _check(lib().ipi_solve_batch(n, H, O, Vp, Pp, infos, sts, _stream(stream)))
    return list(sts), [i.to_dict() for i in infos]


def ipi_get_tuning(handle):
    t = ipi_tuning()
    _check(lib().ipi_get_tuning(handle, ctypes.byref(t)))
    return {k: getattr(t, k) for k, _ in t._fields_}


def ipi_set_tuning(handle, bellman_lanes=0, bellman_states_per_tile=0, spmv_lanes=0, spmv_states_per_tile=0,
                   bellman_chunk=0, spmv_chunk=0, spmv_schedule=0, spmv_workgroups=0, band_rows=0, ppi_cached=0,
                   blocked_prefetch=0):
    t = ipi_tuning(bellman_lanes, bellman_states_per_tile, spmv_lanes, spmv_states_per_tile, bellman_chunk, spmv_chunk,
                   spmv_schedule, spmv_workgroups, band_rows, ppi_cached, blocked_prefetch)
    _check(lib().ipi_set_tuning(handle, ctypes.byref(t)))


def ipi_autotune(handle, precision=IPI_FP64, cache_path=None, stream=None):
    _check(lib().ipi_autotune(handle, int(precision), cache_path.encode() if cache_path else None,
                              _stream(stream)))


def ipi_footprint_bytes(S, A, nnz, k_max, opts=None):
    return lib().ipi_footprint_bytes(int(S), int(A), int(nnz), int(k_max),
                                     ctypes.byref(opts) if opts is not None else None)


def ipi_stream_read(buf, nbytes, xor_out, stream=None):
    _check(lib().ipi_stream_read(_ptr(buf), int(nbytes), _ptr(xor_out), _stream(stream)))


def ipi_last_error():
    return lib().ipi_last_error().decode()


def ipi_version():
    return lib().ipi_version().decode()


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

def make_opts(**kw):
    """ipi_solve_opts from Table 1 style keywords (atol=..., alpha=..., ksp_type=...)."""
    o = ipi_opts_default()
    names = {"atol": "atol_pi", "max_outer": "max_iter_pi", "max_inner": "max_iter_ksp",
             "inner": "ksp_type", "ksp_type": "ksp_type", "pc": "pc_type", "omega": "ksp_richardson_scale",
             "restart": "ksp_gmres_restart", "reorth": "ksp_gmres_cgs_passes",
             "richardson_block": "ksp_richardson_block"}
    for k, v in kw.items():
        if k == "v0":
            o.v0 = _ptr(v)
            continue
        ipi_opts_set(o, names.get(k, k), v)
    return o


class MDP:
    """Owns one ipi_mdp_t handle."""

    def __init__(self, handle, S, A):
        self.handle = handle
        self.S = S
        self.A = A

    @classmethod
    def from_data(cls, d, flags=IPI_VAL_FP32, stream=None):
        """Create from a workloads.MDPData (host arrays are uploaded by the library)."""
        h = ipi_mdp_create_csr(d.S, d.A, d.nnz, np.ascontiguousarray(d.row_ptr, np.int64),
                               np.ascontiguousarray(d.col, np.int32), np.ascontiguousarray(d.val, np.float64),
                               np.ascontiguousarray(d.g, np.float64), d.gamma, flags, stream)
        return cls(h, d.S, d.A)

    def describe(self):
        return ipi_mdp_describe(self.handle)

    def bellman(self, V, precision=IPI_FP64, stream=None):
        import torch
        dev = V.device
        TV = torch.empty(self.S, dtype=torch.float64, device=dev)
        pi = torch.empty(self.S, dtype=torch.int32, device=dev)
        resid = torch.empty(self.S, dtype=torch.float64, device=dev)
        rho = torch.empty(1, dtype=torch.float64, device=dev)
        ipi_bellman(self.handle, V, TV, pi, resid, rho, precision, stream)
        return TV, pi, resid, rho

    def solve(self, device=None, stream=None, **kw):
        import torch
        dev = device or torch.device("cuda:0")
        V = torch.empty(self.S, dtype=torch.float64, device=dev)
        pi = torch.empty(self.S, dtype=torch.int32, device=dev)
        opts = make_opts(**kw)
        st, info = ipi_solve(self.handle, opts, V, pi, stream)
        return V, pi, info, st

    def tuning(self):
        return ipi_get_tuning(self.handle)

    def set_tuning(self, **kw):
        ipi_set_tuning(self.handle, **kw)

    def close(self):
        if self.handle:
            ipi_mdp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# serving loop (include/ipi_server.h)
# ---------------------------------------------------------------------------

class ipi_server_opts(Structure):
    _fields_ = [("hbm_budget_bytes", c_int64), ("max_slots", c_int32), ("n_streams", c_int32),
                ("small_nnz_threshold", c_int64), ("max_batch", c_int32), ("backfill", c_int32)]


class ipi_latency(Structure):
    _fields_ = [("arrival_ms", c_double), ("admit_ms", c_double), ("start_ms", c_double), ("done_ms", c_double),
                ("batched", c_int32), ("batch_size", c_int32)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _server_lib():
    L = lib()
    if not hasattr(L, "_server_ready"):
        st = c_int32
        L.ipi_server_opts_default.restype = None
        L.ipi_server_opts_default.argtypes = [POINTER(ipi_server_opts)]
        L.ipi_server_create.restype = st
        L.ipi_server_create.argtypes = [POINTER(ipi_server_opts), POINTER(c_void_p)]
        L.ipi_server_submit.restype = st
        L.ipi_server_submit.argtypes = [c_void_p, c_int64, c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_double, c_uint32, POINTER(ipi_solve_opts), POINTER(ctypes.c_uint64)]
        L.ipi_server_poll.restype = st
        L.ipi_server_poll.argtypes = [c_void_p, ctypes.c_uint64, POINTER(c_int32)]
        L.ipi_server_wait.restype = st
        L.ipi_server_wait.argtypes = [c_void_p, ctypes.c_uint64, c_void_p, c_void_p, POINTER(ipi_solve_info),
                                      POINTER(ipi_latency)]
        L.ipi_server_cancel.restype = st
        L.ipi_server_cancel.argtypes = [c_void_p, ctypes.c_uint64]
        L.ipi_server_destroy.restype = st
        L.ipi_server_destroy.argtypes = [c_void_p]
        L._server_ready = True
    return L


def ipi_server_opts_default():
    o = ipi_server_opts()
    _server_lib().ipi_server_opts_default(ctypes.byref(o))
    return o


def ipi_server_create(opts=None, **kw):
    o = opts or ipi_server_opts_default()
    for k, v in kw.items():
        setattr(o, k, v)
    h = c_void_p()
    _check(_server_lib().ipi_server_create(ctypes.byref(o), ctypes.byref(h)))
    return h.value


def ipi_server_submit(srv, d, opts=None, flags=0):
    """Queue the solve of a workloads.MDPData (host arrays, copied by the call)."""
    o = opts or ipi_opts_default()
    t = ctypes.c_uint64()
    rp = np.ascontiguousarray(d.row_ptr, np.int64)
    col = np.ascontiguousarray(d.col, np.int32)
    val = np.ascontiguousarray(d.val, np.float64)
    g = np.ascontiguousarray(d.g, np.float64)
    _check(_server_lib().ipi_server_submit(srv, d.S, d.A, d.nnz, _ptr(rp), _ptr(col), _ptr(val), _ptr(g),
                                           d.gamma, flags, ctypes.byref(o), ctypes.byref(t)))
    return t.value


def ipi_server_poll(srv, ticket):
    done = c_int32()
    _check(_server_lib().ipi_server_poll(srv, ticket, ctypes.byref(done)))
    return bool(done.value)


def ipi_server_wait(srv, ticket, S):
    """Wait for a ticket; returns (status, V, pi, info, latency) with host numpy outputs."""
    V = np.empty(S, np.float64)
    pi = np.empty(S, np.int32)
    info = ipi_solve_info()
    lat = ipi_latency()
    st = _server_lib().ipi_server_wait(srv, ticket, _ptr(V), _ptr(pi), ctypes.byref(info), ctypes.byref(lat))
    if st == IPI_E_NOT_FOUND:
        _check(st)
    info = info.to_dict()
    if st != IPI_OK:
        info["error"] = ipi_last_error()
    return st, V, pi, info, lat.to_dict()


def ipi_server_cancel(srv, ticket):
    return _server_lib().ipi_server_cancel(srv, ticket)


def ipi_server_destroy(srv):
    _check(_server_lib().ipi_server_destroy(srv))
