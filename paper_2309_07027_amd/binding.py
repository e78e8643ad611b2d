"""ctypes binding of libbbfg.so (include/bbfg.h), argument marshalling only.

Matrices may be numpy arrays (host) or torch tensors (host or ``cuda``); they
must be complex128 and are made contiguous.  Every computation runs in the HIP
library; this module never computes a permanent itself, and it raises
``ImportError`` when the library has not been built.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "libbbfg.so"

BBFG_OK = 0
BBFG_EINVAL = -1
BBFG_ERANGE = -2
BBFG_ENOMEM = -3
BBFG_EDEVICE = -4
BBFG_EBUSY = -5
BBFG_ENOTFOUND = -6
BBFG_ECANCELED = -7
BBFG_FP64 = 0
BBFG_FP32 = 1
BBFG_MINORS = 2
BBFG_RYSER = 4
BBFG_COLS = 3
MAX_N = 48
MAX_N_FP32 = 24


class BBFGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bbfg error {code}: {msg}")
        self.code = code


class Info(ctypes.Structure):
    _fields_ = [("rel_err_est", ctypes.c_double), ("kappa", ctypes.c_double),
                ("n_addends", ctypes.c_uint64), ("n_units", ctypes.c_uint64),
                ("kernel_ms", ctypes.c_double), ("flops", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanSummary(ctypes.Structure):
    _fields_ = [("n_cols", ctypes.c_int32), ("n_rows_kept", ctypes.c_int32), ("pivot_row", ctypes.c_int32),
                ("n_lane_digits", ctypes.c_int32), ("n_high_digits", ctypes.c_int32),
                ("n_low_digits", ctypes.c_int32), ("lane_product", ctypes.c_uint32),
                ("lane_groups", ctypes.c_uint32), ("low_count", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("high_count", ctypes.c_uint64), ("n_addends", ctypes.c_uint64), ("n_units", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class ServerStats(ctypes.Structure):
    _fields_ = [("jobs_submitted", ctypes.c_uint64), ("jobs_done", ctypes.c_uint64),
                ("iterations", ctypes.c_uint64), ("samples_done", ctypes.c_uint64),
                ("max_active", ctypes.c_uint64), ("max_queued", ctypes.c_uint64),
                ("jobs_cancelled", ctypes.c_uint64), ("busy_s", ctypes.c_double),
                ("host_s", ctypes.c_double), ("wait_s", ctypes.c_double), ("flops", ctypes.c_double),
                ("walk_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PD = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes): every symbol of include/bbfg.h
SIGNATURES = {
    "bbfg_last_error": (ctypes.c_char_p, []),
    "bbfg_version": (ctypes.c_int, []),
    "bbfg_init": (ctypes.c_int, []),
    "bbfg_set_stream": (ctypes.c_int, [_P]),
    "bbfg_set_cache_limits": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64]),
    "perm_bbfg": (ctypes.c_int, [_P, _I32, _PI32, _I32, _P, ctypes.POINTER(Info)]),
    "perm_bbfg_noalloc": (ctypes.c_int, [_P, _I32, _PI32, _I32, _P, ctypes.POINTER(Info)]),
    "perm_ryser": (ctypes.c_int, [_P, _I32, _PI32, _I32, _P, ctypes.POINTER(Info)]),
    "perm_batch": (ctypes.c_int, [_I32, _P, _PI64, _PI32, _PI32, _PI64, _PI32, _I32, _P, _PD]),
    "perm_minors": (ctypes.c_int, [_P, _I32, _PI32, _I32, _P, _PD]),
    "perm_bbfg_cols": (ctypes.c_int, [_P, _I32, _PI32, _I32, _PI32, _P, ctypes.POINTER(Info)]),
    "perm_batch_last_kernel_ms": (ctypes.c_double, []),
    "perm_batch_last_was_graph": (ctypes.c_int, []),
    "bs_sample": (ctypes.c_int, [_P, _I32, _PI32, _I32, ctypes.c_double, ctypes.c_uint64, _PI32,
                                 ctypes.POINTER(Info)]),
    "bs_sample_lossy": (ctypes.c_int, [_P, _I32, _PI32, _I32, ctypes.c_uint64, _PI32, ctypes.POINTER(Info)]),
    "bs_sample_extracted": (ctypes.c_int, [_P, _I32, _PI32, _I32, ctypes.c_double, ctypes.c_uint64, _PI32,
                                           ctypes.POINTER(Info)]),
    "bs_server_create": (ctypes.c_int, [ctypes.c_size_t, _I32, ctypes.POINTER(_P)]),
    "bs_server_submit": (ctypes.c_int, [_P, _P, _I32, _PI32, _I32, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "bs_server_submit_lossy": (ctypes.c_int, [_P, _P, _I32, _PI32, _I32, ctypes.c_uint64,
                                              ctypes.POINTER(ctypes.c_uint64)]),
    "bs_server_submit_extracted": (ctypes.c_int, [_P, _P, _I32, _PI32, _I32, ctypes.c_double, ctypes.c_uint64,
                                                  ctypes.POINTER(ctypes.c_uint64)]),
    "bs_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, _PI32, _PD, _PD]),
    "bs_server_cancel": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "bs_server_drain": (ctypes.c_int, [_P]),
    "bs_server_destroy": (ctypes.c_int, [_P]),
    "bs_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ServerStats)]),
    "bbfg_plan_query": (ctypes.c_int, [_PI32, _I32, _I32, _I32, ctypes.POINTER(PlanSummary)]),
    "bbfg_gray_table": (ctypes.c_int, [_PI32, _I32, _I32, _PI32, _PI32]),
    "bbfg_walk_occupancy": (ctypes.c_int, [_I32, _I32, _PI32, _PI32]),
    "bbfg_fp64_fma_peak": (ctypes.c_int, [_PD, _PD]),
    "bbfg_autotune": (ctypes.c_int, [_I32, _I32, _I32, ctypes.c_char_p]),
    "bbfg_autotune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "bbfg_batch_unit_length": (ctypes.c_int, [_I32, _I32, ctypes.POINTER(ctypes.c_uint64)]),
}

_lib = None


def lib():
    """The loaded library (raises ImportError if it was not built)."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2309_07027_amd.build`"
                              "; there is no fallback path")
        # torch ships its own HIP runtime.  Loading it first makes libbbfg.so bind
        # to that same runtime (one HIP/HSA runtime per process); loading
        # libbbfg.so first would bring in a second runtime that torch cannot use.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(str(_LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def library_path() -> str:
    return str(_LIB_PATH)


def _check(rc: int):
    if rc != BBFG_OK:
        raise BBFGError(rc, lib().bbfg_last_error().decode(errors="replace"))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _cmat_ptr(A):
    """(pointer, keepalive, shape) of a complex128 matrix (numpy or torch)."""
    if _is_torch(A):
        import torch
        if A.dtype != torch.complex128:
            raise TypeError("matrix must be torch.complex128")
        t = A.contiguous()
        return ctypes.c_void_p(t.data_ptr()), t, tuple(t.shape)
    a = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    return ctypes.c_void_p(a.ctypes.data), a, a.shape


def _i32(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int32))
    return a, a.ctypes.data_as(_PI32)


def _i64(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
    return a, a.ctypes.data_as(_PI64)


def init():
    _check(lib().bbfg_init())


def set_cache_limits(max_plans: int = 0, max_table_entries: int = 0):
    """Bounds of the plan and Gray-table caches (0 = default)."""
    _check(lib().bbfg_set_cache_limits(int(max_plans), int(max_table_entries)))


def set_stream(stream=None):
    """Use a torch.cuda.Stream (or a raw hipStream_t int, or None) for later calls."""
    if stream is None:
        h = None
    elif isinstance(stream, int):
        h = stream
    else:
        h = stream.cuda_stream
    _check(lib().bbfg_set_stream(ctypes.c_void_p(h)))


def perm_bbfg(A, row_mult=None, with_info: bool = False):
    """Permanent of A with row multiplicities (default all ones): Eq. (bbfgrepeated)."""
    ptr, keep, shape = _cmat_ptr(A)
    r, n = shape
    mult, mp = _i32(np.ones(r, dtype=np.int32) if row_mult is None else row_mult)
    out = np.zeros(1, dtype=np.complex128)
    info = Info()
    _check(lib().perm_bbfg(ptr, r, mp, n, ctypes.c_void_p(out.ctypes.data), ctypes.byref(info)))
    del keep
    return (complex(out[0]), info.as_dict()) if with_info else complex(out[0])


def perm_ryser(A, row_mult=None, with_info: bool = False):
    """The same permanent by Eq. (ryser) with row multiplicities, FP64, on the same walk."""
    ptr, keep, shape = _cmat_ptr(A)
    r, n = shape
    mult, mp = _i32(np.ones(r, dtype=np.int32) if row_mult is None else row_mult)
    out = np.zeros(1, dtype=np.complex128)
    info = Info()
    _check(lib().perm_ryser(ptr, r, mp, n, ctypes.c_void_p(out.ctypes.data), ctypes.byref(info)))
    del keep
    return (complex(out[0]), info.as_dict()) if with_info else complex(out[0])


def perm_bbfg_noalloc(A, row_mult=None, with_info: bool = False):
    """perm_bbfg through the entry point that allocates no device memory."""
    ptr, keep, shape = _cmat_ptr(A)
    r, n = shape
    mult, mp = _i32(np.ones(r, dtype=np.int32) if row_mult is None else row_mult)
    out = np.zeros(1, dtype=np.complex128)
    info = Info()
    _check(lib().perm_bbfg_noalloc(ptr, r, mp, n, ctypes.c_void_p(out.ctypes.data), ctypes.byref(info)))
    del keep
    return (complex(out[0]), info.as_dict()) if with_info else complex(out[0])


def pack_batch(mats):
    """Pack [(A, M), ...] into the perm_batch arrays (host numpy)."""
    shapes = [np.asarray(A).shape for A, _ in mats]
    n_rows = np.array([s[0] for s in shapes], dtype=np.int32)
    n_cols = np.array([s[1] for s in shapes], dtype=np.int32)
    a_off = np.zeros(len(mats), dtype=np.int64)
    m_off = np.zeros(len(mats), dtype=np.int64)
    if len(mats):
        a_off[1:] = np.cumsum(n_rows.astype(np.int64) * n_cols)[:-1]
        m_off[1:] = np.cumsum(n_rows.astype(np.int64))[:-1]
    A_packed = np.concatenate([np.asarray(A, dtype=np.complex128).ravel() for A, _ in mats]) if mats else \
        np.zeros(1, dtype=np.complex128)
    M_packed = np.concatenate([np.asarray(M, dtype=np.int32).ravel() for _, M in mats]) if mats else \
        np.zeros(1, dtype=np.int32)
    return A_packed, a_off, n_rows, M_packed, m_off, n_cols


def perm_batch_packed(A_packed, a_off, n_rows, M_packed, m_off, n_cols, precision: int = BBFG_FP64,
                      out=None, with_err: bool = False):
    """perm_batch on pre-packed arrays; A_packed / out may be torch cuda tensors."""
    ptr, keep, _ = _cmat_ptr(A_packed) if _is_torch(A_packed) else _cmat_ptr(np.ravel(A_packed))
    a_off, pa = _i64(a_off)
    n_rows, pr = _i32(n_rows)
    M_packed, pm = _i32(M_packed)
    m_off, pmo = _i64(m_off)
    n_cols, pc = _i32(n_cols)
    b = len(n_cols)
    host_out = out is None
    if host_out:
        out = np.zeros(b, dtype=np.complex128)
        optr = ctypes.c_void_p(out.ctypes.data)
    else:
        optr = ctypes.c_void_p(out.data_ptr()) if _is_torch(out) else ctypes.c_void_p(out.ctypes.data)
    err = np.zeros(b, dtype=np.float64)
    _check(lib().perm_batch(b, ptr, pa, pr, pm, pmo, pc, int(precision), optr, err.ctypes.data_as(_PD)))
    del keep
    return (out, err) if with_err else out


def perm_batch(mats, precision: int = BBFG_FP64, with_err: bool = False):
    """Permanents of [(A, M), ...] (host matrices) in one batched launch."""
    return perm_batch_packed(*pack_batch(mats), precision=precision, with_err=with_err)


def perm_bbfg_cols(A, row_mult, col_mult, with_info: bool = False):
    """Permanent with row and column multiplicities (Eq. bbfgrepeated): A holds the
    distinct rows and columns; sum(row_mult) == sum(col_mult)."""
    ptr, keep, shape = _cmat_ptr(A)
    r, c = shape
    m, pm = _i32(row_mult)
    cm, pc = _i32(col_mult)
    out = np.zeros(1, dtype=np.complex128)
    info = Info()
    _check(lib().perm_bbfg_cols(ptr, r, pm, c, pc, ctypes.c_void_p(out.ctypes.data), ctypes.byref(info)))
    del keep
    return (complex(out[0]), info.as_dict()) if with_info else complex(out[0])


def perm_minors(A, M, with_err: bool = False):
    """[perm(A without column l, M) for l in range(n_cols)] (host numpy complex128);
    sum(M) == n_cols - 1.  A may be a torch cuda tensor.  with_err: also the
    per-minor relative error estimates."""
    ptr, keep, shape = _cmat_ptr(A)
    m, pm = _i32(M)
    out = np.zeros(shape[1], dtype=np.complex128)
    err = np.zeros(shape[1], dtype=np.float64)
    _check(lib().perm_minors(ptr, shape[0], pm, shape[1], ctypes.c_void_p(out.ctypes.data), err.ctypes.data_as(_PD)))
    del keep
    return (out, err) if with_err else out


def batch_last_kernel_ms() -> float:
    return float(lib().perm_batch_last_kernel_ms())


def batch_last_was_graph() -> bool:
    return bool(lib().perm_batch_last_was_graph())


def bs_sample(U, input_occupation, n_samples: int, loss: float = 0.0, seed: int = 0, with_info: bool = False):
    """Clifford & Clifford samples: (n_samples, m) int32 output occupations."""
    ptr, keep, shape = _cmat_ptr(U)
    m = shape[0]
    occ, po = _i32(input_occupation)
    out = np.zeros((n_samples, m), dtype=np.int32)
    info = Info()
    _check(lib().bs_sample(ptr, m, po, int(n_samples), float(loss), ctypes.c_uint64(seed & (2**64 - 1)),
                           out.ctypes.data_as(_PI32), ctypes.byref(info)))
    del keep
    return (out, info.as_dict()) if with_info else out


def bs_sample_lossy(T, input_occupation, n_samples: int, seed: int = 0, with_info: bool = False):
    """Samples through the lossy interferometer matrix T (a contraction): (n_samples, m) int32."""
    ptr, keep, shape = _cmat_ptr(T)
    m = shape[0]
    occ, po = _i32(input_occupation)
    out = np.zeros((n_samples, m), dtype=np.int32)
    info = Info()
    _check(lib().bs_sample_lossy(ptr, m, po, int(n_samples), ctypes.c_uint64(seed & (2**64 - 1)),
                                 out.ctypes.data_as(_PI32), ctypes.byref(info)))
    del keep
    return (out, info.as_dict()) if with_info else out


def bs_sample_extracted(U, input_occupation, n_samples: int, loss: float = 0.0, seed: int = 0,
                        with_info: bool = False):
    """Samples with the uniform loss applied to the input photons (survivors
    sampled on U's m modes): (n_samples, m) int32."""
    ptr, keep, shape = _cmat_ptr(U)
    m = shape[0]
    occ, po = _i32(input_occupation)
    out = np.zeros((n_samples, m), dtype=np.int32)
    info = Info()
    _check(lib().bs_sample_extracted(ptr, m, po, int(n_samples), float(loss), ctypes.c_uint64(seed & (2**64 - 1)),
                                     out.ctypes.data_as(_PI32), ctypes.byref(info)))
    del keep
    return (out, info.as_dict()) if with_info else out


class Server:
    """Continuous-batching sampling server (bs_server_*)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_active_jobs: int = 64):
        h = ctypes.c_void_p()
        _check(lib().bs_server_create(ctypes.c_size_t(hbm_budget_bytes), int(max_active_jobs), ctypes.byref(h)))
        self._h = h
        self._m = {}

    def submit(self, U, input_occupation, n_samples: int, loss: float = 0.0, seed: int = 0) -> int:
        ptr, keep, shape = _cmat_ptr(U)
        occ, po = _i32(input_occupation)
        jid = ctypes.c_uint64()
        _check(lib().bs_server_submit(self._h, ptr, shape[0], po, int(n_samples), float(loss),
                                      ctypes.c_uint64(seed & (2**64 - 1)), ctypes.byref(jid)))
        self._m[jid.value] = (int(n_samples), shape[0])
        del keep
        return jid.value

    def submit_lossy(self, T, input_occupation, n_samples: int, seed: int = 0) -> int:
        ptr, keep, shape = _cmat_ptr(T)
        occ, po = _i32(input_occupation)
        jid = ctypes.c_uint64()
        _check(lib().bs_server_submit_lossy(self._h, ptr, shape[0], po, int(n_samples),
                                            ctypes.c_uint64(seed & (2**64 - 1)), ctypes.byref(jid)))
        self._m[jid.value] = (int(n_samples), shape[0])
        del keep
        return jid.value

    def submit_extracted(self, U, input_occupation, n_samples: int, loss: float = 0.0, seed: int = 0) -> int:
        ptr, keep, shape = _cmat_ptr(U)
        occ, po = _i32(input_occupation)
        jid = ctypes.c_uint64()
        _check(lib().bs_server_submit_extracted(self._h, ptr, shape[0], po, int(n_samples), float(loss),
                                                ctypes.c_uint64(seed & (2**64 - 1)), ctypes.byref(jid)))
        self._m[jid.value] = (int(n_samples), shape[0])
        del keep
        return jid.value

    def poll(self, job_id: int, with_err: bool = False):
        """None while running, else (samples, latency_s) -- with_err: (samples,
        latency_s, err_est).  A cancelled job raises BBFGError (BBFG_ECANCELED)."""
        ns, m = self._m.get(job_id, (0, 1))
        out = np.zeros((max(ns, 1), m), dtype=np.int32)
        lat = ctypes.c_double()
        err = ctypes.c_double()
        rc = lib().bs_server_poll(self._h, ctypes.c_uint64(job_id), out.ctypes.data_as(_PI32), ctypes.byref(lat),
                                  ctypes.byref(err))
        if rc == BBFG_EBUSY:
            return None
        self._m.pop(job_id, None)
        _check(rc)
        return (out[:ns], lat.value, err.value) if with_err else (out[:ns], lat.value)

    def cancel(self, job_id: int):
        """Cancel a queued or active job (its later poll raises BBFG_ECANCELED)."""
        _check(lib().bs_server_cancel(self._h, ctypes.c_uint64(job_id)))

    def drain(self):
        _check(lib().bs_server_drain(self._h))

    def stats(self):
        s = ServerStats()
        _check(lib().bs_server_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self._h:
            _check(lib().bs_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def plan_query(row_mult, n_cols: int, slots: int = 0):
    m, pm = _i32(row_mult)
    s = PlanSummary()
    _check(lib().bbfg_plan_query(pm, len(m), int(n_cols), int(slots), ctypes.byref(s)))
    return s.as_dict()


def gray_table(radices):
    r, pr = _i32(radices)
    n = int(np.prod(r)) if len(r) else 1
    ch = np.zeros(n, dtype=np.int32)
    dr = np.zeros(n, dtype=np.int32)
    _check(lib().bbfg_gray_table(pr, len(r), n, ch.ctypes.data_as(_PI32), dr.ctypes.data_as(_PI32)))
    return ch, dr


def autotune(n_lo: int, n_hi: int, precision: int = BBFG_FP64, cache_path: str | None = None):
    """Tune the batched unit length for n in [n_lo, n_hi] on this device."""
    _check(lib().bbfg_autotune(int(n_lo), int(n_hi), int(precision),
                               None if cache_path is None else str(cache_path).encode()))


def autotune_load(cache_path: str):
    _check(lib().bbfg_autotune_load(str(cache_path).encode()))


def batch_unit_length(n_cols: int, precision: int = BBFG_FP64) -> int:
    L = ctypes.c_uint64()
    _check(lib().bbfg_batch_unit_length(int(n_cols), int(precision), ctypes.byref(L)))
    return L.value


def fp64_fma_peak():
    """(TFLOP/s, ms) of the device's measured FP64 FMA throughput."""
    t = ctypes.c_double()
    ms = ctypes.c_double()
    _check(lib().bbfg_fp64_fma_peak(ctypes.byref(t), ctypes.byref(ms)))
    return t.value, ms.value


def walk_occupancy(n_cols: int, precision: int = BBFG_FP64):
    w = ctypes.c_int32()
    c = ctypes.c_int32()
    _check(lib().bbfg_walk_occupancy(int(n_cols), int(precision), ctypes.byref(w), ctypes.byref(c)))
    return w.value, c.value
