"""ctypes wrapper of the double-double CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke entry point and the
CPU-baseline leg of the benchmark may import this module; the product library
never does.  It imports nothing from the product package.

Every function takes numpy arrays (complex matrices as complex128, row-major)
and returns Python/numpy values.  Complex results come back as a pair
``(value, lo)`` where ``value`` is the complex128 rounding of the
double-double result and ``lo`` the complex low parts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"

# x86-64-v3 (AVX2 + FMA) so the library built here also runs on the GPU hosts.
GCC_CMD = ["gcc", "-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           str(_SRC), "-o", str(_LIB), "-lm"]


def build(force: bool = True) -> Path:
    """Compile liboracle.so with gcc (always, when ``force``)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        subprocess.run(GCC_CMD, check=True)
    return _LIB


_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build()
        L = ctypes.CDLL(str(_LIB))
        L.oracle_version.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_get_threads.restype = ctypes.c_int
        L.oracle_dd_add.argtypes = [_D, _D, _D]
        L.oracle_dd_mul.argtypes = [_D, _D, _D]
        L.oracle_perm_bruteforce.argtypes = [ctypes.c_int, _D, _D]
        L.oracle_perm_ryser.argtypes = [ctypes.c_int, _D, _D]
        L.oracle_perm_glynn.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D]
        L.oracle_perm_glynn_gray.argtypes = [ctypes.c_int, _D, ctypes.c_int64, ctypes.c_int64, _D]
        L.oracle_perm_generalized.argtypes = [ctypes.c_int, ctypes.c_int, _D, _I, ctypes.c_int, _D, _D]
        L.oracle_perm_generalized_full.argtypes = [ctypes.c_int, ctypes.c_int, _D, _I, _D]
        L.oracle_binom.argtypes = [ctypes.c_int, ctypes.c_int]
        L.oracle_binom.restype = ctypes.c_uint64
        L.oracle_default_pivot.argtypes = [ctypes.c_int, _I]
        L.oracle_bs_prob.argtypes = [ctypes.c_int, _D, _I, _I, _D]
        L.oracle_splitmix64_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_splitmix64_draw.restype = ctypes.c_uint64
        L.oracle_lossy_dilation.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D]
        L.oracle_cc_weights.argtypes = [ctypes.c_int, ctypes.c_int, _D, _I, ctypes.c_int, _I, _D]
        L.oracle_cc_sample.argtypes = [ctypes.c_int, _D, _I, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_uint64, _I]
        L.oracle_perm_ryser_generalized.argtypes = [ctypes.c_int, ctypes.c_int, _D, _I, _D, _D]
        L.oracle_contraction_isometry.argtypes = [ctypes.c_int, _D, _D]
        L.oracle_cc_sample_lossy.argtypes = [ctypes.c_int, _D, _I, ctypes.c_int, ctypes.c_uint64, _I]
        L.oracle_cc_sample_extracted.argtypes = [ctypes.c_int, _D, _I, ctypes.c_int, ctypes.c_double,
                                                 ctypes.c_uint64, _I]
        L.oracle_uniform_transmission.argtypes = [ctypes.c_int, _D]
        L.oracle_uniform_transmission.restype = ctypes.c_double
        _lib = L
    return _lib


def _cmat(A) -> np.ndarray:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    return A


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_I)


def _ivec(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def _result(out: np.ndarray):
    val = complex(out[0] + out[1], out[2] + out[3])
    return val, out


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def dd_add(a, b):
    out = np.zeros(2)
    lib().oracle_dd_add(_dp(np.asarray(a, dtype=np.float64)), _dp(np.asarray(b, dtype=np.float64)), _dp(out))
    return out


def dd_mul(a, b):
    out = np.zeros(2)
    lib().oracle_dd_mul(_dp(np.asarray(a, dtype=np.float64)), _dp(np.asarray(b, dtype=np.float64)), _dp(out))
    return out


def perm_bruteforce(A) -> complex:
    """Eq. (perm_def): sum over all permutations (n <= 12)."""
    A = _cmat(A)
    n = A.shape[0]
    assert A.shape == (n, n)
    out = np.zeros(4)
    rc = lib().oracle_perm_bruteforce(n, _dp(A), _dp(out))
    if rc:
        raise ValueError(f"oracle_perm_bruteforce rc={rc}")
    return _result(out)[0]


def perm_ryser(A) -> complex:
    """Eq. (ryser), subsets in Gray order, double-double."""
    A = _cmat(A)
    n = A.shape[0]
    assert A.shape == (n, n)
    out = np.zeros(4)
    rc = lib().oracle_perm_ryser(n, _dp(A), _dp(out))
    if rc:
        raise ValueError(f"oracle_perm_ryser rc={rc}")
    return _result(out)[0]


def perm_glynn(A, with_abs: bool = False):
    """Eq. (bbfg), every addend from scratch; any rows x cols shape."""
    A = _cmat(A)
    rows, cols = A.shape
    out = np.zeros(4)
    ab = np.zeros(1)
    rc = lib().oracle_perm_glynn(rows, cols, _dp(A), _dp(out), _dp(ab))
    if rc:
        raise ValueError(f"oracle_perm_glynn rc={rc}")
    v = _result(out)[0]
    return (v, float(ab[0])) if with_abs else v


def perm_glynn_gray(A, first: int = 0, count: int = -1, full: bool = False):
    """Sec. 2.1 Gray-coded Eq. (bbfg); optionally only indices [first, first+count)."""
    A = _cmat(A)
    n = A.shape[0]
    assert A.shape == (n, n)
    out = np.zeros(4)
    rc = lib().oracle_perm_glynn_gray(n, _dp(A), int(first), int(count), _dp(out))
    if rc:
        raise ValueError(f"oracle_perm_glynn_gray rc={rc}")
    return _result(out) if full else _result(out)[0]


def perm_generalized(A, M, pivot: int = -1, with_abs: bool = False, full: bool = False):
    """Eq. (bbfgrepeated), N = 1, lexicographic order, double-double."""
    A = _cmat(A)
    r, n = A.shape
    M = _ivec(M)
    assert M.shape == (r,)
    out = np.zeros(4)
    ab = np.zeros(1)
    rc = lib().oracle_perm_generalized(r, n, _dp(A), _ip(M), int(pivot), _dp(out), _dp(ab))
    if rc:
        raise ValueError(f"oracle_perm_generalized rc={rc}")
    res = _result(out)
    v = res if full else res[0]
    return (v, float(ab[0])) if with_abs else v


def perm_generalized_full(A, M) -> complex:
    """Eq. (bbfgrepeated) read with every row's Delta in [0, M_k], prefactor 2^-n."""
    A = _cmat(A)
    r, n = A.shape
    M = _ivec(M)
    out = np.zeros(4)
    rc = lib().oracle_perm_generalized_full(r, n, _dp(A), _ip(M), _dp(out))
    if rc:
        raise ValueError(f"oracle_perm_generalized_full rc={rc}")
    return _result(out)[0]


def perm_ryser_generalized(A, M, with_abs: bool = False, full: bool = False):
    """Eq. (ryser) over row subsets with row multiplicities, lexicographic, double-double."""
    A = _cmat(A)
    r, n = A.shape
    M = _ivec(M)
    assert M.shape == (r,)
    out = np.zeros(4)
    ab = np.zeros(1)
    rc = lib().oracle_perm_ryser_generalized(r, n, _dp(A), _ip(M), _dp(out), _dp(ab))
    if rc:
        raise ValueError(f"oracle_perm_ryser_generalized rc={rc}")
    res = _result(out)
    v = res if full else res[0]
    return (v, float(ab[0])) if with_abs else v


def binom(m: int, k: int) -> int:
    return int(lib().oracle_binom(int(m), int(k)))


def default_pivot(M) -> int:
    M = _ivec(M)
    return int(lib().oracle_default_pivot(len(M), _ip(M)))


def bs_prob(U, S, T) -> float:
    """Eq. (bs_p)."""
    U = _cmat(U)
    m = U.shape[0]
    S, T = _ivec(S), _ivec(T)
    out = np.zeros(1)
    rc = lib().oracle_bs_prob(m, _dp(U), _ip(S), _ip(T), _dp(out))
    if rc:
        raise ValueError(f"oracle_bs_prob rc={rc}")
    return float(out[0])


def splitmix64_draw(key: int, c: int) -> int:
    return int(lib().oracle_splitmix64_draw(key & (2**64 - 1), c & (2**64 - 1)))


def lossy_dilation(U, eta: float) -> np.ndarray:
    U = _cmat(U)
    m = U.shape[0]
    W = np.zeros((2 * m, 2 * m), dtype=np.complex128)
    rc = lib().oracle_lossy_dilation(m, _dp(U), float(eta), _dp(W))
    if rc:
        raise ValueError(f"oracle_lossy_dilation rc={rc}")
    return W


def cc_weights(A, prefix, pi, k: int) -> np.ndarray:
    """Unnormalised C&C step-k weights |perm A[(prefix, r), pi[:k]]|^2 for every row r."""
    A = _cmat(A)
    rows, n = A.shape
    prefix = _ivec(list(prefix) + [0])
    pi = _ivec(pi)
    w = np.zeros(rows)
    rc = lib().oracle_cc_weights(rows, n, _dp(A), _ip(prefix), int(k), _ip(pi), _dp(w))
    if rc:
        raise ValueError(f"oracle_cc_weights rc={rc}")
    return w


def cc_sample(U, input_occ, n_samples: int, loss: float, seed: int) -> np.ndarray:
    """Clifford & Clifford samples (n_samples x m occupations)."""
    U = _cmat(U)
    m = U.shape[0]
    occ = _ivec(input_occ)
    out = np.zeros((n_samples, m), dtype=np.int32)
    rc = lib().oracle_cc_sample(m, _dp(U), _ip(occ), int(n_samples), float(loss),
                                ctypes.c_uint64(seed & (2**64 - 1)), _ip(out))
    if rc:
        raise ValueError(f"oracle_cc_sample rc={rc}")
    return out


def cc_sample_extracted(U, input_occ, n_samples: int, loss: float, seed: int) -> np.ndarray:
    """Clifford & Clifford samples with the uniform loss taken out at the input
    (Sec. 4): each photon survives with probability 1 - loss, the survivors are
    sampled on the m modes of U (n_samples x m occupations)."""
    U = _cmat(U)
    m = U.shape[0]
    occ = _ivec(input_occ)
    out = np.zeros((n_samples, m), dtype=np.int32)
    rc = lib().oracle_cc_sample_extracted(m, _dp(U), _ip(occ), int(n_samples), float(loss),
                                          ctypes.c_uint64(seed & (2**64 - 1)), _ip(out))
    if rc:
        raise ValueError(f"oracle_cc_sample_extracted rc={rc}")
    return out


def uniform_transmission(T) -> float:
    """The uniform part of T's loss taken out at the input by cc_sample_lossy."""
    T = _cmat(T)
    return float(lib().oracle_uniform_transmission(T.shape[0], _dp(T)))


def contraction_isometry(T) -> np.ndarray:
    """V = [T; R] (2m x m) with R the Cholesky factor of I - T^H T (Sec. 4 non-uniform loss)."""
    T = _cmat(T)
    m = T.shape[0]
    V = np.zeros((2 * m, m), dtype=np.complex128)
    rc = lib().oracle_contraction_isometry(m, _dp(T), _dp(V))
    if rc:
        raise ValueError(f"oracle_contraction_isometry rc={rc}")
    return V


def cc_sample_lossy(T, input_occ, n_samples: int, seed: int) -> np.ndarray:
    """Clifford & Clifford samples through the lossy interferometer matrix T (n_samples x m)."""
    T = _cmat(T)
    m = T.shape[0]
    occ = _ivec(input_occ)
    out = np.zeros((n_samples, m), dtype=np.int32)
    rc = lib().oracle_cc_sample_lossy(m, _dp(T), _ip(occ), int(n_samples),
                                      ctypes.c_uint64(seed & (2**64 - 1)), _ip(out))
    if rc:
        raise ValueError(f"oracle_cc_sample_lossy rc={rc}")
    return out
