"""Seeded synthetic inputs shared by the tests, the benchmark and the golden-value
script.

This module only draws random numbers and slices matrices: it holds none of the
method's arithmetic, and it imports neither the GPU library nor the oracle.

The paper's workloads are random (Haar) unitaries with photons placed at random
on the modes (Sec. 3.1 benchmarks; Sec. 3.2 accuracy study; Sec. 4 sampling on a
60-mode interferometer).  No public dataset is involved; these generators stand
in for them.

Conventions
-----------
* Haar unitary: ``Z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))``
  (real block drawn first), ``Q, R = numpy.linalg.qr(Z)``,
  ``U = Q * (diag(R) / |diag(R)|)`` (R-diagonal phase fix).
* Rows of U are output modes, columns are input modes (Sec. 2).
* A "generalized" instance is ``(A, M)``: ``A`` is r x n complex128 with one row
  per distinct output mode and ``M`` the int32 multiplicities, sum M == n.
"""
from __future__ import annotations

import numpy as np

M_MODES = 60


def haar_from_rng(rng: np.random.Generator, m: int = M_MODES) -> np.ndarray:
    z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return np.ascontiguousarray(q * (d / np.abs(d))[None, :])


def haar_unitary(seed, m: int = M_MODES) -> np.ndarray:
    return haar_from_rng(np.random.default_rng(seed), m)


def bunch(modes: np.ndarray, m: int = M_MODES):
    """Occupied output modes (ascending) and their counts for a list of photon modes."""
    cnt = np.bincount(np.asarray(modes, dtype=np.int64), minlength=m)
    rows = np.nonzero(cnt)[0]
    return rows, cnt[rows].astype(np.int32)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def c1():
    """20 distinct rows, first 20 columns of Haar(seed 0), all M = 1."""
    u = haar_unitary(0)
    return np.ascontiguousarray(u[0:20, 0:20]), np.ones(20, dtype=np.int32)


def c2a():
    """n = 30: 30 distinct rows, all M = 1."""
    u = haar_unitary(0)
    return np.ascontiguousarray(u[0:30, 0:30]), np.ones(30, dtype=np.int32)


def c2b():
    """n = 30: 10 distinct rows, each M = 3."""
    u = haar_unitary(0)
    return np.ascontiguousarray(u[0:10, 0:30]), np.full(10, 3, dtype=np.int32)


def c2c():
    """n = 30: 30 photons dropped uniformly at random into 60 modes (seed 2)."""
    rng = np.random.default_rng(2)
    modes = rng.integers(0, M_MODES, 30)
    rows, mult = bunch(modes)
    u = haar_unitary(0)
    return np.ascontiguousarray(u[rows, 0:30]), mult


def c2(case: str):
    return {"a": c2a, "b": c2b, "c": c2c}[case]()


def c3_item(i: int):
    """Item i of the 4096-item uneven batch: n uniform in [8, 24]."""
    rng = np.random.default_rng([3, i])
    n = int(rng.integers(8, 25))
    u = haar_from_rng(rng)
    modes = rng.integers(0, M_MODES, n)
    rows, mult = bunch(modes)
    return np.ascontiguousarray(u[rows, 0:n]), mult


def c3(count: int = 4096):
    return [c3_item(i) for i in range(count)]


def random_instance(rng: np.random.Generator, n: int, m: int = M_MODES, distinct: bool = False):
    """A random (A, M) of n photons: n columns of a fresh Haar unitary (of size
    max(m, n)), rows from n photons placed uniformly on m modes (or n distinct
    rows when ``distinct``)."""
    u = haar_from_rng(rng, max(m, n))
    if distinct:
        rows = np.sort(rng.choice(m, size=n, replace=False))
        mult = np.ones(n, dtype=np.int32)
    else:
        rows, mult = bunch(rng.integers(0, m, n), m)
    return np.ascontiguousarray(u[rows, 0:n]), mult


def c4_job(j: int):
    """Serving job j: (U, input occupation, n_samples, loss, seed)."""
    rng = np.random.default_rng([4, j])
    n = int(rng.choice([20, 24, 28, 30]))
    u = haar_from_rng(rng)
    occ = np.zeros(M_MODES, dtype=np.int32)
    occ[:n] = 1
    return u, occ, 16, 0.0, (4 << 32) | j


def c4_arrivals(rate: float, count: int, lam_index: int):
    """Poisson arrival times (seconds) with the given rate (jobs/s)."""
    rng = np.random.default_rng([40, lam_index])
    gaps = rng.exponential(1.0 / rate, count)
    return np.cumsum(gaps)


def c5(lossy: bool = False):
    """n = 40 photons in the first 40 modes of Haar(seed 5); lossy: transmission 0.5."""
    u = haar_unitary(5)
    occ = np.zeros(M_MODES, dtype=np.int32)
    occ[:40] = 1
    return u, occ, (0.5 if lossy else 0.0)
