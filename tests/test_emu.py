"""CPU emulation of the permanent kernels against the oracle.

tests/emu/walk_emu.cpp runs the kernel's own per-lane code (walk_core.hpp)
with bounds-checked reads, under AddressSanitizer/UBSan, on the host planner's
work split, and reproduces the wavefront and finalize reductions.  These tests
need no GPU: they check that every read stays in bounds, that the walk ends,
and that the algorithm the kernel implements matches the oracle to 1e-10.
"""
import numpy as np
import pytest

from paper_2309_07027_amd import inputs as I
from tests.emu import emu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def built():
    emu.build()


def rel(a, b):
    return abs(a - b) / abs(b)


@pytest.mark.parametrize("slots", [768, 3072])
def test_smoke_and_batch_instances(oracle, slots):
    rng = np.random.default_rng(2024)
    A, M = I.random_instance(rng, 14, m=9)
    v, err, kappa, units = emu.run(A, M, slots)
    assert rel(v, oracle.perm_generalized(A, M)) <= TOL
    for i in range(8):
        A, M = I.c3_item(i)
        v, *_ = emu.run(A, M, slots)
        assert rel(v, oracle.perm_generalized(A, M)) <= TOL, i


@pytest.mark.parametrize("kind", ["distinct", "bunched", "random"])
def test_random_instances(oracle, kind):
    rng = np.random.default_rng({"distinct": 21, "bunched": 22, "random": 23}[kind])
    for n in range(1, 17):
        if kind == "distinct":
            A, M = I.random_instance(rng, n, distinct=True)
        elif kind == "bunched":
            A, M = I.random_instance(rng, n, m=max(2, n // 2))
        else:
            A, M = I.random_instance(rng, n)
        ref = oracle.perm_generalized(A, M)
        for slots in (1, 512):
            v, err, kappa, units = emu.run(A, M, slots)
            assert rel(v, ref) <= TOL, (n, M, slots)
        for L in (64, 512):
            v, err, kappa, units = emu.run(A, M, 1, l_batch=L)
            assert rel(v, ref) <= TOL, (n, M, L)


def test_edge_shapes(oracle):
    rng = np.random.default_rng(5)
    for M in ([1], [2], [1, 1], [1, 2], [3, 0, 2], [5, 1], [2, 2, 2], [7], [1, 1, 1, 1, 1, 1, 1]):
        n = sum(M)
        A = rng.standard_normal((len(M), n)) + 1j * rng.standard_normal((len(M), n))
        v, *_ = emu.run(A, M, 64)
        ref = oracle.perm_generalized(A, M)
        assert rel(v, ref) <= TOL, M


def test_c1_full(oracle):
    A, M = I.c1()
    v, err, kappa, units = emu.run(A, M, 3072)
    assert rel(v, oracle.perm_glynn_gray(A)) <= TOL
    assert err < 1e-10 and kappa > 1


def test_fp32_error_reported(oracle):
    rng = np.random.default_rng(6)
    A, M = I.random_instance(rng, 16)
    v, err, kappa, units = emu.run(A, M, 1024, f32=True)
    e = rel(v, oracle.perm_generalized(A, M))
    assert e < 1e-3
    assert err > 1e-7
