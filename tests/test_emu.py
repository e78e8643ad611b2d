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
# Sums with a conditioning kappa (sum |addend| / |perm|) above this are held to
# their own reported error estimate instead of TOL (the FP64 walk's error grows
# like kappa * u; the estimate is kappa * u * (n + sqrt(Q))).
KAPPA_WELL = 1e6


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


def _minor_case(rng, K, modes):
    """A random (A, M): rows from K-1 photons on `modes` modes, K columns."""
    rows = rng.integers(0, modes, K - 1)
    u = I.haar_from_rng(rng, max(modes, K))
    kept, mult = I.bunch(rows, modes) if K > 1 else (np.array([0]), np.array([0], dtype=np.int32))
    return np.ascontiguousarray(u[kept][:, :K]), mult


@pytest.mark.parametrize("modes,Ks", [(60, (2, 3, 5, 9, 14, 17, 21)), (5, (22, 26, 31, 40))])
def test_minors_walk_matches_oracle(oracle, modes, Ks):
    """Every leave-one-column-out permanent of the joint walk (Laplace minors),
    against the oracle's generalized permanent of the matrix without that column;
    K spans one group (small K) and several groups, with a padded last group
    (K = 21, 31, 40).  Heavy bunching (5 modes) keeps the large-K sums short but
    makes them ill-conditioned (kappa up to ~3e7 at K = 40).  The bar (the
    reading of the relative-error target for ill-conditioned sums): 1e-10 where
    the oracle's kappa is at most KAPPA_WELL, and otherwise the walk's own
    estimate; the error never exceeds that estimate in any case."""
    rng = np.random.default_rng(77 + modes)
    for K in Ks:
        A, M = _minor_case(rng, K, modes)
        refs = [oracle.perm_generalized(np.delete(A, l, axis=1), M, with_abs=True) for l in range(K)]
        for L, slots in ((64, 1), (512, 1), (0, 2048)):
            got, est, kap = emu.run_minors(A, M, L, slots, with_err=True)
            for l, (ref, absum) in enumerate(refs):
                e = rel(got[l], ref)
                assert e <= est[l], (K, l, M, L, e, est[l])
                if absum / abs(ref) <= KAPPA_WELL:
                    assert e <= TOL, (K, l, M, L, e)


@pytest.mark.parametrize("K,M", [(14, [1] * 13), (16, [1] * 15), (24, [2] * 6 + [1] * 11), (36, [4] * 8 + [3])])
def test_minors_kappa_estimate(oracle, K, M):
    """The walk's per-minor conditioning estimate against the oracle's sum of
    |addend| / |perm|, at unit lengths 64, 512 and 4096.  The walk samples the
    modulus of each target's addend at one position per lane (the unit's last)
    in about 32 units per lane group, scaled by the positions they stand for:
    an estimate of a heavy-tailed sum (a product of K - 1 moduli).  Measured
    over these cases: between 0.15 and 5.1 times the exact value; the bar is a
    factor of 8 either way.  The result itself stays within min(1e-10, its own
    estimate)."""
    U = I.haar_unitary(300 + K)
    A = np.ascontiguousarray(U[:len(M)][:, :K])
    refs = [oracle.perm_generalized(np.delete(A, l, axis=1), M, with_abs=True) for l in range(K)]
    for L in (64, 512, 4096):
        got, est, kap = emu.run_minors(A, M, L, 1, with_err=True)
        for l, (ref, absum) in enumerate(refs):
            ratio = kap[l] / (absum / abs(ref))
            assert 1.0 / 8.0 <= ratio <= 8.0, (K, L, l, ratio)
            assert rel(got[l], ref) <= min(TOL, est[l]), (K, L, l)


@pytest.mark.parametrize("K", [12, 26])
def test_minors_estimate_with_a_zero_column(oracle, K):
    """A zero column makes its column sum zero at every Gray position.  Every
    other minor keeps that column, so it is 0 with an infinite estimate; the
    minor that drops it is a generic permanent whose estimate must come from
    the other columns' moduli (a leave-one-out product, no division by the
    zero modulus): finite, positive and covering its error."""
    rng = np.random.default_rng(900 + K)
    A, M = _minor_case(rng, K, 60)
    z = K // 3
    A = A.copy()
    A[:, z] = 0.0
    for L in (64, 512):
        got, est, _ = emu.run_minors(A, M, L, 1, with_err=True)
        ref = oracle.perm_generalized(np.delete(A, z, axis=1), M)
        e = rel(got[z], ref)
        assert np.isfinite(est[z]) and 0.0 < est[z] < 1e-8, (K, L, est[z])
        assert e <= min(TOL, est[z]), (K, L, e, est[z])
        for l in range(K):
            if l != z:
                assert got[l] == 0, (K, L, l, got[l])


@pytest.mark.parametrize("seed", [31, 32])
def test_column_multiplicities_match_oracle(oracle, seed):
    """Column multiplicities (Eq. bbfgrepeated) against the oracle's permanent of
    the column-expanded matrix: equal multiplicities e use (prod_j c_j)^e over the
    distinct columns, mixed ones the expanded matrix."""
    rng = np.random.default_rng(seed)
    cases = [(n, None) for n in (1, 2, 5, 9, 14, 17)] + [(n, e) for n, e in ((4, 2), (12, 2), (15, 3), (16, 4), (18, 6))]
    for n, e in cases:
        rows, M = I.bunch(rng.integers(0, 60, n), 60)
        if e is None:
            cols, N = I.bunch(rng.integers(0, 9, n), 9)
        else:
            cols, N = np.arange(n // e), np.full(n // e, e, dtype=np.int32)
        u = I.haar_from_rng(rng, 60)
        A = np.ascontiguousarray(u[rows][:, cols])
        ref = oracle.perm_generalized(np.repeat(A, N, axis=1), M)
        for slots, L in ((1, 64), (2048, 0)):
            v, err, kappa, units = emu.run_cols(A, M, N, slots, L)
            assert rel(v, ref) <= TOL, (n, M.tolist(), N.tolist(), slots, L)


@pytest.mark.parametrize("kind", ["distinct", "bunched"])
def test_ryser_walk_matches_oracle(oracle, kind):
    """The walk planned for Eq. ryser (no pivot row, base coefficient 0, scale
    2^-n) against the oracle's generalized Ryser and its BB/FG value, single and
    batched splits; its error estimate covers its error."""
    rng = np.random.default_rng({"distinct": 41, "bunched": 42}[kind])
    for n in (1, 2, 3, 6, 11, 15):
        if kind == "distinct":
            A, M = I.random_instance(rng, n, distinct=True)
        else:
            A, M = I.random_instance(rng, n, m=max(2, n // 2))
        ref_r = oracle.perm_ryser_generalized(A, M)
        ref = oracle.perm_generalized(A, M)
        for slots, L in ((512, 0), (1, 64)):
            v, err, kappa, units = emu.run(A, M, slots, l_batch=L, ryser=True)
            e = rel(v, ref)
            assert e <= max(err, 1e-15), (n, M, slots, e, err)
            assert rel(v, ref_r) <= max(err, 1e-15)
            assert e <= 1e-8, (n, e)
