"""GPU tests of Clifford & Clifford sampling (bs_sample) and the continuous-batching
server, against the CPU oracle sampler (same SplitMix64 draws, direct k x k
permanents instead of Laplace minors) and Eq. (bs_p)."""
import sys
import time

import numpy as np
import pytest

from paper_2309_07027_amd import binding as B
from paper_2309_07027_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def patterns(m, n):
    if m == 1:
        yield (n,)
        return
    for k in range(n + 1):
        for rest in patterns(m - 1, n - k):
            yield (k,) + rest


def compare_samples(gpu, cpu, what):
    mism = np.nonzero((gpu != cpu).any(axis=1))[0]
    # both sides draw with the same uniforms; a flip can only come from a weight
    # rounding difference at a CDF boundary, which is vanishingly rare
    assert len(mism) == 0, f"{what}: samples {mism[:10]} differ"


@pytest.mark.parametrize("m,occ,loss,seed", [
    (8, [1, 1, 1, 1, 0, 0, 0, 0], 0.0, 7),
    (6, [1, 0, 2, 0, 1, 0], 0.0, 8),
    (6, [1, 1, 1, 0, 0, 0], 0.4, 9),
    (12, [1] * 6 + [0] * 6, 0.0, 10),
    (10, [2, 1, 1, 1, 0, 0, 0, 0, 0, 0], 0.3, 11),
])
def test_bs_sample_matches_oracle_sampler(oracle, m, occ, loss, seed):
    U = I.haar_unitary(100 + seed, m)
    say(f"case bs_sample m={m} occ={occ} loss={loss}")
    g = B.bs_sample(U, occ, 40, loss=loss, seed=seed)
    c = oracle.cc_sample(U, occ, 40, loss, seed)
    compare_samples(g, c, f"m={m}")
    n = sum(occ)
    if loss == 0.0:
        assert (g.sum(axis=1) == n).all()
    else:
        assert (g.sum(axis=1) <= n).all()


def test_bs_sample_distribution_matches_bs_p(oracle):
    m, occ = 5, [1, 1, 1, 0, 0]
    U = I.haar_unitary(21, m)
    N = 20000
    say("case distribution m=5 n=3")
    s = B.bs_sample(U, occ, N, seed=123)
    counts = {}
    for row in s:
        counts[tuple(row)] = counts.get(tuple(row), 0) + 1
    tv = 0.5 * sum(abs(counts.get(T, 0) / N - oracle.bs_prob(U, occ, T)) for T in patterns(m, 3))
    assert tv < 0.03


def test_hong_ou_mandel():
    H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
    s = B.bs_sample(H, [1, 1], 500, seed=3)
    assert not ((s[:, 0] == 1) & (s[:, 1] == 1)).any()
    frac = (s[:, 0] == 2).mean()
    assert 0.4 < frac < 0.6


def test_lossy_photon_count_distribution():
    # each photon survives with probability eta = 1 - loss, independently
    m, n, loss = 8, 4, 0.5
    U = I.haar_unitary(31, m)
    s = B.bs_sample(U, [1] * n + [0] * (m - n), 4000, loss=loss, seed=5)
    k = s.sum(axis=1)
    from math import comb
    for j in range(n + 1):
        p = comb(n, j) * 0.5 ** n
        assert abs((k == j).mean() - p) < 0.035


def test_sampler_m60_n10_runs(oracle):
    U, occ, ns, loss, seed = I.c4_job(0)
    occ = np.zeros(60, dtype=np.int32)
    occ[:10] = 1
    say("case m=60 n=10")
    g, info = B.bs_sample(U, occ, 8, seed=99, with_info=True)
    c = oracle.cc_sample(U, occ, 8, 0.0, 99)
    compare_samples(g, c, "m60n10")
    assert info["n_addends"] > 0


def test_server_results_same_alone_and_in_mix():
    jobs = []
    for j in range(6):
        rng = np.random.default_rng([77, j])
        m = 12
        n = 3 + j % 3
        U = I.haar_from_rng(rng, m)
        occ = np.zeros(m, dtype=np.int32)
        occ[:n] = 1
        jobs.append((U, occ, 8, 0.2 if j == 4 else 0.0, 1000 + j))
    alone = [B.bs_sample(U, occ, ns, loss=l, seed=s) for U, occ, ns, l, s in jobs]
    say("case server mix")
    with B.Server(max_active_jobs=4) as srv:
        ids = [srv.submit(*jb) for jb in jobs]
        srv.drain()
        res = [srv.poll(i) for i in ids]
        st = srv.stats()
    for a, (s, lat) in zip(alone, res):
        assert np.array_equal(a, s)
        assert lat > 0
    assert st["jobs_done"] == 6 and st["max_active"] <= 4 and st["samples_done"] == 48


def test_server_admission_tiny_budget_queues():
    with B.Server(hbm_budget_bytes=1, max_active_jobs=8) as srv:
        ids = []
        for j in range(3):
            U = I.haar_unitary(200 + j, 8)
            ids.append(srv.submit(U, [1, 1, 1, 0, 0, 0, 0, 0], 4, seed=j))
        srv.drain()
        st = srv.stats()
        for i in ids:
            r = srv.poll(i)
            assert r is not None and r[0].shape == (4, 8)
    # a budget smaller than any job admits one job at a time (never zero)
    assert st["max_active"] == 1 and st["jobs_done"] == 3


def test_server_poll_busy_and_unknown():
    with B.Server(max_active_jobs=2) as srv:
        U = I.haar_unitary(3, 20)
        occ = np.zeros(20, dtype=np.int32)
        occ[:8] = 1
        jid = srv.submit(U, occ, 4, seed=1)
        t0 = time.time()
        r = None
        while r is None and time.time() - t0 < 60:
            r = srv.poll(jid)
            time.sleep(0.001)
        assert r is not None
        with pytest.raises(B.BBFGError) as e:
            srv.poll(jid)  # already collected
        assert e.value.code == B.BBFG_ENOTFOUND


def _rows_of(counts):
    rows = np.nonzero(counts)[0]
    return rows, counts[rows].astype(np.int32)


def test_c5_n40_ideal_and_lossy_sampling(oracle):
    """Large sampling (40 photons in the first 40 of 60 modes of Haar(5)), ideal
    and with transmission 0.5 through the 120 x 120 dilation.  The n = 40
    permanents are beyond the oracle, so their parity rests on spot checks:
    (i) the leave-one-column-out walk at 40 columns against independent single
    permanents (other split, other column order) within their error estimates,
    and the Laplace identity at 40 x 40; (ii) a minor of the same matrix and a
    sampled row pattern that the oracle can evaluate."""
    U, occ, _ = I.c5(False)
    say("case c5 ideal")
    s1 = B.bs_sample(U, occ, 1, 0.0, 5)
    assert s1.sum() == 40 and (s1 >= 0).all()
    assert np.array_equal(B.bs_sample(U, occ, 1, 0.0, 5), s1)
    say("case c5 lossy")
    U2, occ2, loss = I.c5(True)
    s2 = B.bs_sample(U2, occ2, 1, loss, 6)
    assert 0 <= s2.sum() <= 40 and (s2 >= 0).all()
    with B.Server() as srv:
        j = srv.submit(U2, occ2, 1, loss, 6)
        srv.drain()
        got, _ = srv.poll(j)
    assert np.array_equal(got, s2)

    # (i) minors of the sampled pattern with one photon removed, 40 columns
    counts = s1[0].copy()
    r_drop = int(np.nonzero(counts)[0][0])
    counts[r_drop] -= 1
    rows, M = _rows_of(counts)
    A = np.ascontiguousarray(U[rows][:, :40])
    say(f"case c5 minors K=40 rows={len(rows)}")
    minors = B.perm_minors(A, M)
    for l in (0, 13, 39):
        v, info = B.perm_bbfg(np.ascontiguousarray(np.delete(A, l, axis=1)), M, with_info=True)
        assert abs(minors[l] - v) <= 2 * max(1e-10, info["rel_err_est"]) * abs(v), l
    for r in (r_drop, 59):
        lap = np.dot(U[r, :40], minors)
        full = counts.copy()
        full[r] += 1
        rr, Mr = _rows_of(full)
        v, info = B.perm_bbfg(np.ascontiguousarray(U[rr][:, :40]), Mr, with_info=True)
        assert abs(lap - v) <= 2 * max(1e-10, info["rel_err_est"]) * abs(v), r

    # (ii) oracle spot check: 20 of the sampled photons, 21 columns
    sub = np.zeros(60, dtype=np.int64)
    left = 20
    for r in np.nonzero(s1[0])[0]:
        take = min(left, int(s1[0][r]))
        sub[r] = take
        left -= take
        if left == 0:
            break
    rows, M = _rows_of(sub)
    A = np.ascontiguousarray(U[rows][:, :21])
    minors = B.perm_minors(A, M)
    for l in (0, 20):
        ref, absum = oracle.perm_generalized(np.delete(A, l, axis=1), M, with_abs=True)
        assert abs(minors[l] - ref) <= max(1e-10, absum / abs(ref) * 84 * 2.0 ** -53) * abs(ref), l
