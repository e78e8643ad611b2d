"""GPU tests of Clifford & Clifford sampling (bs_sample) and the continuous-batching
server, against the CPU oracle sampler (same SplitMix64 draws, direct k x k
permanents instead of Laplace minors) and Eq. (bs_p)."""
import json
import os
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


@pytest.mark.parametrize("name", ["m60_n16", "m60_n20"])
def test_sampler_matches_stored_oracle_samples(name):
    """Samples of the oracle's sampler (direct k x k permanents of every
    candidate, no Laplace minors) stored by tests/golden/make_golden.py: 16 and
    20 photons in the first modes of a 60-mode Haar unitary, so the steps'
    minors run in the 16- and 24-column kernels.  Same draws, same samples."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "sampler_golden.json")) as fh:
        case = next(c for c in json.load(fh)["cases"] if c["name"] == name)
    U = np.array([complex(x, y) for x, y in case["U"]]).reshape(60, 60)
    say(f"case stored oracle samples {name}")
    g = B.bs_sample(U, case["occ"], case["n_samples"], seed=case["seed"])
    compare_samples(g, np.asarray(case["samples"], dtype=np.int32), name)


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
    minors, est = B.perm_minors(A, M, with_err=True)
    for l in (0, 20):
        ref, absum = oracle.perm_generalized(np.delete(A, l, axis=1), M, with_abs=True)
        e = abs(minors[l] - ref) / abs(ref)
        assert e <= est[l], l
        if absum / abs(ref) <= 1e6:
            assert e <= 1e-10, l


# ---------------------------------------------------------------------------
# Non-uniform loss (Sec. 4): the lossy interferometer matrix T
# ---------------------------------------------------------------------------

def _lossy_matrices(m, seed):
    rng = np.random.default_rng(seed)
    U = I.haar_unitary(500 + seed, m)
    eta_in = rng.uniform(0.2, 1.0, m)
    eta_out = rng.uniform(0.2, 1.0, m)
    Z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    general = 0.95 * Z / np.linalg.norm(Z, 2)          # a generic contraction
    return {"inputs": U * np.sqrt(eta_in)[None, :], "outputs": np.sqrt(eta_out)[:, None] * U,
            "uniform": np.sqrt(0.6) * U, "general": general, "lossless": U}


@pytest.mark.parametrize("m,occ,seed", [
    (6, [1, 1, 1, 0, 0, 0], 1),
    (8, [2, 0, 1, 1, 0, 0, 0, 1], 2),
    (12, [1] * 6 + [0] * 6, 3),
])
def test_bs_sample_lossy_matches_oracle_sampler(oracle, m, occ, seed):
    """bs_sample_lossy against the oracle's sampler on the same isometry
    [T; R] (R the Cholesky factor of I - T^H T, built independently on each
    side): the same draws give the same samples, for per-input-mode,
    per-output-mode, uniform, generic and no loss."""
    for kind, T in _lossy_matrices(m, seed).items():
        say(f"case bs_sample_lossy m={m} occ={occ} {kind}")
        g, info = B.bs_sample_lossy(T, occ, 40, seed=seed, with_info=True)
        c = oracle.cc_sample_lossy(T, occ, 40, seed)
        compare_samples(g, c, f"{kind} m={m}")
        assert (g.sum(axis=1) <= sum(occ)).all()
        if kind == "lossless":
            assert (g.sum(axis=1) == sum(occ)).all()
        assert 0.0 <= info["rel_err_est"] < 1e-9


@pytest.mark.parametrize("m,n,loss,seed", [(12, 6, 0.3, 5), (12, 8, 0.6, 6), (60, 16, 0.5, 7), (60, 20, 0.4, 8)])
def test_bs_sample_extracted_matches_oracle_sampler(oracle, m, n, loss, seed):
    """Uniform loss taken out at the input (Sec. 4): each photon survives with
    probability 1 - loss and the survivors are sampled on U's m modes.  The
    same draws give the same samples as the oracle's extraction sampler."""
    U = I.haar_unitary(60 + seed, m)
    occ = np.zeros(m, dtype=np.int32)
    occ[:n] = 1
    say(f"case bs_sample_extracted m={m} n={n} loss={loss}")
    g, info = B.bs_sample_extracted(U, occ, 30, loss, seed, with_info=True)
    c = oracle.cc_sample_extracted(U, occ, 30, loss, seed)
    compare_samples(g, c, f"extracted m={m} n={n} loss={loss}")
    assert (g.sum(axis=1) <= n).all()
    assert 0.0 <= info["rel_err_est"] < 1e-6


def test_bs_sample_extracted_edges():
    """No loss: exactly the ideal samples of bs_sample.  Heavy loss: samples
    with no surviving photon are all-zero rows, and the number of survivors
    follows Binomial(n, 1 - loss)."""
    U = I.haar_unitary(70, 10)
    occ = [1, 1, 0, 2, 1, 0, 0, 1, 0, 0]
    assert np.array_equal(B.bs_sample_extracted(U, occ, 40, 0.0, 3), B.bs_sample(U, occ, 40, 0.0, 3))
    N, n, keep = 3000, 6, 0.15
    s = B.bs_sample_extracted(U, occ, N, 1 - keep, 4)
    k = s.sum(axis=1)
    assert (k == 0).any() and (k <= n).all()
    assert abs(k.mean() - n * keep) < 4 * np.sqrt(n * keep * (1 - keep) / N)
    assert abs((k == 0).mean() - (1 - keep) ** n) < 4 * np.sqrt((1 - keep) ** n / N)


def test_lossy_per_mode_photon_survival():
    """Losses at the inputs, T = U diag(sqrt(eta)): each photon entering mode i
    is detected with probability eta_i, independently, so the number detected
    follows the Poisson-binomial law of the occupied modes' eta."""
    m = 8
    U = I.haar_unitary(77, m)
    eta = np.array([0.95, 0.8, 0.6, 0.3, 0.5, 0.9, 0.7, 0.4])
    occ = [1, 1, 1, 1, 0, 0, 0, 0]
    N = 6000
    s = B.bs_sample_lossy(U * np.sqrt(eta)[None, :], occ, N, seed=12)
    law = np.array([1.0])
    for e in eta[:4]:
        law = np.convolve(law, [1 - e, e])
    k = s.sum(axis=1)
    emp = np.array([(k == j).mean() for j in range(5)])
    assert 0.5 * np.abs(emp - law).sum() < 0.03, (emp, law)
    # output losses: the detected count has mean sum_j eta_j <n_j> with <n_j> the
    # lossless mean occupation, checked against 6000 lossless samples
    T = np.sqrt(eta)[:, None] * U
    so = B.bs_sample_lossy(T, occ, N, seed=13)
    full = B.bs_sample(U, occ, N, seed=14)
    mean_lossless = full.mean(axis=0)
    assert abs(so.sum(axis=1).mean() - (eta * mean_lossless).sum()) < 0.06


def test_lossy_uniform_matrix_law_equals_scalar_loss(oracle):
    """T = sqrt(eta) U and the scalar loss 1 - eta are the same channel: their
    output histograms agree (different isometries, so different samples)."""
    m, occ, eta = 5, [1, 1, 1, 0, 0], 0.6
    U = I.haar_unitary(88, m)
    N = 20000
    a = B.bs_sample_lossy(np.sqrt(eta) * U, occ, N, seed=1)
    b = B.bs_sample(U, occ, N, loss=1 - eta, seed=2)
    ca, cb = {}, {}
    for row in a:
        ca[tuple(row)] = ca.get(tuple(row), 0) + 1
    for row in b:
        cb[tuple(row)] = cb.get(tuple(row), 0) + 1
    keys = set(ca) | set(cb)
    tv = 0.5 * sum(abs(ca.get(k, 0) - cb.get(k, 0)) / N for k in keys)
    assert tv < 0.04, tv


def test_server_lossy_jobs_and_cancel():
    """Lossy-matrix jobs through the server equal bs_sample_lossy alone; a
    cancelled queued job and a cancelled running job both poll as cancelled,
    and the other jobs' samples are unchanged."""
    m = 10
    T = _lossy_matrices(m, 9)["general"]
    occ = [1] * 5 + [0] * 5
    alone = B.bs_sample_lossy(T, occ, 16, seed=31)
    U, occ4, ns, loss, seed4 = I.c4_job(3)
    occ4 = np.zeros(60, dtype=np.int32)
    occ4[:24] = 1
    with B.Server(max_active_jobs=2) as srv:
        j_long = srv.submit(U, occ4, 64, seed=seed4)          # occupies the device for a while
        j_lossy = srv.submit_lossy(T, occ, 16, seed=31)
        j_queued = srv.submit(U, occ4, 16, seed=5)            # waits for a slot
        srv.cancel(j_queued)
        srv.cancel(j_long)
        srv.drain()
        got = srv.poll(j_lossy, with_err=True)
        assert got is not None
        assert np.array_equal(got[0], alone)
        assert got[2] >= 0.0
        for j in (j_queued, j_long):
            with pytest.raises(B.BBFGError) as e:
                srv.poll(j)
            assert e.value.code == B.BBFG_ECANCELED
        st = srv.stats()
        assert st["jobs_cancelled"] == 2
        # the server keeps working after cancellations
        j2 = srv.submit_lossy(T, occ, 16, seed=31)
        srv.drain()
        assert np.array_equal(srv.poll(j2)[0], alone)


def test_server_extracted_jobs_equal_alone():
    """Input-loss jobs through the server (mixed with ideal jobs, one of them at
    a loss that leaves many samples without photons) equal bs_sample_extracted
    alone, sample for sample."""
    U = I.haar_unitary(81, 60)
    occ = np.zeros(60, dtype=np.int32)
    occ[:20] = 1
    cases = [(0.5, 11), (0.95, 12), (0.2, 13)]
    alone = [B.bs_sample_extracted(U, occ, 16, loss, seed) for loss, seed in cases]
    ideal = B.bs_sample(U, occ, 8, 0.0, 14)
    with B.Server(max_active_jobs=4) as srv:
        jid = [srv.submit_extracted(U, occ, 16, loss, seed) for loss, seed in cases]
        j_ideal = srv.submit(U, occ, 8, seed=14)
        srv.drain()
        for j, a in zip(jid, alone):
            assert np.array_equal(srv.poll(j)[0], a)
        assert np.array_equal(srv.poll(j_ideal)[0], ideal)
    assert (alone[1].sum(axis=1) == 0).any()


def test_sampler_error_estimate_reported():
    """Every sample's law carries an error estimate (sum over its steps of the
    draw distribution's estimated total-variation error, from the minors'
    estimates): positive and small for a 24-photon job, and returned by the
    server's poll for the same job."""
    U, occ, ns, loss, seed = I.c4_job(1)
    occ = np.zeros(60, dtype=np.int32)
    occ[:24] = 1
    s, info = B.bs_sample(U, occ, 8, seed=seed, with_info=True)
    say(f"  24-photon sampler error estimate {info['rel_err_est']:.2e}")
    assert 0.0 < info["rel_err_est"] < 1e-6
    with B.Server() as srv:
        j = srv.submit(U, occ, 8, seed=seed)
        srv.drain()
        got, lat, err = srv.poll(j, with_err=True)
    assert np.array_equal(got, s)
    assert err == info["rel_err_est"]
