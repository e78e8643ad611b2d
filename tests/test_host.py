"""Host-side tests of the C-ABI library (no GPU needed): the library loads and
exports every entry point of include/bbfg.h, arguments are validated before any
device work, and the planner's n-ary Gray code and work split are right."""
import itertools
import math
import os
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2309_07027_amd import binding as B

ROOT = Path(__file__).resolve().parents[1]


def header_functions():
    text = (ROOT / "include" / "bbfg.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "for", "while", "return", "sizeof")))


def test_header_symbols_exported_and_bound():
    L = B.lib()
    names = header_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
        assert n in B.SIGNATURES, n
    assert set(B.SIGNATURES) == set(names)
    assert L.bbfg_version() == 1


def test_library_is_gfx950_code_object():
    data = Path(B.library_path()).read_bytes()
    assert b"gfx950" in data


# ---------------------------------------------------------------------------
# argument validation (returns before touching a device)
# ---------------------------------------------------------------------------

def test_validation_errors():
    A = np.ones((3, 3), dtype=complex)
    with pytest.raises(B.BBFGError) as e:
        B.perm_bbfg(A, [1, 1, 2])  # sum != n_cols
    assert e.value.code == B.BBFG_EINVAL and "differs" in str(e.value)
    with pytest.raises(B.BBFGError) as e:
        B.perm_bbfg(A, [2, -1, 2])
    assert e.value.code == B.BBFG_EINVAL
    big = np.ones((49, 49), dtype=complex)
    with pytest.raises(B.BBFGError) as e:
        B.perm_bbfg(big)
    assert e.value.code == B.BBFG_ERANGE
    with pytest.raises(B.BBFGError) as e:
        B.perm_batch([(A, [1, 1, 1])], precision=7)
    assert e.value.code == B.BBFG_EINVAL
    with pytest.raises(B.BBFGError) as e:
        B.perm_batch([(np.ones((25, 25), dtype=complex), np.ones(25))], precision=B.BBFG_FP32)
    assert e.value.code == B.BBFG_ERANGE
    with pytest.raises(B.BBFGError) as e:
        B.perm_batch([(A, [1, 1, 1]), (A, [3, 0, 1])])
    assert e.value.code == B.BBFG_EINVAL and "item 1" in str(e.value)
    U = np.eye(4, dtype=complex)
    with pytest.raises(B.BBFGError) as e:
        B.bs_sample(U, [1, 1, 0, 0], 2, loss=1.0)
    assert e.value.code == B.BBFG_EINVAL
    with pytest.raises(B.BBFGError) as e:
        B.bs_sample(U, [1, -1, 0, 0], 2)
    assert e.value.code == B.BBFG_EINVAL
    with pytest.raises(B.BBFGError) as e:
        B.bs_sample(np.eye(130, dtype=complex), [1] + [0] * 129, 1, loss=0.5)
    assert e.value.code == B.BBFG_ERANGE
    occ = np.zeros(60, dtype=np.int32)
    occ[:49] = 1
    with pytest.raises(B.BBFGError) as e:
        B.bs_sample(np.eye(60, dtype=complex), occ, 1)
    assert e.value.code == B.BBFG_ERANGE
    # the lossy interferometer matrix must be a contraction (checked on the host)
    with pytest.raises(B.BBFGError) as e:
        B.bs_sample_lossy(1.01 * U, [1, 1, 0, 0], 2)
    assert e.value.code == B.BBFG_EINVAL and "contraction" in str(e.value)
    with pytest.raises(B.BBFGError) as e:
        B.bs_sample_lossy(np.eye(129, dtype=complex), [1] + [0] * 128, 1)
    assert e.value.code == B.BBFG_ERANGE


def test_empty_permanent_is_one_without_device():
    assert B.perm_bbfg(np.zeros((0, 0), dtype=complex), np.zeros(0, dtype=np.int32)) == 1
    # rows with multiplicity zero and no columns
    assert B.perm_bbfg(np.zeros((3, 0), dtype=complex), [0, 0, 0]) == 1
    out = B.perm_batch([(np.zeros((0, 0), dtype=complex), np.zeros(0, dtype=np.int32))] * 3)
    assert (out == 1).all()


# ---------------------------------------------------------------------------
# the n-ary reflected Gray code walked inside a block (Sec. 2.1, 2.2)
# ---------------------------------------------------------------------------

def walk(radices):
    ch, dr = B.gray_table(radices)
    cur = [0] * len(radices)
    seq = [tuple(cur)]
    for t in range(1, len(ch)):
        cur[ch[t]] += dr[t]
        seq.append(tuple(cur))
    return ch, dr, seq


def test_binary_gray_matches_paper_table():
    # Table "gray" (Sec. 2.1): decimal index -> 3-bit reflected Gray code.
    rows = [l.split() for l in (ROOT / "tests" / "golden" / "table_gray.txt").read_text().splitlines()
            if l and not l.startswith("#")]
    _, _, seq = walk([2, 2, 2])
    for (idx, code), digits in zip(rows, seq):
        assert code == "".join(str(d) for d in reversed(digits)), idx
    # the changed bit is the lowest set bit of the index
    ch, _, _ = walk([2] * 6)
    for i in range(1, 64):
        assert ch[i] == (i & -i).bit_length() - 1


@pytest.mark.parametrize("radices", [[3, 3], [2, 4, 3], [4, 1, 2, 5], [5], [2, 2, 2, 2], [7, 3, 2]])
def test_mixed_radix_gray_invariants(radices):
    ch, dr, seq = walk(radices)
    total = math.prod(radices)
    assert len(seq) == total
    # bijection onto the whole box
    assert sorted(seq) == sorted(itertools.product(*[range(r) for r in radices]))
    for t in range(1, total):
        diff = [a - b for a, b in zip(seq[t], seq[t - 1])]
        assert sum(1 for d in diff if d) == 1 and sum(abs(d) for d in diff) == 1
        # the changed digit is the lowest nonzero mixed-radix digit of t
        x, k = t, 0
        while x % radices[k] == 0:
            x //= radices[k]
            k += 1
        assert ch[t] == k
        # the digit moves up exactly when the number above it is even
        q = t
        for r in radices[: k + 1]:
            q //= r
        assert dr[t] == (1 if q % 2 == 0 else -1)


# ---------------------------------------------------------------------------
# planner
# ---------------------------------------------------------------------------

def cprime(M):
    M = [m for m in M if m > 0]
    p = min(range(len(M)), key=lambda i: (M[i], i))
    Mp = list(M)
    Mp[p] -= 1
    return math.prod(m + 1 for m in Mp), p


@pytest.mark.parametrize("M", [[1] * 30, [3] * 10, [1, 2, 0, 4, 1, 3], [5], [2, 2], [1] * 7, [1] * 3,
                               [40], [1] * 48, [2, 1, 1, 3, 1, 2, 1, 1, 1, 2, 1, 1]])
@pytest.mark.parametrize("slots", [1024, 3072, 4096])
def test_plan_split(M, slots):
    n = sum(M)
    s = B.plan_query(M, n, slots=slots)
    C, p = cprime(M)
    assert s["n_addends"] == C
    assert s["lane_product"] * s["high_count"] * s["low_count"] == C
    assert s["lane_groups"] == -(-s["lane_product"] // 64)
    kept = [i for i, m in enumerate(M) if m > 0]
    assert s["pivot_row"] == kept[p]
    assert s["n_rows_kept"] == len(kept)
    assert s["low_count"] <= 4096
    assert s["n_units"] >= s["lane_groups"]
    # large sums fill whole rounds of resident wavefronts
    if s["lane_groups"] * s["high_count"] * s["low_count"] >= slots * 256:
        assert s["n_units"] <= slots * max(1, round(s["lane_groups"] * s["high_count"] * s["low_count"]
                                                      / (slots * 1024)))
    if C >= 64 and all(m == 1 for m in M):
        assert s["lane_product"] == 64


def test_plan_c2_workloads():
    from paper_2309_07027_amd import inputs as I
    s = B.plan_query(*(lambda AM: (AM[1], AM[0].shape[1]))(I.c2a()), slots=3072)
    assert s["n_addends"] == 2 ** 29 and s["n_units"] == 3 * 3072 and s["lane_product"] == 64  # 3 rounds
    s = B.plan_query(*(lambda AM: (AM[1], AM[0].shape[1]))(I.c2b()), slots=3072)
    assert s["n_addends"] == 3 * 4 ** 9 and s["lane_product"] == 64


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with a message (no GPU work)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert p.returncode != 0 and "one GPU" in p.stderr


def test_sampling_cost_model_and_t0_fit():
    """Eq. performance at the paper's fitted T0 and 40 photons on 60 modes is about a
    minute per sample (the paper measured about 80 s); the fit recovers T0 exactly from
    model-generated times."""
    import bench
    from math import comb
    n, m = 40, 60
    direct = n * (m + n) / m * comb(2 * m + n, n + 1) / comb(m + n, n + 1) + n * n * m
    assert bench.cc_cost_model(n, m) == pytest.approx(direct, rel=1e-15)
    assert 50 < 7.5e-11 * bench.cc_cost_model(40, 60) < 80
    pts = [(k, mm, 3.1e-13 * bench.cc_cost_model(k, mm)) for k in (30, 34, 38) for mm in (60, 120)]
    assert bench.fit_t0(pts) == pytest.approx(3.1e-13, rel=1e-12)


def test_cpu_baseline_contract():
    """bench.py's cpu_baseline: the oracle timed as is, on all threads and on one,
    reported with the fields the bench line carries (tiny sample, CPU only)."""
    import bench
    cb = bench.cpu_baseline(1 << 12)
    assert cb["kind"] == "oracle" and cb["unit"] == "GFLOP/s"
    assert cb["value"] > 0 and cb["cores"] >= 1
    assert "addends [0, 4096)" in cb["sample"]
    st = cb["single_thread"]
    assert st["value"] > 0 and st["unit"] == "GFLOP/s" and "addends [0, 128)" in st["sample"]
    from oracle import oracle as O
    assert O.get_threads() == cb["cores"]  # thread count restored
