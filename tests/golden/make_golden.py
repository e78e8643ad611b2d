"""Writes the stored oracle values of the full-size workloads.

Calls only the double-double CPU oracle (oracle/) and the seeded input
generators; nothing here touches the GPU library.

    python tests/golden/make_golden.py perm      # perm_golden.json: n = 30 cases, 32 batch items (~10 min)
    python tests/golden/make_golden.py c3        # c3_all.txt: all 4096 batch items (~30 min on 8 cores)
    python tests/golden/make_golden.py minors    # minors_golden.json: 30-40-column minors (~20 min)
    python tests/golden/make_golden.py sampler   # sampler_golden.json: 60-mode samples (~10 min)
    python tests/golden/make_golden.py cols      # cols_golden.json: column multiplicities, n = 24 .. 48 (~10 min)

perm_golden.json, minors_golden.json and sampler_golden.json store their input
matrices next to the values (as exact float reprs), so the GPU tests compare
against the very inputs the oracle saw, whatever LAPACK build regenerates them.
c3_all.txt stores, per item, a hash of the input bytes instead (the 4096
matrices would take ~16 MB): a test that regenerates an item with different
bits sees the hash differ.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2309_07027_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "perm_golden.json")
OUT_C3 = os.path.join(HERE, "c3_all.txt")
OUT_MINORS = os.path.join(HERE, "minors_golden.json")
OUT_SAMPLER = os.path.join(HERE, "sampler_golden.json")
OUT_COLS = os.path.join(HERE, "cols_golden.json")
C3_SAMPLE = list(range(0, 4096, 128))


def enc(A):
    return [[float(x.real), float(x.imag)] for x in np.asarray(A).ravel()]


def record(name, A, M, full, abs_sum, method, secs):
    v = full[1]
    val = complex(v[0] + v[1], v[2] + v[3])
    return {
        "name": name, "rows": int(A.shape[0]), "cols": int(A.shape[1]), "A": enc(A),
        "M": [int(x) for x in M], "re": [float(v[0]), float(v[1])], "im": [float(v[2]), float(v[3])],
        "abs_sum": abs_sum, "kappa": (abs_sum / abs(val)) if abs_sum else None,
        "method": method, "oracle_seconds": secs,
    }


def input_hash(A, M) -> str:
    """First 16 hex digits of SHA-256 over the complex128 bytes of A and the int32 bytes of M."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(A, dtype=np.complex128).tobytes())
    h.update(np.ascontiguousarray(M, dtype=np.int32).tobytes())
    return h.hexdigest()[:16]


def main_c3():
    """Every item of the 4096-item batch: one text line per item,
    'index n rows hash re im abs_sum' (re, im the double-double value rounded
    to double, abs_sum = 2^{1-n} sum |addend| of Eq. bbfgrepeated)."""
    t0 = time.time()
    lines = ["# item n rows input_sha256_16 re im abs_sum  (Eq. bbfgrepeated, double-double oracle)"]
    for i in range(4096):
        A, M = I.c3_item(i)
        v, ab = O.perm_generalized(A, M, with_abs=True)
        lines.append(f"{i} {A.shape[1]} {A.shape[0]} {input_hash(A, M)} {v.real!r} {v.imag!r} {ab:.6e}")
        if i % 256 == 255:
            print(f"c3 {i + 1}/4096 {time.time() - t0:.0f}s", flush=True)
    with open(OUT_C3, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", OUT_C3)


# Leave-one-column-out (Laplace) minors of one sampler-like step: the first
# len(M) rows of a Haar unitary with multiplicities M and its first K columns.
MINOR_CASES = [
    # (name, Haar seed, K, M): K = 30 with all M = 1 (2^28 addends per minor) runs
    # in the 25-30-column kernel; the bunched cases (kappa 3e4 .. 9e5) in the
    # 31-32- and 33-48-column kernels
    ("k30_distinct", 300, 30, [1] * 29),
    ("k32_bunched", 300, 32, [4, 4, 4, 4, 4, 3, 3, 5]),
    ("k36_bunched", 300, 36, [4] * 8 + [3]),
    ("k37_bunched", 300, 37, [4] * 9),
    ("k40_bunched", 300, 40, [5] * 7 + [4]),
]


def main_minors():
    cases = []
    for name, seed, K, M in MINOR_CASES:
        U = I.haar_unitary(seed)
        A = np.ascontiguousarray(U[:len(M), :K])
        M = np.asarray(M, dtype=np.int32)
        t = time.time()
        vals, absums = [], []
        for l in range(K):
            B = np.ascontiguousarray(np.delete(A, l, axis=1))
            if (M == 1).all():
                (v, lo) = O.perm_glynn_gray(B, full=True)
                ab = None
            else:
                (v, lo), ab = O.perm_generalized(B, M, full=True, with_abs=True)
            vals.append([float(lo[0]), float(lo[1]), float(lo[2]), float(lo[3])])
            absums.append(ab)
            print(name, l, f"{time.time() - t:.0f}s", flush=True)
        cases.append({"name": name, "seed": seed, "K": K, "M": [int(x) for x in M], "A": enc(A),
                      "minors": vals, "abs_sum": absums,
                      "method": "Gray-coded Eq. bbfg (Sec. 2.1)" if (M == 1).all()
                      else "generalized (Eq. bbfgrepeated, lexicographic)",
                      "oracle_seconds": time.time() - t})
    meta = {"oracle_threads": O.get_threads(), "generator": "tests/golden/make_golden.py minors",
            "note": "minors[l] = perm(A without column l, M) as double-double re_hi re_lo im_hi im_lo"}
    with open(OUT_MINORS, "w") as fh:
        json.dump({"meta": meta, "cases": cases}, fh)
    print("wrote", OUT_MINORS)


# Clifford & Clifford samples of the oracle's sampler (direct k x k permanents
# for every candidate, no Laplace expansion): n photons in the first n of 60
# modes of a Haar unitary.
SAMPLER_CASES = [("m60_n16", 61, 16, 8, 1601), ("m60_n20", 61, 20, 4, 2001)]


def main_sampler():
    cases = []
    for name, seed, n, count, sseed in SAMPLER_CASES:
        U = I.haar_unitary(seed)
        occ = np.zeros(I.M_MODES, dtype=np.int32)
        occ[:n] = 1
        t = time.time()
        out = O.cc_sample(U, occ, count, 0.0, sseed)
        cases.append({"name": name, "haar_seed": seed, "U": enc(U), "occ": occ.tolist(), "n_samples": count,
                      "seed": sseed, "samples": out.tolist(), "oracle_seconds": time.time() - t})
        print(name, f"{time.time() - t:.0f}s", flush=True)
    meta = {"oracle_threads": O.get_threads(), "generator": "tests/golden/make_golden.py sampler"}
    with open(OUT_SAMPLER, "w") as fh:
        json.dump({"meta": meta, "cases": cases}, fh)
    print("wrote", OUT_SAMPLER)


# Row AND column multiplicities (Eq. bbfgrepeated): len(M) rows of a Haar
# unitary with multiplicities M, `ncols` distinct columns from column 30 on with
# multiplicities N (None: n photons dropped at random on the columns).  Equal
# N = 2 on 17 .. 24 distinct columns runs the column-power kernel's 24-column
# bucket; mixed N the column-expanded walk at n = 24 .. 32.
COLS_CASES = [
    ("e2_c17", 400, [4] * 6 + [5] * 2, 17, [2] * 17),
    ("e2_c20", 401, [5] * 8, 20, [2] * 20),
    ("e2_c22", 406, [4] * 6 + [5] * 4, 22, [2] * 22),
    ("e2_c24", 402, [6] * 8, 24, [2] * 24),
    ("mixed_n24", 403, [4] * 6, 15, None),
    ("mixed_n28", 404, [4] * 7, 18, None),
    ("mixed_n32", 405, [4] * 8, 20, None),
]


def main_cols():
    cases = []
    for name, seed, M, ncols, N in COLS_CASES:
        U = I.haar_unitary(seed)
        rng = np.random.default_rng(seed)
        n = sum(M)
        if N is None:
            N = np.bincount(rng.integers(0, ncols, n), minlength=ncols)
            N = N[N > 0]
        N = np.asarray(N, dtype=np.int32)
        A = np.ascontiguousarray(U[:len(M), 30:30 + len(N)])
        t = time.time()
        (v, lo), ab = O.perm_generalized(np.repeat(A, N, axis=1), np.asarray(M, dtype=np.int32), full=True,
                                         with_abs=True)
        cases.append({"name": name, "seed": seed, "M": [int(x) for x in M], "N": N.tolist(), "A": enc(A),
                      "re": [float(lo[0]), float(lo[1])], "im": [float(lo[2]), float(lo[3])], "abs_sum": ab,
                      "method": "generalized (Eq. bbfgrepeated, lexicographic) on the column-expanded matrix",
                      "oracle_seconds": time.time() - t})
        print(name, f"{time.time() - t:.0f}s", flush=True)
    meta = {"oracle_threads": O.get_threads(), "generator": "tests/golden/make_golden.py cols",
            "note": "complex results as double-double: value = hi + lo"}
    with open(OUT_COLS, "w") as fh:
        json.dump({"meta": meta, "cases": cases}, fh)
    print("wrote", OUT_COLS)


def main():
    cases = []
    for name, f in (("c2b", I.c2b), ("c2c", I.c2c)):
        A, M = f()
        t = time.time()
        full, ab = O.perm_generalized(A, M, full=True, with_abs=True)
        cases.append(record(name, A, M, full, ab, "generalized (Eq. bbfgrepeated, lexicographic)", time.time() - t))
        print(name, cases[-1]["oracle_seconds"], flush=True)
    A, M = I.c2a()
    t = time.time()
    full = O.perm_glynn_gray(A, full=True)
    cases.append(record("c2a", A, M, full, None, "Gray-coded Eq. bbfg (Sec. 2.1)", time.time() - t))
    print("c2a", cases[-1]["oracle_seconds"], flush=True)
    for i in C3_SAMPLE:
        A, M = I.c3_item(i)
        t = time.time()
        full, ab = O.perm_generalized(A, M, full=True, with_abs=True)
        cases.append(record(f"c3_{i}", A, M, full, ab, "generalized (Eq. bbfgrepeated, lexicographic)",
                            time.time() - t))
    print("c3 sample done", flush=True)
    meta = {"oracle_threads": O.get_threads(), "generator": "tests/golden/make_golden.py",
            "note": "complex results as double-double: value = hi + lo"}
    with open(OUT, "w") as fh:
        json.dump({"meta": meta, "cases": cases}, fh)
    print("wrote", OUT)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "perm"
    {"perm": main, "c3": main_c3, "minors": main_minors, "sampler": main_sampler, "cols": main_cols}[what]()
