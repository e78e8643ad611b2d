"""Writes tests/golden/perm_golden.json: oracle values of the full-size workloads.

Calls only the double-double CPU oracle (oracle/) and the seeded input
generators; nothing here touches the GPU library.  The input matrices are
stored next to the values (as exact float reprs), so the GPU tests compare
against the very inputs the oracle saw, whatever LAPACK build regenerates them.

    python tests/golden/make_golden.py            # all cases (~10 min on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2309_07027_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "perm_golden.json")
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
    main()
