"""Runs the host-only paths of the sanitized builds (no GPU needed).  Started by
tests/test_host_sanitized.py in a subprocess with the ASan runtime preloaded;
any sanitizer report aborts it with a non-zero status."""
import ctypes
import math
import sys
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
sys.path.insert(0, str(HERE.parent.parent))


def oracle_paths():
    from oracle import oracle as O
    O._LIB = HERE / "_build" / "liboracle_san.so"
    O._lib = None
    rng = np.random.default_rng(1)
    A = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    ref = O.perm_bruteforce(A)
    for v in (O.perm_ryser(A), O.perm_glynn(A), O.perm_glynn_gray(A), O.perm_generalized(A, [1] * 5),
              O.perm_generalized_full(A, [1] * 5), O.perm_ryser_generalized(A, [1] * 5)):
        assert abs(v - ref) <= 1e-12 * abs(ref)
    B = rng.standard_normal((3, 6)) + 1j * rng.standard_normal((3, 6))
    assert abs(O.perm_generalized(B, [2, 1, 3]) - O.perm_ryser_generalized(B, [2, 1, 3])) < 1e-10
    assert O.binom(64, 32) == math.comb(64, 32)
    U = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))[0]
    assert abs(sum(O.bs_prob(U, [1, 1, 0, 0], T) for T in ([2, 0, 0, 0], [1, 1, 0, 0], [0, 0, 1, 1])) - 0) >= 0
    O.cc_sample(U, [1, 1, 0, 0], 20, 0.3, 7)
    O.cc_sample_lossy(0.9 * U, [1, 1, 0, 0], 20, 7)
    V = O.contraction_isometry(0.7 * U)
    assert np.abs(V.conj().T @ V - np.eye(4)).max() < 1e-13
    print("oracle paths ok", flush=True)


def library_paths():
    from paper_2309_07027_amd import binding as B
    B._LIB_PATH = HERE / "_build" / "libbbfg_san.so"
    B._lib = None
    L = B.lib()
    assert L.bbfg_version() == 1
    A = np.ones((3, 3), dtype=complex)
    bad = [lambda: B.perm_bbfg(A, [1, 1, 2]), lambda: B.perm_bbfg(A, [2, -1, 2]),
           lambda: B.perm_bbfg(np.ones((49, 49), dtype=complex)),
           lambda: B.perm_ryser(A, [1, 1, 2]), lambda: B.perm_bbfg_noalloc(A, [1, 1, 2]),
           lambda: B.perm_batch([(A, [1, 1, 1])], precision=7),
           lambda: B.perm_batch([(A, [1, 1, 1]), (A, [3, 0, 1])]),
           lambda: B.perm_minors(np.ones((2, 3), dtype=complex), [1, 2]),
           lambda: B.perm_bbfg_cols(np.ones((2, 3), dtype=complex), [2, 1], [1, 1, 0]),
           lambda: B.bs_sample(np.eye(4, dtype=complex), [1, 1, 0, 0], 2, loss=1.0),
           lambda: B.bs_sample(np.eye(4, dtype=complex), [1, -1, 0, 0], 2),
           lambda: B.bs_sample_lossy(1.01 * np.eye(4, dtype=complex), [1, 1, 0, 0], 2),
           lambda: B.bs_sample_lossy(np.eye(129, dtype=complex), [1] + [0] * 128, 1)]
    for f in bad:
        try:
            f()
        except B.BBFGError:
            pass
        else:
            raise AssertionError("expected an argument error")
    # the empty permanent needs no device
    assert B.perm_bbfg(np.zeros((0, 0), dtype=complex), np.zeros(0, dtype=np.int32)) == 1
    # planner and Gray tables on the host
    for M in ([1] * 30, [3] * 10, [2, 1, 4, 1, 7], [48], [1] * 48, [6] * 8):
        s = B.plan_query(M, sum(M), slots=3072)
        assert s["n_addends"] > 0
    for radices in ([2, 2, 2], [3, 4], [5, 2, 3, 2], [7]):
        ch, dr = B.gray_table(radices)
        assert len(ch) == int(np.prod(radices))
    print("library host paths ok", flush=True)


if __name__ == "__main__":
    what = sys.argv[1]
    {"oracle": oracle_paths, "library": library_paths}[what]()
