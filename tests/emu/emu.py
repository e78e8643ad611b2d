"""Build and run the CPU emulation of the permanent kernels (walk_emu.cpp)."""
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent.parent
CSRC = ROOT / "paper_2309_07027_amd" / "csrc"
EXE = HERE / "walk_emu"
SOURCES = [HERE / "walk_emu.cpp", CSRC / "plan.cpp"]
HEADERS = list(CSRC.glob("*.hpp")) + [ROOT / "include" / "bbfg.h"]
CMD = ["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-Wno-unknown-pragmas",
       f"-I{CSRC}", f"-I{ROOT / 'include'}", *map(str, SOURCES), "-o", str(EXE)]


def build():
    """Rebuilds the emulator when a source is newer.  Parallel test workers
    serialise on a lock file, and the binary is replaced atomically, so no
    worker runs a half-written one."""
    import fcntl

    def stale():
        newest = max(p.stat().st_mtime for p in SOURCES + HEADERS)
        return not EXE.exists() or EXE.stat().st_mtime < newest

    if not stale():
        return EXE
    with open(HERE / ".walk_emu.lock", "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        if stale():
            tmp = EXE.with_name(f"walk_emu.tmp{os.getpid()}")
            subprocess.run(CMD[:-1] + [str(tmp)], check=True)
            os.replace(tmp, EXE)
    return EXE


def run(A, M, slots: int, f32: bool = False, l_batch: int = 0, ryser: bool = False):
    """Emulated evaluation: (value, rel_err_est, kappa, units).  l_batch = 0 plans
    the permanent as perm_bbfg does; l_batch > 0 as a batched launch with that
    unit length.  ryser: Eq. ryser with row multiplicities on the same walk."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    r, n = A.shape
    lines = [f"{r} {n} {int(slots)} {1 if f32 else 0} {int(l_batch)} {3 if ryser else 0}",
             " ".join(str(int(m)) for m in M)]
    lines.append(" ".join(f"{float(x.real).hex()} {float(x.imag).hex()}" for x in A.ravel()))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    p = subprocess.run([str(EXE)], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env,
                       timeout=600)
    if p.returncode != 0:
        raise RuntimeError(f"walk_emu failed ({p.returncode}): {p.stderr[-2000:]}")
    re_, im_, err, kappa, units = p.stdout.split()
    return complex(float.fromhex(re_), float.fromhex(im_)), float.fromhex(err), float.fromhex(kappa), int(units)


def run_minors(A, M, l_batch: int, slots: int = 1, with_err: bool = False):
    """Emulated minors walk: [perm(A without column l, M) for each l], planned with
    unit length l_batch, or (l_batch = 0) to fill `slots` wavefront slots.
    with_err: also the per-minor (rel_err_est, kappa) arrays."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    r, n = A.shape
    lines = [f"{r} {n} {int(slots)} 0 {int(l_batch)} 1", " ".join(str(int(m)) for m in M)]
    lines.append(" ".join(f"{float(x.real).hex()} {float(x.imag).hex()}" for x in A.ravel()))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    p = subprocess.run([str(EXE)], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env,
                       timeout=600)
    if p.returncode != 0:
        raise RuntimeError(f"walk_emu failed ({p.returncode}): {p.stderr[-2000:]}")
    v = [float.fromhex(x) for x in p.stdout.split()]
    vals = np.array([complex(v[4 * i], v[4 * i + 1]) for i in range(n)])
    if with_err:
        return vals, np.array(v[2::4]), np.array(v[3::4])
    return vals


def run_cols(A, M, N, slots: int, l_batch: int = 0):
    """Emulated walk with column multiplicities N (A holds the distinct columns):
    (value, rel_err_est, kappa, units)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    r, n = A.shape
    lines = [f"{r} {n} {int(slots)} 0 {int(l_batch)} 2", " ".join(str(int(m)) for m in M),
             " ".join(str(int(x)) for x in N)]
    lines.append(" ".join(f"{float(x.real).hex()} {float(x.imag).hex()}" for x in A.ravel()))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    p = subprocess.run([str(EXE)], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env,
                       timeout=600)
    if p.returncode != 0:
        raise RuntimeError(f"walk_emu failed ({p.returncode}): {p.stderr[-2000:]}")
    re_, im_, err, kappa, units = p.stdout.split()
    return complex(float.fromhex(re_), float.fromhex(im_)), float.fromhex(err), float.fromhex(kappa), int(units)
