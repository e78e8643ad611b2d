"""Builds libbbfg.so (gfx950) in-tree from csrc/ with hipcc.

    python -m paper_2309_07027_amd.build

Every HIP source is compiled with -ffp-contract=off (the kernels spell out
every fused multiply-add, so results do not depend on the compiler's
contraction choices) and with packed FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
BUILD = PKG / "_build"
LIB = PKG / "libbbfg.so"
ROOT = PKG.parent

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-function", f"-I{ROOT / 'include'}", f"-I{CSRC}"]
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(CSRC.glob("*.hip")) + sorted(CSRC.glob("*.cpp"))


def _headers():
    return list(CSRC.glob("*.hpp")) + [ROOT / "include" / "bbfg.h"]


def _compile(src: Path, force: bool = True) -> Path:
    obj = BUILD / (src.stem + ("_hip" if src.suffix == ".hip" else "") + ".o")
    if not force and obj.exists():
        newest = max(p.stat().st_mtime for p in [src, *_headers()])
        if obj.stat().st_mtime > newest:
            return obj
    cmd = [HIPCC, *COMMON]
    if src.suffix == ".hip":
        cmd += HIP_FLAGS
    else:
        cmd += ["-D__HIP_PLATFORM_AMD__"]
    cmd += ["-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True, force: bool = True) -> Path:
    """Compile every source (force=True: always, as the build check requires)."""
    BUILD.mkdir(exist_ok=True)
    srcs = sources()
    t0 = time.time()
    jobs = jobs or min(8, os.cpu_count() or 4, len(srcs))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda p: _compile(p, force), srcs))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs),
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources in {time.time() - t0:.1f}s", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv)
