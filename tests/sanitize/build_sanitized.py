"""Host-code builds under AddressSanitizer and UndefinedBehaviorSanitizer.

* liboracle_san.so: oracle/oracle.c, gcc -fsanitize=address,undefined;
* libbbfg_san.so: the library's host sources (runtime, C ABI, sampler,
  server, planner, autotuner) built with g++ -fsanitize=address,undefined and
  linked with the gfx950 kernel objects of the ordinary build (their device
  code is not instrumented: there is no GPU sanitizer here).

Both go to tests/sanitize/_build/.  The caller preloads g++'s libasan.so.
"""
from __future__ import annotations

import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent.parent
OUT = HERE / "_build"
CSRC = ROOT / "paper_2309_07027_amd" / "csrc"
KOBJ = ROOT / "paper_2309_07027_amd" / "_build"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
HOST_SOURCES = ["autotune.cpp", "capi.cpp", "plan.cpp", "runtime.cpp", "sampler.cpp", "server.cpp"]


def asan_runtime() -> str:
    return subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()


def build_oracle() -> Path:
    OUT.mkdir(exist_ok=True)
    lib = OUT / "liboracle_san.so"
    subprocess.run(["gcc", *SAN, "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
                    "-Wno-unused-function", str(ROOT / "oracle" / "oracle.c"), "-o", str(lib), "-lm"], check=True)
    return lib


def build_library() -> Path:
    """Needs the kernel objects of `python -m paper_2309_07027_amd.build`."""
    OUT.mkdir(exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = OUT / (Path(src).stem + ".o")
        subprocess.run(["g++", *SAN, "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
                        "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{ROOT / 'include'}", f"-I{CSRC}",
                        "-c", str(CSRC / src), "-o", str(obj)], check=True)
        objs.append(str(obj))
    kernels = sorted(str(p) for p in KOBJ.glob("*_hip.o"))
    if not kernels:
        raise FileNotFoundError("kernel objects missing: run python -m paper_2309_07027_amd.build first")
    lib = OUT / "libbbfg_san.so"
    subprocess.run(["g++", *SAN, "-shared", "-o", str(lib), *objs, *kernels, "-L/opt/rocm/lib", "-lamdhip64",
                    "-lpthread", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    return lib
