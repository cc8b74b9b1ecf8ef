"""Build the two drivers that run the library's host code under AddressSanitizer
and UndefinedBehaviorSanitizer.

Every source under csrc/ is compiled with the sanitizers on its host pass only
(each -fsanitize= follows -Xarch_host; the device code is compiled as usual);
the objects are linked by the host compiler with the sanitizer runtimes.

* hostsan_driver (under _build/hostsan/, CPU only): hostsan_driver.hip, which
  compiles the entry-point source into itself and drives the host logic
  without a device.
* tests/hostsan/hostsan_gpu (GPU): hostsan_gpu.cpp, linked with every library
  object, which runs real builds through the C ABI. Built here, on the CPU, and
  run by tests/test_gpu_hostsan.py.

Objects are cached under _build/hostsan/ and rebuilt when a source or header
is newer.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent
ROOT = HERE.parent.parent
CSRC = ROOT / "paper_2304_05505_amd" / "csrc"
OUT = ROOT / "_build" / "hostsan"
CPU_DRIVER = HERE / "hostsan_driver.hip"
GPU_DRIVER = HERE / "hostsan_gpu.cpp"
GPU_EXE = HERE / "hostsan_gpu"

HIPCC = "/opt/rocm/bin/hipcc"
HOST_CXX = "/opt/rocm/llvm/bin/clang++"
HIP_FLAGS = [
    "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-omit-frame-pointer", "-Wno-pass-failed",
    # sanitizers on the host pass only
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
]
# host-compiler lines (no device code): the GPU driver's own source and the links
HOST_SANITIZERS = ["-fsanitize=address,undefined"]
HOST_FLAGS = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
              "-I/opt/rocm/include", *HOST_SANITIZERS]
LINK = ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]


def available() -> bool:
    return os.path.exists(HIPCC) and os.path.exists(HOST_CXX)


def _stale(out, deps):
    return not out.exists() or any(d.stat().st_mtime > out.stat().st_mtime for d in deps)


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"{' '.join(map(str, cmd))}\n{res.stderr[-4000:]}")


def _objects(srcs, extra_deps=None):
    """Compile the HIP sources (host pass sanitized) in parallel; return objects."""
    OUT.mkdir(parents=True, exist_ok=True)
    headers = [*CSRC.glob("*.h"), ROOT / "include" / "exx.h"]
    jobs, objs = [], []
    for s in srcs:
        obj = OUT / (s.stem + ".o")
        objs.append(obj)
        if _stale(obj, [s, *headers, *(extra_deps or {}).get(s, [])]):
            jobs.append([HIPCC, *HIP_FLAGS, "-c", str(s), "-o", str(obj)])
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(_run, jobs))
    return objs


def _library_sources():
    return sorted(CSRC.glob("*.hip"))


def build_cpu_driver() -> pathlib.Path:
    # the entry-point source is compiled into the driver
    srcs = [s for s in _library_sources() if s.name != "api.hip"] + [CPU_DRIVER]
    objs = _objects(srcs, {CPU_DRIVER: [CSRC / "api.hip"]})
    exe = OUT / "hostsan_driver"
    if _stale(exe, objs):
        _run([HOST_CXX, *HOST_SANITIZERS, "-o", str(exe), *map(str, objs), *LINK])
    return exe


def build_gpu_driver() -> pathlib.Path:
    objs = _objects(_library_sources())
    drv = OUT / "hostsan_gpu.o"
    if _stale(drv, [GPU_DRIVER, ROOT / "include" / "exx.h"]):
        _run([HOST_CXX, *HOST_FLAGS, "-c", str(GPU_DRIVER), "-o", str(drv)])
    if _stale(GPU_EXE, [*objs, drv]):
        _run([HOST_CXX, *HOST_SANITIZERS, "-o", str(GPU_EXE), *map(str, objs), str(drv), *LINK])
    return GPU_EXE


def build_all() -> None:
    build_cpu_driver()
    build_gpu_driver()
