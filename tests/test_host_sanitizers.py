"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
on the CPU (no GPU needed, nothing is launched).

Every source under csrc/ is compiled with the sanitizers on its host pass only
(each -fsanitize= follows -Xarch_host; the device code is built as usual and
never runs), together with tests/hostsan/hostsan_driver.hip, which compiles the
entry-point source into itself and drives the host logic behind the C ABI:

* every entry point with a NULL handle, and exx_create without a device;
* the shape and argument checks of every call, one out-of-range field at a
  time, including precisions outside the four constants;
* the scratch layouts of every call form over meshes, grids, sizes and
  precisions (offsets aligned, in order, within the total);
* the conjugate-pair table of every k-mesh up to 64 points (each transfer once,
  m + (-m) = 0 on the mesh);
* the lane plan of the batched call (each item on one lane sized for it, within
  the budget);
* the tile-table file: round trip, malformed, out-of-range and overlong lines,
  CRLF, a missing final newline, missing and unwritable paths.

The objects are linked by the host compiler with the sanitizer runtimes; the run
fails on any sanitizer report (leaks included) or failed check.
"""

import concurrent.futures as cf
import os
import pathlib
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parent.parent
CSRC = ROOT / "paper_2304_05505_amd" / "csrc"
DRIVER = ROOT / "tests" / "hostsan" / "hostsan_driver.hip"
OUT = ROOT / "_build" / "hostsan"

HIPCC = "/opt/rocm/bin/hipcc"
HOST_CXX = "/opt/rocm/llvm/bin/clang++"
COMPILE = [
    "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-omit-frame-pointer", "-Wno-pass-failed",
    # sanitizers on the host pass only
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
]
# the link of host objects by the host compiler (no device code is compiled here)
LINK_SANITIZERS = ["-fsanitize=address,undefined"]


def _stale(obj, deps):
    return not obj.exists() or any(d.stat().st_mtime > obj.stat().st_mtime for d in deps)


def _build():
    OUT.mkdir(parents=True, exist_ok=True)
    headers = [*CSRC.glob("*.h"), ROOT / "include" / "exx.h"]
    # api.hip is compiled into the driver
    srcs = [s for s in sorted(CSRC.glob("*.hip")) if s.name != "api.hip"] + [DRIVER]
    jobs = []
    for s in srcs:
        obj = OUT / (s.stem + ".o")
        deps = [s, *headers] + ([CSRC / "api.hip"] if s == DRIVER else [])
        if _stale(obj, deps):
            jobs.append([HIPCC, *COMPILE, "-c", str(s), "-o", str(obj)])
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for cmd, res in zip(jobs, ex.map(lambda c: subprocess.run(c, capture_output=True, text=True),
                                          jobs)):
            assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stderr[-4000:]}"
    exe = OUT / "hostsan_driver"
    objs = [OUT / (s.stem + ".o") for s in srcs]
    if _stale(exe, objs):
        cmd = [HOST_CXX, *LINK_SANITIZERS, "-o", str(exe), *map(str, objs),
               "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stderr[-4000:]}"
    return exe


@pytest.mark.timeout(600)
def test_host_code_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(HOST_CXX)):
        pytest.skip("the ROCm compilers are not installed")
    exe = _build()
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    res = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, env=env,
                         timeout=300)
    print(res.stdout)
    report = res.stderr
    assert "runtime error" not in report and "Sanitizer" not in report, report[-4000:]
    assert res.returncode == 0, report[-4000:]
    if res.stdout.startswith("hostsan skip"):
        pytest.skip("a GPU is visible: the checks rely on device calls failing")
    assert res.stdout.startswith("hostsan ok"), res.stdout
