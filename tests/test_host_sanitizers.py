"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
on the CPU (no GPU needed, nothing is launched).

tests/hostsan/build_hostsan.py compiles every source under csrc/ with the
sanitizers on its host pass only (the device code is built as usual and never
runs here), together with tests/hostsan/hostsan_driver.hip, which compiles the
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

The run fails on any sanitizer report (leaks included) or failed check. The
same host code under the sanitizers during real GPU builds is
tests/test_gpu_hostsan.py.
"""

import os
import pathlib
import subprocess
import sys

import pytest

sys.path.insert(0, str(pathlib.Path(__file__).resolve().parent / "hostsan"))
import build_hostsan  # noqa: E402


@pytest.mark.timeout(600)
def test_host_code_under_asan_and_ubsan(tmp_path):
    if not build_hostsan.available():
        pytest.skip("the ROCm compilers are not installed")
    exe = build_hostsan.build_cpu_driver()
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
