"""The library's host code under AddressSanitizer, UndefinedBehaviorSanitizer
and LeakSanitizer during real GPU builds.

tests/hostsan/hostsan_gpu is built on the CPU by __graft_entry__.build() (the
library's objects with the sanitizers on their host pass only, linked with a
C++ driver, tests/hostsan/hostsan_gpu.cpp). This test writes four seeded cells
(a ragged 2x2x2 cell, a 3x1x1 and a 3x3x3 paired-path cell, a Gamma cell) and
runs the driver on them: every entry point that builds, including the batched
call with lanes, captured graphs replayed twice and autotuning. It fails on any
sanitizer report (LeakSanitizer with the HIP runtime's own allocations
suppressed) or on a failed check of the driver, which compares the calls with
each other.
"""

import os
import pathlib
import subprocess

import numpy as np
import pytest

import synth
from oracle import select

pytestmark = pytest.mark.gpu

HERE = pathlib.Path(__file__).resolve().parent / "hostsan"
EXE = HERE / "hostsan_gpu"


def _write_inputs(out):
    cells = [
        synth.make_random_cell((6.0, 6.5, 7.0), 2, (12, 15, 10), (2, 2, 2), 3, 30, (11, 1, 1)),
        synth.make_random_cell((6.0, 5.0, 5.0), 2, (12, 10, 10), (3, 1, 1), 2, 24, (11, 13, 1)),
        synth.make_config(1),
        synth.make_random_cell((5.0, 5.0, 5.0), 2, (10, 12, 9), (3, 3, 3), 2, 40, (11, 3, 1)),
    ]
    lines = []
    for i, c in enumerate(cells):
        psi = synth.orbitals_on_grid(c, synth.orbital_coeffs(c))
        pts, _ = select.select_points(psi, c.n_isdf)
        ao = np.stack([synth.ao_at_points(c, n, pts) for n in range(c.N_k)])
        aog = np.stack([synth.ao_on_grid(c, n) for n in range(c.N_k)])
        occ = np.transpose(psi[:, :, pts], (0, 2, 1))
        for name, a, dt in (("psi", psi, np.complex128), ("occ", occ, np.complex128),
                            ("ao", np.transpose(ao, (0, 2, 1)), np.complex128),
                            ("aog", aog, np.complex128), ("pts", pts, np.int32)):
            np.ascontiguousarray(a, dtype=dt).tofile(out / f"{name}{i}.bin")
        lines.append(" ".join(map(str, [*c.L, *c.grid, *c.kmesh, c.n_occ, c.n_ao, len(pts)])))
    (out / "cells.txt").write_text("\n".join(lines) + "\n")


@pytest.mark.timeout(600)
def test_host_code_under_sanitizers_on_the_gpu(tmp_path, gpu):
    assert EXE.exists(), f"{EXE} is not built (__graft_entry__.build() builds it)"
    inp = tmp_path / "in"
    inp.mkdir()
    _write_inputs(inp)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={HERE / 'lsan.supp'}:print_suppressions=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    print(f"running {EXE.name} on {inp}", flush=True)
    res = subprocess.run([str(EXE), str(inp), str(tmp_path)], capture_output=True, text=True,
                         env=env, timeout=300)
    print(res.stdout)
    report = res.stderr
    assert "runtime error" not in report and "Sanitizer" not in report, report[-4000:]
    assert res.returncode == 0, report[-4000:]
    assert "hostsan-gpu ok: 0 failures" in res.stdout, res.stdout
