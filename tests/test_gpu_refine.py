"""One step of iterative refinement after the fit solve (exx_set_refinement).

The refined fit must still match the FP64 oracle (to the parity tolerance of
each mode), and in FP64 it must not leave a larger normal-equation residual
|| S_RR xi_R - Z_R || than the plain solve with the explicit pseudo-inverse
(refinement in the same precision reduces the residual, not the forward error,
so that is what is checked).
"""

import numpy as np
import pytest

import synth
from gpu_helpers import inputs, run_gpu
from oracle import select, thc

pytestmark = pytest.mark.gpu


def _cell():
    return synth.make_random_cell((6.0, 6.5, 7.0), 3, (15, 16, 18), (2, 2, 1), 4, 50, (31, 1, 1))


@pytest.fixture(scope="module")
def case():
    cell = _cell()
    d = inputs(cell)
    pts, _ = select.select_points(d["psi"], cell.n_isdf)
    d = inputs(cell, pts)
    ref = thc.thc_oo_k(cell.L, cell.grid, cell.kmesh, d["psi"], pts, d["ao_pts"],
                       keep_intermediates=("Z", "xi"))
    return cell, d, pts, ref


def _normal_residual(ref, xi):
    out = 0.0
    for m in range(ref["S"].shape[0]):
        R = np.flatnonzero(ref["keep"][m])
        S = ref["S"][m][np.ix_(R, R)]
        r = S @ xi[m][R] - ref["Z"][m][R]
        out = max(out, np.linalg.norm(r) / (np.linalg.norm(S) * np.linalg.norm(xi[m][R])))
    return out


def _tol(ref, eps):
    conds = []
    for m in range(ref["S"].shape[0]):
        R = np.flatnonzero(ref["keep"][m])
        conds.append(np.linalg.cond(ref["S"][m][np.ix_(R, R)]))
    return max(1e-12, 64 * eps * max(conds))


@pytest.mark.parametrize("prec", ["f64", "mixed", "f32"])
def test_refined_fit_matches_the_oracle(case, prec, gpu):
    from paper_2304_05505_amd import exx

    cell, d, pts, ref = case
    h = exx.Handle(0)
    h.set_refinement(1)
    out = run_gpu(cell, d["psi"], pts, d["ao_pts"], prec=prec, handle=h)
    assert np.array_equal(out["rank"], ref["rank"])
    if prec == "f64":
        tol = _tol(ref, np.finfo(np.float64).eps)
        assert abs(out["Ex"] - ref["Ex"]) <= tol * abs(ref["Ex"])
        assert np.abs(out["K"] - ref["K"]).max() <= tol * np.abs(ref["K"]).max()
    else:
        # FP32 storage of xi (and of Z in f32) bounds these modes, refined or not
        tol = _tol(ref, np.finfo(np.float32).eps)
        assert abs(out["Ex"] - ref["Ex"]) <= tol * abs(ref["Ex"])


def test_refinement_does_not_raise_the_fp64_residual(case, gpu):
    from paper_2304_05505_amd import exx

    cell, d, pts, ref = case
    res = []
    for steps in (0, 1):
        h = exx.Handle(0)
        h.set_refinement(steps)
        out = run_gpu(cell, d["psi"], pts, d["ao_pts"], prec="f64", handle=h)
        res.append(_normal_residual(ref, out["xi"]))
    print(f"relative normal-equation residual: plain {res[0]:.3e}, refined {res[1]:.3e}")
    assert res[1] <= 1.05 * res[0] + 1e-16
    assert res[1] <= 1e-12


def test_refinement_setting_is_checked(gpu):
    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    with pytest.raises(exx.ExxError):
        h.set_refinement(2)
    with pytest.raises(exx.ExxError):
        h.set_refinement(-1)
