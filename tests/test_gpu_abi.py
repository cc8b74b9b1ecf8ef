"""Error behaviour of the C ABI on a GPU handle: every bad argument is rejected before launch."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _cell(exx, grid=(12, 12, 12), kmesh=(2, 2, 2), no=3, na=8, ni=20):
    return exx.make_cell((6.0, 6.0, 6.0), grid, kmesh, no, na, ni)


def _fit(exx, h, c, prec, null=False):
    import torch

    dev = torch.device("cuda", 0)
    nk = c.kmesh[0] * c.kmesh[1] * c.kmesh[2]
    ng = c.grid[0] * c.grid[1] * c.grid[2]
    gd = torch.complex128 if prec == exx.EXX_F64 else torch.complex64
    psi = torch.zeros((nk, c.n_occ, ng), dtype=gd, device=dev)
    occ = torch.zeros((nk, c.n_isdf, c.n_occ), dtype=torch.complex128, device=dev)
    pts = torch.arange(c.n_isdf, dtype=torch.int32, device=dev)
    xi = torch.zeros((nk, c.n_isdf, ng), dtype=gd, device=dev)
    S = torch.zeros((nk, c.n_isdf, c.n_isdf), dtype=torch.complex128, device=dev)
    rank = torch.zeros((nk,), dtype=torch.int32, device=dev)
    lib = exx._lib
    st = torch.cuda.current_stream().cuda_stream
    ptrs = [psi.data_ptr(), occ.data_ptr(), pts.data_ptr(), xi.data_ptr(), S.data_ptr(), rank.data_ptr()]
    if null:
        ptrs[1] = None
    return lib.exx_isdf_fit(h.raw, ctypes.byref(c), prec, *ptrs, st)


def test_bad_arguments_are_rejected(gpu):
    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    assert _fit(exx, h, _cell(exx), exx.EXX_F64, null=True) == -1
    assert _fit(exx, h, _cell(exx, grid=(12, 12, 7)), exx.EXX_F64) == -2
    assert _fit(exx, h, _cell(exx, kmesh=(8, 8, 2)), exx.EXX_F64) == -2  # 128 k-points
    assert _fit(exx, h, _cell(exx), exx.EXX_BF16) == 0  # built in: Gamma on the BF16 cores
    assert _fit(exx, h, _cell(exx, ni=2049), exx.EXX_F64) == -2
    assert _fit(exx, h, _cell(exx), 9) == -1
    msg = exx._lib.exx_last_error(h.raw).decode()
    assert "precision" in msg


def test_gradient_and_robust_reject_bad_arguments(gpu):
    """exx_exchange_gradient and exx_build_robust: a null array, a bad shape and a
    precision other than EXX_F64 or EXX_MIXED are rejected before launch, with
    the message."""
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    dev = torch.device("cuda", 0)
    lib = exx._lib
    st = torch.cuda.current_stream().cuda_stream

    def call(fn, c, prec, null_ao_grid=False):
        nk = c.kmesh[0] * c.kmesh[1] * c.kmesh[2]
        ng = c.grid[0] * c.grid[1] * c.grid[2]
        z = lambda *shape: torch.zeros(shape, dtype=torch.complex128, device=dev)  # noqa: E731
        t = [z(nk, c.n_occ, ng), z(nk, c.n_isdf, c.n_occ), z(nk, c.n_isdf, c.n_ao),
             z(nk, c.n_ao, ng), torch.arange(c.n_isdf, dtype=torch.int32, device=dev),
             z(nk, c.n_ao, c.n_ao), z(nk, c.n_ao, c.n_ao),
             torch.zeros((1,), dtype=torch.float64, device=dev),
             torch.zeros((nk,), dtype=torch.int32, device=dev)]
        ptrs = [x.data_ptr() for x in t]
        if null_ao_grid:
            ptrs[3] = None
        if fn == "robust":
            del ptrs[6]  # no Kgrad
            return lib.exx_build_robust(h.raw, ctypes.byref(c), prec, *ptrs, st)
        return lib.exx_exchange_gradient(h.raw, ctypes.byref(c), prec, *ptrs, st)

    for fn in ("gradient", "robust"):
        assert call(fn, _cell(exx), exx.EXX_F64, null_ao_grid=True) == -1
        assert "null array" in exx._lib.exx_last_error(h.raw).decode()
        assert call(fn, _cell(exx, grid=(12, 12, 7)), exx.EXX_F64) == -2
        assert call(fn, _cell(exx), exx.EXX_F32) == -7  # EXX_ERR_UNSUPPORTED
        assert "FP64 or MIXED" in exx._lib.exx_last_error(h.raw).decode()


def test_all_zero_orbitals_drop_every_point(gpu):
    """S = 0: every pivot is dropped, rank 0, xi = 0, and nothing faults."""
    from paper_2304_05505_amd import exx
    import torch

    h = exx.Handle(0)
    c = _cell(exx)
    assert _fit(exx, h, c, exx.EXX_F64) == 0
    torch.cuda.synchronize()


def test_binding_validates_shapes(gpu):
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    c = _cell(exx)
    dev = torch.device("cuda", 0)
    bad = torch.zeros((1, 2, 3), dtype=torch.complex128, device=dev)
    with pytest.raises(ValueError):
        exx.exx_coulomb_V(h, c, exx.EXX_F64, bad, torch.zeros(20, dtype=torch.int32, device=dev),
                          torch.zeros((8, 20, 20), dtype=torch.complex128, device=dev))
    with pytest.raises(TypeError):
        exx.exx_coulomb_V(h, c, exx.EXX_F64, np.zeros(3), None, None)


def _small_build_inputs(exx, torch, kmesh=(2, 1, 1), dup=False, n_isdf=24):
    import synth
    from oracle import select

    cell = synth.make_random_cell((6.0, 5.0, 5.0), 2, (12, 10, 10), kmesh, 3, n_isdf, (11, 40, 1))
    C = synth.orbital_coeffs(cell)
    psi = synth.orbitals_on_grid(cell, C)
    pts, _ = select.select_points(psi, cell.n_isdf)
    if dup:
        pts = pts.copy()
        pts[-1] = pts[0]  # a repeated point: its Schur pivot vanishes on every transfer
    ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
    dev = torch.device("cuda", 0)
    t = dict(
        psi=torch.from_numpy(psi).to(dev),
        occ=torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev),
        ao=torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
        pts=torch.from_numpy(pts.astype(np.int32)).to(dev),
        K=torch.empty((cell.N_k, cell.n_ao, cell.n_ao), dtype=torch.complex128, device=dev),
        Ex=torch.empty((1,), dtype=torch.float64, device=dev),
        rank=torch.empty((cell.N_k,), dtype=torch.int32, device=dev),
    )
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, cell.n_isdf)
    return cell, c, t


def _build_raw(exx, h, c, prec, t, psi=None, occ=None):
    import torch

    st = torch.cuda.current_stream().cuda_stream
    return exx._lib.exx_build(h.raw, ctypes.byref(c), prec, (psi if psi is not None else t["psi"]).data_ptr(),
                              (occ if occ is not None else t["occ"]).data_ptr(), t["ao"].data_ptr(),
                              t["pts"].data_ptr(), t["K"].data_ptr(), t["Ex"].data_ptr(),
                              t["rank"].data_ptr(), st)


def test_caller_workspace_gives_identical_results(gpu):
    """exx_set_workspace: a torch buffer of exx_workspace_size bytes serves every
    scratch request; the build equals the one on library-owned scratch bit for bit,
    the handle then holds no scratch of its own, and a buffer one byte short is
    rejected with EXX_ERR_NOMEM before anything runs."""
    import torch

    from paper_2304_05505_amd import exx

    for kmesh in ((2, 1, 1), (3, 1, 1)):
        h = exx.Handle(0)
        cell, c, t = _small_build_inputs(exx, torch, kmesh)
        for prec in (exx.EXX_F64, exx.EXX_MIXED):
            assert _build_raw(exx, h, c, prec, t) == 0
            torch.cuda.synchronize()
            K0, E0 = t["K"].clone(), t["Ex"].clone()
            need = h.workspace_size(c, prec)
            buf = torch.empty((need,), dtype=torch.uint8, device=gpu)
            h.set_workspace(buf)
            t["K"].zero_()
            assert _build_raw(exx, h, c, prec, t) == 0
            torch.cuda.synchronize()
            assert torch.equal(t["K"], K0) and torch.equal(t["Ex"], E0)
            small = h.scratch_bytes()
            assert small < 1 << 20, small  # only the per-shape tables remain
            h.set_workspace(buf[: need - 256])
            assert _build_raw(exx, h, c, prec, t) == -3  # EXX_ERR_NOMEM
            assert "workspace" in exx._lib.exx_last_error(h.raw).decode()
            h.set_workspace(None)
        del h


def test_nonfinite_psi_is_reported(gpu):
    """A NaN planted in psi_grid on the host reaches K and E_x; with EXX_CHECK_SYNC
    the build returns EXX_ERR_NONFINITE and names the output site; a NaN in occ_pts
    is caught at the input. Every kernel runs to completion on NaN data."""
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    cell, c, t = _small_build_inputs(exx, torch)
    assert _build_raw(exx, h, c, exx.EXX_F64, t) == 0
    assert h.status() == (0, -1, 0)
    bad = t["psi"].clone()
    bad[0, 1, 7] = complex(float("nan"), 0.0)
    h.set_checks(exx.EXX_CHECK_FINITE | exx.EXX_CHECK_SYNC)
    assert _build_raw(exx, h, c, exx.EXX_F64, t, psi=bad) == exx.EXX_ERR_NONFINITE
    assert "non-finite" in exx._lib.exx_last_error(h.raw).decode()
    # asynchronous form: the call returns OK, the status word holds the report
    h.set_checks(exx.EXX_CHECK_FINITE)
    badocc = t["occ"].clone()
    badocc[0, 2, 1] = complex(0.0, float("inf"))
    assert _build_raw(exx, h, c, exx.EXX_F64, t, occ=badocc) == 0
    code, q, site = h.status()
    assert code == exx.EXX_ERR_NONFINITE and site == 1
    # read-and-clear: a clean build afterwards reports nothing
    assert _build_raw(exx, h, c, exx.EXX_F64, t) == 0
    assert h.status() == (0, -1, 0)
    # checks off: no report
    h.set_checks(0)
    assert _build_raw(exx, h, c, exx.EXX_F64, t, psi=bad) == 0
    assert h.status()[0] == 0


@pytest.mark.parametrize("kmesh", [(2, 1, 1), (3, 1, 1)])
def test_strict_pd_reports_the_first_transfer(kmesh, gpu):
    """12 points on a cell whose pair space has dimension N_k n_occ^2 >= 18: every
    fit metric is positive definite and a strict build is OK. Repeating a point
    makes every metric singular; the drop rule removes it (rank 11). Under
    EXX_STRICT_PD the build then reports EXX_ERR_NOT_PD with transfer 0, the first
    that lost a pivot; without it the same build is OK."""
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    cell, c, t = _small_build_inputs(exx, torch, kmesh, n_isdf=12)
    h.set_checks(exx.EXX_CHECK_FINITE | exx.EXX_STRICT_PD | exx.EXX_CHECK_SYNC)
    assert _build_raw(exx, h, c, exx.EXX_F64, t) == 0
    assert t["rank"].cpu().tolist() == [12] * cell.N_k
    h.set_checks(exx.EXX_CHECK_FINITE)
    cell, c, t = _small_build_inputs(exx, torch, kmesh, dup=True, n_isdf=12)
    assert _build_raw(exx, h, c, exx.EXX_F64, t) == 0
    assert h.status()[0] == 0
    assert t["rank"].cpu().tolist() == [11] * cell.N_k
    h.set_checks(exx.EXX_CHECK_FINITE | exx.EXX_STRICT_PD | exx.EXX_CHECK_SYNC)
    assert _build_raw(exx, h, c, exx.EXX_F64, t) == exx.EXX_ERR_NOT_PD
    h.set_checks(exx.EXX_CHECK_FINITE | exx.EXX_STRICT_PD)
    assert _build_raw(exx, h, c, exx.EXX_F64, t) == 0
    code, q, site = h.status()
    assert code == exx.EXX_ERR_NOT_PD and q == 0 and site == 0
