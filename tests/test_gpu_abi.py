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
    assert _fit(exx, h, _cell(exx, kmesh=(5, 1, 1)), exx.EXX_F64) == -7
    assert _fit(exx, h, _cell(exx), exx.EXX_BF16) == -7
    assert _fit(exx, h, _cell(exx, ni=2049), exx.EXX_F64) == -2
    assert _fit(exx, h, _cell(exx), 9) == -1
    msg = exx._lib.exx_last_error(h.raw).decode()
    assert "precision" in msg


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
