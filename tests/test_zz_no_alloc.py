"""exx_build_K_noalloc (scratch in the library's fixed per-GPU array) against
exx_build_K (scratch from the handle), through the C ABI: two calls in a row, the
second on a smaller cell, then a cell too large for the fixed array."""

import ctypes

import numpy as np
import pytest

import synth
from oracle import select

pytestmark = pytest.mark.gpu


def _case(cell):
    import torch

    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    C = synth.orbital_coeffs(cell)
    psi = synth.orbitals_on_grid(cell, C)
    pts, _ = select.select_points(psi, cell.n_isdf)
    ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
    nk, ni, ng = cell.N_k, cell.n_isdf, cell.N_g
    t = dict(
        psi=torch.from_numpy(psi).to(dev),
        occ=torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev),
        ao=torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
        pts=torch.from_numpy(pts.astype(np.int32)).to(dev),
    )
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, ni)
    return c, t


def _V(h, c, t, nk, ni, ng):
    import torch

    from paper_2304_05505_amd import exx

    dev = t["psi"].device
    xi = torch.empty((nk, ni, ng), dtype=torch.complex128, device=dev)
    S = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    V = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    rank = torch.empty((nk,), dtype=torch.int32, device=dev)
    exx.exx_isdf_fit(h, c, exx.EXX_F64, t["psi"], t["occ"], t["pts"], xi, S, rank)
    exx.exx_coulomb_V(h, c, exx.EXX_F64, xi, t["pts"], V)
    return V


def test_noalloc_matches_build_K_on_two_calls(gpu):
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    cells = [
        # first call: 2x2x2 mesh, n_ao 8 < N_ISDF 40 (A^H staged in the scratch)
        synth.make_random_cell((6.0, 6.5, 7.0), 2, (12, 15, 10), (2, 2, 2), 3, 40, (12, 1, 1)),
        # second call, smaller: Gamma only, N_ISDF 6 < n_ao 8 (the tiled K form)
        synth.make_random_cell((5.0, 5.0, 5.0), 2, (8, 8, 10), (1, 1, 1), 2, 6, (12, 2, 1)),
    ]
    for cell in cells:
        c, t = _case(cell)
        nk, ni, na = cell.N_k, cell.n_isdf, cell.n_ao
        V = _V(h, c, t, nk, ni, cell.N_g)
        K_ref = torch.empty((nk, na, na), dtype=torch.complex128, device=gpu)
        E_ref = torch.empty((1,), dtype=torch.float64, device=gpu)
        exx.exx_build_K(h, c, exx.EXX_F64, t["ao"], t["occ"], V, K_ref, E_ref)
        K = torch.full((nk, na, na), float("nan"), dtype=torch.complex128, device=gpu)
        E = torch.full((1,), float("nan"), dtype=torch.float64, device=gpu)
        exx.exx_build_K_noalloc(h, c, exx.EXX_F64, t["ao"], t["occ"], V, K, E)
        torch.cuda.synchronize()
        print(f"{cell.name}: N_k {nk} N_ISDF {ni} n_ao {na}: E_x {float(E.cpu()[0]):.15f} "
              f"ref {float(E_ref.cpu()[0]):.15f}")
        # same kernels on the same inputs: identical bits
        assert torch.equal(K, K_ref)
        assert torch.equal(E, E_ref)
        assert h.status()[0] == 0


def test_noalloc_rejects_cells_beyond_the_fixed_scratch(gpu):
    """A 4x4x4 cell with N_ISDF 420 and n_ao 384 needs about 690 MB; the call fails
    with EXX_ERR_SHAPE before launching anything (the pointers are never read)."""
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    c = exx.make_cell((14.0, 17.8, 12.9), (72, 90, 64), (4, 4, 4), 84, 384, 420)
    dummy = torch.zeros((4,), dtype=torch.float64, device=gpu)
    p = dummy.data_ptr()
    st = torch.cuda.current_stream().cuda_stream
    assert exx._lib.exx_build_K_noalloc(h.raw, ctypes.byref(c), exx.EXX_F64, p, p, p, p, p, st) == -2
    assert "allocation-free scratch" in exx._lib.exx_last_error(h.raw).decode()
