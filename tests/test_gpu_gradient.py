"""The density derivative of the fitted exchange energy (exx_exchange_gradient,
FP64) against the gradient oracle (thc.thc_oo_k_gradient, itself pinned by finite
differences of the fitted energy) on the Gamma point, real-path, odd-grid,
ragged, 3x3x3, 5x1x1 and 4x4x4 meshes (the k-correlations' register, two-pass
register, LDS-staged and direct forms), with the fit at and below the pair rank.

* Ranks equal; E_x, K and Kgrad (relative to max|Kgrad|) to
  min(1e-8, max(1e-12, 64 eps64 cond)), cond the largest cond(S^m) over the
  retained points: every term of the derivative is a product of the fitted
  xi^m (or its potential) with G^n or Gamma^n, so its rounding is the fit's.
  The cap 1e-8 also holds on the cells with cond > 1e8, where xi^m and V^m
  themselves are fixed only to about eps64 cond: like K, Kgrad sees them only
  through products that the factor-form solve W^H (W Z) keeps accurate.
* K equals exx_build's K on the same inputs (the call's K-build is the
  build's, to rounding).
* On the GPU result itself: Kgrad Hermitian, and Euler's identity of a
  degree-two function, -(1/N_k) sum_n Tr(Kgrad^n D^n) = E_x.
* Also: one refinement step, a caller-owned workspace, FP32 rejected, and
  EXX_MIXED (with the robust K) against the oracle on seven meshes.
"""

import numpy as np
import pytest

import synth
from oracle import select, thc

from test_gpu_parity import CELLS

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps

GRAD_CELLS = {
    "k211": lambda: synth.make_random_cell((5.0, 5.5, 6.0), 2, (10, 10, 12), (2, 1, 1), 2, 14,
                                           (7, 7, 7)),
    # N_ISDF 12 below the pair rank N_k n_occ^2 = 18: an approximate fit
    "k211-low": lambda: synth.make_random_cell((5.0, 5.5, 6.0), 2, (10, 10, 12), (2, 1, 1), 3, 12,
                                               (7, 7, 6)),
    "k311": lambda: synth.make_random_cell((6.0, 5.0, 5.0), 2, (12, 10, 10), (3, 1, 1), 2, 16,
                                           (7, 7, 8)),
    "gamma": lambda: synth.make_random_cell((6.0, 6.0, 6.0), 3, (12, 12, 12), (1, 1, 1), 3, 12,
                                            (7, 7, 9)),
    "k222-ragged": CELLS["k222-ragged"],
    "k112-odd": CELLS["k112-odd"],
    "k333": CELLS["k333"],  # the correlations' two-pass register form
    "k511": CELLS["k511"],  # a mesh without a compiled form: LDS staging
    "k444": CELLS["k444"],  # 64 transfers: the correlations' direct form (no staging)
}


def _cond(o):
    conds = []
    for m in range(o["S"].shape[0]):
        R = np.flatnonzero(o["keep"][m])
        conds.append(np.linalg.cond(o["S"][m][np.ix_(R, R)]))
    return float(max(conds))


@pytest.mark.parametrize("name", list(GRAD_CELLS))
def test_exchange_gradient_matches_oracle(name, gpu):
    import torch

    from paper_2304_05505_amd import exx

    cell = GRAD_CELLS[name]()
    C = synth.orbital_coeffs(cell)
    psi = synth.orbitals_on_grid(cell, C)
    phi = np.stack([synth.ao_on_grid(cell, n) for n in range(cell.N_k)])
    pts, _ = select.select_points(psi, cell.n_isdf)
    o = thc.thc_oo_k_gradient(cell.L, cell.grid, cell.kmesh, psi, phi, pts)
    cond = _cond(o)
    tol = min(1e-8, max(1e-12, 64 * EPS64 * cond))

    dev = torch.device("cuda", 0)
    nk, na, ni = cell.N_k, cell.n_ao, len(pts)
    ao = np.stack([phi[n][:, pts] for n in range(nk)])
    t = dict(
        psi_grid=torch.from_numpy(psi).to(dev),
        occ_pts=torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev),
        ao_pts=torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
        ao_grid=torch.from_numpy(np.ascontiguousarray(phi)).to(dev),
        pts=torch.from_numpy(np.asarray(pts, dtype=np.int32)).to(dev),
    )
    K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
    Kg = torch.empty_like(K)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    rank = torch.empty((nk,), dtype=torch.int32, device=dev)
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, ni)
    h = exx.Handle(0)
    exx.exx_exchange_gradient(h, c, t["psi_grid"], t["occ_pts"], t["ao_pts"], t["ao_grid"],
                              t["pts"], K, Kg, Ex, rank)
    torch.cuda.synchronize()
    Kn, Kgn, E, r = K.cpu().numpy(), Kg.cpu().numpy(), float(Ex.cpu()[0]), rank.cpu().numpy()
    dE = abs(E - o["Ex"]) / abs(o["Ex"])
    dK = np.abs(Kn - o["K"]).max() / np.abs(o["K"]).max()
    dG = np.abs(Kgn - o["Kgrad"]).max() / np.abs(o["Kgrad"]).max()
    print(f"{name}: cond {cond:.2e} rank {r.tolist()} tol {tol:.1e} rel dE {dE:.2e} dK {dK:.2e} "
          f"dKgrad {dG:.2e}")
    assert np.array_equal(r, o["rank"])
    assert dE <= tol and dK <= tol and dG <= tol

    # the K-build of the call is exx_build's
    K2 = torch.empty_like(K)
    Ex2 = torch.empty_like(Ex)
    exx.exx_build(h, c, exx.EXX_F64, t["psi_grid"], t["occ_pts"], t["ao_pts"], t["pts"], K2, Ex2,
                  rank)
    torch.cuda.synchronize()
    assert np.abs(K2.cpu().numpy() - Kn).max() <= tol * np.abs(Kn).max()

    # Hermiticity and Euler's identity on the GPU result
    scale = np.abs(Kgn).max()
    D = [Cn @ Cn.conj().T for Cn in C]
    e_euler = -(1.0 / nk) * sum(np.trace(Kgn[n] @ D[n]).real for n in range(nk))
    assert abs(e_euler - E) <= max(tol, 1e-10) * abs(E)
    for n in range(nk):
        assert np.abs(Kgn[n] - Kgn[n].conj().T).max() <= 1e-12 * scale


def test_exchange_gradient_rejects_fp32(gpu):
    import torch

    from paper_2304_05505_amd import exx

    cell = GRAD_CELLS["k211"]()
    dev = torch.device("cuda", 0)
    nk, na, ni, no, ng = cell.N_k, cell.n_ao, cell.n_isdf, cell.n_occ, cell.N_g
    z = lambda *s: torch.zeros(s, dtype=torch.complex128, device=dev)  # noqa: E731
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, no, na, ni)
    h = exx.Handle(0)
    with pytest.raises(RuntimeError, match="FP64 or MIXED"):
        exx.exx_exchange_gradient(h, c, z(nk, no, ng), z(nk, ni, no), z(nk, ni, na), z(nk, na, ng),
                                  torch.arange(ni, dtype=torch.int32, device=dev), z(nk, na, na),
                                  z(nk, na, na), torch.zeros(1, dtype=torch.float64, device=dev),
                                  torch.zeros(nk, dtype=torch.int32, device=dev), prec=exx.EXX_F32)


def test_gradient_and_robust_on_caller_workspace(gpu):
    """exx_workspace_size with EXX_CALL_GRADIENT covers both calls: on a caller
    buffer of exactly that size they give the results of library-owned scratch
    bit for bit, and a buffer 256 bytes short is rejected before anything runs."""
    import torch

    from paper_2304_05505_amd import exx

    cell = GRAD_CELLS["k222-ragged"]()
    C = synth.orbital_coeffs(cell)
    psi = synth.orbitals_on_grid(cell, C)
    phi = np.stack([synth.ao_on_grid(cell, n) for n in range(cell.N_k)])
    pts, _ = select.select_points(psi, cell.n_isdf)
    dev = torch.device("cuda", 0)
    nk, na, ni = cell.N_k, cell.n_ao, len(pts)
    ao = np.stack([phi[n][:, pts] for n in range(nk)])
    args = (torch.from_numpy(psi).to(dev),
            torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev),
            torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
            torch.from_numpy(np.ascontiguousarray(phi)).to(dev),
            torch.from_numpy(np.asarray(pts, dtype=np.int32)).to(dev))
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, ni)

    def run(h):
        K = torch.zeros((nk, na, na), dtype=torch.complex128, device=dev)
        Kg = torch.zeros_like(K)
        Kr = torch.zeros_like(K)
        Ex = torch.zeros((1,), dtype=torch.float64, device=dev)
        rank = torch.zeros((nk,), dtype=torch.int32, device=dev)
        exx.exx_exchange_gradient(h, c, *args, K, Kg, Ex, rank)
        exx.exx_build_robust(h, c, *args, Kr, Ex, rank)
        torch.cuda.synchronize()
        return K, Kg, Kr

    h = exx.Handle(0)
    ref = run(h)
    need = h.workspace_size(c, exx.EXX_F64, exx.EXX_CALL_GRADIENT)
    buf = torch.empty((need,), dtype=torch.uint8, device=dev)
    h.set_workspace(buf)
    got = run(h)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    h.set_workspace(buf[: need - 256])
    with pytest.raises(exx.ExxError, match="workspace"):
        run(h)
    h.set_workspace(None)


def test_gradient_with_one_refinement_step(gpu):
    """With one step of iterative refinement the fit applies the explicit S^+
    and refines it (the path that leaves xi in the caller-side buffer and copies
    it for the potentials): the gradient is still the oracle's to the same
    tolerance (refinement only reduces the solve's residual)."""
    import torch

    from paper_2304_05505_amd import exx

    cell = GRAD_CELLS["k311"]()
    psi = synth.orbitals_on_grid(cell, synth.orbital_coeffs(cell))
    phi = np.stack([synth.ao_on_grid(cell, n) for n in range(cell.N_k)])
    pts, _ = select.select_points(psi, cell.n_isdf)
    o = thc.thc_oo_k_gradient(cell.L, cell.grid, cell.kmesh, psi, phi, pts)
    tol = min(1e-8, max(1e-12, 64 * EPS64 * _cond(o)))
    dev = torch.device("cuda", 0)
    nk, na, ni = cell.N_k, cell.n_ao, len(pts)
    ao = np.stack([phi[n][:, pts] for n in range(nk)])
    K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
    Kg = torch.empty_like(K)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    rank = torch.empty((nk,), dtype=torch.int32, device=dev)
    h = exx.Handle(0)
    h.set_refinement(1)
    exx.exx_exchange_gradient(
        h, exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, na, ni),
        torch.from_numpy(psi).to(dev),
        torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev),
        torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
        torch.from_numpy(np.ascontiguousarray(phi)).to(dev),
        torch.from_numpy(np.asarray(pts, dtype=np.int32)).to(dev), K, Kg, Ex, rank)
    torch.cuda.synchronize()
    dG = np.abs(Kg.cpu().numpy() - o["Kgrad"]).max() / np.abs(o["Kgrad"]).max()
    dE = abs(float(Ex.cpu()[0]) - o["Ex"]) / abs(o["Ex"])
    print(f"refined: rel dE {dE:.2e} dKgrad {dG:.2e} tol {tol:.1e}")
    assert dE <= tol and dG <= tol


MIXED_CELLS = ["k211", "k311", "gamma", "k222-ragged", "k112-odd", "k333", "k511"]


@pytest.mark.parametrize("name", MIXED_CELLS)
def test_mixed_gradient_and_robust_against_oracle(name, gpu):
    """EXX_MIXED: the fit as in the MIXED builds (FP64 Gamma^n, Z^m and solve,
    xi stored as c64), the transforms and the potentials stored as c64 (FP32
    transform arithmetic), the correlations and AO contractions in FP64. The
    FP32 steps are the storage of xi, of F and of Pw and the transform's
    log2(N_g) stages, so K, Kgrad, K_rob and E_x are held to
    16 eps32 log2(N_g) relative (about 2e-5 on these grids)."""
    import torch

    from paper_2304_05505_amd import exx

    cell = GRAD_CELLS[name]()
    psi = synth.orbitals_on_grid(cell, synth.orbital_coeffs(cell))
    phi = np.stack([synth.ao_on_grid(cell, n) for n in range(cell.N_k)])
    pts, _ = select.select_points(psi, cell.n_isdf)
    og = thc.thc_oo_k_gradient(cell.L, cell.grid, cell.kmesh, psi, phi, pts)
    orb = thc.thc_oo_k_robust(cell.L, cell.grid, cell.kmesh, psi, phi, pts)
    cond = _cond(og)
    dev = torch.device("cuda", 0)
    nk, na, ni = cell.N_k, cell.n_ao, len(pts)
    ao = np.stack([phi[n][:, pts] for n in range(nk)])
    args = (torch.from_numpy(psi).to(dev),
            torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev),
            torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
            torch.from_numpy(np.ascontiguousarray(phi)).to(dev),
            torch.from_numpy(np.asarray(pts, dtype=np.int32)).to(dev))
    K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
    Kg = torch.empty_like(K)
    Kr = torch.empty_like(K)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    rank = torch.empty((nk,), dtype=torch.int32, device=dev)
    h = exx.Handle(0)
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, na, ni)
    exx.exx_exchange_gradient(h, c, *args, K, Kg, Ex, rank, prec=exx.EXX_MIXED)
    exx.exx_build_robust(h, c, *args, Kr, Ex, rank, prec=exx.EXX_MIXED)
    torch.cuda.synchronize()
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())  # noqa: E731
    dG, dR, dK = rel(Kg.cpu().numpy(), og["Kgrad"]), rel(Kr.cpu().numpy(), orb["K"]), \
        rel(K.cpu().numpy(), og["K"])
    dE = abs(float(Ex.cpu()[0]) - og["Ex"]) / abs(og["Ex"])
    tol = 16 * np.finfo(np.float32).eps * np.log2(cell.N_g)
    print(f"{name} mixed: cond {cond:.2e} tol {tol:.1e} rel dE {dE:.2e} dK {dK:.2e} "
          f"dKgrad {dG:.2e} dKrob {dR:.2e}")
    assert np.array_equal(rank.cpu().numpy(), og["rank"])
    assert max(dE, dK, dG, dR) <= tol
