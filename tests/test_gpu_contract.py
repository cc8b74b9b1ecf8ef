"""Coulomb contraction on the BF16 matrix cores (exx_set_contraction).

Kernel check (exx_coulomb_V, FP32-stored transforms, seeded random xi): the
BF16 forms and the FP64-matrix-core form contract the same FP32 transforms F,
and the FP64-core form is exact up to FP64 accumulation, so their difference is
the BF16 form's own error. Per term v F_P conj F_Q:
  * EXX_CONTRACT_BF16: each operand rounded to 8 significant bits (relative
    2^-9), so a product is off by at most ~2^-8 of |v F_P F_Q|;
  * EXX_CONTRACT_BF16X3: each operand carried as hi + lo to 2^-18, the dropped
    lo lo product is below 2^-18, so a product is off by at most 3 * 2^-18;
plus FP32 accumulation over at most 256 points (16 k-steps of up to three
32-term products: under 100 * 2^-24 of the summed magnitudes). So
  |dV^m_PQ| <= c B^m_PQ,  B^m_PQ = (Omega/N_g^2) sum_g v^m(g) |F_P(g)| |F_Q(g)|,
with c = 2^-8 + 1e-5 (BF16) and 3 * 2^-18 + 1e-5 (BF16X3), checked entry by
entry (B from the FP64 transform of the same xi). A sign, index or pairing
mistake gives errors of order B and fails it. Cells cover the complex Gamma
point, the 3x3x3 and 3x2x1 meshes, ragged N_ISDF and an odd N_g (the scalar-
load form).

Fused builds (the real path's Re-only form on half grids, the paired complex
path): the BF16X3 build is compared with the same build on the FP64 cores and
must be at least ten times closer than the BF16 build; both are compared with
the FP64 oracle and reported (measured on these cells: BF16X3 rel |dE_x|
5e-8 .. 5.5e-5, BF16 3e-5 .. 3e-2, growing with cond(S)).
"""

import numpy as np
import pytest
import scipy.fft as sfft

import synth
from oracle import coulomb, select, thc

from gpu_helpers import inputs, run_gpu
from test_gpu_parity import CELLS, _cond

pytestmark = pytest.mark.gpu

C_BF16 = 2.0 ** -8 + 1e-5
C_BF16X3 = 3 * 2.0 ** -18 + 1e-5


def _coulomb(cell, xi, form):
    import torch

    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    h = exx.Handle(0)
    h.set_contraction(form)
    nk, ni = xi.shape[0], xi.shape[1]
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, ni)
    pts = np.arange(ni, dtype=np.int32) * 7 % cell.N_g
    V = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    exx.exx_coulomb_V(h, c, exx.EXX_F32, torch.from_numpy(xi).to(dev),
                      torch.from_numpy(pts).to(dev), V)
    torch.cuda.synchronize()
    return V.cpu().numpy()


def _bound_matrix(cell, xi):
    """B^m_PQ = (Omega/N_g^2) sum_g v^m(g) |F_P(g)| |F_Q(g)| from the FP64 transform."""
    nk, ni, ng = xi.shape
    omega = float(np.prod(cell.L))
    out = np.empty((nk, ni, ni))
    for m in range(nk):
        F = sfft.fftn(xi[m].astype(np.complex128).reshape((ni,) + tuple(cell.grid)),
                      axes=(1, 2, 3)).reshape(ni, ng)
        v = coulomb.kernel(cell.L, cell.grid, cell.kmesh, m).reshape(-1)
        A = np.abs(F)
        out[m] = (omega / ng ** 2) * ((A * v[None, :]) @ A.T)
    return out


@pytest.mark.parametrize("name", ["gamma-config1", "k333", "k321", "k112-odd", "k222-ragged"])
def test_bf16_contraction_within_its_rounding_bound(name, gpu):
    from paper_2304_05505_amd import exx

    cell = CELLS[name]()
    ni = cell.n_isdf
    rng = np.random.default_rng([2304, 5505, ni, cell.N_g])
    xi = (rng.standard_normal((cell.N_k, ni, cell.N_g))
          + 1j * rng.standard_normal((cell.N_k, ni, cell.N_g))).astype(np.complex64)
    V0 = _coulomb(cell, xi, exx.EXX_CONTRACT_F64)
    B = _bound_matrix(cell, xi)
    for form, c, floor in ((exx.EXX_CONTRACT_BF16, C_BF16, 1e-4),
                           (exx.EXX_CONTRACT_BF16X3, C_BF16X3, 1e-8)):
        V = _coulomb(cell, xi, form)
        r = np.abs(V - V0) / B
        print(f"{name} form {form}: max |dV|/B {r.max():.3e} (bound {c:.2e}), "
              f"max |dV|/max|V| {np.abs(V - V0).max() / np.abs(V0).max():.2e}")
        assert np.all(np.isfinite(V))
        assert r.max() <= c
        # the rounding is really applied
        assert r.max() >= floor
    # the FP64-core form against the oracle's contraction of the same xi (the FP32
    # transform's rounding only)
    for m in (0, cell.N_k - 1):
        Vo = thc.bloch_gauge(cell.L, cell.grid, cell.kmesh, m, np.arange(ni) * 7 % cell.N_g,
                             thc.coulomb_matrix(cell.L, cell.grid, cell.kmesh, m,
                                                xi[m].astype(np.complex128)))
        assert np.abs(V0[m] - Vo).max() <= 1e-5 * np.abs(Vo).max()


def test_f64_build_rejects_bf16_forms(gpu):
    import torch

    from paper_2304_05505_amd import exx

    cell = CELLS["k333"]()
    h = exx.Handle(0)
    with pytest.raises(exx.ExxError):
        h.set_contraction(7)
    h.set_contraction(exx.EXX_CONTRACT_BF16X3)
    base = inputs(cell)
    pts, _ = select.select_points(base["psi"], cell.n_isdf)
    ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
    with pytest.raises(exx.ExxError) as ei:
        run_gpu(cell, base["psi"], pts, ao, "f64", stages=False, handle=h)
    assert ei.value.status == -7
    torch.cuda.synchronize()
    h.set_contraction(exx.EXX_CONTRACT_AUTO)
    g = run_gpu(cell, base["psi"], pts, ao, "f64", stages=False, handle=h)
    assert np.isfinite(g["Ex"])


@pytest.mark.parametrize("name", ["gamma-config1", "k222-ragged", "k112-odd", "k333", "k321"])
def test_fused_builds_with_bf16_contraction(name, gpu):
    from paper_2304_05505_amd import exx

    cell = CELLS[name]()
    base = inputs(cell)
    pts, _ = select.select_points(base["psi"], cell.n_isdf)
    ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
    o = thc.thc_oo_k(cell.L, cell.grid, cell.kmesh, base["psi"], pts, ao)
    res = {}
    for form in (exx.EXX_CONTRACT_F64, exx.EXX_CONTRACT_BF16, exx.EXX_CONTRACT_BF16X3):
        h = exx.Handle(0)
        h.set_contraction(form)
        res[form] = run_gpu(cell, base["psi"], pts, ao, "f32", stages=False, handle=h)
    g0 = res[exx.EXX_CONTRACT_F64]
    kmax = np.abs(g0["K"]).max()
    d = {}
    for form in (exx.EXX_CONTRACT_BF16, exx.EXX_CONTRACT_BF16X3):
        g = res[form]
        assert np.array_equal(g["rank"], g0["rank"])
        d[form] = (abs(g["Ex"] - g0["Ex"]) / abs(g0["Ex"]), np.abs(g["K"] - g0["K"]).max() / kmax,
                   abs(g["Ex"] - o["Ex"]) / abs(o["Ex"]),
                   np.abs(g["K"] - o["K"]).max() / np.abs(o["K"]).max())
        print(f"{name} form {form} (cond {_cond(o):.1e}): vs FP64-core build rel dE {d[form][0]:.2e} "
              f"rel dK {d[form][1]:.2e}; vs oracle rel dE {d[form][2]:.2e} rel dK {d[form][3]:.2e}")
    e16, k16 = d[exx.EXX_CONTRACT_BF16][:2]
    e3, k3 = d[exx.EXX_CONTRACT_BF16X3][:2]
    if _cond(o) <= 1e8:
        # beyond that the metric amplifies BF16 rounding to order one in K
        # (3x3x3 cell here: cond 1.8e10, rel max|dK| 1.7)
        assert e16 <= 5e-2 and k16 <= 1.0
    assert e3 <= e16 / 10 + 1e-9 and k3 <= k16 / 10 + 1e-9
