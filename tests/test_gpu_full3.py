"""Full-size parity on the 3x3x3 form of the benchmark cell (48-atom four-ring
cell, N = 192, n_occ = 84, grid 60x75x54, N_ISDF = 420, N_k = 27) against stored
FP64 oracle values (tests/golden/make_golden.py, points chosen by the oracle):
the fit metric and Bloch-gauge Coulomb matrices of three transfers, and the
whole K (27 x 192 x 192) and E_x of the fused build in every precision.
"""

import numpy as np
import pytest

import synth

from gpu_helpers import from_cplx_list, load_golden, load_golden_arrays

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def full3():
    import torch

    from paper_2304_05505_amd import exx
    from synth.fast import orbitals_on_grid_torch

    gold = load_golden("config3.json")
    gold["K"] = load_golden_arrays("config3_K.npz")["K"]
    cell = synth.make_config(3)
    dev = torch.device("cuda", 0)
    psi = orbitals_on_grid_torch(cell, synth.orbital_coeffs(cell), dev)
    pts = np.asarray(gold["pts"], dtype=np.int64)
    pts_t = torch.from_numpy(pts.astype(np.int32)).to(dev)
    ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
    t = {
        "psi": psi,
        "occ": psi[:, :, pts_t.long()].permute(0, 2, 1).contiguous(),
        "ao": torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
        "pts": pts_t,
    }
    h = exx.Handle(0)
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, cell.n_isdf)
    return dict(gold=gold, cell=cell, t=t, h=h, c=c, exx=exx, torch=torch, dev=dev)


def test_config3_fit_and_coulomb_match_oracle_samples(full3):
    gold, cell, t, exx, torch, dev = (full3[k] for k in ("gold", "cell", "t", "exx", "torch", "dev"))
    nk, ni, ng = cell.N_k, cell.n_isdf, cell.N_g
    xi = torch.empty((nk, ni, ng), dtype=torch.complex128, device=dev)
    S = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    V = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    rank = torch.empty((nk,), dtype=torch.int32, device=dev)
    exx.exx_isdf_fit(full3["h"], full3["c"], exx.EXX_F64, t["psi"], t["occ"], t["pts"], xi, S, rank)
    exx.exx_coulomb_V(full3["h"], full3["c"], exx.EXX_F64, xi, t["pts"], V)
    torch.cuda.synchronize()
    del xi
    S = S.cpu().numpy()
    V = V.cpu().numpy()
    rank = rank.cpu().numpy()
    for j, m in enumerate(gold["m"]):
        assert rank[m] == gold["rank"][j]
        idx = np.asarray(gold[f"idx_{m}"])
        tol = min(1e-8, max(1e-12, 64 * EPS64 * gold["cond_S"][j]))
        s_ref = from_cplx_list(gold[f"S_{m}"])
        assert np.abs(S[m][idx[:, 0], idx[:, 1]] - s_ref).max() <= 1e-12 * np.abs(s_ref).max()
        v_ref = from_cplx_list(gold[f"Vb_{m}"])
        dv = np.abs(V[m][idx[:, 0], idx[:, 1]] - v_ref).max()
        dd = np.abs(np.diagonal(V[m]) - from_cplx_list(gold[f"Vbdiag_{m}"])).max()
        print(f"m={m}: max|dVb| {dv:.2e} (diag {dd:.2e}) vs tol {tol * gold['maxabs_Vb'][j]:.2e}")
        assert dv <= tol * gold["maxabs_Vb"][j]
        assert dd <= tol * gold["maxabs_Vb"][j]


def _build(full3, prec):
    exx, torch, cell, t, dev = (full3[k] for k in ("exx", "torch", "cell", "t", "dev"))
    psi = t["psi"] if prec in ("f64", "mixed") else t["psi"].to(torch.complex64)
    K = torch.empty((cell.N_k, cell.n_ao, cell.n_ao), dtype=torch.complex128, device=dev)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    rank = torch.empty((cell.N_k,), dtype=torch.int32, device=dev)
    exx.exx_build(full3["h"], full3["c"], exx.PREC[prec], psi, t["occ"], t["ao"], t["pts"], K, Ex,
                  rank)
    torch.cuda.synchronize()
    return K.cpu().numpy(), float(Ex.cpu()[0])


@pytest.mark.parametrize("prec", ["f64", "mixed", "f32"])
def test_config3_fused_build_matches_oracle(full3, prec):
    """The fused build against the oracle's whole K and E_x. FP64: relative
    tolerance min(1e-8, 64 eps64 cond(S)). MIXED and F32: the accuracy target,
    |dE_x| <= 1e-5 Ha/cell and max|dK| <= 1e-6."""
    gold = full3["gold"]
    K, E = _build(full3, prec)
    Kref = gold["K"]
    dK = float(np.abs(K - Kref).max())
    dE = abs(E - gold["Ex"])
    cond = max(gold["cond_S_all"])
    print(f"config3 {prec}: cond {cond:.2e} |dEx| {dE:.3e} Ha/cell max|dK| {dK:.3e} "
          f"(rel {dK / np.abs(Kref).max():.2e})")
    if prec == "f64":
        tol = min(1e-8, 64 * EPS64 * cond)
        assert dE <= tol * abs(gold["Ex"]) and dK <= tol * np.abs(Kref).max()
        herm = max(np.abs(K[n] - K[n].conj().T).max() for n in range(K.shape[0]))
        assert herm <= 1e-10 * np.abs(K).max()
        assert E < 0
    else:
        assert dE <= 1e-5
        assert dK <= 1e-6


def test_config3_fused_build_matches_stages(full3):
    """On the 3x3x3 mesh the fused build fits and contracts one transfer of each
    pair (m, -m) and writes Vb^{-m} = conj Vb^m; the stage-wise calls compute
    every transfer. K, E_x and the ranks agree to the FP64 parity tolerance."""
    gold, cell, t, exx, torch, dev = (full3[k] for k in ("gold", "cell", "t", "exx", "torch", "dev"))
    h, c = full3["h"], full3["c"]
    nk, ni, ng, na = cell.N_k, cell.n_isdf, cell.N_g, cell.n_ao
    K_f, E_f = _build(full3, "f64")
    rank_f = torch.empty((nk,), dtype=torch.int32, device=dev)
    K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    exx.exx_build(h, c, exx.EXX_F64, t["psi"], t["occ"], t["ao"], t["pts"], K, Ex, rank_f)
    xi = torch.empty((nk, ni, ng), dtype=torch.complex128, device=dev)
    S = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    V = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
    rank_s = torch.empty((nk,), dtype=torch.int32, device=dev)
    exx.exx_isdf_fit(h, c, exx.EXX_F64, t["psi"], t["occ"], t["pts"], xi, S, rank_s)
    exx.exx_coulomb_V(h, c, exx.EXX_F64, xi, t["pts"], V)
    del xi
    K_s = torch.empty_like(K)
    E_s = torch.empty_like(Ex)
    exx.exx_build_K(h, c, exx.EXX_F64, t["ao"], t["occ"], V, K_s, E_s)
    torch.cuda.synchronize()
    tol = min(1e-8, max(1e-12, 64 * EPS64 * max(gold["cond_S_all"])))
    dK = float(np.abs(K_f - K_s.cpu().numpy()).max() / np.abs(K_s.cpu().numpy()).max())
    dE = abs(E_f - float(E_s.cpu()[0])) / abs(float(E_s.cpu()[0]))
    print(f"fused (paired) vs stage-wise: rel dK {dK:.2e}, rel dE {dE:.2e} (tol {tol:.2e})")
    assert rank_f.cpu().tolist() == rank_s.cpu().tolist()
    assert dK <= 2 * tol and dE <= 2 * tol



def test_config3_bf16_error_report(full3):
    """EXX_BF16 (Gamma and the Coulomb contraction on the BF16 matrix cores) at
    full size against the oracle: the error is reported and bounded (about five
    times the measured values); it is not within the 1e-5 / 1e-6 target, which
    EXX_MIXED and EXX_F32 meet."""
    gold = full3["gold"]
    K, E = _build(full3, "bf16")
    Kref = gold["K"]
    dK = float(np.abs(K - Kref).max())
    dE = abs(E - gold["Ex"])
    print(f"config3 bf16: |dEx| {dE:.3e} Ha/cell (rel {dE / abs(gold['Ex']):.2e}) max|dK| {dK:.3e} "
          f"(rel {dK / np.abs(Kref).max():.2e})")
    # measured: rel |dE_x| 9.2e-6, rel max|dK| 4.2e-3 (4.4e-6 and 4.2e-3 with the
    # contraction on the FP64 cores)
    assert dE <= 2e-5 * abs(gold["Ex"])
    assert dK <= 2e-2 * np.abs(Kref).max()


@pytest.mark.parametrize("prec", ["mixed", "f32"])
def test_config3_split_bf16_contraction_report(full3, prec):
    """EXX_MIXED and EXX_F32 with the contraction on the BF16 matrix cores in the
    split form (EXX_CONTRACT_BF16X3) against the oracle's whole K and E_x: E_x is
    within the 1e-5 Ha/cell target, max|dK| is not within 1e-6 at this cell
    (measured: MIXED 3.0e-6 Ha/cell and 1.9e-6, F32 2.5e-6 and 2.5e-6; the
    operands' 16-bit significands, against 24 with the FP64-core form, set it).
    Bounded at about five times the measured values."""
    exx = full3["exx"]
    gold = full3["gold"]
    h = full3["h"]
    h.set_contraction(exx.EXX_CONTRACT_BF16X3)
    try:
        K, E = _build(full3, prec)
    finally:
        h.set_contraction(exx.EXX_CONTRACT_AUTO)
    dK = float(np.abs(K - gold["K"]).max())
    dE = abs(E - gold["Ex"])
    print(f"config3 {prec} + split BF16 contraction: |dEx| {dE:.3e} Ha/cell max|dK| {dK:.3e}")
    assert dE <= 1.5e-5
    assert dK <= 1.2e-5
