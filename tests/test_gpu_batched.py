"""Batched builds (exx_build_batched): heterogeneous cells in one call, with and
without graph capture and tile autotuning, against the single-cell build and
the FP64 oracle. Graph replays are checked one by one with eager work and
synchronisations between them."""

import numpy as np
import pytest

import synth
from oracle import select, thc

pytestmark = pytest.mark.gpu


def _cells():
    return [
        synth.make_config(1),
        synth.make_random_cell((6.0, 6.5, 7.0), 2, (12, 15, 10), (2, 2, 2), 3, 30, (12, 1, 1)),
        synth.make_random_cell((5.0, 6.0, 7.5), 3, (16, 18, 20), (3, 2, 1), 5, 100, (12, 2, 1)),
        synth.make_random_cell((5.0, 5.0, 5.0), 2, (10, 12, 9), (3, 3, 3), 2, 40, (12, 3, 1)),
    ]


@pytest.fixture(scope="module")
def batch():
    import torch

    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    cases = []
    for cell in _cells():
        C = synth.orbital_coeffs(cell)
        psi = synth.orbitals_on_grid(cell, C)
        pts, _ = select.select_points(psi, cell.n_isdf)
        ao = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
        ref = thc.thc_oo_k(cell.L, cell.grid, cell.kmesh, psi, pts, ao)
        t = {
            "cell": exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, len(pts)),
            "psi64": torch.from_numpy(psi).to(dev),
            "occ_pts": torch.from_numpy(np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))).to(dev),
            "ao_pts": torch.from_numpy(np.ascontiguousarray(np.transpose(ao, (0, 2, 1)))).to(dev),
            "pts": torch.from_numpy(pts.astype(np.int32)).to(dev),
            "K": torch.empty((cell.N_k, cell.n_ao, cell.n_ao), dtype=torch.complex128, device=dev),
            "Ex": torch.empty((1,), dtype=torch.float64, device=dev),
            "rank": torch.empty((cell.N_k,), dtype=torch.int32, device=dev),
        }
        cases.append((cell, ref, t))
    return cases


def _items(cases, prec):
    import torch

    out = []
    for cell, ref, t in cases:
        psi = t["psi64"] if prec in ("f64", "mixed") else t["psi64"].to(torch.complex64)
        out.append({"cell": t["cell"], "psi_grid": psi, "occ_pts": t["occ_pts"], "ao_pts": t["ao_pts"],
                    "pts": t["pts"], "K": t["K"], "Ex": t["Ex"], "rank": t["rank"]})
    return out


def _single(h, exx, it, prec):
    import torch

    K = torch.empty_like(it["K"])
    Ex = torch.empty_like(it["Ex"])
    rank = torch.empty_like(it["rank"])
    exx.exx_build(h, it["cell"], exx.PREC[prec], it["psi_grid"], it["occ_pts"], it["ao_pts"],
                  it["pts"], K, Ex, rank)
    torch.cuda.synchronize()
    return K.cpu().numpy(), float(Ex.cpu()[0]), rank.cpu().numpy()


@pytest.mark.parametrize("prec", ["f64", "mixed", "f32"])
@pytest.mark.parametrize("flags", [0, 2, 1, 3, 4, 6])
def test_batched_equals_single_builds(batch, prec, flags, gpu):
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    items = _items(batch, prec)
    singles = [_single(h, exx, it, prec) for it in items]
    stream = torch.cuda.Stream() if flags & exx.EXX_BATCH_GRAPH else None
    reps = 3 if flags & exx.EXX_BATCH_GRAPH else 1
    for rep in range(reps):
        for it in items:
            it["K"].zero_()
            it["Ex"].zero_()
            it["rank"].zero_()
        torch.cuda.synchronize()
        if stream is not None:
            stream.wait_stream(torch.cuda.current_stream())
            exx.exx_build_batched(h, items, exx.PREC[prec], flags, stream=stream)
            stream.synchronize()
        else:
            exx.exx_build_batched(h, items, exx.PREC[prec], flags)
            torch.cuda.synchronize()
        # eager work between replays
        _ = (items[0]["K"].abs().sum()).item()
        for (cell, ref, t), it, (Ks, Es, rs) in zip(batch, items, singles):
            K = it["K"].cpu().numpy()
            Ex = float(it["Ex"].cpu()[0])
            assert np.array_equal(it["rank"].cpu().numpy(), rs)
            assert np.abs(K - Ks).max() <= 1e-13 * np.abs(Ks).max(), f"rep {rep}"
            assert abs(Ex - Es) <= 1e-13 * abs(Es), f"rep {rep}"
            assert np.array_equal(rs, ref["rank"])
            # the parity tests' bounds against the oracle, for E_x and the whole K
            conds = []
            for m in range(ref["S"].shape[0]):
                R = np.flatnonzero(ref["keep"][m])
                conds.append(np.linalg.cond(ref["S"][m][np.ix_(R, R)]))
            cond = max(conds)
            dE = abs(Ex - ref["Ex"]) / abs(ref["Ex"])
            dK = np.abs(K - ref["K"]).max() / np.abs(ref["K"]).max()
            # beyond cond 1e10 FP64 itself fixes K only to ~eps64 cond (either side)
            floor = min(1e-5, 4 * np.finfo(np.float64).eps * cond) if cond > 1e10 else 0.0
            msg = f"{cell.name} {prec}: cond {cond:.2e} rel dE {dE:.2e} rel dK {dK:.2e}"
            if prec == "f64":
                tol = min(1e-8, max(1e-12, 64 * np.finfo(np.float64).eps * cond))
                assert dE <= tol and dK <= max(tol, floor), msg
            elif prec == "mixed":
                assert dE <= 3e-7 and dK <= max(3e-7, floor), msg
            elif cond <= 1e10:
                # F32 data is amplified by the metric: beyond cond 1e10 (the 3x2x1
                # cell here, 6e12) its result is not compared with the oracle
                assert dE <= 1e-6, msg
                assert dK <= 8 * np.finfo(np.float32).eps * np.sqrt(cond), msg


@pytest.mark.skip(reason="capturing concurrent lanes into one graph (EXX_BATCH_GRAPH | "
                  "EXX_BATCH_CONCURRENT) ended in a host segmentation fault whose cause is not "
                  "found; the library rejects the combination, and this case stays off the GPU")
def test_graph_with_concurrent_lanes(batch, gpu):
    from paper_2304_05505_amd import exx
    import torch

    h = exx.Handle(0)
    items = _items(batch, "f64")
    exx.exx_build_batched(h, items, exx.EXX_F64, exx.EXX_BATCH_GRAPH | exx.EXX_BATCH_CONCURRENT,
                          stream=torch.cuda.Stream())


def test_graph_and_lanes_is_rejected_before_launch(batch, gpu):
    """The switched-off combination returns EXX_ERR_UNSUPPORTED before anything runs."""
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    items = _items(batch, "f64")
    with pytest.raises(exx.ExxError) as ei:
        exx.exx_build_batched(h, items, exx.EXX_F64,
                              exx.EXX_BATCH_GRAPH | exx.EXX_BATCH_CONCURRENT,
                              stream=torch.cuda.Stream())
    assert ei.value.status == -7


def test_graph_requires_a_stream(batch, gpu):
    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    items = _items(batch, "f64")
    with pytest.raises(ValueError):
        exx.exx_build_batched(h, items, exx.EXX_F64, exx.EXX_BATCH_GRAPH)


def test_tuning_table_round_trip(batch, gpu, tmp_path):
    """The autotuned tile table saved to a file and loaded into a fresh handle
    gives the same table (and the same batched results without re-tuning); a
    malformed file is rejected."""
    import torch

    from paper_2304_05505_amd import exx

    h = exx.Handle(0)
    items = _items(batch, "f64")
    exx.exx_build_batched(h, items, exx.EXX_F64, exx.EXX_BATCH_TUNE)
    torch.cuda.synchronize()
    K0 = [it["K"].clone() for it in items]
    path = tmp_path / "tiles.txt"
    h.save_tuning(str(path))
    lines = [ln for ln in path.read_text().splitlines() if not ln.startswith("#")]
    assert len(lines) == len({(c.n_isdf, c.N_g, c.n_occ, c.N_k) for c, _, _ in batch})
    h2 = exx.Handle(0)
    h2.load_tuning(str(path))
    path2 = tmp_path / "tiles2.txt"
    h2.save_tuning(str(path2))
    assert path2.read_text() == path.read_text()
    exx.exx_build_batched(h2, items, exx.EXX_F64, 0)
    torch.cuda.synchronize()
    for it, k in zip(items, K0):
        assert torch.equal(it["K"], k)
    bad = tmp_path / "bad.txt"
    bad.write_text("420 243000 84 8 0 22\n")
    with pytest.raises(exx.ExxError):
        h2.load_tuning(str(bad))
