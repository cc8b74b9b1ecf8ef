"""Write the stored oracle values used by the full-size GPU parity tests.

Runs only the FP64 oracle (``oracle/``) on the seeded inputs from ``synth``:

* ``config2.json`` + ``config2_K.npz``: the 48-atom four-ring cell on the
  2x2x2 mesh (N = 192, n_occ = 84, grid 60x75x54, N_ISDF = 420). Points chosen
  by the oracle's pivoted-Cholesky selection; E_x (three forms), ranks,
  cond(S^m), seeded samples of Vb^m and S^m, and the whole K^k.
* ``config3.json`` + ``config3_K.npz``: the same cell on the 3x3x3 mesh, all
  27 transfers: E_x (three forms), ranks and cond(S^m) of every transfer,
  seeded samples of S^m and Vb^m for m = 0, 13, 26, and the whole K^k.
* ``config5.json`` + ``config5_K.npz``: the 4x4x4 ring cell with 2s + 2p per atom
  (N = 384, n_occ = 84, grid 72x90x64, N_ISDF = 420), all 64 transfers: E_x,
  ranks, cond(S^m), every diagonal of K and 4000 seeded entries.
* ``config5c.json`` + ``config5c_K.npz``: the same 4x4x4 cell on the coarser
  36x45x32 grid (same seed, basis, n_occ and N_ISDF), with the same contents.
* ``config4.json`` + ``config4_K.npz``: the 24 cells of the batched workload
  (2 x {8, 16, 24, 48 atoms} x {1^3, 2^3, 3^3}), each with its own oracle
  points: E_x (two forms), ranks, cond(S^m), the diagonal of every K^k and
  2000 seeded entries of K.

Each ``.npz`` holds plain complex128 arrays (no pickled objects).

Usage: ``python tests/golden/make_golden.py [config2] [config3] [config4] [config5] [config5c]``.
Wall times on 8 cores: config2 a few minutes (~25 GB RAM), config3 about
half an hour (~30 GB), config4 about an hour (~30 GB), config5c about an hour
(~35 GB), config5 about half a day (~40 GB).
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import direct, select, thc  # noqa: E402


def cl(a):
    a = np.asarray(a).reshape(-1)
    return [[float(x.real), float(x.imag)] for x in a]


def _conds(o, nk):
    """cond(S^m) over the retained points of each transfer."""
    out = []
    for m in range(nk):
        R = np.flatnonzero(o["keep"][m])
        out.append(float(np.linalg.cond(o["S"][m][np.ix_(R, R)])))
    return out


def make_config2(path):
    t0 = time.time()
    c = synth.make_config(2)
    C = synth.orbital_coeffs(c)
    psi = synth.orbitals_on_grid(c, C)
    pts, npiv = select.select_points(psi, c.n_isdf)
    ao = np.stack([synth.ao_at_points(c, n, pts) for n in range(c.N_k)])
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao)
    rng = np.random.default_rng(20230405)
    nk, na, ni = c.N_k, c.n_ao, c.n_isdf
    kn = rng.integers(0, nk, 1000)
    kmu = rng.integers(0, na, 1000)
    knu = rng.integers(0, na, 1000)
    vm = rng.integers(0, nk, 1000)
    vp = rng.integers(0, ni, 1000)
    vq = rng.integers(0, ni, 1000)
    out = {
        "workload": "48-atom four-ring cell, 2x2x2 mesh, N=192, n_occ=84, grid 60x75x54, N_ISDF=420",
        "seed": list(c.seed),
        "pts": [int(x) for x in pts],
        "n_pivot": int(npiv),
        "Ex": o["Ex"],
        "Ex_trVS": o["Ex_trVS"],
        "Ex_fromK": direct.energy_from_K(o["K"], C),
        "rank": [int(x) for x in o["rank"]],
        "cond_S": _conds(o, nk),
        "maxabs_K": float(np.abs(o["K"]).max()),
        "maxabs_Vb": float(np.abs(o["Vb"]).max()),
        "K_idx": [[int(a), int(b), int(d)] for a, b, d in zip(kn, kmu, knu)],
        "K_val": cl(o["K"][kn, kmu, knu]),
        "K0_diag": cl(np.diagonal(o["K"][0])),
        "Vb_idx": [[int(a), int(b), int(d)] for a, b, d in zip(vm, vp, vq)],
        "Vb_val": cl(o["Vb"][vm, vp, vq]),
        "S_val": cl(o["S"][vm, vp, vq]),
        "seconds": time.time() - t0,
    }
    with open(path, "w") as f:
        json.dump(out, f)
    np.savez_compressed(path.replace(".json", "_K.npz"), K=o["K"])
    print(f"wrote {path}: Ex={o['Ex']:.12f} in {out['seconds']:.0f} s", flush=True)


M3 = (0, 13, 26)


def make_config3(path):
    t0 = time.time()
    c = synth.make_config(3)
    C = synth.orbital_coeffs(c)
    psi = synth.orbitals_on_grid(c, C)
    pts, npiv = select.select_points(psi, c.n_isdf)
    print(f"config3: points selected ({npiv} pivots) in {time.time() - t0:.0f} s", flush=True)
    ao = np.stack([synth.ao_at_points(c, n, pts) for n in range(c.N_k)])
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao)
    rng = np.random.default_rng(20230406)
    ni, nk = c.n_isdf, c.N_k
    out = {
        "workload": "48-atom four-ring cell, 3x3x3 mesh, N=192, n_occ=84, grid 60x75x54, N_ISDF=420",
        "seed": list(c.seed),
        "pts": [int(x) for x in pts],
        "n_pivot": int(npiv),
        "Ex": o["Ex"],
        "Ex_trVS": o["Ex_trVS"],
        "Ex_fromK": direct.energy_from_K(o["K"], C),
        "rank_all": [int(x) for x in o["rank"]],
        "cond_S_all": _conds(o, nk),
        "maxabs_K": float(np.abs(o["K"]).max()),
        "m": list(M3),
        "rank": [int(o["rank"][m]) for m in M3],
        "cond_S": [float(np.linalg.cond(o["S"][m])) for m in M3],
        "maxabs_Vb": [float(np.abs(o["Vb"][m]).max()) for m in M3],
        "seconds": 0.0,
    }
    for m in M3:
        vp = rng.integers(0, ni, 1000)
        vq = rng.integers(0, ni, 1000)
        out[f"idx_{m}"] = [[int(a), int(b)] for a, b in zip(vp, vq)]
        out[f"Vb_{m}"] = cl(o["Vb"][m][vp, vq])
        out[f"S_{m}"] = cl(o["S"][m][vp, vq])
        out[f"Vbdiag_{m}"] = cl(np.diagonal(o["Vb"][m]))
    out["seconds"] = time.time() - t0
    with open(path, "w") as f:
        json.dump(out, f)
    np.savez_compressed(path.replace(".json", "_K.npz"), K=o["K"])
    print(f"wrote {path}: Ex={o['Ex']:.12f} in {out['seconds']:.0f} s", flush=True)


def make_config4(path):
    cells = synth.make_batch_cells()
    rng = np.random.default_rng(20230407)
    meta, arrays = [], {}
    for i, c in enumerate(cells):
        t0 = time.time()
        C = synth.orbital_coeffs(c)
        psi = synth.orbitals_on_grid(c, C)
        pts, npiv = select.select_points(psi, c.n_isdf)
        ao = np.stack([synth.ao_at_points(c, n, pts) for n in range(c.N_k)])
        t1 = time.time()
        o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao)
        t_build = time.time() - t1
        nk, na = c.N_k, c.n_ao
        kn = rng.integers(0, nk, 2000)
        kmu = rng.integers(0, na, 2000)
        knu = rng.integers(0, na, 2000)
        meta.append({
            "name": c.name,
            "seed": list(c.seed),
            "kmesh": list(c.kmesh),
            "grid": list(c.grid),
            "n_occ": c.n_occ,
            "n_ao": c.n_ao,
            "n_isdf": c.n_isdf,
            "pts": [int(x) for x in pts],
            "n_pivot": int(npiv),
            "Ex": o["Ex"],
            "Ex_trVS": o["Ex_trVS"],
            "rank": [int(x) for x in o["rank"]],
            "cond_S": _conds(o, nk),
            "maxabs_K": float(np.abs(o["K"]).max()),
            "oracle_build_s": t_build,
        })
        arrays[f"idx_{i}"] = np.stack([kn, kmu, knu], axis=1).astype(np.int32)
        arrays[f"val_{i}"] = o["K"][kn, kmu, knu]
        arrays[f"diag_{i}"] = np.stack([np.diagonal(o["K"][n]) for n in range(nk)])
        print(f"config4 cell {i} ({c.name}): Ex={o['Ex']:.12f}, selection {t1 - t0:.0f} s, "
              f"oracle build {t_build:.0f} s", flush=True)
        del psi, o
    with open(path, "w") as f:
        json.dump({"workload": "24 cells: 2 x {8, 16, 24, 48 atoms} x {1, 2, 3}^3 k-meshes, "
                               "4 functions/atom, n_occ = 0.44 N, N_ISDF = 2.2 N, oracle points",
                   "cells": meta}, f)
    np.savez_compressed(path.replace(".json", "_K.npz"), **arrays)
    print(f"wrote {path}", flush=True)


def make_config5(path, coarse=False):
    """The 4x4x4 ring cell with the 2s + 2p basis (N = 384, n_occ = 84, grid
    72x90x64, N_ISDF = 420; with coarse, the same cell on the 36x45x32 grid):
    oracle points, E_x (two forms), ranks, cond(S^m), the diagonal of every K^k
    and 4000 seeded entries of K."""
    t0 = time.time()
    c = synth.make_config5_coarse() if coarse else synth.make_config(5)
    tag = "config5c" if coarse else "config5"
    C = synth.orbital_coeffs(c)
    psi = synth.orbitals_on_grid(c, C)
    pts, npiv = select.select_points(psi, c.n_isdf)
    print(f"{tag}: points selected ({npiv} pivots) in {time.time() - t0:.0f} s", flush=True)
    ao = np.stack([synth.ao_at_points(c, n, pts) for n in range(c.N_k)])
    t1 = time.time()
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao)
    t_build = time.time() - t1
    rng = np.random.default_rng(20230408)
    nk, na = c.N_k, c.n_ao
    kn = rng.integers(0, nk, 4000)
    kmu = rng.integers(0, na, 4000)
    knu = rng.integers(0, na, 4000)
    out = {
        "workload": "48-atom four-ring cell, 4x4x4 mesh, 2s+2p basis N=384, n_occ=84, grid "
                    f"{'x'.join(map(str, c.grid))}, N_ISDF=420",
        "seed": list(c.seed),
        "pts": [int(x) for x in pts],
        "n_pivot": int(npiv),
        "Ex": o["Ex"],
        "Ex_trVS": o["Ex_trVS"],
        "rank": [int(x) for x in o["rank"]],
        "cond_S": _conds(o, nk),
        "maxabs_K": float(np.abs(o["K"]).max()),
        "oracle_build_s": t_build,
    }
    with open(path, "w") as f:
        json.dump(out, f)
    np.savez_compressed(path.replace(".json", "_K.npz"),
                        idx=np.stack([kn, kmu, knu], axis=1).astype(np.int32),
                        val=o["K"][kn, kmu, knu],
                        diag=np.stack([np.diagonal(o["K"][n]) for n in range(nk)]))
    print(f"wrote {path}: Ex={o['Ex']:.12f}, oracle build {t_build:.0f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["config2", "config3", "config4", "config5"]
    if "config2" in which:
        make_config2(os.path.join(HERE, "config2.json"))
    if "config3" in which:
        make_config3(os.path.join(HERE, "config3.json"))
    if "config4" in which:
        make_config4(os.path.join(HERE, "config4.json"))
    if "config5" in which:
        make_config5(os.path.join(HERE, "config5.json"))
    if "config5c" in which:
        make_config5(os.path.join(HERE, "config5c.json"), coarse=True)
