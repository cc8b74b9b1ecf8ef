"""Write the stored oracle values used by the full-size GPU parity tests.

Runs only the FP64 oracle (``oracle/``) on the seeded inputs from ``synth``:

* ``config2.json``: the 48-atom four-ring cell on the 2x2x2 mesh (N = 192,
  n_occ = 84, grid 60x75x54, N_ISDF = 420). Points chosen by the oracle's
  pivoted-Cholesky selection; E_x, ranks, cond(S^m) and seeded samples of
  K^k, Vb^m and S^m.
* ``config3.json``: the same cell on the 3x3x3 mesh. Points by the oracle's
  selection; the fit and Coulomb steps for three of the 27 transfers
  (m = 0, 13, 26): ranks, cond(S^m) and seeded samples of S^m and of the
  Bloch-gauge Coulomb matrix Vb^m.

Usage: ``python tests/golden/make_golden.py [config2|config3]`` (config2 about
three minutes and ~25 GB RAM, config3 a few minutes and ~30 GB).
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
    conds = [float(np.linalg.cond(o["S"][m])) for m in range(nk)]
    out = {
        "workload": "48-atom four-ring cell, 2x2x2 mesh, N=192, n_occ=84, grid 60x75x54, N_ISDF=420",
        "seed": list(c.seed),
        "pts": [int(x) for x in pts],
        "n_pivot": int(npiv),
        "Ex": o["Ex"],
        "Ex_trVS": o["Ex_trVS"],
        "Ex_fromK": direct.energy_from_K(o["K"], C),
        "rank": [int(x) for x in o["rank"]],
        "cond_S": conds,
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
    print(f"wrote {path}: Ex={o['Ex']:.12f} in {out['seconds']:.0f} s")


M3 = (0, 13, 26)


def make_config3(path):
    t0 = time.time()
    c = synth.make_config(3)
    C = synth.orbital_coeffs(c)
    psi = synth.orbitals_on_grid(c, C)
    pts, npiv = select.select_points(psi, c.n_isdf)
    print(f"config3: points selected ({npiv} pivots) in {time.time() - t0:.0f} s", flush=True)
    ao = np.stack([synth.ao_at_points(c, n, pts) for n in range(c.N_k)])
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao, m_subset=list(M3))
    rng = np.random.default_rng(20230406)
    ni = c.n_isdf
    out = {
        "workload": "48-atom four-ring cell, 3x3x3 mesh, N=192, n_occ=84, grid 60x75x54, N_ISDF=420",
        "seed": list(c.seed),
        "pts": [int(x) for x in pts],
        "n_pivot": int(npiv),
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
    print(f"wrote {path} in {out['seconds']:.0f} s")


if __name__ == "__main__":
    which = sys.argv[1:] or ["config2", "config3"]
    if "config2" in which:
        make_config2(os.path.join(HERE, "config2.json"))
    if "config3" in which:
        make_config3(os.path.join(HERE, "config3.json"))
