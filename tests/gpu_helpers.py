"""Helpers shared by the GPU tests: build inputs, run the HIP path through the C ABI."""

from __future__ import annotations

import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def inputs(cell, pts=None, tr=False):
    C = synth.orbital_coeffs(cell, tr_symmetric=tr)
    psi = synth.orbitals_on_grid(cell, C)
    out = {"C": C, "psi": psi}
    if pts is not None:
        out["ao_pts"] = np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])
        out["occ_pts"] = np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))
    return out


def run_gpu(cell, psi, pts, ao_pts, prec="f64", stages=True, handle=None):
    """Run fit, Coulomb and K on the GPU; return numpy copies of every output."""
    import torch

    from paper_2304_05505_amd import exx

    dev = torch.device("cuda", 0)
    h = handle or exx.Handle(0)
    p = exx.PREC[prec]
    c = exx.make_cell(cell.L, cell.grid, cell.kmesh, cell.n_occ, cell.n_ao, len(pts))
    wide = prec in ("f64", "mixed")
    gd = torch.complex128 if prec == "f64" else torch.complex64
    nk, no, ng, ni, na = cell.N_k, cell.n_occ, cell.N_g, len(pts), cell.n_ao
    t_psi = torch.from_numpy(psi.astype(np.complex128 if wide else np.complex64)).to(dev)
    occ = np.ascontiguousarray(np.transpose(psi[:, :, pts], (0, 2, 1)))
    t_occ = torch.from_numpy(occ).to(dev)
    t_ao = torch.from_numpy(np.ascontiguousarray(np.transpose(ao_pts, (0, 2, 1)))).to(dev)
    t_pts = torch.from_numpy(np.asarray(pts, dtype=np.int32)).to(dev)
    K = torch.empty((nk, na, na), dtype=torch.complex128, device=dev)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    rank = torch.empty((nk,), dtype=torch.int32, device=dev)
    out = {}
    if stages:
        xi = torch.empty((nk, ni, ng), dtype=gd, device=dev)
        S = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
        V = torch.empty((nk, ni, ni), dtype=torch.complex128, device=dev)
        exx.exx_isdf_fit(h, c, p, t_psi, t_occ, t_pts, xi, S, rank)
        exx.exx_coulomb_V(h, c, p, xi, t_pts, V)
        exx.exx_build_K(h, c, p, t_ao, t_occ, V, K, Ex)
        torch.cuda.synchronize()
        out.update(xi=xi.cpu().numpy(), S=S.cpu().numpy(), V=V.cpu().numpy())
    else:
        exx.exx_build(h, c, p, t_psi, t_occ, t_ao, t_pts, K, Ex, rank)
        torch.cuda.synchronize()
    out.update(K=K.cpu().numpy(), Ex=float(Ex.cpu().numpy()[0]), rank=rank.cpu().numpy())
    return out


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def load_golden_arrays(name):
    """Arrays stored beside a golden JSON file (plain numeric .npz, no pickles)."""
    with np.load(os.path.join(GOLDEN, name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def cplx_list(a):
    a = np.asarray(a)
    return [[float(x.real), float(x.imag)] for x in a.reshape(-1)]


def from_cplx_list(v):
    v = np.asarray(v, dtype=np.float64)
    return v[:, 0] + 1j * v[:, 1]
