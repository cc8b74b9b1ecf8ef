"""Device-side evaluation of the synthetic occupied orbitals (input preparation).

``orbitals_on_grid_torch`` evaluates exactly what ``cells.orbitals_on_grid``
defines, psi_i^{k_n}(r) = sum_mu C^k_{mu i} phi_mu^k(r), but builds the basis
functions on the grid from their three 1-D factors with torch on a given
device, one k-point at a time, so that large cells (and many training cells)
are generated in seconds instead of minutes. The 1-D factors, norms and
coefficients come from ``cells``; only the outer product and the contraction
with C run in torch.
"""

from __future__ import annotations

import numpy as np
import torch

from .cells import Cell, _factors_1d, _norms, grid_coords


def ao_on_grid_torch(cell: Cell, n: int, device) -> torch.Tensor:
    """phi_mu^{k_n}(r) on the full grid, shape (n_ao, N_g), complex128 on ``device``."""
    k = cell.kvec(n)
    f = [torch.from_numpy(_factors_1d(cell, k, a, grid_coords(cell, a))).to(device) for a in range(3)]
    nrm = torch.from_numpy(_norms(cell).astype(np.complex128)).to(device)
    out = (nrm[:, None, None, None] * f[0][:, :, None, None]) * f[1][:, None, :, None]
    out = out * f[2][:, None, None, :]
    return out.reshape(cell.n_ao, cell.N_g)


def orbitals_on_grid_torch(cell: Cell, C: list, device, dtype=torch.complex128) -> torch.Tensor:
    """(N_k, n_occ, N_g) orbitals on ``device``; same values as ``orbitals_on_grid``."""
    out = torch.empty((cell.N_k, cell.n_occ, cell.N_g), dtype=dtype, device=device)
    for n in range(cell.N_k):
        phi = ao_on_grid_torch(cell, n, device)
        Ct = torch.from_numpy(np.ascontiguousarray(C[n].T)).to(device)
        out[n] = (Ct @ phi).to(dtype)
        del phi
    return out
