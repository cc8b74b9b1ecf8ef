"""O1: exact periodic exchange by one FFT-Poisson solve per pair density (oracle).

TEST INFRASTRUCTURE ONLY (see package docstring).

This is the plain definition of the k-point exchange matrix (Eq. 2) and of
the closed-shell exchange energy, evaluated on the real-space grid with the
Coulomb operator applied in reciprocal space (GPW, Sec. 3):

* for every k-pair (n, n') with transfer m = n' - n and every occupied pair
  (i, j), the pair density rho(r) = e^{-i q_m.r} conj psi_in(r) psi_jn'(r) is
  cell periodic; one FFT gives its Coulomb self-energy J^m[rho, rho];
* E_x = -(1/N_k^2) sum_{n n' i j} J^m[rho, rho]  (closed shell, per cell);
* K^n_{mu nu} = (1/N_k) sum_{n' j} J^m[rho_{mu j}, rho_{nu j}] with
  rho_{mu j} = e^{-i q_m.r} conj phi_mu^n psi_jn', so that
  E_x = -(1/N_k) sum_n Tr(C^n^H K^n C^n) (P = 2 C C^H, Fock exchange -K).

Cost: N_k^2 n_occ^2 FFTs for the energy, N_k^2 n_occ N FFTs for K; only
small cells.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import coulomb
from ._threads import WORKERS


def _fft(a, grid):
    return sfft.fftn(a.reshape((-1,) + tuple(grid)), axes=(1, 2, 3), workers=WORKERS)


def exchange_energy(L, grid, kmesh, psi: np.ndarray) -> float:
    """E_x (Ha per cell) from occupied orbitals psi (N_k, n_occ, N_g)."""
    nk, no, ng = psi.shape
    E = 0.0
    for n in range(nk):
        for n2 in range(nk):
            m = coulomb.transfer_index(kmesh, n, n2)
            v = coulomb.kernel(L, grid, kmesh, m)
            ph = coulomb.bloch_phase(L, grid, coulomb.qvec(L, kmesh, m))
            rho = (psi[n].conj()[:, None, :] * psi[n2][None, :, :]) * ph
            F = _fft(rho.reshape(no * no, ng), grid)
            E += coulomb.pair_integral_from_fft(L, grid, v, F).sum()
    return float(-E / nk ** 2)


def exchange_matrix(L, grid, kmesh, psi: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """AO-basis K^n (N_k, N, N) from orbitals psi (N_k, n_occ, N_g) and basis phi (N_k, N, N_g)."""
    nk, no, ng = psi.shape
    nao = phi.shape[1]
    K = np.zeros((nk, nao, nao), dtype=np.complex128)
    for n in range(nk):
        for n2 in range(nk):
            m = coulomb.transfer_index(kmesh, n, n2)
            v = coulomb.kernel(L, grid, kmesh, m)
            ph = coulomb.bloch_phase(L, grid, coulomb.qvec(L, kmesh, m))
            for j in range(no):
                rho = phi[n].conj() * (psi[n2, j] * ph)[None, :]
                F = _fft(rho, grid)
                K[n] += coulomb.pair_integral_from_fft(L, grid, v, F, F)
    return K / nk


def energy_from_K(K: np.ndarray, C: list) -> float:
    """-(1/N_k) sum_n Tr(C^n^H K^n C^n)."""
    nk = K.shape[0]
    tot = 0.0
    for n in range(nk):
        tot += np.trace(C[n].conj().T @ K[n] @ C[n]).real
    return float(-tot / nk)
