"""Periodic Coulomb kernel and pair integrals on the FFT grid (oracle).

TEST INFRASTRUCTURE ONLY (see package docstring).

The Coulomb integral of two cell-periodic functions f1, f2 that carry a Bloch
phase e^{i q.r} is evaluated in reciprocal space, as in the GPW scheme the
paper uses for M_PQ (Sec. 2.1, after Eq. 9; M^q in Eq. 15):

    J^m[f1, f2] = (Omega / N_g^2) sum_g v^m(g) F1(g) conj F2(g),
    F(g) = sum_r f(r) exp(-2 pi i sum_i g_i r_i / n_i)   (numpy fftn sign)

with v^m(g) = 4 pi / |K|^2. K is the representative of G + q_m chosen inside
the symmetric FFT box of the Born-von Karman supercell:

    kappa_i = wrap_{N_i n_i}(N_i g_i + m_i),   K = sum_i kappa_i b_i / N_i,
    wrap_L(x) = ((x + floor(L/2)) mod L) - floor(L/2),

and the single K = 0 term (m = 0, g = 0) is dropped (no Madelung term; the
paper's Sec. 3 uses a Madelung correction, the workloads here drop G+q = 0).
With this choice a k-mesh calculation equals the Gamma-point calculation on
the supercell divided by N_k.
"""

from __future__ import annotations

import numpy as np


def transfer_index(kmesh, n: int, n2: int) -> int:
    """Flat index m of q = k_{n2} - k_n reduced onto the mesh: m_i = (n2_i - n_i) mod N_i."""
    a = np.unravel_index(n, kmesh)
    b = np.unravel_index(n2, kmesh)
    m = tuple((int(b[i]) - int(a[i])) % kmesh[i] for i in range(3))
    return int(np.ravel_multi_index(m, kmesh))


def add_index(kmesh, n: int, m: int) -> int:
    """Flat index of k_n + q_m on the mesh (per-axis addition mod N_i)."""
    a = np.unravel_index(n, kmesh)
    b = np.unravel_index(m, kmesh)
    return int(np.ravel_multi_index(tuple((int(a[i]) + int(b[i])) % kmesh[i] for i in range(3)), kmesh))


def qvec(L, kmesh, m: int) -> np.ndarray:
    """q_m = sum_i (m_i / N_i) b_i with b_i = 2 pi / L_i e_i."""
    mi = np.unravel_index(m, kmesh)
    return np.array([mi[i] / kmesh[i] * 2 * np.pi / L[i] for i in range(3)])


def _wrap(x, L):
    h = L // 2
    return np.mod(x + h, L) - h


def kernel(L, grid, kmesh, m: int) -> np.ndarray:
    """v^m(g) = 4 pi / |K|^2 on the FFT box, shape ``grid``; zero at K = 0."""
    mi = np.unravel_index(m, kmesh)
    comps = []
    for i in range(3):
        g = np.arange(grid[i])
        kap = _wrap(kmesh[i] * g + mi[i], kmesh[i] * grid[i])
        comps.append(kap * (2 * np.pi / (kmesh[i] * L[i])))
    K2 = comps[0][:, None, None] ** 2 + comps[1][None, :, None] ** 2 + comps[2][None, None, :] ** 2
    v = np.zeros(K2.shape)
    nz = K2 > 0
    v[nz] = 4 * np.pi / K2[nz]
    return v


def positions(L, grid, flat_idx=None) -> np.ndarray:
    """Cartesian coordinates of grid points (all points if ``flat_idx`` is None)."""
    if flat_idx is None:
        flat_idx = np.arange(int(np.prod(grid)))
    idx = np.unravel_index(np.asarray(flat_idx, dtype=np.int64), grid)
    return np.stack([idx[i] * (L[i] / grid[i]) for i in range(3)], axis=-1)


def bloch_phase(L, grid, q, flat_idx=None, sign=-1.0) -> np.ndarray:
    """exp(sign * i q.r) at the grid points."""
    r = positions(L, grid, flat_idx)
    return np.exp(sign * 1j * (r @ q))


def pair_integral_from_fft(L, grid, v, F1, F2=None):
    """J[f1, f2] = (Omega/N_g^2) sum_g v F1 conj F2 for stacks of transformed functions.

    ``F1`` (a, n1, n2, n3) and ``F2`` (b, n1, n2, n3) give the (a, b) matrix;
    with ``F2`` None the diagonal sum_g v |F1|^2 for each function is returned.
    """
    omega = float(np.prod(L))
    ng = int(np.prod(grid))
    pref = omega / ng ** 2
    a = F1.reshape(F1.shape[0], -1)
    vf = v.reshape(-1)
    if F2 is None:
        return pref * (np.abs(a) ** 2 @ vf)
    b = F2.reshape(F2.shape[0], -1)
    return pref * ((a * vf) @ b.conj().T)
