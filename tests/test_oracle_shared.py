"""Pins of the shared-fit oracle (thc.thc_oo_k_shared: one ISDF fit for the pairs
of every transfer, Sec. 2.2 Eq. 13 on occupied pairs) against facts other than
itself:

* at the Gamma point (one transfer) it is the per-transfer fit;
* its xi is numpy's least-squares solution of the stacked pair matrix of all
  transfers (catches a dropped transfer, a wrong phase or a transposed sum);
* when the points span every pair function of every transfer it reproduces
  direct exchange (O1) for E_x and the occupied block of K;
* the k-convolution form of E_x equals the trace form with the per-transfer
  metrics, and E_x from K (the contraction is the same as the per-q one).

And of the THC-AO-K composition (thc.thc_ao_k: the AO-pair fit done once, the
K-build from the occupied density): exact at full AO pair rank (every entry of
K against direct exchange), and below it E_x from its own K, Hermitian K, and a
fit that does not depend on the occupied orbitals.
"""

import numpy as np
import pytest

import synth
from oracle import coulomb, direct, select, thc


def _orbitals(cell):
    C = synth.orbital_coeffs(cell)
    return C, synth.orbitals_on_grid(cell, C)


def _ao_pts(cell, pts):
    return np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])


def _phi(cell):
    return np.stack([synth.ao_on_grid(cell, n) for n in range(cell.N_k)])


def test_gamma_point_shared_fit_is_the_per_transfer_fit():
    c = synth.make_config(1)
    C, psi = _orbitals(c)
    pts, _ = select.select_points(psi, c.n_isdf)
    ao = _ao_pts(c, pts)
    a = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao)
    b = thc.thc_oo_k_shared(c.L, c.grid, c.kmesh, psi, pts, ao)
    assert b["rank"] == a["rank"][0]
    assert abs(a["Ex"] - b["Ex"]) <= 1e-12 * abs(a["Ex"])
    assert np.abs(a["K"] - b["K"]).max() <= 1e-12 * np.abs(a["K"]).max()


@pytest.fixture(scope="module")
def kshared():
    c = synth.make_random_cell((6.0, 6.5, 7.0), 2, (10, 12, 10), (2, 2, 1), 2, 24, (3, 1, 4))
    C, psi = _orbitals(c)
    pts, _ = select.select_points(psi, c.n_isdf)
    o = thc.thc_oo_k_shared(c.L, c.grid, c.kmesh, psi, pts, _ao_pts(c, pts))
    return c, C, psi, pts, o


def test_shared_fit_is_the_stacked_least_squares_solution(kshared):
    c, C, psi, pts, o = kshared
    Psi = np.stack([psi[n][:, pts].T for n in range(c.N_k)])
    r = coulomb.positions(c.L, c.grid)
    rP = coulomb.positions(c.L, c.grid, pts)
    cols = np.arange(0, c.N_g, 37)
    Bs, As = [], []
    for m in range(c.N_k):
        q = coulomb.qvec(c.L, c.kmesh, m)
        Bs.append(thc.pair_rows(Psi, c.kmesh, m, np.exp(-1j * (rP @ q))))
        for n in range(c.N_k):
            n2 = coulomb.add_index(c.kmesh, n, m)
            blk = psi[n][:, cols].conj()[:, None, :] * psi[n2][:, cols][None, :, :]
            As.append(blk.reshape(-1, len(cols)) * np.exp(-1j * (r[cols] @ q))[None, :])
    B = np.concatenate(Bs)
    A = np.concatenate(As)
    assert o["rank"] == min(B.shape)
    xi_ls = np.linalg.lstsq(B, A, rcond=None)[0]
    ref = o["xi"][:, cols]
    assert np.abs(xi_ls - ref).max() <= 1e-7 * np.abs(ref).max()


def test_shared_fit_energy_identities(kshared):
    c, C, psi, pts, o = kshared
    assert abs(o["Ex"] - o["Ex_trVS"]) <= 1e-10 * abs(o["Ex"])
    assert abs(o["Ex"] - direct.energy_from_K(o["K"], C)) <= 1e-10 * abs(o["Ex"])
    assert o["Ex"] < 0
    for n in range(c.N_k):
        assert np.abs(o["K"][n] - o["K"][n].conj().T).max() <= 1e-12 * np.abs(o["K"]).max()


def test_shared_fit_at_full_pair_rank_reproduces_direct_exchange():
    """2x1x1 mesh, two occupied orbitals: the pairs of both transfers span
    (N_k n_occ)^2 = 16 functions; 40 points span them all, so the shared fit is
    exact for every pair and the THC energy is the direct one."""
    c = synth.make_random_cell((6.0, 5.0, 5.0), 2, (12, 10, 10), (2, 1, 1), 2, 40, (3, 2, 7))
    C, psi = _orbitals(c)
    pts, _ = select.select_points(psi, c.n_isdf)
    o = thc.thc_oo_k_shared(c.L, c.grid, c.kmesh, psi, pts, _ao_pts(c, pts))
    assert o["rank"] == (c.N_k * c.n_occ) ** 2
    E1 = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    assert abs(o["Ex"] - E1) <= 1e-10 * abs(E1)
    K1 = direct.exchange_matrix(c.L, c.grid, c.kmesh, psi, _phi(c))
    for n in range(c.N_k):
        oo2 = C[n].conj().T @ o["K"][n] @ C[n]
        oo1 = C[n].conj().T @ K1[n] @ C[n]
        assert np.abs(oo2 - oo1).max() <= 1e-9 * np.abs(oo1).max()


# ---------------------------------------------------------------------------
# THC-AO-K (the AO-pair fit, done once, and the K-build from the occupied density)
# ---------------------------------------------------------------------------

def test_thc_ao_k_at_full_pair_rank_is_direct_exchange():
    """2x1x1 mesh, one atom (4 AO functions): the AO pairs of a transfer span at
    most N_k N^2 = 32 functions (fewer independent ones on this grid); with every
    grid point offered in QRCP order the fit spans them all and is exact, so K
    (every AO entry, not only the occupied block) and E_x equal direct exchange.
    (In flat grid order the point-order Cholesky keeps nearly dependent points
    of the AO pair space, whose conditioning then ruins the fit: the points are
    an input, and QRCP is the selection this fit needs.)"""
    c = synth.make_random_cell((4.0, 4.5, 5.0), 1, (6, 6, 8), (2, 1, 1), 2, 288, (9, 9, 9))
    C, psi = _orbitals(c)
    phi = _phi(c)
    pts, _ = select.select_points(phi, c.N_g)
    o = thc.thc_ao_k(c.L, c.grid, c.kmesh, phi, psi, pts)
    assert np.all(o["rank"] <= c.N_k * c.n_ao ** 2)
    K1 = direct.exchange_matrix(c.L, c.grid, c.kmesh, psi, phi)
    assert np.abs(o["K"] - K1).max() <= 1e-10 * np.abs(K1).max()
    E1 = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    assert abs(o["Ex"] - E1) <= 1e-12 * abs(E1)


def test_thc_ao_k_below_full_rank_identities():
    """Below full rank: E_x equals the energy of its own K, K is Hermitian, and
    the fit is independent of the occupied orbitals (a second orbital set reuses
    M^q unchanged, as Algorithm 1 does inside the SCF loop)."""
    c = synth.make_random_cell((5.0, 5.0, 6.0), 2, (10, 10, 12), (2, 2, 1), 3, 80, (4, 4, 4))
    C, psi = _orbitals(c)
    phi = _phi(c)
    pts, _ = select.select_points(phi, c.n_isdf)
    o = thc.thc_ao_k(c.L, c.grid, c.kmesh, phi, psi, pts)
    assert abs(o["Ex"] - direct.energy_from_K(o["K"], C)) <= 1e-10 * abs(o["Ex"])
    # Hermitian to the rounding of the AO pair metric's solve (that metric is far
    # worse conditioned than the occupied one)
    for n in range(c.N_k):
        assert np.abs(o["K"][n] - o["K"][n].conj().T).max() <= 1e-9 * np.abs(o["K"]).max()
    C2 = synth.orbital_coeffs(synth.make_random_cell((5.0, 5.0, 6.0), 2, (10, 10, 12), (2, 2, 1),
                                                     3, 80, (4, 4, 5)))
    psi2 = synth.orbitals_on_grid(c, C2)
    o2 = thc.thc_ao_k(c.L, c.grid, c.kmesh, phi, psi2, pts)
    assert np.array_equal(o2["Vb"], o["Vb"])
    assert abs(o2["Ex"] - direct.energy_from_K(o2["K"], C2)) <= 1e-10 * abs(o2["Ex"])
