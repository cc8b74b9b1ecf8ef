"""Pins of the robust-fit oracle (thc.thc_oo_k_robust: one fitted and one exact
pair density in each exchange integral) against facts other than itself:

* the residual identity K_direct - K_rob = K[delta, delta], with the residual
  pair densities delta = rho - rho~ formed explicitly on the grid (every AO-
  orbital pair, every k-pair) and their exchange matrix taken by one FFT-Poisson
  solve per pair, as direct exchange does: a route that shares nothing with the
  oracle's potentials-and-Gamma form of the one-sided term, so a wrong sign,
  phase, conjugate or transfer index in that term fails it;
* at full occupied-pair rank the occupied rows of K_rob are exact
  (C^H K_rob = C^H K_direct, because every delta_{i j} vanishes), while those of
  the plain fit K_fit are not;
* the robust energy equals the fitted one (the fit is a projection of the
  occupied pairs), and equals the energy of K_rob;
* below full rank K_rob is closer to direct exchange than K_fit.
"""

import numpy as np
import pytest
import scipy.fft as sfft

import synth
from oracle import coulomb, direct, select, thc


def _cell(kind):
    if kind == "k211":      # N_ISDF 14 spans the N_k n_occ^2 = 8 pairs: full pair rank
        return synth.make_random_cell((5.0, 5.5, 6.0), 2, (10, 10, 12), (2, 1, 1), 2, 14, (7, 7, 7))
    if kind == "k211-low":  # N_ISDF 12 below the pair rank 18
        return synth.make_random_cell((5.0, 5.5, 6.0), 2, (10, 10, 12), (2, 1, 1), 3, 12, (7, 7, 6))
    if kind == "k311":
        return synth.make_random_cell((6.0, 5.0, 5.0), 2, (12, 10, 10), (3, 1, 1), 2, 10, (7, 7, 8))
    return synth.make_random_cell((6.0, 6.0, 6.0), 3, (12, 12, 12), (1, 1, 1), 3, 7, (7, 7, 9))


def _setup(kind):
    c = _cell(kind)
    C = synth.orbital_coeffs(c)
    psi = synth.orbitals_on_grid(c, C)
    phi = np.stack([synth.ao_on_grid(c, n) for n in range(c.N_k)])
    pts, _ = select.select_points(psi, c.n_isdf)
    return c, C, psi, phi, pts


def _residual_exchange(c, psi, phi, pts, xi):
    """K[delta, delta]^n = (1/N_k) sum_{n' j} J^m[delta_{mu j}, delta_{nu j}] with
    delta_{mu j}(r) = e^{-i q.r} conj phi_mu^n(r) psi_jn'(r)
                      - sum_P xi^m_P(r) e^{-i q.r_P} conj phi_mu^n(r_P) psi_jn'(r_P)."""
    nk, no, ng = psi.shape
    nao = phi.shape[1]
    r = coulomb.positions(c.L, c.grid)
    rP = coulomb.positions(c.L, c.grid, pts)
    K = np.zeros((nk, nao, nao), dtype=np.complex128)
    for n in range(nk):
        for n2 in range(nk):
            m = coulomb.transfer_index(c.kmesh, n, n2)
            q = coulomb.qvec(c.L, c.kmesh, m)
            v = coulomb.kernel(c.L, c.grid, c.kmesh, m)
            for j in range(no):
                exact = phi[n].conj() * (psi[n2, j] * np.exp(-1j * (r @ q)))[None, :]
                coef = phi[n][:, pts].conj() * (psi[n2, j, pts] * np.exp(-1j * (rP @ q)))[None, :]
                delta = exact - coef @ xi[m]
                F = sfft.fftn(delta.reshape((nao,) + tuple(c.grid)), axes=(1, 2, 3))
                K[n] += coulomb.pair_integral_from_fft(c.L, c.grid, v, F, F)
    return K / nk


@pytest.mark.parametrize("kind", ["k211", "k211-low", "k311", "gamma"])
def test_robust_residual_identity(kind):
    c, C, psi, phi, pts = _setup(kind)
    o = thc.thc_oo_k_robust(c.L, c.grid, c.kmesh, psi, phi, pts)
    ao = np.stack([phi[n][:, pts] for n in range(c.N_k)])
    xi = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao, keep_intermediates=("xi",))["xi"]
    Kd = direct.exchange_matrix(c.L, c.grid, c.kmesh, psi, phi)
    Kdd = _residual_exchange(c, psi, phi, pts, xi)
    scale = np.abs(Kd).max()
    err = np.abs(Kd - o["K"] - Kdd).max() / scale
    print(f"{kind}: rank {o['rank'].tolist()} |K_d - K_rob - K[dd]| {err:.2e} "
          f"|K_d - K_fit| {np.abs(Kd - o['K_fit']).max() / scale:.2e} "
          f"|K_d - K_rob| {np.abs(Kd - o['K']).max() / scale:.2e}")
    assert err <= 1e-11
    # the residual term is not negligible: the identity tests the one-sided term
    assert np.abs(Kdd).max() >= 1e-6 * scale
    # energies: robust = fitted = energy of K_rob; K_rob Hermitian
    assert abs(o["Ex_rob"] - o["Ex"]) <= 1e-12 * abs(o["Ex"])
    assert abs(direct.energy_from_K(o["K"], C) - o["Ex"]) <= 1e-10 * abs(o["Ex"])
    for n in range(c.N_k):
        assert np.abs(o["K"][n] - o["K"][n].conj().T).max() <= 1e-12 * scale
    if kind != "k211":
        assert np.abs(Kd - o["K"]).max() < np.abs(Kd - o["K_fit"]).max()


def test_robust_occupied_rows_exact_at_full_pair_rank():
    c, C, psi, phi, pts = _setup("k211")
    o = thc.thc_oo_k_robust(c.L, c.grid, c.kmesh, psi, phi, pts)
    assert np.all(o["rank"] == c.N_k * c.n_occ ** 2)
    Kd = direct.exchange_matrix(c.L, c.grid, c.kmesh, psi, phi)
    rows = lambda K: np.stack([C[n].conj().T @ K[n] for n in range(c.N_k)])  # noqa: E731
    ref = rows(Kd)
    e_rob = np.abs(rows(o["K"]) - ref).max() / np.abs(ref).max()
    e_fit = np.abs(rows(o["K_fit"]) - ref).max() / np.abs(ref).max()
    print(f"occupied rows: robust {e_rob:.2e}, plain fit {e_fit:.2e}")
    assert e_rob <= 1e-9
    assert e_fit >= 1e-4
