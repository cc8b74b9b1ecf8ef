"""Pins of the gradient oracle (thc.thc_oo_k_gradient: the derivative of the fitted
exchange energy in the AO density matrices, whose occupied-virtual block is the
orbital gradient of Eq. 19) against facts other than itself:

* central finite differences of the oracle's fitted energy E(C + eps dC) along
  random complex directions of the orbital coefficients (so every AO entry,
  occupied-virtual included, is exercised), at two step sizes whose error
  ratio shows the second-order convergence of the difference quotient;
* Euler's identity for the energy, homogeneous of degree two in the density:
  -(1/N_k) sum_n Tr(Kgrad^n D^n) = E_x;
* the gradient is not the fixed-V exchange matrix K: along the same directions
  K's directional derivative differs (the fit's own dependence on the
  orbitals matters), and the test requires the two to differ.
"""

import numpy as np
import pytest

import synth
from oracle import select, thc


def _cell(kind):
    if kind == "k211":
        return synth.make_random_cell((5.0, 5.5, 6.0), 2, (10, 10, 12), (2, 1, 1), 2, 14, (7, 7, 7))
    if kind == "k211-low":  # N_ISDF 12 below the pair rank N_k n_occ^2 = 18: an approximate fit
        return synth.make_random_cell((5.0, 5.5, 6.0), 2, (10, 10, 12), (2, 1, 1), 3, 12, (7, 7, 6))
    if kind == "k311":
        return synth.make_random_cell((6.0, 5.0, 5.0), 2, (12, 10, 10), (3, 1, 1), 2, 16, (7, 7, 8))
    return synth.make_random_cell((6.0, 6.0, 6.0), 3, (12, 12, 12), (1, 1, 1), 3, 12, (7, 7, 9))


def _directional(Kg, C, dC, nk):
    return sum(-(2.0 / nk) * np.trace(Kg[n] @ (dC[n] @ C[n].conj().T + C[n] @ dC[n].conj().T)).real
               for n in range(nk))


@pytest.mark.parametrize("kind", ["k211", "k211-low", "k311", "gamma"])
def test_gradient_matches_finite_differences(kind):
    c = _cell(kind)
    C = synth.orbital_coeffs(c)
    psi = synth.orbitals_on_grid(c, C)
    phi = np.stack([synth.ao_on_grid(c, n) for n in range(c.N_k)])
    pts, _ = select.select_points(psi, c.n_isdf)
    g = thc.thc_oo_k_gradient(c.L, c.grid, c.kmesh, psi, phi, pts)
    ao = np.stack([phi[n][:, pts] for n in range(c.N_k)])
    rng = np.random.default_rng([len(kind), c.N_k, 5])
    dC = [rng.standard_normal(Cn.shape) + 1j * rng.standard_normal(Cn.shape) for Cn in C]

    def energy(eps):
        Cp = [Cn + eps * d for Cn, d in zip(C, dC)]
        return thc.thc_oo_k(c.L, c.grid, c.kmesh, synth.orbitals_on_grid(c, Cp), pts, ao)["Ex"]

    an = _directional(g["Kgrad"], C, dC, c.N_k)
    errs = []
    for eps in (1e-3, 1e-4):
        fd = (energy(eps) - energy(-eps)) / (2 * eps)
        errs.append(abs(fd - an) / abs(fd))
    print(f"{kind}: rank {g['rank']}, analytic {an:.10f}, rel errors {errs[0]:.2e}, {errs[1]:.2e}")
    assert errs[1] <= 5e-6
    assert errs[1] <= errs[0] / 30          # O(eps^2): a factor 100 for a factor 10 in eps
    fixed_v = _directional(g["K"], C, dC, c.N_k)
    assert abs(fixed_v - an) > 1e-3 * abs(an)
    # Euler (degree two) and Hermiticity
    D = [Cn @ Cn.conj().T for Cn in C]
    e_euler = -(1.0 / c.N_k) * sum(np.trace(g["Kgrad"][n] @ D[n]).real for n in range(c.N_k))
    assert abs(e_euler - g["Ex"]) <= 1e-10 * abs(g["Ex"])
    for n in range(c.N_k):
        assert np.abs(g["Kgrad"][n] - g["Kgrad"][n].conj().T).max() <= 1e-12 * np.abs(g["Kgrad"]).max()


@pytest.mark.parametrize("m", [0, 1])
def test_potentials_of_a_plane_wave(m):
    """phased_potentials on single Fourier modes: xi_P(r) = e^{2 pi i g_P.c / n}
    (grid index c) has F_P = N_g at g_P alone, so its potential is
    Phi_P = (Omega/N_g) v^m(g_P) e^{2 pi i g_P.c / n}, and the returned
    Pw_P(r) = e^{i q_m.(r_P - r)} conj Phi_P(r) follows in closed form (the
    normalisation, the sign of the exponent, the conjugate and the phase)."""
    from oracle import coulomb

    L, grid, kmesh = (5.0, 6.0, 7.0), (8, 9, 10), (2, 1, 1)
    ng = int(np.prod(grid))
    c = np.stack(np.unravel_index(np.arange(ng), grid), axis=-1)
    modes = np.array([[1, 2, 3], [0, 0, 1], [7, 8, 9], [3, 0, 5]])
    pts = np.array([0, 17, 250, 719])
    arg = 2 * np.pi * (modes[:, None, :] * c[None, :, :] / np.array(grid)).sum(-1)
    xi = np.zeros((2, len(pts), ng), dtype=np.complex128)
    xi[m] = np.exp(1j * arg)
    Pw = thc.phased_potentials(L, grid, kmesh, xi, pts)
    v = coulomb.kernel(L, grid, kmesh, m)
    q = coulomb.qvec(L, kmesh, m)
    r = coulomb.positions(L, grid)
    omega = float(np.prod(L))
    for P, (g, p) in enumerate(zip(modes, pts)):
        phi = (omega / ng) * v[tuple(g)] * np.exp(1j * arg[P])
        ref = np.exp(1j * ((r[p] - r) @ q)) * phi.conj()
        assert np.abs(Pw[m, P] - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)
    assert np.abs(Pw[1 - m]).max() == 0.0


@pytest.mark.parametrize("kmesh", [(3, 1, 1), (3, 2, 1)])
def test_potentials_of_conjugate_transfers_are_conjugate(kmesh):
    """Pw^{-m} = conj Pw^m for every transfer m and its partner -m (the identity
    that lets a build fit one transfer of each conjugate pair), although the
    fitted functions themselves differ by a phase (xi^{-m} != conj xi^m when
    q_{-m} is q_m's partner shifted by a reciprocal lattice vector)."""
    from oracle import coulomb

    c = synth.make_random_cell((6.0, 5.0, 5.0), 2, (12, 10, 10), kmesh, 2, 16, (7, 7, 8))
    psi = synth.orbitals_on_grid(c, synth.orbital_coeffs(c))
    pts, _ = select.select_points(psi, c.n_isdf)
    ao = np.stack([synth.ao_at_points(c, n, pts) for n in range(c.N_k)])
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao, keep_intermediates=("xi",))
    Pw = thc.phased_potentials(c.L, c.grid, c.kmesh, o["xi"], pts)
    differs = False
    for m in range(c.N_k):
        mb = coulomb.transfer_index(c.kmesh, m, 0)  # the transfer -m
        scale = np.abs(Pw[m]).max()
        assert np.abs(Pw[mb] - Pw[m].conj()).max() <= 1e-10 * scale
        if mb != m:
            differs |= np.abs(o["xi"][mb] - o["xi"][m].conj()).max() > 1e-3 * np.abs(o["xi"][m]).max()
    assert differs
