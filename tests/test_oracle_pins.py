"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test ties one oracle function to something other than itself: a closed
form, a brute-force evaluation, an exact identity of the method or a textbook
library routine. Together they are chosen so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails at least one.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import coulomb, direct, select, thc


# ---------------------------------------------------------------------------
# small cells
# ---------------------------------------------------------------------------

def _orbitals(cell, tr=False):
    C = synth.orbital_coeffs(cell, tr_symmetric=tr)
    return C, synth.orbitals_on_grid(cell, C)


def _ao_pts(cell, pts):
    return np.stack([synth.ao_at_points(cell, n, pts) for n in range(cell.N_k)])


def _phi(cell):
    return np.stack([synth.ao_on_grid(cell, n) for n in range(cell.N_k)])


@pytest.fixture(scope="module")
def kcell():
    """2x2x2 mesh, 2 occupied orbitals, 12^3 grid: pair space of dimension 32 per q."""
    c = synth.make_random_cell((6.0, 6.5, 7.0), 2, (12, 12, 12), (2, 2, 2), 2, 40, (1, 2, 3))
    C, psi = _orbitals(c)
    return c, C, psi


@pytest.fixture(scope="module")
def gcell():
    """The Gamma-point workload shape: cubic 8 bohr, 4 atoms, 24^3 grid, n_occ 4, N_ISDF 64."""
    c = synth.make_config(1)
    C, psi = _orbitals(c)
    return c, C, psi


# ---------------------------------------------------------------------------
# pin 1: analytic Gaussian lattice sum for the FFT-Poisson step
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kmesh,m", [((1, 1, 1), 0), ((2, 3, 1), 4), ((2, 3, 1), 3)])
def test_pair_integral_matches_gaussian_lattice_sum(kmesh, m):
    L = np.array([8.0, 8.0, 8.0])
    grid = (48, 48, 48)
    p = 1.6
    c = np.array([1.3, 2.9, 5.1])
    q = coulomb.qvec(L, kmesh, m)
    r = coulomb.positions(L, grid)
    # Bloch-summed Gaussian rho(r) = sum_R e^{i q.R} exp(-p |r - c - R|^2)
    rho = np.zeros(len(r), dtype=np.complex128)
    for R in np.ndindex(3, 3, 3):
        Rv = (np.array(R) - 1) * L
        d = r - c - Rv
        rho += np.exp(1j * q @ Rv) * np.exp(-p * np.sum(d * d, axis=1))
    f = np.exp(-1j * (r @ q)) * rho
    F = np.fft.fftn(f.reshape(grid))[None]
    v = coulomb.kernel(L, grid, kmesh, m)
    J_fft = coulomb.pair_integral_from_fft(L, grid, v, F)[0]
    # closed form: (4 pi/Omega) sum_{K = G + q != 0} (pi/p)^3 exp(-|K|^2/(2p)) / |K|^2
    omega = np.prod(L)
    nmax = 12
    ax = np.arange(-nmax, nmax + 1)
    Gx, Gy, Gz = np.meshgrid(ax, ax, ax, indexing="ij")
    K = np.stack([Gx, Gy, Gz], -1) * (2 * np.pi / L) + q
    K2 = np.sum(K * K, -1)
    mask = K2 > 0
    J_ref = (4 * np.pi / omega) * np.sum((np.pi / p) ** 3 * np.exp(-K2[mask] / (2 * p)) / K2[mask])
    assert abs(J_fft - J_ref) <= 1e-10 * abs(J_ref)


def test_kernel_box_rule_against_explicit_representatives():
    """v^m(g) = 4 pi/|G+q|^2 with G+q the supercell-box representative, K=0 dropped."""
    L = np.array([5.0, 6.0, 7.0])
    grid, kmesh = (6, 5, 4), (2, 3, 1)
    for m in range(6):
        v = coulomb.kernel(L, grid, kmesh, m)
        mi = np.unravel_index(m, kmesh)
        for g in [(0, 0, 0), (3, 2, 1), (5, 4, 3), (1, 0, 2)]:
            # all aliases G = g + t n, keep the one whose supercell index is in the box
            best = None
            for t in np.ndindex(3, 3, 3):
                kap = [kmesh[i] * (g[i] + (t[i] - 1) * grid[i]) + mi[i] for i in range(3)]
                Ls = [kmesh[i] * grid[i] for i in range(3)]
                if all(-(Ls[i] // 2) <= kap[i] < Ls[i] - Ls[i] // 2 for i in range(3)):
                    best = np.array([kap[i] * 2 * np.pi / (kmesh[i] * L[i]) for i in range(3)])
            k2 = best @ best
            expect = 0.0 if k2 == 0 else 4 * np.pi / k2
            assert v[g] == pytest.approx(expect, rel=1e-14, abs=0)


# ---------------------------------------------------------------------------
# pin 2: brute-force real-space double sum (no FFT anywhere)
# ---------------------------------------------------------------------------

def test_exchange_pair_integral_brute_force_real_space():
    c = synth.make_random_cell((5.0, 5.5, 6.0), 2, (8, 8, 8), (2, 1, 1), 2, 8, (7, 7, 7))
    C, psi = _orbitals(c)
    L, grid, kmesh = c.L, c.grid, c.kmesh
    r = coulomb.positions(L, grid)
    omega = c.omega
    dV = c.dV
    # band-limited periodic kernel for transfer m, summed explicitly over K
    for (n, n2, i, j) in [(0, 1, 0, 1), (1, 0, 1, 1), (0, 0, 0, 1)]:
        m = coulomb.transfer_index(kmesh, n, n2)
        mi = np.unravel_index(m, kmesh)
        Ks = []
        for g in np.ndindex(*grid):
            kap = [coulomb._wrap(kmesh[a] * g[a] + mi[a], kmesh[a] * grid[a]) for a in range(3)]
            Ks.append([kap[a] * 2 * np.pi / (kmesh[a] * L[a]) for a in range(3)])
        Ks = np.array(Ks)
        K2 = np.sum(Ks * Ks, 1)
        w = np.where(K2 > 0, 4 * np.pi / np.where(K2 > 0, K2, 1.0), 0.0)
        f = psi[n, i].conj() * psi[n2, j]  # full Bloch product, momentum q
        # sum_{r,r'} conj f(r) v(r - r') f(r') with v(x) = (1/Omega) sum_K w_K e^{iK.x}
        E = np.exp(1j * (r @ Ks.T))  # (N_g, N_K)
        a = E.conj().T @ f  # sum_r f(r) e^{-iK.r}
        J_bf = dV * dV / omega * np.sum(w * np.abs(a) ** 2)
        # the oracle's pair integral of the cell-periodic e^{-iq.r} f
        q = coulomb.qvec(L, kmesh, m)
        F = np.fft.fftn((np.exp(-1j * (r @ q)) * f).reshape(grid))[None]
        J = coulomb.pair_integral_from_fft(L, grid, coulomb.kernel(L, grid, kmesh, m), F)[0]
        assert abs(J - J_bf) <= 1e-12 * abs(J_bf)


# ---------------------------------------------------------------------------
# pin 3: supercell identity for all k/q bookkeeping
# ---------------------------------------------------------------------------

def _supercell_exchange(cell, psi):
    km, g = cell.kmesh, cell.grid
    sg = tuple(km[i] * g[i] for i in range(3))
    SL = np.array([km[i] * cell.L[i] for i in range(3)])
    orbs = []
    for n in range(cell.N_k):
        k = cell.kvec(n)
        for i in range(cell.n_occ):
            f = psi[n, i].reshape(g)
            big = np.zeros(sg, dtype=np.complex128)
            for t in np.ndindex(*km):
                R = np.array([t[a] * cell.L[a] for a in range(3)])
                sl = tuple(slice(t[a] * g[a], (t[a] + 1) * g[a]) for a in range(3))
                big[sl] = np.exp(1j * (k @ R)) * f
            orbs.append(big / np.sqrt(cell.N_k))
    Ks = [np.fft.fftfreq(sg[a], d=1.0 / sg[a]) * 2 * np.pi / SL[a] for a in range(3)]
    K2 = Ks[0][:, None, None] ** 2 + Ks[1][None, :, None] ** 2 + Ks[2][None, None, :] ** 2
    v = np.where(K2 > 0, 4 * np.pi / np.where(K2 > 0, K2, 1.0), 0.0)
    om, ng = np.prod(SL), np.prod(sg)
    E = 0.0
    for a in orbs:
        for b in orbs:
            E += om / ng ** 2 * np.sum(v * np.abs(np.fft.fftn(a.conj() * b)) ** 2)
    return -E


def test_supercell_identity(kcell):
    c, C, psi = kcell
    E_k = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    E_s = _supercell_exchange(c, psi)
    assert abs(E_k - E_s / c.N_k) <= 1e-12 * abs(E_k)


def test_supercell_identity_odd_mesh():
    c = synth.make_random_cell((5.0, 6.0, 5.5), 2, (8, 10, 9), (3, 2, 1), 2, 20, (4, 4, 4))
    C, psi = _orbitals(c)
    E_k = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    E_s = _supercell_exchange(c, psi)
    assert abs(E_k - E_s / c.N_k) <= 1e-12 * abs(E_k)


# ---------------------------------------------------------------------------
# O1 internal consistency: energy from pairs = energy from AO-basis K
# ---------------------------------------------------------------------------

def test_direct_energy_from_K(kcell):
    c, C, psi = kcell
    E = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    K = direct.exchange_matrix(c.L, c.grid, c.kmesh, psi, _phi(c))
    assert abs(direct.energy_from_K(K, C) - E) <= 1e-12 * abs(E)
    for n in range(c.N_k):
        assert np.abs(K[n] - K[n].conj().T).max() <= 1e-13 * np.abs(K[n]).max()
        assert np.linalg.eigvalsh(K[n]).min() >= -1e-12 * np.abs(K[n]).max()
    assert E < 0


# ---------------------------------------------------------------------------
# pin 4: full pair rank -> THC-oo-K equals direct exchange (energy and oo block)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["gamma", "kmesh"])
def test_full_pair_rank_reproduces_direct_exchange(which, gcell, kcell):
    c, C, psi = gcell if which == "gamma" else kcell
    pts, npiv = select.select_points(psi, c.n_isdf)
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, _ao_pts(c, pts))
    assert np.all(o["rank"] == c.N_k * c.n_occ ** 2)
    E1 = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    assert abs(o["Ex"] - E1) <= 1e-10 * abs(E1)
    K1 = direct.exchange_matrix(c.L, c.grid, c.kmesh, psi, _phi(c))
    for n in range(c.N_k):
        oo2 = C[n].conj().T @ o["K"][n] @ C[n]
        oo1 = C[n].conj().T @ K1[n] @ C[n]
        assert np.abs(oo2 - oo1).max() <= 1e-9 * np.abs(oo1).max()


# ---------------------------------------------------------------------------
# pin 5: xi = identity at N_I = N_g reproduces the AO-basis K of O1
# ---------------------------------------------------------------------------

def test_identity_interpolation_reproduces_ao_exchange():
    c = synth.make_random_cell((4.0, 4.5, 5.0), 2, (6, 6, 8), (2, 1, 1), 2, 288, (9, 9, 9))
    C, psi = _orbitals(c)
    pts = np.arange(c.N_g)
    ao = _ao_pts(c, pts)
    Psi, X, G = thc.gather(psi, pts, ao)
    xi = np.eye(c.N_g, dtype=np.complex128)
    Vb = np.stack([thc.bloch_gauge(c.L, c.grid, c.kmesh, m, pts,
                                   thc.coulomb_matrix(c.L, c.grid, c.kmesh, m, xi))
                   for m in range(c.N_k)])
    Y, K, Ex = thc.contract(c.kmesh, G, X, Vb)
    K1 = direct.exchange_matrix(c.L, c.grid, c.kmesh, psi, _phi(c))
    assert np.abs(K - K1).max() <= 1e-12 * np.abs(K1).max()
    E1 = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    assert abs(Ex - E1) <= 1e-12 * abs(E1)


# ---------------------------------------------------------------------------
# pin 6 and 7: energy identities and invariants below full rank
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def lowrank():
    c = synth.make_random_cell((6.0, 6.5, 7.0), 2, (12, 12, 12), (2, 2, 2), 3, 30, (5, 6, 7))
    C, psi = _orbitals(c)
    pts, _ = select.select_points(psi, c.n_isdf)
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, _ao_pts(c, pts))
    return c, C, psi, pts, o


def test_energy_identities(lowrank):
    c, C, psi, pts, o = lowrank
    assert np.all(o["rank"] == c.n_isdf)
    E_K = direct.energy_from_K(o["K"], C)
    assert abs(o["Ex"] - o["Ex_trVS"]) <= 1e-10 * abs(o["Ex"])
    assert abs(o["Ex"] - E_K) <= 1e-10 * abs(o["Ex"])
    assert o["Ex"] < 0


def _neg(kmesh, m):
    mi = np.unravel_index(m, kmesh)
    return int(np.ravel_multi_index(tuple((-x) % N for x, N in zip(mi, kmesh)), kmesh))


def test_invariants(lowrank):
    c, C, psi, pts, o = lowrank
    rP = coulomb.positions(c.L, c.grid, pts)
    for m in range(c.N_k):
        S, V, Vb = o["S"][m], o["V"][m], o["Vb"][m]
        for A in (S, V):
            assert np.abs(A - A.conj().T).max() <= 1e-12 * np.abs(A).max()
            assert np.linalg.eigvalsh(0.5 * (A + A.conj().T)).min() >= -1e-10 * np.abs(A).max()
        mm = _neg(c.kmesh, m)
        # Vb^{-m} = conj Vb^m (relative, scaled by the conditioning of S)
        cond = np.linalg.cond(o["S"][m])
        assert np.abs(o["Vb"][mm] - Vb.conj()).max() <= 1e-15 * cond * np.abs(Vb).max() * 10
        # gauge-free metric T^m = e^{-iq.(r_P - r_Q)} S^m satisfies T^{-m} = conj T^m
        q, qn = coulomb.qvec(c.L, c.kmesh, m), coulomb.qvec(c.L, c.kmesh, mm)
        T = S * np.exp(-1j * np.subtract.outer(rP @ q, rP @ q))
        Tn = o["S"][mm] * np.exp(-1j * np.subtract.outer(rP @ qn, rP @ qn))
        assert np.abs(Tn - T.conj()).max() <= 1e-12 * np.abs(T).max()
    for n in range(c.N_k):
        K = o["K"][n]
        assert np.abs(K - K.conj().T).max() <= 1e-12 * np.abs(K).max()


def test_time_reversal_symmetry():
    c = synth.make_random_cell((6.0, 6.5, 7.0), 2, (12, 12, 12), (2, 2, 1), 2, 24, (8, 8, 8))
    C, psi = _orbitals(c, tr=True)
    pts, _ = select.select_points(psi, c.n_isdf)
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, _ao_pts(c, pts))
    for n in range(c.N_k):
        nn = _neg(c.kmesh, n)
        assert np.abs(o["K"][nn] - o["K"][n].conj()).max() <= 1e-10 * np.abs(o["K"][n]).max()


# ---------------------------------------------------------------------------
# pin 8: Gamma reduction (Sec. 2.1 restricted to occupied pairs)
# ---------------------------------------------------------------------------

def test_gamma_reduction(gcell):
    c, C, psi = gcell
    pts, _ = select.select_points(psi, 12)
    ao = _ao_pts(c, pts)
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, ao, keep_intermediates=("Z",))
    Psi = psi[0][:, pts].T
    G = Psi @ Psi.conj().T
    Gam = Psi @ psi[0].conj()
    assert np.abs(o["S"][0] - np.abs(G) ** 2).max() <= 1e-13 * np.abs(G).max() ** 2
    assert np.abs(o["Z"][0] - np.abs(Gam) ** 2).max() <= 1e-13 * np.abs(Gam).max() ** 2
    X = ao[0].conj()
    K = X @ (o["V"][0] * G) @ X.conj().T
    assert np.abs(o["K"][0] - K).max() <= 1e-13 * np.abs(K).max()


# ---------------------------------------------------------------------------
# pin 9: systematic improvability in N_ISDF (loose)
# ---------------------------------------------------------------------------

def test_error_decreases_with_more_points(kcell):
    c, C, psi = kcell
    E1 = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    pts_all, _ = select.select_points(psi, 32)
    errs = []
    for nI in (6, 12, 20, 32):
        pts = pts_all[:nI]
        o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, _ao_pts(c, pts))
        errs.append(abs(o["Ex"] - E1))
    assert errs[-1] <= 1e-10 * abs(E1)
    assert errs[0] > errs[-1] and errs[1] > errs[-1]
    assert min(errs[:2]) > 10 * errs[2] or errs[2] < 1e-3 * abs(E1)


def test_fitted_exchange_is_a_variational_bound(kcell):
    """Per transfer q the fitted pair functions are the pair functions projected
    onto the row space of their values at the points, and the Coulomb kernel is
    positive, so the fitted exchange recovers at most the exact exchange
    (E_fit >= E_exact, both negative) and more of it for a larger point set."""
    c, C, psi = kcell
    E1 = direct.exchange_energy(c.L, c.grid, c.kmesh, psi)
    order = np.random.default_rng(12).permutation(c.N_g)
    prev = 0.0
    for nI in (4, 9, 17, 30):
        pts = order[:nI]
        Ex = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, _ao_pts(c, pts))["Ex"]
        assert Ex >= E1 - 1e-10 * abs(E1)
        assert Ex <= prev + 1e-10 * abs(E1)
        prev = Ex
    assert prev < 0.5 * E1  # 30 of 32 pair dimensions recover most of it


# ---------------------------------------------------------------------------
# the fit itself: literal least squares, and the k-sum forms used on the GPU
# ---------------------------------------------------------------------------

def test_fit_is_the_least_squares_solution(lowrank):
    """xi from the normal equations equals numpy's lstsq of the pair matrix."""
    c, C, psi, pts, _ = lowrank
    o = thc.thc_oo_k(c.L, c.grid, c.kmesh, psi, pts, _ao_pts(c, pts), keep_intermediates=("xi",))
    Psi = np.stack([psi[n][:, pts].T for n in range(c.N_k)])
    r = coulomb.positions(c.L, c.grid)
    cols = np.arange(0, c.N_g, 97)
    for m in (0, 5):
        q = coulomb.qvec(c.L, c.kmesh, m)
        phP = np.exp(-1j * (coulomb.positions(c.L, c.grid, pts) @ q))
        B = thc.pair_rows(Psi, c.kmesh, m, phP)
        # A(r): the same pair products on the grid columns
        A = []
        for n in range(c.N_k):
            n2 = coulomb.add_index(c.kmesh, n, m)
            blk = psi[n][:, cols].conj()[:, None, :] * psi[n2][:, cols][None, :, :]
            A.append(blk.reshape(-1, len(cols)) * np.exp(-1j * (r[cols] @ q))[None, :])
        A = np.concatenate(A)
        xi_ls = np.linalg.lstsq(B, A, rcond=None)[0]
        ref = o["xi"][m][:, cols]
        assert np.abs(xi_ls - ref).max() <= 1e-7 * np.abs(ref).max()


def test_hadamard_and_kdft_forms_equal_the_literal_sums(lowrank):
    c, C, psi, pts, o = lowrank
    rP = coulomb.positions(c.L, c.grid, pts)
    G = o["G"]
    nk = c.N_k
    for m in range(nk):
        q = coulomb.qvec(c.L, c.kmesh, m)
        T = sum(G[n] * G[coulomb.add_index(c.kmesh, n, m)].conj() for n in range(nk))
        S_h = np.exp(1j * np.subtract.outer(rP @ q, rP @ q)) * T
        assert np.abs(S_h - o["S"][m]).max() <= 1e-13 * np.abs(o["S"][m]).max()
    # Wiener-Khinchin: sum_n a_n conj a_{n+m} = (1/N_k) DFT_k(|DFT_k a|^2)_m
    Gk = G.reshape(c.kmesh + G.shape[1:])
    A = np.fft.fftn(Gk, axes=(0, 1, 2))
    corr = np.fft.fftn(np.abs(A) ** 2, axes=(0, 1, 2)).reshape(G.shape) / nk
    for m in range(nk):
        T = sum(G[n] * G[coulomb.add_index(c.kmesh, n, m)].conj() for n in range(nk))
        assert np.abs(corr[m] - T).max() <= 1e-13 * np.abs(T).max()


def test_cholesky_drop_matches_lapack_and_drops_duplicates():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((40, 12)) + 1j * rng.standard_normal((40, 12))
    S = B.conj().T @ B
    L, keep = thc.cholesky_drop(S)
    assert keep.all()
    assert np.abs(L - np.linalg.cholesky(S)).max() <= 1e-12 * np.abs(L).max()
    # duplicate column 3 at position 7: that point is dropped, solution = lstsq on the rest
    B2 = B.copy()
    B2[:, 7] = B2[:, 3]
    S2 = B2.conj().T @ B2
    L2, keep2 = thc.cholesky_drop(S2)
    assert not keep2[7] and keep2.sum() == 11
    Z = B2.conj().T @ (rng.standard_normal((40, 5)) + 0j)
    xi = thc.solve_drop(L2, keep2, Z)
    R = np.flatnonzero(keep2)
    ref = np.linalg.solve(S2[np.ix_(R, R)], Z[R])
    assert np.abs(xi[R] - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.all(xi[7] == 0)


# ---------------------------------------------------------------------------
# point selection = QR with column pivoting of the pair matrix
# ---------------------------------------------------------------------------

def test_selection_matches_lapack_qrcp(kcell):
    """Pivoted Cholesky of |Gamma|^2 picks LAPACK's QRCP columns of the pair matrix.

    Its stopping rule (Gram pivot below 1e-12 of the first) is the QR rule
    |R_pp| < 1e-6 |R_00|.
    """
    c, C, psi = kcell
    nk, no = c.N_k, c.n_occ
    flat = psi.reshape(nk * no, -1)
    A = (flat.conj()[:, None, :] * flat[None, :, :]).reshape((nk * no) ** 2, -1)
    _, R, piv = sla.qr(A, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    n_qr = int(np.sum(d > 1e-6 * d[0]))
    pts, npiv = select.select_points(psi, (nk * no) ** 2 + 10)
    assert npiv == n_qr
    agree = 0
    while agree < npiv and pts[agree] == piv[agree]:
        agree += 1
    assert agree == npiv


def test_selection_fill_by_density(gcell):
    c, C, psi = gcell
    pts, npiv = select.select_points(psi, c.n_isdf)
    assert npiv == c.n_occ ** 2
    assert len(set(pts.tolist())) == c.n_isdf
    dens = np.sum(np.abs(psi.reshape(-1, c.N_g)) ** 2, axis=0)
    rest = pts[npiv:]
    assert np.all(np.diff(dens[rest]) <= 0)
    chosen = set(pts.tolist())
    unchosen_max = max(dens[r] for r in range(c.N_g) if r not in chosen)
    assert dens[rest].min() >= unchosen_max
