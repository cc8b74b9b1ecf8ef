"""O2: THC-oo-K exchange build with one occupied-pair ISDF fit per transfer q (oracle).

TEST INFRASTRUCTURE ONLY (see package docstring).

Follows Sec. 2.3 (Eqs. 16-18) and the per-iteration body of Algorithm 2
(compute xi, FFT xi, M^q, the k-convolved intermediate, K_ij), with the
per-q fit in the full-Bloch gauge. Notation (orbitals psi_in(r) of k-point n
on the grid, interpolation points r_P, transfer m with q_m):

1. Gather: Psi^n_{Pi} = psi_in(r_P), X^n_{mu P} = conj phi_mu^n(r_P),
   G^n = Psi^n Psi^n^H  (G^n_PQ = sum_i psi_in(r_P) conj psi_in(r_Q)).
2. Fit metric of the least-squares problem (Eqs. 7-8 and 13 restricted to
   occupied pairs): the pair matrix B_m has one row per (n, i, j),
   B_m[(n,i,j), P] = e^{-i q_m.r_P} conj psi_in(r_P) psi_{j,n+m}(r_P),
   and S^m = B_m^H B_m (formed literally).
3. Right-hand side B_m^H A_m(r) (Eq. 7/13), written through
   Gamma^n(P, r) = sum_i psi_in(r_P) conj psi_in(r):
   Z^m_P(r) = e^{i q_m.(r_P - r)} sum_n Gamma^n(P, r) conj Gamma^{n+m}(P, r)
   with a direct sum over n.
4. Solve S^m xi^m(r) = Z^m(r) by an FP64 Cholesky factorisation in the given
   point order; a point whose Schur-complement pivot falls below
   rel_tol * max_P S_PP is dropped (xi_P = 0).
5. F^m_P = FFT(xi^m_P); V^m_PQ = (Omega/N_g^2) sum_g v^m(g) F_P conj F_Q
   (M^q of Eq. 15 by GPW).
6. Bloch-gauge Coulomb matrix Vb^m_PQ = e^{-i q_m.(r_P - r_Q)} V^m_PQ.
7. k-convolution (Algorithm 2, X^k line): Y^n = sum_{n'} Vb^{m(n,n')} o G^{n'}
   by a direct sum.
8. K^n = (1/N_k) X^n Y^n X^n^H  (Eq. 14 restricted to the oo fit).
9. E_x = -(1/N_k^2) sum_n sum_PQ Y^n_PQ conj G^n_PQ (Eq. 18, closed shell per
   cell); also -(1/N_k^2) sum_m Tr(V^m S^m).
"""

from __future__ import annotations

import time

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

from . import coulomb
from ._threads import WORKERS


def cholesky_drop(S: np.ndarray, rel_tol: float = 1e-12):
    """Cholesky of Hermitian PSD S in the given order, dropping tiny pivots.

    Returns (L, keep): L is lower triangular with zero columns for dropped
    points, keep[p] says whether point p was retained. The retained block
    satisfies S[R][:, R] = L[R][:, R] L[R][:, R]^H.
    """
    n = S.shape[0]
    tol = rel_tol * float(np.max(S.diagonal().real))
    L = np.zeros((n, n), dtype=np.complex128)
    keep = np.zeros(n, dtype=bool)
    for p in range(n):
        col = S[p:, p] - L[p:, :p] @ L[p, :p].conj()
        d = float(col[0].real)
        if not (np.isfinite(d) and d > 0.0 and d >= tol):
            continue
        keep[p] = True
        s = np.sqrt(d)
        L[p, p] = s
        L[p + 1:, p] = col[1:] / s
    return L, keep


def solve_drop(L: np.ndarray, keep: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """xi = S_RR^{-1} Z_R on the retained points, zero on dropped points."""
    R = np.flatnonzero(keep)
    Lr = L[np.ix_(R, R)]
    y = sla.solve_triangular(Lr, Z[R], lower=True, check_finite=False)
    x = sla.solve_triangular(Lr, y, lower=True, trans="C", check_finite=False)
    xi = np.zeros_like(Z)
    xi[R] = x
    return xi


def gather(psi: np.ndarray, pts: np.ndarray, ao_pts: np.ndarray):
    """Psi^n (N_I, n_occ), X^n (N, N_I) and G^n (N_I, N_I) for every k."""
    nk = psi.shape[0]
    Psi = np.stack([psi[n][:, pts].T for n in range(nk)])
    X = ao_pts.conj()
    G = np.einsum("npi,nqi->npq", Psi, Psi.conj())
    return Psi, X, G


def pair_rows(psi_pts: np.ndarray, kmesh, m: int, phase_P: np.ndarray) -> np.ndarray:
    """B_m: rows (n, i, j) -> e^{-i q_m.r_P} conj psi_in(r_P) psi_{j,n+m}(r_P)."""
    nk, nI, no = psi_pts.shape
    rows = []
    for n in range(nk):
        n2 = coulomb.add_index(kmesh, n, m)
        blk = psi_pts[n].conj().T[:, None, :] * psi_pts[n2].T[None, :, :]
        rows.append(blk.reshape(no * no, nI) * phase_P[None, :])
    return np.concatenate(rows, axis=0)


def _gamma(Psi_n, psi_n_chunk):
    return Psi_n @ psi_n_chunk.conj()


def coulomb_matrix(L, grid, kmesh, m: int, xi: np.ndarray) -> np.ndarray:
    """Step 5: V^m_PQ = (Omega/N_g^2) sum_g v^m(g) F_P(g) conj F_Q(g), F_P = FFT(xi_P)."""
    grid = tuple(int(x) for x in grid)
    nI, ng = xi.shape
    omega = float(np.prod(L))
    F = sfft.fftn(xi.reshape((nI,) + grid), axes=(1, 2, 3), workers=WORKERS).reshape(nI, ng)
    v = coulomb.kernel(L, grid, kmesh, m).reshape(-1)
    return (omega / ng ** 2) * ((F * v[None, :]) @ F.conj().T)


def bloch_gauge(L, grid, kmesh, m: int, pts, V: np.ndarray) -> np.ndarray:
    """Step 6: Vb^m_PQ = e^{-i q_m.(r_P - r_Q)} V^m_PQ."""
    q = coulomb.qvec(L, kmesh, m)
    ph = np.exp(-1j * (coulomb.positions(L, grid, pts) @ q))
    return V * (ph[:, None] * ph.conj()[None, :])


def contract(kmesh, G: np.ndarray, X: np.ndarray, Vb: np.ndarray):
    """Steps 7-9: Y^n, K^n and E_x from Vb^m (N_k, N_I, N_I), G^n and X^n."""
    nk = G.shape[0]
    Y = np.zeros_like(G)
    for n in range(nk):
        for n2 in range(nk):
            Y[n] += Vb[coulomb.transfer_index(kmesh, n, n2)] * G[n2]
    K = np.stack([X[n] @ Y[n] @ X[n].conj().T for n in range(nk)]) / nk
    Ex = -float(np.sum(Y * G.conj()).real) / nk ** 2
    return Y, K, Ex


def thc_oo_k(L, grid, kmesh, psi, pts, ao_pts, rel_tol=1e-12, keep_intermediates=(),
             gamma_store_bytes=24 << 30, chunk=1 << 15, m_subset=None):
    """Run O2. Returns a dict with K (N_k, N, N), Ex, Ex_trVS, V, Vb, S, G, Y, rank.

    ``keep_intermediates`` may include "Z" and "xi" to also return those
    (N_k, N_I, N_g) arrays (small cells only). ``m_subset`` restricts steps
    2-6 to the listed transfers (timing samples only: K and E_x are then
    incomplete). ``out["seconds"]`` holds wall-clock seconds per section.
    """
    t0 = time.perf_counter()
    L = np.asarray(L, dtype=np.float64)
    grid = tuple(int(x) for x in grid)
    kmesh = tuple(int(x) for x in kmesh)
    pts = np.asarray(pts, dtype=np.int64)
    nk, no, ng = psi.shape
    nI = len(pts)

    Psi, X, G = gather(psi, pts, ao_pts)
    rP = coulomb.positions(L, grid, pts)

    store = nk * nI * ng * 16 <= gamma_store_bytes
    Gam = None
    if store:
        Gam = np.empty((nk, nI, ng), dtype=np.complex128)
        for n in range(nk):
            Gam[n] = _gamma(Psi[n], psi[n])

    t_gamma = time.perf_counter() - t0
    out = {"G": G, "X": X}
    S_all = np.zeros((nk, nI, nI), dtype=np.complex128)
    V_all = np.zeros((nk, nI, nI), dtype=np.complex128)
    Vb_all = np.zeros((nk, nI, nI), dtype=np.complex128)
    rank = np.zeros(nk, dtype=np.int64)
    keep_sets = []
    kept = {k: np.zeros((nk, nI, ng), dtype=np.complex128) for k in keep_intermediates}

    r_all = coulomb.positions(L, grid)
    t_m = []
    for m in (range(nk) if m_subset is None else m_subset):
        tm0 = time.perf_counter()
        q = coulomb.qvec(L, kmesh, m)
        ph_P = np.exp(-1j * (rP @ q))
        # step 2: fit metric, literally B^H B
        B = pair_rows(Psi, kmesh, m, ph_P)
        S = B.conj().T @ B
        del B
        S_all[m] = S
        Lc, keep = cholesky_drop(S, rel_tol)
        rank[m] = int(keep.sum())
        keep_sets.append(keep)
        # step 3: right-hand side, direct k-sum, chunked over r
        xi = np.empty((nI, ng), dtype=np.complex128)
        for c0 in range(0, ng, chunk):
            c1 = min(ng, c0 + chunk)
            Z = np.zeros((nI, c1 - c0), dtype=np.complex128)
            for n in range(nk):
                n2 = coulomb.add_index(kmesh, n, m)
                ga = Gam[n, :, c0:c1] if store else _gamma(Psi[n], psi[n][:, c0:c1])
                gb = Gam[n2, :, c0:c1] if store else _gamma(Psi[n2], psi[n2][:, c0:c1])
                Z += ga * gb.conj()
            ph_r = np.exp(-1j * (r_all[c0:c1] @ q))
            Z *= ph_P.conj()[:, None] * ph_r[None, :]
            if "Z" in kept:
                kept["Z"][m, :, c0:c1] = Z
            # step 4: least-squares solve on the retained points
            xi[:, c0:c1] = solve_drop(Lc, keep, Z)
        if "xi" in kept:
            kept["xi"][m] = xi
        # steps 5-6: Coulomb matrix, Bloch gauge
        V_all[m] = coulomb_matrix(L, grid, kmesh, m, xi)
        del xi
        Vb_all[m] = bloch_gauge(L, grid, kmesh, m, pts, V_all[m])
        t_m.append(time.perf_counter() - tm0)

    # steps 7-9
    tc0 = time.perf_counter()
    Y, K, Ex = contract(kmesh, G, X, Vb_all)
    t_contract = time.perf_counter() - tc0
    Ex_trVS = -float(sum(np.trace(V_all[m] @ S_all[m]).real for m in range(nk))) / nk ** 2

    out.update(dict(K=K, Ex=Ex, Ex_trVS=Ex_trVS, V=V_all, Vb=Vb_all, S=S_all, Y=Y,
                    rank=rank, keep=np.stack(keep_sets),
                    seconds={"gamma": t_gamma, "per_q": t_m, "contract": t_contract}))
    out.update(kept)
    return out


def thc_oo_k_shared(L, grid, kmesh, psi, pts, ao_pts, rel_tol=1e-12, chunk=1 << 15):
    """THC-oo-K with one fit shared by every transfer (Sec. 2.2, Eq. 13: the
    k-point least-squares fit, here over the occupied pairs of Eq. 16).

    The pairs of all transfers enter one least-squares problem for a single set
    of interpolating vectors xi_P(r) (cell-periodic gauge, as the per-transfer
    fit): with the pair matrices B_m and right-hand sides of steps 2-3, the
    normal equations are (sum_m B_m^H B_m) xi = sum_m B_m^H A_m, i.e.
    S = sum_m S^m and Z = sum_m Z^m. One Cholesky-with-drop of S, one solve,
    then per transfer the Coulomb matrix of the same xi with the kernel v^m
    (steps 5-6) and steps 7-9 unchanged. Returns K, Ex, Ex_trVS (with the
    shared S), V, Vb, S (shared), rank (shared, one value), xi.
    """
    L = np.asarray(L, dtype=np.float64)
    grid = tuple(int(x) for x in grid)
    kmesh = tuple(int(x) for x in kmesh)
    pts = np.asarray(pts, dtype=np.int64)
    nk, no, ng = psi.shape
    nI = len(pts)
    Psi, X, G = gather(psi, pts, ao_pts)
    rP = coulomb.positions(L, grid, pts)
    r_all = coulomb.positions(L, grid)
    S = np.zeros((nI, nI), dtype=np.complex128)
    Z = np.zeros((nI, ng), dtype=np.complex128)
    for m in range(nk):
        q = coulomb.qvec(L, kmesh, m)
        ph_P = np.exp(-1j * (rP @ q))
        B = pair_rows(Psi, kmesh, m, ph_P)
        S += B.conj().T @ B
        del B
        for c0 in range(0, ng, chunk):
            c1 = min(ng, c0 + chunk)
            Zc = np.zeros((nI, c1 - c0), dtype=np.complex128)
            for n in range(nk):
                n2 = coulomb.add_index(kmesh, n, m)
                Zc += _gamma(Psi[n], psi[n][:, c0:c1]) * _gamma(Psi[n2], psi[n2][:, c0:c1]).conj()
            ph_r = np.exp(-1j * (r_all[c0:c1] @ q))
            Z[:, c0:c1] += Zc * (ph_P.conj()[:, None] * ph_r[None, :])
    Lc, keep = cholesky_drop(S, rel_tol)
    xi = solve_drop(Lc, keep, Z)
    V_all = np.stack([coulomb_matrix(L, grid, kmesh, m, xi) for m in range(nk)])
    Vb_all = np.stack([bloch_gauge(L, grid, kmesh, m, pts, V_all[m]) for m in range(nk)])
    Y, K, Ex = contract(kmesh, G, X, Vb_all)
    # the per-transfer metrics S^m weight V^m in the trace form of E_x
    Sm = np.stack([pair_rows(Psi, kmesh, m, np.exp(-1j * (rP @ coulomb.qvec(L, kmesh, m))))
                   for m in range(nk)])
    Ex_trVS = -float(sum(np.trace(V_all[m] @ (Sm[m].conj().T @ Sm[m])).real
                         for m in range(nk))) / nk ** 2
    return dict(K=K, Ex=Ex, Ex_trVS=Ex_trVS, V=V_all, Vb=Vb_all, S=S, G=G, Y=Y,
                rank=int(keep.sum()), keep=keep, xi=xi)


def thc_ao_k(L, grid, kmesh, phi, psi, pts, rel_tol=1e-12):
    """THC-AO-K (Algorithm 1): the ISDF fit of the AO pair products
    conj phi_mu^k(r) phi_nu^{k+q}(r) per transfer (Eqs. 7-9 and 13), done once,
    and the K-build from the occupied density at the points (Eq. 14).

    The fit of the AO pairs is the fit of steps 1-6 with the AO functions phi^k
    (N per k) in place of the occupied orbitals, so it is taken from thc_oo_k
    called on phi: its Bloch-gauge Coulomb matrices are M^q of the AO fit. The
    contraction (steps 7-9) then uses the occupied G^n_PQ = sum_i
    psi_in(r_P) conj psi_in(r_Q) and X^n_{mu P} = conj phi_mu^n(r_P):
    Y^n = sum_m Vb^m o G^{n+m}, K^n = (1/N_k) X^n Y^n X^n^H, E_x from Y and G.
    Returns K, Ex, Vb (of the AO fit), rank (per transfer), the AO-pair metrics S
    and the retained points keep.
    """
    pts = np.asarray(pts, dtype=np.int64)
    nk = phi.shape[0]
    ao_pts = np.stack([phi[n][:, pts] for n in range(nk)])
    fit = thc_oo_k(L, grid, kmesh, phi, pts, ao_pts, rel_tol)
    Psi, X, G = gather(psi, pts, ao_pts)
    Y, K, Ex = contract(tuple(int(x) for x in kmesh), G, X, fit["Vb"])
    return dict(K=K, Ex=Ex, Vb=fit["Vb"], rank=fit["rank"], Y=Y, S=fit["S"], keep=fit["keep"])


def phased_potentials(L, grid, kmesh, xi: np.ndarray, pts) -> np.ndarray:
    """Pw^m(P, r) = e^{i q_m.(r_P - r)} conj Phi^m_P(r) for every transfer, with
    Phi^m_P(r) = (Omega/N_g^2) sum_g e^{i g.r} v^m(g) F^m_P(g) the Coulomb potential
    of the fitted function xi^m_P (F^m_P its FFT; the paper's potentials of the
    interpolating vectors, Sec. 2.3 and the discussion of the robust fit)."""
    grid = tuple(int(x) for x in grid)
    nk, nI, ng = xi.shape
    omega = float(np.prod(L))
    rP = coulomb.positions(L, grid, pts)
    r_all = coulomb.positions(L, grid)
    Pw = np.empty((nk, nI, ng), dtype=np.complex128)
    for m in range(nk):
        q = coulomb.qvec(L, kmesh, m)
        F = sfft.fftn(xi[m].reshape((nI,) + grid), axes=(1, 2, 3), workers=WORKERS)
        v = coulomb.kernel(L, grid, kmesh, m)
        Phi = (omega / ng) * sfft.ifftn(F * v[None], axes=(1, 2, 3), workers=WORKERS).reshape(nI, ng)
        Pw[m] = np.exp(1j * (rP @ q))[:, None] * np.exp(-1j * (r_all @ q))[None, :] * Phi.conj()
    return Pw


def thc_oo_k_robust(L, grid, kmesh, psi, phi, pts, rel_tol=1e-12):
    """Robust-fit THC-oo-K (the one-sided fit of the discussion in Sec. 5): the
    exchange matrix with one fitted and one exact pair density in each integral,
      K_rob = K[rho, rho~] + K[rho~, rho] - K[rho~, rho~],
    where K[a, b]^n_{mu nu} = (1/N_k) sum_{n' j} J^m[a_{mu j}, b_{nu j}] (the pair
    densities of direct exchange), rho the exact pairs e^{-i q.r} conj phi_mu^n
    psi_jn' and rho~ their interpolation sum_P xi^m_P(r) e^{-i q.r_P} conj
    phi_mu^n(r_P) psi_jn'(r_P) with the per-transfer occupied-pair fit. Then
    K_direct - K_rob = K[delta, delta] (delta = rho - rho~): second order in the
    fit's residual, where K_fit = K[rho~, rho~] is first order.

    The one-sided term needs the potentials Phi^m of the fitted functions on the
    grid (never the exact pair potentials): with J[f1, f2] = sum_r f1(r) conj
    Phi[f2](r) and the sum over j of the exact pair giving conj Gamma^{n'},
      K[rho, rho~]^n = (1/N_k) conj(phi^n) R^n^T A^n,
      R^n(Q, r) = sum_m Pw^m(Q, r) conj Gamma^{n+m}(Q, r),
    A^n_{Q nu} = phi_nu^n(r_Q) and Pw as in phased_potentials. Its energy
    E_cross = -(1/N_k^2) Re sum_n sum_{Q,r} Gamma^n(Q, r) R^n(Q, r) equals the
    fitted E_x: the least-squares fit projects every occupied pair onto the fit
    space, so the robust energy 2 E_cross - E_x is E_x itself; only K moves.

    phi: AO functions on the grid (N_k, N, N_g). Returns K (robust), K_fit,
    K_cross, Ex (fitted), Ex_rob (2 E_cross - E_x), rank, S, keep.
    """
    L = np.asarray(L, dtype=np.float64)
    grid = tuple(int(x) for x in grid)
    kmesh = tuple(int(x) for x in kmesh)
    pts = np.asarray(pts, dtype=np.int64)
    nk = psi.shape[0]
    ao_pts = np.stack([phi[n][:, pts] for n in range(nk)])
    o = thc_oo_k(L, grid, kmesh, psi, pts, ao_pts, rel_tol, keep_intermediates=("xi",))
    Psi, X, G = gather(psi, pts, ao_pts)
    Gam = np.stack([_gamma(Psi[n], psi[n]) for n in range(nk)])
    Pw = phased_potentials(L, grid, kmesh, o["xi"], pts)
    Kc = np.empty_like(o["K"])
    e_cross = 0.0
    for n in range(nk):
        R = np.zeros_like(Pw[0])
        for m in range(nk):
            R += Pw[m] * Gam[coulomb.add_index(kmesh, n, m)].conj()
        Kc[n] = phi[n].conj() @ R.T @ ao_pts[n].T / nk
        e_cross += np.sum(Gam[n] * R).real
    e_cross = -e_cross / nk ** 2
    Kr = Kc + np.conj(np.transpose(Kc, (0, 2, 1))) - o["K"]
    return dict(K=Kr, K_fit=o["K"], K_cross=Kc, Ex=o["Ex"], Ex_rob=2.0 * e_cross - o["Ex"],
                rank=o["rank"], S=o["S"], keep=o["keep"])


def thc_oo_k_gradient(L, grid, kmesh, psi, phi, pts, rel_tol=1e-12):
    """The derivative of the fitted exchange energy in the AO density matrices:
    the full exchange matrix whose occupied-virtual block is the orbital
    gradient of Sec. 2.3 (Eq. 19; the dM/dtheta step of Algorithm 2).

    With the per-transfer fit xi^m = (S^m)^{-1} Z^m (on the retained points) and
    V^m = xi^m Vop xi^m^H (Vop the Coulomb operator of steps 5-6), the energy of
    step 9 is E = -(1/N_k^2) sum_m Tr(V^m S^m) = -(1/N_k^2) sum_m Tr((S^m)^{-1}
    Z^m Vop Z^m^H), so that
      dE = (1/N_k^2) sum_m [Tr(V^m dS^m) - 2 Re sum_{P,r} dZ^m(P,r) conj Phi^m_P(r)],
      Phi^m_P(r) = (Omega/N_g^2) sum_g e^{i g.r} v^m(g) F^m_P(g)  (the potential of xi^m_P).
    S^m and Z^m depend on the density through G^n and Gamma^n (steps 1-3), and
    those on the AO density matrices D^n = C^n C^n^H through
    Gamma^n(P,r) = sum_{mu,nu} phi_mu^n(r_P) D^n_{mu nu} conj phi_nu^n(r). Collecting
    the coefficient of dD gives dE = Re sum_n sum_{mu nu} dD^n_{mu nu} A^n_{mu nu}
    and, for Hermitian dD, dE = -(2/N_k) sum_n Tr(Kgrad^n dD^n) with
    Kgrad^n = -(N_k/4) (A^n + A^n^H)^T. (Holding V^m fixed instead gives the K of
    steps 7-8 in the same normalisation.) Both terms of each product rule are
    written out (no symmetry between m and -m is used).

    phi: AO functions on the grid (N_k, N, N_g). Returns K, Kgrad, Ex, rank (and
    the metrics S with their retained points keep).
    """
    L = np.asarray(L, dtype=np.float64)
    grid = tuple(int(x) for x in grid)
    kmesh = tuple(int(x) for x in kmesh)
    pts = np.asarray(pts, dtype=np.int64)
    nk, no, ng = psi.shape
    nI = len(pts)
    ao_pts = np.stack([phi[n][:, pts] for n in range(nk)])
    o = thc_oo_k(L, grid, kmesh, psi, pts, ao_pts, rel_tol, keep_intermediates=("xi",))
    Psi, X, G = gather(psi, pts, ao_pts)
    rP = coulomb.positions(L, grid, pts)
    Gam = np.stack([_gamma(Psi[n], psi[n]) for n in range(nk)])
    # Pw^m(P, r) = e^{i q_m.(r_P - r)} conj Phi^m_P(r) and U^m_PQ = V^m_QP e^{i q_m.(r_P - r_Q)}
    Pw = phased_potentials(L, grid, kmesh, o["xi"], pts)
    U = np.empty((nk, nI, nI), dtype=np.complex128)
    for m in range(nk):
        eP = np.exp(1j * (rP @ coulomb.qvec(L, kmesh, m)))
        U[m] = o["V"][m].T * (eP[:, None] * eP.conj()[None, :])
    Kgrad = np.empty_like(o["K"])
    for n in range(nk):
        CS = np.zeros((nI, nI), dtype=np.complex128)
        CZ = np.zeros((nI, ng), dtype=np.complex128)
        for m in range(nk):
            up = coulomb.add_index(kmesh, n, m)                       # n + m
            dn = [k for k in range(nk) if coulomb.add_index(kmesh, k, m) == n][0]  # n - m
            CS += U[m] * G[up].conj() + U[m].conj() * G[dn].conj()
            CZ += Pw[m] * Gam[up].conj() + Pw[m].conj() * Gam[dn].conj()
        NS = ao_pts[n] @ CS @ ao_pts[n].conj().T
        NZ = ao_pts[n] @ CZ @ phi[n].conj().T
        A = (NS - 2.0 * NZ) / nk ** 2
        Kgrad[n] = -(nk / 4.0) * (A + A.conj().T).T
    return dict(K=o["K"], Kgrad=Kgrad, Ex=o["Ex"], rank=o["rank"], S=o["S"], keep=o["keep"])

