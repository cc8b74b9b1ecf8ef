"""Pins of the learned-selector reference (oracle/mlp.py): finite-difference
gradients, the closed-form first Adam step, feature identities, targets, the
non-maximum-suppression rule checked by brute force, and the fit-residual
probe checked against least squares on the explicit pair matrix and against
the pivot order of QRCP."""

import numpy as np

import synth
from oracle import mlp, select


def _data(n=200, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 3))
    t = rng.uniform(0, 1, n) ** 4
    w = 1.0 + 20.0 * t
    return X, t, w


def test_gradient_matches_central_differences():
    X, t, w = _data()
    theta = mlp.init_params(3)
    g = mlp.grad(theta, X, t, w)
    rng = np.random.default_rng(7)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss(theta + e, X, t, w) - mlp.loss(theta - e, X, t, w)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(g[i])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=0.0)
    # bias-corrected moments equal g and g^2 at step 1, so the step is lr * sign(g)
    assert np.allclose(new, theta - 0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_training_lowers_the_loss():
    X, t, w = _data(400)
    theta = mlp.init_params(0)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, t, w)
    for step in range(1, 201):
        theta, m, v = mlp.adam_step(theta, mlp.grad(theta, X, t, w), m, v, step, lr=3e-3)
    assert mlp.loss(theta, X, t, w) < 0.8 * l0


def test_feature_identities():
    # one orbital: the orbital-weight feature is exactly 1; mean of rho/rho_bar is 1
    c = synth.make_random_cell((5.0, 5.5, 6.0), 2, (10, 12, 12), (1, 1, 1), 1, 10, (3, 1, 4))
    psi = synth.orbitals_on_grid(c, synth.orbital_coeffs(c))
    F = mlp.features(c.L, c.grid, psi)
    assert np.allclose(F[:, 2], 1.0, atol=1e-12)
    assert abs(np.mean(np.exp(F[:, 0])) - 1.0) <= 1e-12
    # with several orbitals it lies in (0, 1]
    c2 = synth.make_random_cell((5.0, 5.5, 6.0), 2, (10, 12, 12), (2, 1, 1), 3, 10, (3, 1, 5))
    F2 = mlp.features(c2.L, c2.grid, synth.orbitals_on_grid(c2, synth.orbital_coeffs(c2)))
    assert np.all(F2[:, 2] > 0) and np.all(F2[:, 2] <= 1 + 1e-12)


def test_fourth_order_gradient_on_a_plane_wave_density():
    L = np.array([6.0, 7.0, 8.0])
    grid = (24, 28, 32)
    idx = np.unravel_index(np.arange(np.prod(grid)), grid)
    x = idx[0] * L[0] / grid[0]
    # a single "orbital" whose density is 2 + sin(2 pi x / L0)
    rho = 2.0 + np.sin(2 * np.pi * x / L[0])
    psi = np.sqrt(rho)[None, None, :].astype(np.complex128)
    F = mlp.features(L, grid, psi)
    k = 2 * np.pi / L[0]
    grad = np.abs(k * np.cos(k * x))
    ref = np.log(np.maximum(grad, 1e-300)) - (4.0 / 3.0) * np.log(rho)
    ok = grad > 1e-3
    assert np.abs(F[ok, 1] - ref[ok]).max() <= 2e-4


def test_targets_and_nms_rule():
    L = np.array([5.0, 6.0, 7.0])
    grid = (10, 12, 14)
    rng = np.random.default_rng(4)
    pts = rng.choice(np.prod(grid), 12, replace=False)
    t = mlp.targets(L, grid, pts, mlp.target_width(L, 12))
    assert np.allclose(t[pts], 1.0)
    assert np.all((t > 0) & (t <= 1.0 + 1e-15))
    scores = rng.standard_normal(np.prod(grid))
    sel = mlp.nms_select(L, grid, scores, 12)
    idx = np.unravel_index(np.arange(np.prod(grid)), grid)
    r = np.stack([idx[i] * (L[i] / grid[i]) for i in range(3)], axis=1)
    h2 = mlp.nms_radius(L, 12) ** 2
    d2 = mlp.min_image_dist2(L, r[sel], r[sel])
    np.fill_diagonal(d2, np.inf)
    assert d2.min() >= h2
    # greedy: every unselected point that beats the last pick is suppressed by an earlier pick
    last = scores[sel[-1]]
    for i in np.flatnonzero(scores > last):
        if i in sel:
            continue
        assert mlp.min_image_dist2(L, r[i:i + 1], r[sel]).min() < h2
    assert len(set(sel.tolist())) == 12


def _small_cell(nk=(2, 1, 1), n_occ=2, grid=(6, 6, 8), seed=(5, 5, 5)):
    c = synth.make_random_cell((4.0, 4.5, 5.0), 2, grid, nk, n_occ, 6, seed)
    return synth.orbitals_on_grid(c, synth.orbital_coeffs(c))


def _pair_rows(psi):
    """Explicit pair matrix z[(w, w'), r] = psi_w(r) conj psi_w'(r)."""
    A = psi.reshape(-1, psi.shape[-1])
    return (A[:, None, :] * A[None, :, :].conj()).reshape(-1, A.shape[-1])


def test_probe_residual_is_least_squares_on_the_pair_matrix():
    psi = _small_cell()
    Z = _pair_rows(psi)  # 16 pair functions
    ng = psi.shape[-1]
    rng = np.random.default_rng(11)
    pts = rng.choice(ng, 6, replace=False)
    for r in rng.choice(np.setdiff1d(np.arange(ng), pts), 12, replace=False):
        coef, *_ = np.linalg.lstsq(Z[:, pts], Z[:, r], rcond=None)
        res = np.linalg.norm(Z[:, r] - Z[:, pts] @ coef) ** 2 / np.linalg.norm(Z[:, r]) ** 2
        got = mlp.probe_residual(psi, pts, [r])
        assert abs(got - res) <= 1e-10 + 1e-8 * res


def test_probe_residual_vanishes_on_the_points_and_decreases_with_more_points():
    psi = _small_cell(nk=(1, 1, 1), n_occ=3, seed=(6, 6, 6))
    ng = psi.shape[-1]
    rng = np.random.default_rng(3)
    pts = rng.choice(ng, 8, replace=False)
    assert mlp.probe_residual(psi, pts, pts[:5]) <= 1e-12
    probe = rng.choice(ng, 40, replace=False)
    prev = 1.0 + 1e-12
    for p in range(1, 9):
        cur = mlp.probe_residual(psi, pts[:p], probe)
        assert cur <= prev + 1e-12
        prev = cur
    # 9 pair functions: 9 well-spread points span them, so nothing is left anywhere
    full, _ = select.select_points(psi, 9)
    assert mlp.probe_residual(psi, full, np.arange(ng)) <= 1e-9


def test_probe_schur_diagonal_peaks_at_the_next_qrcp_pivot():
    psi = _small_cell(seed=(7, 7, 7))
    ng = psi.shape[-1]
    A = psi.reshape(-1, ng)
    crr = np.sum(np.abs(A) ** 2, axis=0) ** 2
    for p in (1, 3, 5):
        pts, npiv = select.select_points(psi, p + 1)
        assert npiv == p + 1
        d = np.array([mlp.probe_residual(psi, pts[:p], [r]) * crr[r] for r in range(ng)])
        assert int(np.argmax(d)) == int(pts[p])
