"""Learned interpolation-point selector: FP64 reference (oracle).

TEST INFRASTRUCTURE ONLY (see package docstring).

The paper selects ISDF points by QRCP or CVT k-means (Sec. 2.1 after Eq. 5).
The learned selector proposes points from per-grid-point descriptors of the
occupied density instead, trained to reproduce QRCP selections:

* features (per grid point r, orthorhombic periodic grid):
    f0 = ln(rho / mean rho),  rho(r) = (1/N_k) sum_{n,i} |psi_in(r)|^2
    f1 = ln|grad rho| - (4/3) ln rho   (fourth-order periodic central differences)
    f2 = sum_{n,i} |psi_in(r)|^4 / (sum_{n,i} |psi_in(r)|^2)^2
  each standardised with fixed (mean, scale) constants;
* network: 3 -> 64 -> 64 -> 1 with SiLU after the hidden layers; the score is
  the logit s(r);
* targets: t(r) = exp(-d(r)^2 / (2 sigma^2)) with d the periodic minimum-image
  distance to the nearest QRCP point and a given width sigma (the training
  driver uses sigma = (Omega / N_ISDF)^{1/3} / 4, half the suppression radius);
* loss: weighted binary cross-entropy
    L = sum_r w(r) [softplus(s) - t s] / sum_r w(r),  w = 1 + wpos t;
* optimiser: Adam;
* inference: greedy top-N_ISDF by score with non-maximum suppression within
  radius h = (Omega / N_ISDF)^{1/3} / 2 (periodic minimum image);
* probe: relative fit residual of a point set P on probe points r_j,
  sum_j [C(r_j,r_j) - C(r_j,P) C(P,P)^+ C(P,r_j)]_+ / sum_j C(r_j,r_j), where
  C(r,r') = |Gamma(r,r')|^2 is the Gram matrix of the pair rows
  z_{ww'}(r) = psi_w(r) conj psi_w'(r) that QRCP pivots on (Sec. 2.1): the
  Schur complement is the squared distance of z(r_j) from span{z(r_P)}.

Parameters are one flat FP64 vector: W1 (64x3), b1 (64), W2 (64x64), b2 (64),
w3 (64), b3 (1).
"""

from __future__ import annotations

import numpy as np

H = 64
SIZES = (("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,)))
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def init_params(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.standard_normal((H, 3)) * np.sqrt(1.0 / 3.0),
        "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) * np.sqrt(1.0 / H),
        "b2": np.zeros(H),
        "w3": rng.standard_normal(H) * np.sqrt(1.0 / H),
        "b3": np.array([-4.0]),
    }
    return pack(p)


def features(L, grid, psi: np.ndarray, norm=((0.0, 1.0), (0.0, 1.0), (0.0, 1.0))) -> np.ndarray:
    """(N_g, 3) standardised descriptors from orbitals psi (N_k, n_occ, N_g)."""
    grid = tuple(int(x) for x in grid)
    nk = psi.shape[0]
    a2 = np.abs(psi.reshape(-1, psi.shape[-1])) ** 2
    s2 = a2.sum(axis=0)
    s4 = (a2 * a2).sum(axis=0)
    rho = s2 / nk
    tiny = 1e-300
    f0 = np.log(np.maximum(rho, tiny) / rho.mean())
    r3 = rho.reshape(grid)
    g2 = np.zeros(grid)
    for ax in range(3):
        h = L[ax] / grid[ax]
        d = (np.roll(r3, 2, ax) - 8 * np.roll(r3, 1, ax) + 8 * np.roll(r3, -1, ax)
             - np.roll(r3, -2, ax)) / (12 * h)
        g2 += d * d
    f1 = 0.5 * np.log(np.maximum(g2.reshape(-1), tiny)) - (4.0 / 3.0) * np.log(np.maximum(rho, tiny))
    f2 = s4 / np.maximum(s2 * s2, tiny)
    F = np.stack([f0, f1, f2], axis=1)
    for k in range(3):
        F[:, k] = (F[:, k] - norm[k][0]) / norm[k][1]
    return F


def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def forward(theta: np.ndarray, X: np.ndarray, keep=False):
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(z2)
    s = h2 @ p["w3"] + p["b3"][0]
    if keep:
        return s, (z1, h1, z2, h2)
    return s


def softplus(x):
    return np.logaddexp(0.0, x)


def loss(theta, X, t, w):
    s = forward(theta, X)
    return float(np.sum(w * (softplus(s) - t * s)) / np.sum(w))


def grad(theta, X, t, w):
    """Analytic gradient of ``loss`` (reverse mode through the two hidden layers)."""
    p = unpack(theta)
    s, (z1, h1, z2, h2) = forward(theta, X, keep=True)
    ds = w * (1.0 / (1.0 + np.exp(-s)) - t) / np.sum(w)
    g = {"w3": h2.T @ ds, "b3": np.array([ds.sum()])}
    dz2 = np.outer(ds, p["w3"]) * dsilu(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * dsilu(z1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); returns new (theta, m, v). ``step`` counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def min_image_dist2(L, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Squared periodic minimum-image distances between point sets a (n,3) and b (m,3)."""
    d = a[:, None, :] - b[None, :, :]
    d -= L * np.round(d / L)
    return np.sum(d * d, axis=-1)


def nms_radius(L, n_isdf) -> float:
    return 0.5 * (float(np.prod(L)) / n_isdf) ** (1.0 / 3.0)


def target_width(L, n_isdf) -> float:
    """Default target width sigma = (Omega / N_ISDF)^{1/3} / 4."""
    return 0.25 * (float(np.prod(L)) / n_isdf) ** (1.0 / 3.0)


def targets(L, grid, pts, sigma, chunk=4096) -> np.ndarray:
    """t(r) = exp(-d^2 / (2 sigma^2)) to the nearest of the points ``pts`` (flat indices)."""
    L = np.asarray(L, dtype=np.float64)
    idx = np.unravel_index(np.arange(int(np.prod(grid))), grid)
    r = np.stack([idx[i] * (L[i] / grid[i]) for i in range(3)], axis=1)
    q = r[np.asarray(pts)]
    out = np.empty(len(r))
    for c0 in range(0, len(r), chunk):
        d2 = min_image_dist2(L, r[c0:c0 + chunk], q).min(axis=1)
        out[c0:c0 + chunk] = np.exp(-d2 / (2 * sigma * sigma))
    return out


def nms_select(L, grid, scores: np.ndarray, n_isdf: int) -> np.ndarray:
    """Greedy: highest score first (ties to the smallest flat index), skipping points
    within the suppression radius of an already chosen point."""
    L = np.asarray(L, dtype=np.float64)
    idx = np.unravel_index(np.arange(len(scores)), grid)
    r = np.stack([idx[i] * (L[i] / grid[i]) for i in range(3)], axis=1)
    h2 = nms_radius(L, n_isdf) ** 2
    alive = np.ones(len(scores), dtype=bool)
    order = np.lexsort((np.arange(len(scores)), -scores))
    chosen = []
    for i in order:
        if not alive[i]:
            continue
        chosen.append(int(i))
        if len(chosen) == n_isdf:
            break
        d2 = min_image_dist2(L, r[i:i + 1], r)[0]
        alive &= d2 >= h2
    if len(chosen) < n_isdf:  # radius too large for this grid: fill by score
        rest = [int(i) for i in order if int(i) not in set(chosen)]
        chosen += rest[: n_isdf - len(chosen)]
    return np.asarray(chosen, dtype=np.int64)


def probe_residual(psi: np.ndarray, pts, probe, rel_tol: float = 1e-12) -> float:
    """Relative fit residual of the points ``pts`` on the grid points ``probe``
    (both flat indices; orbitals psi (N_k, n_occ, N_g)), FP64, by the Schur
    complement of the Gram matrix C = |Gamma|^2 with C(P,P) factorised by the
    fit's Cholesky with pivot drop."""
    from . import thc

    nk, no, ng = psi.shape
    A = psi.reshape(nk * no, ng)
    AP = A[:, np.asarray(pts)]
    AR = A[:, np.asarray(probe)]
    Cpp = np.abs(AP.T @ AP.conj()) ** 2
    Cpr = np.abs(AP.T @ AR.conj()) ** 2
    crr = np.sum(np.abs(AR) ** 2, axis=0) ** 2
    L, keep = thc.cholesky_drop(Cpp.astype(np.complex128), rel_tol)
    R = np.flatnonzero(keep)
    y = np.linalg.solve(L[np.ix_(R, R)], Cpr[R].astype(np.complex128))
    q = np.sum(np.abs(y) ** 2, axis=0)
    den = float(np.sum(crr))
    return float(np.sum(np.maximum(crr - q, 0.0)) / den) if den > 0 else 1.0