"""Interpolation-point selection by pivoted Cholesky (oracle).

TEST INFRASTRUCTURE ONLY (see package docstring).

The paper selects the ISDF points by QR with column pivoting (or CVT
k-means; Sec. 2.1 after Eq. 5, Algorithms 1-2 first line), once before the SCF
loop, with one point set for every q. QR with column pivoting of the stacked
pair matrix A[(n,i,n',j), r] = conj psi_in(r) psi_jn'(r) picks the same
columns as greedy pivoted Cholesky of its Gram matrix

    A^H A (r, r') = |Gamma(r, r')|^2,   Gamma(r, r') = sum_{n,i} psi_in(r) conj psi_in(r'),

which is what is written here, in FP64:

* pivot = argmax of the Schur-complement diagonal (ties -> smallest flat
  index); the first diagonal is (sum_{n,i} |psi_in(r)|^2)^2;
* stop pivoting once the pivot falls below rel_tol times the first pivot;
* the remaining slots are filled by descending density
  rho(r) = sum_{n,i} |psi_in(r)|^2 among unselected points (ties -> smallest
  flat index).
"""

from __future__ import annotations

import numpy as np


def select_points(psi: np.ndarray, n_isdf: int, rel_tol: float = 1e-12):
    """Return (points int64 (n_isdf,), n_pivoted)."""
    nk, no, ng = psi.shape
    A = psi.reshape(nk * no, ng)
    dens = np.sum(np.abs(A) ** 2, axis=0)
    d = dens ** 2
    Lf = np.zeros((ng, n_isdf), dtype=np.float64)
    chosen = []
    taken = np.zeros(ng, dtype=bool)
    first = None
    for p in range(n_isdf):
        dm = np.where(taken, -np.inf, d)
        piv = int(np.argmax(dm))
        dp = float(dm[piv])
        if first is None:
            first = dp
        if not dp > rel_tol * first:
            break
        col = np.abs(A.T @ A[:, piv].conj()) ** 2
        if p:
            col = col - Lf[:, :p] @ Lf[piv, :p]
        Lf[:, p] = col / np.sqrt(dp)
        d = d - Lf[:, p] ** 2
        chosen.append(piv)
        taken[piv] = True
    n_piv = len(chosen)
    if n_piv < n_isdf:
        order = np.argsort(-dens, kind="stable")
        for r in order:
            if not taken[r]:
                chosen.append(int(r))
                taken[r] = True
                if len(chosen) == n_isdf:
                    break
    return np.asarray(chosen, dtype=np.int64), n_piv
