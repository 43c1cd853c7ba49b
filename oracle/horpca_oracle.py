"""Independent full-SVD ADMM for the splitting of eq. (2) (test infrastructure only).

TEST INFRASTRUCTURE ONLY; never called by the GPU library.

When every R_n equals I_n the active subspace U_n of eq. (3) is a square
orthogonal matrix, so fold_n(U_n V_n) with V_n = SVT(U_n^T G_n) is
fold_n(SVT(G_n)) for any orthogonal U_n, and Algorithm 1 becomes an ADMM on the
splitting of eq. (2) with a full singular value thresholding of each
unfolding.  This module writes that ADMM out on its own (its own unfolding by
explicit index arithmetic, its own SVT) so that it can pin the PASD oracle
iterate by iterate in that special case.  It is not claimed to match the
step-size schedule of any published HoRPCA code; it uses the penalty schedule
of Algorithm 1 (mu^0, rho, mu_max) so that both follow the same sequence.
"""

from __future__ import annotations

import itertools
from typing import List, Sequence

import numpy as np


def _unfold_loops(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding by explicit index enumeration (small tensors only)."""
    dims = X.shape
    other = [m for m in range(X.ndim) if m != n]
    cols = list(itertools.product(*[range(dims[m]) for m in other]))
    out = np.empty((dims[n], len(cols)))
    for c, idx in enumerate(cols):
        full = [0] * X.ndim
        for m, i in zip(other, idx):
            full[m] = i
        for i in range(dims[n]):
            full[n] = i
            out[i, c] = X[tuple(full)]
    return out


def _fold_loops(M: np.ndarray, n: int, dims: Sequence[int]) -> np.ndarray:
    other = [m for m in range(len(dims)) if m != n]
    cols = list(itertools.product(*[range(dims[m]) for m in other]))
    X = np.empty(tuple(dims))
    for c, idx in enumerate(cols):
        full = [0] * len(dims)
        for m, i in zip(other, idx):
            full[m] = i
        for i in range(dims[n]):
            full[n] = i
            X[tuple(full)] = M[i, c]
    return X


def _svt_full(X: np.ndarray, tau: float) -> np.ndarray:
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    s = np.where(s > tau, s - tau, 0.0)
    return U @ np.diag(s) @ Vt


def _shrink(x: np.ndarray, tau: float) -> np.ndarray:
    out = np.zeros_like(x)
    out[x > tau] = x[x > tau] - tau
    out[x < -tau] = x[x < -tau] + tau
    return out


def horpca_admm(T: np.ndarray, lam: Sequence[float], iters: int, mu0: float = 1e-4,
                rho: float = 1.1, mu_max: float = 1e10):
    """ADMM on eq. (2): per iteration Z_n = fold(SVT_{lam_n/mu}(unfold(T - E + Y_n/mu))),
    E = shrink(mean_n(T - Z_n + Y_n/mu), 1/(mu N)), Y_n += mu (T - Z_n - E),
    mu = min(rho mu, mu_max).  Returns the list of (Z, E, Y) after each iteration.
    """
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    dims = T.shape
    E = np.zeros_like(T)
    Y: List[np.ndarray] = [np.zeros_like(T) for _ in range(N)]
    mu = mu0
    out = []
    for _ in range(iters):
        Z = []
        for n in range(N):
            G = _unfold_loops(T - E + Y[n] / mu, n)
            Z.append(_fold_loops(_svt_full(G, lam[n] / mu), n, dims))
        Hbar = np.zeros_like(T)
        for n in range(N):
            Hbar += T - Z[n] + Y[n] / mu
        Hbar /= N
        E = _shrink(Hbar, 1.0 / (mu * N))
        Y = [Y[n] + mu * (T - Z[n] - E) for n in range(N)]
        mu = min(rho * mu, mu_max)
        out.append(([z.copy() for z in Z], E.copy(), [y.copy() for y in Y]))
    return out
