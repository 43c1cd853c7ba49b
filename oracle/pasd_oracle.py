"""Plain FP64 PASD ADMM: the oracle the GPU path is checked against.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or runs
this module; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It is written for clarity, not speed: every step is one library call
(``numpy.linalg.svd``, ``@``) or an elementwise numpy expression, taken in the
order of Algorithm 1 of the paper (Section 3.2).

Notation follows the paper: ``T`` the observed tensor, ``U_n`` the active
subspace (an I_n x R_n column-orthonormal matrix), ``V_n`` the small R_n x J_n
factor with J_n the product of the other dimensions, ``E`` the sparse part,
``Y_n`` the multipliers, ``mu`` the penalty.  ``P_n`` denotes the matrix the
SVT of eq. (13) is applied to, ``U_n^T G_n``; so ``V_n = SVT(P_n)``.

Readings of points the paper leaves open (each is argued in the design notes):

* Procrustes step (eq. (10)).  Eq. (10) takes the polar factor of
  ``G_n^k (V_n^k)^T``.  Write the thin SVD P_n^k = A S B^T; then
  V_n^k = A diag((s - tau)_+) B^T, so whenever V_n^k has full row rank R_n the
  matrices ``G_n^k (V_n^k)^T`` and ``G_n^k (P_n^k)^T`` have the same range and
  their polar factors span the same subspace.  When V_n^k is rank deficient
  (always at k = 0, where V^0 = 0, and whenever the SVT zeroes a singular
  value) eq. (10) has many minimisers.  The oracle keeps ``U^1 = U^0`` at
  k = 0 and for k >= 1 takes the polar factor of ``G_n^k (P_n^k)^T``: eq. (10)
  itself when V_n^k has full rank (up to a rotation inside the same span,
  which changes no iterate, since Z_n = SVT(U_n U_n^T G_n) depends on the span
  only), and one of its minimisers otherwise.  Using P instead of V also keeps
  the step well conditioned when a singular value has just crossed the
  threshold.
  The alternative tie-break ``tiebreak="keep"`` (reading R1') solves eq. (10)
  with ``G_n^k (V_n^k)^T`` itself and, on the directions where V_n^k vanishes,
  keeps U_n^k: among the maximisers of <U, A> over column-orthonormal U
  (A = G_n^k (V_n^k)^T of rank r, thin SVD A = Ua S Va^T) it takes
  ``Ua_r Va_r^T + C B^T`` with B the last R_n - r columns of Va (the null
  space of A) and C the polar factor of (I - Ua_r Ua_r^T) U_n^k B, the
  orthonormal completion nearest U_n^k (the limit of polar(A + eps U_n^k) as
  eps -> 0+).  At k = 0 (V = 0) this gives U^1 = U^0, as does the default.
  Parity status of this variant: pinned by the same tests (it equals the
  default wherever V_n^k has full rank) and by a brute-force search over the
  completion on small cases.
* The weights ``lambda_n`` default to sqrt(max(I_n, J_n)) / N (Section 5.1).
* The output weights ``alpha_n`` of Algorithm 1 are undefined in the paper;
  the oracle takes ``alpha_n = lambda_n``.
* The stopping test is the strict inequality of Algorithm 1, evaluated with
  E^{k+1}, Z^{k+1} after mu has been updated; the multiplier update uses the
  penalty of the current iteration, mu^k.

Parity status: every function here is pinned by tests against brute force,
closed forms, an independent full-SVD implementation of the R_n = I_n special
case, or the exact optimality conditions of the paper's appendix (eqs. (S1),
(S3)).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


# --------------------------------------------------------------------------
# Tensor algebra (Section 2.1)
# --------------------------------------------------------------------------

def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding: the mode-n fibres of ``X`` become the columns.

    The columns are ordered lexicographically over the remaining indices
    (i_1, ..., i_{n-1}, i_{n+1}, ..., i_N), last index fastest.  The paper's
    results do not depend on the column order.
    """
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def fold(M: np.ndarray, n: int, shape: Sequence[int]) -> np.ndarray:
    """Inverse of :func:`unfold` (the ``fold_n`` of eq. (3))."""
    rest = [int(s) for m, s in enumerate(shape) if m != n]
    return np.moveaxis(M.reshape([int(shape[n])] + rest), 0, n)


# --------------------------------------------------------------------------
# Proximal operators (eqs. (10), (13), (15))
# --------------------------------------------------------------------------

def prox_l1(X: np.ndarray, tau: float) -> np.ndarray:
    """Shrinkage operator of eq. (15): sgn(x) max(|x| - tau, 0), elementwise."""
    return np.sign(X) * np.maximum(np.abs(X) - tau, 0.0)


def svt(X: np.ndarray, tau: float):
    """Singular value thresholding of eq. (13).

    Returns ``(SVT_tau(X), singular values of X)``.  SVT_tau(X) keeps the
    singular vectors of X and replaces every singular value s by max(s - tau, 0).
    """
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    return (U * np.maximum(s - tau, 0.0)) @ Vt, s


def polar(M: np.ndarray) -> np.ndarray:
    """Solution of the orthogonal Procrustes problem of eq. (9): U_hat V_hat^T
    from the thin SVD M = U_hat Sigma_hat V_hat^T (eq. (10))."""
    U, _, Vt = np.linalg.svd(M, full_matrices=False)
    return U @ Vt


def procrustes_keep(A: np.ndarray, r: int, U_prev: np.ndarray) -> np.ndarray:
    """Eq. (10) for A = G V^T of rank r with the completion nearest U_prev on
    the null space of A (reading R1'): Ua_r Va_r^T + C B^T, where A = Ua S Va^T,
    B = Va[:, r:] and C = polar((I - Ua_r Ua_r^T) U_prev B)."""
    R = A.shape[1]
    Ua, _, Vat = np.linalg.svd(A, full_matrices=False)
    Va = Vat.T
    U = Ua[:, :r] @ Va[:, :r].T
    if r < R:
        B = Va[:, r:]
        X = U_prev @ B
        X = X - Ua[:, :r] @ (Ua[:, :r].T @ X)
        U = U + polar(X) @ B.T
    return U


def default_lambdas(dims: Sequence[int]) -> List[float]:
    """lambda_n = sqrt(max(I_n, prod_{m != n} I_m)) / N (Section 5.1)."""
    N = len(dims)
    numel = math.prod(int(d) for d in dims)
    return [math.sqrt(max(int(d), numel // int(d))) / N for d in dims]


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------

@dataclasses.dataclass
class OracleState:
    T: np.ndarray
    ranks: List[int]
    lam: List[float]
    alpha: List[float]
    mu: float
    mu_max: float
    rho: float
    k: int
    U: List[np.ndarray]
    V: List[np.ndarray]
    P: List[Optional[np.ndarray]]
    Z: List[np.ndarray]
    E: np.ndarray
    Y: List[np.ndarray]
    residual: List[float] = dataclasses.field(default_factory=list)
    rank: List[int] = dataclasses.field(default_factory=list)
    history: List[List[float]] = dataclasses.field(default_factory=list)
    # Quantities of the last completed iteration, kept for the invariant tests.
    last: dict = dataclasses.field(default_factory=dict)
    # Procrustes tie-break: "pre" (default, G P^T) or "keep" (reading R1')
    tiebreak: str = "pre"

    @property
    def N(self) -> int:
        return self.T.ndim


def pasd_init(T: np.ndarray, ranks: Sequence[int], lam: Optional[Sequence[float]] = None,
              alpha: Optional[Sequence[float]] = None, mu0: float = 1e-4,
              mu_max: float = 1e10, rho: float = 1.1, tiebreak: str = "pre") -> OracleState:
    """Initialisation of Algorithm 1: U_n^0 = eye(I_n, R_n), V_n^0 = 0,
    Y_n^0 = 0, E^0 = 0, mu^0 = 1e-4, mu_max = 1e10, rho = 1.1."""
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    dims = T.shape
    ranks = [int(r) for r in ranks]
    lam = list(default_lambdas(dims) if lam is None else [float(x) for x in lam])
    alpha = list(lam if alpha is None else [float(x) for x in alpha])
    U = [np.eye(dims[n], ranks[n]) for n in range(N)]
    J = [T.size // dims[n] for n in range(N)]
    V = [np.zeros((ranks[n], J[n])) for n in range(N)]
    return OracleState(
        T=T, ranks=ranks, lam=lam, alpha=alpha, mu=float(mu0), mu_max=float(mu_max),
        rho=float(rho), k=0, U=U, V=V, P=[None] * N, Z=[np.zeros_like(T) for _ in range(N)],
        E=np.zeros_like(T), Y=[np.zeros_like(T) for _ in range(N)], tiebreak=str(tiebreak))


def pasd_iterate(st: OracleState, count: int = 1, tol: Optional[float] = None) -> OracleState:
    """Run ``count`` iterations of Algorithm 1 in place.

    If ``tol`` is given the loop stops after the first iteration whose
    residuals all fall strictly below it (the convergence check of
    Algorithm 1).  Returns the state.
    """
    T = st.T
    N = st.N
    shape = T.shape
    for _ in range(count):
        mu = st.mu
        # G_n^k = T_(n) - E^k_(n) + Y^k_n,(n) / mu^k  (definition under eq. (9))
        G = [unfold(T - st.E + st.Y[n] / mu, n) for n in range(N)]
        # U-step, eq. (10), with the tie-break described in the module notes.
        U_new = []
        for n in range(N):
            if st.k == 0:
                U_new.append(st.U[n].copy())
            elif st.tiebreak == "keep":
                U_new.append(procrustes_keep(G[n] @ st.V[n].T, st.rank[n], st.U[n]))
            else:
                U_new.append(polar(G[n] @ st.P[n].T))
        # V-step, eq. (13): V_n = SVT_{lambda_n / mu^k}(U_n^T G_n^k).
        P_new, V_new, ranks_now, sing = [], [], [], []
        for n in range(N):
            P = U_new[n].T @ G[n]
            Vn, s = svt(P, st.lam[n] / mu)
            P_new.append(P)
            V_new.append(Vn)
            ranks_now.append(int(np.sum(s > st.lam[n] / mu)))
            sing.append(s)
        # Z_n^{k+1} = fold_n(U_n^{k+1} V_n^{k+1})  (Algorithm 1, line 5)
        Z = [fold(U_new[n] @ V_new[n], n, shape) for n in range(N)]
        # E-step, eq. (15): E = prox_{1/(mu N)}( (1/N) sum_n H_n ),
        # H_n = T - Z_n + Y_n / mu.
        H_mean = sum(T - Z[n] + st.Y[n] / mu for n in range(N)) / N
        E_new = prox_l1(H_mean, 1.0 / (mu * N))
        # Multipliers (Algorithm 1, line 6), with mu^k.
        Y_new = [st.Y[n] + mu * (T - Z[n] - E_new) for n in range(N)]
        # Residuals (Algorithm 1, line 8) and penalty update (line 7).
        res = [float(np.max(np.abs(T - Z[n] - E_new))) if T.size else 0.0 for n in range(N)]
        st.last = dict(mu=mu, G=G, E_prev=st.E, Y_prev=st.Y, sing=sing)
        st.U, st.V, st.P, st.Z, st.E, st.Y = U_new, V_new, P_new, Z, E_new, Y_new
        st.residual, st.rank = res, ranks_now
        st.history.append(res)
        st.mu = min(st.rho * mu, st.mu_max)
        st.k += 1
        if tol is not None and max(res) < tol:
            break
    return st


def pasd_output(st: OracleState):
    """Output of Algorithm 1: X = sum_n alpha_n Z_n / sum_n alpha_n, and E."""
    w = np.asarray(st.alpha, dtype=np.float64)
    X = sum(w[n] * st.Z[n] for n in range(st.N)) / w.sum()
    return X, st.E.copy()


def pasd_solve(T: np.ndarray, ranks: Sequence[int], lam=None, alpha=None, tol: float = 1e-5,
               max_iter: int = 1000, mu0: float = 1e-4, mu_max: float = 1e10,
               rho: float = 1.1, tiebreak: str = "pre"):
    """Algorithm 1 to convergence or ``max_iter``; returns (X, E, state)."""
    st = pasd_init(T, ranks, lam, alpha, mu0, mu_max, rho, tiebreak)
    while st.k < max_iter:
        pasd_iterate(st, 1)
        if max(st.residual) < tol:
            break
    X, E = pasd_output(st)
    return X, E, st
