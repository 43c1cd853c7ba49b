"""Pins for the FP64 oracle: each checks it against something other than itself.

Closed forms and brute force for the three proximal steps, the exact
optimality conditions the paper's appendix derives for every iterate
(eqs. (S1) and (S3)), basis invariance of the iteration, an independent
full-SVD ADMM for the R_n = I_n special case, convergence (Theorem 1) and
recovery of a planted decomposition (Section 5.1).
"""

import math

import numpy as np
import pytest

import workloads
from oracle import (default_lambdas, fold, horpca_admm, pasd_init, pasd_iterate, pasd_output,
                    pasd_solve, polar, prox_l1, svt, unfold)
from oracle import pasd_oracle


def _small(dims=(6, 7, 8), ranks=(2, 3, 2), frac=0.1, seed=3):
    return workloads.tucker_workload("small", dims, ranks, frac, seed, value_range=(-5, 5),
                                     scale="rms")


# ---------------------------------------------------------------- tensor algebra

def test_unfold_fold_roundtrip_and_fibres():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3, 4, 5, 2))
    for n in range(4):
        M = unfold(X, n)
        assert M.shape == (X.shape[n], X.size // X.shape[n])
        np.testing.assert_array_equal(fold(M, n, X.shape), X)
        # every column is a mode-n fibre: fixing the other indices
        other = [m for m in range(4) if m != n]
        idx = [1, 2, 1, 0]
        col = 0
        for m in other:
            col = col * X.shape[m] + idx[m]
        sl = list(idx)
        sl[n] = slice(None)
        np.testing.assert_array_equal(M[:, col], X[tuple(sl)])


# ---------------------------------------------------------------- prox (eq. 15)

@pytest.mark.parametrize("tau", [0.05, 0.7, 2.0])
def test_prox_matches_scalar_grid(tau):
    grid = np.linspace(-6, 6, 240001)
    for x in [-4.3, -0.8, -0.01, 0.0, 0.3, 0.69, 1.9, 5.5]:
        f = np.abs(grid) + (grid - x) ** 2 / (2 * tau)
        e_bf = grid[np.argmin(f)]
        assert abs(prox_l1(np.array(x), tau) - e_bf) <= 1e-4


def test_estep_is_minimiser_of_eq14():
    """E^{k+1} from one oracle iteration minimises eq. (14) elementwise."""
    wl = _small()
    st = pasd_init(wl.T, wl.ranks, mu0=0.05)
    pasd_iterate(st, 3)
    mu = st.last["mu"]
    N = st.N
    H = [st.T - st.Z[n] + st.last["Y_prev"][n] / mu for n in range(N)]
    flatH = np.stack([h.reshape(-1) for h in H])
    E = st.E.reshape(-1)
    rng = np.random.default_rng(1)
    for idx in rng.choice(E.size, 40, replace=False):
        h = flatH[:, idx]
        lo, hi = min(h.min(), 0.0) - 1, max(h.max(), 0.0) + 1
        grid = np.linspace(lo, hi, 200001)
        f = np.abs(grid) + 0.5 * mu * ((grid[:, None] - h[None, :]) ** 2).sum(1)
        e_bf = grid[np.argmin(f)]
        assert abs(E[idx] - e_bf) <= 2 * (hi - lo) / 200000


# ---------------------------------------------------------------- SVT (eq. 13)

def test_svt_rank_one_is_vector_shrinkage():
    rng = np.random.default_rng(2)
    for tau in [0.1, 1.0, 5.0]:
        p = rng.standard_normal((1, 9)) * 2
        out, _ = svt(p, tau)
        nrm = np.linalg.norm(p)
        np.testing.assert_allclose(out, max(1 - tau / nrm, 0) * p, atol=1e-13)


def test_svt_is_nuclear_prox():
    """SVT_tau(X) minimises tau ||V||_* + 0.5 ||V - X||_F^2 (eqs. (12)-(13))."""
    rng = np.random.default_rng(3)
    nuc = lambda A: np.linalg.svd(A, compute_uv=False).sum()
    for shape, tau in [((3, 7), 0.5), ((4, 4), 2.0), ((2, 11), 0.1)]:
        X = rng.standard_normal(shape) * 2
        V, s = svt(X, tau)
        f0 = tau * nuc(V) + 0.5 * np.sum((V - X) ** 2)
        for _ in range(2000):
            D = rng.standard_normal(shape) * rng.choice([1e-3, 1e-2, 1e-1])
            W = V + D
            assert tau * nuc(W) + 0.5 * np.sum((W - X) ** 2) >= f0 - 1e-12
        # optimality: X - V lies in tau * subdifferential of ||V||_*
        assert np.linalg.norm(X - V, 2) <= tau * (1 + 1e-12)
        np.testing.assert_allclose(np.sum((X - V) * V), tau * nuc(V), rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------- Procrustes (eq. 10)

def _random_stiefel(rng, I, R):
    q, r = np.linalg.qr(rng.standard_normal((I, R)))
    return q


@pytest.mark.parametrize("I,R", [(2, 1), (3, 1), (3, 2), (5, 2), (4, 3)])
def test_polar_solves_procrustes(I, R):
    """polar(G V^T) minimises ||U V - G||_F over St(I, R) (eqs. (9)-(10))."""
    rng = np.random.default_rng(10 * I + R)
    G = rng.standard_normal((I, 6))
    V = rng.standard_normal((R, 6))
    Us = polar(G @ V.T)
    assert np.allclose(Us.T @ Us, np.eye(R), atol=1e-13)
    best = np.linalg.norm(Us @ V - G)
    if (I, R) == (2, 1):
        for th in np.linspace(0, 2 * np.pi, 100001):
            u = np.array([[math.cos(th)], [math.sin(th)]])
            assert np.linalg.norm(u @ V - G) >= best - 1e-12
    for _ in range(5000):
        U = _random_stiefel(rng, I, R)
        assert np.linalg.norm(U @ V - G) >= best - 1e-12
    S = Us.T @ (G @ V.T)
    np.testing.assert_allclose(S, S.T, atol=1e-12)
    assert np.linalg.eigvalsh((S + S.T) / 2).min() >= -1e-12


# ---------------------------------------------------------------- invariants per iteration

def _check_invariants(st, tol_scale=1e-9):
    T = st.T
    N = st.N
    mu = st.last["mu"]
    G = st.last["G"]
    E_prev = st.last["E_prev"]
    Y_prev = st.last["Y_prev"]
    Tmax = max(1.0, float(np.abs(T).max()))
    # (S1): sum_n Y_n^{k+1} is a subgradient of ||E^{k+1}||_1.
    Ysum = sum(st.Y)
    on = st.E != 0
    atol = tol_scale * mu * Tmax * N + 1e-12
    assert np.all(np.abs(Ysum[on] - np.sign(st.E[on])) <= atol)
    assert np.all(np.abs(Ysum[~on]) <= 1 + atol)
    for n in range(N):
        U = st.U[n]
        R = st.ranks[n]
        # U_n on the Stiefel manifold
        np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-12)
        # (S3): U^T Yhat_(n) = mu (P - V) has spectral norm <= lambda_n, where
        # Yhat^{k+1} = Y^k + mu^k (T - fold(U^{k+1} V^{k+1}) - E^k)  (eq. (16)).
        Yhat = Y_prev[n] + mu * (T - st.Z[n] - E_prev)
        lhs = np.linalg.norm(U.T @ unfold(Yhat, n), 2)
        assert lhs <= st.lam[n] * (1 + 1e-9) + 1e-9
        # Z_n = fold(SVT(U U^T G_n)): the iterate depends on span(U) only.
        Zs, _ = svt(U @ (U.T @ G[n]), st.lam[n] / mu)
        np.testing.assert_allclose(fold(Zs, n, T.shape), st.Z[n], atol=1e-9 * Tmax)


@pytest.mark.parametrize("dims,ranks,mu0", [((6, 7, 8), (2, 3, 2), 1e-4), ((6, 7, 8), (2, 3, 2), 0.05),
                                            ((5, 4, 6, 3), (2, 2, 2, 2), 0.02)])
def test_invariants_every_iteration(dims, ranks, mu0):
    wl = workloads.tucker_workload("inv", dims, ranks, 0.1, 7, value_range=(-5, 5), scale="rms")
    st = pasd_init(wl.T, wl.ranks, mu0=mu0)
    for _ in range(60):
        pasd_iterate(st, 1)
        _check_invariants(st)


def test_procrustes_span_matches_eq10_when_full_rank():
    """range(G P^T) = range(G V^T) on iterations where V has full row rank."""
    wl = _small()
    st = pasd_init(wl.T, wl.ranks, mu0=0.05)
    checked = 0
    for _ in range(40):
        prevP, prevV, prevrank = st.P, st.V, list(st.rank)
        pasd_iterate(st, 1)
        if not prevrank or prevP[0] is None:
            continue
        for n in range(st.N):
            if prevrank[n] != st.ranks[n]:
                continue
            G = st.last["G"][n]
            A = polar(G @ prevV[n].T)
            B = st.U[n]
            cosines = np.linalg.svd(A.T @ B, compute_uv=False)
            assert cosines.min() >= 1 - 1e-9
            checked += 1
    assert checked > 20


# ---------------------------------------------------------------- basis invariance (QR vs polar)

def test_iterates_depend_on_span_only(monkeypatch):
    """Replacing the polar factor by any other orthonormal basis of the same
    span (QR with random column signs and a rotation) leaves Z, E, Y unchanged."""
    wl = _small(dims=(7, 6, 9), ranks=(3, 2, 3))
    ref = pasd_init(wl.T, wl.ranks, mu0=0.02)
    pasd_iterate(ref, 50)
    rng = np.random.default_rng(5)

    def qr_basis(M):
        q, _ = np.linalg.qr(M)
        W = _random_stiefel(rng, M.shape[1], M.shape[1])
        return q @ W

    monkeypatch.setattr(pasd_oracle, "polar", qr_basis)
    alt = pasd_init(wl.T, wl.ranks, mu0=0.02)
    pasd_iterate(alt, 50)
    for n in range(3):
        np.testing.assert_allclose(alt.Z[n], ref.Z[n], atol=1e-10)
        np.testing.assert_allclose(alt.Y[n], ref.Y[n], atol=1e-8)
    np.testing.assert_allclose(alt.E, ref.E, atol=1e-10)


# ---------------------------------------------------------------- special case R_n = I_n

@pytest.mark.parametrize("dims", [(4, 5, 3), (3, 3, 2, 2)])
def test_full_rank_reduces_to_eq2_admm(dims):
    rng = np.random.default_rng(11)
    T = rng.standard_normal(dims)
    T[rng.random(dims) < 0.15] += 8
    lam = default_lambdas(dims)
    iters = 40
    ref = horpca_admm(T, lam, iters, mu0=0.01)
    st = pasd_init(T, list(dims), lam=lam, mu0=0.01)
    for k in range(iters):
        pasd_iterate(st, 1)
        Zr, Er, Yr = ref[k]
        scale = max(1.0, float(np.abs(T).max()))
        for n in range(len(dims)):
            np.testing.assert_allclose(st.Z[n], Zr[n], atol=1e-12 * scale * (k + 1))
            np.testing.assert_allclose(st.Y[n], Yr[n], atol=1e-12 * scale * st.last["mu"] * (k + 1) + 1e-12)
        np.testing.assert_allclose(st.E, Er, atol=1e-12 * scale * (k + 1))


# ---------------------------------------------------------------- Theorem 1, recovery

def test_residual_reaches_tolerance():
    wl = _small(dims=(12, 10, 11), ranks=(2, 2, 2))
    X, E, st = pasd_solve(wl.T, wl.ranks, tol=1e-8, max_iter=1000)
    assert max(st.residual) < 1e-8
    assert st.k < 1000
    # the residual identity of the proof of Theorem 1: T - Z - E = (Y^{k+1} - Y^k) / mu^k
    mu = st.last["mu"]
    for n in range(st.N):
        lhs = st.T - st.Z[n] - st.E
        rhs = (st.Y[n] - st.last["Y_prev"][n]) / mu
        np.testing.assert_allclose(lhs, rhs, atol=1e-9)


def test_recovers_planted_c1():
    """Config c1 (50^3, rank 5, 10% U(-10, 10)): exact support and tiny RSE."""
    wl = workloads.make_config("c1")
    X, E, st = pasd_solve(wl.T, wl.ranks, tol=wl.tol, max_iter=wl.max_iter)
    rse = np.linalg.norm(X - wl.L) / np.linalg.norm(wl.L)
    assert rse < 1e-8
    np.testing.assert_array_equal(E != 0, wl.mask)
    assert st.rank == [5, 5, 5]


def test_default_lambda_rule():
    # Section 5.1: sqrt(max(I_n, prod_{j != n} I_j)) / N
    assert default_lambdas((50, 50, 50)) == pytest.approx([50 / 3] * 3)
    lam = default_lambdas((144, 176, 400))
    assert lam == pytest.approx([math.sqrt(176 * 400) / 3, math.sqrt(144 * 400) / 3,
                                 math.sqrt(144 * 176) / 3])
    assert default_lambdas((64,) * 4) == pytest.approx([128.0] * 4)
