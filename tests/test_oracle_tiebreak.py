"""Pins for the oracle's alternative Procrustes tie-break (reading R1').

Eq. (10) maximises <U, G V^T> over column-orthonormal U.  When V is rank
deficient the maximiser is not unique; the "keep" tie-break takes, on the null
space of G V^T, the orthonormal completion nearest the previous U.  The pins:
it is a maximiser (trace equals the nuclear norm), it is nearest the previous U
among maximisers (brute force over the completions of a rank-one A), it is the
limit of polar(A + eps U_prev), it reduces to the polar factor at full rank and
to U_prev at A = 0, and the whole iteration agrees with the default tie-break
whenever every V_n keeps full rank.
"""

import numpy as np
import pytest

import workloads
from oracle import pasd_init, pasd_iterate, pasd_output, polar, procrustes_keep


def _orth(rng, m, k):
    return np.linalg.qr(rng.standard_normal((m, k)))[0]


def _rank_r(rng, m, n, r):
    return rng.standard_normal((m, r)) @ rng.standard_normal((r, n))


@pytest.mark.parametrize("m,R,r", [(6, 3, 1), (7, 4, 2), (9, 5, 3), (5, 2, 0)])
def test_keep_is_a_maximiser(m, R, r):
    rng = np.random.default_rng(10 + m + R + r)
    A = _rank_r(rng, m, R, r) if r else np.zeros((m, R))
    U_prev = _orth(rng, m, R)
    U = procrustes_keep(A, r, U_prev)
    np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-13)
    # <U, A> equals the nuclear norm of A, the maximum of eq. (10)
    assert abs(np.trace(U.T @ A) - np.linalg.svd(A, compute_uv=False).sum()) < 1e-12 * (1 + abs(A).sum())


def test_keep_is_nearest_completion_brute_force():
    # rank-one A in R^{4 x 2}: the maximisers are a1 b1^T + c b2^T with c a unit
    # vector orthogonal to a1 (a 2-sphere); search it on a fine grid
    rng = np.random.default_rng(5)
    a1 = rng.standard_normal(4)
    a1 /= np.linalg.norm(a1)
    b = _orth(rng, 2, 2)
    A = 3.0 * np.outer(a1, b[:, 0])
    U_prev = _orth(rng, 4, 2)
    U = procrustes_keep(A, 1, U_prev)
    best = np.linalg.norm(U - U_prev)
    Q = np.linalg.qr(np.column_stack([a1, rng.standard_normal((4, 3))]))[0][:, 1:]  # basis of a1-perp
    th = np.linspace(0.0, np.pi, 181)
    ph = np.linspace(0.0, 2 * np.pi, 361)
    T, P = np.meshgrid(th, ph, indexing="ij")
    C = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1) @ Q.T
    a1b1 = np.outer(a1, b[:, 0])
    cand = a1b1[None, None] + C[..., :, None] * b[:, 1][None, None, None, :]
    dist = np.linalg.norm((cand - U_prev).reshape(*T.shape, -1), axis=-1)
    assert dist.min() >= best - 1e-12            # no sampled maximiser is nearer
    assert dist.min() - best < 2e-4              # and the grid comes close to it
    assert abs(np.trace(U.T @ A) - 3.0) < 1e-12


@pytest.mark.parametrize("m,R,r", [(8, 3, 1), (10, 4, 2)])
def test_keep_is_the_limit_of_a_perturbed_polar(m, R, r):
    rng = np.random.default_rng(30 + m)
    A = _rank_r(rng, m, R, r)
    U_prev = _orth(rng, m, R)
    U = procrustes_keep(A, r, U_prev)
    errs = [np.linalg.norm(polar(A + eps * U_prev) - U) for eps in (1e-4, 1e-5, 1e-6)]
    assert errs[0] < 1e-2
    assert errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5   # first order in eps


def test_keep_full_rank_and_zero():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((7, 3))
    U_prev = _orth(rng, 7, 3)
    np.testing.assert_allclose(procrustes_keep(A, 3, U_prev), polar(A), atol=1e-13)
    np.testing.assert_allclose(procrustes_keep(np.zeros((7, 3)), 0, U_prev), U_prev, atol=1e-14)


def _case(dims=(6, 7, 8), ranks=(2, 3, 2), seed=3):
    return workloads.tucker_workload("small", dims, ranks, 0.1, seed, value_range=(-5, 5),
                                     scale="rms").observed()


def test_keep_agrees_with_default_while_v_has_full_rank():
    # a large mu0 makes tau = lambda / mu tiny: every V_n keeps full rank, and
    # both tie-breaks span the same subspace at every step
    T = _case()
    a = pasd_init(T, (2, 3, 2), mu0=1e3)
    b = pasd_init(T, (2, 3, 2), mu0=1e3, tiebreak="keep")
    for _ in range(12):
        pasd_iterate(a, 1)
        pasd_iterate(b, 1)
        assert a.rank == b.rank == [2, 3, 2]
    Xa, Ea = pasd_output(a)
    Xb, Eb = pasd_output(b)
    np.testing.assert_allclose(Xb, Xa, atol=1e-10 * np.abs(Xa).max())
    np.testing.assert_allclose(Eb, Ea, atol=1e-10 * (1 + np.abs(Ea).max()))


def test_keep_holds_u0_while_v_is_zero():
    # the default mu0 = 1e-4 gives tau far above every singular value at first:
    # V = 0, so the keep tie-break leaves U at U^0 = eye(I, R)
    T = _case()
    st = pasd_init(T, (2, 3, 2), tiebreak="keep")
    for _ in range(5):
        pasd_iterate(st, 1)
        assert st.rank == [0, 0, 0]
    for n, U in enumerate(st.U):
        np.testing.assert_array_equal(U, np.eye(T.shape[n], (2, 3, 2)[n]))
