"""BF16-input unfolding GEMMs (PASD_BF16_GEMM) on the GPU.

In this mode both operands of GEMM-M and GEMM-P are rounded to BF16 (round to
nearest, ties to even) and accumulated in FP32; the state is FP32 and QR, the
Gram, the eigensolver and the norms stay FP64.  The tests pin the rounding
exactly where the product has a single term, check that GEMM-M's subspace
follows the BF16-rounded operands, and bound the end-to-end error of a solve
against the FP64 path."""

import numpy as np
import pytest

import workloads
from bf16util import bf16_rne

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_1712_09999_amd import pasd as P  # noqa: E402

DIMS, RANKS = (20, 16, 12), (4, 3, 5)


def _tensor(seed=3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(DIMS).astype(np.float32) * 3.0


def _unfold_cols(T, n):
    """Mode-n unfolding with the solver's column order j = a B + b."""
    A = int(np.prod(T.shape[:n]))
    B = int(np.prod(T.shape[n + 1:]))
    return T.reshape(A, T.shape[n], B).transpose(1, 0, 2).reshape(T.shape[n], A * B)


def test_gemm_p_rounds_operands_to_bf16():
    """k = 0: U_n = eye, Y_n = 0, D = T, so P_n = U_n^T G_n has one term per
    entry and equals the BF16 rounding of the first R_n unfolding rows."""
    T = _tensor()
    with P.Solver(T, RANKS, precision="bf16", tol=0.0, max_iter=1000) as s:
        s.step(1)
        for n, R in enumerate(RANKS):
            Pn = s.export(P.Q_P, n)
            want = bf16_rne(_unfold_cols(T, n)[:R])
            assert np.array_equal(Pn.view(np.uint32), want.view(np.uint32)), n


def test_gemm_p_rounds_operands_to_bf16_rank_tiles():
    """The same pin for ranks above one 16-wide tile, where GEMM-P runs once
    per rank tile: every tile's rows land in their place of P_n (R_1 = 33:
    three tiles, the last one holding a single row)."""
    dims, ranks = (40, 36, 34), (20, 33, 17)
    T = (np.random.default_rng(5).standard_normal(dims) * 3.0).astype(np.float32)
    with P.Solver(T, ranks, precision="bf16", tol=0.0, max_iter=1000) as s:
        s.step(1)
        for n, R in enumerate(ranks):
            Pn = s.export(P.Q_P, n)
            want = bf16_rne(_unfold_cols(T, n)[:R])
            assert np.array_equal(Pn.view(np.uint32), want.view(np.uint32)), n


def _proj_dist(U, V):
    return float(np.linalg.norm(U @ U.T - V @ V.T))


def test_gemm_m_follows_bf16_operands():
    """U_n after the second iteration spans range(bf16(G_n) bf16(P_n)^T) with
    G_n = D + Y_n / mu formed in FP32, not the range of the unrounded product."""
    T = _tensor(4)
    with P.Solver(T, RANKS, precision="bf16", tol=0.0, max_iter=1000) as s:
        s.step(1)
        D = s.export(P.Q_D)
        mu = float(s.export(P.Q_SCALARS)[1])
        inv_mu = np.float32(1.0 / mu)
        G = {n: (D.astype(np.float64) + s.export(P.Q_Y, n).astype(np.float64) * np.float64(inv_mu))
             .astype(np.float32) for n in range(3)}
        Pm = {n: s.export(P.Q_P, n) for n in range(3)}
        s.step(1)
        for n, R in enumerate(RANKS):
            Gn = _unfold_cols(G[n], n)
            Mb = bf16_rne(Gn).astype(np.float64) @ bf16_rne(Pm[n]).astype(np.float64).T
            Mf = Gn.astype(np.float64) @ Pm[n].astype(np.float64).T
            Qb = np.linalg.qr(Mb)[0]
            Qf = np.linalg.qr(Mf)[0]
            U = s.export(P.Q_U, n)
            db, df = _proj_dist(U, Qb), _proj_dist(U, Qf)
            assert db < 1e-4 and db < 0.25 * df, (n, db, df)


def test_bf16_solve_error_vs_fp64():
    """c1-shaped solve: converges under the BF16 stopping level and stays
    within 2e-3 (X) and 1e-2 (E) of the FP64 solve in relative Frobenius
    error; the FP64 path is pinned to the oracle elsewhere."""
    wl = workloads.make_config("c1")
    T32 = wl.observed(np.float32)
    out = {}
    for prec, T in (("bf16", T32), ("fp64", T32.astype(np.float64))):
        with P.Solver(T, wl.ranks, precision=prec, tol=1e-6, max_iter=1000) as s:
            info = s.solve()
            assert info.converged, (prec, info.iterations)
            out[prec] = [np.asarray(v.double().cpu().numpy() if hasattr(v, "cpu") else v, dtype=np.float64)
                         for v in s.result()]
    ex = np.linalg.norm(out["bf16"][0] - out["fp64"][0]) / np.linalg.norm(out["fp64"][0])
    ee = np.linalg.norm(out["bf16"][1] - out["fp64"][1]) / np.linalg.norm(out["fp64"][1])
    print("bf16 vs fp64: X", ex, "E", ee)
    assert ex < 2e-3 and ee < 1e-2, (ex, ee)
