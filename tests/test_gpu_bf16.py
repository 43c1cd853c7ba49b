"""Split-BF16 unfolding GEMMs (PASD_BF16_GEMM) on the GPU against the oracle.

In this mode every operand of GEMM-M and GEMM-P is split into three BF16
terms and the products run on the BF16 matrix cores with FP32 accumulation;
the state is FP32 and QR, the Gram, the eigensolver and the norms stay FP64.
The bar is the mixed-precision one, 1e-5 relative Frobenius error of X, E
and every Z_n against the FP64 oracle run on the same FP32-rounded input.
"""

import numpy as np
import pytest

import workloads
from oracle import pasd_init, pasd_iterate, pasd_output

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_1712_09999_amd import pasd as P  # noqa: E402
from parity_util import _compare, _gpu, rel  # noqa: E402

DIMS, RANKS = (20, 16, 12), (4, 3, 5)


def _tensor(seed=3, dims=DIMS):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(dims).astype(np.float32) * 3.0


def _unfold_cols(T, n):
    """Mode-n unfolding with the solver's column order j = a B + b."""
    A = int(np.prod(T.shape[:n]))
    B = int(np.prod(T.shape[n + 1:]))
    return T.reshape(A, T.shape[n], B).transpose(1, 0, 2).reshape(T.shape[n], A * B)


@pytest.mark.parametrize("dims,ranks", [(DIMS, RANKS), ((40, 36, 34), (20, 33, 17))])
def test_gemm_p_split_is_exact_for_single_terms(dims, ranks):
    """k = 0: U_n = eye, Y_n = 0, D = T, so every entry of P_n = U_n^T G_n is a
    single product 1 * g.  The three-term BF16 split of an FP32 value is exact
    (h1 + h2 + h3 = g), so P_n must equal the FP32 unfolding rows bitwise; with
    R_1 = 33 GEMM-P runs once per 16-wide rank tile and every tile's rows must
    land in their place."""
    T = _tensor(5, dims)
    with P.Solver(T, ranks, precision="bf16", tol=0.0, max_iter=1000) as s:
        s.step(1)
        for n, R in enumerate(ranks):
            Pn = s.export(P.Q_P, n)
            want = _unfold_cols(T, n)[:R]
            assert np.array_equal(Pn.view(np.uint32), want.view(np.uint32)), n


def _proj_dist(U, V):
    return float(np.linalg.norm(U @ U.T - V @ V.T))


def test_gemm_m_split_keeps_fp32_accuracy():
    """U_n after the second iteration spans range(G_n P_n^T) of the stored FP32
    operands to FP32 accuracy: the split products carry no BF16 rounding."""
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
            M = Gn.astype(np.float64) @ Pm[n].astype(np.float64).T
            Q = np.linalg.qr(M)[0]
            d = _proj_dist(s.export(P.Q_U, n), Q)
            assert d < 1e-5, (n, d)


def test_bf16_c1_trajectory_matches_oracle():
    """The 50^3 configuration from the initialisation (default mu0, so the
    V = 0 phase, the threshold crossings and the late iterations are all
    covered), iterate by iterate against the oracle at the 1e-5 bar."""
    wl = workloads.make_config("c1")
    T = wl.observed(np.float32).astype(np.float64)
    st = pasd_init(T, wl.ranks)
    s = _gpu(T, wl.ranks, "bf16")
    done = 0
    for K in [1, 5, 40, 70, 100, 149]:
        pasd_iterate(st, K - done)
        s.step(K - done)
        done = K
        _compare(st, s, "bf16", f"c1/bf16 k={K}")


def test_bf16_video_shaped_matches_oracle():
    """A half-size video-shaped tensor (72 x 88 x 100, background Tucker rank
    (8, 8, 3), moving blocks) with the default mu0 at k = 60 and k = 150."""
    wl = workloads.video_workload("v", dims=(72, 88, 100), bg_ranks=(8, 8, 3), blocks=3,
                                  seed=17120311)
    T = wl.observed(np.float32).astype(np.float64)
    st = pasd_init(T, wl.ranks)
    s = _gpu(T, wl.ranks, "bf16")
    done = 0
    for K in (60, 150):
        pasd_iterate(st, K - done)
        s.step(K - done)
        done = K
        _compare(st, s, "bf16", f"video/bf16 k={K}")


def test_bf16_solve_matches_oracle_and_stops_honestly():
    """c1 solved to tol 1e-6: the solve ends converged (Algorithm 1's test) or
    at the FP32 precision floor, never claiming convergence above tol; X and E
    match the oracle run for the same number of iterations at 1e-5."""
    wl = workloads.make_config("c1")
    T = wl.observed(np.float32).astype(np.float64)
    with P.Solver(T.astype(np.float32), wl.ranks, precision="bf16", tol=1e-6, max_iter=1000) as s:
        info = s.solve()
        X, E = (t.double().cpu().numpy() for t in s.result())
    r = max(info.residual[:3])
    assert info.done in (1, 4), info.done
    assert (info.converged == 1) == (r < 1e-6), (info.converged, r)
    if info.done == 4:
        assert r < info.tol_effective
    st = pasd_init(T, wl.ranks)
    pasd_iterate(st, info.iterations)
    X_o, E_o = pasd_output(st)
    ex, ee = rel(X, X_o), rel(E, E_o)
    print(f"c1 bf16 solve: k={info.iterations} done={info.done} residual {r:.2e} "
          f"X {ex:.2e} E {ee:.2e}", flush=True)
    assert ex <= 1e-5 and ee <= 1e-5, (ex, ee)
