"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Each case runs both sides on the same seeded input for the same number of
iterations (the GPU with tol = 0 so that it cannot stop early) and compares
the basis-free iterates: the low-rank copies Z_n, the sparse part E, the
multipliers Y_n, the output X and the projectors U_n U_n^T.  (U_n and P_n
themselves are unique only up to a rotation.)

Tolerances (relative Frobenius error): 1e-10 in FP64 and 1e-5 in FP32 for X
and E, the bars of the specification; Z_n use the same bar; Y_n, whose
entries are O(1) sums of mu-scaled residuals, use 10x the bar.
"""

import math

import numpy as np
import pytest

import workloads
from oracle import pasd_init, pasd_iterate, pasd_output, pasd_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_09999_amd  # noqa: F401  (raises if the library is missing)


from paper_1712_09999_amd import pasd as P  # noqa: E402

from parity_util import TOL, _compare, _gpu, rel  # noqa: E402


# --------------------------------------------------------------------------- c1 trajectory

def test_c1_fp64_trajectory():
    wl = workloads.make_config("c1")
    st = pasd_init(wl.T, wl.ranks)
    s = _gpu(wl.T, wl.ranks, "fp64")
    done = 0
    for K in [1, 2, 5, 40, 70, 100, 149]:
        pasd_iterate(st, K - done)
        s.step(K - done)
        done = K
        _compare(st, s, "fp64", f"c1 k={K}")


def test_c1_fp64_solve_matches_oracle_and_recovers_support():
    wl = workloads.make_config("c1")
    X_o, E_o, st = pasd_solve(wl.T, wl.ranks, tol=wl.tol, max_iter=wl.max_iter)
    s = _gpu(wl.T, wl.ranks, "fp64", tol=wl.tol, max_iter=wl.max_iter)
    info = s.solve()
    assert info.iterations == st.k and info.converged == 1
    X_g, E_g = (t.cpu().numpy() for t in s.result())
    assert rel(X_g, X_o) <= 1e-10 and rel(E_g, E_o) <= 1e-10
    np.testing.assert_array_equal(E_g != 0, wl.mask)
    assert rel(X_g, wl.L) < 1e-8
    for n in range(3):
        assert abs(info.residual[n] - st.residual[n]) <= 1e-12 + 1e-6 * st.residual[n]


def test_c1_fp32_trajectory():
    wl = workloads.make_config("c1")
    T32 = wl.observed(np.float32).astype(np.float64)
    st = pasd_init(T32, wl.ranks)
    s = _gpu(T32, wl.ranks, "fp32")
    done = 0
    for K in [3, 70, 149]:
        pasd_iterate(st, K - done)
        s.step(K - done)
        done = K
        _compare(st, s, "fp32", f"c1/fp32 k={K}")


# --------------------------------------------------------------------------- shapes and edge cases

SHAPES = [
    # (dims, ranks, mu0, iters)  ragged sizes, 2-way, 4-way, R = 1, R = I, R = 16
    ((23, 17, 19), (3, 2, 4), 0.01, 40),
    ((40, 37), (3, 3), 0.01, 50),
    ((8, 12, 16, 20), (2, 3, 2, 3), 0.01, 30),
    ((30, 20, 12), (1, 1, 1), 0.01, 40),
    ((6, 5, 4), (6, 5, 4), 0.01, 30),
    ((32, 24, 20), (16, 16, 16), 0.05, 25),
    ((130, 9, 70), (5, 4, 6), 0.002, 40),
    ((300, 10, 8), (6, 3, 3), 0.01, 25),     # QR in registers with 5 rows per lane
    ((600, 12, 10), (12, 4, 4), 0.01, 20),   # QR falls back to the LDS kernel
    # last mode contiguous with a partial final 16-row tile narrower than R
    # (A_N mod 16 < R_N): rows past A must be masked in the row operand only
    ((7, 5, 20), (3, 3, 8), 0.01, 30),
    ((111, 41, 36), (7, 14, 8), 0.01, 20),
    # tall modes (I_n R_n > 8192): the block-wide CholeskyQR2 on M_n in global
    # memory, and the eigensolver reading U_n from global memory
    ((1000, 12, 10), (10, 4, 4), 0.01, 25),
    ((2100, 8, 6), (16, 4, 3), 0.01, 12),
    # last two modes 64 x 64: their GEMM-P as one pass over the slabs, with a
    # partial last block (5 slabs, blocks of 4) and R_N = 16
    ((5, 64, 64), (3, 5, 7), 0.01, 25),
    ((2, 3, 64, 64), (2, 3, 11, 16), 0.01, 15),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,ranks,mu0,iters", SHAPES)
def test_shapes(dims, ranks, mu0, iters, precision):
    core = tuple(min(r, 3) for r in ranks)
    wl = workloads.tucker_workload("shape", dims, core, 0.08, 1234 + sum(dims),
                                   value_range=(-5, 5), scale="rms")
    T = wl.observed(np.float32 if precision == "fp32" else np.float64).astype(np.float64)
    st = pasd_init(T, ranks, mu0=mu0)
    pasd_iterate(st, iters)
    s = _gpu(T, ranks, precision, mu0=mu0)
    s.step(iters)
    # the last two modes' GEMM-P as one pass exactly where the plan says
    pair = len(dims) >= 3 and dims[-1] == dims[-2] == 64 and max(ranks) <= 16
    assert s.query().gemm_p_pair == int(pair)
    _compare(st, s, precision, f"{dims}/{ranks}/{precision}")


def _random_case(seed):
    """A seeded random problem: order 2-4, dimensions 3..48 (3..16 for order
    4; every other one a multiple of 4, so that both the scalar and the vector
    paths of the last mode and both GEMM schemes with partial tiles appear),
    Tucker-feasible ranks up to min(16, I_n), planted with the same ranks."""
    rng = np.random.default_rng(900_000 + seed)
    N = 2 + seed % 3
    while True:
        dims = []
        for n in range(N):
            d = int(rng.integers(3, 49 if N < 4 else 17))
            if (seed + n) % 2 == 0:
                d = max(4, d // 4 * 4)
            dims.append(d)
        if int(np.prod(dims)) <= 40_000:
            break
        if N > 2:
            N -= 1
    ranks = [int(rng.integers(1, min(16, d) + 1)) for d in dims]
    for _ in range(8):  # Tucker feasibility: r_n <= prod_{m != n} r_m
        for n in range(N):
            others = int(np.prod([ranks[m] for m in range(N) if m != n]))
            ranks[n] = min(ranks[n], others)
    return tuple(dims), tuple(ranks)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("seed", range(16))
def test_random_shapes(seed, precision):
    dims, ranks = _random_case(seed)
    wl = workloads.tucker_workload("rand", dims, ranks, 0.08, 4321 + seed,
                                   value_range=(-5, 5), scale="rms", ranks=ranks)
    T = wl.observed(np.float32 if precision == "fp32" else np.float64).astype(np.float64)
    mu0 = 0.02
    st = pasd_init(T, ranks, mu0=mu0)
    pasd_iterate(st, 20)
    s = _gpu(T, ranks, precision, mu0=mu0)
    s.step(20)
    _compare(st, s, precision, f"random {seed}: {dims}/{ranks}/{precision}")


# --------------------------------------------------------------------------- full size (200^3)

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c2_full_size_short_schedule(precision):
    """200^3, R = 10 (the benchmarked shape and launch configuration) with a
    larger initial penalty so that the thresholds bite within a few
    iterations; compared iterate by iterate after 6 iterations."""
    wl = workloads.make_config("c2")
    T = wl.observed(np.float32 if precision == "fp32" else np.float64).astype(np.float64)
    st = pasd_init(T, wl.ranks, mu0=0.3)
    pasd_iterate(st, 6)
    assert min(st.rank) > 0  # the SVT is active, not the trivial V = 0 phase
    s = _gpu(T, wl.ranks, precision, mu0=0.3)
    s.step(6)
    _compare(st, s, precision, f"c2/{precision} k=6")


@pytest.mark.parametrize("name,mu0", [("c3", 0.1), ("c4", 1.0)])
def test_full_size_video_and_four_way(name, mu0):
    """144 x 176 x 400 video-shaped (R = (8, 8, 3)) and 64^4 (R = 6) in FP32,
    with an initial penalty large enough for the SVT to act within 6 steps."""
    wl = workloads.make_config(name)
    T = wl.observed(np.float32).astype(np.float64)
    st = pasd_init(T, wl.ranks, mu0=mu0)
    pasd_iterate(st, 6)
    assert min(st.rank) > 0
    s = _gpu(T, wl.ranks, "fp32", mu0=mu0)
    s.step(6)
    _compare(st, s, "fp32", f"{name}/fp32 k=6")


# --------------------------------------------------------------------------- runtime behaviour

def test_checkpoint_restore_is_bitwise():
    wl = workloads.make_config("c1")
    a = _gpu(wl.T, wl.ranks, "fp64")
    a.step(60)
    ck = a.checkpoint()
    a.step(25)
    Xa = a.export(P.Q_X)
    b = _gpu(wl.T, wl.ranks, "fp64")
    b.restore(ck)
    b.step(25)
    np.testing.assert_array_equal(b.export(P.Q_X), Xa)
    np.testing.assert_array_equal(b.export(P.Q_E), a.export(P.Q_E))


# 4-way with a mode-1 slab of 4096 (FP64) or 2048 (FP32) chunks: the fused pass folds in the
# GEMM-M of modes 0 and 1 (blocks of 1024 chunks, several per slab), with the last mode's
# columns kept per thread and, in FP64, mode 2's U W rows and the last mode's P columns
# staged in LDS and the GEMM-M of modes 2 and 3 accumulated too (rows of 64 chunks: lane
# groups of a whole wave; 16 rows per block, so every block holds a quarter of the i_2 rows)
MERGED = ((3, 4, 64, 128), (3, 4, 3, 3))
# (dims, ranks, merged modes in FP64, in FP32)
MERGED_SHAPES = [
    (MERGED, 4, 2),
    # FP64: rows of 48 chunks (the last mode's columns reloaded per chunk, modes 2 and 3
    # left to GEMM-M); FP32: a slab of 960 chunks, not merged
    (((2, 3, 40, 96), (2, 3, 3, 4)), 2, 0),
    # FP64: 300 rows per block, more than the LDS stage holds
    (((2, 2, 300, 8), (2, 2, 4, 3)), 2, 0),
    # rank 10: the largest rank merged with an FP32 state; FP64 folds only modes 0 and 1
    (((2, 3, 64, 64), (2, 3, 10, 10)), 2, 2),
    # every mode in FP64 at rank 6 (one block per slab, 32 rows), rows of 16 chunks
    # (lane groups of a quarter wave), and of 8 chunks with 128 rows, the most the stage
    # holds; in FP32 these slabs hold 512 chunks, not merged
    (((4, 4, 32, 64), (4, 4, 6, 6)), 4, 0),
    (((3, 2, 64, 32), (3, 2, 5, 4)), 4, 0),
    (((2, 2, 128, 16), (2, 2, 6, 5)), 4, 0),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,m64,m32", MERGED_SHAPES)
def test_merged_gemm_m_trajectory(shape, m64, m32, precision):
    dims, ranks = shape
    wl = workloads.tucker_workload("merged", dims, tuple(min(r, 3) for r in ranks), 0.1, 17125100,
                                   value_range=(-5, 5), scale="rms")
    T = wl.observed(np.float32 if precision == "fp32" else np.float64).astype(np.float64)
    st = pasd_init(T, ranks, mu0=0.01)
    s = _gpu(T, ranks, precision, mu0=0.01)
    assert s.query().merged_modes == (m64 if precision == "fp64" else m32), (dims, precision)
    done = 0
    for K in (1, 2, 15, 40):
        pasd_iterate(st, K - done)
        s.step(K - done)
        done = K
        _compare(st, s, precision, f"merged {dims}/{ranks}/{precision} k={K}")


def test_merge_plan_limits():
    """Order-4 problems fold GEMM-M of modes 0 and 1 into the fused pass only
    where that was measured faster: slabs of at least 1024 chunks, and ranks up
    to 10 with an FP32 state (16 with FP64); modes 2 and 3 too with an FP64
    state up to rank 6."""
    T = np.zeros((2, 3, 64, 64))
    for prec, R, want in (("fp64", 16, 2), ("fp64", 7, 2), ("fp64", 6, 4), ("fp32", 6, 2),
                          ("fp32", 10, 2), ("fp32", 12, 0)):
        with P.Solver(T, (2, 3, R, R), precision=prec, tol=0.0, max_iter=10) as s:
            assert s.query().merged_modes == want, (prec, R)
    with P.Solver(np.zeros((32, 48, 40, 56)), (4, 4, 4, 4), precision="fp32", tol=0.0,
                  max_iter=10) as s:
        assert s.query().merged_modes == 0


def test_merged_batch_equals_alone():
    """Problems that fold every mode, two modes and none stepped in one batch
    give the iterates they give alone, bitwise (each keeps its own kernels,
    blocks and reduction order)."""
    specs = [((4, 4, 32, 64), (4, 4, 6, 6)), ((3, 4, 64, 128), (3, 4, 3, 3)),
             ((2, 3, 64, 64), (2, 3, 10, 10)), ((20, 18, 16), (3, 4, 5))]
    alone, mixed = [], []
    for k, (dims, ranks) in enumerate(specs):
        wl = workloads.tucker_workload("mix", dims, tuple(min(r, 3) for r in ranks), 0.1,
                                       17125300 + k, value_range=(-5, 5), scale="rms")
        T = wl.observed(np.float64)
        a = _gpu(T, ranks, "fp64", mu0=0.01)
        a.step(23)
        alone.append(a)
        mixed.append(_gpu(T, ranks, "fp64", mu0=0.01))
    assert [m.query().merged_modes for m in mixed] == [4, 4, 2, 0]
    assert [m.query().gemm_p_pair for m in mixed] == [0, 0, 1, 0]
    for _ in range(3):
        P.step_batch(mixed, 7)
    P.step_batch(mixed, 2)
    for a, b in zip(alone, mixed):
        np.testing.assert_array_equal(a.export(P.Q_D), b.export(P.Q_D))
        np.testing.assert_array_equal(a.export(P.Q_X), b.export(P.Q_X))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_merged_checkpoint_restore_is_bitwise(precision):
    # the restore does not carry the fused pass's GEMM-M partials of the merged
    # modes; they are recomputed from the restored iterate before it continues
    dims, ranks = MERGED
    wl = workloads.tucker_workload("merged", dims, (3, 3, 3, 3), 0.1, 17125100,
                                   value_range=(-5, 5), scale="rms")
    T = wl.observed(np.float32 if precision == "fp32" else np.float64)
    a = _gpu(T, ranks, precision, mu0=0.01)
    a.step(30)
    ck = a.checkpoint()
    a.step(20)
    b = _gpu(T, ranks, precision, mu0=0.01)
    b.step(3)  # a different state before the restore
    b.restore(ck)
    b.step(20)
    np.testing.assert_array_equal(b.export(P.Q_D), a.export(P.Q_D))
    for n in range(4):
        np.testing.assert_array_equal(b.export(P.Q_Y, n), a.export(P.Q_Y, n))


def test_runs_are_bitwise_reproducible():
    wl = workloads.make_config("c1")
    outs = []
    for _ in range(2):
        s = _gpu(wl.T, wl.ranks, "fp64")
        s.step(90)
        outs.append((s.export(P.Q_X), s.export(P.Q_E), s.export(P.Q_Y, 1)))
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_graph_replays_match_direct_launches():
    """Iterations replayed from the captured HIP graph (several replays, with
    eager work and synchronisation in between) equal direct launches bitwise."""
    wl = workloads.make_config("c1")
    a = _gpu(wl.T, wl.ranks, "fp64", graphs=True)
    b = _gpu(wl.T, wl.ranks, "fp64", graphs=False)
    for chunk in (16, 32, 16, 48):
        a.step(chunk)
        b.step(chunk)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.export(P.Q_D), b.export(P.Q_D))
        np.testing.assert_array_equal(a.export(P.Q_Y, 2), b.export(P.Q_Y, 2))
    assert a.query().iterations == b.query().iterations == 112


def test_reset_restarts_from_initialisation():
    wl = workloads.make_config("c1")
    s = _gpu(wl.T, wl.ranks, "fp64")
    s.step(30)
    X1 = s.export(P.Q_X)
    s.step(10)
    s.reset()
    s.step(30)
    np.testing.assert_array_equal(s.export(P.Q_X), X1)
    assert s.query().iterations == 30


def test_max_iter_and_not_converged():
    wl = workloads.make_config("c1")
    s = _gpu(wl.T, wl.ranks, "fp64", tol=1e-30, max_iter=17)
    info = s.solve()
    assert info.iterations == 17 and info.done == 2 and info.converged == 0
    s.step(5)  # skipped on the device
    assert s.query().iterations == 17


def test_nan_input_reports_numeric_error():
    T = np.random.default_rng(0).standard_normal((12, 10, 8))
    T[3, 4, 5] = np.nan
    s = _gpu(T, (2, 2, 2), "fp64", tol=1e-8, max_iter=50)
    with pytest.raises(P.PasdError) as ei:
        s.solve()
    assert ei.value.code == P.ERR_NUMERIC
    assert s.query().done == 3


# --------------------------------------------------------------------------- weights and the penalty cap

def test_unequal_output_weights_on_a_non_cube():
    """alpha_n of the output X = sum alpha_n Z_n / sum alpha_n (reading:
    alpha_n = lambda_n by default) passed explicitly and unequal on a
    non-cubic tensor, where the copies Z_n differ before convergence: a wrong
    weighting of the output is visible at 1e-10."""
    wl = workloads.tucker_workload("alpha", (30, 22, 14), (3, 4, 2), 0.08, 4711,
                                   value_range=(-5, 5), scale="rms")
    alpha = (0.5, 2.0, 7.0)
    lam = (3.0, 2.5, 4.0)
    st = pasd_init(wl.T, wl.ranks, lam=lam, alpha=alpha, mu0=0.01)
    pasd_iterate(st, 25)
    s = _gpu(wl.T, wl.ranks, "fp64", lam=lam, alpha=alpha, mu0=0.01)
    s.step(25)
    errs = _compare(st, s, "fp64", "alpha/lambda explicit k=25")
    # the weighting matters here: the equal-weight mean differs from X
    X_eq = sum(st.Z) / 3.0
    X_o, _ = pasd_output(st)
    assert rel(X_eq, X_o) > 1e-6
    assert errs["X"] <= 1e-10


def test_penalty_cap_binds():
    """mu = min(rho mu, mu_max) (Algorithm 1, line 7) with a cap reached after
    a few iterations (mu0 = 0.5, mu_max = 2, rho = 1.5): both sides run 30
    iterations at the cap; a wrong cap or an update order that skips it would
    change the multipliers, the shrinkage threshold and the SVT threshold."""
    wl = workloads.tucker_workload("cap", (26, 20, 18), (3, 3, 3), 0.1, 4712,
                                   value_range=(-5, 5), scale="rms")
    kw = dict(mu0=0.5, mu_max=2.0, rho=1.5)
    st = pasd_init(wl.T, wl.ranks, **kw)
    pasd_iterate(st, 30)
    assert st.mu == 2.0
    s = _gpu(wl.T, wl.ranks, "fp64", **kw)
    s.step(30)
    assert float(s.export(P.Q_SCALARS)[1]) == 2.0
    _compare(st, s, "fp64", "mu_max binds k=30")


def test_tall_mode_rank_deficient_m_fp64():
    # An exactly rank-3 tensor without corruption and a tall first mode with
    # R_0 = 12 (I_0 R_0 = 10800): M_0 = G_0 P_0^T is numerically rank
    # deficient, the tall kernel's CholeskyQR2 pivots fail and its Householder
    # QR completes the basis.  The completion is not determined (reading R1),
    # so what holds for any completion is checked: U_n orthonormal, the SVT
    # ranks reaching the planted rank, and recovery (the oracle's own solve of
    # this tensor takes 58 iterations to ranks (3, 3, 3) and RSE 1.5e-12).
    dims, core, ranks = (900, 24, 20), (3, 3, 3), (12, 8, 8)
    wl = workloads.tucker_workload("talldef", dims, core, 0.0, 17124800, scale="rms", ranks=ranks)
    s = P.Solver(wl.T, ranks, precision="fp64", tol=1e-9, max_iter=2000, mu0=0.01)
    for K in (2, 10, 25):
        s.step(K - s.query().iterations)
        orth = max(float(np.abs(s.export(P.Q_U, n).T @ s.export(P.Q_U, n) - np.eye(ranks[n])).max())
                   for n in range(3))
        print(f"tall rank-deficient M k={K}: orth {orth:.2e} rank {list(s.query().rank[:3])}",
              flush=True)
        assert orth <= 1e-12
    info = s.solve()
    rse = rel(s.export(P.Q_X), wl.L)
    print(f"tall rank-deficient M: k={info.iterations} converged={info.converged} "
          f"rank={list(info.rank[:3])} RSE={rse:.2e}", flush=True)
    assert info.converged == 1 and list(info.rank[:3]) == [3, 3, 3]
    assert rse <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,ranks", [((3, 64, 64), (3, 5, 7)), ((2, 3, 64, 64), (2, 3, 6, 16))])
def test_gemm_p_pair_places_every_entry(dims, ranks, precision):
    """First iteration (U_n = the leading columns of the identity, Y_n = 0,
    D = T): every entry of P_n = U_n^T G_n is one product 1 * t plus exact
    zeros, so P_n must equal the leading R_n rows of each unfolding bitwise,
    also for the last two modes, which GEMM-P takes in one pass over their
    64 x 64 slabs."""
    dt = np.float64 if precision == "fp64" else np.float32
    T = (np.random.default_rng(77).standard_normal(dims) * 3.0).astype(dt)
    with P.Solver(T, ranks, precision=precision, tol=0.0, max_iter=1000) as s:
        s.step(1)
        assert s.query().gemm_p_pair == 1
        for n, R in enumerate(ranks):
            A = int(np.prod(dims[:n]))
            B = int(np.prod(dims[n + 1:]))
            want = T.reshape(A, dims[n], B).transpose(1, 0, 2).reshape(dims[n], A * B)[:R]
            got = s.export(P.Q_P, n)
            assert got.dtype == dt and got.shape == want.shape, n
            assert np.array_equal(got, want), n
