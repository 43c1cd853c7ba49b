"""GPU parity for ranks beyond one 16-wide rank tile (R_n up to 64).

Such problems keep their rank-indexed factors in 16-column tiles: the
unfolding GEMMs and the GEMM-M reduction run once per tile, and the Gram,
Householder QR, Jacobi eigensolver, keep tie-break and fused pass take their
rank-wide variants.  The R_n = floor(1.2 r) surplus of Section 5.1 at the
Fig. 1 ranks (r up to 50) needs them.  Compared with the oracle on the same
seeded inputs after K iterations: X, E, Z_n to 1e-10 (FP64) / 1e-5 (FP32),
Y_n to 10x that, U_n U_n^T to 100x, and the SVT ranks exactly in FP64.
"""

import json
import os

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
    import paper_1712_09999_amd  # noqa: F401  (raises if the library is missing)


from paper_1712_09999_amd import pasd as P  # noqa: E402

TOL = {"fp64": 1e-10, "fp32": 1e-5}


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def _compare(st, s, precision, label):
    bar = TOL[precision]
    info = s.query()
    assert info.iterations == st.k
    X_o, E_o = pasd_output(st)
    errs = {"X": rel(s.export(P.Q_X).astype(np.float64), X_o),
            "E": rel(s.export(P.Q_E).astype(np.float64), E_o)}
    for n in range(st.T.ndim):
        errs[f"Z{n}"] = rel(s.export(P.Q_Z, n).astype(np.float64), st.Z[n])
        errs[f"Y{n}"] = rel(s.export(P.Q_Y, n).astype(np.float64), st.Y[n])
        U = s.export(P.Q_U, n)
        errs[f"UU{n}"] = rel(U @ U.T, st.U[n] @ st.U[n].T)
        if precision == "fp64":
            assert info.rank[n] == st.rank[n], (label, n, info.rank[n], st.rank[n])
    print(label, list(st.rank), {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        lim = bar * (10 if k.startswith("Y") else 1)
        if k.startswith("Y") and precision == "fp32":
            lim = 1e-3  # mu-scaled FP32 rounding of D and Z, as in the one-tile parity tests
        if k.startswith("UU"):
            lim = bar * 100
        assert v <= lim, (label, k, v)


# dims, Tucker rank of the planted part, R_n, corrupted fraction, iterations compared
CASES = [
    # two tiles in every mode (the last mode too), odd R_1: the Jacobi padding index
    ((40, 36, 34), (12, 12, 12), (18, 17, 20), 0.1, (2, 15, 40)),
    # R = 64 (four tiles), three tiles, and a narrow last mode
    ((70, 66, 64), (30, 30, 8), (64, 40, 10), 0.1, (2, 10, 25)),
    # a wide last mode (transposed factor, tile loop over R_N), ragged sizes
    ((23, 30, 61), (8, 12, 30), (9, 20, 37), 0.15, (2, 12, 30)),
    # I_n R_n = 16384, the largest QR workspace of the rank-wide kernels
    ((256, 20, 20), (40, 5, 5), (64, 6, 6), 0.05, (2, 10)),
    # order 4, Section 5.1's R = floor(1.2 r) at r = 15
    ((20, 20, 20, 20), (15, 15, 15, 15), (18, 18, 18, 18), 0.1, (2, 12, 30)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])) + "-R" + "-".join(map(str, c[2])))
def test_wide_rank_fp64_trajectory(case):
    dims, core, ranks, frac, checks = case
    wl = workloads.tucker_workload("wide", dims, core, frac, 17124000 + sum(dims), ranks=ranks)
    st = pasd_init(wl.T, wl.ranks)
    s = P.Solver(wl.T, wl.ranks, precision="fp64", tol=0.0, max_iter=100000)
    done = 0
    for K in checks:
        print(f"case {dims} R={ranks} k={K}", flush=True)
        pasd_iterate(st, K - done)
        s.step(K - done)
        done = K
        _compare(st, s, "fp64", f"{dims}/R={ranks} k={K}")


def test_wide_rank_fp32_trajectory():
    dims, core, ranks = (40, 36, 34), (12, 12, 12), (18, 17, 20)
    wl = workloads.tucker_workload("wide32", dims, core, 0.1, 17124200, ranks=ranks)
    T32 = wl.observed(np.float32).astype(np.float64)
    st = pasd_init(T32, ranks)
    s = P.Solver(T32.astype(np.float32), ranks, precision="fp32", tol=0.0, max_iter=100000)
    done = 0
    for K in (3, 20, 40):
        pasd_iterate(st, K - done)
        s.step(K - done)
        done = K
        _compare(st, s, "fp32", f"fp32 {dims}/R={ranks} k={K}")


def test_wide_rank_keep_tiebreak_fp64():
    # surplus rank: V_n stays rank deficient, so the two tie-break candidates differ
    dims, core, ranks = (40, 36, 34), (6, 6, 6), (20, 18, 17)
    wl = workloads.tucker_workload("widekeep", dims, core, 0.1, 17124300, value_range=(-5, 5),
                                   scale="rms", ranks=ranks)
    T = wl.observed()
    st = pasd_init(T, ranks, mu0=0.01, tiebreak="keep")
    s = P.Solver(T, ranks, precision="fp64", tol=0.0, max_iter=100000, mu0=0.01, tiebreak="keep")
    done = 0
    for K in (2, 15, 30):
        pasd_iterate(st, K - done)
        s.step(K - done)
        done = K
        _compare(st, s, "fp64", f"keep {dims}/R={ranks} k={K}")
    assert min(st.rank) < min(ranks)


def test_wide_rank_batch_matches_single():
    # a batch mixing one-tile and rank-wide problems: every problem as alone
    specs = [((40, 36, 34), (12, 12, 12), (18, 17, 20)),
             ((30, 32, 28), (5, 5, 5), (6, 6, 6)),
             ((70, 66, 64), (30, 30, 8), (64, 40, 10)),
             ((24, 40, 36), (4, 10, 10), (5, 12, 12))]
    Ts = [workloads.tucker_workload("b", d, c, 0.1, 17124400 + k, ranks=r).T
          for k, (d, c, r) in enumerate(specs)]
    batch = [P.Solver(T, r, precision="fp64", tol=0.0, max_iter=100000)
             for T, (_, _, r) in zip(Ts, specs)]
    P.step_batch(batch, 12)
    for T, (d, c, r), sb in zip(Ts, specs, batch):
        alone = P.Solver(T, r, precision="fp64", tol=0.0, max_iter=100000)
        alone.step(12)
        assert sb.query().iterations == 12
        for q in (P.Q_X, P.Q_E):
            e = rel(sb.export(q), alone.export(q))
            assert e <= 1e-12, (d, r, q, e)


def test_wide_rank_checkpoint_restore_continues_bitwise():
    dims, core, ranks = (40, 36, 34), (12, 12, 12), (18, 17, 20)
    wl = workloads.tucker_workload("wideck", dims, core, 0.1, 17124500, ranks=ranks)
    for tb in ("pre", "keep"):
        a = P.Solver(wl.T, ranks, precision="fp64", tol=0.0, max_iter=100000, tiebreak=tb)
        a.step(17)
        ck = a.checkpoint()
        a.step(9)
        b = P.Solver(wl.T, ranks, precision="fp64", tol=0.0, max_iter=100000, tiebreak=tb)
        b.restore(ck)
        b.step(9)
        np.testing.assert_array_equal(b.export(P.Q_D), a.export(P.Q_D))
        for n in range(3):
            np.testing.assert_array_equal(b.export(P.Q_Y, n), a.export(P.Q_Y, n))
            np.testing.assert_array_equal(b.export(P.Q_U, n), a.export(P.Q_U, n))


FIG1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fig1_points.json")))


@pytest.mark.parametrize("pt", FIG1["points"], ids=lambda p: f"r{p['r']}-rho{p['rho']}")
def test_wide_rank_fig1_points_match_oracle(pt):
    # full FP64 solves at two Fig. 1 settings (Section 5.1), each against the
    # oracle's own full solve (tests/golden/make_fig1_points.py): r = 20 is
    # recovered (RSE <= 1e-3, the paper's success test), r = 40 (R = 48, rank
    # ratio 0.4) is not, on both sides
    r, R = pt["r"], pt["R"]
    wl = workloads.tucker_workload("fig1", tuple(FIG1["dims"]), (r, r, r), pt["rho"], pt["seed"],
                                   ranks=(R, R, R))
    s = P.Solver(wl.T, wl.ranks, precision="fp64", tol=FIG1["tol"], max_iter=FIG1["max_iter"])
    info = s.solve()
    rse = rel(s.export(P.Q_X), wl.L)
    print(f"fig1 r={r} rho={pt['rho']}: k={info.iterations} (oracle {pt['iterations']}) "
          f"rank={list(info.rank[:3])} (oracle {pt['rank']}) RSE={rse:.3e} (oracle {pt['rse']:.3e})",
          flush=True)
    assert info.converged == 1
    assert abs(info.iterations - pt["iterations"]) <= 1
    assert list(info.rank[:3]) == pt["rank"]
    assert (rse <= 1e-3) == (pt["rse"] <= 1e-3)
    assert abs(rse - pt["rse"]) <= 1e-6 + 1e-3 * pt["rse"]


def test_wide_rank_rank_deficient_m_fp64():
    # An exactly rank-3 tensor without corruption and R_n = 20: M_n = G_n P_n^T
    # is numerically rank deficient, the CholeskyQR2 pivots fail and the
    # Householder QR completes the basis.  With the default tie-break the
    # completion is not determined (reading R1: the Procrustes maximiser is not
    # unique while V_n is rank deficient), so the oracle's and this path's
    # iterates differ once it matters; what holds for any completion is checked:
    # U_n orthonormal, the SVT ranks reaching the planted rank, and recovery.
    dims, core, ranks = (40, 36, 34), (3, 3, 3), (20, 18, 17)
    wl = workloads.tucker_workload("widedef", dims, core, 0.0, 17124700, scale="rms", ranks=ranks)
    s = P.Solver(wl.T, ranks, precision="fp64", tol=1e-9, max_iter=2000, mu0=0.01)
    for K in (2, 10, 25):
        s.step(K - s.query().iterations)
        orth = max(float(np.abs(s.export(P.Q_U, n).T @ s.export(P.Q_U, n) - np.eye(ranks[n])).max())
                   for n in range(3))
        print(f"rank-deficient M k={K}: orth {orth:.2e} rank {list(s.query().rank[:3])}", flush=True)
        assert orth <= 1e-12
    info = s.solve()
    rse = rel(s.export(P.Q_X), wl.L)
    print(f"rank-deficient M: k={info.iterations} converged={info.converged} "
          f"rank={list(info.rank[:3])} RSE={rse:.2e}", flush=True)
    assert info.converged == 1 and list(info.rank[:3]) == [3, 3, 3]
    assert rse <= 1e-8
