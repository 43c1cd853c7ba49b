"""pasd_solve_static, the entry point that allocates nothing (its state lives
in the library's static device array), against the allocating path
pasd_create + pasd_solve + pasd_get_result on the same inputs: two calls in a
row, the second with a smaller tensor, in FP64 and FP32 (3-way) and for order-4
FP64 tensors whose fused pass folds in every mode's GEMM-M, plus the size
limit.

Both paths run the same kernels in the same order (the allocating one with
PASD_FLAG_NO_GRAPH here, so both launch directly), so iteration counts,
ranks and residuals must agree and X, E to the parity bars (1e-10 FP64,
1e-5 FP32); the test also reports whether they agree bitwise.
"""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_1712_09999_amd import pasd as P  # noqa: E402

BAR = {"fp64": 1e-10, "fp32": 1e-5}


def _rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def _case(dims, ranks, seed, precision):
    wl = workloads.tucker_workload(f"static{seed}", dims, ranks, 0.1, seed, value_range=(-5, 5),
                                   scale="rms")
    dt = torch.float64 if precision == "fp64" else torch.float32
    T = torch.from_numpy(wl.T).to(device="cuda", dtype=dt).contiguous()
    kw = dict(tol=1e-7 if precision == "fp64" else 1e-5, max_iter=400, precision=precision)
    # the allocating path
    with P.Solver(T, ranks, graphs=False, **kw) as s:
        info_a = s.solve()
        Xa, Ea = (t.double().cpu().numpy() for t in s.result())
    # the static path: caller-owned outputs, filled with garbage first
    X = torch.full_like(T, float("nan"))
    E = torch.full_like(T, float("nan"))
    code, info_s = P.solve_static(T, ranks, X, E, **kw)
    torch.cuda.synchronize()
    Xs, Es = X.double().cpu().numpy(), E.double().cpu().numpy()
    N = len(dims)
    ex, ee = _rel(Xs, Xa), _rel(Es, Ea)
    bitwise = bool(np.array_equal(Xs, Xa) and np.array_equal(Es, Ea))
    print(f"[static {precision} {dims} R={ranks}] code {code} k {info_s.iterations} "
          f"(alloc {info_a.iterations}) X {ex:.2e} E {ee:.2e} bitwise {bitwise}", flush=True)
    assert info_s.iterations == info_a.iterations
    assert info_s.done == info_a.done and info_s.converged == info_a.converged
    assert list(info_s.rank[:N]) == list(info_a.rank[:N])
    assert ex <= BAR[precision] and ee <= BAR[precision], (ex, ee)
    return code


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_solve_matches_allocating_solve_twice(precision):
    # first call, then a smaller one that reuses the same static array
    _case((40, 36, 32), (4, 4, 3), 11, precision)
    _case((24, 20, 18), (3, 3, 2), 12, precision)


def test_static_solve_folded_order4_twice():
    # order 4, FP64, ranks up to 6: the fused pass accumulates every mode's
    # GEMM-M, with its per-block partials and tile counters in the static
    # array too; the second call is smaller
    _case((4, 4, 32, 64), (4, 4, 6, 6), 13, "fp64")
    _case((3, 2, 64, 32), (3, 2, 5, 4), 14, "fp64")


def test_static_solve_rejects_state_above_the_array():
    limit = P.static_scratch_bytes()
    assert limit == 32 << 20
    T = torch.zeros((300, 300, 300), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PasdError) as ei:
        P.solve_static(T, (5, 5, 5), tol=1e-6, max_iter=10, precision="fp64")
    assert ei.value.code == P.ERR_UNSUPPORTED
    assert "static scratch" in str(ei.value)
