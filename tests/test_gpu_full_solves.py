"""Full solves at the configurations' full sizes against the oracle's own full
solves (tests/golden/full_*.json, written by make_full_solves.py from the
oracle alone), from the default initialisation (mu0 = 1e-4, so the V = 0
phase, every threshold crossing and the stopping test are all covered).

Both sides solve the FP32-rounded observed tensor.  The oracle's X and E are
stored at 2048 seeded positions; the GPU result is compared there (relative
Frobenius error over the samples) and through the full-tensor norms.  Bars:
1e-10 and the same iteration count in FP64; 1e-5 in FP32 and with split-BF16
GEMMs, whose solves end by Algorithm 1's test or at the FP32 precision floor
(never claiming convergence above tol).

Planted support: the support recovered is {x : |E(x)| > t} with t the level
the solve's last stopping test certified, tol_effective = max(tol, c u max|D|)
(u the unit roundoff of the state).  The iterate determines E only to about
that level: the oracle's E, too, carries entries of at most 5e-9 (200^3) and
7e-7 (video) off the planted mask, while its smallest planted entry is 2.0e-6
and 4.4e-4.  In FP64 t = tol.  An FP32 state on the video-shaped tensor
(max |T| = 16.8, one unit in the last place 1.9e-6 > tol) stops at its
precision floor, t = 1.6e-5, and its E carries up to ~5e-6 off the mask.  The
recovered support must equal the planted mask exactly on the 200^3 and
video-shaped workloads and on 64^4 with R_n = 7, the multilinear rank of the
min-max normalised Tucker part (the shift adds a constant, so R_n = 6 cannot
recover it exactly).
"""

import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLES = 2048
SAMPLE_SEED = 17129001


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_1712_09999_amd import pasd as P  # noqa: E402


def _golden(name):
    return json.load(open(os.path.join(HERE, "golden", f"full_{name}.json")))


def _positions(numel):
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(numel, size=min(SAMPLES, numel), replace=False))


def _srel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _workload(name):
    if name == "c4r7":
        return workloads.make_config("c4"), (7, 7, 7, 7)
    wl = workloads.make_config(name)
    return wl, tuple(wl.ranks)


CASES = [("c2", "fp64"), ("c2", "fp32"), ("c2", "bf16"),
         ("c3", "fp64"), ("c3", "fp32"), ("c3", "bf16"),
         ("c4", "fp64"), ("c4", "fp32"), ("c4", "bf16"),
         ("c4r7", "fp64")]


@pytest.mark.parametrize("name,precision", CASES)
def test_full_solve_matches_oracle(name, precision):
    g = _golden(name)
    wl, ranks = _workload(name)
    assert list(ranks) == g["ranks"] and list(wl.dims) == g["dims"]
    T32 = wl.observed(np.float32)
    T = T32.astype(np.float64) if precision == "fp64" else T32
    print(f"[{name}/{precision}] solving {wl.dims} R={ranks}", flush=True)
    with P.Solver(T, ranks, precision=precision, tol=g["tol"], max_iter=g["max_iter"]) as s:
        info = s.solve()
        X, E = (t.double().cpu().numpy() for t in s.result())
    N = len(ranks)
    r = max(info.residual[:N])
    pos = _positions(X.size)
    ex = _srel(X.reshape(-1)[pos], np.asarray(g["X_samples"]))
    ee = _srel(E.reshape(-1)[pos], np.asarray(g["E_samples"]))
    nx = abs(np.linalg.norm(X) - g["norm_X"]) / g["norm_X"]
    ne = abs(np.linalg.norm(E) - g["norm_E"]) / g["norm_E"]
    print(f"[{name}/{precision}] k={info.iterations} (oracle {g['iterations']}) done={info.done} "
          f"residual {r:.2e} ranks {list(info.rank[:N])} (oracle {g['rank']}) "
          f"X {ex:.2e} E {ee:.2e} |X| {nx:.1e} |E| {ne:.1e}", flush=True)
    if precision == "fp64":
        assert info.done == 1 and info.converged == 1
        assert info.iterations == g["iterations"]
        assert list(info.rank[:N]) == g["rank"]
        bar = 1e-10
    else:
        assert info.done in (1, 4), info.done
        assert (info.converged == 1) == (r < g["tol"])
        bar = 1e-5
    assert ex <= bar and ee <= bar and nx <= bar and ne <= bar, (ex, ee, nx, ne)
    if name != "c4":
        thr = max(g["tol"], info.tol_effective)
        supp = np.abs(E) > thr
        miss = int(np.count_nonzero(supp != wl.mask))
        off = float(np.abs(E[~wl.mask]).max())
        on = float(np.abs(E[wl.mask]).min())
        print(f"[{name}/{precision}] support |E| > {thr:.2e} vs planted: {miss} mismatches of "
              f"{int(wl.mask.sum())} (false positives {int(np.count_nonzero(supp & ~wl.mask))}, "
              f"max |E| off the mask {off:.2e}, min |E| on it {on:.2e}, "
              f"max |T| {float(np.abs(T).max()):.2e})", flush=True)
        assert miss == 0
