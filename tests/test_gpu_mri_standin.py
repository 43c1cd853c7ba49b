"""The MRI-shaped stand-in of Section 5.2 on the GPU path: 181 x 217 x 181
with R_n = 40 (three rank tiles), a fraction of the voxels replaced by
U(0, 255).  The first iterations are compared element by element with the
oracle at full size; a full FP64 solve is compared with the oracle's own full
solve (tests/golden/make_mri_standin.py): iteration count, SVT ranks, PSNR;
an FP32 solve restores it to the FP32 rounding level.
"""

import json
import os

import numpy as np
import pytest

import workloads
from oracle import pasd_init, pasd_iterate, pasd_output

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mri_standin.json")))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_09999_amd  # noqa: F401  (raises if the library is missing)


@pytest.fixture(scope="module")
def wl():
    return workloads.mri_standin(GOLDEN["rho"], GOLDEN["seed"])


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def test_mri_standin_first_iterations_match_oracle(wl):
    from paper_1712_09999_amd import pasd as P
    st = pasd_init(wl.T, wl.ranks)
    pasd_iterate(st, 3)
    s = P.Solver(wl.T, wl.ranks, precision="fp64", tol=0.0, max_iter=100000)
    s.step(3)
    X_o, E_o = pasd_output(st)
    ex, ee = rel(s.export(P.Q_X), X_o), rel(s.export(P.Q_E), E_o)
    ez = [rel(s.export(P.Q_Z, n), st.Z[n]) for n in range(3)]
    print(f"mri k=3: X {ex:.2e} E {ee:.2e} Z {[f'{e:.2e}' for e in ez]}", flush=True)
    assert max([ex, ee] + ez) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mri_standin_full_solve_matches_oracle(wl, precision):
    from paper_1712_09999_amd import pasd as P
    dt = np.float64 if precision == "fp64" else np.float32
    s = P.Solver(wl.T.astype(dt), wl.ranks, precision=precision, tol=GOLDEN["tol"],
                 max_iter=GOLDEN["max_iter"])
    info = s.solve()
    p = workloads.psnr(s.export(P.Q_X).astype(np.float64), wl.L)
    print(f"mri {precision}: k={info.iterations} (oracle {GOLDEN['iterations']}) "
          f"rank={list(info.rank[:3])} (oracle {GOLDEN['rank']}) PSNR={p:.3f} dB "
          f"(oracle {GOLDEN['psnr_db']:.3f}, observed {GOLDEN['psnr_observed_db']:.2f})", flush=True)
    if precision == "fp64":
        assert info.converged == 1
        # the oracle restores the stand-in to ~2e-9 RMS (PSNR ~222 dB); the GPU
        # iterate differs from the oracle's at the 1e-13 level, which moves the
        # PSNR by hundredths of a dB
        assert abs(p - GOLDEN["psnr_db"]) <= 1.0
        assert abs(info.iterations - GOLDEN["iterations"]) <= 1
        assert list(info.rank[:3]) == GOLDEN["rank"]
    else:
        # FP32 state on values up to 255: the residual cannot be certified
        # below the FP32 rounding level (tol_effective ~ 2e-4 > tol), so the
        # solve ends at the precision floor (or converged), never claiming
        # convergence above tol; the restoration is bounded by FP32 rounding of
        # X (~1e-7 relative), i.e. PSNR near 150 dB
        r = max(info.residual[:3])
        assert info.done in (1, 4) and (info.converged == 1) == (r < GOLDEN["tol"])
        assert p >= 120.0
