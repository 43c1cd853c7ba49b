"""Table 1 of the paper (Section 5.1), PASD only, on the GPU path.

Tucker rank 10 with R_n = floor(1.2 r) = 12 surplus ranks, additive U[-1, 1]
corruption, epsilon = 1e-5, maxiter = 1000, FP64.  The paper prints the mean
RSE over ten random instances (tests/golden/table1_pasd.json); one seeded
instance per entry must land within an order of magnitude of it.  This also
exercises the surplus-rank case, where M_n and the Gram have numerically
tiny directions that the thresholds must keep out of Z_n.
"""

import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_pasd.json")))


@pytest.mark.parametrize("entry", GOLDEN["entries"], ids=lambda e: f"{len(e['dims'])}way-{e['rho']}")
def test_table1_pasd_recovery(entry):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_09999_amd import pasd as P
    dims = tuple(entry["dims"])
    N = len(dims)
    seed = 17121000 + int(entry["rho"] * 100) + 10 * N
    wl = workloads.tucker_workload("table1", dims, (10,) * N, entry["rho"], seed,
                                   value_range=(-1.0, 1.0), ranks=(12,) * N)
    s = P.Solver(wl.T, wl.ranks, precision="fp64", tol=1e-5, max_iter=1000)
    torch.cuda.synchronize()
    info = s.solve()
    X, E = (t.cpu().numpy() for t in s.result())
    rse = float(np.linalg.norm(X - wl.L) / np.linalg.norm(wl.L))
    print(f"{dims} rho={entry['rho']}: k={info.iterations} converged={info.converged} "
          f"rank={list(info.rank[:N])} RSE={rse:.3e} (paper mean {entry['rse']:.2e})", flush=True)
    assert info.converged == 1
    assert rse <= 10 * entry["rse"]
