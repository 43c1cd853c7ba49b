"""Writes full_<config>.json: a full FP64 oracle solve of one full-size
configuration, for the GPU full-solve parity tests.

Configurations (workloads.make_config): c2 (200^3, R_n = 10), c3 (the
video-shaped 144 x 176 x 400, R = (8, 8, 3)), c4 (64^4, R_n = 6) and c4r7
(64^4 with R_n = 7, the multilinear rank of the min-max normalised Tucker
part, for the planted-support check).  Every solve runs on the FP32-rounded
observed tensor cast to FP64, the bytes both GPU precisions are given, with
the configuration's tolerance (1e-6) and iteration cap (1000).

The tensors are too large to store, so each file holds the iteration count,
the final residuals, SVT ranks and penalty, the residual history, the
Frobenius norms of X and E, the support statistics of E against the planted
mask, and X and E at SAMPLES positions drawn by numpy.random.default_rng
(SAMPLE_SEED) without replacement (the tests redraw the same positions).
Calls only the oracle and the seeded generators; run from the repository
root (c2 about 2 minutes on 8 cores, c3 about 5, c4 about 15):

    python tests/golden/make_full_solves.py c2 c3 c4 c4r7
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import pasd_solve  # noqa: E402

SAMPLES = 2048
SAMPLE_SEED = 17129001


def sample_positions(numel: int) -> np.ndarray:
    """Flat indices of the sampled entries (sorted)."""
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(numel, size=min(SAMPLES, numel), replace=False))


def config(name: str):
    """(workload, solver ranks) of a golden configuration."""
    if name == "c4r7":
        wl = workloads.make_config("c4")
        return wl, (7, 7, 7, 7)
    wl = workloads.make_config(name)
    return wl, tuple(wl.ranks)


def main(names):
    here = os.path.dirname(os.path.abspath(__file__))
    for name in names:
        wl, ranks = config(name)
        T = wl.observed(np.float32).astype(np.float64)
        t0 = time.time()
        X, E, st = pasd_solve(T, ranks, tol=wl.tol, max_iter=wl.max_iter)
        dt = time.time() - t0
        pos = sample_positions(T.size)
        supp = E != 0
        out = {
            "source": "oracle/pasd_oracle.py pasd_solve, FP64, on the FP32-rounded T",
            "config": name, "dims": list(wl.dims), "ranks": list(ranks), "tol": wl.tol,
            "max_iter": wl.max_iter, "iterations": int(st.k),
            "residual": [float(r) for r in st.residual], "rank": [int(r) for r in st.rank],
            "mu": float(st.mu), "history": [[float(r) for r in h] for h in st.history],
            "norm_X": float(np.linalg.norm(X)), "norm_E": float(np.linalg.norm(E)),
            "support": {"nnz_E": int(supp.sum()), "planted": int(wl.mask.sum()),
                        "planted_and_E": int((supp & wl.mask).sum()),
                        "min_abs_planted_S": float(np.abs(wl.S[wl.mask]).min()),
                        "max_abs_E_off_mask": float(np.abs(E[~wl.mask]).max()),
                        "min_abs_E_on_mask": float(np.abs(E[wl.mask]).min()),
                        "max_abs_E_minus_S": float(np.abs(E - wl.S).max())},
            "rse_vs_planted": float(np.linalg.norm(X - wl.L) / np.linalg.norm(wl.L)),
            "samples": SAMPLES, "sample_seed": SAMPLE_SEED,
            "X_samples": [float(v) for v in X.reshape(-1)[pos]],
            "E_samples": [float(v) for v in E.reshape(-1)[pos]],
            "oracle_seconds": round(dt, 1),
        }
        path = os.path.join(here, f"full_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"{name}: {st.k} iterations, residual {max(st.residual):.3e}, ranks {st.rank}, "
              f"support {out['support']}, rse {out['rse_vs_planted']:.3e} ({dt:.0f} s)",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c3", "c4", "c4r7"])
