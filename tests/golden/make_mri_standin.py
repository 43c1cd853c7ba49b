"""Writes mri_standin.json: a full FP64 oracle solve of the MRI-shaped
stand-in (Section 5.2's 181 x 217 x 181 restoration with R_n = 40; the MRI
data is not available, so workloads.mri_standin draws a Tucker tensor on
[0, 255] with 10% of the voxels replaced by U(0, 255)).  Calls only the
oracle and the seeded generators; run from the repository root (about ten
minutes on 8 cores):

    python tests/golden/make_mri_standin.py
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import pasd_solve  # noqa: E402

RHO = 0.10
SEED = 17127000


def main():
    wl = workloads.mri_standin(RHO, SEED)
    t0 = time.time()
    X, _, st = pasd_solve(wl.T, wl.ranks, tol=wl.tol, max_iter=wl.max_iter)
    out = {"source": "oracle/pasd_oracle.py pasd_solve, FP64", "dims": list(wl.dims),
           "rho": RHO, "seed": SEED, "core_ranks": [30, 30, 30], "ranks": list(wl.ranks),
           "tol": wl.tol, "max_iter": wl.max_iter, "iterations": int(st.k),
           "rank": [int(x) for x in st.rank], "psnr_db": workloads.psnr(X, wl.L),
           "psnr_observed_db": workloads.psnr(wl.T, wl.L)}
    print(out, f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mri_standin.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
