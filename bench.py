#!/usr/bin/env python3
"""Throughput of the PASD ADMM iteration on one MI355X.

Workload: 200 x 200 x 200 tensor, Tucker core 10^3 with N(0, 1) entries and
orthonormal factors, 20% of entries corrupted by additive U(-20, 20), ranks
R_n = 10, FP32 state (the paper's synthetic recipe, Section 5.1, at the
benchmarked size).  One step is one full ADMM iteration (Algorithm 1: both
unfolding GEMMs, QR, Gram eigensolver and SVT factor, the fused E/Y/residual
pass and the control update) with the input resident in HBM.

Prints one JSON line: ADMM iterations/s over --steps timed iterations, the
full-solve rate to tol 1e-6 in FP32 and FP64 with the FP32-vs-FP64 error of
X and E, per-kernel times from HIP events recorded inside the library on the
launch stream, the roofline figure of the dominant kernel, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TRPCA solves/s + ADMM iters/s at rel.err≤1e-5 vs FP64; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def _measured_traffic():
    """Calibrated HBM bytes per fused-pass launch from the committed counter
    profile, or None once the kernel source differs from the measured one."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "pasd_c2_fp32_hbm_traffic.md")
    try:
        vals = {}
        for line in open(path):
            if ":" in line and line.strip().startswith("fused_"):
                k, v = line.strip().split(":", 1)
                vals[k.strip()] = v.strip()
        src = os.path.join(here, vals["fused_source"])
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if digest != vals["fused_source_sha256"]:
            return None
        return int(vals["fused_traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _rel(a, b):
    import numpy as np
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def kernel_bytes(dims, ranks, es):
    """Algorithmic HBM bytes per launch of the streaming kernels.

    fused : reads T and Y_1..Y_N, writes D and Y_1..Y_N  -> (2N + 2) numel s
            plus one read of every P_n (R_n J_n s)
    gemm_p: reads D and Y_n for every mode               -> 2 N numel s, writes P_n
    gemm_m: reads D and Y_n for every mode               -> 2 N numel s, reads P_n
    """
    import math
    N = len(dims)
    numel = math.prod(dims)
    Pbytes = sum(r * numel // d for d, r in zip(dims, ranks)) * es
    return {
        "fused": (2 * N + 2) * numel * es + Pbytes,
        "gemm_p": 2 * N * numel * es + Pbytes,
        "gemm_m": 2 * N * numel * es + Pbytes,
    }


def cpu_baseline(T64, ranks, iters):
    """The FP64 oracle on the host cores, `iters` iterations from k = 0."""
    import numpy as np
    from oracle import pasd_init, pasd_iterate
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        ncores = len(os.sched_getaffinity(0))
        ctx = threadpool_limits(limits=ncores)
        used = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # threadpoolctl missing: report what numpy's BLAS was left with
        ctx = None
        used = len(os.sched_getaffinity(0))
    st = pasd_init(T64, ranks)
    pasd_iterate(st, 1)  # warm the BLAS and page in the arrays
    t0 = time.perf_counter()
    pasd_iterate(st, iters)
    dt = time.perf_counter() - t0
    if ctx is not None:
        ctx.restore_original_limits()
    return {"value": iters / dt, "unit": "ADMM iters/s", "cores": int(used), "kind": "oracle",
            "sample": f"{iters} FP64 oracle iterations of the same 200^3 R=10 workload "
                      f"(k = 1..{iters}), {dt:.1f} s"}


def serving_bench(count, seq_count):
    """The serving trace: `count` 3-way requests (dims U{32..256}, Tucker ranks
    U{3..15}, 5-20% U(-10, 10), FP32, tol 1e-6).  Saturation throughput with
    everything arriving at once, then Poisson arrivals at 0.8x that rate for
    p50/p99 latency, and the first `seq_count` requests served one at a time by
    plain pasd_solve as the baseline."""
    import torch

    import workloads
    from workloads.torch_gen import tucker_on_device
    from paper_1712_09999_amd import serving

    t0 = time.perf_counter()
    trace = workloads.serving_trace(count=count, qps=1.0)
    tensors = []
    for spec in trace:
        T, _, _ = tucker_on_device(spec["dims"], spec["ranks"], spec["frac"], spec["seed"])
        tensors.append(T)
    torch.cuda.synchronize()
    numel = sum(t.numel() for t in tensors)
    _progress(f"serving: {count} request tensors drawn in {time.perf_counter() - t0:.1f} s")

    def reqs(scale):
        return [serving.Request(s["index"], s["arrival"] * scale, tensors[s["index"]], s["ranks"],
                                tol=1e-6, max_iter=1000) for s in trace]

    srv = serving.Server(precision="fp32", max_slots=64, step_iters=4, keep_results=False)
    sat = serving.latency_summary(srv.run(reqs(0.0), realtime=False))
    _progress(f"serving: saturation {sat['solves_per_s']:.1f} solves/s ({srv.stats['wall_s']:.1f} s)")
    qps = 0.8 * sat["solves_per_s"]
    pois = serving.latency_summary(srv.run(reqs(1.0 / qps), realtime=True))
    _progress(f"serving: Poisson at {qps:.1f}/s p50 {pois['p50_ms']:.1f} ms p99 {pois['p99_ms']:.1f} ms")
    seq_reqs = reqs(1.0 / qps)[:seq_count]
    seq = serving.latency_summary(serving.sequential(seq_reqs))
    _progress(f"serving: sequential {seq['solves_per_s']:.1f} solves/s")
    return {
        "requests": count, "mean_numel": numel / count, "precision": "fp32", "max_slots": 64,
        "saturation": {"solves_per_s": round(sat["solves_per_s"], 2),
                       "converged": sat["converged"]},
        "poisson": {"qps": round(qps, 2), "p50_ms": round(pois["p50_ms"], 2),
                    "p99_ms": round(pois["p99_ms"], 2),
                    "solves_per_s": round(pois["solves_per_s"], 2)},
        "sequential_plain": {"requests": seq_count, "solves_per_s": round(seq["solves_per_s"], 2),
                             "p50_ms": round(seq["p50_ms"], 2), "p99_ms": round(seq["p99_ms"], 2)},
        "speedup_vs_sequential": round(sat["solves_per_s"] / seq["solves_per_s"], 2),
    }


def phase_bench(rs, rhos, trials, dim=100, seed0=17125000):
    """The phase-transition workload of Fig. 1 (Section 5.1) as one batch of
    solves through the serving loop: dim^3 tensors, Tucker rank r in every mode
    (N(0, 1) core, Haar factors, left unscaled), a fraction rho of the entries
    plus U(-1, 1), R_n = floor(1.2 r), epsilon 1e-5, maxiter 1000, FP64; a
    trial succeeds when RSE = ||X - L|| / ||L|| <= 1e-3.  Returns the success
    fraction per (rho, r) cell and the batched solve rate."""
    import torch

    from workloads.torch_gen import tucker_on_device
    from paper_1712_09999_amd import serving

    t0 = time.perf_counter()
    reqs, cells, planted = [], [], []
    for a, rho in enumerate(rhos):
        for b, r in enumerate(rs):
            for t in range(trials):
                seed = seed0 + 100000 * t + 1000 * a + b
                T, L, _ = tucker_on_device((dim,) * 3, (r,) * 3, rho, seed, value_range=(-1.0, 1.0),
                                           dtype=torch.float64, scale=None)
                reqs.append(serving.Request(len(reqs), 0.0, T, (int(1.2 * r),) * 3, tol=1e-5,
                                            max_iter=1000))
                cells.append((a, b))
                planted.append(L)
    torch.cuda.synchronize()
    _progress(f"phase: {len(reqs)} tensors drawn in {time.perf_counter() - t0:.1f} s")
    srv = serving.Server(precision="fp64", max_slots=64, step_iters=4, keep_results=True)
    res = srv.run(reqs, realtime=False)
    wall = srv.stats["wall_s"]
    ok = [[0] * len(rs) for _ in rhos]
    iters = 0
    for q in res:
        a, b = cells[q.rid]
        L = planted[q.rid]
        rse = float(torch.linalg.vector_norm(q.X - L) / torch.linalg.vector_norm(L))
        ok[a][b] += int(rse <= 1e-3)
        iters += q.iterations
    _progress(f"phase: {len(res)} solves in {wall:.1f} s")
    return {"dims": [dim] * 3, "r": list(rs), "rho": list(rhos), "trials": trials,
            "precision": "fp64", "success": [[c / trials for c in row] for row in ok],
            "solves": len(res), "iterations": iters, "wall_s": round(wall, 2),
            "solves_per_s": round(len(res) / wall, 2), "iters_per_s": round(iters / wall, 1)}


def wide_rank_bench(rs, precision="fp64", iters=40):
    """Per-kernel times of one 100^3 solve at Tucker rank r with R_n =
    floor(1.2 r) (the Fig. 1 workload), from HIP events between launches over
    `iters` iterations after 30 warm-up iterations, and the graph-replay
    iteration time; R_n > 16 runs the rank-tiled path."""
    import torch

    from workloads.torch_gen import tucker_on_device
    from paper_1712_09999_amd import pasd as P

    dt = torch.float64 if precision == "fp64" else torch.float32
    rows = []
    for r in rs:
        R = int(1.2 * r)
        T, _, _ = tucker_on_device((100, 100, 100), (r, r, r), 0.1, 17126000 + r,
                                   value_range=(-1.0, 1.0), dtype=dt, scale=None)
        s = P.Solver(T, (R, R, R), precision=precision, tol=0.0, max_iter=100000, device=0)
        s.step(30)
        prof = s.profile(iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(64)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 64 * 1e3
        info = s.query()
        rows.append({"r": r, "R": R, "ms_per_iter": round(ms, 4),
                     "eig_sweeps": list(info.eig_sweeps[:3]),
                     "kernels_us": {k: round(v[0] / max(v[1], 1) * 1e3, 1) for k, v in prof.items()}})
        s.close()
        _progress(f"wide rank r={r} R={R}: {ms:.3f} ms/iter")
    return {"dims": [100, 100, 100], "precision": precision, "rows": rows}


def mri_bench(rhos):
    """The MRI-shaped stand-in of Section 5.2 (181 x 217 x 181, R_n = 40, a
    fraction rho of the voxels replaced by U(0, 255); the MRI data itself is not
    available, see workloads.mri_standin): one FP32 and one FP64 solve per rho
    with the input resident on the GPU, iterations, solve time and PSNR."""
    import torch

    import workloads
    from paper_1712_09999_amd import pasd as P

    rows = []
    for rho in rhos:
        wl = workloads.mri_standin(rho)
        row = {"rho": rho, "psnr_observed_db": round(workloads.psnr(wl.T, wl.L), 2)}
        for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
            Td = torch.from_numpy(wl.T).to(device="cuda", dtype=dt).contiguous()
            s = P.Solver(Td, wl.ranks, precision=prec, tol=wl.tol, max_iter=wl.max_iter, device=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.solve()
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t0
            X = s.result()[0].double().cpu().numpy()
            row[prec] = {"iterations": info.iterations, "converged": bool(info.converged),
                         "solve_ms": round(dt_s * 1e3, 1),
                         "ms_per_iter": round(dt_s * 1e3 / max(info.iterations, 1), 3),
                         "psnr_db": round(workloads.psnr(X, wl.L), 2)}
            s.close()
        rows.append(row)
        _progress(f"mri stand-in rho={rho}: fp32 {row['fp32']['solve_ms']} ms "
                  f"({row['fp32']['iterations']} it), fp64 {row['fp64']['solve_ms']} ms, "
                  f"PSNR {row['psnr_observed_db']} -> {row['fp64']['psnr_db']} dB")
    return {"dims": [181, 217, 181], "ranks": [40, 40, 40], "data": "synthetic stand-in",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--srv-requests", type=int, default=512)
    ap.add_argument("--srv-sequential", type=int, default=128)
    ap.add_argument("--no-phase", action="store_true")
    ap.add_argument("--phase-full", action="store_true",
                    help="the full Fig. 1 grid (r = 2..50 and rho = 2..50%% in steps of 2, "
                         "--phase-trials each) instead of every fourth point")
    ap.add_argument("--phase-trials", type=int, default=1)
    ap.add_argument("--no-mri", action="store_true")
    ap.add_argument("--no-wide", action="store_true")
    ap.add_argument("--pmc-calib", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy (3 times), the "
                         "reference kernel that scales hardware traffic counters to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the solver runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1712_09999_amd import pasd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    wl = workloads.make_config("c2")
    dims, ranks = wl.dims, wl.ranks
    T32 = wl.observed(np.float32)
    T64 = T32.astype(np.float64)

    # ---- timed iterations (FP32, no early stop) ------------------------------
    s = P.Solver(T32, ranks, precision="fp32", tol=0.0, max_iter=10 ** 7, device=0)
    s.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    ms_per_step = total_ms / args.steps
    value = 1000.0 / ms_per_step
    _progress(f"timed {args.steps} iterations: {ms_per_step:.4f} ms each")

    prof_iters = max(10, min(args.steps, 100))
    prof = s.profile(prof_iters)
    kernels = {k: {"ms": t / max(c, 1)} for k, (t, c) in prof.items()}
    kb = kernel_bytes(dims, ranks, 4)
    for k, b in kb.items():
        kernels[k]["alg_bytes"] = b
        kernels[k]["GB/s"] = b / (kernels[k]["ms"] * 1e-3) / 1e9
    dom = max(kb, key=lambda k: kernels[k]["ms"])
    ach = kernels[dom]["GB/s"]
    traffic = _measured_traffic() if dom == "fused" else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": kb[dom], "ms_per_launch": kernels[dom]["ms"]}
    s.close()

    if args.pmc_calib:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").uniform_()
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        _progress("copy calibration: 3 x 256 MiB device copies")

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "ADMM iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "200x200x200 Tucker rank-10 core N(0,1), 20% additive U(-20,20); "
                               "R_n=10, FP32 state and GEMMs, FP64 QR/eig/norms",
                   "dims": list(dims), "ranks": list(ranks), "tol": wl.tol},
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
    }

    # ---- full solves to tol 1e-6: FP32 and FP64 on the same bytes -----------
    if not args.no_solve:
        res = {}
        for prec, T in (("fp32", T32), ("fp64", T64), ("bf16", T32)):
            sv = P.Solver(T, ranks, precision=prec, tol=wl.tol, max_iter=wl.max_iter, device=0)
            sv.solve()  # warm-up solve
            sv.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = sv.solve()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            X, E = (t.double().cpu().numpy() for t in sv.result())
            res[prec] = dict(ms=dt * 1e3, iters=info.iterations, converged=info.converged, X=X, E=E,
                             residual=max(info.residual[:3]))
            sv.close()
        ex = _rel(res["fp32"]["X"], res["fp64"]["X"])
        ee = _rel(res["fp32"]["E"], res["fp64"]["E"])
        out["solve"] = {
            p: {"solves_per_s": round(1e3 / r["ms"], 3), "solve_ms": round(r["ms"], 3),
                "iterations": r["iters"], "converged": bool(r["converged"]),
                "iters_per_s": round(r["iters"] / (r["ms"] * 1e-3), 1),
                "final_residual": r["residual"]} for p, r in res.items()}
        out["solve"]["fp32_vs_fp64_rel_err"] = {"X": ex, "E": ee, "within_1e-5": ex <= 1e-5 and ee <= 1e-5}
        bx = _rel(res["bf16"]["X"], res["fp64"]["X"])
        be = _rel(res["bf16"]["E"], res["fp64"]["E"])
        out["solve"]["bf16_vs_fp64_rel_err"] = {"X": bx, "E": be, "within_1e-5": bx <= 1e-5 and be <= 1e-5}
        out["solve"]["rse_vs_planted_fp64"] = _rel(res["fp64"]["X"], wl.L)
        out["solves_per_s"] = out["solve"]["fp32"]["solves_per_s"]
        _progress("full solves done")
        # Procrustes tie-break of eq. (10): the default (pre-threshold P) against
        # keeping U^k where V^k vanishes; recovery of the planted low-rank part
        tb = {}
        for name in ("c1", "c2"):
            w = wl if name == "c2" else workloads.make_config("c1")
            row = {}
            for t in ("pre", "keep"):
                sv = P.Solver(w.T, w.ranks, precision="fp64", tol=w.tol, max_iter=w.max_iter,
                              device=0, tiebreak=t)
                info = sv.solve()
                X = sv.result()[0].cpu().numpy()
                row[t] = {"iterations": info.iterations, "converged": bool(info.converged),
                          "rse_vs_planted": _rel(X, w.L)}
                sv.close()
            tb[name] = row
        out["solve"]["tiebreak_fp64"] = tb
        _progress("tie-break comparison done")

    if not args.no_serving:
        out["serving"] = serving_bench(args.srv_requests, min(args.srv_sequential, args.srv_requests))

    if not args.no_phase:
        step = 1 if args.phase_full else 4
        rs = list(range(2, 51, 2))[::step]
        rhos = [round(0.02 * k, 2) for k in range(1, 26)][::step]
        out["phase_transition"] = phase_bench(rs, rhos, args.phase_trials)

    if not args.no_wide:
        out["wide_rank"] = wide_rank_bench([10, 30, 50])

    if not args.no_mri:
        out["mri_standin"] = mri_bench([0.05, 0.10, 0.20, 0.30])

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(T64, ranks, args.cpu_iters)
        cb = out["cpu_baseline"]
        cb["value"] = round(cb["value"], 4)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
