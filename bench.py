#!/usr/bin/env python3
"""Benchmark of the *_L-product completion hot path on one MI355X.

A step is one PGA iteration (Alg. 5) over the whole tensor: momentum and masked
gradient step (eqs. (51)-(52), fused into the forward transform), forward L (DCT
along modes 3..N as one MFMA GEMM), per-slice one-sided-Jacobi SVD and singular
value soft-threshold, rank-r rebuild, inverse L with the stopping-rule norms.

Default workload: the video-shaped completion 144x176x3x50 of L-rank 10, 30%
observed (150 frontal slices of 144x176 per step), the continuation schedule
mu0 = 0.9 ||P_Omega(M)||_F, nu = 0.9, mu_bar = 1e-4 mu0, run for --steps
iterations from X = 0 (the full job is 200 iterations).  Inputs are resident in
HBM before the timed region.

Prints one JSON line (rank 0).  Extra fields: slice-SVT/s, the Jacobi kernel's
roofline (VALU-bound: FP64 dots and angles, FP32 rotations), the FP64 oracle
timed on this host on a bounded sample, and the sample's error vs that oracle.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_VALU = 78.6e12
PEAK_FP32_VALU = 157.3e12
PEAK_HBM = 8.0e12


# HBM bytes per k_jacobi_warm launch on the default video workload (FP32,
# Cholesky-QR preconditioned, warm-started, 150 slices of 144 x 144 factors), from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes scaled by a 256 MiB device copy
# in the same run (fetch x2.0, write x1.0), warm launches; the command lines and
# raw figures are in profiles/.  Reported only for that configuration and this
# kernel version (null elsewhere).
JACOBI_WARM_TRAFFIC_VIDEO_BYTES = 42332974


def jacobi_flops(rows, n, sweeps, rotations, slices, dot32=True, rot_rows=None):
    """Algorithmic flops of the one-sided Jacobi SVT kernel summed over `slices`
    slice-SVDs of n columns of `rows` rows (the slice's m, or n when the
    Cholesky-QR preconditioned path runs the Jacobi on R^T) that took `sweeps`
    sweeps and applied `rotations` rotations in total: per sweep and slice,
    n(n-1)/2 pair dot products (2 rows flops each; FP32 when the tolerance is
    1e-6 or looser, FP64 otherwise) and n column norms (2 rows FP64 flops); per
    rotation 6 rot_rows FP32 flops (two columns, 3 flops per entry; rot_rows =
    rows unless the columns carry more rows than the dot products read); per
    slice the final column norms (2 rows n FP64)."""
    pairs = n * (n - 1) // 2
    dots = sweeps * pairs * 2 * rows
    f64 = sweeps * n * 2 * rows + slices * n * 2 * rows + (0 if dot32 else dots)
    f32 = rotations * 6 * (rot_rows or rows) + (dots if dot32 else 0)
    return f64, f32


def threads_used():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        blas = [i for i in info if i.get("user_api") == "blas"]
        if blas:
            return int(blas[0]["num_threads"])
    except Exception:
        pass
    return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed iterations (default: 200 video, 300 large, 30 big; 50 mix ticks)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="f32", choices=["f32", "bf16x3"])
    ap.add_argument("--workload", default="video", choices=["video", "large", "big", "mix", "serve"])
    ap.add_argument("--large-frac", type=float, default=0.1,
                    help="serve workload: share of 512x512x3x64 requests")
    ap.add_argument("--no-lanes", action="store_true",
                    help="serve workload: one batch for all requests (no lane for blocked-kernel requests)")
    ap.add_argument("--requests", type=int, default=200, help="serve workload: number of requests")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serve workload: Poisson arrival rate (1/s); 0 = calibrate to 0.7 x saturation")
    ap.add_argument("--per-request-iters", type=int, default=5,
                    help="mix workload: iterations of the plain per-request form timed for comparison")
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="oracle iterations timed on the host (bounded CPU sample; default 30 for "
                         "video, 10 for large: the iterates are nonzero from the sixth and eighth iterations)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="video/large: run one 256 MiB device copy before the timed region (counter reference)")
    ap.add_argument("--transform", default="dct", choices=["dct", "dft"],
                    help="video workload: transform along the trailing modes (dft: the t-product form)")
    ap.add_argument("--no-precondition", action="store_true",
                    help="run the Jacobi SVD on the slices themselves (no Cholesky-QR factor)")
    ap.add_argument("--warm-restart", type=int, default=0,
                    help="video/large/big: cold Jacobi start every this many iterations "
                         "(0: the library default, 256; -1: every iteration, no warm start)")
    ap.add_argument("--fp32-dots", action="store_true",
                    help="FP32 pair dot products in the Jacobi (default: FP64)")
    ap.add_argument("--lanes", default="auto",
                    help="mix workload: Jacobi lanes per column pair (4..64, 0 = built-in, auto = timed)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"video": 200, "large": 300, "big": 30, "mix": 50, "serve": 0}[args.workload]

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the completion path here is single-GPU "
              "(requests shard by whole problem across GPUs); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_02870_amd import lt
    from paper_2202_02870_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.workload == "mix":
        return bench_mix(args, torch, lt, wl)
    if args.workload == "serve":
        return bench_serve(args, torch, lt, wl)
    if args.workload == "video":
        p = wl.config1(transform=args.transform)
    else:
        p = {"large": wl.config2, "big": wl.config4_large}[args.workload]()
    shape = p.shape
    I1, I2 = shape[0], shape[1]
    P = wl.n_slices(shape)
    m, n = max(I1, I2), min(I1, I2)
    s = p.schedule
    M = lt.to_device(p.M)
    mask = lt.to_device(p.mask, dtype=torch.uint8)
    X = lt.fortran_empty(shape)
    ws = torch.empty(lt.workspace_bytes(shape, p.kinds, "pga", args.precision), dtype=torch.uint8,
                     device="cuda")

    def params(iters):
        return lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0, max_iter=iters,
                             precision=args.precision, precondition=not args.no_precondition,
                             warm_restart=args.warm_restart, fp32_dots=args.fp32_dots)

    # warmup (untimed)
    if args.warmup > 0:
        lt.complete_pga(M, mask, params(args.warmup), p.kinds, out=X, ws=ws)
    torch.cuda.synchronize()

    if args.pmc_calibrate:
        # a plain device copy of known size (256 MiB read + 256 MiB written): the
        # reference that turns hardware byte counters into HBM bytes
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # timed region: exactly --steps iterations, kernel durations recorded with HIP events
    lt.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep, st = lt.complete_pga(M, mask, params(args.steps), p.kinds, out=X, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof, dropped = lt.profile_end()
    elapsed = t1 - t0
    value = args.steps / elapsed

    # Jacobi kernel roofline (dominant kernel): algorithmic flops per launch over
    # its mean event-timed duration
    jcalls, jms = prof["jacobi"]
    path = lt.svt_path(shape, p.kinds, precondition=not args.no_precondition)
    precond = "precond" in path
    jm, jn = (2 * m, 2 * n) if "dft" in p.kinds else (m, n)   # Fourier: real embeddings of the slices
    rows = jn if precond else jm
    # warm-started Jacobi: every rotation also updates the accumulated rotations
    # (a second block of 4 ceil(n/4) rows below the factor's)
    warm = lt.pga_warm(shape, p.kinds, precondition=not args.no_precondition, warm_restart=args.warm_restart)
    rot_rows = rows + 4 * ((jn + 3) // 4) if warm else rows
    f64, f32 = jacobi_flops(rows, jn, rep["total_sweeps"], rep["total_rotations"], rep["total_slices"],
                            rot_rows=rot_rows)
    per_launch = (f64 + f32) / max(jcalls, 1)
    t_launch = jms / 1e3 / max(jcalls, 1)
    t_peak = (f64 / PEAK_FP64_VALU + f32 / PEAK_FP32_VALU) / max(jcalls, 1)
    achieved = per_launch / t_launch / 1e12 if t_launch > 0 else 0.0
    peak = per_launch / t_peak / 1e12 if t_peak > 0 else 0.0
    measured_cfg = (args.workload == "video" and args.transform == "dct" and args.precision == "f32" and precond
                    and warm)
    roofline = {"bound": "alu", "kernel": "k_jacobi_warm" if warm else "k_jacobi", "achieved": round(achieved, 3),
                "peak": round(peak, 2), "unit": "TFLOP/s",
                "frac": round(t_peak / t_launch, 4) if t_launch > 0 else None,
                "traffic": JACOBI_WARM_TRAFFIC_VIDEO_BYTES if measured_cfg else None,
                "flops_per_launch": per_launch, "fp64_share": round(f64 / (f64 + f32), 4),
                "launch_ms": round(t_launch * 1e3, 4), "launches": jcalls,
                "jacobi_rows": rows, "rotated_rows": rot_rows, "preconditioned": precond,
                "warm_start": warm, "svt_path": path}

    line = {
        "metric": "PGA iterations/s (slice-SVT/s alongside) at rel-err <= 1e-4 vs FP64 oracle",
        "value": round(value, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "f32" else "bf16x3+f32",
        "data": "synthetic",
        "config": {"workload": p.name, "shape": list(shape), "slices_per_step": P,
                   "precision": args.precision, "schedule": "mu0=0.9||P_Omega M||, nu=0.9, mu_bar=1e-4 mu0"},
        "slice_svt_per_s": round(value * P, 1),
        "mean_sweeps": round(rep["total_sweeps"] / max(rep["total_slices"], 1), 3),
        "kernel_ms": {k: round(v[1], 3) for k, v in prof.items()},
        "kernel_calls": {k: v[0] for k, v in prof.items()},
        "roofline": roofline,
    }

    cpu_iters = args.cpu_iters if args.cpu_iters is not None else {"video": 30, "large": 10, "big": 1}[args.workload]
    if not args.no_cpu_baseline and cpu_iters > 0:
        import oracle as o
        k = cpu_iters
        mats = o.mats_for(shape, list(p.kinds))
        c0 = time.perf_counter()
        Xo, _ = o.complete_pga(p.M, p.mask, mats, mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"],
                               tol=0.0, max_iter=k)
        c1 = time.perf_counter()
        line["cpu_baseline"] = {"value": round(k / (c1 - c0), 4), "unit": "iters/s",
                                "cores": threads_used(), "kind": "oracle",
                                "sample": "first %d PGA iterations of the same workload, FP64 NumPy/LAPACK" % k}
        Xg, _, _ = lt.complete_pga(M, mask, params(k), p.kinds, out=X, ws=ws)
        Xg = lt.to_host(Xg).astype(np.float64)
        nrm = float(np.linalg.norm(Xo))
        # the first iterations threshold every singular value (mu_k is large), so a
        # sample that short compares zero tensors: report the GPU iterate's own norm then
        if nrm > 0:
            err = {"rel_err_vs_oracle": float(np.linalg.norm(Xg - Xo) / nrm)}
        else:
            err = {"abs_norm_gpu_where_oracle_is_zero": float(np.linalg.norm(Xg))}
        line["parity"] = {"iters": k, **err, "bound": 1e-4 if args.precision == "f32" else 1e-2}

    print(json.dumps(line), flush=True)


def bench_mix(args, torch, lt, wl):
    """64 independent problems of uneven shapes (order 3/4, I1, I2 in 32..256,
    trailing {3,8,16} x {1,10,30}); a step is one tick of the batch engine: one
    PGA iteration of every problem, with all frontal slices of all problems in
    one Jacobi launch (graph-replayed ticks).  The plain per-request form (one
    lt_complete_pga call per problem) is timed alongside."""
    probs = wl.config3(max_iter=args.steps + args.warmup)
    total_slices = sum(wl.n_slices(p.shape) for p in probs)
    dev = []
    for p in probs:
        s = p.schedule
        params = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0,
                               max_iter=args.steps + args.warmup, precision=args.precision)
        M = lt.to_device(p.M)
        mask = lt.to_device(p.mask, dtype=torch.uint8)
        dev.append((p, M, mask, params))
    lanes, tune_ms = args.lanes, None
    if lanes == "auto":
        from paper_2202_02870_amd import autotune
        lanes, tune_ms = autotune.tune([p.shape for p in probs])
    lanes = int(lanes)
    gps = [lt.Problem(M, mask, params, p.kinds) for (p, M, mask, params) in dev]
    batch = lt.Batch(gps, use_graph=True, jacobi_lanes=lanes)
    if args.warmup > 0:
        batch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    reps = [gp.status()[0] for gp in gps]
    batch.close()
    # eager ticks with per-kernel events (same work, no graph) for the kernel split
    gps2 = [lt.Problem(M, mask, params, p.kinds) for (p, M, mask, params) in dev]
    b2 = lt.Batch(gps2, use_graph=False, jacobi_lanes=lanes)
    b2.step(args.warmup)
    lt.profile_begin()
    b2.step(min(args.steps, 20))
    prof, _ = lt.profile_end()
    b2.close()
    # plain FP32 per-request form: one problem after another, the same first iterations
    k = args.per_request_iters
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for (p, M, mask, params) in dev:
        s = p.schedule
        pr = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0, max_iter=k)
        lt.complete_pga(M, mask, pr, p.kinds)
    torch.cuda.synchronize()
    c1 = time.perf_counter()
    per_req_slices = k * total_slices / (c1 - c0)
    value = args.steps / elapsed
    line = {
        "metric": "slice-SVT/s of the batched engine (PGA ticks/s as value) at rel-err <= 1e-4 vs FP64 oracle",
        "value": round(value, 3),
        "unit": "ticks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "f32" else "bf16x3+f32",
        "data": "synthetic",
        "config": {"workload": "mix-64-problems", "problems": len(probs), "slices_per_tick": total_slices,
                   "precision": args.precision},
        "slice_svt_per_s": round(value * total_slices, 1),
        "per_request_f32_slice_svt_per_s": round(per_req_slices, 1),
        "batched_over_per_request": round(value * total_slices / per_req_slices, 3),
        "mean_sweeps": round(sum(r["total_sweeps"] for r in reps) / max(sum(r["total_slices"] for r in reps), 1), 3),
        "kernel_ms_20_eager_ticks": {k2: round(v[1], 3) for k2, v in prof.items()},
        "jacobi_lanes": lanes if lanes else "built-in",
        "autotune_jacobi_ms_per_tick": ({str(g): round(t, 4) for g, t in sorted(tune_ms.items())}
                                        if tune_ms else None),
    }
    print(json.dumps(line), flush=True)


def bench_serve(args, torch, lt, wl):
    """Served stream: Poisson arrivals of completion requests drawn from the
    uneven-mix size distribution, with a share (--large-frac, 10%) of
    512x512x3x64 requests; each runs until the relative change
    ||Y - X|| / ||X|| < 1e-5 (gated until mu reaches its floor) or 500
    iterations; admission by HBM footprint, iterates resident on the device,
    iteration-level continuous batching.  Reports p50/p99 latency and the
    aggregate slice-SVT/s."""
    from paper_2202_02870_amd import serving
    specs = wl.config4_specs(n=args.requests, seed=4, large_frac=args.large_frac)
    n_large = sum(1 for sp in specs if tuple(sp["shape"]) == wl.LARGE_REQUEST_SHAPE)

    def progress(r):
        print("finished request %d %s: %d iterations, latency %.3f s" % (r.rid, "x".join(map(str, r.M.shape)),
                                                                         r.iters, r.latency),
              file=sys.stderr, flush=True)

    reqs = []
    for i, sp in enumerate(specs):
        p = wl.make_problem(sp["shape"], sp["rank"], sp["observed"], sp["seed"])
        prm = dict(wl.pga_schedule_params(p.M, p.mask), max_iter=500, tol=1e-5)
        reqs.append(serving.Request(rid=i, arrival=0.0, M=p.M.astype(np.float32), mask=p.mask,
                                    params=prm, kinds=p.kinds))
    rate = args.rate
    if rate <= 0:
        # saturation estimate: all requests at t = 0 on a small prefix
        probe = [serving.Request(rid=r.rid, arrival=0.0, M=r.M, mask=r.mask, params=r.params, kinds=r.kinds)
                 for r in reqs[:16]]
        srv = serving.CompletionServer(serving.GpuExecutor(lanes=not args.no_lanes), hbm_budget=int(64e9),
                                       ticks_per_round=4, lane_ticks=2, on_finish=progress)
        for r in probe:
            srv.submit(r)
        c0 = time.perf_counter()
        srv.run()
        sat = len(probe) / (time.perf_counter() - c0)
        rate = 0.7 * sat
    arr = serving.poisson_arrivals(len(reqs), rate, seed=4)
    for r, t in zip(reqs, arr):
        r.arrival = float(t)
    srv = serving.CompletionServer(serving.GpuExecutor(lanes=not args.no_lanes), hbm_budget=int(64e9),
                                   ticks_per_round=4, lane_ticks=2, on_finish=progress)
    for r in reqs:
        srv.submit(r)
    c0 = time.perf_counter()
    st = srv.run(sleep=0.001)
    wall = time.perf_counter() - c0
    slices = sum(r.iters * wl.n_slices(r.M.shape) for r in srv.done)
    line = {
        "metric": "served p50/p99 latency and aggregate slice-SVT/s",
        "value": round(slices / wall, 1),
        "unit": "slice-SVT/s",
        "n_gpus": 1,
        "steps": st["ticks"],
        "warmup": 0,
        "ms_per_step": round(1e3 * wall / max(st["ticks"], 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "served-stream", "requests": len(reqs), "large_512x512x3x64": n_large,
                   "rate_per_s": round(rate, 3),
                   "stop": "rel. change < 1e-5 or 500 iterations", "hbm_budget_GB": 64,
                   "lanes": not args.no_lanes},
        "p50_s": round(st.get("p50", float("nan")), 4),
        "p99_s": round(st.get("p99", float("nan")), 4),
        "completed": st["completed"],
        "rejected": st["rejected"],
        "mean_iters": round(float(np.mean([r.iters for r in srv.done])), 2) if srv.done else None,
        "peak_resident_GB": round(st["peak_bytes"] / 1e9, 3),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
