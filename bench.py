#!/usr/bin/env python3
"""Benchmark of the *_L-product completion hot path on one MI355X.

A step is one PGA iteration (Alg. 5) over the whole tensor: momentum and masked
gradient step (eqs. (51)-(52), fused into the forward transform), forward L (DCT
along modes 3..N as one MFMA GEMM), per-slice one-sided-Jacobi SVD and singular
value soft-threshold, rank-r rebuild, inverse L with the stopping-rule norms.

Default workload: the video-shaped completion 144x176x3x50 of L-rank 10, 30%
observed (150 frontal slices of 144x176 per step), continuation schedule
mu0 = 0.9 ||P_Omega(M)||_F, nu = 0.9, mu_bar = 1e-4 mu0.  The timed steps are
iterations start+warmup+1 .. start+warmup+steps of one run: an untimed prefix of
--start iterations (default 100: past the zero iterates of the first ~7
iterations and into the rank-carrying, floor-threshold regime), then --warmup
untimed and --steps timed iterations, each call continuing the previous one
(lt_pga_params.start_iter).  Inputs are resident in HBM before the timed region.

Prints one JSON line.  Besides the contract's keys: slice-SVT/s; the dominant
kernel's roofline (VALU: FP64 dot products and FP32 rotations, counted as the
method needs them); the FP64 oracle on this host (all threads and one thread,
CPU model); and, in the default run, further legs of the metric: the
256x256x3x100 workload with FP32 and BF16x3 transforms and their errors vs the
oracle, the 1080 x 1920 frames, the video under the DFT (complex Hermitian
Jacobi, and the real embeddings beside it), the 64-problem mix through the
batch engine (mixed-precision batched form vs the plain FP32 per-request
form), a bounded served stream (p50/p99), and the whole 200-iteration video
job from X = 0.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_VALU = 78.6e12
PEAK_FP32_VALU = 157.3e12
PEAK_HBM = 8.0e12

JACOBI_SRC = os.path.join(ROOT, "paper_2202_02870_amd", "csrc", "lt_jacobi.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_jacobi_warm_video_144x176x3x50.md")
TRAFFIC_PROFILE_DFT = os.path.join(ROOT, "profiles", "k_jacobi_cx_video_dft_144x176x3x50.md")


def svt_time_at_peak(m, n, sweeps_total):
    """Algorithmic work of the one-sided Jacobi SVD of m x n slices (m rows,
    n columns) summed over slices with sweeps_total sweeps in all: per sweep,
    n(n-1)/2 column pairs, each with three FP64 dot products (6 m flops) and the
    FP32 rotation of the pair's data and rotation-accumulator columns
    (6 m + 6 n flops).  Returns (FP64 flops, FP32 flops, seconds at the MI355X
    vector peaks)."""
    pairs = n * (n - 1) // 2
    f64 = float(sweeps_total) * pairs * 6 * m
    f32 = float(sweeps_total) * pairs * (6 * m + 6 * n)
    return f64, f32, f64 / PEAK_FP64_VALU + f32 / PEAK_FP32_VALU


def svt_time_at_peak_complex(m, n, sweeps_total):
    """The same for complex m x n slices (Fourier transforms) under Hermitian
    rotations: per column pair three complex dot products in FP64 (|a|^2 and
    |b|^2, 4 m flops each, and a^H b, 8 m) and in FP32 the rotation of the pair's
    data and accumulator columns (the phase on one column, 6 flops per entry,
    and the real rotation of both, 12 flops per entry: 18 (m + n) flops)."""
    pairs = n * (n - 1) // 2
    f64 = float(sweeps_total) * pairs * 16 * m
    f32 = float(sweeps_total) * pairs * 18 * (m + n)
    return f64, f32, f64 / PEAK_FP64_VALU + f32 / PEAK_FP32_VALU


def kernel_flops_complex(m, n, sweeps, rotations, slices):
    """What the complex kernel executes: per sweep and slice n(n-1)/2 pair
    products a^H b (8 m FP64 flops) and n column norms (4 m), the final norms,
    and per applied rotation 18 m FP32 flops (phase, then rotation)."""
    pairs = n * (n - 1) // 2
    f64 = sweeps * (pairs * 8 * m + n * 4 * m) + slices * n * 4 * m
    f32 = rotations * 18 * m
    return f64, f32


def kernel_flops(rows, n, sweeps, rotations, slices, dot32=False, rot_rows=None):
    """What the kernel itself executes: per sweep and slice n(n-1)/2 pair dot
    products of 2 rows flops and n column norms of 2 rows FP64 flops (rows: the
    Jacobi's working rows, n on the Cholesky-QR factor); per applied rotation
    6 rot_rows FP32 flops; the final column norms."""
    pairs = n * (n - 1) // 2
    dots = sweeps * pairs * 2 * rows
    f64 = sweeps * n * 2 * rows + slices * n * 2 * rows + (0 if dot32 else dots)
    f32 = rotations * 6 * (rot_rows or rows) + (dots if dot32 else 0)
    return f64, f32


def threads_used():
    try:
        from threadpoolctl import threadpool_info
        blas = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if blas:
            return int(blas[0]["num_threads"])
    except Exception:
        pass
    return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_traffic(profile=TRAFFIC_PROFILE):
    """HBM bytes per Jacobi launch on the video workload (k_jacobi_warm; with the
    DFT, the complex k_jacobi) from the committed FETCH_SIZE / WRITE_SIZE
    summary, if it was taken on the current kernel source (its SHA-256 is
    recorded there), else None."""
    try:
        text = open(profile).read()
        src = hashlib.sha256(open(JACOBI_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    mt = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    ms = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    if mt and ms and ms.group(1) == src:
        return int(mt.group(1))
    return None


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed iterations (default: 200 video, 100 large, 30 big; 50 mix ticks)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--start", type=int, default=None,
                    help="untimed iterations before the warm-up (default 100 video/large, 20 big)")
    ap.add_argument("--precision", default="f32", choices=["f32", "bf16x3"])
    ap.add_argument("--workload", default="video", choices=["video", "large", "big", "frames", "mix", "serve"])
    ap.add_argument("--frame-height", type=int, default=1080, choices=[1080, 2160],
                    help="frames workload: 1080 x 1920 or 2160 x 3840 frontal slices")
    ap.add_argument("--legs", default="all",
                    help="video workload: extra legs, comma list of job,large,frames,dft,mix,serve, 'all' or 'none'")
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
                    help="oracle iterations timed on the host with all threads (default 30 video, 10 large)")
    ap.add_argument("--cpu-iters-1t", type=int, default=None,
                    help="oracle iterations timed on one thread (default 5 video, 2 large)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="run one 256 MiB device copy before the timed region (counter reference)")
    ap.add_argument("--transform", default="dct", choices=["dct", "dft"],
                    help="video workload: transform along the trailing modes (dft: the t-product form)")
    ap.add_argument("--no-precondition", action="store_true",
                    help="run the Jacobi SVD on the slices themselves (no Cholesky-QR factor)")
    ap.add_argument("--warm-restart", type=int, default=0,
                    help="cold Jacobi start every this many iterations (0: library default 256; -1: never warm)")
    ap.add_argument("--fp32-dots", action="store_true", help="FP32 pair dot products in the Jacobi (default FP64)")
    ap.add_argument("--lanes", default="auto",
                    help="mix workload: Jacobi lanes per column pair (4..64, 0 = built-in, auto = timed)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"video": 200, "large": 100, "big": 30, "frames": 10, "mix": 50, "serve": 0}[args.workload]
    if args.start is None:
        args.start = {"video": 100, "large": 100, "big": 20, "frames": 10}.get(args.workload, 0)

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
        print(json.dumps(bench_mix(args, torch, lt, wl)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args, torch, lt, wl)), flush=True)
        return
    line = bench_completion(args, torch, lt, wl)
    if args.workload == "video" and args.transform == "dct":
        legs = set() if args.legs == "none" else (
            {"large", "frames", "dft", "mix", "serve", "job"} if args.legs == "all" else set(args.legs.split(",")))
        extra = {}
        for name, fn in (("job", leg_job), ("large", leg_large), ("frames", leg_frames), ("dft", leg_dft),
                         ("mix", leg_mix), ("serve", leg_serve)):
            if name in legs:
                say("leg", name)
                try:
                    extra[name] = (fn(args, torch, lt, wl, line["ms_per_step"]) if name == "dft"
                                   else fn(args, torch, lt, wl))
                except Exception as e:   # a failed leg is reported; the headline is still printed
                    extra[name] = {"error": "%s: %s" % (type(e).__name__, e)}
                torch.cuda.empty_cache()
        if extra:
            line["legs"] = extra
    print(json.dumps(line), flush=True)


def run_window(lt, M, mask, p, X, ws, args, precision, start, warmup, steps, fp32_dots=False):
    """start untimed iterations from X = 0, warmup more, then steps timed ones,
    each call continuing the run; returns (seconds, report, profile, window)."""
    import torch
    s = p.schedule

    def params(iters, k0):
        return lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0, max_iter=iters,
                             precision=precision, precondition=not args.no_precondition,
                             warm_restart=args.warm_restart, fp32_dots=fp32_dots, start_iter=k0)

    k = 0
    if start > 0:
        lt.complete_pga(M, mask, params(start, 0), p.kinds, out=X, ws=ws)
        k = start
    if warmup > 0:
        lt.complete_pga(M, mask, params(warmup, k), p.kinds, out=X, ws=ws)
        k += warmup
    torch.cuda.synchronize()
    if args.pmc_calibrate:
        # a plain device copy of known size (256 MiB read + 256 MiB written): the
        # reference that turns hardware byte counters into HBM bytes
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    lt.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep, _ = lt.complete_pga(M, mask, params(steps, k), p.kinds, out=X, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof, _ = lt.profile_end()
    return t1 - t0, rep, prof, (k + 1, k + steps)


def oracle_rate(o, p, iters, threads=None):
    """The FP64 oracle's iterations/s over the first `iters` iterations, its
    iterate, and the BLAS threads used."""
    s = p.schedule
    mats = o.mats_for(p.shape, list(p.kinds))

    def run():
        c0 = time.perf_counter()
        Xo, _ = o.complete_pga(p.M, p.mask, mats, mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0,
                               max_iter=iters)
        return iters / (time.perf_counter() - c0), Xo

    if threads is None:
        return run() + (threads_used(),)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=threads):
        return run() + (threads,)


def gpu_iterate(lt, M, mask, p, precision, iters, fp32_dots=False):
    s = p.schedule
    prm = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0, max_iter=iters,
                        precision=precision, fp32_dots=fp32_dots)
    X, _, _ = lt.complete_pga(M, mask, prm, p.kinds)
    return lt.to_host(X).astype(np.float64)


def bench_completion(args, torch, lt, wl):
    if args.workload == "video":
        p = wl.config1(transform=args.transform)
    elif args.workload == "frames":
        p = wl.config_frames(args.frame_height)
    else:
        p = {"large": wl.config2, "big": wl.config4_large}[args.workload]()
    shape = p.shape
    I1, I2 = shape[0], shape[1]
    P = wl.n_slices(shape)
    m, n = max(I1, I2), min(I1, I2)
    M = lt.to_device(p.M)
    mask = lt.to_device(p.mask, dtype=torch.uint8)
    X = lt.fortran_empty(shape)
    ws = torch.empty(lt.workspace_bytes(shape, p.kinds, "pga", args.precision), dtype=torch.uint8, device="cuda")
    elapsed, rep, prof, window = run_window(lt, M, mask, p, X, ws, args, args.precision, args.start, args.warmup,
                                            args.steps, args.fp32_dots)
    value = args.steps / elapsed

    # dominant kernel: the Jacobi SVT.  Work counted as the method needs it (three
    # FP64 dots and the FP32 rotations of data and accumulator per column pair of
    # the m x n slice, at the measured sweeps), over the kernel's mean event-timed
    # launch duration on the library's stream.
    jcalls, jms = prof["jacobi"]
    path = lt.svt_path(shape, p.kinds, precondition=not args.no_precondition)
    precond = "precond" in path
    dft = "dft" in p.kinds
    cx = "complex" in path   # Fourier: complex slices (or factors), or else their real embeddings
    jm, jn = (2 * m, 2 * n) if dft and not cx else (m, n)
    warm = lt.pga_warm(shape, p.kinds, precondition=not args.no_precondition, warm_restart=args.warm_restart)
    t_launch = jms / 1e3 / max(jcalls, 1)
    if cx:
        f64, f32, t_peak = svt_time_at_peak_complex(m, n, rep["total_sweeps"])
    else:
        f64, f32, t_peak = svt_time_at_peak(jm, jn, rep["total_sweeps"])
    flops = (f64 + f32) / max(jcalls, 1)
    t_peak /= max(jcalls, 1)
    rows = jn if precond else jm
    rot_rows = rows + 4 * ((jn + 3) // 4) if warm else rows
    if cx:
        cm = n if precond else m   # complex rows of the Jacobi's columns (the n x n factor, or the slice)
        rows = rot_rows = 2 * cm   # as interleaved real rows
        k64, k32 = kernel_flops_complex(cm, n, rep["total_sweeps"], rep["total_rotations"], rep["total_slices"])
    else:
        k64, k32 = kernel_flops(rows, jn, rep["total_sweeps"], rep["total_rotations"], rep["total_slices"],
                                dot32=args.fp32_dots, rot_rows=rot_rows)
    tk_peak = (k64 / PEAK_FP64_VALU + k32 / PEAK_FP32_VALU) / max(jcalls, 1)
    # the slices run side by side, one workgroup each: a launch lasts as long as
    # its slowest slice, whose sweeps per iteration are reported beside the mean
    mean_sw = rep["total_sweeps"] / max(rep["total_slices"], 1)
    slowest = rep["slowest_sweeps"] / max(rep["iters"], 1)
    default_cfg = (args.workload == "video" and args.transform == "dct" and args.precision == "f32" and precond
                   and warm and not args.fp32_dots)
    dft_cfg = (args.workload == "video" and args.transform == "dft" and args.precision == "f32" and precond
               and cx and not args.fp32_dots)
    roofline = {"bound": "alu", "kernel": "k_jacobi_warm" if warm else "k_jacobi",
                "achieved": round(flops / t_launch / 1e12, 3) if t_launch > 0 else None,
                "peak": round(flops / t_peak / 1e12, 2) if t_peak > 0 else None, "unit": "TFLOP/s",
                "frac": round(t_peak / t_launch, 4) if t_launch > 0 else None,
                "traffic": (measured_traffic() if default_cfg else
                            measured_traffic(TRAFFIC_PROFILE_DFT) if dft_cfg else None),
                "count": ("per sweep of a complex m x n slice: n(n-1)/2 pairs x (16m FP64 + 18(m+n) FP32) flops"
                          if cx else
                          "per sweep of an m x n slice: n(n-1)/2 pairs x (6m FP64 + 6m+6n FP32) flops")
                + ", measured sweeps; peak = time at 78.6 (FP64) and 157.3 (FP32) TFLOP/s",
                "flops_per_launch": flops, "time_at_peak_us": round(t_peak * 1e6, 2),
                "launch_ms": round(t_launch * 1e3, 4), "launches": jcalls,
                "frac_kernel_count": round(tk_peak / t_launch, 4) if t_launch > 0 else None,
                "slowest_slice_sweeps": round(slowest, 3),
                "frac_at_slowest_sweeps": round(t_peak * slowest / mean_sw / t_launch, 4)
                if t_launch > 0 and mean_sw > 0 else None,
                "slice": [jm, jn], "complex": cx, "jacobi_rows": rows, "rotated_rows": rot_rows,
                "preconditioned": precond,
                "warm_start": warm, "svt_path": path, "pair_dots": "fp32" if args.fp32_dots else "fp64"}
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
        "config": {"workload": p.name, "shape": list(shape), "slices_per_step": P, "precision": args.precision,
                   "schedule": "mu0=0.9||P_Omega M||, nu=0.9, mu_bar=1e-4 mu0",
                   "timed_iterations": list(window)},
        "slice_svt_per_s": round(value * P, 1),
        "mean_sweeps": round(mean_sw, 3),
        "slowest_slice_sweeps": round(slowest, 3),
        "kernel_ms": {k: round(v[1], 3) for k, v in prof.items()},
        "kernel_calls": {k: v[0] for k, v in prof.items()},
        "roofline": roofline,
    }
    cpu_iters = args.cpu_iters if args.cpu_iters is not None else \
        {"video": 30, "large": 10, "big": 1, "frames": 0}[args.workload]
    cpu_1t = args.cpu_iters_1t if args.cpu_iters_1t is not None else \
        {"video": 5, "large": 2, "big": 0, "frames": 0}[args.workload]
    if not args.no_cpu_baseline and cpu_iters > 0:
        import oracle as o
        say("oracle on the host:", cpu_iters, "iterations, all threads")
        rate, Xo, cores = oracle_rate(o, p, cpu_iters)
        cb = {"value": round(rate, 4), "unit": "iters/s", "cores": cores, "kind": "oracle",
              "sample": "first %d PGA iterations of the same workload, FP64 NumPy/LAPACK, %d BLAS threads"
                        % (cpu_iters, cores),
              "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        if cpu_1t > 0:
            say("oracle on the host:", cpu_1t, "iterations, one thread")
            r1, _, _ = oracle_rate(o, p, cpu_1t, threads=1)
            cb["single_thread"] = {"value": round(r1, 4), "unit": "iters/s", "cores": 1,
                                   "sample": "first %d PGA iterations, one BLAS thread (the paper's "
                                             "single-core protocol)" % cpu_1t}
        line["cpu_baseline"] = cb
        Xg = gpu_iterate(lt, M, mask, p, args.precision, cpu_iters, args.fp32_dots)
        nrm = float(np.linalg.norm(Xo))
        err = ({"rel_err_vs_oracle": float(np.linalg.norm(Xg - Xo) / nrm)} if nrm > 0 else
               {"abs_norm_gpu_where_oracle_is_zero": float(np.linalg.norm(Xg))})
        bound = 1e-4 if args.precision == "f32" else 1e-2
        ok = err.get("rel_err_vs_oracle", 0.0) <= bound and err.get("abs_norm_gpu_where_oracle_is_zero", 0.0) == 0.0
        if not ok:
            say("PARITY: the GPU iterate after %d iterations is outside the bound %g: %s" % (cpu_iters, bound, err))
        line["parity"] = {"iters": cpu_iters, **err, "bound": bound, "within_bound": ok,
                          "full_length": "200 iterations at full size in tests/test_gpu_configs.py"}
    return line


def leg_job(args, torch, lt, wl):
    """The whole 200-iteration video job from X = 0, one call."""
    p = wl.config1()
    s = p.schedule
    M = lt.to_device(p.M)
    mask = lt.to_device(p.mask, dtype=torch.uint8)
    prm = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0, max_iter=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep, _ = lt.complete_pga(M, mask, prm, p.kinds)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"iterations": 200, "seconds": round(dt, 4), "iters_per_s": round(200 / dt, 2),
            "mean_sweeps": round(rep["total_sweeps"] / rep["total_slices"], 3),
            "nuclear_norm": rep["nuclear_norm"]}


def leg_large(args, torch, lt, wl):
    """256x256x3x100 (300 slices of 256 x 256), FP32 and BF16x3 transforms:
    iterations 103..132 of a run timed, and the error of the first 12
    iterations vs the FP64 oracle (the iterates are nonzero from the eighth)."""
    import oracle as o
    p = wl.config2()
    M = lt.to_device(p.M)
    mask = lt.to_device(p.mask, dtype=torch.uint8)
    X = lt.fortran_empty(p.shape)
    out = {"workload": p.name}
    k_or = 12
    say("  oracle", k_or, "iterations")
    rate, Xo, cores = oracle_rate(o, p, k_or)
    out["oracle"] = {"iters_per_s": round(rate, 4), "cores": cores, "iters": k_or}
    nrm = float(np.linalg.norm(Xo))
    for prec in ("f32", "bf16x3"):
        ws = torch.empty(lt.workspace_bytes(p.shape, p.kinds, "pga", prec), dtype=torch.uint8, device="cuda")
        dt, rep, prof, window = run_window(lt, M, mask, p, X, ws, args, prec, 100, 2, 30)
        del ws
        Xg = gpu_iterate(lt, M, mask, p, prec, k_or)
        e = float(np.linalg.norm(Xg - Xo) / nrm) if nrm > 0 else None
        bound = 1e-4 if prec == "f32" else 1e-2
        if e is None or e > bound:
            say("PARITY: %s large workload after %d iterations: %s (bound %g)" % (prec, k_or, e, bound))
        out[prec] = {"iters_per_s": round(30 / dt, 2), "timed_iterations": list(window),
                     "slice_svt_per_s": round(30 * 300 / dt, 1),
                     "mean_sweeps": round(rep["total_sweeps"] / rep["total_slices"], 3),
                     "jacobi_ms_per_launch": round(prof["jacobi"][1] / max(prof["jacobi"][0], 1), 3),
                     "rel_err_vs_oracle_at_%d" % k_or: e, "bound": bound,
                     "within_bound": e is not None and e <= bound}
    return out


def leg_frames(args, torch, lt, wl):
    """The 1080 x 1920 x 3 x 2 frames (six slices of 1080 x 1920, sr 0.1):
    iterations 11..15 of a run timed (the wide blocked Jacobi on the 1080 x 1080
    Cholesky factors); parity of this path is in tests/test_gpu_wide.py."""
    p = wl.config_frames(1080)
    M = lt.to_device(p.M)
    mask = lt.to_device(p.mask, dtype=torch.uint8)
    X = lt.fortran_empty(p.shape)
    ws = torch.empty(lt.workspace_bytes(p.shape, p.kinds, "pga"), dtype=torch.uint8, device="cuda")
    a = argparse.Namespace(**vars(args))
    a.no_precondition, a.warm_restart, a.pmc_calibrate = False, 0, False
    dt, rep, prof, window = run_window(lt, M, mask, p, X, ws, a, "f32", 9, 1, 5)
    P = wl.n_slices(p.shape)
    return {"workload": p.name, "iters_per_s": round(5 / dt, 3), "timed_iterations": list(window),
            "slice_svt_per_s": round(5 * P / dt, 2), "svt_path": lt.svt_path(p.shape, p.kinds),
            "mean_sweeps": round(rep["total_sweeps"] / rep["total_slices"], 3),
            "kernel_ms": {k: round(v[1], 3) for k, v in prof.items()}}


def leg_dft(args, torch, lt, wl, dct_ms=None):
    """The same video workload under the DFT along both trailing modes (the
    t-product's TNN-PGA-F): iterations 106-125 timed on the complex Hermitian
    Jacobi (76 conjugate-pair representatives of 144 x 176), then on the real
    288 x 352 embeddings (LT_DFT_EMBED=1) for comparison."""
    p = wl.config1(transform="dft")
    M = lt.to_device(p.M)
    mask = lt.to_device(p.mask, dtype=torch.uint8)
    ws = torch.empty(lt.workspace_bytes(p.shape, p.kinds, "pga"), dtype=torch.uint8, device="cuda")
    a = argparse.Namespace(**vars(args))
    a.no_precondition, a.warm_restart, a.pmc_calibrate = False, 0, False
    out = {"workload": p.name}
    for key, embed in (("complex", False), ("embedding", True)):
        if embed:
            os.environ["LT_DFT_EMBED"] = "1"
        try:
            X = lt.fortran_empty(p.shape)
            dt, rep, prof, window = run_window(lt, M, mask, p, X, ws, a, "f32", 100, 5, 20)
            out[key] = {"iters_per_s": round(20 / dt, 3), "ms_per_iter": round(dt / 20 * 1e3, 4),
                        "svt_path": lt.svt_path(p.shape, p.kinds),
                        "mean_sweeps": round(rep["total_sweeps"] / max(rep["total_slices"], 1), 3),
                        "jacobi_ms_per_iter": round(prof["jacobi"][1] / max(prof["jacobi"][0], 1), 4)}
            if not embed:   # HBM bytes per complex Jacobi launch, from the committed counters
                out[key]["jacobi_traffic"] = measured_traffic(TRAFFIC_PROFILE_DFT)
        finally:
            if embed:
                del os.environ["LT_DFT_EMBED"]
    out["timed_iterations"] = list(window)
    if dct_ms:
        out["step_over_dct_step"] = round(out["complex"]["ms_per_iter"] / dct_ms, 3)
    return out


def leg_mix(args, torch, lt, wl):
    """The benchmark spec's comparison on the 64-problem mix: mixed-precision
    batched form (BF16x3 transforms, one batch-engine tick per iteration over
    all problems, graph-replayed) vs the plain FP32 per-request form."""
    a = argparse.Namespace(**vars(args))
    a.steps, a.warmup, a.precision, a.per_request_iters, a.lanes = 30, 5, "bf16x3", 3, "auto"
    r = bench_mix(a, torch, lt, wl)
    keep = ("value", "unit", "slice_svt_per_s", "per_request_f32_slice_svt_per_s", "batched_over_per_request",
            "batched_f32_slice_svt_per_s", "batched_over_batched_f32", "mean_sweeps", "jacobi_lanes", "config")
    return {k: r[k] for k in keep}


def leg_serve(args, torch, lt, wl):
    """A bounded served stream: 40 requests (10% of 512x512x3x64), Poisson
    arrivals at 0.7x the measured saturation rate."""
    a = argparse.Namespace(**vars(args))
    a.requests, a.rate, a.large_frac = 40, 0.0, 0.1
    r = bench_serve(a, torch, lt, wl)
    keep = ("value", "unit", "p50_s", "p99_s", "completed", "rejected", "mean_iters", "peak_resident_GB", "config")
    return {k: r[k] for k in keep}


def bench_mix(args, torch, lt, wl):
    """64 independent problems of uneven shapes (order 3/4, I1, I2 in 32..256,
    trailing {3,8,16} x {1,10,30}); a step is one tick of the batch engine: one
    PGA iteration of every problem, with all frontal slices of all problems in
    one Jacobi launch per kernel family (graph-replayed ticks).  The plain FP32
    per-request form (one lt_complete_pga call per problem) is timed alongside."""
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
    del gps
    # eager ticks with per-kernel events (same work, no graph) for the kernel split
    gps2 = [lt.Problem(M, mask, params, p.kinds) for (p, M, mask, params) in dev]
    b2 = lt.Batch(gps2, use_graph=False, jacobi_lanes=lanes)
    b2.step(args.warmup)
    lt.profile_begin()
    b2.step(min(args.steps, 20))
    prof, _ = lt.profile_end()
    b2.close()
    del gps2
    # the same batch with FP32 transforms: what the BF16x3 split itself buys
    batched_f32 = None
    if args.precision != "f32":
        gps3 = []
        for (p, M, mask, params) in dev:
            s = p.schedule
            pf = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0,
                               max_iter=args.steps + args.warmup, precision="f32")
            gps3.append(lt.Problem(M, mask, pf, p.kinds))
        b3 = lt.Batch(gps3, use_graph=True, jacobi_lanes=lanes)
        if args.warmup > 0:
            b3.step(args.warmup)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        b3.step(args.steps)
        torch.cuda.synchronize()
        batched_f32 = args.steps * total_slices / (time.perf_counter() - f0)
        b3.close()
        del gps3
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
    return {
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
                   "precision": args.precision, "per_request_precision": "f32"},
        "slice_svt_per_s": round(value * total_slices, 1),
        "per_request_f32_slice_svt_per_s": round(per_req_slices, 1),
        "batched_over_per_request": round(value * total_slices / per_req_slices, 3),
        "batched_f32_slice_svt_per_s": round(batched_f32, 1) if batched_f32 else None,
        "batched_over_batched_f32": round(value * total_slices / batched_f32, 3) if batched_f32 else None,
        "mean_sweeps": round(sum(r["total_sweeps"] for r in reps) / max(sum(r["total_slices"] for r in reps), 1), 3),
        "kernel_ms_20_eager_ticks": {k2: round(v[1], 3) for k2, v in prof.items()},
        "jacobi_lanes": lanes if lanes else "built-in",
        "autotune_jacobi_ms_per_tick": ({str(g): round(t, 4) for g, t in sorted(tune_ms.items())}
                                        if tune_ms else None),
    }


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
        say("finished request %d %s: %d iterations, latency %.3f s" % (r.rid, "x".join(map(str, r.M.shape)),
                                                                       r.iters, r.latency))

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
    return {
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


if __name__ == "__main__":
    main()
