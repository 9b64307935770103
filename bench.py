#!/usr/bin/env python3
"""Frequency solves/s at FP64 relative residual 1e-6 on MI355X.

Workload (one "step"): the pressurised spherical cavity in full space,
icosphere level 4 (5120 flat triangles, 15,360 complex unknowns), unit
material (mu = rho = 1, nu = 1/4), 64 Laplace parameters s_k = 0.25 + i k pi/20
with a Heaviside pressure; every frequency is assembled and solved until the
true residual ||b - A x|| / ||b|| with the FP64 operator is <= 1e-6.

Timed paths (same mesh, same s list, same GPU):
  * optimised: FP32 hi-plane GMRES inside FP64 iterative refinement, previous-
    frequency warm start  -> ``value``
  * plain FP64: FP64 storage and GMRES(50) with block-Jacobi, zero x0 -> ``plain_fp64``
Inputs (mesh plan, boundary values) are resident in HBM before timing starts.

Also reported: the roofline of the dominant kernel -- the FP64 far-field
assembly kernel, VALU-bound; its launches are timed with HIP events on the
assembly stream during the timed steps -- with the GEMV that streams the matrix
(HBM-bound) beside it, the lockstep batched path on the same workload, and the
FP64 CPU oracle timed on this host on a bounded sample.

Algorithmic work per unit (counted from the formulas as implemented, closed-
form branch of the radial functions; each sqrt, division, exp and sincos
counted as one operation):
  far field, per quadrature node (7 per source element, every pair m != n):
    geometry 22 + radial functions 118 + traction coefficients 24
    + traction invariants 63 + U.t for b 60 + 7 special functions
    + per-pair expansion 90 / 7  ->  307 FP64 flops
  GEMV: N^2 * 8 bytes (FP32 hi plane) per product.
HBM traffic of these kernels from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE,
FETCH_SIZE scaled by 2.0 (it reads 524,300 KiB for a 1 GiB device copy,
WRITE_SIZE 1,048,576 KiB).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frequency solves/s at rel-res 1e-6: mixed+batched+learned vs plain FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FAR_FLOPS_PER_NODE = 307.0
FAR_NODES = 7
# HBM bytes per launch, rocprofv3 --pmc on this workload (FETCH_SIZE x 2.0 + WRITE_SIZE)
FAR_TRAFFIC_BYTES = (2.0 * 21978.77 + 3736212.70) * 1024
GEMV32_TRAFFIC_BYTES = 2.0 * 923563.31 * 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=4)
    ap.add_argument("--nfreq", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 path")
    ap.add_argument("--no-batched", action="store_true", help="skip the lockstep batched path")
    ap.add_argument("--cpu-freqs", type=int, default=1)
    ap.add_argument("--warm", choices=["none", "prev"], default="prev",
                    help="initial guess of the optimised path")
    ap.add_argument("--batch", type=int, default=0,
                    help="optimised path: 1 = one frequency at a time, 0 = assembly of the next frequency "
                         "overlapped with the Krylov phase of the current one")
    return ap.parse_args()


def timed(P, s, bc, opts, steps, warmup, torch):
    out = None
    for _ in range(warmup):
        out = P.solve(s, bc, opts, out=out, want_ut=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = P.solve(s, bc, opts, out=out, want_ut=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, out


def cpu_baseline(mesh, s_list, nfreq):
    import numpy as np

    from oracle import bem
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    for sk in s_list[1:1 + nfreq]:
        A, b = bem.assemble(mesh, sk)
        bem.solve_dense(A, b)
        del A
    dt = time.perf_counter() - t0
    return {"value": nfreq / dt, "unit": "frequency solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{nfreq} frequency of the same workload (s_1): FP64 oracle assembly (C, OpenMP) "
                      f"+ LAPACK LU solve, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(frequencies shard across GPUs with no communication, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1511_04355_amd as afs
    from synth import meshgen as mg

    torch.cuda.set_device(0)
    mesh = mg.cavity(args.level)
    s = mg.cavity_frequencies(args.nfreq)
    bc = torch.from_numpy(np.stack([np.asarray(mesh.bc_shape, np.complex128) / sk for sk in s])).cuda()
    t0 = time.perf_counter()
    P = afs.Problem.from_mesh(mesh)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    N = P.N

    warm = afs.WARM_PREV if args.warm == "prev" else afs.WARM_NONE
    mixed = afs.SolveOptions(tol=args.tol, precision=afs.PREC_MIXED, warm_start=warm, profile=1, batch=args.batch)
    ms_mixed, out = timed(P, s, bc, mixed, args.steps, args.warmup, torch)
    st = out["stats"]
    worst = max(x["rel_res_fp64"] for x in st)
    assert worst <= args.tol, f"mixed path missed the tolerance: {worst}"
    far_ms = sum(x["t_far_ms"] for x in st) / len(st)
    far_flops = FAR_FLOPS_PER_NODE * FAR_NODES * float(P.n_tri) * (P.n_tri - 1)
    far_tf = far_flops / (far_ms * 1e-3) / 1e12
    g_ms = sum(x["gemv_ms"] for x in st)
    g_n = sum(x["gemv_count"] for x in st)
    g64_ms = sum(x["gemv64_ms"] for x in st)
    g64_n = sum(x["gemv64_count"] for x in st)
    bytes_per_launch = float(N) * N * 8  # hi plane, complex64
    avg_ms = g_ms / max(g_n, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    res = {
        "metric": METRIC,
        "value": args.nfreq / (ms_mixed * 1e-3),
        "unit": "frequency solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 GEMV / f64 assembly, Arnoldi, residual",
        "data": "synthetic",
        "config": {"workload": f"pressurised spherical cavity, icosphere level {args.level} "
                               f"({P.n_tri} triangles, {N} complex unknowns), {args.nfreq} frequencies "
                               f"s_k=0.25+ik*pi/20, FP64 true rel. residual <= {args.tol}",
                   "path": "mixed: FP32 hi-plane GMRES(50) + FP64 refinement, "
                           + ("previous-s warm start" if args.warm == "prev" else "zero start")
                           + (", assembly of s_k+1 overlapped with GMRES of s_k" if args.batch != 1 else ""),
                   "plan_s": plan_s},
        "roofline": {"bound": "alu", "achieved": far_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": far_tf / FP64_PEAK_TFLOPS, "traffic": FAR_TRAFFIC_BYTES,
                     "kernel": "far_assemble_kernel (FP64 far-field rule, split store)",
                     "flops_per_launch": far_flops, "avg_launch_ms": far_ms, "launches": len(st)},
        "gemv": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": achieved / HBM_PEAK_GBS, "traffic": GEMV32_TRAFFIC_BYTES,
                 "kernel": "gemv_split32_kernel (live, sharing the GPU with the next assembly)",
                 "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms, "launches": g_n},
        "solve": {"max_rel_res_fp64": worst,
                  "matvecs_per_solve": sum(x["iters"] for x in st) / len(st),
                  "refine_steps_per_solve": sum(x["refine_steps"] for x in st) / len(st),
                  "assemble_ms_per_solve": sum(x["t_assemble_ms"] for x in st) / len(st),
                  "solve_ms_per_solve": sum(x["t_solve_ms"] for x in st) / len(st),
                  "gemv32_ms_per_solve": g_ms / len(st),
                  "gemv64_ms_per_solve": g64_ms / len(st),
                  "gemv64_avg_ms": g64_ms / max(g64_n, 1)},
    }
    del out
    if not args.no_plain:
        plain = afs.SolveOptions(tol=args.tol, precision=afs.PREC_FP64, warm_start=afs.WARM_NONE, profile=1,
                                 batch=1)
        ms_plain, out = timed(P, s, bc, plain, args.steps, args.warmup, torch)
        sp = out["stats"]
        wp = max(x["rel_res_fp64"] for x in sp)
        gp_ms = sum(x["gemv_ms"] for x in sp)
        gp_n = sum(x["gemv_count"] for x in sp)
        res["plain_fp64"] = {"value": args.nfreq / (ms_plain * 1e-3), "ms_per_step": ms_plain,
                             "max_rel_res_fp64": wp,
                             "matvecs_per_solve": sum(x["iters"] for x in sp) / len(sp),
                             "assemble_ms_per_solve": sum(x["t_assemble_ms"] for x in sp) / len(sp),
                             "gemv_c128_avg_ms": gp_ms / max(gp_n, 1),
                             "gemv_c128_GBs": float(N) * N * 16 / (gp_ms / max(gp_n, 1) * 1e-3) / 1e9}
        res["speedup_vs_plain_fp64"] = res["value"] / res["plain_fp64"]["value"]
        del out
    if not args.no_batched:
        bopts = afs.SolveOptions(tol=args.tol, precision=afs.PREC_MIXED)
        for _ in range(args.warmup):
            outs, _ = afs.solve_batched([P], [s], [bc], bopts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            outs, _ = afs.solve_batched([P], [s], [bc], bopts)
        torch.cuda.synchronize()
        ms_b = (time.perf_counter() - t0) * 1e3 / args.steps
        sb = outs[0]["stats"]
        res["batched_lockstep"] = {"value": args.nfreq / (ms_b * 1e-3), "ms_per_step": ms_b,
                                   "max_rel_res_fp64": max(x["rel_res_fp64"] for x in sb),
                                   "inner_matvecs_per_solve": sum(x["iters"] for x in sb) / len(sb),
                                   "path": "all frequencies in waves solved in lockstep, FP32 inner cycles, "
                                           "FP64 residuals, next wave assembled during the current solve"}
        del outs
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(mesh, s, args.cpu_freqs)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
