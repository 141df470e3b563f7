#!/usr/bin/env python
"""Time-to-solution of the SAP-preconditioned FGCR Wilson-clover solve on one GPU.

One step = one full solve A x = b to true relative residual 1e-10 (all rows
of the hot path: FP64 operator, Schwarz preconditioner with MR block solves,
Gram-Schmidt, solution update), inputs resident in HBM, gauge field and
clover term loaded beforehand.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload C2|C3|C1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve time @rel.res 1e-10; SAP Dslash Gflop/s & %HBM/FP32 peak; mixed vs FP64"
FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", default="sweeps", choices=["queue", "sweeps"],
                    help="block-solve schedule: persistent work queue or one launch per half-sweep")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-preconditioner comparison solve")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this many MiB (a known-size kernel for "
                         "calibrating profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the lattice is solved whole on a single "
              "MI355X; multi-GPU sharding is not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1412_2629_amd import configs, ddqcd, geometry, inputs

    w = configs.WORKLOADS[args.workload]
    log(f"[bench] workload {w.name}: generating inputs")
    U = inputs.random_gauge(w.lattice, w.eps, w.gauge_seed)
    f = inputs.gaussian_source(w.lattice, w.source_seed)
    dev = torch.device("cuda:0")
    Ud = torch.from_numpy(U).to(dev)
    fd = torch.from_numpy(f).to(dev)
    ctx = ddqcd.Context(w.lattice, w.domain, w.kappa, w.csw, w.bc)
    ctx.load_gauge(Ud)
    ctx.set_solver(w.restart, w.tol, 64)
    ctx.set_schedule(args.schedule)
    del Ud

    def solve(prec):
        ctx.set_sap(w.n_cycles, w.n_mr, prec)
        x, info, st = ctx.solve(fd)
        if st != 0:
            raise RuntimeError(f"solve did not converge: {info}")
        return x, info[0]

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration_mib} MiB done")
        del a, b
    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        solve(w.prec)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        x, info = solve(w.prec)
        infos.append(info)
    torch.cuda.synchronize()
    t_solve = (time.perf_counter() - t0) / args.steps
    log(f"[bench] {args.steps} solves, {t_solve * 1e3:.2f} ms each, {infos[-1]['iters']} FGCR steps")

    # true residual of the last solution, FP64 operator on the GPU
    r = fd - ctx.apply_D(x, "f64")
    true_res = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(fd))

    iters = infos[-1]["iters"]
    sap_ms = sum(i["t_sap_ms"] for i in infos) / len(infos)
    nd = w.volume // geometry.volume(w.domain)
    per_dom = geometry.sap_flops_per_domain(w.domain, w.n_mr)
    # one preconditioner call = n_cycles visits of every domain; it is one
    # launch of the work-queue kernel, or 2 * n_cycles half-sweep launches
    call_ms = sap_ms / iters
    launches_per_call = 1 if args.schedule == "queue" else 2 * w.n_cycles
    launch_ms = call_ms / launches_per_call
    flops_call = per_dom["total"] * nd * w.n_cycles
    achieved_tflops = flops_call / (call_ms * 1e-3) / 1e12
    dslash_gflops = per_dom["dslash"] * nd * w.n_cycles / (call_ms * 1e-3) / 1e9
    kernel = "k_sap_queue" if args.schedule == "queue" else "k_sap_lds"

    fp64 = None
    if not args.no_fp64 and w.prec != "f64":
        log("[bench] FP64-preconditioner comparison solve")
        try:
            solve("f64")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, i64 = solve("f64")
            torch.cuda.synchronize()
            fp64 = {"fp64_sap_solve_s": round(time.perf_counter() - t1, 5), "fp64_sap_iters": i64["iters"]}
            fp64["speedup"] = round(fp64["fp64_sap_solve_s"] / t_solve, 3)
        except ddqcd.DDQCDError as e:
            fp64 = {"unavailable": str(e)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, U, f, iters)

    out = {
        "metric": METRIC,
        "value": round(t_solve, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_solve * 1e3, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32+f64", "f16": "f16-storage/f32+f64"}[w.prec],
        "data": "synthetic",
        "config": {"workload": f"{w.name}: lattice {w.lattice}, kappa {w.kappa}, c_sw {w.csw}, eps {w.eps}, "
                               f"domains {w.domain}, SAP {w.n_cycles} cycles x {w.n_mr} MR ({w.prec}), "
                               f"FGCR restart {w.restart} (f64), tol {w.tol}, schedule {args.schedule}",
                   "global_batch": 1, "parallelism": "single GPU"},
        "fgcr_steps": iters,
        "true_rel_residual": true_res,
        "time_split_ms": {k: round(sum(i[k] for i in infos) / len(infos), 3)
                          for k in ("t_sap_ms", "t_A_ms", "t_gs_ms", "t_other_ms")},
        "sap_dslash_gflops": round(dslash_gflops, 1),
        "sap_total_tflops": round(achieved_tflops, 3),
        "sap_call_ms": round(call_ms, 4),
        "sap_launch_ms": round(launch_ms, 5),
        "roofline": {"kernel": kernel, "bound": "alu", "achieved": round(achieved_tflops, 3),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved_tflops / FP32_PEAK_TFLOPS, 4),
                     "traffic": None},
        "mixed_vs_fp64": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(w, U, f, gpu_iters):
    """The FP64 oracle on the host: a bounded sample of the same solve (two
    FGCR steps with the same SAP parameters), scaled to the GPU run's number
    of FGCR steps."""
    import numpy as np

    import oracle as O
    log("[bench] cpu baseline (oracle)")
    C = O.clover_field(w.lattice, U, w.kappa, w.csw)
    Ci = O.clover_inverse(C)
    nstep = 2
    t0 = time.perf_counter()
    O.fgcr(w.lattice, w.domain, w.bc, U, C, Ci, f, n_cycles=w.n_cycles, n_mr=w.n_mr, restart=nstep,
           tol=1e-300, max_cycles=1)
    dt = time.perf_counter() - t0
    per_step = dt / nstep
    return {"value": round(per_step * gpu_iters, 3), "unit": "s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{nstep} FGCR steps of the same solve (FP64 SAP {w.n_cycles}x{w.n_mr}, A, Gram-Schmidt, "
                      f"one restart) in {dt:.1f} s, scaled to the GPU solve's {gpu_iters} steps"}


if __name__ == "__main__":
    main()
