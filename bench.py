#!/usr/bin/env python
"""Time-to-solution of the SAP-preconditioned FGCR Wilson-clover solve on one GPU.

One step = one full solve A x = b to true relative residual 1e-10 of every
right-hand side of the workload (all rows of the hot path: FP64 operator,
Schwarz preconditioner with MR block solves, Gram-Schmidt, solution update),
inputs resident in HBM, gauge field and clover term loaded beforehand.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload C4|C3|C2|C5|C1]

C4 is the default: 12 point sources on the 32^3x64 lattice solved together
(FP16-storage block solves, FP64 FGCR per right-hand side), the largest
single-GPU workload.  C3 is one Gaussian source on that lattice, C2 the
16^3x32 lattice with FP32 block solves, C5 the 24-lattice uneven batch in one
ddqcd_solve_batch call; for the batched workloads one step is the whole batch.
Beside the timed solve the same workload is solved with the FP64
preconditioner (the plain path) and with FP64 BiCGstab (no domain
decomposition), and the oracle is timed on the host.
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
CPU_BUDGET_S = 30.0          # bound on the oracle's host time

# HBM bytes per half-sweep launch of the block-solve kernel, from rocprofv3
# FETCH_SIZE / WRITE_SIZE passes calibrated against a plain device copy
# (profiles/k_sap_tile_32x32x32x64_12rhs_f16.md, profiles/k_sap_lds_32x32x32x64_f16_and_fgcr_blas.md).  They hold for the kernel sources
# they were taken on, identified by a hash; after any change to those sources
# the figure is reported as null until it is measured again.
# Keyed by (workload, domain shape, product form).
KERNEL_SOURCES = ("paper_1412_2629_amd/csrc/dd_sap.hip", "paper_1412_2629_amd/csrc/dd_device.h")
MEASURED_TRAFFIC = {("C4", (4, 4, 4, 4), "tile"): {"bytes_per_launch": 5.1026e9, "sources": "b43375ccdb70b66a"},
                    ("C3", (8, 4, 4, 4), "lane"): {"bytes_per_launch": 602.75e6, "sources": "b43375ccdb70b66a"}}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class System:
    """One lattice of the benchmark with its sources (one or more right-hand sides)."""

    def __init__(self, w, U, srcs, schedule="sweeps", schwarz="multiplicative", product="lane"):
        import numpy as np
        import torch

        from paper_1412_2629_amd import ddqcd
        self.w, self.U, self.srcs = w, U, srcs
        dev = torch.device("cuda:0")
        self.ctx = ddqcd.Context(w.lattice, w.domain, w.kappa, w.csw, w.bc)
        self.ctx.load_gauge(torch.from_numpy(U).to(dev))
        self.ctx.set_solver(w.restart, w.tol, 64)
        self.product = product
        self.ctx.set_sap(w.n_cycles, w.n_mr, w.prec, product)
        self.ctx.set_schedule(schedule)
        self.ctx.set_schwarz(schwarz)
        self.b = torch.from_numpy(np.ascontiguousarray(srcs[0] if len(srcs) == 1 else np.stack(srcs))).to(dev)


def build(name, schedule, tune=False, schwarz="multiplicative", domain=None, product="lane", lattice=None):
    import dataclasses

    import numpy as np
    import torch

    from paper_1412_2629_amd import configs, ddqcd, inputs
    if name == "C5":
        out = []
        for j, w in enumerate(configs.uneven_batch()):
            if lattice is not None and j != lattice:
                continue
            log(f"[bench] lattice {j} {w.lattice}: generating inputs")
            U = inputs.random_gauge(w.lattice, w.eps, w.gauge_seed)
            src = inputs.gaussian_source(w.lattice, w.source_seed)
            if tune:   # the domain shape this lattice solves fastest with (untimed set-up)
                dom, ms = ddqcd.tune_domain(w.lattice, w.kappa, w.csw, torch.from_numpy(U).cuda(),
                                            torch.from_numpy(src).cuda(), w.prec, w.n_cycles, w.n_mr, w.restart,
                                            w.tol, 64, w.bc)
                log(f"[bench] lattice {j}: domain {dom}" + (f" ({ms:.1f} ms)" if ms >= 0 else " (only fit)"))
                w = dataclasses.replace(w, domain=dom)
            out.append(System(w, U, [src], schedule, schwarz))
        return out
    w = configs.WORKLOADS[name]
    if domain is not None:
        w = dataclasses.replace(w, domain=domain)
    log(f"[bench] workload {w.name}: generating inputs")
    U = inputs.random_gauge(w.lattice, w.eps, w.gauge_seed)
    if w.nrhs > 1:   # point sources: every spin and colour at the origin
        srcs = [inputs.point_source(w.lattice, 0, s, c) for s in range(4) for c in range(3)][:w.nrhs]
    else:
        srcs = [inputs.gaussian_source(w.lattice, w.source_seed)]
    if tune and domain is None and product == "auto":
        # the (domain shape, product form) this workload solves fastest with (untimed set-up)
        b = torch.from_numpy(np.ascontiguousarray(srcs[0] if len(srcs) == 1 else np.stack(srcs))).cuda()
        dom, product, ms = ddqcd.tune_sap(w.lattice, w.kappa, w.csw, torch.from_numpy(U).cuda(), b, w.prec,
                                          w.n_cycles, w.n_mr, w.restart, w.tol, 64, w.bc)
        log(f"[bench] tuned: domain {dom}, products {product}" + (f" ({ms:.1f} ms)" if ms >= 0 else " (only fit)"))
        w = dataclasses.replace(w, domain=dom)
        del b
    elif product == "auto":
        product = "lane"
    return [System(w, U, srcs, schedule, schwarz, product)]


def solve_all(systems, ddqcd):
    """One step: every system of the workload to tolerance.  Returns the
    solutions and one info record per right-hand side."""
    if len(systems) == 1:
        x, infos, st = systems[0].ctx.solve(systems[0].b)
        xs = [x]
    else:
        xs, infos, st = ddqcd.solve_batch([s.ctx for s in systems], [s.b for s in systems])
    if st != 0:
        raise RuntimeError(f"solve did not converge: {infos}")
    return xs, infos


def sap_work(systems, iters, additive=False):
    """Algorithmic work of the block solves of one step: (flops, Dslash flops,
    launches, bytes).  iters holds the outer steps of every right-hand side in
    the order of the systems and their sources; each step is one
    preconditioner call of n_cycles cycles visiting every domain once per
    cycle.  Launches: two per cycle (one per colour; one for additive Schwarz)
    per call, systems of one domain shape and precision sharing a launch, so
    the group's longest system counts.  Bytes (geometry's byte model: links and
    clover once per domain visit, spinor data per right-hand side): a system's
    right-hand sides share its launches, so its longest right-hand side counts."""
    from paper_1412_2629_amd import geometry
    per_rhs = [s for s in systems for _ in s.srcs]
    assert len(per_rhs) == len(iters)
    flops = dslash = 0.0
    groups, sys_iters = {}, {}
    for s, it in zip(per_rhs, iters):
        w = s.w
        nd = w.volume // geometry.volume(w.domain)
        pd = geometry.sap_flops_per_domain(w.domain, w.n_mr)
        flops += it * pd["total"] * nd * w.n_cycles
        dslash += it * pd["dslash"] * nd * w.n_cycles
        key = (tuple(w.domain), w.prec)
        groups[key] = max(groups.get(key, 0), it)
        sys_iters[id(s)] = max(sys_iters.get(id(s), 0), it)
    per_call = systems[0].w.n_cycles * (1 if additive else 2)
    launches = sum(per_call * it for it in groups.values())
    sap_bytes = 0.0
    for s in systems:
        w = s.w
        nd = w.volume // geometry.volume(w.domain)
        per = geometry.sap_bytes_per_domain(w.domain, w.prec if w.prec != "f64" else "f32", len(s.srcs))
        sap_bytes += sys_iters[id(s)] * w.n_cycles * nd * per
    return flops, dslash, launches, sap_bytes


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C4", choices=["C1", "C2", "C3", "C4", "C5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", default="sweeps", choices=["sweeps", "graph"],
                    help="block-solve launches issued one by one, or replayed from a captured HIP graph")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-preconditioner comparison solve")
    ap.add_argument("--schwarz", default="multiplicative", choices=["multiplicative", "additive"],
                    help="Schwarz method of the preconditioner (the workloads are defined with multiplicative)")
    ap.add_argument("--domain", default=None,
                    help="override the workload's domain shape, e.g. 4,4,4,4 (single-lattice workloads)")
    ap.add_argument("--product", default="auto", choices=["auto", "lane", "tile", "mfma_f32", "mfma_bf16"],
                    help="block-solve product form: one right-hand side per workgroup, or tiles of four with the "
                         "link products on VALU, FP32 MFMA or BF16-input MFMA (4^4 domains, FP16 storage); auto: "
                         "tuned with the domain shape by ddqcd_tune_sap")
    ap.add_argument("--outer", default="fgcr",
                    help="outer solver: fgcr, or fgmres_dr:M:K (flexible GMRES with deflated restarts, basis M, "
                         "K deflation vectors)")
    ap.add_argument("--lattice", type=int, default=None, help="uneven batch: solve only this lattice")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the listed domain shapes (and one right-hand side per workgroup) instead of autotuning "
                         "them per lattice")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this many MiB (a known-size kernel for "
                         "calibrating profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the lattice is solved whole on a single "
              "MI355X; the library does not shard a lattice across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1412_2629_amd import ddqcd, geometry

    t_tune = time.perf_counter()
    systems = build(args.workload, args.schedule, tune=not args.no_tune, schwarz=args.schwarz,
                    domain=tuple(int(v) for v in args.domain.split(",")) if args.domain else None,
                    product=args.product, lattice=args.lattice)
    if args.outer != "fgcr":
        kind, m, k = args.outer.split(":")
        for s in systems:
            s.ctx.set_solver(int(m), s.w.tol, 64)
            s.ctx.set_outer(kind, int(k))
    t_tune = time.perf_counter() - t_tune
    dev = torch.device("cuda:0")
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
        solve_all(systems, ddqcd)
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runs.append(solve_all(systems, ddqcd))
    torch.cuda.synchronize()
    t_solve = (time.perf_counter() - t0) / args.steps
    xs, infos = runs[-1]
    iters = [i["iters"] for i in infos]
    log(f"[bench] {args.steps} steps, {t_solve * 1e3:.2f} ms each, FGCR steps {iters}")

    # true residual of the last solutions, FP64 operator on the GPU
    true_res = 0.0
    for s, x in zip(systems, xs):
        r = s.b - s.ctx.apply_D(x, "f64")
        rr = torch.linalg.vector_norm(r.reshape(len(s.srcs), -1), dim=1)
        bb = torch.linalg.vector_norm(s.b.reshape(len(s.srcs), -1), dim=1)
        true_res = max(true_res, float((rr / bb).max()))

    flops, dslash, launches, sap_bytes = sap_work(systems, iters, args.schwarz == "additive")
    sap_ms = sum(i["t_sap_ms"] for _, inf in runs for i in inf[:1]) / len(runs)
    launch_ms = sap_ms / launches
    achieved_tflops = flops / (sap_ms * 1e-3) / 1e12
    dslash_gflops = dslash / (sap_ms * 1e-3) / 1e9

    traffic = None
    m = MEASURED_TRAFFIC.get((args.workload, tuple(systems[0].w.domain), systems[0].product))
    if m and m["sources"] == kernel_sources_hash() and args.schwarz == "multiplicative":
        traffic = m["bytes_per_launch"]

    w0 = systems[0].w
    fp64 = None
    if not args.no_fp64 and w0.prec != "f64":
        fp64 = fp64_comparison(systems, xs, iters, t_solve, ddqcd)
    nodd = None
    if not args.no_fp64:
        nodd = non_dd_comparison(systems, t_solve)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(systems, iters)

    if args.workload == "C5":
        doms = sorted({(s.w.lattice, s.w.domain) for s in systems})
        wl = (f"uneven batch of {len(systems)} lattices (8 x 8^4, 8 x 12^3x24, 6 x 16^3x32, 2 x 24^3x48), "
              f"domains {'autotuned' if not args.no_tune else 'as listed'} "
              f"{[(l, d, sum(1 for s in systems if (s.w.lattice, s.w.domain) == (l, d))) for l, d in doms]}, "
              f"kappa in [0.12, 0.136], c_sw 1.5, eps in [0.3, 0.6], FP16-storage SAP {w0.n_cycles}x{w0.n_mr}, "
              f"FGCR restart {w0.restart} (f64), tol {w0.tol}, one ddqcd_solve_batch call, schedule {args.schedule}, "
              f"{args.schwarz} Schwarz, outer {args.outer}"
              + (f", lattice {args.lattice} only" if args.lattice is not None else ""))
        batch = len(systems)
    else:
        wl = (f"{w0.name}: lattice {w0.lattice}, kappa {w0.kappa}, c_sw {w0.csw}, eps {w0.eps}, "
              f"domains {w0.domain}, SAP {w0.n_cycles} cycles x {w0.n_mr} MR ({w0.prec}), "
              f"FGCR restart {w0.restart} (f64), tol {w0.tol}, {len(systems[0].srcs)} right-hand side(s), "
              f"schedule {args.schedule}, {args.schwarz} Schwarz, outer {args.outer}, "
              f"block-solve products {systems[0].product}"
              + (" (domain shape and products autotuned)" if not args.no_tune and not args.domain
                 and args.product == "auto" else ""))
        batch = len(systems[0].srcs)
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
        "dtype": {"f64": "f64", "f32": "f32+f64", "f16": "f16-storage/f32+f64"}[w0.prec],
        "data": "synthetic",
        "config": {"workload": wl, "global_batch": batch, "parallelism": "single GPU"},
        "fgcr_steps": iters if len(iters) > 1 else iters[0],
        "true_rel_residual": true_res,
        "time_split_ms": {k: round(sum(inf[0][k] for _, inf in runs) / len(runs), 3)
                          for k in ("t_sap_ms", "t_A_ms", "t_gs_ms", "t_other_ms")},
        "fgcr_gram_schmidt": gram_schmidt_rate(systems, iters, runs),
        "global_operator": operator_rate(systems, iters, runs),
        "sap_dslash_gflops": round(dslash_gflops, 1),
        "sap_total_tflops": round(achieved_tflops, 3),
        "sap_launches_per_step": int(launches),
        "sap_launch_ms": round(launch_ms, 5),
        "setup_s": round(t_tune, 3),
        "roofline": roofline(systems, achieved_tflops, sap_bytes, sap_ms, launches, traffic),
        "mixed_vs_fp64": fp64,
        "dd_vs_non_dd": nodd,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def gram_schmidt_rate(systems, iters, runs):
    """Algorithmic HBM rate of FGCR's orthogonalisation (FP64 vectors, 192 B
    per site): at step k > 0 of a cycle the multi-dot reads the k earlier
    columns and w, the update reads them, w and r and writes w, the residual
    update reads w and r and writes r (2k + 7 vectors); at step 0 only <w, w>,
    <w, r> (two reads) and the residual update (5 vectors).  Divided by the
    Gram-Schmidt time the library measures on the stream (single passes: a
    repeated pass adds bytes this does not count)."""
    byts = 0.0
    rhs = [s for s in systems for _ in s.srcs]
    for s, n in zip(rhs, iters):
        m = s.w.restart
        vec = s.w.volume * 192
        for step in range(n):
            k = step % m
            byts += (2 * k + 7 if k > 0 else 5) * vec
    t_gs = sum(inf[0]["t_gs_ms"] for _, inf in runs) / len(runs)
    return {"algorithmic_GB": round(byts / 1e9, 3), "t_ms": round(t_gs, 3),
            "GB_per_s": round(byts / (t_gs * 1e-3) / 1e9, 1) if t_gs > 0 else None}


def operator_rate(systems, iters, runs):
    """Algorithmic HBM rate of the outer solver's FP64 operator applications:
    one per FGCR step (w = A z) and one true residual per restart cycle (from a
    zero start the first residual is b itself), 1536 bytes per site each
    (spinor in and out, links and clover); divided by the operator time the
    library measures on the stream."""
    byts = 0.0
    calls = 0
    rhs = [s for s in systems for _ in s.srcs]
    for s, n in zip(rhs, iters):
        m = s.w.restart
        c = n + (n + m - 1) // m
        calls += c
        byts += c * s.w.volume * 1536
    t_a = sum(inf[0]["t_A_ms"] for _, inf in runs) / len(runs)
    return {"applications": calls, "algorithmic_GB": round(byts / 1e9, 3), "t_ms": round(t_a, 3),
            "GB_per_s": round(byts / (t_a * 1e-3) / 1e9, 1) if t_a > 0 else None}


def roofline(systems, achieved_tflops, sap_bytes, sap_ms, launches, traffic):
    """The block-solve kernel against both roofs: its algorithmic flops against
    FP32 vector peak, its algorithmic bytes (geometry's byte model, summed over
    the launches the step made) against HBM peak, both over the block solves'
    time.  The bound is the roof the kernel is closer to.  Where the whole
    working set fits in the 256 MB last-level cache (small lattices), the byte
    rate can exceed HBM peak: then those bytes are not all HBM bytes."""
    w0 = systems[0].w
    launch_ms = sap_ms / launches
    bytes_launch = sap_bytes / launches
    gbs = sap_bytes / (sap_ms * 1e-3) / 1e9
    alu_frac = achieved_tflops / FP32_PEAK_TFLOPS
    hbm_frac = gbs / HBM_PEAK_GBS
    kernel = "k_sap_lds" if w0.prec != "f64" else "k_sap_f64"
    if systems[0].product != "lane":
        kernel = "k_sap_tile"
    common = {"kernel": kernel, "traffic": traffic,
              "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE+WRITE_SIZE)",
              "algorithmic_bytes_per_launch": round(bytes_launch), "launch_ms": round(launch_ms, 5),
              "alu_frac": round(alu_frac, 4), "hbm_frac": round(hbm_frac, 4)}
    if alu_frac >= hbm_frac:
        return {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(alu_frac, 4), **common}
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hbm_frac, 4), **common}


def fp64_comparison(systems, xs, iters, t_solve, ddqcd):
    """The same workload with the FP64 preconditioner on the same domains (the
    plain FP64 SAP + FGCR path): time, steps and the distance between the two
    solutions.  Lattices whose domain shape has no FP64 block-solve kernel keep
    their low-precision preconditioner and are listed."""
    import torch
    log("[bench] FP64-preconditioner comparison solve")
    kept = []
    for s in systems:
        w = s.w
        try:
            s.ctx.set_sap(w.n_cycles, w.n_mr, "f64")
        except ddqcd.DDQCDError:
            kept.append(f"{w.lattice} {w.domain}")
    solve_all(systems, ddqcd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x64, i64 = solve_all(systems, ddqcd)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t1
    for s in systems:
        s.ctx.set_sap(s.w.n_cycles, s.w.n_mr, s.w.prec, s.product)
    diff = max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) for a, b in zip(xs, x64))
    steps64 = [i["iters"] for i in i64]
    return {"fp64_sap_solve_s": round(t64, 5), "fp64_sap_fgcr_steps": steps64 if len(steps64) > 1 else steps64[0],
            "mixed_solve_s": round(t_solve, 6), "mixed_fgcr_steps": iters if len(iters) > 1 else iters[0],
            "speedup_mixed_over_fp64": round(t64 / t_solve, 3),
            "rel_diff_mixed_vs_fp64_solution": diff, "lattices_without_fp64_kernel": kept}


def non_dd_comparison(systems, t_solve):
    """FP64 BiCGstab without preconditioner (the paper's non-DD solver) on the
    same GPU, one right-hand side after the other, after one untimed warm-up
    solve of the first."""
    import torch
    log("[bench] non-DD comparison solves (FP64 BiCGstab)")
    s0 = systems[0]
    s0.ctx.solve_bicgstab(s0.b if len(s0.srcs) == 1 else s0.b[0].contiguous())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    its, ok = [], True
    for s in systems:
        for k in range(len(s.srcs)):
            b = s.b if len(s.srcs) == 1 else s.b[k].contiguous()
            _, ib, st = s.ctx.solve_bicgstab(b, check=False)
            its.append(ib["iters"])
            ok = ok and st == 0 and bool(ib["converged"])
    torch.cuda.synchronize()
    tb = time.perf_counter() - t1
    return {"bicgstab_fp64_solve_s": round(tb, 5), "bicgstab_iters": its if len(its) > 1 else its[0],
            "converged": ok, "speedup_dd_over_non_dd": round(tb / t_solve, 3)}


def cpu_baseline(systems, gpu_iters):
    """The FP64 oracle on the host, same algorithm and parameters.  One FGCR
    step of each distinct lattice shape is timed; if the whole workload's
    oracle solve is then estimated to fit the CPU budget it is run to the
    tolerance and timed, otherwise the per-step times are scaled by the GPU
    run's step counts."""
    import oracle as O
    log("[bench] cpu baseline (oracle)")
    per_step = {}
    samples = []
    for s in systems:
        w = s.w
        key = (w.lattice, w.domain)
        if key in per_step:
            continue
        C = O.clover_field(w.lattice, s.U, w.kappa, w.csw)
        Ci = O.clover_inverse(C)
        t0 = time.perf_counter()
        O.fgcr(w.lattice, w.domain, w.bc, s.U, C, Ci, s.srcs[0], n_cycles=w.n_cycles, n_mr=w.n_mr, restart=1,
               tol=1e-300, max_cycles=1)
        per_step[key] = time.perf_counter() - t0
        samples.append(f"{w.lattice}: {per_step[key]:.2f} s")
    rhs = [s for s in systems for _ in s.srcs]
    est = sum(per_step[(s.w.lattice, s.w.domain)] * it for s, it in zip(rhs, gpu_iters))
    if len(rhs) == 1 and est * 1.5 <= CPU_BUDGET_S:
        s = systems[0]
        w = s.w
        C = O.clover_field(w.lattice, s.U, w.kappa, w.csw)
        Ci = O.clover_inverse(C)
        t0 = time.perf_counter()
        _, st, steps, rr = O.fgcr(w.lattice, w.domain, w.bc, s.U, C, Ci, s.srcs[0], n_cycles=w.n_cycles,
                                  n_mr=w.n_mr, restart=w.restart, tol=w.tol)
        dt = time.perf_counter() - t0
        return {"value": round(dt, 3), "unit": "s", "cores": O.num_threads(), "kind": "oracle",
                "sample": f"the whole solve to {w.tol} ({steps} FGCR steps, status {st}, FP64 SAP "
                          f"{w.n_cycles}x{w.n_mr}) on the host"}
    return {"value": round(est, 3), "unit": "s", "cores": O.num_threads(), "kind": "oracle",
            "sample": "one FGCR step (FP64 SAP call, A, Gram-Schmidt, restart) per lattice shape ("
                      + "; ".join(samples) + "), scaled by the GPU run's FGCR step count of every right-hand side"}


if __name__ == "__main__":
    main()
