"""Parity at the full workload sizes, in the configuration bench.py times.

Operator: sampled output sites (random sites plus every site of two whole
domains) computed one by one by the oracle.  Preconditioner: the whole SAP
output against the oracle's SAP at 16^3x32 (FP32, FP64), 32^3x64 (FP16
storage) and on lattices with four domains per direction for every domain
shape, normwise and per site.  Solve: the true residual |b - A x|/|b|
evaluated with the oracle's operator at every site; the solution against the
oracle's own solve to 1e-12, whole at 16^3x32 and at 512 seeded sites for
the 32^3x64 solves and three lattices of the uneven batch (the oracle's values
there come from tests/golden/make_fullsize_refs.py, which calls only the
oracle).
"""
import functools
import json
import os

import numpy as np
import pytest

from paper_1412_2629_amd import configs, inputs
from tests.gpu_cases import A_TOL, BC, SAP_TOL, SITE_FACTOR, WIDE, dev, fp64_sap, host, rel, site_err

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_refs")
SOL_TOL = 1e-8   # solution against the oracle's solution (oracle solved to 1e-12)


@functools.lru_cache(maxsize=1)
def refs():
    return dict(np.load(GOLDEN + ".npz")), json.load(open(GOLDEN + ".json"))


def check_against_ref(key, x):
    """x (the GPU solution, canonical layout) against the oracle's solution at
    the stored sites, and its norm against the oracle solution's norm."""
    arrays, meta = refs()
    sites, want = arrays[key + "_sites"], arrays[key + "_x"]
    err = rel(x[sites], want)
    nerr = abs(float(np.linalg.norm(x)) - meta[key]["x_norm"]) / meta[key]["x_norm"]
    print(f"{key}: solution error vs oracle at {len(sites)} sites {err:.3e}, norm {nerr:.1e} "
          f"(oracle {meta[key]['oracle_steps']} steps)", flush=True)
    assert err <= SOL_TOL and nerr <= SOL_TOL

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@functools.lru_cache(maxsize=2)
def fields(name):
    w = configs.WORKLOADS[name]
    print(f"[fullsize] generating {name} inputs", flush=True)
    return w, inputs.random_gauge(w.lattice, w.eps, w.gauge_seed), inputs.gaussian_source(w.lattice, w.source_seed)


@functools.lru_cache(maxsize=1)
def oracle_clover(name):
    import oracle as O
    w, U, _ = fields(name)
    C = O.clover_field(w.lattice, U, w.kappa, w.csw)
    return C, O.clover_inverse(C)


def context(w, U):
    from paper_1412_2629_amd import ddqcd
    ctx = ddqcd.Context(w.lattice, w.domain, w.kappa, w.csw, w.bc)
    ctx.load_gauge(dev(U))
    ctx.set_sap(w.n_cycles, w.n_mr, w.prec)
    ctx.set_solver(w.restart, w.tol, 64)
    return ctx


def sample_sites(w, n=3000, seed=0):
    L, b = w.lattice, w.domain
    rng = np.random.default_rng(seed)
    sites = set(rng.integers(0, w.volume, size=n).tolist())
    # two whole domains: the first one and the last one
    for X in ([0, 0, 0, 0], [L[m] // b[m] - 1 for m in range(4)]):
        for lt in range(b[3]):
            for lz in range(b[2]):
                for ly in range(b[1]):
                    for lx in range(b[0]):
                        x = [X[0] * b[0] + lx, X[1] * b[1] + ly, X[2] * b[2] + lz, X[3] * b[3] + lt]
                        sites.add(x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3])))
    return np.array(sorted(sites), dtype=np.int64)


@pytest.mark.parametrize("name", ["C2", "C3"])
def test_apply_D_sampled(name, oracle):
    w, U, f = fields(name)
    ctx = context(w, U)
    sites = sample_sites(w)
    want = oracle.apply_A_sites(w.lattice, w.bc, U, w.kappa, w.csw, f, sites)
    fd = dev(f)
    for prec in ("f64", "f32", "f16", "bf16"):
        got = host(ctx.apply_D(fd, prec))[sites]
        err = rel(got, want)
        print(f"{name} {prec}: operator error on {len(sites)} sampled sites {err:.3e}")
        assert err <= A_TOL[prec]


# ---------------------------------------------------------------------------
# the preconditioner at the benchmarked sizes
# ---------------------------------------------------------------------------

def check_sap(got, want, prec, what):
    err, site = site_err(got, want)
    tol = SAP_TOL[prec]
    print(f"{what} SAP {prec}: error {err:.3e}, largest site error {site:.3e} (bounds {tol:.2e}, "
          f"{SITE_FACTOR * tol:.2e})", flush=True)
    assert err <= tol and site <= SITE_FACTOR * tol


@pytest.mark.parametrize("case", WIDE, ids=repr)
def test_sap_wide(case, oracle):
    """Every domain shape on a lattice with four domains per direction, every
    precision the shape has a kernel for."""
    eta = case.source(25)
    want = oracle.sap(case.L, case.b, BC, case.U, case.C, case.Ci, case.n_cycles, case.n_mr, eta)
    ctx = case.context()
    for prec in ("f64", "f32", "f16", "bf16"):
        if prec == "f64" and not fp64_sap(case):
            continue
        ctx.set_sap(case.n_cycles, case.n_mr, prec)
        check_sap(host(ctx.sap(dev(eta))), want, prec, case)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,precs", [("C2", ("f32", "f64")), ("C3", ("f16",))])
def test_sap_fullsize(name, precs, oracle):
    """ddqcd_sap on the whole 16^3x32 and 32^3x64 lattices, with the benchmark's
    domains and cycle counts, against the oracle's SAP (the FGCR residual r the
    preconditioner sees is a Gaussian field here)."""
    w, U, f = fields(name)
    C, Ci = oracle_clover(name)
    eta = inputs.gaussian_source(w.lattice, w.source_seed + 50)
    want = oracle.sap(w.lattice, w.domain, w.bc, U, C, Ci, w.n_cycles, w.n_mr, eta)
    ctx = context(w, U)
    for prec in precs:
        ctx.set_sap(w.n_cycles, w.n_mr, prec)
        check_sap(host(ctx.sap(dev(eta))), want, prec, f"{name} ({w.domain} domains, {w.n_cycles}x{w.n_mr})")


@pytest.mark.timeout(600)
def test_sap_fullsize_tile(oracle):
    """The 12-source benchmark's block solves: tiles of right-hand sides on 4^4
    domains of the 32^3x64 lattice (FP16 storage, 16 x 5), two Gaussian
    right-hand sides in one tile against the oracle's SAP of each."""
    import dataclasses
    _, U, _ = fields("C3")   # the 12-source workload shares this gauge field
    w = dataclasses.replace(configs.WORKLOADS["C4"], domain=(4, 4, 4, 4))
    C, Ci = oracle_clover("C3")
    etas = np.stack([inputs.gaussian_source(w.lattice, w.source_seed + 70 + k) for k in range(2)])
    ctx = context(w, U)
    ctx.set_sap(w.n_cycles, w.n_mr, "f16", "tile")
    got = host(ctx.sap(dev(etas)))
    for k in range(2):
        want = oracle.sap(w.lattice, w.domain, w.bc, U, C, Ci, w.n_cycles, w.n_mr, etas[k])
        check_sap(got[k], want, "f16", f"32^3x64 tile, rhs {k} (4^4 domains, {w.n_cycles}x{w.n_mr})")


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,prec", [("C2", None), ("C3", None), ("C2", "f64")])
def test_solve_true_residual(name, prec, oracle):
    w, U, f = fields(name)
    ctx = context(w, U)
    if prec is not None:   # the plain FP64 preconditioner on the same domains
        ctx.set_sap(w.n_cycles, w.n_mr, prec)
    x, info, st = ctx.solve(dev(f))
    assert st == 0, info
    x = host(x)
    Ax = oracle.apply_A_sites(w.lattice, w.bc, U, w.kappa, w.csw, x, np.arange(w.volume, dtype=np.int64))
    true_res = rel(Ax, f)
    print(f"{name} {prec or w.prec}: {info[0]['iters']} FGCR steps, true residual (oracle A) {true_res:.3e}, "
          f"reported {info[0]['rel_residual']:.3e}", flush=True)
    assert true_res <= 1e-10
    assert abs(true_res - info[0]["rel_residual"]) <= 1e-12
    if name == "C3":
        check_against_ref("C3", x)
    if name == "C2":
        C, Ci = oracle_clover(name)
        x_or, st_or, steps, rr = oracle.fgcr(w.lattice, w.domain, w.bc, U, C, Ci, f, n_cycles=w.n_cycles,
                                             n_mr=w.n_mr, restart=w.restart, tol=1e-12)
        assert st_or == 0
        err = rel(x, x_or)
        print(f"C2: solution error vs oracle {err:.3e} (oracle {steps} steps)")
        assert err <= SOL_TOL
        if prec == "f64":
            # the plain FP64 path runs the oracle's algorithm: the same step count to 1e-10
            _, st10, steps10, _ = oracle.fgcr(w.lattice, w.domain, w.bc, U, C, Ci, f, n_cycles=w.n_cycles,
                                              n_mr=w.n_mr, restart=w.restart, tol=w.tol)
            print(f"C2 f64: {info[0]['iters']} GPU FGCR steps, oracle {steps10}")
            assert st10 == 0 and info[0]["iters"] == steps10


@pytest.mark.timeout(600)
def test_c4_twelve_point_sources(oracle):
    """12 point sources (every spin and colour at the origin) on the 32^3x64
    lattice, solved together.  Every solution's true residual is evaluated
    with the oracle's operator at every site; right-hand sides 0, 5 and 11
    against the oracle's solutions; right-hand side 5 alone gives the same
    iterate bit for bit."""
    w = configs.C4
    _, U, _ = fields("C3")
    ctx = context(w, U)
    srcs = np.stack([inputs.point_source(w.lattice, 0, s, c) for s in range(4) for c in range(3)])
    x, infos, st = ctx.solve(dev(srcs))
    assert st == 0, infos
    print(f"C4: FGCR steps {[i['iters'] for i in infos]}, batch {infos[0]['t_total_ms']:.1f} ms", flush=True)
    xh = host(x)
    all_sites = np.arange(w.volume, dtype=np.int64)
    for k in range(12):
        Ax = oracle.apply_A_sites(w.lattice, w.bc, U, w.kappa, w.csw, xh[k], all_sites)
        true_res = rel(Ax, srcs[k])
        print(f"C4 rhs {k}: true residual (oracle A) {true_res:.3e}", flush=True)
        assert true_res <= 1e-10
        if f"C4_rhs{k}" in refs()[1]:
            check_against_ref(f"C4_rhs{k}", xh[k])
    x5, info5, st5 = ctx.solve(dev(srcs[5]))
    assert st5 == 0 and info5[0]["iters"] == infos[5]["iters"]
    assert np.array_equal(host(x5), xh[5])


@pytest.mark.timeout(600)
def test_c5_uneven_batch(oracle):
    """The 24-lattice uneven batch solved in one ddqcd_solve_batch call: every
    solution's true residual with the oracle's operator; one lattice of each
    size against the oracle's solution (the smallest solved here, the others
    at stored sites); two lattices alone give the same iterate bit for bit."""
    from paper_1412_2629_amd import ddqcd
    ws = configs.uneven_batch()
    ctxs, Us, fs = [], [], []
    for j, w in enumerate(ws):
        print(f"[fullsize] generating uneven batch lattice {j} {w.lattice}", flush=True)
        U = inputs.random_gauge(w.lattice, w.eps, w.gauge_seed)
        Us.append(U)
        fs.append(inputs.gaussian_source(w.lattice, w.source_seed))
        ctxs.append(context(w, U))
    xs, infos, st = ddqcd.solve_batch(ctxs, [dev(f) for f in fs])
    assert st == ddqcd.OK, infos
    print(f"C5: batch {infos[0]['t_total_ms']:.1f} ms, steps {[i['iters'] for i in infos]}", flush=True)
    for j, (w, U, f, x) in enumerate(zip(ws, Us, fs, xs)):
        C = oracle.clover_field(w.lattice, U, w.kappa, w.csw)
        true_res = rel(oracle.apply_A(w.lattice, w.bc, U, C, host(x)), f)
        print(f"C5 lattice {j} {w.lattice}: true residual (oracle A) {true_res:.3e}", flush=True)
        assert true_res <= 1e-10
        if f"C5_lat{j}" in refs()[1]:
            check_against_ref(f"C5_lat{j}", host(x))
    w, U, f = ws[0], Us[0], fs[0]
    C = oracle.clover_field(w.lattice, U, w.kappa, w.csw)
    x_or, st_or, _, _ = oracle.fgcr(w.lattice, w.domain, w.bc, U, C, oracle.clover_inverse(C), f,
                                    n_cycles=w.n_cycles, n_mr=w.n_mr, restart=w.restart, tol=1e-12)
    assert st_or == 0 and rel(host(xs[0]), x_or) <= SOL_TOL
    for j in (0, len(ws) - 1):
        x1, info1, st1 = ctxs[j].solve(dev(fs[j]))
        assert st1 == 0 and info1[0]["iters"] == infos[j]["iters"]
        assert np.array_equal(host(x1), host(xs[j]))


def test_c2_bicgstab_true_residual(oracle):
    """The non-DD baseline at 16^3x32: FP64 BiCGstab to 1e-10, checked with
    the oracle's operator at every site, and against the DD solve's solution."""
    w, U, f = fields("C2")
    ctx = context(w, U)
    x, info, st = ctx.solve_bicgstab(dev(f))
    assert st == 0, info
    xh = host(x)
    Ax = oracle.apply_A_sites(w.lattice, w.bc, U, w.kappa, w.csw, xh, np.arange(w.volume, dtype=np.int64))
    true_res = rel(Ax, f)
    xd, _, std = ctx.solve(dev(f))
    print(f"C2 BiCGstab: {info['iters']} iterations, true residual {true_res:.3e}, "
          f"vs DD solution {rel(xh, host(xd)):.2e}")
    assert true_res <= 1e-10 and rel(xh, host(xd)) <= 1e-8
