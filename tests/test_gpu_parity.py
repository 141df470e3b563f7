"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerances (normwise relative errors):
  operator A:  1e-13 (FP64), 1e-6 (FP32), 5e-3 (FP16 storage)
  SAP output:  1e-12 (FP64); FP32 and FP16-storage bounds are derived from
               the unit roundoff in the tests below
  solve:       true residual |b - A x|/|b| <= 1e-10 with the oracle's A,
               |x - x_oracle| / |x_oracle| <= 1e-8 (oracle solved to 1e-12)
"""
import numpy as np
import pytest

from tests.gpu_cases import (A_TOL, BC, NO_FP64_SAP, PRODUCT_TOL, SAP_TOL, SITE_FACTOR, SMALL, WIDE, Case, dev, fp64_sap, host,
                             rel, site_err)

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_2629_amd import ddqcd
    ddqcd.lib()


@pytest.mark.parametrize("case", SMALL, ids=repr)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_apply_D(case, prec, oracle):
    psi = case.source()
    want = oracle.apply_A(case.L, BC, case.U, case.C, psi)
    ctx = case.context()
    got = host(ctx.apply_D(dev(psi), prec))
    err = rel(got, want)
    print(f"{case} {prec} operator error {err:.3e}")
    assert err <= A_TOL[prec]


def test_apply_D_batched_rhs(oracle):
    case = SMALL[2]
    ctx = case.context()
    psis = np.stack([case.source(7), case.source(8), case.source(9)])
    got = host(ctx.apply_D(dev(psis), "f64"))
    for k in range(3):
        assert rel(got[k], oracle.apply_A(case.L, BC, case.U, case.C, psis[k])) <= 1e-13


def check_sap(got, want, prec, what):
    err, site = site_err(got, want)
    tol = SAP_TOL[prec]
    print(f"{what} SAP {prec}: error {err:.3e}, largest site error {site:.3e} (bounds {tol:.2e}, "
          f"{SITE_FACTOR * tol:.2e})")
    assert err <= tol and site <= SITE_FACTOR * tol


@pytest.mark.parametrize("case", SMALL, ids=repr)
def test_sap_fp64(case, oracle):
    if not fp64_sap(case):
        pytest.skip(NO_FP64_SAP)
    eta = case.source(5)
    want = oracle.sap(case.L, case.b, BC, case.U, case.C, case.Ci, case.n_cycles, case.n_mr, eta)
    ctx = case.context("f64")
    check_sap(host(ctx.sap(dev(eta))), want, "f64", case)


# The persistent work-queue kernel stalled on the device twice (first with
# acquire polling, then with relaxed system-scope polling); its cause is not
# established, so the kernel is not built into the library, the library
# refuses that schedule, and these cases stay off.
QUEUE_SKIP = "work-queue schedule not built (stalled on the device, cause not established)"


@pytest.mark.parametrize("case", SMALL, ids=repr)
@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("sched", ["sweeps", "queue"])
def test_sap_low_precision(case, prec, sched, oracle):
    if sched == "queue":
        pytest.skip(QUEUE_SKIP)
    eta = case.source(5)
    want = oracle.sap(case.L, case.b, BC, case.U, case.C, case.Ci, case.n_cycles, case.n_mr, eta)
    ctx = case.context(prec)
    ctx.set_schedule(sched)
    check_sap(host(ctx.sap(dev(eta))), want, prec, case)


@pytest.mark.parametrize("case", SMALL[1:], ids=repr)
@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_queue_equals_sweeps_bitwise(case, prec):
    """The work-queue schedule runs the same block solves on the same inputs in
    the same arithmetic order as the per-half-sweep launches: identical bits,
    also over repeated calls (epoch counters advance) with changing cycle counts."""
    pytest.skip(QUEUE_SKIP)
    eta = dev(case.source(9))
    ctx = case.context(prec)
    for n_cycles in (case.n_cycles, 1, 3, case.n_cycles):
        ctx.set_sap(n_cycles, case.n_mr, prec)
        ctx.set_schedule("sweeps")
        a = host(ctx.sap(eta))
        ctx.set_schedule("queue")
        b = host(ctx.sap(eta))
        c = host(ctx.sap(eta))
        assert np.array_equal(a, b) and np.array_equal(b, c), n_cycles


@pytest.mark.parametrize("case", SMALL[:3], ids=repr)
def test_sap_homogeneous(case):
    eta = case.source(6)
    ctx = case.context("f64")
    s = 0.3 + 1.7j
    m1 = host(ctx.sap(dev(eta)))
    m2 = host(ctx.sap(dev(s * eta)))
    assert rel(m2, s * m1) < 1e-13


@pytest.mark.parametrize("case", SMALL, ids=repr)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_solve(case, prec, oracle):
    if prec == "f64" and not fp64_sap(case):
        pytest.skip(NO_FP64_SAP)
    f = case.source(3)
    x_or, st, steps, rr = oracle.fgcr(case.L, case.b, BC, case.U, case.C, case.Ci, f, n_cycles=case.n_cycles,
                                      n_mr=case.n_mr, restart=16, tol=1e-12)
    assert st == 0
    ctx = case.context(prec)
    ctx.set_solver(16, 1e-10, 64)
    x, info, status = ctx.solve(dev(f))
    x = host(x)
    true_res = rel(oracle.apply_A(case.L, BC, case.U, case.C, x), f)
    err = rel(x, x_or)
    print(f"{case} {prec}: steps {info[0]['iters']} (oracle fp64 {steps}), true residual {true_res:.2e}, "
          f"solution error {err:.2e}")
    assert status == 0 and info[0]["converged"] == 1
    assert true_res <= 1e-10
    assert abs(info[0]["rel_residual"] - true_res) <= 1e-12
    assert err <= 1e-8


def test_solve_fp64_matches_oracle_iterates(oracle):
    """The FP64 path runs the same algorithm: same number of FGCR steps."""
    case = SMALL[0]
    f = case.source(4)
    _, st, steps, rr = oracle.fgcr(case.L, case.b, BC, case.U, case.C, case.Ci, f, n_cycles=case.n_cycles,
                                   n_mr=case.n_mr, restart=16, tol=1e-10)
    ctx = case.context("f64")
    x, info, status = ctx.solve(dev(f))
    assert status == 0 and info[0]["iters"] == steps


def test_solve_multi_rhs_and_guess(oracle):
    case = SMALL[2]
    ctx = case.context("f32")
    fs = np.stack([case.source(21), case.source(22)])
    x, info, status = ctx.solve(dev(fs))
    assert status == 0 and len(info) == 2
    for k in range(2):
        assert rel(oracle.apply_A(case.L, BC, case.U, case.C, host(x)[k]), fs[k]) <= 1e-10
    # restart from the converged solution: no further steps
    x2, info2, status2 = ctx.solve(dev(fs), x0=x)
    assert status2 == 0 and all(i["iters"] == 0 for i in info2)


def test_queue_schedule_switched_off():
    from paper_1412_2629_amd import ddqcd
    ctx = SMALL[0].context("f32")
    with pytest.raises(ddqcd.DDQCDError) as e:
        ctx.set_schedule("queue")
    assert e.value.status == ddqcd.ERR_ARG
    ctx.set_schedule("sweeps")


def test_solve_edge_cases():
    from paper_1412_2629_amd import ddqcd
    case = SMALL[0]
    ctx = case.context("f64")
    z = np.zeros((case.V, 4, 3), dtype=np.complex128)
    x, info, st = ctx.solve(dev(z))
    assert st == 0 and np.abs(host(x)).max() == 0 and info[0]["iters"] == 0
    ctx.set_solver(1, 1e-10, 1)
    x, info, st = ctx.solve(dev(case.source(1)))
    assert st == ddqcd.ERR_NOT_CONVERGED and info[0]["iters"] == 1 and 0 < info[0]["rel_residual"] < 1
    ctx.set_solver(16, 1e-10, 64)
    bad = case.source(2)
    bad[3, 1, 2] = np.nan
    x, info, st = ctx.solve(dev(bad), check=False)
    assert st == ddqcd.ERR_NONFINITE
    U = case.U.copy()
    U[5, 2, 1, 1] = np.inf
    with pytest.raises(ddqcd.DDQCDError) as e:
        ctx.load_gauge(dev(U))
    assert e.value.status == ddqcd.ERR_NONFINITE


def test_two_contexts_independent(oracle):
    a, b = SMALL[0], SMALL[1]
    ca, cb = a.context("f64"), b.context("f64")
    pa, pb = a.source(31), b.source(32)
    ga = host(ca.apply_D(dev(pa)))
    gb = host(cb.apply_D(dev(pb)))
    assert rel(ga, oracle.apply_A(a.L, BC, a.U, a.C, pa)) <= 1e-13
    assert rel(gb, oracle.apply_A(b.L, BC, b.U, b.C, pb)) <= 1e-13


def test_fp64_sap_rejected_on_padded_domains():
    from paper_1412_2629_amd import ddqcd
    ctx = SMALL[5].context()
    with pytest.raises(ddqcd.DDQCDError) as e:
        ctx.set_sap(4, 5, "f64")
    assert e.value.status == ddqcd.ERR_GEOMETRY


# ---------------------------------------------------------------------------
# additive Schwarz (Eq. 4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", SMALL, ids=repr)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_sap_additive(case, prec, oracle):
    if prec == "f64" and not fp64_sap(case):
        pytest.skip(NO_FP64_SAP)
    eta = case.source(15)
    want = oracle.sap_additive(case.L, case.b, BC, case.U, case.C, case.Ci, case.n_cycles, case.n_mr, eta)
    ctx = case.context(prec)
    ctx.set_schwarz("additive")
    check_sap(host(ctx.sap(dev(eta))), want, prec, f"{case} additive")


@pytest.mark.parametrize("case", [SMALL[0], SMALL[2], SMALL[3], SMALL[5]], ids=repr)
@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_solve_additive(case, prec, oracle):
    f = case.source(16)
    x_or, st, steps, _ = oracle.fgcr(case.L, case.b, BC, case.U, case.C, case.Ci, f, n_cycles=case.n_cycles,
                                     n_mr=case.n_mr, restart=16, tol=1e-12, additive=True)
    assert st == 0
    ctx = case.context(prec)
    ctx.set_schwarz("additive")
    ctx.set_solver(16, 1e-10, 64)
    x, info, status = ctx.solve(dev(f))
    x = host(x)
    true_res = rel(oracle.apply_A(case.L, BC, case.U, case.C, x), f)
    err = rel(x, x_or)
    print(f"{case} additive {prec}: steps {info[0]['iters']} (oracle fp64 {steps}), true residual {true_res:.2e}, "
          f"solution error {err:.2e}")
    assert status == 0 and true_res <= 1e-10 and err <= 1e-8


def test_additive_graph_and_batch():
    """Graph replays of the additive launches equal the eager ones bit for bit;
    batched additive solves equal single ones; mixed Schwarz variants in one
    batch are rejected."""
    from paper_1412_2629_amd import ddqcd
    case = SMALL[2]
    ctx = case.context("f16")
    ctx.set_schwarz("additive")
    eta = dev(case.source(17))
    eager = host(ctx.sap(eta))
    ctx.set_schedule("graph")
    for _ in range(3):
        assert np.array_equal(host(ctx.sap(eta)), eager)
        ctx.apply_D(eta, "f64")
    ctx.set_schedule("sweeps")
    other = SMALL[3].context("f32")
    other.set_sap(case.n_cycles, 5, "f32")
    other.set_schwarz("additive")
    fa, fb = dev(case.source(18)), dev(SMALL[3].source(19))
    xs, infos, st = ddqcd.solve_batch([ctx, other], [fa, fb])
    assert st == ddqcd.OK
    x1, _, _ = ctx.solve(fa)
    assert np.array_equal(host(x1), host(xs[0]))
    other.set_schwarz("multiplicative")
    with pytest.raises(ddqcd.DDQCDError) as e:
        ddqcd.solve_batch([ctx, other], [fa, fb])
    assert e.value.status == ddqcd.ERR_ARG


# ---------------------------------------------------------------------------
# the solver without domain decomposition (FP64 BiCGstab, Sec. IV-C)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", [SMALL[0], SMALL[2], SMALL[3]], ids=repr)
def test_bicgstab(case, oracle):
    f = case.source(20)
    x_or, st, _, _ = oracle.fgcr(case.L, case.b, BC, case.U, case.C, case.Ci, f, n_cycles=case.n_cycles,
                                 n_mr=case.n_mr, restart=16, tol=1e-12)
    assert st == 0
    ctx = case.context()
    ctx.set_solver(16, 1e-10, 64)
    x, info, status = ctx.solve_bicgstab(dev(f))
    x = host(x)
    true_res = rel(oracle.apply_A(case.L, BC, case.U, case.C, x), f)
    err = rel(x, x_or)
    print(f"{case} BiCGstab: {info['iters']} iterations, {info['restarts']} restarts, true residual {true_res:.2e}, "
          f"solution error {err:.2e}")
    assert status == 0 and info["converged"] == 1
    assert true_res <= 1e-10 and abs(info["rel_residual"] - true_res) <= 1e-12 and err <= 1e-8
    # zero source and exact guess
    z, info0, st0 = ctx.solve_bicgstab(dev(np.zeros_like(f)))
    assert st0 == 0 and info0["iters"] == 0 and not np.any(host(z))
    x2, info2, st2 = ctx.solve_bicgstab(dev(f), x0=dev(x))
    assert st2 == 0 and info2["iters"] == 0


# ---------------------------------------------------------------------------
# tiles of four right-hand sides per workgroup, link products on VALU or MFMA
# ---------------------------------------------------------------------------

TILE_PRODUCTS = ["tile", "mfma_f32", "mfma_bf16"]
_tile_refs = {}


def tile_reference(case, oracle, n):
    """n seeded sources of the case and the oracle's SAP of each."""
    if case.name not in _tile_refs:
        etas = np.stack([case.source(60 + k) for k in range(n)])
        want = [oracle.sap(case.L, case.b, BC, case.U, case.C, case.Ci, case.n_cycles, case.n_mr, e) for e in etas]
        _tile_refs[case.name] = (etas, want)
    return _tile_refs[case.name]


TILE_FORMS = [("f16", "tile"), ("f16", "mfma_f32"), ("f16", "mfma_bf16"), ("bf16", "tile"), ("bf16", "mfma_bf16")]


@pytest.mark.parametrize("case", [SMALL[2], WIDE[1]], ids=repr)
@pytest.mark.parametrize("prec,product", TILE_FORMS)
def test_sap_tile(case, prec, product, oracle):
    """Five right-hand sides (a full tile and a tile of one) against the
    oracle's SAP of each; a right-hand side solved alone (a tile of one) gives
    the bits it gets inside a full tile."""
    etas, want = tile_reference(case, oracle, 5)
    ctx = case.context()
    ctx.set_sap(case.n_cycles, case.n_mr, prec, product)
    got = host(ctx.sap(dev(etas)))
    tol = max(PRODUCT_TOL[product], SAP_TOL[prec])
    for k in range(len(etas)):
        err, site = site_err(got[k], want[k])
        print(f"{case} {prec} {product} rhs {k}: error {err:.3e}, largest site error {site:.3e} (bounds {tol:.2e}, "
              f"{SITE_FACTOR * tol:.2e})")
        assert err <= tol and site <= SITE_FACTOR * tol
    alone = host(ctx.sap(dev(etas[1])))
    assert np.array_equal(alone, got[1])


@pytest.mark.parametrize("prec,product", TILE_FORMS)
def test_solve_tile(prec, product, oracle):
    """Five right-hand sides solved together with the tile forms: true residual
    and solution against the oracle's solve of each."""
    case = SMALL[2]
    fs = np.stack([case.source(70 + k) for k in range(5)])
    ctx = case.context()
    ctx.set_sap(case.n_cycles, case.n_mr, prec, product)
    ctx.set_solver(16, 1e-10, 64)
    x, info, status = ctx.solve(dev(fs))
    assert status == 0
    x = host(x)
    for k in range(len(fs)):
        x_or, st, steps, _ = oracle.fgcr(case.L, case.b, BC, case.U, case.C, case.Ci, fs[k], n_cycles=case.n_cycles,
                                         n_mr=case.n_mr, restart=16, tol=1e-12)
        true_res = rel(oracle.apply_A(case.L, BC, case.U, case.C, x[k]), fs[k])
        err = rel(x[k], x_or)
        print(f"{case} {product} rhs {k}: steps {info[k]['iters']} (oracle fp64 {steps}), true residual "
              f"{true_res:.2e}, solution error {err:.2e}")
        assert st == 0 and true_res <= 1e-10 and err <= 1e-8


def test_tile_graph_batch_and_rejects():
    """Graph replays of tile launches give the eager bits; a batch mixing a
    tiled lattice with another gives each system's own result; shapes and
    precisions without a tile kernel are refused."""
    from paper_1412_2629_amd import ddqcd
    case = SMALL[2]
    ctx = case.context()
    ctx.set_sap(case.n_cycles, case.n_mr, "f16", "mfma_f32")
    etas = dev(np.stack([case.source(80 + k) for k in range(3)]))
    eager = host(ctx.sap(etas))
    ctx.set_schedule("graph")
    for _ in range(3):
        assert np.array_equal(host(ctx.sap(etas)), eager)
        ctx.apply_D(etas[0].contiguous(), "f64")
    ctx.set_schedule("sweeps")
    other = SMALL[3].context("f32")
    other.set_sap(case.n_cycles, 5, "f32")
    fa, fb = dev(case.source(81)), dev(SMALL[3].source(82))
    xs, infos, st = ddqcd.solve_batch([ctx, other, ctx], [fa, fb, fa])
    assert st == ddqcd.OK
    x1, _, _ = ctx.solve(fa)
    assert np.array_equal(host(x1), host(xs[0])) and np.array_equal(host(x1), host(xs[2]))
    for bad in ((SMALL[3], "f16"), (SMALL[3], "bf16"), (SMALL[2], "f32"), (SMALL[2], "f64")):
        c = bad[0].context()
        with pytest.raises(ddqcd.DDQCDError) as e:
            c.set_sap(4, 5, bad[1], "mfma_f32")
        assert e.value.status == ddqcd.ERR_GEOMETRY


# ---------------------------------------------------------------------------
# flexible GMRES with deflated restarts (the paper's outer solver)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", [SMALL[0], SMALL[1], SMALL[3]], ids=repr)
@pytest.mark.parametrize("prec", ["f64", "f16"])
@pytest.mark.parametrize("m,k", [(8, 4), (16, 6), (6, 0)])
def test_solve_fgmres_dr(case, prec, m, k, oracle):
    """Solution and true residual against the oracle; the FP64 path takes the
    oracle's FGMRES-DR step count."""
    f = case.source(30)
    x_or, st, steps_or, _ = oracle.fgmres_dr(case.L, case.b, BC, case.U, case.C, case.Ci, f, m, k,
                                             n_cycles=case.n_cycles, n_mr=case.n_mr, tol=1e-10)
    assert st == 0
    ctx = case.context(prec)
    ctx.set_solver(m, 1e-10, 64)
    ctx.set_outer("fgmres_dr", k)
    x, info, status = ctx.solve(dev(f))
    x = host(x)
    true_res = rel(oracle.apply_A(case.L, BC, case.U, case.C, x), f)
    x_ex, st_ex, _, _ = oracle.fgcr(case.L, case.b, BC, case.U, case.C, case.Ci, f, n_cycles=case.n_cycles,
                                    n_mr=case.n_mr, restart=16, tol=1e-12)
    err = rel(x, x_ex)
    print(f"{case} {prec} FGMRES-DR({m},{k}): steps {info[0]['iters']} in {info[0]['restarts']} cycles "
          f"(oracle fp64 {steps_or}), true residual {true_res:.2e}, solution error {err:.2e}")
    assert status == 0 and true_res <= 1e-10 and err <= 1e-8
    assert abs(info[0]["rel_residual"] - true_res) <= 1e-12
    if prec == "f64":
        assert info[0]["iters"] == steps_or


def test_fgmres_dr_multi_rhs_batch_and_settings(oracle):
    """Several right-hand sides and a batch (solved one after the other), a
    converged guess takes no step, bad settings are refused."""
    from paper_1412_2629_amd import ddqcd
    case = SMALL[2]
    ctx = case.context("f32")
    ctx.set_solver(8, 1e-10, 64)
    ctx.set_outer("fgmres_dr", 4)
    fs = np.stack([case.source(31), case.source(32)])
    x, info, st = ctx.solve(dev(fs))
    assert st == 0
    for q in range(2):
        assert rel(oracle.apply_A(case.L, BC, case.U, case.C, host(x)[q]), fs[q]) <= 1e-10
    x2, info2, st2 = ctx.solve(dev(fs), x0=x)
    assert st2 == 0 and all(i["iters"] == 0 for i in info2)
    other = SMALL[3].context("f32")
    other.set_solver(8, 1e-10, 64)
    with pytest.raises(ddqcd.DDQCDError) as e:     # outer solvers differ
        ddqcd.solve_batch([ctx, other], [dev(fs[0]), dev(SMALL[3].source(33))])
    assert e.value.status == ddqcd.ERR_ARG
    other.set_outer("fgmres_dr", 4)
    xs, infos, st3 = ddqcd.solve_batch([ctx, other], [dev(fs[0]), dev(SMALL[3].source(33))])
    assert st3 == 0 and np.array_equal(host(xs[0]), host(x)[0])
    for k in (8, -1):                              # deflation vectors outside [0, basis size)
        with pytest.raises(ddqcd.DDQCDError):
            ctx.set_outer("fgmres_dr", k)


@pytest.mark.parametrize("case", [SMALL[0], SMALL[1], SMALL[3], SMALL[5]], ids=repr)
@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_solve_mixed_outer(case, prec, oracle):
    """The mixed-precision outer solver (FP64 refinement around FP32 FGCR
    cycles): true residual and solution against the oracle."""
    f = case.source(40)
    x_ex, st, _, _ = oracle.fgcr(case.L, case.b, BC, case.U, case.C, case.Ci, f, n_cycles=case.n_cycles,
                                 n_mr=case.n_mr, restart=16, tol=1e-12)
    assert st == 0
    ctx = case.context(prec)
    ctx.set_solver(16, 1e-10, 64)
    ctx.set_outer("fgcr_mixed")
    x, info, status = ctx.solve(dev(f))
    x = host(x)
    true_res = rel(oracle.apply_A(case.L, BC, case.U, case.C, x), f)
    err = rel(x, x_ex)
    print(f"{case} {prec} mixed outer: {info[0]['iters']} steps in {info[0]['restarts']} refinements, true residual "
          f"{true_res:.2e}, solution error {err:.2e}")
    assert status == 0 and true_res <= 1e-10 and err <= 1e-8
    assert abs(info[0]["rel_residual"] - true_res) <= 1e-12


def test_mixed_outer_settings():
    from paper_1412_2629_amd import ddqcd
    ctx = SMALL[2].context("f64")
    with pytest.raises(ddqcd.DDQCDError):          # an FP64 preconditioner has no FP32 input
        ctx.set_outer("fgcr_mixed")
    ctx.set_sap(4, 5, "f32")
    ctx.set_outer("fgcr_mixed")
    with pytest.raises(ddqcd.DDQCDError):
        ctx.set_sap(4, 5, "f64")
    with pytest.raises(ddqcd.DDQCDError):
        ctx.set_outer("fgcr_mixed", 2)
