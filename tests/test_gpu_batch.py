"""Batched systems on the GPU: many right-hand sides of one lattice, and many
lattices of different sizes, domain shapes and block-solve precisions solved
together (ddqcd_sap with nrhs > 1, ddqcd_solve_batch).

Each system in a batch runs exactly the arithmetic it runs alone (one
workgroup per (system, domain), per-system reductions), so batched results
are compared bit for bit with single-system calls, and against the oracle to
the solve bar: true residual <= 1e-10 with the oracle's A, solution within
1e-8 of the oracle's solve to 1e-12.
"""
import numpy as np
import pytest

from tests.gpu_cases import BC, SMALL, dev, host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("ci,prec", [(0, "f64"), (0, "f16"), (2, "f32"), (2, "f16"), (3, "f32")],
                         ids=lambda v: str(v))
def test_sap_nrhs_equals_single(ci, prec):
    case = SMALL[ci]
    ctx = case.context(prec)
    etas = np.stack([case.source(40 + k) for k in range(3)])
    got = host(ctx.sap(dev(etas)))
    for k in range(3):
        alone = host(ctx.sap(dev(etas[k])))
        assert np.array_equal(got[k], alone), (case, prec, k)


@pytest.mark.parametrize("ci,prec", [(0, "f32"), (2, "f16"), (2, "f64"), (3, "f32")], ids=lambda v: str(v))
def test_solve_nrhs_equals_single(ci, prec):
    """Three right-hand sides solved together give each one's single solve bit
    for bit: with domains of at most 256 sites the outer solver applies A to
    two right-hand sides per launch (the first two here) and to the third
    alone, so this checks the paired operator against the single one."""
    case = SMALL[ci]
    ctx = case.context(prec)
    bs = np.stack([case.source(60 + k) for k in range(3)])
    xs, infos, st = ctx.solve(dev(bs))
    assert st == 0
    got = host(xs)
    for k in range(3):
        x1, info1, st1 = ctx.solve(dev(bs[k]))
        assert st1 == 0 and info1[0]["iters"] == infos[k]["iters"], (case, prec, k)
        assert np.array_equal(got[k], host(x1)), (case, prec, k)


def _batch_systems():
    """(case, prec, n_mr, source seed): four block-solve groups (2^4 FP64, 2^4
    FP32, 4^4 FP16, 8x4^3 FP32), two right-hand sides on one lattice."""
    return [(SMALL[2], "f16", 5, 50), (SMALL[0], "f32", 4, 51), (SMALL[2], "f16", 5, 52),
            (SMALL[3], "f32", 5, 53), (SMALL[1], "f64", 3, 54)]


def test_solve_batch_mixed_lattices(oracle):
    from paper_1412_2629_amd import ddqcd
    n_cycles = 4
    ctxs, cache = [], {}
    for case, prec, n_mr, _ in _batch_systems():
        key = (case.name, prec)
        if key not in cache:
            c = case.context()
            c.set_sap(n_cycles, n_mr, prec)
            c.set_solver(16, 1e-10, 64)
            cache[key] = c
        ctxs.append(cache[key])
    srcs = [case.source(seed) for case, _, _, seed in _batch_systems()]
    xs, infos, st = ddqcd.solve_batch(ctxs, [dev(f) for f in srcs])
    assert st == ddqcd.OK
    for (case, prec, n_mr, seed), c, f, x, inf in zip(_batch_systems(), ctxs, srcs, xs, infos):
        x = host(x)
        # the same system alone: the same iterate, bit for bit
        x1, info1, st1 = c.solve(dev(f))
        assert st1 == ddqcd.OK
        assert info1[0]["iters"] == inf["iters"]
        assert np.array_equal(host(x1), x), (case, prec)
        # against the oracle
        x_or, st_or, _, _ = oracle.fgcr(case.L, case.b, BC, case.U, case.C, case.Ci, f, n_cycles=n_cycles,
                                        n_mr=n_mr, restart=16, tol=1e-12)
        assert st_or == 0
        true_res = rel(oracle.apply_A(case.L, BC, case.U, case.C, x), f)
        err = rel(x, x_or)
        print(f"{case} {prec}: steps {inf['iters']}, true residual {true_res:.2e}, solution error {err:.2e}")
        assert inf["converged"] == 1 and true_res <= 1e-10 and err <= 1e-8


def test_solve_batch_uneven_convergence(oracle):
    """Systems that converge at once (zero source, exact guess) stop while the
    others go on; a not-converged system is reported as such."""
    from paper_1412_2629_amd import ddqcd
    case = SMALL[2]
    ctx = case.context("f32")
    ctx.set_solver(16, 1e-10, 64)
    f = case.source(60)
    x_ref, info_ref, _ = ctx.solve(dev(f))
    zero = np.zeros_like(f)
    xs, infos, st = ddqcd.solve_batch([ctx, ctx, ctx], [dev(f), dev(zero), dev(f)],
                                      x0s=[dev(zero), dev(zero), x_ref])
    assert st == ddqcd.OK
    assert infos[0]["iters"] == info_ref[0]["iters"]
    assert np.array_equal(host(xs[0]), host(x_ref))
    assert infos[1]["iters"] == 0 and not np.any(host(xs[1]))
    assert infos[2]["iters"] == 0 and np.array_equal(host(xs[2]), host(x_ref))
    # a cycle limit too small for one system: that one is reported not converged
    hard = case.context("f32")
    hard.set_solver(2, 1e-10, 1)
    easy = SMALL[0].context("f32")
    easy.set_sap(case.n_cycles, 4, "f32")
    easy.set_solver(2, 1e-10, 1)
    xs, infos, st = ddqcd.solve_batch([hard, easy], [dev(f), dev(np.zeros(SMALL[0].V * 12).reshape(-1, 4, 3))])
    assert st == ddqcd.ERR_NOT_CONVERGED
    assert infos[0]["converged"] == 0 and infos[1]["converged"] == 1


def test_solve_batch_rejects_mixed_settings():
    from paper_1412_2629_amd import ddqcd
    a = SMALL[2].context("f32")
    b = SMALL[3].context("f32")
    b.set_solver(8, 1e-10, 64)
    f_a, f_b = SMALL[2].source(70), SMALL[3].source(71)
    with pytest.raises(ddqcd.DDQCDError) as e:
        ddqcd.solve_batch([a, b], [dev(f_a), dev(f_b)])
    assert e.value.status == ddqcd.ERR_ARG


@pytest.mark.parametrize("ci,prec", [(0, "f64"), (2, "f16"), (2, "f64"), (3, "f32")], ids=lambda v: str(v))
def test_graph_schedule_replays_match_eager(ci, prec):
    """The captured launch graph gives the eager launches' result bit for bit,
    on every replay, with other (eager) GPU work between the replays."""
    case = SMALL[ci]
    ctx = case.context(prec)
    etas = [case.source(80 + k) for k in range(3)]
    eager = [host(ctx.sap(dev(e))) for e in etas]
    ctx.set_schedule("graph")
    for rep in range(3):
        for k, e in enumerate(etas):
            got = host(ctx.sap(dev(e)))
            assert np.array_equal(got, eager[k]), (rep, k)
            ctx.apply_D(dev(e), "f64")   # eager work between replays
    f = case.source(90)
    x_g, info_g, st_g = ctx.solve(dev(f))
    ctx.set_schedule("sweeps")
    x_s, info_s, st_s = ctx.solve(dev(f))
    assert st_g == st_s == 0 and info_g[0]["iters"] == info_s[0]["iters"]
    assert np.array_equal(host(x_g), host(x_s))


def test_graph_schedule_batch():
    from paper_1412_2629_amd import ddqcd
    a = SMALL[2].context()
    a.set_sap(4, 5, "f16")
    b = SMALL[3].context()
    b.set_sap(4, 5, "f32")
    fs = [dev(SMALL[2].source(91)), dev(SMALL[3].source(92)), dev(SMALL[2].source(93))]
    xs_s, inf_s, st_s = ddqcd.solve_batch([a, b, a], fs)
    a.set_schedule("graph")
    for _ in range(2):
        xs_g, inf_g, st_g = ddqcd.solve_batch([a, b, a], fs)
        assert st_g == st_s == 0
        for xg, xs in zip(xs_g, xs_s):
            assert np.array_equal(host(xg), host(xs))


def test_tune_domain_picks_a_converging_shape():
    from paper_1412_2629_amd import ddqcd
    case = SMALL[2]   # 8^4: 2^4 and 4^4 domains fit
    f = dev(case.source(95))
    dom, ms = ddqcd.tune_domain(case.L, case.kappa, case.csw, dev(case.U), f, prec="f16", n_cycles=4, n_mr=5)
    print(f"tuned domain {dom} ({ms:.2f} ms)")
    assert dom in ((2, 2, 2, 2), (4, 4, 4, 4)) and ms > 0
    ctx = ddqcd.Context(case.L, dom, case.kappa, case.csw, BC)
    ctx.load_gauge(dev(case.U))
    ctx.set_sap(4, 5, "f16")
    x, info, st = ctx.solve(f)
    assert st == ddqcd.OK


def test_tune_domain_respects_precision():
    """12x12x4x8 is tiled by 2^4 and by 6x6x2x4; 6x6x2x4 has no FP64 kernel,
    so an FP64 tuning returns 2^4 untimed while FP16 times both."""
    from paper_1412_2629_amd import ddqcd
    case = SMALL[5]
    f = dev(case.source(96))
    dom, ms = ddqcd.tune_domain(case.L, case.kappa, case.csw, dev(case.U), f, prec="f64", n_cycles=4, n_mr=5)
    assert dom == (2, 2, 2, 2) and ms == -1
    dom, ms = ddqcd.tune_domain(case.L, case.kappa, case.csw, dev(case.U), f, prec="f16", n_cycles=4, n_mr=5)
    assert dom in ((2, 2, 2, 2), (6, 6, 2, 4)) and ms > 0


def test_tune_cache(tmp_path, monkeypatch):
    """With DDQCD_TUNE_CACHE set, the first tuning times the candidates and
    appends its result; the same problem again is answered from the file (same
    pair and time, nothing appended); another gauge field is another key."""
    from paper_1412_2629_amd import ddqcd, inputs
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("DDQCD_TUNE_CACHE", str(path))
    case = SMALL[2]   # 8^4: 2^4 and 4^4 domains fit
    f = dev(case.source(97))
    U = dev(case.U)
    dom1, ms1 = ddqcd.tune_domain(case.L, case.kappa, case.csw, U, f, prec="f16", n_cycles=4, n_mr=5)
    assert ms1 > 0 and len(path.read_text().splitlines()) == 1
    dom2, ms2 = ddqcd.tune_domain(case.L, case.kappa, case.csw, U, f, prec="f16", n_cycles=4, n_mr=5)
    assert dom2 == dom1 and abs(ms2 - ms1) < 1e-5
    assert len(path.read_text().splitlines()) == 1
    U3 = dev(inputs.random_gauge(case.L, case.eps, 977))
    dom3, ms3 = ddqcd.tune_domain(case.L, case.kappa, case.csw, U3, f, prec="f16", n_cycles=4, n_mr=5)
    assert ms3 > 0 and dom3 in ((2, 2, 2, 2), (4, 4, 4, 4))
    assert len(path.read_text().splitlines()) == 2


def test_graph_batch_with_fp64_systems(oracle):
    from paper_1412_2629_amd import ddqcd
    a = SMALL[0].context()
    a.set_sap(4, 4, "f64")
    b = SMALL[2].context()
    b.set_sap(4, 5, "f64")
    fs = [dev(SMALL[0].source(97)), dev(SMALL[2].source(98))]
    xs, infos, st = ddqcd.solve_batch([a, b], fs)
    a.set_schedule("graph")
    xg, infog, stg = ddqcd.solve_batch([a, b], fs)
    assert st == stg == ddqcd.OK
    for c, x, y, f in zip((SMALL[0], SMALL[2]), xs, xg, fs):
        assert np.array_equal(host(x), host(y))
        assert rel(oracle.apply_A(c.L, BC, c.U, c.C, host(x)), host(f)) <= 1e-10
