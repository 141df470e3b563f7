"""Host-side accounting of bench.py (no GPU): the block solves' flops, launches
and bytes over an uneven batch, the roofline's bound and fractions, and the
Gram-Schmidt byte model."""
import types

import pytest

import bench
from paper_1412_2629_amd import geometry


def system(L, b, prec, nsrc, n_cycles=16, n_mr=5, restart=16, product="lane"):
    w = types.SimpleNamespace(lattice=L, volume=L[0] * L[1] * L[2] * L[3], domain=b, prec=prec, n_cycles=n_cycles,
                              n_mr=n_mr, restart=restart)
    return types.SimpleNamespace(w=w, srcs=list(range(nsrc)), product=product)


def test_sap_work_over_an_uneven_batch():
    """Systems leave the batch at different steps: flops follow every right-hand
    side's own step count, a launch group's count is its longest system's, and
    a system's bytes its longest right-hand side's."""
    a = system((8, 8, 8, 8), (4, 4, 4, 4), "f16", 1)
    b = system((16, 16, 16, 32), (8, 4, 4, 4), "f16", 2)
    c = system((8, 8, 8, 8), (4, 4, 4, 4), "f16", 1)
    iters = [3, 5, 4, 10]   # a: 3; b: 5 and 4; c: 10
    flops, dslash, launches, byts = bench.sap_work([a, b, c], iters)
    f44 = geometry.sap_flops_per_domain((4, 4, 4, 4), 5)
    f84 = geometry.sap_flops_per_domain((8, 4, 4, 4), 5)
    nd_a, nd_b = 8 ** 4 // 256, 16 * 16 * 16 * 32 // 512
    assert flops == pytest.approx(16 * nd_a * (3 + 10) * f44["total"] + 16 * nd_b * (5 + 4) * f84["total"])
    assert dslash == pytest.approx(16 * nd_a * (3 + 10) * f44["dslash"] + 16 * nd_b * (5 + 4) * f84["dslash"])
    assert launches == 2 * 16 * (10 + 5)
    per_a = geometry.sap_bytes_per_domain((4, 4, 4, 4), "f16", 1)
    per_b = geometry.sap_bytes_per_domain((8, 4, 4, 4), "f16", 2)
    assert byts == pytest.approx(16 * nd_a * (3 + 10) * per_a + 16 * nd_b * 5 * per_b)
    # additive Schwarz: one launch per cycle
    assert bench.sap_work([a, b, c], iters, additive=True)[2] == 16 * (10 + 5)


def test_sap_work_single_lattice_matches_the_per_launch_model():
    """One lattice, every right-hand side the same steps: bytes per launch are
    half the domains times the per-domain figure for all right-hand sides."""
    s = system((32, 32, 32, 64), (4, 4, 4, 4), "f16", 12, product="tile")
    flops, _, launches, byts = bench.sap_work([s], [3] * 12)
    nd = 32 ** 3 * 64 // 256
    assert launches == 96
    assert byts / launches == pytest.approx(nd / 2 * geometry.sap_bytes_per_domain((4, 4, 4, 4), "f16", 12))
    assert flops / launches == pytest.approx(12 * nd / 2 * geometry.sap_flops_per_domain((4, 4, 4, 4), 5)["total"])


def test_roofline_takes_the_nearer_roof():
    s = system((8, 8, 8, 8), (4, 4, 4, 4), "f16", 4, product="tile")
    # 1 GB in 1 ms: 1000 GB/s, 0.125 of HBM
    r = bench.roofline([s], 20.0, 1e9, 1.0, 10, None)
    assert r["bound"] == "alu" and r["kernel"] == "k_sap_tile"
    assert r["frac"] == pytest.approx(20.0 / bench.FP32_PEAK_TFLOPS, abs=1e-4)
    assert r["hbm_frac"] == pytest.approx(0.125, abs=1e-4)
    assert r["algorithmic_bytes_per_launch"] == 100000000 and r["launch_ms"] == pytest.approx(0.1)
    r = bench.roofline([s], 5.0, 1e9, 1.0, 10, 1.2e8)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1000.0) and r["frac"] == pytest.approx(0.125, abs=1e-4)
    assert r["traffic"] == 1.2e8


def test_gram_schmidt_byte_model():
    """Step 0: <w, w>-free first step, 5 vectors; step k > 0: 2k + 7."""
    s = system((32, 32, 32, 64), (8, 4, 4, 4), "f16", 1)
    vec = 32 ** 3 * 64 * 192
    runs = [(None, [{"t_gs_ms": 2.0}])]
    g = bench.gram_schmidt_rate([s], [3], runs)
    want = (5 + 9 + 11) * vec
    assert g["algorithmic_GB"] == pytest.approx(want / 1e9, abs=1e-3)
    assert g["GB_per_s"] == pytest.approx(want / 2e-3 / 1e9, rel=1e-3)
    # a restart: step 16 of a restart-16 cycle is step 0 of the next
    g = bench.gram_schmidt_rate([s], [17], runs)
    want = (5 + sum(2 * k + 7 for k in range(1, 16)) + 5) * vec
    assert g["algorithmic_GB"] == pytest.approx(want / 1e9, abs=1e-3)


def test_operator_byte_model():
    """One application per outer step and one true residual per restart
    cycle, 1536 bytes per site each."""
    s = system((32, 32, 32, 64), (4, 4, 4, 4), "f16", 2)
    runs = [(None, [{"t_A_ms": 4.0}])]
    g = bench.operator_rate([s], [3, 17], runs)
    calls = (3 + 1) + (17 + 2)
    assert g["applications"] == calls
    assert g["algorithmic_GB"] == pytest.approx(calls * 32 ** 3 * 64 * 1536 / 1e9, abs=1e-3)
    assert g["GB_per_s"] == pytest.approx(calls * 32 ** 3 * 64 * 1536 / 4e-3 / 1e9, rel=1e-3)
