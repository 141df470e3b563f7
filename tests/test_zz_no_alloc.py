"""ddqcd_sap_noalloc (the preconditioner without allocation, for callers that
cannot allocate) through the C-ABI, against ddqcd_sap: the same kernels in the
same order, so the same bits.  Two contexts on one device share the
library's scratch array; the second call uses a smaller lattice, the third
goes back to the first."""
import numpy as np
import pytest

from tests.gpu_cases import SAP_TOL, Case, dev, host, site_err

pytestmark = pytest.mark.gpu

BIG = Case("16x8x8x8/8x4^3", (16, 8, 8, 8), (8, 4, 4, 4), 0.1355, 1.5, 0.5, 131, 4, 5)
SMALL = Case("4^4/2^4", (4, 4, 4, 4), (2, 2, 2, 2), 0.12, 1.0, 0.3, 101, 8, 4)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check(ctx, case, prec, seed):
    eta = dev(case.source(seed))
    want = host(ctx.sap(eta))
    got = host(ctx.sap_noalloc(eta))
    err, site = site_err(got, want)
    print(f"{case} {prec}: noalloc vs sap error {err:.1e}, largest site {site:.1e}", flush=True)
    assert err <= SAP_TOL[prec] and np.array_equal(got, want)


def test_noalloc_matches_sap():
    big = BIG.context("f32")
    small = SMALL.context("f16")
    check(big, BIG, "f32", 41)
    check(small, SMALL, "f16", 42)     # smaller input, same scratch
    check(big, BIG, "f32", 43)
    for prec in ("f64", "f16"):
        big.set_sap(BIG.n_cycles, BIG.n_mr, prec)
        check(big, BIG, prec, 44)
    small.set_schwarz("additive")
    check(small, SMALL, "f16", 45)


def test_noalloc_rejects_lattice_over_the_limit():
    from paper_1412_2629_amd import ddqcd
    case = Case("16^3x64/8x4^3", (16, 16, 16, 64), (8, 4, 4, 4), 0.1355, 1.5, 0.5, 151, 1, 1)
    ctx = case.context("f32")
    eta = dev(np.zeros((case.V, 4, 3), dtype=np.complex128))
    with pytest.raises(ddqcd.DDQCDError) as e:
        ctx.sap_noalloc(eta)
    assert e.value.status == ddqcd.ERR_NOMEM and "limit" in str(e.value)
