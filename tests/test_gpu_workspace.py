"""A context whose device memory is one caller-owned (torch) allocation
(ddqcd_workspace_size / ddqcd_set_workspace): the same results bit for bit as
a context that allocates its own, no device allocation by the library, and
DDQCD_ERR_NOMEM where the workspace is too small."""
import numpy as np
import pytest

from tests.gpu_cases import BC, WIDE, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def outside_torch_bytes():
    """Device memory in use that torch's allocator does not account for."""
    import torch
    torch.cuda.synchronize()
    free, total = torch.cuda.mem_get_info()
    return (total - free) - torch.cuda.memory_reserved()


def test_workspace_matches_own_allocation():
    import torch

    from paper_1412_2629_amd import ddqcd
    case = WIDE[1]                       # 16^4 lattice, 4^4 domains
    fs = dev(np.stack([case.source(90 + k) for k in range(3)]))
    ref = case.context()
    ref.set_sap(case.n_cycles, case.n_mr, "f16", "tile")
    x_ref, _, st = ref.solve(fs)
    m_ref = host(ref.sap(fs))
    a_ref = host(ref.apply_D(fs[0].contiguous(), "f32"))
    assert st == 0
    U = dev(case.U)
    x = torch.zeros_like(fs)
    m = torch.empty_like(fs)
    a = torch.empty_like(fs[0])
    before = outside_torch_bytes()
    ctx = ddqcd.Context(case.L, case.b, case.kappa, case.csw, BC)
    nbytes = ctx.workspace_size(3)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ctx.set_workspace(ws)
    ctx.load_gauge(U)
    ctx.set_sap(case.n_cycles, case.n_mr, "f16", "tile")
    x, _, st = ctx.solve(fs, x0=None)
    ctx.sap(fs, out=m)
    ctx.apply_D(fs[0].contiguous(), "f32", out=a)
    grown = outside_torch_bytes() - before
    print(f"workspace {nbytes / 2**20:.1f} MiB; device memory outside torch grew by {grown / 2**20:.1f} MiB")
    assert st == 0
    assert np.array_equal(host(x), host(x_ref)) and np.array_equal(host(m), m_ref) and np.array_equal(host(a), a_ref)
    assert grown < 32 * 2 ** 20          # the library's own arrays would be about 1 GiB here
    # a fourth right-hand side needs a slot the workspace does not hold
    with pytest.raises(ddqcd.DDQCDError) as e:
        ctx.solve(dev(np.stack([case.source(95 + k) for k in range(4)])))
    assert e.value.status == ddqcd.ERR_NOMEM
    ctx.close()


def test_workspace_too_small():
    import torch

    from paper_1412_2629_amd import ddqcd
    case = WIDE[1]
    ctx = ddqcd.Context(case.L, case.b, case.kappa, case.csw, BC)
    need = ctx.workspace_size(1)
    ws = torch.empty(need - 4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(ddqcd.DDQCDError) as e:
        ctx.set_workspace(ws)
    assert e.value.status == ddqcd.ERR_NOMEM
