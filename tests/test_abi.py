"""The C-ABI library loads and exports every entry point of include/ddqcd.h;
host-side validation paths (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1412_2629_amd import ddqcd

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ddqcd.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ddqcd_[A-Za-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_solver_calls():
    names = declared()
    for n in ["ddqcd_create", "ddqcd_load_gauge", "ddqcd_apply_D", "ddqcd_sap", "ddqcd_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = ddqcd.lib()
    for n in declared():
        assert hasattr(L, n), n
    assert set(declared()) == set(ddqcd.EXPORTS)


def _create(L=(8, 8, 8, 8), b=(4, 4, 4, 4), kappa=0.12, csw=1.0, bc=(1, 1, 1, -1)):
    h = ctypes.c_void_p()
    st = ddqcd.lib().ddqcd_create((ctypes.c_int * 4)(*L), (ctypes.c_int * 4)(*b), kappa, csw,
                                  (ctypes.c_double * 4)(*bc), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("L,b", [((8, 8, 8, 8), (8, 4, 4, 4)),      # one domain in x
                                 ((12, 8, 8, 8), (4, 4, 4, 4)),     # three domains in x
                                 ((8, 8, 8, 8), (3, 4, 4, 4)),      # odd extent
                                 ((8, 8, 8, 10), (4, 4, 4, 5)),     # odd extent
                                 ((16, 16, 16, 16), (4, 4, 8, 4))])  # no compiled block-solve shape
def test_create_rejects_geometry(L, b):
    st, h = _create(L, b)
    assert st == ddqcd.ERR_GEOMETRY and not h.value


@pytest.mark.parametrize("kw", [dict(kappa=0.0), dict(kappa=-0.1), dict(kappa=float("nan")), dict(csw=float("inf")),
                                dict(bc=(1, 1, 1, 0.5)), dict(bc=(1, 1, 2, -1))])
def test_create_rejects_arguments(kw):
    st, h = _create(**kw)
    assert st == ddqcd.ERR_ARG and not h.value


def test_create_settings_and_state_errors():
    st, h = _create()
    assert st == ddqcd.OK and h.value
    L = ddqcd.lib()
    try:
        lane, mfma = ddqcd.PRODUCT["lane"], ddqcd.PRODUCT["mfma_f32"]
        assert L.ddqcd_set_sap(h, 0, 5, 1, lane) == ddqcd.ERR_ARG
        assert L.ddqcd_set_sap(h, 16, 0, 1, lane) == ddqcd.ERR_ARG
        assert L.ddqcd_set_sap(h, 16, 5, 7, lane) == ddqcd.ERR_ARG
        assert L.ddqcd_set_sap(h, 16, 5, ddqcd.FP16, 9) == ddqcd.ERR_ARG
        # the tile forms need FP16 storage (and 4^4 domains, which this context has)
        assert L.ddqcd_set_sap(h, 16, 5, ddqcd.FP32, mfma) == ddqcd.ERR_GEOMETRY
        assert L.ddqcd_set_sap(h, 16, 5, ddqcd.FP16, mfma) == ddqcd.OK
        assert L.ddqcd_set_sap(h, 16, 5, ddqcd.FP16, lane) == ddqcd.OK
        assert L.ddqcd_set_sap(h, 16, 5, ddqcd.FP64, lane) == ddqcd.OK
        assert L.ddqcd_set_schwarz(h, 2) == ddqcd.ERR_ARG
        assert L.ddqcd_set_schwarz(h, 1) == ddqcd.OK
        assert L.ddqcd_set_schwarz(h, 0) == ddqcd.OK
        assert L.ddqcd_set_solver(h, 0, 1e-10, 10) == ddqcd.ERR_ARG
        assert L.ddqcd_set_solver(h, 17, 1e-10, 10) == ddqcd.ERR_ARG
        assert L.ddqcd_set_solver(h, 16, 0.0, 10) == ddqcd.ERR_ARG
        assert L.ddqcd_set_solver(h, 16, 1e-10, 0) == ddqcd.ERR_ARG
        assert L.ddqcd_set_solver(h, 8, 1e-10, 10) == ddqcd.OK
        assert L.ddqcd_set_outer(h, 2, 0) == ddqcd.ERR_ARG           # no such solver
        assert L.ddqcd_set_outer(h, 0, 3) == ddqcd.ERR_ARG           # FGCR has no deflation
        assert L.ddqcd_set_outer(h, 1, 8) == ddqcd.ERR_ARG           # deflation >= basis size
        assert L.ddqcd_set_outer(h, 1, 4) == ddqcd.OK
        assert L.ddqcd_set_solver(h, 4, 1e-10, 10) == ddqcd.ERR_ARG  # basis no larger than the deflation
        assert L.ddqcd_set_outer(h, 0, 0) == ddqcd.OK
        dummy = ctypes.c_void_p(4096)
        dummy2 = ctypes.c_void_p(8192)
        # no gauge field loaded yet: rejected before any device work
        assert L.ddqcd_apply_D(h, dummy, dummy2, 1, 0, None) == ddqcd.ERR_STATE
        assert L.ddqcd_sap(h, dummy, dummy2, 1, None) == ddqcd.ERR_STATE
        assert L.ddqcd_sap_noalloc(h, dummy, dummy2, None) == ddqcd.ERR_STATE
        assert L.ddqcd_solve(h, dummy, dummy2, 1, 0, None, None) == ddqcd.ERR_STATE
        assert b"load_gauge" in L.ddqcd_last_error(h)
        assert L.ddqcd_solve_bicgstab(h, dummy, dummy2, 0, 100, None, None) == ddqcd.ERR_STATE
        assert L.ddqcd_solve_bicgstab(h, dummy, dummy, 0, 100, None, None) == ddqcd.ERR_ARG    # aliasing
        assert L.ddqcd_solve_bicgstab(h, dummy, dummy2, 0, 0, None, None) == ddqcd.ERR_ARG     # max_iter
        # argument errors
        assert L.ddqcd_apply_D(h, dummy, dummy, 1, 0, None) == ddqcd.ERR_ARG      # aliasing
        assert L.ddqcd_apply_D(h, dummy, dummy2, 0, 0, None) == ddqcd.ERR_ARG     # nrhs
        assert L.ddqcd_apply_D(h, dummy, dummy2, 1, 5, None) == ddqcd.ERR_ARG     # precision
        assert L.ddqcd_load_gauge(h, None, None) == ddqcd.ERR_ARG
    finally:
        assert L.ddqcd_destroy(h) == ddqcd.OK
    assert L.ddqcd_destroy(None) == ddqcd.OK


def test_solve_batch_host_checks():
    L = ddqcd.lib()
    st1, h1 = _create()
    st2, h2 = _create((8, 8, 8, 16), (4, 4, 4, 4))
    assert st1 == st2 == ddqcd.OK
    try:
        vp = ctypes.c_void_p
        hs = (vp * 2)(h1.value, h2.value)
        xs = (vp * 2)(4096, 8192)
        bs = (vp * 2)(12288, 16384)
        assert L.ddqcd_solve_batch(None, 2, xs, bs, 0, None, None) == ddqcd.ERR_ARG
        assert L.ddqcd_solve_batch(hs, 0, xs, bs, 0, None, None) == ddqcd.ERR_ARG
        assert L.ddqcd_solve_batch((vp * 2)(h1.value, None), 2, xs, bs, 0, None, None) == ddqcd.ERR_ARG
        assert L.ddqcd_solve_batch(hs, 2, (vp * 2)(4096, None), bs, 0, None, None) == ddqcd.ERR_ARG
        assert L.ddqcd_solve_batch(hs, 2, xs, (vp * 2)(4096, 16384), 0, None, None) == ddqcd.ERR_ARG  # aliasing
        # no gauge field loaded: rejected before any device work
        assert L.ddqcd_solve_batch(hs, 2, xs, bs, 0, None, None) == ddqcd.ERR_STATE
        assert b"load_gauge" in L.ddqcd_last_error(h1)
    finally:
        assert L.ddqcd_destroy(h1) == ddqcd.OK
        assert L.ddqcd_destroy(h2) == ddqcd.OK


def test_tune_domain_host_paths():
    """Shape enumeration happens before any device work: no fitting shape is a
    geometry error, a single fitting shape is returned without timing."""
    L = ddqcd.lib()
    dom = (ctypes.c_int * 4)()
    ms = ctypes.c_double(0)
    bc = (ctypes.c_double * 4)(1, 1, 1, -1)
    dummy, dummy2 = ctypes.c_void_p(4096), ctypes.c_void_p(8192)

    def tune(lat):
        return L.ddqcd_tune_domain((ctypes.c_int * 4)(*lat), 0.13, 1.5, bc, dummy, dummy2, 2, 16, 5, 16, 1e-10, 64,
                                   dom, ctypes.byref(ms), None)
    assert L.ddqcd_tune_domain(None, 0.13, 1.5, bc, dummy, dummy2, 2, 16, 5, 16, 1e-10, 64, dom, None,
                               None) == ddqcd.ERR_ARG
    assert tune((6, 6, 6, 6)) == ddqcd.ERR_GEOMETRY          # 6 = 2 x 3: odd domain count
    assert tune((4, 4, 4, 4)) == ddqcd.OK                     # only 2^4 tiles it
    assert tuple(dom) == (2, 2, 2, 2) and ms.value == -1


def test_workspace_host_paths():
    """Workspace sizes grow with the number of right-hand sides by at least
    the FGCR basis; misaligned, too small and repeated workspaces are refused
    before any device work."""
    L = ddqcd.lib()
    st, h = _create((16, 16, 16, 16), (4, 4, 4, 4))
    assert st == ddqcd.OK
    try:
        n = ctypes.c_size_t()
        sizes = []
        for k in (1, 2, 4):
            assert L.ddqcd_workspace_size(h, k, ctypes.byref(n)) == ddqcd.OK
            sizes.append(n.value)
        V = 16 ** 4
        assert sizes[0] > V * (576 + 576 + 576)                    # FP64 links, clover, C_e / C_o^-1
        assert sizes[1] - sizes[0] >= V * 192 * (4 + 2 * 16)       # a slot: four FP64 vectors and the basis
        assert sizes[2] - sizes[1] > sizes[1] - sizes[0]
        assert L.ddqcd_workspace_size(h, 0, ctypes.byref(n)) == ddqcd.ERR_ARG
        assert L.ddqcd_set_workspace(h, ctypes.c_void_p(4096 + 8), sizes[2]) == ddqcd.ERR_ARG
        assert L.ddqcd_set_workspace(h, ctypes.c_void_p(4096), sizes[0] - 1) == ddqcd.ERR_NOMEM
        assert L.ddqcd_set_workspace(h, ctypes.c_void_p(1 << 20), sizes[1]) == ddqcd.OK
        assert L.ddqcd_set_workspace(h, ctypes.c_void_p(1 << 20), sizes[1]) == ddqcd.ERR_STATE
    finally:
        assert L.ddqcd_destroy(h) == ddqcd.OK


def test_status_strings():
    assert ddqcd.status_string(ddqcd.ERR_NOT_CONVERGED) == "DDQCD_ERR_NOT_CONVERGED"
    assert ddqcd.status_string(99) == "unknown status"


def test_bench_runs_on_one_gpu_only():
    """bench.py --gpus N with N > 1 exits with status 2 and says why, before any GPU work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""
