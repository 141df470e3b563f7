"""Python binding of the ddqcd C-ABI (include/ddqcd.h).

Argument marshalling only: torch tensors on the GPU become device pointers,
the current torch stream becomes the hipStream_t.  Every step of the solver
runs in libddqcd.so; there is no fallback.  Fields are complex128 tensors in
the canonical layouts: gauge (V, 4, 3, 3), spinor (V, 4, 3) or (nrhs, V, 4, 3).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddqcd.so")

OK, ERR_ARG, ERR_GEOMETRY, ERR_STATE, ERR_DEVICE, ERR_NOMEM, ERR_NOT_CONVERGED, ERR_NONFINITE = range(8)
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
PREC = {"f64": FP64, "f32": FP32, "f16": FP16, "bf16": BF16, FP64: FP64, FP32: FP32, FP16: FP16, BF16: BF16}

SCHED_SWEEPS, SCHED_QUEUE, SCHED_GRAPH = 0, 1, 2
PRODUCT = {"lane": 0, "tile": 1, "mfma_f32": 2, "mfma_bf16": 3}

EXPORTS = ["ddqcd_create", "ddqcd_destroy", "ddqcd_workspace_size", "ddqcd_set_workspace", "ddqcd_set_sap", "ddqcd_set_schedule", "ddqcd_set_schwarz", "ddqcd_set_outer",
           "ddqcd_set_solver", "ddqcd_load_gauge",
           "ddqcd_apply_D", "ddqcd_sap", "ddqcd_sap_noalloc", "ddqcd_solve", "ddqcd_solve_batch", "ddqcd_solve_bicgstab", "ddqcd_tune_domain",
           "ddqcd_tune_sap",
           "ddqcd_last_error",
           "ddqcd_status_string"]


class Info(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int), ("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("t_total_ms", ctypes.c_double), ("t_sap_ms", ctypes.c_double),
                ("t_A_ms", ctypes.c_double), ("t_gs_ms", ctypes.c_double), ("t_other_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DDQCDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1412_2629_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.ddqcd_create.argtypes = [ctypes.POINTER(i), ctypes.POINTER(i), d, d, ctypes.POINTER(d), ctypes.POINTER(vp)]
        L.ddqcd_destroy.argtypes = [vp]
        L.ddqcd_workspace_size.argtypes = [vp, i, ctypes.POINTER(ctypes.c_size_t)]
        L.ddqcd_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
        L.ddqcd_set_sap.argtypes = [vp, i, i, i, i]
        L.ddqcd_set_solver.argtypes = [vp, i, d, i]
        L.ddqcd_set_schedule.argtypes = [vp, i]
        L.ddqcd_set_schwarz.argtypes = [vp, i]
        L.ddqcd_set_outer.argtypes = [vp, i, i]
        L.ddqcd_load_gauge.argtypes = [vp, vp, vp]
        L.ddqcd_apply_D.argtypes = [vp, vp, vp, i, i, vp]
        L.ddqcd_sap.argtypes = [vp, vp, vp, i, vp]
        L.ddqcd_sap_noalloc.argtypes = [vp, vp, vp, vp]
        L.ddqcd_solve.argtypes = [vp, vp, vp, i, i, ctypes.POINTER(Info), vp]
        L.ddqcd_solve_batch.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(vp), ctypes.POINTER(vp), i,
                                        ctypes.POINTER(Info), vp]
        L.ddqcd_solve_bicgstab.argtypes = [vp, vp, vp, i, i, ctypes.POINTER(Info), vp]
        L.ddqcd_tune_domain.argtypes = [ctypes.POINTER(i), d, d, ctypes.POINTER(d), vp, vp, i, i, i, i, d, i,
                                        ctypes.POINTER(i), ctypes.POINTER(d), vp]
        L.ddqcd_tune_sap.argtypes = [ctypes.POINTER(i), d, d, ctypes.POINTER(d), vp, vp, i, i, i, i, i, d, i,
                                     ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(d), vp]
        L.ddqcd_last_error.argtypes = [vp]
        L.ddqcd_last_error.restype = ctypes.c_char_p
        L.ddqcd_status_string.argtypes = [i]
        L.ddqcd_status_string.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("ddqcd_last_error", "ddqcd_status_string"):
                getattr(L, name).restype = i
        _LIB = L
    return _LIB


def status_string(st):
    return lib().ddqcd_status_string(st).decode()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous complex128 tensor")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One lattice: geometry, operator parameters, gauge field and solver state."""

    def __init__(self, lattice, domain, kappa, csw, boundary=(1.0, 1.0, 1.0, -1.0)):
        self.lattice = tuple(int(v) for v in lattice)
        self.domain = tuple(int(v) for v in domain)
        self.V = self.lattice[0] * self.lattice[1] * self.lattice[2] * self.lattice[3]
        h = ctypes.c_void_p()
        st = lib().ddqcd_create((ctypes.c_int * 4)(*self.lattice), (ctypes.c_int * 4)(*self.domain),
                                ctypes.c_double(kappa), ctypes.c_double(csw),
                                (ctypes.c_double * 4)(*[float(b) for b in boundary]), ctypes.byref(h))
        if st != OK:
            raise DDQCDError(st, f"ddqcd_create({self.lattice}, {self.domain}) failed: {status_string(st)}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ddqcd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != OK:
            raise DDQCDError(st, f"{what}: {status_string(st)}: {lib().ddqcd_last_error(self._h).decode()}")

    def workspace_size(self, nrhs=1):
        """Bytes of device memory the context needs for nrhs right-hand sides
        (ddqcd_workspace_size)."""
        n = ctypes.c_size_t()
        self._check(lib().ddqcd_workspace_size(self._h, nrhs, ctypes.byref(n)), "workspace_size")
        return n.value

    def set_workspace(self, ws):
        """Hands the context a device tensor (uint8, contiguous) as its whole
        device memory (ddqcd_set_workspace); the tensor is kept alive with the
        context."""
        import torch
        if not isinstance(ws, torch.Tensor) or not ws.is_cuda or not ws.is_contiguous():
            raise TypeError("workspace must be a contiguous CUDA (HIP) tensor")
        self._check(lib().ddqcd_set_workspace(self._h, ctypes.c_void_p(ws.data_ptr()),
                                              ws.numel() * ws.element_size()), "set_workspace")
        self._workspace = ws

    def set_sap(self, n_cycles=16, n_mr=5, prec="f32", product="lane"):
        """product: "lane" (one right-hand side per workgroup), "tile" (four per
        workgroup, VALU products), "mfma_f32" or "mfma_bf16" (four per workgroup,
        link products on matrix instructions)."""
        self._check(lib().ddqcd_set_sap(self._h, n_cycles, n_mr, PREC[prec], PRODUCT[product]), "set_sap")

    def set_schedule(self, schedule):
        """"sweeps" (one launch per colour of a half-sweep), "graph" (the same launches replayed
        from a captured HIP graph) or "queue" (persistent work-queue kernel, switched off)."""
        mode = {"sweeps": SCHED_SWEEPS, "queue": SCHED_QUEUE, "graph": SCHED_GRAPH}.get(schedule, schedule)
        self._check(lib().ddqcd_set_schedule(self._h, mode), "set_schedule")

    def set_schwarz(self, kind):
        """"multiplicative" (the default) or "additive" Schwarz preconditioner."""
        mode = {"multiplicative": 0, "additive": 1}.get(kind, kind)
        self._check(lib().ddqcd_set_schwarz(self._h, mode), "set_schwarz")

    def set_outer(self, kind="fgcr", deflate=0):
        """"fgcr" (the default), "fgmres_dr" with `deflate` deflation vectors
        (the basis size is the restart of set_solver) or "fgcr_mixed" (FP64
        iterative refinement around FP32 FGCR cycles)."""
        mode = {"fgcr": 0, "fgmres_dr": 1, "fgcr_mixed": 2}.get(kind, kind)
        self._check(lib().ddqcd_set_outer(self._h, mode, deflate), "set_outer")

    def set_solver(self, restart=16, tol=1e-10, max_cycles=64):
        self._check(lib().ddqcd_set_solver(self._h, restart, ctypes.c_double(tol), max_cycles), "set_solver")

    def load_gauge(self, U):
        assert U.shape == (self.V, 4, 3, 3), U.shape
        self._check(lib().ddqcd_load_gauge(self._h, _ptr(U, "U"), _stream()), "load_gauge")

    def _nrhs(self, t):
        if t.shape == (self.V, 4, 3):
            return 1
        assert t.dim() == 4 and t.shape[1:] == (self.V, 4, 3), t.shape
        return t.shape[0]

    def apply_D(self, psi, prec="f64", out=None):
        import torch
        out = torch.empty_like(psi) if out is None else out
        self._check(lib().ddqcd_apply_D(self._h, _ptr(out, "out"), _ptr(psi, "in"), self._nrhs(psi), PREC[prec],
                                        _stream()), "apply_D")
        return out

    def sap(self, eta, out=None):
        import torch
        out = torch.empty_like(eta) if out is None else out
        self._check(lib().ddqcd_sap(self._h, _ptr(out, "out"), _ptr(eta, "in"), self._nrhs(eta), _stream()), "sap")
        return out

    def sap_noalloc(self, eta, out=None):
        """out = M eta for one right-hand side through ddqcd_sap_noalloc (the
        library allocates nothing; out is allocated here unless given)."""
        import torch
        assert eta.shape == (self.V, 4, 3), eta.shape
        out = torch.empty_like(eta) if out is None else out
        self._check(lib().ddqcd_sap_noalloc(self._h, _ptr(out, "out"), _ptr(eta, "in"), _stream()), "sap_noalloc")
        return out

    def solve_bicgstab(self, b, x0=None, max_iter=20000, check=True):
        """FP64 BiCGstab without preconditioner (one right-hand side).  Returns (x, info dict, status)."""
        import torch
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        info = Info()
        st = lib().ddqcd_solve_bicgstab(self._h, _ptr(x, "x"), _ptr(b, "b"), 0 if x0 is None else 1, max_iter,
                                        ctypes.byref(info), _stream())
        if check and st not in (OK, ERR_NOT_CONVERGED):
            self._check(st, "solve_bicgstab")
        return x, info.as_dict(), st

    def solve(self, b, x0=None, check=True):
        """Returns (x, [info dicts], status)."""
        import torch
        nrhs = self._nrhs(b)
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        infos = (Info * nrhs)()
        st = lib().ddqcd_solve(self._h, _ptr(x, "x"), _ptr(b, "b"), nrhs, 0 if x0 is None else 1, infos, _stream())
        if check and st not in (OK, ERR_NOT_CONVERGED):
            self._check(st, "solve")
        return x, [i.as_dict() for i in infos], st


def solve_batch(contexts, bs, x0s=None, check=True):
    """Solves contexts[i] x_i = bs[i] for all i at once (ddqcd_solve_batch).

    bs[i] is one (V_i, 4, 3) field of contexts[i]; a context may appear more
    than once.  Returns ([x_i], [info dicts], status)."""
    import torch
    n = len(contexts)
    assert len(bs) == n and n > 0
    for c, b in zip(contexts, bs):
        assert b.shape == (c.V, 4, 3), b.shape
    xs = [torch.zeros_like(b) if x0s is None else x0s[i].clone() for i, b in enumerate(bs)]
    hs = (ctypes.c_void_p * n)(*[c._h for c in contexts])
    xp = (ctypes.c_void_p * n)(*[_ptr(x, "x").value for x in xs])
    bp = (ctypes.c_void_p * n)(*[_ptr(b, "b").value for b in bs])
    infos = (Info * n)()
    st = lib().ddqcd_solve_batch(hs, n, xp, bp, 0 if x0s is None else 1, infos, _stream())
    if check and st not in (OK, ERR_NOT_CONVERGED):
        msg = lib().ddqcd_last_error(contexts[0]._h).decode()
        raise DDQCDError(st, f"solve_batch: {status_string(st)}: {msg}")
    return xs, [i.as_dict() for i in infos], st


def tune_domain(lattice, kappa, csw, U, b, prec="f16", n_cycles=16, n_mr=5, restart=16, tol=1e-10, max_cycles=64,
                boundary=(1.0, 1.0, 1.0, -1.0)):
    """The fastest compiled domain shape for this lattice and gauge field
    (ddqcd_tune_domain).  Returns (domain, ms); ms is -1 when only one shape
    fits and nothing was timed."""
    dom = (ctypes.c_int * 4)()
    ms = ctypes.c_double()
    st = lib().ddqcd_tune_domain((ctypes.c_int * 4)(*[int(v) for v in lattice]), ctypes.c_double(kappa),
                                 ctypes.c_double(csw), (ctypes.c_double * 4)(*[float(v) for v in boundary]),
                                 _ptr(U, "U"), _ptr(b, "b"), PREC[prec], n_cycles, n_mr, restart,
                                 ctypes.c_double(tol), max_cycles, dom, ctypes.byref(ms), _stream())
    if st != OK:
        raise DDQCDError(st, f"tune_domain({tuple(lattice)}): {status_string(st)}")
    return tuple(dom), ms.value


def tune_sap(lattice, kappa, csw, U, b, prec="f16", n_cycles=16, n_mr=5, restart=16, tol=1e-10, max_cycles=64,
             boundary=(1.0, 1.0, 1.0, -1.0)):
    """The fastest (domain shape, product form) for solving the right-hand
    sides b ((V, 4, 3) or (nrhs, V, 4, 3)) together on this lattice and gauge
    field (ddqcd_tune_sap).  Returns (domain, product name, ms); ms is -1 when
    only one pair fits and nothing was timed."""
    V = int(lattice[0]) * int(lattice[1]) * int(lattice[2]) * int(lattice[3])
    nrhs = 1 if tuple(b.shape) == (V, 4, 3) else b.shape[0]
    dom = (ctypes.c_int * 4)()
    prod = ctypes.c_int()
    ms = ctypes.c_double()
    st = lib().ddqcd_tune_sap((ctypes.c_int * 4)(*[int(v) for v in lattice]), ctypes.c_double(kappa),
                              ctypes.c_double(csw), (ctypes.c_double * 4)(*[float(v) for v in boundary]),
                              _ptr(U, "U"), _ptr(b, "b"), nrhs, PREC[prec], n_cycles, n_mr, restart,
                              ctypes.c_double(tol), max_cycles, dom, ctypes.byref(prod), ctypes.byref(ms), _stream())
    if st != OK:
        raise DDQCDError(st, f"tune_sap({tuple(lattice)}): {status_string(st)}")
    name = {v: k for k, v in PRODUCT.items()}[prod.value]
    return tuple(dom), name, ms.value
