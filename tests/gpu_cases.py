"""Shared set-up of the GPU parity tests: seeded lattices, oracle fields and
torch <-> numpy transfers.  Inputs come from paper_1412_2629_amd.inputs only;
expected values from the oracle only."""
import functools

import numpy as np

from paper_1412_2629_amd import inputs

BC = (1.0, 1.0, 1.0, -1.0)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def site_err(got, want):
    """(normwise relative error, largest error of one site relative to the
    RMS site norm of want): an error confined to a few sites (a face layer, one
    domain) shows in the second figure even where the norm hides it."""
    g = np.asarray(got).reshape(-1, 12)
    w = np.asarray(want).reshape(-1, 12)
    d = np.linalg.norm(g - w, axis=1)
    n = np.linalg.norm(w, axis=1)
    return float(np.linalg.norm(d) / np.linalg.norm(n)), float(d.max() / np.sqrt(np.mean(n * n)))


# Block-solve output against the FP64 oracle:
# FP32 arithmetic accumulates a few unit roundoffs per MR step; FP16 storage
# rounds each stored link, clover entry, block residual and boundary term once
# per half-sweep (BF16 storage likewise, with its u = 2^-8).  Each Schwarz
# cycle contracts the error the earlier cycles left, so the error does not
# grow with the cycle count.  Normwise bounds: 8 u (FP32, u = 2^-24) and 4 u
# (FP16 and BF16 storage); one site's error may reach SITE_FACTOR times that
# relative to the RMS site norm.
SAP_TOL = {"f64": 1e-12, "f32": 8 * 2.0 ** -24, "f16": 4 * 2.0 ** -11, "bf16": 4 * 2.0 ** -8}
# The operator with reduced storage (spec bounds; BF16 storage is held
# to the FP16 bound, about 1.3 u_bf16)
A_TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 5e-3, "bf16": 5e-3}
SITE_FACTOR = 4.0
# The tile forms of the FP16-storage block solve (ddqcd_set_sap product):
# VALU and FP32-MFMA products keep the FP16 bound; BF16-input MFMA rounds the
# link and the projected half-spinor to BF16 (u = 2^-8) in every product, a
# relative perturbation of the block operator of at most about 2u per
# application, which the block solve passes on to its output: 2 u_bf16.
PRODUCT_TOL = {"lane": SAP_TOL["f16"], "tile": SAP_TOL["f16"], "mfma_f32": SAP_TOL["f16"],
               "mfma_bf16": 2 * 2.0 ** -8}


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


class Case:
    def __init__(self, name, L, b, kappa, csw, eps, seed, n_cycles=16, n_mr=5):
        self.name, self.L, self.b = name, tuple(L), tuple(b)
        self.kappa, self.csw, self.eps, self.seed = kappa, csw, eps, seed
        self.n_cycles, self.n_mr = n_cycles, n_mr
        self.V = int(np.prod(L))

    def __repr__(self):
        return self.name

    @functools.cached_property
    def U(self):
        return inputs.random_gauge(self.L, self.eps, self.seed)

    @functools.cached_property
    def C(self):
        import oracle as O
        return O.clover_field(self.L, self.U, self.kappa, self.csw)

    @functools.cached_property
    def Ci(self):
        import oracle as O
        return O.clover_inverse(self.C)

    def source(self, seed=None):
        return inputs.gaussian_source(self.L, self.seed + 1 if seed is None else seed)

    def context(self, prec=None):
        from paper_1412_2629_amd import ddqcd
        ctx = ddqcd.Context(self.L, self.b, self.kappa, self.csw, BC)
        ctx.load_gauge(dev(self.U))
        if prec is not None:
            ctx.set_sap(self.n_cycles, self.n_mr, prec)
        return ctx



SMALL = [
    Case("4^4/2^4", (4, 4, 4, 4), (2, 2, 2, 2), 0.12, 1.0, 0.3, 101, 8, 4),
    Case("4x8x4x12/2^4", (4, 8, 4, 12), (2, 2, 2, 2), 0.1365, 1.7, 0.6, 111, 4, 3),
    Case("8^4/4^4", (8, 8, 8, 8), (4, 4, 4, 4), 0.13, 1.5, 0.5, 121, 4, 5),
    Case("16x8x8x8/8x4^3", (16, 8, 8, 8), (8, 4, 4, 4), 0.1355, 1.5, 0.5, 131, 4, 5),
    Case("8x8x8x16/4^3x8", (8, 8, 8, 16), (4, 4, 4, 8), 0.13, 1.5, 0.5, 141, 4, 5),
    Case("12x12x4x8/6x6x2x4", (12, 12, 4, 8), (6, 6, 2, 4), 0.13, 1.5, 0.5, 151, 4, 5),
]

# Four or more domains in every direction, so the -mu and +mu neighbour
# domains of every domain differ (with two per direction they coincide): the
# neighbour and face indexing of each compiled domain shape.
WIDE = [
    Case("8^4/2^4", (8, 8, 8, 8), (2, 2, 2, 2), 0.13, 1.5, 0.5, 161, 8, 4),
    Case("16^4/4^4", (16, 16, 16, 16), (4, 4, 4, 4), 0.13, 1.5, 0.5, 171, 8, 5),
    Case("32x16x16x16/8x4^3", (32, 16, 16, 16), (8, 4, 4, 4), 0.1355, 1.5, 0.5, 181, 8, 5),
    Case("16x16x16x32/4^3x8", (16, 16, 16, 32), (4, 4, 4, 8), 0.13, 1.5, 0.5, 191, 8, 5),
    Case("24x24x8x16/6x6x2x4", (24, 24, 8, 16), (6, 6, 2, 4), 0.13, 1.5, 0.5, 199, 8, 5),
]

# Block solves on 288-site domains run in 320-thread workgroups with idle
# padding threads; the FP64 block-solve kernels are built for whole waves (or
# 16-site domains) only, and the library rejects FP64 for this shape.
NO_FP64_SAP = "no FP64 block-solve kernel for 6x6x2x4 domains (padded workgroups)"


def fp64_sap(case):
    return case.b != (6, 6, 2, 4)
