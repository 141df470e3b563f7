"""The five synthetic workloads, with their solver parameters and seeds.

Mass parameter: the paper writes A = (4 + m) - D_w/2 + D_cl (Sec. II-B, Eq. 1);
the workloads are quoted in kappa, with 4 + m = 1/(2 kappa).  Boundary phases:
periodic in x, y, z and antiperiodic in t.  The Schwarz and block-solver
iteration counts (I_Schwarz, I_domain) follow Sec. II-D / Sec. IV-C; where a
workload gives none, the paper's tuned values (16 cycles, 5 MR iterations)
are used.
"""
from dataclasses import dataclass, field
import numpy as np

BC_APT = (1.0, 1.0, 1.0, -1.0)


@dataclass
class Workload:
    name: str
    lattice: tuple          # (Lx, Ly, Lz, Lt)
    domain: tuple           # (bx, by, bz, bt)
    kappa: float
    csw: float
    eps: float
    n_cycles: int           # I_Schwarz
    n_mr: int               # I_domain
    prec: str               # SAP storage precision: "f64", "f32" or "f16"
    restart: int = 16
    tol: float = 1e-10
    nrhs: int = 1
    gauge_seed: int = 0
    source_seed: int = 0
    bc: tuple = BC_APT

    @property
    def volume(self):
        L = self.lattice
        return L[0] * L[1] * L[2] * L[3]


C1 = Workload("4^4 plain FP64", (4, 4, 4, 4), (2, 2, 2, 2), 0.12, 1.0, 0.3,
              8, 4, "f64", gauge_seed=101, source_seed=102)
C2 = Workload("16^3x32 FP32 SAP", (16, 16, 16, 32), (8, 4, 4, 4), 0.1355, 1.5, 0.5,
              16, 5, "f32", gauge_seed=201, source_seed=202)
C3 = Workload("32^3x64 FP16-storage SAP", (32, 32, 32, 64), (8, 4, 4, 4), 0.1365, 1.7, 0.6,
              16, 5, "f16", gauge_seed=301, source_seed=302)
C4 = Workload("32^3x64 12 point sources", (32, 32, 32, 64), (8, 4, 4, 4), 0.1365, 1.7, 0.6,
              16, 5, "f16", nrhs=12, gauge_seed=301, source_seed=0)

WORKLOADS = {"C1": C1, "C2": C2, "C3": C3, "C4": C4}


def uneven_batch():
    """The 24-lattice uneven batch: 8 x 8^4, 8 x 12^3x24, 6 x 16^3x32, 2 x 24^3x48.

    (eps_j, kappa_j) are drawn from PCG64(4999); lattice j uses gauge seed
    5000+j and source seed 6000+j.  Domain shapes are chosen per lattice
    among those with an even domain count (>= 2) in every direction.
    """
    shapes = [(8, 8, 8, 8)] * 8 + [(12, 12, 12, 24)] * 8 + [(16, 16, 16, 32)] * 6 + [(24, 24, 24, 48)] * 2
    doms = {(8, 8, 8, 8): (4, 4, 4, 4), (12, 12, 12, 24): (2, 2, 2, 2),
            (16, 16, 16, 32): (8, 4, 4, 4), (24, 24, 24, 48): (4, 4, 4, 4)}
    rng = np.random.Generator(np.random.PCG64(4999))
    eps = rng.uniform(0.3, 0.6, size=len(shapes))
    kap = rng.uniform(0.12, 0.136, size=len(shapes))
    out = []
    for j, L in enumerate(shapes):
        out.append(Workload(f"batch[{j}] {L}", L, doms[L], float(kap[j]), 1.5, float(eps[j]),
                            16, 5, "f16", gauge_seed=5000 + j, source_seed=6000 + j))
    return out
