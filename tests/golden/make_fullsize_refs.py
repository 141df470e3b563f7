"""Writes tests/golden/fullsize_refs.npz: the oracle's solutions of the large
workloads at a seeded sample of sites, for the GPU solution-parity tests.

    python tests/golden/make_fullsize_refs.py [case ...]

Only the oracle (oracle/) and the seeded input generators
(paper_1412_2629_amd/inputs.py) are called.  Each solution is the oracle's own
FGCR solve (FP64 SAP preconditioner with the workload's domains, I_S = 16,
I_D = 5) to true relative residual 1e-12; a whole 32^3x64 solution is 403 MB,
so the file keeps the solution at 512 seeded random sites together with its
full norm, the oracle's step count and its final residual.  The inputs are
regenerated from their seeds by the tests.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1412_2629_amd import configs, inputs  # noqa: E402

OUT = os.path.join(HERE, "fullsize_refs.npz")
N_SITES = 512
TOL = 1e-12

# point source (spin, colour) of each 12-source right-hand side: rhs = 3 * spin + colour
C4_RHS = (0, 5, 11)
C5_LATTICES = (8, 16, 22)   # one lattice of each size above 8^4


def cases():
    """(key, workload, source builder)"""
    out = [("C3", configs.C3, lambda w: inputs.gaussian_source(w.lattice, w.source_seed))]
    for k in C4_RHS:
        out.append((f"C4_rhs{k}", configs.C4, lambda w, k=k: inputs.point_source(w.lattice, 0, k // 3, k % 3)))
    ws = configs.uneven_batch()
    for j in C5_LATTICES:
        out.append((f"C5_lat{j}", ws[j], lambda w: inputs.gaussian_source(w.lattice, w.source_seed)))
    return out


def sample_sites(key, V):
    seed = sum(ord(ch) for ch in key)
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(V, size=N_SITES, replace=False)).astype(np.int64)


def main(only):
    store = dict(np.load(OUT)) if os.path.exists(OUT) else {}
    meta_path = OUT.replace(".npz", ".json")
    meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
    gauge_cache = {}
    for key, w, src in cases():
        if only and key not in only:
            continue
        t0 = time.time()
        gk = (w.lattice, w.eps, w.gauge_seed)
        if gk not in gauge_cache:
            gauge_cache.clear()
            gauge_cache[gk] = inputs.random_gauge(w.lattice, w.eps, w.gauge_seed)
        U = gauge_cache[gk]
        f = src(w)
        C = O.clover_field(w.lattice, U, w.kappa, w.csw)
        Ci = O.clover_inverse(C)
        x, st, steps, rr = O.fgcr(w.lattice, w.domain, w.bc, U, C, Ci, f, n_cycles=w.n_cycles, n_mr=w.n_mr,
                                  restart=w.restart, tol=TOL, max_cycles=200)
        assert st == 0, (key, st, rr)
        sites = sample_sites(key, w.volume)
        store[key + "_sites"] = sites
        store[key + "_x"] = np.ascontiguousarray(x[sites])
        meta[key] = {"lattice": list(w.lattice), "domain": list(w.domain), "kappa": w.kappa, "csw": w.csw,
                     "eps": w.eps, "gauge_seed": w.gauge_seed, "n_cycles": w.n_cycles, "n_mr": w.n_mr,
                     "restart": w.restart, "tol": TOL, "oracle_steps": steps, "oracle_relres": rr,
                     "x_norm": float(np.linalg.norm(x)), "n_sites": N_SITES}
        del x, C, Ci
        np.savez(OUT, **store)
        json.dump(meta, open(meta_path, "w"), indent=1, sort_keys=True)
        print(f"{key}: {steps} oracle steps, residual {rr:.2e}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(set(sys.argv[1:]))
