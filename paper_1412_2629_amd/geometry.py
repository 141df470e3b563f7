"""Host-side geometry of the domain decomposition: domain counts, the load
model, domain working sets and the flop/byte accounting used by the
benchmark.  No GPU code and no solver arithmetic lives here.

Flop conventions.  The paper counts 1344 flop/site for the Wilson hopping
term and 504 for the clover term, 1848 for A (Sec. II-B).  The throughput
figures here use 165 flop per computed hop (1320 per site for eight hops;
the remaining 24 of the paper's 1344 are the final summation, counted
with the site term) and 504 per clover (or inverse clover) application.
"""
import math

HOP_FLOPS = 165            # project, SU(3) x half-spinor, reconstruct+accumulate
DSLASH_FLOPS = 8 * HOP_FLOPS   # 1320
CLOVER_FLOPS = 504         # two Hermitian 6x6 complex mat-vecs (incl. the 4+m diagonal)
A_FLOPS = DSLASH_FLOPS + CLOVER_FLOPS  # 1824 per site
PAPER_DW_FLOPS = 1344
PAPER_A_FLOPS = 1848


def volume(L):
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def domain_grid(L, b):
    return tuple(int(L[m]) // int(b[m]) for m in range(4))


def check_domains(L, b):
    """True if b divides L and every direction has an even number >= 2 of
    domains (needed for a consistent black/white colouring on the torus)."""
    for m in range(4):
        if b[m] < 1 or L[m] % b[m]:
            return False
        n = L[m] // b[m]
        if n < 2 or n % 2:
            return False
    return True


def n_domain(V, V_domain):
    """Domains that can be processed at once in multiplicative Schwarz: half of
    all domains, one colour at a time (Sec. IV-B2, Eq. n_domain)."""
    return V // (2 * V_domain)


def load(n_dom, n_core):
    """Average load of n_dom independent domains on n_core workers handed out
    round-robin (Sec. IV-B2, Eq. load)."""
    return n_dom / (n_core * math.ceil(n_dom / n_core))


def domain_working_set(b, spinor_bytes=4, gauge_bytes=4, n_half_spinors=7):
    """Bytes of one domain's block-solve working set as counted in Sec. III-B:
    seven half-lattice spinors, the four forward links of every site and the
    two packed 6x6 clover blocks of every site."""
    Vd = volume(b)
    spinors = n_half_spinors * (Vd // 2) * 24 * spinor_bytes
    links = Vd * 4 * 18 * gauge_bytes
    clover = Vd * 72 * gauge_bytes
    return {"spinors": spinors, "links": links, "clover": clover, "total": spinors + links + clover}


def in_domain_hops(b):
    """Number of (site, direction, sign) hops with both ends in one domain."""
    Vd = volume(b)
    return sum(2 * (b[m] - 1) * (Vd // b[m]) for m in range(4))


def face_hops(b):
    """Hops that cross the domain boundary, counted at the receiving site."""
    Vd = volume(b)
    return sum(2 * (Vd // b[m]) for m in range(4))


def sap_flops_per_domain(b, n_mr):
    """Algorithmic flops of one block update in a SAP half-sweep, counted from
    the geometry (165 per hop, 504 per clover or inverse-clover apply,
    24 per complex 12-vector add, 96/48 per complex dot/norm, 96 per axpy):

      staging     face hops into the domain (the R term of the previous sweep)
      prep        C_o^-1 on odd sites, hops odd->even, subtraction
      MR x n_mr   hops even->odd, C_o^-1, hops odd->even, C_e, combine,
                  <p,r>, <p,p>, two axpys
      reconstruct hops even->odd, subtraction, C_o^-1
      epilogue    psi += delta

    Returns a dict with the 'dslash' part (hops and clovers only) and 'total'."""
    Vd = volume(b)
    h = Vd // 2
    hin = in_domain_hops(b)          # split evenly between the two parities
    he = hin // 2
    ho = hin - he
    fh = face_hops(b)
    dslash = fh * HOP_FLOPS
    dslash += h * CLOVER_FLOPS + he * HOP_FLOPS                     # prep
    dslash += n_mr * ((ho + he) * HOP_FLOPS + 2 * h * CLOVER_FLOPS)  # MR
    dslash += ho * HOP_FLOPS + h * CLOVER_FLOPS                     # reconstruct
    blas = h * 24 + n_mr * h * (24 + 96 + 48 + 96 + 96) + h * 24 + Vd * 24
    return {"dslash": dslash, "total": dslash + blas}


def sap_call_flops(L, b, n_cycles, n_mr, nrhs=1):
    Vd = volume(b)
    nd = volume(L) // Vd
    f = sap_flops_per_domain(b, n_mr)
    return {k: v * nd * n_cycles * nrhs for k, v in f.items()}


def a_bytes_per_site(prec):
    """Minimum HBM bytes of one application of A per site (spinor in, links,
    clover, spinor out), each field read once."""
    if prec == "f64":
        return 192 + 576 + 576 + 192
    if prec == "f32":
        return 96 + 4 * 12 * 4 + 72 * 4 + 96
    if prec == "f16":
        return 48 + 4 * 12 * 2 + 72 * 2 + 48
    raise ValueError(prec)


def face_sites(b):
    """Sites on the faces of a domain, counted once per face (a site on two
    faces counts twice): the boundary half-spinors one domain writes."""
    Vd = volume(b)
    return sum(2 * (Vd // b[m]) for m in range(4))


def sap_bytes_per_domain(b, prec, nrhs=1):
    """Algorithmic HBM bytes of one visit of one domain by nrhs right-hand
    sides in a SAP half-sweep (each field read once, each result written once):
    the two-row links and the site clover blocks (C_e / C_o^-1) once, and per
    right-hand side the stored block residual of the even sites (read and
    written), the solution accumulator (FP32, read and written) and the
    boundary half-spinors (read from the neighbours, written for them).  prec:
    "f32" or "f16" storage of links, clover, residual and boundary terms."""
    Vd = volume(b)
    c = {"f32": 8, "f16": 4}[prec]          # bytes per stored complex number
    shared = Vd * (4 * 6 * c + 36 * c)
    per_rhs = Vd // 2 * 12 * c * 2 + Vd * 12 * 8 * 2 + face_sites(b) * 6 * c * 2
    return shared + nrhs * per_rhs
