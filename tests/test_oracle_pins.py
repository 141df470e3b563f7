"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks one part of the oracle against something other than the
oracle itself: a closed form, an invariant, a textbook routine applied to a
dense matrix, or brute force on a tiny lattice.
"""
import numpy as np
import pytest

from paper_1412_2629_amd import inputs
from tests import dense_ref as R

BC = (1.0, 1.0, 1.0, -1.0)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------------------
# A: free field closed form in momentum space (Sec. II-B, Eqs. 1-2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc", [(1.0, 1.0, 1.0, -1.0), (1.0, 1.0, 1.0, 1.0), (-1.0, 1.0, -1.0, 1.0)])
def test_free_field_plane_waves(oracle, bc):
    """With U = 1 the clover vanishes and a plane wave e^{ipx} u with
    p_mu = (2 pi n + pi [bc=-1]) / L_mu is an eigenfunction in position space:
    A -> 1/(2 kappa) - sum_mu cos p_mu + i sum_mu gamma_mu sin p_mu."""
    L = (3, 4, 5, 6)
    kappa, csw = 0.13, 1.7
    U = inputs.unit_gauge(L)
    C = oracle.clover_field(L, U, kappa, csw)
    assert np.abs(C - np.eye(12) / (2 * kappa)).max() < 1e-15
    rng = np.random.default_rng(5)
    c = R.coords(L)
    for trial in range(6):
        n = rng.integers(0, 7, size=4)
        p = np.array([(2 * np.pi * n[m] + (np.pi if bc[m] < 0 else 0)) / L[m] for m in range(4)])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (c @ p))
        psi = phase[:, None, None] * u[None]
        out = oracle.apply_A(L, bc, U, C, psi)
        K = (1 / (2 * kappa) - np.cos(p).sum()) * np.eye(4) + 1j * sum(R.GAMMA[m] * np.sin(p[m]) for m in range(4))
        want = phase[:, None, None] * (K @ u)[None]
        assert rel(out, want) < 1e-14, trial


# ---------------------------------------------------------------------------
# A: gamma5-hermiticity and gauge covariance
# ---------------------------------------------------------------------------

def test_gamma5_hermiticity(oracle):
    """gamma5 A is Hermitian: <phi, g5 A psi> = <g5 A phi, psi>."""
    L = (4, 4, 4, 6)
    U = inputs.random_gauge(L, 0.6, 11)
    C = oracle.clover_field(L, U, 0.1365, 1.7)
    V = R.coords(L).shape[0]
    phi = inputs.gaussian_spinor(V, 12)
    psi = inputs.gaussian_spinor(V, 13)
    g5 = np.diag(R.GAMMA5).real
    lhs = np.vdot(phi, np.einsum("s,nsc->nsc", g5, oracle.apply_A(L, BC, U, C, psi)))
    rhs = np.vdot(np.einsum("s,nsc->nsc", g5, oracle.apply_A(L, BC, U, C, phi)), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_gamma5_is_diag(oracle):
    assert np.allclose(R.GAMMA5, np.diag([-1, -1, 1, 1]))


def _gauge_transform(L, U, Om):
    Un = np.empty_like(U)
    for mu in range(4):
        fwd = R.shift(L, mu, +1)
        Un[:, mu] = Om @ U[:, mu] @ Om[fwd].conj().transpose(0, 2, 1)
    return Un


def test_gauge_covariance(oracle):
    """A[U^Om](Om psi) = Om A[U] psi, U^Om_mu(x) = Om(x) U_mu(x) Om(x+mu)^dag."""
    L = (4, 4, 6, 4)
    kappa, csw = 0.125, 1.9
    U = inputs.random_gauge(L, 0.5, 21)
    V = U.shape[0]
    Om = inputs.random_su3(V, 22)
    Ug = _gauge_transform(L, U, Om)
    psi = inputs.gaussian_spinor(V, 23)
    C = oracle.clover_field(L, U, kappa, csw)
    Cg = oracle.clover_field(L, Ug, kappa, csw)
    lhs = oracle.apply_A(L, BC, Ug, Cg, np.einsum("nab,nsb->nsa", Om, psi))
    rhs = np.einsum("nab,nsb->nsa", Om, oracle.apply_A(L, BC, U, C, psi))
    assert rel(lhs, rhs) < 1e-13


# ---------------------------------------------------------------------------
# Clover term (Sec. II-B, Eq. 3)
# ---------------------------------------------------------------------------

def _constant_field(L, mu, nu, k):
    """Abelian field with every (mu,nu) plaquette equal to exp(i theta T),
    T = diag(1,-1,0), theta = 2 pi k / L_mu: U_nu(x) = exp(i theta x_mu T),
    all other links 1."""
    theta = 2 * np.pi * k / L[mu]
    U = inputs.unit_gauge(L)
    xm = R.coords(L)[:, mu]
    U[:, nu, 0, 0] = np.exp(1j * theta * xm)
    U[:, nu, 1, 1] = np.exp(-1j * theta * xm)
    return U, theta


@pytest.mark.parametrize("mu,nu", [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])
def test_clover_constant_field(oracle, mu, nu):
    """For a constant abelian field in one plane, Q_munu = 4 P with P the
    plaquette, so D_cl = -(c_sw/2) sigma_munu (x) sin(theta T) at every site."""
    L = (4, 6, 4, 8)
    kappa, csw = 0.13, 1.3
    U, theta = _constant_field(L, mu, nu, 1)
    C = oracle.clover_field(L, U, kappa, csw)
    sinT = np.diag(np.sin(theta * np.array([1.0, -1.0, 0.0])))
    want = np.eye(12) / (2 * kappa) - (csw / 2) * np.kron(R.sigma(mu, nu), sinT)
    assert np.abs(C - want[None]).max() < 1e-14


def test_clover_constant_field_block_forms(oracle):
    """Hand-derived chiral blocks: sigma_xy = -diag(s3, s3) and
    sigma_zt = diag(-s3, s3), so the xy field gives +(c_sw/2) diag(s3, s3) sinT and
    the zt field gives +(c_sw/2) diag(s3, -s3) sinT (spin-major, colour-minor)."""
    L = (4, 4, 4, 4)
    kappa, csw = 0.12, 1.0
    s3 = np.diag([1.0, -1.0])
    for (mu, nu), spin in [((0, 1), np.kron(np.eye(2), s3)), ((2, 3), np.kron(np.diag([1.0, -1.0]), s3))]:
        U, theta = _constant_field(L, mu, nu, 1)
        sinT = np.diag(np.sin(theta * np.array([1.0, -1.0, 0.0])))
        C = oracle.clover_field(L, U, kappa, csw)
        want = np.eye(12) / (2 * kappa) + (csw / 2) * np.kron(spin, sinT)
        assert np.abs(C[7] - want).max() < 1e-14


def test_clover_pure_gauge_and_linearity(oracle):
    L = (4, 4, 4, 4)
    V = 256
    Om = inputs.random_su3(V, 31)
    U = _gauge_transform(L, inputs.unit_gauge(L), Om)
    C = oracle.clover_field(L, U, 0.12, 1.7)
    assert np.abs(C - np.eye(12) / 0.24).max() < 1e-13
    U = inputs.random_gauge(L, 0.5, 32)
    D1 = oracle.clover_field(L, U, 0.12, 1.0) - np.eye(12) / 0.24
    D2 = oracle.clover_field(L, U, 0.12, 2.5) - np.eye(12) / 0.24
    assert np.abs(D2 - 2.5 * D1).max() < 1e-13
    assert np.abs(D1 - D1.conj().transpose(0, 2, 1)).max() < 1e-15
    assert np.abs(D1[:, :6, 6:]).max() == 0 and np.abs(D1[:, 6:, :6]).max() == 0
    assert np.abs(D1).max() > 0.05


def test_clover_inverse(oracle):
    L = (4, 4, 4, 4)
    U = inputs.random_gauge(L, 0.6, 33)
    C = oracle.clover_field(L, U, 0.1365, 1.7)
    Ci = oracle.clover_inverse(C)
    assert np.abs(np.einsum("nij,njk->nik", C, Ci) - np.eye(12)).max() < 1e-14


def test_apply_sites_matches_full(oracle):
    L = (4, 4, 4, 6)
    U = inputs.random_gauge(L, 0.5, 41)
    C = oracle.clover_field(L, U, 0.13, 1.5)
    psi = inputs.gaussian_spinor(U.shape[0], 42)
    full = oracle.apply_A(L, BC, U, C, psi)
    sites = np.array([0, 5, 17, 63, 200, 383])
    part = oracle.apply_A_sites(L, BC, U, 0.13, 1.5, psi, sites)
    assert np.abs(part - full[sites]).max() < 1e-14


# ---------------------------------------------------------------------------
# Domain split A = D + R (Sec. II-D)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("L,b", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 4, 4, 8), (4, 2, 2, 2)),
                                 ((6, 4, 4, 4), (3, 2, 2, 2))])
def test_split_D_plus_R(oracle, L, b):
    U = inputs.random_gauge(L, 0.5, 51)
    C = oracle.clover_field(L, U, 0.13, 1.5)
    V = U.shape[0]
    psi = inputs.gaussian_spinor(V, 52)
    A = oracle.apply_A(L, BC, U, C, psi)
    D = oracle.apply_Dblock(L, b, BC, U, C, psi)
    Rr = oracle.apply_R(L, b, BC, U, C, psi)
    assert rel(D + Rr, A) < 1e-15
    dom, _ = R.domain_ids(L, b)
    sel = dom == 3
    v = psi * sel[:, None, None]
    assert np.abs(oracle.apply_Dblock(L, b, BC, U, C, v)[~sel]).max() == 0
    assert np.abs(oracle.apply_R(L, b, BC, U, C, v)[sel]).max() == 0
    assert np.abs(oracle.apply_R(L, b, BC, U, C, v)[~sel]).max() > 0


def test_bad_geometry_rejected(oracle):
    """Two-colour Schwarz needs an even number (>= 2) of domains per direction."""
    for L, b in [((4, 4, 4, 4), (4, 2, 2, 2)),      # one domain in x
                 ((4, 4, 4, 4), (3, 2, 2, 2)),      # extent does not divide
                 ((6, 4, 4, 4), (2, 2, 2, 2))]:     # three domains in x
        V = int(np.prod(L))
        U = inputs.unit_gauge(L)
        C = oracle.clover_field(L, U, 0.12, 1.0)
        psi = inputs.gaussian_spinor(V, 1)
        with pytest.raises(ValueError):
            oracle.apply_Dblock(L, b, BC, U, C, psi)


# ---------------------------------------------------------------------------
# Block solve: even-odd Schur complement + MR (Sec. II-D, Eq. 5)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("L,b,d,n_mr", [((4, 4, 4, 4), (2, 2, 2, 2), 5, 4), ((8, 4, 4, 4), (4, 2, 2, 2), 2, 5),
                                        ((4, 4, 4, 8), (2, 2, 2, 4), 9, 7)])
def test_blocksolve_dense(oracle, L, b, d, n_mr):
    """The oracle's block solve equals textbook MR on the dense Schur
    complement built from the dense domain block of D."""
    U = inputs.random_gauge(L, 0.6, 61)
    C = oracle.clover_field(L, U, 0.1365, 1.7)
    Ci = oracle.clover_inverse(C)
    V = U.shape[0]
    rho = inputs.gaussian_spinor(V, 62)
    delta, res = oracle.blocksolve(L, b, U, C, Ci, d, n_mr, rho)
    dom, _ = R.domain_ids(L, b)
    sites = np.where(dom == d)[0]
    dof = (sites[:, None] * 12 + np.arange(12)[None]).reshape(-1)

    def applyD(v):
        full = np.zeros(V * 12, dtype=np.complex128)
        full[dof] = v
        return oracle.apply_Dblock(L, b, BC, U, C, full.reshape(V, 4, 3)).reshape(-1)[dof]

    Ablk = R.dense_operator(applyD, len(dof))
    par = np.repeat(R.site_parity(L)[sites], 12)
    want_d, want_r = R.dense_block_solve(Ablk, par, rho.reshape(-1)[dof], n_mr)
    assert rel(delta.reshape(-1)[dof], want_d) < 1e-13
    assert rel(res.reshape(-1)[dof], want_r) < 1e-12
    # the block residual is rho - D delta exactly
    assert rel(rho.reshape(-1)[dof] - Ablk @ want_d, want_r) < 1e-12
    outside = np.setdiff1d(np.arange(V), sites)
    assert np.abs(delta[outside]).max() == 0


def test_mr_residual_monotone(oracle):
    """MR minimises the residual along r at each step, so the block residual
    norm never increases with the number of MR steps."""
    L = (4, 4, 4, 4)
    U = inputs.random_gauge(L, 0.6, 71)
    C = oracle.clover_field(L, U, 0.13, 1.7)
    Ci = oracle.clover_inverse(C)
    rho = inputs.gaussian_spinor(256, 72)
    norms = []
    for n in range(0, 7):
        _, res = oracle.blocksolve(L, (2, 2, 2, 2), U, C, Ci, 0, n, rho)
        norms.append(np.linalg.norm(res))
    assert all(norms[i + 1] <= norms[i] * (1 + 1e-14) for i in range(len(norms) - 1))
    assert norms[-1] < 0.5 * norms[1]


# ---------------------------------------------------------------------------
# SAP (multiplicative Schwarz, Sec. II-D and the algorithm of Table I)
# ---------------------------------------------------------------------------

def _dense_sap(L, b, Adense, Dblocks, eta, n_cycles, n_mr):
    """SAP written with dense matrices: for each cycle, black then white, every
    domain of the colour adds the dense block solve of (eta - A psi) on it."""
    V = Adense.shape[0] // 12
    dom, col = R.domain_ids(L, b)
    par = R.site_parity(L)
    psi = np.zeros(V * 12, dtype=np.complex128)
    for _ in range(n_cycles):
        for colour in (0, 1):
            res = eta - Adense @ psi
            upd = np.zeros_like(psi)
            for d in np.unique(dom[col == colour]):
                sites = np.where(dom == d)[0]
                dof = (sites[:, None] * 12 + np.arange(12)[None]).reshape(-1)
                delta, _ = R.dense_block_solve(Dblocks[d], np.repeat(par[sites], 12), res[dof], n_mr)
                upd[dof] = delta
            psi = psi + upd
    return psi


@pytest.fixture(scope="module")
def dense_4444(oracle):
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = inputs.random_gauge(L, 0.3, 101)
    kappa, csw = 0.12, 1.0
    C = oracle.clover_field(L, U, kappa, csw)
    Ci = oracle.clover_inverse(C)
    V = 256
    A = R.dense_operator(lambda v: oracle.apply_A(L, BC, U, C, v.reshape(V, 4, 3)), V * 12)
    Dfull = R.dense_operator(lambda v: oracle.apply_Dblock(L, b, BC, U, C, v.reshape(V, 4, 3)), V * 12)
    dom, _ = R.domain_ids(L, b)
    blocks = {}
    for d in np.unique(dom):
        sites = np.where(dom == d)[0]
        dof = (sites[:, None] * 12 + np.arange(12)[None]).reshape(-1)
        blocks[d] = Dfull[np.ix_(dof, dof)]
    return dict(L=L, b=b, U=U, C=C, Ci=Ci, A=A, blocks=blocks, kappa=kappa, csw=csw)


def test_sap_dense(oracle, dense_4444):
    g = dense_4444
    eta = inputs.gaussian_source(g["L"], 102)
    psi = oracle.sap(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], 3, 4, eta)
    want = _dense_sap(g["L"], g["b"], g["A"], g["blocks"], eta.reshape(-1), 3, 4)
    assert rel(psi.reshape(-1), want) < 1e-13


def test_sap_exact_blocks_is_block_gauss_seidel(oracle, dense_4444):
    """With converged block solves one SAP cycle is one block Gauss-Seidel
    sweep: psi_B = D_BB^-1 eta_B, psi_W = D_WW^-1 (eta_W - A_WB psi_B)."""
    g = dense_4444
    eta = inputs.gaussian_source(g["L"], 103).reshape(-1)
    psi = oracle.sap(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], 1, 60, eta.reshape(-1, 4, 3)).reshape(-1)
    dom, col = R.domain_ids(g["L"], g["b"])
    black = np.repeat(col == 0, 12)
    white = ~black
    A = g["A"]
    D_BB = A[np.ix_(black, black)] * 0
    # D_BB: block diagonal of the black domains (no couplings between different black domains)
    Bsites = np.where(black)[0]
    Wsites = np.where(white)[0]
    D_BB = np.zeros((len(Bsites), len(Bsites)), dtype=np.complex128)
    D_WW = np.zeros((len(Wsites), len(Wsites)), dtype=np.complex128)
    posB = {s: i for i, s in enumerate(Bsites)}
    posW = {s: i for i, s in enumerate(Wsites)}
    for d, blk in g["blocks"].items():
        sites = np.where(dom == d)[0]
        dof = (sites[:, None] * 12 + np.arange(12)[None]).reshape(-1)
        if col[sites[0]] == 0:
            ix = [posB[q] for q in dof]
            D_BB[np.ix_(ix, ix)] = blk
        else:
            ix = [posW[q] for q in dof]
            D_WW[np.ix_(ix, ix)] = blk
    want = np.zeros_like(eta)
    want[black] = np.linalg.solve(D_BB, eta[black])
    want[white] = np.linalg.solve(D_WW, eta[white] - A[np.ix_(white, black)] @ want[black])
    assert rel(psi, want) < 1e-12


def test_sap_additive_dense(oracle, dense_4444):
    """Additive Schwarz (Eq. 4) written with dense matrices: every cycle, all
    domains add the dense block solve of the same residual eta - A psi."""
    g = dense_4444
    eta = inputs.gaussian_source(g["L"], 106)
    psi = oracle.sap_additive(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], 3, 4, eta)
    dom, _ = R.domain_ids(g["L"], g["b"])
    par = R.site_parity(g["L"])
    want = np.zeros(eta.size, dtype=np.complex128)
    for _ in range(3):
        res = eta.reshape(-1) - g["A"] @ want
        upd = np.zeros_like(want)
        for d in np.unique(dom):
            sites = np.where(dom == d)[0]
            dof = (sites[:, None] * 12 + np.arange(12)[None]).reshape(-1)
            upd[dof], _ = R.dense_block_solve(g["blocks"][d], np.repeat(par[sites], 12), res[dof], 4)
        want = want + upd
    assert rel(psi.reshape(-1), want) < 1e-13
    # not the multiplicative method
    mult = oracle.sap(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], 3, 4, eta)
    assert rel(psi, mult) > 1e-3


def test_sap_additive_exact_blocks_is_block_jacobi(oracle, dense_4444):
    """With converged block solves, two additive cycles are two block Jacobi
    steps: psi_1 = D^-1 eta, psi_2 = psi_1 + D^-1 (eta - A psi_1), with D the
    block diagonal of A over all domains (solved by LAPACK)."""
    g = dense_4444
    eta = inputs.gaussian_source(g["L"], 107).reshape(-1)
    psi = oracle.sap_additive(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], 2, 60, eta.reshape(-1, 4, 3)).reshape(-1)
    dom, _ = R.domain_ids(g["L"], g["b"])
    A = g["A"]
    D = np.zeros_like(A)
    for d in np.unique(dom):
        sites = np.where(dom == d)[0]
        dof = (sites[:, None] * 12 + np.arange(12)[None]).reshape(-1)
        D[np.ix_(dof, dof)] = A[np.ix_(dof, dof)]
    p1 = np.linalg.solve(D, eta)
    p2 = p1 + np.linalg.solve(D, eta - A @ p1)
    assert rel(psi, p2) < 1e-12


def test_fgcr_additive_sap_dense_solve(oracle, dense_4444):
    g = dense_4444
    f = inputs.gaussian_source(g["L"], 108)
    x, st, steps, relres = oracle.fgcr(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], f, precond=True, n_cycles=8,
                                       n_mr=4, restart=16, tol=1e-12, additive=True)
    assert st == 0 and relres <= 1e-12
    assert rel(x.reshape(-1), np.linalg.solve(g["A"], f.reshape(-1))) < 1e-10


def test_sap_homogeneous(oracle, dense_4444):
    g = dense_4444
    eta = inputs.gaussian_source(g["L"], 104)
    s = 0.37 - 1.9j
    m1 = oracle.sap(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], 2, 4, eta)
    m2 = oracle.sap(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], 2, 4, s * eta)
    assert rel(m2, s * m1) < 1e-14


def test_sap_reduces_residual(oracle, dense_4444):
    g = dense_4444
    eta = inputs.gaussian_source(g["L"], 105).reshape(-1)
    r = [np.linalg.norm(eta - g["A"] @ oracle.sap(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], n, 4,
                                                  eta.reshape(-1, 4, 3)).reshape(-1)) for n in (1, 2, 4, 8)]
    assert r[0] < np.linalg.norm(eta) and all(r[i + 1] < r[i] for i in range(3))


# ---------------------------------------------------------------------------
# FGCR (outer solver) and the whole solve
# ---------------------------------------------------------------------------

def test_gcr_minimal_residual(oracle):
    """With M = 1, GCR's residual after k steps is GMRES(k)'s minimum of
    |f - A y| over the Krylov space span{f, Af, ..., A^{k-1} f}."""
    L = (2, 2, 2, 4)
    U = inputs.random_gauge(L, 0.5, 81)
    C = oracle.clover_field(L, U, 0.13, 1.5)
    V = 32
    f = inputs.gaussian_source(L, 82)
    _, st, steps, _, hist = oracle.fgcr(L, None, BC, U, C, None, f, precond=False, restart=12, tol=1e-300,
                                        max_cycles=1, history=True)
    A = R.dense_operator(lambda v: oracle.apply_A(L, BC, U, C, v.reshape(V, 4, 3)), V * 12)
    fv = f.reshape(-1)
    K = [fv]
    for k in range(1, 12):
        K.append(A @ K[-1])
    fn = np.linalg.norm(fv)
    for k in range(1, 11):
        Q, _ = np.linalg.qr(np.stack(K[:k], axis=1))
        y, *_ = np.linalg.lstsq(A @ Q, fv, rcond=None)
        want = np.linalg.norm(fv - A @ Q @ y) / fn
        assert abs(hist[k] - want) <= 1e-10 * max(want, 1e-3), k


@pytest.mark.slow
def test_fgcr_sap_dense_solve(oracle, dense_4444):
    """The 4^4 workload (2^4 domains, 8 cycles, 4 MR steps): the FGCR+SAP
    solution equals LAPACK's dense solve."""
    g = dense_4444
    f = inputs.gaussian_source(g["L"], 102)
    x, st, steps, relres = oracle.fgcr(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], f, precond=True, n_cycles=8,
                                       n_mr=4, restart=16, tol=1e-12)
    assert st == 0 and relres <= 1e-12
    want = np.linalg.solve(g["A"], f.reshape(-1))
    assert rel(x.reshape(-1), want) < 1e-10
    assert steps < 20


def test_gcr_unpreconditioned_dense_solve(oracle):
    L = (2, 2, 2, 2)
    U = inputs.random_gauge(L, 0.5, 91)
    C = oracle.clover_field(L, U, 0.12, 1.0)
    f = inputs.gaussian_source(L, 92)
    x, st, steps, relres = oracle.fgcr(L, None, BC, U, C, None, f, precond=False, restart=16, tol=1e-12,
                                       max_cycles=100)
    A = R.dense_operator(lambda v: oracle.apply_A(L, BC, U, C, v.reshape(16, 4, 3)), 192)
    assert st == 0
    assert rel(x.reshape(-1), np.linalg.solve(A, f.reshape(-1))) < 1e-10


def test_fgcr_zero_source_and_guess(oracle, dense_4444):
    g = dense_4444
    z = np.zeros((256, 4, 3), dtype=np.complex128)
    x, st, steps, relres = oracle.fgcr(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], z, n_cycles=2, n_mr=2)
    assert st == 0 and steps == 0 and np.abs(x).max() == 0
    f = inputs.gaussian_source(g["L"], 106)
    want = np.linalg.solve(g["A"], f.reshape(-1)).reshape(256, 4, 3)
    x, st, steps, relres = oracle.fgcr(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], f, n_cycles=2, n_mr=2,
                                       x0=want)
    assert st == 0 and steps == 0
    x, st, steps, relres = oracle.fgcr(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], f, n_cycles=2, n_mr=2,
                                       max_cycles=1, restart=1, tol=1e-10)
    assert st == 6 and steps == 1 and relres < 1


# ---------------------------------------------------------------------------
# flexible GMRES with deflated restarts (Sec. II-C)
# ---------------------------------------------------------------------------

def _hessenberg_like(rng, m, dense_block=0):
    """(m+1) x m: upper Hessenberg, or, after a deflated restart, with a dense
    (k+1) x k leading block."""
    H = np.triu(rng.standard_normal((m + 1, m)) + 1j * rng.standard_normal((m + 1, m)), -1)
    if dense_block:
        H[:dense_block + 1, :dense_block] = (rng.standard_normal((dense_block + 1, dense_block))
                                             + 1j * rng.standard_normal((dense_block + 1, dense_block)))
    return H


@pytest.mark.parametrize("m,k,dense", [(6, 1, 0), (8, 3, 0), (8, 4, 3), (16, 6, 0), (16, 6, 5)])
def test_harmonic_ritz_pairs(oracle, m, k, dense):
    """The oracle's harmonic Ritz pairs are those of the generalized problem
    (Hbar^H Hbar) g = theta H_m^H g (LAPACK through scipy): the k values of
    smallest magnitude, and the span of their vectors."""
    import scipy.linalg as sl
    H = _hessenberg_like(np.random.default_rng(m * 10 + k + dense), m, dense)
    th, P = oracle.harmonic_ritz(H, k)
    w, vr = sl.eig(H.conj().T @ H, H[:m].conj().T)
    o = np.argsort(np.abs(w))
    assert np.allclose(th, w[o[:k]], rtol=1e-10, atol=1e-12)
    assert np.allclose(P.conj().T @ P, np.eye(k), atol=1e-12)
    Q, _ = np.linalg.qr(vr[:, o[:k]])
    assert sl.subspace_angles(P, Q).max() < 1e-9
    # the defining property of each pair: Hbar^H (Hbar g - theta [g; 0]) = 0
    for q in range(k):
        g = vr[:, o[q]]
        assert np.linalg.norm(H.conj().T @ (H @ g - w[o[q]] * np.append(g, 0))) < 1e-9 * np.linalg.norm(H) ** 2


def _arnoldi(A, r, m):
    """m steps of Arnoldi (modified Gram-Schmidt): V (n x m+1), Hbar."""
    n = len(r)
    V = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    V[:, 0] = r / np.linalg.norm(r)
    for j in range(m):
        w = A @ V[:, j]
        for i in range(j + 1):
            H[i, j] = np.vdot(V[:, i], w)
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
    return V, H


@pytest.mark.parametrize("m,k", [(6, 2), (8, 3)])
def test_fgmres_dr_deflated_restart_space(oracle, m, k):
    """With M = 1: the first cycle is GMRES(m) (least squares over the Krylov
    space of f); the second cycle minimises |f - A x| over x_1 plus the span of
    the k harmonic Ritz vectors of the first cycle and the Krylov vectors
    r_1, A r_1, ..., A^{m-k-1} r_1 (GMRES-DR's search space), built here from
    dense numpy Arnoldi and scipy's generalized eigensolver."""
    import scipy.linalg as sl
    L = (2, 2, 2, 4)
    U = inputs.random_gauge(L, 0.5, 83)
    C = oracle.clover_field(L, U, 0.13, 1.5)
    V = 32
    f = inputs.gaussian_source(L, 84)
    A = R.dense_operator(lambda v: oracle.apply_A(L, BC, U, C, v.reshape(V, 4, 3)), V * 12)
    fv = f.reshape(-1)
    # cycle 1: GMRES(m) from x0 = 0
    Vb, H = _arnoldi(A, fv, m)
    c = np.zeros(m + 1, dtype=np.complex128)
    c[0] = np.linalg.norm(fv)
    y, *_ = np.linalg.lstsq(H, c, rcond=None)
    x1 = Vb[:, :m] @ y
    x, st, steps, _ = oracle.fgmres_dr(L, None, BC, U, C, None, f, m, k, precond=False, tol=1e-300, max_cycles=1)
    assert steps == m and rel(x.reshape(-1), x1) < 1e-11
    # cycle 2 over the deflated space
    w, vr = sl.eig(H.conj().T @ H, H[:m].conj().T)
    o = np.argsort(np.abs(w))
    Y = Vb[:, :m] @ vr[:, o[:k]]
    r1 = fv - A @ x1
    S = [Y[:, q] for q in range(k)] + [r1]
    for _ in range(m - k - 1):
        S.append(A @ S[-1])
    S, _ = np.linalg.qr(np.stack(S, axis=1))
    coef, *_ = np.linalg.lstsq(A @ S, r1, rcond=None)
    x2 = x1 + S @ coef
    x, st, steps, _ = oracle.fgmres_dr(L, None, BC, U, C, None, f, m, k, precond=False, tol=1e-300, max_cycles=2)
    assert steps == 2 * m - k
    assert rel(x.reshape(-1), x2) < 1e-9
    # without deflation the second cycle is plain restarted GMRES(m) instead
    x0d, _, _, _ = oracle.fgmres_dr(L, None, BC, U, C, None, f, m, 0, precond=False, tol=1e-300, max_cycles=2)
    assert rel(x0d.reshape(-1), x2) > 1e-6


def test_fgmres_dr_residual_estimates_are_gmres(oracle):
    """Within the first cycle, the residual estimate after step j is GMRES(j)'s
    minimum over the Krylov space (M = 1)."""
    L = (2, 2, 2, 4)
    U = inputs.random_gauge(L, 0.5, 85)
    C = oracle.clover_field(L, U, 0.13, 1.5)
    V = 32
    f = inputs.gaussian_source(L, 86)
    _, st, steps, _, hist = oracle.fgmres_dr(L, None, BC, U, C, None, f, 12, 4, precond=False, tol=1e-300,
                                             max_cycles=1, history=True)
    A = R.dense_operator(lambda v: oracle.apply_A(L, BC, U, C, v.reshape(V, 4, 3)), V * 12)
    fv = f.reshape(-1)
    K = [fv]
    for _ in range(1, 12):
        K.append(A @ K[-1])
    fn = np.linalg.norm(fv)
    for j in range(1, 12):
        Q, _ = np.linalg.qr(np.stack(K[:j], axis=1))
        y, *_ = np.linalg.lstsq(A @ Q, fv, rcond=None)
        want = np.linalg.norm(fv - A @ Q @ y) / fn
        assert abs(hist[j] - want) <= 1e-10 * max(want, 1e-3), j


@pytest.mark.slow
@pytest.mark.parametrize("m,k", [(8, 4), (16, 6)])
def test_fgmres_dr_sap_dense_solve(oracle, dense_4444, m, k):
    """FGMRES-DR with the SAP preconditioner (the paper's basis and deflation
    sizes, Sec. IV-C) reaches LAPACK's dense solution."""
    g = dense_4444
    f = inputs.gaussian_source(g["L"], 107)
    x, st, steps, relres = oracle.fgmres_dr(g["L"], g["b"], BC, g["U"], g["C"], g["Ci"], f, m, k, n_cycles=8,
                                            n_mr=4, tol=1e-12)
    assert st == 0 and relres <= 1e-12
    assert rel(x.reshape(-1), np.linalg.solve(g["A"], f.reshape(-1))) < 1e-10


def test_fgmres_dr_unpreconditioned_restarts_dense_solve(oracle):
    """Many deflated restarts (M = 1, basis 6, 3 deflation vectors) still reach
    the dense solution; the zero source and an exact guess take no step."""
    L = (2, 2, 2, 2)
    U = inputs.random_gauge(L, 0.5, 93)
    C = oracle.clover_field(L, U, 0.12, 1.0)
    f = inputs.gaussian_source(L, 94)
    A = R.dense_operator(lambda v: oracle.apply_A(L, BC, U, C, v.reshape(16, 4, 3)), 192)
    want = np.linalg.solve(A, f.reshape(-1))
    x, st, steps, relres = oracle.fgmres_dr(L, None, BC, U, C, None, f, 6, 3, precond=False, tol=1e-12,
                                            max_cycles=200)
    assert st == 0 and rel(x.reshape(-1), want) < 1e-10
    x0, st0, steps0, _ = oracle.fgmres_dr(L, None, BC, U, C, None, np.zeros_like(f), 6, 3, precond=False)
    assert st0 == 0 and steps0 == 0 and not np.any(x0)
    xg, stg, stepsg, _ = oracle.fgmres_dr(L, None, BC, U, C, None, f, 6, 3, precond=False,
                                          x0=want.reshape(16, 4, 3))
    assert stg == 0 and stepsg == 0
