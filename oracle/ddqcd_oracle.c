/*
 * FP64 CPU oracle for the SAP-preconditioned flexible GCR solve of the
 * Wilson-clover Dirac equation (Heybrock et al., SC14, arXiv:1412.2629).
 *
 * TEST INFRASTRUCTURE.  This file is the plain, slow, obviously correct
 * statement of what the GPU path computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * library never calls it and shares no code, header or table with it.
 *
 * Everything is double precision complex, lexicographic site loops, dense
 * 12x12 site matrices and explicit 4x4 gamma matrices: no half-spinor
 * tricks, no packing, no blocking.
 *
 * Conventions (the readings of the paper that this oracle fixes):
 *  - site i = x + Lx*(y + Ly*(z + Lz*t)); mu = 0,1,2,3 <-> x,y,z,t.
 *  - gauge U[site][mu][row][col]; spinor psi[site][spin][colour].
 *  - A = (4+m) - D_w/2 + D_cl (Sec. II-B, Eq. 1) with 4+m = 1/(2 kappa).
 *  - D_w as in Sec. II-B Eq. 2: forward hop (1-gamma_mu) U_mu(x) psi(x+mu),
 *    backward hop (1+gamma_mu) U_mu(x-mu)^dagger psi(x-mu).  A hop that wraps
 *    around the lattice in direction mu is multiplied by bc[mu] (+1 or -1).
 *  - gamma matrices in the chiral basis: gamma_k = [[0,-i s_k],[i s_k,0]]
 *    (s_k Pauli), gamma_t = [[0,-1],[-1,0]]; sigma_munu = (i/2)[g_mu,g_nu].
 *    In this basis the clover term is block diagonal in spins {0,1} and
 *    {2,3}, the two Hermitian 6x6 blocks of Sec. II-B.
 *  - clover (Sec. II-B Eq. 3): D_cl = c_sw sum_{mu != nu} (i/8) sigma_munu F_munu
 *    with F_munu = (Q_munu - Q_munu^dagger)/4 and Q_munu the sum of the four
 *    plaquette leaves at x in the (mu,nu) plane, each oriented mu -> nu.
 *    No traceless projection; leaves use the bare links.
 *
 * Parity pins live in tests/ (free-field momentum-space closed form,
 * gamma5-hermiticity, gauge covariance, constant-field clover closed form,
 * D + R = A, dense block solves, dense SAP (multiplicative and additive),
 * dense LU solve, GMRES minimal residual).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_GEOMETRY = 2, OR_ERR_NOMEM = 5, OR_ERR_NOT_CONVERGED = 6 };

/* ------------------------------------------------------------------ */
/* gamma matrices                                                     */
/* ------------------------------------------------------------------ */

static cplx GAMMA[4][4][4];
static int gamma_ready = 0;

static void build_gamma(void)
{
    if (gamma_ready) return;
    cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAMMA, 0, sizeof(GAMMA));
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                GAMMA[k][a][2 + b] = -I * pauli[k][a][b];
                GAMMA[k][2 + a][b] = I * pauli[k][a][b];
            }
    for (int a = 0; a < 2; a++) {
        GAMMA[3][a][2 + a] = -1;
        GAMMA[3][2 + a][a] = -1;
    }
    gamma_ready = 1;
}

/* ------------------------------------------------------------------ */
/* geometry                                                           */
/* ------------------------------------------------------------------ */

static long volume(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static long site_index(const int L[4], const int x[4])
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

static void site_coords(const int L[4], long i, int x[4])
{
    x[0] = (int)(i % L[0]); i /= L[0];
    x[1] = (int)(i % L[1]); i /= L[1];
    x[2] = (int)(i % L[2]); i /= L[2];
    x[3] = (int)i;
}

/* neighbour of site i one step (+1/-1) in direction mu; *wrap = 1 if the step
   crosses the lattice edge */
static long neighbour(const int L[4], long i, int mu, int step, int *wrap)
{
    int x[4];
    site_coords(L, i, x);
    x[mu] += step;
    *wrap = 0;
    if (x[mu] >= L[mu]) { x[mu] -= L[mu]; *wrap = 1; }
    if (x[mu] < 0) { x[mu] += L[mu]; *wrap = 1; }
    return site_index(L, x);
}

static int parity_of(const int L[4], long i)
{
    int x[4];
    site_coords(L, i, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* the domain grid: domain extents b divide L; domain coordinates X = x / b */
static int check_domains(const int L[4], const int b[4])
{
    for (int mu = 0; mu < 4; mu++) {
        if (b[mu] < 1 || L[mu] % b[mu] != 0) return OR_ERR_GEOMETRY;
        int n = L[mu] / b[mu];
        if (n < 2 || (n & 1)) return OR_ERR_GEOMETRY;
    }
    return OR_OK;
}

static long domain_of(const int L[4], const int b[4], long i)
{
    int x[4];
    site_coords(L, i, x);
    int n[4] = {L[0] / b[0], L[1] / b[1], L[2] / b[2], L[3] / b[3]};
    return x[0] / b[0] + (long)n[0] * (x[1] / b[1] + (long)n[1] * (x[2] / b[2] + (long)n[2] * (x[3] / b[3])));
}

/* colour of domain d: parity of the sum of its domain coordinates (black = 0) */
static int domain_colour(const int L[4], const int b[4], long d)
{
    int n[4] = {L[0] / b[0], L[1] / b[1], L[2] / b[2], L[3] / b[3]};
    int X0 = (int)(d % n[0]); d /= n[0];
    int X1 = (int)(d % n[1]); d /= n[1];
    int X2 = (int)(d % n[2]); d /= n[2];
    int X3 = (int)d;
    return (X0 + X1 + X2 + X3) & 1;
}

/* list the global sites of domain d in lexicographic order of the local
   coordinates; returns the number of sites */
static long domain_sites(const int L[4], const int b[4], long d, long *sites)
{
    int n[4] = {L[0] / b[0], L[1] / b[1], L[2] / b[2], L[3] / b[3]};
    int X[4];
    X[0] = (int)(d % n[0]); d /= n[0];
    X[1] = (int)(d % n[1]); d /= n[1];
    X[2] = (int)(d % n[2]); d /= n[2];
    X[3] = (int)d;
    long k = 0;
    int l[4], x[4];
    for (l[3] = 0; l[3] < b[3]; l[3]++)
        for (l[2] = 0; l[2] < b[2]; l[2]++)
            for (l[1] = 0; l[1] < b[1]; l[1]++)
                for (l[0] = 0; l[0] < b[0]; l[0]++) {
                    for (int mu = 0; mu < 4; mu++) x[mu] = X[mu] * b[mu] + l[mu];
                    sites[k++] = site_index(L, x);
                }
    return k;
}

/* ------------------------------------------------------------------ */
/* 3x3 colour algebra                                                 */
/* ------------------------------------------------------------------ */

static void m3_mul(cplx out[9], const cplx a[9], const cplx b[9])
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[i * 3 + k] * b[k * 3 + j];
            t[i * 3 + j] = s;
        }
    memcpy(out, t, sizeof(t));
}

static void m3_dag(cplx out[9], const cplx a[9])
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[i * 3 + j] = conj(a[j * 3 + i]);
    memcpy(out, t, sizeof(t));
}

static const cplx *link(const cplx *U, long i, int mu) { return U + ((size_t)i * 4 + mu) * 9; }

/* ------------------------------------------------------------------ */
/* the hopping term of one direction                                  */
/* ------------------------------------------------------------------ */

/* out += coef * (1 - sgn*gamma_mu) (W v), with W = U (dagger = 0) or
   W = U^dagger (dagger = 1) acting on colour, for a 12-component v */
static void add_hop(cplx out[12], const cplx *Ul, int dagger, int mu, double sgn, cplx coef, const cplx *v)
{
    cplx w[12];
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++) {
            cplx acc = 0;
            for (int c = 0; c < 3; c++) {
                cplx Wac = dagger ? conj(Ul[c * 3 + a]) : Ul[a * 3 + c];
                acc += Wac * v[s * 3 + c];
            }
            w[s * 3 + a] = acc;
        }
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++) {
            cplx acc = w[s * 3 + a];
            for (int t = 0; t < 4; t++) acc -= sgn * GAMMA[mu][s][t] * w[t * 3 + a];
            out[s * 3 + a] += coef * acc;
        }
}

/* ------------------------------------------------------------------ */
/* clover term (Sec. II-B, Eq. 3)                                     */
/* ------------------------------------------------------------------ */

/* Q_munu(x): sum of the four plaquette leaves at x in the (mu,nu) plane */
static void clover_leaves(const int L[4], const cplx *U, long x, int mu, int nu, cplx Q[9])
{
    int w;
    long xpm = neighbour(L, x, mu, +1, &w);
    long xmm = neighbour(L, x, mu, -1, &w);
    long xpn = neighbour(L, x, nu, +1, &w);
    long xmn = neighbour(L, x, nu, -1, &w);
    long xpn_mm = neighbour(L, xpn, mu, -1, &w);   /* x + nu - mu */
    long xmm_mn = neighbour(L, xmm, nu, -1, &w);   /* x - mu - nu */
    long xmn_pm = neighbour(L, xmn, mu, +1, &w);   /* x - nu + mu */
    cplx d[9], leaf[9];
    memset(Q, 0, 9 * sizeof(cplx));

    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
    m3_mul(leaf, link(U, x, mu), link(U, xpm, nu));
    m3_dag(d, link(U, xpn, mu)); m3_mul(leaf, leaf, d);
    m3_dag(d, link(U, x, nu)); m3_mul(leaf, leaf, d);
    for (int k = 0; k < 9; k++) Q[k] += leaf[k];

    /* U_nu(x) U_mu(x+nu-mu)^dag U_nu(x-mu)^dag U_mu(x-mu) */
    m3_dag(d, link(U, xpn_mm, mu)); m3_mul(leaf, link(U, x, nu), d);
    m3_dag(d, link(U, xmm, nu)); m3_mul(leaf, leaf, d);
    m3_mul(leaf, leaf, link(U, xmm, mu));
    for (int k = 0; k < 9; k++) Q[k] += leaf[k];

    /* U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu) */
    m3_dag(leaf, link(U, xmm, mu));
    m3_dag(d, link(U, xmm_mn, nu)); m3_mul(leaf, leaf, d);
    m3_mul(leaf, leaf, link(U, xmm_mn, mu));
    m3_mul(leaf, leaf, link(U, xmn, nu));
    for (int k = 0; k < 9; k++) Q[k] += leaf[k];

    /* U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag */
    m3_dag(leaf, link(U, xmn, nu));
    m3_mul(leaf, leaf, link(U, xmn, mu));
    m3_mul(leaf, leaf, link(U, xmn_pm, nu));
    m3_dag(d, link(U, x, mu)); m3_mul(leaf, leaf, d);
    for (int k = 0; k < 9; k++) Q[k] += leaf[k];
}

/* dense 12x12 site matrix C(x) = (1/(2 kappa)) 1 + D_cl(x); index (s*3+a, t*3+b) */
void oracle_clover_site(const int L[4], const cplx *U, double kappa, double csw, long x, cplx *C)
{
    build_gamma();
    memset(C, 0, 144 * sizeof(cplx));
    for (int k = 0; k < 12; k++) C[k * 12 + k] = 1.0 / (2.0 * kappa);
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++) {
            if (mu == nu) continue;
            cplx Q[9], F[9], sig[4][4];
            clover_leaves(L, U, x, mu, nu, Q);
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) F[a * 3 + b] = (Q[a * 3 + b] - conj(Q[b * 3 + a])) / 4.0;
            for (int s = 0; s < 4; s++)
                for (int t = 0; t < 4; t++) {
                    cplx gg = 0;
                    for (int r = 0; r < 4; r++)
                        gg += GAMMA[mu][s][r] * GAMMA[nu][r][t] - GAMMA[nu][s][r] * GAMMA[mu][r][t];
                    sig[s][t] = 0.5 * I * gg;
                }
            for (int s = 0; s < 4; s++)
                for (int t = 0; t < 4; t++)
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            C[(s * 3 + a) * 12 + t * 3 + b] += csw * (I / 8.0) * sig[s][t] * F[a * 3 + b];
        }
}

void oracle_clover_field(const int L[4], const cplx *U, double kappa, double csw, cplx *C)
{
    long V = volume(L);
    build_gamma();
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++) oracle_clover_site(L, U, kappa, csw, x, C + (size_t)x * 144);
}

/* inverse of a dense 12x12 complex matrix, Gauss-Jordan with partial pivoting */
static int inv12(const cplx *A, cplx *Ainv)
{
    cplx M[12][24];
    for (int i = 0; i < 12; i++)
        for (int j = 0; j < 24; j++) M[i][j] = j < 12 ? A[i * 12 + j] : (j - 12 == i ? 1 : 0);
    for (int c = 0; c < 12; c++) {
        int p = c;
        for (int r = c + 1; r < 12; r++)
            if (cabs(M[r][c]) > cabs(M[p][c])) p = r;
        if (cabs(M[p][c]) == 0) return OR_ERR_ARG;
        if (p != c)
            for (int j = 0; j < 24; j++) { cplx t = M[c][j]; M[c][j] = M[p][j]; M[p][j] = t; }
        cplx piv = M[c][c];
        for (int j = 0; j < 24; j++) M[c][j] /= piv;
        for (int r = 0; r < 12; r++) {
            if (r == c) continue;
            cplx f = M[r][c];
            if (f != 0)
                for (int j = 0; j < 24; j++) M[r][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < 12; i++)
        for (int j = 0; j < 12; j++) Ainv[i * 12 + j] = M[i][12 + j];
    return OR_OK;
}

int oracle_clover_inverse_field(long V, const cplx *C, cplx *Cinv)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long x = 0; x < V; x++) bad |= inv12(C + (size_t)x * 144, Cinv + (size_t)x * 144) != OR_OK;
    return bad ? OR_ERR_ARG : OR_OK;
}

static void mat12_vec(cplx out[12], const cplx *M, const cplx *v)
{
    for (int i = 0; i < 12; i++) {
        cplx s = 0;
        for (int j = 0; j < 12; j++) s += M[i * 12 + j] * v[j];
        out[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* the operator A (Sec. II-B, Eqs. 1-2)                               */
/* ------------------------------------------------------------------ */

static void apply_A_site(const int L[4], const double bc[4], const cplx *U, const cplx *Cx, const cplx *in, long x,
                         cplx out[12])
{
    mat12_vec(out, Cx, in + (size_t)x * 12);
    for (int mu = 0; mu < 4; mu++) {
        int w;
        long y = neighbour(L, x, mu, +1, &w);
        add_hop(out, link(U, x, mu), 0, mu, +1.0, -0.5 * (w ? bc[mu] : 1.0), in + (size_t)y * 12);
        y = neighbour(L, x, mu, -1, &w);
        add_hop(out, link(U, y, mu), 1, mu, -1.0, -0.5 * (w ? bc[mu] : 1.0), in + (size_t)y * 12);
    }
}

void oracle_apply_A(const int L[4], const double bc[4], const cplx *U, const cplx *C, const cplx *in, cplx *out)
{
    long V = volume(L);
    build_gamma();
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++) apply_A_site(L, bc, U, C + (size_t)x * 144, in, x, out + (size_t)x * 12);
}

/* (A psi)(x) at a list of sites, building the clover matrix of each site on
   the fly (no full clover field needed) */
void oracle_apply_A_sites(const int L[4], const double bc[4], const cplx *U, double kappa, double csw,
                          const cplx *in, long nsites, const long *sites, cplx *out)
{
    build_gamma();
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < nsites; k++) {
        cplx Cx[144];
        oracle_clover_site(L, U, kappa, csw, sites[k], Cx);
        apply_A_site(L, bc, U, Cx, in, sites[k], out + (size_t)k * 12);
    }
}

/* ------------------------------------------------------------------ */
/* the split A = D + R (Sec. II-D)                                    */
/* ------------------------------------------------------------------ */

/* which = 0: D (site term + hops with both ends in one domain);
   which = 1: R (hops between domains, with boundary phases) */
static void apply_split(const int L[4], const int b[4], const double bc[4], const cplx *U, const cplx *C,
                        const cplx *in, cplx *out, int which)
{
    long V = volume(L);
    build_gamma();
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++) {
        cplx acc[12];
        long dx = domain_of(L, b, x);
        if (which == 0) mat12_vec(acc, C + (size_t)x * 144, in + (size_t)x * 12);
        else memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; mu++) {
            int w;
            long y = neighbour(L, x, mu, +1, &w);
            if ((domain_of(L, b, y) == dx) == (which == 0))
                add_hop(acc, link(U, x, mu), 0, mu, +1.0, -0.5 * (w ? bc[mu] : 1.0), in + (size_t)y * 12);
            y = neighbour(L, x, mu, -1, &w);
            if ((domain_of(L, b, y) == dx) == (which == 0))
                add_hop(acc, link(U, y, mu), 1, mu, -1.0, -0.5 * (w ? bc[mu] : 1.0), in + (size_t)y * 12);
        }
        memcpy(out + (size_t)x * 12, acc, sizeof(acc));
    }
}

int oracle_apply_Dblock(const int L[4], const int b[4], const double bc[4], const cplx *U, const cplx *C,
                        const cplx *in, cplx *out)
{
    int e = check_domains(L, b);
    if (e) return e;
    apply_split(L, b, bc, U, C, in, out, 0);
    return OR_OK;
}

int oracle_apply_R(const int L[4], const int b[4], const double bc[4], const cplx *U, const cplx *C,
                   const cplx *in, cplx *out)
{
    int e = check_domains(L, b);
    if (e) return e;
    apply_split(L, b, bc, U, C, in, out, 1);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* block solve on one domain: even-odd Schur complement + MR          */
/* (Sec. II-D, Eq. 5 and the MR iteration)                            */
/* ------------------------------------------------------------------ */

typedef struct {
    const int *L, *b;
    const cplx *U, *C, *Cinv;
    long n;          /* sites in the domain */
    long *site;      /* global index of local site k (lexicographic in the domain) */
    int *par;        /* global parity of local site k */
    long *nbr;       /* [k][mu][dir]: local index of the neighbour, or -1 outside */
} dom_t;

static int dom_init(dom_t *D, const int L[4], const int b[4], const cplx *U, const cplx *C, const cplx *Cinv, long d)
{
    D->L = L; D->b = b; D->U = U; D->C = C; D->Cinv = Cinv;
    D->site = NULL; D->par = NULL; D->nbr = NULL;
    D->n = (long)b[0] * b[1] * b[2] * b[3];
    D->site = malloc(D->n * sizeof(long));
    D->par = malloc(D->n * sizeof(int));
    D->nbr = malloc(D->n * 8 * sizeof(long));
    if (!D->site || !D->par || !D->nbr) return OR_ERR_NOMEM;
    domain_sites(L, b, d, D->site);
    for (long k = 0; k < D->n; k++) {
        D->par[k] = parity_of(L, D->site[k]);
        int l[4];
        long r = k;
        l[0] = (int)(r % b[0]); r /= b[0];
        l[1] = (int)(r % b[1]); r /= b[1];
        l[2] = (int)(r % b[2]); r /= b[2];
        l[3] = (int)r;
        for (int mu = 0; mu < 4; mu++)
            for (int dir = 0; dir < 2; dir++) {
                int m[4] = {l[0], l[1], l[2], l[3]};
                m[mu] += dir == 0 ? +1 : -1;
                long idx = -1;
                if (m[mu] >= 0 && m[mu] < b[mu])
                    idx = m[0] + (long)b[0] * (m[1] + (long)b[1] * (m[2] + (long)b[2] * m[3]));
                D->nbr[(k * 4 + mu) * 2 + dir] = idx;
            }
    }
    return OR_OK;
}

static void dom_free(dom_t *D)
{
    free(D->site); free(D->par); free(D->nbr);
}

/* out(k) = sum of the in-domain hopping terms -1/2 (1 -+ gamma) W v(nbr) at every
   local site k of parity `target` (zero elsewhere); v is a local field.  Hops
   inside a domain never wrap the lattice (at least two domains per direction),
   so no boundary phase enters. */
static void dom_hops(const dom_t *D, int target, const cplx *v, cplx *out)
{
    memset(out, 0, D->n * 12 * sizeof(cplx));
    for (long k = 0; k < D->n; k++) {
        if (D->par[k] != target) continue;
        for (int mu = 0; mu < 4; mu++) {
            long f = D->nbr[(k * 4 + mu) * 2 + 0];
            long bk = D->nbr[(k * 4 + mu) * 2 + 1];
            if (f >= 0) add_hop(out + k * 12, link(D->U, D->site[k], mu), 0, mu, +1.0, -0.5, v + f * 12);
            if (bk >= 0) add_hop(out + k * 12, link(D->U, D->site[bk], mu), 1, mu, -1.0, -0.5, v + bk * 12);
        }
    }
}

/* out(k) = M(site k) v(k) at sites of parity `target` (M = C or C^-1), zero elsewhere */
static void dom_site_mat(const dom_t *D, const cplx *M, int target, const cplx *v, cplx *out)
{
    for (long k = 0; k < D->n; k++) {
        if (D->par[k] == target) mat12_vec(out + k * 12, M + (size_t)D->site[k] * 144, v + k * 12);
        else memset(out + k * 12, 0, 12 * sizeof(cplx));
    }
}

static cplx dom_dot(const dom_t *D, int target, const cplx *a, const cplx *b)
{
    cplx s = 0;
    for (long k = 0; k < D->n; k++)
        if (D->par[k] == target)
            for (int c = 0; c < 12; c++) s += conj(a[k * 12 + c]) * b[k * 12 + c];
    return s;
}

/* approximate solution of D_Omega delta = rho on one domain:
   rho_e~ = rho_e - D_eo C_o^-1 rho_o; MR on Dt_ee = C_e - D_eo C_o^-1 D_oe from
   x = 0 for n_mr steps; delta_e = x; delta_o = C_o^-1 (rho_o - D_oe x).
   rho, delta, res: local fields (n x 12); res receives the block residual
   rho - D_Omega delta (the MR residual on even sites, zero on odd sites). */
static void dom_blocksolve(const dom_t *D, int n_mr, const cplx *rho, cplx *delta, cplx *res)
{
    const int E = 0, O = 1;
    long n = D->n;
    cplx *t1 = calloc(n * 12, sizeof(cplx)), *t2 = calloc(n * 12, sizeof(cplx));
    cplx *x = calloc(n * 12, sizeof(cplx)), *r = calloc(n * 12, sizeof(cplx)), *p = calloc(n * 12, sizeof(cplx));

    /* rho_e~ */
    dom_site_mat(D, D->Cinv, O, rho, t1);           /* C_o^-1 rho_o          */
    dom_hops(D, E, t1, t2);                          /* D_eo C_o^-1 rho_o     */
    for (long k = 0; k < n; k++)
        for (int c = 0; c < 12; c++)
            r[k * 12 + c] = D->par[k] == E ? rho[k * 12 + c] - t2[k * 12 + c] : 0;

    /* minimal residual on the Schur complement */
    for (int it = 0; it < n_mr; it++) {
        dom_hops(D, O, r, t1);                       /* D_oe r                */
        dom_site_mat(D, D->Cinv, O, t1, t2);         /* C_o^-1 D_oe r         */
        dom_hops(D, E, t2, t1);                      /* D_eo C_o^-1 D_oe r    */
        dom_site_mat(D, D->C, E, r, p);              /* C_e r                 */
        for (long k = 0; k < n * 12; k++) p[k] -= t1[k];
        cplx pr = dom_dot(D, E, p, r);
        double pp = creal(dom_dot(D, E, p, p));
        cplx alpha = pp > 0 ? pr / pp : 0;
        for (long k = 0; k < n * 12; k++) {
            x[k] += alpha * r[k];
            r[k] -= alpha * p[k];
        }
    }

    /* odd sites */
    dom_hops(D, O, x, t1);                           /* D_oe x                */
    for (long k = 0; k < n * 12; k++) t2[k] = rho[k] - t1[k];
    dom_site_mat(D, D->Cinv, O, t2, t1);             /* C_o^-1 (rho_o - D_oe x) */
    for (long k = 0; k < n; k++)
        for (int c = 0; c < 12; c++) {
            delta[k * 12 + c] = D->par[k] == E ? x[k * 12 + c] : t1[k * 12 + c];
            if (res) res[k * 12 + c] = D->par[k] == E ? r[k * 12 + c] : 0;
        }
    free(t1); free(t2); free(x); free(r); free(p);
}

/* block solve of domain d with rho and delta given as full lattice fields;
   only the sites of domain d are read and written */
int oracle_blocksolve(const int L[4], const int b[4], const cplx *U, const cplx *C, const cplx *Cinv, long d,
                      int n_mr, const cplx *rho, cplx *delta, cplx *blockres)
{
    int e = check_domains(L, b);
    if (e) return e;
    build_gamma();
    dom_t D;
    if (dom_init(&D, L, b, U, C, Cinv, d)) { dom_free(&D); return OR_ERR_NOMEM; }
    cplx *rl = malloc(D.n * 12 * sizeof(cplx)), *dl = malloc(D.n * 12 * sizeof(cplx)), *bl = malloc(D.n * 12 * sizeof(cplx));
    for (long k = 0; k < D.n; k++) memcpy(rl + k * 12, rho + (size_t)D.site[k] * 12, 12 * sizeof(cplx));
    dom_blocksolve(&D, n_mr, rl, dl, bl);
    for (long k = 0; k < D.n; k++) {
        memcpy(delta + (size_t)D.site[k] * 12, dl + k * 12, 12 * sizeof(cplx));
        if (blockres) memcpy(blockres + (size_t)D.site[k] * 12, bl + k * 12, 12 * sizeof(cplx));
    }
    free(rl); free(dl); free(bl);
    dom_free(&D);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Schwarz alternating procedure (multiplicative Schwarz, Sec. II-D)  */
/* ------------------------------------------------------------------ */

/* psi = M eta: psi = 0; for each of n_cycles cycles, for colour black then
   white, every domain of that colour adds its block solve of the current
   residual (eta - A psi) restricted to the domain. */
int oracle_sap(const int L[4], const int b[4], const double bc[4], const cplx *U, const cplx *C, const cplx *Cinv,
               int n_cycles, int n_mr, const cplx *eta, cplx *psi)
{
    int e = check_domains(L, b);
    if (e) return e;
    build_gamma();
    long V = volume(L);
    long nd = V / ((long)b[0] * b[1] * b[2] * b[3]);
    cplx *res = malloc((size_t)V * 12 * sizeof(cplx));
    if (!res) return OR_ERR_NOMEM;
    memset(psi, 0, (size_t)V * 12 * sizeof(cplx));
    int fail = 0;
    for (int s = 0; s < n_cycles; s++)
        for (int colour = 0; colour < 2; colour++) {
            oracle_apply_A(L, bc, U, C, psi, res);
            for (long k = 0; k < V * 12; k++) res[k] = eta[k] - res[k];
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
            for (long d = 0; d < nd; d++) {
                if (domain_colour(L, b, d) != colour) continue;
                dom_t D;
                if (dom_init(&D, L, b, U, C, Cinv, d)) { dom_free(&D); fail |= 1; continue; }
                cplx *rl = malloc(D.n * 12 * sizeof(cplx)), *dl = malloc(D.n * 12 * sizeof(cplx));
                for (long k = 0; k < D.n; k++) memcpy(rl + k * 12, res + (size_t)D.site[k] * 12, 12 * sizeof(cplx));
                dom_blocksolve(&D, n_mr, rl, dl, NULL);
                for (long k = 0; k < D.n; k++)
                    for (int c = 0; c < 12; c++) psi[(size_t)D.site[k] * 12 + c] += dl[k * 12 + c];
                free(rl); free(dl);
                dom_free(&D);
            }
        }
    free(res);
    return fail ? OR_ERR_NOMEM : OR_OK;
}

/* Additive Schwarz (Sec. II-D, Eq. 4): every cycle, all domains solve
 * their block of the same residual eta - A psi, and the corrections are
 * summed.  No colouring; psi starts at zero. */
int oracle_sap_additive(const int L[4], const int b[4], const double bc[4], const cplx *U, const cplx *C,
                        const cplx *Cinv, int n_cycles, int n_mr, const cplx *eta, cplx *psi)
{
    int e = check_domains(L, b);
    if (e) return e;
    build_gamma();
    long V = volume(L);
    long nd = V / ((long)b[0] * b[1] * b[2] * b[3]);
    cplx *res = malloc((size_t)V * 12 * sizeof(cplx));
    if (!res) return OR_ERR_NOMEM;
    memset(psi, 0, (size_t)V * 12 * sizeof(cplx));
    int fail = 0;
    for (int s = 0; s < n_cycles; s++) {
        oracle_apply_A(L, bc, U, C, psi, res);
        for (long k = 0; k < V * 12; k++) res[k] = eta[k] - res[k];
        /* domains are disjoint: each adds only to its own sites */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
        for (long d = 0; d < nd; d++) {
            dom_t D;
            if (dom_init(&D, L, b, U, C, Cinv, d)) { dom_free(&D); fail |= 1; continue; }
            cplx *rl = malloc(D.n * 12 * sizeof(cplx)), *dl = malloc(D.n * 12 * sizeof(cplx));
            for (long k = 0; k < D.n; k++) memcpy(rl + k * 12, res + (size_t)D.site[k] * 12, 12 * sizeof(cplx));
            dom_blocksolve(&D, n_mr, rl, dl, NULL);
            for (long k = 0; k < D.n; k++)
                for (int c = 0; c < 12; c++) psi[(size_t)D.site[k] * 12 + c] += dl[k * 12 + c];
            free(rl); free(dl);
            dom_free(&D);
        }
    }
    free(res);
    return fail ? OR_ERR_NOMEM : OR_OK;
}

/* ------------------------------------------------------------------ */
/* flexible GCR (outer solver, right preconditioning, Sec. II-C)      */
/* ------------------------------------------------------------------ */

static cplx vdot(long n, const cplx *a, const cplx *b)
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long k = 0; k < n; k++) {
        cplx t = conj(a[k]) * b[k];
        re += creal(t);
        im += cimag(t);
    }
    return re + I * im;
}

static double vnorm(long n, const cplx *a) { return sqrt(creal(vdot(n, a, a))); }

/* Solves A x = f.  precond = 0: M = 1 (plain GCR); precond = 1: M = SAP with
   the given domains, n_cycles and n_mr.  Each cycle takes up to `restart`
   steps z_k = M r, w = A z_k, modified Gram-Schmidt of w against the earlier
   w-hat, r -= <w-hat_k, r> w-hat_k; then back-substitution for the
   coefficients, x += sum alpha_k z_k and the true residual r = f - A x.
   Stops when |r| <= tol |f| (true residual) or after max_cycles cycles.
   x holds the initial guess on entry if x_is_guess, else starts at zero.
   history (optional, length max_cycles*restart+1) receives |r|/|f| after
   every step (recursive residual inside a cycle, true residual at a restart). */
int oracle_fgcr(const int L[4], const int b[4], const double bc[4], const cplx *U, const cplx *C, const cplx *Cinv,
                int precond, int n_cycles, int n_mr, int restart, double tol, int max_cycles, const cplx *f, cplx *x,
                int x_is_guess, int *n_steps, double *relres, double *history)
{
    if (restart < 1 || max_cycles < 1 || !(tol > 0)) return OR_ERR_ARG;
    if (precond) {
        int e = check_domains(L, b);
        if (e) return e;
    }
    build_gamma();
    long V = volume(L), n = V * 12;
    cplx *r = malloc(n * sizeof(cplx)), *w = malloc(n * sizeof(cplx));
    cplx **z = malloc(restart * sizeof(cplx *)), **wh = malloc(restart * sizeof(cplx *));
    cplx *a = calloc((size_t)restart * restart, sizeof(cplx)), *c = calloc(restart, sizeof(cplx)),
         *alpha = calloc(restart, sizeof(cplx));
    double *bb = calloc(restart, sizeof(double));
    if (!r || !w || !z || !wh || !a || !c || !alpha || !bb) return OR_ERR_NOMEM;
    for (int k = 0; k < restart; k++) {
        z[k] = malloc(n * sizeof(cplx));
        wh[k] = malloc(n * sizeof(cplx));
        if (!z[k] || !wh[k]) return OR_ERR_NOMEM;
    }
    if (!x_is_guess) memset(x, 0, n * sizeof(cplx));
    double fn = vnorm(n, f);
    int steps = 0, status = OR_ERR_NOT_CONVERGED, hcount = 0;
    double rel = 0;
    if (fn == 0) {
        memset(x, 0, n * sizeof(cplx));
        status = OR_OK;
        goto done;
    }
    oracle_apply_A(L, bc, U, C, x, r);
    for (long k = 0; k < n; k++) r[k] = f[k] - r[k];
    rel = vnorm(n, r) / fn;
    if (history) history[hcount++] = rel;
    if (rel <= tol) { status = OR_OK; goto done; }

    for (int cyc = 0; cyc < max_cycles; cyc++) {
        int kend = 0;
        for (int k = 0; k < restart; k++) {
            if (precond == 2) oracle_sap_additive(L, b, bc, U, C, Cinv, n_cycles, n_mr, r, z[k]);
            else if (precond) oracle_sap(L, b, bc, U, C, Cinv, n_cycles, n_mr, r, z[k]);
            else memcpy(z[k], r, n * sizeof(cplx));
            oracle_apply_A(L, bc, U, C, z[k], w);
            for (int j = 0; j < k; j++) {
                cplx ajk = vdot(n, wh[j], w);
                a[j * restart + k] = ajk;
                for (long q = 0; q < n; q++) w[q] -= ajk * wh[j][q];
            }
            bb[k] = vnorm(n, w);
            for (long q = 0; q < n; q++) wh[k][q] = w[q] / bb[k];
            c[k] = vdot(n, wh[k], r);
            for (long q = 0; q < n; q++) r[q] -= c[k] * wh[k][q];
            steps++;
            kend = k + 1;
            rel = vnorm(n, r) / fn;
            if (history && hcount < max_cycles * restart) history[hcount++] = rel;
            if (rel <= tol) break;
        }
        for (int k = kend - 1; k >= 0; k--) {
            cplx s = c[k];
            for (int j = k + 1; j < kend; j++) s -= a[k * restart + j] * alpha[j];
            alpha[k] = s / bb[k];
        }
        for (int k = 0; k < kend; k++)
            for (long q = 0; q < n; q++) x[q] += alpha[k] * z[k][q];
        oracle_apply_A(L, bc, U, C, x, r);
        for (long q = 0; q < n; q++) r[q] = f[q] - r[q];
        rel = vnorm(n, r) / fn;
        if (history && hcount > 0) history[hcount - 1] = rel;
        if (rel <= tol) { status = OR_OK; break; }
    }
done:
    if (n_steps) *n_steps = steps;
    if (relres) *relres = rel;
    for (int k = 0; k < restart; k++) { free(z[k]); free(wh[k]); }
    free(z); free(wh); free(a); free(c); free(alpha); free(bb); free(r); free(w);
    return status;
}

/* ------------------------------------------------------------------ */
/* flexible GMRES with deflated restarts (outer solver, Sec. II-C)     */
/* ------------------------------------------------------------------ */

/* Small dense complex matrices are row-major: M[i*ld + j]. */

/* Least squares min_y |c - H y| for H (rows x cols, rows > cols, full column
   rank), by Householder QR; returns |c - H y|. */
static double small_lsq(int rows, int cols, const cplx *H, int ldh, const cplx *c, cplx *y)
{
    cplx *A = malloc(sizeof(cplx) * rows * cols), *b = malloc(sizeof(cplx) * rows);
    for (int i = 0; i < rows; i++) {
        for (int j = 0; j < cols; j++) A[i * cols + j] = H[i * ldh + j];
        b[i] = c[i];
    }
    for (int j = 0; j < cols; j++) {
        /* Householder vector u = x + e^{i arg x_0} |x| e_0 for column j, rows j.. */
        double nx = 0;
        for (int i = j; i < rows; i++) nx += creal(conj(A[i * cols + j]) * A[i * cols + j]);
        nx = sqrt(nx);
        if (nx == 0) continue;
        cplx x0 = A[j * cols + j];
        cplx ph = cabs(x0) > 0 ? x0 / cabs(x0) : 1.0;
        cplx *u = malloc(sizeof(cplx) * rows);
        for (int i = 0; i < rows; i++) u[i] = i >= j ? A[i * cols + j] : 0;
        u[j] += ph * nx;
        double uu = 0;
        for (int i = j; i < rows; i++) uu += creal(conj(u[i]) * u[i]);
        /* apply (1 - 2 u u^H / u^H u) to the remaining columns and to b */
        for (int q = j; q < cols; q++) {
            cplx t = 0;
            for (int i = j; i < rows; i++) t += conj(u[i]) * A[i * cols + q];
            t *= 2.0 / uu;
            for (int i = j; i < rows; i++) A[i * cols + q] -= t * u[i];
        }
        cplx t = 0;
        for (int i = j; i < rows; i++) t += conj(u[i]) * b[i];
        t *= 2.0 / uu;
        for (int i = j; i < rows; i++) b[i] -= t * u[i];
        free(u);
    }
    for (int j = cols - 1; j >= 0; j--) {
        cplx t = b[j];
        for (int q = j + 1; q < cols; q++) t -= A[j * cols + q] * y[q];
        y[j] = t / A[j * cols + j];
    }
    double res = 0;
    for (int i = cols; i < rows; i++) res += creal(conj(b[i]) * b[i]);
    free(A);
    free(b);
    return sqrt(res);
}

/* Solves M X = B (M n x n, B n x nr) by Gaussian elimination with partial
   pivoting; returns nonzero if M is singular. */
static int small_solve(int n, const cplx *M, int nr, cplx *B)
{
    cplx *A = malloc(sizeof(cplx) * n * n);
    memcpy(A, M, sizeof(cplx) * n * n);
    int bad = 0;
    for (int c = 0; c < n && !bad; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (cabs(A[r * n + c]) > cabs(A[p * n + c])) p = r;
        if (cabs(A[p * n + c]) == 0) { bad = 1; break; }
        if (p != c) {
            for (int q = 0; q < n; q++) { cplx t = A[c * n + q]; A[c * n + q] = A[p * n + q]; A[p * n + q] = t; }
            for (int q = 0; q < nr; q++) { cplx t = B[c * nr + q]; B[c * nr + q] = B[p * nr + q]; B[p * nr + q] = t; }
        }
        for (int r = c + 1; r < n; r++) {
            cplx f = A[r * n + c] / A[c * n + c];
            for (int q = c; q < n; q++) A[r * n + q] -= f * A[c * n + q];
            for (int q = 0; q < nr; q++) B[r * nr + q] -= f * B[c * nr + q];
        }
    }
    for (int c = n - 1; c >= 0 && !bad; c--)
        for (int q = 0; q < nr; q++) {
            cplx t = B[c * nr + q];
            for (int j = c + 1; j < n; j++) t -= A[c * n + j] * B[j * nr + q];
            B[c * nr + q] = t / A[c * n + c];
        }
    free(A);
    return bad;
}

/* Eigenvalues and eigenvectors of a general complex n x n matrix B: reduction
   to upper Hessenberg form by Householder reflections, then the shifted QR
   iteration (Givens rotations, Wilkinson shift, deflation at negligible
   subdiagonal entries) to the Schur form B = Z T Z^H, and eigenvectors of the
   triangular T by back substitution, mapped back with Z.  lam[i] and the
   columns of X (row-major n x n, X[r*n+i]) hold the pairs. */
static void small_eig(int n, const cplx *B, cplx *lam, cplx *X)
{
    cplx *T = malloc(sizeof(cplx) * n * n), *Z = malloc(sizeof(cplx) * n * n);
    memcpy(T, B, sizeof(cplx) * n * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Z[i * n + j] = i == j;
    /* Hessenberg reduction: T <- Q^H T Q, Z <- Z Q */
    for (int j = 0; j + 2 < n; j++) {
        double nx = 0;
        for (int i = j + 1; i < n; i++) nx += creal(conj(T[i * n + j]) * T[i * n + j]);
        nx = sqrt(nx);
        if (nx == 0) continue;
        cplx *u = calloc(n, sizeof(cplx));
        cplx x0 = T[(j + 1) * n + j];
        cplx ph = cabs(x0) > 0 ? x0 / cabs(x0) : 1.0;
        for (int i = j + 1; i < n; i++) u[i] = T[i * n + j];
        u[j + 1] += ph * nx;
        double uu = 0;
        for (int i = j + 1; i < n; i++) uu += creal(conj(u[i]) * u[i]);
        for (int q = 0; q < n; q++) {   /* rows: T <- (1 - 2uu^H/uu) T */
            cplx t = 0;
            for (int i = j + 1; i < n; i++) t += conj(u[i]) * T[i * n + q];
            t *= 2.0 / uu;
            for (int i = j + 1; i < n; i++) T[i * n + q] -= t * u[i];
        }
        for (int r = 0; r < n; r++) {   /* columns: T <- T (1 - 2uu^H/uu), Z likewise */
            cplx t = 0, tz = 0;
            for (int i = j + 1; i < n; i++) {
                t += T[r * n + i] * u[i];
                tz += Z[r * n + i] * u[i];
            }
            t *= 2.0 / uu;
            tz *= 2.0 / uu;
            for (int i = j + 1; i < n; i++) {
                T[r * n + i] -= t * conj(u[i]);
                Z[r * n + i] -= tz * conj(u[i]);
            }
        }
        free(u);
        for (int i = j + 2; i < n; i++) T[i * n + j] = 0;
    }
    /* shifted QR iteration on the active block [lo, hi] */
    int hi = n - 1, iter = 0;
    while (hi > 0 && iter < 100 * n) {
        /* deflate */
        int l = hi;
        while (l > 0) {
            double s = cabs(T[(l - 1) * n + l - 1]) + cabs(T[l * n + l]);
            if (cabs(T[l * n + l - 1]) <= 1e-15 * (s > 0 ? s : 1.0)) {
                T[l * n + l - 1] = 0;
                break;
            }
            l--;
        }
        if (l == hi) {
            hi--;
            iter = 0;
            continue;
        }
        iter++;
        /* Wilkinson shift from the trailing 2x2 block, or an exceptional shift */
        cplx a = T[(hi - 1) * n + hi - 1], b2 = T[(hi - 1) * n + hi], c2 = T[hi * n + hi - 1], d = T[hi * n + hi];
        cplx tr = a + d, det = a * d - b2 * c2, disc = csqrt(tr * tr / 4 - det);
        cplx mu1 = tr / 2 + disc, mu2 = tr / 2 - disc;
        cplx mu = cabs(mu1 - d) < cabs(mu2 - d) ? mu1 : mu2;
        if (iter % 20 == 0) mu = d + cabs(T[hi * n + hi - 1]);
        /* QR of (T - mu) on rows/cols l..hi by Givens rotations, then RQ + mu */
        int nb = hi - l + 1;
        cplx *cs = malloc(sizeof(cplx) * nb), *sn = malloc(sizeof(cplx) * nb);
        for (int i = l; i <= hi; i++) T[i * n + i] -= mu;
        for (int i = l; i < hi; i++) {
            cplx x = T[i * n + i], y = T[(i + 1) * n + i];
            double r = sqrt(creal(conj(x) * x) + creal(conj(y) * y));
            cplx cc = r > 0 ? x / r : 1.0, ss = r > 0 ? y / r : 0.0;
            cs[i - l] = cc;
            sn[i - l] = ss;
            for (int q = i; q < n; q++) {   /* G^H rows i, i+1 */
                cplx t1 = T[i * n + q], t2 = T[(i + 1) * n + q];
                T[i * n + q] = conj(cc) * t1 + conj(ss) * t2;
                T[(i + 1) * n + q] = -ss * t1 + cc * t2;
            }
        }
        for (int i = l; i < hi; i++) {   /* multiply by G on the right: columns i, i+1 */
            cplx cc = cs[i - l], ss = sn[i - l];
            for (int r = 0; r <= (i + 1 < hi ? i + 1 : hi); r++) {
                cplx t1 = T[r * n + i], t2 = T[r * n + i + 1];
                T[r * n + i] = cc * t1 + ss * t2;
                T[r * n + i + 1] = -conj(ss) * t1 + conj(cc) * t2;
            }
            for (int r = 0; r < n; r++) {
                cplx t1 = Z[r * n + i], t2 = Z[r * n + i + 1];
                Z[r * n + i] = cc * t1 + ss * t2;
                Z[r * n + i + 1] = -conj(ss) * t1 + conj(cc) * t2;
            }
        }
        for (int i = l; i <= hi; i++) T[i * n + i] += mu;
        free(cs);
        free(sn);
    }
    for (int i = 0; i < n; i++) lam[i] = T[i * n + i];
    /* eigenvectors of T, then X = Z Y */
    double tn = 0;
    for (int i = 0; i < n * n; i++) tn += cabs(T[i]);
    cplx *Y = calloc(n, sizeof(cplx));
    for (int e = 0; e < n; e++) {
        for (int i = 0; i < n; i++) Y[i] = 0;
        Y[e] = 1;
        for (int j = e - 1; j >= 0; j--) {
            cplx t = 0;
            for (int q = j + 1; q <= e; q++) t -= T[j * n + q] * Y[q];
            cplx den = T[j * n + j] - lam[e];
            if (cabs(den) < 1e-14 * tn) den = 1e-14 * tn;
            Y[j] = t / den;
        }
        double nrm = 0;
        for (int r = 0; r < n; r++) {
            cplx v = 0;
            for (int q = 0; q <= e; q++) v += Z[r * n + q] * Y[q];
            X[r * n + e] = v;
            nrm += creal(conj(v) * v);
        }
        nrm = sqrt(nrm);
        for (int r = 0; r < n; r++) X[r * n + e] /= nrm;
    }
    free(Y);
    free(T);
    free(Z);
}

/* The k harmonic Ritz pairs of smallest magnitude of a flexible Arnoldi
   relation A Z_m = V_{m+1} Hbar (Hbar (m+1) x m, row-major): the pairs
   (theta, g) with Hbar^H (Hbar g - theta [g; 0]) = 0, i.e. the eigenpairs of
   H_m^{-H} Hbar^H Hbar with H_m the first m rows of Hbar.  P (m x k, row-major)
   receives an orthonormal basis of span{g_1..g_k} (modified Gram-Schmidt, two
   passes), theta the k values in increasing magnitude.  Returns nonzero if
   H_m is singular. */
int oracle_harmonic_ritz(int m, const cplx *Hbar, int k, cplx *P, cplx *theta)
{
    if (m < 1 || k < 1 || k > m) return OR_ERR_ARG;
    cplx *G = malloc(sizeof(cplx) * m * m), *HmH = malloc(sizeof(cplx) * m * m);
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++) {
            cplx s = 0;
            for (int q = 0; q <= m; q++) s += conj(Hbar[q * m + i]) * Hbar[q * m + j];
            G[i * m + j] = s;                     /* Hbar^H Hbar */
            HmH[i * m + j] = conj(Hbar[j * m + i]);   /* H_m^H */
        }
    if (small_solve(m, HmH, m, G)) {
        free(G);
        free(HmH);
        return OR_ERR_ARG;
    }
    cplx *lam = malloc(sizeof(cplx) * m), *X = malloc(sizeof(cplx) * m * m);
    small_eig(m, G, lam, X);
    int *ord = malloc(sizeof(int) * m);
    for (int i = 0; i < m; i++) ord[i] = i;
    for (int i = 0; i < m; i++)
        for (int j = i + 1; j < m; j++)
            if (cabs(lam[ord[j]]) < cabs(lam[ord[i]])) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
    for (int q = 0; q < k; q++) {
        theta[q] = lam[ord[q]];
        for (int r = 0; r < m; r++) P[r * k + q] = X[r * m + ord[q]];
        for (int pass = 0; pass < 2; pass++)
            for (int p = 0; p < q; p++) {
                cplx d = 0;
                for (int r = 0; r < m; r++) d += conj(P[r * k + p]) * P[r * k + q];
                for (int r = 0; r < m; r++) P[r * k + q] -= d * P[r * k + p];
            }
        double nrm = 0;
        for (int r = 0; r < m; r++) nrm += creal(conj(P[r * k + q]) * P[r * k + q]);
        nrm = sqrt(nrm);
        for (int r = 0; r < m; r++) P[r * k + q] /= nrm;
    }
    free(ord);
    free(lam);
    free(X);
    free(G);
    free(HmH);
    return OR_OK;
}

/* Solves A x = f by flexible GMRES with deflated restarts, right-preconditioned
   by M (precond: 0 M = 1, 1 multiplicative SAP, 2 additive SAP).  A cycle runs
   the flexible Arnoldi process z_j = M v_j, w = A z_j, modified Gram-Schmidt of
   w against v_1..v_j (Hbar column j), v_{j+1} = w / |w|, up to m steps,
   keeping A Z = V Hbar; after each step the least squares problem
   min |c - Hbar y| gives the residual estimate, and the cycle ends at m steps
   or when it falls below tol |f|.  Then x += Z y and the true residual f - A x
   decides convergence.  Restart: with k > 0 deflation vectors after a full
   cycle, the k harmonic Ritz vectors of smallest magnitude (oracle_harmonic_ritz)
   and the least squares residual s = c - Hbar y form the orthonormal (m+1) x
   (k+1) matrix P = [[P_k; 0], p] (p: s orthogonalised against them), and the
   next cycle starts from V_{k+1} = V P, Z_k = Z P_k, Hbar_k = P^H Hbar P_k,
   c = P^H s, with the Arnoldi process continued from step k+1 (orthogonalising
   against all earlier v); otherwise (k = 0, or a cycle stopped early) it
   restarts from the true residual.  n_steps counts preconditioner
   applications; history (length max_cycles*m+1) gets the residual estimate of
   every step, and the true residual at each cycle's end. */
int oracle_fgmres_dr(const int L[4], const int b[4], const double bc[4], const cplx *U, const cplx *C,
                     const cplx *Cinv, int precond, int n_cycles, int n_mr, int m, int k, double tol, int max_cycles,
                     const cplx *f, cplx *x, int x_is_guess, int *n_steps, double *relres, double *history)
{
    if (m < 1 || k < 0 || k >= m || max_cycles < 1 || !(tol > 0)) return OR_ERR_ARG;
    if (precond) {
        int e = check_domains(L, b);
        if (e) return e;
    }
    build_gamma();
    long V = volume(L), n = V * 12;
    cplx **Vb = malloc(sizeof(cplx *) * (m + 1)), **Zb = malloc(sizeof(cplx *) * m);
    cplx *r = malloc(n * sizeof(cplx)), *w = malloc(n * sizeof(cplx));
    cplx *H = calloc((size_t)(m + 1) * m, sizeof(cplx)), *c = calloc(m + 1, sizeof(cplx)), *y = calloc(m, sizeof(cplx));
    for (int j = 0; j <= m; j++) Vb[j] = malloc(n * sizeof(cplx));
    for (int j = 0; j < m; j++) Zb[j] = malloc(n * sizeof(cplx));
    if (!x_is_guess) memset(x, 0, n * sizeof(cplx));
    double fn = vnorm(n, f), rel = 0;
    int steps = 0, status = OR_ERR_NOT_CONVERGED, hcount = 0, j0 = 0;
    if (fn == 0) {
        memset(x, 0, n * sizeof(cplx));
        status = OR_OK;
        goto done;
    }
    oracle_apply_A(L, bc, U, C, x, r);
    for (long q = 0; q < n; q++) r[q] = f[q] - r[q];
    rel = vnorm(n, r) / fn;
    if (history) history[hcount++] = rel;
    if (rel <= tol) { status = OR_OK; goto done; }
    for (int cyc = 0; cyc < max_cycles; cyc++) {
        if (j0 == 0) {   /* plain (re)start from the true residual */
            double beta = vnorm(n, r);
            for (long q = 0; q < n; q++) Vb[0][q] = r[q] / beta;
            memset(H, 0, sizeof(cplx) * (m + 1) * m);
            memset(c, 0, sizeof(cplx) * (m + 1));
            c[0] = beta;
        }
        int jend = m;
        for (int j = j0; j < m; j++) {
            if (precond == 2) oracle_sap_additive(L, b, bc, U, C, Cinv, n_cycles, n_mr, Vb[j], Zb[j]);
            else if (precond) oracle_sap(L, b, bc, U, C, Cinv, n_cycles, n_mr, Vb[j], Zb[j]);
            else memcpy(Zb[j], Vb[j], n * sizeof(cplx));
            oracle_apply_A(L, bc, U, C, Zb[j], w);
            for (int i = 0; i <= j; i++) {
                cplx h = vdot(n, Vb[i], w);
                H[i * m + j] = h;
                for (long q = 0; q < n; q++) w[q] -= h * Vb[i][q];
            }
            double hn = vnorm(n, w);
            H[(j + 1) * m + j] = hn;
            for (long q = 0; q < n; q++) Vb[j + 1][q] = w[q] / hn;
            steps++;
            double est = small_lsq(j + 2, j + 1, H, m, c, y) / fn;
            if (history && hcount <= max_cycles * m) history[hcount++] = est;
            if (est <= tol) { jend = j + 1; break; }
        }
        for (int j = 0; j < jend; j++)
            for (long q = 0; q < n; q++) x[q] += y[j] * Zb[j][q];
        oracle_apply_A(L, bc, U, C, x, r);
        for (long q = 0; q < n; q++) r[q] = f[q] - r[q];
        rel = vnorm(n, r) / fn;
        if (history && hcount > 0) history[hcount - 1] = rel;
        if (rel <= tol) { status = OR_OK; break; }
        if (k == 0 || jend < m) { j0 = 0; continue; }
        /* deflated restart */
        cplx *s = malloc(sizeof(cplx) * (m + 1)), *Pk = malloc(sizeof(cplx) * m * k), *th = malloc(sizeof(cplx) * k);
        cplx *P = calloc((size_t)(m + 1) * (k + 1), sizeof(cplx));
        for (int i = 0; i <= m; i++) {
            cplx t = c[i];
            for (int j = 0; j < m; j++) t -= H[i * m + j] * y[j];
            s[i] = t;
        }
        if (oracle_harmonic_ritz(m, H, k, Pk, th)) {
            free(s); free(Pk); free(th); free(P);
            j0 = 0;
            continue;
        }
        for (int i = 0; i < m; i++)
            for (int q = 0; q < k; q++) P[i * (k + 1) + q] = Pk[i * k + q];
        for (int i = 0; i <= m; i++) P[i * (k + 1) + k] = s[i];
        for (int pass = 0; pass < 2; pass++)
            for (int q = 0; q < k; q++) {
                cplx d = 0;
                for (int i = 0; i <= m; i++) d += conj(P[i * (k + 1) + q]) * P[i * (k + 1) + k];
                for (int i = 0; i <= m; i++) P[i * (k + 1) + k] -= d * P[i * (k + 1) + q];
            }
        double pn = 0;
        for (int i = 0; i <= m; i++) pn += creal(conj(P[i * (k + 1) + k]) * P[i * (k + 1) + k]);
        pn = sqrt(pn);
        for (int i = 0; i <= m; i++) P[i * (k + 1) + k] /= pn;
        /* new bases: V_{k+1} = V P, Z_k = Z P_k (through w and r as scratch) */
        cplx **nV = malloc(sizeof(cplx *) * (k + 1)), **nZ = malloc(sizeof(cplx *) * k);
        for (int q = 0; q <= k; q++) nV[q] = calloc(n, sizeof(cplx));
        for (int q = 0; q < k; q++) nZ[q] = calloc(n, sizeof(cplx));
        for (int q = 0; q <= k; q++)
            for (int i = 0; i <= m; i++)
                for (long t = 0; t < n; t++) nV[q][t] += Vb[i][t] * P[i * (k + 1) + q];
        for (int q = 0; q < k; q++)
            for (int i = 0; i < m; i++)
                for (long t = 0; t < n; t++) nZ[q][t] += Zb[i][t] * P[i * (k + 1) + q];
        for (int q = 0; q <= k; q++) { memcpy(Vb[q], nV[q], n * sizeof(cplx)); free(nV[q]); }
        for (int q = 0; q < k; q++) { memcpy(Zb[q], nZ[q], n * sizeof(cplx)); free(nZ[q]); }
        free(nV);
        free(nZ);
        /* Hbar_k = P^H Hbar P_k, c = P^H s */
        cplx *Hn = calloc((size_t)(m + 1) * m, sizeof(cplx));
        for (int a = 0; a <= k; a++)
            for (int q = 0; q < k; q++) {
                cplx t = 0;
                for (int i = 0; i <= m; i++)
                    for (int j = 0; j < m; j++) t += conj(P[i * (k + 1) + a]) * H[i * m + j] * P[j * (k + 1) + q];
                Hn[a * m + q] = t;
            }
        memcpy(H, Hn, sizeof(cplx) * (m + 1) * m);
        free(Hn);
        memset(c, 0, sizeof(cplx) * (m + 1));
        for (int a = 0; a <= k; a++) {
            cplx t = 0;
            for (int i = 0; i <= m; i++) t += conj(P[i * (k + 1) + a]) * s[i];
            c[a] = t;
        }
        free(s); free(Pk); free(th); free(P);
        j0 = k;
    }
done:
    if (n_steps) *n_steps = steps;
    if (relres) *relres = rel;
    for (int j = 0; j <= m; j++) free(Vb[j]);
    for (int j = 0; j < m; j++) free(Zb[j]);
    free(Vb); free(Zb); free(r); free(w); free(H); free(c); free(y);
    return status;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
