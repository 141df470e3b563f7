// Layout conversion, clover set-up, the global operator A and the FP64
// linear algebra of the outer solver.
#include <hip/hip_runtime.h>

#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

static inline unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ===========================================================================
// layout conversion
// ===========================================================================

__device__ __forceinline__ long canon_index(const Geo &g, const int x[4])
{
    return x[0] + (long)g.L[0] * (x[1] + (long)g.L[1] * (x[2] + (long)g.L[2] * x[3]));
}

template <typename S> __global__ void k_import_spinor(Geo g, const double2 *canon, v2<S> *out)
{
    long I = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.V) return;
    int x[4], d, loc;
    decode(g, I, x, d, loc);
    long c = canon_index(g, x) * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) st<double, S>(out, ((long)d * 12 + k) * g.Vd + loc, ld<double, double>(canon, c + k));
}

template <typename S> __global__ void k_export_spinor(Geo g, const v2<S> *in, double2 *canon)
{
    long I = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.V) return;
    int x[4], d, loc;
    decode(g, I, x, d, loc);
    long c = canon_index(g, x) * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) st<double, double>(canon, c + k, ld<double, S>(in, ((long)d * 12 + k) * g.Vd + loc));
}

// The same conversions through LDS, one workgroup per domain of VD sites
// (VD threads): the canonical side is moved as the domain's x-runs (b0 sites
// x 12 components, contiguous in memory), consecutive threads on consecutive
// 16-byte entries; the internal side one component at a time, consecutive
// threads on consecutive sites.  buf holds the domain as [local lexicographic
// site][12].
__device__ __forceinline__ long dom_run_base(const Geo &g, int d, int j)
{
    // canonical index of the first site of x-run j (= (ly, lz, lt)) of domain d
    int r = d, x[4];
    x[0] = (r % g.n[0]) * g.b[0]; r /= g.n[0];
    x[1] = (r % g.n[1]) * g.b[1]; r /= g.n[1];
    x[2] = (r % g.n[2]) * g.b[2];
    x[3] = (r / g.n[2]) * g.b[3];
    x[1] += j % g.b[1]; j /= g.b[1];
    x[2] += j % g.b[2];
    x[3] += j / g.b[2];
    return canon_index(g, x);
}

__device__ __forceinline__ int local_lex(const Geo &g, const int x[4])
{
    return x[0] % g.b[0] + g.b[0] * (x[1] % g.b[1] + g.b[1] * (x[2] % g.b[2] + g.b[2] * (x[3] % g.b[3])));
}

template <int VD, typename S> __global__ __launch_bounds__(VD) void k_import_dom(Geo g, const double2 *canon, v2<S> *out)
{
    __shared__ double2 buf[12 * VD];
    const int d = blockIdx.x, t = threadIdx.x;
    const int runlen = g.b[0] * 12;
    for (int e = t; e < 12 * VD; e += VD) {
        const int j = e / runlen, o = e - j * runlen;
        buf[e] = canon[dom_run_base(g, d, j) * 12 + o];
    }
    __syncthreads();
    int x[4], dd, loc;
    decode(g, (long)d * VD + t, x, dd, loc);
    const int ll = local_lex(g, x);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const double2 v = buf[ll * 12 + k];
        st<double, S>(out, ((long)d * 12 + k) * VD + t, cx<double>{v.x, v.y});
    }
}

template <int VD, typename S> __global__ __launch_bounds__(VD) void k_export_dom(Geo g, const v2<S> *in, double2 *canon)
{
    __shared__ double2 buf[12 * VD];
    const int d = blockIdx.x, t = threadIdx.x;
    int x[4], dd, loc;
    decode(g, (long)d * VD + t, x, dd, loc);
    const int ll = local_lex(g, x);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const cx<double> v = ld<double, S>(in, ((long)d * 12 + k) * VD + t);
        buf[ll * 12 + k] = make_double2(v.r, v.i);
    }
    __syncthreads();
    const int runlen = g.b[0] * 12;
    for (int e = t; e < 12 * VD; e += VD) {
        const int j = e / runlen, o = e - j * runlen;
        canon[dom_run_base(g, d, j) * 12 + o] = buf[e];
    }
}

template <int VD>
static void launch_convert_dom(const Geo &g, const double *canon, void *internal, int prec, bool import,
                               hipStream_t s)
{
    const unsigned nb = (unsigned)g.nd;
    if (import) {
        const double2 *c = (const double2 *)canon;
        if (prec == P64) hipLaunchKernelGGL((k_import_dom<VD, double>), nb, VD, 0, s, g, c, (double2 *)internal);
        else if (prec == P32) hipLaunchKernelGGL((k_import_dom<VD, float>), nb, VD, 0, s, g, c, (float2 *)internal);
        else if (prec == P16) hipLaunchKernelGGL((k_import_dom<VD, half_t>), nb, VD, 0, s, g, c, (half2_t *)internal);
        else hipLaunchKernelGGL((k_import_dom<VD, bf16_t>), nb, VD, 0, s, g, c, (bf162_t *)internal);
    } else {
        double2 *c = (double2 *)canon;
        if (prec == P64) hipLaunchKernelGGL((k_export_dom<VD, double>), nb, VD, 0, s, g, (const double2 *)internal, c);
        else if (prec == P32) hipLaunchKernelGGL((k_export_dom<VD, float>), nb, VD, 0, s, g, (const float2 *)internal, c);
        else if (prec == P16) hipLaunchKernelGGL((k_export_dom<VD, half_t>), nb, VD, 0, s, g, (const half2_t *)internal, c);
        else hipLaunchKernelGGL((k_export_dom<VD, bf16_t>), nb, VD, 0, s, g, (const bf162_t *)internal, c);
    }
}

// domains of 256 or 512 sites through LDS, others one thread per site
static bool convert_dom(const Geo &g, const double *canon, void *internal, int prec, bool import, hipStream_t s)
{
    if (g.Vd == 256) launch_convert_dom<256>(g, canon, internal, prec, import, s);
    else if (g.Vd == 512) launch_convert_dom<512>(g, canon, internal, prec, import, s);
    else return false;
    return true;
}

hipError_t import_spinor(const Geo &g, const double *canon, void *internal, int prec, hipStream_t s)
{
    if (convert_dom(g, canon, internal, prec, true, s)) return hipGetLastError();
    unsigned nb = nblocks(g.V, 256);
    if (prec == P64) hipLaunchKernelGGL(k_import_spinor<double>, nb, 256, 0, s, g, (const double2 *)canon, (double2 *)internal);
    else if (prec == P32) hipLaunchKernelGGL(k_import_spinor<float>, nb, 256, 0, s, g, (const double2 *)canon, (float2 *)internal);
    else if (prec == P16) hipLaunchKernelGGL(k_import_spinor<half_t>, nb, 256, 0, s, g, (const double2 *)canon, (half2_t *)internal);
    else hipLaunchKernelGGL(k_import_spinor<bf16_t>, nb, 256, 0, s, g, (const double2 *)canon, (bf162_t *)internal);
    return hipGetLastError();
}

hipError_t export_spinor(const Geo &g, const void *internal, int prec, double *canon, hipStream_t s)
{
    if (convert_dom(g, canon, const_cast<void *>(internal), prec, false, s)) return hipGetLastError();
    unsigned nb = nblocks(g.V, 256);
    if (prec == P64) hipLaunchKernelGGL(k_export_spinor<double>, nb, 256, 0, s, g, (const double2 *)internal, (double2 *)canon);
    else if (prec == P32) hipLaunchKernelGGL(k_export_spinor<float>, nb, 256, 0, s, g, (const float2 *)internal, (double2 *)canon);
    else if (prec == P16) hipLaunchKernelGGL(k_export_spinor<half_t>, nb, 256, 0, s, g, (const half2_t *)internal, (double2 *)canon);
    else hipLaunchKernelGGL(k_export_spinor<bf16_t>, nb, 256, 0, s, g, (const bf162_t *)internal, (double2 *)canon);
    return hipGetLastError();
}

__global__ void k_import_gauge(Geo g, const double2 *canon, double2 *U)
{
    long I = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.V) return;
    int x[4], d, loc;
    decode(g, I, x, d, loc);
    long c = canon_index(g, x) * 36;
    for (int mu = 0; mu < 4; mu++)
#pragma unroll
        for (int e = 0; e < 9; e++) U[(((long)d * 4 + mu) * 9 + e) * g.Vd + loc] = canon[c + mu * 9 + e];
}

hipError_t import_gauge(const Geo &g, const double *canon, double2 *U64, hipStream_t s)
{
    hipLaunchKernelGGL(k_import_gauge, nblocks(g.V, 256), 256, 0, s, g, (const double2 *)canon, U64);
    return hipGetLastError();
}

template <typename S> __global__ void k_compress_links(Geo g, const double2 *U, v2<S> *out)
{
    long I = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.V) return;
    int d = (int)(I / g.Vd), loc = (int)(I - (long)d * g.Vd);
    for (int mu = 0; mu < 4; mu++)
#pragma unroll
        for (int e = 0; e < 6; e++)
            st<double, S>(out, (((long)d * 4 + mu) * 6 + e) * g.Vd + loc,
                          ld<double, double>(U, (((long)d * 4 + mu) * 9 + e) * g.Vd + loc));
}

hipError_t compress_links(const Geo &g, const double2 *U64, void *out, int prec, hipStream_t s)
{
    unsigned nb = nblocks(g.V, 256);
    if (prec == P32) hipLaunchKernelGGL(k_compress_links<float>, nb, 256, 0, s, g, U64, (float2 *)out);
    else if (prec == P16) hipLaunchKernelGGL(k_compress_links<half_t>, nb, 256, 0, s, g, U64, (half2_t *)out);
    else hipLaunchKernelGGL(k_compress_links<bf16_t>, nb, 256, 0, s, g, U64, (bf162_t *)out);
    return hipGetLastError();
}

template <typename S> __global__ void k_convert_pairs(const double2 *in, v2<S> *out, long n)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) st<double, S>(out, i, ld<double, double>(in, i));
}

hipError_t convert_pairs(const double2 *in, void *out, long n, int prec, hipStream_t s)
{
    unsigned nb = nblocks(n, 256);
    if (prec == P32) hipLaunchKernelGGL(k_convert_pairs<float>, nb, 256, 0, s, in, (float2 *)out, n);
    else if (prec == P16) hipLaunchKernelGGL(k_convert_pairs<half_t>, nb, 256, 0, s, in, (half2_t *)out, n);
    else hipLaunchKernelGGL(k_convert_pairs<bf16_t>, nb, 256, 0, s, in, (bf162_t *)out, n);
    return hipGetLastError();
}

__global__ void k_count_nonfinite(const double2 *v, long n, int *cnt)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    for (; i < n; i += (long)gridDim.x * blockDim.x) bad |= !isfinite(v[i].x) || !isfinite(v[i].y);
    if (bad) atomicOr(cnt, 1);
}

hipError_t count_nonfinite(const double2 *v, long n, int *cnt, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_nonfinite, 1024, 256, 0, s, v, n, cnt);
    return hipGetLastError();
}

// ===========================================================================
// clover term (Sec. II-B, Eq. 3) and its odd-site inverse (Sec. II-D, Eq. 5)
// ===========================================================================

struct m3 {
    cx<double> e[9];
};

__device__ __forceinline__ m3 m3_load(const Geo &g, const double2 *U, const int x[4], int mu)
{
    long J = encode(g, x);
    int d = (int)(J / g.Vd), loc = (int)(J - (long)d * g.Vd);
    m3 r;
    for (int e = 0; e < 9; e++) r.e[e] = ld<double, double>(U, (((long)d * 4 + mu) * 9 + e) * g.Vd + loc);
    return r;
}

// a * b with optional daggers
__device__ __forceinline__ m3 m3_mul(const m3 &a, bool da, const m3 &b, bool db)
{
    m3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cx<double> s = czero<double>();
            for (int k = 0; k < 3; k++) {
                cx<double> av = da ? cx<double>{a.e[k * 3 + i].r, -a.e[k * 3 + i].i} : a.e[i * 3 + k];
                cx<double> bv = db ? cx<double>{b.e[j * 3 + k].r, -b.e[j * 3 + k].i} : b.e[k * 3 + j];
                s = s + av * bv;
            }
            r.e[i * 3 + j] = s;
        }
    return r;
}

__device__ __forceinline__ void shift(const Geo &g, const int x[4], int mu, int step, int y[4])
{
    for (int m = 0; m < 4; m++) y[m] = x[m];
    y[mu] += step;
    if (y[mu] >= g.L[mu]) y[mu] -= g.L[mu];
    if (y[mu] < 0) y[mu] += g.L[mu];
}

// F_munu = (Q - Q^dag) / 8, Q = sum of the four leaves at x oriented mu -> nu
__device__ m3 field_strength(const Geo &g, const double2 *U, const int x[4], int mu, int nu)
{
    int xpm[4], xmm[4], xpn[4], xmn[4], a[4], b[4], c[4];
    shift(g, x, mu, +1, xpm);
    shift(g, x, mu, -1, xmm);
    shift(g, x, nu, +1, xpn);
    shift(g, x, nu, -1, xmn);
    shift(g, xpn, mu, -1, a);   // x + nu - mu
    shift(g, xmm, nu, -1, b);   // x - mu - nu
    shift(g, xmn, mu, +1, c);   // x - nu + mu
    m3 Q, t;
    // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    t = m3_mul(m3_load(g, U, x, mu), false, m3_load(g, U, xpm, nu), false);
    t = m3_mul(t, false, m3_load(g, U, xpn, mu), true);
    Q = m3_mul(t, false, m3_load(g, U, x, nu), true);
    // leaf 2: U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    t = m3_mul(m3_load(g, U, x, nu), false, m3_load(g, U, a, mu), true);
    t = m3_mul(t, false, m3_load(g, U, xmm, nu), true);
    t = m3_mul(t, false, m3_load(g, U, xmm, mu), false);
    for (int e = 0; e < 9; e++) Q.e[e] = Q.e[e] + t.e[e];
    // leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    t = m3_mul(m3_load(g, U, xmm, mu), true, m3_load(g, U, b, nu), true);
    t = m3_mul(t, false, m3_load(g, U, b, mu), false);
    t = m3_mul(t, false, m3_load(g, U, xmn, nu), false);
    for (int e = 0; e < 9; e++) Q.e[e] = Q.e[e] + t.e[e];
    // leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+
    t = m3_mul(m3_load(g, U, xmn, nu), true, m3_load(g, U, xmn, mu), false);
    t = m3_mul(t, false, m3_load(g, U, c, nu), false);
    t = m3_mul(t, false, m3_load(g, U, x, mu), true);
    for (int e = 0; e < 9; e++) Q.e[e] = Q.e[e] + t.e[e];
    m3 F;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cx<double> q = Q.e[i * 3 + j], qd = {Q.e[j * 3 + i].r, -Q.e[j * 3 + i].i};
            F.e[i * 3 + j] = scal(0.125, q - qd);
        }
    return F;
}

// In the chiral basis sigma_jk = -eps_jkl diag(s_l, s_l) (j,k spatial) and
// sigma_kt = diag(-s_k, s_k), so with E_l the colour matrices multiplying
// s_l, each chiral block of D_cl is [[E3, E1 - i E2], [E1 + i E2, -E3]] with
//   upper: E1 = -(i c/2)(F_yz + F_xt), E2 = (i c/2)(F_xz - F_yt), E3 = -(i c/2)(F_xy + F_zt)
//   lower: E1 = -(i c/2)(F_yz - F_xt), E2 = (i c/2)(F_xz + F_yt), E3 = -(i c/2)(F_xy - F_zt)
__global__ void k_clover_build(Geo g, const double2 *U, double kappa, double csw, double2 *C)
{
    long I = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.V) return;
    int x[4], d, loc;
    decode(g, I, x, d, loc);
    m3 Fxy = field_strength(g, U, x, 0, 1), Fxz = field_strength(g, U, x, 0, 2), Fxt = field_strength(g, U, x, 0, 3);
    m3 Fyz = field_strength(g, U, x, 1, 2), Fyt = field_strength(g, U, x, 1, 3), Fzt = field_strength(g, U, x, 2, 3);
    const double diag = 1.0 / (2.0 * kappa);
    for (int blk = 0; blk < 2; blk++) {
        const double sg = blk == 0 ? 1.0 : -1.0;
        cx<double> M[6][6];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                int e = i * 3 + j;
                // -(i c/2) X = (c/2) (X.i, -X.r)
                cx<double> s1 = Fyz.e[e] + scal(sg, Fxt.e[e]);
                cx<double> s2 = Fxz.e[e] - scal(sg, Fyt.e[e]);
                cx<double> s3 = Fxy.e[e] + scal(sg, Fzt.e[e]);
                cx<double> E1 = scal(0.5 * csw, cx<double>{s1.i, -s1.r});
                cx<double> E2 = scal(0.5 * csw, cx<double>{-s2.i, s2.r});
                cx<double> E3 = scal(0.5 * csw, cx<double>{s3.i, -s3.r});
                M[i][j] = E3;
                M[3 + i][3 + j] = neg(E3);
                M[i][3 + j] = E1 - times_i(E2);
                M[3 + i][j] = E1 + times_i(E2);
            }
        for (int i = 0; i < 6; i++) M[i][i].r += diag;
        long base = ((long)d * 36 + blk * 18) * g.Vd + loc;
        for (int q = 0; q < 3; q++) C[base + q * g.Vd] = make_double2(M[2 * q][2 * q].r, M[2 * q + 1][2 * q + 1].r);
        for (int i = 1; i < 6; i++)
            for (int j = 0; j < i; j++) C[base + (3 + tri_index(i, j)) * g.Vd] = make_double2(M[i][j].r, M[i][j].i);
    }
}

hipError_t clover_build(const Geo &g, const double2 *U64, double kappa, double csw, double2 *C64, hipStream_t s)
{
    hipLaunchKernelGGL(k_clover_build, nblocks(g.V, 128), 128, 0, s, g, U64, kappa, csw, C64);
    return hipGetLastError();
}

// one thread per (site, chiral block): copy on even sites, Gauss-Jordan
// inverse with partial pivoting on odd sites
__global__ void k_clover_schur(Geo g, const double2 *C, double2 *Cs, int *bad)
{
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * g.V) return;
    long I = t >> 1;
    int blk = (int)(t & 1);
    int d = (int)(I / g.Vd), loc = (int)(I - (long)d * g.Vd);
    long base = ((long)d * 36 + blk * 18) * g.Vd + loc;
    if (loc < g.Vh) {
        for (int q = 0; q < 18; q++) Cs[base + q * g.Vd] = C[base + q * g.Vd];
        return;
    }
    cx<double> M[6][12];
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 12; j++) M[i][j] = czero<double>();
    for (int q = 0; q < 3; q++) {
        double2 v = C[base + q * g.Vd];
        M[2 * q][2 * q].r = v.x;
        M[2 * q + 1][2 * q + 1].r = v.y;
    }
    for (int i = 1; i < 6; i++)
        for (int j = 0; j < i; j++) {
            double2 v = C[base + (3 + tri_index(i, j)) * g.Vd];
            M[i][j] = {v.x, v.y};
            M[j][i] = {v.x, -v.y};
        }
    for (int i = 0; i < 6; i++) M[i][6 + i].r = 1.0;
    for (int c = 0; c < 6; c++) {
        int p = c;
        double best = M[c][c].r * M[c][c].r + M[c][c].i * M[c][c].i;
        for (int r = c + 1; r < 6; r++) {
            double v = M[r][c].r * M[r][c].r + M[r][c].i * M[r][c].i;
            if (v > best) { best = v; p = r; }
        }
        if (!(best > 0)) { atomicOr(bad, 1); return; }
        if (p != c)
            for (int j = 0; j < 12; j++) { cx<double> tmp = M[c][j]; M[c][j] = M[p][j]; M[p][j] = tmp; }
        cx<double> piv = M[c][c];
        double inv = 1.0 / best;
        cx<double> ip = {piv.r * inv, -piv.i * inv};
        for (int j = 0; j < 12; j++) M[c][j] = M[c][j] * ip;
        for (int r = 0; r < 6; r++) {
            if (r == c) continue;
            cx<double> f = M[r][c];
            for (int j = 0; j < 12; j++) M[r][j] = M[r][j] - f * M[c][j];
        }
    }
    for (int q = 0; q < 3; q++) Cs[base + q * g.Vd] = make_double2(M[2 * q][6 + 2 * q].r, M[2 * q + 1][6 + 2 * q + 1].r);
    for (int i = 1; i < 6; i++)
        for (int j = 0; j < i; j++) {
            // Hermitian inverse: average the two triangles to remove rounding asymmetry
            cx<double> a = M[i][6 + j], b = M[j][6 + i];
            Cs[base + (3 + tri_index(i, j)) * g.Vd] = make_double2(0.5 * (a.r + b.r), 0.5 * (a.i - b.i));
        }
}

hipError_t clover_schur(const Geo &g, const double2 *C64, double2 *Cs64, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_clover_schur, nblocks(2 * g.V, 128), 128, 0, s, g, C64, Cs64, bad);
    return hipGetLastError();
}

// ===========================================================================
// global operator A (Sec. II-B, Eqs. 1-2): one thread per site
// ===========================================================================

// one hop: DIR = +1 forward, -1 backward
template <int MU, int DIR, typename T, typename SI, typename G, int NLC>
__device__ __forceinline__ void a_hop(const Geo &g, const int x[4], int d, int loc, const v2<SI> *in,
                                      const v2<G> *links, cx<T> acc[12])
{
    const long Vd = g.Vd;
    int y[4] = {x[0], x[1], x[2], x[3]};
    bool wrap = false;
    if constexpr (DIR > 0) {
        y[MU] = x[MU] + 1;
        if (y[MU] == g.L[MU]) { y[MU] = 0; wrap = true; }
    } else {
        y[MU] = x[MU] - 1;
        if (y[MU] < 0) { y[MU] = g.L[MU] - 1; wrap = true; }
    }
    const long J = encode(g, y);
    const int dj = (int)(J / Vd), lj = (int)(J - (long)dj * Vd);
    cx<T> v[12], h[6], uh[6];
#pragma unroll
    for (int k = 0; k < 12; k++) v[k] = ld<T, SI>(in, ((long)dj * 12 + k) * Vd + lj);
    if constexpr (DIR > 0) {
        // -1/2 (1 - gamma_mu) U_mu(x) psi(x + mu)
        proj<MU, -1>(v, h);
        su3<T> U = ld_link<T, G, NLC>(links, ((long)d * 4 + MU) * NLC * Vd + loc, Vd);
        su3_mul(U, h, uh);
        recon_acc<MU, -1>(acc, uh, T(wrap ? -0.5 * g.bc[MU] : -0.5));
    } else {
        // -1/2 (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu)
        proj<MU, +1>(v, h);
        su3<T> U = ld_link<T, G, NLC>(links, ((long)dj * 4 + MU) * NLC * Vd + lj, Vd);
        su3_dag_mul(U, h, uh);
        recon_acc<MU, +1>(acc, uh, T(wrap ? -0.5 * g.bc[MU] : -0.5));
    }
}

template <typename T, typename SI, typename SO, typename G, int NLC>
__global__ __launch_bounds__(256) void k_apply_A(Geo g, const v2<SI> *in, v2<SO> *out, const v2<G> *links,
                                                 const v2<G> *clov)
{
    // Workgroup w runs on XCD w mod 8.  Blocks are handed out so that each
    // XCD sweeps one contiguous eighth of the domain-blocked site order: most
    // neighbour spinors and links a workgroup reads were brought into the
    // same XCD's L2 by its neighbours (a plain order spreads neighbouring
    // blocks over all eight L2s).
    const unsigned nbk = gridDim.x, w = blockIdx.x;
    const unsigned blk = nbk % 8 == 0 ? (w % 8) * (nbk / 8) + w / 8 : w;
    long I = (long)blk * blockDim.x + threadIdx.x;
    if (I >= g.V) return;
    int x[4], d, loc;
    decode(g, I, x, d, loc);
    const long Vd = g.Vd;
    cx<T> acc[12];
    {
        cx<T> s[12];
#pragma unroll
        for (int k = 0; k < 12; k++) s[k] = ld<T, SI>(in, ((long)d * 12 + k) * Vd + loc);
        clover_apply<T, G>(clov, (long)d * 36 * Vd + loc, Vd, s, acc);
    }
    // The eight hops one after another (a loop the compiler keeps rolled): only
    // one neighbour's spinor and link are live at a time.  Unrolled, the
    // compiler issues every load of the site up front, which needs several
    // hundred registers and spills to scratch.
#pragma unroll 1
    for (int k = 0; k < 8; k++) {
        switch (k) {
            case 0: a_hop<0, +1, T, SI, G, NLC>(g, x, d, loc, in, links, acc); break;
            case 1: a_hop<0, -1, T, SI, G, NLC>(g, x, d, loc, in, links, acc); break;
            case 2: a_hop<1, +1, T, SI, G, NLC>(g, x, d, loc, in, links, acc); break;
            case 3: a_hop<1, -1, T, SI, G, NLC>(g, x, d, loc, in, links, acc); break;
            case 4: a_hop<2, +1, T, SI, G, NLC>(g, x, d, loc, in, links, acc); break;
            case 5: a_hop<2, -1, T, SI, G, NLC>(g, x, d, loc, in, links, acc); break;
            case 6: a_hop<3, +1, T, SI, G, NLC>(g, x, d, loc, in, links, acc); break;
            default: a_hop<3, -1, T, SI, G, NLC>(g, x, d, loc, in, links, acc); break;
        }
    }
#pragma unroll
    for (int k = 0; k < 12; k++) st<T, SO>(out, ((long)d * 12 + k) * Vd + loc, acc[k]);
}

// A on whole domains: a workgroup takes NT consecutive sites of the
// domain-blocked order (NT / Vd whole domains) for R right-hand sides, one
// thread per (site, right-hand side) with the R threads of a site adjacent,
// so their link and clover loads are one request.  The workgroup's input
// spinors are staged in LDS, and each site pushes its backward term
// U_mu(x)^+ (1 + gamma_mu) psi(x) to the site x + mu through LDS, so inside a
// domain every link and spinor is read from memory once (by its own site);
// only hops that leave the domain read a neighbour domain's spinor (and,
// backwards, its link).  The hops are summed in the order of k_apply_A (per
// direction: forward, then backward) with the same products, so both kernels
// give the same bits, for any R.  Field offsets are 32-bit byte offsets (the
// host checks that every field is under 4 GiB), which keeps an address in
// one VGPR.
template <int R, typename SI, typename SO> struct RhsPtrs {
    const v2<SI> *in[R];
    v2<SO> *out[R];
};

template <int MU, int NT, int R, typename T, typename SI, typename G, int NLC>
__device__ __forceinline__ void a_dom_dir(const Geo &g, const int x[4], int d, int loc, int ts, int r,
                                          const v2<SI> *in, const v2<G> *links, cx<T> (*sp)[NT * R],
                                          cx<T> (*ex)[NT * R], cx<T> acc[12])
{
    const unsigned Vd = (unsigned)g.Vd;
    const int base = ts - loc;                // first site of this site's domain in the workgroup
    const int me = ts * R + r;                // this thread's LDS slot
    const int lx = x[MU] % g.b[MU];           // coordinate inside the domain
    cx<T> h[6], uh[6];
    {
        const unsigned lb = ((unsigned)d * 4 + MU) * NLC * Vd + loc;
        const su3<T> U = ld_link_with<T, NLC>([&](int e) { return ld32<T, G>(links, lb + e * Vd); });
        // forward: -1/2 (1 - gamma_mu) U_mu(x) psi(x + mu)
        {
            cx<T> v[12];
            int y[4] = {x[0], x[1], x[2], x[3]};
            bool wrap = false;
            y[MU] = x[MU] + 1;
            if (lx + 1 < g.b[MU]) {
                const int lj = (int)(encode(g, y) - (long)d * Vd);
#pragma unroll
                for (int k = 0; k < 12; k++) v[k] = sp[k][(base + lj) * R + r];
            } else {
                if (y[MU] == g.L[MU]) { y[MU] = 0; wrap = true; }
                const long J = encode(g, y);
                const unsigned dj = (unsigned)(J / Vd), lj = (unsigned)(J - (long)dj * Vd);
#pragma unroll
                for (int k = 0; k < 12; k++) v[k] = ld32<T, SI>(in, (dj * 12 + k) * Vd + lj);
            }
            proj<MU, -1>(v, h);
            su3_mul(U, h, uh);
            recon_acc<MU, -1>(acc, uh, T(wrap ? -0.5 * g.bc[MU] : -0.5));
        }
        // push U_mu(x)^+ (1 + gamma_mu) psi(x) for the site x + mu
        {
            cx<T> v[12];
#pragma unroll
            for (int k = 0; k < 12; k++) v[k] = sp[k][me];
            proj<MU, +1>(v, h);
        }
        su3_dag_mul(U, h, uh);
#pragma unroll
        for (int k = 0; k < 6; k++) ex[k][me] = uh[k];
    }
    __syncthreads();   // every push of this direction is in LDS
    // backward: -1/2 (1 + gamma_mu) U_mu(x - mu)^+ psi(x - mu)
    if (lx > 0) {
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[MU] = x[MU] - 1;
        const int lj = (int)(encode(g, y) - (long)d * Vd);
#pragma unroll
        for (int k = 0; k < 6; k++) uh[k] = ex[k][(base + lj) * R + r];
        recon_acc<MU, +1>(acc, uh, T(-0.5));
    } else {
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[MU] = x[MU] - 1;
        bool wrap = false;
        if (y[MU] < 0) { y[MU] = g.L[MU] - 1; wrap = true; }
        const long J = encode(g, y);
        const unsigned dj = (unsigned)(J / Vd), lj = (unsigned)(J - (long)dj * Vd);
        cx<T> v[12];
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = ld32<T, SI>(in, (dj * 12 + k) * Vd + lj);
        proj<MU, +1>(v, h);
        const unsigned lb = (dj * 4 + MU) * NLC * Vd + lj;
        const su3<T> W = ld_link_with<T, NLC>([&](int e) { return ld32<T, G>(links, lb + e * Vd); });
        su3_dag_mul(W, h, uh);
        recon_acc<MU, +1>(acc, uh, T(wrap ? -0.5 * g.bc[MU] : -0.5));
    }
    __syncthreads();   // the pushes are consumed before the next direction's
}

template <int NT, int R, typename T, typename SI, typename SO, typename G, int NLC>
__global__ __launch_bounds__(NT * R, 2) void k_apply_A_dom(Geo g, RhsPtrs<R, SI, SO> io, const v2<G> *links,
                                                           const v2<G> *clov)
{
    __shared__ cx<T> sp[12][NT * R];   // the workgroup's input spinors
    __shared__ cx<T> ex[6][NT * R];    // backward terms pushed to x + mu
    // XCD-aware order as in k_apply_A: each XCD sweeps one contiguous eighth
    const unsigned nbk = gridDim.x, w = blockIdx.x;
    const unsigned blk = nbk % 8 == 0 ? (w % 8) * (nbk / 8) + w / 8 : w;
    const int t = threadIdx.x, ts = t / R, r = t - ts * R;
    const long I = (long)blk * NT + ts;   // V is a multiple of NT: every thread has a site
    const v2<SI> *in = io.in[0];
    v2<SO> *out = io.out[0];
#pragma unroll
    for (int q = 1; q < R; q++)
        if (r == q) {
            in = io.in[q];
            out = io.out[q];
        }
    int x[4], d, loc;
    decode(g, I, x, d, loc);
    const unsigned Vd = (unsigned)g.Vd;
    cx<T> acc[12];
    {
        cx<T> s[12];
#pragma unroll
        for (int k = 0; k < 12; k++) s[k] = ld32<T, SI>(in, ((unsigned)d * 12 + k) * Vd + loc);
#pragma unroll
        for (int k = 0; k < 12; k++) sp[k][t] = s[k];
        const unsigned cb = (unsigned)d * 36 * Vd + loc;
        clover_block_with<T>([&](int q) { return ld32<T, G>(clov, cb + q * Vd); }, s, acc);
        clover_block_with<T>([&](int q) { return ld32<T, G>(clov, cb + (18 + q) * Vd); }, s + 6, acc + 6);
    }
    __syncthreads();
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++) {
        // the site's indices made opaque per direction: what is formed from
        // them (neighbour indices, offsets) is formed here, not hoisted out of
        // the loop and held in registers through it
        int xs[4] = {x[0], x[1], x[2], x[3]}, ds = d, ls = loc, tss = ts;
        asm volatile("" : "+v"(xs[0]), "+v"(xs[1]), "+v"(xs[2]), "+v"(xs[3]), "+v"(ds), "+v"(ls), "+v"(tss));
        switch (mu) {
            case 0: a_dom_dir<0, NT, R, T, SI, G, NLC>(g, xs, ds, ls, tss, r, in, links, sp, ex, acc); break;
            case 1: a_dom_dir<1, NT, R, T, SI, G, NLC>(g, xs, ds, ls, tss, r, in, links, sp, ex, acc); break;
            case 2: a_dom_dir<2, NT, R, T, SI, G, NLC>(g, xs, ds, ls, tss, r, in, links, sp, ex, acc); break;
            default: a_dom_dir<3, NT, R, T, SI, G, NLC>(g, xs, ds, ls, tss, r, in, links, sp, ex, acc); break;
        }
    }
    {
        int ds = d, ls = loc;   // output offsets formed here, not held through the hops
        asm volatile("" : "+v"(ds), "+v"(ls));
#pragma unroll
        for (int k = 0; k < 12; k++) st32<T, SO>(out, ((unsigned)ds * 12 + k) * Vd + ls, acc[k]);
    }
}

template <int NT, int R, typename T, typename S, int NLC>
static void launch_A_dom(const Geo &g, const void *const *in, void *const *out, const void *links, const void *clov,
                         hipStream_t s)
{
    RhsPtrs<R, S, S> io;
    for (int q = 0; q < R; q++) {
        io.in[q] = (const v2<S> *)in[q];
        io.out[q] = (v2<S> *)out[q];
    }
    hipLaunchKernelGGL((k_apply_A_dom<NT, R, T, S, S, S, NLC>), (unsigned)(g.V / NT), NT * R, 0, s, g, io,
                       (const v2<S> *)links, (const v2<S> *)clov);
}

template <int NT, int R>
static void launch_apply_A_dom(const Geo &g, const void *const *in, void *const *out, const void *links,
                               const void *clov, int prec, hipStream_t s)
{
    if (prec == P64) launch_A_dom<NT, R, double, double, 9>(g, in, out, links, clov, s);
    else if (prec == P32) launch_A_dom<NT, R, float, float, 6>(g, in, out, links, clov, s);
    else if (prec == P16) launch_A_dom<NT, R, float, half_t, 6>(g, in, out, links, clov, s);
    else launch_A_dom<NT, R, float, bf16_t, 6>(g, in, out, links, clov, s);
}

// whole domains per workgroup where the domain size divides the workgroup's
// site count (V is then a multiple of it) and every field is under 4 GiB (the
// largest, links and clover, hold 36 complex numbers per site)
static int dom_sites(const Geo &g, int prec)
{
    const size_t elem = prec == P64 ? 16 : prec == P32 ? 8 : 4;
    if ((size_t)g.V * 36 * elem >= ((size_t)1 << 32)) return 0;
    if (g.Vd <= 256 && 256 % g.Vd == 0 && g.V % 256 == 0) return 256;
    if (g.Vd == 512 && g.V % 512 == 0) return 512;
    return 0;
}

bool apply_A_pairs(const Geo &g, int prec) { return dom_sites(g, prec) == 256; }

hipError_t apply_A_pair(const Geo &g, const void *in0, void *out0, const void *in1, void *out1, const void *links,
                        const void *clov, int prec, hipStream_t s)
{
    if (!apply_A_pairs(g, prec)) return hipErrorInvalidValue;
    const void *in[2] = {in0, in1};
    void *out[2] = {out0, out1};
    launch_apply_A_dom<256, 2>(g, in, out, links, clov, prec, s);
    return hipGetLastError();
}

hipError_t apply_A(const Geo &g, const void *in, void *out, const void *links, const void *clov, int prec,
                   hipStream_t s)
{
    unsigned nb = nblocks(g.V, 256);
    const int nt = dom_sites(g, prec);
    if (nt) {
        const void *ins[1] = {in};
        void *outs[1] = {out};
        if (nt == 256) launch_apply_A_dom<256, 1>(g, ins, outs, links, clov, prec, s);
        else launch_apply_A_dom<512, 1>(g, ins, outs, links, clov, prec, s);
        return hipGetLastError();
    }
    if (prec == P64)
        hipLaunchKernelGGL((k_apply_A<double, double, double, double, 9>), nb, 256, 0, s, g, (const double2 *)in,
                           (double2 *)out, (const double2 *)links, (const double2 *)clov);
    else if (prec == P32)
        hipLaunchKernelGGL((k_apply_A<float, float, float, float, 6>), nb, 256, 0, s, g, (const float2 *)in,
                           (float2 *)out, (const float2 *)links, (const float2 *)clov);
    else if (prec == P16)
        hipLaunchKernelGGL((k_apply_A<float, half_t, half_t, half_t, 6>), nb, 256, 0, s, g, (const half2_t *)in,
                           (half2_t *)out, (const half2_t *)links, (const half2_t *)clov);
    else
        hipLaunchKernelGGL((k_apply_A<float, bf16_t, bf16_t, bf16_t, 6>), nb, 256, 0, s, g, (const bf162_t *)in,
                           (bf162_t *)out, (const bf162_t *)links, (const bf162_t *)clov);
    return hipGetLastError();
}

// ===========================================================================
// FP64 linear algebra (deterministic two-stage reductions)
// ===========================================================================

constexpr int BS = 256;

template <int N> __device__ __forceinline__ void block_reduce_store(double (&v)[N], double2 *dst_pairs)
{
    // wave64 butterfly, then the waves of the block through LDS in fixed order
    __shared__ double red[BS / 64][N];
#pragma unroll
    for (int q = 0; q < N; q++)
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o);
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; q++) red[w][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q + 1 < N + 1; q += 2) {
            double a = 0, b = 0;
            for (int k = 0; k < BS / 64; k++) {
                a += red[k][q];
                if (q + 1 < N) b += red[k][q + 1];
            }
            dst_pairs[q / 2] = make_double2(a, b);
        }
    }
}

// blocks of a BLAS launch over n complex elements: about four elements per
// thread, at most BLAS_NBLK (the size of the partial-sum buffer)
static int blas_blocks(long n)
{
    const long b = (n + 4L * BS - 1) / (4L * BS);
    return (int)(b < 1 ? 1 : b > BLAS_NBLK ? BLAS_NBLK : b);
}

// stage 2: result[j] = sum over blocks of partial[b][j], j < m pairs
__global__ void k_finish(const double2 *partial, int nblk, int m, double2 *result)
{
    __shared__ double2 red[BS];
    for (int j = 0; j < m; j++) {
        double2 s = make_double2(0, 0);
        for (int b = threadIdx.x; b < nblk; b += BS) {
            double2 v = partial[(long)b * 32 + j];
            s.x += v.x;
            s.y += v.y;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = BS / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                red[threadIdx.x].x += red[threadIdx.x + o].x;
                red[threadIdx.x].y += red[threadIdx.x + o].y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) result[j] = red[0];
        __syncthreads();
    }
}

template <int K> __global__ __launch_bounds__(BS) void k_multidot(const double2 *W, long ldw, const double2 *v, long n, double2 *partial)
{
    double acc[2 * K];
#pragma unroll
    for (int q = 0; q < 2 * K; q++) acc[q] = 0;
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        double2 b = v[i];
#pragma unroll
        for (int j = 0; j < K; j++) {
            double2 a = W[j * ldw + i];
            acc[2 * j] += a.x * b.x + a.y * b.y;
            acc[2 * j + 1] += a.x * b.y - a.y * b.x;
        }
    }
    block_reduce_store<2 * K>(acc, partial + (long)blockIdx.x * 32);
}

template <int K> static void launch_multidot(const double2 *W, long ldw, const double2 *v, long n, double2 *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_multidot<K>, blas_blocks(n), BS, 0, s, W, ldw, v, n, partial);
}

hipError_t Blas::init()
{
    hipError_t e = hipMalloc(&partial, sizeof(double2) * BLAS_NBLK * 32);
    if (e == hipSuccess) e = hipMalloc(&result, sizeof(double2) * 32);
    if (e == hipSuccess) e = hipMalloc(&coef, sizeof(double2) * 32);
    return e;
}

void Blas::release()
{
    if (partial) (void)hipFree(partial);
    if (result) (void)hipFree(result);
    if (coef) (void)hipFree(coef);
    partial = result = coef = nullptr;
}

hipError_t multidot(Blas &B, const double2 *W, long ldw, int k, const double2 *v, long n, hipStream_t s)
{
    switch (k) {
#define MD(K) case K: launch_multidot<K>(W, ldw, v, n, B.partial, s); break;
        MD(1) MD(2) MD(3) MD(4) MD(5) MD(6) MD(7) MD(8) MD(9) MD(10) MD(11) MD(12) MD(13) MD(14) MD(15) MD(16)
#undef MD
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), k, B.result);
    return hipGetLastError();
}

template <int K>
__global__ __launch_bounds__(BS) void k_cgs_update(double2 *w, const double2 *W, long ldw, const double2 *coef, const double2 *r,
                                                   long n, double2 *partial)
{
    double2 c[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; j++) c[j] = coef[j];
    double acc[4] = {0, 0, 0, 0};
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        double2 x = w[i];
#pragma unroll
        for (int j = 0; j < K; j++) {
            double2 a = W[j * ldw + i];
            x.x -= c[j].x * a.x - c[j].y * a.y;
            x.y -= c[j].x * a.y + c[j].y * a.x;
        }
        w[i] = x;
        double2 b = r[i];
        acc[0] += x.x * x.x + x.y * x.y;
        acc[2] += x.x * b.x + x.y * b.y;
        acc[3] += x.x * b.y - x.y * b.x;
    }
    block_reduce_store<4>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t cgs_update(Blas &B, double2 *w, const double2 *W, long ldw, int k, const double2 *r, long n, hipStream_t s)
{
    switch (k) {
#define CU(K) case K: hipLaunchKernelGGL(k_cgs_update<K>, blas_blocks(n), BS, 0, s, w, W, ldw, B.coef, r, n, B.partial); break;
        CU(0) CU(1) CU(2) CU(3) CU(4) CU(5) CU(6) CU(7) CU(8) CU(9) CU(10) CU(11) CU(12) CU(13) CU(14) CU(15) CU(16)
#undef CU
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), 2, B.result);
    return hipGetLastError();
}

__global__ __launch_bounds__(BS) void k_residual_update(const double2 *w, double2 *r, double2 c, long n,
                                                        double2 *partial)
{
    double acc[2] = {0, 0};
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        const double2 x = w[i];
        double2 y = r[i];
        y.x -= c.x * x.x - c.y * x.y;
        y.y -= c.x * x.y + c.y * x.x;
        r[i] = y;
        acc[0] += y.x * y.x + y.y * y.y;
    }
    block_reduce_store<2>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t residual_update(Blas &B, const double2 *w, double2 *r, double2 c, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual_update, blas_blocks(n), BS, 0, s, w, r, c, n, B.partial);
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), 1, B.result);
    return hipGetLastError();
}

template <int K> __global__ __launch_bounds__(BS) void k_axpy_multi(double2 *x, const double2 *Z, long ldz, const double2 *coef, long n)
{
    double2 c[K];
#pragma unroll
    for (int j = 0; j < K; j++) c[j] = coef[j];
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        double2 y = x[i];
#pragma unroll
        for (int j = 0; j < K; j++) {
            double2 a = Z[j * ldz + i];
            y.x += c[j].x * a.x - c[j].y * a.y;
            y.y += c[j].x * a.y + c[j].y * a.x;
        }
        x[i] = y;
    }
}

hipError_t axpy_multi(Blas &B, double2 *x, const double2 *Z, long ldz, int k, long n, hipStream_t s)
{
    switch (k) {
#define AX(K) case K: hipLaunchKernelGGL(k_axpy_multi<K>, blas_blocks(n), BS, 0, s, x, Z, ldz, B.coef, n); break;
        AX(1) AX(2) AX(3) AX(4) AX(5) AX(6) AX(7) AX(8) AX(9) AX(10) AX(11) AX(12) AX(13) AX(14) AX(15) AX(16)
#undef AX
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(BS) void k_residual(const double2 *b, double2 *r, long n, double2 *partial)
{
    double acc[2] = {0, 0};
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        double2 y = b[i], a = r[i];
        y.x -= a.x;
        y.y -= a.y;
        r[i] = y;
        acc[0] += y.x * y.x + y.y * y.y;
    }
    block_reduce_store<2>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t residual(Blas &B, const double2 *b, double2 *r, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, blas_blocks(n), BS, 0, s, b, r, n, B.partial);
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), 1, B.result);
    return hipGetLastError();
}

__global__ __launch_bounds__(BS) void k_norm2(const double2 *v, long n, double2 *partial)
{
    double acc[2] = {0, 0};
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        double2 y = v[i];
        acc[0] += y.x * y.x + y.y * y.y;
    }
    block_reduce_store<2>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t norm2(Blas &B, const double2 *v, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm2, blas_blocks(n), BS, 0, s, v, n, B.partial);
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), 1, B.result);
    return hipGetLastError();
}

// result[0] = <t, s>, result[1] = (|t|^2, 0)
__global__ __launch_bounds__(BS) void k_dot2(const double2 *t, const double2 *sv, long n, double2 *partial)
{
    double acc[4] = {0, 0, 0, 0};
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        const double2 a = t[i], b = sv[i];
        acc[0] += a.x * b.x + a.y * b.y;
        acc[1] += a.x * b.y - a.y * b.x;
        acc[2] += a.x * a.x + a.y * a.y;
    }
    block_reduce_store<4>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t dot2(Blas &B, const double2 *t, const double2 *sv, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot2, blas_blocks(n), BS, 0, s, t, sv, n, B.partial);
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), 2, B.result);
    return hipGetLastError();
}

// out = ca a + cb b + cc c (complex coefficients; c may be null; out may alias a, b or c)
__global__ __launch_bounds__(BS) void k_lincomb(double2 *out, const double2 *a, double2 ca, const double2 *b,
                                                double2 cb, const double2 *c, double2 cc, long n)
{
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        const double2 x = a[i], y = b[i];
        double2 o;
        o.x = ca.x * x.x - ca.y * x.y + cb.x * y.x - cb.y * y.y;
        o.y = ca.x * x.y + ca.y * x.x + cb.x * y.y + cb.y * y.x;
        if (c) {
            const double2 z = c[i];
            o.x += cc.x * z.x - cc.y * z.y;
            o.y += cc.x * z.y + cc.y * z.x;
        }
        out[i] = o;
    }
}

hipError_t lincomb(double2 *out, const double2 *a, double2 ca, const double2 *b, double2 cb, const double2 *c,
                   double2 cc, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_lincomb, blas_blocks(n), BS, 0, s, out, a, ca, b, cb, c, cc, n);
    return hipGetLastError();
}

// ---- FP32 vectors with FP64 accumulation (the inner solve of the
// mixed-precision outer solver) ----------------------------------------------

template <int K>
__global__ __launch_bounds__(BS) void k_multidot32(const float2 *W, long ldw, const float2 *v, long n, double2 *partial)
{
    double acc[2 * K];
#pragma unroll
    for (int q = 0; q < 2 * K; q++) acc[q] = 0;
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        const float2 b = v[i];
#pragma unroll
        for (int j = 0; j < K; j++) {
            const float2 a = W[j * ldw + i];
            acc[2 * j] += (double)a.x * b.x + (double)a.y * b.y;
            acc[2 * j + 1] += (double)a.x * b.y - (double)a.y * b.x;
        }
    }
    block_reduce_store<2 * K>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t multidot32(Blas &B, const float2 *W, long ldw, int k, const float2 *v, long n, hipStream_t s)
{
    switch (k) {
#define MD(K) case K: hipLaunchKernelGGL(k_multidot32<K>, blas_blocks(n), BS, 0, s, W, ldw, v, n, B.partial); break;
        MD(1) MD(2) MD(3) MD(4) MD(5) MD(6) MD(7) MD(8) MD(9) MD(10) MD(11) MD(12) MD(13) MD(14) MD(15) MD(16)
#undef MD
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), k, B.result);
    return hipGetLastError();
}

template <int K>
__global__ __launch_bounds__(BS) void k_cgs_update32(float2 *w, const float2 *W, long ldw, const double2 *coef, long n,
                                                     double2 *partial)
{
    double2 c[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; j++) c[j] = coef[j];
    double acc[2] = {0, 0};
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        const float2 x0 = w[i];
        double xr = x0.x, xi = x0.y;
#pragma unroll
        for (int j = 0; j < K; j++) {
            const float2 a = W[j * ldw + i];
            xr -= c[j].x * a.x - c[j].y * a.y;
            xi -= c[j].x * a.y + c[j].y * a.x;
        }
        const float2 x = make_float2((float)xr, (float)xi);
        w[i] = x;
        acc[0] += (double)x.x * x.x + (double)x.y * x.y;
    }
    block_reduce_store<2>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t cgs_update32(Blas &B, float2 *w, const float2 *W, long ldw, int k, long n, hipStream_t s)
{
    switch (k) {
#define CU(K) case K: hipLaunchKernelGGL(k_cgs_update32<K>, blas_blocks(n), BS, 0, s, w, W, ldw, B.coef, n, B.partial); break;
        CU(0) CU(1) CU(2) CU(3) CU(4) CU(5) CU(6) CU(7) CU(8) CU(9) CU(10) CU(11) CU(12) CU(13) CU(14) CU(15) CU(16)
#undef CU
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), 1, B.result);
    return hipGetLastError();
}

// w *= inv_b; then result[0] = <w, r>, after which r -= c w with c = that dot
// is left to k_axpy32 (c is only known on the host)
__global__ __launch_bounds__(BS) void k_scale_dot32(float2 *w, double inv_b, const float2 *r, long n, double2 *partial)
{
    double acc[2] = {0, 0};
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        float2 x = w[i];
        x.x = (float)(x.x * inv_b);
        x.y = (float)(x.y * inv_b);
        w[i] = x;
        const float2 b = r[i];
        acc[0] += (double)x.x * b.x + (double)x.y * b.y;
        acc[1] += (double)x.x * b.y - (double)x.y * b.x;
    }
    block_reduce_store<2>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t scale_dot32(Blas &B, float2 *w, double inv_b, const float2 *r, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_dot32, blas_blocks(n), BS, 0, s, w, inv_b, r, n, B.partial);
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), 1, B.result);
    return hipGetLastError();
}

// r -= c w; result[0] = (|r|^2, 0)
__global__ __launch_bounds__(BS) void k_axpy32(float2 *r, double2 c, const float2 *w, long n, double2 *partial)
{
    double acc[2] = {0, 0};
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        const float2 x = w[i];
        float2 y = r[i];
        y.x = (float)(y.x - (c.x * x.x - c.y * x.y));
        y.y = (float)(y.y - (c.x * x.y + c.y * x.x));
        r[i] = y;
        acc[0] += (double)y.x * y.x + (double)y.y * y.y;
    }
    block_reduce_store<2>(acc, partial + (long)blockIdx.x * 32);
}

hipError_t axpy32(Blas &B, float2 *r, double2 c, const float2 *w, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy32, blas_blocks(n), BS, 0, s, r, c, w, n, B.partial);
    hipLaunchKernelGGL(k_finish, 1, BS, 0, s, B.partial, blas_blocks(n), 1, B.result);
    return hipGetLastError();
}

// x += scale * sum_j coef[j] Z_j (FP64 x, FP32 Z)
template <int K>
__global__ __launch_bounds__(BS) void k_axpy_mixed(double2 *x, const float2 *Z, long ldz, const double2 *coef,
                                                   double scale, long n)
{
    double2 c[K];
#pragma unroll
    for (int j = 0; j < K; j++) c[j] = make_double2(scale * coef[j].x, scale * coef[j].y);
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        double2 y = x[i];
#pragma unroll
        for (int j = 0; j < K; j++) {
            const float2 a = Z[j * ldz + i];
            y.x += c[j].x * a.x - c[j].y * a.y;
            y.y += c[j].x * a.y + c[j].y * a.x;
        }
        x[i] = y;
    }
}

hipError_t axpy_mixed(Blas &B, double2 *x, const float2 *Z, long ldz, int k, double scale, long n, hipStream_t s)
{
    switch (k) {
#define AX(K) case K: hipLaunchKernelGGL(k_axpy_mixed<K>, blas_blocks(n), BS, 0, s, x, Z, ldz, B.coef, scale, n); break;
        AX(1) AX(2) AX(3) AX(4) AX(5) AX(6) AX(7) AX(8) AX(9) AX(10) AX(11) AX(12) AX(13) AX(14) AX(15) AX(16)
#undef AX
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// out = s * in, rounded to FP32
__global__ __launch_bounds__(BS) void k_to_f32(const double2 *in, double sc, float2 *out, long n)
{
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        const double2 v = in[i];
        out[i] = make_float2((float)(sc * v.x), (float)(sc * v.y));
    }
}

hipError_t to_f32(const double2 *in, double sc, float2 *out, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f32, blas_blocks(n), BS, 0, s, in, sc, out, n);
    return hipGetLastError();
}

// out_q = sum_i W_i P[i][q] for q < nq (columns of n complex numbers, W_i =
// W + i*ldw, out_q = out + q*ldo; P row-major nin x nq on the device, nin, nq
// <= RECOMB_MAX).  Each element of the inputs is read once; the outputs of one
// element accumulate in registers.
constexpr int RECOMB_MAX = 24;
__global__ __launch_bounds__(BS) void k_recombine(const double2 *W, long ldw, int nin, const double2 *P, int nq,
                                                  double2 *out, long ldo, long n)
{
    __shared__ double2 sp[RECOMB_MAX * RECOMB_MAX];
    for (int t = threadIdx.x; t < nin * nq; t += BS) sp[t] = P[t];
    __syncthreads();
    for (long e = (long)blockIdx.x * BS + threadIdx.x; e < n; e += (long)gridDim.x * BS) {
        double2 acc[RECOMB_MAX];
#pragma unroll
        for (int q = 0; q < RECOMB_MAX; q++) acc[q] = make_double2(0, 0);
        for (int i = 0; i < nin; i++) {
            const double2 w = W[i * ldw + e];
#pragma unroll
            for (int q = 0; q < RECOMB_MAX; q++) {
                if (q >= nq) break;
                const double2 c = sp[i * nq + q];
                acc[q].x += c.x * w.x - c.y * w.y;
                acc[q].y += c.x * w.y + c.y * w.x;
            }
        }
#pragma unroll
        for (int q = 0; q < RECOMB_MAX; q++) {
            if (q >= nq) break;
            out[q * ldo + e] = acc[q];
        }
    }
}

hipError_t recombine(const double2 *W, long ldw, int nin, const double2 *P, int nq, double2 *out, long ldo, long n,
                     hipStream_t s)
{
    if (nin < 1 || nq < 1 || nin > RECOMB_MAX || nq > RECOMB_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_recombine, blas_blocks(n), BS, 0, s, W, ldw, nin, P, nq, out, ldo, n);
    return hipGetLastError();
}

__global__ void k_zero(double2 *v, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        v[i] = make_double2(0, 0);
}

hipError_t zero(double2 *v, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero, 2048, 256, 0, s, v, n);
    return hipGetLastError();
}

}  // namespace dd
