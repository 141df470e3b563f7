// Device-side building blocks of the Wilson-clover operator on gfx950.
//
// Internal (library-private) data layout, shared by every kernel:
//  * sites are blocked by Schwarz domain: internal index I = d*Vd + loc, with
//    d the lexicographic domain number and loc = parity*Vd/2 + (lexicographic
//    local index >> 1), i.e. even sites first, then odd (all domain extents
//    are even, so local and global site parity agree);
//  * every field is an array of 2-vectors (a complex number, or a pair of
//    reals), component-major inside a domain so that consecutive threads
//    (consecutive loc) touch consecutive addresses:
//      spinor  [d][12 = spin*3+colour][Vd]      complex
//      link    [d][mu][9 or 6][Vd]              complex (full or first two rows)
//      clover  [d][36][Vd]                      real pairs: two packed Hermitian 6x6
//    A packed 6x6 block holds its 6 real diagonal entries as 3 pairs, then
//    the 15 entries below the diagonal, row by row (Sec. II-B: 2 x (6 + 15
//    complex) = 72 reals per site).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dd {

typedef _Float16 half_t;
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16_t;
typedef __bf16 bf162_t __attribute__((ext_vector_type(2)));

template <typename S> struct vec2;
template <> struct vec2<double> { typedef double2 type; };
template <> struct vec2<float> { typedef float2 type; };
template <> struct vec2<half_t> { typedef half2_t type; };
template <> struct vec2<bf16_t> { typedef bf162_t type; };
template <typename S> using v2 = typename vec2<S>::type;

template <typename T> struct cx {
    T r, i;
};

template <typename T> __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T> __device__ __forceinline__ cx<T> scal(T s, cx<T> a) { return {s * a.r, s * a.i}; }
// conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b)
{
    return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
// a * b + c with one rounding
template <typename T> __device__ __forceinline__ T fmad(T a, T b, T c)
{
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}
// acc + a * b and acc + conj(a) * b as chains of fused multiply-adds (two per
// component, where acc + (a * b) costs a multiply, a fused multiply-add and an
// add per component: the sum cannot be fused without reassociating it)
template <typename T> __device__ __forceinline__ cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b)
{
    acc.r = fmad(a.r, b.r, acc.r);
    acc.r = fmad(-a.i, b.i, acc.r);
    acc.i = fmad(a.r, b.i, acc.i);
    acc.i = fmad(a.i, b.r, acc.i);
    return acc;
}
template <typename T> __device__ __forceinline__ cx<T> cmacc(cx<T> acc, cx<T> a, cx<T> b)
{
    acc.r = fmad(a.r, b.r, acc.r);
    acc.r = fmad(a.i, b.i, acc.r);
    acc.i = fmad(a.r, b.i, acc.i);
    acc.i = fmad(-a.i, b.r, acc.i);
    return acc;
}
// -0.0 hidden from the compiler.  a * b + (-0.0) equals a * b exactly for
// every a, b, so products written as fused multiply-adds onto it keep their
// value, and the compiler cannot turn them back into multiplies: with
// reduced-precision operands a multiply needs the operand converted first,
// while a mixed-precision fused multiply-add takes it as stored.
template <typename T> __device__ __forceinline__ T opaque_neg_zero()
{
    T z = T(-0.0);
    asm("" : "+v"(z));
    return z;
}
// a * b as fused multiply-adds onto -0.0 (the same value as a * b, see above)
template <typename T> __device__ __forceinline__ cx<T> cmul_f(cx<T> a, cx<T> b, T z)
{
    return {fmad(a.r, b.r, -fmad(a.i, b.i, z)), fmad(a.r, b.i, fmad(a.i, b.r, z))};
}
template <typename T> __device__ __forceinline__ cx<T> cmulc_f(cx<T> a, cx<T> b, T z)
{
    return {fmad(a.r, b.r, fmad(a.i, b.i, z)), fmad(a.r, b.i, -fmad(a.i, b.r, z))};
}
template <typename T> __device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.i, a.r}; }
template <typename T> __device__ __forceinline__ cx<T> times_mi(cx<T> a) { return {a.i, -a.r}; }
template <typename T> __device__ __forceinline__ cx<T> neg(cx<T> a) { return {-a.r, -a.i}; }
template <typename T> __device__ __forceinline__ cx<T> czero() { return {T(0), T(0)}; }

// ---- loads and stores with precision conversion -------------------------

template <typename T, typename S> __device__ __forceinline__ cx<T> ld(const v2<S> *p, long idx)
{
    v2<S> v = p[idx];
    return {static_cast<T>(v.x), static_cast<T>(v.y)};
}
template <typename T, typename S> __device__ __forceinline__ void st(v2<S> *p, long idx, cx<T> a)
{
    v2<S> v;
    v.x = static_cast<S>(a.r);
    v.y = static_cast<S>(a.i);
    p[idx] = v;
}
// The same at a 32-bit byte offset from the array's base (arrays under 4 GiB):
// one VGPR per address, and a uniform base can stay in SGPRs.
template <typename T, typename S> __device__ __forceinline__ cx<T> ld32(const v2<S> *p, unsigned idx)
{
    const v2<S> v = *(const v2<S> *)((const char *)p + idx * (unsigned)sizeof(v2<S>));
    return {static_cast<T>(v.x), static_cast<T>(v.y)};
}
template <typename T, typename S> __device__ __forceinline__ void st32(v2<S> *p, unsigned idx, cx<T> a)
{
    v2<S> v;
    v.x = static_cast<S>(a.r);
    v.y = static_cast<S>(a.i);
    *(v2<S> *)((char *)p + idx * (unsigned)sizeof(v2<S>)) = v;
}

// ---- SU(3) ---------------------------------------------------------------

template <typename T> struct su3 {
    cx<T> m[9];
};

// Loads U with NLC stored complex entries per link (9: all rows; 6: rows 0
// and 1, row 2 rebuilt as conj(row0 x row1), exact for SU(3)); load(e)
// returns stored entry e.
template <typename T, int NLC, typename Load> __device__ __forceinline__ su3<T> ld_link_with(Load load)
{
    su3<T> U;
#pragma unroll
    for (int e = 0; e < NLC; e++) U.m[e] = load(e);
    if constexpr (NLC == 6) {
        const cx<T> *a = U.m, *b = U.m + 3;
        U.m[6] = {a[1].r * b[2].r - a[1].i * b[2].i - a[2].r * b[1].r + a[2].i * b[1].i,
                  -(a[1].r * b[2].i + a[1].i * b[2].r - a[2].r * b[1].i - a[2].i * b[1].r)};
        U.m[7] = {a[2].r * b[0].r - a[2].i * b[0].i - a[0].r * b[2].r + a[0].i * b[2].i,
                  -(a[2].r * b[0].i + a[2].i * b[0].r - a[0].r * b[2].i - a[0].i * b[2].r)};
        U.m[8] = {a[0].r * b[1].r - a[0].i * b[1].i - a[1].r * b[0].r + a[1].i * b[0].i,
                  -(a[0].r * b[1].i + a[0].i * b[1].r - a[1].r * b[0].i - a[1].i * b[0].r)};
    }
    return U;
}

template <typename T, typename G, int NLC>
__device__ __forceinline__ su3<T> ld_link(const v2<G> *p, long base, long stride)
{
    return ld_link_with<T, NLC>([&](int e) { return ld<T, G>(p, base + e * stride); });
}

// out[s][a] = sum_b U[a][b] h[s][b]   (two spin components of a half-spinor)
template <typename T> __device__ __forceinline__ void su3_mul(const su3<T> &U, const cx<T> h[6], cx<T> out[6])
{
    const T z = opaque_neg_zero<T>();
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int a = 0; a < 3; a++)
            out[s * 3 + a] = cmac(cmac(cmul_f(U.m[a * 3 + 0], h[s * 3 + 0], z), U.m[a * 3 + 1], h[s * 3 + 1]),
                                  U.m[a * 3 + 2], h[s * 3 + 2]);
}

// out[s][a] = sum_b conj(U[b][a]) h[s][b]
template <typename T> __device__ __forceinline__ void su3_dag_mul(const su3<T> &U, const cx<T> h[6], cx<T> out[6])
{
    const T z = opaque_neg_zero<T>();
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int a = 0; a < 3; a++)
            out[s * 3 + a] = cmacc(cmacc(cmulc_f(U.m[0 * 3 + a], h[s * 3 + 0], z), U.m[1 * 3 + a], h[s * 3 + 1]),
                                   U.m[2 * 3 + a], h[s * 3 + 2]);
}

// ---- spin projection in the chiral basis ----------------------------------
//
// gamma_k = [[0, -i s_k], [i s_k, 0]] (k = x, y, z), gamma_t = [[0, -1], [-1, 0]].
// With psi = (u; l) split into spins {0,1} and {2,3}, (1 -+ gamma_mu) psi has
// rank two: its upper half h is a 2-spinor and its lower half is a fixed
// multiple of h.  SG = -1 is the forward projector (1 - gamma_mu), SG = +1
// the backward projector (1 + gamma_mu).

template <int MU, int SG, typename T> __device__ __forceinline__ void proj(const cx<T> s[12], cx<T> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<T> u0 = s[c], u1 = s[3 + c], l0 = s[6 + c], l1 = s[9 + c];
        if constexpr (MU == 0) {
            if constexpr (SG < 0) { h[c] = u0 + times_i(l1); h[3 + c] = u1 + times_i(l0); }
            else { h[c] = u0 - times_i(l1); h[3 + c] = u1 - times_i(l0); }
        } else if constexpr (MU == 1) {
            if constexpr (SG < 0) { h[c] = u0 + l1; h[3 + c] = u1 - l0; }
            else { h[c] = u0 - l1; h[3 + c] = u1 + l0; }
        } else if constexpr (MU == 2) {
            if constexpr (SG < 0) { h[c] = u0 + times_i(l0); h[3 + c] = u1 - times_i(l1); }
            else { h[c] = u0 - times_i(l0); h[3 + c] = u1 + times_i(l1); }
        } else {
            if constexpr (SG < 0) { h[c] = u0 + l0; h[3 + c] = u1 + l1; }
            else { h[c] = u0 - l0; h[3 + c] = u1 - l1; }
        }
    }
}

// out += k * (h; lower(h)), the full spinor whose projection is h
template <int MU, int SG, typename T>
__device__ __forceinline__ void recon_acc(cx<T> out[12], const cx<T> h[6], T k)
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<T> h0 = scal(k, h[c]), h1 = scal(k, h[3 + c]);
        out[c] = out[c] + h0;
        out[3 + c] = out[3 + c] + h1;
        cx<T> l0, l1;
        if constexpr (MU == 0) {
            if constexpr (SG < 0) { l0 = times_mi(h1); l1 = times_mi(h0); }
            else { l0 = times_i(h1); l1 = times_i(h0); }
        } else if constexpr (MU == 1) {
            if constexpr (SG < 0) { l0 = neg(h1); l1 = h0; }
            else { l0 = h1; l1 = neg(h0); }
        } else if constexpr (MU == 2) {
            if constexpr (SG < 0) { l0 = times_mi(h0); l1 = times_i(h1); }
            else { l0 = times_i(h0); l1 = times_mi(h1); }
        } else {
            if constexpr (SG < 0) { l0 = h0; l1 = h1; }
            else { l0 = neg(h0); l1 = neg(h1); }
        }
        out[6 + c] = out[6 + c] + l0;
        out[9 + c] = out[9 + c] + l1;
    }
}

// ---- packed Hermitian 6x6 clover blocks ----------------------------------

__host__ __device__ constexpr int tri_index(int i, int j) { return i * (i - 1) / 2 + j; }  // i > j

// out[0..5] = M in[0..5] for one packed block; load(q) returns its pair q
template <typename T, typename Load>
__device__ __forceinline__ void clover_block_with(Load load, const cx<T> in[6], cx<T> out[6])
{
    T dg[6];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        cx<T> v = load(q);
        dg[2 * q] = v.r;
        dg[2 * q + 1] = v.i;
    }
#pragma unroll
    for (int i = 0; i < 6; i++) out[i] = scal(dg[i], in[i]);
#pragma unroll
    for (int i = 1; i < 6; i++)
#pragma unroll
        for (int j = 0; j < i; j++) {
            cx<T> m = load(3 + tri_index(i, j));
            out[i] = cmac(out[i], m, in[j]);
            out[j] = cmacc(out[j], m, in[i]);
        }
}

template <typename T, typename G>
__device__ __forceinline__ void clover_block(const v2<G> *p, long base, long stride, const cx<T> in[6], cx<T> out[6])
{
    clover_block_with<T>([&](int q) { return ld<T, G>(p, base + q * stride); }, in, out);
}

template <typename T, typename G>
__device__ __forceinline__ void clover_apply(const v2<G> *p, long base, long stride, const cx<T> in[12], cx<T> out[12])
{
    clover_block<T, G>(p, base, stride, in, out);
    clover_block<T, G>(p, base + 18 * stride, stride, in + 6, out + 6);
}

// ---- lattice geometry -----------------------------------------------------

struct Geo {
    int L[4];
    int b[4];
    int n[4];
    int Vd, Vh, nd;
    long V;
    double bc[4];
};

__device__ __forceinline__ void decode(const Geo &g, long I, int x[4], int &d, int &loc)
{
    d = (int)(I / g.Vd);
    loc = (int)(I - (long)d * g.Vd);
    int p = loc >= g.Vh;
    int h = loc - p * g.Vh;
    int bxh = g.b[0] >> 1;
    int row = h / bxh;
    int xh = h - row * bxh;
    int l1 = row % g.b[1];
    row /= g.b[1];
    int l2 = row % g.b[2];
    int l3 = row / g.b[2];
    int l0 = 2 * xh + ((p + l1 + l2 + l3) & 1);
    int r = d;
    int D0 = r % g.n[0]; r /= g.n[0];
    int D1 = r % g.n[1]; r /= g.n[1];
    int D2 = r % g.n[2];
    int D3 = r / g.n[2];
    x[0] = D0 * g.b[0] + l0;
    x[1] = D1 * g.b[1] + l1;
    x[2] = D2 * g.b[2] + l2;
    x[3] = D3 * g.b[3] + l3;
}

__host__ __device__ __forceinline__ long encode(const Geo &g, const int x[4])
{
    int D[4], l[4];
#pragma unroll
    for (int m = 0; m < 4; m++) {
        D[m] = x[m] / g.b[m];
        l[m] = x[m] - D[m] * g.b[m];
    }
    int d = D[0] + g.n[0] * (D[1] + g.n[1] * (D[2] + g.n[2] * D[3]));
    int Ll = l[0] + g.b[0] * (l[1] + g.b[1] * (l[2] + g.b[2] * l[3]));
    int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    return (long)d * g.Vd + p * g.Vh + (Ll >> 1);
}

}  // namespace dd
