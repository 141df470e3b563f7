// One half-sweep of the Schwarz alternating procedure (multiplicative
// Schwarz, Sec. II-D and the algorithm of Table I): every domain of one colour
// solves D_Omega delta = rho_Omega approximately and adds delta to the
// solution.  One workgroup per domain, one thread per site; the spinors the
// block solve exchanges between sites live in LDS for the whole solve.
//
// Residual bookkeeping.  After a domain's block solve its residual is known
// exactly: the MR residual on the even sites and zero on the odd sites
// (Sec. II-D, Eq. 5).  Between two solves of a domain only its neighbours
// (the other colour) change the solution, by their own delta, so the domain
// next sees
//     rho = stored block residual - R delta_neighbours .
// Each domain therefore stores, after its solve, its block residual and the
// boundary half-spinors of its delta (the terms of R that its neighbours
// need: (1 - gamma_mu) delta on its -mu face, U_mu^dagger (1 + gamma_mu) delta
// on its +mu face), and gathers its neighbours' at the start of its next
// solve.  This is the paper's packed boundary buffers (Sec. III-A) with the
// gather done by the reading domain, so no two workgroups write the same
// address and no atomics are needed.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

template <int BX, int BY, int BZ, int BT> struct Shape {
    static constexpr int VD = BX * BY * BZ * BT;
    static constexpr int VH = VD / 2;
    // threads of a one-domain block-solve workgroup: whole waves (idle padding
    // threads beyond VD) for domains of 64 sites or more
    static constexpr int NT = VD >= 64 ? (VD + 63) / 64 * 64 : VD;
    static constexpr int B[4] = {BX, BY, BZ, BT};
    static constexpr int FS[4] = {VD / BX, VD / BY, VD / BZ, VD / BT};
    static constexpr int FTOT = 2 * (VD / BX + VD / BY + VD / BZ + VD / BT);
    static_assert(BX % 2 == 0 && BY % 2 == 0 && BZ % 2 == 0 && BT % 2 == 0, "domain extents must be even");

    // face f = 2*mu + side (side 0: l_mu = 0, side 1: l_mu = B_mu - 1)
    static constexpr int foff(int f)
    {
        int o = 0;
        for (int q = 0; q < f; q++) o += FS[q >> 1];
        return o;
    }
    __device__ static void coords(int loc, int l[4])
    {
        int p = loc >= VH;
        int h = loc - p * VH;
        int xh = h % (BX / 2);
        int row = h / (BX / 2);
        l[1] = row % BY;
        row /= BY;
        l[2] = row % BZ;
        l[3] = row / BZ;
        l[0] = 2 * xh + ((p + l[1] + l[2] + l[3]) & 1);
    }
    // index within the half-lattice of the site's own parity
    __device__ static int half_index(const int l[4]) { return (l[0] + BX * (l[1] + BY * (l[2] + BZ * l[3]))) >> 1; }
    template <int MU> __device__ static int face_index(const int l[4])
    {
        if constexpr (MU == 0) return l[1] + BY * (l[2] + BZ * l[3]);
        else if constexpr (MU == 1) return l[0] + BX * (l[2] + BZ * l[3]);
        else if constexpr (MU == 2) return l[0] + BX * (l[1] + BY * l[3]);
        else return l[0] + BX * (l[1] + BY * l[2]);
    }
};

// ---- block reductions over all VD threads (deterministic order) -----------

// Sum over the 64 lanes of a wave, returned to every lane (all lanes active):
// DPP permutes within each 16-lane row (lane ^ 1, lane ^ 2, then the mirrored
// halves of 8 and of 16 lanes) leave every lane with its row's sum; the four
// row sums are read out and added.
__device__ __forceinline__ float wave_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));  // row_half_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));  // row_mirror
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int VD, typename T, int N> __device__ __forceinline__ void block_sum(T (&v)[N], T *red)
{
    if constexpr (VD >= 64) {
        constexpr int NW = VD / 64;
#pragma unroll
        for (int q = 0; q < N; q++) v[q] = wave_sum(v[q]);
        int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int q = 0; q < N; q++) red[q * NW + w] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < N; q++) {
            T s = 0;
            for (int k = 0; k < NW; k++) s += red[q * NW + k];
            v[q] = s;
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int q = 0; q < N; q++) red[q * VD + threadIdx.x] = v[q];
        __syncthreads();
        for (int o = VD / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o)
#pragma unroll
                for (int q = 0; q < N; q++) red[q * VD + threadIdx.x] += red[q * VD + threadIdx.x + o];
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < N; q++) v[q] = red[q * VD];
        __syncthreads();
    }
}

template <int VD, typename T> __device__ __forceinline__ T block_max(T v, T *red)
{
    if constexpr (VD >= 64) {
        constexpr int NW = VD / 64;
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        T m = red[0];
        for (int k = 1; k < NW; k++) m = fmax(m, red[k]);
        __syncthreads();
        return m;
    } else {
        red[threadIdx.x] = v;
        __syncthreads();
        for (int o = VD / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
            __syncthreads();
        }
        T m = red[0];
        __syncthreads();
        return m;
    }
}

// Reductions over the sites of each domain when NDW domains share a
// workgroup: wave 0 holds the even sites and wave 1 the odd sites of all NDW
// domains (NDW * VD / 2 = 64), VD / 2 consecutive lanes per domain.
template <int VD, int NDW, typename T, int N> __device__ __forceinline__ void slot_sum(T (&v)[N], T *red)
{
    if constexpr (NDW == 1) {
        block_sum<VD, T, N>(v, red);
    } else {
        constexpr int VH = VD / 2;
        static_assert(NDW * VH == 64, "one wave per parity");
#pragma unroll
        for (int q = 0; q < N; q++)
            for (int o = VH / 2; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o);
        const int par = threadIdx.x >> 6, sub = (threadIdx.x & 63) / VH;
        if ((threadIdx.x % VH) == 0)
#pragma unroll
            for (int q = 0; q < N; q++) red[(q * 2 + par) * NDW + sub] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < N; q++) v[q] = red[(q * 2) * NDW + sub] + red[(q * 2 + 1) * NDW + sub];
        __syncthreads();
    }
}

template <int VD, int NDW, typename T> __device__ __forceinline__ T slot_max(T v, T *red)
{
    if constexpr (NDW == 1) {
        return block_max<VD, T>(v, red);
    } else {
        constexpr int VH = VD / 2;
        static_assert(NDW * VH == 64, "one wave per parity");
        for (int o = VH / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        const int par = threadIdx.x >> 6, sub = (threadIdx.x & 63) / VH;
        if ((threadIdx.x % VH) == 0) red[par * NDW + sub] = v;
        __syncthreads();
        const T m = fmax(red[sub], red[NDW + sub]);
        __syncthreads();
        return m;
    }
}

// smallest power of two >= m (m > 0), 1 for m == 0
template <typename T> __device__ __forceinline__ T pow2_ceil(T m)
{
    if (!(m > T(0))) return T(1);
    int e;
    T f = frexp(m, &e);   // m = f * 2^e, f in [0.5, 1)
    (void)f;
    return ldexp(T(1), e);
}

template <typename T> __device__ __forceinline__ T maxabs12(const cx<T> a[12])
{
    T m = 0;
#pragma unroll
    for (int k = 0; k < 12; k++) m = fmax(m, fmax(fabs(a[k].r), fabs(a[k].i)));
    return m;
}

// ---- in-domain hopping terms from an LDS half-lattice spinor --------------
//
// acc += sum over in-domain neighbours of (1 - gamma_mu) U_mu(x) v(x+mu) and
// (1 + gamma_mu) U_mu(x-mu)^dagger v(x-mu); the -1/2 of Eq. 1 is applied by
// the caller.  v holds the sites of the other parity.

template <class Sh, int MU, typename T, typename G, int NLC>
__device__ __forceinline__ void dom_hop(const cx<T> (*v)[Sh::VH], const int l[4], long lbase, int loc,
                                        const v2<G> *links, cx<T> acc[12], T scale = T(1))
{
    constexpr int VD = Sh::VD;
    int n[4] = {l[0], l[1], l[2], l[3]};
    cx<T> s[12], h[6], uh[6];
    if (l[MU] + 1 < Sh::B[MU]) {
        n[MU] = l[MU] + 1;
        int nh = Sh::half_index(n);
#pragma unroll
        for (int k = 0; k < 12; k++) s[k] = v[k][nh];
        proj<MU, -1>(s, h);
        su3<T> U = ld_link<T, G, NLC>(links, lbase + (long)MU * NLC * VD + loc, VD);
        su3_mul(U, h, uh);
        recon_acc<MU, -1>(acc, uh, scale);
    }
    if (l[MU] > 0) {
        n[MU] = l[MU] - 1;
        int nh = Sh::half_index(n);
        int nloc = (1 - (loc >= Sh::VH)) * Sh::VH + nh;
#pragma unroll
        for (int k = 0; k < 12; k++) s[k] = v[k][nh];
        proj<MU, +1>(s, h);
        su3<T> U = ld_link<T, G, NLC>(links, lbase + (long)MU * NLC * VD + nloc, VD);
        su3_dag_mul(U, h, uh);
        recon_acc<MU, +1>(acc, uh, scale);
    }
}

template <class Sh, typename T, typename G, int NLC>
__device__ __forceinline__ void dom_hops(const cx<T> (*v)[Sh::VH], const int l[4], long lbase, int loc,
                                         const v2<G> *links, cx<T> acc[12])
{
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = czero<T>();
    dom_hop<Sh, 0, T, G, NLC>(v, l, lbase, loc, links, acc);
    dom_hop<Sh, 1, T, G, NLC>(v, l, lbase, loc, links, acc);
    dom_hop<Sh, 2, T, G, NLC>(v, l, lbase, loc, links, acc);
    dom_hop<Sh, 3, T, G, NLC>(v, l, lbase, loc, links, acc);
}

// The hop sum of every site of parity po, shared by the site's thread pair:
// the thread of parity po takes directions 0 and 1 of its own site, the thread
// of the other parity with the same half index takes directions 2 and 3 of
// that site (partner coordinates lp, index locp) and hands its partial sum over
// through X ([12][VH] in LDS).  XFREE: nothing reads X during the hops, so the
// partial is written at once; otherwise after a barrier.  Every thread of the
// workgroup calls this (it holds barriers); on return the po thread's acc is
// the whole sum, the other thread's acc is its own partial.
template <class Sh, typename T, typename G, int NLC, bool XFREE>
__device__ __forceinline__ void pair_hops(const cx<T> (*v)[Sh::VH], cx<T> (*X)[Sh::VH], int po, int par, int hi,
                                          const int l[4], int loc, const int lp[4], int locp, long lbase,
                                          const v2<G> *links, cx<T> acc[12])
{
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = czero<T>();
    if (par == po) {
        dom_hop<Sh, 0, T, G, NLC>(v, l, lbase, loc, links, acc);
        dom_hop<Sh, 1, T, G, NLC>(v, l, lbase, loc, links, acc);
    } else if (par == 1 - po) {
        dom_hop<Sh, 2, T, G, NLC>(v, lp, lbase, locp, links, acc);
        dom_hop<Sh, 3, T, G, NLC>(v, lp, lbase, locp, links, acc);
        if constexpr (XFREE)
#pragma unroll
            for (int k = 0; k < 12; k++) X[k][hi] = acc[k];
    }
    if constexpr (!XFREE) {
        __syncthreads();
        if (par == 1 - po)
#pragma unroll
            for (int k = 0; k < 12; k++) X[k][hi] = acc[k];
    }
    __syncthreads();
    if (par == po)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = acc[k] + X[k][hi];
}

// A uniform pointer the compiler must treat as unknown from here on: the
// addresses derived from it are formed at their use instead of being
// precomputed and held in registers across loops.
template <typename P> __device__ __forceinline__ P opaque(P p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// acc (= 0 first if ZERO) += scale * (in-domain hops), directions visited in
// a loop that is not unrolled: one direction's temporaries live at a time
// (fewer registers)
template <class Sh, typename T, typename G, int NLC, bool ZERO>
__device__ __forceinline__ void dom_hops_rolled(const cx<T> (*v)[Sh::VH], const int l[4], long lbase, int loc,
                                                const v2<G> *links, cx<T> acc[12], T scale)
{
    if constexpr (ZERO)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = czero<T>();
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++) {
        const v2<G> *lk = opaque(links);
        switch (mu) {
            case 0: dom_hop<Sh, 0, T, G, NLC>(v, l, lbase, loc, lk, acc, scale); break;
            case 1: dom_hop<Sh, 1, T, G, NLC>(v, l, lbase, loc, lk, acc, scale); break;
            case 2: dom_hop<Sh, 2, T, G, NLC>(v, l, lbase, loc, lk, acc, scale); break;
            default: dom_hop<Sh, 3, T, G, NLC>(v, l, lbase, loc, lk, acc, scale); break;
        }
    }
}

// pair_hops with the directions visited in a loop that is not unrolled and a
// scale: the po thread's acc (zeroed first if ZERO) gains scale x its share
// and then the helper's; the helper's acc is zeroed and takes its share.
template <class Sh, typename T, typename G, int NLC, bool XFREE, bool ZERO>
__device__ __forceinline__ void pair_hops_rolled(const cx<T> (*v)[Sh::VH], cx<T> (*X)[Sh::VH], int po, int par,
                                                 int hi, const int l[4], int loc, const int lp[4], int locp,
                                                 long lbase, const v2<G> *links, cx<T> acc[12], T scale)
{
    const bool own = par == po, help = par == 1 - po;
    if (ZERO || !own)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = czero<T>();
    if (own || help) {
        int ls[4];
#pragma unroll
        for (int q = 0; q < 4; q++) ls[q] = own ? l[q] : lp[q];
        const int ss = own ? loc : locp;
#pragma unroll 1
        for (int mu = own ? 0 : 2; mu < (own ? 2 : 4); mu++) {
            const v2<G> *lk = opaque(links);
            switch (mu) {
                case 0: dom_hop<Sh, 0, T, G, NLC>(v, ls, lbase, ss, lk, acc, scale); break;
                case 1: dom_hop<Sh, 1, T, G, NLC>(v, ls, lbase, ss, lk, acc, scale); break;
                case 2: dom_hop<Sh, 2, T, G, NLC>(v, ls, lbase, ss, lk, acc, scale); break;
                default: dom_hop<Sh, 3, T, G, NLC>(v, ls, lbase, ss, lk, acc, scale); break;
            }
        }
    }
    if constexpr (XFREE) {
        if (help)
#pragma unroll
            for (int k = 0; k < 12; k++) X[k][hi] = acc[k];
    } else {
        __syncthreads();
        if (help)
#pragma unroll
            for (int k = 0; k < 12; k++) X[k][hi] = acc[k];
    }
    __syncthreads();
    if (own)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = acc[k] + X[k][hi];
}

// ---- boundary terms --------------------------------------------------------

template <class Sh> __device__ __forceinline__ long face_base(int d, int f) { return ((long)d * Sh::FTOT + Sh::foff(f)) * 6; }

// rho += 1/2 phi * (the hop from the neighbouring domain across each face)
template <class Sh, int MU, typename T, typename SS, typename G, int NLC, bool SCALED>
__device__ __forceinline__ void gather_face(const SapArgs &a, const int D[4], int d, const int l[4], int loc,
                                            cx<T> rho[12])
{
    constexpr int VD = Sh::VD;
    const v2<SS> *face = (const v2<SS> *)a.face_in;
    int Dn[4] = {D[0], D[1], D[2], D[3]};
    cx<T> h[6];
    if (l[MU] == 0) {
        // backward hop from x - mu, in the -mu neighbour's +mu face
        bool wrap = D[MU] == 0;
        Dn[MU] = wrap ? a.g.n[MU] - 1 : D[MU] - 1;
        int dn = Dn[0] + a.g.n[0] * (Dn[1] + a.g.n[1] * (Dn[2] + a.g.n[2] * Dn[3]));
        T sc = SCALED ? T(a.face_in_scale[dn]) : T(1);
        long fb = face_base<Sh>(dn, 2 * MU + 1);
        int fi = Sh::template face_index<MU>(l);
#pragma unroll
        for (int k = 0; k < 6; k++) h[k] = scal(sc, ld<T, SS>(face, fb + (long)k * Sh::FS[MU] + fi));
        recon_acc<MU, +1>(rho, h, T(wrap ? 0.5 * a.g.bc[MU] : 0.5));
    } else if (l[MU] == Sh::B[MU] - 1) {
        // forward hop from x + mu, in the +mu neighbour's -mu face
        bool wrap = D[MU] == a.g.n[MU] - 1;
        Dn[MU] = wrap ? 0 : D[MU] + 1;
        int dn = Dn[0] + a.g.n[0] * (Dn[1] + a.g.n[1] * (Dn[2] + a.g.n[2] * Dn[3]));
        T sc = SCALED ? T(a.face_in_scale[dn]) : T(1);
        long fb = face_base<Sh>(dn, 2 * MU);
        int fi = Sh::template face_index<MU>(l);
#pragma unroll
        for (int k = 0; k < 6; k++) h[k] = scal(sc, ld<T, SS>(face, fb + (long)k * Sh::FS[MU] + fi));
        cx<T> uh[6];
        su3<T> U = ld_link<T, G, NLC>((const v2<G> *)a.links, ((long)d * 4 + MU) * NLC * VD + loc, VD);
        su3_mul(U, h, uh);
        recon_acc<MU, -1>(rho, uh, T(wrap ? 0.5 * a.g.bc[MU] : 0.5));
    }
}

// gather_face for all four directions at once, split in two steps so that
// the boundary loads of every direction are in flight together: face_fetch
// loads the site's boundary half-spinor along MU (if it has one) and its
// weight, face_apply adds its contribution.
template <class Sh, int MU, typename T, typename SS, bool SCALED>
__device__ __forceinline__ void face_fetch(const SapArgs &a, const int D[4], const int l[4], cx<T> h[6], T &w,
                                           int &side)
{
    const bool bwd = l[MU] == 0, fwd = l[MU] == Sh::B[MU] - 1;
    side = bwd ? 1 : fwd ? 2 : 0;
    if (!(bwd || fwd)) return;
    const v2<SS> *face = (const v2<SS> *)a.face_in;
    int Dn[4] = {D[0], D[1], D[2], D[3]};
    const bool wrap = bwd ? D[MU] == 0 : D[MU] == a.g.n[MU] - 1;
    Dn[MU] = bwd ? (wrap ? a.g.n[MU] - 1 : D[MU] - 1) : (wrap ? 0 : D[MU] + 1);
    const int dn = Dn[0] + a.g.n[0] * (Dn[1] + a.g.n[1] * (Dn[2] + a.g.n[2] * Dn[3]));
    // backward hop: the -mu neighbour's +mu face; forward: the +mu neighbour's -mu face
    const long fb = face_base<Sh>(dn, 2 * MU + (bwd ? 1 : 0));
    const int fi = Sh::template face_index<MU>(l);
#pragma unroll
    for (int k = 0; k < 6; k++) h[k] = ld<T, SS>(face, fb + (long)k * Sh::FS[MU] + fi);
    const T sc = SCALED ? T(a.face_in_scale[dn]) : T(1);
    w = sc * T(wrap ? 0.5 * a.g.bc[MU] : 0.5);
}

template <class Sh, int MU, typename T, typename G, int NLC, int LNLC, bool FROM_LDS, int LSTR = Sh::VD>
__device__ __forceinline__ void face_apply(const SapArgs &a, int d, int loc, const v2<G> *slink, const cx<T> h[6],
                                           T w, int side, cx<T> rho[12])
{
    constexpr int VD = Sh::VD;
    if (side == 1) {
        recon_acc<MU, +1>(rho, h, w);
    } else if (side == 2) {
        cx<T> uh[6];
        su3<T> U;
        if constexpr (FROM_LDS) U = ld_link<T, G, LNLC>(slink, (long)MU * LNLC * LSTR + loc, LSTR);
        else U = ld_link<T, G, NLC>((const v2<G> *)a.links, ((long)d * 4 + MU) * NLC * VD + loc, VD);
        su3_mul(U, h, uh);
        recon_acc<MU, -1>(rho, uh, w);
    }
}

template <class Sh, int MU, typename T, typename SS, typename G, int NLC, int LNLC = NLC, bool FROM_LDS = false,
          int LSTR = Sh::VD>
__device__ __forceinline__ void write_face(const SapArgs &a, int d, const int l[4], int loc, const cx<T> delta[12],
                                           T inv_sc, const v2<G> *slink = nullptr)
{
    constexpr int VD = Sh::VD;
    v2<SS> *face = (v2<SS> *)a.face;
    cx<T> h[6];
    if (l[MU] == 0) {
        proj<MU, -1>(delta, h);
        long fb = face_base<Sh>(d, 2 * MU);
        int fi = Sh::template face_index<MU>(l);
#pragma unroll
        for (int k = 0; k < 6; k++) st<T, SS>(face, fb + (long)k * Sh::FS[MU] + fi, scal(inv_sc, h[k]));
    } else if (l[MU] == Sh::B[MU] - 1) {
        cx<T> uh[6];
        proj<MU, +1>(delta, h);
        // FROM_LDS: the domain's links staged in slink ([mu][LNLC][LSTR]), else global
        su3<T> U;
        if constexpr (FROM_LDS) U = ld_link<T, G, LNLC>(slink, (long)MU * LNLC * LSTR + loc, LSTR);
        else U = ld_link<T, G, NLC>((const v2<G> *)a.links, ((long)d * 4 + MU) * NLC * VD + loc, VD);
        su3_dag_mul(U, h, uh);
        long fb = face_base<Sh>(d, 2 * MU + 1);
        int fi = Sh::template face_index<MU>(l);
#pragma unroll
        for (int k = 0; k < 6; k++) st<T, SS>(face, fb + (long)k * Sh::FS[MU] + fi, scal(inv_sc, uh[k]));
    }
}

// ---- the half-sweep kernel --------------------------------------------------
//
// One workgroup per domain, one thread per (even site, odd site) pair: thread
// t owns the even site with half-lattice index t and the odd site with
// half-lattice index t, so in every phase of the block solve (which works on
// one parity at a time) all threads are busy.  The MR residual r of the even
// site stays in registers; the MR solution x, the odd-site right-hand side
// rho_o and the exchanged half-lattice spinors live in LDS.
//
// T: arithmetic; SS: storage of the block residual and the boundary terms;
// PS: storage of the solution accumulator; G: storage of links and clover;
// RHO_LDS: keep rho_o in LDS (else in a per-domain global buffer, used when
// four FP64 half-lattice spinors would not fit in LDS).

template <class Sh, typename T, typename SS, typename G, int NLC, bool SCALED>
__device__ __forceinline__ void stage_site(const SapArgs &a, const int D[4], int d, const int l[4], int loc,
                                           cx<T> rho[12])
{
    constexpr int VD = Sh::VD, VH = Sh::VH;
    const long sidx = (long)d * 12 * VD + loc;
    if (a.first) {
#pragma unroll
        for (int k = 0; k < 12; k++) rho[k] = ld<T, double>(a.eta, sidx + (long)k * VD);
    } else if (loc < VH) {
        T sc = SCALED ? T(a.res_scale[d]) : T(1);
        const v2<SS> *res = (const v2<SS> *)a.res;
#pragma unroll
        for (int k = 0; k < 12; k++) rho[k] = scal(sc, ld<T, SS>(res, ((long)d * 12 + k) * VH + loc));
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) rho[k] = czero<T>();
    }
    if (a.faces_in) {
        gather_face<Sh, 0, T, SS, G, NLC, SCALED>(a, D, d, l, loc, rho);
        gather_face<Sh, 1, T, SS, G, NLC, SCALED>(a, D, d, l, loc, rho);
        gather_face<Sh, 2, T, SS, G, NLC, SCALED>(a, D, d, l, loc, rho);
        gather_face<Sh, 3, T, SS, G, NLC, SCALED>(a, D, d, l, loc, rho);
    }
}

template <class Sh, typename T, typename SS, typename PS, typename G, int NLC>
__device__ __forceinline__ void write_site(const SapArgs &a, int d, const int l[4], int loc, const cx<T> delta[12],
                                           T inv_face_sc)
{
    constexpr int VD = Sh::VD;
    const long sidx = (long)d * 12 * VD + loc;
    const v2<PS> *psi_in = (const v2<PS> *)a.psi;
    v2<PS> *psi_out = (v2<PS> *)a.psi;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        cx<T> ps = a.first ? delta[k] : ld<T, PS>(psi_in, sidx + (long)k * VD) + delta[k];
        if (a.last) st<T, double>(a.out, sidx + (long)k * VD, ps);
        else st<T, PS>(psi_out, sidx + (long)k * VD, ps);
    }
    if (a.faces_out) {
        write_face<Sh, 0, T, SS, G, NLC>(a, d, l, loc, delta, inv_face_sc);
        write_face<Sh, 1, T, SS, G, NLC>(a, d, l, loc, delta, inv_face_sc);
        write_face<Sh, 2, T, SS, G, NLC>(a, d, l, loc, delta, inv_face_sc);
        write_face<Sh, 3, T, SS, G, NLC>(a, d, l, loc, delta, inv_face_sc);
    }
}

template <class Sh, typename T, typename SS, typename PS, typename G, int NLC, bool SCALED, bool RHO_LDS>
__device__ __forceinline__ void pair_block_solve(const SapArgs &a, const int d)
{
    constexpr int VD = Sh::VD, VH = Sh::VH;
    __shared__ cx<T> she[12][VH];                                  // even-site spinor being hopped
    __shared__ cx<T> sho[12][VH];                                  // odd-site spinor being hopped
    __shared__ cx<T> shx[12][VH];                                  // MR solution on the even sites
    __shared__ cx<T> shr[RHO_LDS ? 12 : 1][RHO_LDS ? VH : 1];      // rho on the odd sites
    __shared__ T red[VH >= 64 ? 3 * (VH / 64) : 3 * VH];

    const int t = threadIdx.x;
    const int loc_e = t, loc_o = VH + t;
    int le[4], lo[4];
    Sh::coords(loc_e, le);
    Sh::coords(loc_o, lo);
    int D[4];
    {
        int r = d;
        D[0] = r % a.g.n[0]; r /= a.g.n[0];
        D[1] = r % a.g.n[1]; r /= a.g.n[1];
        D[2] = r % a.g.n[2];
        D[3] = r / a.g.n[2];
    }
    const v2<G> *links = (const v2<G> *)a.links;
    const v2<G> *cs = (const v2<G> *)a.cs;
    const long lbase = (long)d * 4 * NLC * VD;
    const long cbase = (long)d * 36 * VD;
    v2<T> *rho_g = (v2<T> *)a.rho_tmp;

    cx<T> r[12], P[12];

    // ---- staging (Sec. II-D: the residual restricted to the domain)
    {
        cx<T> ro[12];
        stage_site<Sh, T, SS, G, NLC, SCALED>(a, D, d, lo, loc_o, ro);
        // odd part of the preparation: C_o^-1 rho_o
        clover_apply<T, G>(cs, cbase + loc_o, VD, ro, P);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            sho[k][t] = P[k];
            if constexpr (RHO_LDS) shr[k][t] = ro[k];
            else st<T, T>(rho_g, ((long)d * 12 + k) * VH + t, ro[k]);
            shx[k][t] = czero<T>();
        }
    }
    stage_site<Sh, T, SS, G, NLC, SCALED>(a, D, d, le, loc_e, r);
    __syncthreads();
    // r = rho_e - D_eo C_o^-1 rho_o  (D_eo = -1/2 hops)
    dom_hops<Sh, T, G, NLC>(sho, le, lbase, loc_e, links, P);
#pragma unroll
    for (int k = 0; k < 12; k++) r[k] = r[k] + scal(T(0.5), P[k]);

    // ---- minimal residual on the Schur complement C_e - D_eo C_o^-1 D_oe
    for (int it = 0; it < a.n_mr; it++) {
#pragma unroll
        for (int k = 0; k < 12; k++) she[k][t] = r[k];
        __syncthreads();
        {
            cx<T> q[12];
            dom_hops<Sh, T, G, NLC>(she, lo, lbase, loc_o, links, q);
#pragma unroll
            for (int k = 0; k < 12; k++) q[k] = scal(T(-0.5), q[k]);   // D_oe r
            clover_apply<T, G>(cs, cbase + loc_o, VD, q, P);           // C_o^-1 D_oe r
#pragma unroll
            for (int k = 0; k < 12; k++) sho[k][t] = P[k];
        }
        __syncthreads();
        T dots[3] = {0, 0, 0};
        {
            cx<T> q[12];
            dom_hops<Sh, T, G, NLC>(sho, le, lbase, loc_e, links, q);
            clover_apply<T, G>(cs, cbase + loc_e, VD, r, P);           // C_e r
#pragma unroll
            for (int k = 0; k < 12; k++) {
                P[k] = P[k] + scal(T(0.5), q[k]);                      // p = C_e r - D_eo C_o^-1 D_oe r
                dots[0] = fmad(P[k].i, r[k].i, fmad(P[k].r, r[k].r, dots[0]));
                dots[1] = fmad(-P[k].i, r[k].r, fmad(P[k].r, r[k].i, dots[1]));
                dots[2] = fmad(P[k].i, P[k].i, fmad(P[k].r, P[k].r, dots[2]));
            }
        }
        block_sum<VH, T, 3>(dots, red);
        const cx<T> alpha = dots[2] > T(0) ? cx<T>{dots[0] / dots[2], dots[1] / dots[2]} : czero<T>();
#pragma unroll
        for (int k = 0; k < 12; k++) {
            shx[k][t] = cmac(shx[k][t], alpha, r[k]);
            r[k] = cmac(r[k], neg(alpha), P[k]);
        }
    }
    __syncthreads();

    // ---- odd sites: delta_o = C_o^-1 (rho_o - D_oe x)
    {
        cx<T> q[12];
        dom_hops<Sh, T, G, NLC>(shx, lo, lbase, loc_o, links, q);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<T> ro;
            if constexpr (RHO_LDS) ro = shr[k][t];
            else ro = ld<T, T>(rho_g, ((long)d * 12 + k) * VH + t);
            q[k] = ro + scal(T(0.5), q[k]);
        }
        clover_apply<T, G>(cs, cbase + loc_o, VD, q, P);               // P = delta_o
    }

    // ---- epilogue: psi += delta, stored residual, boundary terms
    T face_sc = T(1);
    if (a.res_out) {
        T sc = T(1);
        if constexpr (SCALED) {
            sc = pow2_ceil(block_max<VH, T>(maxabs12(r), red));
            if (t == 0) a.res_scale[d] = (float)sc;
        }
        v2<SS> *res = (v2<SS> *)a.res;
        T inv = T(1) / sc;
#pragma unroll
        for (int k = 0; k < 12; k++) st<T, SS>(res, ((long)d * 12 + k) * VH + t, scal(inv, r[k]));
    }
#pragma unroll
    for (int k = 0; k < 12; k++) r[k] = shx[k][t];                    // r <- delta_e
    if (a.faces_out) {
        if constexpr (SCALED) {
            face_sc = T(8) * pow2_ceil(block_max<VH, T>(fmax(maxabs12(r), maxabs12(P)), red));
            if (t == 0) a.face_scale[d] = (float)face_sc;
        }
    }
    write_site<Sh, T, SS, PS, G, NLC>(a, d, lo, loc_o, P, T(1) / face_sc);
    write_site<Sh, T, SS, PS, G, NLC>(a, d, le, loc_e, r, T(1) / face_sc);
}

// ---- the LDS-resident half-sweep kernel (FP32 arithmetic) -----------------
//
// One workgroup per domain, one thread per site.  At the start of the block
// solve the domain's links are staged once into LDS and each thread loads its
// own site's clover block (C on even sites, C^-1 on odd sites) into
// registers, so the MR steps read no global memory at all: the hopping terms
// take the neighbour spinor and the link from LDS, the site terms from
// registers.  x and r of the even sites and rho/delta of the odd sites stay in
// the registers of the site's own thread.

template <typename T, typename G>
__device__ __forceinline__ void clover_block_reg(const v2<G> *c, const cx<T> in[6], cx<T> out[6])
{
    const T z = opaque_neg_zero<T>();
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const T d0 = static_cast<T>(c[q].x), d1 = static_cast<T>(c[q].y);
        out[2 * q] = {fmad(d0, in[2 * q].r, z), fmad(d0, in[2 * q].i, z)};
        out[2 * q + 1] = {fmad(d1, in[2 * q + 1].r, z), fmad(d1, in[2 * q + 1].i, z)};
    }
#pragma unroll
    for (int i = 1; i < 6; i++)
#pragma unroll
        for (int j = 0; j < i; j++) {
            v2<G> mv = c[3 + tri_index(i, j)];
            cx<T> m = {static_cast<T>(mv.x), static_cast<T>(mv.y)};
            out[i] = cmac(out[i], m, in[j]);
            out[j] = cmacc(out[j], m, in[i]);
        }
}

template <typename T, typename G>
__device__ __forceinline__ void clover_reg(const v2<G> cl[36], const cx<T> in[12], cx<T> out[12])
{
    clover_block_reg<T, G>(cl, in, out);
    clover_block_reg<T, G>(cl + 18, in + 6, out + 6);
}

// T: arithmetic; SS: storage of the block residual and faces; PS: storage of
// the solution accumulator; G: links and clover; NLC: complex numbers stored
// per link (6: two rows, 9: full).  LINK_LDS stages the domain's links into
// LDS (else they are read from global memory at each use); CL_REG keeps the
// site's clover block in registers (else it is read from global memory).
//
// NDW domains share a workgroup (NDW > 1 for domains of fewer than 64 sites):
// wave 0 then holds the even sites and wave 1 the odd sites of all of them,
// so each phase of the even-odd MR step runs one full wave; d is the calling
// thread's domain.
//
// LNLC: complex numbers per link kept in LDS (6, as stored, or 9: the third
// row rebuilt once at staging instead of at every use).
template <class Sh, int NDW, typename T, typename SS, typename PS, typename G, int NLC, int LNLC, bool SCALED,
          bool LINK_LDS, bool CL_REG>
__device__ __forceinline__ void lds_block_solve(const SapArgs &a, const int d, const Visit f)
{
    constexpr int VD = Sh::VD, VH = Sh::VH;
    constexpr int NT = NDW > 1 ? NDW * VD : Sh::NT;   // threads of the workgroup
    constexpr int RV = NDW > 1 ? VD : NT;             // reduction width argument
    constexpr int HNLC = LINK_LDS ? LNLC : NLC;   // link layout the hops read
    static_assert(NDW == 1 || NDW * VH == 64, "packed domains: one wave per parity");
    static_assert(LNLC == NLC || (LNLC == 9 && NLC == 6), "links in LDS: as stored, or two rows made three");
    __shared__ v2<G> slink_all[NDW][LINK_LDS ? 4 * LNLC * VD : 1];   // [mu][LNLC][VD] per domain
    __shared__ cx<T> she_all[NDW][12][VH];
    __shared__ cx<T> sho_all[NDW][12][VH];
    __shared__ T red[NDW > 1 ? 6 * NDW : NT >= 64 ? 3 * (NT / 64) : 3 * NT];

    const int par = (int)threadIdx.x / (NDW * VH);
    const int idx = (int)threadIdx.x - par * (NDW * VH);
    const int sub = idx / VH;   // this thread's domain within the workgroup
    const int hi = idx - sub * VH;
    const int loc = par * VH + hi;
    // padding threads (threadIdx >= VD, only when VD is not a multiple of 64)
    // take part in barriers and reductions with zeros and touch no memory
    const bool live = NDW > 1 || NT == VD || (int)threadIdx.x < VD;
    v2<G> *slink = slink_all[sub];
    cx<T>(*she)[VH] = she_all[sub];
    cx<T>(*sho)[VH] = sho_all[sub];
    int l[4];
    Sh::coords(loc, l);
    // the site of the other parity with the same half index: its hops in
    // directions 2 and 3 are this thread's share of its hop sums
    const int locp = (1 - par) * VH + hi;
    int lp[4];
    Sh::coords(par < 2 ? locp : loc, lp);
    int D[4];
    {
        int r = d;
        D[0] = r % a.g.n[0]; r /= a.g.n[0];
        D[1] = r % a.g.n[1]; r /= a.g.n[1];
        D[2] = r % a.g.n[2];
        D[3] = r / a.g.n[2];
    }
    const v2<G> *glinks = (const v2<G> *)a.links;
    const v2<G> *cs = (const v2<G> *)a.cs;
    const long sbase = (long)d * 12 * VD + loc;

    // ---- stage the links into LDS, the site's clover block into registers.
    // Every global load is issued before the first LDS store: the loads go
    // through generic pointers, so a load placed after an LDS store must wait
    // for it, and with loads and stores interleaved each load would wait for
    // the previous one's data.
    const v2<G> *links = slink;
    long lbase = 0;
    v2<G> lt[LINK_LDS ? 4 * NLC : 1];
    if constexpr (LINK_LDS) {
        if (live) {
            const long lb = (long)d * 4 * NLC * VD + loc;
#pragma unroll
            for (int q = 0; q < 4 * NLC; q++) lt[q] = glinks[lb + (long)q * VD];
        }
    } else {
        links = glinks;
        lbase = (long)d * 4 * NLC * VD;
    }
    const long cbase = (long)d * 36 * VD + loc;
    v2<G> cl[CL_REG ? 36 : 1];
    if constexpr (CL_REG) {
#pragma unroll
        for (int q = 0; q < 36; q++) cl[q] = live ? cs[cbase + (long)q * VD] : v2<G>{};
    }
    if (!live) {
    } else if constexpr (LINK_LDS && LNLC == NLC) {
#pragma unroll
        for (int q = 0; q < 4 * NLC; q++) slink[q * VD + loc] = lt[q];
    } else if constexpr (LINK_LDS) {
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            const su3<T> U = ld_link<T, G, NLC>(lt + mu * NLC, 0, 1);
#pragma unroll
            for (int e = 0; e < 9; e++) st<T, G>(slink, (long)(mu * 9 + e) * VD + loc, U.m[e]);
        }
    }
    // this site's clover block (C_e on even sites, C_o^-1 on odd sites) times in
    auto clover = [&](const cx<T> in[12], cx<T> out[12]) {
        if constexpr (CL_REG) clover_reg<T, G>(cl, in, out);
        else clover_apply<T, G>(cs, cbase, VD, in, out);
    };

    // A: even sites x (MR solution), odd sites rho_o then delta_o
    cx<T> A[12], P[12];
    if (!live) {
#pragma unroll
        for (int k = 0; k < 12; k++) A[k] = czero<T>();
    } else if (f.first) {
        if (a.io32) {
#pragma unroll
            for (int k = 0; k < 12; k++) A[k] = ld<T, float>((const float2 *)a.eta, sbase + (long)k * VD);
        } else {
#pragma unroll
            for (int k = 0; k < 12; k++) A[k] = ld<T, double>(a.eta, sbase + (long)k * VD);
        }
    } else if (par == 0) {
        T sc = SCALED ? T(a.res_scale[d]) : T(1);
        const v2<SS> *res = (const v2<SS> *)a.res;
#pragma unroll
        for (int k = 0; k < 12; k++) A[k] = scal(sc, ld<T, SS>(res, ((long)d * 12 + k) * VH + hi));
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) A[k] = czero<T>();
    }
    if (f.faces_in && live) {
        cx<T> hf[4][6];
        T wf[4] = {0, 0, 0, 0};
        int sf[4];
        face_fetch<Sh, 0, T, SS, SCALED>(a, D, l, hf[0], wf[0], sf[0]);
        face_fetch<Sh, 1, T, SS, SCALED>(a, D, l, hf[1], wf[1], sf[1]);
        face_fetch<Sh, 2, T, SS, SCALED>(a, D, l, hf[2], wf[2], sf[2]);
        face_fetch<Sh, 3, T, SS, SCALED>(a, D, l, hf[3], wf[3], sf[3]);
        face_apply<Sh, 0, T, G, NLC, LNLC, LINK_LDS>(a, d, loc, slink, hf[0], wf[0], sf[0], A);
        face_apply<Sh, 1, T, G, NLC, LNLC, LINK_LDS>(a, d, loc, slink, hf[1], wf[1], sf[1], A);
        face_apply<Sh, 2, T, G, NLC, LNLC, LINK_LDS>(a, d, loc, slink, hf[2], wf[2], sf[2], A);
        face_apply<Sh, 3, T, G, NLC, LNLC, LINK_LDS>(a, d, loc, slink, hf[3], wf[3], sf[3], A);
    }

    // ---- even-odd preparation: r = rho_e - D_eo C_o^-1 rho_o, x = 0
    if (par == 1) {
        clover(A, P);
#pragma unroll
        for (int k = 0; k < 12; k++) sho[k][hi] = P[k];
    }
    __syncthreads();   // also publishes slink
    // the even-site MR residual r lives in its own slot of she for the whole
    // solve (fewer live registers); x stays in the registers of A.  she is
    // free until r is written, so it carries the odd threads' partial sums.
    pair_hops<Sh, T, G, HNLC, true>(sho, she, 0, par, hi, l, loc, lp, locp, lbase, links, P);
    if (par == 0) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            she[k][hi] = A[k] + scal(T(0.5), P[k]);
            A[k] = czero<T>();
        }
    }

    // ---- minimal residual on the Schur complement
#pragma unroll 1
    for (int it = 0; it < a.n_mr; it++) {
        if constexpr (CL_REG && sizeof(v2<G>) == 4) {
            // keep the clover block in its 16-bit storage form: stops the
            // compiler from hoisting its widening out of the loop, which would
            // double the registers it occupies
#pragma unroll
            for (int q = 0; q < 36; q++) asm volatile("" : "+v"(cl[q]));
        }
        __syncthreads();
        // sho is dead here (its last readers passed the reduction's barriers),
        // so it carries the even threads' partial sums
        cx<T> t[12];
        pair_hops<Sh, T, G, HNLC, true>(she, sho, 1, par, hi, l, loc, lp, locp, lbase, links, t);
        if (par == 1) {
#pragma unroll
            for (int k = 0; k < 12; k++) t[k] = scal(T(-0.5), t[k]);   // D_oe r
            clover(t, P);                                // C_o^-1 D_oe r
#pragma unroll
            for (int k = 0; k < 12; k++) sho[k][hi] = P[k];
        } else if (par == 0) {
            // meanwhile the even sites form C_e r, which needs only r
            cx<T> rr[12];
#pragma unroll
            for (int k = 0; k < 12; k++) rr[k] = she[k][hi];
            clover(rr, P);
        }
        __syncthreads();
        T dots[3] = {0, 0, 0};
        pair_hops<Sh, T, G, HNLC, false>(sho, sho, 0, par, hi, l, loc, lp, locp, lbase, links, t);
        if (par == 0) {
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const cx<T> rk = she[k][hi];
                P[k] = P[k] + scal(T(0.5), t[k]);
                dots[0] = fmad(P[k].i, rk.i, fmad(P[k].r, rk.r, dots[0]));
                dots[1] = fmad(-P[k].i, rk.r, fmad(P[k].r, rk.i, dots[1]));
                dots[2] = fmad(P[k].i, P[k].i, fmad(P[k].r, P[k].r, dots[2]));
            }
        }
        slot_sum<RV, NDW, T, 3>(dots, red);
        if (par == 0) {
            cx<T> alpha = dots[2] > T(0) ? cx<T>{dots[0] / dots[2], dots[1] / dots[2]} : czero<T>();
#pragma unroll
            for (int k = 0; k < 12; k++) {
                cx<T> rk = she[k][hi];
                A[k] = cmac(A[k], alpha, rk);
                she[k][hi] = cmac(rk, neg(alpha), P[k]);
            }
        }
    }

    // ---- odd sites: delta_o = C_o^-1 (rho_o - D_oe x); x goes through sho
    // (free since the last reduction), she keeps r for the epilogue
    if (par == 0)
#pragma unroll
        for (int k = 0; k < 12; k++) sho[k][hi] = A[k];
    __syncthreads();
    {
        cx<T> t[12];
        pair_hops<Sh, T, G, HNLC, false>(sho, sho, 1, par, hi, l, loc, lp, locp, lbase, links, t);
        if (par == 1) {
#pragma unroll
            for (int k = 0; k < 12; k++) t[k] = A[k] + scal(T(0.5), t[k]);
            clover(t, A);
        }
    }

    // ---- epilogue
    if (live) {
        const v2<PS> *psi_in = (const v2<PS> *)a.psi;
        v2<PS> *psi_out = (v2<PS> *)a.psi;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<T> ps = f.first ? A[k] : ld<T, PS>(psi_in, sbase + (long)k * VD) + A[k];
            if (f.last && a.io32) st<T, float>((float2 *)a.out, sbase + (long)k * VD, ps);
            else if (f.last) st<T, double>(a.out, sbase + (long)k * VD, ps);
            else st<T, PS>(psi_out, sbase + (long)k * VD, ps);
        }
    }
    if (f.res_out) {
        cx<T> rr[12];
#pragma unroll
        for (int k = 0; k < 12; k++) rr[k] = par == 0 ? she[k][hi] : czero<T>();
        T sc = T(1);
        if constexpr (SCALED) {
            sc = pow2_ceil(slot_max<RV, NDW, T>(maxabs12(rr), red));
            if (loc == 0) a.res_scale[d] = (float)sc;
        }
        if (par == 0) {
            v2<SS> *res = (v2<SS> *)a.res;
            T inv = T(1) / sc;
#pragma unroll
            for (int k = 0; k < 12; k++) st<T, SS>(res, ((long)d * 12 + k) * VH + hi, scal(inv, rr[k]));
        }
    }
    if (f.faces_out) {
        T sc = T(1);
        if constexpr (SCALED) {
            sc = T(8) * pow2_ceil(slot_max<RV, NDW, T>(maxabs12(A), red));
            if (loc == 0) a.face_scale[d] = (float)sc;
        }
        T inv = T(1) / sc;
        if (live) {
            write_face<Sh, 0, T, SS, G, NLC, LNLC, LINK_LDS>(a, d, l, loc, A, inv, slink);
            write_face<Sh, 1, T, SS, G, NLC, LNLC, LINK_LDS>(a, d, l, loc, A, inv, slink);
            write_face<Sh, 2, T, SS, G, NLC, LNLC, LINK_LDS>(a, d, l, loc, A, inv, slink);
            write_face<Sh, 3, T, SS, G, NLC, LNLC, LINK_LDS>(a, d, l, loc, A, inv, slink);
        }
    }
}


// ---- the FP64 block solve for domains of 256 and more sites -------------------
//
// The same schedule as lds_block_solve (one workgroup per domain, one thread
// per site, Schur complement MR on the even sites), laid out for FP64's
// register cost: the even-site r and x live in LDS, links and clover blocks
// are read from global memory at each use (they stay in the L1/L2 caches
// within a block solve), the odd-site right-hand side is parked in global
// memory until the reconstruction, and the hop directions are visited in a
// loop, so no thread holds more than two 12-component vectors at a time.

template <class Sh>
__device__ __forceinline__ void f64_block_solve(const SapArgs &a, const int d, const Visit f)
{
    using T = double;
    using G = double;
    constexpr int VD = Sh::VD, VH = Sh::VH, NLC = 9;
    __shared__ cx<T> she[12][VH];   // even sites: MR residual r
    __shared__ cx<T> sho[12][VH];   // odd sites: C_o^-1 D_oe r
    __shared__ cx<T> shx[12][VH];   // even sites: MR solution x
    __shared__ T red[VD >= 64 ? 3 * (VD / 64) : 3 * VD];

    const int loc = threadIdx.x;
    const int par = loc >= VH;
    const int hi = loc - par * VH;
    int l[4];
    Sh::coords(loc, l);
    // the site of the other parity with the same half index (its hops in
    // directions 2 and 3 are this thread's share)
    const int locp = (1 - par) * VH + hi;
    int lp[4];
    Sh::coords(locp, lp);
    int D[4];
    {
        int r = d;
        D[0] = r % a.g.n[0]; r /= a.g.n[0];
        D[1] = r % a.g.n[1]; r /= a.g.n[1];
        D[2] = r % a.g.n[2];
        D[3] = r / a.g.n[2];
    }
    const v2<G> *links = (const v2<G> *)a.links;
    const long lbase = (long)d * 4 * NLC * VD;
    const v2<G> *cs = (const v2<G> *)a.cs;
    const long cbase = (long)d * 36 * VD + loc;
    v2<T> *rho_g = (v2<T> *)a.rho_tmp;
    const long sbase = (long)d * 12 * VD + loc;

    // ---- the block right-hand side rho
    cx<T> A[12], P[12];
    if (f.first) {
#pragma unroll
        for (int k = 0; k < 12; k++) A[k] = ld<T, double>(a.eta, sbase + (long)k * VD);
    } else if (par == 0) {
        const v2<T> *res = (const v2<T> *)a.res;
#pragma unroll
        for (int k = 0; k < 12; k++) A[k] = ld<T, T>(res, ((long)d * 12 + k) * VH + hi);
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) A[k] = czero<T>();
    }
    if (f.faces_in) {
        gather_face<Sh, 0, T, T, G, NLC, false>(a, D, d, l, loc, A);
        gather_face<Sh, 1, T, T, G, NLC, false>(a, D, d, l, loc, A);
        gather_face<Sh, 2, T, T, G, NLC, false>(a, D, d, l, loc, A);
        gather_face<Sh, 3, T, T, G, NLC, false>(a, D, d, l, loc, A);
    }

    // ---- even-odd preparation: r = rho_e - D_eo C_o^-1 rho_o, x = 0
    if (par == 1) {
        clover_apply<T, G>(opaque(cs), cbase, VD, A, P);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            sho[k][hi] = P[k];
            st<T, T>(rho_g, ((long)d * 12 + k) * VH + hi, A[k]);
        }
    }
    __syncthreads();
    // she is free until r is written: it carries the odd threads' partial sums
    pair_hops_rolled<Sh, T, G, NLC, true, true>(sho, she, 0, par, hi, l, loc, lp, locp, lbase, links, P, T(0.5));
    if (par == 0) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            she[k][hi] = A[k] + P[k];
            shx[k][hi] = czero<T>();
        }
    }

    // ---- minimal residual on the Schur complement
#pragma unroll 1
    for (int it = 0; it < a.n_mr; it++) {
        __syncthreads();
        // sho is dead here (its readers passed the reduction's barriers): it
        // carries the even threads' partial sums
        pair_hops_rolled<Sh, T, G, NLC, true, true>(she, sho, 1, par, hi, l, loc, lp, locp, lbase, links, P,
                                                    T(-0.5));   // D_oe r
        if (par == 1) {
            clover_apply<T, G>(opaque(cs), cbase, VD, P, A);                                       // C_o^-1 D_oe r
#pragma unroll
            for (int k = 0; k < 12; k++) sho[k][hi] = A[k];
        } else {
            // meanwhile the even sites form C_e r, which needs only r
#pragma unroll
            for (int k = 0; k < 12; k++) A[k] = she[k][hi];
            clover_apply<T, G>(opaque(cs), cbase, VD, A, P);                                       // C_e r
        }
        __syncthreads();
        T dots[3] = {0, 0, 0};
        pair_hops_rolled<Sh, T, G, NLC, false, false>(sho, sho, 0, par, hi, l, loc, lp, locp, lbase, links, P,
                                                      T(0.5));   // - D_eo C_o^-1 D_oe r
        if (par == 0) {
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const cx<T> rk = she[k][hi];
                dots[0] = fmad(P[k].i, rk.i, fmad(P[k].r, rk.r, dots[0]));
                dots[1] = fmad(-P[k].i, rk.r, fmad(P[k].r, rk.i, dots[1]));
                dots[2] = fmad(P[k].i, P[k].i, fmad(P[k].r, P[k].r, dots[2]));
            }
        }
        block_sum<VD, T, 3>(dots, red);
        if (par == 0) {
            const cx<T> alpha = dots[2] > T(0) ? cx<T>{dots[0] / dots[2], dots[1] / dots[2]} : czero<T>();
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const cx<T> rk = she[k][hi];
                shx[k][hi] = cmac(shx[k][hi], alpha, rk);
                she[k][hi] = cmac(rk, neg(alpha), P[k]);
            }
        }
    }
    __syncthreads();

    // ---- delta: x on even sites, C_o^-1 (rho_o - D_oe x) on odd sites
    // x moves to the even threads' registers; shx then carries their partial sums
    if (par == 1) {
#pragma unroll
        for (int k = 0; k < 12; k++) P[k] = ld<T, T>(rho_g, ((long)d * 12 + k) * VH + hi);
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) A[k] = shx[k][hi];
    }
    pair_hops_rolled<Sh, T, G, NLC, false, false>(shx, shx, 1, par, hi, l, loc, lp, locp, lbase, links, P, T(0.5));
    if (par == 1) clover_apply<T, G>(opaque(cs), cbase, VD, P, A);

    // ---- epilogue: psi += delta, stored residual, boundary terms
    {
        const v2<T> *psi_in = (const v2<T> *)a.psi;
        v2<T> *psi_out = (v2<T> *)a.psi;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const cx<T> ps = f.first ? A[k] : ld<T, T>(psi_in, sbase + (long)k * VD) + A[k];
            if (f.last) st<T, double>(a.out, sbase + (long)k * VD, ps);
            else st<T, T>(psi_out, sbase + (long)k * VD, ps);
        }
    }
    if (f.res_out && par == 0) {
        v2<T> *res = (v2<T> *)a.res;
#pragma unroll
        for (int k = 0; k < 12; k++) st<T, T>(res, ((long)d * 12 + k) * VH + hi, she[k][hi]);
    }
    if (f.faces_out) {
        write_face<Sh, 0, T, T, G, NLC>(a, d, l, loc, A, T(1));
        write_face<Sh, 1, T, T, G, NLC>(a, d, l, loc, A, T(1));
        write_face<Sh, 2, T, T, G, NLC>(a, d, l, loc, A, T(1));
        write_face<Sh, 3, T, T, G, NLC>(a, d, l, loc, A, T(1));
    }
}

// The boundary terms a visit reads (face_in) and writes (face): one buffer for
// the multiplicative schedule (the two colours alternate), two alternating
// buffers for the additive one (all domains read the previous cycle's terms
// while writing their own).
__device__ __forceinline__ void bind_faces(SapArgs &a, const Visit &v)
{
    if (a.face_alt) {
        if (v.flip) {
            a.face_in = a.face;
            a.face_in_scale = a.face_scale;
            a.face = a.face_alt;
            a.face_scale = a.face_scale_alt;
        } else {
            a.face_in = a.face_alt;
            a.face_in_scale = a.face_scale_alt;
        }
    } else {
        a.face_in = a.face;
        a.face_in_scale = a.face_scale;
    }
}

// ---- batched half-sweeps ------------------------------------------------------
//
// One launch covers one colour of one half-sweep for many systems (right-hand
// sides and lattices of one domain shape): workgroup i takes item i = (system,
// domain) and that system's arguments.  Items with system < 0 are padding;
// systems with active == 0 (already converged) are skipped.

// With NDW > 1, items come in runs of NDW domains of one system (the plan
// never splits or pads a run), and workgroup i takes run i.
template <class Sh, int NDW, typename T, typename SS, typename PS, typename G, int NLC, int LNLC, bool SCALED,
          bool LINK_LDS, bool CL_REG>
__global__ __launch_bounds__(NDW > 1 ? Sh::VD * NDW : Sh::NT) void k_sap_lds(const SapArgs *args, const int2 *items,
                                                                             Visit v)
{
    const int2 it = items[(long)blockIdx.x * NDW];
    if (it.x < 0) return;
    SapArgs a = args[it.x];
    if (!a.active) return;
    bind_faces(a, v);
    int d = it.y;
    if constexpr (NDW > 1) d = items[(long)blockIdx.x * NDW + ((int)threadIdx.x & 63) / Sh::VH].y;
    lds_block_solve<Sh, NDW, T, SS, PS, G, NLC, LNLC, SCALED, LINK_LDS, CL_REG>(a, d, v);
}

template <class Sh>
__global__ __launch_bounds__(Sh::VD) void k_sap_f64(const SapArgs *args, const int2 *items, Visit v)
{
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    SapArgs a = args[it.x];
    if (!a.active) return;
    bind_faces(a, v);
    f64_block_solve<Sh>(a, it.y, v);
}

template <class Sh, typename T, typename SS, typename PS, typename G, int NLC, bool SCALED, bool RHO_LDS>
__global__ __launch_bounds__(Sh::VH) void k_sap_sweep(const SapArgs *args, const int2 *items, Visit v)
{
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    SapArgs a = args[it.x];
    if (!a.active) return;
    bind_faces(a, v);
    a.first = v.first;
    a.faces_in = v.faces_in;
    a.last = v.last;
    a.faces_out = v.faces_out;
    a.res_out = v.res_out;
    pair_block_solve<Sh, T, SS, PS, G, NLC, SCALED, RHO_LDS>(a, it.y);
}

// ---- dispatch ---------------------------------------------------------------

// ---- block solves of a tile of right-hand sides ---------------------------------
//
// One workgroup solves one domain for a tile of up to RT = 4 right-hand sides
// of one lattice (systems sys0 .. sys0 + nt - 1), so the domain's links are
// staged into LDS once for the tile and each link entry read from LDS serves
// all of them.  Thread t works on the even and the odd site with half index
// h = t / 4 for right-hand side r = t % 4, so the four threads of a site are
// four consecutive lanes, and every thread is busy in both parity phases of
// the MR step.  Spinors in LDS are [component][half index][right-hand side].
//
// Those four lanes are one 4x4 block of the 16-block MFMA instructions.  In
// a hop, the SU(3) product U h (U the link or its adjoint, h the projected
// half-spinor) is, in real form, a 6x6 matrix (rows Re y_a and Im y_a, columns
// Re h_b and Im h_b) times a 6-vector; for the four right-hand sides and one
// spin component of h it is a 6x6 times 6x4 product, done as two 4-row blocks
// of the site's quad: lane r supplies row r of each block of U and column r
// (its own half-spinor), and receives column r of the result.  PROD selects
// the product: VALU (per-thread fused multiply-adds, as in k_sap_lds), FP32
// MFMA (4x4x1, six steps over the inner dimension) or BF16-input MFMA with
// FP32 accumulation (4x4x4, two steps; the link and half-spinor rounded to
// BF16).  Lanes of right-hand sides beyond the tile work on zeros and touch no
// memory.

enum { PROD_VALU = 0, PROD_MFMA_F32 = 1, PROD_MFMA_BF16 = 2 };
constexpr int RT = 4;
// Link entries in LDS lie LSTR = VD + 16 entries apart: the four lanes of a
// quad read four different entries of one site (rows or columns of U for the
// matrix operands), and with a stride of VD (a multiple of the 64 banks) all
// four would fall in one bank.
template <class Sh> constexpr int tile_lstr() { return Sh::VD + 16; }

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));

// sum of v over the threads of this thread's right-hand side (lanes with equal
// lane % 4), for all NW waves of the workgroup; fixed order, every thread joins
template <int NW, int N> __device__ __forceinline__ void rhs_sum(float (&v)[N], float *red)
{
#pragma unroll
    for (int q = 0; q < N; q++)
#pragma unroll
        for (int o = 4; o < 64; o <<= 1) v[q] += __shfl_xor(v[q], o);
    const int w = threadIdx.x >> 6, r = threadIdx.x & 3;
    if ((threadIdx.x & 63) < RT)
#pragma unroll
        for (int q = 0; q < N; q++) red[(w * RT + r) * N + q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; q++) {
        float s = 0;
        for (int k = 0; k < NW; k++) s += red[(k * RT + r) * N + q];
        v[q] = s;
    }
    // no closing barrier: the MR step's next two barriers pass before red is
    // written again (the next step's sums, or the epilogue's maxima)
}

// The maximum of v over the workgroup for this lane's right-hand side, through
// red[0 .. NW * RT); no closing barrier: the callers (the epilogue) give each
// maximum its own part of red and write none of it again.
template <int NW> __device__ __forceinline__ float rhs_max(float v, float *red)
{
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6, r = threadIdx.x & 3;
    if ((threadIdx.x & 63) < RT) red[w * RT + r] = v;
    __syncthreads();
    float m = red[r];
    for (int k = 1; k < NW; k++) m = fmax(m, red[k * RT + r]);
    return m;
}

// Row `row` of U (forward hop, SIGN < 0) or of U^dagger (backward hop): u[b] =
// U[row][b], or conj(U[b][row]); links in LDS as three rows [mu][9][VD].
template <class Sh, int SIGN, typename G>
__device__ __forceinline__ void link_row(const v2<G> *slink, int mu, int lloc, int row, cx<float> u[3])
{
#pragma unroll
    for (int b = 0; b < 3; b++) {
        const int e = SIGN < 0 ? row * 3 + b : b * 3 + row;
        const v2<G> v = slink[(mu * 9 + e) * tile_lstr<Sh>() + lloc];
        u[b] = {static_cast<float>(v.x), SIGN < 0 ? static_cast<float>(v.y) : -static_cast<float>(v.y)};
    }
}

// uh = (U or U^dagger) h for the four right-hand sides of the quad (h: this
// lane's half-spinor, both spin components) on the matrix cores.
template <class Sh, int SIGN, int PROD, typename G>
__device__ __forceinline__ void quad_product(const v2<G> *slink, int mu, int lloc, int r, const cx<float> h[6],
                                             cx<float> uh[6])
{
    // block 0 rows: Re y_0, Re y_1, Re y_2, Im y_0; block 1: Im y_1, Im y_2, 0, 0
    cx<float> u0[3], u1[3];
    link_row<Sh, SIGN, G>(slink, mu, lloc, r < 3 ? r : 0, u0);
    link_row<Sh, SIGN, G>(slink, mu, lloc, r == 0 ? 1 : 2, u1);
    const bool re0 = r < 3, use1 = r < 2;
    float a0[6], a1[6];
#pragma unroll
    for (int b = 0; b < 3; b++) {
        a0[b] = re0 ? u0[b].r : u0[b].i;
        a0[3 + b] = re0 ? -u0[b].i : u0[b].r;
        a1[b] = use1 ? u1[b].i : 0.f;
        a1[3 + b] = use1 ? u1[b].r : 0.f;
    }
    f32x4_t acc[2][2];
#pragma unroll
    for (int s = 0; s < 2; s++) acc[s][0] = acc[s][1] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    if constexpr (PROD == PROD_MFMA_F32) {
#pragma unroll
        for (int k = 0; k < 6; k++)
#pragma unroll
            for (int s = 0; s < 2; s++) {
                const float bk = k < 3 ? h[s * 3 + k].r : h[s * 3 + k - 3].i;
                acc[s][0] = __builtin_amdgcn_mfma_f32_4x4x1f32(a0[k], bk, acc[s][0], 0, 0, 0);
                acc[s][1] = __builtin_amdgcn_mfma_f32_4x4x1f32(a1[k], bk, acc[s][1], 0, 0, 0);
            }
    } else {
        const bf16x4_t A0lo = {(__bf16)a0[0], (__bf16)a0[1], (__bf16)a0[2], (__bf16)a0[3]};
        const bf16x4_t A0hi = {(__bf16)a0[4], (__bf16)a0[5], (__bf16)0.f, (__bf16)0.f};
        const bf16x4_t A1lo = {(__bf16)a1[0], (__bf16)a1[1], (__bf16)a1[2], (__bf16)a1[3]};
        const bf16x4_t A1hi = {(__bf16)a1[4], (__bf16)a1[5], (__bf16)0.f, (__bf16)0.f};
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const cx<float> *hs = h + 3 * s;
            const bf16x4_t Blo = {(__bf16)hs[0].r, (__bf16)hs[1].r, (__bf16)hs[2].r, (__bf16)hs[0].i};
            const bf16x4_t Bhi = {(__bf16)hs[1].i, (__bf16)hs[2].i, (__bf16)0.f, (__bf16)0.f};
            acc[s][0] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A0lo, Blo, acc[s][0], 0, 0, 0);
            acc[s][0] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A0hi, Bhi, acc[s][0], 0, 0, 0);
            acc[s][1] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A1lo, Blo, acc[s][1], 0, 0, 0);
            acc[s][1] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A1hi, Bhi, acc[s][1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int s = 0; s < 2; s++) {
        uh[s * 3 + 0] = {acc[s][0][0], acc[s][0][3]};
        uh[s * 3 + 1] = {acc[s][0][1], acc[s][1][0]};
        uh[s * 3 + 2] = {acc[s][0][2], acc[s][1][1]};
    }
}

// acc += the in-domain hop into site l (local index loc) along MU; SIGN < 0:
// from x + mu with (1 - gamma_mu) U_mu(x), SIGN > 0: from x - mu with
// (1 + gamma_mu) U_mu(x - mu)^dagger.  v holds the other parity's sites.
template <class Sh, int MU, int SIGN, int PROD, typename G>
__device__ __forceinline__ void tile_hop(const cx<float> (*v)[Sh::VH][RT], const int l[4], int loc, int r,
                                         const v2<G> *slink, cx<float> acc[12])
{
    constexpr int VH = Sh::VH;
    const bool has = SIGN < 0 ? l[MU] + 1 < Sh::B[MU] : l[MU] > 0;
    int n[4] = {l[0], l[1], l[2], l[3]};
    if (has) n[MU] += SIGN < 0 ? 1 : -1;
    const int nh = Sh::half_index(n);   // without a neighbour: a valid index, its value unused
    const int lloc = SIGN < 0 ? loc : (1 - (loc >= VH)) * VH + nh;
    cx<float> s[12], h[6], uh[6];
    if constexpr (PROD == PROD_VALU) {
        if (!has) return;
#pragma unroll
        for (int k = 0; k < 12; k++) s[k] = v[k][nh][r];
        proj<MU, SIGN>(s, h);
        const su3<float> U = ld_link<float, G, 9>(slink, (long)MU * 9 * tile_lstr<Sh>() + lloc, tile_lstr<Sh>());
        if constexpr (SIGN < 0) su3_mul(U, h, uh);
        else su3_dag_mul(U, h, uh);
        recon_acc<MU, SIGN>(acc, uh, 1.0f);
    } else {
        // every lane takes part in the matrix instructions; a site without this
        // neighbour multiplies a finite stand-in (its own index's entry) and
        // adds the product with weight 0
#pragma unroll
        for (int k = 0; k < 12; k++) s[k] = v[k][nh][r];
        proj<MU, SIGN>(s, h);
        quad_product<Sh, SIGN, PROD, G>(slink, MU, lloc, r, h, uh);
        recon_acc<MU, SIGN>(acc, uh, has ? 1.0f : 0.0f);
    }
}

template <class Sh, int PROD, typename G>
__device__ __forceinline__ void tile_hops(const cx<float> (*v)[Sh::VH][RT], const int l[4], int loc, int r,
                                          const v2<G> *slink, cx<float> acc[12])
{
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = czero<float>();
    if constexpr (PROD != PROD_VALU) {
        // one hop's operands live at a time (a loop the compiler keeps rolled)
#pragma unroll 1
        for (int k = 0; k < 8; k++) {
            switch (k) {
                case 0: tile_hop<Sh, 0, -1, PROD, G>(v, l, loc, r, slink, acc); break;
                case 1: tile_hop<Sh, 0, +1, PROD, G>(v, l, loc, r, slink, acc); break;
                case 2: tile_hop<Sh, 1, -1, PROD, G>(v, l, loc, r, slink, acc); break;
                case 3: tile_hop<Sh, 1, +1, PROD, G>(v, l, loc, r, slink, acc); break;
                case 4: tile_hop<Sh, 2, -1, PROD, G>(v, l, loc, r, slink, acc); break;
                case 5: tile_hop<Sh, 2, +1, PROD, G>(v, l, loc, r, slink, acc); break;
                case 6: tile_hop<Sh, 3, -1, PROD, G>(v, l, loc, r, slink, acc); break;
                default: tile_hop<Sh, 3, +1, PROD, G>(v, l, loc, r, slink, acc); break;
            }
        }
        return;
    }
    tile_hop<Sh, 0, -1, PROD, G>(v, l, loc, r, slink, acc);
    tile_hop<Sh, 0, +1, PROD, G>(v, l, loc, r, slink, acc);
    tile_hop<Sh, 1, -1, PROD, G>(v, l, loc, r, slink, acc);
    tile_hop<Sh, 1, +1, PROD, G>(v, l, loc, r, slink, acc);
    tile_hop<Sh, 2, -1, PROD, G>(v, l, loc, r, slink, acc);
    tile_hop<Sh, 2, +1, PROD, G>(v, l, loc, r, slink, acc);
    tile_hop<Sh, 3, -1, PROD, G>(v, l, loc, r, slink, acc);
    tile_hop<Sh, 3, +1, PROD, G>(v, l, loc, r, slink, acc);
}

// Items: x = first system of the tile | (systems in the tile) << 24, y = domain.
// SS: storage of block residual and boundary terms; G: links and clover (two
// rows stored, three rows in LDS); arithmetic and accumulator FP32.
template <class Sh, int PROD, typename SS, typename G, bool SCALED>
__global__ __launch_bounds__(Sh::VH * RT) void k_sap_tile(const SapArgs *args, const int2 *items, Visit v)
{
    using T = float;
    using PS = float;
    constexpr int VD = Sh::VD, VH = Sh::VH, NT = VH * RT, NW = NT / 64, NLC = 6, LNLC = 9;
    static_assert(NT % 64 == 0 && NT <= 1024 && NT == 2 * VD, "whole waves; two threads per site for staging");
    constexpr int LSTR = tile_lstr<Sh>();
    __shared__ v2<G> slink[4 * LNLC * LSTR];   // [mu][9][LSTR]
    __shared__ v2<G> sclo[36][VH];            // C_o^-1 of the odd sites
    __shared__ cx<T> she[12][VH][RT];
    __shared__ cx<T> sho[12][VH][RT];
    __shared__ T red[NW * RT * 3];

    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding (XCD lists of unequal length)
    const int sys0 = it.x & 0xffffff, nt = it.x >> 24, d = it.y;
    const int t = threadIdx.x, hi = t >> 2, r = t & 3;
    // this lane's right-hand side; what the tile shares (geometry, links,
    // clover, MR steps) is taken from the first system, so it stays uniform
    const SapArgs &a0 = args[sys0];
    SapArgs a = args[sys0 + (r < nt ? r : 0)];
    a.g = a0.g;
    a.links = a0.links;
    a.cs = a0.cs;
    a.n_mr = a0.n_mr;
    const bool live = r < nt && a.active;
    bind_faces(a, v);
    const int loc_e = hi, loc_o = VH + hi;
    int le[4], lo[4];
    Sh::coords(loc_e, le);
    Sh::coords(loc_o, lo);
    int D[4];
    {
        int q = d;
        D[0] = q % a.g.n[0]; q /= a.g.n[0];
        D[1] = q % a.g.n[1]; q /= a.g.n[1];
        D[2] = q % a.g.n[2];
        D[3] = q / a.g.n[2];
    }
    const v2<G> *glinks = (const v2<G> *)a.links;
    const v2<G> *cs = (const v2<G> *)a.cs;

    // ---- links and the odd sites' C_o^-1 into LDS (two threads per site, two
    // link directions each), the even site's C_e into registers; every global
    // load before the first LDS store
    v2<G> cle[36];
    {
        const int q = t % VD, m0 = (t / VD) * 2;
        v2<G> lt[2 * NLC];
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < NLC; e++) lt[j * NLC + e] = glinks[(((long)d * 4 + m0 + j) * NLC + e) * VD + q];
        const long cb = (long)d * 36 * VD;
#pragma unroll
        for (int k = 0; k < 36; k++) cle[k] = cs[cb + (long)k * VD + loc_e];
        constexpr int NCO = 36 * VH / NT;
        static_assert(36 * VH % NT == 0, "odd clover entries per thread");
        v2<G> ct[NCO];
#pragma unroll
        for (int j = 0; j < NCO; j++) {
            const int i = t + j * NT, k = i / VH;
            ct[j] = cs[cb + (long)k * VD + VH + (i - k * VH)];
        }
#pragma unroll
        for (int j = 0; j < NCO; j++) {
            const int i = t + j * NT, k = i / VH;
            sclo[k][i - k * VH] = ct[j];
        }
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const su3<T> U = ld_link<T, G, NLC>(lt + j * NLC, 0, 1);
#pragma unroll
            for (int e = 0; e < 9; e++) st<T, G>(slink, (long)((m0 + j) * 9 + e) * LSTR + q, U.m[e]);
        }
    }

    // ---- the block right-hand side of both sites
    cx<T> Ae[12], Ao[12], P[12], tt[12];
    const long se = (long)d * 12 * VD + loc_e, so = (long)d * 12 * VD + loc_o;
    if (!live) {
#pragma unroll
        for (int k = 0; k < 12; k++) Ae[k] = Ao[k] = czero<T>();
    } else if (v.first && a.io32) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            Ae[k] = ld<T, float>((const float2 *)a.eta, se + (long)k * VD);
            Ao[k] = ld<T, float>((const float2 *)a.eta, so + (long)k * VD);
        }
    } else if (v.first) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            Ae[k] = ld<T, double>(a.eta, se + (long)k * VD);
            Ao[k] = ld<T, double>(a.eta, so + (long)k * VD);
        }
    } else {
        const T sc = SCALED ? T(a.res_scale[d]) : T(1);
        const v2<SS> *res = (const v2<SS> *)a.res;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            Ae[k] = scal(sc, ld<T, SS>(res, ((long)d * 12 + k) * VH + hi));
            Ao[k] = czero<T>();
        }
    }
    __syncthreads();   // links staged
    if (v.faces_in && live) {
#pragma unroll
        for (int p = 0; p < 2; p++) {
            const int *l = p ? lo : le;
            const int loc = p ? loc_o : loc_e;
            cx<T> *A = p ? Ao : Ae;
            cx<T> hf[4][6];
            T wf[4] = {0, 0, 0, 0};
            int sf[4];
            face_fetch<Sh, 0, T, SS, SCALED>(a, D, l, hf[0], wf[0], sf[0]);
            face_fetch<Sh, 1, T, SS, SCALED>(a, D, l, hf[1], wf[1], sf[1]);
            face_fetch<Sh, 2, T, SS, SCALED>(a, D, l, hf[2], wf[2], sf[2]);
            face_fetch<Sh, 3, T, SS, SCALED>(a, D, l, hf[3], wf[3], sf[3]);
            face_apply<Sh, 0, T, G, NLC, LNLC, true, LSTR>(a, d, loc, slink, hf[0], wf[0], sf[0], A);
            face_apply<Sh, 1, T, G, NLC, LNLC, true, LSTR>(a, d, loc, slink, hf[1], wf[1], sf[1], A);
            face_apply<Sh, 2, T, G, NLC, LNLC, true, LSTR>(a, d, loc, slink, hf[2], wf[2], sf[2], A);
            face_apply<Sh, 3, T, G, NLC, LNLC, true, LSTR>(a, d, loc, slink, hf[3], wf[3], sf[3], A);
        }
    }

    // ---- even-odd preparation: r = rho_e - D_eo C_o^-1 rho_o, x = 0.  With
    // the matrix-instruction products rho_o waits in this right-hand side's
    // global buffer until the reconstruction (their operands leave no room
    // for it in registers); the VALU form keeps it in registers.
    constexpr bool PARK = PROD != PROD_VALU;
    clover_apply<T, G>(&sclo[0][0], hi, VH, Ao, P);
    v2<T> *rho_g = (v2<T> *)a.rho_tmp;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        sho[k][hi][r] = P[k];
        if (PARK && live) st<T, T>(rho_g, ((long)d * 12 + k) * VH + hi, Ao[k]);
    }
    __syncthreads();
    tile_hops<Sh, PROD, G>(sho, le, loc_e, r, slink, tt);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        she[k][hi][r] = Ae[k] + scal(T(0.5), tt[k]);
        Ae[k] = czero<T>();
    }

    // ---- minimal residual on the Schur complement, per right-hand side
#pragma unroll 1
    for (int itr = 0; itr < a.n_mr; itr++) {
        if constexpr (sizeof(v2<G>) == 4) {
            // keep the clover blocks in their 16-bit storage form (see k_sap_lds)
#pragma unroll
            for (int q = 0; q < 36; q++) asm volatile("" : "+v"(cle[q]));
        }
        __syncthreads();
        tile_hops<Sh, PROD, G>(she, lo, loc_o, r, slink, tt);
#pragma unroll
        for (int k = 0; k < 12; k++) tt[k] = scal(T(-0.5), tt[k]);   // D_oe r
        clover_apply<T, G>(&sclo[0][0], hi, VH, tt, P);             // C_o^-1 D_oe r
#pragma unroll
        for (int k = 0; k < 12; k++) sho[k][hi][r] = P[k];
        __syncthreads();
        tile_hops<Sh, PROD, G>(sho, le, loc_e, r, slink, tt);
        cx<T> rr[12];
#pragma unroll
        for (int k = 0; k < 12; k++) rr[k] = she[k][hi][r];
        clover_reg<T, G>(cle, rr, P);                               // C_e r
        T dots[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < 12; k++) {
            P[k] = P[k] + scal(T(0.5), tt[k]);                      // p = C_e r - D_eo C_o^-1 D_oe r
            dots[0] = fmad(P[k].i, rr[k].i, fmad(P[k].r, rr[k].r, dots[0]));
            dots[1] = fmad(-P[k].i, rr[k].r, fmad(P[k].r, rr[k].i, dots[1]));
            dots[2] = fmad(P[k].i, P[k].i, fmad(P[k].r, P[k].r, dots[2]));
        }
        rhs_sum<NW, 3>(dots, red);
        const cx<T> alpha = dots[2] > T(0) ? cx<T>{dots[0] / dots[2], dots[1] / dots[2]} : czero<T>();
#pragma unroll
        for (int k = 0; k < 12; k++) {
            Ae[k] = cmac(Ae[k], alpha, rr[k]);
            she[k][hi][r] = cmac(rr[k], neg(alpha), P[k]);
        }
    }

    // ---- odd sites: delta_o = C_o^-1 (rho_o - D_oe x); x goes through sho
#pragma unroll
    for (int k = 0; k < 12; k++) sho[k][hi][r] = Ae[k];
    __syncthreads();
    tile_hops<Sh, PROD, G>(sho, lo, loc_o, r, slink, tt);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const cx<T> ro = !PARK ? Ao[k] : live ? ld<T, T>(rho_g, ((long)d * 12 + k) * VH + hi) : czero<T>();
        tt[k] = ro + scal(T(0.5), tt[k]);
    }
    clover_apply<T, G>(&sclo[0][0], hi, VH, tt, Ao);                // Ao = delta_o, Ae = delta_e = x

    // ---- epilogue: psi += delta, stored residual, boundary terms
    if (live) {
        const v2<PS> *psi_in = (const v2<PS> *)a.psi;
        v2<PS> *psi_out = (v2<PS> *)a.psi;
#pragma unroll
        for (int p = 0; p < 2; p++) {
            const long sb = p ? so : se;
            const cx<T> *A = p ? Ao : Ae;
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const cx<T> ps = v.first ? A[k] : ld<T, PS>(psi_in, sb + (long)k * VD) + A[k];
                if (v.last && a.io32) st<T, float>((float2 *)a.out, sb + (long)k * VD, ps);
                else if (v.last) st<T, double>(a.out, sb + (long)k * VD, ps);
                else st<T, PS>(psi_out, sb + (long)k * VD, ps);
            }
        }
    }
    if (v.res_out) {
        cx<T> rr[12];
#pragma unroll
        for (int k = 0; k < 12; k++) rr[k] = she[k][hi][r];
        T sc = T(1);
        if constexpr (SCALED) {
            sc = pow2_ceil(rhs_max<NW>(maxabs12(rr), red));
            if (hi == 0 && live) a.res_scale[d] = (float)sc;
        }
        if (live) {
            v2<SS> *res = (v2<SS> *)a.res;
            const T inv = T(1) / sc;
#pragma unroll
            for (int k = 0; k < 12; k++) st<T, SS>(res, ((long)d * 12 + k) * VH + hi, scal(inv, rr[k]));
        }
    }
    if (v.faces_out) {
        T sc = T(1);
        if constexpr (SCALED) {
            sc = T(8) * pow2_ceil(rhs_max<NW>(fmax(maxabs12(Ae), maxabs12(Ao)), red + NW * RT));
            if (hi == 0 && live) a.face_scale[d] = (float)sc;
        }
        const T inv = T(1) / sc;
        if (live) {
            write_face<Sh, 0, T, SS, G, NLC, LNLC, true, LSTR>(a, d, le, loc_e, Ae, inv, slink);
            write_face<Sh, 1, T, SS, G, NLC, LNLC, true, LSTR>(a, d, le, loc_e, Ae, inv, slink);
            write_face<Sh, 2, T, SS, G, NLC, LNLC, true, LSTR>(a, d, le, loc_e, Ae, inv, slink);
            write_face<Sh, 3, T, SS, G, NLC, LNLC, true, LSTR>(a, d, le, loc_e, Ae, inv, slink);
            write_face<Sh, 0, T, SS, G, NLC, LNLC, true, LSTR>(a, d, lo, loc_o, Ao, inv, slink);
            write_face<Sh, 1, T, SS, G, NLC, LNLC, true, LSTR>(a, d, lo, loc_o, Ao, inv, slink);
            write_face<Sh, 2, T, SS, G, NLC, LNLC, true, LSTR>(a, d, lo, loc_o, Ao, inv, slink);
            write_face<Sh, 3, T, SS, G, NLC, LNLC, true, LSTR>(a, d, lo, loc_o, Ao, inv, slink);
        }
    }
}

// Every block-solve launch goes through here: the workgroup size must not
// exceed the kernel's launch bound (the register allocation is made for that
// bound), which is read from the code object once per kernel and checked on
// the host before the launch.
template <typename... P, typename... A>
static hipError_t launch_bounded(void (*kernel)(P...), unsigned grid, unsigned block, hipStream_t s, A... args)
{
    static std::mutex mu;
    static std::unordered_map<const void *, int> bound;
    const void *key = reinterpret_cast<const void *>(kernel);
    int maxt;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = bound.find(key);
        if (it == bound.end()) {
            hipFuncAttributes at;
            const hipError_t e = hipFuncGetAttributes(&at, key);
            if (e != hipSuccess) return e;
            it = bound.emplace(key, at.maxThreadsPerBlock).first;
        }
        maxt = it->second;
    }
    if (block == 0 || (int)block > maxt) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, args...);
    return hipGetLastError();
}

template <class Sh>
static hipError_t launch_batch(const SapArgs *args, const int2 *items, int nitems, int prec, int product, Visit v,
                               hipStream_t s)
{
    if (product != PRODUCT_LANE) {
        // a tile of right-hand sides per workgroup: 4^4 domains, FP16 storage
        if constexpr (std::is_same<Sh, Shape<4, 4, 4, 4>>::value) {
            constexpr int NT = Sh::VH * RT;
            if (prec == PB16) {
                switch (product) {
                    case PRODUCT_TILE_VALU:
                        return launch_bounded(k_sap_tile<Sh, PROD_VALU, bf16_t, bf16_t, false>, nitems, NT, s, args,
                                              items, v);
                    case PRODUCT_TILE_MFMA_F32:
                        return launch_bounded(k_sap_tile<Sh, PROD_MFMA_F32, bf16_t, bf16_t, false>, nitems, NT, s, args,
                                              items, v);
                    case PRODUCT_TILE_MFMA_BF16:
                        return launch_bounded(k_sap_tile<Sh, PROD_MFMA_BF16, bf16_t, bf16_t, false>, nitems, NT, s,
                                              args, items, v);
                    default: return hipErrorInvalidValue;
                }
            }
            if (prec != P16) return hipErrorInvalidValue;
            switch (product) {
                case PRODUCT_TILE_VALU:
                    return launch_bounded(k_sap_tile<Sh, PROD_VALU, half_t, half_t, true>, nitems, NT, s, args, items, v);
                case PRODUCT_TILE_MFMA_F32:
                    return launch_bounded(k_sap_tile<Sh, PROD_MFMA_F32, half_t, half_t, true>, nitems, NT, s, args, items,
                                          v);
                case PRODUCT_TILE_MFMA_BF16:
                    return launch_bounded(k_sap_tile<Sh, PROD_MFMA_BF16, half_t, half_t, true>, nitems, NT, s, args,
                                          items, v);
                default: return hipErrorInvalidValue;
            }
        }
        return hipErrorInvalidValue;
    }
    if (prec == P64) {
        // FP64: one thread per even/odd site pair on 2^4 domains, else the LDS
        // layout (whole waves only: no FP64 kernel for padded workgroups)
        if constexpr (Sh::VD == 16)
            return launch_bounded(k_sap_sweep<Sh, double, double, double, double, 9, false, false>, nitems, Sh::VH, s,
                                  args, items, v);
        else if constexpr (Sh::VD % 64 == 0)
            return launch_bounded(k_sap_f64<Sh>, nitems, Sh::VD, s, args, items, v);
        else
            return hipErrorInvalidValue;
    } else {
        constexpr int NDW = Sh::VD < 64 ? 128 / Sh::VD : 1;
        constexpr int NT = NDW > 1 ? Sh::VD * NDW : Sh::NT;
        if (nitems % NDW) return hipErrorInvalidValue;
        if (prec == P32)
            return launch_bounded(k_sap_lds<Sh, NDW, float, float, float, float, 6, 6, false, true, true>, nitems / NDW,
                                  NT, s, args, items, v);
        else if (prec == P16)
            return launch_bounded(k_sap_lds<Sh, NDW, float, half_t, float, half_t, 6, 9, true, true, true>,
                                  nitems / NDW, NT, s, args, items, v);
        else
            return launch_bounded(k_sap_lds<Sh, NDW, float, bf16_t, float, bf16_t, 6, 9, false, true, true>,
                                  nitems / NDW, NT, s, args, items, v);
    }
}

int sap_domains_per_workgroup(int shape, int prec, int product)
{
    return shape == 0 && prec != P64 && product == PRODUCT_LANE ? 8 : 1;
}

int sap_rhs_per_workgroup(int product) { return product == PRODUCT_LANE ? 1 : RT; }

bool sap_product_supported(const int b[4], int prec, int product)
{
    if (product == PRODUCT_LANE) return sap_prec_supported(b, prec);
    if (product < PRODUCT_TILE_VALU || product > PRODUCT_TILE_MFMA_BF16) return false;
    return sap_shape_id(b) == 1 && (prec == P16 || prec == PB16);
}

int sap_shape_id(const int b[4])
{
    if (b[0] == 2 && b[1] == 2 && b[2] == 2 && b[3] == 2) return 0;
    if (b[0] == 4 && b[1] == 4 && b[2] == 4 && b[3] == 4) return 1;
    if (b[0] == 8 && b[1] == 4 && b[2] == 4 && b[3] == 4) return 2;
    if (b[0] == 4 && b[1] == 4 && b[2] == 4 && b[3] == 8) return 3;
    if (b[0] == 6 && b[1] == 6 && b[2] == 2 && b[3] == 4) return 4;
    return -1;
}

int sap_shape_count() { return 5; }

void sap_shape_extents(int shape, int b[4])
{
    static const int E[5][4] = {{2, 2, 2, 2}, {4, 4, 4, 4}, {8, 4, 4, 4}, {4, 4, 4, 8}, {6, 6, 2, 4}};
    for (int m = 0; m < 4; m++) b[m] = E[shape][m];
}

bool sap_shape_supported(const int b[4]) { return sap_shape_id(b) >= 0; }

// FP64 block solves need 16 sites or whole waves (no padded FP64 workgroups)
bool sap_prec_supported(const int b[4], int prec)
{
    const int id = sap_shape_id(b);
    if (id < 0 || prec < P64 || prec > PB16) return false;
    const int vd = b[0] * b[1] * b[2] * b[3];
    return prec != P64 || vd == 16 || vd % 64 == 0;
}

long sap_face_sites(const int b[4])
{
    long Vd = (long)b[0] * b[1] * b[2] * b[3];
    return 2 * (Vd / b[0] + Vd / b[1] + Vd / b[2] + Vd / b[3]);
}

// item i < nd/2: the i-th black domain (item.x = x), item nd/2 + i: the i-th
// white one, in increasing domain number.  The domain grid's x extent is even,
// so domains 2i and 2i + 1 lie in one x row and have opposite colours: the
// i-th domain of colour c is the one of that pair with colour c.
__global__ void k_schedule_items(Geo g, int x, int2 *items)
{
    const int half = g.nd / 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nd) return;
    const int c = i >= half, j = i - c * half;
    const int d0 = 2 * j;
    const int rest = d0 / g.n[0];
    const int D1 = rest % g.n[1], D2 = (rest / g.n[1]) % g.n[2], D3 = rest / (g.n[1] * g.n[2]);
    const int colour0 = (D1 + D2 + D3) & 1;   // colour of domain 2j (its x coordinate is even)
    items[i] = make_int2(x, d0 + ((c + colour0) & 1));
}

__global__ void k_put_args(SapArgs a, SapArgs *dst) { *dst = a; }

hipError_t sap_schedule_items(const Geo &g, int x, int2 *items, hipStream_t s)
{
    hipLaunchKernelGGL(k_schedule_items, (g.nd + 255) / 256, 256, 0, s, g, x, items);
    return hipGetLastError();
}

hipError_t sap_put_args(const SapArgs &a, SapArgs *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_put_args, 1, 1, 0, s, a, dst);
    return hipGetLastError();
}

hipError_t sap_sweep_batch(const SapArgs *args, const int2 *items, int nitems, int shape, int prec, int product,
                           Visit v, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    switch (shape) {
        case 0: return launch_batch<Shape<2, 2, 2, 2>>(args, items, nitems, prec, product, v, s);
        case 1: return launch_batch<Shape<4, 4, 4, 4>>(args, items, nitems, prec, product, v, s);
        case 2: return launch_batch<Shape<8, 4, 4, 4>>(args, items, nitems, prec, product, v, s);
        case 3: return launch_batch<Shape<4, 4, 4, 8>>(args, items, nitems, prec, product, v, s);
        case 4: return launch_batch<Shape<6, 6, 2, 4>>(args, items, nitems, prec, product, v, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dd
