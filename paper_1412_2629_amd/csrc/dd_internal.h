// Host-side interface between the C-ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include "dd_device.h"

namespace dd {

enum { P64 = 0, P32 = 1, P16 = 2, PB16 = 3 };   // FP64, FP32, FP16, BF16 storage

// Canonical FP64 spinor [V][12] complex <-> internal layout in precision prec.
hipError_t import_spinor(const Geo &g, const double *canon, void *internal, int prec, hipStream_t s);
hipError_t export_spinor(const Geo &g, const void *internal, int prec, double *canon, hipStream_t s);

// Canonical FP64 links -> internal FP64 full links [d][mu][9][Vd].
hipError_t import_gauge(const Geo &g, const double *canon, double2 *U64, hipStream_t s);
// Internal FP64 full links -> first two rows in FP32 or FP16 [d][mu][6][Vd].
hipError_t compress_links(const Geo &g, const double2 *U64, void *out, int prec, hipStream_t s);
// Clover term C(x) = 1/(2 kappa) + D_cl(x), packed [d][36][Vd] FP64.
hipError_t clover_build(const Geo &g, const double2 *U64, double kappa, double csw, double2 *C64, hipStream_t s);
// Site matrices used by the block solves: C on even sites, C^-1 on odd sites.
// *bad (device int) is set to 1 if a block is singular.
hipError_t clover_schur(const Geo &g, const double2 *C64, double2 *Cs64, int *bad, hipStream_t s);
// Elementwise FP64 pairs -> FP32 / FP16 pairs.
hipError_t convert_pairs(const double2 *in, void *out, long n, int prec, hipStream_t s);
// Number of non-finite values in n FP64 pairs (device counter *cnt, accumulated).
hipError_t count_nonfinite(const double2 *v, long n, int *cnt, hipStream_t s);

// out = A in (internal layouts; links/clover in the given precision).
hipError_t apply_A(const Geo &g, const void *in, void *out, const void *links, const void *clov, int prec,
                   hipStream_t s);
// out0 = A in0 and out1 = A in1 on one lattice in one launch (the two
// right-hand sides share each link and clover load); same bits as two apply_A
// calls.  Available where apply_A_pairs(g, prec) (domains of at most 256
// sites, fields under 4 GiB); hipErrorInvalidValue otherwise.
bool apply_A_pairs(const Geo &g, int prec);
hipError_t apply_A_pair(const Geo &g, const void *in0, void *out0, const void *in1, void *out1, const void *links,
                        const void *clov, int prec, hipStream_t s);

// What one visit of a domain reads and writes.
struct Visit {
    int first;      // first visit in this preconditioner call: residual is eta
    int faces_in;   // add the neighbours' boundary terms
    int last;       // last visit: write psi to the FP64 output
    int faces_out;  // write this domain's boundary terms
    int res_out;    // store the block residual
    int flip;       // additive schedule: which of the two boundary buffers is written
};

// Arguments of the block solves of one system (one lattice, one right-hand side).
struct SapArgs {
    Geo g;
    int first;          // first visit of these domains: residual is eta
    int faces_in;       // add the boundary terms of the previous half-sweep
    int last;           // last visit: write psi (+ delta) to out
    int faces_out;      // write this sweep's boundary terms
    int res_out;        // store the block residual
    int n_mr;
    const double2 *eta; // FP64 input of the preconditioner
    double2 *out;       // FP64 output
    void *psi;          // solution accumulator (FP64, or FP32 for FP32/FP16 storage)
    void *res;          // block residual on even sites [d][12][Vd/2]
    float *res_scale;   // per-domain scale of res (FP16 storage)
    void *face;         // boundary half-spinors [d][8 faces][6][face sites]
    float *face_scale;  // per-domain scale of face (FP16 storage)
    void *face_alt;     // second boundary buffer (additive schedule), else null
    float *face_scale_alt;
    const void *face_in;          // set in the kernel: the buffer this visit reads
    const float *face_in_scale;
    const void *links;  // [d][mu][9 or 6][Vd]
    const void *cs;     // C_e on even / C_o^-1 on odd sites [d][36][Vd]
    void *rho_tmp;      // odd-site right-hand sides [d][12][Vd/2] when not kept in LDS
    int active;         // 0: skip this system (already converged)
    int io32;           // eta and out are FP32 (float2) vectors (FP32/FP16/BF16 block solves only)
};
bool sap_shape_supported(const int b[4]);
bool sap_prec_supported(const int b[4], int prec);
long sap_face_sites(const int b[4]);
int sap_shape_id(const int b[4]);
// How a block-solve workgroup forms the SU(3) products of its hops:
// PRODUCT_LANE, one right-hand side per workgroup and one site per thread
// (VALU); the TILE forms take a tile of four right-hand sides of one lattice
// per workgroup (4^4 domains, FP16 storage) with the product on the VALU, on
// FP32 MFMA, or on BF16-input MFMA with FP32 accumulation.
enum { PRODUCT_LANE = 0, PRODUCT_TILE_VALU = 1, PRODUCT_TILE_MFMA_F32 = 2, PRODUCT_TILE_MFMA_BF16 = 3 };
bool sap_product_supported(const int b[4], int prec, int product);
// Right-hand sides one workgroup takes (1, or 4 for the tile forms): the items
// of a tile launch are (first system | systems in the tile << 24, domain).
int sap_rhs_per_workgroup(int product);
// Domains one block-solve workgroup takes for (shape, precision, product): the
// items of a launch come in runs of this many domains of one system, and a run
// is never split or padded.
int sap_domains_per_workgroup(int shape, int prec, int product);
// The compiled domain shapes: ids 0 .. sap_shape_count() - 1 and their extents.
int sap_shape_count();
void sap_shape_extents(int shape, int b[4]);
// Work items of one system on the device: [0, nd/2) its black domains, then
// its white domains, each in increasing domain number (the order a plan of
// one system uses), with item.x = x.  items holds nd entries.
hipError_t sap_schedule_items(const Geo &g, int x, int2 *items, hipStream_t s);
// *dst = a on the device, in stream order (no host copy).
hipError_t sap_put_args(const SapArgs &a, SapArgs *dst, hipStream_t s);
// One colour of one half-sweep for a list of (system, domain) items; args and
// items are device arrays.  All systems share one domain shape (shape id).
hipError_t sap_sweep_batch(const SapArgs *args, const int2 *items, int nitems, int shape, int prec, int product,
                           Visit v, hipStream_t s);

// ---- FP64 linear algebra on flat complex vectors (double2) ---------------
struct Blas {
    double2 *partial = nullptr;   // [NBLK][32]
    double2 *result = nullptr;    // [32] device
    double2 *coef = nullptr;      // [32] device coefficients
    hipError_t init();
    void release();
};
enum { BLAS_NBLK = 1024, BLAS_MAXK = 16 };
// result[j] = <W_j, v>, j < k (k <= 16); W_j = W + j*ldw
hipError_t multidot(Blas &B, const double2 *W, long ldw, int k, const double2 *v, long n, hipStream_t s);
// w -= sum_j coef[j] W_j (coef on device, k <= 16); result[0] = (|w|^2, 0), result[1] = <w, r>
hipError_t cgs_update(Blas &B, double2 *w, const double2 *W, long ldw, int k, const double2 *r, long n,
                      hipStream_t s);
// r -= c w; result[0] = (|r|^2, 0)
hipError_t residual_update(Blas &B, const double2 *w, double2 *r, double2 c, long n, hipStream_t s);
// x += sum_j coef[j] Z_j (coef on device, k <= 16)
hipError_t axpy_multi(Blas &B, double2 *x, const double2 *Z, long ldz, int k, long n, hipStream_t s);
// r = b - r; result[0] = (|r|^2, 0)
hipError_t residual(Blas &B, const double2 *b, double2 *r, long n, hipStream_t s);
// result[0] = (|v|^2, 0)
hipError_t norm2(Blas &B, const double2 *v, long n, hipStream_t s);
hipError_t zero(double2 *v, long n, hipStream_t s);
// FP32 vectors, FP64 accumulation: result[j] = <W_j, v> (k <= 16);
// w -= sum_j coef[j] W_j with result[0] = |w|^2; w *= inv_b with result[0] =
// <w, r>; r -= c w with result[0] = |r|^2; x (FP64) += scale sum_j coef[j] Z_j;
// out = sc * in rounded to FP32
hipError_t multidot32(Blas &B, const float2 *W, long ldw, int k, const float2 *v, long n, hipStream_t s);
hipError_t cgs_update32(Blas &B, float2 *w, const float2 *W, long ldw, int k, long n, hipStream_t s);
hipError_t scale_dot32(Blas &B, float2 *w, double inv_b, const float2 *r, long n, hipStream_t s);
hipError_t axpy32(Blas &B, float2 *r, double2 c, const float2 *w, long n, hipStream_t s);
hipError_t axpy_mixed(Blas &B, double2 *x, const float2 *Z, long ldz, int k, double scale, long n, hipStream_t s);
hipError_t to_f32(const double2 *in, double sc, float2 *out, long n, hipStream_t s);
// out_q = sum_i W_i P[i][q], q < nq, i < nin (<= 24 each; P row-major on the
// device; out must not overlap W)
hipError_t recombine(const double2 *W, long ldw, int nin, const double2 *P, int nq, double2 *out, long ldo, long n,
                     hipStream_t s);
// result[0] = <t, s>, result[1] = (|t|^2, 0)
hipError_t dot2(Blas &B, const double2 *t, const double2 *s_vec, long n, hipStream_t s);
// out = ca a + cb b + cc c; c may be null; out may alias an input
hipError_t lincomb(double2 *out, const double2 *a, double2 ca, const double2 *b, double2 cb, const double2 *c,
                   double2 cc, long n, hipStream_t s);

}  // namespace dd
