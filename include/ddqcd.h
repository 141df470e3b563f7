/*
 * ddqcd: SAP-preconditioned flexible GCR solver for the Wilson-clover Dirac
 * equation on one AMD MI355X (gfx950), after Heybrock et al., "Lattice QCD
 * with Domain Decomposition on Intel Xeon Phi Co-Processors", SC14
 * (arXiv:1412.2629).
 *
 * The operator (Sec. II-B, Eqs. 1-3):
 *   A = (4 + m) - D_w / 2 + D_cl,    4 + m = 1 / (2 kappa),
 *   D_w psi(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *              + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu),
 *   D_cl = c_sw sum_{mu,nu} (i/8) sigma_munu F_munu   (clover-leaf field strength),
 * gamma matrices in the chiral basis (the clover term is then two Hermitian
 * 6x6 blocks per site), mu = 0..3 <-> x, y, z, t.  A hop that wraps around
 * the lattice in direction mu is multiplied by boundary[mu] (+1 or -1).
 *
 * The solver (Sec. II-C, II-D and the algorithm of Table I): flexible GCR
 * with restart, right-preconditioned by the Schwarz alternating procedure
 * (multiplicative Schwarz over a black/white colouring of the domains), each
 * block solved approximately by minimal-residual (MR) steps on the even-odd
 * Schur complement (Sec. II-D, Eq. 5).  The outer solver, its residuals and
 * the solution update are FP64; the preconditioner runs in FP64, FP32, or
 * FP32 arithmetic with FP16 storage (Sec. III, III-B).
 *
 * Canonical layouts at this interface (all device pointers, C-contiguous):
 *   site index      i = x + Lx*(y + Ly*(z + Lz*t))
 *   gauge field     double[V][4][3][3][2]   U_mu(x)[row][col], re/im interleaved
 *   spinor field    double[nrhs][V][4][3][2] psi(x)[spin][colour]
 * Pointers must be 16-byte aligned device memory of the current device.
 *
 * Ownership: the caller owns every pointer it passes.  The device memory of a
 * context (internal copies of the links and clover terms, solver work
 * vectors, launch plans) is either allocated by the library and freed in
 * ddqcd_destroy, or carved from a workspace the caller hands over with
 * ddqcd_set_workspace (the caller frees it after ddqcd_destroy).
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  apply_D
 * and sap are asynchronous on that stream; load_gauge and solve return
 * after the stream has drained (solve reads residual norms on the host).
 *
 * Errors: every entry point returns a ddqcd_status; nothing throws across
 * the interface.  ddqcd_last_error(ctx) describes the last failure.
 * One context must not be used by two host threads at once.
 */
#ifndef DDQCD_H
#define DDQCD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddqcd_ctx *ddqcd_t;

typedef enum {
    DDQCD_OK = 0,
    DDQCD_ERR_ARG = 1,           /* bad argument (null pointer, kappa <= 0, |boundary| != 1, ...) */
    DDQCD_ERR_GEOMETRY = 2,      /* domain shape does not tile the lattice in an even count >= 2 per direction,
                                    an odd domain extent, or a domain shape without a compiled kernel */
    DDQCD_ERR_STATE = 3,         /* call out of order (e.g. solve before load_gauge) */
    DDQCD_ERR_DEVICE = 4,        /* a HIP runtime call failed */
    DDQCD_ERR_NOMEM = 5,         /* device allocation failed */
    DDQCD_ERR_NOT_CONVERGED = 6, /* solve stopped at max_cycles; x holds the last iterate */
    DDQCD_ERR_NONFINITE = 7      /* NaN or Inf in the input or in a residual */
} ddqcd_status;

/* Storage and arithmetic of the block solves and of ddqcd_apply_D: FP64; FP32;
 * FP16 storage (links as two rows, clover, block residual and boundary terms;
 * power-of-two scales per domain for the spinors) with FP32 arithmetic; BF16
 * storage (the same fields, FP32's exponent range, so no scales; 8-bit
 * significand) with FP32 arithmetic (Sec. III-B: reduced-precision storage). */
typedef enum { DDQCD_FP64 = 0, DDQCD_FP32 = 1, DDQCD_FP16 = 2, DDQCD_BF16 = 3 } ddqcd_prec;

typedef enum { DDQCD_SCHED_SWEEPS = 0, DDQCD_SCHED_QUEUE = 1, DDQCD_SCHED_GRAPH = 2 } ddqcd_schedule;
typedef enum { DDQCD_SCHWARZ_MULTIPLICATIVE = 0, DDQCD_SCHWARZ_ADDITIVE = 1 } ddqcd_schwarz;

typedef struct {
    int converged;        /* 1 if |b - A x| / |b| <= tol */
    int iters;            /* FGCR steps (= preconditioner applications) */
    int restarts;         /* FGCR cycles */
    double rel_residual;  /* true residual |b - A x| / |b|, recomputed in FP64 at exit */
    double t_total_ms;    /* wall time of the call */
    double t_sap_ms;      /* preconditioner M (stream time, events) */
    double t_A_ms;        /* operator A */
    double t_gs_ms;       /* Gram-Schmidt */
    double t_other_ms;    /* remaining linear algebra */
} ddqcd_info;

/* Creates a context for one lattice (host metadata only; no device memory).
 * lattice[4]: Lx, Ly, Lz, Lt.  domain[4]: Schwarz domain extents; each must be
 * even, divide the lattice extent, and leave an even number >= 2 of domains
 * per direction (black/white colouring of Sec. IV-B2), and be one of the
 * compiled block-solve shapes 2x2x2x2, 4x4x4x4, 8x4x4x4, 4x4x4x8, 6x6x2x4.  kappa > 0 gives
 * 4 + m = 1/(2 kappa) (Sec. II-B).  boundary[mu] in {+1, -1}.
 * Defaults: SAP 16 cycles, 5 MR steps, FP32 (Sec. IV-C); FGCR restart 16,
 * tol 1e-10, max 64 cycles.  Returns DDQCD_ERR_GEOMETRY / DDQCD_ERR_ARG on
 * invalid input; *out is set only on success. */
int ddqcd_create(const int lattice[4], const int domain[4], double kappa, double c_sw, const double boundary[4],
                 ddqcd_t *out);

/* Frees the context and all device memory it owns.  NULL is allowed. */
int ddqcd_destroy(ddqcd_t ctx);

/* How the block solves form the SU(3) link x half-spinor products of their
 * hops (the hop structure of Sec. II-B: project, multiply by the link,
 * reconstruct).  DDQCD_PRODUCT_LANE: one right-hand side per workgroup, one
 * site per thread, products on the vector ALUs.  The tile forms solve one
 * domain for a tile of four right-hand sides of a lattice per workgroup (the
 * link is staged once for the tile): DDQCD_PRODUCT_TILE_VALU with the products
 * on the vector ALUs, DDQCD_PRODUCT_MFMA_F32 on FP32 matrix instructions
 * (U in real form, 6x6, times the 6x4 block of the four right-hand sides'
 * half-spinors, FP32 inputs and accumulation), DDQCD_PRODUCT_MFMA_BF16 on
 * BF16-input matrix instructions with FP32 accumulation (link and half-spinor
 * rounded to BF16 for the product).  The tile forms need 4x4x4x4 domains and
 * DDQCD_FP16 or DDQCD_BF16 storage; a solve or preconditioner call with nrhs
 * right-hand sides uses ceil(nrhs / 4) tiles. */
typedef enum {
    DDQCD_PRODUCT_LANE = 0,
    DDQCD_PRODUCT_TILE_VALU = 1,
    DDQCD_PRODUCT_MFMA_F32 = 2,
    DDQCD_PRODUCT_MFMA_BF16 = 3
} ddqcd_product;

/* Schwarz preconditioner settings: n_cycles = I_Schwarz >= 1, n_mr = I_domain
 * >= 1 (Sec. II-D), prec = storage/arithmetic of the block solves, a
 * ddqcd_prec (reduced storage with FP32 arithmetic and an FP32 solution
 * accumulator); product = a
 * ddqcd_product.  Every precision is available with DDQCD_PRODUCT_LANE for
 * every domain shape ddqcd_create accepts, except FP64 on 6x6x2x4 domains.
 * DDQCD_ERR_GEOMETRY for a combination without a kernel, DDQCD_ERR_ARG for
 * values out of range. */
int ddqcd_set_sap(ddqcd_t ctx, int n_cycles, int n_mr, int prec, int product);

/* How the block solves of one preconditioner call are scheduled.
 * DDQCD_SCHED_SWEEPS (the default) launches one kernel per colour of each
 * half-sweep: all domains of one colour at once, Sec. IV-B2's n_domain.
 * DDQCD_SCHED_GRAPH issues the same launches from a HIP graph captured once
 * per set of systems and replayed for every preconditioner call (results are
 * identical bit for bit; the launch cost is paid once).  DDQCD_SCHED_QUEUE,
 * one persistent kernel taking (cycle, domain) tasks from a work queue with
 * per-domain epoch counters so that consecutive half-sweeps overlap, is
 * switched off: selecting it returns DDQCD_ERR_ARG.  In a ddqcd_solve_batch
 * call the schedule of the first context applies. */
int ddqcd_set_schedule(ddqcd_t ctx, int schedule);

/* Which Schwarz method the preconditioner runs (Sec. II-D).
 * DDQCD_SCHWARZ_MULTIPLICATIVE (the default, the paper's choice): each cycle
 * visits the black domains, then the white ones, each from the residual that
 * includes the other colour's latest corrections.  DDQCD_SCHWARZ_ADDITIVE
 * (Eq. 4): each cycle every domain solves its block of the same residual and
 * the corrections are summed, so one launch per cycle covers all domains
 * (twice the block solves in flight, no colouring).  Applies to ddqcd_sap and
 * ddqcd_solve; ddqcd_solve_batch requires it to be equal on all contexts. */
int ddqcd_set_schwarz(ddqcd_t ctx, int kind);

/* Device memory of a context supplied by the caller (for instance one torch
 * allocation).  ddqcd_workspace_size writes to *bytes what the context needs to
 * solve nrhs >= 1 right-hand sides at once (or apply the preconditioner or
 * operator to them) with its current restart length: the copies of links,
 * clover term and C_e / C_o^-1 in every precision; per right-hand side the
 * work slot (solution accumulator, block residual, boundary terms of both
 * Schwarz variants, FP64 vectors, reduction buffers, the FGCR basis of 2 x
 * max(restart, 5) vectors); the apply_D operands; the reduction area; and a
 * region for launch plans.  ddqcd_set_workspace hands the context dev_ptr
 * (device memory of the device ddqcd_load_gauge will run on, 256-byte
 * aligned, at least ddqcd_workspace_size(ctx, 1) bytes), before
 * ddqcd_load_gauge and once per context: from then on every device array of
 * the context is carved from it and the context calls no hipMalloc (the
 * ddqcd_tune_* calls make contexts of their own).  The workspace serves the
 * largest nrhs whose size fits; a call that needs more (more right-hand sides,
 * a longer restart set afterwards, a ddqcd_solve_batch led by this context
 * with more than max(nrhs, 64) systems) returns DDQCD_ERR_NOMEM.  The caller
 * keeps the memory alive and unused by anything else until ddqcd_destroy,
 * which does not free it.  Errors: DDQCD_ERR_ARG (null or misaligned pointer),
 * DDQCD_ERR_NOMEM (smaller than one right-hand side needs), DDQCD_ERR_STATE
 * (the context already holds device memory or a workspace). */
int ddqcd_workspace_size(ddqcd_t ctx, int nrhs, size_t *bytes);
int ddqcd_set_workspace(ddqcd_t ctx, void *dev_ptr, size_t bytes);

/* The outer solver of ddqcd_solve and ddqcd_solve_batch (Sec. II-C).
 * DDQCD_OUTER_FGCR (the default): flexible GCR, restart = basis vectors per
 * cycle, all right-hand sides in lockstep.  DDQCD_OUTER_FGMRES_DR: flexible
 * GMRES with deflated restarts, the paper's outer solver (Table I): restart =
 * maximum basis size m, deflate = k harmonic Ritz vectors of smallest magnitude
 * kept at each restart (0 <= k < m; the paper uses m = 8, k = 4 and m = 16,
 * k = 6, Sec. IV-C), right-hand sides one after the other.  Both keep the
 * orthogonalisation, residuals and solution update in FP64 and stop on the
 * true residual recomputed at each cycle's end.  DDQCD_OUTER_FGCR_MIXED
 * (deflate 0): the mixed-precision outer solver of Sec. VI: FP64 iterative
 * refinement (true residual r = b - A x, x += |r| e) around FGCR cycles in FP32
 * (vectors, operator with two-row links, Gram-Schmidt with FP64 accumulation)
 * that reduce their residual by 1e-5 each (or to what the tolerance needs),
 * with the SAP preconditioner reading and writing FP32; needs a
 * reduced-precision preconditioner; right-hand sides one after the other.  ddqcd_solve_batch needs equal
 * settings on all contexts.  DDQCD_ERR_ARG for values out of range,
 * DDQCD_ERR_STATE on a workspace context that already has work slots (their
 * basis size is fixed). */
typedef enum { DDQCD_OUTER_FGCR = 0, DDQCD_OUTER_FGMRES_DR = 1, DDQCD_OUTER_FGCR_MIXED = 2 } ddqcd_outer;
int ddqcd_set_outer(ddqcd_t ctx, int kind, int deflate);

/* Outer solver settings: restart >= 1 basis vectors per cycle, tol > 0 on the
 * true relative residual |b - A x|/|b| (Sec. IV-C1), max_cycles >= 1. */
int ddqcd_set_solver(ddqcd_t ctx, int restart, double tol, int max_cycles);

/* Loads the gauge field U (device pointer, canonical layout, FP64), builds the
 * clover term (Sec. II-B, Eq. 3), its odd-site inverse (needed by the Schur
 * complement of Sec. II-D, Eq. 5) and the reduced-precision copies.  The
 * caller may reuse U once this returns.  Allocates the context's device
 * memory on the current device on first call. */
int ddqcd_load_gauge(ddqcd_t ctx, const double *U, void *stream);

/* out = A in for nrhs spinor fields (canonical layout, FP64 at the interface).
 * prec selects the arithmetic and storage of the application: DDQCD_FP64, or
 * DDQCD_FP32 / DDQCD_FP16 (input rounded to that precision, 2-row compressed
 * links, result rounded before widening to FP64).  in and out must not alias. */
int ddqcd_apply_D(ddqcd_t ctx, double *out, const double *in, int nrhs, int prec, void *stream);

/* out = M in: the Schwarz alternating procedure with the settings of
 * ddqcd_set_sap (Sec. II-D; the algorithm of Table I without the outer loop).
 * in and out must not alias. */
int ddqcd_sap(ddqcd_t ctx, double *out, const double *in, int nrhs, void *stream);

/* out = M in for one right-hand side, as ddqcd_sap, without allocating any
 * memory: for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  All work space
 * (internal copies of in and out, the solution accumulator, block residuals,
 * boundary terms, the launch arguments and the domain lists) is carved from
 * one device array of the library, 128 MiB per device, which every device the
 * library runs on holds until the process ends; ddqcd_load_gauge looks up its
 * address on the context's device.  A lattice whose work space does not fit
 * (about 940 bytes per site with 8x4x4x4 domains, more with smaller domains or
 * the additive variant; 16^3x32 with 8x4x4x4 domains fits) returns
 * DDQCD_ERR_NOMEM.  Every call on one device uses that same array: calls that
 * overlap on one device (two streams, two host threads) race and give wrong
 * results; calls ordered in one stream are safe, and nothing of an earlier
 * call's contents is read.  Settings as for ddqcd_sap (ddqcd_set_sap,
 * ddqcd_set_schwarz); the launches are issued one by one whatever
 * ddqcd_set_schedule says.  The kernels and their order are those of
 * ddqcd_sap with nrhs = 1, so the result is the same bit for bit.  in and out:
 * device pointers, canonical layout, must not alias.  Asynchronous on stream. */
int ddqcd_sap_noalloc(ddqcd_t ctx, double *out, const double *in, void *stream);

/* Solves A x = b for nrhs right-hand sides with SAP-preconditioned FGCR.  If
 * x_is_guess, x holds the initial guess; else it starts from zero.  info
 * (optional) receives nrhs records.  Returns DDQCD_OK when every right-hand
 * side converged, DDQCD_ERR_NOT_CONVERGED otherwise (x then holds the last
 * iterate).  b and x must not alias. */
int ddqcd_solve(ddqcd_t ctx, double *x, const double *b, int nrhs, int x_is_guess, ddqcd_info *info, void *stream);

/* Solves n independent systems A_i x_i = b_i at once: system i belongs to
 * context ctxs[i] (a context may appear several times: its right-hand sides),
 * and x[i], b[i] are device pointers to one spinor field each in that
 * context's canonical layout.  The contexts may differ in lattice, domain
 * shape, kappa, c_sw, gauge field and block-solve precision, but must share
 * restart, tol, max_cycles and n_cycles (DDQCD_ERR_ARG otherwise).  Each half-
 * sweep of the preconditioner is one launch per (domain shape, precision)
 * over the domains of every system, so small lattices fill the device
 * together; each system stops when it has converged.  The parallelism over
 * configurations and sources is the batch dimension of Sec. IV-B2 (n_domain
 * per half-sweep times the number of systems).  x_is_guess and info as for
 * ddqcd_solve (info receives n records).  The return value is that of
 * ddqcd_solve over all systems; an error names the context in its
 * ddqcd_last_error. */
int ddqcd_solve_batch(const ddqcd_t *ctxs, int n, double *const *x, const double *const *b, int x_is_guess,
                      ddqcd_info *info, void *stream);

/* Solves A x = b (one right-hand side, canonical layouts, device pointers) with
 * BiCGstab in FP64 on the full operator and no preconditioner: the solver
 * without domain decomposition that the paper measures its method against
 * (Sec. IV-C: double-precision BiCGstab).  The same stopping rule as
 * ddqcd_solve (true relative residual <= the tol of ddqcd_set_solver; a
 * recursive residual below tol is confirmed with b - A x, and the iteration
 * restarts from it if not met).  At most max_iter iterations (each two
 * applications of A).  info (optional) receives iters, restarts,
 * rel_residual, converged and t_total_ms.  Returns DDQCD_OK,
 * DDQCD_ERR_NOT_CONVERGED (x holds the last iterate) or DDQCD_ERR_NONFINITE
 * on breakdown. */
int ddqcd_solve_bicgstab(ddqcd_t ctx, double *x, const double *b, int x_is_guess, int max_iter, ddqcd_info *info,
                         void *stream);

/* Picks a domain shape for a lattice.  The domain size trades the number of
 * independent block solves per half-sweep (Sec. IV-B2's n_domain, the
 * parallelism) against the strength of the preconditioner (larger blocks,
 * fewer outer iterations; Sec. II-D, IV-C), and the best trade depends on the
 * lattice and the gauge field, so it is measured: for every compiled
 * block-solve shape (2x2x2x2, 4x4x4x4, 8x4x4x4, 4x4x4x8, 6x6x2x4; 6x6x2x4 has
 * no FP64 kernel) that tiles the lattice with an even number (>= 2) of
 * domains in each direction and has a kernel for prec, a context is created, U loaded (device pointer,
 * canonical layout) and b solved (device pointer, canonical layout, one
 * right-hand side) twice with the given settings; the second solve is timed.
 * The fastest shape that converged is written to domain_out and its solve time
 * in milliseconds to ms_out (optional).  Products: DDQCD_PRODUCT_LANE.  If only one shape fits, it is
 * returned without timing and ms_out is set to -1.  Allocates and frees its
 * own device memory (one solution vector and the candidates' contexts, one at
 * a time).  Returns DDQCD_ERR_GEOMETRY if no compiled shape fits, otherwise
 * the error of the last failing candidate if none converged. */
int ddqcd_tune_domain(const int lattice[4], double kappa, double c_sw, const double boundary[4], const double *U,
                      const double *b, int prec, int n_cycles, int n_mr, int restart, double tol, int max_cycles,
                      int domain_out[4], double *ms_out, void *stream);

/* ddqcd_tune_domain for nrhs right-hand sides solved together (b: nrhs
 * spinor fields, canonical layout, one after the other) over the pairs (domain
 * shape, product form): for every compiled shape that tiles the lattice and
 * every ddqcd_product its kernels offer for prec (the tile forms only when
 * nrhs >= 2: they take four right-hand sides per workgroup), a context is
 * created, U loaded and the nrhs systems solved twice, the second solve timed;
 * the fastest pair that converged is written to domain_out and product_out
 * (optional), its time in milliseconds to ms_out (optional; -1 when only one
 * pair fits and nothing was timed).  Allocates and frees its own device memory
 * (nrhs solution vectors and the candidates' contexts, one at a time).  Errors
 * as ddqcd_tune_domain.  When the environment variable DDQCD_TUNE_CACHE names
 * a file, both calls keep their results there, one text line per problem, the
 * key made of every argument above except b and stream, with a fingerprint of U
 * (a hash of its first 64 numbers); a problem found in the file (whose pair is
 * still a candidate) is answered from it without any timing, with the stored
 * time; a new result is appended.  The file is read and appended with plain
 * stdio: processes tuning at once may interleave lines. */
int ddqcd_tune_sap(const int lattice[4], double kappa, double c_sw, const double boundary[4], const double *U,
                   const double *b, int nrhs, int prec, int n_cycles, int n_mr, int restart, double tol, int max_cycles,
                   int domain_out[4], int *product_out, double *ms_out, void *stream);

/* Text of the last error on this context (never NULL; "" if none). */
const char *ddqcd_last_error(ddqcd_t ctx);

/* Name of a status code. */
const char *ddqcd_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* DDQCD_H */
