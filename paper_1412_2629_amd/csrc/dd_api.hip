// The C-ABI of include/ddqcd.h: context management, argument validation,
// the preconditioner driver and the flexible GCR outer solver.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ddqcd.h"
#include "dd_internal.h"

using namespace dd;

struct ddqcd_ctx {
    Geo g{};
    double kappa = 0, csw = 0;
    int n_cycles = 16, n_mr = 5, sap_prec = DDQCD_FP32;
    int restart = 16, max_cycles = 64;
    int schedule = DDQCD_SCHED_SWEEPS;
    int n_cu = 0;
    int epoch_base = 0;
    std::vector<int> order_host;
    double tol = 1e-10;
    std::string err;
    std::vector<int> dom_host[2];
    bool loaded = false;
    int device = -1;

    // device memory (owned)
    int *d_dom[2] = {nullptr, nullptr};
    int *d_flag = nullptr;
    int *d_epoch = nullptr, *d_counter = nullptr, *d_qerr = nullptr, *d_order = nullptr;
    double2 *U64 = nullptr;      // [d][mu][9][Vd]
    void *U32 = nullptr, *U16 = nullptr;   // [d][mu][6][Vd]
    double2 *C64 = nullptr;      // [d][36][Vd]
    void *C32 = nullptr, *C16 = nullptr;
    double2 *Cs64 = nullptr;     // C_e / C_o^-1
    void *Cs32 = nullptr, *Cs16 = nullptr;
    // spinor work space
    double2 *t_in = nullptr, *t_out = nullptr;     // FP64 internal
    void *t_lo_in = nullptr, *t_lo_out = nullptr;  // FP32/FP16 internal (max size)
    void *psi = nullptr, *res = nullptr, *face = nullptr, *rho_tmp = nullptr;
    float *res_scale = nullptr, *face_scale = nullptr;
    double2 *x = nullptr, *r = nullptr, *b = nullptr, *Z = nullptr, *W = nullptr;
    int zw_restart = 0;
    Blas blas;
    std::vector<void *> owned;
};

namespace {

int fail(ddqcd_t c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                                   \
    do {                                                                                                    \
        hipError_t _e = (expr);                                                                             \
        if (_e != hipSuccess)                                                                               \
            return fail(ctx, _e == hipErrorOutOfMemory ? DDQCD_ERR_NOMEM : DDQCD_ERR_DEVICE,                \
                        std::string(#expr) + ": " + hipGetErrorString(_e));                                 \
    } while (0)

long nsites(const Geo &g) { return g.V; }
long ncomplex(const Geo &g) { return g.V * 12; }

size_t elem_bytes(int prec) { return prec == DDQCD_FP64 ? 16 : prec == DDQCD_FP32 ? 8 : 4; }

int dev_alloc(ddqcd_t c, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, DDQCD_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    c->owned.push_back(*p);
    return DDQCD_OK;
}

template <typename P> int alloc(ddqcd_t c, P **p, size_t bytes) { return dev_alloc(c, (void **)p, bytes); }

int check_device(ddqcd_t c)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(c, DDQCD_ERR_DEVICE, "no HIP device");
    if (c->device >= 0 && dev != c->device)
        return fail(c, DDQCD_ERR_STATE, "context was loaded on device " + std::to_string(c->device));
    return DDQCD_OK;
}

const void *links_for(ddqcd_t c, int prec) { return prec == DDQCD_FP64 ? (void *)c->U64 : prec == DDQCD_FP32 ? c->U32 : c->U16; }
const void *clover_for(ddqcd_t c, int prec) { return prec == DDQCD_FP64 ? (void *)c->C64 : prec == DDQCD_FP32 ? c->C32 : c->C16; }
const void *schur_for(ddqcd_t c, int prec) { return prec == DDQCD_FP64 ? (void *)c->Cs64 : prec == DDQCD_FP32 ? c->Cs32 : c->Cs16; }

int ensure_spinor_tmp(ddqcd_t c)
{
    if (c->t_in) return DDQCD_OK;
    size_t n = (size_t)ncomplex(c->g);
    int e;
    if ((e = alloc(c, &c->t_in, n * 16))) return e;
    if ((e = alloc(c, &c->t_out, n * 16))) return e;
    if ((e = alloc(c, &c->t_lo_in, n * 8))) return e;
    if ((e = alloc(c, &c->t_lo_out, n * 8))) return e;
    return DDQCD_OK;
}

int ensure_sap_space(ddqcd_t c)
{
    if (c->psi) return DDQCD_OK;
    const Geo &g = c->g;
    size_t n = (size_t)ncomplex(g);
    int e;
    if ((e = dev_alloc(c, &c->psi, n * 16))) return e;                    // FP64 or FP32 accumulator
    if ((e = dev_alloc(c, &c->res, (size_t)g.nd * 12 * g.Vh * 16))) return e;
    if ((e = dev_alloc(c, &c->rho_tmp, (size_t)g.nd * 12 * g.Vh * 16))) return e;
    if ((e = dev_alloc(c, &c->face, (size_t)g.nd * sap_face_sites(g.b) * 6 * 16))) return e;
    if ((e = alloc(c, &c->res_scale, (size_t)g.nd * 4))) return e;
    if ((e = alloc(c, &c->face_scale, (size_t)g.nd * 4))) return e;
    return DDQCD_OK;
}

int ensure_solver_space(ddqcd_t c)
{
    size_t n = (size_t)ncomplex(c->g);
    int e;
    if (!c->x) {
        if ((e = alloc(c, &c->x, n * 16))) return e;
        if ((e = alloc(c, &c->r, n * 16))) return e;
        if ((e = alloc(c, &c->b, n * 16))) return e;
    }
    if (c->zw_restart < c->restart) {
        // grow the basis (the old one, if any, stays owned until destroy)
        if ((e = alloc(c, &c->Z, n * 16 * c->restart))) return e;
        if ((e = alloc(c, &c->W, n * 16 * c->restart))) return e;
        c->zw_restart = c->restart;
    }
    return DDQCD_OK;
}

// psi = M eta on internal FP64 vectors
int run_sap(ddqcd_t c, const double2 *eta, double2 *out, hipStream_t s)
{
    int e = ensure_sap_space(c);
    if (e) return e;
    const int prec = c->sap_prec;
    SapArgs a{};
    a.g = c->g;
    a.n_mr = c->n_mr;
    a.eta = eta;
    a.out = out;
    a.psi = c->psi;
    a.res = c->res;
    a.res_scale = c->res_scale;
    a.face = c->face;
    a.face_scale = c->face_scale;
    a.rho_tmp = c->rho_tmp;
    a.links = links_for(c, prec);
    a.cs = schur_for(c, prec);
    if (c->schedule == DDQCD_SCHED_QUEUE && prec != DDQCD_FP64) {
        QueueArgs q{};
        q.epoch = c->d_epoch;
        q.counter = c->d_counter;
        q.error = c->d_qerr;
        q.base = c->epoch_base;
        q.n_cycles = c->n_cycles;
        q.nd = c->g.nd;
        q.nblack = (int)c->dom_host[0].size();
        q.order = c->d_order;
        HIPCHK(c, sap_queue(a, q, prec, c->n_cu, s));
        int qerr = 0;
        HIPCHK(c, hipMemcpyAsync(&qerr, c->d_qerr, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if (qerr) {
            HIPCHK(c, queue_reset_epochs(c->d_epoch, c->g.nd, c->d_qerr, s));
            c->epoch_base = 0;
            return fail(c, DDQCD_ERR_DEVICE, "SAP work queue: a dependency wait exceeded its limit");
        }
        c->epoch_base += c->n_cycles;
        if (c->epoch_base > (1 << 30)) {
            HIPCHK(c, queue_reset_epochs(c->d_epoch, c->g.nd, c->d_qerr, s));
            c->epoch_base = 0;
        }
        return DDQCD_OK;
    }
    for (int cyc = 0; cyc < c->n_cycles; cyc++)
        for (int col = 0; col < 2; col++) {
            a.dom = c->d_dom[col];
            a.ndom = (int)c->dom_host[col].size();
            a.first = cyc == 0;
            a.faces_in = !(cyc == 0 && col == 0);
            a.last = cyc == c->n_cycles - 1;
            a.faces_out = !(a.last && col == 1);
            a.res_out = !a.last;
            HIPCHK(c, sap_sweep(a, prec, s));
        }
    return DDQCD_OK;
}

int apply_A64(ddqcd_t c, const double2 *in, double2 *out, hipStream_t s)
{
    HIPCHK(c, apply_A(c->g, in, out, c->U64, c->C64, P64, s));
    return DDQCD_OK;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    double *acc;
    Timer(hipStream_t s_, double *acc_) : s(s_), acc(acc_)
    {
        if (acc) {
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            (void)hipEventRecord(a, s);
        }
    }
    void stop()
    {
        if (!acc) return;
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        *acc += ms;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        acc = nullptr;
    }
    ~Timer() { stop(); }
};

// reads result[0..m-1] of the last reduction
int fetch(ddqcd_t c, double2 *host, int m, hipStream_t s)
{
    HIPCHK(c, hipMemcpyAsync(host, c->blas.result, sizeof(double2) * m, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return DDQCD_OK;
}

int put_coef(ddqcd_t c, const std::vector<std::complex<double>> &v, hipStream_t s)
{
    static_assert(sizeof(std::complex<double>) == sizeof(double2), "layout");
    HIPCHK(c, hipMemcpyAsync(c->blas.coef, v.data(), sizeof(double2) * v.size(), hipMemcpyHostToDevice, s));
    return DDQCD_OK;
}

// FGCR on internal FP64 vectors b -> x (x holds the guess if guess)
int fgcr(ddqcd_t c, bool guess, ddqcd_info *info, hipStream_t s)
{
    const long n = ncomplex(c->g);
    const int m = c->restart;
    double2 *Z = c->Z, *W = c->W;
    double tsap = 0, tA = 0, tgs = 0, tother = 0;
    double2 h[32];
    int e;
    using C = std::complex<double>;
    std::vector<C> a((size_t)m * m), cc(m), alpha(m);
    std::vector<double> bb(m);

    if (!guess) HIPCHK(c, zero(c->x, n, s));
    HIPCHK(c, norm2(c->blas, c->b, n, s));
    if ((e = fetch(c, h, 1, s))) return e;
    const double bn = std::sqrt(h[0].x);
    int steps = 0, cycles = 0, status = DDQCD_ERR_NOT_CONVERGED;
    double rel = 0;
    if (!std::isfinite(bn)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite right-hand side");
    if (bn == 0) {
        HIPCHK(c, zero(c->x, n, s));
        status = DDQCD_OK;
        goto done;
    }
    {
        Timer t(s, &tA);
        if ((e = apply_A64(c, c->x, c->r, s))) return e;
    }
    {
        Timer t(s, &tother);
        HIPCHK(c, residual(c->blas, c->b, c->r, n, s));
        if ((e = fetch(c, h, 1, s))) return e;
    }
    rel = std::sqrt(h[0].x) / bn;
    if (!std::isfinite(rel)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite residual");
    if (rel <= c->tol) {
        status = DDQCD_OK;
        goto done;
    }
    for (cycles = 0; cycles < c->max_cycles;) {
        int kend = 0;
        for (int k = 0; k < m; k++) {
            double2 *zk = Z + (long)k * n, *wk = W + (long)k * n;
            {
                Timer t(s, &tsap);
                if ((e = run_sap(c, c->r, zk, s))) return e;
            }
            {
                Timer t(s, &tA);
                if ((e = apply_A64(c, zk, wk, s))) return e;
            }
            {
                Timer t(s, &tgs);
                // classical Gram-Schmidt against the earlier w-hat, repeated once
                // if the new vector lost more than half its norm
                for (int j = 0; j < k; j++) a[(size_t)j * m + k] = 0;
                double before = 0, wn2 = 0;
                C wr;
                for (int pass = 0; pass < 2; pass++) {
                    std::vector<C> coef(k);
                    if (k > 0) {
                        HIPCHK(c, multidot(c->blas, W, n, k, wk, n, s));
                        if ((e = fetch(c, h, k, s))) return e;
                        for (int j = 0; j < k; j++) {
                            coef[j] = C(h[j].x, h[j].y);
                            a[(size_t)j * m + k] += coef[j];
                        }
                        if ((e = put_coef(c, coef, s))) return e;
                    }
                    if (pass == 0) {
                        HIPCHK(c, norm2(c->blas, wk, n, s));
                        if ((e = fetch(c, h, 1, s))) return e;
                        before = h[0].x;
                    }
                    HIPCHK(c, cgs_update(c->blas, wk, W, n, k, c->r, n, s));
                    if ((e = fetch(c, h, 2, s))) return e;
                    wn2 = h[0].x;
                    wr = C(h[1].x, h[1].y);
                    if (k == 0 || wn2 > 0.25 * before) break;
                    before = wn2;
                }
                bb[k] = std::sqrt(wn2);
                if (!(bb[k] > 0) || !std::isfinite(bb[k]))
                    return fail(c, DDQCD_ERR_NONFINITE, "breakdown: A M r vanished or is non-finite");
                cc[k] = wr / bb[k];
                HIPCHK(c, normalize_update(c->blas, wk, 1.0 / bb[k], c->r, make_double2(cc[k].real(), cc[k].imag()), n, s));
                if ((e = fetch(c, h, 1, s))) return e;
            }
            steps++;
            kend = k + 1;
            rel = std::sqrt(h[0].x) / bn;
            if (!std::isfinite(rel)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite residual");
            if (rel <= c->tol) break;
        }
        {
            Timer t(s, &tother);
            for (int k = kend - 1; k >= 0; k--) {
                C sum = cc[k];
                for (int j = k + 1; j < kend; j++) sum -= a[(size_t)k * m + j] * alpha[j];
                alpha[k] = sum / bb[k];
            }
            std::vector<C> al(alpha.begin(), alpha.begin() + kend);
            if ((e = put_coef(c, al, s))) return e;
            HIPCHK(c, axpy_multi(c->blas, c->x, Z, n, kend, n, s));
        }
        {
            Timer t(s, &tA);
            if ((e = apply_A64(c, c->x, c->r, s))) return e;
        }
        {
            Timer t(s, &tother);
            HIPCHK(c, residual(c->blas, c->b, c->r, n, s));
            if ((e = fetch(c, h, 1, s))) return e;
        }
        cycles++;
        rel = std::sqrt(h[0].x) / bn;
        if (!std::isfinite(rel)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite residual");
        if (rel <= c->tol) {
            status = DDQCD_OK;
            break;
        }
    }
done:
    if (info) {
        info->converged = status == DDQCD_OK;
        info->iters = steps;
        info->restarts = cycles;
        info->rel_residual = rel;
        info->t_sap_ms = tsap;
        info->t_A_ms = tA;
        info->t_gs_ms = tgs;
        info->t_other_ms = tother;
    }
    if (status != DDQCD_OK) c->err = "not converged: relative residual " + std::to_string(rel);
    return status;
}

bool is_pm1(double v) { return v == 1.0 || v == -1.0; }

}  // namespace

// ===========================================================================
// exported entry points
// ===========================================================================

extern "C" {

const char *ddqcd_status_string(int st)
{
    switch (st) {
        case DDQCD_OK: return "DDQCD_OK";
        case DDQCD_ERR_ARG: return "DDQCD_ERR_ARG";
        case DDQCD_ERR_GEOMETRY: return "DDQCD_ERR_GEOMETRY";
        case DDQCD_ERR_STATE: return "DDQCD_ERR_STATE";
        case DDQCD_ERR_DEVICE: return "DDQCD_ERR_DEVICE";
        case DDQCD_ERR_NOMEM: return "DDQCD_ERR_NOMEM";
        case DDQCD_ERR_NOT_CONVERGED: return "DDQCD_ERR_NOT_CONVERGED";
        case DDQCD_ERR_NONFINITE: return "DDQCD_ERR_NONFINITE";
        default: return "unknown status";
    }
}

const char *ddqcd_last_error(ddqcd_t c) { return c ? c->err.c_str() : "null context"; }

int ddqcd_create(const int lattice[4], const int domain[4], double kappa, double c_sw, const double boundary[4],
                 ddqcd_t *out)
{
    if (!lattice || !domain || !boundary || !out) return DDQCD_ERR_ARG;
    if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(c_sw)) return DDQCD_ERR_ARG;
    for (int m = 0; m < 4; m++) {
        if (!is_pm1(boundary[m])) return DDQCD_ERR_ARG;
        if (lattice[m] < 2 || domain[m] < 2) return DDQCD_ERR_GEOMETRY;
        if (domain[m] % 2 || lattice[m] % domain[m]) return DDQCD_ERR_GEOMETRY;
        int n = lattice[m] / domain[m];
        if (n < 2 || n % 2) return DDQCD_ERR_GEOMETRY;
    }
    if (!sap_shape_supported(domain)) return DDQCD_ERR_GEOMETRY;
    long V = (long)lattice[0] * lattice[1] * lattice[2] * lattice[3];
    if (V * 12 > (1L << 40)) return DDQCD_ERR_GEOMETRY;
    ddqcd_ctx *c = new (std::nothrow) ddqcd_ctx();
    if (!c) return DDQCD_ERR_NOMEM;
    Geo &g = c->g;
    for (int m = 0; m < 4; m++) {
        g.L[m] = lattice[m];
        g.b[m] = domain[m];
        g.n[m] = lattice[m] / domain[m];
        g.bc[m] = boundary[m];
    }
    g.Vd = domain[0] * domain[1] * domain[2] * domain[3];
    g.Vh = g.Vd / 2;
    g.nd = g.n[0] * g.n[1] * g.n[2] * g.n[3];
    g.V = V;
    c->kappa = kappa;
    c->csw = c_sw;
    for (int d = 0; d < g.nd; d++) {
        int r = d, s = 0;
        for (int m = 0; m < 4; m++) {
            s += r % g.n[m];
            r /= g.n[m];
        }
        c->dom_host[s & 1].push_back(d);
    }
    c->order_host = c->dom_host[0];
    c->order_host.insert(c->order_host.end(), c->dom_host[1].begin(), c->dom_host[1].end());
    *out = c;
    return DDQCD_OK;
}

int ddqcd_destroy(ddqcd_t c)
{
    if (!c) return DDQCD_OK;
    for (void *p : c->owned) (void)hipFree(p);
    c->blas.release();
    delete c;
    return DDQCD_OK;
}

int ddqcd_set_sap(ddqcd_t c, int n_cycles, int n_mr, int prec)
{
    if (!c) return DDQCD_ERR_ARG;
    if (n_cycles < 1 || n_mr < 1 || n_cycles > 1000 || n_mr > 1000) return fail(c, DDQCD_ERR_ARG, "bad SAP iteration counts");
    if (prec != DDQCD_FP64 && prec != DDQCD_FP32 && prec != DDQCD_FP16) return fail(c, DDQCD_ERR_ARG, "bad precision");
    if (!sap_prec_supported(c->g.b, prec))
        return fail(c, DDQCD_ERR_GEOMETRY, "FP64 block solves are available for 2x2x2x2 domains only");
    c->n_cycles = n_cycles;
    c->n_mr = n_mr;
    c->sap_prec = prec;
    return DDQCD_OK;
}

int ddqcd_set_schedule(ddqcd_t c, int schedule)
{
    if (!c) return DDQCD_ERR_ARG;
    if (schedule != DDQCD_SCHED_SWEEPS && schedule != DDQCD_SCHED_QUEUE) return fail(c, DDQCD_ERR_ARG, "bad schedule");
    if (schedule == DDQCD_SCHED_QUEUE)
        return fail(c, DDQCD_ERR_ARG, "the work-queue schedule is switched off: it stalled on the device and its cause "
                                      "is not established");
    c->schedule = schedule;
    return DDQCD_OK;
}

int ddqcd_set_solver(ddqcd_t c, int restart, double tol, int max_cycles)
{
    if (!c) return DDQCD_ERR_ARG;
    if (restart < 1 || restart > BLAS_MAXK) return fail(c, DDQCD_ERR_ARG, "restart must be in [1, 16]");
    if (!(tol > 0) || !std::isfinite(tol) || max_cycles < 1) return fail(c, DDQCD_ERR_ARG, "bad tolerance or cycle limit");
    c->restart = restart;
    c->tol = tol;
    c->max_cycles = max_cycles;
    return DDQCD_OK;
}

int ddqcd_load_gauge(ddqcd_t c, const double *U, void *stream)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!U) return fail(c, DDQCD_ERR_ARG, "null gauge field");
    int e = check_device(c);
    if (e) return e;
    hipStream_t s = (hipStream_t)stream;
    const Geo &g = c->g;
    const size_t V = (size_t)g.V;
    if (c->device < 0) {
        HIPCHK(c, hipGetDevice(&c->device));
        HIPCHK(c, c->blas.init());
        for (int col = 0; col < 2; col++) {
            if ((e = alloc(c, &c->d_dom[col], c->dom_host[col].size() * sizeof(int)))) return e;
            HIPCHK(c, hipMemcpy(c->d_dom[col], c->dom_host[col].data(), c->dom_host[col].size() * sizeof(int),
                                hipMemcpyHostToDevice));
        }
        if ((e = alloc(c, &c->d_flag, sizeof(int)))) return e;
        if ((e = alloc(c, &c->d_epoch, sizeof(int) * g.nd))) return e;
        if ((e = alloc(c, &c->d_counter, sizeof(int)))) return e;
        if ((e = alloc(c, &c->d_qerr, sizeof(int)))) return e;
        if ((e = alloc(c, &c->d_order, sizeof(int) * g.nd))) return e;
        HIPCHK(c, hipMemcpy(c->d_order, c->order_host.data(), sizeof(int) * g.nd, hipMemcpyHostToDevice));
        HIPCHK(c, queue_reset_epochs(c->d_epoch, g.nd, c->d_qerr, s));
        c->epoch_base = 0;
        HIPCHK(c, hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
        if ((e = alloc(c, &c->U64, V * 4 * 9 * 16))) return e;
        if ((e = dev_alloc(c, &c->U32, V * 4 * 6 * 8))) return e;
        if ((e = dev_alloc(c, &c->U16, V * 4 * 6 * 4))) return e;
        if ((e = alloc(c, &c->C64, V * 36 * 16))) return e;
        if ((e = dev_alloc(c, &c->C32, V * 36 * 8))) return e;
        if ((e = dev_alloc(c, &c->C16, V * 36 * 4))) return e;
        if ((e = alloc(c, &c->Cs64, V * 36 * 16))) return e;
        if ((e = dev_alloc(c, &c->Cs32, V * 36 * 8))) return e;
        if ((e = dev_alloc(c, &c->Cs16, V * 36 * 4))) return e;
    }
    HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
    HIPCHK(c, count_nonfinite((const double2 *)U, (long)V * 36, c->d_flag, s));
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (bad) return fail(c, DDQCD_ERR_NONFINITE, "non-finite gauge field");
    HIPCHK(c, import_gauge(g, U, c->U64, s));
    HIPCHK(c, compress_links(g, c->U64, c->U32, P32, s));
    HIPCHK(c, compress_links(g, c->U64, c->U16, P16, s));
    HIPCHK(c, clover_build(g, c->U64, c->kappa, c->csw, c->C64, s));
    HIPCHK(c, convert_pairs(c->C64, c->C32, (long)V * 36, P32, s));
    HIPCHK(c, convert_pairs(c->C64, c->C16, (long)V * 36, P16, s));
    HIPCHK(c, clover_schur(g, c->C64, c->Cs64, c->d_flag, s));
    HIPCHK(c, convert_pairs(c->Cs64, c->Cs32, (long)V * 36, P32, s));
    HIPCHK(c, convert_pairs(c->Cs64, c->Cs16, (long)V * 36, P16, s));
    HIPCHK(c, hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (bad) return fail(c, DDQCD_ERR_ARG, "singular clover block on an odd site");
    c->loaded = true;
    return DDQCD_OK;
}

int ddqcd_apply_D(ddqcd_t c, double *out, const double *in, int nrhs, int prec, void *stream)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!out || !in || nrhs < 1 || out == in) return fail(c, DDQCD_ERR_ARG, "bad apply_D arguments");
    if (prec != DDQCD_FP64 && prec != DDQCD_FP32 && prec != DDQCD_FP16) return fail(c, DDQCD_ERR_ARG, "bad precision");
    if (!c->loaded) return fail(c, DDQCD_ERR_STATE, "apply_D before load_gauge");
    int e = check_device(c);
    if (e || (e = ensure_spinor_tmp(c))) return e;
    hipStream_t s = (hipStream_t)stream;
    const Geo &g = c->g;
    const long n = ncomplex(g);
    for (int k = 0; k < nrhs; k++) {
        const double *ik = in + (size_t)k * n * 2;
        double *ok = out + (size_t)k * n * 2;
        void *ti = prec == DDQCD_FP64 ? (void *)c->t_in : c->t_lo_in;
        void *to = prec == DDQCD_FP64 ? (void *)c->t_out : c->t_lo_out;
        HIPCHK(c, import_spinor(g, ik, ti, prec, s));
        HIPCHK(c, apply_A(g, ti, to, links_for(c, prec), clover_for(c, prec), prec, s));
        HIPCHK(c, export_spinor(g, to, prec, ok, s));
    }
    return DDQCD_OK;
}

int ddqcd_sap(ddqcd_t c, double *out, const double *in, int nrhs, void *stream)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!out || !in || nrhs < 1 || out == in) return fail(c, DDQCD_ERR_ARG, "bad sap arguments");
    if (!c->loaded) return fail(c, DDQCD_ERR_STATE, "sap before load_gauge");
    int e = check_device(c);
    if (e || (e = ensure_spinor_tmp(c))) return e;
    hipStream_t s = (hipStream_t)stream;
    const Geo &g = c->g;
    const long n = ncomplex(g);
    for (int k = 0; k < nrhs; k++) {
        HIPCHK(c, import_spinor(g, in + (size_t)k * n * 2, c->t_in, P64, s));
        if ((e = run_sap(c, c->t_in, c->t_out, s))) return e;
        HIPCHK(c, export_spinor(g, c->t_out, P64, out + (size_t)k * n * 2, s));
    }
    return DDQCD_OK;
}

int ddqcd_solve(ddqcd_t c, double *x, const double *b, int nrhs, int x_is_guess, ddqcd_info *info, void *stream)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!x || !b || nrhs < 1 || x == b) return fail(c, DDQCD_ERR_ARG, "bad solve arguments");
    if (!c->loaded) return fail(c, DDQCD_ERR_STATE, "solve before load_gauge");
    int e = check_device(c);
    if (e || (e = ensure_solver_space(c))) return e;
    hipStream_t s = (hipStream_t)stream;
    const Geo &g = c->g;
    const long n = ncomplex(g);
    int status = DDQCD_OK;
    for (int k = 0; k < nrhs; k++) {
        auto t0 = std::chrono::steady_clock::now();
        ddqcd_info inf{};
        HIPCHK(c, import_spinor(g, b + (size_t)k * n * 2, c->b, P64, s));
        if (x_is_guess) HIPCHK(c, import_spinor(g, x + (size_t)k * n * 2, c->x, P64, s));
        int st = fgcr(c, x_is_guess != 0, &inf, s);
        if (st != DDQCD_OK && st != DDQCD_ERR_NOT_CONVERGED) return st;
        HIPCHK(c, export_spinor(g, c->x, P64, x + (size_t)k * n * 2, s));
        HIPCHK(c, hipStreamSynchronize(s));
        inf.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (info) info[k] = inf;
        if (st != DDQCD_OK) status = st;
    }
    return status;
}

}  // extern "C"
