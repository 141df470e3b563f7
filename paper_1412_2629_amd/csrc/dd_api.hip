// The C-ABI of include/ddqcd.h: context management, argument validation,
// the preconditioner driver and the flexible GCR outer solver.
//
// A "system" is one right-hand side of one lattice (context).  Solves and
// preconditioner calls work on a list of systems in lockstep: one block-solve
// launch per colour of a half-sweep covers every system of one domain shape
// and storage precision, and the outer solver's reductions for all systems are
// read back with one host synchronisation per round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <array>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ddqcd.h"
#include "dd_internal.h"

using namespace dd;

// ---- device scratch of ddqcd_sap_noalloc ------------------------------------
//
// One copy of this array lives on every device the library runs on, for the
// life of the process.  Host code never uses its name as an address: the
// device address is looked up once per device (scratch_setup) and kept in
// scratch_dev.
constexpr size_t SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

std::mutex scratch_mu;
std::map<int, unsigned char *> scratch_dev;   // device -> address of its scratch

// Looks up this device's scratch address (the device must be current).
hipError_t scratch_setup(int device)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev.count(device)) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_dev[device] = (unsigned char *)p;
    return hipSuccess;
}

unsigned char *scratch_for(int device)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    auto it = scratch_dev.find(device);
    return it == scratch_dev.end() ? nullptr : it->second;
}

// work space of one right-hand side of a context
struct Slot {
    void *psi = nullptr, *res = nullptr, *face = nullptr, *rho_tmp = nullptr;   // block solves
    float *res_scale = nullptr, *face_scale = nullptr;
    void *face_alt = nullptr;                                                    // additive schedule
    float *face_scale_alt = nullptr;
    double2 *x = nullptr, *r = nullptr, *b = nullptr;                            // FP64 vectors
    double2 *Z = nullptr, *W = nullptr;                                          // FGCR basis
    int zw_restart = 0;
    double2 *rcoef = nullptr;   // restart recombination matrix (FGMRES-DR)
    Blas blas;
};

// Device-side description of the block solves of a list of systems: the
// per-system argument array and, per (domain shape, precision) group and
// colour, the list of (system, domain) work items.  Workgroup i of a launch
// runs on XCD i mod 8; the items of one lattice domain (the right-hand sides
// of one context) are placed on one XCD, so that domain's links and clover
// blocks are fetched into one L2.
struct Plan {
    struct Group {
        int shape = 0, prec = 0, product = 0;
        int2 *items[3] = {nullptr, nullptr, nullptr};   // black, white, all domains
        int nitems[3] = {0, 0, 0};
    };
    bool additive = false;
    std::vector<Group> groups;
    SapArgs *d_args = nullptr;
    std::vector<SapArgs> h_args;
    hipGraphExec_t graph = nullptr;   // the launches of one preconditioner call
    int graph_cycles = -1;
    bool in_workspace = false;        // device arrays carved from the caller's workspace
    ~Plan()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (in_workspace) return;
        (void)hipFree(d_args);
        for (Group &G : groups)
            for (int c = 0; c < 3; c++) (void)hipFree(G.items[c]);
    }
};

constexpr int N_XCD = 8;
constexpr int RCOEF = 24 * 24;   // entries of a slot's restart recombination matrix
constexpr size_t MAX_PLANS = 32;

}  // namespace

struct ddqcd_ctx {
    Geo g{};
    double kappa = 0, csw = 0;
    int n_cycles = 16, n_mr = 5, sap_prec = DDQCD_FP32, product = DDQCD_PRODUCT_LANE;
    int restart = 16, max_cycles = 64;
    int outer = DDQCD_OUTER_FGCR, deflate = 0;   // outer solver, FGMRES-DR deflation vectors
    double tol = 1e-10;
    int schedule = DDQCD_SCHED_SWEEPS;
    int schwarz = DDQCD_SCHWARZ_MULTIPLICATIVE;
    std::string err;
    std::vector<int> dom_host[2];   // black (0) and white (1) domains
    bool loaded = false;
    int device = -1;

    // device memory (owned)
    int *d_flag = nullptr;
    double2 *U64 = nullptr;                // [d][mu][9][Vd]
    void *U32 = nullptr, *U16 = nullptr, *UB16 = nullptr;   // [d][mu][6][Vd]
    double2 *C64 = nullptr;                // [d][36][Vd]
    void *C32 = nullptr, *C16 = nullptr, *CB16 = nullptr;
    double2 *Cs64 = nullptr;               // C_e / C_o^-1
    void *Cs32 = nullptr, *Cs16 = nullptr, *CsB16 = nullptr;
    void *t_lo_in = nullptr, *t_lo_out = nullptr;   // FP32/FP16 operands of apply_D
    hipStream_t capture = nullptr;   // private stream on which launch graphs are captured
    // reduction results of the systems of a solve led by this context, side by
    // side (32 pairs each) on the device and in pinned host memory
    double2 *res_dev = nullptr, *res_host = nullptr;
    int res_cap = 0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::map<std::string, std::unique_ptr<Plan>> plans;   // batch plans led by this context
    std::vector<void *> owned;
    // caller-owned workspace (ddqcd_set_workspace): every device array of the
    // context is carved from it (bump allocation, 256-byte aligned) instead of
    // hipMalloc; the plans live in a region at its top that is reset when full
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0, ws_used = 0;
    unsigned char *ws_plan = nullptr;
    size_t ws_plan_bytes = 0, ws_plan_used = 0;
    int ws_nrhs = 0;
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

long ncomplex(const Geo &g) { return g.V * 12; }

size_t aligned(size_t bytes) { return (bytes + 255) / 256 * 256; }

int dev_alloc(ddqcd_t c, void **p, size_t bytes)
{
    if (c->ws) {
        const size_t need = aligned(bytes);
        if (c->ws_used + need > c->ws_bytes - c->ws_plan_bytes) {
            *p = nullptr;
            return fail(c, DDQCD_ERR_NOMEM, "the workspace is too small: " + std::to_string(need) +
                                                " more bytes needed (ddqcd_workspace_size)");
        }
        *p = c->ws + c->ws_used;
        c->ws_used += need;
        return DDQCD_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, DDQCD_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    c->owned.push_back(*p);
    return DDQCD_OK;
}

template <typename P> int alloc(ddqcd_t c, P **p, size_t bytes) { return dev_alloc(c, (void **)p, bytes); }

// device array of a plan: hipMalloc, or carved from the workspace's plan
// region (false when the region is full)
bool plan_alloc(ddqcd_t lead, void **p, size_t bytes)
{
    if (!lead->ws) return hipMalloc(p, bytes) == hipSuccess;
    const size_t need = aligned(bytes);
    if (lead->ws_plan_used + need > lead->ws_plan_bytes) return false;
    *p = lead->ws_plan + lead->ws_plan_used;
    lead->ws_plan_used += need;
    return true;
}

int check_device(ddqcd_t c)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(c, DDQCD_ERR_DEVICE, "no HIP device");
    if (c->device >= 0 && dev != c->device)
        return fail(c, DDQCD_ERR_STATE, "context was loaded on device " + std::to_string(c->device));
    return DDQCD_OK;
}

int check_ready(ddqcd_t c, const char *what)
{
    if (!c->loaded) return fail(c, DDQCD_ERR_STATE, std::string(what) + " before load_gauge");
    return check_device(c);
}

// the copies of the links, clover term and C_e / C_o^-1 in one storage precision
const void *links_for(ddqcd_t c, int prec)
{
    const void *f[4] = {c->U64, c->U32, c->U16, c->UB16};
    return f[prec];
}
const void *clover_for(ddqcd_t c, int prec)
{
    const void *f[4] = {c->C64, c->C32, c->C16, c->CB16};
    return f[prec];
}
const void *schur_for(ddqcd_t c, int prec)
{
    const void *f[4] = {c->Cs64, c->Cs32, c->Cs16, c->CsB16};
    return f[prec];
}
bool valid_prec(int prec) { return prec >= DDQCD_FP64 && prec <= DDQCD_BF16; }

// ---- per right-hand-side work space ----------------------------------------

int ensure_slots(ddqcd_t c, int n)
{
    const Geo &g = c->g;
    const size_t nc = (size_t)ncomplex(g);
    while ((int)c->slots.size() < n) {
        auto sl = std::make_unique<Slot>();
        int e;
        if ((e = dev_alloc(c, &sl->psi, nc * 16))) return e;   // FP64 or FP32 accumulator
        if ((e = dev_alloc(c, &sl->res, (size_t)g.nd * 12 * g.Vh * 16))) return e;
        if ((e = dev_alloc(c, &sl->rho_tmp, (size_t)g.nd * 12 * g.Vh * 16))) return e;
        if ((e = dev_alloc(c, &sl->face, (size_t)g.nd * sap_face_sites(g.b) * 6 * 16))) return e;
        if ((e = alloc(c, &sl->res_scale, (size_t)g.nd * 4))) return e;
        if ((e = alloc(c, &sl->face_scale, (size_t)g.nd * 4))) return e;
        if ((e = alloc(c, &sl->x, nc * 16))) return e;
        if ((e = alloc(c, &sl->r, nc * 16))) return e;
        if ((e = alloc(c, &sl->b, nc * 16))) return e;
        if ((e = alloc(c, &sl->blas.partial, sizeof(double2) * BLAS_NBLK * 32))) return e;
        if ((e = alloc(c, &sl->blas.result, sizeof(double2) * 32))) return e;
        if ((e = alloc(c, &sl->blas.coef, sizeof(double2) * 32))) return e;
        if ((e = alloc(c, &sl->rcoef, sizeof(double2) * RCOEF))) return e;
        c->slots.push_back(std::move(sl));
    }
    return DDQCD_OK;
}

// columns of each of the two basis arrays: FGCR's z and w (restart), FGMRES-DR's
// z and v with room for the restart recombination (restart + deflate + 2), at
// least 5 (the BiCGstab work vectors)
int basis_columns(ddqcd_t c)
{
    const int outer = c->outer == DDQCD_OUTER_FGMRES_DR ? c->restart + c->deflate + 2 : c->restart;
    return std::max(outer, 5);
}

int ensure_basis(ddqcd_t c, Slot &sl, int columns = 0)
{
    const int want = std::max(columns, basis_columns(c));
    if (sl.zw_restart >= want) return DDQCD_OK;
    const size_t nc = (size_t)ncomplex(c->g);
    int e;
    // grow the basis (a smaller old one stays owned until destroy)
    if ((e = alloc(c, &sl.Z, nc * 16 * want))) return e;
    if ((e = alloc(c, &sl.W, nc * 16 * want))) return e;
    sl.zw_restart = want;
    return DDQCD_OK;
}

// ---- systems and batch plans ------------------------------------------------

struct Sys {
    ddqcd_t c;
    Slot *sl;
    int slot;
};

// the plan depends on each system's context, slot, precision and geometry
std::string plan_key(const std::vector<Sys> &sys)
{
    std::string k = sys[0].c->schwarz == DDQCD_SCHWARZ_ADDITIVE ? "A;" : "M;";
    char buf[160];
    for (const Sys &s : sys) {
        const Geo &g = s.c->g;
        snprintf(buf, sizeof buf, "%p:%d:%d:%d:%d,%d,%d,%d:%d,%d,%d,%d;", (void *)s.c, s.slot, s.c->sap_prec,
                 s.c->product, g.L[0], g.L[1], g.L[2], g.L[3], g.b[0], g.b[1], g.b[2], g.b[3]);
        k += buf;
    }
    return k;
}

int build_plan_once(const std::vector<Sys> &sys, const std::string &key, Plan *&out);

int build_plan(const std::vector<Sys> &sys, Plan *&out)
{
    ddqcd_t lead = sys[0].c;
    const std::string key = plan_key(sys);
    auto it = lead->plans.find(key);
    if (it != lead->plans.end()) {
        out = it->second.get();
        return DDQCD_OK;
    }
    if (lead->plans.size() >= MAX_PLANS) {
        HIPCHK(lead, hipDeviceSynchronize());   // no launch may still read an old plan
        lead->plans.clear();
        lead->ws_plan_used = 0;
    }
    int e = build_plan_once(sys, key, out);
    if (e == DDQCD_ERR_NOMEM && lead->ws && !lead->plans.empty()) {
        // the workspace's plan region is full: drop the cached plans and retry
        HIPCHK(lead, hipDeviceSynchronize());
        lead->plans.clear();
        lead->ws_plan_used = 0;
        e = build_plan_once(sys, key, out);
    }
    return e;
}

int build_plan_once(const std::vector<Sys> &sys, const std::string &key, Plan *&out)
{
    ddqcd_t lead = sys[0].c;
    auto plan = std::make_unique<Plan>();
    plan->in_workspace = lead->ws != nullptr;
    if (!plan_alloc(lead, (void **)&plan->d_args, sizeof(SapArgs) * sys.size()))
        return fail(lead, DDQCD_ERR_NOMEM, "no device memory for a launch plan (workspace plan region full)");
    plan->h_args.resize(sys.size());
    // group the systems by (domain shape, precision, product form)
    std::vector<std::array<int, 3>> gk;
    std::vector<std::vector<int>> members;
    for (size_t i = 0; i < sys.size(); i++) {
        const std::array<int, 3> k{sap_shape_id(sys[i].c->g.b), sys[i].c->sap_prec, sys[i].c->product};
        size_t gi = std::find(gk.begin(), gk.end(), k) - gk.begin();
        if (gi == gk.size()) {
            gk.push_back(k);
            members.emplace_back();
        }
        members[gi].push_back((int)i);
    }
    for (size_t gi = 0; gi < gk.size(); gi++) {
        plan->groups.emplace_back();
        Plan::Group &G = plan->groups.back();
        G.shape = gk[gi][0];
        G.prec = gk[gi][1];
        G.product = gk[gi][2];
        const int ndw = sap_domains_per_workgroup(G.shape, G.prec, G.product);
        const int rt = sap_rhs_per_workgroup(G.product);
        // tiles: up to rt systems of one context with consecutive system
        // numbers (one system each for the one-right-hand-side kernels)
        std::vector<std::pair<int, int>> tiles;   // (first system, count)
        for (int si : members[gi]) {
            if (!tiles.empty()) {
                auto &tl = tiles.back();
                const int last = tl.first + tl.second - 1;
                if (tl.second < rt && si == last + 1 && sys[si].c == sys[last].c) {
                    tl.second++;
                    continue;
                }
            }
            tiles.emplace_back(si, 1);
        }
        for (int col = 0; col < 3; col++) {
            // runs of ndw domains of one tile (one workgroup each), one list
            // of runs per XCD; the runs of one (context, domain run) share a list
            std::vector<std::vector<std::vector<int2>>> lane(N_XCD);
            std::map<std::pair<ddqcd_t, int>, int> key_lane;
            int next = 0;
            for (const auto &tl : tiles) {
                const int si = tl.first;
                const int x = rt > 1 ? si | (tl.second << 24) : si;
                std::vector<int> all_doms;
                if (col == 2) {
                    all_doms = sys[si].c->dom_host[0];
                    all_doms.insert(all_doms.end(), sys[si].c->dom_host[1].begin(), sys[si].c->dom_host[1].end());
                }
                const std::vector<int> &doms = col == 2 ? all_doms : sys[si].c->dom_host[col];
                if (doms.size() % ndw)
                    return fail(lead, DDQCD_ERR_GEOMETRY, "domain count per colour not a multiple of the workgroup's");
                for (size_t r = 0; r * ndw < doms.size(); r++) {
                    const auto kd = std::make_pair(sys[si].c, (int)r);
                    auto f = key_lane.find(kd);
                    const int ln = f == key_lane.end() ? (key_lane[kd] = next++ % N_XCD) : f->second;
                    std::vector<int2> run;
                    for (int q = 0; q < ndw; q++) run.push_back(make_int2(x, doms[r * ndw + q]));
                    lane[ln].push_back(run);
                }
            }
            size_t len = 0;
            for (auto &l : lane) len = std::max(len, l.size());
            std::vector<int2> items(len * N_XCD * ndw, make_int2(-1, -1));
            for (int ln = 0; ln < N_XCD; ln++)
                for (size_t j = 0; j < lane[ln].size(); j++)
                    for (int q = 0; q < ndw; q++) items[(j * N_XCD + ln) * ndw + q] = lane[ln][j][q];
            while (!items.empty() && items[items.size() - ndw].x < 0) items.resize(items.size() - ndw);
            G.nitems[col] = (int)items.size();
            if (!plan_alloc(lead, (void **)&G.items[col], sizeof(int2) * std::max<size_t>(1, items.size())))
                return fail(lead, DDQCD_ERR_NOMEM, "no device memory for a launch plan (workspace plan region full)");
            HIPCHK(lead, hipMemcpy(G.items[col], items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
        }
    }
    plan->additive = lead->schwarz == DDQCD_SCHWARZ_ADDITIVE;
    out = plan.get();
    lead->plans[key] = std::move(plan);
    return DDQCD_OK;
}

// the launches of one preconditioner call: black domains first (colour 0),
// then white, n_cycles times, one launch per (shape, precision) group
hipError_t enqueue_sweeps(const Plan &plan, int n_cycles, hipStream_t s)
{
    if (plan.additive) {
        // one launch per cycle over all domains; the boundary buffers alternate
        for (int cyc = 0; cyc < n_cycles; cyc++) {
            Visit v;
            v.first = cyc == 0;
            v.faces_in = cyc > 0;
            v.last = cyc == n_cycles - 1;
            v.faces_out = !v.last;
            v.res_out = !v.last;
            v.flip = cyc & 1;
            for (const Plan::Group &G : plan.groups) {
                hipError_t e =
                    sap_sweep_batch(plan.d_args, G.items[2], G.nitems[2], G.shape, G.prec, G.product, v, s);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    }
    for (int cyc = 0; cyc < n_cycles; cyc++)
        for (int col = 0; col < 2; col++) {
            Visit v;
            v.first = cyc == 0;
            v.faces_in = !(cyc == 0 && col == 0);
            v.last = cyc == n_cycles - 1;
            v.faces_out = !(v.last && col == 1);
            v.res_out = !v.last;
            v.flip = 0;
            for (const Plan::Group &G : plan.groups) {
                hipError_t e =
                    sap_sweep_batch(plan.d_args, G.items[col], G.nitems[col], G.shape, G.prec, G.product, v, s);
                if (e != hipSuccess) return e;
            }
        }
    return hipSuccess;
}

int capture_graph(ddqcd_t lead, Plan &plan, int n_cycles)
{
    if (plan.graph) {
        (void)hipGraphExecDestroy(plan.graph);
        plan.graph = nullptr;
    }
    if (!lead->capture) HIPCHK(lead, hipStreamCreateWithFlags(&lead->capture, hipStreamNonBlocking));
    HIPCHK(lead, hipStreamBeginCapture(lead->capture, hipStreamCaptureModeThreadLocal));
    const hipError_t e = enqueue_sweeps(plan, n_cycles, lead->capture);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(lead->capture, &g);   // always ends the capture
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        HIPCHK(lead, e);
        HIPCHK(lead, e2);
    }
    const hipError_t e3 = hipGraphInstantiate(&plan.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(lead, e3);
    plan.graph_cycles = n_cycles;
    return DDQCD_OK;
}

// out_i = M eta_i for the listed systems (internal FP64 vectors); systems with
// on[i] == 0 are left out (their out_i is not written).  All systems share the
// SAP cycle count.
int run_sap(const std::vector<Sys> &all, const std::vector<const double2 *> &eta_all,
            const std::vector<double2 *> &out_all, const std::vector<int> &on, hipStream_t s, bool io32 = false)
{
    std::vector<Sys> sys;
    std::vector<const double2 *> eta;
    std::vector<double2 *> out;
    for (size_t i = 0; i < all.size(); i++)
        if (on[i]) {
            sys.push_back(all[i]);
            eta.push_back(eta_all[i]);
            out.push_back(out_all[i]);
        }
    if (sys.empty()) return DDQCD_OK;
    ddqcd_t lead = all[0].c;
    const int n_cycles = lead->n_cycles;
    Plan *plan;
    int e = build_plan(sys, plan);
    if (e) return e;
    for (size_t i = 0; i < sys.size(); i++) {
        ddqcd_t c = sys[i].c;
        Slot *sl = sys[i].sl;
        SapArgs &a = plan->h_args[i];
        a = SapArgs{};
        a.g = c->g;
        a.n_mr = c->n_mr;
        a.eta = eta[i];
        a.out = out[i];
        a.psi = sl->psi;
        a.res = sl->res;
        a.res_scale = sl->res_scale;
        a.face = sl->face;
        a.face_scale = sl->face_scale;
        if (plan->additive) {
            if (!sl->face_alt) {
                const Geo &g = c->g;
                if ((e = dev_alloc(c, &sl->face_alt, (size_t)g.nd * sap_face_sites(g.b) * 6 * 16))) return e;
                if ((e = alloc(c, &sl->face_scale_alt, (size_t)g.nd * 4))) return e;
            }
            a.face_alt = sl->face_alt;
            a.face_scale_alt = sl->face_scale_alt;
        }
        a.rho_tmp = sl->rho_tmp;
        a.links = links_for(c, c->sap_prec);
        a.cs = schur_for(c, c->sap_prec);
        a.active = 1;
        a.io32 = io32;
    }
    HIPCHK(lead, hipMemcpyAsync(plan->d_args, plan->h_args.data(), sizeof(SapArgs) * sys.size(),
                                hipMemcpyHostToDevice, s));
    if (lead->schedule == DDQCD_SCHED_GRAPH) {
        if (!plan->graph || plan->graph_cycles != n_cycles)
            if ((e = capture_graph(lead, *plan, n_cycles))) return e;
        HIPCHK(lead, hipGraphLaunch(plan->graph, s));
        return DDQCD_OK;
    }
    HIPCHK(lead, enqueue_sweeps(*plan, n_cycles, s));
    return DDQCD_OK;
}

int apply_A64(ddqcd_t c, const double2 *in, double2 *out, hipStream_t s)
{
    HIPCHK(c, apply_A(c->g, in, out, c->U64, c->C64, P64, s));
    return DDQCD_OK;
}

// out_i = A in_i (FP64) for the listed systems; two consecutive systems of one
// context share a launch where the kernel allows it (each link and clover
// load then serves both), with the bits of two single calls
template <typename In, typename Out>
int apply_A64_list(const std::vector<Sys> &sys, const std::vector<int> &list, In in_of, Out out_of, hipStream_t s)
{
    for (size_t q = 0; q < list.size();) {
        const int i = list[q];
        ddqcd_t c = sys[i].c;
        if (q + 1 < list.size() && sys[list[q + 1]].c == c && apply_A_pairs(c->g, P64)) {
            const int j = list[q + 1];
            HIPCHK(c, apply_A_pair(c->g, in_of(i), out_of(i), in_of(j), out_of(j), c->U64, c->C64, P64, s));
            q += 2;
        } else {
            const int e = apply_A64(c, in_of(i), out_of(i), s);
            if (e) return e;
            q += 1;
        }
    }
    return DDQCD_OK;
}

// Phase timings of a solve: each phase is bracketed by two events on the
// launch stream; the elapsed times are read once at the end (no extra
// synchronisation between phases).
struct Clock {
    struct Span {
        hipEvent_t a, b;
        double *acc;
    };
    std::vector<Span> spans;
    hipStream_t s;
    explicit Clock(hipStream_t s_) : s(s_) {}
    void collect()
    {
        if (spans.empty()) return;
        (void)hipEventSynchronize(spans.back().b);
        for (Span &p : spans) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) *p.acc += ms;
        }
        release();
    }
    void release()
    {
        for (Span &p : spans) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        spans.clear();
    }
    ~Clock() { release(); }
};

struct Timer {
    Clock &clk;
    Clock::Span sp{nullptr, nullptr, nullptr};
    Timer(Clock &c, double *acc) : clk(c)
    {
        if (hipEventCreate(&sp.a) != hipSuccess) return;
        if (hipEventCreate(&sp.b) != hipSuccess) {
            (void)hipEventDestroy(sp.a);
            sp.a = nullptr;
            return;
        }
        sp.acc = acc;
        (void)hipEventRecord(sp.a, clk.s);
    }
    ~Timer()
    {
        if (!sp.acc) return;
        (void)hipEventRecord(sp.b, clk.s);
        clk.spans.push_back(sp);
    }
};

using C = std::complex<double>;

// ---- flexible GCR over many systems in lockstep ------------------------------

struct FgcrState {
    double bn = 0, rel = 0;
    int steps = 0, cycles = 0, kend = 0;
    bool done = false;      // converged, or a zero source
    bool in_cycle = false;  // still taking steps in the current cycle
    int status = DDQCD_ERR_NOT_CONVERGED;
    std::vector<C> a, cc, alpha;
    std::vector<double> bb;
    double2 h[32];          // results of the last reduction
};

// During a solve every system's reduction results live side by side in the
// lead context's result area (system i at pairs [32 i, 32 i + 32)), so one
// copy into pinned memory and one wait read all of them back.
struct ResultArea {
    const std::vector<Sys> &sys;
    std::vector<double2 *> saved;
    ddqcd_t lead;
    explicit ResultArea(const std::vector<Sys> &s) : sys(s), lead(s[0].c) {}
    int bind()
    {
        const int ns = (int)sys.size();
        if (lead->res_cap < ns && lead->ws)
            return fail(lead, DDQCD_ERR_NOMEM, "more systems than the workspace's reduction area holds (" +
                                                   std::to_string(lead->res_cap) + ")");
        if (!lead->res_host && lead->res_cap > 0)   // pinned host copy of a workspace's reduction area
            HIPCHK(lead, hipHostMalloc((void **)&lead->res_host, sizeof(double2) * 32 * lead->res_cap,
                                       hipHostMallocDefault));
        if (lead->res_cap < ns) {
            int e;
            if ((e = alloc(lead, &lead->res_dev, sizeof(double2) * 32 * ns))) return e;
            if (lead->res_host) (void)hipHostFree(lead->res_host);
            lead->res_host = nullptr;
            lead->res_cap = 0;
            HIPCHK(lead, hipHostMalloc((void **)&lead->res_host, sizeof(double2) * 32 * ns, hipHostMallocDefault));
            lead->res_cap = ns;
        }
        for (int i = 0; i < ns; i++) {
            saved.push_back(sys[i].sl->blas.result);
            sys[i].sl->blas.result = lead->res_dev + 32L * i;
        }
        return DDQCD_OK;
    }
    ~ResultArea()
    {
        for (size_t i = 0; i < saved.size(); i++) sys[i].sl->blas.result = saved[i];
    }
};

// read back result[0..m-1] of every listed system with one copy and one wait
int fetch_all(const std::vector<Sys> &sys, std::vector<FgcrState> &st, const std::vector<int> &which, int m,
              hipStream_t s)
{
    if (which.empty()) return DDQCD_OK;
    ddqcd_t lead = sys[0].c;
    const int lo = *std::min_element(which.begin(), which.end());
    const int hi = *std::max_element(which.begin(), which.end());
    const size_t off = 32L * lo, len = 32L * (hi - lo) + m;
    HIPCHK(lead, hipMemcpyAsync(lead->res_host + off, lead->res_dev + off, sizeof(double2) * len,
                                hipMemcpyDeviceToHost, s));
    HIPCHK(lead, hipStreamSynchronize(s));
    for (int i : which) std::copy(lead->res_host + 32L * i, lead->res_host + 32L * i + m, st[i].h);
    return DDQCD_OK;
}

int put_coef(const Sys &y, const std::vector<C> &v, hipStream_t s)
{
    static_assert(sizeof(C) == sizeof(double2), "layout");
    if (v.empty()) return DDQCD_OK;
    HIPCHK(y.c, hipMemcpyAsync(y.sl->blas.coef, v.data(), sizeof(double2) * v.size(), hipMemcpyHostToDevice, s));
    return DDQCD_OK;
}

// Solves A x = b for every system (x, b: the slot's internal FP64 vectors; x
// holds a guess where guess[i]).  The timings are those of the whole batch.
int fgcr(const std::vector<Sys> &sys, const std::vector<int> &guess, std::vector<ddqcd_info> &info, hipStream_t s)
{
    const int ns = (int)sys.size();
    ddqcd_t lead = sys[0].c;
    const int m = lead->restart;
    const int max_cycles = lead->max_cycles;
    const double tol = lead->tol;
    double tsap = 0, tA = 0, tgs = 0, tother = 0;
    Clock clk(s);
    std::vector<FgcrState> st(ns);
    int e;
    ResultArea area(sys);
    if ((e = area.bind())) return e;
    for (int i = 0; i < ns; i++) {
        st[i].a.assign((size_t)m * m, 0);
        st[i].cc.assign(m, 0);
        st[i].alpha.assign(m, 0);
        st[i].bb.assign(m, 0);
        if ((e = ensure_basis(sys[i].c, *sys[i].sl))) return e;
    }
    auto nc = [&](int i) { return ncomplex(sys[i].c->g); };
    auto Zk = [&](int i, int k) { return sys[i].sl->Z + (long)k * nc(i); };
    auto Wk = [&](int i, int k) { return sys[i].sl->W + (long)k * nc(i); };

    // |b| and the initial residual
    std::vector<int> all(ns), live;
    for (int i = 0; i < ns; i++) {
        all[i] = i;
        if (!guess[i]) HIPCHK(sys[i].c, zero(sys[i].sl->x, nc(i), s));
        HIPCHK(sys[i].c, norm2(sys[i].sl->blas, sys[i].sl->b, nc(i), s));
    }
    if ((e = fetch_all(sys, st, all, 1, s))) return e;
    for (int i = 0; i < ns; i++) {
        st[i].bn = std::sqrt(st[i].h[0].x);
        if (!std::isfinite(st[i].bn)) return fail(sys[i].c, DDQCD_ERR_NONFINITE, "non-finite right-hand side");
        if (st[i].bn == 0) {
            HIPCHK(sys[i].c, zero(sys[i].sl->x, nc(i), s));
            st[i].done = true;
            st[i].status = DDQCD_OK;
        } else live.push_back(i);
    }
    // r = b - A x; from x = 0 that is b itself (A 0 = 0 exactly), a copy
    std::vector<int> guessed;
    {
        Timer t(clk, &tother);
        for (int i : live) {
            if (guess[i]) guessed.push_back(i);
            else HIPCHK(sys[i].c, hipMemcpyAsync(sys[i].sl->r, sys[i].sl->b, sizeof(double2) * nc(i),
                                                 hipMemcpyDeviceToDevice, s));
        }
    }
    {
        Timer t(clk, &tA);
        if ((e = apply_A64_list(
                 sys, guessed, [&](int i) { return (const double2 *)sys[i].sl->x; },
                 [&](int i) { return sys[i].sl->r; }, s)))
            return e;
    }
    {
        Timer t(clk, &tother);
        for (int i : guessed) HIPCHK(sys[i].c, residual(sys[i].sl->blas, sys[i].sl->b, sys[i].sl->r, nc(i), s));
        if (!guessed.empty() && (e = fetch_all(sys, st, guessed, 1, s))) return e;
    }
    for (int i : live) {
        st[i].rel = guess[i] ? std::sqrt(st[i].h[0].x) / st[i].bn : 1.0;
        if (!std::isfinite(st[i].rel)) return fail(sys[i].c, DDQCD_ERR_NONFINITE, "non-finite residual");
        if (st[i].rel <= tol) {
            st[i].done = true;
            st[i].status = DDQCD_OK;
        }
    }

    for (int cyc = 0; cyc < max_cycles; cyc++) {
        std::vector<int> cur;
        for (int i = 0; i < ns; i++) {
            st[i].in_cycle = !st[i].done;
            st[i].kend = 0;
            if (!st[i].done) cur.push_back(i);
        }
        if (cur.empty()) break;
        for (int k = 0; k < m; k++) {
            std::vector<int> act;
            for (int i : cur)
                if (st[i].in_cycle) act.push_back(i);
            if (act.empty()) break;
            // z_k = M r
            {
                Timer t(clk, &tsap);
                std::vector<const double2 *> eta(ns);
                std::vector<double2 *> out(ns);
                std::vector<int> on(ns, 0);
                for (int i = 0; i < ns; i++) {
                    eta[i] = sys[i].sl->r;
                    out[i] = Zk(i, k);
                }
                for (int i : act) on[i] = 1;
                if ((e = run_sap(sys, eta, out, on, s))) return e;
            }
            // w_k = A z_k
            {
                Timer t(clk, &tA);
                if ((e = apply_A64_list(
                         sys, act, [&](int i) { return (const double2 *)Zk(i, k); }, [&](int i) { return Wk(i, k); },
                         s)))
                    return e;
            }
            {
                Timer t(clk, &tgs);
                // classical Gram-Schmidt against the earlier w-hat, repeated
                // once for a system whose new vector lost more than half its norm
                std::vector<double> before(ns, 0), wn2(ns, 0);
                std::vector<C> wr(ns);
                std::vector<int> todo = act;
                for (int pass = 0; pass < 2 && !todo.empty(); pass++) {
                    // the first pass also takes <w, w> (column k of W is w itself),
                    // which only the repeat test reads: not for the first vector
                    const int nd = pass == 0 && k > 0 ? k + 1 : k;
                    if (nd > 0) {
                        for (int i : todo)
                            HIPCHK(sys[i].c, multidot(sys[i].sl->blas, sys[i].sl->W, nc(i), nd, Wk(i, k), nc(i), s));
                        if ((e = fetch_all(sys, st, todo, nd, s))) return e;
                        for (int i : todo) {
                            if (pass == 0) before[i] = st[i].h[k].x;
                            if (k == 0) continue;
                            // the columns of W are kept unnormalised, W_j = b_j w-hat_j:
                            // <w-hat_j, w> = <W_j, w> / b_j, and w -= sum <w-hat_j, w> w-hat_j
                            // takes the coefficients <W_j, w> / b_j^2 on the columns
                            std::vector<C> coef(k);
                            for (int j = 0; j < k; j++) {
                                const C cj = C(st[i].h[j].x, st[i].h[j].y) / st[i].bb[j];
                                st[i].a[(size_t)j * m + k] += cj;
                                coef[j] = cj / st[i].bb[j];
                            }
                            if ((e = put_coef(sys[i], coef, s))) return e;
                        }
                    }
                    for (int i : todo)
                        HIPCHK(sys[i].c, cgs_update(sys[i].sl->blas, Wk(i, k), sys[i].sl->W, nc(i), k, sys[i].sl->r,
                                                    nc(i), s));
                    if ((e = fetch_all(sys, st, todo, 2, s))) return e;
                    std::vector<int> again;
                    for (int i : todo) {
                        wn2[i] = st[i].h[0].x;
                        wr[i] = C(st[i].h[1].x, st[i].h[1].y);
                        if (k > 0 && !(wn2[i] > 0.25 * before[i])) {
                            before[i] = wn2[i];
                            again.push_back(i);
                        }
                    }
                    todo = again;
                }
                for (int i : act) {
                    FgcrState &f = st[i];
                    f.bb[k] = std::sqrt(wn2[i]);
                    if (!(f.bb[k] > 0) || !std::isfinite(f.bb[k]))
                        return fail(sys[i].c, DDQCD_ERR_NONFINITE, "breakdown: A M r vanished or is non-finite");
                    f.cc[k] = wr[i] / f.bb[k];
                    // r -= <w-hat, r> w-hat = (<w, r> / b^2) w; w stays unnormalised
                    const C al = f.cc[k] / f.bb[k];
                    HIPCHK(sys[i].c, residual_update(sys[i].sl->blas, Wk(i, k), sys[i].sl->r,
                                                     make_double2(al.real(), al.imag()), nc(i), s));
                }
                if ((e = fetch_all(sys, st, act, 1, s))) return e;
            }
            for (int i : act) {
                FgcrState &f = st[i];
                f.steps++;
                f.kend = k + 1;
                f.rel = std::sqrt(f.h[0].x) / f.bn;
                if (!std::isfinite(f.rel)) return fail(sys[i].c, DDQCD_ERR_NONFINITE, "non-finite residual");
                if (f.rel <= tol) f.in_cycle = false;
            }
        }
        // x += sum_k alpha_k z_k, then the true residual r = b - A x
        {
            Timer t(clk, &tother);
            for (int i : cur) {
                FgcrState &f = st[i];
                for (int k = f.kend - 1; k >= 0; k--) {
                    C sum = f.cc[k];
                    for (int j = k + 1; j < f.kend; j++) sum -= f.a[(size_t)k * m + j] * f.alpha[j];
                    f.alpha[k] = sum / f.bb[k];
                }
                std::vector<C> al(f.alpha.begin(), f.alpha.begin() + f.kend);
                if ((e = put_coef(sys[i], al, s))) return e;
                HIPCHK(sys[i].c, axpy_multi(sys[i].sl->blas, sys[i].sl->x, sys[i].sl->Z, nc(i), f.kend, nc(i), s));
                std::fill(f.a.begin(), f.a.end(), C(0));
            }
        }
        {
            Timer t(clk, &tA);
            if ((e = apply_A64_list(
                     sys, cur, [&](int i) { return (const double2 *)sys[i].sl->x; },
                     [&](int i) { return sys[i].sl->r; }, s)))
                return e;
        }
        {
            Timer t(clk, &tother);
            for (int i : cur) HIPCHK(sys[i].c, residual(sys[i].sl->blas, sys[i].sl->b, sys[i].sl->r, nc(i), s));
            if ((e = fetch_all(sys, st, cur, 1, s))) return e;
        }
        for (int i : cur) {
            FgcrState &f = st[i];
            f.cycles++;
            f.rel = std::sqrt(f.h[0].x) / f.bn;
            if (!std::isfinite(f.rel)) return fail(sys[i].c, DDQCD_ERR_NONFINITE, "non-finite residual");
            if (f.rel <= tol) {
                f.done = true;
                f.status = DDQCD_OK;
            }
        }
    }
    clk.collect();
    int status = DDQCD_OK;
    for (int i = 0; i < ns; i++) {
        ddqcd_info &inf = info[i];
        inf.converged = st[i].status == DDQCD_OK;
        inf.iters = st[i].steps;
        inf.restarts = st[i].cycles;
        inf.rel_residual = st[i].rel;
        inf.t_sap_ms = tsap;
        inf.t_A_ms = tA;
        inf.t_gs_ms = tgs;
        inf.t_other_ms = tother;
        if (st[i].status != DDQCD_OK) {
            status = DDQCD_ERR_NOT_CONVERGED;
            sys[i].c->err = "not converged: relative residual " + std::to_string(st[i].rel);
        }
    }
    return status;
}

// ---- flexible GMRES with deflated restarts ------------------------------------
//
// Small dense complex matrices on the host are row-major vectors.

// min |c - H y| (H rows x cols, row stride ld, full column rank): QR of H by
// modified Gram-Schmidt with a second orthogonalisation pass, R y = Q^H c;
// returns |c - H y|, evaluated directly.
double lsq_mgs(int rows, int cols, const C *H, int ld, const C *c, C *y)
{
    std::vector<C> Q((size_t)rows * cols), Rm((size_t)cols * cols, 0.0);
    for (int j = 0; j < cols; j++) {
        for (int i = 0; i < rows; i++) Q[(size_t)i * cols + j] = H[(size_t)i * ld + j];
        for (int pass = 0; pass < 2; pass++)
            for (int p = 0; p < j; p++) {
                C d = 0;
                for (int i = 0; i < rows; i++) d += std::conj(Q[(size_t)i * cols + p]) * Q[(size_t)i * cols + j];
                Rm[(size_t)p * cols + j] += d;
                for (int i = 0; i < rows; i++) Q[(size_t)i * cols + j] -= d * Q[(size_t)i * cols + p];
            }
        double nq = 0;
        for (int i = 0; i < rows; i++) nq += std::norm(Q[(size_t)i * cols + j]);
        nq = std::sqrt(nq);
        Rm[(size_t)j * cols + j] = nq;
        for (int i = 0; i < rows; i++) Q[(size_t)i * cols + j] /= nq;
    }
    for (int j = cols - 1; j >= 0; j--) {
        C t = 0;
        for (int i = 0; i < rows; i++) t += std::conj(Q[(size_t)i * cols + j]) * c[i];
        for (int p = j + 1; p < cols; p++) t -= Rm[(size_t)j * cols + p] * y[p];
        y[j] = t / Rm[(size_t)j * cols + j];
    }
    double res = 0;
    for (int i = 0; i < rows; i++) {
        C t = c[i];
        for (int j = 0; j < cols; j++) t -= H[(size_t)i * ld + j] * y[j];
        res += std::norm(t);
    }
    return std::sqrt(res);
}

// x = M^-1 b for a small n x n matrix (Gaussian elimination, partial pivoting);
// false if singular
bool small_solve(int n, std::vector<C> M, std::vector<C> &x)
{
    for (int col = 0; col < n; col++) {
        int p = col;
        for (int r = col + 1; r < n; r++)
            if (std::abs(M[(size_t)r * n + col]) > std::abs(M[(size_t)p * n + col])) p = r;
        if (!(std::abs(M[(size_t)p * n + col]) > 0)) return false;
        if (p != col) {
            for (int q = 0; q < n; q++) std::swap(M[(size_t)p * n + q], M[(size_t)col * n + q]);
            std::swap(x[p], x[col]);
        }
        for (int r = col + 1; r < n; r++) {
            const C f = M[(size_t)r * n + col] / M[(size_t)col * n + col];
            for (int q = col; q < n; q++) M[(size_t)r * n + q] -= f * M[(size_t)col * n + q];
            x[r] -= f * x[col];
        }
    }
    for (int r = n - 1; r >= 0; r--) {
        C t = x[r];
        for (int q = r + 1; q < n; q++) t -= M[(size_t)r * n + q] * x[q];
        x[r] = t / M[(size_t)r * n + r];
    }
    return true;
}

// Eigenvalues of a small general complex matrix: QR iterations on the full
// matrix (Wilkinson shift from the trailing 2x2 block, the QR factor by
// modified Gram-Schmidt), deflating the last row of the active block when
// its off-diagonal part is negligible.
std::vector<C> small_eigenvalues(int n, std::vector<C> A)
{
    std::vector<C> lam;
    double an = 0;
    for (const C &v : A) an += std::norm(v);
    an = std::sqrt(an);
    int act = n, iters = 0;
    while (act > 0) {
        const int a = act - 1;
        double off = 0;
        for (int j = 0; j < a; j++) off += std::norm(A[(size_t)a * n + j]);
        if (act == 1 || std::sqrt(off) <= 1e-15 * an || iters > 200) {
            lam.push_back(A[(size_t)a * n + a]);
            act--;
            iters = 0;
            continue;
        }
        iters++;
        const C p = A[(size_t)(a - 1) * n + a - 1], q = A[(size_t)(a - 1) * n + a], r = A[(size_t)a * n + a - 1],
                d = A[(size_t)a * n + a];
        const C half = 0.5 * (p + d), disc = std::sqrt(0.25 * (p - d) * (p - d) + q * r);
        C mu = std::abs(half + disc - d) < std::abs(half - disc - d) ? half + disc : half - disc;
        if (iters % 25 == 0) mu = d + std::sqrt(off);   // exceptional shift
        std::vector<C> Qm((size_t)act * act), Rm((size_t)act * act, 0.0);
        for (int j = 0; j < act; j++) {
            for (int i = 0; i < act; i++) Qm[(size_t)i * act + j] = A[(size_t)i * n + j] - (i == j ? mu : C(0));
            for (int pass = 0; pass < 2; pass++)
                for (int pp = 0; pp < j; pp++) {
                    C dd = 0;
                    for (int i = 0; i < act; i++) dd += std::conj(Qm[(size_t)i * act + pp]) * Qm[(size_t)i * act + j];
                    Rm[(size_t)pp * act + j] += dd;
                    for (int i = 0; i < act; i++) Qm[(size_t)i * act + j] -= dd * Qm[(size_t)i * act + pp];
                }
            double nq = 0;
            for (int i = 0; i < act; i++) nq += std::norm(Qm[(size_t)i * act + j]);
            nq = std::sqrt(nq);
            Rm[(size_t)j * act + j] = nq;
            for (int i = 0; i < act; i++) Qm[(size_t)i * act + j] = nq > 0 ? Qm[(size_t)i * act + j] / nq : C(0);
        }
        for (int i = 0; i < act; i++)   // A_act = R Q + mu
            for (int j = 0; j < act; j++) {
                C t = i == j ? mu : C(0);
                for (int l = i; l < act; l++) t += Rm[(size_t)i * act + l] * Qm[(size_t)l * act + j];
                A[(size_t)i * n + j] = t;
            }
    }
    return lam;
}

// Orthonormal basis (m x k, row-major) of the span of the k harmonic Ritz
// vectors of smallest |theta| of the relation A Z = V Hbar (Hbar (m+1) x m,
// last row h e_m^T): the eigenvectors of H_m + |h|^2 H_m^-H e_m e_m^H, found by
// inverse iteration at each selected eigenvalue, each start vector and
// iterate orthogonalised against the vectors already taken (so a cluster of
// close eigenvalues yields its invariant subspace).
bool harmonic_ritz_basis(int m, int k, const std::vector<C> &H, std::vector<C> &P)
{
    std::vector<C> Hm((size_t)m * m), HmH((size_t)m * m);
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++) {
            Hm[(size_t)i * m + j] = H[(size_t)i * m + j];
            HmH[(size_t)i * m + j] = std::conj(H[(size_t)j * m + i]);
        }
    std::vector<C> f(m, 0.0);
    f[m - 1] = 1.0;
    if (!small_solve(m, HmH, f)) return false;
    const double h2 = std::norm(H[(size_t)m * m + m - 1]);
    std::vector<C> B = Hm;
    for (int i = 0; i < m; i++) B[(size_t)i * m + m - 1] += h2 * f[i];
    std::vector<C> lam = small_eigenvalues(m, B);
    std::sort(lam.begin(), lam.end(), [](const C &a, const C &b) { return std::abs(a) < std::abs(b); });
    double bn = 0;
    for (const C &v : B) bn += std::norm(v);
    bn = std::sqrt(bn);
    P.assign((size_t)m * k, 0.0);
    for (int q = 0; q < k; q++) {
        const C shift = lam[q] + C(1e-13 * bn, 1e-13 * bn);
        std::vector<C> Ms = B;
        for (int i = 0; i < m; i++) Ms[(size_t)i * m + i] -= shift;
        std::vector<C> v(m);
        for (int i = 0; i < m; i++) v[i] = C(1.0 + 0.1 * i, 0.3 * (i % 3));
        for (int it = 0; it < 4; it++) {
            for (int pass = 0; pass < 2; pass++)
                for (int p = 0; p < q; p++) {
                    C d = 0;
                    for (int i = 0; i < m; i++) d += std::conj(P[(size_t)i * k + p]) * v[i];
                    for (int i = 0; i < m; i++) v[i] -= d * P[(size_t)i * k + p];
                }
            double nv = 0;
            for (const C &t : v) nv += std::norm(t);
            nv = std::sqrt(nv);
            for (C &t : v) t /= nv;
            if (it < 3 && !small_solve(m, Ms, v)) return false;
        }
        for (int i = 0; i < m; i++) P[(size_t)i * k + q] = v[i];
    }
    return true;
}

// Solves A x = b for one system (x, b: the slot's FP64 vectors; x holds a
// guess if guess) by FGMRES-DR(m = restart, k = deflate), right-preconditioned
// by the context's SAP: the same algorithm as the oracle's (flexible Arnoldi,
// least squares residual estimate after each step, x += Z y and the true FP64
// residual at each cycle's end, deflated restart from the harmonic Ritz
// vectors and the least squares residual), with classical Gram-Schmidt
// repeated once when the new vector loses more than half its norm.
int fgmres_dr(const Sys &y, bool guess, ddqcd_info &info, hipStream_t s)
{
    ddqcd_t c = y.c;
    Slot &sl = *y.sl;
    const int m = c->restart, k = c->deflate;
    const long n = ncomplex(c->g);
    int e;
    if ((e = ensure_basis(c, sl))) return e;
    double2 *Vb = sl.W, *Zb = sl.Z;
    auto Vc = [&](int j) { return Vb + (long)j * n; };
    auto Zc = [&](int j) { return Zb + (long)j * n; };
    double tsap = 0, tA = 0, tgs = 0, tother = 0;
    Clock clk(s);
    double2 h[32];
    auto fetch = [&](int cnt) -> int {
        HIPCHK(c, hipMemcpyAsync(h, sl.blas.result, sizeof(double2) * cnt, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return DDQCD_OK;
    };
    auto put = [&](const std::vector<C> &v, double2 *dst) -> int {
        HIPCHK(c, hipMemcpyAsync(dst, v.data(), sizeof(double2) * v.size(), hipMemcpyHostToDevice, s));
        return DDQCD_OK;
    };
    info = ddqcd_info{};
    if (!guess) HIPCHK(c, zero(sl.x, n, s));
    HIPCHK(c, norm2(sl.blas, sl.b, n, s));
    if ((e = fetch(1))) return e;
    const double bn = std::sqrt(h[0].x);
    if (!std::isfinite(bn)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite right-hand side");
    if (bn == 0) {
        HIPCHK(c, zero(sl.x, n, s));
        info.converged = 1;
        return DDQCD_OK;
    }
    double rn;
    {
        Timer t(clk, &tA);
        if ((e = apply_A64(c, sl.x, sl.r, s))) return e;
    }
    HIPCHK(c, residual(sl.blas, sl.b, sl.r, n, s));
    if ((e = fetch(1))) return e;
    rn = std::sqrt(h[0].x);
    double rel = rn / bn;
    if (!std::isfinite(rel)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite residual");
    std::vector<C> H((size_t)(m + 1) * m, 0.0), cv(m + 1, 0.0), yv(m, 0.0);
    int steps = 0, cycles = 0, j0 = 0, status = rel <= c->tol ? DDQCD_OK : DDQCD_ERR_NOT_CONVERGED;
    for (int cyc = 0; cyc < c->max_cycles && status != DDQCD_OK; cyc++) {
        if (j0 == 0) {   // (re)start from the true residual
            const double2 one = make_double2(1.0 / rn, 0), z0 = make_double2(0, 0);
            HIPCHK(c, lincomb(Vc(0), sl.r, one, sl.r, z0, nullptr, z0, n, s));
            std::fill(H.begin(), H.end(), C(0));
            std::fill(cv.begin(), cv.end(), C(0));
            cv[0] = rn;
        }
        int jend = m;
        for (int j = j0; j < m; j++) {
            {
                Timer t(clk, &tsap);
                if ((e = run_sap({y}, {Vc(j)}, {Zc(j)}, {1}, s))) return e;
            }
            {
                Timer t(clk, &tA);
                if ((e = apply_A64(c, Zc(j), Vc(j + 1), s))) return e;
            }
            double wn2;
            {
                Timer t(clk, &tgs);
                double2 *w = Vc(j + 1);
                double before;
                std::vector<C> hsum(j + 1, 0.0);
                // first pass; <w, w> in the same multi-dot where the column fits
                const bool joint = j + 2 <= BLAS_MAXK;
                HIPCHK(c, multidot(sl.blas, Vb, n, joint ? j + 2 : j + 1, w, n, s));
                if ((e = fetch(joint ? j + 2 : j + 1))) return e;
                std::vector<C> coef(j + 1);
                for (int i = 0; i <= j; i++) coef[i] = C(h[i].x, h[i].y);
                if (joint) before = h[j + 1].x;
                else {
                    HIPCHK(c, norm2(sl.blas, w, n, s));
                    if ((e = fetch(1))) return e;
                    before = h[0].x;
                }
                for (int pass = 0; pass < 2; pass++) {
                    for (int i = 0; i <= j; i++) hsum[i] += coef[i];
                    if ((e = put(coef, sl.blas.coef))) return e;
                    HIPCHK(c, cgs_update(sl.blas, w, Vb, n, j + 1, w, n, s));
                    if ((e = fetch(1))) return e;
                    wn2 = h[0].x;
                    if (pass == 1 || wn2 > 0.25 * before) break;
                    before = wn2;
                    HIPCHK(c, multidot(sl.blas, Vb, n, j + 1, w, n, s));
                    if ((e = fetch(j + 1))) return e;
                    for (int i = 0; i <= j; i++) coef[i] = C(h[i].x, h[i].y);
                }
                const double hn = std::sqrt(wn2);
                if (!(hn > 0) || !std::isfinite(hn))
                    return fail(c, DDQCD_ERR_NONFINITE, "breakdown: A M v vanished or is non-finite");
                for (int i = 0; i <= j; i++) H[(size_t)i * m + j] = hsum[i];
                H[(size_t)(j + 1) * m + j] = hn;
                const double2 inv = make_double2(1.0 / hn, 0), z0 = make_double2(0, 0);
                HIPCHK(c, lincomb(w, w, inv, w, z0, nullptr, z0, n, s));
            }
            steps++;
            const double est = lsq_mgs(j + 2, j + 1, H.data(), m, cv.data(), yv.data()) / bn;
            if (!std::isfinite(est)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite residual estimate");
            if (est <= c->tol) {
                jend = j + 1;
                break;
            }
        }
        {
            Timer t(clk, &tother);
            if ((e = put(std::vector<C>(yv.begin(), yv.begin() + jend), sl.blas.coef))) return e;
            HIPCHK(c, axpy_multi(sl.blas, sl.x, Zb, n, jend, n, s));
        }
        {
            Timer t(clk, &tA);
            if ((e = apply_A64(c, sl.x, sl.r, s))) return e;
        }
        HIPCHK(c, residual(sl.blas, sl.b, sl.r, n, s));
        if ((e = fetch(1))) return e;
        rn = std::sqrt(h[0].x);
        rel = rn / bn;
        cycles++;
        if (!std::isfinite(rel)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite residual");
        if (rel <= c->tol) {
            status = DDQCD_OK;
            break;
        }
        if (k == 0 || jend < m) {
            j0 = 0;
            continue;
        }
        // deflated restart
        Timer t(clk, &tother);
        std::vector<C> sres(m + 1), Pk;
        for (int i = 0; i <= m; i++) {
            C tt = cv[i];
            for (int j = 0; j < m; j++) tt -= H[(size_t)i * m + j] * yv[j];
            sres[i] = tt;
        }
        if (!harmonic_ritz_basis(m, k, H, Pk)) {
            j0 = 0;
            continue;
        }
        const int k1 = k + 1;
        std::vector<C> P((size_t)(m + 1) * k1, 0.0), Pz((size_t)m * k);
        for (int i = 0; i < m; i++)
            for (int q = 0; q < k; q++) P[(size_t)i * k1 + q] = Pz[(size_t)i * k + q] = Pk[(size_t)i * k + q];
        for (int i = 0; i <= m; i++) P[(size_t)i * k1 + k] = sres[i];
        for (int pass = 0; pass < 2; pass++)
            for (int q = 0; q < k; q++) {
                C d = 0;
                for (int i = 0; i <= m; i++) d += std::conj(P[(size_t)i * k1 + q]) * P[(size_t)i * k1 + k];
                for (int i = 0; i <= m; i++) P[(size_t)i * k1 + k] -= d * P[(size_t)i * k1 + q];
            }
        double pn = 0;
        for (int i = 0; i <= m; i++) pn += std::norm(P[(size_t)i * k1 + k]);
        pn = std::sqrt(pn);
        for (int i = 0; i <= m; i++) P[(size_t)i * k1 + k] /= pn;
        // V_{k+1} = V P and Z_k = Z P_k, formed in the spare columns, then moved
        if ((e = put(P, sl.rcoef))) return e;
        HIPCHK(c, recombine(Vb, n, m + 1, sl.rcoef, k1, Vc(m + 1), n, n, s));
        HIPCHK(c, hipMemcpyAsync(Vc(0), Vc(m + 1), sizeof(double2) * n * k1, hipMemcpyDeviceToDevice, s));
        if ((e = put(Pz, sl.rcoef))) return e;
        HIPCHK(c, recombine(Zb, n, m, sl.rcoef, k, Zc(m), n, n, s));
        HIPCHK(c, hipMemcpyAsync(Zc(0), Zc(m), sizeof(double2) * n * k, hipMemcpyDeviceToDevice, s));
        // Hbar_k = P^H Hbar P_k, c = P^H s
        std::vector<C> Hn((size_t)(m + 1) * m, 0.0);
        for (int a = 0; a < k1; a++)
            for (int q = 0; q < k; q++) {
                C tt = 0;
                for (int i = 0; i <= m; i++) {
                    C hp = 0;
                    for (int j = 0; j < m; j++) hp += H[(size_t)i * m + j] * Pk[(size_t)j * k + q];
                    tt += std::conj(P[(size_t)i * k1 + a]) * hp;
                }
                Hn[(size_t)a * m + q] = tt;
            }
        H = Hn;
        std::fill(cv.begin(), cv.end(), C(0));
        for (int a = 0; a < k1; a++) {
            C tt = 0;
            for (int i = 0; i <= m; i++) tt += std::conj(P[(size_t)i * k1 + a]) * sres[i];
            cv[a] = tt;
        }
        j0 = k;
    }
    clk.collect();
    info.converged = status == DDQCD_OK;
    info.iters = steps;
    info.restarts = cycles;
    info.rel_residual = rel;
    info.t_sap_ms = tsap;
    info.t_A_ms = tA;
    info.t_gs_ms = tgs;
    info.t_other_ms = tother;
    if (status != DDQCD_OK) c->err = "not converged: relative residual " + std::to_string(rel);
    return status;
}

// ---- mixed-precision outer solver (iterative refinement) ------------------------
//
// Solves A x = b for one system by FP64 iterative refinement around an FP32
// flexible GCR: each outer step takes the true residual r = b - A x in FP64,
// solves A e = r / |r| by one FGCR cycle whose vectors, operator (two-row FP32
// links, FP32 clover) and Gram-Schmidt are FP32 (dot products accumulated in
// FP64), preconditioned by the context's SAP reading and writing FP32
// vectors, until its residual has fallen by MIXED_INNER_REDUCTION (or below
// what the outer tolerance needs), and adds |r| e to x in FP64.
constexpr double MIXED_INNER_REDUCTION = 1e-5;

int fgcr_mixed(const Sys &y, bool guess, ddqcd_info &info, hipStream_t s)
{
    ddqcd_t c = y.c;
    Slot &sl = *y.sl;
    const int m = c->restart;
    const long n = ncomplex(c->g);
    int e;
    if ((e = ensure_basis(c, sl))) return e;
    // FP32 work vectors in the FP64 basis arrays: Z32 (m columns) in Z, W32 (m)
    // and r32 in W (each FP64 column holds two FP32 ones)
    float2 *Z32 = (float2 *)sl.Z, *W32 = (float2 *)sl.W, *r32 = W32 + (long)m * n;
    double tsap = 0, tA = 0, tgs = 0, tother = 0;
    Clock clk(s);
    double2 h[32];
    auto fetch = [&](int cnt) -> int {
        HIPCHK(c, hipMemcpyAsync(h, sl.blas.result, sizeof(double2) * cnt, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return DDQCD_OK;
    };
    auto put = [&](const std::vector<C> &v) -> int {
        HIPCHK(c, hipMemcpyAsync(sl.blas.coef, v.data(), sizeof(double2) * v.size(), hipMemcpyHostToDevice, s));
        return DDQCD_OK;
    };
    info = ddqcd_info{};
    if (!guess) HIPCHK(c, zero(sl.x, n, s));
    HIPCHK(c, norm2(sl.blas, sl.b, n, s));
    if ((e = fetch(1))) return e;
    const double bn = std::sqrt(h[0].x);
    if (!std::isfinite(bn)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite right-hand side");
    if (bn == 0) {
        HIPCHK(c, zero(sl.x, n, s));
        info.converged = 1;
        return DDQCD_OK;
    }
    const void *U32 = links_for(c, DDQCD_FP32), *C32 = clover_for(c, DDQCD_FP32);
    std::vector<C> a((size_t)m * m), cc(m), alpha(m);
    std::vector<double> bb(m);
    int steps = 0, outer = 0, status = DDQCD_ERR_NOT_CONVERGED;
    double rel = 0;
    for (;;) {
        {
            Timer t(clk, &tA);
            if ((e = apply_A64(c, sl.x, sl.r, s))) return e;
        }
        HIPCHK(c, residual(sl.blas, sl.b, sl.r, n, s));
        if ((e = fetch(1))) return e;
        const double rn = std::sqrt(h[0].x);
        rel = rn / bn;
        if (!std::isfinite(rel)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite residual");
        if (rel <= c->tol) {
            status = DDQCD_OK;
            break;
        }
        if (outer >= c->max_cycles) break;
        outer++;
        HIPCHK(c, to_f32(sl.r, 1.0 / rn, r32, n, s));
        const double target = std::max(MIXED_INNER_REDUCTION, 0.5 * c->tol / rel);
        int kend = 0;
        std::fill(a.begin(), a.end(), C(0));
        for (int k = 0; k < m; k++) {
            float2 *zk = Z32 + (long)k * n, *wk = W32 + (long)k * n;
            {
                Timer t(clk, &tsap);
                if ((e = run_sap({y}, {(const double2 *)r32}, {(double2 *)zk}, {1}, s, true))) return e;
            }
            {
                Timer t(clk, &tA);
                HIPCHK(c, apply_A(c->g, zk, wk, U32, C32, P32, s));
            }
            Timer t(clk, &tgs);
            double before = 0, wn2 = 0;
            if (k > 0) {
                HIPCHK(c, multidot32(sl.blas, W32, n, k + 1, wk, n, s));   // column k is w itself
                if ((e = fetch(k + 1))) return e;
                before = h[k].x;
                for (int pass = 0; pass < 2; pass++) {
                    std::vector<C> coef(k);
                    for (int j = 0; j < k; j++) {
                        coef[j] = C(h[j].x, h[j].y);
                        a[(size_t)j * m + k] += coef[j];
                    }
                    if ((e = put(coef))) return e;
                    HIPCHK(c, cgs_update32(sl.blas, wk, W32, n, k, n, s));
                    if ((e = fetch(1))) return e;
                    wn2 = h[0].x;
                    if (pass == 1 || wn2 > 0.25 * before) break;
                    before = wn2;
                    HIPCHK(c, multidot32(sl.blas, W32, n, k, wk, n, s));
                    if ((e = fetch(k))) return e;
                }
            } else {
                HIPCHK(c, multidot32(sl.blas, wk, n, 1, wk, n, s));
                if ((e = fetch(1))) return e;
                wn2 = h[0].x;
            }
            bb[k] = std::sqrt(wn2);
            if (!(bb[k] > 0) || !std::isfinite(bb[k]))
                return fail(c, DDQCD_ERR_NONFINITE, "breakdown: A M r vanished or is non-finite");
            HIPCHK(c, scale_dot32(sl.blas, wk, 1.0 / bb[k], r32, n, s));
            if ((e = fetch(1))) return e;
            cc[k] = C(h[0].x, h[0].y);
            HIPCHK(c, axpy32(sl.blas, r32, make_double2(cc[k].real(), cc[k].imag()), wk, n, s));
            if ((e = fetch(1))) return e;
            steps++;
            kend = k + 1;
            if (std::sqrt(h[0].x) <= target) break;
        }
        {
            Timer t(clk, &tother);
            for (int k = kend - 1; k >= 0; k--) {
                C sum = cc[k];
                for (int j = k + 1; j < kend; j++) sum -= a[(size_t)k * m + j] * alpha[j];
                alpha[k] = sum / bb[k];
            }
            if ((e = put(std::vector<C>(alpha.begin(), alpha.begin() + kend)))) return e;
            HIPCHK(c, axpy_mixed(sl.blas, sl.x, Z32, n, kend, rn, n, s));
        }
    }
    clk.collect();
    info.converged = status == DDQCD_OK;
    info.iters = steps;
    info.restarts = outer;
    info.rel_residual = rel;
    info.t_sap_ms = tsap;
    info.t_A_ms = tA;
    info.t_gs_ms = tgs;
    info.t_other_ms = tother;
    if (status != DDQCD_OK) c->err = "not converged: relative residual " + std::to_string(rel);
    return status;
}

// shared body of ddqcd_solve and ddqcd_solve_batch
int solve_systems(const std::vector<Sys> &sys, double *const *x, const double *const *b, int x_is_guess,
                  ddqcd_info *info, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (size_t i = 0; i < sys.size(); i++) {
        const Geo &g = sys[i].c->g;
        HIPCHK(sys[i].c, import_spinor(g, b[i], sys[i].sl->b, P64, s));
        if (x_is_guess) HIPCHK(sys[i].c, import_spinor(g, x[i], sys[i].sl->x, P64, s));
    }
    std::vector<ddqcd_info> inf(sys.size());
    int st = DDQCD_OK;
    if (sys[0].c->outer != DDQCD_OUTER_FGCR) {
        // one system after the other
        for (size_t i = 0; i < sys.size(); i++) {
            const int si = sys[0].c->outer == DDQCD_OUTER_FGMRES_DR ? fgmres_dr(sys[i], x_is_guess != 0, inf[i], s)
                                                                     : fgcr_mixed(sys[i], x_is_guess != 0, inf[i], s);
            if (si != DDQCD_OK && si != DDQCD_ERR_NOT_CONVERGED) return si;
            if (si != DDQCD_OK) st = si;
        }
    } else {
        st = fgcr(sys, std::vector<int>(sys.size(), x_is_guess != 0), inf, s);
    }
    if (st != DDQCD_OK && st != DDQCD_ERR_NOT_CONVERGED) return st;
    for (size_t i = 0; i < sys.size(); i++) HIPCHK(sys[i].c, export_spinor(sys[i].c->g, sys[i].sl->x, P64, x[i], s));
    HIPCHK(sys[0].c, hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (size_t i = 0; i < sys.size(); i++) {
        inf[i].t_total_ms = ms;
        if (info) info[i] = inf[i];
    }
    return st;
}

// BiCGstab (van der Vorst 1992) on A in FP64, no preconditioner: the solver
// without domain decomposition that the paper compares against (Sec. IV-C).
// x and b are the slot's internal vectors; work vectors are basis columns.
int bicgstab(ddqcd_t c, Slot &sl, bool guess, int max_iter, ddqcd_info &info, hipStream_t s)
{
    const long n = ncomplex(c->g);
    int e;
    if ((e = ensure_basis(c, sl, 5))) return e;
    double2 *r0 = sl.Z, *p = sl.Z + n, *v = sl.Z + 2 * n, *sv = sl.Z + 3 * n, *t = sl.Z + 4 * n;
    double2 *x = sl.x, *r = sl.r, *b = sl.b;
    double2 h[2];
    auto fetch = [&](int m) -> int {
        HIPCHK(c, hipMemcpyAsync(h, sl.blas.result, sizeof(double2) * m, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return DDQCD_OK;
    };
    auto dot = [&](const double2 *a, const double2 *bb, C &out) -> int {   // <a, bb>
        HIPCHK(c, multidot(sl.blas, a, n, 1, bb, n, s));
        int e2 = fetch(1);
        out = C(h[0].x, h[0].y);
        return e2;
    };
    const double2 one = make_double2(1, 0), zero2 = make_double2(0, 0);
    auto cd = [](C z) { return make_double2(z.real(), z.imag()); };
    if (!guess) HIPCHK(c, zero(x, n, s));
    HIPCHK(c, norm2(sl.blas, b, n, s));
    if ((e = fetch(1))) return e;
    const double bn = std::sqrt(h[0].x);
    info = ddqcd_info{};
    if (!std::isfinite(bn)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite right-hand side");
    if (bn == 0) {
        HIPCHK(c, zero(x, n, s));
        info.converged = 1;
        return DDQCD_OK;
    }
    // r = b - A x, r0 = r, p = v = 0
    if ((e = apply_A64(c, x, r, s))) return e;
    HIPCHK(c, residual(sl.blas, b, r, n, s));
    if ((e = fetch(1))) return e;
    double rel = std::sqrt(h[0].x) / bn;
    HIPCHK(c, lincomb(r0, r, one, r, zero2, nullptr, zero2, n, s));
    HIPCHK(c, zero(p, n, s));
    HIPCHK(c, zero(v, n, s));
    C rho_old = 1, alpha = 1, omega = 1;
    int it = 0, restarts = 0, breakdowns = 0;
    // restart from the current x: r = b - A x (unless r already is), r0 = r,
    // p = v = 0
    auto restart = [&](bool have_r) -> int {
        int e2;
        if (!have_r) {
            if ((e2 = apply_A64(c, x, r, s))) return e2;
            HIPCHK(c, residual(sl.blas, b, r, n, s));
            if ((e2 = fetch(1))) return e2;
            rel = std::sqrt(h[0].x) / bn;
        }
        HIPCHK(c, lincomb(r0, r, one, r, zero2, nullptr, zero2, n, s));
        HIPCHK(c, zero(p, n, s));
        HIPCHK(c, zero(v, n, s));
        rho_old = alpha = omega = 1;
        restarts++;
        return DDQCD_OK;
    };
    while (rel > c->tol && it < max_iter) {
        C rho;
        if ((e = dot(r0, r, rho))) return e;
        if (std::abs(rho) == 0 || std::abs(omega) == 0) {
            // breakdown (rho or omega vanished): restart from the current
            // iterate with the true residual as the new shadow vector
            if (++breakdowns > 100) return fail(c, DDQCD_ERR_NONFINITE, "BiCGstab breakdown");
            if ((e = restart(false))) return e;
            continue;
        }
        const C beta = (rho / rho_old) * (alpha / omega);
        // p = r + beta (p - omega v)
        HIPCHK(c, lincomb(p, r, one, p, cd(beta), v, cd(-beta * omega), n, s));
        if ((e = apply_A64(c, p, v, s))) return e;
        C r0v;
        if ((e = dot(r0, v, r0v))) return e;
        alpha = rho / r0v;
        if (!std::isfinite(alpha.real()) || !std::isfinite(alpha.imag())) {
            // <r0, A p> vanished: restart before x takes the step
            if (++breakdowns > 100) return fail(c, DDQCD_ERR_NONFINITE, "BiCGstab breakdown");
            if ((e = restart(false))) return e;
            continue;
        }
        // s = r - alpha v, t = A s, omega = <t, s> / <t, t>
        HIPCHK(c, lincomb(sv, r, one, v, cd(-alpha), nullptr, zero2, n, s));
        if ((e = apply_A64(c, sv, t, s))) return e;
        HIPCHK(c, dot2(sl.blas, t, sv, n, s));
        if ((e = fetch(2))) return e;
        omega = h[1].x > 0 && std::isfinite(h[0].x) && std::isfinite(h[0].y) ? C(h[0].x, h[0].y) / h[1].x : C(0);
        // x += alpha p + omega s, r = s - omega t
        HIPCHK(c, lincomb(x, x, one, p, cd(alpha), sv, cd(omega), n, s));
        HIPCHK(c, lincomb(r, sv, one, t, cd(-omega), nullptr, zero2, n, s));
        HIPCHK(c, norm2(sl.blas, r, n, s));
        if ((e = fetch(1))) return e;
        rel = std::sqrt(h[0].x) / bn;
        rho_old = rho;
        it++;
        if (!std::isfinite(rel)) return fail(c, DDQCD_ERR_NONFINITE, "non-finite residual");
        if (rel <= c->tol) {
            // confirm with the true residual; restart from it if the recursion drifted
            if ((e = apply_A64(c, x, r, s))) return e;
            HIPCHK(c, residual(sl.blas, b, r, n, s));
            if ((e = fetch(1))) return e;
            rel = std::sqrt(h[0].x) / bn;
            if (rel > c->tol && (e = restart(true))) return e;
        }
    }
    info.converged = rel <= c->tol;
    info.iters = it;
    info.restarts = restarts;
    info.rel_residual = rel;
    if (!info.converged) {
        c->err = "BiCGstab not converged: relative residual " + std::to_string(rel);
        return DDQCD_ERR_NOT_CONVERGED;
    }
    return DDQCD_OK;
}

bool is_pm1(double v) { return v == 1.0 || v == -1.0; }

// ---- workspace layout ---------------------------------------------------------
// The sum of every device array the context allocates for nrhs right-hand
// sides (each rounded up to 256 bytes), in three parts: the reduction area at
// the bottom, the arrays of load_gauge, the work slots and the apply_D
// temporaries above it, and the plan region at the top.
size_t ws_result_bytes(int nrhs) { return aligned(sizeof(double2) * 32 * std::max(nrhs, 64)); }

size_t ws_plan_bytes(const Geo &g, int nrhs)
{
    const size_t per_plan =
        aligned(sizeof(SapArgs) * nrhs) + 3 * aligned(sizeof(int2) * ((size_t)nrhs * g.nd + 64));
    return (size_t)(nrhs + 3) * per_plan;
}

size_t ws_main_bytes(ddqcd_t c, int nrhs)
{
    const Geo &g = c->g;
    const size_t V = (size_t)g.V, nc = V * 12, half = (size_t)g.nd * 12 * g.Vh;
    const size_t faces = (size_t)g.nd * sap_face_sites(g.b) * 6;
    size_t gauge = aligned(sizeof(int)) + aligned(V * 4 * 9 * 16) + aligned(V * 4 * 6 * 8) + 2 * aligned(V * 4 * 6 * 4);
    gauge += 2 * (aligned(V * 36 * 16) + aligned(V * 36 * 8) + 2 * aligned(V * 36 * 4));   // clover, C_e / C_o^-1
    size_t slot = 4 * aligned(nc * 16) + 2 * aligned(half * 16) + aligned(faces * 16) + 2 * aligned((size_t)g.nd * 4);
    slot += aligned(sizeof(double2) * BLAS_NBLK * 32) + 2 * aligned(sizeof(double2) * 32);
    slot += aligned(sizeof(double2) * RCOEF);
    slot += 2 * aligned(nc * 16 * basis_columns(c));                        // outer solver basis
    slot += aligned(faces * 16) + aligned((size_t)g.nd * 4);                 // additive Schwarz
    return gauge + (size_t)nrhs * slot + 2 * aligned(nc * 8);               // + apply_D operands
}

size_t ws_total_bytes(ddqcd_t c, int nrhs)
{
    return ws_result_bytes(nrhs) + ws_main_bytes(c, nrhs) + ws_plan_bytes(c->g, nrhs);
}

}  // namespace

// ===========================================================================
// exported entry points
// ===========================================================================

namespace {

// ---- tuner cache: a text file of lines "<key> | b0 b1 b2 b3 product ms", the
// key holding every argument that decides the result (lattice, kappa, c_sw,
// boundary, right-hand sides, precision, SAP and solver parameters) and a
// fingerprint of the gauge field (FNV-1a of its first 64 numbers)
std::string tune_key(const int lattice[4], double kappa, double c_sw, const double boundary[4], const double *U,
                     int nrhs, int prec, int n_cycles, int n_mr, int restart, double tol, int max_cycles,
                     hipStream_t s, int &err)
{
    double head[64] = {};
    err = DDQCD_OK;
    if (hipMemcpyAsync(head, U, sizeof(head), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        err = DDQCD_ERR_DEVICE;
        return "";
    }
    unsigned long long h = 1469598103934665603ull;
    const unsigned char *p = (const unsigned char *)head;
    for (size_t i = 0; i < sizeof(head); i++) h = (h ^ p[i]) * 1099511628211ull;
    char buf[512];
    snprintf(buf, sizeof(buf), "L=%d,%d,%d,%d kappa=%.17g csw=%.17g bc=%.17g,%.17g,%.17g,%.17g nrhs=%d prec=%d "
             "sap=%d,%d solver=%d,%.17g,%d U=%016llx",
             lattice[0], lattice[1], lattice[2], lattice[3], kappa, c_sw, boundary[0], boundary[1], boundary[2],
             boundary[3], nrhs, prec, n_cycles, n_mr, restart, tol, max_cycles, h);
    return buf;
}

bool tune_cache_get(const char *path, const std::string &key, int b[4], int &product, double &ms)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool hit = false;
    while (fgets(line, sizeof(line), f)) {
        const char *bar = strstr(line, " | ");
        if (!bar || (size_t)(bar - line) != key.size() || key.compare(0, key.size(), line, key.size())) continue;
        int v[5];
        double t;
        if (sscanf(bar + 3, "%d %d %d %d %d %lf", &v[0], &v[1], &v[2], &v[3], &v[4], &t) == 6) {
            for (int m = 0; m < 4; m++) b[m] = v[m];
            product = v[4];
            ms = t;
            hit = true;   // the last entry for a key wins
        }
    }
    fclose(f);
    return hit;
}

void tune_cache_put(const char *path, const std::string &key, const int b[4], int product, double ms)
{
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s | %d %d %d %d %d %.6f\n", key.c_str(), b[0], b[1], b[2], b[3], product, ms);
    fclose(f);
}

}  // namespace

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
        const int n = lattice[m] / domain[m];
        if (n < 2 || n % 2) return DDQCD_ERR_GEOMETRY;
    }
    if (!sap_shape_supported(domain)) return DDQCD_ERR_GEOMETRY;
    const long V = (long)lattice[0] * lattice[1] * lattice[2] * lattice[3];
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
    *out = c;
    return DDQCD_OK;
}

int ddqcd_destroy(ddqcd_t c)
{
    if (!c) return DDQCD_OK;
    c->plans.clear();
    if (c->capture) (void)hipStreamDestroy(c->capture);
    if (c->res_host) (void)hipHostFree(c->res_host);
    for (void *p : c->owned) (void)hipFree(p);
    delete c;
    return DDQCD_OK;
}

int ddqcd_set_sap(ddqcd_t c, int n_cycles, int n_mr, int prec, int product)
{
    if (!c) return DDQCD_ERR_ARG;
    if (n_cycles < 1 || n_mr < 1 || n_cycles > 1000 || n_mr > 1000) return fail(c, DDQCD_ERR_ARG, "bad SAP iteration counts");
    if (!valid_prec(prec)) return fail(c, DDQCD_ERR_ARG, "bad precision");
    if (product < DDQCD_PRODUCT_LANE || product > DDQCD_PRODUCT_MFMA_BF16) return fail(c, DDQCD_ERR_ARG, "bad product form");
    if (!sap_prec_supported(c->g.b, prec))
        return fail(c, DDQCD_ERR_GEOMETRY, "no block-solve kernel for this domain shape and precision");
    if (!sap_product_supported(c->g.b, prec, product))
        return fail(c, DDQCD_ERR_GEOMETRY, "the right-hand-side tile forms need 4x4x4x4 domains and FP16 or BF16 "
                                           "storage");
    if (prec == DDQCD_FP64 && c->outer == DDQCD_OUTER_FGCR_MIXED)
        return fail(c, DDQCD_ERR_ARG, "the mixed-precision outer solver needs a reduced-precision preconditioner");
    c->n_cycles = n_cycles;
    c->n_mr = n_mr;
    c->sap_prec = prec;
    c->product = product;
    return DDQCD_OK;
}

int ddqcd_set_schedule(ddqcd_t c, int schedule)
{
    if (!c) return DDQCD_ERR_ARG;
    if (schedule != DDQCD_SCHED_SWEEPS && schedule != DDQCD_SCHED_QUEUE && schedule != DDQCD_SCHED_GRAPH)
        return fail(c, DDQCD_ERR_ARG, "bad schedule");
    if (schedule == DDQCD_SCHED_QUEUE)
        return fail(c, DDQCD_ERR_ARG, "the work-queue schedule is switched off: it stalled on the device and its cause "
                                      "is not established");
    c->schedule = schedule;
    return DDQCD_OK;
}

int ddqcd_set_schwarz(ddqcd_t c, int kind)
{
    if (!c) return DDQCD_ERR_ARG;
    if (kind != DDQCD_SCHWARZ_MULTIPLICATIVE && kind != DDQCD_SCHWARZ_ADDITIVE)
        return fail(c, DDQCD_ERR_ARG, "bad Schwarz variant");
    c->schwarz = kind;
    return DDQCD_OK;
}

int ddqcd_workspace_size(ddqcd_t c, int nrhs, size_t *bytes)
{
    if (!c) return DDQCD_ERR_ARG;
    if (nrhs < 1 || !bytes) return fail(c, DDQCD_ERR_ARG, "bad workspace_size arguments");
    *bytes = ws_total_bytes(c, nrhs);
    return DDQCD_OK;
}

int ddqcd_set_workspace(ddqcd_t c, void *dev_ptr, size_t bytes)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return fail(c, DDQCD_ERR_ARG, "workspace must be 256-byte aligned");
    if (c->ws || c->device >= 0 || !c->owned.empty())
        return fail(c, DDQCD_ERR_STATE, "set_workspace must come before load_gauge, once per context");
    int nrhs = 0;
    while (nrhs < 4096 && ws_total_bytes(c, nrhs + 1) <= bytes) nrhs++;
    if (nrhs == 0)
        return fail(c, DDQCD_ERR_NOMEM, "the workspace is smaller than ddqcd_workspace_size(ctx, 1) = " +
                                            std::to_string(ws_total_bytes(c, 1)));
    c->ws = (unsigned char *)dev_ptr;
    c->ws_bytes = bytes;
    c->ws_plan_bytes = ws_plan_bytes(c->g, nrhs);
    c->ws_plan = c->ws + (bytes - c->ws_plan_bytes) / 256 * 256;
    c->ws_plan_bytes = bytes - (size_t)(c->ws_plan - c->ws);
    c->ws_nrhs = nrhs;
    // the reduction area of the solves this context leads, at the bottom
    c->res_dev = (double2 *)c->ws;
    c->ws_used = ws_result_bytes(nrhs);
    c->res_cap = std::max(nrhs, 64);
    return DDQCD_OK;
}

int ddqcd_set_outer(ddqcd_t c, int kind, int deflate)
{
    if (!c) return DDQCD_ERR_ARG;
    if (kind != DDQCD_OUTER_FGCR && kind != DDQCD_OUTER_FGMRES_DR && kind != DDQCD_OUTER_FGCR_MIXED)
        return fail(c, DDQCD_ERR_ARG, "bad outer solver");
    if (kind != DDQCD_OUTER_FGMRES_DR && deflate != 0) return fail(c, DDQCD_ERR_ARG, "FGCR takes no deflation vectors");
    if (kind == DDQCD_OUTER_FGCR_MIXED && c->sap_prec == DDQCD_FP64)
        return fail(c, DDQCD_ERR_ARG, "the mixed-precision outer solver needs a reduced-precision preconditioner");
    if (deflate < 0 || (kind == DDQCD_OUTER_FGMRES_DR && deflate >= c->restart))
        return fail(c, DDQCD_ERR_ARG, "deflation vectors must be in [0, restart)");
    if (c->ws && !c->slots.empty())
        return fail(c, DDQCD_ERR_STATE, "outer solver fixed once a workspace context has work slots");
    c->outer = kind;
    c->deflate = deflate;
    return DDQCD_OK;
}

int ddqcd_set_solver(ddqcd_t c, int restart, double tol, int max_cycles)
{
    if (!c) return DDQCD_ERR_ARG;
    if (restart < 1 || restart > BLAS_MAXK) return fail(c, DDQCD_ERR_ARG, "restart must be in [1, 16]");
    if (c->outer == DDQCD_OUTER_FGMRES_DR && c->deflate >= restart)
        return fail(c, DDQCD_ERR_ARG, "restart must exceed the deflation vectors");
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
        HIPCHK(c, scratch_setup(c->device));
        if ((e = alloc(c, &c->d_flag, sizeof(int)))) return e;
        if ((e = alloc(c, &c->U64, V * 4 * 9 * 16))) return e;
        if ((e = dev_alloc(c, &c->U32, V * 4 * 6 * 8))) return e;
        if ((e = dev_alloc(c, &c->U16, V * 4 * 6 * 4))) return e;
        if ((e = dev_alloc(c, &c->UB16, V * 4 * 6 * 4))) return e;
        if ((e = alloc(c, &c->C64, V * 36 * 16))) return e;
        if ((e = dev_alloc(c, &c->C32, V * 36 * 8))) return e;
        if ((e = dev_alloc(c, &c->C16, V * 36 * 4))) return e;
        if ((e = dev_alloc(c, &c->CB16, V * 36 * 4))) return e;
        if ((e = alloc(c, &c->Cs64, V * 36 * 16))) return e;
        if ((e = dev_alloc(c, &c->Cs32, V * 36 * 8))) return e;
        if ((e = dev_alloc(c, &c->Cs16, V * 36 * 4))) return e;
        if ((e = dev_alloc(c, &c->CsB16, V * 36 * 4))) return e;
    }
    c->loaded = false;
    HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
    HIPCHK(c, count_nonfinite((const double2 *)U, (long)V * 36, c->d_flag, s));
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (bad) return fail(c, DDQCD_ERR_NONFINITE, "non-finite gauge field");
    HIPCHK(c, import_gauge(g, U, c->U64, s));
    HIPCHK(c, compress_links(g, c->U64, c->U32, P32, s));
    HIPCHK(c, compress_links(g, c->U64, c->U16, P16, s));
    HIPCHK(c, compress_links(g, c->U64, c->UB16, PB16, s));
    HIPCHK(c, clover_build(g, c->U64, c->kappa, c->csw, c->C64, s));
    HIPCHK(c, convert_pairs(c->C64, c->C32, (long)V * 36, P32, s));
    HIPCHK(c, convert_pairs(c->C64, c->C16, (long)V * 36, P16, s));
    HIPCHK(c, convert_pairs(c->C64, c->CB16, (long)V * 36, PB16, s));
    HIPCHK(c, clover_schur(g, c->C64, c->Cs64, c->d_flag, s));
    HIPCHK(c, convert_pairs(c->Cs64, c->Cs32, (long)V * 36, P32, s));
    HIPCHK(c, convert_pairs(c->Cs64, c->Cs16, (long)V * 36, P16, s));
    HIPCHK(c, convert_pairs(c->Cs64, c->CsB16, (long)V * 36, PB16, s));
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
    if (!valid_prec(prec)) return fail(c, DDQCD_ERR_ARG, "bad precision");
    int e = check_ready(c, "apply_D");
    if (e || (e = ensure_slots(c, 1))) return e;
    hipStream_t s = (hipStream_t)stream;
    const Geo &g = c->g;
    const long n = ncomplex(g);
    if (prec != DDQCD_FP64 && !c->t_lo_in) {
        if ((e = dev_alloc(c, &c->t_lo_in, (size_t)n * 8))) return e;
        if ((e = dev_alloc(c, &c->t_lo_out, (size_t)n * 8))) return e;
    }
    Slot &sl = *c->slots[0];
    void *ti = prec == DDQCD_FP64 ? (void *)sl.b : c->t_lo_in;
    void *to = prec == DDQCD_FP64 ? (void *)sl.x : c->t_lo_out;
    for (int k = 0; k < nrhs; k++) {
        HIPCHK(c, import_spinor(g, in + (size_t)k * n * 2, ti, prec, s));
        HIPCHK(c, apply_A(g, ti, to, links_for(c, prec), clover_for(c, prec), prec, s));
        HIPCHK(c, export_spinor(g, to, prec, out + (size_t)k * n * 2, s));
    }
    return DDQCD_OK;
}

int ddqcd_sap(ddqcd_t c, double *out, const double *in, int nrhs, void *stream)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!out || !in || nrhs < 1 || out == in) return fail(c, DDQCD_ERR_ARG, "bad sap arguments");
    int e = check_ready(c, "sap");
    if (e || (e = ensure_slots(c, nrhs))) return e;
    hipStream_t s = (hipStream_t)stream;
    const Geo &g = c->g;
    const long n = ncomplex(g);
    std::vector<Sys> sys;
    std::vector<const double2 *> eta;
    std::vector<double2 *> o;
    for (int k = 0; k < nrhs; k++) {
        Slot *sl = c->slots[k].get();
        sys.push_back({c, sl, k});
        HIPCHK(c, import_spinor(g, in + (size_t)k * n * 2, sl->b, P64, s));
        eta.push_back(sl->b);
        o.push_back(sl->x);
    }
    if ((e = run_sap(sys, eta, o, std::vector<int>(nrhs, 1), s))) return e;
    for (int k = 0; k < nrhs; k++) HIPCHK(c, export_spinor(g, c->slots[k]->x, P64, out + (size_t)k * n * 2, s));
    return DDQCD_OK;
}

int ddqcd_sap_noalloc(ddqcd_t c, double *out, const double *in, void *stream)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!out || !in || out == in) return fail(c, DDQCD_ERR_ARG, "bad sap_noalloc arguments");
    int e = check_ready(c, "sap_noalloc");
    if (e) return e;
    unsigned char *base = scratch_for(c->device);
    if (!base) return fail(c, DDQCD_ERR_STATE, "no scratch address for this device");
    hipStream_t s = (hipStream_t)stream;
    const Geo &g = c->g;
    const bool additive = c->schwarz == DDQCD_SCHWARZ_ADDITIVE;
    // carve the scratch into 256-byte aligned pieces
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    const size_t nc = (size_t)ncomplex(g), half = (size_t)g.nd * 12 * g.Vh;
    const size_t faces = (size_t)g.nd * sap_face_sites(g.b) * 6;
    SapArgs *d_args = (SapArgs *)take(sizeof(SapArgs));
    int2 *items = (int2 *)take(sizeof(int2) * g.nd);
    double2 *eta = (double2 *)take(nc * 16), *res_out = (double2 *)take(nc * 16);
    void *psi = take(nc * 16), *res = take(half * 16), *rho_tmp = take(half * 16), *face = take(faces * 16);
    void *face_alt = additive ? take(faces * 16) : nullptr;
    float *res_scale = (float *)take((size_t)g.nd * 4), *face_scale = (float *)take((size_t)g.nd * 4);
    float *face_scale_alt = additive ? (float *)take((size_t)g.nd * 4) : nullptr;
    if (off > SCRATCH_BYTES)
        return fail(c, DDQCD_ERR_NOMEM, "sap_noalloc needs " + std::to_string(off) + " bytes of scratch for this "
                                        "lattice; the limit is " + std::to_string(SCRATCH_BYTES));
    SapArgs a{};
    a.g = g;
    a.n_mr = c->n_mr;
    a.eta = eta;
    a.out = res_out;
    a.psi = psi;
    a.res = res;
    a.res_scale = res_scale;
    a.face = face;
    a.face_scale = face_scale;
    a.face_alt = face_alt;
    a.face_scale_alt = face_scale_alt;
    a.rho_tmp = rho_tmp;
    a.links = links_for(c, c->sap_prec);
    a.cs = schur_for(c, c->sap_prec);
    a.active = 1;
    HIPCHK(c, import_spinor(g, in, eta, P64, s));
    HIPCHK(c, sap_put_args(a, d_args, s));
    HIPCHK(c, sap_schedule_items(g, sap_rhs_per_workgroup(c->product) > 1 ? 1 << 24 : 0, items, s));
    const int shape = sap_shape_id(g.b), prec = c->sap_prec, half_nd = g.nd / 2;
    for (int cyc = 0; cyc < c->n_cycles; cyc++) {
        Visit v{};
        v.first = cyc == 0;
        v.last = cyc == c->n_cycles - 1;
        v.res_out = !v.last;
        if (additive) {   // one launch per cycle over all domains, alternating boundary buffers
            v.faces_in = cyc > 0;
            v.faces_out = !v.last;
            v.flip = cyc & 1;
            HIPCHK(c, sap_sweep_batch(d_args, items, g.nd, shape, prec, c->product, v, s));
            continue;
        }
        for (int col = 0; col < 2; col++) {
            v.faces_in = !(cyc == 0 && col == 0);
            v.faces_out = !(v.last && col == 1);
            HIPCHK(c, sap_sweep_batch(d_args, items + col * half_nd, half_nd, shape, prec, c->product, v, s));
        }
    }
    HIPCHK(c, export_spinor(g, res_out, P64, out, s));
    return DDQCD_OK;
}

int ddqcd_solve(ddqcd_t c, double *x, const double *b, int nrhs, int x_is_guess, ddqcd_info *info, void *stream)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!x || !b || nrhs < 1 || x == b) return fail(c, DDQCD_ERR_ARG, "bad solve arguments");
    int e = check_ready(c, "solve");
    if (e || (e = ensure_slots(c, nrhs))) return e;
    const long n = ncomplex(c->g);
    std::vector<Sys> sys;
    std::vector<double *> xs;
    std::vector<const double *> bs;
    for (int k = 0; k < nrhs; k++) {
        sys.push_back({c, c->slots[k].get(), k});
        xs.push_back(x + (size_t)k * n * 2);
        bs.push_back(b + (size_t)k * n * 2);
    }
    return solve_systems(sys, xs.data(), bs.data(), x_is_guess, info, (hipStream_t)stream);
}

int ddqcd_solve_batch(const ddqcd_t *ctxs, int n, double *const *x, const double *const *b, int x_is_guess,
                      ddqcd_info *info, void *stream)
{
    if (!ctxs || n < 1 || !x || !b) return DDQCD_ERR_ARG;
    for (int i = 0; i < n; i++)
        if (!ctxs[i]) return DDQCD_ERR_ARG;
    for (int i = 0; i < n; i++)
        if (!x[i] || !b[i] || (const double *)x[i] == b[i])
            return fail(ctxs[i], DDQCD_ERR_ARG, "bad solve_batch arguments for system " + std::to_string(i));
    ddqcd_t c0 = ctxs[0];
    std::vector<Sys> sys;
    std::map<ddqcd_t, int> used;
    for (int i = 0; i < n; i++) {
        ddqcd_t c = ctxs[i];
        int e = check_ready(c, "solve_batch");
        if (e) return e;
        if (c->restart != c0->restart || c->tol != c0->tol || c->max_cycles != c0->max_cycles ||
            c->n_cycles != c0->n_cycles || c->schwarz != c0->schwarz || c->outer != c0->outer ||
            c->deflate != c0->deflate)
            return fail(c, DDQCD_ERR_ARG,
                        "batched contexts need equal solver settings, SAP cycle counts and Schwarz variant");
        const int k = used[c]++;
        if ((e = ensure_slots(c, k + 1))) return e;
        sys.push_back({c, c->slots[k].get(), k});
    }
    return solve_systems(sys, x, b, x_is_guess, info, (hipStream_t)stream);
}

int ddqcd_solve_bicgstab(ddqcd_t c, double *x, const double *b, int x_is_guess, int max_iter, ddqcd_info *info,
                         void *stream)
{
    if (!c) return DDQCD_ERR_ARG;
    if (!x || !b || x == b || max_iter < 1) return fail(c, DDQCD_ERR_ARG, "bad bicgstab arguments");
    int e = check_ready(c, "solve_bicgstab");
    if (e || (e = ensure_slots(c, 1))) return e;
    hipStream_t s = (hipStream_t)stream;
    Slot &sl = *c->slots[0];
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(c, import_spinor(c->g, b, sl.b, P64, s));
    if (x_is_guess) HIPCHK(c, import_spinor(c->g, x, sl.x, P64, s));
    ddqcd_info inf{};
    const int st = bicgstab(c, sl, x_is_guess != 0, max_iter, inf, s);
    if (st != DDQCD_OK && st != DDQCD_ERR_NOT_CONVERGED) return st;
    HIPCHK(c, export_spinor(c->g, sl.x, P64, x, s));
    HIPCHK(c, hipStreamSynchronize(s));
    inf.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return st;
}

int ddqcd_tune_sap(const int lattice[4], double kappa, double c_sw, const double boundary[4], const double *U,
                   const double *b, int nrhs, int prec, int n_cycles, int n_mr, int restart, double tol, int max_cycles,
                   int domain_out[4], int *product_out, double *ms_out, void *stream)
{
    if (!lattice || !boundary || !U || !b || !domain_out || nrhs < 1) return DDQCD_ERR_ARG;
    // the compiled (shape, product) pairs that tile this lattice; the tile
    // forms only for several right-hand sides
    struct Cand {
        int b[4], product;
    };
    std::vector<Cand> cand;
    for (int sh = 0; sh < sap_shape_count(); sh++) {
        Cand cd;
        sap_shape_extents(sh, cd.b);
        bool ok = true;
        for (int m = 0; m < 4; m++) {
            if (lattice[m] < 2 || lattice[m] % cd.b[m]) ok = false;
            else if ((lattice[m] / cd.b[m]) % 2 || lattice[m] / cd.b[m] < 2) ok = false;
        }
        if (!ok) continue;
        for (int pr = DDQCD_PRODUCT_LANE; pr <= DDQCD_PRODUCT_MFMA_BF16; pr++) {
            if (pr != DDQCD_PRODUCT_LANE && nrhs < 2) continue;
            if (!sap_product_supported(cd.b, prec, pr)) continue;
            cd.product = pr;
            cand.push_back(cd);
        }
    }
    if (cand.empty()) return DDQCD_ERR_GEOMETRY;
    if (cand.size() == 1) {   // nothing to choose: no timing
        for (int m = 0; m < 4; m++) domain_out[m] = cand[0].b[m];
        if (product_out) *product_out = cand[0].product;
        if (ms_out) *ms_out = -1;
        return DDQCD_OK;
    }
    // a cached result for exactly this problem, if it names a candidate
    const char *cache = getenv("DDQCD_TUNE_CACHE");
    std::string key;
    if (cache && *cache) {
        int err;
        key = tune_key(lattice, kappa, c_sw, boundary, U, nrhs, prec, n_cycles, n_mr, restart, tol, max_cycles,
                       (hipStream_t)stream, err);
        if (err) return err;
        int cb[4], cp;
        double cms;
        if (tune_cache_get(cache, key, cb, cp, cms))
            for (const Cand &cd : cand)
                if (cd.product == cp && std::equal(cd.b, cd.b + 4, cb)) {
                    for (int m = 0; m < 4; m++) domain_out[m] = cb[m];
                    if (product_out) *product_out = cp;
                    if (ms_out) *ms_out = cms;
                    return DDQCD_OK;
                }
    }
    const size_t bytes = (size_t)lattice[0] * lattice[1] * lattice[2] * lattice[3] * 12 * 16 * nrhs;
    double *x = nullptr;
    if (hipMalloc(&x, bytes) != hipSuccess) return DDQCD_ERR_NOMEM;
    double best = 0;
    int found = 0, last = DDQCD_ERR_GEOMETRY, best_product = DDQCD_PRODUCT_LANE;
    for (const Cand &cd : cand) {
        ddqcd_t c = nullptr;
        int st = ddqcd_create(lattice, cd.b, kappa, c_sw, boundary, &c);
        if (st == DDQCD_OK) st = ddqcd_set_sap(c, n_cycles, n_mr, prec, cd.product);
        if (st == DDQCD_OK) st = ddqcd_set_solver(c, restart, tol, max_cycles);
        if (st == DDQCD_OK) st = ddqcd_load_gauge(c, U, stream);
        if (st == DDQCD_OK) st = ddqcd_solve(c, x, b, nrhs, 0, nullptr, stream);   // first call builds the plans
        double ms = 0;
        if (st == DDQCD_OK) {
            const auto t0 = std::chrono::steady_clock::now();
            st = ddqcd_solve(c, x, b, nrhs, 0, nullptr, stream);
            ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        ddqcd_destroy(c);
        if (st == DDQCD_OK && (!found || ms < best)) {
            best = ms;
            best_product = cd.product;
            found = 1;
            for (int m = 0; m < 4; m++) domain_out[m] = cd.b[m];
            if (product_out) *product_out = cd.product;
        } else if (st != DDQCD_OK) {
            last = st;
        }
    }
    (void)hipFree(x);
    if (!found) return last;
    if (ms_out) *ms_out = best;
    if (!key.empty()) tune_cache_put(cache, key, domain_out, best_product, best);
    return DDQCD_OK;
}

int ddqcd_tune_domain(const int lattice[4], double kappa, double c_sw, const double boundary[4], const double *U,
                      const double *b, int prec, int n_cycles, int n_mr, int restart, double tol, int max_cycles,
                      int domain_out[4], double *ms_out, void *stream)
{
    return ddqcd_tune_sap(lattice, kappa, c_sw, boundary, U, b, 1, prec, n_cycles, n_mr, restart, tol, max_cycles,
                          domain_out, nullptr, ms_out, stream);
}

}  // extern "C"
