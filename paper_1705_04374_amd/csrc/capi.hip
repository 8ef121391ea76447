// C ABI of the library: contexts, validation, the batched solve driver and
// the estimator entry points.  Everything numeric runs in the kernels of
// flow_kernels.hip / mlmc_kernels.hip; this file only lays out memory,
// launches and waits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "flow_kernels.h"
#include "ofm_error.h"
#include "tuning.h"

struct ofm_ctx {
    int device = 0;
    std::string err;
    // grow-only device scratch owned by the context
    void* arena = nullptr;  size_t arena_bytes = 0;     // sample states of solves
    void* meta = nullptr;   size_t meta_bytes = 0;      // descriptors, states, partials, work list
    void* bub = nullptr;    size_t bub_bytes = 0;       // bubbles of the samples
    ofm::SampleState* host_state = nullptr; size_t host_state_cap = 0;  // pinned
    hipStream_t stream = nullptr;   // solves run here (capturable, default priority)
    double last_init_s = 0, last_step_s = 0, last_cell_steps = 0;
    bool timing = false;          // per-launch events around stage kernels
    int64_t t_launches = 0;
    double t_ms = 0.0, t_cells = 0.0;
    ofm::Tuning tuning;
};

namespace ofm {

static thread_local std::string t_err;

int fail(ofm_ctx* ctx, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    t_err = buf;
    return code;
}

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ofm::fail(ctx, OFM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static int grow(ofm_ctx* ctx, void** p, size_t* have, size_t need)
{
    if (need <= *have) return OFM_OK;
    if (*p) { (void)hipFree(*p); *p = nullptr; *have = 0; }
    size_t want = std::max(need, (size_t)1 << 20);
    if (hipMalloc(p, want) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, OFM_ENOMEM, "device allocation of %zu bytes failed", want);
    }
    *have = want;
    return OFM_OK;
}

static PhysD make_phys(const ofm_solve_spec& s)
{
    PhysD p;
    p.g1inv = 1.0 / (s.eos.gamma1 - 1.0);
    p.g2inv = 1.0 / (s.eos.gamma2 - 1.0);
    p.pi1 = s.eos.gamma1 * s.eos.pc1 / (s.eos.gamma1 - 1.0);
    p.pi2 = s.eos.gamma2 * s.eos.pc2 / (s.eos.gamma2 - 1.0);
    p.gamma1 = s.eos.gamma1;
    p.pc1 = s.eos.pc1;
    p.gamma2 = s.eos.gamma2;
    p.pc2 = s.eos.pc2;
    p.eps = s.weno_eps;
    p.rho1 = s.rho1;
    p.rho2 = s.rho2;
    p.p_far = s.p_inf;
    p.order = s.weno_order == 3 ? 3 : 5;
    p.pad = 0;
    return p;
}

static int validate(ofm_ctx* ctx, const ofm_solve_spec* s)
{
    if (!s) return fail(ctx, OFM_EINVAL, "null spec");
    if (s->ndim < 1 || s->ndim > 3) return fail(ctx, OFM_EINVAL, "ndim must be 1, 2 or 3 (got %d)", s->ndim);
    if (s->n < 8 || s->n > 4096) return fail(ctx, OFM_EINVAL, "n must be in [8, 4096] (got %d)", s->n);
    if (s->precision != OFM_F32 && s->precision != OFM_F64) return fail(ctx, OFM_EINVAL, "bad precision");
    if (s->bc != OFM_BC_ZERO_GRADIENT && s->bc != OFM_BC_PERIODIC && s->bc != OFM_BC_CHARACTERISTIC)
        return fail(ctx, OFM_EINVAL, "bad bc");
    int nsub = 1;
    for (int a = 0; a < s->ndim; ++a) nsub *= s->n_sub;
    if (s->n_sub < 1 || nsub > 64) return fail(ctx, OFM_EINVAL, "n_sub^ndim must be in [1, 64]");
    if (!(s->cfl > 0.0 && s->cfl <= 1.0)) return fail(ctx, OFM_EINVAL, "cfl must be in (0, 1]");
    if (!(s->eos.gamma1 > 1.0) || !(s->eos.gamma2 > 1.0)) return fail(ctx, OFM_EINVAL, "gamma must exceed 1");
    if (!(s->weno_eps > 0.0)) return fail(ctx, OFM_EINVAL, "weno_eps must be positive");
    if (s->weno_order != 0 && s->weno_order != 3 && s->weno_order != 5)
        return fail(ctx, OFM_EINVAL, "weno_order must be 0, 3 or 5 (got %d)", s->weno_order);
    if (!(s->rho1 > 0.0) || !(s->rho2 > 0.0)) return fail(ctx, OFM_EINVAL, "densities must be positive");
    if (!(s->ramp_width > 0.0)) return fail(ctx, OFM_EINVAL, "ramp_width must be positive");
    if (s->max_steps < 1) return fail(ctx, OFM_EINVAL, "max_steps must be >= 1");
    if (s->n_steps <= 0 && !(s->t_end > 0.0)) return fail(ctx, OFM_EINVAL, "need t_end > 0 or n_steps > 0");
    return OFM_OK;
}

static int64_t cells_of(const ofm_solve_spec& s)
{
    int64_t c = 1;
    for (int a = 0; a < s.ndim; ++a) c *= s.n;
    return c;
}

static size_t state_bytes(const ofm_solve_spec& s)
{
    return (size_t)(4 + s.ndim) * (size_t)cells_of(s) * (s.precision == OFM_F64 ? 8 : 4);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Descriptor of one sample of a launch: its arrays, tiling (its tiles are
// tile0 .. tile0 + ntiles - 1 of the launch's partials), step control and the
// sensors' balls.
static SampleDesc make_desc(const ofm_solve_spec& s, const TileChoice& tc, int tile0, void* b0, void* b1, void* du)
{
    SampleDesc d{};
    const int nd = s.ndim;
    d.buf[0] = b0;
    d.buf[1] = b1;
    d.du = du;
    d.n = s.n;
    d.ntx = (s.n + tc.tx - 1) / tc.tx;
    d.nty = nd >= 2 ? (s.n + tc.ty - 1) / tc.ty : 1;
    d.nzc = nd == 3 ? (s.n + tc.zchunk - 1) / tc.zchunk : 1;
    d.tile0 = tile0;
    d.ntiles = d.ntx * d.nty * d.nzc;
    d.h = 1.0 / (double)s.n;
    d.cfl = s.cfl;
    d.t_end = s.n_steps > 0 ? INFINITY : s.t_end;
    d.n_steps = s.n_steps;
    d.max_steps = s.max_steps;
    // sensors (ofm_qoi): pressure ball of radius max(R_c / 40, 1.01 half
    // cell diagonals), gas-fraction ball of radius R_c, at the cloud centre
    for (int a = 0; a < 3; ++a) d.centre[a] = s.center[a];
    double rp = s.cloud_radius / 40.0;
    const double hd = 1.01 * 0.5 * d.h * sqrt((double)s.ndim);
    if (hd > rp) rp = hd;
    d.r2_p = rp * rp;
    d.r2_a = s.cloud_radius * s.cloud_radius;
    return d;
}

// One batched run: all members share ndim/precision/bc/eos.
struct Member {
    ofm_solve_spec spec;
    const double* bubbles;  // host
    int32_t nb;
    void* buf0; void* buf1; void* du;   // device arrays (caller's, the context's arena or the run's)
};

}  // namespace ofm

// A batched run in progress: the members, their device descriptors and
// sample states, the captured graph of K steps and the step count.  The
// synchronous entry points build one, advance it to the end and drop it; an
// ofm_run handle keeps it between calls.  Device metadata and the pinned
// host mirror are the run's own when `own` is set (handles), else the
// context's cached buffers.
struct ofm_run {
    ofm_ctx* ctx = nullptr;
    bool own = false;
    std::vector<ofm::Member> mem;
    std::vector<ofm::SampleDesc> desc;
    std::vector<ofm::SampleState> state;   // host copy after the last advance
    ofm::TileChoice tc{};
    ofm::LaunchArgs la{};
    void* meta = nullptr;                   // own metadata (when own)
    ofm::SampleState* pinned = nullptr;     // own pinned mirror (when own)
    ofm::SampleState* host_state = nullptr;
    ofm::SampleState* d_state = nullptr;
    ofm::SampleDesc* d_desc = nullptr;
    ofm::TilePartial* d_part = nullptr;
    double* d_dt = nullptr;
    ofm::WorkItem* d_work = nullptr;
    std::vector<int> order;                 // samples, larger grids first
    int64_t dts_len = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t kev[2] = { nullptr, nullptr };
    bool eager = false;
    int K = 2;
    int64_t taken = 0, cap = 0;
    double live_cells = 0.0;
    double init_s = 0.0, step_s = 0.0;
    void* arena = nullptr;                  // state arrays owned by a handle
    bool finished = false;

    ~ofm_run()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : kev)
            if (e) (void)hipEventDestroy(e);
        if (own) {
            if (meta) (void)hipFree(meta);
            if (pinned) (void)hipHostFree(pinned);
            if (arena) (void)hipFree(arena);
        }
    }
};

namespace ofm {

static double elapsed_s(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms * 1e-3;
}

// Capture K steps of the run (its current work list) into r.gexec.
static int run_capture(ofm_run& r)
{
    ofm_ctx* ctx = r.ctx;
    hipStream_t stream = ctx->stream;
    const ofm_solve_spec& s0 = r.mem[0].spec;
    const int ns = (int)r.mem.size();
    if (r.gexec) { (void)hipGraphExecDestroy(r.gexec); r.gexec = nullptr; }
    if (r.graph) { (void)hipGraphDestroy(r.graph); r.graph = nullptr; }
    HIPCHK(ctx, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    int rc = OFM_OK;
    for (int g = 0; g < r.K && rc == OFM_OK; ++g)
        for (int stg = 0; stg < 3 && rc == OFM_OK; ++stg) {
            r.la.src = (g + stg) & 1;     // replayed at even step indices only
            hipError_t le = launch_stage(s0.precision, s0.ndim, r.tc.tx, r.tc.ty, r.la, stg, stream);
            if (le == hipSuccess && stg == 2)
                le = launch_finalize(r.d_desc, r.d_state, r.d_part, ns, 0, r.d_dt, r.dts_len, stream);
            if (le != hipSuccess) rc = fail(ctx, OFM_EHIP, "launch failed: %s", hipGetErrorString(le));
        }
    hipError_t ce = hipStreamEndCapture(stream, &r.graph);
    if (rc) return rc;
    if (ce != hipSuccess) return fail(ctx, OFM_EHIP, "graph capture failed: %s", hipGetErrorString(ce));
    HIPCHK(ctx, hipGraphInstantiate(&r.gexec, r.graph, nullptr, nullptr, 0));
    return OFM_OK;
}

// Drop the tiles of finished samples from the work list once they are more
// than a tenth of it.  The launch index is mapped to work items in
// contiguous ranges per XCD, so tiles that exit at once would otherwise
// leave some XCDs idle while others carry the live samples; the graph is
// captured again for the shorter grid.  Results do not depend on the tile
// order (each cell's arithmetic and each sample's reduction order are fixed).
static int run_compact(ofm_run& r)
{
    int64_t live = 0;
    for (size_t i = 0; i < r.mem.size(); ++i)
        if (!r.host_state[i].done) live += r.desc[i].ntiles;
    if (live == 0 || (double)live > 0.9 * (double)r.la.n_work) return OFM_OK;
    std::vector<WorkItem> work;
    work.reserve(live);
    for (int i : r.order)
        if (!r.host_state[i].done)
            for (int t = 0; t < r.desc[i].ntiles; ++t) work.push_back(WorkItem{ i, t });
    ofm_ctx* ctx = r.ctx;
    HIPCHK(ctx, hipMemcpyAsync(r.d_work, work.data(), sizeof(WorkItem) * work.size(), hipMemcpyHostToDevice,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    r.la.n_work = (int)work.size();
    return r.eager ? OFM_OK : run_capture(r);
}

// Set up a run of r.mem: descriptors, work list, (init: Q_0 from the
// bubbles, else buf0 as given), the initial reduction and the step graph.
// dts_len > 0 records the step sizes on the device (eager launches).
static int run_begin(ofm_ctx* ctx, ofm_run& r, bool init, int64_t dts_len, hipStream_t user_stream)
{
    // Work already queued by the caller comes first; the solve itself runs on
    // the context's own non-blocking stream, which graph capture requires.
    HIPCHK(ctx, hipStreamSynchronize(user_stream));
    hipStream_t stream = ctx->stream;
    std::vector<Member>& mem = r.mem;
    r.ctx = ctx;
    r.dts_len = dts_len;
    const int ns = (int)mem.size();
    const ofm_solve_spec& s0 = mem[0].spec;
    const int prec = s0.precision, nd = s0.ndim, bc = s0.bc;
    for (const Member& m : mem) {
        if (m.spec.ndim != nd || m.spec.precision != prec || m.spec.bc != bc || m.spec.weno_eps != s0.weno_eps ||
            (m.spec.weno_order == 3) != (s0.weno_order == 3) || m.spec.rho1 != s0.rho1 || m.spec.rho2 != s0.rho2 ||
            memcmp(&m.spec.eos, &s0.eos, sizeof(ofm_eos)) != 0)
            return fail(ctx, OFM_EINVAL,
                        "batched items must share ndim, precision, bc, eos, rho1, rho2, weno_eps and weno_order");
        if (bc == OFM_BC_PERIODIC && m.spec.n < 6) return fail(ctx, OFM_EINVAL, "periodic grids need n >= 6");
        if (bc == OFM_BC_CHARACTERISTIC && m.spec.p_inf != s0.p_inf)
            return fail(ctx, OFM_EINVAL, "batched items with the far-field boundary must share p_inf");
    }
    // tiling
    int maxn = 0;
    for (const Member& m : mem) maxn = std::max(maxn, m.spec.n);
    r.tc = ctx->tuning.choose(prec, nd, maxn, ns);
    const TileChoice& tc = r.tc;
    r.desc.assign(ns, SampleDesc{});
    int tiles = 0;
    for (int i = 0; i < ns; ++i) {
        r.desc[i] = make_desc(mem[i].spec, tc, tiles, mem[i].buf0, mem[i].buf1, mem[i].du);
        tiles += r.desc[i].ntiles;
    }
    // work list: larger samples first, tiles of a sample contiguous
    r.order.resize(ns);
    for (int i = 0; i < ns; ++i) r.order[i] = i;
    std::stable_sort(r.order.begin(), r.order.end(), [&](int a, int b) { return mem[a].spec.n > mem[b].spec.n; });
    std::vector<WorkItem> work;
    work.reserve(tiles);
    for (int i : r.order)
        for (int t = 0; t < r.desc[i].ntiles; ++t) work.push_back(WorkItem{ i, t });

    const size_t o_desc = 0;
    const size_t o_state = align256(o_desc + sizeof(SampleDesc) * ns);
    const size_t o_part = align256(o_state + sizeof(SampleState) * ns);
    const size_t o_work = align256(o_part + sizeof(TilePartial) * tiles);
    const size_t o_dt = align256(o_work + sizeof(WorkItem) * work.size());
    const size_t meta_need = o_dt + sizeof(double) * (size_t)std::max<int64_t>(dts_len, 1);
    char* meta;
    if (r.own) {
        HIPCHK(ctx, hipMalloc(&r.meta, meta_need));
        HIPCHK(ctx, hipHostMalloc((void**)&r.pinned, sizeof(SampleState) * ns, hipHostMallocDefault));
        meta = (char*)r.meta;
        r.host_state = r.pinned;
    } else {
        int rc = grow(ctx, &ctx->meta, &ctx->meta_bytes, meta_need);
        if (rc) return rc;
        if (ctx->host_state_cap < (size_t)ns) {
            if (ctx->host_state) (void)hipHostFree(ctx->host_state);
            ctx->host_state = nullptr;
            ctx->host_state_cap = 0;
            HIPCHK(ctx, hipHostMalloc((void**)&ctx->host_state, sizeof(SampleState) * ns, hipHostMallocDefault));
            ctx->host_state_cap = ns;
        }
        meta = (char*)ctx->meta;
        r.host_state = ctx->host_state;
    }
    r.d_desc = (SampleDesc*)(meta + o_desc);
    r.d_state = (SampleState*)(meta + o_state);
    r.d_part = (TilePartial*)(meta + o_part);
    WorkItem* d_work = r.d_work = (WorkItem*)(meta + o_work);
    r.d_dt = dts_len > 0 ? (double*)(meta + o_dt) : nullptr;

    std::vector<SampleState> st0(ns);
    for (auto& s : st0) memset(&s, 0, sizeof s);
    HIPCHK(ctx, hipMemcpyAsync(r.d_desc, r.desc.data(), sizeof(SampleDesc) * ns, hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemcpyAsync(r.d_state, st0.data(), sizeof(SampleState) * ns, hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemcpyAsync(d_work, work.data(), sizeof(WorkItem) * work.size(), hipMemcpyHostToDevice, stream));

    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    HIPCHK(ctx, hipEventRecord(e0, stream));

    const PhysD ph = make_phys(s0);
    if (init) {
        size_t nbub = 0;
        for (const Member& m : mem) nbub += (size_t)m.nb;
        int rc = grow(ctx, &ctx->bub, &ctx->bub_bytes, sizeof(double) * 4 * std::max<size_t>(nbub, 1));
        if (rc) return rc;
        std::vector<double> hb;
        hb.reserve(4 * nbub);
        for (const Member& m : mem) hb.insert(hb.end(), m.bubbles, m.bubbles + 4 * (size_t)m.nb);
        if (nbub)
            HIPCHK(ctx, hipMemcpyAsync(ctx->bub, hb.data(), sizeof(double) * hb.size(), hipMemcpyHostToDevice, stream));
        size_t off = 0;
        for (const Member& m : mem) {
            InitLaunch L;
            L.ph = ph;
            L.bubbles = (const double*)ctx->bub + 4 * off;
            L.nb = m.nb;
            L.n = m.spec.n;
            L.n_sub = m.spec.n_sub;
            L.rho1 = m.spec.rho1; L.rho2 = m.spec.rho2;
            L.p_bubble = m.spec.p_bubble; L.p_inf = m.spec.p_inf;
            for (int a = 0; a < 3; ++a) L.center[a] = m.spec.center[a];
            L.radius = m.spec.cloud_radius; L.delta = m.spec.ramp_delta; L.width = m.spec.ramp_width;
            L.u = m.buf0;
            HIPCHK(ctx, launch_init(prec, nd, L, stream));
            off += (size_t)m.nb;
        }
        // the host bubbles vector must outlive the copy
        HIPCHK(ctx, hipStreamSynchronize(stream));
    }
    LaunchArgs& la = r.la;
    la.ph = ph;
    la.work = d_work;
    la.n_work = (int)work.size();
    la.zchunk = tc.zchunk;
    la.desc = r.d_desc;
    la.state = r.d_state;
    la.part = r.d_part;
    la.bc = bc;
    la.src = 0;
    HIPCHK(ctx, launch_reduce(prec, nd, tc.tx, tc.ty, la, stream));
    HIPCHK(ctx, launch_finalize(r.d_desc, r.d_state, r.d_part, ns, 1, r.d_dt, dts_len, stream));
    HIPCHK(ctx, hipEventRecord(e1, stream));
    HIPCHK(ctx, hipEventSynchronize(e1));
    r.init_s = elapsed_s(e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);

    r.cap = 0;
    for (const Member& m : mem) r.cap = std::max(r.cap, m.spec.n_steps > 0 ? m.spec.n_steps : m.spec.max_steps);
    // eager launches for the low-level stepper (per-step control) and while
    // kernels are being timed; captured graphs otherwise
    r.eager = dts_len > 0 || ctx->timing;
    r.K = r.eager ? 2 : tc.graph_steps;
    if (ctx->timing) {
        HIPCHK(ctx, hipEventCreate(&r.kev[0]));
        HIPCHK(ctx, hipEventCreate(&r.kev[1]));
    }
    r.live_cells = 0.0;
    for (int i = 0; i < ns; ++i) r.live_cells += (double)cells_of(mem[i].spec);
    r.state.assign(st0.begin(), st0.end());
    if (!r.eager) return run_capture(r);
    return OFM_OK;
}

// Eager launches of steps g0 .. g0+nsteps-1 (the state of step g sits in
// buffer g & 1; stage stg of step g reads buffer (3 g + stg) & 1).
static int run_enqueue(ofm_run& r, int nsteps, int64_t g0)
{
    ofm_ctx* ctx = r.ctx;
    hipStream_t stream = ctx->stream;
    const ofm_solve_spec& s0 = r.mem[0].spec;
    const int ns = (int)r.mem.size();
    for (int g = 0; g < nsteps; ++g)
        for (int stg = 0; stg < 3; ++stg) {
            r.la.src = (int)((g0 + g + stg) & 1);
            if (ctx->timing) HIPCHK(ctx, hipEventRecord(r.kev[0], stream));
            HIPCHK(ctx, launch_stage(s0.precision, s0.ndim, r.tc.tx, r.tc.ty, r.la, stg, stream));
            if (ctx->timing) {
                HIPCHK(ctx, hipEventRecord(r.kev[1], stream));
                HIPCHK(ctx, hipEventSynchronize(r.kev[1]));
                float ms = 0.f;
                HIPCHK(ctx, hipEventElapsedTime(&ms, r.kev[0], r.kev[1]));
                ctx->t_launches += 1;
                ctx->t_ms += ms;
                ctx->t_cells += r.live_cells;
            }
            if (stg == 2)
                HIPCHK(ctx, launch_finalize(r.d_desc, r.d_state, r.d_part, ns, 0, r.d_dt, r.dts_len, stream));
        }
    return OFM_OK;
}

// Advance until every sample is done or at least max_steps more steps have
// been enqueued (whole graphs of K steps); r.state holds the states after.
static int run_advance(ofm_run& r, int64_t max_steps)
{
    ofm_ctx* ctx = r.ctx;
    hipStream_t stream = ctx->stream;
    const int ns = (int)r.mem.size();
    if (r.finished) return OFM_OK;
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    HIPCHK(ctx, hipEventRecord(e0, stream));
    const int64_t start = r.taken;
    int result = OFM_OK;
    for (;;) {
        int todo = r.K;
        int rc;
        if (r.eager) {
            // no launches past the step cap (they would find every sample done)
            todo = (int)std::min<int64_t>(r.K, std::max<int64_t>(1, r.cap - r.taken));
            rc = run_enqueue(r, todo, r.taken);
        } else {
            hipError_t le = hipGraphLaunch(r.gexec, stream);
            rc = le == hipSuccess ? OFM_OK : fail(ctx, OFM_EHIP, "graph launch failed: %s", hipGetErrorString(le));
        }
        if (rc) { result = rc; break; }
        r.taken += todo;
        hipError_t ce = hipMemcpyAsync(r.host_state, r.d_state, sizeof(SampleState) * ns, hipMemcpyDeviceToHost, stream);
        if (ce == hipSuccess) ce = hipStreamSynchronize(stream);
        if (ce != hipSuccess) { result = fail(ctx, OFM_EHIP, "state read-back failed: %s", hipGetErrorString(ce)); break; }
        bool all = true;
        r.live_cells = 0.0;
        for (int i = 0; i < ns; ++i) {
            all = all && r.host_state[i].done;
            if (!r.host_state[i].done) r.live_cells += (double)cells_of(r.mem[i].spec);
        }
        r.state.assign(r.host_state, r.host_state + ns);
        if (all) { r.finished = true; break; }
        if ((rc = run_compact(r)) != OFM_OK) { result = rc; break; }
        if (r.taken > r.cap + 2 * r.K) { result = fail(ctx, OFM_EHIP, "samples did not finish within the step cap"); break; }
        if (r.taken - start >= max_steps) break;
    }
    (void)hipEventRecord(e1, stream);
    (void)hipEventSynchronize(e1);
    r.step_s += elapsed_s(e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return result;
}

// Statistics of a finished run into the context; the step sizes to the host.
static int run_stats(ofm_run& r, double* dts_host)
{
    ofm_ctx* ctx = r.ctx;
    ctx->last_init_s = r.init_s;
    ctx->last_step_s = r.step_s;
    double cs = 0;
    for (size_t i = 0; i < r.mem.size(); ++i) cs += (double)cells_of(r.mem[i].spec) * (double)r.state[i].steps;
    ctx->last_cell_steps = cs;
    if (dts_host && r.dts_len > 0)
        HIPCHK(ctx, hipMemcpy(dts_host, r.d_dt, sizeof(double) * r.dts_len, hipMemcpyDeviceToHost));
    return OFM_OK;
}

// Runs members to completion.  init: 1 = build Q_0 from bubbles, 0 = use buf0.
static int run(ofm_ctx* ctx, std::vector<Member>& mem, bool init, double* dts_host, int64_t dts_len,
               std::vector<SampleState>& out, hipStream_t user_stream)
{
    ofm_run r;
    r.mem = mem;
    int rc = run_begin(ctx, r, init, dts_host ? dts_len : 0, user_stream);
    if (rc == OFM_OK) rc = run_advance(r, INT64_MAX);
    if (rc == OFM_OK) rc = run_stats(r, dts_host);
    if (rc == OFM_OK) out = r.state;
    return rc;
}

static void to_qoi(const ofm_solve_spec& s, const SampleState& st, ofm_qoi* q)
{
    memset(q, 0, sizeof *q);
    q->p_max = st.p_max;
    q->t_at_max = st.t_at_max;
    q->t = st.t;
    q->argmax = st.argmax;
    q->steps = st.steps;
    q->status = st.status;
    const int64_t n = s.n;
    const int64_t a = st.argmax < 0 || st.argmax == INT64_MAX ? 0 : st.argmax;
    q->x[0] = ((double)(a % n) + 0.5) / (double)n;
    if (s.ndim > 1) q->x[1] = ((double)((a / n) % n) + 0.5) / (double)n;
    if (s.ndim > 2) q->x[2] = ((double)(a / (n * n)) + 0.5) / (double)n;
    q->p_sensor = st.p_sensor;
    q->t_p_sensor = st.t_p_sensor;
    q->gas_min = st.gas_min;
    q->t_gas_min = st.t_gas_min;
    q->c_max = st.c_max;
    double dd = 0.0;
    for (int k = 0; k < s.ndim; ++k) dd = dd + (q->x[k] - s.center[k]) * (q->x[k] - s.center[k]);
    q->peak_distance = sqrt(dd);
}

}  // namespace ofm

// ---------------------------------------------------------------------------
// Stepping without allocation (ofm_step_noalloc)
// ---------------------------------------------------------------------------
// The stepper's scratch lives in a fixed device array: the sample
// descriptor, its dynamic state, one reduction partial per tile, the work
// list and the step-size log.  Every GPU the library runs on holds its own
// copy until the process ends; all calls on that GPU share it.
static __device__ __align__(256) unsigned char scratch[OFM_NOALLOC_SCRATCH_BYTES];

namespace ofm {

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// Resolve the device address of `scratch` on ctx's device (current), once
// per device.  Host code uses only this address: the array's name is a
// host-side stand-in.
static int resolve_scratch(ofm_ctx* ctx)
{
    if (ctx->device >= kMaxDevices) return fail(ctx, OFM_EUNSUPPORTED, "device %d beyond %d", ctx->device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[ctx->device]) return OFM_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(ctx, OFM_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch[ctx->device] = (char*)p;
    return OFM_OK;
}

static char* scratch_of(const ofm_ctx* ctx)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return ctx->device < kMaxDevices ? g_scratch[ctx->device] : nullptr;
}

// Descriptor, a zeroed dynamic state and the work list (tiles 0..ntiles-1
// of sample 0), written by the device from kernel arguments (no copies from
// host memory).
__global__ void __launch_bounds__(256) noalloc_setup_kernel(SampleDesc d, SampleDesc* dd, SampleState* ds,
                                                            WorkItem* work, int ntiles)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i == 0) {
        *dd = d;
        SampleState z{};
        *ds = z;
    }
    if (i < ntiles) work[i] = WorkItem{ 0, i };
}

}  // namespace ofm

using namespace ofm;

extern "C" {

int ofm_ctx_create(int device, ofm_ctx** out)
{
    if (!out) return fail(nullptr, OFM_EINVAL, "ofm_ctx_create: null out");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(nullptr, OFM_EHIP, "ofm_ctx_create: no HIP device %d (found %d)", device, count);
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, OFM_EHIP, "ofm_ctx_create: hipSetDevice failed");
    ofm_ctx* c = new ofm_ctx();
    c->device = device;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(nullptr, OFM_EHIP, "ofm_ctx_create: stream creation failed");
    }
    const int rc = resolve_scratch(c);
    if (rc) {
        const std::string msg = c->err;
        (void)hipStreamDestroy(c->stream);
        delete c;
        return fail(nullptr, rc, "ofm_ctx_create: %s", msg.c_str());
    }
    *out = c;
    return OFM_OK;
}

void ofm_ctx_destroy(ofm_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->meta) (void)hipFree(ctx->meta);
    if (ctx->bub) (void)hipFree(ctx->bub);
    if (ctx->host_state) (void)hipHostFree(ctx->host_state);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* ofm_last_error(const ofm_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : t_err.c_str();
}

int ofm_state_init(ofm_ctx* ctx, const ofm_solve_spec* spec, const double* bubbles, int32_t nb, ofm_state_view* st,
                   void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    int rc = validate(ctx, spec);
    if (rc) return rc;
    if (!st || !st->u || (nb > 0 && !bubbles) || nb < 0) return fail(ctx, OFM_EINVAL, "ofm_state_init: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    rc = grow(ctx, &ctx->bub, &ctx->bub_bytes, sizeof(double) * 4 * std::max(nb, 1));
    if (rc) return rc;
    if (nb) HIPCHK(ctx, hipMemcpyAsync(ctx->bub, bubbles, sizeof(double) * 4 * nb, hipMemcpyHostToDevice, s));
    InitLaunch L;
    L.ph = make_phys(*spec);
    L.bubbles = (const double*)ctx->bub;
    L.nb = nb;
    L.n = spec->n;
    L.n_sub = spec->n_sub;
    L.rho1 = spec->rho1; L.rho2 = spec->rho2; L.p_bubble = spec->p_bubble; L.p_inf = spec->p_inf;
    for (int a = 0; a < 3; ++a) L.center[a] = spec->center[a];
    L.radius = spec->cloud_radius; L.delta = spec->ramp_delta; L.width = spec->ramp_width;
    L.u = st->u;
    HIPCHK(ctx, launch_init(spec->precision, spec->ndim, L, s));
    HIPCHK(ctx, hipStreamSynchronize(s));   // the host bubbles may go away
    return OFM_OK;
}

int ofm_state_from_primitive(ofm_ctx* ctx, const ofm_solve_spec* spec, const void* w, ofm_state_view* st,
                             void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    int rc = validate(ctx, spec);
    if (rc) return rc;
    if (!w || !st || !st->u) return fail(ctx, OFM_EINVAL, "ofm_state_from_primitive: null pointer");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_prim_to_cons(spec->precision, spec->ndim, make_phys(*spec), w, st->u, cells_of(*spec),
                                    (hipStream_t)stream));
    return OFM_OK;
}

int ofm_state_to_conserved(ofm_ctx* ctx, const ofm_solve_spec* spec, const ofm_state_view* st, double* q,
                           void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    int rc = validate(ctx, spec);
    if (rc) return rc;
    if (!q || !st || !st->u) return fail(ctx, OFM_EINVAL, "ofm_state_to_conserved: null pointer");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_to_conserved(spec->precision, spec->ndim, make_phys(*spec), st->u, q, cells_of(*spec),
                                    (hipStream_t)stream));
    return OFM_OK;
}

int ofm_step(ofm_ctx* ctx, const ofm_solve_spec* spec, ofm_state_view* st, int64_t n_steps, ofm_qoi* qoi,
             double* dts, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    int rc = validate(ctx, spec);
    if (rc) return rc;
    if (!st || !st->u || !st->u_tmp || !st->du || n_steps < 1 || !qoi)
        return fail(ctx, OFM_EINVAL, "ofm_step: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    std::vector<Member> mem(1);
    mem[0].spec = *spec;
    mem[0].spec.n_steps = n_steps;
    mem[0].spec.max_steps = n_steps;
    mem[0].bubbles = nullptr;
    mem[0].nb = 0;
    mem[0].buf0 = st->u;
    mem[0].buf1 = st->u_tmp;
    mem[0].du = st->du;
    std::vector<double> dloc;
    double* dptr = dts;
    if (!dptr) { dloc.resize(n_steps); dptr = dloc.data(); }
    std::vector<SampleState> out;
    rc = run(ctx, mem, false, dptr, n_steps, out, (hipStream_t)stream);
    if (rc) return rc;
    to_qoi(mem[0].spec, out[0], qoi);
    if (out[0].steps & 1) std::swap(st->u, st->u_tmp);
    return OFM_OK;
}

int ofm_step_noalloc(ofm_ctx* ctx, const ofm_solve_spec* spec, ofm_state_view* st, int64_t n_steps, ofm_qoi* qoi,
                     double* dts, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    int rc = validate(ctx, spec);
    if (rc) return rc;
    if (!st || !st->u || !st->u_tmp || !st->du || n_steps < 1 || !qoi)
        return fail(ctx, OFM_EINVAL, "ofm_step_noalloc: bad arguments");
    ofm_solve_spec s = *spec;
    s.n_steps = n_steps;
    s.max_steps = n_steps;
    const TileChoice tc = ctx->tuning.choose(s.precision, s.ndim, s.n, 1);
    const SampleDesc d = make_desc(s, tc, 0, st->u, st->u_tmp, st->du);
    // scratch layout: descriptor | state | partials | work list | step sizes
    const size_t o_state = align256(sizeof(SampleDesc));
    const size_t o_part = align256(o_state + sizeof(SampleState));
    const size_t o_work = align256(o_part + sizeof(TilePartial) * (size_t)d.ntiles);
    const size_t o_dt = align256(o_work + sizeof(WorkItem) * (size_t)d.ntiles);
    const size_t need = o_dt + (dts ? sizeof(double) * (size_t)n_steps : 0);
    if (need > (size_t)OFM_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, OFM_EINVAL,
                    "ofm_step_noalloc: %d tiles%s need %zu bytes of scratch; the fixed scratch holds %zu",
                    d.ntiles, dts ? " and the step-size log" : "", need, (size_t)OFM_NOALLOC_SCRATCH_BYTES);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    char* base = scratch_of(ctx);
    if (!base) return fail(ctx, OFM_EHIP, "ofm_step_noalloc: scratch of device %d not resolved", ctx->device);
    SampleDesc* d_desc = (SampleDesc*)base;
    SampleState* d_state = (SampleState*)(base + o_state);
    TilePartial* d_part = (TilePartial*)(base + o_part);
    WorkItem* d_work = (WorkItem*)(base + o_work);
    double* d_dt = dts ? (double*)(base + o_dt) : nullptr;
    const int64_t dt_len = dts ? n_steps : 0;
    hipStream_t hs = (hipStream_t)stream;
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3((d.ntiles + 255) / 256), dim3(256), 0, hs, d, d_desc, d_state,
                       d_work, d.ntiles);
    HIPCHK(ctx, hipGetLastError());
    LaunchArgs la{};
    la.ph = make_phys(s);
    la.work = d_work;
    la.n_work = d.ntiles;
    la.zchunk = tc.zchunk;
    la.desc = d_desc;
    la.state = d_state;
    la.part = d_part;
    la.bc = s.bc;
    la.src = 0;
    // the same launches as ofm_step: the reduction of the initial level, then
    // per step three stages (stage k of step g reads buffer (g + k) & 1) and
    // the finalisation
    HIPCHK(ctx, launch_reduce(s.precision, s.ndim, tc.tx, tc.ty, la, hs));
    HIPCHK(ctx, launch_finalize(d_desc, d_state, d_part, 1, 1, d_dt, dt_len, hs));
    for (int64_t g = 0; g < n_steps; ++g)
        for (int stg = 0; stg < 3; ++stg) {
            la.src = (int)((g + stg) & 1);
            HIPCHK(ctx, launch_stage(s.precision, s.ndim, tc.tx, tc.ty, la, stg, hs));
            if (stg == 2) HIPCHK(ctx, launch_finalize(d_desc, d_state, d_part, 1, 0, d_dt, dt_len, hs));
        }
    SampleState out;
    HIPCHK(ctx, hipMemcpyAsync(&out, d_state, sizeof out, hipMemcpyDeviceToHost, hs));
    if (dts) HIPCHK(ctx, hipMemcpyAsync(dts, d_dt, sizeof(double) * (size_t)n_steps, hipMemcpyDeviceToHost, hs));
    HIPCHK(ctx, hipStreamSynchronize(hs));
    to_qoi(s, out, qoi);
    if (out.steps & 1) std::swap(st->u, st->u_tmp);
    return OFM_OK;
}

static int solve_members(ofm_ctx* ctx, const ofm_batch_item* items, int32_t n, ofm_qoi* qoi, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (!items || n < 1 || !qoi) return fail(ctx, OFM_EINVAL, "bad batch arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    std::vector<Member> mem(n);
    size_t need = 0;
    for (int i = 0; i < n; ++i) {
        int rc = validate(ctx, items[i].spec);
        if (rc) return rc;
        if (items[i].n_bubbles < 0 || (items[i].n_bubbles > 0 && !items[i].bubbles))
            return fail(ctx, OFM_EINVAL, "item %d: bad bubbles", i);
        mem[i].spec = *items[i].spec;
        mem[i].bubbles = items[i].bubbles;
        mem[i].nb = items[i].n_bubbles;
        need += 3 * align256(state_bytes(mem[i].spec));
    }
    int rc = grow(ctx, &ctx->arena, &ctx->arena_bytes, need);
    if (rc) return rc;
    char* p = (char*)ctx->arena;
    for (int i = 0; i < n; ++i) {
        const size_t b = align256(state_bytes(mem[i].spec));
        mem[i].buf0 = p; p += b;
        mem[i].buf1 = p; p += b;
        mem[i].du = p; p += b;
    }
    std::vector<SampleState> out;
    rc = run(ctx, mem, true, nullptr, 0, out, (hipStream_t)stream);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) to_qoi(mem[i].spec, out[i], qoi + i);
    return OFM_OK;
}

int ofm_solve(ofm_ctx* ctx, const ofm_solve_spec* spec, const double* bubbles, int32_t nb, ofm_qoi* qoi,
              void* stream)
{
    ofm_batch_item it;
    it.spec = spec;
    it.bubbles = bubbles;
    it.n_bubbles = nb;
    it.reserved = 0;
    return solve_members(ctx, &it, 1, qoi, stream);
}

int ofm_solve_batch(ofm_ctx* ctx, const ofm_batch_item* items, int32_t n, ofm_qoi* qoi, void* stream)
{
    return solve_members(ctx, items, n, qoi, stream);
}

int ofm_run_begin(ofm_ctx* ctx, const ofm_batch_item* items, int32_t n, ofm_run** out, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (!items || n < 1 || !out) return fail(ctx, OFM_EINVAL, "ofm_run_begin: bad arguments");
    *out = nullptr;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    ofm_run* r = new ofm_run();
    r->own = true;
    r->mem.resize(n);
    size_t need = 0;
    for (int i = 0; i < n; ++i) {
        int rc = validate(ctx, items[i].spec);
        if (rc) { delete r; return rc; }
        if (items[i].n_bubbles < 0 || (items[i].n_bubbles > 0 && !items[i].bubbles)) {
            delete r;
            return fail(ctx, OFM_EINVAL, "item %d: bad bubbles", i);
        }
        r->mem[i].spec = *items[i].spec;
        r->mem[i].bubbles = items[i].bubbles;
        r->mem[i].nb = items[i].n_bubbles;
        need += 3 * align256(state_bytes(r->mem[i].spec));
    }
    if (hipMalloc(&r->arena, need) != hipSuccess) {
        r->arena = nullptr;
        (void)hipGetLastError();
        delete r;
        return fail(ctx, OFM_ENOMEM, "ofm_run_begin: device allocation of %zu bytes failed", need);
    }
    char* p = (char*)r->arena;
    for (int i = 0; i < n; ++i) {
        const size_t b = align256(state_bytes(r->mem[i].spec));
        r->mem[i].buf0 = p; p += b;
        r->mem[i].buf1 = p; p += b;
        r->mem[i].du = p; p += b;
    }
    int rc = run_begin(ctx, *r, true, 0, (hipStream_t)stream);
    if (rc) { delete r; return rc; }
    *out = r;
    return OFM_OK;
}

int ofm_run_advance(ofm_run* run, int64_t max_steps, int32_t* done)
{
    if (!run) return fail(nullptr, OFM_EINVAL, "null run");
    if (max_steps < 1) return fail(run->ctx, OFM_EINVAL, "ofm_run_advance: max_steps must be >= 1");
    HIPCHK(run->ctx, hipSetDevice(run->ctx->device));
    int rc = run_advance(*run, max_steps);
    if (done) *done = run->finished ? 1 : 0;
    return rc;
}

int ofm_run_status(const ofm_run* run, ofm_qoi* qoi, int64_t* steps_taken, double* init_s, double* step_s)
{
    if (!run) return fail(nullptr, OFM_EINVAL, "null run");
    if (qoi)
        for (size_t i = 0; i < run->mem.size(); ++i) to_qoi(run->mem[i].spec, run->state[i], qoi + i);
    if (steps_taken) *steps_taken = run->taken;
    if (init_s) *init_s = run->init_s;
    if (step_s) *step_s = run->step_s;
    return OFM_OK;
}

void ofm_run_destroy(ofm_run* run)
{
    if (!run) return;
    (void)hipSetDevice(run->ctx->device);
    (void)hipStreamSynchronize(run->ctx->stream);
    delete run;
}

int ofm_last_solve_stats(const ofm_ctx* ctx, double* init_s, double* step_s, double* cell_steps)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (init_s) *init_s = ctx->last_init_s;
    if (step_s) *step_s = ctx->last_step_s;
    if (cell_steps) *cell_steps = ctx->last_cell_steps;
    return OFM_OK;
}

int ofm_tune_set(ofm_ctx* ctx, int32_t precision, int32_t ndim, int32_t n, int32_t tx, int32_t ty, int32_t zchunk,
                 int32_t graph_steps)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (!tile_supported(precision, ndim, tx, ty))
        return fail(ctx, OFM_EUNSUPPORTED, "tile %dx%d not compiled for precision %d, ndim %d", tx, ty, precision, ndim);
    if (zchunk < 1 || zchunk > 4096 || graph_steps < 2 || (graph_steps & 1))
        return fail(ctx, OFM_EINVAL, "zchunk must be >= 1 and graph_steps even and >= 2");
    ctx->tuning.set(precision, ndim, n, TileChoice{ tx, ty, zchunk, graph_steps });
    return OFM_OK;
}

int ofm_tune_get(const ofm_ctx* ctx, int32_t precision, int32_t ndim, int32_t n, ofm_tune_result* out)
{
    if (!ctx || !out) return fail(nullptr, OFM_EINVAL, "ofm_tune_get: null argument");
    if (ndim < 1 || ndim > 3 || (precision != OFM_F32 && precision != OFM_F64) || n < 1)
        return fail(const_cast<ofm_ctx*>(ctx), OFM_EINVAL, "ofm_tune_get: bad precision, ndim or n");
    const TileChoice t = ctx->tuning.choose(precision, ndim, n, 1);
    *out = ofm_tune_result{ t.tx, t.ty, t.zchunk, t.graph_steps, 0.0, 0, 0 };
    return OFM_OK;
}

int ofm_autotune(ofm_ctx* ctx, const ofm_solve_spec* spec, ofm_state_view* st, int32_t steps,
                 ofm_tune_result* out, ofm_tune_result* all, int32_t all_cap, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    int rc = validate(ctx, spec);
    if (rc) return rc;
    if (!st || !st->u || !st->u_tmp || !st->du || steps < 1 || steps > 1000 || !out || all_cap < 0 ||
        (all_cap > 0 && !all))
        return fail(ctx, OFM_EINVAL, "ofm_autotune: bad arguments");
    int tiles[32][2];
    const int nt = std::min(tile_list(spec->precision, spec->ndim, tiles, 32), 32);
    int cus = 0;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) cus = 0;
    // z-chunks of a tile: fixed sizes, and those whose workgroup count fills
    // whole rounds of the GPU (every CU holding its resident workgroups; a
    // last round partly empty leaves CUs idle while it runs)
    auto zchunks = [&](int tx, int ty) {
        std::vector<int> z;
        if (spec->ndim != 3) return std::vector<int>{ 1 };
        for (int c : { 8, 16, 32, 64 })
            if (c <= spec->n) z.push_back(c);
        const int per = stage_blocks_per_cu(spec->precision, spec->ndim, tx, ty, spec->weno_order == 3 ? 3 : 5);
        const long long slots = (long long)cus * per;
        const long long xy = (long long)((spec->n + tx - 1) / tx) * ((spec->n + ty - 1) / ty);
        for (int r = 1; slots > 0 && r <= 8; ++r) {
            const long long nzc = (r * slots + xy - 1) / xy;
            if (nzc > spec->n) break;
            const int c = (int)((spec->n + nzc - 1) / nzc);
            if (c >= 4 && std::find(z.begin(), z.end(), c) == z.end()) z.push_back(c);
        }
        if (z.empty()) z.push_back(spec->n);
        return z;
    };
    const TileChoice before = ctx->tuning.choose(spec->precision, spec->ndim, spec->n, 1);
    const bool had_timing = ctx->timing;
    const int64_t l0 = ctx->t_launches;
    const double m0 = ctx->t_ms, c0 = ctx->t_cells;
    TileChoice best = before;
    double best_ms = INFINITY;
    int tried = 0;
    ofm_qoi q;
    for (int i = 0; i < nt && rc == OFM_OK; ++i)
        for (int z : zchunks(tiles[i][0], tiles[i][1])) {
            ctx->tuning.set(spec->precision, spec->ndim, spec->n, TileChoice{ tiles[i][0], tiles[i][1], z, 2 });
            ctx->timing = true;
            ctx->t_launches = 0;
            ctx->t_ms = 0.0;
            ctx->t_cells = 0.0;
            rc = ofm_step(ctx, spec, st, steps, &q, nullptr, stream);
            if (rc == OFM_OK && q.status != OFM_SAMPLE_OK)
                rc = fail(ctx, OFM_EINVAL, "ofm_autotune: the state failed while stepping (status %d)", q.status);
            if (rc) break;
            const double ms = ctx->t_ms * 3.0 / (double)std::max<int64_t>(ctx->t_launches, 1);
            if (tried < all_cap)
                all[tried] = ofm_tune_result{ tiles[i][0], tiles[i][1], z, before.graph_steps, ms, 1, 0 };
            ++tried;
            if (ms < best_ms) {
                best_ms = ms;
                best = TileChoice{ tiles[i][0], tiles[i][1], z, before.graph_steps };
            }
        }
    ctx->timing = had_timing;
    ctx->t_launches = l0;
    ctx->t_ms = m0;
    ctx->t_cells = c0;
    ctx->tuning.set(spec->precision, spec->ndim, spec->n, rc == OFM_OK ? best : before);
    if (rc) return rc;
    out->tx = best.tx;
    out->ty = best.ty;
    out->zchunk = best.zchunk;
    out->graph_steps = best.graph_steps;
    out->stage_ms_per_step = best_ms;
    out->candidates = tried;
    out->reserved = 0;
    return OFM_OK;
}

int ofm_kernel_timing(ofm_ctx* ctx, int32_t enable)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    ctx->timing = enable != 0;
    ctx->t_launches = 0;
    ctx->t_ms = 0.0;
    ctx->t_cells = 0.0;
    return OFM_OK;
}

int ofm_kernel_times(const ofm_ctx* ctx, int64_t* launches, double* total_ms, double* cells)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (launches) *launches = ctx->t_launches;
    if (total_ms) *total_ms = ctx->t_ms;
    if (cells) *cells = ctx->t_cells;
    return OFM_OK;
}

int ofm_mlmc_moments(ofm_ctx* ctx, const double* qf, const double* qc, const int32_t* ok, int64_t M, double* out,
                     void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (!qf || !out || M < 0) return fail(ctx, OFM_EINVAL, "ofm_mlmc_moments: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_moments(qf, qc, ok, M, out, (hipStream_t)stream));
    return OFM_OK;
}

int ofm_ofmlmc_coefficients(ofm_ctx* ctx, int32_t L, const double* mom, const double* W, double* alpha,
                            int32_t* flag, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (L < 0 || L > 31 || !mom || !W || !alpha || !flag) return fail(ctx, OFM_EINVAL, "ofm_ofmlmc_coefficients: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_coefficients(L, mom, W, alpha, flag, (hipStream_t)stream));
    return OFM_OK;
}

int ofm_ofmlmc_errors(ofm_ctx* ctx, int32_t L, const double* mom, const double* alpha, double* sig, double* eps2,
                      void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (L < 0 || L > 31 || !mom || !alpha || !sig || !eps2) return fail(ctx, OFM_EINVAL, "ofm_ofmlmc_errors: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_errors(L, mom, alpha, sig, eps2, (hipStream_t)stream));
    return OFM_OK;
}

int ofm_ofmlmc_estimate(ofm_ctx* ctx, int32_t L, const double* mom, const double* alpha, double* E, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (L < 0 || L > 31 || !mom || !alpha || !E) return fail(ctx, OFM_EINVAL, "ofm_ofmlmc_estimate: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_estimate(L, mom, alpha, E, (hipStream_t)stream));
    return OFM_OK;
}

int ofm_ofmlmc_optimal_M(ofm_ctx* ctx, int32_t L, const double* sig, const double* W, const int64_t* have,
                         int32_t mode, double target, int64_t* out, int32_t* flag, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (L < 0 || L > 31 || !sig || !W || !have || !out || !flag || (mode != OFM_MODE_TOLERANCE && mode != OFM_MODE_BUDGET) ||
        !(target > 0.0))
        return fail(ctx, OFM_EINVAL, "ofm_ofmlmc_optimal_M: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_optimal_M(L, sig, W, have, mode, target, out, flag, (hipStream_t)stream));
    return OFM_OK;
}

int ofm_mlmc_merge_moments(ofm_ctx* ctx, int32_t n_terms, const double* a, const double* b, double* out,
                           void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (n_terms < 1 || n_terms > 32 || !a || !b || !out)
        return fail(ctx, OFM_EINVAL, "ofm_mlmc_merge_moments: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_merge(n_terms, a, b, out, (hipStream_t)stream));
    return OFM_OK;
}

int ofm_ofmlmc_fit_indicators(ofm_ctx* ctx, int32_t L, int32_t first, int32_t m_floor, double* mom, double* v_hat,
                              int32_t* flag, void* stream)
{
    if (!ctx) return fail(nullptr, OFM_EINVAL, "null context");
    if (L < 1 || L > 31 || first < 0 || first > L || m_floor < 0 || !mom || !v_hat || !flag)
        return fail(ctx, OFM_EINVAL, "ofm_ofmlmc_fit_indicators: bad arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_fit(L, first, m_floor, mom, v_hat, flag, (hipStream_t)stream));
    return OFM_OK;
}

}  // extern "C"
