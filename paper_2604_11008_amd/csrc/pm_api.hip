// pm_api.hip -- host side of the C ABI declared in include/pm.h: argument
// checks, workspace layout, launch configuration, HIP-graph capture of the
// fused step, kernel timing and the launch-shape autotuner.
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

#include "pm_internal.h"

namespace {

thread_local std::string g_err;

pm_status arg_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return PM_ERR_ARG;
}

pm_status hip_error(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return PM_ERR_HIP;
}

#define PM_HIP(call, what)                       \
    do {                                         \
        hipError_t e_ = (call);                  \
        if (e_ != hipSuccess)                    \
            return hip_error(e_, what);          \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// pm_field_interleave: one node per thread, the three components read from
// their arrays, converted to the output type (double to float rounds to
// nearest) and written next to each other (the node's 3 values are one run
// of the output; a wave's stores cover consecutive runs).
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_interleave(const Ti *__restrict__ u0,
                                                    const Ti *__restrict__ u1,
                                                    const Ti *__restrict__ u2,
                                                    To *__restrict__ out, int64_t nodes)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nodes;
         i += (int64_t)gridDim.x * 256) {
        const To a = (To)u0[i], b = (To)u1[i], c = (To)u2[i];
        out[3 * i] = a;
        out[3 * i + 1] = b;
        out[3 * i + 2] = c;
    }
}

struct WsLayout {
    size_t hdr, tile_start, stay, migtot, stg_start, lb, slot, stg, total;
    int64_t max_tiles, stg_extent;
};

// Device workspace: header words, per-segment tables, one look-back word per
// tile, the plain path's stayer slots (slot = false: none, for a workspace
// that serves the fused step only), and the staging area of the leavers
// (one record per send-buffer slot, 8-byte fields, plus a direction byte).
WsLayout ws_layout(int64_t pool_extent, int64_t send_extent, int32_t nsub, bool slot = true)
{
    WsLayout L{};
    size_t o = 0;
    const size_t ns = (size_t)std::max(nsub, 1);
    L.hdr = o;
    o += align256(pm::kHdrWords * sizeof(uint32_t));
    L.tile_start = o;
    o += align256((PM_MAX_NSUB + 1) * sizeof(int64_t));
    L.stay = o;
    o += align256(ns * sizeof(int64_t));
    L.migtot = o;
    o += align256(ns * sizeof(int64_t));
    L.stg_start = o;
    o += align256((PM_MAX_NSUB + 1) * sizeof(int64_t));
    L.max_tiles = pool_extent / pm::kMinTile + nsub + 2;
    L.lb = o;
    o += align256((size_t)L.max_tiles * sizeof(uint64_t));
    L.slot = o;
    if (slot)
        o += align256((size_t)std::max<int64_t>(pool_extent, 1) * sizeof(uint32_t));
    // every segment's staging area is rounded up to a multiple of 16 records
    L.stg_extent = send_extent + 16 * (int64_t)ns + 16;
    L.stg = o;
    // x, v, tau, id, and the mid-step fields xs, vs, a of per-stage migration
    o += 17 * align256((size_t)L.stg_extent * 8) + align256((size_t)L.stg_extent);
    L.total = o;
    return L;
}

// Device pointers of a workspace at w laid out by L, and its extents.
void bind_ws(pm::DWS &ws, char *w, const WsLayout &L, int64_t pool_extent,
             int64_t send_extent, bool slot)
{
    ws.hdr = (uint32_t *)(w + L.hdr);
    ws.tile_start = (int64_t *)(w + L.tile_start);
    ws.stay = (int64_t *)(w + L.stay);
    ws.migtot = (int64_t *)(w + L.migtot);
    ws.stg_start = (int64_t *)(w + L.stg_start);
    ws.lb = (uint64_t *)(w + L.lb);
    ws.slot = slot ? (uint32_t *)(w + L.slot) : nullptr;
    const size_t fs = align256((size_t)L.stg_extent * 8);
    char *g = w + L.stg;
    for (int c = 0; c < 3; ++c) {
        ws.stg_x[c] = (double *)(g + c * fs);
        ws.stg_v[c] = (double *)(g + (3 + c) * fs);
    }
    ws.stg_tau = (double *)(g + 6 * fs);
    ws.stg_id = (uint64_t *)(g + 7 * fs);
    for (int c = 0; c < 3; ++c) {
        ws.stg_xs[c] = (double *)(g + (8 + c) * fs);
        ws.stg_vs[c] = (double *)(g + (11 + c) * fs);
        ws.stg_a[c] = (double *)(g + (14 + c) * fs);
    }
    ws.stg_d = (uint8_t *)(g + 17 * fs);
    ws.max_tiles = L.max_tiles;
    ws.pool_extent = pool_extent;
    ws.send_extent = send_extent;
    ws.stg_extent = L.stg_extent;
}

struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraphExec_t exec;
};

}  // namespace

struct pm_ctx {
    int device = 0;
    int cus = 0;
    pm::DWS ws{};
    int32_t nsub_max = 0;
    pm::Shape shape{256, 4};
    bool shape_auto = true;         // no pm_set_tuning / pm_autotune yet
    pm::Shape last_shape{256, 4};   // the shape of the last launch
    int blocks_per_cu = 0;
    int xcd_block = 0;              // pm_tuning.xcd_block
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry> graphs;
    int32_t tmax = 0;
    int32_t tcount = 0;
    std::vector<hipEvent_t> events;
};

namespace {

// ---------------------------------------------------------------------------
// argument conversion
// ---------------------------------------------------------------------------

pm_status conv_field(const pm_field *f, pm::DField &d, bool &mixed)
{
    if (!f)
        return arg_error("field is NULL");
    if (f->halo != 0 && f->halo != 1)
        return arg_error("field.halo must be 0 or 1");
    if (f->dtype != PM_F64 && f->dtype != PM_F32)
        return arg_error("field.dtype must be PM_F64 or PM_F32");
    if (f->stagger != 0 && f->stagger != 1)
        return arg_error("field.stagger must be 0 or 1");
    if (f->layout != PM_LAYOUT_SPLIT && f->layout != PM_LAYOUT_INTERLEAVED)
        return arg_error("field.layout must be PM_LAYOUT_SPLIT or PM_LAYOUT_INTERLEAVED");
    const bool ilv = f->layout == PM_LAYOUT_INTERLEAVED;
    if (ilv && f->stagger)
        return arg_error("an interleaved field must be collocated (stagger 0)");
    if (ilv && (f->u[1] || f->u[2]))
        return arg_error("field.u[1] and field.u[2] must be NULL for an interleaved field");
    for (int a = 0; a < 3; ++a) {
        if (f->n[a] < 2 || f->n[a] > (1 << 20))
            return arg_error("field.n[%d] = %d out of range", a, f->n[a]);
        if (!(f->L[a] > 0.0) || !std::isfinite(f->L[a]))
            return arg_error("field.L[%d] must be positive and finite", a);
        if (!f->u[a] && (a == 0 || !ilv))
            return arg_error("field.u[%d] is NULL", a);
    }
    const int64_t sx = f->n[0] + 2 * f->halo, sy = f->n[1] + 2 * f->halo,
                  sz = f->n[2] + 2 * f->halo;
    if (sx * sy * sz > (int64_t)1 << 40)
        return arg_error("field too large");
    for (int a = 0; a < 3; ++a) {
        d.u[a] = f->u[a];
        d.n[a] = f->n[a];
        d.r[a] = (double)f->n[a] / f->L[a];
    }
    d.halo = f->halo;
    d.stagger = f->stagger;
    d.layout = f->layout;
    d.sx = sx;
    d.sxy = sx * sy;
    mixed = f->dtype == PM_F32;
    return PM_OK;
}

pm_status conv_decomp(const pm_decomp *dc, const double *Lfield, pm::DDecomp &d)
{
    if (!dc)
        return arg_error("decomp is NULL");
    int64_t nsub = 1;
    for (int a = 0; a < 3; ++a) {
        const int P = dc->p[a];
        if (P < 1 || P > PM_MAX_P)
            return arg_error("decomp.p[%d] = %d not in 1..%d", a, P, PM_MAX_P);
        if (!dc->bounds[a])
            return arg_error("decomp.bounds[%d] is NULL", a);
        const double *b = dc->bounds[a];
        if (b[0] != 0.0)
            return arg_error("decomp.bounds[%d][0] must be 0", a);
        for (int k = 0; k < P; ++k)
            if (!(b[k] < b[k + 1]) || !std::isfinite(b[k + 1]))
                return arg_error("decomp.bounds[%d] must increase strictly", a);
        if (Lfield && b[P] != Lfield[a])
            return arg_error("decomp.bounds[%d][%d] must equal field.L[%d]", a, P, a);
        d.p[a] = P;
        for (int k = 0; k <= PM_MAX_P; ++k)
            d.b[a][k] = k <= P ? b[k] : b[P];
        d.L[a] = b[P];
        d.predL[a] = std::nextafter(b[P], 0.0);
        nsub *= P;
    }
    if (nsub > PM_MAX_NSUB)
        return arg_error("%lld subdomains exceed %d", (long long)nsub, PM_MAX_NSUB);
    d.nsub = (int32_t)nsub;
    return PM_OK;
}

pm_status conv_pool(const pm_particles *p, const char *name, bool mixed, pm::DPool &d)
{
    if (!p)
        return arg_error("%s is NULL", name);
    if (p->vdtype != (mixed ? PM_F32 : PM_F64))
        return arg_error("%s.vdtype must be %s with a %s field", name,
                         mixed ? "PM_F32" : "PM_F64", mixed ? "PM_F32" : "PM_F64");
    if (!p->base || !p->cap || !p->count || !p->tau || !p->id)
        return arg_error("%s has a NULL array", name);
    for (int a = 0; a < 3; ++a)
        if (!p->x[a] || !p->v[a])
            return arg_error("%s has a NULL array", name);
    d.base = p->base;
    d.cap = p->cap;
    d.count = p->count;
    for (int a = 0; a < 3; ++a) {
        d.x[a] = p->x[a];
        d.v[a] = p->v[a];
    }
    d.tau = p->tau;
    d.id = p->id;
    return PM_OK;
}

pm_status conv_send(const pm_sendbufs *s, pm::DPool &d)
{
    if (!s)
        return arg_error("send is NULL");
    if (!s->base || !s->cap || !s->count || !s->tau || !s->id)
        return arg_error("send has a NULL array");
    for (int a = 0; a < 3; ++a)
        if (!s->x[a] || !s->v[a])
            return arg_error("send has a NULL array");
    d.base = s->base;
    d.cap = s->cap;
    d.count = s->count;
    for (int a = 0; a < 3; ++a) {
        d.x[a] = s->x[a];
        d.v[a] = s->v[a];
    }
    d.tau = s->tau;
    d.id = s->id;
    return PM_OK;
}

// The mid-step pools of per-stage migration: the plain fields plus xs, vs, a.
template <typename P>
pm_status conv_stage(const P *p, const char *name, pm::DPool &d)
{
    if (!p)
        return arg_error("%s is NULL", name);
    if (!p->base || !p->cap || !p->count || !p->tau || !p->id)
        return arg_error("%s has a NULL array", name);
    for (int a = 0; a < 3; ++a)
        if (!p->x[a] || !p->v[a] || !p->xs[a] || !p->vs[a] || !p->a[a])
            return arg_error("%s has a NULL array", name);
    d.base = p->base;
    d.cap = p->cap;
    d.count = p->count;
    for (int a = 0; a < 3; ++a) {
        d.x[a] = p->x[a];
        d.v[a] = p->v[a];
        d.xs[a] = p->xs[a];
        d.vs[a] = p->vs[a];
        d.a[a] = p->a[a];
    }
    d.tau = p->tau;
    d.id = p->id;
    return PM_OK;
}

pm_status conv_params(const pm_params *pr, pm::KArgs &k)
{
    if (!pr)
        return arg_error("params is NULL");
    if (!std::isfinite(pr->dt) || !std::isfinite(pr->g[0]) || !std::isfinite(pr->g[1]) ||
        !std::isfinite(pr->g[2]))
        return arg_error("params must be finite");
    if (pr->drag != PM_DRAG_STOKES && pr->drag != PM_DRAG_NONLINEAR)
        return arg_error("params.drag = %d is not a pm_drag", pr->drag);
    if (pr->drag == PM_DRAG_NONLINEAR &&
        !(std::isfinite(pr->nu) && pr->nu > 0 && std::isfinite(pr->density_ratio) &&
          pr->density_ratio > 0))
        return arg_error("nonlinear drag needs positive finite nu and density_ratio");
    k.drag = pr->drag;
    // Re_p = 2 r |V - U| / nu with r^2 = 9 nu tau / (2 rho_p/rho), i.e.
    // Re_p = sqrt(18 tau / (rho_p/rho nu)) |V - U|
    k.kappa = pr->drag == PM_DRAG_NONLINEAR ? std::sqrt(18.0 / (pr->density_ratio * pr->nu)) : 0.0;
    k.kappaf = (float)k.kappa;
    k.dt = pr->dt;
    k.half_dt = 0.5 * pr->dt;
    k.dtf = (float)pr->dt;
    k.half_dtf = (float)(0.5 * pr->dt);
    for (int c = 0; c < 3; ++c) {
        k.g[c] = pr->g[c];
        k.gf[c] = (float)pr->g[c];
    }
    return PM_OK;
}

pm_status check_range(pm_ctx *ctx, int32_t nsub, int32_t first, int32_t count)
{
    if (nsub < 1 || nsub > ctx->nsub_max)
        return arg_error("nsub = %d not in 1..%d (context limit)", nsub, ctx->nsub_max);
    if (first < 0 || count < 0 || (int64_t)first + count > nsub)
        return arg_error("segment range [%d, %d) outside 0..%d", first, first + count, nsub);
    return PM_OK;
}

// Records per thread of the default shape: at most max_items, halved while
// the context's pool extent would give fewer than two tiles per compute unit
// (a pool of 65,536 particles steps in 0.045 ms at 256 x 1 against 0.059 ms
// at 256 x 4: its 64 large tiles leave most of the chip idle).
int auto_items(const pm_ctx *ctx, int max_items)
{
    int items = max_items;
    while (items > 1 && ctx->ws.pool_extent / (256 * (int64_t)items) < 2 * (int64_t)ctx->cus)
        items /= 2;
    return items;
}

// Launch shape of a call: the tuned one, else a measured default — 256
// threads x 4 records, except the mixed periodic kernels on an interleaved
// field, 2-3% faster so on the 1024^3 workload (x 2 records); fewer records
// per thread for small pools (auto_items).
pm::Shape shape_for(pm_ctx *ctx, bool mixed, bool halo, bool ilv = false)
{
    pm::Shape sh = ctx->shape;
    const bool two = !halo && mixed && ilv;
    if (ctx->shape_auto)
        sh = pm::Shape{256, auto_items(ctx, two ? 2 : 4)};
    ctx->last_shape = sh;
    return sh;
}

int persistent_grid(pm_ctx *ctx, pm::Shape sh, bool mixed, bool halo, bool nonlinear,
                    int arr)
{
    // An explicit figure may exceed the runtime's occupancy estimate: workgroups
    // that do not fit start as others retire.  Tiles are claimed by ticket when
    // a workgroup runs, so a running workgroup only waits on tiles that a
    // running workgroup holds or that its ticket group will hand to one: each
    // group has running workgroups, since workgroups start in index order.
    const int per = ctx->blocks_per_cu > 0 ? ctx->blocks_per_cu
                                           : pm::step_occupancy(sh, mixed, halo, nonlinear,
                                                                arr);
    return std::max(1, ctx->cus * per);
}

// Ticket groups of a persistent launch of `grid` workgroups: one counter, or
// one per XCD handing out blocks of xcd_block tiles.
void set_groups(const pm_ctx *ctx, pm::KArgs &k, int grid)
{
    const bool grouped = ctx->xcd_block > 0 && grid >= pm::kMaxGroups;
    k.xg = grouped ? pm::kMaxGroups : 1;
    k.xb = grouped ? ctx->xcd_block : 1;
}

int append_cpt(int32_t count) { return std::max(1, 2048 / std::max(1, count)); }

// Queue the fused step (prep, fused kernel, exchange) on `st`.
pm_status queue_step(pm_ctx *ctx, pm::KArgs &k, bool mixed, hipStream_t st, bool timed)
{
    const pm::Shape sh = shape_for(ctx, mixed, k.f.halo != 0, k.f.layout != 0);
    k.tile = sh.wg * sh.items;
    k.cpt = append_cpt(k.sub_count);
    PM_HIP(pm::launch_prep(k,
                           pm::kPrepTiles | pm::kPrepStaging | pm::kPrepZeroLb |
                               pm::kPrepZeroCounts | pm::kPrepCheckIn | pm::kPrepCheckOut |
                               pm::kPrepCheckSend,
                           st),
           "prep launch");
    if (timed)
        PM_HIP(hipEventRecord(ctx->events[2 * ctx->tcount], st), "event record");
    const int grid =
        persistent_grid(ctx, sh, mixed, k.f.halo != 0, k.drag != 0, pm::field_arr(k.f));
    set_groups(ctx, k, grid);
    PM_HIP(pm::launch_step(k, sh, mixed, grid, st), "fused step launch");
    if (timed) {
        PM_HIP(hipEventRecord(ctx->events[2 * ctx->tcount + 1], st), "event record");
        ctx->tcount++;
    }
    PM_HIP(pm::launch_route(k, mixed, true, st), "route launch");
    return PM_OK;
}

void base_args(pm_ctx *ctx, pm::KArgs &k)
{
    std::memset(&k, 0, sizeof k);
    k.ws = ctx->ws;
}

// Launch the graph captured for `key` on `st`, capturing it first (from what
// `queue` enqueues on the context's capture stream) if this key is new.  At
// most 16 graphs are kept, the oldest dropped first.
template <typename Queue>
pm_status run_captured(pm_ctx *ctx, const std::vector<unsigned char> &key,
                              hipStream_t st, Queue queue)
{
    for (auto &g : ctx->graphs)
        if (g.key == key) {
            PM_HIP(hipGraphLaunch(g.exec, st), "graph launch");
            return PM_OK;
        }
    if (!ctx->cap_stream)
        PM_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "stream create");
    PM_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal),
           "begin capture");
    const pm_status qs = queue(ctx->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (qs) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return qs;
    }
    if (ce != hipSuccess)
        return hip_error(ce, "end capture");
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess)
        return hip_error(ie, "graph instantiate");
    if (ctx->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back({key, exec});
    PM_HIP(hipGraphLaunch(exec, st), "graph launch");
    return PM_OK;
}

// Graph key: a tag, the launch arguments, the shape and the tuning that
// decides the grid and the tile order.
std::vector<unsigned char> graph_key(const pm_ctx *ctx, char tag,
                                            const pm::KArgs *ks, int nk, pm::Shape sh)
{
    std::vector<unsigned char> key(1 + nk * sizeof(pm::KArgs) + sizeof sh + 2 * sizeof(int));
    unsigned char *p = key.data();
    *p++ = (unsigned char)tag;
    for (int i = 0; i < nk; ++i, p += sizeof(pm::KArgs))
        std::memcpy(p, &ks[i], sizeof(pm::KArgs));
    std::memcpy(p, &sh, sizeof sh);
    p += sizeof sh;
    std::memcpy(p, &ctx->blocks_per_cu, sizeof(int));
    p += sizeof(int);
    std::memcpy(p, &ctx->xcd_block, sizeof(int));
    return key;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char *pm_last_error(void) { return g_err.c_str(); }

// Extents a context accepts (records).
constexpr int64_t kMaxExtent = (int64_t)1 << 34;

size_t pm_workspace_bytes(int64_t pool_extent, int64_t send_extent, int32_t nsub)
{
    if (pool_extent < 0 || pool_extent > kMaxExtent || send_extent < 0 ||
        send_extent > kMaxExtent || nsub < 1 || nsub > PM_MAX_NSUB)
        return 0;
    return ws_layout(pool_extent, send_extent, nsub).total;
}

pm_status pm_create(pm_ctx **out, void *workspace, size_t ws_bytes, int64_t pool_extent,
                    int64_t send_extent, int32_t nsub)
{
    if (!out)
        return arg_error("ctx pointer is NULL");
    *out = nullptr;
    if (nsub < 1 || nsub > PM_MAX_NSUB)
        return arg_error("nsub = %d not in 1..%d", nsub, PM_MAX_NSUB);
    if (pool_extent < 0 || pool_extent > kMaxExtent || send_extent < 0 ||
        send_extent > kMaxExtent)
        return arg_error("pool or send extent out of range (0..2^34)");
    const WsLayout L = ws_layout(pool_extent, send_extent, nsub);
    if (!workspace || ws_bytes < L.total)
        return arg_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                         L.total);
    if (((uintptr_t)workspace & 255u) != 0)
        return arg_error("workspace must be 256-byte aligned");
    pm_ctx *ctx = new pm_ctx();
    hipError_t e = hipGetDevice(&ctx->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess) {
        delete ctx;
        return hip_error(e, "device query");
    }
    bind_ws(ctx->ws, (char *)workspace, L, pool_extent, send_extent, true);
    ctx->nsub_max = nsub;
    // start from a clean header, tables and look-back state
    e = hipMemset(workspace, 0, L.slot);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete ctx;
        return hip_error(e, "workspace clear");
    }
    *out = ctx;
    return PM_OK;
}

pm_status pm_destroy(pm_ctx *ctx)
{
    if (!ctx)
        return PM_OK;
    for (auto &g : ctx->graphs)
        (void)hipGraphExecDestroy(g.exec);
    for (auto e : ctx->events)
        (void)hipEventDestroy(e);
    if (ctx->cap_stream)
        (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return PM_OK;
}

pm_status pm_interp(pm_ctx *ctx, const pm_field *field, int64_t n, const double *x,
                    const double *y, const double *z, void *ux, void *uy, void *uz,
                    void *stream)
{
    if (!ctx)
        return arg_error("ctx is NULL");
    pm::KArgs k;
    base_args(ctx, k);
    bool mixed = false;
    pm_status s = conv_field(field, k.f, mixed);
    if (s)
        return s;
    if (n < 0)
        return arg_error("n < 0");
    if (n == 0)
        return PM_OK;
    if (!x || !y || !z || !ux || !uy || !uz)
        return arg_error("NULL array");
    PM_HIP(pm::launch_interp(k, mixed, n, x, y, z, ux, uy, uz, (hipStream_t)stream),
           "interp launch");
    return PM_OK;
}

pm_status pm_field_interleave(const pm_field *field, int32_t out_dtype, void *out,
                              void *stream)
{
    pm::DField d;
    bool mixed = false;
    pm_status s = conv_field(field, d, mixed);
    if (s)
        return s;
    if (field->layout != PM_LAYOUT_SPLIT || field->stagger)
        return arg_error("pm_field_interleave takes a collocated field stored as one array "
                         "per component");
    if (out_dtype != PM_F64 && out_dtype != PM_F32)
        return arg_error("out_dtype must be PM_F64 or PM_F32");
    if (mixed && out_dtype == PM_F64)
        return arg_error("pm_field_interleave does not widen a PM_F32 field");
    if (!out)
        return arg_error("out is NULL");
    const int64_t nodes = d.sxy * (field->n[2] + 2 * field->halo);
    const size_t ein = mixed ? sizeof(float) : sizeof(double);
    const size_t eout = out_dtype == PM_F32 ? sizeof(float) : sizeof(double);
    const uintptr_t o0 = (uintptr_t)out, o1 = o0 + 3 * (size_t)nodes * eout;
    for (int c = 0; c < 3; ++c) {
        const uintptr_t a0 = (uintptr_t)field->u[c], a1 = a0 + (size_t)nodes * ein;
        if (a0 < o1 && o0 < a1)
            return arg_error("out overlaps field.u[%d]", c);
    }
    const int grid = (int)std::min<int64_t>(65536, std::max<int64_t>(1, (nodes + 255) / 256));
    hipStream_t st = (hipStream_t)stream;
    if (mixed)
        hipLaunchKernelGGL((k_interleave<float, float>), dim3(grid), dim3(256), 0, st,
                           (const float *)field->u[0], (const float *)field->u[1],
                           (const float *)field->u[2], (float *)out, nodes);
    else if (out_dtype == PM_F32)
        hipLaunchKernelGGL((k_interleave<double, float>), dim3(grid), dim3(256), 0, st,
                           (const double *)field->u[0], (const double *)field->u[1],
                           (const double *)field->u[2], (float *)out, nodes);
    else
        hipLaunchKernelGGL((k_interleave<double, double>), dim3(grid), dim3(256), 0, st,
                           (const double *)field->u[0], (const double *)field->u[1],
                           (const double *)field->u[2], (double *)out, nodes);
    PM_HIP(hipGetLastError(), "interleave launch");
    return PM_OK;
}

pm_status pm_interp_advance(pm_ctx *ctx, const pm_field *field, pm_particles *inout,
                            const pm_params *params, int32_t sub_first, int32_t sub_count,
                            void *stream)
{
    if (!ctx)
        return arg_error("ctx is NULL");
    pm::KArgs k;
    base_args(ctx, k);
    bool mixed = false;
    pm_status s = conv_field(field, k.f, mixed);
    if (!s)
        s = conv_pool(inout, "inout", mixed, k.in);
    if (!s)
        s = conv_params(params, k);
    if (!s)
        s = check_range(ctx, inout->nsub, sub_first, sub_count);
    if (s)
        return s;
    if (sub_count == 0)
        return PM_OK;
    hipStream_t st = (hipStream_t)stream;
    k.sub_first = sub_first;
    k.sub_count = sub_count;
    const pm::Shape sh = shape_for(ctx, mixed, k.f.halo != 0, k.f.layout != 0);
    k.tile = sh.wg * sh.items;
    PM_HIP(pm::launch_prep(k, pm::kPrepTiles | pm::kPrepCheckIn, st), "prep launch");
    const int grid =
        persistent_grid(ctx, sh, mixed, k.f.halo != 0, k.drag != 0, pm::field_arr(k.f));
    set_groups(ctx, k, grid);
    PM_HIP(pm::launch_advance(k, sh, mixed, grid, st),
           "advance launch");
    return PM_OK;
}

pm_status pm_classify_scan_pack(pm_ctx *ctx, const pm_decomp *decomp, const pm_particles *in,
                                pm_sendbufs *send, int32_t sub_first, int32_t sub_count,
                                void *stream)
{
    if (!ctx)
        return arg_error("ctx is NULL");
    pm::KArgs k;
    base_args(ctx, k);
    pm_status s = conv_decomp(decomp, nullptr, k.dc);
    if (s)
        return s;
    if (!in)
        return arg_error("in is NULL");
    const bool mixed = in->vdtype == PM_F32;
    s = conv_pool(in, "in", mixed, k.in);
    if (!s)
        s = conv_send(send, k.send);
    if (!s)
        s = check_range(ctx, in->nsub, sub_first, sub_count);
    if (!s && in->nsub != k.dc.nsub)
        s = arg_error("in.nsub = %d but the decomposition has %d subdomains", in->nsub,
                      k.dc.nsub);
    if (s)
        return s;
    if (sub_count == 0)
        return PM_OK;
    hipStream_t st = (hipStream_t)stream;
    k.sub_first = sub_first;
    k.sub_count = sub_count;
    const pm::Shape sh = shape_for(ctx, mixed, false);
    k.tile = sh.wg * sh.items;
    PM_HIP(pm::launch_prep(k,
                           pm::kPrepTiles | pm::kPrepStaging | pm::kPrepZeroLb |
                               pm::kPrepZeroCounts | pm::kPrepCheckIn | pm::kPrepCheckSend,
                           st),
           "prep launch");
    const int grid = persistent_grid(ctx, sh, mixed, false, false, pm::kFieldSplit);
    set_groups(ctx, k, grid);
    PM_HIP(pm::launch_classify(k, sh, mixed, grid, st),
           "classify launch");
    PM_HIP(pm::launch_route(k, mixed, false, st), "route launch");
    return PM_OK;
}

pm_status pm_compact_append(pm_ctx *ctx, const pm_decomp *decomp, const pm_particles *in,
                            const pm_sendbufs *send, pm_particles *out, int32_t sub_first,
                            int32_t sub_count, void *stream)
{
    if (!ctx)
        return arg_error("ctx is NULL");
    pm::KArgs k;
    base_args(ctx, k);
    pm_status s = conv_decomp(decomp, nullptr, k.dc);
    if (s)
        return s;
    if (!in)
        return arg_error("in is NULL");
    const bool mixed = in->vdtype == PM_F32;
    s = conv_pool(in, "in", mixed, k.in);
    if (!s)
        s = conv_pool(out, "out", mixed, k.out);
    if (!s)
        s = conv_send(send, k.send);
    if (!s)
        s = check_range(ctx, in->nsub, sub_first, sub_count);
    if (!s && (in->nsub != k.dc.nsub || out->nsub != k.dc.nsub))
        s = arg_error("pool nsub does not match the decomposition (%d)", k.dc.nsub);
    if (s)
        return s;
    if (sub_count == 0)
        return PM_OK;
    hipStream_t st = (hipStream_t)stream;
    k.sub_first = sub_first;
    k.sub_count = sub_count;
    const pm::Shape sh = shape_for(ctx, mixed, false);
    k.tile = sh.wg * sh.items;
    k.cpt = append_cpt(sub_count);
    PM_HIP(pm::launch_prep(k, pm::kPrepTiles | pm::kPrepCheckIn | pm::kPrepCheckOut |
                                  pm::kPrepCheckSend,
                           st),
           "prep launch");
    const int cgrid = persistent_grid(ctx, sh, mixed, false, false, pm::kFieldSplit);
    PM_HIP(pm::launch_compact(k, sh, mixed, cgrid, st), "compact launch");
    const int grid = std::min(4096, sub_count * k.cpt);
    PM_HIP(pm::launch_append(k, mixed, std::max(1, grid), st), "append launch");
    return PM_OK;
}

static pm_status step_args(pm_ctx *ctx, const pm_field *field, const pm_decomp *decomp,
                           const pm_particles *in, pm_particles *out, pm_sendbufs *send,
                           const pm_params *params, pm::KArgs &k, bool &mixed)
{
    if (!ctx)
        return arg_error("ctx is NULL");
    base_args(ctx, k);
    pm_status s = conv_field(field, k.f, mixed);
    if (!s)
        s = conv_decomp(decomp, field->L, k.dc);
    if (!s)
        s = conv_pool(in, "in", mixed, k.in);
    if (!s)
        s = conv_pool(out, "out", mixed, k.out);
    if (!s)
        s = conv_send(send, k.send);
    if (!s)
        s = conv_params(params, k);
    if (!s && (in->nsub != k.dc.nsub || out->nsub != k.dc.nsub))
        s = arg_error("pool nsub does not match the decomposition (%d)", k.dc.nsub);
    if (!s)
        s = check_range(ctx, in->nsub, 0, in->nsub);
    if (s)
        return s;
    if (in->x[0] == out->x[0])
        return arg_error("pm_step is out of place: in and out must differ");
    k.sub_first = 0;
    k.sub_count = in->nsub;
    return PM_OK;
}

// One stage of per-stage migration: prep, the stage's fused kernel, and the
// exchange (mid-step records after stage 1, plain ones after stage 2).
static pm_status queue_stage(pm_ctx *ctx, pm::KArgs &k, bool mixed, int stage, pm::Shape sh,
                             hipStream_t st, bool timed)
{
    k.tile = sh.wg * sh.items;
    k.cpt = append_cpt(k.sub_count);
    PM_HIP(pm::launch_prep(k,
                           pm::kPrepTiles | pm::kPrepStaging | pm::kPrepZeroLb |
                               pm::kPrepZeroCounts | pm::kPrepCheckIn | pm::kPrepCheckOut |
                               pm::kPrepCheckSend,
                           st),
           "prep launch");
    const int per = ctx->blocks_per_cu > 0
                        ? ctx->blocks_per_cu
                        : pm::stage_occupancy(sh, mixed, k.f.halo != 0, k.drag != 0, stage,
                                              k.f.layout != 0);
    const int grid = std::max(1, ctx->cus * per);
    set_groups(ctx, k, grid);
    if (timed)
        PM_HIP(hipEventRecord(ctx->events[2 * ctx->tcount], st), "event record");
    PM_HIP(pm::launch_stage(k, sh, mixed, stage, grid, st), "stage launch");
    if (timed) {
        PM_HIP(hipEventRecord(ctx->events[2 * ctx->tcount + 1], st), "event record");
        ctx->tcount++;
    }
    PM_HIP(pm::launch_route(k, mixed, true, st, stage == 1), "route launch");
    return PM_OK;
}

pm_status pm_step_staged(pm_ctx *ctx, const pm_field *field, const pm_decomp *decomp,
                         const pm_particles *in, pm_stage_particles *mid,
                         pm_stage_sendbufs *mid_send, pm_particles *out, pm_sendbufs *send,
                         const pm_params *params, void *stream)
{
    pm::KArgs k;
    bool mixed = false;
    pm_status s = step_args(ctx, field, decomp, in, out, send, params, k, mixed);
    if (s)
        return s;
    if (field->stagger)
        return arg_error("per-stage migration takes a collocated field");
    pm::DPool dmid, dms;
    std::memset(&dmid, 0, sizeof dmid);  // the bytes are part of a graph key
    std::memset(&dms, 0, sizeof dms);
    s = conv_stage(mid, "mid", dmid);
    if (!s)
        s = conv_stage(mid_send, "mid_send", dms);
    if (s)
        return s;
    if (mid->vdtype != (mixed ? PM_F32 : PM_F64))
        return arg_error("mid.vdtype must match the field");
    if (mid->nsub != in->nsub)
        return arg_error("mid.nsub must equal in.nsub");
    if (mid->x[0] == in->x[0] || mid->x[0] == out->x[0])
        return arg_error("mid must differ from in and out");
    const pm::Shape sh = ctx->shape_auto ? pm::Shape{256, auto_items(ctx, 2)} : ctx->shape;
    if (!pm::stage_shape_supported(sh))
        return arg_error("launch shape wg=%d items=%d is not built for per-stage migration",
                         sh.wg, sh.items);
    ctx->last_shape = sh;
    hipStream_t st = (hipStream_t)stream;
    pm::KArgs ks[2] = {k, k};
    ks[0].out = dmid;  // stage 1: in -> mid, leavers through mid_send
    ks[0].send = dms;
    ks[1].in = dmid;   // stage 2: mid -> out, leavers through send
    auto queue = [&](hipStream_t qs, bool timed) {
        pm::KArgs k1 = ks[0], k2 = ks[1];
        pm_status r = queue_stage(ctx, k1, mixed, 1, sh, qs, timed);
        return r ? r : queue_stage(ctx, k2, mixed, 2, sh, qs, timed);
    };
    if (!ctx->use_graph)
        return queue(st, ctx->tmax > 0 && ctx->tcount + 1 < ctx->tmax);
    // graph path: one captured graph (both stages) per argument set and shape
    return run_captured(ctx, graph_key(ctx, 'S', ks, 2, sh), st,
                        [&](hipStream_t cs) { return queue(cs, false); });
}

pm_status pm_step(pm_ctx *ctx, const pm_field *field, const pm_decomp *decomp,
                  const pm_particles *in, pm_particles *out, pm_sendbufs *send,
                  const pm_params *params, void *stream)
{
    pm::KArgs k;
    bool mixed = false;
    pm_status s = step_args(ctx, field, decomp, in, out, send, params, k, mixed);
    if (s)
        return s;
    hipStream_t st = (hipStream_t)stream;
    if (!ctx->use_graph) {
        const bool timed = ctx->tmax > 0 && ctx->tcount < ctx->tmax;
        return queue_step(ctx, k, mixed, st, timed);
    }
    // graph path: one captured graph per distinct argument set and shape
    const pm::Shape sh = shape_for(ctx, mixed, k.f.halo != 0, k.f.layout != 0);
    k.tile = sh.wg * sh.items;
    k.cpt = append_cpt(k.sub_count);
    return run_captured(ctx, graph_key(ctx, 'P', &k, 1, sh), st, [&](hipStream_t cs) {
        pm::KArgs kk = k;
        return queue_step(ctx, kk, mixed, cs, false);
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// pm_step_noalloc: pm_step with its scratch in a fixed device array of the
// library instead of a caller's workspace
// ---------------------------------------------------------------------------

// The scratch of pm_step_noalloc (header words, tile and staging tables,
// look-back words, the leavers' staging area): one copy per device, zero at
// load, shared by every call on that device.  In host code this name is not
// a device address; the address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[PM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocDevices = 64;

struct NoAllocDevice {
    bool ready;
    int cus;
    char *ptr;  // device address of `scratch` on this device
};

NoAllocDevice g_noalloc[kNoAllocDevices];
std::mutex g_noalloc_mu;

// The current device's scratch address and CU count, looked up once per
// device (with that device current).
pm_status noalloc_device(NoAllocDevice **out)
{
    int dev = 0;
    PM_HIP(hipGetDevice(&dev), "device query");
    if (dev < 0 || dev >= kNoAllocDevices)
        return arg_error("device %d is beyond the %d that pm_step_noalloc serves", dev,
                         kNoAllocDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoAllocDevice &d = g_noalloc[dev];
    if (!d.ready) {
        void *p = nullptr;
        PM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
        if (!p || ((uintptr_t)p & 255u) != 0)
            return hip_error(hipErrorInvalidSymbol, "scratch address");
        int cus = 0;
        PM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
               "device query");
        d.cus = cus;
        d.ptr = (char *)p;
        d.ready = true;
    }
    *out = &d;
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status pm_step_noalloc(const pm_field *field, const pm_decomp *decomp,
                          const pm_particles *in, pm_particles *out, pm_sendbufs *send,
                          const pm_params *params, int64_t pool_extent, int64_t send_extent,
                          uint32_t *flags, void *stream)
{
    if (!flags)
        return arg_error("flags is NULL");
    if (!in)
        return arg_error("in is NULL");
    if (in->nsub < 1 || in->nsub > PM_MAX_NSUB)
        return arg_error("nsub = %d not in 1..%d", in->nsub, PM_MAX_NSUB);
    if (pool_extent < 0 || pool_extent > kMaxExtent || send_extent < 0 ||
        send_extent > kMaxExtent)
        return arg_error("pool or send extent out of range (0..2^34)");
    const WsLayout L = ws_layout(pool_extent, send_extent, in->nsub, false);
    if (L.total > PM_NOALLOC_SCRATCH_BYTES)
        return arg_error("pm_step_noalloc: %lld pool records, %lld send records and %d "
                         "subdomains need %zu bytes of scratch, more than its %zu",
                         (long long)pool_extent, (long long)send_extent, in->nsub, L.total,
                         (size_t)PM_NOALLOC_SCRATCH_BYTES);
    NoAllocDevice *d = nullptr;
    pm_status s = noalloc_device(&d);
    if (s)
        return s;
    // host-side settings only (the default launch shape; no graphs, no
    // timing): nothing here allocates
    pm_ctx ctx;
    ctx.cus = d->cus;
    ctx.nsub_max = in->nsub;
    bind_ws(ctx.ws, d->ptr, L, pool_extent, send_extent, false);
    pm::KArgs k;
    bool mixed = false;
    s = step_args(&ctx, field, decomp, in, out, send, params, k, mixed);
    if (s)
        return s;
    hipStream_t st = (hipStream_t)stream;
    // the array keeps the last call's contents: start without its flags
    PM_HIP(pm::launch_flags_move(ctx.ws.hdr, nullptr, st), "flags launch");
    s = queue_step(&ctx, k, mixed, st, false);
    if (s)
        return s;
    PM_HIP(pm::launch_flags_move(ctx.ws.hdr, flags, st), "flags launch");
    return PM_OK;
}

pm_status pm_get_status(pm_ctx *ctx, void *stream, uint32_t *flags)
{
    if (!ctx || !flags)
        return arg_error("NULL argument");
    hipStream_t st = (hipStream_t)stream;
    PM_HIP(hipStreamSynchronize(st), "stream sync");
    uint32_t f = 0;
    PM_HIP(hipMemcpy(&f, ctx->ws.hdr + pm::kHdrFlags, sizeof f, hipMemcpyDeviceToHost),
           "status read");
    const uint32_t zero = 0;
    PM_HIP(hipMemcpy(ctx->ws.hdr + pm::kHdrFlags, &zero, sizeof zero, hipMemcpyHostToDevice),
           "status clear");
    *flags = f;
    return PM_OK;
}

pm_status pm_set_tuning(pm_ctx *ctx, const pm_tuning *t)
{
    if (!ctx || !t)
        return arg_error("NULL argument");
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 32)
        return arg_error("blocks_per_cu out of range");
    if (t->xcd_block < 0 || t->xcd_block > 65536)
        return arg_error("xcd_block out of range");
    ctx->xcd_block = t->xcd_block;
    if (t->wg == 0) {  // back to the per-variant defaults
        ctx->shape_auto = true;
        ctx->blocks_per_cu = t->blocks_per_cu;
        return PM_OK;
    }
    const pm::Shape sh{t->wg, t->items};
    if (!pm::shape_supported(sh))
        return arg_error("launch shape wg=%d items=%d is not built", t->wg, t->items);
    ctx->shape = sh;
    ctx->shape_auto = false;
    ctx->blocks_per_cu = t->blocks_per_cu;
    return PM_OK;
}

pm_status pm_get_tuning(pm_ctx *ctx, pm_tuning *t)
{
    if (!ctx || !t)
        return arg_error("NULL argument");
    const pm::Shape sh = ctx->shape_auto ? ctx->last_shape : ctx->shape;
    t->wg = sh.wg;
    t->items = sh.items;
    t->blocks_per_cu = ctx->blocks_per_cu;
    t->xcd_block = ctx->xcd_block;
    return PM_OK;
}

pm_status pm_set_graph(pm_ctx *ctx, int32_t enable)
{
    if (!ctx)
        return arg_error("ctx is NULL");
    ctx->use_graph = enable != 0;
    return PM_OK;
}

pm_status pm_set_timing(pm_ctx *ctx, int32_t max_records)
{
    if (!ctx)
        return arg_error("ctx is NULL");
    if (max_records < 0 || max_records > (1 << 16))
        return arg_error("max_records out of range");
    for (auto e : ctx->events)
        (void)hipEventDestroy(e);
    ctx->events.clear();
    ctx->tcount = 0;
    ctx->tmax = max_records;
    for (int i = 0; i < 2 * max_records; ++i) {
        hipEvent_t e;
        PM_HIP(hipEventCreate(&e), "event create");
        ctx->events.push_back(e);
    }
    return PM_OK;
}

pm_status pm_kernel_times(pm_ctx *ctx, int32_t *n, double *total_ms, float *ms, int32_t max_ms)
{
    if (!ctx || !n || !total_ms)
        return arg_error("NULL argument");
    double tot = 0.0;
    for (int i = 0; i < ctx->tcount; ++i) {
        PM_HIP(hipEventSynchronize(ctx->events[2 * i + 1]), "event sync");
        float t = 0.f;
        PM_HIP(hipEventElapsedTime(&t, ctx->events[2 * i], ctx->events[2 * i + 1]), "elapsed");
        tot += t;
        if (ms && i < max_ms)
            ms[i] = t;
    }
    *n = ctx->tcount;
    *total_ms = tot;
    return PM_OK;
}

// Context settings that a tuning sweep changes, put back on every way out of
// pm_autotune unless the sweep finished and chose new ones.
struct TuneGuard {
    pm_ctx *ctx;
    pm::Shape shape;
    bool shape_auto;
    int bpc;
    bool graph;
    int32_t tmax;
    bool commit = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    explicit TuneGuard(pm_ctx *c)
        : ctx(c), shape(c->shape), shape_auto(c->shape_auto), bpc(c->blocks_per_cu),
          graph(c->use_graph), tmax(c->tmax)
    {
    }
    ~TuneGuard()
    {
        if (!commit) {
            ctx->shape = shape;
            ctx->shape_auto = shape_auto;
            ctx->blocks_per_cu = bpc;
        }
        ctx->use_graph = graph;
        ctx->tmax = tmax;
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
    }
};

pm_status pm_autotune(pm_ctx *ctx, const pm_field *field, const pm_decomp *decomp,
                      const pm_particles *in, pm_particles *out, pm_sendbufs *send,
                      const pm_params *params, void *stream, const char *cache_path)
{
    pm::KArgs k;
    bool mixed = false;
    pm_status s = step_args(ctx, field, decomp, in, out, send, params, k, mixed);
    if (s)
        return s;
    hipStream_t st = (hipStream_t)stream;
    // everything the fastest shape depends on: grid, field arrangement and
    // precision, drag law, decomposition, pool extent, tile order
    char key[320];
    snprintf(key, sizeof key,
             "n=%d,%d,%d halo=%d dtype=%d stagger=%d layout=%d drag=%d nsub=%d extent=%lld "
             "xcd=%d",
             field->n[0], field->n[1], field->n[2], field->halo, field->dtype, field->stagger,
             field->layout, params->drag, k.dc.nsub, (long long)ctx->ws.pool_extent,
             ctx->xcd_block);
    if (cache_path) {
        if (FILE *fp = fopen(cache_path, "r")) {
            char line[512];
            int wg = 0, items = 0, bpc = 0;
            bool hit = false;
            while (fgets(line, sizeof line, fp)) {
                char *bar = strchr(line, '|');
                if (!bar)
                    continue;
                *bar = 0;
                if (strcmp(line, key) == 0 &&
                    sscanf(bar + 1, " wg=%d items=%d bpc=%d", &wg, &items, &bpc) == 3) {
                    hit = true;
                }
            }
            fclose(fp);
            if (hit && pm::shape_supported({wg, items}) && bpc >= 0 && bpc <= 32) {
                ctx->shape = {wg, items};
                ctx->shape_auto = false;
                ctx->blocks_per_cu = bpc;
                return PM_OK;
            }
        }
    }
    const pm::Shape shapes[] = {{256, 1}, {256, 2}, {256, 4}, {256, 8},
                                {512, 1}, {512, 2}, {512, 4}};
    const int bpcs[] = {0, 2, 3, 4, 6};
    TuneGuard guard(ctx);
    ctx->use_graph = false;
    ctx->tmax = 0;
    PM_HIP(hipEventCreate(&guard.e0), "event create");
    PM_HIP(hipEventCreate(&guard.e1), "event create");
    float best = 1e30f;
    pm::Shape best_sh = shape_for(ctx, mixed, k.f.halo != 0, k.f.layout != 0);
    int best_bpc = ctx->blocks_per_cu;
    ctx->shape_auto = false;  // the sweep sets the shape of every trial
    for (const auto &sh : shapes) {
        for (int bpc : bpcs) {
            ctx->shape = sh;
            ctx->blocks_per_cu = bpc;
            pm::KArgs kk = k;
            for (int it = 0; it < 2; ++it) {
                const pm_status r = queue_step(ctx, kk, mixed, st, false);
                if (r)
                    return r;
            }
            PM_HIP(hipEventRecord(guard.e0, st), "event record");
            const int reps = 5;
            for (int it = 0; it < reps; ++it) {
                const pm_status r = queue_step(ctx, kk, mixed, st, false);
                if (r)
                    return r;
            }
            PM_HIP(hipEventRecord(guard.e1, st), "event record");
            PM_HIP(hipEventSynchronize(guard.e1), "event sync");
            float ms = 0.f;
            PM_HIP(hipEventElapsedTime(&ms, guard.e0, guard.e1), "elapsed");
            ms /= reps;
            if (getenv("PM_TUNE_VERBOSE"))
                fprintf(stderr, "pm_autotune: wg=%d items=%d bpc=%d %.4f ms/step\n", sh.wg,
                        sh.items, bpc, ms);
            if (ms < best) {
                best = ms;
                best_sh = sh;
                best_bpc = bpc;
            }
        }
    }
    ctx->shape = best_sh;
    ctx->blocks_per_cu = best_bpc;
    guard.commit = true;
    if (cache_path) {
        if (FILE *fp = fopen(cache_path, "a")) {
            fprintf(fp, "%s| wg=%d items=%d bpc=%d ms=%.4f\n", key, best_sh.wg, best_sh.items,
                    best_bpc, best);
            fclose(fp);
        }
    }
    return PM_OK;
}

// Layout of the re-sort workspace.
struct SortLayout {
    size_t keys[2], vals[2], hist, off, total;
    int64_t tiles;
};

static SortLayout sort_layout(int64_t pool_extent, int32_t nsub)
{
    SortLayout L{};
    const size_t pe = (size_t)std::max<int64_t>(pool_extent, 1);
    const size_t tiles = (size_t)(pool_extent / pm::sort_tile()) + (size_t)nsub + 1;
    L.tiles = (int64_t)tiles;
    size_t o = 0;
    for (int b = 0; b < 2; ++b) {
        L.keys[b] = o;
        o += align256(pe * sizeof(uint64_t));
    }
    for (int b = 0; b < 2; ++b) {
        L.vals[b] = o;
        o += align256(pe * sizeof(uint32_t));
    }
    L.hist = o;
    o += align256(tiles * 256 * sizeof(uint32_t));
    L.off = o;
    o += align256(tiles * 256 * sizeof(int64_t));
    L.total = o;
    return L;
}

size_t pm_sort_workspace_bytes(int64_t pool_extent, int32_t nsub)
{
    if (pool_extent < 0 || pool_extent >= ((int64_t)1 << 32) || nsub < 1 || nsub > PM_MAX_NSUB)
        return 0;
    return sort_layout(pool_extent, nsub).total;
}

pm_status pm_sort(pm_ctx *ctx, const pm_field *field, const pm_particles *in,
                  pm_particles *out, void *workspace, size_t ws_bytes, void *stream)
{
    if (!ctx)
        return arg_error("ctx is NULL");
    pm::KArgs k;
    base_args(ctx, k);
    bool mixed = false;
    pm_status s = conv_field(field, k.f, mixed);
    if (!s)
        s = conv_pool(in, "in", mixed, k.in);
    if (!s)
        s = conv_pool(out, "out", mixed, k.out);
    if (!s)
        s = check_range(ctx, in->nsub, 0, in->nsub);
    if (s)
        return s;
    if (out->nsub != in->nsub)
        return arg_error("out.nsub must equal in.nsub");
    if (in->x[0] == out->x[0])
        return arg_error("in and out must be different pools");
    if (ctx->ws.pool_extent >= ((int64_t)1 << 32))
        return arg_error("the re-sort takes pool extents below 2^32");
    const SortLayout L = sort_layout(ctx->ws.pool_extent, in->nsub);
    if (!workspace || ws_bytes < L.total)
        return arg_error("sort workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                         L.total);
    if (((uintptr_t)workspace & 255u) != 0)
        return arg_error("sort workspace must be 256-byte aligned");
    char *w = (char *)workspace;
    pm::DSort d;
    for (int b = 0; b < 2; ++b) {
        d.keys[b] = (uint64_t *)(w + L.keys[b]);
        d.vals[b] = (uint32_t *)(w + L.vals[b]);
    }
    d.hist = (uint32_t *)(w + L.hist);
    d.off = (int64_t *)(w + L.off);
    d.tiles = L.tiles;
    // radix passes over the key's bits: 3 bits per Z-order level plus the
    // parity bit of x
    int m = std::max({(field->n[0] - 1) >> 1, field->n[1] - 1, field->n[2] - 1, 1});
    int bits = 0;
    while (m) {
        ++bits;
        m >>= 1;
    }
    const int passes = (3 * bits + 1 + 7) / 8;
    k.sub_first = 0;
    k.sub_count = in->nsub;
    k.tile = pm::sort_tile();
    hipStream_t st = (hipStream_t)stream;
    PM_HIP(pm::launch_prep(k, pm::kPrepTiles | pm::kPrepCheckIn | pm::kPrepCheckOut, st),
           "prep launch");
    PM_HIP(pm::launch_sort(k, d, passes, mixed, std::max(1, ctx->cus * 4), st), "sort launch");
    return PM_OK;
}

pm_status pm_touched_nodes(pm_ctx *ctx, const pm_field *field, const pm_particles *in,
                           const pm_params *params, uint64_t *bitmap, int64_t nbits,
                           void *stream, int64_t *touched)
{
    if (!ctx || !touched)
        return arg_error("NULL argument");
    pm::KArgs k;
    base_args(ctx, k);
    bool mixed = false;
    pm_status s = conv_field(field, k.f, mixed);
    if (!s)
        s = conv_pool(in, "in", mixed, k.in);
    if (!s)
        s = conv_params(params, k);
    if (!s)
        s = check_range(ctx, in->nsub, 0, in->nsub);
    if (s)
        return s;
    const int64_t nodes = k.f.sxy * (field->n[2] + 2 * field->halo) * (k.f.stagger ? 3 : 1);
    if (!bitmap || nbits < nodes)
        return arg_error("bitmap needs %lld bits", (long long)nodes);
    hipStream_t st = (hipStream_t)stream;
    k.sub_first = 0;
    k.sub_count = in->nsub;
    const pm::Shape sh = shape_for(ctx, mixed, false);
    k.tile = sh.wg * sh.items;
    const int64_t words = (nbits + 63) / 64;
    PM_HIP(pm::launch_fill(bitmap, words, st), "fill launch");
    PM_HIP(pm::launch_prep(k, pm::kPrepTiles | pm::kPrepCheckIn, st), "prep launch");
    PM_HIP(pm::launch_touch(k, mixed, bitmap, st), "touch launch");
    unsigned long long *cnt = (unsigned long long *)(ctx->ws.hdr + 8);
    PM_HIP(hipMemsetAsync(cnt, 0, sizeof *cnt, st), "count clear");
    PM_HIP(pm::launch_popcount(bitmap, words, cnt, st), "popcount launch");
    unsigned long long h = 0;
    PM_HIP(hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, st), "count read");
    PM_HIP(hipStreamSynchronize(st), "stream sync");
    *touched = k.f.stagger ? (int64_t)((h + 1) / 3) : (int64_t)h;
    return PM_OK;
}

}  // extern "C"
