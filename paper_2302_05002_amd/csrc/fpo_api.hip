// Host side of libfpo: argument checks, workspace layout and the launch
// sequence of one build (C ABI in include/fpo.h).
#include <chrono>
#include <functional>
#include <mutex>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <string>
#include <vector>

#include "../../include/fpo.h"
#include "fpo_host.h"
#include "fpo_internal.h"

#include <algorithm>

using namespace fpo;

namespace {
thread_local std::string g_err;
}  // namespace

namespace fpo {

fpo_status fail(fpo_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

void set_error_text(const std::string &text) { g_err = text; }
std::string error_text() { return g_err; }

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

std::chrono::milliseconds wait_limit()
{
    static const long long ms = [] {
        const char *v = getenv("FPO_WAIT_LIMIT_MS");
        const long long t = v ? strtoll(v, nullptr, 10) : 0;
        return t > 0 ? t : 300000ll;
    }();
    return std::chrono::milliseconds(ms);
}

bool alloc_fault(fpo_context *c)
{
    if (!c || !c->fault_at) return false;
    return c->allocs.fetch_add(1) + 1 == c->fault_at;
}

void ctx_retain(fpo_context *c) { c->refs.fetch_add(1); }

void ctx_release(fpo_context *c)
{
    if (c->refs.fetch_sub(1) != 1) return;
    // last reference: no job, batch or server of the context is left
    (void)hipSetDevice(c->device);
    destroy_batch_pool(c);
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    for (void *p : c->pinned_free) (void)hipHostFree(p);
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // namespace fpo

namespace {

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(FPO_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool is_pow2(uint32_t v) { return v && !(v & (v - 1)); }
int ilog2(uint32_t v)
{
    int l = 0;
    while ((1u << l) < v) ++l;
    return l;
}
size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// Smallest host-to-device batch of pinned inputs (keeps the partial count bounded).
constexpr uint64_t MIN_STREAM_BATCH = 1u << 20;

// Capacities of one cut's lists (CutArgs) for n points: heavy nodes of a
// level number at most min(8^l, n) above lmin and min(8^l, n / (thresh + 1))
// from lmin on (disjoint nodes holding more than thresh points), and never
// more than eight per heavy node above; entries of a level number at most
// eight per heavy node above (and 8^l, and n).
struct CutPlan {
    uint64_t open_cap = 1;
    uint64_t ent_off[MAXD + 1] = {};
    uint64_t st_off[MAXD + 1] = {};
};

CutPlan cut_plan(uint64_t n, int lam, uint32_t thresh, int lmin)
{
    CutPlan c;
    uint64_t prev = 1;   // level 0: the root
    c.ent_off[0] = 0;
    c.ent_off[1] = lmin == 0 ? 1 : 0;
    for (int l = 1; l <= lam; ++l) {
        const uint64_t cells = 1ull << (3 * l);
        uint64_t ent = l < lmin ? 0 : std::min(std::min(cells, 8 * prev), n);
        c.ent_off[l + 1] = c.ent_off[l] + ent;
        uint64_t open = 0;
        if (l < lam) open = std::min(std::min(cells, l < lmin ? n : n / ((uint64_t)thresh + 1)), 8 * prev);
        c.open_cap = std::max(c.open_cap, open);
        prev = open;
    }
    const uint64_t tiles = (c.open_cap + FR_BLOCK - 1) / FR_BLOCK;
    for (int l = 0; l <= lam + 1; ++l) c.st_off[l] = l >= 1 ? (uint64_t)(l - 1) * tiles : 0;
    return c;
}

// Byte offsets of every region of the workspace for (n, params).
struct Plan {
    uint64_t n;
    int g, s, lam_w, d0, lt;
    uint64_t G3, W3, P;      // finest cells, work-chunk-level cells, pyramid words
    uint64_t maxC, maxW;
    size_t total;
    // results
    size_t xyz, box, bbox_part, ctrs, grid, c_level, c_key, c_count, c_begin, perm;
    size_t n_depth, n_key, n_mask, n_begin, n_count, n_points, pv_index;
    // temporaries
    size_t code, pyr, w_level, w_key, w_count, w_start, w_begin, c_start;
    CutPlan cp[2];   // chunk cut, work-chunk cut
    size_t cut_open[2], cut_ent[2], cut_st[2], cut_ctr[2], cut_idx[2];
    size_t c_count_scan, code_perm, wc_orig, wc_code, ms_temp, scan_temp, seg_b0, seg_nb, wc_nested, wc_chunk;
    size_t gtab, gtab2, t, fr, alive, alive_scan, kd, loff, owned, node_base, lnode_key, lnode_mask, cut;
    size_t big_list, big_nr, big_node, big_hkey, big_hval, cls_list;
    size_t np_tmp, np_glist, np_cnt, np_scan, np_nb, np_l0, np_l1, np_l2, np_l3, np_jobs, np_cp, np_single, pv_tiles, pv_offs,
        cellmin, pv_bits;
    uint64_t pv_ntiles;
    size_t shared_bytes;   // the region of ms_temp (split temporaries, then the subsample and node_points buffers)
};

Plan make_plan(uint64_t n, const fpo_params &p, bool host_in = false)
{
    Plan P{};
    P.n = n;
    P.g = ilog2(p.count_grid);
    P.s = ilog2(p.subsample_grid);
    P.lam_w = P.g;                          // work chunks as deep as the count grid
    P.d0 = P.g > P.s ? P.g - P.s : 0;       // shared depths decided globally
    P.G3 = 1ull << (3 * P.g);
    P.W3 = 1ull << (3 * P.lam_w);
    P.P = pyr_off(P.g + 1);
    P.lt = P.g < 7 ? P.g : 7;
    const uint64_t nn = n ? n : 1;
    P.maxC = nn < P.G3 ? nn : P.G3;
    P.maxW = nn < P.W3 ? nn : P.W3;
    {
        // a work chunk deeper than level d0 has a parent with more than
        // WC_CAP points; such parents are disjoint within a level and have at most
        // eight children each, and level d0 holds at most 8^d0 work chunks
        const uint64_t heavy = nn / (WC_CAP + 1);
        const uint64_t bound = (1ull << (3 * P.d0)) + 8ull * (uint64_t)(P.lam_w - P.d0) * heavy;
        if (bound < P.maxW) P.maxW = bound;
    }
    P.pv_ntiles = bits_tiles(nn);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += a256(bytes ? bytes : 1);
        return r;
    };
    // pinned host inputs: device staging of x, y, z (a256-aligned thirds)
    P.xyz = host_in ? take(3 * a256(4 * nn)) : 0;
    // counters, then the box 256 bytes later: the host reads both with one
    // copy into the same layout of its pinned staging
    P.ctrs = take(sizeof(Ctrs));
    P.box = take(sizeof(DevBox));
    // bounding-box partials: at most one per 1024 points per batch, plus one
    // per batch (batches of at least MIN_STREAM_BATCH points)
    P.bbox_part = take(8 * 4 * (nn / 1024 + nn / MIN_STREAM_BATCH + 1 + BBOX_MAX_BLOCKS));
    P.grid = take(4 * P.G3);
    P.c_level = take(P.maxC);
    P.c_key = take(8 * P.maxC);
    P.c_count = take(4 * P.maxC);
    P.c_begin = take(8 * P.maxC);
    P.perm = take(4 * nn);
    P.n_depth = take(nn);
    P.n_key = take(8 * nn);
    P.n_mask = take(nn + 4);
    P.n_begin = take(8 * nn);
    P.n_count = take(4 * nn);
    P.n_points = take(4 * nn);
    P.pv_index = take(4 * nn);
    // the Morton codes in input order and in chunk order, side by side: both
    // are dead once the work-chunk split has read them, and the subsample
    // path's hash values take their place
    P.code = take(8 * nn);
    P.code_perm = take(8 * nn);
    P.pyr = take(4 * P.P);
    P.c_start = take(8 * P.maxC);
    P.cp[0] = cut_plan(nn, P.g, p.max_points_per_chunk, 0);
    P.cp[1] = cut_plan(nn, P.lam_w, WC_CAP, P.d0);
    for (int k = 0; k < 2; ++k) {
        P.cut_open[k] = take(2 * 8 * P.cp[k].open_cap);
        P.cut_ent[k] = take(8 * P.cp[k].ent_off[P.g + 1]);
        P.cut_st[k] = take(8 * P.cp[k].st_off[P.g + 1]);
        P.cut_ctr[k] = take(4 * 3 * MAXD);
        P.cut_idx[k] = take(4 * ((1ull << (3 * P.lt)) + 1));
    }
    P.w_level = take(P.maxW);
    P.w_key = take(8 * P.maxW);
    P.w_count = take(4 * P.maxW);
    P.w_start = take(8 * P.maxW);
    P.w_begin = take(4 * P.maxW);
    P.c_count_scan = take(4 * P.maxC);
    P.wc_orig = take(4 * nn);
    P.seg_b0 = take(4 * P.maxC);
    P.seg_nb = take(4 * P.maxC);
    P.wc_nested = take(P.maxW);
    P.wc_chunk = take(4 * P.maxW);
    P.wc_code = take(8 * nn);
    // One region serves three phases in turn, each done before the next
    // begins on the stream: the stable splits' temporaries (the chunk split
    // and the work-chunk split), then the global-memory subsample path's
    // hash keys (4 slots per point, 8 B each) and node scratch (3 words per
    // point), then the buffers of node_points.  The hash values (4 B per
    // slot) go where the two code arrays were.
    {
        // chunks, work chunks and nodes each number at most n
        const size_t a = multisplit_temp_bound(nn, nn);
        // segmented work-chunk scatter: count matrix bounded by n + #work chunks
        const size_t b = multisplit_seg_temp_bytes(nn, (uint32_t)P.maxC, nn + P.maxW);
        const size_t split = a > b ? a : b;
        const size_t base = o;
        size_t q = base;
        auto sub = [&](size_t bytes) {
            size_t r = q;
            q += a256(bytes ? bytes : 1);
            return r;
        };
        P.big_hkey = sub(8 * 4 * nn);
        P.big_node = sub(12 * nn);
        P.big_hval = P.code;   // 16 B per point: code and code_perm, 256-aligned each
        const size_t big = q - base;
        q = base;
        P.np_tmp = sub(4 * nn);
        P.np_nb = sub(4 * (nn + 1));
        P.np_l0 = sub(4 * np_list_entries(nn, 0));
        P.np_l1 = sub(4 * np_list_entries(nn, 1));
        P.np_l2 = sub(4 * np_list_entries(nn, 2));
        P.np_l3 = sub(8 * np_list_entries(nn, 3));
        P.np_jobs = sub(8 * np_job_entries(nn));
        P.np_cp = sub(8 * np_copy_entries(nn));
        P.np_single = sub(nn);
        const size_t np = q - base;
        size_t region = split > big ? split : big;
        if (np > region) region = np;
        P.ms_temp = take(region);
        P.shared_bytes = region;
    }
    uint64_t scan_max = (uint64_t)MAXD * P.maxW;
    if (P.pv_ntiles > scan_max) scan_max = P.pv_ntiles;
    if (nn > scan_max) scan_max = nn;   // node sizes (nodes number at most n)
    P.scan_temp = take(scan_temp_bytes(scan_max));
    // cells of the deepest globally decided depth (level d0 - 1 + s)
    P.gtab = P.d0 > 0 ? take(4ull << (3 * (P.d0 - 1 + P.s))) : 0;
    P.gtab2 = P.d0 > 1 ? take(4ull << (3 * (P.d0 - 2 + P.s))) : 0;
    P.t = take(nn);
    P.fr = take(4 * nn);
    P.alive = take(4 * MAXD * P.maxW);
    P.alive_scan = take(4 * (MAXD * P.maxW + 1));
    P.kd = take(4 * MAXD * P.maxW);
    P.loff = take(4 * MAXD * P.maxW);
    P.owned = take(4 * MAXD * P.maxW);
    P.node_base = take(4 * MAXD * P.maxW);
    P.lnode_key = take(8 * nn);
    P.lnode_mask = take(nn);
    P.cut = take(P.maxW);
    P.big_list = take(4 * P.maxW);
    P.cls_list = take(4 * (uint64_t)WC_CLASSES * P.maxW);
    P.big_nr = take(4 * nn);
    P.np_cnt = take(4 * MAXD * P.maxW);
    P.np_glist = take(4 * P.maxW);
    P.np_scan = take(4 * (MAXD * P.maxW + 1));
    P.pv_tiles = take(4 * P.pv_ntiles);
    P.pv_offs = take(4 * P.pv_ntiles);
    P.cellmin = (p.flags & FPO_PREVIEW_GRID) ? take(8 * P.G3) : 0;
    P.pv_bits = take(4 * ((nn + 31) / 32));
    P.total = o;
    return P;
}

}  // namespace

namespace fpo {

fpo_status check_params(uint64_t n, const fpo_params *p)
{
    if (!p) return fail(FPO_ERR_INVALID_ARG, "params is NULL");
    if (!is_pow2(p->count_grid) || p->count_grid > 512)
        return fail(FPO_ERR_INVALID_ARG, "count_grid must be a power of two in 1..512 (got %u)", p->count_grid);
    if (!is_pow2(p->subsample_grid) || p->subsample_grid > 256)
        return fail(FPO_ERR_INVALID_ARG, "subsample_grid must be a power of two in 1..256 (got %u)", p->subsample_grid);
    if (p->max_points_per_chunk == 0) return fail(FPO_ERR_INVALID_ARG, "max_points_per_chunk must be >= 1");
    if (p->leaf_capacity == 0) return fail(FPO_ERR_INVALID_ARG, "leaf_capacity must be >= 1");
    if (p->preview_modulus == 0) return fail(FPO_ERR_INVALID_ARG, "preview_modulus must be >= 1");
    if (n > 0xffffffffull) return fail(FPO_ERR_INVALID_ARG, "n = %llu exceeds 2^32 - 1", (unsigned long long)n);
    if (p->flags & ~(FPO_BBOX_GIVEN | FPO_PREVIEW_STRIDE | FPO_PREVIEW_GRID))
        return fail(FPO_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
    if ((p->flags & FPO_PREVIEW_STRIDE) && (p->flags & FPO_PREVIEW_GRID))
        return fail(FPO_ERR_INVALID_ARG, "FPO_PREVIEW_STRIDE and FPO_PREVIEW_GRID exclude each other");
    if (p->flags & FPO_BBOX_GIVEN)
        for (int a = 0; a < 3; ++a) {
            const float lo = p->bbox_min[a], hi = p->bbox_max[a];
            if (!(lo == lo) || !(hi == hi) || lo - lo != 0.0f || hi - hi != 0.0f || lo > hi)
                return fail(FPO_ERR_INVALID_ARG, "given bbox must be finite with min <= max on axis %d", a);
        }
    return FPO_OK;
}

uint64_t workspace_bytes(uint64_t n, const fpo_params &p, bool host_input) { return make_plan(n, p, host_input).total; }

}  // namespace fpo

namespace {

constexpr size_t PINNED_BYTES = 1024;

void *get_pinned(fpo_context *c)
{
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->pinned_free.empty()) {
        void *p = c->pinned_free.back();
        c->pinned_free.pop_back();
        return p;
    }
    void *p = nullptr;
    if (alloc_fault(c) || hipHostMalloc(&p, PINNED_BYTES, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
}

void put_pinned(fpo_context *c, void *p)
{
    std::lock_guard<std::mutex> g(c->mu);
    c->pinned_free.push_back(p);
}

hipEvent_t get_event(fpo_context *c)
{
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (!c->ev_free.empty()) {
            hipEvent_t e = c->ev_free.back();
            c->ev_free.pop_back();
            return e;
        }
    }
    // timing only: their elapsed times are read once the job's completion
    // event (system-scope release) has been seen, so they need no fence of
    // their own, whose cache writeback and invalidation would slow the work
    // they bracket
    hipEvent_t e = nullptr;
    if (alloc_fault(c) || hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Brackets launches with a pair of timing events, kept by the job.
struct JobTimer final : LaunchTimer {
    fpo_job *job;
    int which;
    hipEvent_t first = nullptr;
    JobTimer(fpo_job *j, int w) : job(j), which(w) {}
    void begin(hipStream_t st) override;
    void end(hipStream_t st) override;
};

void JobTimer::begin(hipStream_t st)
{
    first = job->timed && ((job->timer_mask >> which) & 1u) ? get_event(job->ctx) : nullptr;
    if (first) (void)hipEventRecord(first, st);
}

void JobTimer::end(hipStream_t st)
{
    if (!first) return;
    hipEvent_t second = get_event(job->ctx);
    if (!second) return;
    (void)hipEventRecord(second, st);
    job->tm[which].push_back({first, second});
    first = nullptr;
}

}  // namespace

extern "C" {

const char *fpo_last_error(void) { return g_err.c_str(); }

fpo_status fpo_context_create(int device, fpo_context **out)
{
    if (!out) return fail(FPO_ERR_INVALID_ARG, "out is NULL");
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(FPO_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, count);
    HIPCHK(hipSetDevice(device));
    {
        const fpo_status si = select_static_init(device);
        if (si != FPO_OK) return si;
    }
    fpo_context *c = new fpo_context();
    c->device = device;
    if (const char *f = getenv("FPO_FAULT"))
        if (strncmp(f, "alloc:", 6) == 0) c->fault_at = strtoull(f + 6, nullptr, 10);
    memset(c->qz_variant, 0xff, sizeof(c->qz_variant));
    tune_cache_load(c);
    if (alloc_fault(c) || hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(FPO_ERR_OUT_OF_MEMORY, "could not create the context's stream");
    }
    *out = c;
    return FPO_OK;
}

void fpo_context_destroy(fpo_context *c)
{
    if (c) ctx_release(c);
}

fpo_status fpo_workspace_size(uint64_t n, const fpo_params *p, uint64_t *bytes)
{
    fpo_status s = check_params(n, p);
    if (s != FPO_OK) return s;
    if (!bytes) return fail(FPO_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = make_plan(n, *p).total;
    return FPO_OK;
}

fpo_status fpo_preview_modulus(uint64_t n, uint64_t target, uint32_t *out)
{
    if (!out) return fail(FPO_ERR_INVALID_ARG, "out is NULL");
    if (target == 0) return fail(FPO_ERR_INVALID_ARG, "target must be >= 1");
    if (n > 0xffffffffull) return fail(FPO_ERR_INVALID_ARG, "n = %llu exceeds 2^32 - 1", (unsigned long long)n);
    const uint64_t m = (n + target - 1) / target;
    *out = (uint32_t)(m ? m : 1);
    return FPO_OK;
}

fpo_status fpo_workspace_size_cloud(const fpo_cloud *cloud, const fpo_params *p, uint64_t *bytes)
{
    if (!cloud) return fail(FPO_ERR_INVALID_ARG, "cloud is NULL");
    fpo_status s = check_params(cloud->n, p);
    if (s != FPO_OK) return s;
    if (!bytes) return fail(FPO_ERR_INVALID_ARG, "bytes is NULL");
    if (cloud->location != FPO_DEVICE && cloud->location != FPO_HOST_PINNED)
        return fail(FPO_ERR_INVALID_ARG, "unknown location %u", cloud->location);
    *bytes = make_plan(cloud->n, *p, cloud->location == FPO_HOST_PINNED).total;
    return FPO_OK;
}

}  // extern "C"

namespace fpo {

// Checks every argument of a build; fills the stream batch and the plan size.
static fpo_status check_build(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                              uint64_t workspace_bytes)
{
    if (!ctx || !cloud) return fail(FPO_ERR_INVALID_ARG, "NULL context or cloud");
    fpo_status s = check_params(cloud->n, p);
    if (s != FPO_OK) return s;
    const uint64_t n = cloud->n;
    if (n > 0 && (!cloud->x || !cloud->y || !cloud->z)) return fail(FPO_ERR_INVALID_ARG, "NULL coordinate array");
    if (!workspace) return fail(FPO_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(FPO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (cloud->location != FPO_DEVICE && cloud->location != FPO_HOST_PINNED)
        return fail(FPO_ERR_INVALID_ARG, "unknown location %u", cloud->location);
    const bool host_in = cloud->location == FPO_HOST_PINNED && n > 0;
    if (host_in) {
        // the copies run asynchronously: the arrays must be pinned host memory
        for (const float *a : {cloud->x, cloud->y, cloud->z}) {
            hipPointerAttribute_t attr;
            if (hipPointerGetAttributes(&attr, a) != hipSuccess || attr.type != hipMemoryTypeHost) {
                (void)hipGetLastError();
                return fail(FPO_ERR_INVALID_ARG, "location FPO_HOST_PINNED needs pinned host arrays (hipHostMalloc)");
            }
        }
    }
    const uint64_t need = make_plan(n, *p, host_in).total;
    if (workspace_bytes < need)
        return fail(FPO_ERR_OUT_OF_MEMORY, "workspace holds %llu bytes, the build needs %llu",
                    (unsigned long long)workspace_bytes, (unsigned long long)need);
    return FPO_OK;
}

// A job for a build on st (its events and pinned staging).
static fpo_status new_job(fpo_context *ctx, hipStream_t st, const fpo_params *p, uint64_t grid_cells,
                          uint64_t plan_bytes, fpo_job **out)
{
    fpo_job *job = new fpo_job();
    job->ctx = ctx;
    job->stream = st;
    job->status = FPO_OK;
    job->waited = false;
    job->timed = ctx->timing;
    job->timer_mask = ctx->timer_mask;
    job->t_submit = now_ns();
    job->t_done = 0;
    job->grid_cells = grid_cells;
    job->plan_bytes = plan_bytes;
    job->params = *p;
    job->ev_preview = job->ev_done = nullptr;
    job->pinned = get_pinned(ctx);
    if (!job->pinned) {
        delete job;
        return fail(FPO_ERR_OUT_OF_MEMORY, "pinned host staging allocation failed");
    }
    if (alloc_fault(ctx) || hipEventCreateWithFlags(&job->ev_preview, hipEventDisableTiming) != hipSuccess ||
        alloc_fault(ctx) || hipEventCreateWithFlags(&job->ev_done, hipEventDisableTiming) != hipSuccess) {
        if (job->ev_preview) (void)hipEventDestroy(job->ev_preview);
        put_pinned(ctx, job->pinned);
        delete job;
        return fail(FPO_ERR_OUT_OF_MEMORY, "could not create the job's events");
    }
    *out = job;
    return FPO_OK;
}

bool small_eligible(uint64_t limit, uint64_t n, const fpo_params &p, bool host_in)
{
    return !host_in && n >= 1 && n <= limit && n <= SB_MAX_N && n <= p.max_points_per_chunk &&
           p.count_grid <= SB_MAX_G && p.subsample_grid <= SB_MAX_S && !(p.flags & FPO_PREVIEW_GRID) &&
           n / ((uint64_t)p.leaf_capacity + 1) <= SB_MAX_INNER;
}

fpo_status issue_small_group(fpo_context *ctx, uint32_t count, const fpo_cloud *const *clouds,
                             const fpo_params *const *params, void *const *workspaces, hipStream_t st,
                             fpo_job **jobs_out)
{
    if (count == 0 || count > SB_GROUP) return fail(FPO_ERR_INVALID_ARG, "internal: %u clouds in one group", count);
    HIPCHK(hipSetDevice(ctx->device));
    SmallGroup grp{};
    std::vector<fpo_job *> jobs(count, nullptr);
    std::vector<SmallLayout> lay(count);
    auto drop = [&]() {   // nothing was enqueued: the jobs were never handed out
        for (fpo_job *j : jobs)
            if (j) fpo_job_release(j);
    };
    for (uint32_t i = 0; i < count; ++i) {
        const fpo_cloud &c = *clouds[i];
        const fpo_params &p = *params[i];
        const uint64_t n = c.n;
        const int g = (int)ilog2(p.count_grid);
        const Plan P = make_plan(n, p);
        lay[i] = small_layout(n, g);
        if (!small_eligible(SB_MAX_N, n, p, c.location == FPO_HOST_PINNED) || lay[i].total > P.total) {
            drop();
            return fail(FPO_ERR_INVALID_ARG, "internal: cloud %u does not take the single-workgroup path", i);
        }
        const fpo_status js = new_job(ctx, st, &p, P.G3, P.total, &jobs[i]);
        if (js != FPO_OK) {
            drop();
            return js;
        }
        fpo_job *job = jobs[i];
        job->small = true;
        char *ws = static_cast<char *>(workspaces[i]);
        const SmallLayout &Lo = lay[i];
        fpo_result &R = job->res;
        memset(&R, 0, sizeof(R));
        R.n = n;
        R.count_grid = reinterpret_cast<const uint32_t *>(ws + Lo.grid);
        R.chunk_level = reinterpret_cast<const uint8_t *>(ws + Lo.c_level);
        R.chunk_key = reinterpret_cast<const uint64_t *>(ws + Lo.c_key);
        R.chunk_count = reinterpret_cast<const uint32_t *>(ws + Lo.c_count);
        R.chunk_begin = reinterpret_cast<const uint64_t *>(ws + Lo.c_begin);
        R.perm = reinterpret_cast<const uint32_t *>(ws + Lo.perm);
        R.node_depth = reinterpret_cast<const uint8_t *>(ws + Lo.n_depth);
        R.node_key = reinterpret_cast<const uint64_t *>(ws + Lo.n_key);
        R.node_child_mask = reinterpret_cast<const uint8_t *>(ws + Lo.n_mask);
        R.node_begin = reinterpret_cast<const uint64_t *>(ws + Lo.n_begin);
        R.node_count = reinterpret_cast<const uint32_t *>(ws + Lo.n_count);
        R.node_points = reinterpret_cast<const uint32_t *>(ws + Lo.n_points);
        R.preview_index = reinterpret_cast<const uint32_t *>(ws + Lo.pv_index);
        SmallDesc &d = grp.d[i];
        d.x = c.x;
        d.y = c.y;
        d.z = c.z;
        d.ws = ws;
        d.n = (uint32_t)n;
        d.g = (uint32_t)g;
        d.s = ilog2(p.subsample_grid);
        d.L = p.leaf_capacity;
        d.M = p.preview_modulus;
        d.given = (p.flags & FPO_BBOX_GIVEN) ? 1u : 0u;
        d.stride = (p.flags & FPO_PREVIEW_STRIDE) ? 1u : 0u;
        for (int a = 0; a < 3; ++a) {
            d.glo[a] = p.bbox_min[a];
            d.ghi[a] = p.bbox_max[a];
        }
    }
    std::vector<JobTimer> tmr;
    tmr.reserve(count);
    for (uint32_t i = 0; i < count; ++i) {
        tmr.emplace_back(jobs[i], FPO_TIMER_FUSED);
        tmr[i].begin(st);
    }
    launch_small_build(grp, count, st);
    for (uint32_t i = 0; i < count; ++i) tmr[i].end(st);
    hipError_t e = hipGetLastError();
    for (uint32_t i = 0; i < count && e == hipSuccess; ++i) e = hipEventRecord(jobs[i]->ev_preview, st);
    // counters and box of every build (the counts of chunks and nodes come
    // with them)
    for (uint32_t i = 0; i < count && e == hipSuccess; ++i)
        e = hipMemcpyAsync(jobs[i]->pinned, static_cast<char *>(workspaces[i]) + lay[i].ctrs, 256 + sizeof(DevBox),
                           hipMemcpyDeviceToHost, st);
    for (uint32_t i = 0; i < count && e == hipSuccess; ++i) e = hipEventRecord(jobs[i]->ev_done, st);
    if (e != hipSuccess) {
        // the launch may be in flight: the jobs end with the error, their
        // done events recorded where possible
        for (fpo_job *j : jobs) {
            j->status = FPO_ERR_DEVICE;
            (void)hipEventRecord(j->ev_done, st);
        }
        for (uint32_t i = 0; i < count; ++i) jobs_out[i] = jobs[i];
        return FPO_OK;
    }
    for (uint32_t i = 0; i < count; ++i) jobs_out[i] = jobs[i];
    return FPO_OK;
}

// Enqueues one whole build on st, with the host round trips it needs (the
// counts of chunks, work chunks and nodes size later launches).  on_preview,
// if given, receives the job as soon as the preview kernels are enqueued;
// from then on the job is never freed here: an error later ends it with its
// status set (and its done event recorded) for the caller to release.
fpo_status issue_build(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                       uint64_t workspace_bytes, hipStream_t st, fpo_job **out,
                       const std::function<void(fpo_job *)> &on_preview)
{
    if (!ctx || !cloud || !out) return fail(FPO_ERR_INVALID_ARG, "NULL context, cloud or out");
    fpo_status s = check_params(cloud->n, p);
    if (s != FPO_OK) return s;
    const uint64_t n = cloud->n;
    if (n > 0 && (!cloud->x || !cloud->y || !cloud->z)) return fail(FPO_ERR_INVALID_ARG, "NULL coordinate array");
    if (!workspace) return fail(FPO_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(FPO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (cloud->location != FPO_DEVICE && cloud->location != FPO_HOST_PINNED)
        return fail(FPO_ERR_INVALID_ARG, "unknown location %u", cloud->location);
    const bool host_in = cloud->location == FPO_HOST_PINNED && n > 0;
    if (host_in) {
        // the copies run asynchronously: the arrays must be pinned host memory
        for (const float *a : {cloud->x, cloud->y, cloud->z}) {
            hipPointerAttribute_t attr;
            if (hipPointerGetAttributes(&attr, a) != hipSuccess || attr.type != hipMemoryTypeHost) {
                (void)hipGetLastError();
                return fail(FPO_ERR_INVALID_ARG, "location FPO_HOST_PINNED needs pinned host arrays (hipHostMalloc)");
            }
        }
    }
    uint64_t sbatch = host_in ? (cloud->stream_batch ? cloud->stream_batch : FPO_DEFAULT_STREAM_BATCH) : n;
    if (host_in && sbatch < MIN_STREAM_BATCH) sbatch = MIN_STREAM_BATCH;
    sbatch = (sbatch + 63) / 64 * 64;   // batches start on 256-byte boundaries
    const Plan P = make_plan(n, *p, host_in);
    if (workspace_bytes < P.total)
        return fail(FPO_ERR_OUT_OF_MEMORY, "workspace holds %llu bytes, the build needs %llu",
                    (unsigned long long)workspace_bytes, (unsigned long long)P.total);
    HIPCHK(hipSetDevice(ctx->device));

    if (small_eligible(ctx->small_max.load(), n, *p, host_in)) {
        // the whole build in one workgroup
        void *w = workspace;
        fpo_job *job = nullptr;
        const fpo_status ss = issue_small_group(ctx, 1, &cloud, &p, &w, st, &job);
        if (ss != FPO_OK) return ss;
        if (on_preview) on_preview(job);
        *out = job;
        return FPO_OK;
    }
    fpo_job *job = nullptr;
    {
        const fpo_status js = new_job(ctx, st, p, P.G3, P.total, &job);
        if (js != FPO_OK) return js;
    }

    char *ws = static_cast<char *>(workspace);
    auto U32 = [&](size_t off) { return reinterpret_cast<uint32_t *>(ws + off); };
    auto U64 = [&](size_t off) { return reinterpret_cast<uint64_t *>(ws + off); };
    auto U8 = [&](size_t off) { return reinterpret_cast<uint8_t *>(ws + off); };
    DevBox *box = reinterpret_cast<DevBox *>(ws + P.box);
    Ctrs *ctrs = reinterpret_cast<Ctrs *>(ws + P.ctrs);
    Ctrs *hctrs = static_cast<Ctrs *>(job->pinned);
    DevBox *hbox = reinterpret_cast<DevBox *>(static_cast<char *>(job->pinned) + 256);
    const int g = P.g, s_ = P.s;
    const uint32_t G = p->count_grid;
    (void)G;
    const uint64_t M = p->preview_modulus;
    void *stemp = ws + P.scan_temp;

    fpo_result &R = job->res;
    memset(&R, 0, sizeof(R));
    R.n = n;
    R.count_grid = U32(P.grid);
    R.chunk_level = U8(P.c_level);
    R.chunk_key = U64(P.c_key);
    R.chunk_count = U32(P.c_count);
    R.chunk_begin = U64(P.c_begin);
    R.perm = U32(P.perm);
    R.node_depth = U8(P.n_depth);
    R.node_key = U64(P.n_key);
    R.node_child_mask = U8(P.n_mask);
    R.node_begin = U64(P.n_begin);
    R.node_count = U32(P.n_count);
    R.node_points = U32(P.n_points);
    R.preview_index = U32(P.pv_index);

    bool published = false;
    // ends the job with status fs: freed if nobody holds it yet, else left to
    // its holder with the done event recorded
    auto end_job = [&](fpo_status fs) {
        if (!published) {
            fpo_job_release(job);
        } else {
            job->status = fs;
            (void)hipEventRecord(job->ev_done, st);
        }
        return fs;
    };
#define JCHK(call)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            fpo_status fs_ = fail(FPO_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_));      \
            return end_job(fs_);                                                                \
        }                                                                                       \
    } while (0)

    JobTimer t_prev(job, FPO_TIMER_PREVIEW);
    // the counters start at zero: cleared here, or by the first preview kernel
    // when that is the build's first launch (hash and stride previews)
    const bool early_preview = !(p->flags & FPO_PREVIEW_GRID) && n > 0;
    if (!(p->flags & FPO_PREVIEW_GRID)) t_prev.begin(st);
    if (!early_preview) launch_fill_u32(reinterpret_cast<uint32_t *>(ctrs), 0u, sizeof(Ctrs) / 4, st);
    if (n == 0) {
        t_prev.end(st);
        launch_fill_u32(U32(P.grid), 0u, P.G3, st);
        JCHK(hipEventRecord(job->ev_preview, st));
        JCHK(hipEventRecord(job->ev_done, st));
        published = true;
        if (on_preview) on_preview(job);
        if (p->flags & FPO_BBOX_GIVEN)
            for (int a = 0; a < 3; ++a) { R.bbox_min[a] = p->bbox_min[a]; R.bbox_max[a] = p->bbox_max[a]; }
        *out = job;
        return FPO_OK;
    }

    // ---- step 5 first: hash and stride previews depend on n and M only ----
    PreviewArgs pa{};
    pa.n = n;
    pa.m = M;
    pa.mode = (p->flags & FPO_PREVIEW_GRID) ? PV_GRID : (p->flags & FPO_PREVIEW_STRIDE) ? PV_STRIDE : PV_HASH;
    pa.code = U64(P.code);
    pa.cellmin = U64(P.cellmin);
    pa.shift = 3 * (KB - g);
    if (early_preview) {
        pa.zero = reinterpret_cast<uint32_t *>(ctrs);
        pa.zero_words = sizeof(Ctrs) / 4;
    }
    // ordered compaction of the kept indices, then the preview event (from
    // here on the job belongs to its holder)
    auto emit_preview = [&]() {
        if (pa.mode == PV_GRID) t_prev.begin(st);
        uint32_t *bits = U32(P.pv_bits);
        if (pa.mode == PV_GRID && P.G3 <= 2 * n) {
            // fewer cells than 2n: a pass over the cell minima
            launch_fill_u32(bits, 0u, (n + 31) / 32, st);
            launch_grid_picks(pa.cellmin, P.G3, n, bits, st);
            launch_bits_count(bits, n, U32(P.pv_tiles), st);
        } else {
            launch_preview_bits(pa, bits, U32(P.pv_tiles), st);   // the predicate and the tile counts
        }
        scan_exclusive(U32(P.pv_tiles), U32(P.pv_offs), bits_tiles(n), &ctrs->preview_count, stemp, st);
        launch_bits_write(bits, n, U32(P.pv_offs), U32(P.pv_index), st);
        t_prev.end(st);
        const hipError_t e = hipEventRecord(job->ev_preview, st);
        if (e == hipSuccess) {
            published = true;
            if (on_preview) on_preview(job);
        }
        return e;
    };
    if (pa.mode != PV_GRID) JCHK(emit_preview());

    // ---- step 1: bbox, quantise, count ----
    const int given = (p->flags & FPO_BBOX_GIVEN) ? 1 : 0;
    const int qv = quantize_variant(ctx, n, P.g);
    // the binned quantise + count pass: one pass over device-resident input
    // without the grid preview; its temporaries sit in the region the splits
    // use later and where the chunk-ordered codes go
    const bool binned = qv == QZ_BINNED && !host_in && pa.mode != PV_GRID && quantize_binned_ok(n, P.g) &&
                        quantize_binned_temp_bytes(P.g) <= P.shared_bytes;
    // Timed regions (when timing): contiguous runs of launches that together
    // cover every kernel of the build; only the host round trips fall between
    // them.
    JobTimer t_bbox(job, FPO_TIMER_BBOX), t_quant(job, FPO_TIMER_QUANTIZE), t_cut(job, FPO_TIMER_CUT),
        t_chunk(job, FPO_TIMER_CHUNK_SPLIT), t_sub(job, FPO_TIMER_SUBSAMPLE), t_ncnt(job, FPO_TIMER_NODE_COUNTS),
        t_place(job, FPO_TIMER_NODE_PLACE), t_nsort(job, FPO_TIMER_NODE_SORT);
    const float *X = cloud->x, *Y = cloud->y, *Z = cloud->z;
    if (host_in) {
        // pinned host input: batches copied into the workspace on the copy
        // stream (after the work enqueued on st so far, which may still use
        // the workspace), one event per batch
        hipStream_t cs;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            if (!ctx->copy_stream &&
                (alloc_fault(ctx) || hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking) != hipSuccess))
                ctx->copy_stream = nullptr;
            cs = ctx->copy_stream;
        }
        if (!cs) return end_job(fail(FPO_ERR_OUT_OF_MEMORY, "could not create the copy stream"));
        float *dx = reinterpret_cast<float *>(ws + P.xyz);
        float *dy = reinterpret_cast<float *>(ws + P.xyz + a256(4 * n));
        float *dz = reinterpret_cast<float *>(ws + P.xyz + 2 * a256(4 * n));
        hipEvent_t before;
        JCHK(hipEventCreateWithFlags(&before, hipEventDisableTiming));
        job->stream_events.push_back(before);
        JCHK(hipEventRecord(before, st));
        JCHK(hipStreamWaitEvent(cs, before, 0));
        for (uint64_t o = 0; o < n; o += sbatch) {
            const uint64_t c = n - o < sbatch ? n - o : sbatch;
            JCHK(hipMemcpyAsync(dx + o, cloud->x + o, 4 * c, hipMemcpyHostToDevice, cs));
            JCHK(hipMemcpyAsync(dy + o, cloud->y + o, 4 * c, hipMemcpyHostToDevice, cs));
            JCHK(hipMemcpyAsync(dz + o, cloud->z + o, 4 * c, hipMemcpyHostToDevice, cs));
            hipEvent_t e;
            JCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            job->stream_events.push_back(e);
            JCHK(hipEventRecord(e, cs));
        }
        X = dx;
        Y = dy;
        Z = dz;
    }
    uint32_t *pyr = U32(P.pyr);
    uint32_t *fine = pyr + pyr_off(g);
    const bool box_region = !given;   // a given box has no bounding-box pass: its fills go with quantise
    // the count grid is cleared by the bounding-box pass of a one-batch build
    // (device input), else here; the binned pass writes every cell
    const bool zero_in_bbox = !given && !host_in && !binned;
    (box_region ? t_bbox : t_quant).begin(st);
    if (!zero_in_bbox && !binned) launch_fill_u32(fine, 0u, P.G3, st);
    uint64_t *cellmin = pa.mode == PV_GRID ? U64(P.cellmin) : nullptr;
    if (cellmin) launch_fill_u32(U32(P.cellmin), 0xffffffffu, 2 * P.G3, st);
    (box_region ? t_bbox : t_quant).end(st);
    if (given) {
        // a given box: no bounding-box pass.  The quantise + count pass of a
        // batch starts as soon as it has landed and also flags non-finite
        // coordinates and counts points outside the box
        t_quant.begin(st);
        launch_setup(box, U32(P.bbox_part), 0, given, p->bbox_min, p->bbox_max, 0, st);
        t_quant.end(st);
        size_t bi = 1;
        for (uint64_t o = 0; o < n; o += sbatch) {
            const uint64_t c = n - o < sbatch ? n - o : sbatch;
            if (host_in) JCHK(hipStreamWaitEvent(st, job->stream_events[bi++], 0));
            t_quant.begin(st);
            if (binned)
                launch_quantize_binned(X, Y, Z, n, box, g, 1, U64(P.code), fine, box, ws + P.ms_temp,
                                       reinterpret_cast<uint16_t *>(ws + P.code_perm), stemp, st);
            else
                launch_quantize(X + o, Y + o, Z + o, c, box, g, 1, U64(P.code) + o, fine, box, o, cellmin, st, qv);
            t_quant.end(st);
        }
    } else {
        // bounding box of each batch as it lands, then the box and one
        // quantise + count pass over all points
        uint32_t nparts = 0;
        size_t bi = 1;
        for (uint64_t o = 0; o < n; o += sbatch) {
            const uint64_t c = n - o < sbatch ? n - o : sbatch;
            if (host_in) JCHK(hipStreamWaitEvent(st, job->stream_events[bi++], 0));
            t_bbox.begin(st);
            launch_bbox(X + o, Y + o, Z + o, c, U32(P.bbox_part) + 8ull * nparts, st, zero_in_bbox ? fine : nullptr,
                        zero_in_bbox ? P.G3 : 0);
            t_bbox.end(st);
            nparts += bbox_blocks(c);
        }
        t_bbox.begin(st);
        launch_setup(box, U32(P.bbox_part), nparts, 0, p->bbox_min, p->bbox_max, 0, st);
        t_bbox.end(st);
        t_quant.begin(st);
        if (binned)
            launch_quantize_binned(X, Y, Z, n, box, g, 0, U64(P.code), fine, box, ws + P.ms_temp,
                                   reinterpret_cast<uint16_t *>(ws + P.code_perm), stemp, st);
        else
            launch_quantize(X, Y, Z, n, box, g, 0, U64(P.code), fine, box, 0, cellmin, st, qv);
        t_quant.end(st);
    }

    // grid preview: the least H64 of every occupied cell is known now
    if (pa.mode == PV_GRID) JCHK(emit_preview());

    // ---- step 2: pyramid, chunk cut, work-chunk cut ----
    t_cut.begin(st);
    launch_pyramid(pyr, g, U32(P.grid), st);   // with the row-major count grid
    CutArgs cut[2];
    for (int k = 0; k < 2; ++k) {
        CutArgs &c = cut[k];
        const CutPlan &cp = P.cp[k];
        c.thresh = k == 0 ? p->max_points_per_chunk : WC_CAP;
        c.lmin = k == 0 ? 0 : P.d0;
        c.lam = g;
        c.lt = P.lt;
        c.open[0] = U64(P.cut_open[k]);
        c.open[1] = U64(P.cut_open[k]) + cp.open_cap;
        c.open_cap = (uint32_t)cp.open_cap;
        c.n_open = U32(P.cut_ctr[k]);
        c.n_ent = c.n_open + MAXD;
        c.tile_ctr = c.n_open + 2 * MAXD;
        c.ent = U64(P.cut_ent[k]);
        c.status = reinterpret_cast<unsigned long long *>(ws + P.cut_st[k]);
        for (int l = 0; l <= MAXD; ++l) {
            c.ent_off[l] = l <= g + 1 ? cp.ent_off[l] : cp.ent_off[g + 1];
            c.st_off[l] = l <= g + 1 ? cp.st_off[l] : cp.st_off[g + 1];
        }
        c.over = k == 0 ? &ctrs->oversized : &ctrs->wc_over;
        c.err = &ctrs->internal_error;
        c.num_out = k == 0 ? &ctrs->num_chunks : &ctrs->num_wc;
        c.max_out = (uint32_t)(k == 0 ? P.maxC : P.maxW);
        c.out_level = k == 0 ? U8(P.c_level) : U8(P.w_level);
        c.out_key = k == 0 ? U64(P.c_key) : U64(P.w_key);
        c.out_count = k == 0 ? U32(P.c_count) : U32(P.w_count);
        c.out_start = k == 0 ? U64(P.c_start) : U64(P.w_start);
        c.idx = U32(P.cut_idx[k]);
    }
    launch_cut(pyr, cut[0], cut[1], st);
    CutIndex chunk_index{U64(P.c_start), U32(P.cut_idx[0]), 3 * (g - P.lt)};
    CutIndex wc_index{U64(P.w_start), U32(P.cut_idx[1]), 3 * (g - P.lt)};
    launch_wc_chunks(&ctrs->num_wc, P.maxW, U64(P.w_key), U8(P.w_level), g, pyr, chunk_index, U8(P.c_level),
                     &ctrs->num_chunks, P.maxC, U32(P.wc_chunk), U32(P.seg_b0), U32(P.seg_nb), U8(P.wc_nested),
                     ctrs->wc_flags, U32(P.w_count), p->leaf_capacity, s_, ctrs->lists_pre, st);
    t_cut.end(st);
    JCHK(hipMemcpyAsync(hctrs, ctrs, 256 + sizeof(DevBox), hipMemcpyDeviceToHost, st));   // counters and box
    JCHK(hipStreamSynchronize(st));
    if (hbox->nonfinite) {
        return end_job(fail(FPO_ERR_NONFINITE, "a coordinate is NaN or infinite"));
    }
    const uint32_t num_chunks = hctrs->num_chunks, num_wc = hctrs->num_wc;
    if (hctrs->internal_error || num_wc > P.maxW || num_chunks > P.maxC)
        return end_job(fail(FPO_ERR_DEVICE, "internal: %u chunks, %u work chunks exceed the plan", num_chunks, num_wc));

    // chunk begins (u64) and work-chunk begins
    t_chunk.begin(st);
    if (num_chunks <= SCAN_PAIR_MAX && num_wc <= SCAN_PAIR_MAX) {
        scan_exclusive_pair(U32(P.c_count), U32(P.c_count_scan), U64(P.c_begin), num_chunks, U32(P.w_count),
                            U32(P.w_begin), num_wc, st);
    } else {
        scan_exclusive(U32(P.c_count), U32(P.c_count_scan), num_chunks, nullptr, stemp, st);
        launch_u32_to_u64(U32(P.c_count_scan), U64(P.c_begin), num_chunks, st);
        scan_exclusive(U32(P.w_count), U32(P.w_begin), num_wc, nullptr, stemp, st);
    }

    // ---- step 3: stable scatter by chunk (perm) and by work chunk ----
    {
        MsInput in;
        in.code = U64(P.code);
        in.cut = chunk_index;
        in.code_shift = 3 * (KB - g);
        in.pay = U64(P.code);
        in.bucket_begin = U64(P.c_begin);   // the chunk begins: one pass, no counting pass
        in.err = &ctrs->internal_error;
        MsOutput o;
        o.vals = U32(P.perm);
        o.pay = U64(P.code_perm);
        // every point's work chunk, in chunk order, for the work-chunk split
        // (the subsample's node list buffer is free until then)
        o.cut2_keys = U32(P.big_nr);
        o.cut2 = wc_index;
        o.cut2_shift = 3 * (KB - P.lam_w);
        multisplit(in, n, num_chunks, o, ws + P.ms_temp, st);
    }
    t_chunk.end(st);
    // work-chunk order from perm order: chunk by chunk when every work chunk
    // lies inside one chunk (one pass, few buckets per chunk), else globally
    t_sub.begin(st);
    {
        MsInput in;
        in.keys = U32(P.big_nr);   // the work chunk of every point, written by the chunk split
        in.pay = U64(P.code_perm);
        MsOutput o;
        o.pay = U64(P.wc_code);
        if (hctrs->wc_flags[0] == 0 && hctrs->wc_flags[1] == 0) {
            MsSegments sg;
            sg.nseg = num_chunks;
            sg.begin = U32(P.c_count_scan);
            sg.len = U32(P.c_count);
            sg.b0 = U32(P.seg_b0);
            sg.nb = U32(P.seg_nb);
            sg.max_cells = n + num_wc;
            in.vals = U32(P.perm);   // original indices ride along
            o.vals = U32(P.wc_orig);
            multisplit_segmented(in, n, sg, (n + MS_SEG_TILE - 1) / MS_SEG_TILE + num_chunks, o, ws + P.ms_temp, st);
        } else {
            in.vals = U32(P.perm);
            o.vals = U32(P.wc_orig);
            multisplit(in, n, num_wc, o, ws + P.ms_temp, st);
        }
    }

    // ---- step 4: subsample ----
    WcArgs A{};
    A.num_wc = num_wc;
    A.wc_begin = U32(P.w_begin);
    A.wc_count = U32(P.w_count);
    A.wc_level = U8(P.w_level);
    A.wc_key = U64(P.w_key);
    A.wc_start = U64(P.w_start);
    A.wc_orig = U32(P.wc_orig);
    A.perm = U32(P.perm);
    A.wc_nested = U8(P.wc_nested);
    A.wc_code = U64(P.wc_code);
    A.t = U8(P.t);
    A.fr = U32(P.fr);
    A.alive = U32(P.alive);
    A.alive_scan = U32(P.alive_scan);
    A.kd = U32(P.kd);
    A.loff = U32(P.loff);
    A.lnode_key = U64(P.lnode_key);
    A.lnode_mask = U8(P.lnode_mask);
    A.cut = U8(P.cut);
    A.big_list = U32(P.big_list);
    A.num_big_dev = &ctrs->num_big;
    A.cls_list = U32(P.cls_list);
    A.cls_cnt = ctrs->cls_cnt;
    A.big_nr = U32(P.big_nr);
    A.big_node = U32(P.big_node);
    A.big_hkey = U64(P.big_hkey);
    A.big_hval = U32(P.big_hval);
    A.lam_w = P.lam_w;
    A.d0 = P.d0;
    A.s = s_;
    A.L = p->leaf_capacity;
    A.dmax = KB - s_;
    // every point alive (0xff) until a depth keeps it; the shared depths above
    // the work-chunk levels first, over all points (their first table is
    // cleared with the other two)
    {
        FillSpec f[4];
        f[0] = {U32(P.kd), 0u, (uint64_t)MAXD * num_wc};
        f[1] = {reinterpret_cast<uint32_t *>(U8(P.t)), 0xffffffffu, (n + 3) / 4};
        if (P.d0 > 0) f[2] = {global_depth_table(U32(P.gtab), U32(P.gtab2), P.d0, 0), 0xffffffffu, 1ull << (3 * P.s)};
        launch_fill_many(f, st);
    }
    launch_global_depths(A, n, U32(P.gtab), U32(P.gtab2), st, true);
    // only the lists the counters read back show non-empty are launched; a
    // general-class work chunk whose table overflows LDS joins the
    // global-memory list, so that list runs whenever a general class does
    launch_subsample_small(A, hctrs->lists_pre, st);
    bool big = hctrs->lists_pre[WC_CLASSES] != 0;
    for (int k = WC_GENERAL; k < WC_CLASSES; ++k) big = big || hctrs->lists_pre[k] != 0;
    if (big) launch_subsample_big(A, st);
    scan_exclusive(U32(P.alive), U32(P.alive_scan), (uint64_t)MAXD * num_wc, U32(P.alive_scan) + (uint64_t)MAXD * num_wc,
                   stemp, st);
    launch_decide(A, st);
    launch_node_counts(A, U32(P.owned), st);
    scan_exclusive(U32(P.owned), U32(P.node_base), (uint64_t)MAXD * num_wc, &ctrs->num_nodes, stemp, st);
    t_sub.end(st);
    // points per node (node_count) need no host count: enqueued before the
    // read-back, they keep the device busy while the host waits for it
    t_ncnt.begin(st);
    launch_np_counts(A, U32(P.node_base), U32(P.np_cnt), U32(P.np_scan), U32(P.n_count), U32(P.owned),
                     U32(P.np_glist), &ctrs->np_general, &ctrs->np_max, U8(P.np_single), stemp, st);
    t_ncnt.end(st);
    JCHK(hipMemcpyAsync(hctrs, ctrs, sizeof(Ctrs), hipMemcpyDeviceToHost, st));
    JCHK(hipStreamSynchronize(st));
    const uint32_t num_nodes = hctrs->num_nodes;
    if (num_nodes > NP_MAX_NODES) return end_job(fail(FPO_ERR_INVALID_ARG, "%u nodes: at most 2^31 - 1", num_nodes));
    t_place.begin(st);
    launch_fill_u32(U32(P.n_mask), 0u, (num_nodes + 3) / 4, st);
    launch_node_fill(A, U32(P.node_base), U8(P.n_depth), U64(P.n_key), U8(P.n_mask), st);
    // node_points: every point placed in its node's range, then each range
    // sorted by original index
    {
        NpWork w{};
        w.nb = U32(P.np_nb);
        w.tmp = U32(P.np_tmp);
        w.fill = U32(P.big_nr);
        w.general = hctrs->np_general > 0;
        w.err = &ctrs->internal_error;
        w.out = U32(P.n_points);
        w.lists.c0 = U32(P.np_l0);
        w.lists.c1 = U32(P.np_l1);
        w.lists.c2 = U32(P.np_l2);
        w.lists.c3 = U64(P.np_l3);
        w.lists.jobs = U64(P.np_jobs);
        w.lists.cp = U64(P.np_cp);
        w.lists.single = U8(P.np_single);
        w.lists.counts = ctrs->np_lists;
        w.scan_temp = stemp;
        w.place_timer = &t_place;
        w.sort_timer = &t_nsort;
        launch_np_points(A, U32(P.node_base), U32(P.owned), U32(P.np_cnt), U32(P.n_count), num_nodes, hctrs->np_max, n,
                         w, st);
    }
    launch_u32_to_u64(U32(P.np_nb), U64(P.n_begin), num_nodes, st);
    t_nsort.end(st);

    JCHK(hipMemcpyAsync(hctrs, ctrs, 256 + sizeof(DevBox), hipMemcpyDeviceToHost, st));   // counters and box
    JCHK(hipEventRecord(job->ev_done, st));
    JCHK(hipGetLastError());
    R.num_chunks = num_chunks;
    R.num_nodes = num_nodes;
    *out = job;
    return FPO_OK;
#undef JCHK
}

}  // namespace fpo

extern "C" {

fpo_status fpo_build_submit(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                            uint64_t workspace_bytes, void *hip_stream, fpo_job **out)
{
    if (!out) return fail(FPO_ERR_INVALID_ARG, "out is NULL");
    const fpo_status s = check_build(ctx, cloud, p, workspace, workspace_bytes);
    if (s != FPO_OK) return s;
    return queue_build(ctx, cloud, p, workspace, workspace_bytes,
                       hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream, out);
}

// A batch or server job first waits for its build to be submitted; its
// calls then act on the submitted build.
#define FPO_RESOLVE_(job, block, preview)                         \
    do {                                                          \
        if ((job)->def) {                                         \
            fpo_job *inner_ = nullptr;                            \
            const fpo_status r_ = deferred_resolve(job, block, preview, &inner_); \
            if (r_ != FPO_OK) return r_;                          \
            job = inner_;                                         \
        }                                                         \
    } while (0)
#define FPO_RESOLVE(job, block) FPO_RESOLVE_(job, block, false)

fpo_status fpo_job_preview_ready(fpo_job *job)
{
    if (!job) return fail(FPO_ERR_INVALID_ARG, "job is NULL");
    FPO_RESOLVE_(job, false, true);
    hipError_t e = hipEventQuery(job->ev_preview);
    if (e == hipSuccess) return FPO_OK;
    if (e == hipErrorNotReady) return FPO_NOT_READY;
    return fail(FPO_ERR_DEVICE, "hipEventQuery: %s", hipGetErrorString(e));
}

static fpo_status finish(fpo_job *job)
{
    if (!job->waited) {
        job->waited = true;
        job->t_done = now_ns();
        if (job->status == FPO_OK) {
            const Ctrs *hc = static_cast<const Ctrs *>(job->pinned);
            const DevBox *hb = reinterpret_cast<const DevBox *>(static_cast<const char *>(job->pinned) + 256);
            fpo_result &R = job->res;
            if (R.n > 0) {
                for (int a = 0; a < 3; ++a) {
                    R.bbox_min[a] = hb->lo[a];
                    R.bbox_max[a] = hb->hi[a];
                }
                R.cube_size = hb->size;
                R.scale = hb->scale;
                R.n_outside = hb->n_outside;
                R.preview_count = hc->preview_count;
                R.chunk_oversized_any = hc->oversized ? 1 : 0;
                if (job->small) {
                    // counted by the device: the host never saw them mid-build
                    R.num_chunks = hc->num_chunks;
                    R.num_nodes = hc->num_nodes;
                    if (hb->nonfinite) job->status = FPO_ERR_NONFINITE;
                }
                if (hc->internal_error && job->status == FPO_OK) job->status = FPO_ERR_DEVICE;
            }
        }
    }
    if (job->status == FPO_ERR_DEVICE) return fail(FPO_ERR_DEVICE, "internal error: a point was left without a node");
    if (job->status == FPO_ERR_NONFINITE) return fail(FPO_ERR_NONFINITE, "a coordinate is NaN or infinite");
    return job->status == FPO_OK ? FPO_OK : fail(job->status, "build failed (status %d)", (int)job->status);
}

fpo_status fpo_job_poll(fpo_job *job)
{
    if (!job) return fail(FPO_ERR_INVALID_ARG, "job is NULL");
    FPO_RESOLVE(job, false);
    hipError_t e = hipEventQuery(job->ev_done);
    if (e == hipErrorNotReady) return FPO_NOT_READY;
    if (e != hipSuccess) return fail(FPO_ERR_DEVICE, "hipEventQuery: %s", hipGetErrorString(e));
    return finish(job);
}

fpo_status fpo_job_wait(fpo_job *job)
{
    if (!job) return fail(FPO_ERR_INVALID_ARG, "job is NULL");
    FPO_RESOLVE(job, true);
    hipError_t e = hipEventSynchronize(job->ev_done);
    if (e != hipSuccess) return fail(FPO_ERR_DEVICE, "hipEventSynchronize: %s", hipGetErrorString(e));
    return finish(job);
}

fpo_status fpo_job_result(fpo_job *job, fpo_result *out)
{
    if (!job || !out) return fail(FPO_ERR_INVALID_ARG, "NULL job or out");
    FPO_RESOLVE(job, false);
    if (!job->waited) return fail(FPO_ERR_INVALID_ARG, "the job has not been waited for");
    if (job->status != FPO_OK) return fail(job->status, "the build failed");
    *out = job->res;
    return FPO_OK;
}

// Packed export layout (see include/fpo.h): {pointer, bytes} per array.
static void export_parts(const fpo_job *job, std::vector<std::pair<const void *, uint64_t>> &parts)
{
    const fpo_result &R = job->res;
    const uint64_t nc = R.num_chunks, nn = R.num_nodes, n = R.n;
    parts = {{R.count_grid, 4 * job->grid_cells}, {R.chunk_level, nc},     {R.chunk_key, 8 * nc},
             {R.chunk_count, 4 * nc},             {R.chunk_begin, 8 * nc}, {R.perm, 4 * n},
             {R.node_depth, nn},                  {R.node_key, 8 * nn},    {R.node_child_mask, nn},
             {R.node_begin, 8 * nn},              {R.node_count, 4 * nn},  {R.node_points, 4 * n},
             {R.preview_index, 4 * R.preview_count}};
}

}  // extern "C"

namespace fpo {

// Fingerprint of every array of a completed job (and of its scalars): equal
// for equal results.  Synchronous; allocates 8 bytes of device memory.
fpo_status job_fingerprint(fpo_job *job, uint64_t *out)
{
    FPO_RESOLVE(job, false);
    if (!job->waited || job->status != FPO_OK) return fail(FPO_ERR_INVALID_ARG, "the job has not completed");
    HIPCHK(hipSetDevice(job->ctx->device));
    std::vector<std::pair<const void *, uint64_t>> parts;
    export_parts(job, parts);
    uint64_t *acc = nullptr;
    HIPCHK(hipMalloc(&acc, sizeof(uint64_t)));
    hipStream_t st = job->ctx->stream;
    launch_fill_u32(reinterpret_cast<uint32_t *>(acc), 0u, 2, st);
    uint64_t salt = 0;
    for (auto &pr : parts) launch_fingerprint(pr.first, pr.second, (salt += 0x9E3779B97F4A7C15ull), acc, st);
    uint64_t h = 0;
    hipError_t e = hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(acc);
    if (e != hipSuccess) return fail(FPO_ERR_DEVICE, "fingerprint: %s", hipGetErrorString(e));
    const fpo_result &R = job->res;
    uint32_t sc[8];
    memcpy(sc, R.bbox_min, 12);
    memcpy(sc + 3, R.bbox_max, 12);
    memcpy(sc + 6, &R.cube_size, 4);
    memcpy(sc + 7, &R.scale, 4);
    for (int i = 0; i < 8; ++i) h = (h ^ sc[i]) * 0x100000001B3ull;
    h = (h ^ R.num_chunks ^ ((uint64_t)R.num_nodes << 32)) * 0x100000001B3ull;
    h = (h ^ R.preview_count ^ (R.n_outside << 20)) * 0x100000001B3ull;
    *out = h;
    return FPO_OK;
}

}  // namespace fpo

extern "C" {

fpo_status fpo_job_export_bytes(fpo_job *job, uint64_t *bytes)
{
    if (!job || !bytes) return fail(FPO_ERR_INVALID_ARG, "NULL job or bytes");
    FPO_RESOLVE(job, false);
    if (!job->waited || job->status != FPO_OK) return fail(FPO_ERR_INVALID_ARG, "the job has not completed");
    std::vector<std::pair<const void *, uint64_t>> parts;
    export_parts(job, parts);
    uint64_t off = 0;
    for (auto &pr : parts) off = ((off + 7) & ~7ull) + pr.second;
    *bytes = off;
    return FPO_OK;
}

fpo_status fpo_job_copy_to_host(fpo_job *job, void *host_dst, uint64_t bytes)
{
    if (!job || !host_dst) return fail(FPO_ERR_INVALID_ARG, "NULL job or destination");
    uint64_t need = 0;
    fpo_status s = fpo_job_export_bytes(job, &need);
    if (s != FPO_OK) return s;
    if (bytes < need) return fail(FPO_ERR_INVALID_ARG, "destination holds %llu bytes, the export needs %llu",
                                  (unsigned long long)bytes, (unsigned long long)need);
    FPO_RESOLVE(job, false);
    HIPCHK(hipSetDevice(job->ctx->device));
    std::vector<std::pair<const void *, uint64_t>> parts;
    export_parts(job, parts);
    uint64_t off = 0;
    for (auto &pr : parts) {
        off = (off + 7) & ~7ull;
        // synchronous copies: the job's stream may already run another build
        if (pr.second) HIPCHK(hipMemcpy(static_cast<char *>(host_dst) + off, pr.first, pr.second, hipMemcpyDeviceToHost));
        off += pr.second;
    }
    return FPO_OK;
}

fpo_status fpo_job_gather(fpo_job *job, const fpo_cloud *cloud, const uint8_t *color, uint32_t color_stride,
                          float *out_xyz, uint8_t *out_color, void *hip_stream)
{
    if (!job || !cloud || (cloud->n && !out_xyz)) return fail(FPO_ERR_INVALID_ARG, "NULL job, cloud or output");
    if ((color_stride > 0) != (color != nullptr) || (color_stride > 0 && !out_color) || color_stride > 64)
        return fail(FPO_ERR_INVALID_ARG, "colour: pass the array, a stride of 1..64 and the output together");
    fpo_context *ctx = job->ctx;
    FPO_RESOLVE(job, false);
    if (!job->waited || job->status != FPO_OK) return fail(FPO_ERR_INVALID_ARG, "the job has not completed");
    if (cloud->n != job->res.n) return fail(FPO_ERR_INVALID_ARG, "the cloud has %llu points, the build %llu",
                                            (unsigned long long)cloud->n, (unsigned long long)job->res.n);
    if (cloud->n && (!cloud->x || !cloud->y || !cloud->z)) return fail(FPO_ERR_INVALID_ARG, "NULL coordinate array");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream;
    launch_gather_points(job->res.node_points, cloud->n, cloud->x, cloud->y, cloud->z, color, color_stride, out_xyz,
                         out_color, st);
    HIPCHK(hipGetLastError());
    return FPO_OK;
}

fpo_status fpo_job_write_file(fpo_job *job, const fpo_cloud *cloud, const uint8_t *color, uint32_t color_stride,
                              const char *path)
{
    if (!job || !cloud || !path) return fail(FPO_ERR_INVALID_ARG, "NULL job, cloud or path");
    fpo_job *pub = job;
    FPO_RESOLVE(job, false);
    if (!job->waited || job->status != FPO_OK) return fail(FPO_ERR_INVALID_ARG, "the job has not completed");
    const fpo_result &R = job->res;
    const uint64_t n = R.n;
    // node table and points to the host
    std::vector<uint8_t> depth(R.num_nodes), mask(R.num_nodes);
    std::vector<uint32_t> count(R.num_nodes);
    std::vector<uint64_t> key(R.num_nodes), begin(R.num_nodes);
    HIPCHK(hipSetDevice(job->ctx->device));
    if (R.num_nodes) {
        HIPCHK(hipMemcpy(depth.data(), R.node_depth, R.num_nodes, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(mask.data(), R.node_child_mask, R.num_nodes, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(count.data(), R.node_count, 4ull * R.num_nodes, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(key.data(), R.node_key, 8ull * R.num_nodes, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(begin.data(), R.node_begin, 8ull * R.num_nodes, hipMemcpyDeviceToHost));
    }
    std::vector<float> xyz(3 * n);
    std::vector<uint8_t> col((uint64_t)color_stride * n);
    if (n) {
        float *d_xyz = nullptr;
        uint8_t *d_col = nullptr;
        HIPCHK(hipMalloc(&d_xyz, 12 * n));
        if (color_stride && hipMalloc(&d_col, (uint64_t)color_stride * n) != hipSuccess) {
            (void)hipFree(d_xyz);
            return fail(FPO_ERR_OUT_OF_MEMORY, "device memory for the colours");
        }
        fpo_status s = fpo_job_gather(pub, cloud, color, color_stride, d_xyz, d_col, nullptr);
        hipError_t e = hipSuccess;
        if (s == FPO_OK) {
            e = hipStreamSynchronize(job->ctx->stream);
            if (e == hipSuccess) e = hipMemcpy(xyz.data(), d_xyz, 12 * n, hipMemcpyDeviceToHost);
            if (e == hipSuccess && color_stride) e = hipMemcpy(col.data(), d_col, col.size(), hipMemcpyDeviceToHost);
        }
        (void)hipFree(d_xyz);
        if (d_col) (void)hipFree(d_col);
        if (s != FPO_OK) return s;
        if (e != hipSuccess) return fail(FPO_ERR_DEVICE, "gather: %s", hipGetErrorString(e));
    }
    FILE *f = fopen(path, "wb");
    if (!f) return fail(FPO_ERR_INVALID_ARG, "cannot open %s for writing", path);
    bool ok = true;
    auto put = [&](const void *p, size_t b) { ok = ok && (b == 0 || fwrite(p, 1, b, f) == b); };
    const uint32_t version = 1, nn = R.num_nodes, cs = color_stride;
    const uint32_t G = job->params.count_grid, S = job->params.subsample_grid;
    put("FPO1", 4);
    put(&version, 4);
    put(&n, 8);
    put(&nn, 4);
    put(&cs, 4);
    put(R.bbox_min, 12);
    put(&R.cube_size, 4);
    put(&G, 4);
    put(&S, 4);
    for (uint32_t k = 0; k < nn; ++k) {
        const uint16_t zero = 0;
        put(&depth[k], 1);
        put(&mask[k], 1);
        put(&zero, 2);
        put(&count[k], 4);
        put(&key[k], 8);
        put(&begin[k], 8);
    }
    put(xyz.data(), 12 * n);
    put(col.data(), col.size());
    if (fclose(f) != 0) ok = false;
    return ok ? FPO_OK : fail(FPO_ERR_INVALID_ARG, "writing %s failed", path);
}

fpo_status fpo_job_timestamps(fpo_job *job, uint64_t *submitted_ns, uint64_t *started_ns, uint64_t *completed_ns)
{
    if (!job) return fail(FPO_ERR_INVALID_ARG, "job is NULL");
    uint64_t sub = job->t_submit, start = job->t_submit, end = 0;
    if (job->def) {
        start = deferred_start_ns(job);
        end = deferred_end_ns(job);
        FPO_RESOLVE(job, false);
    }
    if (!job->waited) return fail(FPO_ERR_INVALID_ARG, "the job has not completed");
    if (submitted_ns) *submitted_ns = sub;
    if (started_ns) *started_ns = start;
    if (completed_ns) *completed_ns = end ? end : job->t_done;
    return FPO_OK;
}

fpo_status fpo_job_get_stats(fpo_job *job, fpo_job_stats *out)
{
    if (!job || !out) return fail(FPO_ERR_INVALID_ARG, "NULL job or out");
    fpo_job_stats st;
    memset(&st, 0, sizeof(st));
    const fpo_status ts = fpo_job_timestamps(job, &st.submitted_ns, &st.started_ns, &st.completed_ns);
    if (ts != FPO_OK) return ts;
    FPO_RESOLVE(job, false);
    if (!job->waited || job->status != FPO_OK) return fail(FPO_ERR_INVALID_ARG, "the job has not completed");
    const fpo_result &R = job->res;
    st.n = R.n;
    st.num_chunks = R.num_chunks;
    st.num_nodes = R.num_nodes;
    st.chunk_oversized_any = R.chunk_oversized_any;
    st.n_outside = R.n_outside;
    st.preview_count = R.preview_count;
    st.workspace_bytes = job->plan_bytes;
    if (R.num_nodes) {
        // nodes are listed by depth: the last one is the deepest
        uint8_t d = 0;
        HIPCHK(hipSetDevice(job->ctx->device));
        HIPCHK(hipMemcpy(&d, R.node_depth + (R.num_nodes - 1), 1, hipMemcpyDeviceToHost));
        st.max_depth = d;
    }
    static_assert(FPO_TIMER_COUNT <= 16, "region_ms holds every timer");
    for (int t = 0; t < 16; ++t) st.region_ms[t] = -1.0f;
    if (job->timed)
        for (int t = 0; t < FPO_TIMER_COUNT; ++t) {
            if (!((job->timer_mask >> t) & 1u)) continue;
            float total = 0.0f;
            for (auto &pr : job->tm[t]) {
                float v = 0.0f;
                HIPCHK(hipEventElapsedTime(&v, pr.first, pr.second));
                total += v;
            }
            st.region_ms[t] = total;
        }
    *out = st;
    return FPO_OK;
}

void fpo_job_release(fpo_job *job)
{
    if (!job) return;
    if (job->def) {
        deferred_release(job);
        return;
    }
    (void)hipEventSynchronize(job->ev_done);
    (void)hipEventDestroy(job->ev_preview);
    (void)hipEventDestroy(job->ev_done);
    for (hipEvent_t e : job->stream_events) (void)hipEventDestroy(e);
    if (job->pinned) put_pinned(job->ctx, job->pinned);
    {
        std::lock_guard<std::mutex> g(job->ctx->mu);
        for (auto &v : job->tm)
            for (auto &pr : v) {
                job->ctx->ev_free.push_back(pr.first);
                job->ctx->ev_free.push_back(pr.second);
            }
    }
    delete job;
}

fpo_status fpo_context_set_single_block_max(fpo_context *ctx, uint32_t plain_max, uint32_t batch_max)
{
    if (!ctx) return fail(FPO_ERR_INVALID_ARG, "context is NULL");
    if (plain_max > SB_MAX_N || batch_max > SB_MAX_N)
        return fail(FPO_ERR_INVALID_ARG, "limits must be at most %u (got %u, %u)", SB_MAX_N, plain_max, batch_max);
    ctx->small_max.store(plain_max);
    ctx->small_max_batch.store(batch_max);
    return FPO_OK;
}

fpo_status fpo_context_set_timing(fpo_context *ctx, int enable)
{
    return fpo_context_set_timers(ctx, enable ? (1u << FPO_TIMER_COUNT) - 1u : 0u);
}

fpo_status fpo_context_set_timers(fpo_context *ctx, uint32_t mask)
{
    if (!ctx) return fail(FPO_ERR_INVALID_ARG, "context is NULL");
    if (mask >> FPO_TIMER_COUNT) return fail(FPO_ERR_INVALID_ARG, "unknown timers in mask 0x%x", mask);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->timing = mask != 0;
    ctx->timer_mask = mask;
    return FPO_OK;
}

fpo_status fpo_job_timer(fpo_job *job, fpo_timer which, float *ms, uint32_t *launches)
{
    if (!job) return fail(FPO_ERR_INVALID_ARG, "job is NULL");
    FPO_RESOLVE(job, false);
    if ((int)which < 0 || (int)which >= FPO_TIMER_COUNT) return fail(FPO_ERR_INVALID_ARG, "unknown timer %d", (int)which);
    if (!job->timed) return fail(FPO_ERR_INVALID_ARG, "the job was submitted without timing");
    if (!job->waited || job->status != FPO_OK) return fail(FPO_ERR_INVALID_ARG, "the job has not completed");
    float total = 0.0f;
    for (auto &pr : job->tm[which]) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, pr.first, pr.second));
        total += t;
    }
    if (ms) *ms = total;
    if (launches) *launches = (uint32_t)job->tm[which].size();
    return FPO_OK;
}

}  // extern "C"
