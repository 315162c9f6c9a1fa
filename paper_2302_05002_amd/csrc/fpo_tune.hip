// Autotuning of libfpo: the choices below change only how fast a build runs,
// never its result, and are picked by timing the candidates on the caller's
// own clouds.
//
//  - The quantise + count pass's shape (fpo_internal.h, QZ_VARIANTS): block
//    size and LDS hash-table slots.  Per size class (log2 n) and count grid.
//  - The number of worker streams of batched builds.
//
// The tuner builds the cloud once per candidate (plus repetitions for the
// timing), checks that every candidate's result has the same fingerprint as
// the first candidate's (a mismatch is reported as an internal error), and
// records the fastest in the context.  With FPO_AUTOTUNE_CACHE set, the table
// is read when a context is created and written after every tuning call
// (text: "qz <log2 n> <log2 G> <variant>" and "batch_workers <w>" lines).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "fpo_host.h"
#include "fpo_internal.h"

using namespace fpo;

namespace {

int ilog2_floor(uint64_t v)
{
    int l = 0;
    while (v > 1) {
        v >>= 1;
        ++l;
    }
    return l;
}

int ilog2_ceil(uint32_t v)
{
    int l = 0;
    while ((1u << l) < v) ++l;
    return l;
}

void tune_cache_save(fpo_context *c)
{
    const char *path = getenv("FPO_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "fpo-autotune 1\n");
    {
        std::lock_guard<std::mutex> g(c->mu);
        for (int k = 0; k < 33; ++k)
            for (int gl = 0; gl < 10; ++gl)
                if (c->qz_variant[k][gl] != 0xff) fprintf(f, "qz %d %d %d\n", k, gl, (int)c->qz_variant[k][gl]);
        fprintf(f, "batch_workers %d\n", c->batch_workers);
    }
    const bool ok = fclose(f) == 0;
    if (ok) (void)rename(tmp.c_str(), path);
}

double median(std::vector<double> v)
{
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0 : v[v.size() / 2];
}

struct TimingGuard {   // the context's own timing settings, restored on exit
    fpo_context *c;
    bool timing;
    uint32_t mask;
    uint32_t small_max, small_max_batch;
    explicit TimingGuard(fpo_context *ctx) : c(ctx)
    {
        std::lock_guard<std::mutex> g(c->mu);
        timing = c->timing;
        mask = c->timer_mask;
        small_max = c->small_max.load();
        small_max_batch = c->small_max_batch.load();
    }
    ~TimingGuard()
    {
        std::lock_guard<std::mutex> g(c->mu);
        c->timing = timing;
        c->timer_mask = mask;
        c->qz_force = -1;
        c->small_max.store(small_max);
        c->small_max_batch.store(small_max_batch);
    }
};

}  // namespace

namespace fpo {

int quantize_variant(fpo_context *c, uint64_t n, int g)
{
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->qz_force >= 0) return c->qz_force;
    const uint8_t v = c->qz_variant[ilog2_floor(n ? n : 1)][g];
    // untuned: the binned pass for the 2^27-cell grid (G = 512), else shape 0
    return v < QZ_VARIANTS ? v : g >= 9 ? QZ_BINNED : 0;
}

void tune_cache_load(fpo_context *c)
{
    const char *path = getenv("FPO_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[128];
    while (fgets(line, sizeof(line), f)) {
        int k, gl, v;
        if (sscanf(line, "qz %d %d %d", &k, &gl, &v) == 3) {
            if (k >= 0 && k < 33 && gl >= 0 && gl < 10 && v >= 0 && v < QZ_VARIANTS) c->qz_variant[k][gl] = (uint8_t)v;
        } else if (sscanf(line, "batch_workers %d", &v) == 1) {
            if (v >= 1 && v <= 16) c->batch_workers = v;
        }
    }
    fclose(f);
}

}  // namespace fpo

extern "C" {

fpo_status fpo_context_force_quantize_variant(fpo_context *ctx, int variant)
{
    if (!ctx) return fail(FPO_ERR_INVALID_ARG, "context is NULL");
    if (variant < -1 || variant >= QZ_VARIANTS)
        return fail(FPO_ERR_INVALID_ARG, "variant must be -1 or 0..%d (got %d)", QZ_VARIANTS - 1, variant);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->qz_force = variant;
    return FPO_OK;
}

fpo_status fpo_autotune(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                        uint64_t workspace_bytes, uint32_t reps, fpo_tuning *out)
{
    if (!ctx || !cloud || !p || !out) return fail(FPO_ERR_INVALID_ARG, "NULL context, cloud, params or out");
    if (reps < 1 || reps > 100) return fail(FPO_ERR_INVALID_ARG, "reps must be in 1..100 (got %u)", reps);
    if (p->flags & FPO_PREVIEW_GRID) return fail(FPO_ERR_INVALID_ARG, "the grid preview has a single shape");
    const fpo_status chk = check_params(cloud->n, p);
    if (chk != FPO_OK) return chk;
    if (cloud->n == 0) return fail(FPO_ERR_INVALID_ARG, "nothing to tune on an empty cloud");
    TimingGuard guard(ctx);
    // the shapes are those of the multi-kernel path, also for a cloud that
    // would take the single-workgroup one
    ctx->small_max.store(0);
    memset(out, 0, sizeof(*out));
    uint64_t ref = 0;
    // the binned pass (the last variant) needs device input and a count grid
    // of 2^24 cells or more; it also spares the bounding-box pass the
    // clearing of the grid, so every shape is timed over both regions
    const bool binned_ok = cloud->location == FPO_DEVICE && quantize_binned_ok(cloud->n, ilog2_ceil(p->count_grid));
    const int nv = binned_ok ? QZ_VARIANTS : QZ_BINNED;
    for (int v = 0; v < nv; ++v) {
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            ctx->qz_force = v;
            ctx->timing = true;
            ctx->timer_mask = 1u << FPO_TIMER_QUANTIZE | 1u << FPO_TIMER_BBOX;
        }
        std::vector<double> ms;
        for (uint32_t r = 0; r <= reps; ++r) {   // the first build also warms up the shape
            fpo_job *job = nullptr;
            fpo_status s = fpo_build_submit(ctx, cloud, p, workspace, workspace_bytes, nullptr, &job);
            if (s != FPO_OK) return s;
            s = fpo_job_wait(job);
            float t = 0.0f, tb = 0.0f;
            if (s == FPO_OK) s = fpo_job_timer(job, FPO_TIMER_QUANTIZE, &t, nullptr);
            if (s == FPO_OK) s = fpo_job_timer(job, FPO_TIMER_BBOX, &tb, nullptr);
            t += tb;
            if (s == FPO_OK && r == 0) {
                uint64_t fp = 0;
                s = job_fingerprint(job, &fp);
                if (s == FPO_OK && v == 0) ref = fp;
                if (s == FPO_OK && fp != ref)
                    s = fail(FPO_ERR_DEVICE, "internal: quantise variant %d changed the result", v);
            }
            const std::string err = s == FPO_OK ? std::string() : error_text();
            fpo_job_release(job);
            if (s != FPO_OK) return fail(s, "%s", err.c_str());
            if (r) ms.push_back(t);
        }
        out->quantize_ms[v] = (float)median(ms);
    }
    int best = 0;
    for (int v = 1; v < nv; ++v)
        if (out->quantize_ms[v] < out->quantize_ms[best]) best = v;
    const int k = ilog2_floor(cloud->n), gl = ilog2_ceil(p->count_grid);
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->qz_variant[k][gl] = (uint8_t)best;
    }
    out->quantize_variant = (uint32_t)best;
    out->size_class = (uint32_t)k;
    out->count_grid_log2 = (uint32_t)gl;
    out->candidates = (uint32_t)nv;
    tune_cache_save(ctx);
    return FPO_OK;
}

fpo_status fpo_autotune_batch(fpo_context *ctx, const fpo_cloud *clouds, const fpo_params *params, uint32_t count,
                              void *workspace, uint64_t workspace_bytes, uint32_t reps, uint32_t *workers_out,
                              float *ms_out)
{
    if (!ctx || !workers_out || !count || !clouds || !params)
        return fail(FPO_ERR_INVALID_ARG, "NULL argument or empty batch");
    if (reps < 1 || reps > 100) return fail(FPO_ERR_INVALID_ARG, "reps must be in 1..100 (got %u)", reps);
    static const uint32_t cand[] = {2, 4, 8};
    constexpr int NC = (int)(sizeof(cand) / sizeof(cand[0]));
    uint32_t before;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        before = (uint32_t)ctx->batch_workers;
    }
    std::vector<uint64_t> ref(count, 0);
    std::vector<fpo_job *> jobs(count, nullptr);
    double best_ms = 0.0;
    uint32_t best = before;
    for (int c = 0; c < NC; ++c) {
        fpo_status s = fpo_context_set_batch_workers(ctx, cand[c]);
        if (s != FPO_OK) return s;
        std::vector<double> ms;
        for (uint32_t r = 0; r <= reps; ++r) {
            const uint64_t t0 = now_ns();
            s = fpo_build_batch(ctx, clouds, params, count, workspace, workspace_bytes, nullptr, jobs.data());
            if (s != FPO_OK) {
                (void)fpo_context_set_batch_workers(ctx, before);
                return s;
            }
            fpo_status bad = FPO_OK;
            std::string err;
            for (uint32_t i = 0; i < count; ++i) {
                const fpo_status w = fpo_job_wait(jobs[i]);
                if (w != FPO_OK && bad == FPO_OK) {
                    bad = w;
                    err = error_text();
                }
            }
            const uint64_t t1 = now_ns();
            for (uint32_t i = 0; bad == FPO_OK && r == 0 && i < count; ++i) {
                uint64_t fp = 0;
                fpo_status f = job_fingerprint(jobs[i], &fp);
                if (f == FPO_OK && c == 0) ref[i] = fp;
                if (f == FPO_OK && fp != ref[i]) f = fail(FPO_ERR_DEVICE, "internal: %u workers changed cloud %u", cand[c], i);
                if (f != FPO_OK) {
                    bad = f;
                    err = error_text();
                }
            }
            for (uint32_t i = 0; i < count; ++i) fpo_job_release(jobs[i]);
            if (bad != FPO_OK) {
                (void)fpo_context_set_batch_workers(ctx, before);
                return fail(bad, "%s", err.c_str());
            }
            if (r) ms.push_back((t1 - t0) / 1e6);
        }
        const double m = median(ms);
        if (ms_out) ms_out[c] = (float)m;
        if (c == 0 || m < best_ms) {
            best_ms = m;
            best = cand[c];
        }
    }
    (void)fpo_context_set_batch_workers(ctx, best);
    *workers_out = best;
    tune_cache_save(ctx);
    return FPO_OK;
}

}  // extern "C"
