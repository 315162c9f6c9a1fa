// Executors of libfpo: worker threads that run plain builds on HIP streams of
// their own, for batched builds (fpo_build_batch) and for the request server
// (fpo_server_*), and the server's device memory arena.
//
// Lifetimes: every job holds a reference to its context (and a served job one
// to its server), so handles may be released in any order; destroying a
// context or a server only drops the owner's reference and never blocks.  The
// last release tears the object down.  Waits on other host threads are
// bounded by wait_limit() and end with FPO_ERR_TIMEOUT.
//
// Small and mid-sized builds are latency bound: a few dozen short kernels
// and two short host round trips each.  Running several on separate streams
// keeps the device busy while one build waits for the host, and lets the
// kernels of different builds share the compute units.  Jobs are handed out
// before their build starts; every job call first waits for that start.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "fpo_host.h"
#include "fpo_internal.h"
#include "fpo_sched.h"

namespace fpo {

struct Server;

struct Deferred {
    // QUEUED -> RUNNING -> PREVIEW (preview kernels enqueued, inner known)
    // -> SUBMITTED (whole build enqueued; server jobs: ended) or FAILED
    enum State { QUEUED, RUNNING, PREVIEW, SUBMITTED, FAILED, CANCELLED };
    std::mutex m;
    std::condition_variable cv;
    State state = QUEUED;
    fpo_job *inner = nullptr;     // the plain build, once submitted
    fpo_status status = FPO_OK;
    std::string err;
    fpo_cloud cloud{};
    fpo_params params{};
    void *ws = nullptr;
    uint64_t ws_bytes = 0;
    hipEvent_t after = nullptr;   // the build waits for it (work the caller enqueued before the batch)
    hipStream_t stream = nullptr; // the caller's stream (plain builds); else the worker's
    Pool *pool = nullptr;         // batch pool the job is queued in
    Server *server = nullptr;
    uint64_t arena_off = 0;
    bool has_memory = false;
    uint64_t t_start = 0;
    uint64_t t_end = 0;           // server jobs: when the slot saw the build end
    // a queue entry for single-workgroup builds launched together: the jobs
    // of those clouds (not queued themselves); the entry is internal and
    // deleted once it ran
    std::vector<fpo_job *> group;
};

struct Pool {
    fpo_context *ctx = nullptr;
    Server *server = nullptr;     // the server whose slots these workers are, or null (batch)
    std::mutex m;
    std::condition_variable cv;
    std::deque<fpo_job *> q;
    std::vector<std::thread> threads;
    std::vector<hipStream_t> streams;
    bool stop = false;
};

struct Server {
    Server(uint64_t budget_, uint32_t slots) : budget(budget_), adm(budget_, slots) {}
    std::atomic<int> refs{1};   // the owner's plus one per job submitted
    fpo_context *ctx = nullptr;
    uint64_t budget = 0;
    char *arena = nullptr;
    std::mutex m;
    std::condition_variable cv;
    Admission<fpo_job *> adm;   // arena, waiting requests (FIFO), running builds (under m)
    Pool *pool = nullptr;
};

}  // namespace fpo

struct fpo_server : fpo::Server {
    using fpo::Server::Server;
};

namespace fpo {

namespace {

inline uint64_t a256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

void server_finished(Server *S);

// Runs a group entry: every member's build in one launch.  A member is
// never queued itself, so it cannot be cancelled, and its release waits
// until this has set its final state.
void run_group(Pool *P, fpo_job *entry, hipStream_t st)
{
    std::vector<fpo_job *> mem;
    mem.swap(entry->def->group);
    delete entry->def;
    delete entry;
    const uint64_t t0 = now_ns();
    std::vector<const fpo_cloud *> clouds;
    std::vector<const fpo_params *> params;
    std::vector<void *> ws;
    for (fpo_job *j : mem) {
        Deferred *d = j->def;
        {
            std::lock_guard<std::mutex> g(d->m);
            d->state = Deferred::RUNNING;
            d->t_start = t0;
        }
        if (d->after) (void)hipStreamWaitEvent(st, d->after, 0);
        clouds.push_back(&d->cloud);
        params.push_back(&d->params);
        ws.push_back(d->ws);
    }
    std::vector<fpo_job *> inner(mem.size(), nullptr);
    const fpo_status s = issue_small_group(P->ctx, (uint32_t)mem.size(), clouds.data(), params.data(), ws.data(), st,
                                           inner.data());
    const std::string err = s == FPO_OK ? std::string() : error_text();
    for (size_t k = 0; k < mem.size(); ++k) {
        Deferred *d = mem[k]->def;
        std::lock_guard<std::mutex> g(d->m);
        d->inner = inner[k];
        d->status = s;
        d->err = err;
        d->state = s == FPO_OK ? Deferred::SUBMITTED : Deferred::FAILED;
        d->cv.notify_all();
    }
}

void run_job(Pool *P, fpo_job *job, hipStream_t st)
{
    Deferred *d = job->def;
    if (!d->group.empty()) {
        run_group(P, job, st);
        return;
    }
    {
        std::lock_guard<std::mutex> g(d->m);
        if (d->state == Deferred::CANCELLED) return;
        d->state = Deferred::RUNNING;
        d->t_start = now_ns();
    }
    if (d->stream) st = d->stream;
    if (d->after) (void)hipStreamWaitEvent(st, d->after, 0);
    fpo_job *inner = nullptr;
    const fpo_status s = issue_build(P->ctx, &d->cloud, &d->params, d->ws, d->ws_bytes, st, &inner,
                                     [d](fpo_job *j) {
                                         std::lock_guard<std::mutex> g(d->m);
                                         d->inner = j;
                                         d->state = Deferred::PREVIEW;
                                         d->cv.notify_all();
                                     });
    const std::string err = s == FPO_OK ? std::string() : error_text();
    // a server slot stays taken until its build has ended
    uint64_t t_end = 0;
    if (s == FPO_OK && P->server) {
        (void)hipEventSynchronize(inner->ev_done);
        t_end = now_ns();
    }
    {
        // notified under the lock: once a releaser sees the final state, this
        // thread no longer touches the job
        std::lock_guard<std::mutex> g(d->m);
        if (inner) d->inner = inner;   // (a build that failed after its preview keeps the published job)
        d->status = s;
        d->err = err;
        d->t_end = t_end;
        d->state = s == FPO_OK ? Deferred::SUBMITTED : Deferred::FAILED;
        d->cv.notify_all();
    }
    if (P->server) server_finished(P->server);
}

void worker(Pool *P, int idx)
{
    (void)hipSetDevice(P->ctx->device);
    const hipStream_t st = P->streams[idx];
    for (;;) {
        fpo_job *job;
        {
            std::unique_lock<std::mutex> lk(P->m);
            P->cv.wait(lk, [&] { return P->stop || !P->q.empty(); });
            if (P->q.empty()) return;   // stopping, nothing left
            job = P->q.front();
            P->q.pop_front();
        }
        run_job(P, job, st);
    }
}

Pool *make_pool(fpo_context *ctx, Server *server, int workers)
{
    Pool *P = new Pool();
    P->ctx = ctx;
    P->server = server;
    for (int i = 0; i < workers; ++i) {
        hipStream_t st = nullptr;
        if (alloc_fault(ctx) || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) break;
        P->streams.push_back(st);
    }
    if ((int)P->streams.size() < workers) {
        for (hipStream_t st : P->streams) (void)hipStreamDestroy(st);
        delete P;
        return nullptr;
    }
    for (size_t i = 0; i < P->streams.size(); ++i) P->threads.emplace_back(worker, P, (int)i);
    return P;
}

void stop_pool(Pool *P)
{
    if (!P) return;
    {
        std::lock_guard<std::mutex> g(P->m);
        P->stop = true;
    }
    P->cv.notify_all();
    for (auto &t : P->threads) t.join();
    for (hipStream_t st : P->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    delete P;
}

void pool_push(Pool *P, fpo_job *job)
{
    {
        std::lock_guard<std::mutex> g(P->m);
        P->q.push_back(job);
    }
    P->cv.notify_one();
}

bool pool_remove(Pool *P, fpo_job *job)
{
    std::lock_guard<std::mutex> g(P->m);
    auto it = std::find(P->q.begin(), P->q.end(), job);
    if (it == P->q.end()) return false;
    P->q.erase(it);
    return true;
}

// Admits waiting requests in arrival order while a slot and memory are free
// (the head waits for memory rather than being overtaken).  S->m held.
void try_admit(Server *S)
{
    S->adm.admit([S](fpo_job *j, uint64_t off) {
        Deferred *d = j->def;
        d->arena_off = off;
        d->ws = S->arena + off;
        d->has_memory = true;
        pool_push(S->pool, j);
    });
}

void server_finished(Server *S)
{
    {
        std::lock_guard<std::mutex> g(S->m);
        S->adm.finished();
        try_admit(S);
    }
    S->cv.notify_all();
}

bool server_remove_waiting(Server *S, fpo_job *job)
{
    std::lock_guard<std::mutex> g(S->m);
    if (!S->adm.remove_waiting(job)) return false;
    S->cv.notify_all();
    return true;
}

fpo_job *new_deferred_job(fpo_context *ctx)
{
    ctx_retain(ctx);   // dropped by deferred_release (or free_unqueued)
    fpo_job *job = new fpo_job();
    job->ctx = ctx;
    job->stream = nullptr;
    job->ev_preview = job->ev_done = nullptr;
    job->pinned = nullptr;
    job->status = FPO_OK;
    job->waited = false;
    job->timed = false;
    job->t_submit = now_ns();
    job->t_done = 0;
    job->def = new Deferred();
    return job;
}

// A job that was never queued (an error before the batch was handed over).
void free_unqueued(fpo_job *job)
{
    fpo_context *ctx = job->ctx;
    if (job->def->after) (void)hipEventDestroy(job->def->after);
    delete job->def;
    delete job;
    ctx_release(ctx);
}

void server_release(Server *S)
{
    if (S->refs.fetch_sub(1) != 1) return;
    // last reference: the owner destroyed the server and every job of it has
    // been released, so nothing waits, runs or holds arena memory
    fpo_context *ctx = S->ctx;
    stop_pool(S->pool);
    (void)hipSetDevice(ctx->device);
    (void)hipFree(S->arena);
    delete static_cast<fpo_server *>(S);
    ctx_release(ctx);
}

fpo_status check_cloud(const fpo_cloud *c, const fpo_params *p)
{
    if (!c || !p) return fail(FPO_ERR_INVALID_ARG, "NULL cloud or params");
    const fpo_status s = check_params(c->n, p);
    if (s != FPO_OK) return s;
    if (c->n > 0 && (!c->x || !c->y || !c->z)) return fail(FPO_ERR_INVALID_ARG, "NULL coordinate array");
    return FPO_OK;
}

// Takes a job that has not started out of its queue; false if it started.
bool cancel_queued(fpo_job *job)
{
    Deferred *d = job->def;
    bool removed = false;
    if (d->server) removed = server_remove_waiting(d->server, job);
    else if (d->pool) removed = pool_remove(d->pool, job);
    if (!removed) return false;
    {
        std::lock_guard<std::mutex> g(d->m);
        d->state = Deferred::CANCELLED;
        d->status = FPO_ERR_CANCELLED;
        d->cv.notify_all();
    }
    return true;
}

}  // namespace

fpo_status deferred_resolve(fpo_job *job, bool block, bool preview, fpo_job **inner)
{
    Deferred *d = job->def;
    std::unique_lock<std::mutex> lk(d->m);
    auto pending = [&] {
        return d->state == Deferred::QUEUED || d->state == Deferred::RUNNING ||
               (!preview && d->state == Deferred::PREVIEW);
    };
    if (block && !d->cv.wait_for(lk, wait_limit(), [&] { return !pending(); }))
        return fail(FPO_ERR_TIMEOUT, "gave up after %lld ms waiting for the build to be enqueued",
                    (long long)wait_limit().count());
    if (pending()) return FPO_NOT_READY;
    switch (d->state) {
    case Deferred::PREVIEW:
    case Deferred::SUBMITTED:
        *inner = d->inner;
        return FPO_OK;
    case Deferred::FAILED:
        set_error_text(d->err);
        return d->status;
    case Deferred::CANCELLED:
    default:
        set_error_text("the job was cancelled");
        return FPO_ERR_CANCELLED;
    }
}

uint64_t deferred_start_ns(const fpo_job *job)
{
    Deferred *d = job->def;
    std::lock_guard<std::mutex> g(d->m);
    return d->t_start;
}

uint64_t deferred_end_ns(const fpo_job *job)
{
    Deferred *d = job->def;
    std::lock_guard<std::mutex> g(d->m);
    return d->t_end;
}

void deferred_release(fpo_job *job)
{
    Deferred *d = job->def;
    (void)cancel_queued(job);   // a job that has not started never will
    {
        std::unique_lock<std::mutex> lk(d->m);
        if (!d->cv.wait_for(lk, wait_limit(), [&] {
                return d->state != Deferred::QUEUED && d->state != Deferred::RUNNING && d->state != Deferred::PREVIEW;
            })) {
            // its build is still being enqueued: leave the job (and its
            // references) alive rather than free what the worker still uses
            (void)fail(FPO_ERR_TIMEOUT, "release gave up after %lld ms; the job was left allocated",
                 (long long)wait_limit().count());
            return;
        }
    }
    if (d->inner) fpo_job_release(d->inner);
    if (d->server && d->has_memory) {
        Server *S = d->server;
        {
            std::lock_guard<std::mutex> g(S->m);
            S->adm.release(d->arena_off, d->ws_bytes);
            try_admit(S);
        }
        S->cv.notify_all();
    }
    if (d->after) (void)hipEventDestroy(d->after);
    Server *S = d->server;
    fpo_context *ctx = job->ctx;
    delete d;
    delete job;
    if (S) server_release(S);
    ctx_release(ctx);
}

void destroy_batch_pool(fpo_context *ctx)
{
    Pool *I = nullptr;
    std::vector<Pool *> B;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        I = ctx->issue_pool;
        ctx->issue_pool = nullptr;
        for (Pool *&P : ctx->batch_pools) {
            if (P) B.push_back(P);
            P = nullptr;
        }
    }
    stop_pool(I);
    for (Pool *P : B) stop_pool(P);
}

fpo_status queue_build(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                       uint64_t workspace_bytes, hipStream_t st, fpo_job **out)
{
    Pool *P;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        if (!ctx->issue_pool) ctx->issue_pool = make_pool(ctx, nullptr, 1);
        P = ctx->issue_pool;
    }
    if (!P) return fail(FPO_ERR_OUT_OF_MEMORY, "could not create the issuing thread's stream");
    fpo_job *job = new_deferred_job(ctx);
    Deferred *d = job->def;
    d->cloud = *cloud;
    d->params = *p;
    d->ws = workspace;
    d->ws_bytes = workspace_bytes;
    d->stream = st;
    d->pool = P;
    *out = job;
    pool_push(P, job);
    return FPO_OK;
}

}  // namespace fpo

using namespace fpo;

extern "C" {

fpo_status fpo_job_cancel(fpo_job *job)
{
    if (!job) return fail(FPO_ERR_INVALID_ARG, "job is NULL");
    if (!job->def) return fail(FPO_ERR_INVALID_ARG, "only batch and server jobs can be cancelled");
    if (!cancel_queued(job)) return fail(FPO_ERR_INVALID_ARG, "the job has already started (or was cancelled)");
    return FPO_OK;
}

fpo_status fpo_context_set_batch_workers(fpo_context *ctx, uint32_t workers)
{
    if (!ctx) return fail(FPO_ERR_INVALID_ARG, "context is NULL");
    if (workers < 1 || workers > 16) return fail(FPO_ERR_INVALID_ARG, "workers must be in 1..16 (got %u)", workers);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->batch_workers = (int)workers;
    return FPO_OK;
}

fpo_status fpo_batch_workspace_size(const fpo_cloud *clouds, const fpo_params *params, uint32_t count,
                                    uint64_t *bytes)
{
    if (!bytes || (count && (!clouds || !params))) return fail(FPO_ERR_INVALID_ARG, "NULL clouds, params or bytes");
    uint64_t total = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const fpo_status s = check_cloud(&clouds[i], &params[i]);
        if (s != FPO_OK) return s;
        total += a256(workspace_bytes(clouds[i].n, params[i]));
    }
    *bytes = total;
    return FPO_OK;
}

fpo_status fpo_build_batch(fpo_context *ctx, const fpo_cloud *clouds, const fpo_params *params, uint32_t count,
                           void *workspace, uint64_t workspace_bytes_, void *hip_stream, fpo_job **jobs_out)
{
    if (!ctx || !jobs_out || (count && (!clouds || !params))) return fail(FPO_ERR_INVALID_ARG, "NULL argument");
    if (count == 0) return FPO_OK;
    if (!workspace) return fail(FPO_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(FPO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    std::vector<uint64_t> off(count), sz(count);
    uint64_t total = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const fpo_status s = check_cloud(&clouds[i], &params[i]);
        if (s != FPO_OK) return fail(s, "cloud %u: %s", i, error_text().c_str());
        sz[i] = workspace_bytes(clouds[i].n, params[i]);
        off[i] = total;
        total += a256(sz[i]);
    }
    if (workspace_bytes_ < total)
        return fail(FPO_ERR_OUT_OF_MEMORY, "workspace holds %llu bytes, the batch needs %llu",
                    (unsigned long long)workspace_bytes_, (unsigned long long)total);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(FPO_ERR_DEVICE, "hipSetDevice failed");
    Pool *P;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        // one pool per worker count, kept until the context is torn down
        // (queued jobs refer to theirs)
        Pool *&slot = ctx->batch_pools[ctx->batch_workers];
        if (!slot) slot = make_pool(ctx, nullptr, ctx->batch_workers);
        P = slot;
    }
    if (!P) return fail(FPO_ERR_OUT_OF_MEMORY, "could not create the worker streams");
    std::vector<fpo_job *> jobs(count, nullptr);
    for (uint32_t i = 0; i < count; ++i) {
        fpo_job *job = new_deferred_job(ctx);
        jobs[i] = job;
        Deferred *d = job->def;
        d->cloud = clouds[i];
        d->params = params[i];
        d->ws = static_cast<char *>(workspace) + off[i];
        d->ws_bytes = sz[i];
        d->pool = P;
        bool ok = true;
        if (hip_stream) {
            ok = !alloc_fault(ctx) && hipEventCreateWithFlags(&d->after, hipEventDisableTiming) == hipSuccess;
            if (!ok) d->after = nullptr;
            ok = ok && hipEventRecord(d->after, static_cast<hipStream_t>(hip_stream)) == hipSuccess;
        }
        if (!ok) {   // nothing is queued yet: undo
            for (uint32_t k = 0; k <= i; ++k) free_unqueued(jobs[k]);
            return fail(FPO_ERR_OUT_OF_MEMORY, "could not record an event on the caller's stream");
        }
    }
    // largest first: the small builds fill in behind the long ones.  Clouds
    // of the single-workgroup path go in groups of up to SB_GROUP per
    // launch, queued first so that their workgroups share the device with
    // the long builds
    std::vector<uint32_t> order(count);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return clouds[a].n > clouds[b].n; });
    std::vector<uint32_t> small, rest;
    for (uint32_t i : order)
        (small_eligible(ctx->small_max_batch.load(), clouds[i].n, params[i], clouds[i].location == FPO_HOST_PINNED)
             ? small
             : rest)
            .push_back(i);
    std::vector<fpo_job *> entries;
    for (size_t k = 0; k < small.size(); k += SB_GROUP) {
        fpo_job *e = new fpo_job();
        e->ctx = ctx;
        e->def = new Deferred();
        e->def->pool = P;
        for (size_t m = k; m < small.size() && m < k + SB_GROUP; ++m) e->def->group.push_back(jobs[small[m]]);
        entries.push_back(e);
    }
    for (uint32_t i = 0; i < count; ++i) jobs_out[i] = jobs[i];
    for (fpo_job *e : entries) pool_push(P, e);
    for (uint32_t i : rest) pool_push(P, jobs[i]);
    return FPO_OK;
}

fpo_status fpo_server_create(fpo_context *ctx, uint64_t hbm_budget_bytes, uint32_t max_slots, fpo_server **out)
{
    if (!ctx || !out) return fail(FPO_ERR_INVALID_ARG, "NULL context or out");
    if (max_slots == 0 || max_slots > 64) return fail(FPO_ERR_INVALID_ARG, "max_slots must be in 1..64 (got %u)", max_slots);
    const uint64_t budget = hbm_budget_bytes & ~(uint64_t)255;
    if (budget == 0) return fail(FPO_ERR_INVALID_ARG, "hbm_budget_bytes must be at least 256");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(FPO_ERR_DEVICE, "hipSetDevice failed");
    fpo_server *S = new fpo_server(budget, max_slots);
    S->ctx = ctx;
    void *arena = nullptr;
    if (alloc_fault(ctx) || hipMalloc(&arena, budget) != hipSuccess) {
        delete S;
        return fail(FPO_ERR_OUT_OF_MEMORY, "could not allocate the %llu-byte arena", (unsigned long long)budget);
    }
    S->arena = static_cast<char *>(arena);
    S->pool = make_pool(ctx, S, (int)max_slots);
    if (!S->pool) {
        (void)hipFree(arena);
        delete S;
        return fail(FPO_ERR_OUT_OF_MEMORY, "could not create the slot streams");
    }
    ctx_retain(ctx);   // dropped when the server is torn down
    *out = S;
    return FPO_OK;
}

fpo_status fpo_server_submit(fpo_server *S, const fpo_cloud *cloud, const fpo_params *params, fpo_job **out)
{
    if (!S || !out) return fail(FPO_ERR_INVALID_ARG, "NULL server or out");
    const fpo_status s = check_cloud(cloud, params);
    if (s != FPO_OK) return s;
    const uint64_t bytes = a256(workspace_bytes(cloud->n, *params));
    if (bytes > S->budget)
        return fail(FPO_ERR_REJECTED, "the build needs %llu bytes, more than the server's budget of %llu",
                    (unsigned long long)bytes, (unsigned long long)S->budget);
    fpo_job *job = new_deferred_job(S->ctx);
    Deferred *d = job->def;
    d->cloud = *cloud;
    d->params = *params;
    d->ws_bytes = bytes;
    d->server = S;
    S->refs.fetch_add(1);   // dropped by the job's release
    *out = job;
    {
        std::lock_guard<std::mutex> g(S->m);
        S->adm.submit(job, bytes);
        try_admit(S);
    }
    return FPO_OK;
}

void fpo_server_destroy(fpo_server *S)
{
    // queued and running requests go on; the arena is freed when the last
    // job of the server has been released
    if (S) server_release(S);
}

}  // extern "C"
