// Host-side state shared by the sources of libfpo: the context and job
// objects behind the opaque handles of include/fpo.h, and the helpers the
// executors (batch, server) use.  Not part of the public C ABI.
#pragma once
#include <stdint.h>
#include <atomic>
#include <chrono>
#include <functional>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/fpo.h"

namespace fpo {

// Sets the calling thread's error text (fpo_last_error) and returns s.
fpo_status fail(fpo_status s, const char *fmt, ...);
void set_error_text(const std::string &text);
std::string error_text();
fpo_status check_params(uint64_t n, const fpo_params *p);
uint64_t workspace_bytes(uint64_t n, const fpo_params &p, bool host_input = false);   // worst case of one build
uint64_t now_ns();                                           // steady clock
// Longest time a library call waits on another host thread (a job that has
// not started, a build still being enqueued) before it gives up with
// FPO_ERR_TIMEOUT: FPO_WAIT_LIMIT_MS from the environment, else 300 s.
std::chrono::milliseconds wait_limit();

struct Deferred;   // job created before its build starts (batch, server)
struct Pool;       // worker threads with their own streams

}  // namespace fpo

struct fpo_context {
    // The owner's reference plus one per live batch, server or plain job and
    // one per server: the context is torn down when the last one is dropped,
    // so a job released after fpo_context_destroy still finds its context.
    std::atomic<int> refs{1};
    // FPO_FAULT=alloc:<k> at creation: the k-th allocation the context makes
    // (pinned staging, events, streams, server arenas) fails, counted from 1.
    uint64_t fault_at = 0;
    std::atomic<uint64_t> allocs{0};
    int device;
    hipStream_t stream;
    std::mutex mu;
    std::vector<void *> pinned_free;
    bool timing = false;
    uint32_t timer_mask = 0;           // bit t: timer t is recorded (when timing)
    std::vector<hipEvent_t> ev_free;   // timing events, reused across jobs
    fpo::Pool *batch_pools[17] = {};   // worker pools of batches, by worker count (created on first use)
    int batch_workers = 4;             // workers of the next batch (fpo_context_set_batch_workers)
    // autotuned quantise variant per (log2 n, log2 G); 0xff = not tuned (variant 0)
    uint8_t qz_variant[33][10];
    int qz_force = -1;                 // fpo_context_force_quantize_variant, else -1
    fpo::Pool *issue_pool = nullptr;   // issues plain builds in submission order (created by the first)
    hipStream_t copy_stream = nullptr; // host-to-device batches of pinned inputs (created on first use)
    // single-workgroup builds up to this many points (0: off): plain and
    // served builds, batches
    std::atomic<uint32_t> small_max{65536};
    std::atomic<uint32_t> small_max_batch{262143};
};

struct fpo_job {
    fpo_context *ctx;
    hipStream_t stream;
    hipEvent_t ev_preview, ev_done;
    void *pinned;                 // Ctrs + DevBox staging
    fpo_status status;
    fpo_result res;
    bool waited;
    bool timed;
    uint32_t timer_mask = 0;      // the context's timers when it was submitted
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tm[FPO_TIMER_COUNT];
    uint64_t t_submit, t_done;    // host steady clock, ns (t_done: when a wait or poll saw it end)
    uint64_t grid_cells;          // G^3
    uint64_t plan_bytes = 0;      // the build's worst-case workspace plan
    fpo_params params;            // of the build
    std::vector<hipEvent_t> stream_events;   // one per host-to-device batch
    fpo::Deferred *def = nullptr; // set for batch and server jobs (the build runs later)
    bool small = false;           // a single-workgroup build (counts come with the final read-back)
};

namespace fpo {

// Records the device address of fpo_select_nodes_static's scratch for the
// current device (once per device; fpo_context_create calls it).
fpo_status select_static_init(int device);

void ctx_retain(fpo_context *c);
void ctx_release(fpo_context *c);   // tears the context down at zero references
// Fingerprint of a completed job's result (equal for equal results).
fpo_status job_fingerprint(fpo_job *job, uint64_t *out);

// Quantise variant of a build of n points with count grid 2^g.
int quantize_variant(fpo_context *c, uint64_t n, int g);
// Loads FPO_AUTOTUNE_CACHE into a new context's table (missing file: nothing).
void tune_cache_load(fpo_context *c);

// True when the allocation about to be made is the one FPO_FAULT names.
bool alloc_fault(fpo_context *c);

// For a deferred job: FPO_OK with *inner once its build has been enqueued
// whole (preview: once its preview kernels have), the status that ended it
// otherwise (with the error text set), FPO_NOT_READY before that when block
// is false.
fpo_status deferred_resolve(fpo_job *job, bool block, bool preview, fpo_job **inner);
void deferred_release(fpo_job *job);
void destroy_batch_pool(fpo_context *ctx);

// True when a build of n points with p runs as one workgroup (limit: the
// context's size limit for the kind of build).
bool small_eligible(uint64_t limit, uint64_t n, const fpo_params &p, bool host_in);
// Enqueues count single-workgroup builds (each small_eligible) as one launch
// on st; jobs_out[i] receives the job of clouds[i].  On an error no job is
// left.
fpo_status issue_small_group(fpo_context *ctx, uint32_t count, const fpo_cloud *const *clouds,
                             const fpo_params *const *params, void *const *workspaces, hipStream_t st,
                             fpo_job **jobs_out);
// Enqueues a whole build on st from the calling thread (see fpo_api.hip).
fpo_status issue_build(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                       uint64_t workspace_bytes, hipStream_t st, fpo_job **out,
                       const std::function<void(fpo_job *)> &on_preview);
// Hands a checked build to the context's issuing thread; *out at once.
fpo_status queue_build(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                       uint64_t workspace_bytes, hipStream_t st, fpo_job **out);
uint64_t deferred_start_ns(const fpo_job *job);
uint64_t deferred_end_ns(const fpo_job *job);   // 0 unless a server slot saw the end

}  // namespace fpo
