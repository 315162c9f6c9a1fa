/*
 * fpo.h -- C ABI of libfpo, an MI355X (gfx950) library that builds the
 * shallow out-of-core octree and the immediate decimated preview of FastPoints
 * (arXiv 2302.05002) from a point buffer already resident in GPU memory.
 *
 * The problem statement follows the paper's program structure (sections
 * "Program Structure" and "Implementation"): a point cloud comes in, a
 * uniformly decimated preview is available first, and an octree is built
 * without blocking the caller (section "Octree Construction": points are
 * sorted hierarchically into chunks, chunks are indexed into local octrees,
 * the local trees form one global tree; section "Immediate Low-Resolution
 * Rendering": a decimation that visits every point).  The paper fixes no
 * constants or orderings; the readings this library implements are:
 *
 *   - lattice: K = 21 bits per axis.  The cube is anchored at the bounding-box
 *     minimum with side = the largest extent; scale = 2^21 / side computed in
 *     double and rounded once to float (0 for side 0); the fine coordinate of
 *     an axis value a is clamp(floor((a - min) * scale), 0, 2^21 - 1) with one
 *     float subtraction and one float multiplication (NaN products map to 0).
 *     A computed -0.0 extreme is reported as +0.0.
 *   - count grid: G^3 cells, cell = fine >> (21 - log2 G), row-major [x][y][z].
 *   - chunks: the maximal pyramid nodes holding 0 < count <= C points; a finest
 *     cell with more than C points is an oversized chunk.  Chunks are listed in
 *     Morton pre-order (octant = x<<2 | y<<1 | z); perm lists the points chunk
 *     by chunk, ascending original index inside a chunk.
 *   - octree: top-down from the root, which receives every point.  A node at
 *     depth d receiving the set R is a leaf when |R| <= L or d == 21 - log2 S;
 *     otherwise it keeps, for every occupied cell of an S^3 grid over its cube,
 *     the point of lowest original index, and pushes the others to the child
 *     octants.  Only non-empty children exist.  Nodes are listed by (depth,
 *     Morton key); each node's points ascend.  The tree does not depend on G or
 *     C.
 *   - preview: every index i with H64(i) mod M == 0, ascending, where H64 is
 *     h = i; h ^= h >> 31; h *= 0x9E3779B97F4A7C15; h ^= h >> 29;
 *     h *= 0x9E3779B97F4A7C15; h ^= h >> 32 (all mod 2^64).  Two variants
 *     (section "Future Work" proposes a spatially constrained sampler in place
 *     of the uniform decimation; section "Results" decimates to a fixed target
 *     count): an exact stride, i mod M == 0; and one pick per occupied count-
 *     grid cell, the point of least H64 in the cell (H64 is a bijection, so the
 *     pick is unique).  Hash and stride previews depend on n and M only and are
 *     ready before the bounding box; the grid preview follows the count pass.
 *
 * Conventions for every entry point:
 *   - Every call returns an fpo_status; fpo_last_error() gives the text of the
 *     last non-OK status of the calling thread.  Arguments are validated
 *     before any GPU work is enqueued.
 *   - Pointers marked "device" are HIP device pointers on the context's device;
 *     the library never frees memory it did not allocate.
 *   - The caller owns the workspace (size from fpo_workspace_size); result
 *     arrays are views into it, valid until the workspace is reused or freed.
 *   - Inputs must stay valid and unmodified until fpo_job_wait/poll reports a
 *     status other than FPO_NOT_READY.
 *   - A context may be used from several threads; a job from one at a time.
 */
#ifndef FPO_H
#define FPO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FPO_OK = 0,
    FPO_ERR_INVALID_ARG = 1,   /* bad parameter, size or pointer */
    FPO_ERR_NONFINITE = 2,     /* a coordinate is NaN or infinite (reported by poll/wait) */
    FPO_ERR_OUT_OF_MEMORY = 3, /* workspace too small, or a host/device allocation failed */
    FPO_ERR_DEVICE = 4,        /* a HIP runtime call failed */
    FPO_NOT_READY = 5,         /* poll: the build is still running */
    FPO_ERR_REJECTED = 6,      /* fpo_server_submit: the build needs more than the server's whole budget */
    FPO_ERR_CANCELLED = 7,     /* wait/poll of a batch or server job taken out of its queue by fpo_job_cancel */
    FPO_ERR_TIMEOUT = 8        /* a wait on another host thread of the library (a job not yet started, a build
                                  still being enqueued) exceeded FPO_WAIT_LIMIT_MS (environment; default 300000) */
} fpo_status;

typedef struct fpo_context fpo_context;
typedef struct fpo_job fpo_job;

#define FPO_BBOX_GIVEN 1u      /* fpo_params.flags: use bbox_min/bbox_max instead of computing it */
#define FPO_PREVIEW_STRIDE 2u  /* flags: preview = every index with i mod M == 0 */
#define FPO_PREVIEW_GRID 4u    /* flags: preview = least-H64 point of every occupied count-grid cell (M unused);
                                  the workspace then holds 8 * G^3 more bytes */

/* Build parameters (names after the paper's "maxPointsPerChunk" style):
 *   count_grid G: power of two, 1..512;  max_points_per_chunk C >= 1;
 *   subsample_grid S: power of two, 1..256;  leaf_capacity L >= 1;
 *   preview_modulus M >= 1 (fpo_preview_modulus gives M for a target count).
 * At most one of FPO_PREVIEW_STRIDE and FPO_PREVIEW_GRID; neither selects the
 * H64 predicate.  With FPO_BBOX_GIVEN, bbox_min <= bbox_max per axis, all finite; points
 * outside the box clamp to its faces and are counted in fpo_result.n_outside. */
typedef struct {
    uint32_t count_grid;
    uint32_t max_points_per_chunk;
    uint32_t subsample_grid;
    uint32_t leaf_capacity;
    uint32_t preview_modulus;
    uint32_t flags;
    float bbox_min[3];
    float bbox_max[3];
} fpo_params;

#define FPO_DEVICE 0u           /* fpo_cloud.location: arrays in device memory */
#define FPO_HOST_PINNED 1u      /* arrays in pinned host memory, streamed in batches */
#define FPO_DEFAULT_STREAM_BATCH 16000000ull

/* A point cloud: n points as three float32 arrays (structure of arrays),
 * n <= 2^32 - 1 (indices are 32-bit).  Point i is (x[i], y[i], z[i]); i is
 * its original index.  With location FPO_HOST_PINNED the arrays are pinned
 * host memory (hipHostMalloc): they are copied into the workspace in batches
 * of stream_batch points (0: FPO_DEFAULT_STREAM_BATCH) on a copy stream of
 * the context, and the bounding-box pass of each batch (and, with a given
 * box, its quantise + count pass) starts as soon as the batch has landed. */
typedef struct {
    uint64_t n;
    const float *x;
    const float *y;
    const float *z;
    uint32_t location;
    uint64_t stream_batch;
} fpo_cloud;

/* Result of a build.  Scalars are host values; arrays are device pointers
 * into the workspace.
 *   count_grid   uint32[G^3], row-major [cx][cy][cz]
 *   chunk_*      num_chunks entries in Morton pre-order: level, key (Morton
 *                key of the chunk's cell at that level), count, begin (offset
 *                of the chunk in perm); chunk_oversized_any = 1 when some
 *                finest cell holds more than C points
 *   perm         uint32[n]: original indices, chunk by chunk, ascending inside
 *   node_*       num_nodes entries in (depth, key) order: depth, key (Morton
 *                key at that depth), child_mask (bit o = child octant o
 *                exists), begin (offset into node_points), count
 *   node_points  uint32[n]: original indices, node by node, ascending inside
 *   preview_index uint32[preview_count], ascending */
typedef struct {
    uint64_t n;
    float bbox_min[3], bbox_max[3];
    float cube_size, scale;
    uint64_t n_outside;
    const uint32_t *count_grid;
    uint32_t num_chunks;
    const uint8_t *chunk_level;
    const uint64_t *chunk_key;
    const uint32_t *chunk_count;
    const uint64_t *chunk_begin;
    uint8_t chunk_oversized_any;
    const uint32_t *perm;
    uint32_t num_nodes;
    const uint8_t *node_depth;
    const uint64_t *node_key;
    const uint8_t *node_child_mask;
    const uint64_t *node_begin;
    const uint32_t *node_count;
    const uint32_t *node_points;
    uint64_t preview_count;
    const uint32_t *preview_index;
} fpo_result;

/* Creates a context on HIP device `device` (its streams, events and pinned
 * host staging).  *out receives the handle.  With FPO_FAULT=alloc:<k> in the
 * environment at creation, the k-th allocation the context makes (pinned
 * staging, events, streams, server arenas; counted from 1) fails as if the
 * memory were exhausted, for failure tests: the call that needed it returns
 * FPO_ERR_OUT_OF_MEMORY and the context stays usable.
 *
 * fpo_context_destroy drops the caller's handle and never blocks.  Every job
 * and server holds its context, so jobs may still be waited for, read and
 * released afterwards; the streams, threads and staging are freed when the
 * last of them is released. */
fpo_status fpo_context_create(int device, fpo_context **out);
void fpo_context_destroy(fpo_context *ctx);

/* Text of the last non-OK status returned to the calling thread ("" if none).
 * The pointer stays valid until the thread's next fpo call. */
const char *fpo_last_error(void);

/* Worst-case workspace bytes of one build of n device-resident points with *p. */
fpo_status fpo_workspace_size(uint64_t n, const fpo_params *p, uint64_t *bytes);

/* Preview modulus for a target preview size: max(1, ceil(n / target)).  With
 * FPO_PREVIEW_STRIDE the preview then holds ceil(n / M) <= target indices; with
 * the H64 predicate about n / M.  FPO_ERR_INVALID_ARG if target == 0, n >
 * 2^32 - 1 or out is NULL. */
fpo_status fpo_preview_modulus(uint64_t n, uint64_t target, uint32_t *out);

/* The same for a given cloud: adds the device staging of pinned host inputs
 * (12 bytes per point). */
fpo_status fpo_workspace_size_cloud(const fpo_cloud *cloud, const fpo_params *p, uint64_t *bytes);

/* Queues a build of *cloud on hip_stream (a hipStream_t; NULL = the
 * context's own stream) using `workspace` (device, >= fpo_workspace_size_cloud
 * bytes, 256-byte aligned, owned by the caller) and returns at once: the
 * caller is never blocked by the build.  A thread of the context enqueues the
 * builds in submission order, the preview kernels first, so the preview is
 * ready (fpo_job_preview_ready) long before the tree; the rest of the build
 * needs a few host round trips, which that thread takes.  *out receives the
 * job; release it with fpo_job_release.  Argument errors are returned here,
 * before anything is queued; a non-finite coordinate (FPO_ERR_NONFINITE) is
 * reported by fpo_job_poll / fpo_job_wait. */
fpo_status fpo_build_submit(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                            uint64_t workspace_bytes, void *hip_stream, fpo_job **out);

/* FPO_OK once the preview of the job is complete, FPO_NOT_READY before. */
fpo_status fpo_job_preview_ready(fpo_job *job);

/* FPO_OK when the whole build is complete, FPO_NOT_READY while it runs, or
 * the error that ended it.  Never blocks. */
fpo_status fpo_job_poll(fpo_job *job);

/* Blocks until the build is complete; returns its status.  A batch or
 * server job that does not start within FPO_WAIT_LIMIT_MS (default 300 s)
 * returns FPO_ERR_TIMEOUT instead (the job stays valid; wait again or
 * release it). */
fpo_status fpo_job_wait(fpo_job *job);

/* Fills *out for a completed job (call after fpo_job_wait returned FPO_OK). */
fpo_status fpo_job_result(fpo_job *job, fpo_result *out);

/* Waits for the job if it still runs, then frees the handle (not the
 * workspace; a server job's share of the arena returns to the server).  A job
 * that has not started is taken out of its queue first.  If a batch or
 * server job is still being enqueued after FPO_WAIT_LIMIT_MS, the handle is
 * left allocated rather than freed under its worker, and fpo_last_error says
 * so. */
void fpo_job_release(fpo_job *job);

/* Packed host copy of a completed job's arrays, for tests and export: the
 * arrays of fpo_result in this order, each starting at a multiple of 8 bytes:
 * count_grid (uint32, G^3), chunk_level (uint8), chunk_key (uint64),
 * chunk_count (uint32), chunk_begin (uint64) (num_chunks each), perm
 * (uint32, n), node_depth (uint8), node_key (uint64), node_child_mask
 * (uint8), node_begin (uint64), node_count (uint32) (num_nodes each),
 * node_points (uint32, n), preview_index (uint32, preview_count).
 * fpo_job_export_bytes gives the size; host_dst must hold that many bytes.
 * Works for every kind of job (the only way to read server results from the
 * host). */
fpo_status fpo_job_export_bytes(fpo_job *job, uint64_t *bytes);
fpo_status fpo_job_copy_to_host(fpo_job *job, void *host_dst, uint64_t bytes);

/* ---- node-ordered points and hierarchy export (after a build) ---------------
 * The far side of the path in the paper's octree pipeline: the points of the
 * tree written node by node after the hierarchy ("Octree Construction"). */

/* Gathers the coordinates (and optional per-point colour bytes) of a
 * completed job into node order, k = 0..n-1:
 *   out_xyz[3k + a] = coordinate a of point node_points[k]   (float32, xyz interleaved)
 *   out_color[color_stride * k + c] = color[color_stride * node_points[k] + c]
 * cloud: the build's input, device arrays (a pinned-host build: pass device
 * copies).  color: device bytes, color_stride per point (3 rgb, 4 rgba), NULL
 * with stride 0 for none.  out_xyz: device, 12 n bytes; out_color: device,
 * color_stride n bytes.  Enqueued on hip_stream (NULL: the context's stream);
 * complete when that stream reaches it. */
fpo_status fpo_job_gather(fpo_job *job, const fpo_cloud *cloud, const uint8_t *color, uint32_t color_stride,
                          float *out_xyz, uint8_t *out_color, void *hip_stream);

/* Writes the hierarchy and the node-ordered points of a completed job to one
 * file (little endian; blocks back to back):
 *   header   "FPO1", uint32 version = 1, uint64 n, uint32 num_nodes,
 *            uint32 color_stride, float32 bbox_min[3], float32 cube_size,
 *            uint32 count_grid, uint32 subsample_grid (48 bytes)
 *   nodes    num_nodes records of 24 bytes in (depth, key) order: uint8 depth,
 *            uint8 child_mask, uint16 0, uint32 count, uint64 key, uint64 begin
 *   points   n x 3 float32 (xyz) in node order, then n x color_stride bytes
 * cloud / color as for fpo_job_gather.  Blocks until the file is written. */
fpo_status fpo_job_write_file(fpo_job *job, const fpo_cloud *cloud, const uint8_t *color, uint32_t color_stride,
                              const char *path);

/* Host steady-clock times (ns) of a completed job: when it was submitted, when
 * its build started (later than submitted for batch and server jobs that
 * waited for a worker, a slot or memory) and when it completed (server jobs:
 * when their slot saw the build end; others: when a wait or poll first saw
 * it).  FPO_ERR_INVALID_ARG before a wait or poll has seen the completion. */
fpo_status fpo_job_timestamps(fpo_job *job, uint64_t *submitted_ns, uint64_t *started_ns, uint64_t *completed_ns);

/* Statistics of a completed job (for logs and monitoring). */
typedef struct {
    uint64_t n;                   /* points */
    uint32_t num_chunks;
    uint32_t num_nodes;
    uint32_t max_depth;           /* depth of the deepest node (0 for an empty cloud) */
    uint32_t chunk_oversized_any; /* 1 when a finest count-grid cell holds more than C points */
    uint64_t n_outside;           /* points clamped to a given box */
    uint64_t preview_count;
    uint64_t workspace_bytes;     /* the build's worst-case plan (what fpo_workspace_size_cloud returns) */
    uint64_t submitted_ns, started_ns, completed_ns;   /* as fpo_job_timestamps */
    float region_ms[16];          /* device ms of each fpo_timer region when the job was timed, else -1 */
} fpo_job_stats;

/* Fills *out for a completed job (after fpo_job_wait returned FPO_OK); reads
 * one byte of the node table back from the device.  FPO_ERR_INVALID_ARG
 * before completion. */
fpo_status fpo_job_get_stats(fpo_job *job, fpo_job_stats *out);

/* ---- batched builds ----------------------------------------------------------
 * Many independent clouds in one call (the paper's import of several clouds,
 * each with its own preview and tree).  The builds run concurrently on the
 * context's worker streams (a few, one per hardware queue), largest first,
 * so that latency-bound small builds overlap; each result is the one a plain
 * build of that cloud gives. */

/* Number of worker streams (and issuing threads) of later fpo_build_batch
 * calls on ctx: 1..16, default 4 (one per hardware queue of a process).  Each
 * count has its own workers, kept until the context is torn down. */
fpo_status fpo_context_set_batch_workers(fpo_context *ctx, uint32_t workers);

/* Workspace bytes of a batch: the worst case of every cloud, each rounded up
 * to 256 bytes, back to back in the order of the clouds. */
fpo_status fpo_batch_workspace_size(const fpo_cloud *clouds, const fpo_params *params, uint32_t count,
                                    uint64_t *bytes);

/* Enqueues count builds: clouds[i] (device arrays) with params[i], results in
 * slice i of `workspace` (device, >= fpo_batch_workspace_size bytes,
 * 256-byte aligned, owned by the caller).  The builds start after the work
 * enqueued on hip_stream so far (NULL: no dependency).  jobs_out[i] receives
 * the job of cloud i; release every one.  Returns once the builds are queued;
 * argument errors come back before anything is queued, build errors (a
 * non-finite coordinate) from that build's job. */
fpo_status fpo_build_batch(fpo_context *ctx, const fpo_cloud *clouds, const fpo_params *params, uint32_t count,
                           void *workspace, uint64_t workspace_bytes, void *hip_stream, fpo_job **jobs_out);

/* ---- serving ------------------------------------------------------------------
 * A request loop with continuous batching: requests are admitted in arrival
 * order as soon as a slot and enough of the HBM budget are free, and the
 * builds of admitted requests overlap on the device.  Workspace comes from an
 * arena of hbm_budget_bytes allocated by the server; a request holds its
 * share from admission until fpo_job_release. */
typedef struct fpo_server fpo_server;

/* max_slots (1..64) builds run at once, each on a stream of its own. */
fpo_status fpo_server_create(fpo_context *ctx, uint64_t hbm_budget_bytes, uint32_t max_slots, fpo_server **out);

/* Queues a build of *cloud (device arrays, valid until the job completes)
 * and never blocks.  FPO_ERR_REJECTED when its workspace exceeds the whole
 * budget.  *out receives the job (poll, wait, result, cancel, release). */
fpo_status fpo_server_submit(fpo_server *srv, const fpo_cloud *cloud, const fpo_params *params, fpo_job **out);

/* Takes a batch or server job that has not started out of its queue; its
 * wait then returns FPO_ERR_CANCELLED.  FPO_ERR_INVALID_ARG once it started. */
fpo_status fpo_job_cancel(fpo_job *job);

/* Drops the caller's handle and never blocks.  Queued and running requests
 * go on; every served job holds its server, whose arena (where the job's
 * results live) and slot streams are freed when the last job has been
 * released.  No further fpo_server_submit may use the handle. */
void fpo_server_destroy(fpo_server *srv);

/* ---- autotuning ----------------------------------------------------------------
 * Choices that change only how fast a build runs, never its result, picked by
 * timing every candidate on the caller's own cloud.  The tuner checks that
 * every candidate gives a result with the same fingerprint (a hash of every
 * output array) as the first and reports FPO_ERR_DEVICE otherwise.  Choices
 * are kept in the context; with FPO_AUTOTUNE_CACHE=<path> in the environment
 * they are read when a context is created and written after every tuning
 * call.  Tuning a context while other builds run on it changes only their
 * speed. */
typedef struct {
    uint32_t quantize_variant;  /* the chosen shape of the quantise + count pass (0 .. 4) */
    uint32_t size_class;        /* floor(log2 n): the choice applies to clouds of this size class ... */
    uint32_t count_grid_log2;   /* ... built with this count grid */
    uint32_t candidates;        /* number of shapes timed (4, or 5 with the binned pass) */
    float quantize_ms[5];       /* median device time per shape of the pass and the box pass before it */
} fpo_tuning;

/* Times the quantise + count pass, with the bounding-box pass before it, of
 * `reps` builds (after one warm-up) of *cloud with every candidate shape: one
 * 1024-thread block per compute unit with a 16K-slot LDS table, two
 * 512-thread blocks with 8K slots, four 256-thread blocks with 4K slots, each
 * over a contiguous range of points and taking eight points per thread
 * between table flushes, or the first shape taking two points per thread
 * between flushes (the table then keeps up to 10K cells between flushes: for
 * count grids with few points per cell).  For device input of at least 2^16
 * points and G >= 8 (and 256 points per bin or more) also shape 4, the
 * binned pass: codes and per-block histograms of bins of the grid's Morton
 * order (2^15 cells each from G = 256 on, else 64 bins), each point's cell
 * put into its bin's range, then one workgroup per bin counting in LDS and
 * writing its part of the grid whole (no clearing).  Untuned builds take
 * shape 4 where it applies with G = 512, else shape 0.  Later
 * builds of the size class and count grid use the fastest.  workspace as for
 * fpo_build_submit; reps 1..100.  Blocks until done.  Not for the grid
 * preview (FPO_ERR_INVALID_ARG), which has one shape. */
fpo_status fpo_autotune(fpo_context *ctx, const fpo_cloud *cloud, const fpo_params *p, void *workspace,
                        uint64_t workspace_bytes, uint32_t reps, fpo_tuning *out);

/* Times `reps` whole batches (after one warm-up) with 2, 4 and 8 worker
 * streams and keeps the fastest for later batches of ctx (*workers_out);
 * ms_out (3 floats, may be NULL) receives the median batch time per
 * candidate.  Arguments as for fpo_build_batch (no stream dependency).
 * Blocks until done. */
fpo_status fpo_autotune_batch(fpo_context *ctx, const fpo_cloud *clouds, const fpo_params *params, uint32_t count,
                              void *workspace, uint64_t workspace_bytes, uint32_t reps, uint32_t *workers_out,
                              float *ms_out);

/* Forces the quantise shape of later builds of ctx (0..4; shape 4 where it
 * does not apply runs shape 0), or -1 to use the tuned choices again (for
 * tests: every shape gives the same result). */
fpo_status fpo_context_force_quantize_variant(fpo_context *ctx, int variant);

/* ---- single-workgroup builds ------------------------------------------------
 * A small cloud is built whole by one workgroup in one launch (box, quantise
 * and count, chunk, preview and the tree level by level), instead of a few
 * dozen launches and two host round trips.  A build takes this path when its
 * cloud is in device memory, n >= 1, n <= C (the root is the only chunk),
 * G <= 64, S <= 32, the preview is the hash or stride one, n / (L + 1) <= 64
 * (at most 64 nodes above L points per depth), and n is at most the
 * context's limit: plain_max for plain and served builds (default 65536,
 * where one workgroup stops being faster than the whole device), batch_max in
 * fpo_build_batch (default 262143), which puts up to 32 such clouds in one
 * launch, one workgroup each, beside the other builds (those jobs start with
 * their launch and cannot be cancelled).  Both limits are at most 262143; 0
 * turns the path off.  The results are those of the multi-kernel path, in
 * the same workspace. */
fpo_status fpo_context_set_single_block_max(fpo_context *ctx, uint32_t plain_max, uint32_t batch_max);

/* ---- kernel timing (for benchmarks) ----------------------------------------
 * With timing enabled on a context, every later submit of it brackets each
 * region below with a pair of HIP events recorded on the build's stream (a
 * few microseconds of host time per event; off by default).  The regions are
 * contiguous runs of launches that together hold every kernel of a build; only
 * the build's host round trips fall between them.  After fpo_job_wait
 * returned FPO_OK, fpo_job_timer gives a region's summed device time and its
 * number of brackets (0 when the region did not run in this build). */
typedef enum {
    FPO_TIMER_BBOX = 0,          /* step 1: grid fills, bounding-box passes, box reduction (empty with a given box) */
    FPO_TIMER_QUANTIZE = 1,      /* step 1: quantise + count (one bracket per streamed batch) */
    FPO_TIMER_CHUNK_SPLIT = 2,   /* step 3: chunk begins and the stable split into chunks (count, scan, scatter) */
    FPO_TIMER_SUBSAMPLE = 3,     /* step 4: work-chunk split, shared depths, subsample classes, leaf decision,
                                    node numbering */
    FPO_TIMER_NODE_COUNTS = 4,   /* step 4: points per node */
    FPO_TIMER_NODE_PLACE = 5,    /* step 4: node table, node begins, every point into its node's range */
    FPO_TIMER_PREVIEW = 6,       /* step 5: counters' fill and the preview kernels */
    FPO_TIMER_NODE_SORT = 7,     /* step 4: node ranges sorted by original index, merges, 64-bit begins */
    FPO_TIMER_CUT = 8,           /* step 2: pyramid, count-grid export, chunk and work-chunk cuts */
    FPO_TIMER_FUSED = 9,         /* steps 1-5 of a single-workgroup build (fpo_context_set_single_block_max):
                                    the one launch; such a build has no other region */
    FPO_TIMER_COUNT = 10
} fpo_timer;

/* enable: 1 to time later submits of ctx (every timer), 0 to stop. */
fpo_status fpo_context_set_timing(fpo_context *ctx, int enable);

/* Times later submits of ctx with the timers whose bits are set in mask
 * (bit t for fpo_timer t; 0 stops timing): fewer events, less perturbation of
 * the build.  The others report 0 launches.  FPO_ERR_INVALID_ARG for bits at
 * or above FPO_TIMER_COUNT. */
fpo_status fpo_context_set_timers(fpo_context *ctx, uint32_t mask);

/* *ms = summed elapsed time of the timer's launches in the job, *launches =
 * their number (either pointer may be NULL).  FPO_ERR_INVALID_ARG for an
 * unknown timer, a job that was not timed or is not complete. */
fpo_status fpo_job_timer(fpo_job *job, fpo_timer which, float *ms, uint32_t *launches);

/* ---- LAS point records --------------------------------------------------------
 * Section "File Importing": clouds arrive as LAS files.  A LAS file (ASPRS LAS
 * 1.0-1.4) holds a public header block, variable-length records, then n
 * fixed-size little-endian point records whose first twelve bytes are the
 * int32 coordinates X, Y, Z (point data record formats 0-10; LAZ-compressed
 * records are not supported).  The decode turns records into the float32
 * structure of arrays a build takes, per axis:
 *     x = (float)((X * scale_x + offset_x) - origin_x)
 * with IEEE double arithmetic rounded to nearest after each operation (no
 * fused multiply-add) and one rounding to float32.  The caller picks the
 * origin (the header's minimum, say) so that float32 keeps the file's
 * precision near the data. */
typedef struct {
    uint8_t version_major, version_minor;
    uint8_t point_format;      /* 0..10 */
    uint8_t has_rgb;           /* 1 if the format stores R, G, B */
    uint16_t record_length;    /* bytes per point record (>= the format's minimum: 20 28 26 34 57 63 30 36 38 59 67) */
    uint16_t rgb_offset;       /* byte offset of R, G, B (uint16 each) in a record when has_rgb */
    uint32_t offset_to_points; /* file offset of the first point record */
    uint64_t num_points;       /* LAS 1.4: the 64-bit count; earlier versions: the 32-bit one */
    double scale[3], offset[3];
    double min[3], max[3];     /* the header's box, x y z */
} fpo_las_header;

/* Parses the public header block in bytes[0..len) (host memory).
 * FPO_ERR_INVALID_ARG if it is not a LAS header, is shorter than its version
 * requires, has an unknown or compressed record format, a record length
 * below the format's minimum, points that start inside the header, or a
 * non-finite scale or offset. */
fpo_status fpo_las_parse_header(const void *bytes, uint64_t len, fpo_las_header *out);

/* The header's box in the decoded frame: lo = (float)(min - origin), hi =
 * (float)(max - origin), per axis (for FPO_BBOX_GIVEN). */
fpo_status fpo_las_header_box(const fpo_las_header *h, const double origin[3], float lo[3], float hi[3]);

/* Enqueues the decode of the n records at `records` (device, record_length
 * bytes each, any alignment, records_bytes >= n * record_length readable
 * bytes) on hip_stream (NULL = the context's stream):
 * x, y, z (device float32[n]) as above and, if rgb is not NULL, R, G, B
 * (device uint16[3n], interleaved per point; the format must have them).
 * Returns once enqueued; the outputs are ready when the stream reaches the
 * decode.  FPO_ERR_INVALID_ARG for NULL arguments, n > 2^32 - 1, records_bytes
 * below n * record_length, an inconsistent header or a non-finite origin. */
fpo_status fpo_las_decode(fpo_context *ctx, const fpo_las_header *h, const void *records, uint64_t records_bytes,
                          uint64_t n, const double origin[3], float *x, float *y, float *z, uint16_t *rgb,
                          void *hip_stream);

/* ---- view-dependent node selection -----------------------------------------------
 * Section "Octree Rendering": a traversal thread walks the octree with the
 * camera's position and frustum, checks every node's visibility and queues the
 * nodes to draw.  Here one data-parallel pass decides every node at once.
 * Readings (all IEEE double, one rounding per operation, no fused
 * multiply-add; m = the cloud's box minimum and side its cube side, both
 * float32 values taken as doubles):
 *   - a node at depth d with cell c (its key de-interleaved, x the most
 *     significant bit of each triple) spans m + c*s .. m + (c+1)*s per axis,
 *     s = side / 2^d; centre m + (2c+1)*(s/2); radius (s/2) * 1.7320508075688772;
 *   - a plane (a, b, c, e) keeps a*x + b*y + c*z + e >= 0; a node is visible
 *     unless for some plane ((a*px + b*py) + c*pz) + e < 0 at its corner
 *     farthest along the normal (hi where a component is >= 0, else lo);
 *   - its size on screen is proj_factor * (radius / dist) pixels, dist =
 *     sqrt((dx*dx + dy*dy) + dz*dz) from the eye to the centre, and infinite
 *     when dist <= radius;
 *   - a node is drawn iff it and all its ancestors are visible and every
 *     ancestor's size is >= min_size (a node is refined into its children when
 *     it covers at least min_size pixels); this is the top-down traversal's
 *     result.  Nodes deeper than 21 are never drawn. */
typedef struct {
    double eye[3];          /* camera position */
    double planes[6][4];    /* frustum planes (a, b, c, e) */
    double proj_factor;     /* viewport height / (2 tan(fov_y / 2)), > 0 */
    double min_size;        /* pixels, >= 0 (+inf: draw visible roots only) */
} fpo_view;

/* Device scratch bytes of fpo_select_nodes for num_nodes nodes. */
fpo_status fpo_select_workspace_size(uint64_t num_nodes, uint64_t *bytes);

/* Enqueues the selection of the nodes of one view on hip_stream (NULL = the
 * context's stream).  node_depth, node_key, node_count: device arrays of a
 * node table (fpo_result's, or one read from a file and copied back);
 * bbox_min, cube_size: its cloud's box minimum and cube side.  Writes the
 * drawn nodes' indices, ascending, to out_nodes (device, num_nodes entries
 * at most) and out_totals[0] = their number, out_totals[1] = their points
 * (device uint32[2]).  workspace: device, fpo_select_workspace_size bytes,
 * 256-byte aligned; calls that share a workspace must not overlap.
 * FPO_ERR_INVALID_ARG for NULL arrays, a too small workspace, num_nodes >
 * 2^32 - 1, or non-finite view values (min_size may be +inf). */
fpo_status fpo_select_nodes(fpo_context *ctx, uint64_t num_nodes, const uint8_t *node_depth, const uint64_t *node_key,
                            const uint32_t *node_count, const float bbox_min[3], float cube_size,
                            const fpo_view *view, void *workspace, uint64_t workspace_bytes, uint32_t *out_nodes,
                            uint32_t *out_totals, void *hip_stream);

/* ---- node selection without allocation ------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, render or serving loops that forbid hipMalloc): fpo_select_nodes
 * with the library's own static scratch in place of a workspace.  That
 * scratch is FPO_SELECT_STATIC_BYTES of device memory per device, held from
 * the first fpo_context_create on that device until the process ends; it
 * serves tables of at most FPO_SELECT_STATIC_MAX_NODES nodes.  Arguments,
 * outputs and results are those of fpo_select_nodes; the call makes no
 * hipMalloc, hipFree or other allocating call.  FPO_ERR_INVALID_ARG for more
 * than FPO_SELECT_STATIC_MAX_NODES nodes, before anything is enqueued.
 * Every call on a device shares that device's scratch: calls that overlap on
 * one device (two streams, or two threads) race and give wrong results;
 * calls in order on one stream are safe. */
#define FPO_SELECT_STATIC_MAX_NODES 4194304u
#define FPO_SELECT_STATIC_BYTES 655360u
fpo_status fpo_select_nodes_static(fpo_context *ctx, uint64_t num_nodes, const uint8_t *node_depth,
                                   const uint64_t *node_key, const uint32_t *node_count, const float bbox_min[3],
                                   float cube_size, const fpo_view *view, uint32_t *out_nodes, uint32_t *out_totals,
                                   void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
