// View-dependent node selection: the nodes a renderer draws for one camera
// (section "Octree Rendering": the traversal thread checks every node's
// visibility against the camera's frustum and position and queues the nodes to
// draw).  The top-down traversal is replaced by a test per node of its own
// chain of ancestors, whose cubes follow from the node's key alone, so every
// node is decided independently; the drawn nodes are then compacted in order.
#include <math.h>
#include <stdint.h>

#include <mutex>

#include <hip/hip_runtime.h>

#include "fpo_host.h"
#include "fpo_internal.h"

namespace {

using fpo::fail;

constexpr double kSqrt3 = 1.7320508075688772;   // the double nearest sqrt(3)
constexpr int SEL_BLOCK = 256;

struct SelArgs {
    uint64_t num_nodes;
    const uint8_t *depth;
    const uint64_t *key;
    const uint32_t *count;
    double m[3], side;
    double eye[3];
    double planes[6][4];
    double proj_factor, min_size;
    uint32_t *bits;        // one bit per node
    uint32_t *points;      // total points of the drawn nodes
};

// Bits 3b + shift of a Morton key, gathered into an integer.
__device__ __forceinline__ uint32_t compact3(uint64_t k, int shift)
{
    uint64_t x = (k >> shift) & 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x100f00f00f00f00full;
    x = (x | (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x | (x >> 16)) & 0x1f00000000ffffull;
    x = (x | (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

// Visible and, for an ancestor, refined: the node at depth j with cell c.
__device__ bool passes(const SelArgs &a, int j, const uint32_t c[3], bool refine)
{
    const double s = __ddiv_rn(a.side, (double)(1u << j));
    const double h = __ddiv_rn(s, 2.0);
    double lo[3], hi[3], ctr[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = __dadd_rn(a.m[k], __dmul_rn((double)c[k], s));
        hi[k] = __dadd_rn(a.m[k], __dmul_rn((double)(c[k] + 1u), s));
        ctr[k] = __dadd_rn(a.m[k], __dmul_rn((double)(2u * c[k] + 1u), h));
    }
    for (int p = 0; p < 6; ++p) {
        const double *q = a.planes[p];
        const double px = q[0] >= 0.0 ? hi[0] : lo[0];
        const double py = q[1] >= 0.0 ? hi[1] : lo[1];
        const double pz = q[2] >= 0.0 ? hi[2] : lo[2];
        const double v = __dadd_rn(__dadd_rn(__dadd_rn(__dmul_rn(q[0], px), __dmul_rn(q[1], py)), __dmul_rn(q[2], pz)),
                                   q[3]);
        if (v < 0.0) return false;
    }
    if (!refine) return true;
    const double r = __dmul_rn(h, kSqrt3);
    const double dx = __dsub_rn(ctr[0], a.eye[0]), dy = __dsub_rn(ctr[1], a.eye[1]), dz = __dsub_rn(ctr[2], a.eye[2]);
    const double dist = __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)));
    if (dist <= r) return true;   // infinite size
    return !(__dmul_rn(a.proj_factor, __ddiv_rn(r, dist)) < a.min_size);
}

// One node per thread; a wave's 64 decisions are two words of the bit map.
__global__ __launch_bounds__(SEL_BLOCK) void k_select_nodes(SelArgs a)
{
    __shared__ uint32_t red[SEL_BLOCK / 64];
    const uint64_t words = (a.num_nodes + 31) / 32;
    const uint64_t i = (uint64_t)blockIdx.x * SEL_BLOCK + threadIdx.x;
    bool drawn = false;
    if (i < a.num_nodes) {
        const int d = a.depth[i];
        const uint64_t k = a.key[i];
        if (d <= 21) {
            const uint32_t c[3] = {compact3(k, 2), compact3(k, 1), compact3(k, 0)};
            drawn = true;
            for (int j = 0; j <= d && drawn; ++j) {
                const uint32_t cj[3] = {c[0] >> (d - j), c[1] >> (d - j), c[2] >> (d - j)};
                drawn = passes(a, j, cj, j < d);
            }
        }
    }
    const uint64_t m = __ballot(drawn);
    const uint64_t i0 = i & ~63ull;
    const uint32_t lane = __lane_id();
    if (lane == 0 && i0 / 32 < words) a.bits[i0 / 32] = (uint32_t)m;
    if (lane == 1 && i0 / 32 + 1 < words) a.bits[i0 / 32 + 1] = (uint32_t)(m >> 32);
    // points of the drawn nodes: one atomic per block
    uint32_t pts = drawn ? a.count[i] : 0u;
    for (int o = 32; o > 0; o >>= 1) pts += __shfl_xor(pts, o, 64);
    if (lane == 0) red[threadIdx.x >> 6] = pts;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < SEL_BLOCK / 64; ++w) t += red[w];
        if (t) atomicAdd(a.points, t);
    }
}

struct SelPlan {
    size_t bits, tiles, offs, scan, total;
};

SelPlan sel_plan(uint64_t n)
{
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const uint64_t nn = n ? n : 1;
    SelPlan p;
    p.bits = 0;
    p.tiles = p.bits + a256(4 * ((nn + 31) / 32));
    p.offs = p.tiles + a256(4 * fpo::bits_tiles(nn));
    p.scan = p.offs + a256(4 * fpo::bits_tiles(nn));
    p.total = p.scan + a256(fpo::scan_temp_bytes(fpo::bits_tiles(nn)));
    return p;
}

// Scratch of fpo_select_nodes_static, for callers that cannot allocate: one
// selection's bit map, tile counts, tile offsets and scan partials.  Each
// device holds its own copy for the life of the process.  Every word a call
// reads was written earlier in the same call, so nothing needs clearing.
static_assert(FPO_SELECT_STATIC_BYTES % 256 == 0, "whole 256-byte blocks");
__device__ __align__(256) unsigned char scratch[FPO_SELECT_STATIC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch`, per device

// Validates a selection and enqueues it with the workspace at ws.
fpo_status select_nodes(fpo_context *ctx, uint64_t num_nodes, const uint8_t *node_depth, const uint64_t *node_key,
                        const uint32_t *node_count, const float bbox_min[3], float cube_size, const fpo_view *view,
                        char *ws, uint32_t *out_nodes, uint32_t *out_totals, void *hip_stream)
{
    const SelPlan P = sel_plan(num_nodes);
    bool finite = isfinite(cube_size) && isfinite(view->proj_factor) && view->proj_factor > 0.0 &&
                  !isnan(view->min_size) && view->min_size >= 0.0;
    for (int k = 0; k < 3; ++k) finite = finite && isfinite(bbox_min[k]) && isfinite(view->eye[k]);
    for (int p = 0; p < 6; ++p)
        for (int k = 0; k < 4; ++k) finite = finite && isfinite(view->planes[p][k]);
    if (!finite) return fail(FPO_ERR_INVALID_ARG, "view, box and cube must be finite (min_size may be +inf), "
                                                  "proj_factor > 0, min_size >= 0");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(FPO_ERR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream;
    fpo::launch_fill_u32(out_totals, 0u, 2, st);
    if (num_nodes) {
        SelArgs a;
        a.num_nodes = num_nodes;
        a.depth = node_depth;
        a.key = node_key;
        a.count = node_count;
        for (int k = 0; k < 3; ++k) {
            a.m[k] = (double)bbox_min[k];
            a.eye[k] = view->eye[k];
        }
        a.side = (double)cube_size;
        for (int p = 0; p < 6; ++p)
            for (int k = 0; k < 4; ++k) a.planes[p][k] = view->planes[p][k];
        a.proj_factor = view->proj_factor;
        a.min_size = view->min_size;
        a.bits = reinterpret_cast<uint32_t *>(ws + P.bits);
        a.points = out_totals + 1;
        const uint64_t blocks = (num_nodes + SEL_BLOCK - 1) / SEL_BLOCK;
        hipLaunchKernelGGL(k_select_nodes, dim3((uint32_t)blocks), dim3(SEL_BLOCK), 0, st, a);
        uint32_t *tiles = reinterpret_cast<uint32_t *>(ws + P.tiles), *offs = reinterpret_cast<uint32_t *>(ws + P.offs);
        fpo::launch_bits_count(a.bits, num_nodes, tiles, st);
        fpo::scan_exclusive(tiles, offs, fpo::bits_tiles(num_nodes), out_totals, ws + P.scan, st);
        fpo::launch_bits_write(a.bits, num_nodes, offs, out_nodes, st);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return fail(FPO_ERR_DEVICE, "node selection launch: %s", hipGetErrorString(e));
    return FPO_OK;
}

fpo_status check_select_args(fpo_context *ctx, uint64_t num_nodes, const uint8_t *node_depth, const uint64_t *node_key,
                             const uint32_t *node_count, const float bbox_min[3], const fpo_view *view,
                             uint32_t *out_nodes, uint32_t *out_totals)
{
    if (!ctx || !bbox_min || !view || !out_totals) return fail(FPO_ERR_INVALID_ARG, "NULL context, box, view or totals");
    if (num_nodes > 0xffffffffull) return fail(FPO_ERR_INVALID_ARG, "num_nodes exceeds 2^32 - 1");
    if (num_nodes && (!node_depth || !node_key || !node_count || !out_nodes))
        return fail(FPO_ERR_INVALID_ARG, "NULL node array or output");
    return FPO_OK;
}

}  // namespace

namespace fpo {

// Called by fpo_context_create with `device` current: records the device
// address of the static scratch once per device.
fpo_status select_static_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(FPO_ERR_DEVICE, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch[device]) return FPO_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(FPO_ERR_DEVICE, "hipGetSymbolAddress of the selection scratch: %s", hipGetErrorString(e));
    g_scratch[device] = ptr;
    return FPO_OK;
}

}  // namespace fpo

extern "C" {

fpo_status fpo_select_workspace_size(uint64_t num_nodes, uint64_t *bytes)
{
    if (!bytes) return fail(FPO_ERR_INVALID_ARG, "bytes is NULL");
    if (num_nodes > 0xffffffffull) return fail(FPO_ERR_INVALID_ARG, "num_nodes exceeds 2^32 - 1");
    *bytes = sel_plan(num_nodes).total;
    return FPO_OK;
}

fpo_status fpo_select_nodes(fpo_context *ctx, uint64_t num_nodes, const uint8_t *node_depth, const uint64_t *node_key,
                            const uint32_t *node_count, const float bbox_min[3], float cube_size,
                            const fpo_view *view, void *workspace, uint64_t workspace_bytes, uint32_t *out_nodes,
                            uint32_t *out_totals, void *hip_stream)
{
    const fpo_status s =
        check_select_args(ctx, num_nodes, node_depth, node_key, node_count, bbox_min, view, out_nodes, out_totals);
    if (s != FPO_OK) return s;
    const SelPlan P = sel_plan(num_nodes);
    if (!workspace || workspace_bytes < P.total || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return fail(FPO_ERR_INVALID_ARG, "workspace must be 256-byte aligned with %llu bytes",
                    (unsigned long long)P.total);
    return select_nodes(ctx, num_nodes, node_depth, node_key, node_count, bbox_min, cube_size, view,
                        static_cast<char *>(workspace), out_nodes, out_totals, hip_stream);
}

fpo_status fpo_select_nodes_static(fpo_context *ctx, uint64_t num_nodes, const uint8_t *node_depth,
                                   const uint64_t *node_key, const uint32_t *node_count, const float bbox_min[3],
                                   float cube_size, const fpo_view *view, uint32_t *out_nodes, uint32_t *out_totals,
                                   void *hip_stream)
{
    const fpo_status s =
        check_select_args(ctx, num_nodes, node_depth, node_key, node_count, bbox_min, view, out_nodes, out_totals);
    if (s != FPO_OK) return s;
    if (num_nodes > FPO_SELECT_STATIC_MAX_NODES || sel_plan(num_nodes).total > FPO_SELECT_STATIC_BYTES)
        return fail(FPO_ERR_INVALID_ARG, "%llu nodes: the static scratch holds at most %u",
                    (unsigned long long)num_nodes, (unsigned)FPO_SELECT_STATIC_MAX_NODES);
    char *ws = nullptr;
    if (ctx->device >= 0 && ctx->device < kMaxDevices) {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        ws = static_cast<char *>(g_scratch[ctx->device]);
    }
    if (!ws) return fail(FPO_ERR_DEVICE, "the static scratch of device %d has no address", ctx->device);
    return select_nodes(ctx, num_nodes, node_depth, node_key, node_count, bbox_min, cube_size, view, ws, out_nodes,
                        out_totals, hip_stream);
}

}  // extern "C"
