// HIP kernels (gfx950, wave64) of the online shallow-octree build and the
// decimated preview of FastPoints (arXiv 2302.05002).
//
// Path (section "Octree Construction": chunking, per-chunk indexing into local
// octrees, one global tree; section "Immediate Low-Resolution Rendering": a
// decimation that visits every point):
//   1. bbox reduction, quantisation to the 21-bit lattice, count histogram
//   2. count pyramid, chunk cut (and the internal work-chunk cut)
//   3. stable multisplit by chunk -> perm; by work chunk -> work-chunk order
//   4. per-node grid subsample (lowest original index wins a cell), computed
//      per work chunk in LDS, then node ids and a stable multisplit by node
//   5. hash-of-index preview with an ordered compaction
// Nothing here is a dense contraction, so no MFMA: the bounds are HBM
// bandwidth, LDS/global atomics and scan latency.
#include "fpo_device.h"

namespace fpo {

// Slot hash of the global-memory cell tables: the 64-bit finaliser of
// MurmurHash3 (fmix64, Austin Appleby, public domain), used as published.
__device__ __forceinline__ uint64_t mix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ uint64_t match_peers(uint32_t key, bool valid, int nbits)
{
    uint64_t m = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (key >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return valid ? m : 0ull;
}

constexpr uint32_t ilog2_c(uint32_t v) { return v <= 1 ? 0 : 1 + ilog2_c(v >> 1); }

__device__ __forceinline__ uint32_t ceil_log2_dev(uint32_t v)
{
    return v <= 1 ? 0u : 32u - __clz(v - 1u);
}

static inline uint32_t ceil_log2(uint64_t v)
{
    uint32_t l = 0;
    while ((1ull << l) < v) ++l;
    return l;
}
static inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// ---- step 1a: bounding box ------------------------------------------------------


// zero (or null): zero_words words cleared on the way (the count grid).
__global__ __launch_bounds__(256) void k_bbox(const float *__restrict__ x, const float *__restrict__ y,
                                              const float *__restrict__ z, uint64_t n, int vec4, uint32_t *part,
                                              uint32_t *zero, uint64_t zero_words)
{
    if (zero)   // (a pyramid level: 4-byte aligned only)
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < zero_words;
             i += (uint64_t)gridDim.x * blockDim.x)
            zero[i] = 0u;
    uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
    uint32_t bad = 0;
    const uint64_t n4 = vec4 ? n / 4 : 0;   // float4 loads only on 16-byte aligned inputs
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const float4 *px = reinterpret_cast<const float4 *>(x), *py = reinterpret_cast<const float4 *>(y),
                 *pz = reinterpret_cast<const float4 *>(z);
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // four float4 per axis in flight per thread
    for (; i + 3 * stride < n4; i += 4 * stride) {
        float4 a[4], b[4], c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = px[i + u * stride];
            b[u] = py[i + u * stride];
            c[u] = pz[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            bbox_acc(mn[0], mx[0], bad, a[u].x); bbox_acc(mn[0], mx[0], bad, a[u].y);
            bbox_acc(mn[0], mx[0], bad, a[u].z); bbox_acc(mn[0], mx[0], bad, a[u].w);
            bbox_acc(mn[1], mx[1], bad, b[u].x); bbox_acc(mn[1], mx[1], bad, b[u].y);
            bbox_acc(mn[1], mx[1], bad, b[u].z); bbox_acc(mn[1], mx[1], bad, b[u].w);
            bbox_acc(mn[2], mx[2], bad, c[u].x); bbox_acc(mn[2], mx[2], bad, c[u].y);
            bbox_acc(mn[2], mx[2], bad, c[u].z); bbox_acc(mn[2], mx[2], bad, c[u].w);
        }
    }
    for (; i < n4; i += stride) {
        const float4 a0 = px[i], b0 = py[i], c0 = pz[i];
        bbox_acc(mn[0], mx[0], bad, a0.x); bbox_acc(mn[0], mx[0], bad, a0.y);
        bbox_acc(mn[0], mx[0], bad, a0.z); bbox_acc(mn[0], mx[0], bad, a0.w);
        bbox_acc(mn[1], mx[1], bad, b0.x); bbox_acc(mn[1], mx[1], bad, b0.y);
        bbox_acc(mn[1], mx[1], bad, b0.z); bbox_acc(mn[1], mx[1], bad, b0.w);
        bbox_acc(mn[2], mx[2], bad, c0.x); bbox_acc(mn[2], mx[2], bad, c0.y);
        bbox_acc(mn[2], mx[2], bad, c0.z); bbox_acc(mn[2], mx[2], bad, c0.w);
    }
    for (uint64_t j = n4 * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        bbox_acc(mn[0], mx[0], bad, x[j]);
        bbox_acc(mn[1], mx[1], bad, y[j]);
        bbox_acc(mn[2], mx[2], bad, z[j]);
    }
    // per-block partial box (same-address global atomics from every block
    // would serialise); k_setup reduces the partials
    __shared__ uint32_t s[7][4];
    const int w = threadIdx.x >> 6;
    for (int a = 0; a < 3; ++a) {
        uint32_t v = mn[a], u = mx[a];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            v = min(v, (uint32_t)__shfl_xor(v, o, 64));
            u = max(u, (uint32_t)__shfl_xor(u, o, 64));
        }
        if (lane_id() == 0) { s[a][w] = v; s[3 + a][w] = u; }
    }
    const uint64_t anybad = __ballot(bad != 0);
    if (lane_id() == 0) s[6][w] = anybad ? 1u : 0u;
    __syncthreads();
    if (threadIdx.x < 7) {
        const int a = threadIdx.x;
        uint32_t v = s[a][0];
        for (int k = 1; k < 4; ++k) v = a < 3 ? min(v, s[a][k]) : (a < 6 ? max(v, s[a][k]) : (v | s[a][k]));
        part[(uint64_t)blockIdx.x * 8 + a] = v;
    }
}

// Reduces the per-block partial boxes (nparts of them), then, unless the box
// is given: cube anchored at the box minimum, side = largest extent,
// scale = 2^21/side computed in double and rounded once to float (0 for a
// zero side).
__global__ __launch_bounds__(256) void k_setup(DevBox *box, const uint32_t *part, uint32_t nparts, int given, float gx0,
                                               float gy0, float gz0, float gx1, float gy1, float gz1, int flag_only)
{
    __shared__ uint32_t red[7][4];
    uint32_t v[7] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u, 0u};
    for (uint32_t b = threadIdx.x; b < nparts; b += 256) {
        for (int a = 0; a < 3; ++a) {
            v[a] = min(v[a], part[(uint64_t)b * 8 + a]);
            v[3 + a] = max(v[3 + a], part[(uint64_t)b * 8 + 3 + a]);
        }
        v[6] |= part[(uint64_t)b * 8 + 6];
    }
    // wave reductions, then the four wave results
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        for (int a = 0; a < 3; ++a) {
            v[a] = min(v[a], (uint32_t)__shfl_xor(v[a], o, 64));
            v[3 + a] = max(v[3 + a], (uint32_t)__shfl_xor(v[3 + a], o, 64));
        }
        v[6] |= (uint32_t)__shfl_xor(v[6], o, 64);
    }
    if (lane_id() == 0)
        for (int a = 0; a < 7; ++a) red[a][threadIdx.x >> 6] = v[a];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (uint32_t t = 1; t < 4; ++t) {
        for (int a = 0; a < 3; ++a) {
            v[a] = min(v[a], red[a][t]);
            v[3 + a] = max(v[3 + a], red[3 + a][t]);
        }
        v[6] |= red[6][t];
    }
    box->nonfinite = v[6];
    if (flag_only) return;   // the box is set already (and points outside it counted)
    const float g0[3] = {gx0, gy0, gz0}, g1[3] = {gx1, gy1, gz1};
    box_set(box, v, v + 3, given != 0, g0, g1);
}

// ---- step 1b: quantise + count ---------------------------------------------------
// One Morton code per point (x the most significant bit of each triple) and a
// count per finest cell.  Global atomics cost ~40 ns each on this part, so a
// block first aggregates the cells of its contiguous range of points in an
// LDS hash table and flushes one atomic per distinct cell: scans emit points
// surface by surface, so a range touches far fewer cells than it has points.
// With the grid preview the same table also keeps the least H64 of each cell
// (fewer slots, 64-bit minima) and flushes it with a 64-bit atomic minimum.
// Shapes of the pass (autotuned per size class, result-identical: the counts
// do not depend on which block aggregates which points): a block of BLOCK
// threads with a table of 2^HLOG slots.  Variant 0 is one 1024-thread block
// per compute unit with 16K slots (128 KB); variants 1 and 2 are two 512-
// thread blocks with 8K slots and four 256-thread blocks with 4K slots per
// compute unit, over shorter ranges of points.  All three take IT = 8 points
// per thread between flushes, so the table keeps at most 3/4 of its slots
// minus a round (4K cells for variant 0).  Variant 3 is variant 0 with two
// points per thread: up to 10K cells between flushes, for count grids with
// few points per cell, where a flush per round costs one atomic for nearly
// every point.  The grid preview always takes variant 0's shape with 8K slots
// of 64-bit minima.
template <bool GRID, int BLOCK = 1024, int HLOG = 14, int IT = 8> struct Qz {
    static constexpr int ITEMS = GRID ? 2 : IT;
    static constexpr uint32_t ROUND = BLOCK * ITEMS;
    static constexpr uint32_t HASH = GRID ? 8192 : (1u << HLOG);   // slots
    // flushed when a round could fill the table past half (grid preview)
    // or three quarters of its slots
    static constexpr uint32_t FLUSH_AT = (GRID ? HASH / 2 : HASH - HASH / 4) - ROUND;
    static_assert(HASH - HASH / 4 > ROUND, "a round fits the table");
};

// Slot hash of the quantise pass's LDS cell table: the "lowbias32" integer
// hash of Chris Wellons' hash-prospector (public domain), used as published.
__device__ __forceinline__ uint32_t hash32(uint32_t k)
{
    k ^= k >> 16;
    k *= 0x7feb352du;
    k ^= k >> 15;
    k *= 0x846ca68bu;
    k ^= k >> 16;
    return k;
}

template <bool GRID, int BLOCK, uint32_t HASH>
__device__ void qz_flush(uint32_t *hk, uint32_t *hc, unsigned long long *hm, uint32_t *fine,
                         unsigned long long *cellmin)
{
    for (uint32_t h = threadIdx.x; h < HASH; h += BLOCK) {
        const uint32_t k = hk[h];
        if (k != 0xffffffffu) {
            atomicAdd(&fine[k], hc[h]);
            hk[h] = 0xffffffffu;
            hc[h] = 0;
            if constexpr (GRID) {
                atomicMin(&cellmin[k], hm[h]);
                hm[h] = ~0ull;
            }
        }
    }
}

// Claims or finds the slot of cell `cl`, starting at slot h whose key was
// read as k (linear probing; entries stay until the next flush).
template <uint32_t HASH>
__device__ __forceinline__ uint32_t qz_slot(uint32_t *hk, uint32_t *used, uint32_t cl, uint32_t h, uint32_t k)
{
    while (true) {
        if (k == 0xffffffffu) {
            k = atomicCAS(&hk[h], 0xffffffffu, cl);
            if (k == 0xffffffffu) {
                atomicAdd(used, 1u);
                return h;
            }
        }
        if (k == cl) return h;
        h = (h + 1) & (HASH - 1);
        k = hk[h];
    }
}

// 32-bit byte offsets from a block's own base pointers (a block covers at
// most 2^32 / 256 points), so the loads and stores take a scalar base.
template <typename T> __device__ __forceinline__ const T &at_byte(const T *p, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + off);
}
template <typename T> __device__ __forceinline__ T &at_byte(T *p, uint32_t off)
{
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(p) + off);
}

// One block per compute unit, each over a contiguous range of points.  The
// coordinates of the next round are loaded before the hash updates of the
// current one, so the loads stay in flight while the LDS work runs.  The
// first probe of every item is read before any is used: a cell already in
// the table (the usual case) then costs one read and one atomic.  `base` is
// the original index of x[0] (batches of a streamed cloud).
template <bool GRID, int QZ_BLOCK = 1024, int HLOG = 14, int IT = 8>
__global__ __launch_bounds__(QZ_BLOCK) void k_quantize(const float *__restrict__ x, const float *__restrict__ y,
                                                       const float *__restrict__ z, uint64_t n, const DevBox *box,
                                                       int g, int given, uint64_t *__restrict__ code,
                                                       uint32_t *__restrict__ fine, DevBox *box_rw, uint64_t per_block,
                                                       uint64_t base, unsigned long long *__restrict__ cellmin)
{
    using C = Qz<GRID, QZ_BLOCK, HLOG, IT>;
    constexpr int ITEMS = C::ITEMS;
    constexpr uint32_t ROUND = C::ROUND, HASH = C::HASH;
    __shared__ uint32_t hk[HASH];
    __shared__ uint32_t hc[HASH];
    __shared__ unsigned long long hm[GRID ? HASH : 1];
    __shared__ uint32_t used;
    __shared__ uint32_t wsum[QZ_BLOCK / 64];
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint32_t cnt = (uint32_t)((lo + per_block < n ? lo + per_block : n) - lo);
    const float *bx = x + lo, *by = y + lo, *bz = z + lo;
    uint64_t *bcode = code + lo;
    float px[ITEMS], py[ITEMS], pz[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t o = (uint32_t)j * QZ_BLOCK + threadIdx.x;
        px[j] = o < cnt ? at_byte(bx, 4 * o) : 0.0f;
        py[j] = o < cnt ? at_byte(by, 4 * o) : 0.0f;
        pz[j] = o < cnt ? at_byte(bz, 4 * o) : 0.0f;
    }
    const float lx = box->lo[0], ly = box->lo[1], lz = box->lo[2], sc = box->scale;
    const float hx = box->hi[0], hy = box->hi[1], hz = box->hi[2];
    const int sh = 3 * (KB - g);
    for (uint32_t h = threadIdx.x; h < HASH; h += QZ_BLOCK) {
        hk[h] = 0xffffffffu;
        hc[h] = 0;
        if constexpr (GRID) hm[h] = ~0ull;
    }
    if (threadIdx.x == 0) used = 0;
    __syncthreads();
    uint32_t outside = 0;
    bool bad = false;
    for (uint32_t r0 = 0; r0 < cnt; r0 += ROUND) {
        uint32_t cell[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t o = r0 + (uint32_t)j * QZ_BLOCK + threadIdx.x;
            const uint32_t ux = quantize1(px[j], lx, sc), uy = quantize1(py[j], ly, sc), uz = quantize1(pz[j], lz, sc);
            const uint64_t c = (split3(ux) << 2) | (split3(uy) << 1) | split3(uz);
            cell[j] = o < cnt ? (uint32_t)(c >> sh) : 0xffffffffu;
            if (o < cnt) at_byte(bcode, 8 * o) = c;
            if (given && o < cnt) {
                outside += (px[j] < lx || px[j] > hx || py[j] < ly || py[j] > hy || pz[j] < lz || pz[j] > hz) ? 1u : 0u;
                // NaN fails every comparison, an infinity exceeds the largest float
                bad |= !(fabsf(px[j]) <= FLT_MAX && fabsf(py[j]) <= FLT_MAX && fabsf(pz[j]) <= FLT_MAX);
            }
        }
        // next round's coordinates
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t o = r0 + ROUND + (uint32_t)j * QZ_BLOCK + threadIdx.x;
            px[j] = o < cnt ? at_byte(bx, 4 * o) : 0.0f;
            py[j] = o < cnt ? at_byte(by, 4 * o) : 0.0f;
            pz[j] = o < cnt ? at_byte(bz, 4 * o) : 0.0f;
        }
        uint32_t slot[ITEMS], seen[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            slot[j] = hash32(cell[j]) & (HASH - 1);
            seen[j] = hk[slot[j]];
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t cl = cell[j];
            if (cl == 0xffffffffu) continue;
            const uint32_t h = seen[j] == cl ? slot[j] : qz_slot<HASH>(hk, &used, cl, slot[j], seen[j]);
            atomicAdd(&hc[h], 1u);
            if constexpr (GRID)
                atomicMin(&hm[h], (unsigned long long)h64(base + lo + r0 + (uint64_t)j * QZ_BLOCK + threadIdx.x));
        }
        __syncthreads();
        // at most ROUND new cells per round
        if (used > C::FLUSH_AT) {
            qz_flush<GRID, QZ_BLOCK, HASH>(hk, hc, hm, fine, cellmin);
            __syncthreads();
            if (threadIdx.x == 0) used = 0;
            __syncthreads();
        }
    }
    __syncthreads();
    qz_flush<GRID, QZ_BLOCK, HASH>(hk, hc, hm, fine, cellmin);
    if (given) {
        // one atomic per block (the same counters for every block)
        outside = wave_sum(outside);
        const bool wbad = __ballot(bad) != 0;
        if (lane_id() == 0) wsum[threadIdx.x >> 6] = outside | (wbad ? 0x80000000u : 0u);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0, b = 0;
            for (int w = 0; w < QZ_BLOCK / 64; ++w) {
                t += wsum[w] & 0x7fffffffu;
                b |= wsum[w] >> 31;
            }
            if (t) atomicAdd(&box_rw->n_outside, (unsigned long long)t);
            if (b) atomicOr(&box_rw->nonfinite, 1u);
        }
    }
}

// Binned form of the pass (variant QZ_BINNED), for clouds whose points
// mostly fall in cells of their own, where the table form flushes about one
// global atomic per point (the uniform cube), and for count grids of 2^24
// cells and more, where those atomics land all over a grid larger than the
// last-level cache (G = 512: 512 MiB) at a few tens of G atomics/s.  The
// grid's Morton order falls into bins of 2^cb cells (cb = qb_cell_bits(g):
// 2^15 from G = 256 on, else 64 bins); one pass writes the codes and each
// block's histogram of bins, a scan of the histograms (bin-major) gives every
// (bin, block) its range, a second pass puts the cb low bits of each point's
// cell into its bin's range, and one block per bin counts its cells in LDS
// and writes its counts whole, so the grid needs no clearing.  Counts are
// sums: the order in which a bin's points are placed does not matter.
constexpr int QB_MAX_CELL_BITS = 15;
constexpr uint32_t QB_CELLS = 1u << QB_MAX_CELL_BITS;   // 128 KB of LDS counters
__host__ __device__ constexpr int qb_cell_bits(int g) { return 3 * g - 6 < QB_MAX_CELL_BITS ? 3 * g - 6 : QB_MAX_CELL_BITS; }
constexpr uint32_t QB_MAX_BINS = 4096;              // G = 512
constexpr int QB_BLOCK = 1024, QB_IT = 8;
constexpr uint32_t QB_BLOCKS = 256;                 // one range of points per compute unit

__global__ __launch_bounds__(QB_BLOCK) void k_qz_bin_code(const float *__restrict__ x, const float *__restrict__ y,
                                                          const float *__restrict__ z, uint64_t n, const DevBox *box,
                                                          int g, int given, uint64_t *__restrict__ code,
                                                          uint32_t *__restrict__ bhist, DevBox *box_rw,
                                                          uint64_t per_block)
{
    constexpr uint32_t ROUND = QB_BLOCK * QB_IT;
    __shared__ uint32_t hist[QB_MAX_BINS];
    __shared__ uint32_t wsum[QB_BLOCK / 64];
    const int cb = qb_cell_bits(g);
    const uint32_t nbins = 1u << (3 * g - cb);
    for (uint32_t b = threadIdx.x; b < nbins; b += QB_BLOCK) hist[b] = 0;
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint32_t cnt = (uint32_t)((lo + per_block < n ? lo + per_block : n) - lo);
    const float *bx = x + lo, *by = y + lo, *bz = z + lo;
    uint64_t *bcode = code + lo;
    float px[QB_IT], py[QB_IT], pz[QB_IT];
#pragma unroll
    for (int j = 0; j < QB_IT; ++j) {
        const uint32_t o = (uint32_t)j * QB_BLOCK + threadIdx.x;
        px[j] = o < cnt ? at_byte(bx, 4 * o) : 0.0f;
        py[j] = o < cnt ? at_byte(by, 4 * o) : 0.0f;
        pz[j] = o < cnt ? at_byte(bz, 4 * o) : 0.0f;
    }
    const float lx = box->lo[0], ly = box->lo[1], lz = box->lo[2], sc = box->scale;
    const float hx = box->hi[0], hy = box->hi[1], hz = box->hi[2];
    const int bsh = 3 * (KB - g) + cb;
    __syncthreads();
    uint32_t outside = 0;
    bool bad = false;
    for (uint32_t r0 = 0; r0 < cnt; r0 += ROUND) {
#pragma unroll
        for (int j = 0; j < QB_IT; ++j) {
            const uint32_t o = r0 + (uint32_t)j * QB_BLOCK + threadIdx.x;
            const uint32_t ux = quantize1(px[j], lx, sc), uy = quantize1(py[j], ly, sc), uz = quantize1(pz[j], lz, sc);
            const uint64_t c = (split3(ux) << 2) | (split3(uy) << 1) | split3(uz);
            if (o < cnt) {
                at_byte(bcode, 8 * o) = c;
                atomicAdd(&hist[(uint32_t)(c >> bsh)], 1u);
            }
            if (given && o < cnt) {
                outside += (px[j] < lx || px[j] > hx || py[j] < ly || py[j] > hy || pz[j] < lz || pz[j] > hz) ? 1u : 0u;
                bad |= !(fabsf(px[j]) <= FLT_MAX && fabsf(py[j]) <= FLT_MAX && fabsf(pz[j]) <= FLT_MAX);
            }
        }
#pragma unroll
        for (int j = 0; j < QB_IT; ++j) {
            const uint32_t o = r0 + ROUND + (uint32_t)j * QB_BLOCK + threadIdx.x;
            px[j] = o < cnt ? at_byte(bx, 4 * o) : 0.0f;
            py[j] = o < cnt ? at_byte(by, 4 * o) : 0.0f;
            pz[j] = o < cnt ? at_byte(bz, 4 * o) : 0.0f;
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nbins; b += QB_BLOCK) bhist[(uint64_t)b * gridDim.x + blockIdx.x] = hist[b];
    if (given) {
        outside = wave_sum(outside);
        const bool wbad = __ballot(bad) != 0;
        if (lane_id() == 0) wsum[threadIdx.x >> 6] = outside | (wbad ? 0x80000000u : 0u);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0, b = 0;
            for (int w = 0; w < QB_BLOCK / 64; ++w) {
                t += wsum[w] & 0x7fffffffu;
                b |= wsum[w] >> 31;
            }
            if (t) atomicAdd(&box_rw->n_outside, (unsigned long long)t);
            if (b) atomicOr(&box_rw->nonfinite, 1u);
        }
    }
}

// Each block re-reads the codes of its range and hands out the positions of
// its (bin, block) ranges with LDS counters.
__global__ __launch_bounds__(QB_BLOCK) void k_qz_bin_place(const uint64_t *__restrict__ code, uint64_t n, int g,
                                                           const uint32_t *__restrict__ boff,
                                                           uint16_t *__restrict__ cells, uint64_t per_block)
{
    constexpr uint32_t ROUND = QB_BLOCK * QB_IT;
    __shared__ uint32_t fill[QB_MAX_BINS];
    const int cb = qb_cell_bits(g);
    const uint32_t nbins = 1u << (3 * g - cb);
    for (uint32_t b = threadIdx.x; b < nbins; b += QB_BLOCK) fill[b] = boff[(uint64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint32_t cnt = (uint32_t)((lo + per_block < n ? lo + per_block : n) - lo);
    const uint64_t *bcode = code + lo;
    const int csh = 3 * (KB - g);
    for (uint32_t r0 = 0; r0 < cnt; r0 += ROUND) {
        uint64_t c[QB_IT];
#pragma unroll
        for (int j = 0; j < QB_IT; ++j) {
            const uint32_t o = r0 + (uint32_t)j * QB_BLOCK + threadIdx.x;
            c[j] = o < cnt ? at_byte(bcode, 8 * o) : 0ull;
        }
#pragma unroll
        for (int j = 0; j < QB_IT; ++j) {
            const uint32_t o = r0 + (uint32_t)j * QB_BLOCK + threadIdx.x;
            if (o >= cnt) continue;
            const uint32_t cell = (uint32_t)(c[j] >> csh);
            const uint32_t slot = atomicAdd(&fill[cell >> cb], 1u);
            cells[slot] = (uint16_t)(cell & ((1u << cb) - 1u));
        }
    }
}

// One block per bin: its cells counted in LDS, its 2^cb counts written.
// Sixteen loads per thread are issued before their atomics, so a bin's
// points are not read one memory latency at a time.
constexpr int QB_GRID_IT = 16;
__global__ __launch_bounds__(1024) void k_qz_bin_grid(const uint16_t *__restrict__ cells,
                                                      const uint32_t *__restrict__ boff, uint32_t nblocks,
                                                      uint32_t nbins, int cb, uint64_t n,
                                                      uint32_t *__restrict__ fine)
{
    __shared__ uint32_t hist[QB_CELLS];
    const uint32_t cells_per_bin = 1u << cb;
    for (uint32_t bin = blockIdx.x; bin < nbins; bin += gridDim.x) {
        for (uint32_t i = threadIdx.x; i < cells_per_bin; i += 1024) hist[i] = 0;
        __syncthreads();
        const uint32_t b0 = boff[(uint64_t)bin * nblocks];
        const uint32_t b1 = bin + 1 < nbins ? boff[(uint64_t)(bin + 1) * nblocks] : (uint32_t)n;
        for (uint32_t j0 = b0; j0 < b1; j0 += 1024 * QB_GRID_IT) {
            uint32_t c[QB_GRID_IT];
#pragma unroll
            for (int k = 0; k < QB_GRID_IT; ++k) {
                const uint32_t j = j0 + (uint32_t)k * 1024 + threadIdx.x;
                c[k] = j < b1 ? cells[j] : 0xffffffffu;
            }
#pragma unroll
            for (int k = 0; k < QB_GRID_IT; ++k)
                if (c[k] != 0xffffffffu) atomicAdd(&hist[c[k]], 1u);
        }
        __syncthreads();
        uint32_t *dst = fine + ((uint64_t)bin << cb);
        for (uint32_t i = threadIdx.x; i < cells_per_bin; i += 1024) dst[i] = hist[i];
        __syncthreads();
    }
}

// ---- step 2a: count pyramid ---------------------------------------------------------
// Level l-1 cell k = sum of level-l cells 8k..8k+7 (Morton order).
// The top levels (at most 32768 cells at level `top`) in one block: one
// launch instead of one per level.
// The eight level-l cells 8k..8k+7 (Morton order) into the row-major export
// of the finest level (l = g).
__device__ __forceinline__ void pyr_export(const uint32_t *c, uint64_t k, int l, uint32_t *out)
{
    const uint64_t G = 1ull << l;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const uint64_t m = 8 * k + (uint64_t)o;
        const uint32_t cx = compact3(m >> 2), cy = compact3(m >> 1), cz = compact3(m);
        out[((uint64_t)cx * G + cy) * G + cz] = c[o];
    }
}

// exp_out (or null): the finest level is level `top`, exported row-major on
// the way.
__global__ __launch_bounds__(1024) void k_pyr_top(uint32_t *pyr, int top, uint32_t *exp_out)
{
    for (int l = top; l >= 1; --l) {
        const uint32_t ncell = 1u << (3 * (l - 1));
        const uint32_t *src = pyr + pyr_off(l);
        uint32_t *dst = pyr + pyr_off(l - 1);
        for (uint32_t k = threadIdx.x; k < ncell; k += blockDim.x) {
            const uint32_t *c = src + 8 * k;
            dst[k] = c[0] + c[1] + c[2] + c[3] + c[4] + c[5] + c[6] + c[7];
            if (exp_out && l == top) pyr_export(c, k, l, exp_out);
        }
        __syncthreads();
    }
}

// Level l - 1 from level l: a thread per child, loads coalesced, the eight
// children of a parent summed across eight lanes (a parent's children are
// consecutive, and the stride is a multiple of 8, so its lanes are active
// together).
__global__ void k_pyr_level(uint32_t *pyr, int l)
{
    const uint64_t nchild = 1ull << (3 * l);
    const uint32_t *src = pyr + pyr_off(l);
    uint32_t *dst = pyr + pyr_off(l - 1);
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nchild;
         c += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t s = src[c];
        s += (uint32_t)__shfl_xor(s, 1, 64);
        s += (uint32_t)__shfl_xor(s, 2, 64);
        s += (uint32_t)__shfl_xor(s, 4, 64);
        if ((c & 7) == 0) dst[c >> 3] = s;
    }
}

// The finest level g >= 5: level g - 1 and the row-major export in one pass.
// A block takes 2^14 Morton-contiguous cells (a 16 x 32 x 32 box: x, y, z),
// reads them coalesced (all loads first), sums the parents across lanes, and
// stages the box in LDS in row-major order (z XOR-swizzled by x and y against
// bank conflicts), so that the export is written in whole 128-byte rows of
// 32 cells.  64 KB of LDS: two blocks per compute unit.
constexpr uint32_t PE_CELLS = 1u << 14;
constexpr int PE_BLOCK = 1024, PE_ITEMS = PE_CELLS / PE_BLOCK;
__device__ __forceinline__ uint32_t pe_slot(uint32_t x, uint32_t y, uint32_t z)
{
    return (x * 32u + y) * 32u + (z ^ (((y & 7u) << 2) | (x & 3u)));
}
__global__ __launch_bounds__(PE_BLOCK) void k_pyr_export(uint32_t *pyr, int g, uint32_t *exp_out)
{
    __shared__ uint32_t box[PE_CELLS];
    const uint64_t G = 1ull << g;
    const uint32_t *src = pyr + pyr_off(g);
    uint32_t *dst = pyr + pyr_off(g - 1);
    const uint64_t nboxes = (1ull << (3 * g)) / PE_CELLS;
    for (uint64_t bx = blockIdx.x; bx < nboxes; bx += gridDim.x) {
        const uint64_t m0 = bx * PE_CELLS;
        uint32_t v[PE_ITEMS];
#pragma unroll
        for (int j = 0; j < PE_ITEMS; ++j) v[j] = src[m0 + (uint32_t)j * PE_BLOCK + threadIdx.x];
#pragma unroll
        for (int j = 0; j < PE_ITEMS; ++j) {
            const uint32_t lm = (uint32_t)j * PE_BLOCK + threadIdx.x;   // Morton index inside the box
            box[pe_slot(compact3(lm >> 2), compact3(lm >> 1), compact3(lm))] = v[j];
            uint32_t s = v[j];
            s += (uint32_t)__shfl_xor(s, 1, 64);
            s += (uint32_t)__shfl_xor(s, 2, 64);
            s += (uint32_t)__shfl_xor(s, 4, 64);
            if ((lm & 7) == 0) dst[(m0 + lm) >> 3] = s;
        }
        __syncthreads();
        const uint64_t ox = compact3(m0 >> 2), oy = compact3(m0 >> 1), oz = compact3(m0);   // the box's corner
#pragma unroll
        for (int j = 0; j < PE_ITEMS; ++j) {
            const uint32_t r = (uint32_t)j * PE_BLOCK + threadIdx.x;
            const uint32_t x = r >> 10, y = (r >> 5) & 31u, z = r & 31u;
            exp_out[((ox + x) * G + (oy + y)) * G + (oz + z)] = box[pe_slot(x, y, z)];
        }
        __syncthreads();
    }
}

// Row-major [cx][cy][cz] export of the finest counts.
__global__ void k_grid_export(const uint32_t *fine, int g, uint32_t *out)
{
    const uint64_t G = 1ull << g, ncell = G * G * G;
    for (uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; m < ncell;
         m += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t cx = compact3(m >> 2), cy = compact3(m >> 1), cz = compact3(m);
        out[((uint64_t)cx * G + cy) * G + cz] = fine[m];
    }
}

// ---- step 2b: chunk cut ---------------------------------------------------------------
// A pyramid node (l, a), lmin <= l <= lam, is a chunk when it is non-empty,
// holds at most thresh points or l == lam, and l == lmin or its parent holds
// more than thresh.  flags[m] = 1 at the first level-lam cell m of every chunk; lev[m] =
// its level.  Chunks are disjoint, so at most one level can start at m.
// ---- step 2b: chunk and work-chunk cuts ---------------------------------------------------
// A node of a cut is heavy when it lies above the cut's first level lmin, or
// holds more than the cut's threshold (C for chunks, WC_CAP for work chunks)
// and is not a finest cell.  The cut's entries are the non-empty children of
// heavy nodes that are not heavy themselves (the maximal nodes at or below
// threshold; oversized finest cells), and the root when it is not heavy.
// They are found top-down from the heavy nodes alone, one launch per level:
// a launch classifies the eight children of every heavy node of the level
// above and compacts the heavy children and the entries, each in key order,
// with a single-pass chained scan over tiles of parents.  Work is
// proportional to the heavy nodes (at most n / (threshold + 1) per level), not
// to the G^3 cells of the finest level.  k_cut_rank then merges the per-level
// lists into Morton pre-order, and k_cut_index builds the coarse index that
// maps a finest cell to its entry.
constexpr uint64_t FR_SPIN_LIMIT = 1ull << 22;   // look-back polls before giving up (internal error)

__device__ __forceinline__ uint64_t fr_load(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fr_store(unsigned long long *p, uint64_t v)
{
    __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// status word of a tile: flag (1 aggregate, 2 inclusive prefix) << 62 |
// heavy count << 31 | entry count
__device__ __forceinline__ uint64_t fr_word(uint64_t flag, uint64_t o, uint64_t e) { return flag << 62 | o << 31 | e; }

__global__ void k_cut_init(const uint32_t *pyr, CutArgs c0, CutArgs c1)
{
    for (int which = 0; which < 2; ++which) {
        const CutArgs &a = which ? c1 : c0;
        const uint64_t ns = a.st_off[a.lam + 1];
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns;
             i += (uint64_t)gridDim.x * blockDim.x)
            a.status[i] = 0ull;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            for (int l = 0; l < MAXD; ++l) a.n_open[l] = a.n_ent[l] = a.tile_ctr[l] = 0u;
            const uint32_t n = pyr[0];
            if (n == 0) continue;
            if (a.lmin == 0 && (n <= a.thresh || a.lam == 0)) {
                a.ent[a.ent_off[0]] = 0ull;   // the root is the only entry
                a.n_ent[0] = 1u;
                if (n > a.thresh) atomicOr(a.over, 1u);
            } else {
                a.open[0][0] = 0ull;
                a.n_open[0] = 1u;
            }
        }
    }
}

// Children (level l) of the heavy nodes of level l - 1; blockIdx.y = cut.
__global__ __launch_bounds__(FR_BLOCK) void k_frontier(const uint32_t *pyr, int l, CutArgs c0, CutArgs c1)
{
    const CutArgs &a = blockIdx.y ? c1 : c0;
    __shared__ uint32_t lds[FR_BLOCK / 64 + 1];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_po, s_pe;
    const uint32_t n_in = min(a.n_open[l - 1], a.open_cap);
    const uint32_t live = (n_in + FR_BLOCK - 1) / FR_BLOCK;
    if (blockIdx.x >= live) return;   // exactly `live` blocks take tiles
    if (threadIdx.x == 0) s_tile = atomicAdd(&a.tile_ctr[l], 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t i = tile * FR_BLOCK + threadIdx.x;
    const uint64_t *in = a.open[(l - 1) & 1];
    uint64_t pk = 0;
    uint32_t om = 0, em = 0;
    bool over = false;
    if (i < n_in) {
        pk = in[i];
        const uint32_t *ch = pyr + pyr_off(l) + (pk << 3);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const uint32_t c = ch[o];
            if (c == 0) continue;
            if (l < a.lmin || (c > a.thresh && l < a.lam)) {
                om |= 1u << o;
            } else {
                em |= 1u << o;
                over |= c > a.thresh;
            }
        }
    }
    const uint32_t no = __popc(om), ne = __popc(em);
    uint32_t tot;
    const uint32_t ex = block_excl_scan<FR_BLOCK>(no | ne << 16, lds, &tot);   // at most 8 * FR_BLOCK each
    const uint64_t bo = tot & 0xffffu, be = tot >> 16;
    unsigned long long *st = a.status + a.st_off[l];
    if (threadIdx.x == 0) {
        uint64_t po = 0, pe = 0;
        if (tile == 0) {
            fr_store(&st[0], fr_word(2, bo, be));
        } else {
            fr_store(&st[tile], fr_word(1, bo, be));
            uint32_t j = tile - 1;
            uint64_t spins = 0;
            for (;;) {
                const uint64_t w = fr_load(&st[j]);
                const uint64_t f = w >> 62;
                if (f == 0) {
                    if (++spins > FR_SPIN_LIMIT) {   // never expected: report, and end the wait
                        atomicOr(a.err, 1u);
                        break;
                    }
                    continue;
                }
                po += (w >> 31) & 0x7fffffffull;
                pe += w & 0x7fffffffull;
                if (f == 2 || j == 0) break;
                --j;
            }
            fr_store(&st[tile], fr_word(2, po + bo, pe + be));
        }
        if (tile == live - 1) {   // the last tile knows the level's totals
            a.n_open[l] = (uint32_t)(po + bo);
            a.n_ent[l] = (uint32_t)(pe + be);
        }
        s_po = po;
        s_pe = pe;
    }
    __syncthreads();
    uint64_t oo = s_po + (ex & 0xffffu), oe = s_pe + (ex >> 16);
    const uint64_t ecap = a.ent_off[l + 1] - a.ent_off[l];
    uint64_t *out = a.open[l & 1];
    bool full = false;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        if (om >> o & 1u) {
            if (oo < a.open_cap) out[oo] = pk << 3 | (uint64_t)o; else full = true;
            ++oo;
        }
        if (em >> o & 1u) {
            if (oe < ecap) a.ent[a.ent_off[l] + oe] = pk << 3 | (uint64_t)o; else full = true;
            ++oe;
        }
    }
    if (full) atomicOr(a.err, 1u);
    if (over) atomicOr(a.over, 1u);
}

// Both cuts in one launch when every level's heavy nodes are few (at most
// CS_MAX_OPEN per level, from the plan): one block per cut takes the levels
// one after another, with block-wide scans instead of a launch per level and
// a chained scan across tiles.  The same classification, the same lists in
// the same key order, and the same capacity checks as k_cut_init and
// k_frontier.
constexpr uint32_t CS_BLOCK = 1024, CS_MAX_OPEN = 16384;
__global__ __launch_bounds__(CS_BLOCK) void k_cut_small(const uint32_t *pyr, CutArgs c0, CutArgs c1)
{
    const CutArgs &a = blockIdx.x ? c1 : c0;
    __shared__ uint32_t lds[CS_BLOCK / 64 + 1];
    if (threadIdx.x == 0) {
        for (int l = 0; l < MAXD; ++l) a.n_open[l] = a.n_ent[l] = a.tile_ctr[l] = 0u;
        const uint32_t n = pyr[0];
        if (n != 0) {
            if (a.lmin == 0 && (n <= a.thresh || a.lam == 0)) {
                a.ent[a.ent_off[0]] = 0ull;   // the root is the only entry
                a.n_ent[0] = 1u;
                if (n > a.thresh) atomicOr(a.over, 1u);
            } else {
                a.open[0][0] = 0ull;
                a.n_open[0] = 1u;
            }
        }
    }
    __syncthreads();
    for (int l = 1; l <= a.lam; ++l) {
        const uint32_t n_in = min(a.n_open[l - 1], a.open_cap);
        const uint64_t *in = a.open[(l - 1) & 1];
        uint64_t *out = a.open[l & 1];
        const uint64_t ecap = a.ent_off[l + 1] - a.ent_off[l];
        uint64_t bo_run = 0, be_run = 0;   // heavy children and entries of the parents before this round
        bool full = false, over = false;
        for (uint32_t i0 = 0; i0 < n_in; i0 += CS_BLOCK) {
            const uint32_t i = i0 + threadIdx.x;
            uint64_t pk = 0;
            uint32_t om = 0, em = 0;
            if (i < n_in) {
                pk = in[i];
                const uint32_t *ch = pyr + pyr_off(l) + (pk << 3);
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const uint32_t c = ch[o];
                    if (c == 0) continue;
                    if (l < a.lmin || (c > a.thresh && l < a.lam)) {
                        om |= 1u << o;
                    } else {
                        em |= 1u << o;
                        over |= c > a.thresh;
                    }
                }
            }
            uint32_t tot;
            // at most 8 * CS_BLOCK of each: both counts fit 16 bits
            const uint32_t ex = block_excl_scan<CS_BLOCK>(__popc(om) | __popc(em) << 16, lds, &tot);
            uint64_t oo = bo_run + (ex & 0xffffu), oe = be_run + (ex >> 16);
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                if (om >> o & 1u) {
                    if (oo < a.open_cap) out[oo] = pk << 3 | (uint64_t)o; else full = true;
                    ++oo;
                }
                if (em >> o & 1u) {
                    if (oe < ecap) a.ent[a.ent_off[l] + oe] = pk << 3 | (uint64_t)o; else full = true;
                    ++oe;
                }
            }
            bo_run += tot & 0xffffu;
            be_run += tot >> 16;
        }
        if (full) atomicOr(a.err, 1u);
        if (over) atomicOr(a.over, 1u);
        if (threadIdx.x == 0) {
            a.n_open[l] = (uint32_t)bo_run;
            a.n_ent[l] = (uint32_t)be_run;
        }
        __syncthreads();   // the level's list and counts before the next level reads them
    }
}

// First index of keys[0..n) not below v (keys ascending).
__device__ __forceinline__ uint32_t fr_lower_bound(const uint64_t *keys, uint32_t n, uint64_t v)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Every entry's place in Morton pre-order (by first finest cell): its index in
// its level's list plus, for every other level, how many of that level's
// entries start before it (entries are disjoint, so a coarser one starts
// before it iff its key is below the entry's ancestor key there, a finer one
// iff its ancestor at the entry's level is below the entry's key).
__global__ void k_cut_rank(const uint32_t *pyr, CutArgs c0, CutArgs c1)
{
    const CutArgs &a = blockIdx.y ? c1 : c0;
    uint32_t ne[MAXD];
    uint32_t total = 0;
#pragma unroll
    for (int l = 0; l < MAXD; ++l) {
        const uint64_t cap = l <= a.lam ? a.ent_off[l + 1] - a.ent_off[l] : 0;
        ne[l] = l <= a.lam ? (uint32_t)min((uint64_t)a.n_ent[l], cap) : 0u;
        total += ne[l];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.num_out = total;
        if (total > a.max_out) atomicOr(a.err, 1u);
    }
    const uint64_t slots = a.ent_off[a.lam + 1];
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        int l = 0;
        while (a.ent_off[l + 1] <= s) ++l;
        const uint32_t i = (uint32_t)(s - a.ent_off[l]);
        if (i >= ne[l]) continue;
        const uint64_t key = a.ent[s];
        uint64_t rank = i;
        for (int m = 0; m <= a.lam; ++m) {
            if (m == l || ne[m] == 0) continue;
            const uint64_t v = m < l ? key >> (3 * (l - m)) : key << (3 * (m - l));
            rank += fr_lower_bound(a.ent + a.ent_off[m], ne[m], v);
        }
        if (rank >= a.max_out) continue;   // reported above
        a.out_level[rank] = (uint8_t)l;
        a.out_key[rank] = key;
        a.out_count[rank] = pyr[pyr_off(l) + key];
        a.out_start[rank] = key << (3 * (a.lam - l));
    }
}

// idx[c] = number of entries whose first finest cell lies before coarse cell
// c of level lt (c = 0 .. 8^lt).
// A thread takes CI_RUN consecutive coarse cells: one binary search for the
// first, then a walk over the few entries that start inside the run (the
// index is monotone); the block stages its cells in LDS and writes them
// coalesced.
constexpr int CI_BLOCK = 256, CI_RUN = 16;
constexpr uint32_t CI_SPAN = CI_BLOCK * CI_RUN;

__global__ __launch_bounds__(CI_BLOCK) void k_cut_index(CutArgs c0, CutArgs c1)
{
    __shared__ uint32_t buf[CI_SPAN + CI_SPAN / 32];   // one pad word per 32 against bank conflicts
    const CutArgs &a = blockIdx.y ? c1 : c0;
    const uint32_t num = min(*a.num_out, a.max_out);
    const uint64_t cells = 1ull << (3 * a.lt);   // the index has cells + 1 words
    const int sh = 3 * (a.lam - a.lt);
    for (uint64_t cb = (uint64_t)blockIdx.x * CI_SPAN; cb <= cells; cb += (uint64_t)gridDim.x * CI_SPAN) {
        const uint64_t first = cb + (uint64_t)threadIdx.x * CI_RUN;
        uint32_t lo = first <= cells ? fr_lower_bound(a.out_start, num, first << sh) : num;
        for (int k = 0; k < CI_RUN; ++k) {
            const uint64_t bound = (first + k) << sh;
            while (lo < num && a.out_start[lo] < bound) ++lo;
            const uint32_t i = threadIdx.x * CI_RUN + k;
            buf[i + (i >> 5)] = lo;
        }
        __syncthreads();
        for (int k = 0; k < CI_RUN; ++k) {
            const uint32_t i = k * CI_BLOCK + threadIdx.x;
            if (cb + i <= cells) a.idx[cb + i] = buf[i + (i >> 5)];
        }
        __syncthreads();
    }
}

__global__ void k_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

// ---- device-wide exclusive scan ------------------------------------------------------------

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const uint32_t *in, uint64_t n, const uint32_t *n_dev,
                                                            uint32_t *tile_sum)
{
    __shared__ uint32_t lds[SCAN_BLOCK / 64 + 1];
    if (n_dev && *n_dev < n) n = *n_dev;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const uint64_t e = base + (uint64_t)j * SCAN_BLOCK + threadIdx.x;
        if (e < n) s += in[e];
    }
    s = block_sum<SCAN_BLOCK>(s, lds);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s;
}

// Single block: exclusive scan of the tile sums in place; *total = sum.
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *tile_sum, uint32_t ntiles, uint32_t *total)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    // tiles past a device-side length hold 0 (k_scan_reduce wrote 0 for them)
    uint32_t carry = 0;
    for (uint32_t b = 0; b < ntiles; b += 1024) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < ntiles ? tile_sum[i] : 0u;
        uint32_t t;
        const uint32_t ex = block_excl_scan<1024>(v, lds, &t);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += t;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// With TOP, tile_off holds the raw tile sums and every block adds up those
// before its own (at most SCAN_FUSED_TILES of them, read from L2), and the
// last block writes the total: the separate top pass is not launched.
constexpr uint32_t SCAN_FUSED_TILES = 4096;

template <bool TOP>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_down(const uint32_t *in, uint32_t *out, uint64_t n,
                                                          const uint32_t *n_dev, const uint32_t *tile_off,
                                                          uint32_t *total)
{
    __shared__ uint32_t lds[SCAN_BLOCK / 64 + 1];
    __shared__ uint32_t buf[SCAN_TILE];
    uint32_t prior = 0;
    if constexpr (TOP) {
        uint32_t v = 0;
        for (uint32_t t = threadIdx.x; t < blockIdx.x; t += SCAN_BLOCK) v += tile_off[t];
        prior = block_sum<SCAN_BLOCK>(v, lds);
        if (blockIdx.x == gridDim.x - 1 && total && threadIdx.x == 0) *total = prior + tile_off[blockIdx.x];
    } else {
        prior = tile_off[blockIdx.x];
    }
    if (n_dev && *n_dev < n) n = *n_dev;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    if (base >= n) return;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const uint64_t e = base + (uint64_t)j * SCAN_BLOCK + threadIdx.x;
        buf[j * SCAN_BLOCK + threadIdx.x] = e < n ? in[e] : 0u;
    }
    __syncthreads();
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        v[j] = buf[threadIdx.x * SCAN_ITEMS + j];
        s += v[j];
    }
    uint32_t t;
    uint32_t run = block_excl_scan<SCAN_BLOCK>(s, lds, &t) + prior;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        buf[threadIdx.x * SCAN_ITEMS + j] = run;
        run += v[j];
    }
    __syncthreads();
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const uint64_t e = base + (uint64_t)j * SCAN_BLOCK + threadIdx.x;
        if (e < n) out[e] = buf[j * SCAN_BLOCK + threadIdx.x];
    }
}

// Short arrays: one block, SS_ROUND elements per round with a running carry
// (one launch instead of three).  A round loads coalesced rows into LDS
// (padded by one word per 32 against bank conflicts), each thread scans 16
// consecutive values, and the results leave the same way.
constexpr uint64_t SCAN_SMALL_MAX = 16384;
constexpr int SS_PT = 16;
constexpr uint32_t SS_ROUND = 1024 * SS_PT;
__device__ __forceinline__ uint32_t ss_pad(uint32_t i) { return i + (i >> 5); }

// One round over in[b, min(n, b + SS_ROUND)): out (and wide, when given) get
// carry + the exclusive prefix; returns the round's sum.
__device__ __forceinline__ uint32_t ss_round(const uint32_t *in, uint32_t *out, uint64_t *wide, uint64_t n, uint64_t b,
                                             uint32_t carry, uint32_t *buf, uint32_t *lds)
{
#pragma unroll
    for (int j = 0; j < SS_PT; ++j) {
        const uint64_t e = b + (uint64_t)j * 1024 + threadIdx.x;
        buf[ss_pad(j * 1024 + threadIdx.x)] = e < n ? in[e] : 0u;
    }
    __syncthreads();
    uint32_t v[SS_PT], s = 0;
#pragma unroll
    for (int k = 0; k < SS_PT; ++k) {
        v[k] = buf[ss_pad(SS_PT * threadIdx.x + k)];
        s += v[k];
    }
    uint32_t t;
    uint32_t run = carry + block_excl_scan<1024>(s, lds, &t);   // its barriers order the reads above
#pragma unroll
    for (int k = 0; k < SS_PT; ++k) {
        buf[ss_pad(SS_PT * threadIdx.x + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SS_PT; ++j) {
        const uint64_t e = b + (uint64_t)j * 1024 + threadIdx.x;
        if (e < n) {
            const uint32_t r = buf[ss_pad(j * 1024 + threadIdx.x)];
            out[e] = r;
            if (wide) wide[e] = r;
        }
    }
    __syncthreads();   // the next round refills buf
    return t;
}

__global__ __launch_bounds__(1024) void k_scan_small(const uint32_t *in, uint32_t *out, uint64_t n,
                                                     const uint32_t *n_dev, uint32_t *total)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    __shared__ uint32_t buf[SS_ROUND + SS_ROUND / 32];
    if (n_dev && *n_dev < n) n = *n_dev;
    uint32_t carry = 0;
    for (uint64_t b = 0; b < n; b += SS_ROUND) carry += ss_round(in, out, nullptr, n, b, carry, buf, lds);
    if (threadIdx.x == 0 && total) *total = carry;
}

// Block b scans its own array (b = 0: in0 into out0 and out0_wide; b = 1:
// in1 into out1), SS_ROUND values per round with a running carry.
__global__ __launch_bounds__(1024) void k_scan_pair(const uint32_t *in0, uint32_t *out0, uint64_t *out0_wide,
                                                    uint64_t n0, const uint32_t *in1, uint32_t *out1, uint64_t n1)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    __shared__ uint32_t buf[SS_ROUND + SS_ROUND / 32];
    const uint32_t *in = blockIdx.x ? in1 : in0;
    uint32_t *out = blockIdx.x ? out1 : out0;
    uint64_t *wide = blockIdx.x ? nullptr : out0_wide;
    const uint64_t n = blockIdx.x ? n1 : n0;
    uint32_t carry = 0;
    for (uint64_t b = 0; b < n; b += SS_ROUND) carry += ss_round(in, out, wide, n, b, carry, buf, lds);
}

void scan_exclusive_pair(const uint32_t *in0, uint32_t *out0, uint64_t *out0_wide, uint64_t n0, const uint32_t *in1,
                         uint32_t *out1, uint64_t n1, hipStream_t st)
{
    if (n0 == 0 && n1 == 0) return;
    hipLaunchKernelGGL(k_scan_pair, dim3(2), dim3(1024), 0, st, in0, out0, out0_wide, n0, in1, out1, n1);
}

size_t scan_temp_bytes(uint64_t n)
{
    const uint64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    return ((tiles + 1) * 4 + 255) & ~(size_t)255;
}

void scan_exclusive(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total, void *temp, hipStream_t st)
{
    if (n == 0) {
        if (total) launch_fill_u32(total, 0u, 1, st);
        return;
    }
    if (n <= SCAN_SMALL_MAX) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, in, out, n, nullptr, total);
        return;
    }
    const uint32_t tiles = div_up(n, SCAN_TILE);
    uint32_t *ts = static_cast<uint32_t *>(temp);
    hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(SCAN_BLOCK), 0, st, in, n, nullptr, ts);
    if (tiles <= SCAN_FUSED_TILES) {
        hipLaunchKernelGGL(k_scan_down<true>, dim3(tiles), dim3(SCAN_BLOCK), 0, st, in, out, n, nullptr, ts, total);
        return;
    }
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, ts, tiles, total);
    hipLaunchKernelGGL(k_scan_down<false>, dim3(tiles), dim3(SCAN_BLOCK), 0, st, in, out, n, nullptr, ts, nullptr);
}

void scan_exclusive_dev(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint64_t n_max, void *temp,
                        hipStream_t st)
{
    if (n_max == 0) return;
    if (n_max <= SCAN_SMALL_MAX) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, in, out, n_max, n_dev, nullptr);
        return;
    }
    const uint32_t tiles = div_up(n_max, SCAN_TILE);
    uint32_t *ts = static_cast<uint32_t *>(temp);
    hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(SCAN_BLOCK), 0, st, in, n_max, n_dev, ts);
    if (tiles <= SCAN_FUSED_TILES) {
        hipLaunchKernelGGL(k_scan_down<true>, dim3(tiles), dim3(SCAN_BLOCK), 0, st, in, out, n_max, n_dev, ts,
                           nullptr);
        return;
    }
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, ts, tiles, nullptr);
    hipLaunchKernelGGL(k_scan_down<false>, dim3(tiles), dim3(SCAN_BLOCK), 0, st, in, out, n_max, n_dev, ts, nullptr);
}


// ---- stable multisplit ------------------------------------------------------------------------
// Counting sort of n elements by a key with at most MS_MAX_BINS buckets per
// pass, stable (equal keys keep their input order).  Input ranges can be cut
// into segments, each with its own contiguous range of buckets (a segment's
// tiles only see its own buckets, so the count matrix stays small).
//
// Tile = MS_TILE elements.  Wave w owns the contiguous sub-tile [w*T/4,
// (w+1)*T/4) and walks it in rounds of 64 lanes in input order; inside a
// round, ranks among equal keys come from a ballot match over the key bits.
// The scatter stages the tile in LDS in bucket order and then writes whole
// bucket runs, so global writes are coalesced.

// Keys of items wlo + r*64 + lane, r < N, of a tile ending at hi (hi > the
// tile's first element).  Indices past hi are clamped to hi - 1, so every load
// is in bounds and none waits on a branch; the caller masks those items.  The
// key source is chosen once, and all first-level loads are issued before the
// dependent table loads.
template <int N>
__device__ __forceinline__ void ms_load_keys(const MsArgs &A, uint64_t wlo, uint64_t hi, int lane, uint32_t (&full)[N])
{
    if (A.keys) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const uint64_t e = wlo + (uint64_t)r * 64 + lane;
            full[r] = A.keys[e < hi ? e : hi - 1];
        }
    } else {
        uint64_t c[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const uint64_t e = wlo + (uint64_t)r * 64 + lane;
            c[r] = A.code[e < hi ? e : hi - 1];
        }
#pragma unroll
        for (int r = 0; r < N; ++r) full[r] = cut_find(A.cut, c[r] >> A.code_shift);
    }
}

// Tile t -> [lo, hi), its segment's bucket range, count-matrix location.
struct MsTile {
    uint64_t lo, hi;
    uint32_t b0, nb, mat, ntile, tis;
    bool ok;
};

template <bool SEG, int IT>
__device__ __forceinline__ MsTile ms_tile(const MsArgs &A, uint32_t t)
{
    constexpr uint32_t TILE = MS_BLOCK * IT;
    MsTile T{};
    if (!SEG) {
        T.lo = (uint64_t)t * TILE;
        T.hi = T.lo + TILE < A.n ? T.lo + TILE : A.n;
        T.b0 = 0;
        T.nb = A.nbins;
        T.mat = 0;
        T.ntile = A.tiles;
        T.tis = t;
        T.ok = t < A.tiles;
        return T;
    }
    T.ok = t < *A.seg_total_tiles;
    if (!T.ok) return T;
    uint32_t lo = 0, hi = A.nseg;   // last segment with tile_first <= t
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A.seg_tile_first[mid] <= t) lo = mid; else hi = mid;
    }
    const uint32_t sgm = lo;
    T.tis = t - A.seg_tile_first[sgm];
    const uint64_t sb = A.seg_begin[sgm], se = A.seg_begin[sgm] + A.seg_len[sgm];
    T.lo = sb + (uint64_t)T.tis * TILE;
    T.hi = T.lo + TILE < se ? T.lo + TILE : se;
    T.b0 = A.seg_b0[sgm];
    T.nb = A.seg_nb[sgm];
    T.mat = A.seg_mat[sgm];
    T.ntile = A.seg_tile_first[sgm + 1] - A.seg_tile_first[sgm];
    return T;
}

// Count pass: equal keys of a wave round are grouped by a ballot match and
// added once (consecutive points usually share their chunk), so LDS atomics
// do not pile up on one counter.  The segmented split (work chunks inside a
// chunk) adds each element on its own (20M planes: subsample region 0.532 ->
// 0.518 ms).
template <bool SEG, int IT = MS_ITEMS>
__global__ __launch_bounds__(MS_BLOCK) void k_ms_count(MsArgs A)
{
    constexpr int PER_WAVE = IT * 64;
    __shared__ uint32_t hist[MS_MAX_BINS];
    const MsTile T = ms_tile<SEG, IT>(A, blockIdx.x);
    if (!T.ok) return;
    const int w = threadIdx.x >> 6, lane = lane_id();
    const uint64_t wlo = T.lo + (uint64_t)w * PER_WAVE;
    // all loads of the tile first, so their latencies overlap
    uint32_t full[IT];
    ms_load_keys(A, wlo, T.hi, lane, full);
    for (uint32_t b = threadIdx.x; b < T.nb; b += MS_BLOCK) hist[b] = 0;
    __syncthreads();
    const uint32_t dmask = (1u << A.dbits) - 1u;
    const int nbits = (int)ceil_log2_dev(T.nb);
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint64_t e = wlo + (uint64_t)r * 64 + lane;
        const bool valid = e < T.hi;
        const uint32_t key = valid ? ((full[r] >> A.shift) & dmask) - T.b0 : 0u;
        if constexpr (SEG) {
            // work-chunk keys in chunk order rarely repeat inside a round:
            // one atomic per element is cheaper than the ballot match
            if (valid) atomicAdd(&hist[key], 1u);
        } else {
            const uint64_t peers = match_peers(key, valid, nbits);
            if (valid && (peers & ((1ull << lane) - 1ull)) == 0) atomicAdd(&hist[key], (uint32_t)__popcll(peers));
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < T.nb; b += MS_BLOCK)
        A.counts[(uint64_t)T.mat + (uint64_t)b * T.ntile + T.tis] = hist[b];
}

// ONE (unsegmented, at most MS_ONE_PASS_BINS buckets, known bucket starts):
// no counting pass.  A tile takes its number from a ticket counter, so every
// tile before it has started; it publishes its count per bucket, then walks
// back over the tiles before it, bucket by bucket, until one has published its
// inclusive prefix (a decoupled look-back), and publishes its own.
constexpr uint64_t MS_AGG = 1ull << 62, MS_PREFIX = 2ull << 62, MS_VALUE = (1ull << 62) - 1ull;
constexpr uint32_t MS_ONE_PER = MS_ONE_PASS_BINS / MS_BLOCK;   // buckets per thread
constexpr int MS_WINDOW = 8;                                  // look-back words per round trip
// The look-back is a chain across the tiles: with thousands of tiles it cost
// more than the counting pass it saves (20M points: 0.26 against 0.21 ms for
// the whole split; 1M points: 0.037 against 0.043 ms), so it is used up to
// this many tiles.
constexpr uint32_t MS_ONE_PASS_TILES = 1024;

template <bool SEG, int IT = MS_ITEMS, bool ONE = false>
__global__ __launch_bounds__(MS_BLOCK) void k_ms_scatter(MsArgs A)
{
    static_assert(!(SEG && ONE), "the one-pass split is unsegmented");
    constexpr uint32_t TILE = MS_BLOCK * IT;
    constexpr int W = MS_BLOCK / 64;
    constexpr int PER_WAVE = IT * 64;
    __shared__ uint16_t pre[W][MS_MAX_BINS];
    __shared__ uint32_t gbase[MS_MAX_BINS];   // global position of local slot 0 of a bucket (mod 2^32)
    __shared__ unsigned long long stage[TILE];   // (key, value) pairs, then payloads
    // scan scratch, in the stage (unused until phase 3): 40 KB in all, four
    // blocks per compute unit
    uint32_t *red = reinterpret_cast<uint32_t *>(stage);
    uint32_t tile = blockIdx.x;
    if constexpr (ONE) {
        // the ticket passes through the last bucket base, which a one-pass
        // split (at most MS_ONE_PASS_BINS buckets) never uses
        static_assert(MS_ONE_PASS_BINS < MS_MAX_BINS, "a spare bucket base");
        if (threadIdx.x == 0) gbase[MS_MAX_BINS - 1] = atomicAdd(A.tile_ctr, 1u);
        __syncthreads();
        tile = gbase[MS_MAX_BINS - 1];
    }
    const MsTile T = ms_tile<SEG, IT>(A, tile);
    if (!T.ok) return;
    const int w = threadIdx.x >> 6, lane = lane_id();
    const uint32_t dmask = (1u << A.dbits) - 1u;
    const int nbits = (int)ceil_log2_dev(T.nb);
    // all loads of the tile first (keys, values, payloads), so their
    // latencies overlap
    const uint64_t wlo = T.lo + (uint64_t)w * PER_WAVE;
    uint32_t full[IT], val[IT];
    unsigned long long pay[IT];
    ms_load_keys(A, wlo, T.hi, lane, full);
    if (A.vals) {
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const uint64_t e = wlo + (uint64_t)r * 64 + lane;
            val[r] = A.vals[e < T.hi ? e : T.hi - 1];
        }
    } else {
#pragma unroll
        for (int r = 0; r < IT; ++r) val[r] = (uint32_t)(wlo + (uint64_t)r * 64 + lane);
    }
    if (A.pay) {
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const uint64_t e = wlo + (uint64_t)r * 64 + lane;
            pay[r] = A.pay[e < T.hi ? e : T.hi - 1];
        }
    } else {
#pragma unroll
        for (int r = 0; r < IT; ++r) pay[r] = wlo + (uint64_t)r * 64 + lane;
    }
    for (uint32_t b = threadIdx.x; b < T.nb; b += MS_BLOCK)
        for (int k = 0; k < W; ++k) pre[k][b] = 0;
    __syncthreads();
    // phase 1: per-wave running counts; each lane keeps its offset inside its wave
    uint16_t wof[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint64_t e = wlo + (uint64_t)r * 64 + lane;
        const bool valid = e < T.hi;
        const uint32_t key = valid ? ((full[r] >> A.shift) & dmask) - T.b0 : 0u;
        const uint64_t peers = match_peers(key, valid, nbits);
        const uint64_t lt = peers & ((1ull << lane) - 1ull);
        const uint32_t before = valid ? pre[w][key] : 0u;
        wof[r] = (uint16_t)(before + __popcll(lt));
        if (valid && lt == 0) pre[w][key] = (uint16_t)(before + __popcll(peers));
    }
    __syncthreads();
    // phase 2: bucket starts inside the tile (exclusive scan over buckets, each
    // thread owning a run of consecutive buckets), per-wave bases, global bases
    {
        const uint32_t per = (T.nb + MS_BLOCK - 1) / MS_BLOCK;
        const uint32_t b0 = threadIdx.x * per;
        uint32_t sum = 0;
        for (uint32_t b = b0; b < b0 + per && b < T.nb; ++b)
            for (int k = 0; k < W; ++k) sum += pre[k][b];
        uint32_t tot;
        uint32_t run = block_excl_scan<MS_BLOCK>(sum, red, &tot);
        if constexpr (ONE) {
            uint32_t loffs[MS_ONE_PER], hs[MS_ONE_PER];
#pragma unroll
            for (uint32_t q = 0; q < MS_ONE_PER; ++q) {
                const uint32_t b = b0 + q;
                if (q >= per || b >= T.nb) break;
                loffs[q] = run;
                for (int k = 0; k < W; ++k) {
                    const uint32_t h = pre[k][b];
                    pre[k][b] = (uint16_t)run;
                    run += h;
                }
                hs[q] = run - loffs[q];
                unsigned long long *st = A.status + (uint64_t)tile * A.nbins + b;
                fr_store(st, (tile == 0 ? MS_PREFIX : MS_AGG) | hs[q]);
            }
#pragma unroll
            for (uint32_t q = 0; q < MS_ONE_PER; ++q) {
                const uint32_t b = b0 + q;
                if (q >= per || b >= T.nb) break;
                uint64_t excl = 0;
                if (tile > 0) {
                    // MS_WINDOW predecessors' words per round trip, walked in order
                    int64_t j = (int64_t)tile - 1;
                    uint64_t spins = 0;
                    bool done = false;
                    while (!done) {
                        uint64_t wd[MS_WINDOW];
#pragma unroll
                        for (int u = 0; u < MS_WINDOW; ++u)
                            wd[u] = j - u >= 0 ? fr_load(A.status + (uint64_t)(j - u) * A.nbins + b) : MS_PREFIX;
                        int used = 0;
#pragma unroll
                        for (int u = 0; u < MS_WINDOW; ++u) {
                            if (done || used < u || wd[u] == 0) continue;   // stop at the first unpublished word
                            excl += wd[u] & MS_VALUE;
                            used = u + 1;
                            done = (wd[u] & ~MS_VALUE) == MS_PREFIX || j - u == 0;
                        }
                        j -= used;
                        if (!done && used < MS_WINDOW && ++spins > FR_SPIN_LIMIT) {   // never expected: report
                            atomicOr(A.err, 1u);
                            done = true;
                        }
                    }
                    fr_store(A.status + (uint64_t)tile * A.nbins + b, MS_PREFIX | (excl + hs[q]));
                }
                gbase[b] = (uint32_t)A.bucket_begin[b] + (uint32_t)excl - loffs[q];
            }
        } else {
            for (uint32_t b = b0; b < b0 + per && b < T.nb; ++b) {
                const uint32_t loff = run;
                for (int k = 0; k < W; ++k) {
                    const uint32_t h = pre[k][b];
                    pre[k][b] = (uint16_t)run;
                    run += h;
                }
                gbase[b] = A.offsets[(uint64_t)T.mat + (uint64_t)b * T.ntile + T.tis] - loff;
            }
        }
    }
    __syncthreads();
    // phase 3: stage (key, value) in bucket order
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        const uint64_t e = wlo + (uint64_t)r * 64 + lane;
        if (e >= T.hi) continue;
        const uint32_t key = ((full[r] >> A.shift) & dmask) - T.b0;
        const uint32_t slot = pre[w][key] + wof[r];
        stage[slot] = ((unsigned long long)full[r] << 32) | val[r];
        wof[r] = (uint16_t)slot;
    }
    __syncthreads();
    // phase 4: write bucket runs
    const uint32_t cnt = (uint32_t)(T.hi - T.lo);
    uint32_t gp[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const uint32_t k = i * MS_BLOCK + threadIdx.x;
        if (k >= cnt) continue;
        const unsigned long long kv = stage[k];
        const uint32_t fk = (uint32_t)(kv >> 32);
        const uint32_t key = ((fk >> A.shift) & dmask) - T.b0;
        const uint32_t pos = gbase[key] + k;
        gp[i] = pos;
        if (A.vals_out) A.vals_out[pos] = (uint32_t)kv;
        if (A.keys_out) A.keys_out[pos] = fk;
    }
    if (A.src_out || A.pay_out) {
        // the input position (and payload) of every slot, through the same stage
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const uint64_t e = wlo + (uint64_t)r * 64 + lane;
            if (e >= T.hi) continue;
            stage[wof[r]] = pay[r];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t k = i * MS_BLOCK + threadIdx.x;
            if (k >= cnt) continue;
            if (A.pay_out) A.pay_out[gp[i]] = stage[k];
            if (A.cut2_out) A.cut2_out[gp[i]] = cut_find(A.cut2, stage[k] >> A.cut2_shift);
        }
        if (A.src_out && A.pay_out) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                const uint64_t e = wlo + (uint64_t)r * 64 + lane;
                if (e >= T.hi) continue;
                stage[wof[r]] = e;
            }
            __syncthreads();
        }
        if (A.src_out) {
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t k = i * MS_BLOCK + threadIdx.x;
                if (k >= cnt) continue;
                A.src_out[gp[i]] = (uint32_t)stage[k];
            }
        }
    }
}

// Segment preparation: tiles per segment and count-matrix cells per segment.
__global__ void k_ms_seg_prep(uint32_t nseg, const uint32_t *len, const uint32_t *nb, uint32_t *ntile, uint32_t *cells,
                              uint32_t tile)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) ntile[nseg] = 0;
    for (uint32_t sg = blockIdx.x * blockDim.x + threadIdx.x; sg < nseg; sg += gridDim.x * blockDim.x) {
        const uint32_t t = (len[sg] + tile - 1) / tile;
        ntile[sg] = t;
        cells[sg] = t * nb[sg];
    }
}

// The same for at most SEG_PREP_ONE segments in one block, with both scans:
// tile_first (nseg + 1 entries, the last = all tiles), mat, tot[0] = tiles,
// tot[1] = cells.
constexpr uint32_t SEG_PREP_ONE = 1024;
__global__ __launch_bounds__(SEG_PREP_ONE) void k_ms_seg_prep_one(uint32_t nseg, const uint32_t *len,
                                                                  const uint32_t *nb, uint32_t tile,
                                                                  uint32_t *tile_first, uint32_t *mat, uint32_t *tot)
{
    __shared__ uint32_t lds[SEG_PREP_ONE / 64 + 1];
    const uint32_t sg = threadIdx.x;
    uint32_t t = 0, c = 0;
    if (sg < nseg) {
        t = (len[sg] + tile - 1) / tile;
        c = t * nb[sg];
    }
    uint32_t tiles, cells;
    const uint32_t et = block_excl_scan<SEG_PREP_ONE>(t, lds, &tiles);
    const uint32_t ec = block_excl_scan<SEG_PREP_ONE>(c, lds, &cells);
    if (sg < nseg) {
        tile_first[sg] = et;
        mat[sg] = ec;
    }
    if (sg == 0) {
        tile_first[nseg] = tiles;
        tot[0] = tiles;
        tot[1] = cells;
    }
}

struct MsLayout {
    uint32_t passes, dbits[4], shift[4], nb[4];
    uint32_t tiles;
    uint64_t counts_words;
};

// With many buckets a tile's elements fall into short runs per bucket (344
// chunks of 200M points: about six of a tile's 2048 per bucket), and the
// scatter's writes, spread over hundreds of destinations per tile, ran at a
// third of its rate with long runs.  Two stable passes by digits of half the
// key bits (LSD order) keep the runs long: twice the bytes, still faster
// (200M points, 344 chunks: the chunk split 5.6 -> 4.8 ms).
constexpr uint32_t MS_TWO_PASS_BINS = 128;
constexpr uint64_t MS_TWO_PASS_MIN_N = 1ull << 24;

static MsLayout ms_layout(uint64_t n, uint32_t nbins)
{
    MsLayout L{};
    L.tiles = div_up(n ? n : 1, MS_TILE);
    const uint32_t bits = ceil_log2(nbins);
    const bool two = nbins >= MS_TWO_PASS_BINS && n >= MS_TWO_PASS_MIN_N;
    if (nbins <= MS_ONE_PASS_BINS && !two) {
        L.passes = 1;
        L.dbits[0] = bits;
        L.nb[0] = nbins;
        L.shift[0] = 0;
    } else {
        L.passes = (bits + MS_DIGIT_BITS - 1) / MS_DIGIT_BITS;
        if (L.passes < 2) L.passes = 2;
        const uint32_t per = (bits + L.passes - 1) / L.passes;
        uint32_t done = 0;
        for (uint32_t p = 0; p < L.passes; ++p) {
            const uint32_t b = (bits - done) < per ? (bits - done) : per;
            L.dbits[p] = b;
            L.nb[p] = 1u << b;
            L.shift[p] = done;
            done += b;
        }
    }
    uint32_t maxnb = 0;
    for (uint32_t p = 0; p < L.passes; ++p) maxnb = L.nb[p] > maxnb ? L.nb[p] : maxnb;
    L.counts_words = (uint64_t)maxnb * L.tiles;
    return L;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t multisplit_temp_bytes(uint64_t n, uint32_t nbins)
{
    const MsLayout L = ms_layout(n, nbins);
    size_t b = 2 * align256(L.counts_words * 4) + scan_temp_bytes(L.counts_words);
    if (L.passes > 1) b += 2 * (align256(n * 4) * 2 + align256(n * 8));
    return b;
}

size_t multisplit_temp_bound(uint64_t n, uint64_t max_bins)
{
    // the largest single pass and the multi-pass form (digits of at most
    // MS_DIGIT_BITS bits)
    const uint32_t one = (uint32_t)(max_bins < MS_ONE_PASS_BINS ? max_bins : MS_ONE_PASS_BINS);
    size_t b = multisplit_temp_bytes(n, one ? one : 1);
    if (max_bins > MS_ONE_PASS_BINS) {
        const uint64_t tiles = div_up(n ? n : 1, MS_TILE);
        const uint64_t w = (1ull << MS_DIGIT_BITS) * tiles;
        const size_t m = 2 * align256(w * 4) + scan_temp_bytes(w) + 2 * (align256(n * 4) * 2 + align256(n * 8));
        if (m > b) b = m;
    }
    return b;
}

void multisplit(const MsInput &in, uint64_t n, uint32_t nbins, const MsOutput &out, void *temp, hipStream_t st,
                LaunchTimer *scatter_timer)
{
    if (n == 0) return;
    const MsLayout L = ms_layout(n, nbins);
    char *p = static_cast<char *>(temp);
    uint32_t *counts = reinterpret_cast<uint32_t *>(p); p += align256(L.counts_words * 4);
    uint32_t *offs = reinterpret_cast<uint32_t *>(p); p += align256(L.counts_words * 4);
    void *stemp = p; p += scan_temp_bytes(L.counts_words);
    uint32_t *kb[2] = {nullptr, nullptr}, *vb[2] = {nullptr, nullptr};
    uint64_t *pb[2] = {nullptr, nullptr};
    if (L.passes > 1) {
        for (int i = 0; i < 2; ++i) {
            kb[i] = reinterpret_cast<uint32_t *>(p); p += align256(n * 4);
            vb[i] = reinterpret_cast<uint32_t *>(p); p += align256(n * 4);
            pb[i] = reinterpret_cast<uint64_t *>(p); p += align256(n * 8);
        }
    }
    MsArgs A{};
    A.n = n;
    A.keys = in.keys;
    A.code = in.code;
    A.cut = in.cut;
    A.code_shift = in.code_shift;
    A.vals = in.vals;
    A.pay = in.pay;
    A.tiles = L.tiles;
    A.counts = counts;
    A.offsets = offs;
    if (in.bucket_begin && L.passes == 1 && L.tiles <= MS_ONE_PASS_TILES) {
        // one pass: the count matrix's two arrays hold the status words (a
        // 64-bit word per tile and bucket), the scan's temporary the ticket
        // counter; all cleared by one fill
        A.shift = L.shift[0];
        A.dbits = L.dbits[0];
        A.nbins = L.nb[0];
        A.vals_out = out.vals;
        A.keys_out = out.keys;
        A.pay_out = out.pay;
        A.src_out = out.src;
        A.bucket_begin = in.bucket_begin;
        A.cut2_out = out.cut2_keys;
        A.cut2 = out.cut2;
        A.cut2_shift = out.cut2_shift;
        A.status = reinterpret_cast<unsigned long long *>(counts);
        A.tile_ctr = static_cast<uint32_t *>(stemp);
        A.err = in.err;
        launch_fill_u32(counts, 0u, (static_cast<char *>(stemp) - reinterpret_cast<char *>(counts)) / 4 + 1, st);
        if (scatter_timer) scatter_timer->begin(st);
        hipLaunchKernelGGL((k_ms_scatter<false, MS_ITEMS, true>), dim3(L.tiles), dim3(MS_BLOCK), 0, st, A);
        if (scatter_timer) scatter_timer->end(st);
        return;
    }
    for (uint32_t ps = 0; ps < L.passes; ++ps) {
        const bool last = ps + 1 == L.passes;
        A.shift = L.shift[ps];
        A.dbits = L.dbits[ps];
        A.nbins = L.nb[ps];
        A.vals_out = last ? out.vals : vb[ps & 1];
        A.keys_out = last ? out.keys : kb[ps & 1];
        A.pay_out = last ? out.pay : (in.pay ? pb[ps & 1] : nullptr);
        A.src_out = (last && ps == 0) ? out.src : nullptr;
        A.cut2_out = last ? out.cut2_keys : nullptr;
        A.cut2 = out.cut2;
        A.cut2_shift = out.cut2_shift;
        hipLaunchKernelGGL(k_ms_count<false>, dim3(L.tiles), dim3(MS_BLOCK), 0, st, A);
        scan_exclusive(counts, offs, (uint64_t)L.nb[ps] * L.tiles, nullptr, stemp, st);
        if (scatter_timer) scatter_timer->begin(st);
        hipLaunchKernelGGL(k_ms_scatter<false>, dim3(L.tiles), dim3(MS_BLOCK), 0, st, A);
        if (scatter_timer) scatter_timer->end(st);
        A.keys = A.keys_out;
        A.code = nullptr;
        A.vals = A.vals_out;
        A.pay = A.pay_out;
    }
}

size_t multisplit_seg_temp_bytes(uint64_t n, uint32_t nseg, uint64_t max_cells)
{
    return 5 * align256(4ull * (nseg + 1)) + 2 * align256(4 * max_cells) + scan_temp_bytes(max_cells > nseg + 1 ? max_cells : nseg + 1) + 256;
}

void multisplit_segmented(const MsInput &in, uint64_t n, const MsSegments &sg, uint64_t max_tiles,
                          const MsOutput &out, void *temp, hipStream_t st)
{
    if (n == 0 || sg.nseg == 0) return;
    char *p = static_cast<char *>(temp);
    uint32_t *ntile = reinterpret_cast<uint32_t *>(p); p += align256(4ull * (sg.nseg + 1));
    uint32_t *cells = reinterpret_cast<uint32_t *>(p); p += align256(4ull * (sg.nseg + 1));
    uint32_t *tile_first = reinterpret_cast<uint32_t *>(p); p += align256(4ull * (sg.nseg + 1));
    uint32_t *mat = reinterpret_cast<uint32_t *>(p); p += align256(4ull * (sg.nseg + 1));
    uint32_t *tot = reinterpret_cast<uint32_t *>(p); p += align256(4ull * (sg.nseg + 1));
    uint32_t *counts = reinterpret_cast<uint32_t *>(p); p += align256(4 * sg.max_cells);
    uint32_t *offs = reinterpret_cast<uint32_t *>(p); p += align256(4 * sg.max_cells);
    void *stemp = p;
    if (sg.nseg <= SEG_PREP_ONE) {
        hipLaunchKernelGGL(k_ms_seg_prep_one, dim3(1), dim3(SEG_PREP_ONE), 0, st, sg.nseg, sg.len, sg.nb, MS_SEG_TILE,
                           tile_first, mat, tot);
    } else {
        hipLaunchKernelGGL(k_ms_seg_prep, dim3(div_up(sg.nseg, 256)), dim3(256), 0, st, sg.nseg, sg.len, sg.nb, ntile,
                           cells, MS_SEG_TILE);
        // tile_first has nseg + 1 entries (the last one = total tiles)
        scan_exclusive(ntile, tile_first, sg.nseg + 1, tot, stemp, st);
        scan_exclusive(cells, mat, sg.nseg, tot + 1, stemp, st);
    }
    MsArgs A{};
    A.n = n;
    A.keys = in.keys;
    A.code = in.code;
    A.cut = in.cut;
    A.code_shift = in.code_shift;
    A.vals = in.vals;
    A.pay = in.pay;
    A.shift = 0;
    A.dbits = 31;
    A.counts = counts;
    A.offsets = offs;
    A.nseg = sg.nseg;
    A.seg_begin = sg.begin;
    A.seg_len = sg.len;
    A.seg_b0 = sg.b0;
    A.seg_nb = sg.nb;
    A.seg_mat = mat;
    A.seg_tile_first = tile_first;
    A.seg_total_tiles = tot;
    A.vals_out = out.vals;
    A.keys_out = out.keys;
    A.pay_out = out.pay;
    A.src_out = out.src;
    hipLaunchKernelGGL((k_ms_count<true, MS_SEG_ITEMS>), dim3((uint32_t)max_tiles), dim3(MS_BLOCK), 0, st, A);
    scan_exclusive_dev(counts, offs, tot + 1, sg.max_cells, stemp, st);
    hipLaunchKernelGGL((k_ms_scatter<true, MS_SEG_ITEMS>), dim3((uint32_t)max_tiles), dim3(MS_BLOCK), 0, st, A);
}

// ---- step 4: per-node grid subsample -----------------------------------------------------------
//
// Work chunks (WCs) are the maximal pyramid nodes holding at most WC_CAP
// points, at levels d0 = max(0, g - s) to g.  The subsample cells of a node
// at depth d lie at lattice level d + s; from depth d0 on (d + s >= g >= lw)
// they never straddle two WCs, so each cell's lowest-index point is found
// inside one WC.  The shared depths above d0 (cells spanning several WCs)
// are decided first by a global pass over all points.  The only other
// cross-WC question is whether a node above a WC (a "shared" node, depth
// < lw) is inner or a leaf, which depends on how many points reach it.  Each
// WC therefore runs its subtree assuming its shared ancestors are inner,
// posting its reaching count at every shared depth; a top-down pass then
// finds the first shared leaf of each WC (its "cut"), and points whose
// tentative depth is at or below the cut belong to that leaf.

// Global shared depths d < d0, in work-chunk order.  Every alive point
// (state 0xff) offers its original index to its cell of level d + s; with
// the table of depth d - 1 given (prev), a point first checks whether it
// holds its cell's minimum there, and then stays at depth d - 1 instead (the
// marking of depth d - 1 rides on this pass).  The
// order is spatially coherent, so a tile of GD_TILE consecutive points falls
// in few cells: the tile keeps the minimum of each of its cells in an LDS
// hash table (at least twice as many slots as points, so it never fills),
// lists the slots it takes, and flushes one global atomic per distinct cell,
// clearing just those slots for the next tile.
constexpr int GD_BLOCK = 256, GD_ITEMS = 8;   // (item j of a wave: 64 consecutive points)
constexpr uint32_t GD_TILE = GD_BLOCK * GD_ITEMS;   // 2048 points
constexpr uint32_t GD_HASH = 2 * GD_TILE;           // slots
__global__ __launch_bounds__(GD_BLOCK) void k_gdepth_min(const uint64_t *__restrict__ code,
                                                         const uint32_t *__restrict__ orig,
                                                         uint8_t *__restrict__ t, uint64_t n, int csh,
                                                         uint32_t *gtab, const uint32_t *__restrict__ prev,
                                                         int csh_prev, int d_prev)
{
    __shared__ uint32_t hk[GD_HASH], hv[GD_HASH];
    __shared__ uint16_t taken[GD_TILE];   // slots in use (at most one per point of the tile)
    __shared__ uint32_t used;
    for (uint32_t h = threadIdx.x; h < GD_HASH; h += GD_BLOCK) {
        hk[h] = 0xffffffffu;
        hv[h] = 0xffffffffu;
    }
    if (threadIdx.x == 0) used = 0;
    __syncthreads();
    const uint64_t tiles = (n + GD_TILE - 1) / GD_TILE;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        // cells of level d + s < g number at most 8^8, so a cell id fits 32 bits
        uint32_t cell[GD_ITEMS], o[GD_ITEMS];
#pragma unroll
        for (int j = 0; j < GD_ITEMS; ++j) {
            const uint64_t q = tile * GD_TILE + (uint64_t)j * GD_BLOCK + threadIdx.x;
            bool alive = q < n && t[q] == 0xffu;
            const uint64_t c = alive ? code[q] : 0ull;
            const uint32_t oi = alive ? orig[q] : 0xffffffffu;
            if (prev && alive && prev[c >> csh_prev] == oi) {   // the winner of its cell at depth d - 1
                t[q] = (uint8_t)d_prev;
                alive = false;
            }
            cell[j] = alive ? (uint32_t)(c >> csh) : 0xffffffffu;
            o[j] = alive ? oi : 0xffffffffu;
        }
#pragma unroll
        for (int j = 0; j < GD_ITEMS; ++j) {
            // a point whose left neighbour (the previous point, one lane down)
            // offers the same cell a smaller index cannot be the minimum:
            // inside a work chunk the indices ascend, so a run of one cell
            // sends one offer
            const uint32_t pc = (uint32_t)__shfl_up((int)cell[j], 1, 64), po = (uint32_t)__shfl_up((int)o[j], 1, 64);
            if (cell[j] == 0xffffffffu || (lane_id() > 0 && pc == cell[j] && po < o[j])) continue;
            uint32_t h = hash32(cell[j]) & (GD_HASH - 1);
            for (;;) {   // linear probing; the table is at most half full
                uint32_t k = hk[h];
                if (k == 0xffffffffu) {
                    k = atomicCAS(&hk[h], 0xffffffffu, cell[j]);
                    if (k == 0xffffffffu) {
                        taken[atomicAdd(&used, 1u)] = (uint16_t)h;
                        break;
                    }
                }
                if (k == cell[j]) break;
                h = (h + 1) & (GD_HASH - 1);
            }
            atomicMin(&hv[h], o[j]);
        }
        __syncthreads();
        const uint32_t nu = used;
        for (uint32_t i = threadIdx.x; i < nu; i += GD_BLOCK) {
            const uint32_t h = taken[i];
            atomicMin(&gtab[hk[h]], hv[h]);
            hk[h] = 0xffffffffu;
            hv[h] = 0xffffffffu;
        }
        __syncthreads();
        if (threadIdx.x == 0) used = 0;
        __syncthreads();
    }
}

// Rows of the global shared depths: points of each WC alive at depth d < d0
// (d0 = g - s <= 9), one block per WC: every thread marks the winners of the
// last global depth (alive points holding their cell's minimum in `last`),
// counts its points placed at each global depth, and the block sums them in
// LDS.
constexpr int AR_BLOCK = 256;
constexpr int AR_IT = 8;
constexpr int AR_MAXD0 = 10;   // global depths d < d0 <= 9
__global__ __launch_bounds__(AR_BLOCK) void k_wc_alive_rows(WcArgs a, const uint32_t *__restrict__ last, int csh_last)
{
    __shared__ uint32_t placed[AR_MAXD0];
    const int d0 = a.d0 < AR_MAXD0 ? a.d0 : AR_MAXD0;
    for (uint32_t w = blockIdx.x; w < a.num_wc; w += gridDim.x) {
        if (threadIdx.x < AR_MAXD0) placed[threadIdx.x] = 0;
        __syncthreads();
        const uint32_t base = a.wc_begin[w], n = a.wc_count[w];
        uint32_t c[AR_MAXD0];
#pragma unroll
        for (int d = 0; d < AR_MAXD0; ++d) c[d] = 0;
        // AR_IT points per thread and round, each level of loads (state,
        // then code and index, then the table) issued before it is used
        for (uint32_t p0 = 0; p0 < n; p0 += AR_BLOCK * AR_IT) {
            uint32_t t[AR_IT], oi[AR_IT], win[AR_IT];
            uint64_t cd[AR_IT];
#pragma unroll
            for (int k = 0; k < AR_IT; ++k) {
                const uint32_t p = p0 + (uint32_t)k * AR_BLOCK + threadIdx.x;
                t[k] = p < n ? a.t[base + p] : 0xfeu;
            }
#pragma unroll
            for (int k = 0; k < AR_IT; ++k) {
                const uint32_t p = p0 + (uint32_t)k * AR_BLOCK + threadIdx.x;
                cd[k] = t[k] == 0xffu ? a.wc_code[base + p] : 0ull;
                oi[k] = t[k] == 0xffu ? a.wc_orig[base + p] : 0u;
            }
#pragma unroll
            for (int k = 0; k < AR_IT; ++k) win[k] = t[k] == 0xffu ? last[cd[k] >> csh_last] : 0xffffffffu;
#pragma unroll
            for (int k = 0; k < AR_IT; ++k) {
                const uint32_t p = p0 + (uint32_t)k * AR_BLOCK + threadIdx.x;
                if (t[k] == 0xffu && win[k] == oi[k]) {
                    t[k] = (uint32_t)(d0 - 1);
                    a.t[base + p] = (uint8_t)t[k];
                }
#pragma unroll
                for (int d = 0; d < AR_MAXD0; ++d) c[d] += t[k] == (uint32_t)d ? 1u : 0u;
            }
        }
#pragma unroll
        for (int d = 0; d < AR_MAXD0; ++d) {
            const uint32_t s = d < d0 ? wave_sum(c[d]) : 0u;
            if (lane_id() == 0 && s) atomicAdd(&placed[d], s);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t alive = n;
            for (int d = 0; d < d0; ++d) {
                a.alive[(uint64_t)d * a.num_wc + w] = alive;
                alive -= placed[d];
            }
        }
        __syncthreads();   // placed is cleared for the next WC after every read
    }
}

// Global-memory table (full 64-bit keys, separate values) for the work
// chunks handled outside LDS.
__device__ __forceinline__ void hash_insert_min(unsigned long long *hk, uint32_t *hv, uint64_t mask, uint64_t key,
                                                uint32_t val)
{
    uint64_t h = mix64(key) & mask;
    while (true) {
        const unsigned long long k = *((volatile unsigned long long *)&hk[h]);
        if (k == key) break;
        if (k == ~0ull) {
            const unsigned long long prev = atomicCAS(&hk[h], ~0ull, (unsigned long long)key);
            if (prev == ~0ull || prev == key) break;
        }
        h = (h + 1) & mask;
    }
    atomicMin(&hv[h], val);
}

__device__ __forceinline__ uint32_t hash_lookup(const unsigned long long *hk, const uint32_t *hv, uint64_t mask,
                                                uint64_t key)
{
    uint64_t h = mix64(key) & mask;
    while (hk[h] != key) h = (h + 1) & mask;
    return hv[h];
}

// LDS cell table: packed 64-bit entries (key << POS_BITS | position), one
// atomicMin keeps the lowest position of a key.  Keys are relative to the work
// chunk and hold at most 63 - POS_BITS bits, so an entry is never all ones
// (the empty value).

// Exclusive scan in place of arr[0..K) by the whole block; returns the total.
template <int BLOCK>
__device__ uint32_t block_scan_array(uint32_t *arr, uint32_t K, uint32_t *lds)
{
    uint32_t carry = 0;
    for (uint32_t b = 0; b < K; b += BLOCK) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < K ? arr[i] : 0u;
        uint32_t t;
        const uint32_t ex = block_excl_scan<BLOCK>(v, lds, &t);
        if (i < K) arr[i] = carry + ex;
        carry += t;
        __syncthreads();
    }
    return carry;
}

// Item states during the work-chunk loop: 0..21 = final (tentative) depth,
// ST_ALIVE = not yet placed, ST_INNER = not yet placed and in an inner node
// at the current depth.
constexpr uint32_t ST_ALIVE = 0xffu;
constexpr uint32_t ST_INNER = 0xfeu;

// Per-item state (code, state, current node rank, final node rank) in
// registers (LDS path) or in global memory (BIG path).
// LDS path: one packed word per item, state/depth in bits 0-7, the node rank
// at the current depth in bits 8-19 and the rank of the node it is placed in
// in bits 20-31 (at most 4096 points, so ranks fit 12 bits).
template <int BLOCK, int ITEMS, bool BIG>
struct Items {
    static_assert(BLOCK * ITEMS <= 4096, "ranks are packed in 12 bits");
    uint64_t code[ITEMS];
    uint32_t w[ITEMS];
    uint32_t n;
    __device__ uint32_t st(int j) const { return w[j] & 0xffu; }
    __device__ uint32_t nr(int j) const { return (w[j] >> 8) & 0xfffu; }
    __device__ void set_st(int j, uint32_t v) { w[j] = (w[j] & ~0xffu) | v; }
    __device__ void place(int j, uint32_t d) { w[j] = (w[j] & 0x000fff00u) | d | (nr(j) << 20); }
    __device__ void load(const WcArgs &a, uint32_t base, uint32_t n_)
    {
        n = n_;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t pos = j * BLOCK + threadIdx.x;
            code[j] = pos < n ? a.wc_code[base + pos] : 0ull;
            w[j] = pos < n ? a.t[base + pos] : ST_ALIVE;   // alive, or placed at a global depth
        }
    }
    template <class F>
    __device__ void each(F &&f)
    {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t pos = j * BLOCK + threadIdx.x;
            if (pos < n) {
                uint32_t s = w[j] & 0xffu, r = (w[j] >> 8) & 0xfffu, q = w[j] >> 20;
                f(pos, code[j], s, r, q);
                w[j] = s | (r << 8) | (q << 20);
            }
        }
    }
    __device__ void store(const WcArgs &a, uint32_t base)
    {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t pos = j * BLOCK + threadIdx.x;
            if (pos < n) {
                a.t[base + pos] = (uint8_t)(w[j] & 0xffu);
                a.fr[base + pos] = w[j] >> 20;
            }
        }
    }
};

template <int BLOCK, int ITEMS>
struct Items<BLOCK, ITEMS, true> {
    const uint64_t *code;
    uint8_t *t;
    uint32_t *nr, *fr;
    uint32_t n;
    __device__ void load(const WcArgs &a, uint32_t base, uint32_t n_)
    {
        code = a.wc_code + base;
        t = a.t + base;
        nr = a.big_nr + base;
        fr = a.fr + base;
        n = n_;
        for (uint32_t pos = threadIdx.x; pos < n; pos += BLOCK) {   // t: alive, or placed at a global depth
            nr[pos] = 0;
            fr[pos] = 0;
        }
        __syncthreads();
    }
    template <class F>
    __device__ void each(F &&f)
    {
        for (uint32_t pos = threadIdx.x; pos < n; pos += BLOCK) {
            const uint64_t c = code[pos];
            uint32_t s = t[pos], r = nr[pos], q = fr[pos];
            f(pos, c, s, r, q);
            t[pos] = (uint8_t)s;
            nr[pos] = r;
            fr[pos] = q;
        }
    }
    __device__ void store(const WcArgs &, uint32_t) {}
};

// Runs the subtree of work chunk w assuming its shared ancestors are inner.
// LDS path (BIG = false, at most CAP = BLOCK * ITEMS points): points in
// registers; one LDS region of 3 * CAP words holds the node scratch (parent
// masks, child bases, node counts) and then the cell table (2 * CAP packed
// 32-bit entries).  BIG path: per-position state, node scratch and the cell table in
// global memory; winners are decided on original indices.  Returns false (LDS path only) when the
// relative cell keys outgrow the packed entries: the chunk is then redone by
// the BIG path.
template <int BLOCK, int ITEMS, bool BIG>
__device__ bool subsample_wc(const WcArgs &a, uint32_t w, uint32_t *region, uint32_t *red,
                             uint32_t *counter, uint32_t *gnode, unsigned long long *ghk, uint32_t *ghv,
                             uint64_t gmask)
{
    constexpr uint32_t CAP = BLOCK * ITEMS;
    constexpr uint32_t HASH = 2 * CAP;
    constexpr uint32_t HLOG = ilog2_c(HASH);
    constexpr int POS_BITS = (CAP <= 2048) ? 11 : (CAP <= 4096 ? 12 : 13);
    constexpr int KEY_BITS = 31 - POS_BITS;   // packed 32-bit entries, never all ones
    const uint32_t n = a.wc_count[w];
    const uint32_t base = a.wc_begin[w];
    const int lw = a.wc_level[w];
    const uint64_t wkey = a.wc_key[w];
    uint32_t *pmask, *pbase, *ncnt;
    if (BIG) {
        pmask = gnode;
        pbase = gnode + n;
        ncnt = gnode + 2 * n;
    } else {
        pmask = region;
        pbase = region + CAP;
        ncnt = region + 2 * CAP;
    }
    __shared__ uint32_t alive_at[MAXD];
    if (threadIdx.x < MAXD) alive_at[threadIdx.x] = 0;   // the block may have run another work chunk
    if (threadIdx.x == 0) { counter[0] = 0; counter[1] = 0; }
    Items<BLOCK, ITEMS, BIG> it;
    it.load(a, base, n);
    __syncthreads();
    // alive points at depth d0 (the global depths may have placed some)
    uint32_t A0 = 0;
    it.each([&](uint32_t, uint64_t, uint32_t &st, uint32_t &, uint32_t &) { A0 += st == ST_ALIVE ? 1u : 0u; });
    uint32_t A = block_sum<BLOCK>(A0, red);
    uint32_t Kprev = 0, prev_off = 0, loff = 0;
    for (int d = a.d0; d < MAXD; ++d) {
        if (A == 0) {
            if (d - 1 >= lw)
                for (uint32_t r = threadIdx.x; r < Kprev; r += BLOCK) a.lnode_mask[base + prev_off + r] = 0;
            break;
        }
        const bool deepest = d >= a.dmax;
        uint32_t Kd = 0;
        bool single_inner = false;   // d <= lw: one node holds every alive point
        if (d < lw) {
            // shared node, assumed inner (d < lw <= s <= dmax)
            if (threadIdx.x == 0) alive_at[d] = A;
            single_inner = true;
        } else if (d == lw) {
            if (threadIdx.x == 0) alive_at[d] = A;
            Kd = 1;
            single_inner = !deepest && A > a.L;
            it.each([&](uint32_t, uint64_t, uint32_t &st, uint32_t &r, uint32_t &) { if (st == ST_ALIVE) r = 0; });
            if (threadIdx.x == 0) a.lnode_key[base + loff] = wkey;
        } else {
            for (uint32_t r = threadIdx.x; r < Kprev; r += BLOCK) pmask[r] = 0;
            __syncthreads();
            const int osh = 3 * (KB - d);
            it.each([&](uint32_t, uint64_t c, uint32_t &st, uint32_t &r, uint32_t &) {
                if (st == ST_ALIVE) atomicOr(&pmask[r], 1u << ((c >> osh) & 7u));
            });
            __syncthreads();
            for (uint32_t r = threadIdx.x; r < Kprev; r += BLOCK) {
                const uint32_t m = pmask[r];
                a.lnode_mask[base + prev_off + r] = (uint8_t)m;
                pbase[r] = __popc(m);
            }
            __syncthreads();
            Kd = block_scan_array<BLOCK>(pbase, Kprev, red);
            for (uint32_t r = threadIdx.x; r < Kd; r += BLOCK) ncnt[r] = 0;
            __syncthreads();
            it.each([&](uint32_t, uint64_t c, uint32_t &st, uint32_t &r, uint32_t &) {
                if (st != ST_ALIVE) return;
                const uint32_t o = (c >> osh) & 7u;
                const uint32_t m = pmask[r];
                r = pbase[r] + __popc(m & ((1u << o) - 1u));
                atomicAdd(&ncnt[r], 1u);
                a.lnode_key[base + loff + r] = c >> osh;
            });
            __syncthreads();
        }
        if (d >= lw && threadIdx.x == 0) {
            a.kd[(uint64_t)w * MAXD + d] = Kd;
            a.loff[(uint64_t)w * MAXD + d] = loff;
        }
        // inner flag per item (read before the region becomes the cell table)
        if (d > lw)
            it.each([&](uint32_t, uint64_t, uint32_t &st, uint32_t &r, uint32_t &) {
                if (st == ST_ALIVE && !deepest && ncnt[r] > a.L) st = ST_INNER;
            });
        else if (single_inner)
            it.each([&](uint32_t, uint64_t, uint32_t &st, uint32_t &, uint32_t &) {
                if (st == ST_ALIVE) st = ST_INNER;
            });
        // cells of lattice level d + s; keys relative to the work chunk
        const int csh = 3 * (KB - d - a.s);
        const int rel_bits = 3 * (d + a.s - lw);
        const uint64_t rel_mask = rel_bits >= 64 ? ~0ull : ((1ull << rel_bits) - 1ull);
        bool mine_inner = false;
        it.each([&](uint32_t, uint64_t, uint32_t &st, uint32_t &, uint32_t &) { mine_inner |= st == ST_INNER; });
        // (also the barrier after which the node scratch becomes the cell table)
        const bool any_inner = __syncthreads_or(mine_inner);
        if (!any_inner) {
            // every alive point sits in a leaf
            it.each([&](uint32_t, uint64_t, uint32_t &st, uint32_t &r, uint32_t &f) {
                if (st == ST_ALIVE) {
                    st = (uint32_t)d;
                    f = r;
                }
            });
            A = 0;
            if (d >= lw) {
                prev_off = loff;
                loff += Kd;
                Kprev = Kd;
            }
            continue;
        }
        if (!BIG && rel_bits > KEY_BITS) return false;
        // LDS table of 2^hb slots, at least twice the alive points
        uint32_t hb = ceil_log2_dev(2 * A);
        if (hb < 6) hb = 6;
        if (hb > HLOG) hb = HLOG;
        const uint32_t hsize = 1u << hb;
        if (BIG) {
            for (uint64_t h = threadIdx.x; h <= gmask; h += BLOCK) {
                ghk[h] = ~0ull;
                ghv[h] = 0xffffffffu;
            }
        } else {
            for (uint32_t h = threadIdx.x; h < hsize; h += BLOCK) region[h] = ~0u;
        }
        __syncthreads();
        uint32_t survive = 0;
        if constexpr (BIG) {
            // winners by original index: a work chunk spanning several chunks
            // is not in index order
            it.each([&](uint32_t pos, uint64_t c, uint32_t &st, uint32_t &, uint32_t &) {
                if (st != ST_INNER) return;
                hash_insert_min(ghk, ghv, gmask, (c >> csh) & rel_mask, a.wc_orig[base + pos]);
            });
            __syncthreads();
            it.each([&](uint32_t pos, uint64_t c, uint32_t &st, uint32_t &r, uint32_t &f) {
                if (st == ST_ALIVE) {   // leaf: every reaching point stays
                    st = (uint32_t)d;
                    f = r;
                } else if (st == ST_INNER) {
                    if (hash_lookup(ghk, ghv, gmask, (c >> csh) & rel_mask) == a.wc_orig[base + pos]) {
                        st = (uint32_t)d;
                        f = r;
                    } else {
                        st = ST_ALIVE;
                        ++survive;
                    }
                }
            });
        } else {
            uint32_t slot[ITEMS];
            uint32_t mine[ITEMS];   // key << POS_BITS | position; all ones once placed (or not inserting)
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t pos = j * BLOCK + threadIdx.x;
                const uint32_t key = (uint32_t)((it.code[j] >> csh) & rel_mask);
                mine[j] = (pos < n && it.st(j) == ST_INNER) ? ((key << POS_BITS) | pos) : 0xffffffffu;
                slot[j] = rel_bits <= (int)hb ? key : (key * 0x9E3779B1u) >> (32 - hb);
            }
            bool any = true;
            while (any) {
                any = false;
                uint32_t cur[ITEMS];
#pragma unroll
                for (int j = 0; j < ITEMS; ++j)
                    if (mine[j] != 0xffffffffu) cur[j] = region[slot[j]];
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) {
                    if (mine[j] == 0xffffffffu) continue;
                    uint32_t c = cur[j];
                    if (c == 0xffffffffu) {
                        c = atomicCAS(&region[slot[j]], 0xffffffffu, mine[j]);
                        if (c == 0xffffffffu) { mine[j] = 0xffffffffu; continue; }   // new key: done
                    }
                    if ((c >> POS_BITS) == (mine[j] >> POS_BITS)) {
                        if (c > mine[j]) atomicMin(&region[slot[j]], mine[j]);
                        mine[j] = 0xffffffffu;                                      // our key: done
                    } else {
                        slot[j] = (slot[j] + 1) & (hsize - 1);                       // another key
                        any = true;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t pos = j * BLOCK + threadIdx.x;
                if (pos >= n) continue;
                if (it.st(j) == ST_ALIVE) {   // leaf: every reaching point stays
                    it.place(j, (uint32_t)d);
                } else if (it.st(j) == ST_INNER) {
                    if ((region[slot[j]] & ((1u << POS_BITS) - 1u)) == pos) {
                        it.place(j, (uint32_t)d);
                    } else {
                        it.set_st(j, ST_ALIVE);
                        ++survive;
                    }
                }
            }
        }
        // survivors, counted per wave into an alternating counter
        survive = wave_sum(survive);
        if (lane_id() == 0 && survive) atomicAdd(&counter[(d + 1) & 1], survive);
        __syncthreads();
        A = counter[(d + 1) & 1];
        if (threadIdx.x == 0) counter[d & 1] = 0;   // reused two depths later, after the next barrier
        if (d >= lw) {
            prev_off = loff;
            loff += Kd;
            Kprev = Kd;
        }
    }
    // points reaching each shared ancestor from this work chunk, one row per
    // depth, and at depth lw the points reaching its own root.  Plain stores, summed per ancestor later: thousands of work
    // chunks share the top ancestors, and atomics on those few addresses
    // would serialise and stall the memory pipeline.
    if (threadIdx.x < (uint32_t)MAXD && (int)threadIdx.x >= a.d0) {   // rows above d0: the global pass
        const int d = threadIdx.x;
        a.alive[(uint64_t)d * a.num_wc + w] = d <= lw ? alive_at[d] : 0u;
    }
    it.store(a, base);
    __syncthreads();
    return true;
}

// LDS path: the work chunks of one size class (at most BLOCK * ITEMS points
// each), from the class list.
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_subsample_lds(WcArgs a, int cls)
{
    constexpr uint32_t CAP = BLOCK * ITEMS;
    __shared__ uint32_t region[3 * CAP];   // node scratch, then the cell table (2 * CAP entries)
    __shared__ uint32_t red[BLOCK / 64 + 1];
    __shared__ uint32_t counter[2];
    const uint32_t cnt = a.cls_cnt[cls];
    const uint32_t *list = a.cls_list + (uint64_t)cls * a.num_wc;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const uint32_t w = list[i];
        const bool ok = subsample_wc<BLOCK, ITEMS, false>(a, w, region, red, counter, nullptr, nullptr, nullptr, 0);
        if (!ok && threadIdx.x == 0) a.big_list[atomicAdd(a.num_big_dev, 1u)] = w;
        __syncthreads();
    }
}

// Sorts the work chunks into the LDS size classes; those too large for every
// class, and those spanning several chunks (their positions are not in
// original index order), go to the global-memory list.  One atomic per wave
// and class.
__device__ __forceinline__ uint32_t wc_size_class(uint32_t n)
{
    return n <= 256 ? 0u : n <= 512 ? 1u : n <= 1024 ? 2u : n <= 2048 ? 3u : n <= WC_CAP ? 4u : n <= 2 * WC_CAP ? 5u : 0xffu;
}

// Shared-ancestor pass of a work chunk whose own root is a leaf (at most L
// points, so no local subtree below it; up to 8192 points, which only work
// chunks at the deepest work-chunk level can hold): at every shared depth d < lw each
// alive point competes for its cell of level d + s (relative to the work
// chunk: 3(d + s - lw) bits), the lowest position wins and stays at depth d,
// the others go on; what is left sits in the root at depth lw.  Each point
// carries only its relative cell key at level lw - 1 + s (3(s - 1) <= 18
// bits for s <= 7) and its state, packed in one word; the key of every
// position is also kept in LDS.
//
// Cell table, one atomicMin of the position per point and round:
//  - while the cell key fits the table it is the slot, and the entry is
//    (31 - d) << 12 (13) | position, so entries of shallower depths are replaced
//    by the same atomicMin (no clearing per depth);
//  - longer keys are hashed without probing: every point writes its cell key
//    and position, key << 12 (13) | position, into slot h_r(cell) with an
//    atomicMin, and reads the slot back: the smallest key among the cells
//    that met there owns the slot, and its entry holds the lowest position of
//    that cell; points whose cell owns the slot are decided, the cells that
//    collided try again with the next multiplier.  (Keys have at most 18
//    bits, positions 13.)  With at most a quarter of the slots used, few
//    cells collide per round, and a round costs one LDS read, where linear
//    probing costs as many load and CAS round trips as the longest probe
//    chain of the block.
// LDS operations of all items are issued together and waited for once.
__constant__ uint32_t kFastMul[8] = {0x9E3779B1u, 0x85EBCA77u, 0xC2B2AE3Du, 0x27D4EB2Fu,
                                     0x165667B1u, 0xD3A2646Du, 0xFD7046C5u, 0xB55A4F09u};

// Eight items per thread are held to six waves per SIMD (80 registers, a
// few per-chunk constants spilled): on the 20M-point planes the 512 x 8
// class then runs three blocks per CU instead of two (119 -> 97 us), and
// 256 x 8 for the 2048-point class six blocks of four waves instead of four
// blocks of eight at 512 x 4 (106 -> 84 us).  Eight waves per SIMD spill in
// the depth loop.
template <int BLOCK, int ITEMS, int TLOG>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BLOCK <= 512 && ITEMS == 8 ? 6 : 1)))
void k_subsample_fast(WcArgs a, int cls)
{
    constexpr uint32_t CAP = BLOCK * ITEMS;
    constexpr uint32_t TSZ = 1u << TLOG;        // table entries
    constexpr int NW = BLOCK / 64;
    constexpr uint32_t ALIVE = 0xffu << 24;
    constexpr uint32_t EMPTY = 0xffffffffu;
    constexpr int PB = CAP <= 4096 ? 12 : 13;   // position bits of a table entry
    static_assert(CAP <= 8192, "positions are packed in 13 bits");
    static_assert(TSZ >= 2 * CAP, "table of at least two slots per point");
    __shared__ uint4 table4[TSZ / 4];
    uint32_t *table = reinterpret_cast<uint32_t *>(table4);
    __shared__ uint32_t wsum[2][NW];
    __shared__ uint32_t alive_at[MAXD];
    const uint32_t cnt = a.cls_cnt[cls];
    const uint32_t *list = a.cls_list + (uint64_t)cls * a.num_wc;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    // block-wide sum (every thread gets it); buffers alternate by parity
    auto block_sum2 = [&](uint32_t v, int parity) -> uint32_t {
        v = wave_sum(v);
        if constexpr (NW == 1) {
            return v;
        } else {
            if (lane == 0) wsum[parity][wv] = v;
            __syncthreads();
            uint32_t t = 0;
#pragma unroll
            for (int k = 0; k < NW; ++k) t += wsum[parity][k];
            return t;
        }
    };
    int par = 0;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const uint32_t w = list[i];
        const uint32_t n = a.wc_count[w], base = a.wc_begin[w];
        const int lw = a.wc_level[w];
        const int ksh = 3 * (KB - (lw - 1 + a.s));
        const uint32_t kmask = (1u << (3 * (a.s - 1))) - 1u;
        uint32_t it[ITEMS];   // relative key | state << 24 (0xff alive, else the depth it stays at)
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t pos = j * BLOCK + threadIdx.x;
            const uint64_t c = a.wc_code[base + (pos < n ? pos : n - 1)];
            // alive, or placed at a global depth (none without global depths)
            const uint32_t st = a.d0 > 0 ? a.t[base + (pos < n ? pos : n - 1)] : 0xffu;
            it[j] = pos < n ? ((uint32_t)(c >> ksh) & kmask) | (st << 24) : 0u;
        }
        if (threadIdx.x < (uint32_t)MAXD) alive_at[threadIdx.x] = 0;
        for (uint32_t h = threadIdx.x; h < TSZ / 4; h += BLOCK) table4[h] = make_uint4(EMPTY, EMPTY, EMPTY, EMPTY);
        uint32_t alive0 = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) alive0 += it[j] >= ALIVE ? 1u : 0u;
        uint32_t A = block_sum2(alive0, par);   // its barrier also ends the clearing (one wave: program order)
        par ^= 1;
        bool clean = true;   // the table holds no hashed entries
        for (int d = a.d0; d < lw && A > 0; ++d) {
            if (threadIdx.x == 0) alive_at[d] = A;
            const int rb = 3 * (d + a.s - lw);   // relative key bits at this depth
            const int sh = 3 * (lw - 1 - d);
            uint32_t won = 0;                    // bit j: item j stays at depth d
            if (rb <= TLOG) {
                if (!clean) {   // block-uniform
                    for (uint32_t h = threadIdx.x; h < TSZ / 4; h += BLOCK)
                        table4[h] = make_uint4(EMPTY, EMPTY, EMPTY, EMPTY);
                    clean = true;
                    __syncthreads();
                }
                const uint32_t tag = (31u - (uint32_t)d) << PB;
#pragma unroll
                for (int j = 0; j < ITEMS; ++j)
                    if (it[j] >= ALIVE) atomicMin(&table[(it[j] & 0xffffffu) >> sh], tag | (j * BLOCK + threadIdx.x));
                __syncthreads();
                uint32_t cur[ITEMS];
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) cur[j] = table[(it[j] & 0xffffffu) >> sh];
#pragma unroll
                for (int j = 0; j < ITEMS; ++j)
                    if (it[j] >= ALIVE && cur[j] == (tag | (j * BLOCK + threadIdx.x))) won |= 1u << j;
            } else {
                // table of 2^hb slots, at least four per alive point
                uint32_t hb = ceil_log2_dev(4 * A);
                hb = hb < 6 ? 6 : (hb > (uint32_t)TLOG ? (uint32_t)TLOG : hb);
                uint32_t pend = 0;   // bit j: item j's cell is not decided yet
#pragma unroll
                for (int j = 0; j < ITEMS; ++j)
                    if (it[j] >= ALIVE) pend |= 1u << j;
                for (int r = 0;; ++r) {
                    const uint32_t mul = kFastMul[r & 7] + 2u * (uint32_t)(r >> 3);
                    for (uint32_t h = threadIdx.x; h < (1u << hb) / 4; h += BLOCK)
                        table4[h] = make_uint4(EMPTY, EMPTY, EMPTY, EMPTY);
                    __syncthreads();
                    uint32_t slot[ITEMS];
#pragma unroll
                    for (int j = 0; j < ITEMS; ++j) {
                        const uint32_t key = (it[j] & 0xffffffu) >> sh;
                        slot[j] = (key * mul) >> (32 - hb);
                        if ((pend >> j) & 1u) atomicMin(&table[slot[j]], (key << PB) | (j * BLOCK + threadIdx.x));
                    }
                    __syncthreads();
                    uint32_t cur[ITEMS];
#pragma unroll
                    for (int j = 0; j < ITEMS; ++j) cur[j] = table[slot[j]];
#pragma unroll
                    for (int j = 0; j < ITEMS; ++j) {
                        if (!((pend >> j) & 1u)) continue;
                        if ((cur[j] >> PB) == ((it[j] & 0xffffffu) >> sh)) {   // the slot is this cell's
                            pend &= ~(1u << j);
                            if ((cur[j] & ((1u << PB) - 1u)) == j * BLOCK + threadIdx.x) won |= 1u << j;
                        }
                    }
                    clean = false;
                    if (!__syncthreads_or(pend != 0)) break;
                }
            }
            uint32_t surv = 0;
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                if (it[j] < ALIVE) continue;
                if ((won >> j) & 1u) it[j] = (it[j] & 0xffffffu) | ((uint32_t)d << 24);
                else ++surv;
            }
            // every table read of this depth has completed before the sum's
            // barrier (one wave: in program order), so the next depth may
            // write the table
            A = block_sum2(surv, par);
            par ^= 1;
        }
        // the rest sits in the root (a leaf) at depth lw; ranks among own
        // nodes (fr) are read only for work chunks with nodes below their
        // root, so none is written here
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t pos = j * BLOCK + threadIdx.x;
            if (pos < n) a.t[base + pos] = (uint8_t)(it[j] >= ALIVE ? (uint32_t)lw : it[j] >> 24);
        }
        __syncthreads();
        if (threadIdx.x < (uint32_t)MAXD && (int)threadIdx.x >= a.d0) {   // rows above d0: the global pass
            const int d = threadIdx.x;
            a.alive[(uint64_t)d * a.num_wc + w] = d < lw ? alive_at[d] : d == lw ? A : 0u;
        }
        if (threadIdx.x == 0 && A > 0) {
            a.kd[(uint64_t)w * MAXD + lw] = 1;
            a.loff[(uint64_t)w * MAXD + lw] = 0;
            a.lnode_key[base] = a.wc_key[w];
            a.lnode_mask[base] = 0;
        }
        __syncthreads();
    }
}

// One pass over the work chunks in blocks of 256: each wave counts its work
// chunks per class with ballots into the block's LDS counters, one global
// atomic per block and class reserves the block's run, then the waves write.
// List of a work chunk of n points: a fast class (its own root a leaf), a
// general class, or WC_CLASSES for the global-memory path (work chunks across
// chunks, or too large for LDS).
__device__ __forceinline__ uint32_t wc_list_class(uint32_t n, bool nested, uint32_t L, int s)
{
    uint32_t c = wc_size_class(n);
    if (!nested) c = 0xffu;
    else if (c != 0xffu && !(n <= L && s <= 7)) c = c < 5 ? c + WC_GENERAL : 0xffu;
    return c == 0xffu ? (uint32_t)WC_CLASSES : c;
}

__global__ __launch_bounds__(256) void k_list_classes(WcArgs a)
{
    constexpr uint32_t NC = WC_CLASSES + 1;   // the last one: the global-memory list
    __shared__ uint32_t bcnt[NC], bbase[NC];
    for (uint32_t b0 = blockIdx.x * 256u; b0 < a.num_wc; b0 += gridDim.x * 256u) {
        if (threadIdx.x < NC) bcnt[threadIdx.x] = 0;
        __syncthreads();
        const uint32_t w = b0 + threadIdx.x;
        const bool valid = w < a.num_wc;
        // counter index (0xfe: none)
        const uint32_t ci = valid ? wc_list_class(a.wc_count[w], a.wc_nested[w] != 0, a.L, a.s) : 0xfeu;
        uint32_t rank = 0;
        for (uint32_t k = 0; k < NC; ++k) {
            const uint64_t m = __ballot(ci == k);
            if (!m) continue;
            const int leader = __ffsll((long long)m) - 1;
            uint32_t wb = 0;
            if ((int)lane_id() == leader) wb = atomicAdd(&bcnt[k], (uint32_t)__popcll(m));
            wb = __shfl(wb, leader, 64);
            if (ci == k) rank = wb + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull));
        }
        __syncthreads();
        if (threadIdx.x < NC && bcnt[threadIdx.x])
            bbase[threadIdx.x] = atomicAdd(threadIdx.x == (uint32_t)WC_CLASSES ? a.num_big_dev : &a.cls_cnt[threadIdx.x],
                                           bcnt[threadIdx.x]);
        __syncthreads();
        if (ci < NC) {
            const uint32_t r = bbase[ci] + rank;
            if (ci == (uint32_t)WC_CLASSES) a.big_list[r] = w;
            else a.cls_list[(uint64_t)ci * a.num_wc + r] = w;
        }
        __syncthreads();
    }
}

// Work chunks listed for the global-memory path (too large, or keys too
// long): table and node scratch in a region of 4 slots (table) and 3 words
// (nodes) per point of the work chunk, at its position range, so any number
// of blocks can run.
__global__ __launch_bounds__(P1_BLOCK) void k_subsample_big(WcArgs a)
{
    __shared__ uint32_t red[P1_BLOCK / 64 + 1];
    __shared__ uint32_t counter[2];
    const uint32_t nb = *a.num_big_dev;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint32_t w = a.big_list[b];
        const uint32_t base = a.wc_begin[w], n = a.wc_count[w];
        uint64_t cap = 1;
        while (cap * 2 <= 4ull * n) cap *= 2;
        unsigned long long *hk = reinterpret_cast<unsigned long long *>(a.big_hkey) + 4ull * base;
        uint32_t *hv = a.big_hval + 4ull * base;
        subsample_wc<P1_BLOCK, 1, true>(a, w, nullptr, red, counter, a.big_node + 3ull * base, hk, hv, cap - 1);
    }
}

// First shared depth of each WC whose node is a leaf (or empty); lw if none.
// Reaching count of every shared ancestor (the sum of the rows posted by the
// work chunks inside it: a range of the work-chunk order, found by binary
// search on the first cells, summed as a difference of the row scan; u32
// modular arithmetic is exact since every count is below 2^32), then per work
// chunk the first shared depth whose node is a leaf (lw if none).  The
// reaching counts up to that depth replace the posted rows.
__device__ __forceinline__ uint32_t wc_lower_bound(const uint64_t *start, uint32_t lo, uint32_t hi, uint64_t v)
{
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// The depths of a work chunk in parallel: DC_LANES lanes per work chunk,
// lane d finds the reaching count of its depth-d ancestor; a ballot gives
// the first leaf (the cut), and lanes up to it replace their rows.  (Work
// chunks sit at levels up to g <= 9, so they have at most nine shared depths.)
constexpr int DC_LANES = 16;
__global__ void k_decide(WcArgs a)
{
    const uint32_t W = a.num_wc;
    const uint32_t lane = lane_id();
    const int d = (int)(lane & (DC_LANES - 1)), grp = (int)(lane / DC_LANES);
    constexpr int PER_WAVE = 64 / DC_LANES;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t w0 = wave * PER_WAVE; w0 < W; w0 += nwaves * PER_WAVE) {
        const uint32_t w = (uint32_t)w0 + (uint32_t)grp;
        const bool valid = w < W;
        const int lw = valid ? a.wc_level[w] : 0;
        const bool mine = valid && d < lw;
        uint32_t R = 0;
        bool leaf = false;
        if (mine) {
            const uint64_t key = a.wc_key[w];
            const int sh = 3 * (a.lam_w - d);
            const uint64_t node_start = (key >> (3 * (lw - d))) << sh;
            const uint32_t lo = wc_lower_bound(a.wc_start, 0, w, node_start);
            const uint32_t hi = wc_lower_bound(a.wc_start, w + 1, W, node_start + (1ull << sh));
            R = a.alive_scan[(uint64_t)d * W + hi] - a.alive_scan[(uint64_t)d * W + lo];
            leaf = R <= a.L || d >= a.dmax;
        }
        const uint32_t leaves = (uint32_t)(__ballot(leaf) >> (grp * DC_LANES)) & ((1u << DC_LANES) - 1u);
        const int cut = leaves ? __ffs((int)leaves) - 1 : lw;
        if (mine && d <= cut) a.alive[(uint64_t)d * W + w] = R;
        if (valid && d == 0) a.cut[w] = (uint8_t)cut;
    }
}

// Index of the first WC inside the depth-d node that contains WC w.
__device__ __forceinline__ uint32_t owner_of(const WcArgs &a, uint32_t w, int d)
{
    const int lw = a.wc_level[w];
    const uint64_t node_start = (a.wc_key[w] >> (3 * (lw - d))) << (3 * (a.lam_w - d));
    uint32_t lo = 0, hi = w;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.wc_start[mid] < node_start) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// owned[d * num_wc + w] = number of nodes at depth d attributed to WC w: the
// shared node at depth d < lw when w is the first WC inside it, or w's local
// nodes at depth d >= lw.  Depth-major order of (d, w) equals (depth, key).
__global__ void k_node_counts(WcArgs a, uint32_t *owned)
{
    const uint64_t total = (uint64_t)MAXD * a.num_wc;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const int d = (int)(i / a.num_wc);
        const uint32_t w = (uint32_t)(i % a.num_wc);
        const int lw = a.wc_level[w];
        const int cut = a.cut[w];
        uint32_t v = 0;
        if (d < lw) {
            if (d <= cut) {
                bool first = true;
                if (w > 0) {
                    const int lp = a.wc_level[w - 1];
                    if (lp > d && (a.wc_key[w - 1] >> (3 * (lp - d))) == (a.wc_key[w] >> (3 * (lw - d)))) first = false;
                }
                const bool exists = d < cut || a.alive[(uint64_t)d * a.num_wc + w] > 0;
                v = (first && exists) ? 1u : 0u;
            }
        } else if (cut == lw) {
            v = a.kd[(uint64_t)w * MAXD + d];
        }
        owned[i] = v;
    }
}

// ---- node_points: the points of every node in ascending original index ------------------------
//
// A point's node is fixed by its final depth t: a shared ancestor above its
// work chunk when t < lw, else one of the work chunk's own nodes (rank fr
// among those of depth t).  The points of work chunk w in the shared node of
// depth d form one piece.  Piece sizes are differences of the reaching counts
// the subsample pass posts, and the depth-major exclusive scan S of the piece
// sizes gives every shared node's size (a difference of S over its work
// chunks, which are consecutive) and every piece's offset inside its node.  A
// root that is its work chunk's only own node holds every point reaching it;
// only work chunks with own nodes below their root count their points.  With
// the node begins (scan of the node sizes in node order) every point is put
// inside its node's range, and each range is then sorted by original index:
// an LDS radix sort per tile (tiles sized to the node), merge rounds for
// nodes above one tile.

constexpr int NP_BLOCK = 256;
constexpr int NP_ITEMS = 16;          // positions per thread and step (one step covers a work chunk)
constexpr uint32_t NP_LCAP = 4096;    // own nodes of a work chunk counted in LDS
constexpr uint32_t NP_GROUP = 32;     // consecutive small nodes sorted as one tile
constexpr uint32_t NP_GROUP_FLAG = 0x80000000u;
constexpr uint32_t NP_NONE = 0xffffffffu;

__device__ __forceinline__ int np_final_depth(int t, int lw, int cut) { return (cut < lw && t >= cut) ? cut : t; }

// One LDS atomic per distinct key of the wave: adds the number of active
// lanes holding each key to cnt[key].
__device__ __forceinline__ void wave_lds_count(uint32_t *cnt, uint32_t key, bool active)
{
    uint64_t todo = __ballot(active);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const uint64_t m = __ballot(active && key == k);
        if ((int)lane_id() == leader) atomicAdd(&cnt[k], (uint32_t)__popcll(m));
        todo &= ~m;
    }
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
    return v;
}

// The own nodes of a work chunk, per depth: how many (kd), the slot of the
// first one among all its own nodes (loff) and its node id (first).
struct NpOwn {
    uint32_t kd[MAXD], loff[MAXD], first[MAXD];
    __device__ void load(const WcArgs &a, const uint32_t *node_base, uint32_t w, int lw, int cut)
    {
        if (threadIdx.x < (uint32_t)MAXD) {
            const int d = threadIdx.x;
            const bool own = cut == lw && d >= lw;
            kd[d] = own ? a.kd[(uint64_t)w * MAXD + d] : 0u;
            loff[d] = own ? a.loff[(uint64_t)w * MAXD + d] : 0u;
            first[d] = own ? node_base[(uint64_t)d * a.num_wc + w] : 0u;
        }
    }
    __device__ uint32_t total(int lw) const
    {
        uint32_t t = 0;
        for (int d = lw; d < MAXD; ++d)
            if (kd[d]) t = loff[d] + kd[d];
        return t;
    }
    __device__ uint32_t id_of_slot(uint32_t slot, int lw) const
    {
        int d = lw;
        while (d < MAXD - 1 && !(kd[d] && slot < loff[d] + kd[d])) ++d;
        return first[d] + slot - loff[d];
    }
};

// The LDS key of an own-node point (its slot among the work chunk's own
// nodes), NP_NONE when beyond the LDS counters; gid = the node id.
__device__ __forceinline__ uint32_t np_own_key(const NpOwn &own, int t, uint32_t f, uint32_t &gid)
{
    gid = own.first[t] + f;
    const uint32_t slot = own.loff[t] + f;
    return slot < NP_LCAP ? slot : NP_NONE;
}

// Piece sizes from the reaching counts of the work chunks (their scan, taken
// before k_decide replaced rows): at a shared depth d above its cut a work
// chunk leaves a(d) - a(d+1) of its points (row lw: those reaching its own
// root), at the cut all a(cut).
__global__ void k_np_pieces(WcArgs a, uint32_t *cnt_dw)
{
    const uint32_t W = a.num_wc;
    const uint64_t total = (uint64_t)MAXD * W;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const int d = (int)(i / W);
        const uint32_t w = (uint32_t)(i % W);
        const int lw = a.wc_level[w], cut = a.cut[w];
        uint32_t v = 0;
        if (d < lw && d <= cut) {
            v = a.alive_scan[i + 1] - a.alive_scan[i];
            if (d < cut) v -= a.alive_scan[i + W + 1] - a.alive_scan[i + W];
        }
        cnt_dw[i] = v;
    }
}

// Per (depth d, work chunk w): the node holding w's points of depth d when
// one offset places them (pnode, NP_NONE otherwise) and that offset (poff):
// a piece of a shared node (d < lw), or w's own root when it is its only own
// node (d = lw).  Sizes: of each shared node at its first work chunk (a
// difference of S over its work chunks, found by binary search on their first
// cells), of such roots (the points reaching them).  Work chunks with own
// nodes below their root are listed for k_np_count.
__global__ void k_np_shared(WcArgs a, const uint32_t *node_base, const uint32_t *S, uint32_t *cnt_node,
                            uint32_t *pnode, uint32_t *poff, uint32_t *glist, uint32_t *gcount, uint32_t *maxc,
                            uint8_t *single)
{
    const uint32_t W = a.num_wc;
    const uint64_t total = (uint64_t)MAXD * W;
    uint32_t mymax = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const int d = (int)(i / W);
        const uint32_t w = (uint32_t)(i % W);
        const int lw = a.wc_level[w], cut = a.cut[w];
        uint32_t node = NP_NONE, off = 0;
        if (d < lw && d <= cut) {
            const uint64_t wkey = a.wc_key[w];
            bool first = true;
            if (w > 0) {
                const int lp = a.wc_level[w - 1];
                if (lp > d && (a.wc_key[w - 1] >> (3 * (lp - d))) == (wkey >> (3 * (lw - d)))) first = false;
            }
            if (first && (d < cut || a.alive[i] > 0)) {
                const int sh = 3 * (a.lam_w - d);
                const uint64_t node_start = (wkey >> (3 * (lw - d))) << sh;
                const uint32_t we = wc_lower_bound(a.wc_start, w + 1, W, node_start + (1ull << sh));
                const uint32_t c = S[(uint64_t)d * W + we] - S[i];
                cnt_node[node_base[i]] = c;
                mymax = max(mymax, c);
                // one piece: the first non-empty piece of w .. we - 1 holds all c
                // points, and its work chunk lies inside one chunk (so work-chunk
                // order is index order there)
                uint32_t lo = w, hi = we;   // first w' with a non-empty piece (S rises after it)
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (S[(uint64_t)d * W + mid + 1] > S[i]) hi = mid; else lo = mid + 1;
                }
                single[node_base[i]] =
                    lo < we && S[(uint64_t)d * W + lo + 1] == S[(uint64_t)d * W + we] && a.wc_nested[lo] ? 1 : 0;
            }
            if (S[i + 1] > S[i]) {
                const uint32_t o = first ? w : owner_of(a, w, d);
                node = node_base[(uint64_t)d * W + o];
                off = S[i] - S[(uint64_t)d * W + o];
            }
        } else if (d == lw && cut == lw) {
            const uint32_t reach = a.alive_scan[i + 1] - a.alive_scan[i];
            if (reach > 0) {
                if (a.kd[(uint64_t)w * MAXD + lw + 1] == 0) {   // a leaf root, or every point kept there
                    node = node_base[i];
                    cnt_node[node] = reach;
                    single[node] = a.wc_nested[w];   // placed from this work chunk alone, in index order if nested
                    mymax = max(mymax, reach);
                } else {
                    glist[atomicAdd(gcount, 1u)] = w;
                }
            }
        }
        pnode[i] = node;
        poff[i] = off;
    }
    mymax = wave_max(mymax);
    if (lane_id() == 0 && mymax) atomicMax(maxc, mymax);
}

// Per listed work chunk (one block each): the size of each of its own nodes
// into cnt_node[id].
__global__ __launch_bounds__(NP_BLOCK) void k_np_count(WcArgs a, const uint32_t *node_base, const uint32_t *glist,
                                                       const uint32_t *gcount, uint32_t *cnt_node, uint32_t *maxc,
                                                       uint8_t *single)
{
    __shared__ uint32_t cnt[NP_LCAP];
    __shared__ NpOwn own;
    const uint32_t G = *gcount;
    uint32_t mymax = 0;
    for (uint32_t gi = blockIdx.x; gi < G; gi += gridDim.x) {
        const uint32_t w = glist[gi];
        const int lw = a.wc_level[w], cut = a.cut[w];
        const uint32_t base = a.wc_begin[w], n = a.wc_count[w];
        own.load(a, node_base, w, lw, cut);
        __syncthreads();
        const uint32_t nown = own.total(lw), nl = nown < NP_LCAP ? nown : NP_LCAP;
        for (uint32_t i = threadIdx.x; i < nl; i += NP_BLOCK) cnt[i] = 0;
        // own nodes beyond the LDS counters count in global memory
        for (uint32_t i = NP_LCAP + threadIdx.x; i < nown; i += NP_BLOCK) cnt_node[own.id_of_slot(i, lw)] = 0;
        __syncthreads();
        for (uint32_t c0 = 0; c0 < n; c0 += NP_BLOCK * NP_ITEMS) {
            uint32_t t8[NP_ITEMS], f[NP_ITEMS];
#pragma unroll
            for (int j = 0; j < NP_ITEMS; ++j) {
                const uint32_t p = c0 + j * NP_BLOCK + threadIdx.x;
                t8[j] = p < n ? a.t[base + p] : (uint32_t)MAXD;
                f[j] = p < n ? a.fr[base + p] : 0u;
            }
#pragma unroll
            for (int j = 0; j < NP_ITEMS; ++j) {
                const int t = (int)t8[j];
                const bool mine = t < MAXD && t >= lw;   // the cut is lw here
                uint32_t gid = 0;
                const uint32_t key = mine ? np_own_key(own, t, f[j], gid) : 0u;
                wave_lds_count(cnt, key, mine && key != NP_NONE);
                if (mine && key == NP_NONE) atomicAdd(&cnt_node[gid], 1u);
            }
        }
        __syncthreads();
        // own nodes below a subdivided root are filled through counters (any
        // order within a wave): sorted
        for (uint32_t i = threadIdx.x; i < nl; i += NP_BLOCK) {
            const uint32_t c = cnt[i];
            const uint32_t id = own.id_of_slot(i, lw);
            cnt_node[id] = c;
            single[id] = 0;
            mymax = max(mymax, c);
        }
        for (uint32_t i = NP_LCAP + threadIdx.x; i < nown; i += NP_BLOCK) {   // settled by the barrier above
            const uint32_t id = own.id_of_slot(i, lw);
            single[id] = 0;
            mymax = max(mymax, atomicAdd(&cnt_node[id], 0u));
        }
        __syncthreads();
    }
    mymax = wave_max(mymax);
    if (lane_id() == 0 && mymax) atomicMax(maxc, mymax);
}

// Sort tile classes: values per tile (threads x values per thread).
constexpr uint32_t NP_T0 = 64 * 16, NP_T1 = 256 * 16, NP_T2 = 256 * 32, NP_T3 = 512 * 32;
constexpr uint32_t NPM_OUT = 2048;   // outputs per merge job (measured: 4096 and 1024 slower); divides NP_T3

// Work lists of the sort (one thread per node): groups of NP_GROUP
// consecutive nodes holding at most NP_T1 points together (entry
// g | NP_GROUP_FLAG, class 0 or 1 by size); other nodes by size into classes
// 0..2 (entry: the node), or class 3 for longer ones (entries node << 32 |
// part, plus merge jobs of NPM_OUT outputs, node << 32 | job, above one tile).
// One atomic per wave and list reserves the entries.
__global__ void k_np_lists(const uint32_t *nb, uint32_t nn, NpLists L)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t x0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); x0 < nn; x0 += stride) {
        const uint32_t x = x0 + lane_id();
        const bool valid = x < nn;
        uint32_t n0 = 0, n1 = 0, n2 = 0, n3 = 0, nj = 0, ncp = 0, g = 0;
        bool grouped = false;
        if (valid) {
            g = x / NP_GROUP;
            const uint32_t gx0 = g * NP_GROUP, gx1 = min(gx0 + NP_GROUP, nn);
            const uint32_t gt = nb[gx1] - nb[gx0];
            const uint32_t c = nb[x + 1] - nb[x];
            grouped = gx1 - gx0 > 1 && gt <= NP_T1;
            if (grouped) {
                if (x == gx0) {
                    bool all = true;   // every node of the group already ascends: copied
                    for (uint32_t y = gx0; y < gx1 && all; ++y) all = L.single[y] != 0;
                    if (all) {
                        ncp = 1;
                    } else {
                        n0 = gt <= NP_T0 ? 1u : 0u;
                        n1 = 1u - n0;
                    }
                }
            } else if (L.single[x]) {
                ncp = c ? (c + NP_T3 - 1) / NP_T3 : 0u;
            } else if (c <= NP_T0) {
                n0 = 1;
            } else if (c <= NP_T1) {
                n1 = 1;
            } else if (c <= NP_T2) {
                n2 = 1;
            } else {
                n3 = (c + NP_T3 - 1) / NP_T3;
                if (c > NP_T3) nj = (c + NPM_OUT - 1) / NPM_OUT;
            }
        }
        auto reserve = [&](uint32_t v, uint32_t *counter) -> uint32_t {
            const uint32_t inc = wave_incl_sum(v);
            uint32_t b = 0;
            if (lane_id() == 63 && inc) b = atomicAdd(counter, inc);
            return (uint32_t)__builtin_amdgcn_readlane((int)b, 63) + inc - v;
        };
        const uint32_t o0 = reserve(n0, &L.counts[0]), o1 = reserve(n1, &L.counts[1]);
        const uint32_t o2 = reserve(n2, &L.counts[2]), o3 = reserve(n3, &L.counts[3]);
        const uint32_t oj = reserve(nj, &L.counts[4]);
        const uint32_t oc = reserve(ncp, &L.counts[5]);
        const uint32_t entry = grouped ? (g | NP_GROUP_FLAG) : x;
        if (n0) L.c0[o0] = entry;
        if (n1) L.c1[o1] = entry;
        if (n2) L.c2[o2] = entry;
        for (uint32_t k = 0; k < n3; ++k) L.c3[o3 + k] = ((uint64_t)x << 32) | k;
        for (uint32_t k = 0; k < nj; ++k) L.jobs[oj + k] = ((uint64_t)x << 32) | k;
        for (uint32_t k = 0; k < ncp; ++k) L.cp[oc + k] = ((uint64_t)entry << 32) | k;
    }
}

// Ranges already in ascending order, copied from the placement buffer to
// node_points in parts of NP_T3 values (an entry: node or group << 32 | part).
__global__ void k_np_copy(const uint64_t *list, const uint32_t *list_cnt, const uint32_t *nb, uint32_t nn,
                          const uint32_t *src, uint32_t *dst)
{
    const uint32_t cnt = *list_cnt;
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const uint64_t v = list[e];
        const uint32_t x = (uint32_t)(v >> 32), part = (uint32_t)v;
        uint32_t lo, hi;
        if (x & NP_GROUP_FLAG) {
            const uint32_t g = x & ~NP_GROUP_FLAG;
            lo = nb[g * NP_GROUP];
            hi = nb[min(g * NP_GROUP + NP_GROUP, nn)];
        } else {
            lo = nb[x];
            hi = nb[x + 1];
        }
        const uint32_t b = lo + part * NP_T3, end = min(hi, b + NP_T3);
        for (uint32_t i = b + threadIdx.x; i < end; i += blockDim.x) dst[i] = src[i];
    }
}

// One wave per work chunk: every point into its node's range.  Where one
// offset places a depth's points (a piece of a shared node, or the own root),
// positions are handed out from it: the wave keeps depth d's next position in
// LDS, a row of 64 points groups its lanes by depth with a ballot match over
// the depth's five bits, each lane takes the group's base plus its rank in
// the group (so a piece keeps the row order), and the group's first lane
// advances the base.  Points of own nodes below a subdivided root take
// theirs from global fill counters (zeroed before).
constexpr int NPP_ITEMS = 8;    // positions per lane and step (measured: 4, 16 and 32 slower)
constexpr int NPP_WAVES = 4;

__global__ __launch_bounds__(64 * NPP_WAVES) void k_np_place(WcArgs a, const uint32_t *node_base, const uint32_t *pnode,
                                                             const uint32_t *poff, const uint32_t *nb, uint32_t *fill,
                                                             uint32_t *out, uint32_t n_total, uint32_t *err)
{
    static_assert(MAXD <= 32, "depths fit five bits");
    __shared__ uint32_t nxt_all[NPP_WAVES][MAXD];
    const uint32_t lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    const uint32_t W = a.num_wc;
    uint32_t *nxt = nxt_all[threadIdx.x >> 6];   // this wave's next position per depth
    for (uint32_t w = blockIdx.x * NPP_WAVES + (threadIdx.x >> 6); w < W; w += gridDim.x * NPP_WAVES) {
        const int lw = a.wc_level[w], cut = a.cut[w];
        const uint32_t base = a.wc_begin[w], n = a.wc_count[w];
        uint32_t next = NP_NONE;   // lane d < MAXD: first position of depth d
        if (lane < (uint32_t)MAXD) {
            const uint64_t i = (uint64_t)lane * W + w;
            const uint32_t node = pnode[i];
            if (node != NP_NONE) next = nb[node] + poff[i];
            nxt[lane] = next;
        }
        __builtin_amdgcn_wave_barrier();
        // own nodes below a subdivided root (their points find no offset)
        const bool general = cut == lw && (uint32_t)__builtin_amdgcn_readlane((int)next, lw) == NP_NONE;
        bool bad = false;
        for (uint32_t c0 = 0; c0 < n; c0 += 64 * NPP_ITEMS) {
            uint32_t t8[NPP_ITEMS], o[NPP_ITEMS];
#pragma unroll
            for (int j = 0; j < NPP_ITEMS; ++j) {
                const uint32_t p = c0 + j * 64 + lane;
                t8[j] = p < n ? a.t[base + p] : 0xffu;
                o[j] = p < n ? a.wc_orig[base + p] : 0u;
            }
#pragma unroll
            for (int j = 0; j < NPP_ITEMS; ++j) {
                const uint32_t p = c0 + j * 64 + lane;
                int t = (int)t8[j];
                bad |= p < n && t >= MAXD;   // never placed: an internal error
                const bool ok = p < n && t < MAXD;
                t = np_final_depth(ok ? t : 0, lw, cut);
                const uint64_t peers = match_peers((uint32_t)t, ok, 5);
                const uint32_t rank = (uint32_t)__popcll(peers & below);
                const uint32_t b = ok ? nxt[t] : NP_NONE;
                __builtin_amdgcn_wave_barrier();
                if (ok && rank == 0 && b != NP_NONE) nxt[t] = b + (uint32_t)__popcll(peers);
                __builtin_amdgcn_wave_barrier();
                uint32_t dst = (ok && b != NP_NONE) ? b + rank : NP_NONE;
                if (general && ok && dst == NP_NONE && t >= lw) {
                    const uint32_t id = node_base[(uint64_t)t * W + w] + a.fr[base + p];
                    dst = nb[id] + atomicAdd(&fill[id], 1u);
                }
                if (dst < n_total) out[dst] = o[j];
                else bad |= ok;
            }
        }
        if (__ballot(bad) && lane == 0) atomicOr(err, 1u);
    }
}

// Inclusive sum over the wave with DPP row shifts and row broadcasts.
__device__ __forceinline__ uint32_t wave_incl_sum_dpp(uint32_t v)
{
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return (uint32_t)x;
}

// Exclusive scan of one value per thread across the block (DPP within waves);
// *total = sum.  lds: BLOCK / 64 + 1 words.  Ends with a barrier.
template <int BLOCK>
__device__ __forceinline__ uint32_t np_block_scan(uint32_t v, uint32_t *lds, uint32_t *total)
{
    constexpr int NW = BLOCK / 64;
    const uint32_t inc = wave_incl_sum_dpp(v);
    if constexpr (NW == 1) {
        *total = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        return inc - v;
    } else {
        const int w = threadIdx.x >> 6;
        if (lane_id() == 63) lds[w] = inc;
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const uint32_t x = lds[k];
            before += k < w ? x : 0u;
            all += x;
        }
        *total = all;
        __syncthreads();
        return before + inc - v;
    }
}

template <int BLOCK, int KPT, bool CHECK>
__device__ __forceinline__ void np_radix_count(const uint32_t (&k)[KPT], uint32_t (&loc)[KPT / 2], int sh,
                                               uint32_t *cnt, uint32_t col, uint32_t first, uint32_t len)
{
    constexpr uint32_t ROW = BLOCK + BLOCK / 16;
    // every atomic is issued before any result is used, so they overlap
    uint32_t r[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        r[j] = 0;
        if (!CHECK || first + j < len) {
            const uint32_t d = k[j] >> sh;
            r[j] = atomicAdd(&cnt[(d & 15u) * ROW + col], 1u << (d & 16u));
        }
    }
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const uint32_t l = (r[j] >> ((k[j] >> sh) & 16u)) & 0xffffu;
        if (j % 2 == 0) loc[j / 2] = l;
        else loc[j / 2] |= l << 16;
    }
}

template <int BLOCK, int KPT, bool CHECK>
__device__ __forceinline__ void np_radix_scatter(const uint32_t (&k)[KPT], const uint32_t (&loc)[KPT / 2], int sh,
                                                 const uint32_t *cnt, uint32_t *keys, uint32_t col, uint32_t low_total,
                                                 uint32_t first, uint32_t len)
{
    constexpr uint32_t ROW = BLOCK + BLOCK / 16;
    constexpr int KSH = ilog2_c(KPT);
    uint32_t dst[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const uint32_t d = k[j] >> sh;
        const uint32_t h = d & 16u;
        const uint32_t pre = cnt[(d & 15u) * ROW + col];
        dst[j] = ((pre >> h) & 0xffffu) + (h ? low_total : 0u) + ((loc[j / 2] >> (16 * (j % 2))) & 0xffffu);
    }
#pragma unroll
    for (int j = 0; j < KPT; ++j)
        if (!CHECK || first + j < len) keys[dst[j] + (dst[j] >> KSH)] = k[j];
}

// LDS radix sort of the block's first len keys (KPT per thread, blocked:
// thread i holds elements i * KPT ..; the rest is padding), 5 bits per pass
// from bit 0 up to `bits`; stable, so the passes compose.  Each thread counts
// its own keys per digit in 16-bit halves (digit d in word d & 15, half
// d >> 4; words [d & 15][thread], one padding word per 16), the words are
// scanned in that order (both halves at once; the high half then adds the low
// total), and keys move through LDS.  A thread's counter words are its own
// outside the scan, so it clears them right after reading its offsets.  Waves
// holding only padding skip the passes; only the wave at the end of the keys
// checks each key (with SKIP: measured faster for 8192-value tiles only; the
// larger code is slower for the others).  The sorted keys are left in keys[]
// (element e < len at e + e / KPT).  cnt must be zero on entry; it is zero on
// exit.
template <int BLOCK, int KPT, bool SKIP>
__device__ void np_radix(uint32_t (&k)[KPT], uint32_t len, int bits, uint32_t *keys, uint32_t *cnt, uint32_t *red)
{
    static_assert(BLOCK * KPT <= 65535, "16-bit counters");
    constexpr uint32_t ROW = BLOCK + BLOCK / 16;   // counter words per digit row, padding included
    const uint32_t tid = threadIdx.x;
    const uint32_t col = tid + (tid >> 4);         // the thread's column
    const uint32_t first = tid * KPT;
    const uint32_t wave_first = (tid & ~63u) * KPT;
    // full, partly, no keys (without SKIP every wave counts as full: the
    // padding then sorts last, its keys being all ones)
    const int mode = !SKIP || wave_first + 64 * KPT <= len ? 2 : wave_first < len ? 1 : 0;
    for (int sh = 0; sh < bits; sh += 5) {
        // the thread's rank among its own keys of the same digit (16 bits each)
        uint32_t loc[KPT / 2];
        if (mode == 2) np_radix_count<BLOCK, KPT, false>(k, loc, sh, cnt, col, first, len);
        else if (mode == 1) np_radix_count<BLOCK, KPT, true>(k, loc, sh, cnt, col, first, len);
        __syncthreads();
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) s += cnt[tid * 17 + i];
        uint32_t tot;
        uint32_t ex = np_block_scan<BLOCK>(s, red, &tot);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t v = cnt[tid * 17 + i];
            cnt[tid * 17 + i] = ex;
            ex += v;
        }
        const uint32_t low_total = tot & 0xffffu;
        __syncthreads();
        if (mode == 2) np_radix_scatter<BLOCK, KPT, false>(k, loc, sh, cnt, keys, col, low_total, first, len);
        else if (mode == 1) np_radix_scatter<BLOCK, KPT, true>(k, loc, sh, cnt, keys, col, low_total, first, len);
#pragma unroll
        for (int i = 0; i < 16; ++i) cnt[i * ROW + col] = 0;
        __syncthreads();
        if (sh + 5 < bits && mode != 0) {
#pragma unroll
            for (int j = 0; j < KPT; ++j) k[j] = keys[tid * (KPT + 1) + j];
        }
    }
}

__device__ __forceinline__ uint32_t bits_for(uint32_t span) { return span ? 32u - (uint32_t)__clz(span) : 0u; }

// Sorts src[r0, r0 + len) (len <= BLOCK * KPT) into dst[r0, ..): by segment
// (nseg > 1: segment s starts at segb[s], relative) and then by value.
template <int BLOCK, int KPT, bool SKIP>
__device__ void np_sort_range(const uint32_t *src, uint32_t *dst, uint32_t r0, uint32_t len, uint32_t nseg,
                              const uint32_t *segb, uint32_t *keys, uint32_t *cnt, uint32_t *red)
{
    const uint32_t tid = threadIdx.x;
#pragma unroll 4
    for (int j = 0; j < KPT; ++j) {
        const uint32_t e = j * BLOCK + tid;
        keys[e + e / KPT] = e < len ? src[r0 + e] : 0u;
    }
    __syncthreads();
    uint32_t k[KPT];
    uint32_t mn = 0xffffffffu, mx = 0;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        k[j] = keys[tid * (KPT + 1) + j];
        if (tid * KPT + j < len) {
            mn = min(mn, k[j]);
            mx = max(mx, k[j]);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = min(mn, (uint32_t)__shfl_xor(mn, o, 64));
        mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
    }
    if constexpr (BLOCK > 64) {
        if (lane_id() == 0) {
            red[2 * (tid >> 6)] = mn;
            red[2 * (tid >> 6) + 1] = mx;
        }
        __syncthreads();
        mn = 0xffffffffu;
        mx = 0;
        for (int w = 0; w < BLOCK / 64; ++w) {
            mn = min(mn, red[2 * w]);
            mx = max(mx, red[2 * w + 1]);
        }
        __syncthreads();
    }
    const uint32_t kb = bits_for(mx - mn);
    const uint32_t kmask = kb >= 32 ? 0xffffffffu : (1u << kb) - 1u;
    uint32_t bits = kb;
    if (nseg > 1) {
        // segment index above the value bits (at most 32 segments: 5 bits)
        bits = kb + 5;
        uint32_t e = tid * KPT, s = 0;
#pragma unroll
        for (int j = 0; j < KPT; ++j, ++e) {
            while (s + 1 < nseg && segb[s + 1] <= e) ++s;
            k[j] = e < len ? (s << kb) | (k[j] - mn) : 0xffffffffu;
        }
    } else {
#pragma unroll
        for (int j = 0; j < KPT; ++j) k[j] = tid * KPT + j < len ? k[j] - mn : 0xffffffffu;
    }
    // padding keys are all ones: every digit maximal, and they start after
    // the real keys, so a stable sort leaves them last
    np_radix<BLOCK, KPT, SKIP>(k, len, (int)bits, keys, cnt, red);
#pragma unroll 4
    for (int j = 0; j < KPT; ++j) {
        const uint32_t e = j * BLOCK + tid;
        if (e < len) dst[r0 + e] = bits ? (keys[e + e / KPT] & kmask) + mn : keys[e + e / KPT];
    }
    __syncthreads();
}

// One tile per list entry.  Classes 0..2 (LONG = false): a group of small
// nodes (sorted by node, then value) or one node.  Class 3 (LONG): one part of
// NP_T3 values of a node; a node of R merge rounds leaves its sorted parts
// where round 0 reads them: dst when R is even, alt when odd (the rounds
// alternate, the last one writes dst).
// waves per SIMD each tile size is compiled for (registers held to it, no spills)
constexpr int np_sort_waves(int block, int kpt) { return block * kpt <= 4096 ? 3 : 2; }

template <int BLOCK, int KPT, bool LONG, bool SKIP = false>
__global__ __launch_bounds__(BLOCK, np_sort_waves(BLOCK, KPT)) void k_np_sort(const void *list, const uint32_t *list_cnt, const uint32_t *nb,
                                                   uint32_t nn, const uint32_t *src, uint32_t *dst, uint32_t *alt)
{
    constexpr uint32_t T = BLOCK * KPT;
    __shared__ uint32_t keys[T + BLOCK];
    __shared__ uint32_t cnt[17 * BLOCK];
    __shared__ uint32_t red[2 * (BLOCK / 64) + 2];
    __shared__ uint32_t segb[NP_GROUP + 1];
    const uint32_t count = *list_cnt;
    for (uint32_t i = threadIdx.x; i < 17 * BLOCK; i += BLOCK) cnt[i] = 0;   // the radix passes keep it zero
    __syncthreads();
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        uint32_t r0, len, nseg = 0, nsub = 1;
        uint32_t *out = dst;
        if constexpr (LONG) {
            const uint64_t e = static_cast<const uint64_t *>(list)[i];
            const uint32_t x = (uint32_t)(e >> 32), part = (uint32_t)e;
            const uint32_t b = nb[x], c = nb[x + 1] - b;
            const uint32_t R = ceil_log2_dev((c + T - 1) / T);
            r0 = b + part * T;
            len = min(T, c - part * T);
            if (R & 1u) out = alt;
        } else {
            const uint32_t e = static_cast<const uint32_t *>(list)[i];
            if (e & NP_GROUP_FLAG) {
                const uint32_t x0 = (e & ~NP_GROUP_FLAG) * NP_GROUP, x1 = min(x0 + NP_GROUP, nn);
                nseg = x1 - x0;
                r0 = nb[x0];
                len = nb[x1] - r0;
                if (threadIdx.x <= nseg) segb[threadIdx.x] = nb[x0 + threadIdx.x] - r0;
                // the segment index fits above the values when their span
                // needs at most 27 bits; else the nodes go one by one
                uint32_t mn = 0xffffffffu, mx = 0;
                for (uint32_t j = threadIdx.x; j < len; j += BLOCK) {
                    const uint32_t v = src[r0 + j];
                    mn = min(mn, v);
                    mx = max(mx, v);
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    mn = min(mn, (uint32_t)__shfl_xor(mn, o, 64));
                    mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
                }
                if (!__syncthreads_and(len == 0 || bits_for(mx - mn) <= 27)) {
                    nsub = nseg;
                    nseg = 0;
                }
            } else {
                r0 = nb[e];
                len = nb[e + 1] - r0;
            }
        }
        for (uint32_t sub = 0; sub < nsub; ++sub) {
            uint32_t rr = r0, ll = len;
            if (nsub > 1) {
                rr = r0 + segb[sub];
                ll = segb[sub + 1] - segb[sub];
            }
            np_sort_range<BLOCK, KPT, SKIP>(src, out, rr, ll, nseg, segb, keys, cnt, red);
        }
    }
}

// Merge path: how many of the first k outputs of merging sorted A and B
// (distinct values) come from A.  Wave-wide: 64 probes per step.
__device__ uint32_t merge_split_wave(const uint32_t *A, uint32_t la, const uint32_t *B, uint32_t lb, uint32_t k)
{
    uint32_t lo = k > lb ? k - lb : 0, hi = k < la ? k : la;
    // P(i): A[i] < B[k - 1 - i], true exactly for i below the answer
    while (lo < hi) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t i = lo + lane_id() * step;
        const bool p = i < hi && A[i] < B[k - 1 - i];
        const uint32_t t = (uint32_t)__popcll(__ballot(p));
        const uint32_t nlo = t == 0 ? lo : lo + (t - 1) * step + 1;
        const uint32_t nhi = lo + t * step < hi ? lo + t * step : hi;
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Merge round r of the long nodes: runs of NP_T3 << r sorted values, merged in
// pairs, NPM_OUT outputs per job; nodes needing fewer rounds are done.
constexpr int NPM_BLOCK = 256;
constexpr int NPM_KPT = NPM_OUT / NPM_BLOCK;

__global__ __launch_bounds__(NPM_BLOCK) void k_np_merge(const uint64_t *jobs, const uint32_t *njobs, const uint32_t *nb,
                                                        int r, uint32_t *dst_final, uint32_t *alt)
{
    __shared__ uint32_t in[NPM_OUT];
    __shared__ uint32_t out[NPM_OUT + NPM_OUT / NPM_KPT];
    __shared__ uint32_t split[2];
    const uint32_t nj = *njobs;
    const uint32_t tid = threadIdx.x;
    for (uint32_t q = blockIdx.x; q < nj; q += gridDim.x) {
        const uint64_t e = jobs[q];
        const uint32_t x = (uint32_t)(e >> 32), j = (uint32_t)e;
        const uint32_t b = nb[x], c = nb[x + 1] - b;
        const uint32_t R = ceil_log2_dev((c + NP_T3 - 1) / NP_T3);
        if ((uint32_t)r >= R) continue;
        // after k rounds a node's values sit in dst_final when R - k is even
        const uint32_t *S = (((R - r) & 1u) == 0 ? dst_final : alt) + b;
        uint32_t *D = (((R - r) & 1u) == 0 ? alt : dst_final) + b;
        const uint64_t L = (uint64_t)NP_T3 << r;
        const uint32_t o0 = j * NPM_OUT, o1 = min(o0 + NPM_OUT, c);
        const uint32_t a0 = (uint32_t)(o0 / (2 * L) * (2 * L));
        const uint32_t a1 = (uint32_t)min((uint64_t)a0 + L, (uint64_t)c);
        const uint32_t b1 = (uint32_t)min((uint64_t)a0 + 2 * L, (uint64_t)c);
        if (a1 >= b1) {   // an unpaired last run: already sorted
            for (uint32_t i = o0 + tid; i < o1; i += NPM_BLOCK) D[i] = S[i];
            continue;
        }
        const uint32_t la = a1 - a0, lb = b1 - a1, k0 = o0 - a0, k1 = o1 - a0;
        if (tid < 128) {
            const uint32_t s = merge_split_wave(S + a0, la, S + a1, lb, tid < 64 ? k0 : k1);
            if (lane_id() == 0) split[tid >> 6] = s;
        }
        __syncthreads();
        const uint32_t i0 = split[0], i1 = split[1];
        const uint32_t na = i1 - i0, nbv = (k1 - i1) - (k0 - i0), tot = k1 - k0;
        for (uint32_t i = tid; i < na; i += NPM_BLOCK) in[i] = S[a0 + i0 + i];
        for (uint32_t i = tid; i < nbv; i += NPM_BLOCK) in[na + i] = S[a1 + (k0 - i0) + i];
        __syncthreads();
        const uint32_t d0 = tid * NPM_KPT;
        if (d0 < tot) {
            uint32_t lo = d0 > nbv ? d0 - nbv : 0, hi = d0 < na ? d0 : na;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (in[mid] < in[na + d0 - 1 - mid]) lo = mid + 1; else hi = mid;
            }
            uint32_t ia = lo, ib = d0 - lo;
            for (int s = 0; s < NPM_KPT && d0 + s < tot; ++s) {
                const bool takeA = ib >= nbv || (ia < na && in[ia] < in[na + ib]);
                const uint32_t v = takeA ? in[ia++] : in[na + ib++];
                const uint32_t o = d0 + s;
                out[o + o / NPM_KPT] = v;
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < tot; i += NPM_BLOCK) D[o0 + i] = out[i + i / NPM_KPT];
        __syncthreads();
    }
}

// Chunk of every work chunk: the chunk holding the first occupied finest cell
// of the work chunk (found by descending the count pyramid; an occupied cell
// always lies inside a chunk).
__global__ void k_wc_chunks(const uint32_t *num_wc_dev, uint32_t max_wc, const uint64_t *wc_key, const uint8_t *wc_level, int g,
                            const uint32_t *pyr, CutIndex chunks, const uint8_t *chunk_level,
                            uint32_t *wc_chunk, uint8_t *wc_nested, uint32_t *flags, const uint32_t *wc_count,
                            uint32_t L, int s, uint32_t *class_counts)
{
    const uint32_t num_wc = min(*num_wc_dev, max_wc);
    for (uint32_t w0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); w0 < num_wc; w0 += gridDim.x * blockDim.x) {
        // per-list counts of the work chunks, for the host to skip empty launches
        const uint32_t w = w0 + lane_id();
        uint32_t ci = 0xffffffffu;
        if (w < num_wc) {
            uint64_t m = wc_key[w];
            for (int l = wc_level[w]; l < g; ++l) {
                const uint32_t *ch = pyr + pyr_off(l + 1) + (m << 3);
                uint32_t o = 0;
                while (o < 7 && ch[o] == 0) ++o;   // the work chunk holds a point, so some child does
                m = (m << 3) | o;
            }
            const uint32_t c = cut_find(chunks, m);
            wc_chunk[w] = c;
            const bool nested = chunk_level[c] <= wc_level[w];
            wc_nested[w] = nested ? 1 : 0;
            if (!nested) atomicOr(&flags[0], 1u);
            ci = wc_list_class(wc_count[w], nested, L, s);
        }
        for (uint32_t k = 0; k <= (uint32_t)WC_CLASSES; ++k) {
            const uint64_t b = __ballot(ci == k);
            if (b && lane_id() == (uint32_t)(__ffsll((long long)b) - 1)) atomicAdd(&class_counts[k], (uint32_t)__popcll(b));
        }
    }
}

// Work-chunk range of every chunk: the chunk of each work chunk (that of its
// first finest cell) never decreases in Morton order, so chunk c's work chunks
// are those from the first with a chunk >= c to the first with a chunk > c,
// found by binary search.  flags[1]: a chunk holds more than MS_MAX_BINS.
__device__ __forceinline__ uint32_t wc_first_of(const uint32_t *wc_chunk, uint32_t n, uint32_t c)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (wc_chunk[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__global__ void k_wc_segs(const uint32_t *num_wc_dev, uint32_t max_wc, const uint32_t *num_chunks_dev,
                          uint32_t max_chunks, const uint32_t *wc_chunk, uint32_t *seg_b0, uint32_t *seg_nb,
                          uint32_t *flags)
{
    const uint32_t num_wc = min(*num_wc_dev, max_wc), num_chunks = min(*num_chunks_dev, max_chunks);
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < num_chunks; c += gridDim.x * blockDim.x) {
        const uint32_t b0 = wc_first_of(wc_chunk, num_wc, c), e = wc_first_of(wc_chunk, num_wc, c + 1);
        seg_b0[c] = b0;
        seg_nb[c] = e - b0;
        if (e - b0 > MS_MAX_BINS) atomicOr(&flags[1], 1u);
    }
}


// Node table: depth and key of every node, and child masks.  Local nodes
// carry the masks computed inside their WC; a shared node's mask is the OR of
// the octants of its children (shared nodes or WC roots).
__global__ void k_node_fill(WcArgs a, const uint32_t *node_base, uint8_t *depth, uint64_t *key, uint8_t *mask)
{
    const uint64_t total = (uint64_t)MAXD * a.num_wc;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const int d = (int)(i / a.num_wc);
        const uint32_t w = (uint32_t)(i % a.num_wc);
        const int lw = a.wc_level[w];
        const int cut = a.cut[w];
        const uint64_t wkey = a.wc_key[w];
        if (d < lw) {
            if (d > cut) continue;
            bool first = true;
            if (w > 0) {
                const int lp = a.wc_level[w - 1];
                if (lp > d && (a.wc_key[w - 1] >> (3 * (lp - d))) == (wkey >> (3 * (lw - d)))) first = false;
            }
            if (!first) continue;
            if (!(d < cut || a.alive[(uint64_t)d * a.num_wc + w] > 0)) continue;
            const uint32_t id = node_base[i];
            const uint64_t k = wkey >> (3 * (lw - d));
            depth[id] = (uint8_t)d;
            key[id] = k;
            if (d > 0) {
                const uint32_t pid = node_base[(uint64_t)(d - 1) * a.num_wc + owner_of(a, w, d - 1)];
                atomicOr(reinterpret_cast<uint32_t *>(mask + (pid & ~3u)), (1u << (k & 7u)) << (8 * (pid & 3u)));
            }
        } else if (cut == lw) {
            const uint32_t K = a.kd[(uint64_t)w * MAXD + d];
            if (K == 0) continue;
            const uint32_t id0 = node_base[i];
            const uint64_t lo = a.wc_begin[w] + a.loff[(uint64_t)w * MAXD + d];
            for (uint32_t r = 0; r < K; ++r) {
                depth[id0 + r] = (uint8_t)d;
                key[id0 + r] = a.lnode_key[lo + r];
                const uint32_t m = a.lnode_mask[lo + r];
                if (m) atomicOr(reinterpret_cast<uint32_t *>(mask + ((id0 + r) & ~3u)), m << (8 * ((id0 + r) & 3u)));
            }
            if (d == lw && lw > 0) {
                const uint32_t pid = node_base[(uint64_t)(d - 1) * a.num_wc + owner_of(a, w, d - 1)];
                atomicOr(reinterpret_cast<uint32_t *>(mask + (pid & ~3u)), (1u << (wkey & 7u)) << (8 * (pid & 3u)));
            }
        }
    }
}

// ---- step 5: preview ---------------------------------------------------------------------------
// Modes: keep index i iff H64(i) mod M == 0, iff i mod M == 0 (an exact
// stride), or iff i is the point of least H64 in its count-grid cell (one pick
// per occupied cell; H64 is a bijection, so there are no ties).  The kept
// indices form an n-bit map, compacted in order: count per tile, scan, write.

__device__ __forceinline__ bool keep(const PreviewArgs &p, uint64_t i)
{
    if (p.mode == PV_GRID) return h64(i) == p.cellmin[p.code[i] >> p.shift];
    const uint64_t v = p.mode == PV_STRIDE ? i : h64(i);
    return (p.m & (p.m - 1)) == 0 ? (v & (p.m - 1)) == 0 : (v % p.m) == 0;
}

// The predicate of every index into an n-bit map: a wave covers 64
// consecutive indices per step, and its ballot is two words of the map.
// A block covers one tile of the compaction (4096 indices, 128 words) and
// also writes the tile's count.
constexpr int PV_BLOCK = 256, PV_ITEMS = 16;
constexpr uint64_t PV_TILE = PV_BLOCK * PV_ITEMS;

__global__ __launch_bounds__(PV_BLOCK) void k_preview_bits(PreviewArgs p, uint32_t *__restrict__ bits,
                                                           uint32_t *__restrict__ tile_counts)
{
    __shared__ uint32_t wsum[PV_BLOCK / 64];
    if (p.zero && blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < p.zero_words; i += PV_BLOCK) p.zero[i] = 0u;
    const uint64_t words = (p.n + 31) / 32;
    const uint64_t base = (uint64_t)blockIdx.x * PV_TILE + (uint64_t)(threadIdx.x >> 6) * (64 * PV_ITEMS);
    const uint32_t lane = lane_id();
    uint32_t cnt = 0, mine = 0;   // lane k < 2 * PV_ITEMS keeps word k of the wave's run
#pragma unroll
    for (int j = 0; j < PV_ITEMS; ++j) {
        const uint64_t i = base + (uint64_t)j * 64 + lane;
        const uint64_t m = __ballot(i < p.n && keep(p, i));
        cnt += (uint32_t)__popcll(m);
        if (lane == (uint32_t)(2 * j)) mine = (uint32_t)m;
        if (lane == (uint32_t)(2 * j + 1)) mine = (uint32_t)(m >> 32);
    }
    // the wave's words in one store
    const uint64_t w = base / 32 + lane;
    if (lane < (uint32_t)(2 * PV_ITEMS) && w < words) bits[w] = mine;
    if (tile_counts) {
        if (lane_id() == 0) wsum[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int k = 0; k < PV_BLOCK / 64; ++k) t += wsum[k];
            tile_counts[blockIdx.x] = t;
        }
    }
}

// Grid preview from the per-cell minima (computed by the quantise pass): the
// pick of an occupied cell is the index whose hash is the cell's minimum, so
// inverting the hash gives it directly; its bit is set in an n-bit map.
__global__ void k_grid_picks(const unsigned long long *__restrict__ cellmin, uint64_t cells, uint64_t n,
                             uint32_t *__restrict__ bits)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += stride) {
        const unsigned long long h = cellmin[c];
        if (h == ~0ull) continue;
        const uint64_t i = h64_inverse(h);
        if (i < n) atomicOr(&bits[i >> 5], 1u << (i & 31));
    }
}

// Ordered compaction of a bit map, a word per thread.
constexpr int BW_BLOCK = 128, BW_ITEMS = 1;
constexpr uint64_t BW_TILE = (uint64_t)BW_BLOCK * BW_ITEMS;   // words per tile

__global__ __launch_bounds__(BW_BLOCK) void k_bits_count(const uint32_t *__restrict__ bits, uint64_t words,
                                                         uint32_t *tc)
{
    __shared__ uint32_t red[BW_BLOCK / 64 + 1];
    const uint64_t base = (uint64_t)blockIdx.x * BW_TILE;
    uint32_t c = 0;
    for (int j = 0; j < BW_ITEMS; ++j) {
        const uint64_t w = base + (uint64_t)j * BW_BLOCK + threadIdx.x;
        c += w < words ? (uint32_t)__popc(bits[w]) : 0u;
    }
    c = block_sum<BW_BLOCK>(c, red);
    if (threadIdx.x == 0) tc[blockIdx.x] = c;
}

__global__ __launch_bounds__(BW_BLOCK) void k_bits_write(const uint32_t *__restrict__ bits, uint64_t words,
                                                         const uint32_t *toff, uint32_t *out)
{
    __shared__ uint32_t lds[BW_BLOCK / 64 + 1];
    const uint64_t base = (uint64_t)blockIdx.x * BW_TILE;
    uint32_t run = toff[blockIdx.x];
    for (int j = 0; j < BW_ITEMS; ++j) {
        const uint64_t w = base + (uint64_t)j * BW_BLOCK + threadIdx.x;
        uint32_t b = w < words ? bits[w] : 0u;
        uint32_t tot;
        uint32_t o = run + block_excl_scan<BW_BLOCK>((uint32_t)__popc(b), lds, &tot);
        while (b) {
            const int k = __ffs(b) - 1;
            out[o++] = (uint32_t)(w * 32 + (uint64_t)k);
            b &= b - 1;
        }
        run += tot;
    }
}

// ---- launchers -----------------------------------------------------------------------------------

static uint32_t grid_for(uint64_t n, uint32_t block, uint32_t cap = 4096)
{
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

struct FillSpecs {
    FillSpec f[4];
};
__global__ void k_fill_many(FillSpecs s)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t *p = s.f[k].p;
        const uint32_t v = s.f[k].v;
        const uint64_t words = p ? s.f[k].words : 0;
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = v;
    }
}

void launch_fill_many(const FillSpec (&f)[4], hipStream_t st)
{
    FillSpecs s;
    uint64_t most = 0;
    for (int k = 0; k < 4; ++k) {
        s.f[k] = f[k];
        if (f[k].p && f[k].words > most) most = f[k].words;
    }
    if (most == 0) return;
    hipLaunchKernelGGL(k_fill_many, dim3(grid_for(most, 256, 2048)), dim3(256), 0, st, s);
}

void launch_fill_u32(uint32_t *p, uint32_t v, uint64_t words, hipStream_t st)
{
    if (words == 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words, 256, 2048)), dim3(256), 0, st, p, v, words);
}

// at most 2048 blocks of four waves: one resident wave of blocks on 256 compute units
uint32_t bbox_blocks(uint64_t n) { return grid_for((n + 3) / 4, 256, BBOX_MAX_BLOCKS); }

void launch_bbox(const float *x, const float *y, const float *z, uint64_t n, uint32_t *part, hipStream_t st,
                 uint32_t *zero, uint64_t zero_words)
{
    const int vec4 = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(z)) & 15) == 0;
    hipLaunchKernelGGL(k_bbox, dim3(bbox_blocks(n)), dim3(256), 0, st, x, y, z, n, vec4, part, zero, zero_words);
}

void launch_setup(DevBox *box, const uint32_t *part, uint32_t nparts, int given, const float *lo, const float *hi,
                  int flag_only, hipStream_t st)
{
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, st, box, part, nparts, given, lo[0], lo[1], lo[2], hi[0], hi[1],
                       hi[2], flag_only);
}

void launch_quantize(const float *x, const float *y, const float *z, uint64_t n, const DevBox *box, int g,
                     int given, uint64_t *code, uint32_t *fine_cnt, DevBox *box_rw, uint64_t base,
                     uint64_t *cellmin, hipStream_t st, int variant)
{
    if (n == 0) return;
    // one contiguous range per block: 256 blocks (one per compute unit) for
    // variants 0 and 3 and the grid preview, 512 for variant 1, 1024 for
    // variant 2
    if (cellmin) variant = 0;
    const uint64_t blocks = variant == 2 ? 1024 : variant == 1 ? 512 : 256;
    uint64_t per = (n + blocks - 1) / blocks;
    per = (per + 63) / 64 * 64;
    const uint32_t grid = (uint32_t)((n + per - 1) / per);
    auto *cm = reinterpret_cast<unsigned long long *>(cellmin);
    if (cellmin)
        hipLaunchKernelGGL((k_quantize<true>), dim3(grid), dim3(1024), 0, st, x, y, z, n, box, g, given, code,
                           fine_cnt, box_rw, per, base, cm);
    else if (variant == 2)
        hipLaunchKernelGGL((k_quantize<false, 256, 12>), dim3(grid), dim3(256), 0, st, x, y, z, n, box, g, given,
                           code, fine_cnt, box_rw, per, base, cm);
    else if (variant == 1)
        hipLaunchKernelGGL((k_quantize<false, 512, 13>), dim3(grid), dim3(512), 0, st, x, y, z, n, box, g, given,
                           code, fine_cnt, box_rw, per, base, cm);
    else if (variant == 3)
        hipLaunchKernelGGL((k_quantize<false, 1024, 14, 2>), dim3(grid), dim3(1024), 0, st, x, y, z, n, box, g,
                           given, code, fine_cnt, box_rw, per, base, cm);
    else
        hipLaunchKernelGGL((k_quantize<false>), dim3(grid), dim3(1024), 0, st, x, y, z, n, box, g, given, code,
                           fine_cnt, box_rw, per, base, cm);
}

// 64 bins or more, and no more (bin, block) histogram words than points (the
// scan's temporaries are sized by n)
bool quantize_binned_ok(uint64_t n, int g)
{
    return g >= 3 && g <= 9 && n >= QB_MIN_POINTS && n >= (1ull << (3 * g - qb_cell_bits(g))) * QB_BLOCKS;
}

size_t quantize_binned_temp_bytes(int g)
{
    const uint64_t words = (1ull << (3 * g - qb_cell_bits(g))) * QB_BLOCKS;
    return 2 * ((4 * words + 255) & ~(size_t)255);
}

void launch_quantize_binned(const float *x, const float *y, const float *z, uint64_t n, const DevBox *box, int g,
                            int given, uint64_t *code, uint32_t *fine_cnt, DevBox *box_rw, void *temp,
                            uint16_t *cells, void *scan_temp, hipStream_t st)
{
    if (n == 0) return;
    uint64_t per = (n + QB_BLOCKS - 1) / QB_BLOCKS;
    per = (per + 63) / 64 * 64;
    const uint32_t grid = (uint32_t)((n + per - 1) / per);
    const int cb = qb_cell_bits(g);
    const uint32_t nbins = 1u << (3 * g - cb);
    const uint64_t words = (uint64_t)nbins * grid;
    uint32_t *bhist = static_cast<uint32_t *>(temp);
    uint32_t *boff = bhist + (((4 * (uint64_t)nbins * QB_BLOCKS + 255) & ~255ull) / 4);
    hipLaunchKernelGGL(k_qz_bin_code, dim3(grid), dim3(QB_BLOCK), 0, st, x, y, z, n, box, g, given, code, bhist, box_rw,
                       per);
    scan_exclusive(bhist, boff, words, nullptr, scan_temp, st);
    hipLaunchKernelGGL(k_qz_bin_place, dim3(grid), dim3(QB_BLOCK), 0, st, code, n, g, boff, cells, per);
    hipLaunchKernelGGL(k_qz_bin_grid, dim3(nbins < 1024 ? nbins : 1024), dim3(1024), 0, st, cells, boff, grid, nbins,
                       cb, n, fine_cnt);
}

void launch_pyramid(uint32_t *pyr, int g, uint32_t *exp_out, hipStream_t st)
{
    // the finest level (g >= 5) with its export, levels above 5 one launch
    // each, the rest (level 5 = 32768 cells and up) in one block
    int l = g;
    if (g >= 5 && exp_out) {
        const uint64_t nboxes = (1ull << (3 * g)) / PE_CELLS;
        hipLaunchKernelGGL(k_pyr_export, dim3((uint32_t)(nboxes < 8192 ? nboxes : 8192)), dim3(PE_BLOCK), 0, st,
                           pyr, g, exp_out);
        --l;
    }
    for (; l >= 1 && l > 5; --l) {
        const uint64_t nchild = 1ull << (3 * l);
        hipLaunchKernelGGL(k_pyr_level, dim3(grid_for(nchild, 256)), dim3(256), 0, st, pyr, l);
    }
    if (l >= 1) hipLaunchKernelGGL(k_pyr_top, dim3(1), dim3(1024), 0, st, pyr, l, l == g ? exp_out : nullptr);
    else if (exp_out && g == 0) launch_grid_export(pyr, 0, exp_out, st);   // G = 1: the root is the finest level
}

void launch_grid_export(const uint32_t *fine, int g, uint32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_grid_export, dim3(grid_for(1ull << (3 * g), 256)), dim3(256), 0, st, fine, g, out);
}


uint32_t *global_depth_table(uint32_t *gtab, uint32_t *gtab2, int d0, int d) { return ((d0 - 1 - d) & 1) ? gtab2 : gtab; }

void launch_global_depths(const WcArgs &a, uint64_t n, uint32_t *gtab, uint32_t *gtab2, hipStream_t st,
                          bool first_filled)
{
    if (n == 0 || a.d0 == 0) return;
    for (int d = 0; d < a.d0; ++d) {
        uint32_t *tab = global_depth_table(gtab, gtab2, a.d0, d);
        const uint32_t *prev = d > 0 ? global_depth_table(gtab, gtab2, a.d0, d - 1) : nullptr;
        if (d > 0 || !first_filled) launch_fill_u32(tab, 0xffffffffu, 1ull << (3 * (d + a.s)), st);
        hipLaunchKernelGGL(k_gdepth_min, dim3(grid_for(n, GD_TILE, 8192)), dim3(GD_BLOCK), 0, st, a.wc_code, a.wc_orig,
                           a.t, n, 3 * (KB - d - a.s), tab, prev, 3 * (KB - d + 1 - a.s), d - 1);
    }
    // a work chunk holds at least one point, so every point is marked
    hipLaunchKernelGGL(k_wc_alive_rows, dim3(a.num_wc < 8192 ? a.num_wc : 8192), dim3(AR_BLOCK), 0, st, a,
                       global_depth_table(gtab, gtab2, a.d0, a.d0 - 1), 3 * (KB - (a.d0 - 1) - a.s));
}

void launch_cut(const uint32_t *pyr, const CutArgs &chunks, const CutArgs &wcs, hipStream_t st)
{
    if (chunks.open_cap <= CS_MAX_OPEN && wcs.open_cap <= CS_MAX_OPEN) {
        hipLaunchKernelGGL(k_cut_small, dim3(2), dim3(CS_BLOCK), 0, st, pyr, chunks, wcs);
    } else {
        const uint64_t ns = chunks.st_off[chunks.lam + 1] > wcs.st_off[wcs.lam + 1] ? chunks.st_off[chunks.lam + 1]
                                                                                      : wcs.st_off[wcs.lam + 1];
        hipLaunchKernelGGL(k_cut_init, dim3(grid_for(ns, 256, 1024)), dim3(256), 0, st, pyr, chunks, wcs);
        for (int l = 1; l <= chunks.lam; ++l) {
            const uint64_t t0 = chunks.st_off[l + 1] - chunks.st_off[l], t1 = wcs.st_off[l + 1] - wcs.st_off[l];
            const uint64_t tiles = t0 > t1 ? t0 : t1;
            if (tiles)
                hipLaunchKernelGGL(k_frontier, dim3((uint32_t)tiles, 2), dim3(FR_BLOCK), 0, st, pyr, l, chunks, wcs);
        }
    }
    const uint64_t slots = chunks.ent_off[chunks.lam + 1] > wcs.ent_off[wcs.lam + 1] ? chunks.ent_off[chunks.lam + 1]
                                                                                      : wcs.ent_off[wcs.lam + 1];
    hipLaunchKernelGGL(k_cut_rank, dim3(grid_for(slots, 256, 2048), 2), dim3(256), 0, st, pyr, chunks, wcs);
    const uint64_t cells = (1ull << (3 * chunks.lt)) + 1;
    hipLaunchKernelGGL(k_cut_index, dim3(grid_for(cells, CI_SPAN, 2048), 2), dim3(CI_BLOCK), 0, st, chunks, wcs);
}


void launch_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_u32_to_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, in, out, n);
}

void launch_subsample_small(const WcArgs &a, const uint32_t *lists, hipStream_t st)
{
    if (a.num_wc == 0) return;
    hipLaunchKernelGGL(k_list_classes, dim3(grid_for(a.num_wc, 256)), dim3(256), 0, st, a);
    // lists[c]: work chunks of class c (counted before the read-back); an
    // empty class is not launched, the others get at most one block per work
    // chunk.
    auto grid = [&](int c, uint32_t cap) { return lists[c] < cap ? lists[c] : cap; };
    // work chunks whose own root is a leaf: shared ancestors only
    // (few points per thread: a work chunk's depths run one after another, so
    // its latency bounds these kernels and the blocks resident per CU set
    // their speed.  Measured on the 20M-point planes: four points per thread
    // up to 1024 points, eight above)
    if (lists[0]) hipLaunchKernelGGL((k_subsample_fast<64, 4, 10>), dim3(grid(0, 8192)), dim3(64), 0, st, a, 0);
    if (lists[1]) hipLaunchKernelGGL((k_subsample_fast<128, 4, 11>), dim3(grid(1, 8192)), dim3(128), 0, st, a, 1);
    if (lists[2]) hipLaunchKernelGGL((k_subsample_fast<256, 4, 12>), dim3(grid(2, 8192)), dim3(256), 0, st, a, 2);
    if (lists[3]) hipLaunchKernelGGL((k_subsample_fast<256, 8, 12>), dim3(grid(3, 8192)), dim3(256), 0, st, a, 3);
    if (lists[4]) hipLaunchKernelGGL((k_subsample_fast<512, 8, 13>), dim3(grid(4, 8192)), dim3(512), 0, st, a, 4);
    // oversized work chunks at the deepest work-chunk level (dense clusters)
    if (lists[5]) hipLaunchKernelGGL((k_subsample_fast<1024, 8, 14>), dim3(grid(5, 2048)), dim3(1024), 0, st, a, 5);
    // the general subtree: single-wave blocks for the small classes, many per
    // CU.  Only work chunks with more than L points or subsample grids above
    // 2^7 go there
    if (lists[WC_GENERAL + 0])
        hipLaunchKernelGGL((k_subsample_lds<64, 4>), dim3(grid(WC_GENERAL + 0, 8192)), dim3(64), 0, st, a, WC_GENERAL + 0);
    if (lists[WC_GENERAL + 1])
        hipLaunchKernelGGL((k_subsample_lds<64, 8>), dim3(grid(WC_GENERAL + 1, 8192)), dim3(64), 0, st, a, WC_GENERAL + 1);
    if (lists[WC_GENERAL + 2])
        hipLaunchKernelGGL((k_subsample_lds<64, 16>), dim3(grid(WC_GENERAL + 2, 8192)), dim3(64), 0, st, a, WC_GENERAL + 2);
    if (lists[WC_GENERAL + 3])
        hipLaunchKernelGGL((k_subsample_lds<256, 8>), dim3(grid(WC_GENERAL + 3, 2048)), dim3(256), 0, st, a, WC_GENERAL + 3);
    if (lists[WC_GENERAL + 4])
        hipLaunchKernelGGL((k_subsample_lds<512, 8>), dim3(grid(WC_GENERAL + 4, 1024)), dim3(512), 0, st, a, WC_GENERAL + 4);
}

void launch_subsample_big(const WcArgs &a, hipStream_t st)
{
    if (a.num_wc == 0) return;
    const uint32_t grid = a.num_wc < 256 ? a.num_wc : 256;
    hipLaunchKernelGGL(k_subsample_big, dim3(grid), dim3(P1_BLOCK), 0, st, a);
}

void launch_decide(const WcArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_decide, dim3(grid_for(a.num_wc, 256 / DC_LANES)), dim3(256), 0, st, a);
}

void launch_node_counts(const WcArgs &a, uint32_t *owned, hipStream_t st)
{
    hipLaunchKernelGGL(k_node_counts, dim3(grid_for((uint64_t)MAXD * a.num_wc, 256)), dim3(256), 0, st, a, owned);
}

void launch_wc_chunks(const uint32_t *num_wc_dev, uint64_t max_wc, const uint64_t *wc_key, const uint8_t *wc_level,
                      int g, const uint32_t *pyr, const CutIndex &chunks, const uint8_t *chunk_level,
                      const uint32_t *num_chunks_dev, uint64_t max_chunks, uint32_t *wc_chunk, uint32_t *seg_b0,
                      uint32_t *seg_nb, uint8_t *wc_nested, uint32_t *flags, const uint32_t *wc_count, uint32_t L,
                      int s, uint32_t *class_counts, hipStream_t st)
{
    hipLaunchKernelGGL(k_wc_chunks, dim3(grid_for(max_wc, 256)), dim3(256), 0, st, num_wc_dev, (uint32_t)max_wc, wc_key,
                       wc_level, g, pyr,
                       chunks, chunk_level, wc_chunk, wc_nested, flags, wc_count, L, s, class_counts);
    hipLaunchKernelGGL(k_wc_segs, dim3(grid_for(max_chunks, 256)), dim3(256), 0, st, num_wc_dev, (uint32_t)max_wc,
                       num_chunks_dev, (uint32_t)max_chunks, wc_chunk, seg_b0, seg_nb, flags);
}

void launch_node_fill(const WcArgs &a, const uint32_t *node_base, uint8_t *depth, uint64_t *key, uint8_t *mask,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_node_fill, dim3(grid_for((uint64_t)MAXD * a.num_wc, 256)), dim3(256), 0, st, a, node_base,
                       depth, key, mask);
}

void launch_np_counts(const WcArgs &a, const uint32_t *node_base, uint32_t *cnt_dw, uint32_t *S, uint32_t *cnt_node,
                      uint32_t *pnode, uint32_t *glist, uint32_t *gcount, uint32_t *maxc, uint8_t *single,
                      void *scan_temp, hipStream_t st)
{
    if (a.num_wc == 0) return;
    const uint64_t rows = (uint64_t)MAXD * a.num_wc;
    hipLaunchKernelGGL(k_np_pieces, dim3(grid_for(rows, 256)), dim3(256), 0, st, a, cnt_dw);
    scan_exclusive(cnt_dw, S, rows, S + rows, scan_temp, st);
    // the piece offsets replace the piece sizes (scanned into S already)
    hipLaunchKernelGGL(k_np_shared, dim3(grid_for(rows, 256)), dim3(256), 0, st, a, node_base, S, cnt_node, pnode,
                       cnt_dw, glist, gcount, maxc, single);
    hipLaunchKernelGGL(k_np_count, dim3(a.num_wc < 2048 ? a.num_wc : 2048), dim3(NP_BLOCK), 0, st, a, node_base, glist,
                       gcount, cnt_node, maxc, single);
}

void launch_np_points(const WcArgs &a, const uint32_t *node_base, const uint32_t *pnode, const uint32_t *poff,
                      const uint32_t *cnt_node, uint32_t num_nodes, uint32_t max_count, uint64_t n, const NpWork &w,
                      hipStream_t st)
{
    if (n == 0 || num_nodes == 0) return;
    scan_exclusive(cnt_node, w.nb, num_nodes, w.nb + num_nodes, w.scan_temp, st);
    hipLaunchKernelGGL(k_np_lists, dim3(grid_for(num_nodes, 256, 1024)), dim3(256), 0, st, w.nb, num_nodes, w.lists);
    if (w.general) launch_fill_u32(w.fill, 0u, num_nodes, st);
    const uint32_t pg = (a.num_wc + NPP_WAVES - 1) / NPP_WAVES;
    hipLaunchKernelGGL(k_np_place, dim3(pg < 4096 ? pg : 4096), dim3(64 * NPP_WAVES), 0, st, a, node_base, pnode, poff,
                       w.nb, w.fill, w.tmp, (uint32_t)n, w.err);
    const uint64_t ncp = n / NP_T3 + num_nodes / NP_GROUP + 1;
    hipLaunchKernelGGL(k_np_copy, dim3(ncp < 4096 ? (uint32_t)ncp : 4096), dim3(256), 0, st, w.lists.cp, w.lists.counts + 5,
                       w.nb, num_nodes, w.tmp, w.out);
    if (w.place_timer) w.place_timer->end(st);
    if (w.sort_timer) w.sort_timer->begin(st);
    const uint32_t g0 = num_nodes < 8192 ? num_nodes : 8192;
    const uint64_t n1 = n / 1024 + num_nodes / NP_GROUP + 1, n2 = n / 4096 + 1, n3 = n / 8192 + n / NP_T3 + 1;
    hipLaunchKernelGGL((k_np_sort<64, 16, false>), dim3(g0), dim3(64), 0, st, w.lists.c0, w.lists.counts, w.nb,
                       num_nodes, w.tmp, w.out, w.tmp);
    hipLaunchKernelGGL((k_np_sort<256, 16, false>), dim3(n1 < 4096 ? (uint32_t)n1 : 4096), dim3(256), 0, st, w.lists.c1,
                       w.lists.counts + 1, w.nb, num_nodes, w.tmp, w.out, w.tmp);
    hipLaunchKernelGGL((k_np_sort<256, 32, false, true>), dim3(n2 < 2048 ? (uint32_t)n2 : 2048), dim3(256), 0, st,
                       w.lists.c2,
                       w.lists.counts + 2, w.nb, num_nodes, w.tmp, w.out, w.tmp);
    hipLaunchKernelGGL((k_np_sort<512, 32, true>), dim3(n3 < 1024 ? (uint32_t)n3 : 1024), dim3(512), 0, st, w.lists.c3,
                       w.lists.counts + 3, w.nb, num_nodes, w.tmp, w.out, w.tmp);
    const uint32_t rounds = ceil_log2((max_count + NP_T3 - 1) / NP_T3);
    const uint64_t njobs = np_job_entries(n);
    for (uint32_t r = 0; r < rounds; ++r)
        hipLaunchKernelGGL(k_np_merge, dim3(njobs < 4096 ? (uint32_t)njobs : 4096), dim3(NPM_BLOCK), 0, st,
                           w.lists.jobs, w.lists.counts + 4, w.nb, (int)r, w.out, w.tmp);
}

uint64_t np_list_entries(uint64_t n, int cls)
{
    // nodes number at most n; class 1 holds nodes above NP_T0 values and
    // groups, class 2 nodes above NP_T1, class 3 parts of nodes above NP_T2
    switch (cls) {
    case 0: return n + 1;
    case 1: return n / NP_T0 + n / NP_GROUP + 2;
    case 2: return n / NP_T1 + 1;
    default: return n / NP_T2 + n / NP_T3 + 2;
    }
}
uint64_t np_job_entries(uint64_t n) { return n / NPM_OUT + n / NP_T3 + 2; }
uint64_t np_copy_entries(uint64_t n) { return n + n / NP_T3 + 2; }

static uint64_t preview_tiles(uint64_t n) { return (n + PV_TILE - 1) / PV_TILE; }

static_assert(PV_TILE == BW_TILE * 32, "a preview block covers one compaction tile");

void launch_preview_bits(const PreviewArgs &p, uint32_t *bits, uint32_t *tile_counts, hipStream_t st)
{
    if (p.n == 0) return;
    hipLaunchKernelGGL(k_preview_bits, dim3((uint32_t)preview_tiles(p.n)), dim3(PV_BLOCK), 0, st, p, bits,
                       tile_counts);
}

uint64_t bits_tiles(uint64_t n) { return ((n + 31) / 32 + BW_TILE - 1) / BW_TILE; }

void launch_grid_picks(const uint64_t *cellmin, uint64_t cells, uint64_t n, uint32_t *bits, hipStream_t st)
{
    hipLaunchKernelGGL(k_grid_picks, dim3(grid_for(cells, 256, 8192)), dim3(256), 0, st,
                       reinterpret_cast<const unsigned long long *>(cellmin), cells, n, bits);
}

void launch_bits_count(const uint32_t *bits, uint64_t n, uint32_t *tc, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_bits_count, dim3((uint32_t)bits_tiles(n)), dim3(BW_BLOCK), 0, st, bits, (n + 31) / 32, tc);
}

void launch_bits_write(const uint32_t *bits, uint64_t n, const uint32_t *toff, uint32_t *out, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_bits_write, dim3((uint32_t)bits_tiles(n)), dim3(BW_BLOCK), 0, st, bits, (n + 31) / 32, toff,
                       out);
}

}  // namespace fpo

namespace fpo {

// ---- node-ordered points --------------------------------------------------------------------
// Gathers in node order: reads are random (one point each), writes coalesced.
__global__ void k_gather_points(const uint32_t *__restrict__ idx, uint64_t n, const float *__restrict__ x,
                                const float *__restrict__ y, const float *__restrict__ z,
                                const uint8_t *__restrict__ color, uint32_t stride, float *__restrict__ out_xyz,
                                uint8_t *__restrict__ out_color)
{
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = idx[k];
        out_xyz[3 * k + 0] = x[i];
        out_xyz[3 * k + 1] = y[i];
        out_xyz[3 * k + 2] = z[i];
        for (uint32_t c = 0; c < stride; ++c) out_color[(uint64_t)stride * k + c] = color[(uint64_t)stride * i + c];
    }
}

// Fingerprint of a byte range: the wrapping sum over its bytes b at offsets i
// of mix64((i << 8) | b + salt), so equal ranges give equal sums whatever the
// order of the additions, and a changed byte or a moved value changes the sum
// with high probability.  For comparing results of equivalent builds.
__global__ void k_fingerprint(const uint8_t *p, uint64_t bytes, uint64_t salt, unsigned long long *out)
{
    uint64_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes;
         i += (uint64_t)gridDim.x * blockDim.x)
        acc += mix64(((i << 8) | p[i]) + salt);
    acc = wave_sum64(acc);
    if (lane_id() == 0 && acc) atomicAdd(out, (unsigned long long)acc);
}

void launch_fingerprint(const void *p, uint64_t bytes, uint64_t salt, uint64_t *out, hipStream_t st)
{
    if (bytes == 0) return;
    hipLaunchKernelGGL(k_fingerprint, dim3(grid_for(bytes, 256, 4096)), dim3(256), 0, st,
                       static_cast<const uint8_t *>(p), bytes, salt, reinterpret_cast<unsigned long long *>(out));
}

void launch_gather_points(const uint32_t *idx, uint64_t n, const float *x, const float *y, const float *z,
                          const uint8_t *color, uint32_t stride, float *out_xyz, uint8_t *out_color, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_points, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, idx, n, x, y, z,
                       color, stride, out_xyz, out_color);
}

}  // namespace fpo
