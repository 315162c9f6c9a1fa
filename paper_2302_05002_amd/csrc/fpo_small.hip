// Single-workgroup builds of small clouds: every step of the path for one
// cloud in one workgroup of 1024 threads, and many clouds in one launch.
//
// The multi-kernel path spends a few dozen launches and two host round trips
// on every build, which dominates clouds of some ten thousand points.  Here a
// workgroup runs the steps back to back with barriers in between:
//   1. bounding box (or the given box), quantisation to the 21-bit lattice and
//      the count grid (section "Octree Construction", counting pass);
//   2. chunks: with n <= C the root is the only maximal node of at most C
//      points, so there is one chunk and perm is the identity;
//   3. the preview: the hash (or stride) predicate of every index, compacted
//      in order (section "Immediate Low-Resolution Rendering");
//   4. the tree top-down, one depth at a time (the node subsampling of
//      "Octree Construction"): the points reaching a depth are kept grouped by
//      node in key order, each group in ascending original index.  A node with
//      at most L points, or at the deepest depth, keeps them all.  Otherwise
//      each cell of its S^3 grid keeps its point of least original index and
//      the others go on to their child octants, stably.  The cell table of a
//      node lives in LDS: a cell's entry is (tag << 18 | position in the
//      node), the tag decreasing from node to node, so one atomic minimum
//      both replaces an entry of an earlier node and keeps the least position
//      of this one, and the table is never cleared.
// Every result array is the one the multi-kernel path writes, in the same
// layout; the node table is in (depth, key) order since depths are processed
// in turn and each depth's nodes are in key order.
#include "fpo_device.h"

namespace fpo {
namespace {

constexpr int SB_BLOCK = 1024;
constexpr int SB_W = SB_BLOCK / 64;
constexpr uint32_t SB_TAB = SB_MAX_S * SB_MAX_S * SB_MAX_S;
constexpr uint32_t SB_NODES = 8 * SB_MAX_INNER;       // nodes of one depth
constexpr uint32_t SB_POS_BITS = 18;
constexpr uint32_t SB_TAG_MAX = (1u << (32 - SB_POS_BITS)) - 1u;
constexpr int SB_U = 4;   // loads in flight per thread in the passes over points
static_assert(SB_MAX_N < (1u << SB_POS_BITS), "positions fit their field");

__device__ __forceinline__ bool sb_keep(uint32_t i, uint32_t m, bool stride)
{
    const uint64_t v = stride ? (uint64_t)i : h64(i);
    return (m & (m - 1u)) == 0 ? (v & (m - 1u)) == 0 : (v % m) == 0;
}

__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

// Category of point j of an inner node (range [b, b + c) of the depth's
// arrays): 8 when it wins its cell, else its child octant.
__device__ __forceinline__ uint32_t sb_category(const uint32_t *tab, uint64_t cc, uint32_t tagged_pos, int csh,
                                                uint32_t cmask, int osh)
{
    return tab[(uint32_t)(cc >> csh) & cmask] == tagged_pos ? 8u : (uint32_t)(cc >> osh) & 7u;
}

__global__ __launch_bounds__(SB_BLOCK) void k_small_build(SmallGroup grp)
{
    __shared__ uint32_t tab[SB_TAB];
    __shared__ unsigned long long nkey[2][SB_NODES];
    __shared__ uint32_t nbeg[2][SB_NODES], ncnt[2][SB_NODES];
    __shared__ uint32_t wcat[SB_W][9];     // per wave and category: count, then offset
    __shared__ uint32_t red[7][SB_W];
    __shared__ uint32_t cat_tot[9], cat_base[9];
    __shared__ float s_box[7];             // lo x, y, z, hi x, y, z, scale
    // [0] stop (non-finite input), [1] nodes of the next depth, [2] next
    // depth's array fill, [3] overflow
    __shared__ uint32_t s_u[4];

    const SmallDesc &D = grp.d[blockIdx.x];
    const uint32_t n = D.n;
    const SmallLayout Lo = small_layout(n, (int)D.g);
    char *ws = D.ws;
    Ctrs *ctrs = reinterpret_cast<Ctrs *>(ws + Lo.ctrs);
    DevBox *box = reinterpret_cast<DevBox *>(ws + Lo.box);
    const float *X = D.x, *Y = D.y, *Z = D.z;
    const uint32_t tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    const bool given = D.given != 0;

    for (uint32_t i = tid; i < sizeof(Ctrs) / 4; i += SB_BLOCK) reinterpret_cast<uint32_t *>(ctrs)[i] = 0u;

    // ---- 1. box ----
    if (!given) {
        uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u}, bad = 0;
        // SB_U points per thread and round, every load issued first
        for (uint32_t i0 = tid; i0 < n; i0 += SB_U * SB_BLOCK) {
            float px[SB_U], py[SB_U], pz[SB_U];
#pragma unroll
            for (int u = 0; u < SB_U; ++u) {
                const uint32_t i = min(i0 + u * SB_BLOCK, n - 1u);   // a repeat of the last point changes no extreme
                px[u] = X[i];
                py[u] = Y[i];
                pz[u] = Z[i];
            }
#pragma unroll
            for (int u = 0; u < SB_U; ++u) {
                bbox_acc(mn[0], mx[0], bad, px[u]);
                bbox_acc(mn[1], mx[1], bad, py[u]);
                bbox_acc(mn[2], mx[2], bad, pz[u]);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            for (int a = 0; a < 3; ++a) {
                mn[a] = min(mn[a], (uint32_t)__shfl_xor(mn[a], o, 64));
                mx[a] = max(mx[a], (uint32_t)__shfl_xor(mx[a], o, 64));
            }
            bad |= (uint32_t)__shfl_xor(bad, o, 64);
        }
        if (lane == 0) {
            for (int a = 0; a < 3; ++a) {
                red[a][w] = mn[a];
                red[3 + a][w] = mx[a];
            }
            red[6][w] = bad;
        }
        __syncthreads();
        if (tid == 0) {
            for (int v = 1; v < SB_W; ++v) {
                for (int a = 0; a < 3; ++a) {
                    mn[a] = min(mn[a], red[a][v]);
                    mx[a] = max(mx[a], red[3 + a][v]);
                }
                bad |= red[6][v];
            }
            box->nonfinite = bad;
            if (!bad) box_set(box, mn, mx, false, nullptr, nullptr);
            s_u[0] = bad;
        }
    } else if (tid == 0) {
        const float glo[3] = {D.glo[0], D.glo[1], D.glo[2]}, ghi[3] = {D.ghi[0], D.ghi[1], D.ghi[2]};
        box->nonfinite = 0u;
        box_set(box, nullptr, nullptr, true, glo, ghi);
        s_u[0] = 0u;
    }
    if (tid == 0 && !s_u[0]) {
        for (int a = 0; a < 3; ++a) {
            s_box[a] = box->lo[a];
            s_box[3 + a] = box->hi[a];
        }
        s_box[6] = box->scale;
    }
    __syncthreads();
    if (s_u[0]) return;   // a non-finite coordinate: the host reports it

    // ---- 1. quantise + count ----
    // The count grid is either cleared and counted with global atomics (few
    // points per cell), or, from n >= G^3 / 16 on, counted in LDS one range
    // of SB_TAB cells at a time from each point's cell id (kept in the ia
    // array until the tree needs it) and written once: a single workgroup
    // issues global atomics far more slowly than LDS ones.
    uint32_t *grid = reinterpret_cast<uint32_t *>(ws + Lo.grid);
    const uint32_t G = 1u << D.g, G3 = 1u << (3 * D.g);
    const bool lds_count = n >= (G3 >> 4);
    uint32_t *cell_id = reinterpret_cast<uint32_t *>(ws + Lo.ia);
    if (!lds_count) {
        for (uint32_t c = tid; c < G3; c += SB_BLOCK) grid[c] = 0u;
        __syncthreads();
    }
    uint64_t *code = reinterpret_cast<uint64_t *>(ws + Lo.code);
    {
        const float lx = s_box[0], ly = s_box[1], lz = s_box[2], hx = s_box[3], hy = s_box[4], hz = s_box[5];
        const float sc = s_box[6];
        const int gsh = KB - (int)D.g;
        uint32_t outside = 0, bad = 0;
        for (uint32_t i0 = tid; i0 < n; i0 += SB_U * SB_BLOCK) {
            float px[SB_U], py[SB_U], pz[SB_U];
#pragma unroll
            for (int u = 0; u < SB_U; ++u) {
                const uint32_t i = min(i0 + u * SB_BLOCK, n - 1u);
                px[u] = X[i];
                py[u] = Y[i];
                pz[u] = Z[i];
            }
#pragma unroll
            for (int u = 0; u < SB_U; ++u) {
                const uint32_t i = i0 + u * SB_BLOCK;
                if (i >= n) break;
                const uint32_t ux = quantize1(px[u], lx, sc), uy = quantize1(py[u], ly, sc), uz = quantize1(pz[u], lz, sc);
                code[i] = (split3(ux) << 2) | (split3(uy) << 1) | split3(uz);
                const uint32_t cell = ((ux >> gsh) * G + (uy >> gsh)) * G + (uz >> gsh);
                if (lds_count) cell_id[i] = cell;
                else atomicAdd(&grid[cell], 1u);
                if (given) {
                    outside += (px[u] < lx || px[u] > hx || py[u] < ly || py[u] > hy || pz[u] < lz || pz[u] > hz) ? 1u : 0u;
                    // NaN fails every comparison, an infinity exceeds the largest float
                    bad |= !(fabsf(px[u]) <= FLT_MAX && fabsf(py[u]) <= FLT_MAX && fabsf(pz[u]) <= FLT_MAX) ? 1u : 0u;
                }
            }
        }
        if (given) {
            outside = wave_sum(outside);
            const bool wbad = __ballot(bad != 0) != 0;
            if (lane == 0) {
                red[0][w] = outside;
                red[1][w] = wbad ? 1u : 0u;
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t t = 0, b = 0;
                for (int v = 0; v < SB_W; ++v) {
                    t += red[0][v];
                    b |= red[1][v];
                }
                box->n_outside = t;
                if (b) box->nonfinite = 1u;
                s_u[0] = b;
            }
        }
    }
    __syncthreads();
    if (s_u[0]) return;
    if (lds_count) {
        for (uint32_t r0 = 0; r0 < G3; r0 += SB_TAB) {
            const uint32_t span = min(SB_TAB, G3 - r0);
            for (uint32_t c = tid; c < span; c += SB_BLOCK) tab[c] = 0u;
            __syncthreads();
            for (uint32_t i0 = tid; i0 < n; i0 += SB_U * SB_BLOCK) {
                uint32_t cl[SB_U];
#pragma unroll
                for (int u = 0; u < SB_U; ++u) cl[u] = cell_id[min(i0 + u * SB_BLOCK, n - 1u)];
#pragma unroll
                for (int u = 0; u < SB_U; ++u)
                    if (i0 + u * SB_BLOCK < n && cl[u] - r0 < span) atomicAdd(&tab[cl[u] - r0], 1u);
            }
            __syncthreads();
            for (uint32_t c = tid; c < span; c += SB_BLOCK) grid[r0 + c] = tab[c];
            __syncthreads();
        }
    }

    // ---- 2. the one chunk ----
    if (tid == 0) {
        reinterpret_cast<uint8_t *>(ws + Lo.c_level)[0] = 0;
        reinterpret_cast<uint64_t *>(ws + Lo.c_key)[0] = 0;
        reinterpret_cast<uint32_t *>(ws + Lo.c_count)[0] = n;
        reinterpret_cast<uint64_t *>(ws + Lo.c_begin)[0] = 0;
        ctrs->num_chunks = 1u;
    }
    uint32_t *perm = reinterpret_cast<uint32_t *>(ws + Lo.perm);
    for (uint32_t i = tid; i < n; i += SB_BLOCK) perm[i] = i;

    // ---- 3. preview: each wave compacts a contiguous run of indices ----
    {
        uint32_t *pv = reinterpret_cast<uint32_t *>(ws + Lo.pv_index);
        const bool stride = D.stride != 0;
        const uint32_t M = D.M;
        const uint32_t seg = (n + SB_BLOCK - 1) / SB_BLOCK * 64;
        const uint32_t lo = min(n, w * seg), hi = min(n, lo + seg);
        uint32_t cnt = 0;
        for (uint32_t i0 = lo; i0 < hi; i0 += 64) {
            const uint32_t i = i0 + lane;
            cnt += (uint32_t)__popcll(__ballot(i < hi && sb_keep(i, M, stride)));
        }
        if (lane == 0) red[0][w] = cnt;
        __syncthreads();
        uint32_t base = 0, tot = 0;
        for (uint32_t v = 0; v < (uint32_t)SB_W; ++v) {
            const uint32_t t = red[0][v];
            base += v < w ? t : 0u;
            tot += t;
        }
        for (uint32_t i0 = lo; i0 < hi; i0 += 64) {
            const uint32_t i = i0 + lane;
            const bool k = i < hi && sb_keep(i, M, stride);
            const uint64_t b = __ballot(k);
            if (k) pv[base + __popcll(b & lanes_below())] = i;
            base += (uint32_t)__popcll(b);
        }
        if (tid == 0) ctrs->preview_count = tot;
    }

    // ---- 4. the tree, one depth at a time ----
    const uint32_t S3 = 1u << (3 * D.s), cmask = S3 - 1u;
    for (uint32_t c = tid; c < S3; c += SB_BLOCK) tab[c] = 0xffffffffu;
    if (tid == 0) {
        nkey[0][0] = 0;
        nbeg[0][0] = 0;
        ncnt[0][0] = n;
        s_u[3] = 0;
    }
    uint8_t *n_depth = reinterpret_cast<uint8_t *>(ws + Lo.n_depth);
    uint64_t *n_key = reinterpret_cast<uint64_t *>(ws + Lo.n_key);
    uint8_t *n_mask = reinterpret_cast<uint8_t *>(ws + Lo.n_mask);
    uint64_t *n_begin = reinterpret_cast<uint64_t *>(ws + Lo.n_begin);
    uint32_t *n_count = reinterpret_cast<uint32_t *>(ws + Lo.n_count);
    uint32_t *n_points = reinterpret_cast<uint32_t *>(ws + Lo.n_points);
    uint32_t *ia = reinterpret_cast<uint32_t *>(ws + Lo.ia), *ib = reinterpret_cast<uint32_t *>(ws + Lo.ib);
    uint64_t *ca = reinterpret_cast<uint64_t *>(ws + Lo.ca), *cb = reinterpret_cast<uint64_t *>(ws + Lo.cb);
    // the depth's points (index, code), grouped by node: depth 0 is the input
    // order itself; the next depth's are written to (nidx, ncode)
    const uint32_t *cidx = nullptr;
    const uint64_t *ccode = code;
    uint32_t *nidx = ia;
    uint64_t *ncode = ca;
    const uint32_t L = D.L;
    const int dmax = KB - (int)D.s;
    uint32_t ncur = 1, node_base = 0, out = 0, tag = SB_TAG_MAX;
    int cur = 0;
    bool err = false;
    for (int d = 0; ncur > 0; ++d) {
        const bool last = d >= dmax;
        const int nx = cur ^ 1;
        if (tid == 0) {
            s_u[1] = 0;
            s_u[2] = 0;
        }
        __syncthreads();
        uint32_t k = 0;
        while (k < ncur) {
            const uint32_t b = nbeg[cur][k], c = ncnt[cur][k];
            if (c <= L || last) {
                // a run of leaves: their points go to node_points as they are
                uint32_t k2 = k + 1;
                while (k2 < ncur && (ncnt[cur][k2] <= L || last)) ++k2;
                const uint32_t e = nbeg[cur][k2 - 1] + ncnt[cur][k2 - 1];
                for (uint32_t t = k + tid; t < k2 && node_base + t < n; t += SB_BLOCK) {
                    const uint32_t id = node_base + t;
                    n_depth[id] = (uint8_t)d;
                    n_key[id] = nkey[cur][t];
                    n_mask[id] = 0;
                    n_begin[id] = out + (nbeg[cur][t] - b);
                    n_count[id] = ncnt[cur][t];
                }
                for (uint32_t j = b + tid; j < e && out + (j - b) < n; j += SB_BLOCK)
                    n_points[out + (j - b)] = cidx ? cidx[j] : j;
                out += e - b;
                k = k2;
                continue;
            }
            // an inner node: cells of level d + s, children at level d + 1
            const int csh = 3 * (KB - d - (int)D.s), osh = 3 * (KB - d - 1);
            const uint32_t tg = tag << SB_POS_BITS;
            for (uint32_t j0 = b + tid; j0 < b + c; j0 += SB_U * SB_BLOCK) {
                uint64_t cc[SB_U];
#pragma unroll
                for (int u = 0; u < SB_U; ++u) cc[u] = ccode[min(j0 + u * SB_BLOCK, b + c - 1u)];
#pragma unroll
                for (int u = 0; u < SB_U; ++u) {
                    const uint32_t j = j0 + u * SB_BLOCK;
                    if (j < b + c) atomicMin(&tab[(uint32_t)(cc[u] >> csh) & cmask], tg | (j - b));
                }
            }
            __syncthreads();
            // each wave classifies a contiguous run of the node's points
            const uint32_t seg = (c + SB_BLOCK - 1) / SB_BLOCK * 64;
            const uint32_t lo = b + min(c, w * seg), hi = b + min(c, w * seg + seg);
            uint32_t cnt[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (uint32_t j0 = lo; j0 < hi; j0 += 64 * SB_U) {
                uint64_t cc[SB_U];
#pragma unroll
                for (int u = 0; u < SB_U; ++u) cc[u] = ccode[min(j0 + u * 64 + lane, hi - 1u)];
#pragma unroll
                for (int u = 0; u < SB_U; ++u) {
                    const uint32_t j = j0 + u * 64 + lane;
                    const uint32_t cat = j < hi ? sb_category(tab, cc[u], tg | (j - b), csh, cmask, osh) : 9u;
#pragma unroll
                    for (int q = 0; q < 9; ++q) cnt[q] += (uint32_t)__popcll(__ballot(cat == (uint32_t)q));
                }
            }
#pragma unroll
            for (int q = 0; q < 9; ++q)
                if (lane == (uint32_t)q) wcat[w][q] = cnt[q];
            __syncthreads();
            if (tid < 9) {
                uint32_t run = 0;
                for (int v = 0; v < SB_W; ++v) {
                    const uint32_t t = wcat[v][tid];
                    wcat[v][tid] = run;
                    run += t;
                }
                cat_tot[tid] = run;
            }
            __syncthreads();
            if (tid == 0) {
                // children in octant order, so the next depth stays in key order
                uint32_t at = s_u[2], mask = 0, q = s_u[1];
                const uint64_t key = nkey[cur][k];
                for (uint32_t o = 0; o < 8; ++o) {
                    cat_base[o] = at;
                    const uint32_t t = cat_tot[o];
                    if (t) {
                        mask |= 1u << o;
                        if (q < SB_NODES) {
                            nkey[nx][q] = key * 8u + o;
                            nbeg[nx][q] = at;
                            ncnt[nx][q] = t;
                        } else {
                            s_u[3] = 1u;
                        }
                        ++q;
                    }
                    at += t;
                }
                s_u[1] = q;
                s_u[2] = at;
                cat_base[8] = out;
                const uint32_t id = node_base + k;
                if (id < n) {
                    n_depth[id] = (uint8_t)d;
                    n_key[id] = key;
                    n_mask[id] = (uint8_t)mask;
                    n_begin[id] = out;
                    n_count[id] = cat_tot[8];
                }
            }
            __syncthreads();
            // the same classification again, now writing: winners to
            // node_points, the others to their child's run of the next depth
            uint32_t off[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) off[q] = cat_base[q] + wcat[w][q];
            for (uint32_t j0 = lo; j0 < hi; j0 += 64 * SB_U) {
                uint64_t cc[SB_U];
                uint32_t ix[SB_U];
#pragma unroll
                for (int u = 0; u < SB_U; ++u) {
                    const uint32_t j = min(j0 + u * 64 + lane, hi - 1u);
                    cc[u] = ccode[j];
                    ix[u] = cidx ? cidx[j] : j;
                }
#pragma unroll
                for (int u = 0; u < SB_U; ++u) {
                    const uint32_t j = j0 + u * 64 + lane;
                    const uint32_t cat = j < hi ? sb_category(tab, cc[u], tg | (j - b), csh, cmask, osh) : 9u;
                    uint32_t pos = 0;
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        const uint64_t bq = __ballot(cat == (uint32_t)q);
                        if (cat == (uint32_t)q) pos = off[q] + (uint32_t)__popcll(bq & lanes_below());
                        off[q] += (uint32_t)__popcll(bq);
                    }
                    // (every position is below n by construction; the bound
                    // keeps a broken count from writing past the arrays)
                    if (cat < 9u && pos < n) {
                        if (cat == 8u) {
                            n_points[pos] = ix[u];
                        } else {
                            nidx[pos] = ix[u];
                            ncode[pos] = cc[u];
                        }
                    }
                }
            }
            out += cat_tot[8];
            if (tag == 0) err = true;   // more inner nodes than tags (not reachable within the size limits)
            --tag;
            ++k;
            __syncthreads();   // the table, counts and bases are reused by the next node
        }
        node_base += ncur;
        __syncthreads();
        ncur = s_u[1];
        if (s_u[3] || err) {
            err = true;
            break;
        }
        cur = nx;
        cidx = nidx;
        ccode = ncode;
        nidx = cidx == ia ? ib : ia;
        ncode = ccode == ca ? cb : ca;
        __syncthreads();   // every thread has read the next depth's count before it is reset
    }
    if (tid == 0) {
        ctrs->num_nodes = node_base;
        if (err || out != n || node_base > n) ctrs->internal_error = 1u;
    }
}

}  // namespace

void launch_small_build(const SmallGroup &g, uint32_t count, hipStream_t st)
{
    if (count) hipLaunchKernelGGL(k_small_build, dim3(count), dim3(SB_BLOCK), 0, st, g);
}

}  // namespace fpo
