/*
 * CPU oracle -- TEST INFRASTRUCTURE ONLY (see fpo_oracle.h).
 *
 * Plain, slow, single-threaded C that writes out each step of the path as
 * its definition reads.  Compiled with -ffp-contract=off so that every float
 * operation below is one IEEE-754 binary32 operation rounded to nearest even.
 *
 * Notation: N points indexed 0..N-1 in input order (the "original index");
 * K = 21 bits per axis of the shared integer lattice; G = 2^g count grid;
 * C = max points per chunk; S = 2^s subsample grid; L = leaf capacity;
 * M = preview modulus.  u(p) is the fine lattice coordinate of point p.
 * The node/cell/chunk at level l that holds p is u(p) >> (K - l) per axis.
 * Morton keys interleave the axes with x as the most significant bit of each
 * triple, so the octant of a child is (bx<<2)|(by<<1)|bz and
 * child key = parent key * 8 + octant.
 */
#include "fpo_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define K_BITS 21
#define U_MAX ((1u << K_BITS) - 1u)

/* ---- preview hash (reading of "hash(idx)"): a xorshift-multiply mix with the
 * golden-ratio constant floor(2^64/phi); all arithmetic mod 2^64. ---------- */
uint64_t oracle_h64(uint64_t i)
{
    const uint64_t phi = 0x9E3779B97F4A7C15ull;
    uint64_t h = i;
    h ^= h >> 31;
    h *= phi;
    h ^= h >> 29;
    h *= phi;
    h ^= h >> 32;
    return h;
}

static int is_pow2(uint32_t v) { return v != 0 && (v & (v - 1)) == 0; }
static uint32_t ilog2(uint32_t v) { uint32_t l = 0; while ((1u << l) < v) ++l; return l; }

/* Morton key of the level-l cell (cx, cy, cz), each < 2^l. */
static uint64_t morton(uint32_t cx, uint32_t cy, uint32_t cz, uint32_t l)
{
    uint64_t k = 0;
    for (int b = (int)l - 1; b >= 0; --b) {
        k = (k << 3) | ((uint64_t)((cx >> b) & 1u) << 2) | ((uint64_t)((cy >> b) & 1u) << 1)
            | (uint64_t)((cz >> b) & 1u);
    }
    return k;
}

/* Row-major count-grid cell [cx][cy][cz] of fine coordinates u[0..2]. */
static uint64_t grid_cell(const uint32_t *u, uint32_t G, uint32_t g)
{
    return ((uint64_t)(u[0] >> (K_BITS - g)) * G + (u[1] >> (K_BITS - g))) * G + (u[2] >> (K_BITS - g));
}

/* ---- step 1a: quantization onto the 21-bit lattice ------------------------
 * Reading: the cube is anchored at the box minimum with side = the largest
 * extent; scale = 2^21 / side computed in double and rounded once to float
 * (0 when the side is 0); u = clamp(floor((a - min) * scale), 0, 2^21-1) with
 * one float subtraction and one float multiplication.  A NaN product (0*inf
 * when the side underflows) maps to 0. */
static uint32_t quantize(float a, float lo, float scale)
{
    float t = (a - lo) * scale;
    if (!(t > 0.0f)) return 0u;
    if (t >= (float)U_MAX) return U_MAX;
    return (uint32_t)floorf(t);
}

typedef struct {
    uint32_t d;
    uint64_t key;
    uint8_t child_mask;
    uint32_t *pts;
    uint32_t npts;
} onode;

typedef struct {
    const uint32_t *u;
    uint32_t s, S, L, dmax;
    int32_t *best;          /* S^3 cell table, -1 = empty */
    uint32_t *touched;
    onode *nodes;
    size_t nnodes, cap;
    int oom;
} octree_ctx;

static onode *push_node(octree_ctx *c)
{
    if (c->nnodes == c->cap) {
        size_t nc = c->cap ? c->cap * 2 : 1024;
        onode *nn = (onode *)realloc(c->nodes, nc * sizeof(onode));
        if (!nn) { c->oom = 1; return NULL; }
        c->nodes = nn;
        c->cap = nc;
    }
    onode *n = &c->nodes[c->nnodes++];
    memset(n, 0, sizeof(*n));
    return n;
}

/* ---- step 4: top-down node subsampling -----------------------------------
 * A node at depth d receives the set R of points that reach it (ascending
 * original index).  If |R| <= L, or d is the deepest depth 21 - s at which a
 * node still has an S^3 grid of lattice cells, the node is a leaf and keeps
 * all of R.  Otherwise the node lays an S^3 grid over its cube; for every
 * occupied grid cell it keeps the point of lowest original index (the first
 * one met, since R is ascending) and pushes every other point to the child
 * octant that contains it.  Only non-empty children are created.
 * Returns the index of the node in c->nodes. */
static size_t build_node(octree_ctx *c, uint32_t d, uint64_t key, uint32_t *R, uint32_t nR)
{
    onode *me = push_node(c);
    if (!me) return 0;
    size_t me_idx = c->nnodes - 1;
    me->d = d;
    me->key = key;
    me->child_mask = 0;

    if (nR <= c->L || d == c->dmax) {
        me->pts = (uint32_t *)malloc((size_t)(nR ? nR : 1) * sizeof(uint32_t));
        if (!me->pts) { c->oom = 1; return me_idx; }
        memcpy(me->pts, R, (size_t)nR * sizeof(uint32_t));
        me->npts = nR;
        return me_idx;
    }

    const uint32_t cell_shift = K_BITS - d - c->s;   /* cells are lattice level d + s */
    const uint32_t oct_bit = K_BITS - 1 - d;          /* children are lattice level d + 1 */
    uint32_t *kept = (uint32_t *)malloc((size_t)nR * sizeof(uint32_t));
    uint32_t *rest = (uint32_t *)malloc((size_t)nR * sizeof(uint32_t));
    if (!kept || !rest) { free(kept); free(rest); c->oom = 1; return me_idx; }
    uint32_t nk = 0, nrest = 0, ntouched = 0;
    for (uint32_t j = 0; j < nR; ++j) {
        uint32_t i = R[j];
        const uint32_t *ui = &c->u[(size_t)i * 3];
        uint32_t cx = (ui[0] >> cell_shift) & (c->S - 1);
        uint32_t cy = (ui[1] >> cell_shift) & (c->S - 1);
        uint32_t cz = (ui[2] >> cell_shift) & (c->S - 1);
        uint32_t cell = (cx * c->S + cy) * c->S + cz;
        if (c->best[cell] < 0) {
            c->best[cell] = (int32_t)i;
            c->touched[ntouched++] = cell;
            kept[nk++] = i;
        } else {
            rest[nrest++] = i;
        }
    }
    for (uint32_t t = 0; t < ntouched; ++t) c->best[c->touched[t]] = -1;

    me = &c->nodes[me_idx];
    me->pts = kept;
    me->npts = nk;

    /* split the pushed points by octant, keeping their order */
    uint32_t cnt[8] = {0}, off[8];
    for (uint32_t j = 0; j < nrest; ++j) {
        const uint32_t *ui = &c->u[(size_t)rest[j] * 3];
        uint32_t o = (((ui[0] >> oct_bit) & 1u) << 2) | (((ui[1] >> oct_bit) & 1u) << 1) | ((ui[2] >> oct_bit) & 1u);
        cnt[o]++;
    }
    uint32_t acc = 0;
    for (int o = 0; o < 8; ++o) { off[o] = acc; acc += cnt[o]; }
    uint32_t *split = (uint32_t *)malloc((size_t)(nrest ? nrest : 1) * sizeof(uint32_t));
    if (!split) { free(rest); c->oom = 1; return me_idx; }
    uint32_t fill[8];
    memcpy(fill, off, sizeof(fill));
    for (uint32_t j = 0; j < nrest; ++j) {
        const uint32_t *ui = &c->u[(size_t)rest[j] * 3];
        uint32_t o = (((ui[0] >> oct_bit) & 1u) << 2) | (((ui[1] >> oct_bit) & 1u) << 1) | ((ui[2] >> oct_bit) & 1u);
        split[fill[o]++] = rest[j];
    }
    free(rest);
    uint8_t mask = 0;
    for (uint32_t o = 0; o < 8; ++o) {
        if (cnt[o] == 0) continue;
        mask |= (uint8_t)(1u << o);
        build_node(c, d + 1, key * 8u + o, split + off[o], cnt[o]);
        if (c->oom) break;
    }
    free(split);
    c->nodes[me_idx].child_mask = mask;
    return me_idx;
}

static int cmp_node(const void *a, const void *b)
{
    const onode *x = (const onode *)a, *y = (const onode *)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return 0;
}

typedef struct {
    uint32_t g, C;
    uint32_t **lvl;           /* lvl[l]: 2^l x 2^l x 2^l counts, row-major */
    uint8_t *level; uint64_t *key; uint32_t *count;
    uint32_t n, cap;
    int oom;
} cut_ctx;

/* ---- step 2b: chunk cut ---------------------------------------------------
 * A pyramid node is a chunk when it is non-empty and holds at most C points
 * (or is a finest cell, which may then hold more: an oversized chunk), and
 * its parent holds more than C.  Visiting top-down in octant order emits the
 * chunks in Morton pre-order. */
static void cut(cut_ctx *c, uint32_t l, uint32_t cx, uint32_t cy, uint32_t cz)
{
    uint32_t side = 1u << l;
    uint32_t cnt = c->lvl[l][((size_t)cx * side + cy) * side + cz];
    if (cnt == 0) return;
    if (cnt <= c->C || l == c->g) {
        if (c->n == c->cap) {
            uint32_t nc = c->cap ? c->cap * 2 : 256;
            uint8_t *nl = (uint8_t *)realloc(c->level, nc);
            uint64_t *nk = (uint64_t *)realloc(c->key, nc * sizeof(uint64_t));
            uint32_t *nn = (uint32_t *)realloc(c->count, nc * sizeof(uint32_t));
            if (nl) c->level = nl;
            if (nk) c->key = nk;
            if (nn) c->count = nn;
            if (!nl || !nk || !nn) { c->oom = 1; return; }
            c->cap = nc;
        }
        c->level[c->n] = (uint8_t)l;
        c->key[c->n] = morton(cx, cy, cz, l);
        c->count[c->n] = cnt;
        c->n++;
        return;
    }
    for (uint32_t o = 0; o < 8 && !c->oom; ++o)
        cut(c, l + 1, 2 * cx + ((o >> 2) & 1u), 2 * cy + ((o >> 1) & 1u), 2 * cz + (o & 1u));
}

void oracle_free(oracle_result *r)
{
    if (!r) return;
    free(r->u); free(r->count_grid);
    free(r->chunk_level); free(r->chunk_key); free(r->chunk_count); free(r->chunk_begin);
    free(r->perm);
    free(r->node_depth); free(r->node_key); free(r->node_child_mask);
    free(r->node_begin); free(r->node_count); free(r->node_points);
    free(r->preview_index);
    memset(r, 0, sizeof(*r));
}

#define CHK(p) do { if (!(p)) { st = ORACLE_ERR_OOM; goto done; } } while (0)

int oracle_build(uint64_t n, const float *x, const float *y, const float *z,
                 const oracle_params *p, oracle_result *out)
{
    int st = ORACLE_OK;
    memset(out, 0, sizeof(*out));
    out->n = n;

    if (!p || !is_pow2(p->count_grid) || p->count_grid > 512 || !is_pow2(p->subsample_grid)
        || p->subsample_grid > 256 || p->max_points_per_chunk == 0 || p->leaf_capacity == 0
        || p->preview_modulus == 0 || p->preview_mode > ORACLE_PREVIEW_GRID || n > 0xFFFFFFFFull || (n > 0 && (!x || !y || !z))) {
        out->status = ORACLE_ERR_INVALID_ARG;
        return out->status;
    }
    if (p->bbox_given) {
        for (int a = 0; a < 3; ++a)
            if (!isfinite(p->bbox_min[a]) || !isfinite(p->bbox_max[a]) || p->bbox_min[a] > p->bbox_max[a]) {
                out->status = ORACLE_ERR_INVALID_ARG;
                return out->status;
            }
    }

    const uint32_t G = p->count_grid, g = ilog2(G);
    const uint32_t S = p->subsample_grid, s = ilog2(S);
    const uint32_t C = p->max_points_per_chunk, L = p->leaf_capacity, M = p->preview_modulus;
    const float *xyz[3] = {x, y, z};

    /* ---- step 1a: bounding box (exact min/max; any NaN/Inf is an error) ---- */
    for (uint64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            if (!isfinite(xyz[a][i])) { out->status = ORACLE_ERR_NONFINITE; return out->status; }
    if (p->bbox_given) {
        for (int a = 0; a < 3; ++a) { out->bbox_min[a] = p->bbox_min[a]; out->bbox_max[a] = p->bbox_max[a]; }
        for (uint64_t i = 0; i < n; ++i) {
            int outside = 0;
            for (int a = 0; a < 3; ++a)
                if (xyz[a][i] < p->bbox_min[a] || xyz[a][i] > p->bbox_max[a]) outside = 1;
            out->n_outside += (uint64_t)outside;
        }
    } else if (n > 0) {
        for (int a = 0; a < 3; ++a) { out->bbox_min[a] = xyz[a][0]; out->bbox_max[a] = xyz[a][0]; }
        for (uint64_t i = 1; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                if (xyz[a][i] < out->bbox_min[a]) out->bbox_min[a] = xyz[a][i];
                if (xyz[a][i] > out->bbox_max[a]) out->bbox_max[a] = xyz[a][i];
            }
        /* -0.0 and +0.0 compare equal, so which one a min/max keeps depends on
         * the visiting order; report +0.0 (x + 0.0f maps -0.0 to +0.0 and
         * leaves every other value unchanged) */
        for (int a = 0; a < 3; ++a) {
            out->bbox_min[a] = out->bbox_min[a] + 0.0f;
            out->bbox_max[a] = out->bbox_max[a] + 0.0f;
        }
    }
    /* cube: side = largest extent (float subtraction), scale = 2^21 / side */
    float side = 0.0f;
    for (int a = 0; a < 3; ++a) {
        float ext = out->bbox_max[a] - out->bbox_min[a];
        if (ext > side) side = ext;
    }
    out->cube_size = side;
    out->scale = side > 0.0f ? (float)((double)(1u << K_BITS) / (double)side) : 0.0f;

    /* fine coordinates */
    CHK(out->u = (uint32_t *)malloc((size_t)(n ? n : 1) * 3 * sizeof(uint32_t)));
    for (uint64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            out->u[i * 3 + a] = quantize(xyz[a][i], out->bbox_min[a], out->scale);

    /* ---- step 1b: count grid, row-major [cx][cy][cz], c = u >> (21 - g) ---- */
    const size_t G3 = (size_t)G * G * G;
    CHK(out->count_grid = (uint32_t *)calloc(G3, sizeof(uint32_t)));
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t *ui = &out->u[i * 3];
        uint32_t cx = ui[0] >> (K_BITS - g), cy = ui[1] >> (K_BITS - g), cz = ui[2] >> (K_BITS - g);
        out->count_grid[((size_t)cx * G + cy) * G + cz]++;
    }

    /* ---- step 2a: count pyramid, each level the 2x2x2 sums of the next ---- */
    {
        cut_ctx cc;
        memset(&cc, 0, sizeof(cc));
        cc.g = g;
        cc.C = C;
        CHK(cc.lvl = (uint32_t **)calloc(g + 1, sizeof(uint32_t *)));
        cc.lvl[g] = out->count_grid;
        for (int l = (int)g - 1; l >= 0; --l) {
            uint32_t sd = 1u << l, sc = 2u * sd;
            cc.lvl[l] = (uint32_t *)calloc((size_t)sd * sd * sd, sizeof(uint32_t));
            if (!cc.lvl[l]) { cc.oom = 1; break; }
            for (uint32_t cx = 0; cx < sc; ++cx)
                for (uint32_t cy = 0; cy < sc; ++cy)
                    for (uint32_t cz = 0; cz < sc; ++cz)
                        cc.lvl[l][((size_t)(cx / 2) * sd + cy / 2) * sd + cz / 2] +=
                            cc.lvl[l + 1][((size_t)cx * sc + cy) * sc + cz];
        }
        if (!cc.oom) cut(&cc, 0, 0, 0, 0);
        for (uint32_t l = 0; l < g; ++l) free(cc.lvl[l]);
        free(cc.lvl);
        out->num_chunks = cc.n;
        out->chunk_level = cc.level;
        out->chunk_key = cc.key;
        out->chunk_count = cc.count;
        if (cc.oom) { st = ORACLE_ERR_OOM; goto done; }
    }
    CHK(out->chunk_begin = (uint64_t *)malloc((size_t)(out->num_chunks ? out->num_chunks : 1) * sizeof(uint64_t)));
    {
        uint64_t acc = 0;
        for (uint32_t k = 0; k < out->num_chunks; ++k) {
            out->chunk_begin[k] = acc;
            acc += out->chunk_count[k];
            if (out->chunk_count[k] > C) out->chunk_oversized_any = 1;
        }
    }

    /* ---- step 3: stable scatter; visiting points in index order, each goes to
     * the next free slot of its chunk ---- */
    CHK(out->perm = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t)));
    {
        uint32_t *chunk_of = (uint32_t *)malloc(G3 * sizeof(uint32_t));
        uint64_t *fill = (uint64_t *)malloc((size_t)(out->num_chunks ? out->num_chunks : 1) * sizeof(uint64_t));
        if (!chunk_of || !fill) { free(chunk_of); free(fill); st = ORACLE_ERR_OOM; goto done; }
        for (uint32_t k = 0; k < out->num_chunks; ++k) {
            /* paint every finest cell inside the chunk with its id */
            uint32_t l = out->chunk_level[k], span = 1u << (g - l);
            uint32_t ccx = 0, ccy = 0, ccz = 0;
            uint64_t key = out->chunk_key[k];
            for (uint32_t b = 0; b < l; ++b) {
                ccz |= (uint32_t)((key >> (3 * b)) & 1u) << b;
                ccy |= (uint32_t)((key >> (3 * b + 1)) & 1u) << b;
                ccx |= (uint32_t)((key >> (3 * b + 2)) & 1u) << b;
            }
            for (uint32_t dx = 0; dx < span; ++dx)
                for (uint32_t dy = 0; dy < span; ++dy)
                    for (uint32_t dz = 0; dz < span; ++dz)
                        chunk_of[((size_t)(ccx * span + dx) * G + (ccy * span + dy)) * G + (ccz * span + dz)] = k;
            fill[k] = out->chunk_begin[k];
        }
        for (uint64_t i = 0; i < n; ++i) {
            const uint32_t *ui = &out->u[i * 3];
            uint32_t cx = ui[0] >> (K_BITS - g), cy = ui[1] >> (K_BITS - g), cz = ui[2] >> (K_BITS - g);
            uint32_t k = chunk_of[((size_t)cx * G + cy) * G + cz];
            out->perm[fill[k]++] = (uint32_t)i;
        }
        free(chunk_of);
        free(fill);
    }

    /* ---- step 4: octree; the root receives every point in index order ---- */
    CHK(out->node_points = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t)));
    if (n > 0) {
        octree_ctx oc;
        memset(&oc, 0, sizeof(oc));
        oc.u = out->u;
        oc.s = s;
        oc.S = S;
        oc.L = L;
        oc.dmax = K_BITS - s;
        oc.best = (int32_t *)malloc((size_t)S * S * S * sizeof(int32_t));
        oc.touched = (uint32_t *)malloc((size_t)S * S * S * sizeof(uint32_t));
        uint32_t *R = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
        if (!oc.best || !oc.touched || !R) {
            free(oc.best); free(oc.touched); free(R);
            st = ORACLE_ERR_OOM; goto done;
        }
        for (size_t c = 0; c < (size_t)S * S * S; ++c) oc.best[c] = -1;
        for (uint64_t i = 0; i < n; ++i) R[i] = (uint32_t)i;
        build_node(&oc, 0, 0, R, (uint32_t)n);
        free(R);
        free(oc.best);
        free(oc.touched);
        if (!oc.oom) {
            /* nodes in (depth, key) order; each node's points stay ascending */
            qsort(oc.nodes, oc.nnodes, sizeof(onode), cmp_node);
            size_t nn = oc.nnodes;
            out->num_nodes = (uint32_t)nn;
            out->node_depth = (uint8_t *)malloc(nn);
            out->node_key = (uint64_t *)malloc(nn * sizeof(uint64_t));
            out->node_child_mask = (uint8_t *)malloc(nn);
            out->node_begin = (uint64_t *)malloc(nn * sizeof(uint64_t));
            out->node_count = (uint32_t *)malloc(nn * sizeof(uint32_t));
            if (!out->node_depth || !out->node_key || !out->node_child_mask || !out->node_begin || !out->node_count)
                oc.oom = 1;
            uint64_t acc = 0;
            for (size_t k = 0; k < nn && !oc.oom; ++k) {
                out->node_depth[k] = (uint8_t)oc.nodes[k].d;
                out->node_key[k] = oc.nodes[k].key;
                out->node_child_mask[k] = oc.nodes[k].child_mask;
                out->node_begin[k] = acc;
                out->node_count[k] = oc.nodes[k].npts;
                memcpy(out->node_points + acc, oc.nodes[k].pts, (size_t)oc.nodes[k].npts * sizeof(uint32_t));
                acc += oc.nodes[k].npts;
            }
        }
        for (size_t k = 0; k < oc.nnodes; ++k) free(oc.nodes[k].pts);
        free(oc.nodes);
        if (oc.oom) { st = ORACLE_ERR_OOM; goto done; }
    }

    /* ---- step 5: preview, ascending indices ----
     * hash:   H64(i) mod M == 0 (section "Immediate Low-Resolution Rendering")
     * stride: i mod M == 0 (the fixed-target decimation of section "Results")
     * grid:   H64(i) is the least H64 among the points of i's count-grid cell
     *         (section "Future Work"); H64 is a bijection, so one point per
     *         occupied cell qualifies */
    {
        uint64_t *best = NULL;
        uint8_t *kept = NULL;
        CHK(kept = (uint8_t *)malloc((size_t)(n ? n : 1)));
        if (p->preview_mode == ORACLE_PREVIEW_GRID) {
            const uint64_t cells = (uint64_t)G * G * G;
            best = (uint64_t *)malloc((size_t)cells * sizeof(uint64_t));
            if (!best) { free(kept); st = ORACLE_ERR_OOM; goto done; }
            for (uint64_t c = 0; c < cells; ++c) best[c] = UINT64_MAX;
            for (uint64_t i = 0; i < n; ++i) {
                const uint64_t c = grid_cell(out->u + 3 * i, G, g);
                const uint64_t h = oracle_h64(i);
                if (h < best[c]) best[c] = h;
            }
        }
        uint64_t cnt = 0;
        for (uint64_t i = 0; i < n; ++i) {
            if (p->preview_mode == ORACLE_PREVIEW_GRID)
                kept[i] = oracle_h64(i) == best[grid_cell(out->u + 3 * i, G, g)];
            else if (p->preview_mode == ORACLE_PREVIEW_STRIDE)
                kept[i] = i % M == 0;
            else
                kept[i] = oracle_h64(i) % M == 0;
            cnt += kept[i];
        }
        free(best);
        out->preview_count = cnt;
        out->preview_index = (uint32_t *)malloc((size_t)(cnt ? cnt : 1) * sizeof(uint32_t));
        if (!out->preview_index) { free(kept); st = ORACLE_ERR_OOM; goto done; }
        uint64_t w = 0;
        for (uint64_t i = 0; i < n; ++i)
            if (kept[i]) out->preview_index[w++] = (uint32_t)i;
        free(kept);
    }

done:
    out->status = st;
    return st;
}
