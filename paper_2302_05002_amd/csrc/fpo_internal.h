// Internal declarations shared by the kernels and the host orchestration of
// libfpo.  Not part of the public C ABI (that is include/fpo.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fpo {

constexpr int KB = 21;                       // bits per axis of the shared lattice
constexpr uint32_t UMAX = (1u << KB) - 1u;
constexpr int MAXD = 22;                     // depths 0..21

// Work chunks (internal decomposition of the subsample step) up to WC_CAP
// points are processed with their points in registers and LDS hash tables.
constexpr int P1_BLOCK = 1024;
constexpr int P1_ITEMS = 4;
constexpr uint32_t WC_CAP = P1_BLOCK * P1_ITEMS;   // 4096
constexpr uint32_t WC_HASH = 2 * WC_CAP;           // 8192 slots, load <= 1/2
// Size classes of the LDS path.  Classes 0-5: work chunks of at most L points
// (their own root is a leaf, so only the shared ancestors are subsampled),
// up to 256 / 512 / 1024 / 2048 / 4096 / 8192 points.  Classes 6-10: the
// general subtree, up to 256 ... 4096 points.
constexpr int WC_CLASSES = 11;
constexpr int WC_GENERAL = 6;

constexpr int MS_BLOCK = 256;                // multisplit block (4 waves)
constexpr int MS_ITEMS = 8;                  // elements per thread
constexpr uint32_t MS_TILE = MS_BLOCK * MS_ITEMS;  // 2048
// Segmented splits (many small buckets per segment) take longer tiles, so a
// bucket's run inside a tile is long enough to write whole lines.
constexpr int MS_SEG_ITEMS = 12;
constexpr uint32_t MS_SEG_TILE = MS_BLOCK * MS_SEG_ITEMS;  // 3072
constexpr uint32_t MS_MAX_BINS = 2048;       // buckets a tile can hold (segments)
constexpr uint32_t MS_ONE_PASS_BINS = 1024;  // beyond this, sort by digits (keeps the count matrix small)
constexpr uint32_t MS_DIGIT_BITS = 10;

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr uint32_t SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Values the device derives from the bounding box (written by k_setup).
struct DevBox {
    float lo[3];
    float hi[3];
    float size;
    float scale;
    uint32_t nonfinite;  // some coordinate is NaN or infinite
    uint32_t pad;
    unsigned long long n_outside;
};

// Device counters of a build, read back by the host (with the box 256 bytes
// after them).
struct Ctrs {
    uint32_t num_chunks;
    uint32_t num_wc;
    uint32_t num_big;
    uint32_t max_big;
    uint32_t num_nodes;
    uint32_t preview_count;
    uint32_t oversized;
    uint32_t internal_error;
    uint32_t wc_flags[2];      // [0] a work chunk spans several chunks, [1] a chunk holds too many
    uint32_t cls_cnt[WC_CLASSES];   // work chunks per LDS size class
    uint32_t np_max;                // points of the largest node
    uint32_t np_lists[6];           // node_points: tile lists of four sizes, merge jobs, copies
    uint32_t np_general;            // work chunks with own nodes below their root
    uint32_t wc_over;               // a work chunk holds more than WC_CAP points (one finest cell)
    uint32_t lists_pre[WC_CLASSES + 1];   // work chunks per subsample list (and the global-memory path)
};
static_assert(sizeof(Ctrs) <= 256, "the box follows the counters 256 bytes later");

// Offsets of level l in a pyramid array holding levels 0..g back to back.
__host__ __device__ inline uint64_t pyr_off(int l) { return ((1ull << (3 * l)) - 1ull) / 7ull; }

// Optional bracket around selected kernel launches (event timing).
struct LaunchTimer {
    virtual void begin(hipStream_t st) = 0;
    virtual void end(hipStream_t st) = 0;
    virtual ~LaunchTimer() {}
};

// ---- launchers (fpo_kernels.hip) -------------------------------------------
// Fill kernel (in place of hipMemsetAsync, which costs far more host time per
// call and is not safe to record in a graph).
void launch_fill_u32(uint32_t *p, uint32_t v, uint64_t words, hipStream_t st);
// Up to four fills in one launch (null or empty ones skipped).
struct FillSpec {
    uint32_t *p = nullptr;
    uint32_t v = 0;
    uint64_t words = 0;
};
void launch_fill_many(const FillSpec (&f)[4], hipStream_t st);
// Bounding box: per-block partials (8 words each: 3 min, 3 max in an
// order-preserving integer encoding, a non-finite flag), reduced by k_setup.
constexpr uint32_t BBOX_MAX_BLOCKS = 2048;
uint32_t bbox_blocks(uint64_t n);
// zero (or null): zero_words words cleared by the same launch.
void launch_bbox(const float *x, const float *y, const float *z, uint64_t n, uint32_t *part, hipStream_t st,
                 uint32_t *zero = nullptr, uint64_t zero_words = 0);
// flag_only: only the non-finite flag is reduced (the box was set before).
void launch_setup(DevBox *box, const uint32_t *part, uint32_t nparts, int given, const float *lo, const float *hi,
                  int flag_only, hipStream_t st);
// base = original index of x[0]; cellmin (grid preview only, else nullptr)
// receives the least H64 of each count-grid cell.
// variant: the pass's block and LDS-table shape, 0..QZ_VARIANTS-1 (autotuned;
// every variant gives the same codes and counts).
// Variant QZ_BINNED is the binned form (launch_quantize_binned), for device
// input without the grid preview when quantize_binned_ok(n, g).
constexpr int QZ_VARIANTS = 5;
constexpr int QZ_BINNED = 4;
constexpr uint64_t QB_MIN_POINTS = 1ull << 16;
void launch_quantize(const float *x, const float *y, const float *z, uint64_t n, const DevBox *box,
                     int g, int given, uint64_t *code, uint32_t *fine_cnt, DevBox *box_rw,
                     uint64_t base, uint64_t *cellmin, hipStream_t st, int variant);
// G >= 8 and at least 2^16 points, and at least 256 points per bin (64 bins
// up to G = 128, 512 at G = 256, 4096 at G = 512).
bool quantize_binned_ok(uint64_t n, int g);
// temp: quantize_binned_temp_bytes(g) bytes; cells: 2 B per point; scan_temp:
// scan temporaries for 2^(3g - 15) * 256 values.  Writes every cell of the
// count grid (no clearing needed) and the codes.
size_t quantize_binned_temp_bytes(int g);
void launch_quantize_binned(const float *x, const float *y, const float *z, uint64_t n, const DevBox *box, int g,
                            int given, uint64_t *code, uint32_t *fine_cnt, DevBox *box_rw, void *temp,
                            uint16_t *cells, void *scan_temp, hipStream_t st);
// exp_out (or null): the finest level's row-major export, written by the
// launch that reads it.
void launch_pyramid(uint32_t *pyr, int g, uint32_t *exp_out, hipStream_t st);
void launch_grid_export(const uint32_t *fine_morton, int g, uint32_t *rowmajor, hipStream_t st);
constexpr int FR_BLOCK = 256;   // parents per tile of a frontier launch

// The chunk cut and the work-chunk cut (entries = maximal nodes at or below a
// threshold, oversized finest cells), found top-down over the heavy nodes.
// One per cut; the host sizes every list from n (see cut_plan in fpo_api.hip).
struct CutArgs {
    uint32_t thresh;             // light: count <= thresh
    int lmin;                    // entries only at levels >= lmin
    int lam;                     // finest level (log2 G)
    int lt;                      // level of the coarse index (min(lam, 7))
    uint64_t *open[2];           // heavy nodes of a level (ping-pong by level parity), open_cap each
    uint32_t open_cap;
    uint32_t *n_open;            // [MAXD] heavy nodes per level
    uint64_t *ent;               // entry keys; level l's at ent + ent_off[l], capacity ent_off[l + 1] - ent_off[l]
    uint64_t ent_off[MAXD + 1];
    uint32_t *n_ent;             // [MAXD] entries per level
    unsigned long long *status;  // chained-scan words; level l's tiles at status + st_off[l]
    uint64_t st_off[MAXD + 1];
    uint32_t *tile_ctr;          // [MAXD]
    uint32_t *over;              // set when an entry holds more than thresh points (oversized)
    uint32_t *err;               // set when a list exceeds its capacity
    uint32_t *num_out;           // number of entries
    uint32_t max_out;            // capacity of the outputs below
    uint8_t *out_level;          // entries in Morton pre-order: level, key, count, first finest cell
    uint64_t *out_key;
    uint32_t *out_count;
    uint64_t *out_start;
    uint32_t *idx;               // 8^lt + 1 words: entries starting before each coarse cell
};
// cut init, one frontier launch per level, rank, coarse index
void launch_cut(const uint32_t *pyr, const CutArgs &chunks, const CutArgs &wcs, hipStream_t st);

// Entry containing finest cell m (a cell holding points): the last entry
// starting at or before m, searched among those starting inside m's coarse
// cell (indices idx[c] .. idx[c + 1]) and else the one before them.
struct CutIndex {
    const uint64_t *starts;      // first finest cell of every entry, ascending
    const uint32_t *idx;         // CutArgs::idx
    int tsh;                     // 3 * (lam - lt)
};
__device__ __forceinline__ uint32_t cut_find(const CutIndex &X, uint64_t m)
{
    if (X.tsh == 0) {   // the index is at the finest level: entries starting at or before m
        const uint32_t v = X.idx[m + 1];
        return v ? v - 1 : 0u;
    }
    const uint64_t c = m >> X.tsh;
    uint32_t lo = X.idx[c], hi = X.idx[c + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (X.starts[mid] <= m) lo = mid + 1; else hi = mid;
    }
    return lo ? lo - 1 : 0u;
}

void launch_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, hipStream_t st);
// Two independent exclusive scans of at most SCAN_PAIR_MAX values each in one
// launch (one block each); out0_wide (optional) gets the first as u64.
constexpr uint64_t SCAN_PAIR_MAX = 16384;
void scan_exclusive_pair(const uint32_t *in0, uint32_t *out0, uint64_t *out0_wide, uint64_t n0, const uint32_t *in1,
                         uint32_t *out1, uint64_t n1, hipStream_t st);
// Device-wide exclusive scan of n u32 values; *total (device) gets the sum.
size_t scan_temp_bytes(uint64_t n);
void scan_exclusive(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total, void *temp,
                    hipStream_t st);

// Stable multisplit (counting sort) by u32 keys.
struct MsInput {
    const uint32_t *keys = nullptr;    // explicit keys, or
    const uint64_t *code = nullptr;    // key = the cut entry holding cell code[e] >> code_shift
    CutIndex cut{};
    int code_shift = 0;
    const uint32_t *vals = nullptr;    // values (null: the input position)
    const uint64_t *pay = nullptr;     // optional payload carried along
    // Known start of every bucket in the output (the exclusive scan of the
    // bucket sizes): a split of few tiles then runs in one pass, each tile
    // finding its offsets by a look-back over its predecessors' per-bucket
    // counts instead of a counting pass and a scan.  err receives 1 if a
    // look-back ever gives up waiting (never expected).
    const uint64_t *bucket_begin = nullptr;
    uint32_t *err = nullptr;
};
struct MsOutput {
    uint32_t *vals = nullptr;          // values in sorted order (optional)
    uint32_t *keys = nullptr;          // keys in sorted order (optional)
    uint32_t *src = nullptr;           // input position of every output (optional, one pass only)
    uint64_t *pay = nullptr;           // payload in sorted order (optional)
    // optional, with pay: the entry of a second cut holding each output's
    // payload cell (pay >> cut2_shift), in sorted order (last pass only)
    uint32_t *cut2_keys = nullptr;
    CutIndex cut2{};
    int cut2_shift = 0;
};
// Segments: contiguous input ranges, each sorted into its own contiguous
// bucket range [b0, b0 + nb) (nb <= MS_MAX_BINS); output positions are global.
struct MsSegments {
    uint32_t nseg = 0;
    const uint32_t *begin = nullptr, *len = nullptr, *b0 = nullptr, *nb = nullptr;
    uint64_t max_cells = 0;            // bound on sum(nb * tiles)
};
struct MsArgs {
    uint64_t n;
    const uint32_t *keys;
    const uint64_t *code;
    CutIndex cut;
    int code_shift;
    const uint32_t *vals;
    const uint64_t *pay;
    uint32_t shift, dbits, nbins, tiles;
    uint32_t *counts, *offsets;
    uint32_t *vals_out, *keys_out, *src_out;
    uint64_t *pay_out;
    uint32_t nseg;
    const uint32_t *seg_begin, *seg_len, *seg_b0, *seg_nb, *seg_mat, *seg_tile_first, *seg_total_tiles;
    // one-pass split: bucket starts, per-(tile, bucket) status words, the
    // tile ticket counter, the error flag
    const uint64_t *bucket_begin;
    unsigned long long *status;
    uint32_t *tile_ctr, *err;
    // MsOutput::cut2_keys
    uint32_t *cut2_out;
    CutIndex cut2;
    int cut2_shift;
};
size_t multisplit_temp_bytes(uint64_t n, uint32_t nbins);
size_t multisplit_temp_bound(uint64_t n, uint64_t max_bins);   // for any nbins <= max_bins
// scatter_timer (optional) brackets every scatter-kernel launch.
void multisplit(const MsInput &in, uint64_t n, uint32_t nbins, const MsOutput &out, void *temp, hipStream_t st,
                LaunchTimer *scatter_timer = nullptr);
size_t multisplit_seg_temp_bytes(uint64_t n, uint32_t nseg, uint64_t max_cells);
void multisplit_segmented(const MsInput &in, uint64_t n, const MsSegments &sg, uint64_t max_tiles,
                          const MsOutput &out, void *temp, hipStream_t st);
// Exclusive scan whose length is read on the device (*n_dev <= n_max).
void scan_exclusive_dev(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint64_t n_max, void *temp,
                        hipStream_t st);

// Subsample step.
struct WcArgs {
    uint32_t num_wc;
    const uint32_t *wc_begin;    // position of the work chunk's first point in work-chunk order
    const uint32_t *wc_count;
    const uint8_t *wc_level;
    const uint64_t *wc_key;
    const uint64_t *wc_start;    // first lattice cell (level lam_w) of each work chunk
    const uint32_t *wc_orig;     // original index of every work-chunk position
    const uint32_t *perm;        // original index per perm position
    const uint8_t *wc_nested;    // 1 when the work chunk lies inside one chunk
    const uint64_t *wc_code;     // Morton code per position
    uint8_t *t;                  // tentative depth per position
    uint32_t *fr;                // local node rank per position
    uint32_t *alive;             // [MAXD][num_wc] points reaching each shared ancestor from a work
                                 // chunk (row lw: reaching its own root); after k_decide, rows d <= cut
                                 // hold the ancestor's whole reaching count
    const uint32_t *alive_scan;  // exclusive scan of alive over the flattened matrix (MAXD * num_wc + 1)
    uint32_t *kd;                // [num_wc][MAXD] local node count per depth
    uint32_t *loff;              // [num_wc][MAXD] offset of a depth's local nodes
    uint64_t *lnode_key;         // local node keys, per work chunk region
    uint8_t *lnode_mask;         // local node child masks
    uint8_t *cut;                // per work chunk: first depth whose shared node is a leaf (or lw)
    // work chunks for the global-memory path (more than WC_CAP points, or
    // cell keys too long for the LDS table), listed on the device
    uint32_t *big_list;
    uint32_t *num_big_dev;
    // work chunks of the LDS path by size class (WC_CLASSES lists of up to
    // num_wc entries each) and their counts
    uint32_t *cls_list;
    uint32_t *cls_cnt;
    uint32_t *big_nr;            // per position scratch
    uint32_t *big_node;          // 3 words of node scratch per position
    uint64_t *big_hkey;          // 4 table slots per position
    uint32_t *big_hval;
    int lam_w;                   // deepest work-chunk level (g)
    int d0;                      // shared depths below it are decided globally: max(0, g - s)
    int s;
    uint32_t L;
    int dmax;
};
// Shared depths d < d0 over all points (t filled with 0xff before): winners
// get t = d, and the reaching-count rows of those depths are written.  Two
// cell tables alternate over the depths (the pass of depth d reads the table
// of depth d - 1): depth d uses global_depth_table(gtab, gtab2, d0, d), so
// gtab (4 * 8^(d0 - 1 + s) bytes) serves d0 - 1, d0 - 3, ... and gtab2
// (4 * 8^(d0 - 2 + s) bytes, only when d0 >= 2) serves d0 - 2, d0 - 4, ...
// first_filled: the table of depth 0 was cleared to all ones already.
uint32_t *global_depth_table(uint32_t *gtab, uint32_t *gtab2, int d0, int d);
void launch_global_depths(const WcArgs &a, uint64_t n, uint32_t *gtab, uint32_t *gtab2, hipStream_t st,
                          bool first_filled = false);
// lists[c] (host): number of work chunks in list c, 0 .. WC_CLASSES (the last:
// the global-memory path), as counted by the cut; empty lists are skipped.
void launch_subsample_small(const WcArgs &a, const uint32_t *lists, hipStream_t st);
void launch_subsample_big(const WcArgs &a, hipStream_t st);
void launch_decide(const WcArgs &a, hipStream_t st);
void launch_node_counts(const WcArgs &a, uint32_t *owned, hipStream_t st);
// node_points, sizes first: cnt_dw[d * W + w] = points of work chunk w in the
// shared node of depth d (from the reaching counts), S its exclusive scan
// (MAXD * W + 1 entries), cnt_node[id] = points of every node; per (d, w) the
// node whose range one offset places w's depth-d points in (pnode, all ones
// for none) and that offset (in place of cnt_dw); work chunks with own nodes
// below their root in glist (*gcount, zeroed before).  *maxc = the largest
// node (zeroed before).
// single[id] = 1 for every node filled by one piece in work-chunk order
// (one work chunk contributes to it, not through the fill counters), so its
// placed range already ascends; 0 for the others.
void launch_np_counts(const WcArgs &a, const uint32_t *node_base, uint32_t *cnt_dw, uint32_t *S, uint32_t *cnt_node,
                      uint32_t *pnode, uint32_t *glist, uint32_t *gcount, uint32_t *maxc, uint8_t *single,
                      void *scan_temp, hipStream_t st);
constexpr uint32_t NP_MAX_NODES = 0x7fffffffu;   // the tile lists flag groups of nodes in bit 31
struct NpLists {
    uint32_t *c0, *c1, *c2;   // tiles of up to 1024, 4096, 8192 values: a node, or a group of small nodes
    uint64_t *c3;             // parts of up to 16384 values of longer nodes
    uint64_t *jobs;           // merge jobs of the nodes above 16384 values
    uint64_t *cp;             // parts of up to 16384 values of nodes (or groups) already in order: copied
    const uint8_t *single;    // per node: 1 when one piece in work-chunk order fills it (already ascending)
    uint32_t *counts;         // 6 list lengths (c0..c3, jobs, cp), zeroed before
};
struct NpWork {
    uint32_t *nb;         // node begins (num_nodes + 1)
    uint32_t *tmp;        // n: points placed in node order; then the merges' other buffer
    uint32_t *fill;       // per node id: fill counters of own nodes below subdivided roots
    bool general;         // some work chunk has such nodes (fill is zeroed then)
    uint32_t *err;        // set when a point was never placed
    uint32_t *out;        // n: node_points
    NpLists lists;
    void *scan_temp;
    LaunchTimer *place_timer, *sort_timer;   // the placement; the sorts and merges
};
// Then the points of every node in ascending original index, at the begins nb.
void launch_np_points(const WcArgs &a, const uint32_t *node_base, const uint32_t *pnode, const uint32_t *poff,
                      const uint32_t *cnt_node, uint32_t num_nodes, uint32_t max_count, uint64_t n, const NpWork &w,
                      hipStream_t st);
uint64_t np_list_entries(uint64_t n, int cls);   // entries of tile list cls (0..3) for n points
uint64_t np_job_entries(uint64_t n);
uint64_t np_copy_entries(uint64_t n);
// Chunk of every work chunk (the chunk holding its first occupied finest
// cell), per chunk the range of its work chunks [b0, b0 + nb), per work chunk
// whether it lies inside that chunk; flags[0] is set when some work chunk
// spans several chunks, flags[1] when a chunk holds more than MS_MAX_BINS work
// chunks.  Counts are read on the device; grids cover max_wc / max_chunks.
void launch_wc_chunks(const uint32_t *num_wc_dev, uint64_t max_wc, const uint64_t *wc_key, const uint8_t *wc_level,
                      int g, const uint32_t *pyr, const CutIndex &chunks, const uint8_t *chunk_level,
                      const uint32_t *num_chunks_dev, uint64_t max_chunks, uint32_t *wc_chunk, uint32_t *seg_b0,
                      uint32_t *seg_nb, uint8_t *wc_nested, uint32_t *flags, const uint32_t *wc_count, uint32_t L,
                      int s, uint32_t *class_counts, hipStream_t st);
void launch_node_fill(const WcArgs &a, const uint32_t *node_base, uint8_t *depth, uint64_t *key,
                      uint8_t *mask, hipStream_t st);

// *out += fingerprint of bytes [p, p + bytes) (order-independent sum; out
// zeroed by the caller): equal for equal ranges.
void launch_fingerprint(const void *p, uint64_t bytes, uint64_t salt, uint64_t *out, hipStream_t st);

// Node-ordered gather: out_xyz[3k + a] = coord_a[idx[k]], colour bytes alike.
void launch_gather_points(const uint32_t *idx, uint64_t n, const float *x, const float *y, const float *z,
                          const uint8_t *color, uint32_t stride, float *out_xyz, uint8_t *out_color, hipStream_t st);

// Preview.
enum { PV_HASH = 0, PV_STRIDE = 1, PV_GRID = 2 };
struct PreviewArgs {
    uint64_t n;
    uint64_t m;                  // modulus (hash, stride)
    int mode;
    const uint64_t *code;        // grid: Morton code per original index
    const uint64_t *cellmin;     // grid: least H64 per count-grid cell
    int shift;                   // grid: code >> shift = cell
    uint32_t *zero = nullptr;    // words cleared by the first block (the build's counters), or null
    uint32_t zero_words = 0;
};
// bits (ceil(n / 32) words) = the predicate of every index
// tile_counts (or null): the kept indices of every compaction tile (what
// launch_bits_count gives), counted by the same launch.
void launch_preview_bits(const PreviewArgs &p, uint32_t *bits, uint32_t *tile_counts, hipStream_t st);
// Grid preview: the quantise pass leaves the least H64 of every count-grid
// cell in cellmin (G^3 entries, all ones where empty); the picks follow either
// from the inverse hash (into bits, zeroed before) or from the predicate
// H64(i) == cellmin[cell(i)] (PV_GRID).  The map is then compacted in order.
void launch_grid_picks(const uint64_t *cellmin, uint64_t cells, uint64_t n, uint32_t *bits, hipStream_t st);
uint64_t bits_tiles(uint64_t n);
void launch_bits_count(const uint32_t *bits, uint64_t n, uint32_t *tile_counts, hipStream_t st);
void launch_bits_write(const uint32_t *bits, uint64_t n, const uint32_t *tile_offsets, uint32_t *out,
                       hipStream_t st);

// ---- single-workgroup builds of small clouds ----
// A cloud whose root is its only chunk (n <= C), with at most SB_MAX_N
// points, S <= SB_MAX_S, G <= SB_MAX_G and at most SB_MAX_INNER nodes above L
// points per level (there are at most n / (L + 1) of them), is built whole by
// one workgroup: box, quantise and count, the chunk, the preview, and the tree
// level by level with a node's subsample grid as a table in LDS.  Up to
// SB_GROUP clouds go in one launch, one workgroup each.
constexpr uint32_t SB_MAX_N = (1u << 18) - 1;   // a position inside a node fits 18 bits
constexpr uint32_t SB_MAX_S = 32;               // the S^3 table: 128 KB of LDS
constexpr uint32_t SB_MAX_G = 64;               // the count grid: at most 1 MB to clear
constexpr uint32_t SB_MAX_INNER = 64;
constexpr uint32_t SB_GROUP = 32;

struct SmallDesc {
    const float *x, *y, *z;
    char *ws;                  // the cloud's workspace, laid out by small_layout
    uint32_t n, g, s, L, M;    // points, log2 G, log2 S, leaf capacity, preview modulus
    uint32_t given, stride;    // box given; stride preview (else the hash preview)
    float glo[3], ghi[3];      // the given box
};
struct SmallGroup {
    SmallDesc d[SB_GROUP];
};

// Byte offsets of a single-workgroup build's arrays in its workspace (the
// counters first, the box 256 bytes after them).
struct SmallLayout {
    uint64_t ctrs, box, grid, c_level, c_key, c_count, c_begin, perm;
    uint64_t n_depth, n_key, n_mask, n_begin, n_count, n_points, pv_index;
    uint64_t code, ia, ib, ca, cb, total;
};
__host__ __device__ inline uint64_t sb_take(uint64_t &at, uint64_t bytes)
{
    const uint64_t r = at;
    at += bytes ? (bytes + 255) & ~(uint64_t)255 : 256;
    return r;
}
__host__ __device__ inline SmallLayout small_layout(uint64_t n, int g)
{
    SmallLayout o{};
    uint64_t at = 0;
    o.ctrs = sb_take(at, 256);
    o.box = sb_take(at, sizeof(DevBox));
    o.grid = sb_take(at, 4ull << (3 * g));
    o.c_level = sb_take(at, 1);
    o.c_key = sb_take(at, 8);
    o.c_count = sb_take(at, 4);
    o.c_begin = sb_take(at, 8);
    o.perm = sb_take(at, 4 * n);
    o.n_depth = sb_take(at, n);
    o.n_key = sb_take(at, 8 * n);
    o.n_mask = sb_take(at, n);
    o.n_begin = sb_take(at, 8 * n);
    o.n_count = sb_take(at, 4 * n);
    o.n_points = sb_take(at, 4 * n);
    o.pv_index = sb_take(at, 4 * n);
    o.code = sb_take(at, 8 * n);
    o.ia = sb_take(at, 4 * n);
    o.ib = sb_take(at, 4 * n);
    o.ca = sb_take(at, 8 * n);
    o.cb = sb_take(at, 8 * n);
    o.total = at;
    return o;
}
// One workgroup per cloud: g.d[0 .. count).
void launch_small_build(const SmallGroup &g, uint32_t count, hipStream_t st);

}  // namespace fpo
