/*
 * CPU oracle for the online shallow-octree build and decimated preview
 * (FastPoints, arXiv 2302.05002).  TEST INFRASTRUCTURE ONLY: this code is
 * linked by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  The library under paper_2302_05002_amd/ never includes, links
 * or calls it, and it shares no source with that library.
 *
 * What it computes, step by step, in the paper's order:
 *   Section "Octree Construction" (and the Prior Work paragraph of the same
 *   name): the Potree-2.0-style pipeline -- points are sorted hierarchically
 *   into chunks, each chunk is indexed into a local octree, the local trees
 *   form one global tree.
 *   Section "Immediate Low-Resolution Rendering": a uniform decimation that
 *   visits every point once.
 * The paper gives no constants, rounding rules or orderings for either; the
 * readings used here (21-bit lattice, min-corner cube, lowest index wins a
 * subsample cell, hash-of-index preview, ...) are stated in the comments of
 * fpo_oracle.c at the step they govern.
 */
#ifndef FPO_ORACLE_H
#define FPO_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Preview variants: H64(i) mod M == 0; i mod M == 0; least H64 of every
 * occupied count-grid cell (section "Future Work": a spatially constrained
 * sampler instead of uniform decimation). */
enum { ORACLE_PREVIEW_HASH = 0, ORACLE_PREVIEW_STRIDE = 1, ORACLE_PREVIEW_GRID = 2 };

enum { ORACLE_OK = 0, ORACLE_ERR_INVALID_ARG = 1, ORACLE_ERR_NONFINITE = 2, ORACLE_ERR_OOM = 3 };

typedef struct {
    uint32_t count_grid;           /* G, power of two, 1..512 */
    uint32_t max_points_per_chunk; /* C >= 1 */
    uint32_t subsample_grid;       /* S, power of two, 1..256 */
    uint32_t leaf_capacity;        /* L >= 1 */
    uint32_t preview_modulus;      /* M >= 1 */
    uint32_t bbox_given;           /* 0: computed from the points; 1: use bbox_min/max */
    float bbox_min[3], bbox_max[3];
    uint32_t preview_mode;         /* ORACLE_PREVIEW_HASH, _STRIDE or _GRID */
} oracle_params;

typedef struct {
    int status;
    uint64_t n;
    float bbox_min[3], bbox_max[3];
    float cube_size, scale;
    uint64_t n_outside;            /* points outside a caller-given box (clamped) */
    uint32_t *u;                   /* 3*n fine coordinates, [i*3+axis] */
    uint32_t *count_grid;          /* G^3, row-major [cx][cy][cz] */
    uint32_t num_chunks;
    uint8_t  *chunk_level;
    uint64_t *chunk_key;
    uint32_t *chunk_count;
    uint64_t *chunk_begin;
    uint8_t   chunk_oversized_any;
    uint32_t *perm;                /* n */
    uint32_t num_nodes;
    uint8_t  *node_depth;
    uint64_t *node_key;
    uint8_t  *node_child_mask;
    uint64_t *node_begin;
    uint32_t *node_count;
    uint32_t *node_points;         /* n */
    uint64_t preview_count;
    uint32_t *preview_index;
} oracle_result;

/* Runs the whole path.  x, y, z: n float32 each (host memory, borrowed).
 * Fills *out (arrays malloc'ed here; release with oracle_free).  Returns the
 * status, also stored in out->status. */
int  oracle_build(uint64_t n, const float *x, const float *y, const float *z,
                  const oracle_params *p, oracle_result *out);
void oracle_free(oracle_result *r);

/* The preview hash on its own (used by the known-answer tests). */
uint64_t oracle_h64(uint64_t i);

#ifdef __cplusplus
}
#endif
#endif
