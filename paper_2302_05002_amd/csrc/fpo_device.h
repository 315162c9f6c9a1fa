// Device helpers shared by the kernels of libfpo (wave64 reductions, the
// Morton bit spread, the lattice quantisation, the box derivation and the
// preview hash), so that every kernel computing one of these values computes
// it the same way.
#pragma once
#include <float.h>

#include "fpo_internal.h"

namespace fpo {

// ---- small helpers ------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Order-preserving map of a float to an unsigned integer (for min/max atomics).
__device__ __forceinline__ uint32_t f2o(float f)
{
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float o2f(uint32_t o)
{
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(b);
}

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if ((int)lane_id() >= o) v += t;
    }
    return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive scan of one value per thread across the block; *total = sum.
// lds must hold BLOCK/64 + 1 words.  Ends with a barrier so lds can be reused.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds, uint32_t *total)
{
    constexpr int W = BLOCK / 64;
    const uint32_t inc = wave_incl_sum(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    if (threadIdx.x < 64) {
        uint32_t x = threadIdx.x < W ? lds[threadIdx.x] : 0u;
        uint32_t xi = wave_incl_sum(x);
        if (threadIdx.x < W) lds[threadIdx.x] = xi - x;
        if (threadIdx.x == W - 1) lds[W] = xi;
    }
    __syncthreads();
    const uint32_t r = lds[w] + inc - v;
    *total = lds[W];
    __syncthreads();
    return r;
}

template <int BLOCK>
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *lds)
{
    constexpr int W = BLOCK / 64;
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) lds[w] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) t += lds[i];
    __syncthreads();
    return t;
}

// Spread the low 21 bits of a so that bit b lands on bit 3b.
__device__ __forceinline__ uint64_t split3(uint32_t a)
{
    uint64_t x = a & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}
__device__ __forceinline__ uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

// Branch-free min/max accumulation of one coordinate in the order-preserving
// integer map; non-finite values are flagged and left out.
__device__ __forceinline__ void bbox_acc(uint32_t &mn, uint32_t &mx, uint32_t &bad, float e)
{
    const bool fin = isfinite(e);
    const uint32_t o = f2o(e);
    mn = min(mn, fin ? o : 0xffffffffu);
    mx = max(mx, fin ? o : 0u);
    bad |= fin ? 0u : 1u;
}

// The box a build works in, from the reduced extremes (mn[a] = f2o of the
// least coordinate of axis a, mx[a] of the largest) or from a given box:
// cube anchored at the box minimum, side = largest extent, scale = 2^21/side
// computed in double and rounded once to float (0 for a zero side).  Sets
// every field but nonfinite.
__device__ inline void box_set(DevBox *box, const uint32_t *mn, const uint32_t *mx, bool given, const float *glo,
                               const float *ghi)
{
    box->n_outside = 0;
    float lo[3], hi[3];
    if (given) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = glo[a];
            hi[a] = ghi[a];
        }
    } else {
        for (int a = 0; a < 3; ++a) {
            // +0.0f turns a -0.0 extreme into +0.0 (the two compare equal, so
            // which one a reduction meets first must not show in the result)
            lo[a] = __fadd_rn(o2f(mn[a]), 0.0f);
            hi[a] = __fadd_rn(o2f(mx[a]), 0.0f);
        }
    }
    float side = 0.0f;
    for (int a = 0; a < 3; ++a) {
        const float ext = __fsub_rn(hi[a], lo[a]);
        if (ext > side) side = ext;
        box->lo[a] = lo[a];
        box->hi[a] = hi[a];
    }
    box->size = side;
    box->scale = side > 0.0f ? (float)(2097152.0 / (double)side) : 0.0f;
}

// Clamped to [0, UMAX] before the conversion (NaN and t <= 0 give 0, t >=
// UMAX gives UMAX), so no branch: on t >= 0 truncation is the floor.
__device__ __forceinline__ uint32_t quantize1(float a, float lo, float scale)
{
    const float t = __fmul_rn(__fsub_rn(a, lo), scale);
    return (uint32_t)fminf(fmaxf(t, 0.0f), 2097151.0f);
}

// ---- preview hash H64 and its inverse ----------------------------------------------
// H64: xorshift-multiply mix with the golden-ratio constant, all mod 2^64.
// Every step is invertible (an odd multiplier has an inverse mod 2^64; x ^= x
// >> k is undone by folding the shifts back in), so H64 is a bijection and the
// index of a hash value is recovered exactly.
constexpr uint64_t H64_PHI = 0x9E3779B97F4A7C15ull;

__host__ __device__ constexpr uint64_t inverse_odd64(uint64_t a)
{
    uint64_t x = a;                      // a * a == 1 mod 8: 3 correct bits
    for (int k = 0; k < 5; ++k) x *= 2 - a * x;   // Newton: correct bits double each step
    return x;
}
constexpr uint64_t H64_PHI_INV = inverse_odd64(H64_PHI);
static_assert(H64_PHI * H64_PHI_INV == 1ull, "inverse of the hash multiplier");

__host__ __device__ constexpr uint64_t h64(uint64_t i)
{
    uint64_t h = i;
    h ^= h >> 31;
    h *= H64_PHI;
    h ^= h >> 29;
    h *= H64_PHI;
    h ^= h >> 32;
    return h;
}

__host__ __device__ constexpr uint64_t h64_inverse(uint64_t h)
{
    h ^= h >> 32;
    h *= H64_PHI_INV;
    h ^= (h >> 29) ^ (h >> 58);
    h *= H64_PHI_INV;
    h ^= (h >> 31) ^ (h >> 62);
    return h;
}
static_assert(h64(1) == 0xd8a77e5280806164ull && h64(5) == 0xe1a5a16ee48bea94ull, "hash known answers");
static_assert(h64_inverse(h64(0)) == 0 && h64_inverse(h64(1)) == 1 && h64_inverse(h64(12345678901ull)) == 12345678901ull &&
                  h64_inverse(h64(~0ull)) == ~0ull && h64_inverse(h64(0xffffffffull)) == 0xffffffffull,
              "hash inverse");

}  // namespace fpo
