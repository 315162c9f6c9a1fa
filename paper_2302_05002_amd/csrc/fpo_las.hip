// LAS fixed-record decode: AoS point records with int32 coordinates and the
// header's scale and offset become float32 x, y, z arrays (and uint16 R, G, B).
// Section "File Importing" of the paper (clouds arrive as LAS files); record
// and header layouts from the ASPRS LAS specification, versions 1.0-1.4.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "fpo_host.h"

namespace {

using fpo::fail;

// minimum record length of point data record formats 0-10, and the byte
// offset of R, G, B in them (0: the format has no colour)
constexpr uint16_t kMinLength[11] = {20, 28, 26, 34, 57, 63, 30, 36, 38, 59, 67};
constexpr uint16_t kRgbOffset[11] = {0, 0, 20, 28, 0, 28, 0, 30, 30, 0, 30};

struct LasArgs {
    const uint8_t *rec;
    uint64_t n;
    uint32_t R;           // record length
    uint32_t per_block;   // records per block
    double scale[3], offset[3], origin[3];
    float *x, *y, *z;
    uint16_t *rgb;        // nullptr: no colour
    uint32_t rgb_off;
};

__device__ __forceinline__ float decode1(int32_t X, double scale, double offset, double origin)
{
    return __double2float_rn(__dsub_rn(__dadd_rn(__dmul_rn((double)X, scale), offset), origin));
}

// ---- staged decode --------------------------------------------------------------------
// A block decodes a contiguous run of records.  Its byte range is copied into
// LDS with aligned 16-byte loads (the bytes before the first and after the
// last 16-byte boundary inside the range one by one, so nothing outside the
// records is read), then every thread reads its records' fields from LDS and
// writes x, y, z coalesced.
constexpr int LD_BLOCK = 256;
constexpr uint32_t LD_BYTES = 32768;

__device__ __forceinline__ uint32_t lds_u32(const uint32_t *w, uint32_t o)
{
    const uint32_t k = o >> 2, s = (o & 3u) * 8u;
    const uint32_t lo = w[k];
    return s ? (lo >> s) | (w[k + 1] << (32u - s)) : lo;
}

__global__ __launch_bounds__(LD_BLOCK) void k_las_decode(LasArgs a)
{
    __shared__ uint4 buf[LD_BYTES / 16 + 1];   // one spare line for the word after the last byte
    uint8_t *lb = reinterpret_cast<uint8_t *>(buf);
    const uint64_t p0 = (uint64_t)blockIdx.x * a.per_block;
    const uint64_t p1 = p0 + a.per_block < a.n ? p0 + a.per_block : a.n;
    const uint64_t base = reinterpret_cast<uintptr_t>(a.rec);
    const uint64_t b0 = base + p0 * a.R, b1 = base + p1 * a.R;
    const uint64_t a0 = b0 & ~15ull;
    const uint64_t c0 = (b0 + 15) & ~15ull;   // first 16-byte boundary at or after b0
    const uint64_t c1 = b1 & ~15ull;          // last one at or before b1
    const uint32_t t = threadIdx.x;
    for (uint64_t q = c0 + 16ull * t; q + 16 <= c1; q += 16ull * LD_BLOCK)
        *reinterpret_cast<uint4 *>(lb + (q - a0)) = *reinterpret_cast<const uint4 *>(q);
    if (t < 16) {
        const uint64_t q = b0 + t;   // head: [b0, min(c0, b1))
        if (q < c0 && q < b1) lb[q - a0] = *reinterpret_cast<const uint8_t *>(q);
    } else if (t < 32) {
        const uint64_t q = (c1 > c0 ? c1 : c0) + (t - 16);   // tail: [max(c1, c0), b1)
        if (q < b1) lb[q - a0] = *reinterpret_cast<const uint8_t *>(q);
    }
    __syncthreads();
    const uint32_t *w = reinterpret_cast<const uint32_t *>(buf);
    const uint32_t first = (uint32_t)(b0 - a0);
    for (uint64_t p = p0 + t; p < p1; p += LD_BLOCK) {
        const uint32_t o = first + (uint32_t)(p - p0) * a.R;
        a.x[p] = decode1((int32_t)lds_u32(w, o), a.scale[0], a.offset[0], a.origin[0]);
        a.y[p] = decode1((int32_t)lds_u32(w, o + 4), a.scale[1], a.offset[1], a.origin[1]);
        a.z[p] = decode1((int32_t)lds_u32(w, o + 8), a.scale[2], a.offset[2], a.origin[2]);
        if (a.rgb) {
            const uint32_t rg = lds_u32(w, o + a.rgb_off), b = lds_u32(w, o + a.rgb_off + 4);
            a.rgb[3 * p] = (uint16_t)(rg & 0xffffu);
            a.rgb[3 * p + 1] = (uint16_t)(rg >> 16);
            a.rgb[3 * p + 2] = (uint16_t)(b & 0xffffu);
        }
    }
}

// Records too long for a useful LDS run (more than LD_BYTES / 64 bytes): each
// thread reads its record's fields byte by byte from global memory.
__device__ __forceinline__ uint32_t ld_bytes32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

__global__ __launch_bounds__(LD_BLOCK) void k_las_decode_direct(LasArgs a)
{
    for (uint64_t p = (uint64_t)blockIdx.x * LD_BLOCK + threadIdx.x; p < a.n; p += (uint64_t)gridDim.x * LD_BLOCK) {
        const uint8_t *r = a.rec + p * a.R;
        a.x[p] = decode1((int32_t)ld_bytes32(r), a.scale[0], a.offset[0], a.origin[0]);
        a.y[p] = decode1((int32_t)ld_bytes32(r + 4), a.scale[1], a.offset[1], a.origin[1]);
        a.z[p] = decode1((int32_t)ld_bytes32(r + 8), a.scale[2], a.offset[2], a.origin[2]);
        if (a.rgb) {
            const uint8_t *c = r + a.rgb_off;
            a.rgb[3 * p] = (uint16_t)(c[0] | (c[1] << 8));
            a.rgb[3 * p + 1] = (uint16_t)(c[2] | (c[3] << 8));
            a.rgb[3 * p + 2] = (uint16_t)(c[4] | (c[5] << 8));
        }
    }
}

template <typename T> T get(const uint8_t *b, size_t off)
{
    T v;
    memcpy(&v, b + off, sizeof(T));   // little-endian host
    return v;
}

fpo_status check_header(const fpo_las_header *h)
{
    if (!h) return fail(FPO_ERR_INVALID_ARG, "header is NULL");
    if (h->point_format > 10) return fail(FPO_ERR_INVALID_ARG, "point format %u is not 0..10", h->point_format);
    if (h->record_length < kMinLength[h->point_format])
        return fail(FPO_ERR_INVALID_ARG, "record length %u is below format %u's %u bytes", h->record_length,
                    h->point_format, kMinLength[h->point_format]);
    if (h->has_rgb != (kRgbOffset[h->point_format] != 0) || (h->has_rgb && h->rgb_offset != kRgbOffset[h->point_format]))
        return fail(FPO_ERR_INVALID_ARG, "colour fields do not match point format %u", h->point_format);
    for (int a = 0; a < 3; ++a)
        if (!isfinite(h->scale[a]) || !isfinite(h->offset[a]))
            return fail(FPO_ERR_INVALID_ARG, "scale and offset must be finite");
    return FPO_OK;
}

}  // namespace

extern "C" {

fpo_status fpo_las_parse_header(const void *bytes, uint64_t len, fpo_las_header *out)
{
    if (!bytes || !out) return fail(FPO_ERR_INVALID_ARG, "NULL bytes or output");
    const uint8_t *b = static_cast<const uint8_t *>(bytes);
    if (len < 227 || memcmp(b, "LASF", 4) != 0) return fail(FPO_ERR_INVALID_ARG, "not a LAS public header block");
    fpo_las_header h;
    memset(&h, 0, sizeof(h));
    h.version_major = b[24];
    h.version_minor = b[25];
    const uint16_t header_size = get<uint16_t>(b, 94);
    const bool v14 = h.version_major > 1 || (h.version_major == 1 && h.version_minor >= 4);
    if (header_size < (v14 ? 375 : 227) || (v14 && len < 375))
        return fail(FPO_ERR_INVALID_ARG, "header of %u bytes is too short for LAS %u.%u", header_size, h.version_major,
                    h.version_minor);
    h.offset_to_points = get<uint32_t>(b, 96);
    const uint8_t fmt = b[104];
    if (fmt & 0x80) return fail(FPO_ERR_INVALID_ARG, "compressed (LAZ) point records are not supported");
    h.point_format = fmt;
    h.record_length = get<uint16_t>(b, 105);
    h.num_points = v14 ? get<uint64_t>(b, 247) : get<uint32_t>(b, 107);
    for (int a = 0; a < 3; ++a) {
        h.scale[a] = get<double>(b, 131 + 8 * a);
        h.offset[a] = get<double>(b, 155 + 8 * a);
        h.max[a] = get<double>(b, 179 + 16 * a);   // max x, min x, max y, min y, max z, min z
        h.min[a] = get<double>(b, 187 + 16 * a);
    }
    if (fmt <= 10) {
        h.has_rgb = kRgbOffset[fmt] != 0;
        h.rgb_offset = kRgbOffset[fmt];
    }
    fpo_status s = check_header(&h);
    if (s != FPO_OK) return s;
    if (h.offset_to_points < header_size)
        return fail(FPO_ERR_INVALID_ARG, "point records start at %u, inside the %u-byte header", h.offset_to_points,
                    header_size);
    *out = h;
    return FPO_OK;
}

fpo_status fpo_las_header_box(const fpo_las_header *h, const double origin[3], float lo[3], float hi[3])
{
    if (!h || !origin || !lo || !hi) return fail(FPO_ERR_INVALID_ARG, "NULL argument");
    for (int a = 0; a < 3; ++a) {
        const double l = h->min[a] - origin[a], u = h->max[a] - origin[a];
        lo[a] = (float)l;
        hi[a] = (float)u;
    }
    return FPO_OK;
}

fpo_status fpo_las_decode(fpo_context *ctx, const fpo_las_header *h, const void *records, uint64_t records_bytes,
                          uint64_t n, const double origin[3], float *x, float *y, float *z, uint16_t *rgb,
                          void *hip_stream)
{
    if (!ctx || !origin) return fail(FPO_ERR_INVALID_ARG, "NULL context or origin");
    fpo_status s = check_header(h);
    if (s != FPO_OK) return s;
    if (n > 0xffffffffull) return fail(FPO_ERR_INVALID_ARG, "n = %llu exceeds 2^32 - 1", (unsigned long long)n);
    if (n && (!records || !x || !y || !z)) return fail(FPO_ERR_INVALID_ARG, "NULL records or output");
    if (n * h->record_length > records_bytes)
        return fail(FPO_ERR_INVALID_ARG, "%llu records of %u bytes exceed the %llu bytes given", (unsigned long long)n,
                    h->record_length, (unsigned long long)records_bytes);
    if (rgb && !h->has_rgb) return fail(FPO_ERR_INVALID_ARG, "point format %u has no colour", h->point_format);
    for (int a = 0; a < 3; ++a)
        if (!isfinite(origin[a])) return fail(FPO_ERR_INVALID_ARG, "origin must be finite");
    if (n == 0) return FPO_OK;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(FPO_ERR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream;
    LasArgs a;
    a.rec = static_cast<const uint8_t *>(records);
    a.n = n;
    a.R = h->record_length;
    for (int k = 0; k < 3; ++k) {
        a.scale[k] = h->scale[k];
        a.offset[k] = h->offset[k];
        a.origin[k] = origin[k];
    }
    a.x = x;
    a.y = y;
    a.z = z;
    a.rgb = rgb;
    a.rgb_off = h->rgb_offset;
    // records per block: as many as fit the LDS run (15 bytes of alignment
    // slack), a multiple of 64, at most 16 per thread
    uint32_t per = (LD_BYTES - 16) / a.R;
    per = per > 16u * LD_BLOCK ? 16u * LD_BLOCK : per & ~63u;
    if (per >= 64) {
        a.per_block = per;
        const uint64_t blocks = (n + per - 1) / per;
        hipLaunchKernelGGL(k_las_decode, dim3((uint32_t)blocks), dim3(LD_BLOCK), 0, st, a);
    } else {
        a.per_block = 0;
        uint64_t blocks = (n + LD_BLOCK - 1) / LD_BLOCK;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_las_decode_direct, dim3((uint32_t)blocks), dim3(LD_BLOCK), 0, st, a);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return fail(FPO_ERR_DEVICE, "LAS decode launch: %s", hipGetErrorString(e));
    return FPO_OK;
}

}  // extern "C"
