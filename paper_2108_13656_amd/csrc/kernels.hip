// HIP kernels (gfx950) of the colour-temperature decolorization, Eqs. (1)-(6)
// of Ambalathankandy et al. (arXiv 2108.13656, Sec. II-B), and of the global
// tone map on its luminance (Sec. III-B.1, read as a centred sigmoid in the log
// domain, slope normalised by the image's standard deviation).
//
// The work is an elementwise stream bounded by HBM bandwidth, so there is no
// MFMA here: each thread owns whole 48-byte groups of interleaved RGB (16 px
// of u8, 8 of f16, 4 of f32), loads them with three 16-byte loads, decodes
// them in registers, evaluates the luminance in FP32 with the hardware
// square-root / reciprocal-square-root / reciprocal instructions, and writes
// its outputs with 4-16 byte stores.
#include "dc_internal.h"

namespace dc {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ math

__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// L in code units for 8-bit input (R, G, B are integers 0..255 held exactly).
// Eqs. (4)-(6) are multiplied through by sqrt(3) S, with S = R + G + B and
// Q = sqrt(R^2 + G^2 + B^2) = sqrt(3) L_white:
//   sqrt(3) S L_warm = R sqrt(3 beta_R R^2 + 3 (1 - beta_R) G^2) + (G + B) Q =: A
//   sqrt(3) S L_cool = B (sqrt(3) (R + G) + Q)                                =: C
//   L^2 = (beta_k/3 A^2 + (1 - beta_k)/3 C^2) / S^2 =: Y / S^2
//   L   = Y / sqrt(Y S^2),
// so the 1/3 of Eq. (1) and the weights fold into the constants, and one
// reciprocal square root replaces a square root and a division. Squares and
// sums of code values are exact in FP32 (R^2 + G^2 + B^2 <= 195075). The two
// tiny addends (1e-20 on Y, 1e-6 on S^2) make a black pixel give ~1e-7 instead
// of 0 * inf; for any other pixel S^2 >= 1 and Y >= 0.05, so they change L by
// less than 5e-7 relative.
__device__ __forceinline__ float lum_code(float R, float G, float B, Coef k)
{
    const float rr = R * R, gg = G * G;
    const float Q = hw_sqrt(fmaf(B, B, rr + gg));                 // sqrt(3) * Eq. (1)
    const float Lgr3 = hw_sqrt(fmaf(k.cr, rr, k.cg * gg));        // sqrt(3) * Eq. (3)
    const float rg = R + G;
    const float S = rg + B;
    const float A = fmaf(R, Lgr3, (G + B) * Q);                   // sqrt(3) S * Eq. (4)
    const float C = B * fmaf(1.73205080756887729f, rg, Q);        // sqrt(3) S * Eq. (5)
    const float Y = fmaf(k.ck * A, A, fmaf(k.cc, C * C, 1e-20f)); // S^2 * Eq. (6)^2
    return Y * hw_rsq(Y * fmaf(S, S, 1e-6f));
}

// L for linear float input. The pixel is first normalised by S, so every
// intermediate lies in [0, 1] whatever the radiance scale (binary16 spans
// 6e-8 .. 65504), and L = S * L(r, g, b) by degree-1 homogeneity. NaN and
// negative channels read as 0 (max returns the non-NaN operand).
__device__ __forceinline__ float lum_linear(float R, float G, float B, Coef k)
{
    R = fmaxf(R, 0.0f);
    G = fmaxf(G, 0.0f);
    B = fmaxf(B, 0.0f);
    const float S = (R + G) + B;
    const float inv = hw_rcp(fmaxf(S, 1e-30f));
    const float r = R * inv, g = G * inv, b = B * inv;
    const float rr = r * r, gg = g * g;
    const float lw = hw_sqrt(fmaf(b, b, rr + gg) * (1.0f / 3.0f)); // Eq. (1)
    const float lgr = hw_sqrt(fmaf(k.cr, rr, k.cg * gg));           // Eq. (3)
    const float warm = fmaf(r, lgr - lw, lw);                       // Eq. (4)
    const float cool = b * ((1.0f - b) + lw);                       // Eq. (5), L_b = b
    const float X = fmaf(k.ck * warm, warm, k.cc * (cool * cool));  // Eq. (6)^2
    return S * hw_sqrt(X);
}

template <int SRC>
__device__ __forceinline__ float lum(float R, float G, float B, Coef k)
{
    if constexpr (SRC == 0)
        return lum_code(R, G, B, k);
    else
        return lum_linear(R, G, B, k);
}

// ------------------------------------------------------------ memory

// Image pointers come from descriptors in memory, so the compiler cannot tell
// they are global; these casts give global_load/global_store instead of flat.
#define DC_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const DC_GLOBAL T *gp(const void *p)
{
    return (const DC_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ DC_GLOBAL T *gpw(void *p)
{
    return (DC_GLOBAL T *)p;
}

// ------------------------------------------------------------ decode

__device__ __forceinline__ float half_lo(unsigned w)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
}
__device__ __forceinline__ float half_hi(unsigned w)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}

// Channel c of element e of a 48-byte group held as 12 dwords.
template <int SRC>
__device__ __forceinline__ float chan(const unsigned (&w)[12], int e)
{
    if constexpr (SRC == 0) {
        // The empty asm hides that the value is a small integer, so the
        // compiler keeps the arithmetic in FP32 instead of re-deriving squares
        // and sums with integer multiplies and extra conversions.
        float v = (float)((w[e >> 2] >> (8 * (e & 3))) & 0xffu);
        asm("" : "+v"(v));
        return v;
    } else if constexpr (SRC == 1) {
        return (e & 1) ? half_hi(w[e >> 1]) : half_lo(w[e >> 1]);
    } else {
        return __builtin_bit_cast(float, w[e]);
    }
}

template <int SRC>
__device__ __forceinline__ void load_group(const uint8_t *p, unsigned (&w)[12])
{
    const DC_GLOBAL u32x4 *q = gp<u32x4>(p);
    const u32x4 a = q[0], b = q[1], c = q[2];
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    w[8] = c.x; w[9] = c.y; w[10] = c.z; w[11] = c.w;
}

template <int SRC>
__device__ __forceinline__ void load_px(const uint8_t *p, float &R, float &G, float &B)
{
    if constexpr (SRC == 0) {
        const DC_GLOBAL uint8_t *b = gp<uint8_t>(p);
        R = b[0];
        G = b[1];
        B = b[2];
    } else if constexpr (SRC == 1) {
        const DC_GLOBAL _Float16 *h = gp<_Float16>(p);
        R = (float)h[0];
        G = (float)h[1];
        B = (float)h[2];
    } else {
        const DC_GLOBAL float *f = gp<float>(p);
        R = f[0];
        G = f[1];
        B = f[2];
    }
}

// ------------------------------------------------------------ encode

// Output encodings: f32 / f16 store v * fscale; u8 stores floor(v * u8scale +
// 0.5) clamped to [0, 255] (the conversion instruction saturates; the explicit
// min covers HDR values above 1).
__device__ __forceinline__ unsigned u8_code(float v, float u8scale)
{
    return (unsigned)fminf(floorf(fmaf(v, u8scale, 0.5f)), 255.0f);
}

__device__ __forceinline__ unsigned pack_u8x4(float a, float b, float c, float d, float s)
{
    unsigned w = __builtin_amdgcn_cvt_pk_u8_f32(fminf(floorf(fmaf(a, s, 0.5f)), 255.0f), 0, 0u);
    w = __builtin_amdgcn_cvt_pk_u8_f32(fminf(floorf(fmaf(b, s, 0.5f)), 255.0f), 1, w);
    w = __builtin_amdgcn_cvt_pk_u8_f32(fminf(floorf(fmaf(c, s, 0.5f)), 255.0f), 2, w);
    w = __builtin_amdgcn_cvt_pk_u8_f32(fminf(floorf(fmaf(d, s, 0.5f)), 255.0f), 3, w);
    return w;
}

__device__ __forceinline__ unsigned pack_f16x2(float a, float b)
{
    const unsigned short ha = __builtin_bit_cast(unsigned short, (_Float16)a);
    const unsigned short hb = __builtin_bit_cast(unsigned short, (_Float16)b);
    return (unsigned)ha | ((unsigned)hb << 16);
}

// Stores GPX consecutive values at pixel index px of a 1-channel row.
template <int GPX>
__device__ __forceinline__ void store_group(uint8_t *base, int dtype, int64_t px,
                                            const float (&v)[GPX], float fscale, float u8scale)
{
    if (dtype == 0) {
        unsigned w[GPX / 4];
#pragma unroll
        for (int i = 0; i < GPX / 4; ++i)
            w[i] = pack_u8x4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3], u8scale);
        uint8_t *p = base + px;
        if constexpr (GPX == 16)
            *gpw<u32x4>(p) = u32x4{w[0], w[1], w[2], w[3]};
        else if constexpr (GPX == 8)
            *gpw<u32x2>(p) = u32x2{w[0], w[1]};
        else
            *gpw<unsigned>(p) = w[0];
    } else if (dtype == 1) {
        unsigned w[GPX / 2];
#pragma unroll
        for (int i = 0; i < GPX / 2; ++i)
            w[i] = pack_f16x2(v[2 * i] * fscale, v[2 * i + 1] * fscale);
        uint8_t *p = base + 2 * px;
        if constexpr (GPX == 4) {
            *gpw<u32x2>(p) = u32x2{w[0], w[1]};
        } else {
#pragma unroll
            for (int i = 0; i < GPX / 8; ++i)
                gpw<u32x4>(p)[i] =
                    u32x4{w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]};
        }
    } else {
        uint8_t *p = base + 4 * px;
#pragma unroll
        for (int i = 0; i < GPX / 4; ++i)
            gpw<u32x4>(p)[i] =
                u32x4{__builtin_bit_cast(unsigned, v[4 * i] * fscale),
                      __builtin_bit_cast(unsigned, v[4 * i + 1] * fscale),
                      __builtin_bit_cast(unsigned, v[4 * i + 2] * fscale),
                      __builtin_bit_cast(unsigned, v[4 * i + 3] * fscale)};
    }
}

__device__ __forceinline__ void store_px(uint8_t *base, int dtype, int64_t px, float v,
                                         float fscale, float u8scale)
{
    if (dtype == 0)
        gpw<uint8_t>(base)[px] = (uint8_t)u8_code(v, u8scale);
    else if (dtype == 1)
        gpw<_Float16>(base)[px] = (_Float16)(v * fscale);
    else
        gpw<float>(base)[px] = v * fscale;
}

// ------------------------------------------------------------ tile walk

// Addresses of one tile: segment base pointers and the pixel range.
struct TileRef {
    const uint8_t *src;
    uint8_t *dst;
    uint8_t *dst2;
    int64_t px0; // first pixel of the tile within the segment
    int64_t n;   // pixels in the segment
};

__device__ __forceinline__ TileRef tile_ref(const DevImage &im, int64_t tile, int64_t tile_px)
{
    const int64_t seg = tile / im.tiles_per_seg;
    const int64_t ts = tile - seg * im.tiles_per_seg;
    TileRef t;
    t.src = im.src + seg * im.src_seg_stride;
    t.dst = im.dst + seg * im.dst_seg_stride;
    t.dst2 = im.dst2 ? im.dst2 + seg * im.dst2_seg_stride : nullptr;
    t.px0 = ts * tile_px;
    t.n = im.seg_len;
    return t;
}

// Luminance of all pixels a thread owns in one tile (G vector groups of GPX
// pixels, or the same count of single pixels on the scalar walk). lv holds L
// in input units; valid marks pixels inside the segment. Returns the pixel
// index of slot 0 of each group through gpx0.
template <int SRC, int G>
__device__ __forceinline__ void tile_lum(const DevImage &im, const TileRef &t, Coef k,
                                         float (&lv)[G * group_px(SRC)],
                                         bool (&valid)[G * group_px(SRC)])
{
    constexpr int GPX = group_px(SRC);
    constexpr int ES = elem_size(SRC);
    const int tid = threadIdx.x;
    if (im.walk != kWalkScalar) {
        unsigned w[G][12];
        bool full[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t gp = t.px0 + (int64_t)(g * kBlock + tid) * GPX;
            full[g] = gp + GPX <= t.n;
            if (full[g])
                load_group<SRC>(t.src + gp * 3 * ES, w[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t gp = t.px0 + (int64_t)(g * kBlock + tid) * GPX;
            if (full[g]) {
#pragma unroll
                for (int i = 0; i < GPX; ++i) {
                    lv[g * GPX + i] = lum<SRC>(chan<SRC>(w[g], 3 * i), chan<SRC>(w[g], 3 * i + 1),
                                               chan<SRC>(w[g], 3 * i + 2), k);
                    valid[g * GPX + i] = true;
                }
            } else {
#pragma unroll
                for (int i = 0; i < GPX; ++i) {
                    const int64_t p = gp + i;
                    valid[g * GPX + i] = p < t.n;
                    lv[g * GPX + i] = 0.0f;
                    if (p < t.n) {
                        float R, G_, B;
                        load_px<SRC>(t.src + p * 3 * ES, R, G_, B);
                        lv[g * GPX + i] = lum<SRC>(R, G_, B, k);
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < G * GPX; ++j) {
            const int64_t p = t.px0 + (int64_t)j * kBlock + tid;
            valid[j] = p < t.n;
            lv[j] = 0.0f;
            if (p < t.n) {
                float R, G_, B;
                load_px<SRC>(t.src + p * 3 * ES, R, G_, B);
                lv[j] = lum<SRC>(R, G_, B, k);
            }
        }
    }
}

// Writes per-pixel values v (G*GPX of them, laid out as tile_lum produced
// them) to one output.
template <int SRC, int G>
__device__ __forceinline__ void tile_store(const DevImage &im, const TileRef &t, uint8_t *out,
                                           int dtype, const float (&v)[G * group_px(SRC)],
                                           float fscale, float u8scale)
{
    constexpr int GPX = group_px(SRC);
    const int tid = threadIdx.x;
    if (im.walk != kWalkScalar) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t gp = t.px0 + (int64_t)(g * kBlock + tid) * GPX;
            if (gp + GPX <= t.n) {
                float vv[GPX];
#pragma unroll
                for (int i = 0; i < GPX; ++i)
                    vv[i] = v[g * GPX + i];
                store_group<GPX>(out, dtype, gp, vv, fscale, u8scale);
            } else {
#pragma unroll
                for (int i = 0; i < GPX; ++i)
                    if (gp + i < t.n)
                        store_px(out, dtype, gp + i, v[g * GPX + i], fscale, u8scale);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < G * GPX; ++j) {
            const int64_t p = t.px0 + (int64_t)j * kBlock + tid;
            if (p < t.n)
                store_px(out, dtype, p, v[j], fscale, u8scale);
        }
    }
}

// ------------------------------------------------------- decolorization

// Luminance of one full vector group (GPX pixels) held as 12 dwords.
template <int SRC>
__device__ __forceinline__ void group_lum(const unsigned (&w)[12], Coef k,
                                          float (&v)[group_px(SRC)])
{
#pragma unroll
    for (int i = 0; i < group_px(SRC); ++i)
        v[i] = lum<SRC>(chan<SRC>(w, 3 * i), chan<SRC>(w, 3 * i + 1), chan<SRC>(w, 3 * i + 2), k);
}

// Decolorization of one tile: every load of the thread's G groups is issued
// first, then each group is evaluated and stored while later loads are still
// in flight.
template <int SRC, int G>
__device__ __forceinline__ void decolor_tile(const DevImage &im, int64_t tile, Coef k)
{
    constexpr int GPX = group_px(SRC);
    constexpr int ES = elem_size(SRC);
    const TileRef t = tile_ref(im, tile, (int64_t)kBlock * G * GPX);
    const float u8s = 255.0f * im.unit;
    const int tid = threadIdx.x;
    if (im.walk != kWalkScalar) {
        unsigned w[G][12];
        bool full[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t gp = t.px0 + (int64_t)(g * kBlock + tid) * GPX;
            full[g] = gp + GPX <= t.n;
            if (full[g])
                load_group<SRC>(t.src + gp * 3 * ES, w[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t gp = t.px0 + (int64_t)(g * kBlock + tid) * GPX;
            if (full[g]) {
                float v[GPX];
                group_lum<SRC>(w[g], k, v);
                store_group<GPX>(t.dst, im.dst_dtype, gp, v, im.unit, u8s);
                if (t.dst2)
                    store_group<GPX>(t.dst2, im.dst2_dtype, gp, v, im.unit, u8s);
            } else {
                for (int64_t p = gp; p < t.n && p < gp + GPX; ++p) {
                    float R, G_, B;
                    load_px<SRC>(t.src + p * 3 * ES, R, G_, B);
                    const float v = lum<SRC>(R, G_, B, k);
                    store_px(t.dst, im.dst_dtype, p, v, im.unit, u8s);
                    if (t.dst2)
                        store_px(t.dst2, im.dst2_dtype, p, v, im.unit, u8s);
                }
            }
        }
    } else {
        for (int j = 0; j < G * GPX; ++j) {
            const int64_t p = t.px0 + (int64_t)j * kBlock + tid;
            if (p < t.n) {
                float R, G_, B;
                load_px<SRC>(t.src + p * 3 * ES, R, G_, B);
                const float v = lum<SRC>(R, G_, B, k);
                store_px(t.dst, im.dst_dtype, p, v, im.unit, u8s);
                if (t.dst2)
                    store_px(t.dst2, im.dst2_dtype, p, v, im.unit, u8s);
            }
        }
    }
}

template <int SRC, int G>
__global__ __launch_bounds__(kBlock) void k_decolor_single(DevImage im, int64_t ntiles)
{
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        decolor_tile<SRC, G>(im, tile, im.k);
}

// Index of the image owning global tile `tile`: the first i with
// tile_end[i] > tile (tile_end is the inclusive prefix sum of tile counts).
__device__ __forceinline__ int find_image(const int64_t *tile_end, int nimg, int64_t tile)
{
    int lo = 0, hi = nimg - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tile_end[mid] > tile)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// One launch over the tiles of many images. MIXED = the input element type
// varies per image (a uniform branch per tile); otherwise it is SRC.
template <int SRC, int G, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_decolor_table(const DevImage *__restrict__ table,
                                                          const int64_t *__restrict__ tile_end,
                                                          int nimg, int64_t total_tiles)
{
    for (int64_t tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
        const int i = find_image(tile_end, nimg, tile);
        const DevImage im = table[i];
        const int64_t lt = tile - im.tile_begin;
        if constexpr (MIXED) {
            // Tile sizes are per image: G groups of its own group width.
            if (im.src_dtype == 0)
                decolor_tile<0, G>(im, lt, im.k);
            else if (im.src_dtype == 1)
                decolor_tile<1, G>(im, lt, im.k);
            else
                decolor_tile<2, G>(im, lt, im.k);
        } else {
            decolor_tile<SRC, G>(im, lt, im.k);
        }
    }
}

// ------------------------------------------------------------ tone map

__device__ __forceinline__ Part part_empty()
{
    return Part{0.0f, 0.0f, 0.0f, __builtin_inff(), -__builtin_inff()};
}

// Chan-Golub-LeVeque combination of two partials (count, mean, sum of squared
// deviations); extremes by min/max.
__device__ __forceinline__ Part merge(const Part &a, const Part &b)
{
    if (b.n == 0.0f)
        return a;
    if (a.n == 0.0f)
        return b;
    Part r;
    r.n = a.n + b.n;
    const float d = b.mean - a.mean;
    const float f = b.n / r.n;
    r.mean = fmaf(d, f, a.mean);
    r.m2 = (a.m2 + b.m2) + d * d * a.n * f;
    r.lo = fminf(a.lo, b.lo);
    r.hi = fmaxf(a.hi, b.hi);
    return r;
}

// Statistics pass: one tile = one fixed chunk of kStatsChunkPx pixels (16 per
// thread), so the partials, and the statistics merged from them in a fixed
// order, depend only on the image, never on the other images of the call.
template <int SRC>
__device__ __forceinline__ void tm_pass1_tile(const DevImage &im, int64_t tile, Coef k,
                                              TmArgs tm, Part *parts, Part *sh)
{
    constexpr int G = kStatsPxPerThread / group_px(SRC);
    constexpr int NV = kStatsPxPerThread;
    const TileRef t = tile_ref(im, tile, kStatsChunkPx);
    float lv[NV];
    bool valid[NV];
    tile_lum<SRC, G>(im, t, k, lv, valid);
    if (t.dst2)
        tile_store<SRC, G>(im, t, t.dst2, im.dst2_dtype, lv, im.unit, 255.0f * im.unit);

    // Per-thread exact two-pass statistics over its own pixels (in registers).
    float x[NV];
    float cnt = 0.0f, sum = 0.0f, lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const float lh = lv[i] * im.unit;
        x[i] = hw_log2(lh + tm.eps);
        if (valid[i]) {
            cnt += 1.0f;
            sum += x[i];
            lo = fminf(lo, lh);
            hi = fmaxf(hi, lh);
        }
    }
    Part p = part_empty();
    if (cnt > 0.0f) {
        const float mean = sum / cnt;
        float m2 = 0.0f;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const float d = x[i] - mean;
            m2 = valid[i] ? fmaf(d, d, m2) : m2;
        }
        p = Part{cnt, mean, m2, lo, hi};
    }
    const int tid = threadIdx.x;
    sh[tid] = p;
    __syncthreads();
    if (tid < 64) {
        // Wave 0: each lane folds four consecutive thread partials, then a
        // fixed butterfly over the 64 lanes.
        Part a = merge(merge(sh[4 * tid], sh[4 * tid + 1]), merge(sh[4 * tid + 2], sh[4 * tid + 3]));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            Part b;
            b.n = __shfl_down(a.n, off, 64);
            b.mean = __shfl_down(a.mean, off, 64);
            b.m2 = __shfl_down(a.m2, off, 64);
            b.lo = __shfl_down(a.lo, off, 64);
            b.hi = __shfl_down(a.hi, off, 64);
            a = merge(a, b);
        }
        if (tid == 0)
            parts[im.chunk_begin + tile] = a;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_tm_pass1(const DevImage *__restrict__ table,
                                                     const int64_t *__restrict__ tile_end,
                                                     int nimg, int64_t total_tiles, TmArgs tm,
                                                     Part *__restrict__ parts)
{
    __shared__ Part sh[kBlock];
    for (int64_t tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
        const int i = find_image(tile_end, nimg, tile);
        const DevImage im = table[i];
        const int64_t lt = tile - im.tile_begin;
        if (im.src_dtype == 0)
            tm_pass1_tile<0>(im, lt, im.k, tm, parts, sh);
        else if (im.src_dtype == 1)
            tm_pass1_tile<1>(im, lt, im.k, tm, parts, sh);
        else
            tm_pass1_tile<2>(im, lt, im.k, tm, parts, sh);
    }
}

// One workgroup per image: fixed-order merge of the image's chunk partials,
// then the curve coefficients (and optionally the statistics for the caller).
__global__ __launch_bounds__(kBlock) void k_tm_finalize(const DevImage *__restrict__ table,
                                                        const int64_t *__restrict__ tile_end,
                                                        TmArgs tm, const Part *__restrict__ parts,
                                                        Curve *__restrict__ curves,
                                                        StatsOut *__restrict__ stats)
{
    __shared__ Part sh[kBlock];
    const int img = blockIdx.x;
    const DevImage im = table[img];
    const int64_t nch = tile_end[img] - im.tile_begin;
    const int tid = threadIdx.x;
    Part a = part_empty();
    for (int64_t c = tid; c < nch; c += kBlock)
        a = merge(a, parts[im.chunk_begin + c]);
    sh[tid] = a;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (tid < s)
            sh[tid] = merge(sh[tid], sh[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        const Part tot = sh[0];
        const float ln2 = 0.693147180559945309f;
        const float log2e = 1.442695040888963407f;
        const float sigma2 = tot.n > 0.0f ? sqrtf(tot.m2 / tot.n) : 0.0f; // log2 units
        const float s2 = fmaxf(sigma2, tm.sigma_floor * log2e);
        // T = 1 / (1 + exp(-c (x - mu) / s)) = 1 / (1 + exp2(a (x2 - mu2)))
        curves[img] = Curve{-tm.contrast * log2e / s2, tot.mean};
        if (stats) {
            StatsOut o;
            o.log_mean = tot.mean * ln2;
            o.log_std = sigma2 * ln2;
            o.l_min = tot.lo;
            o.l_max = tot.hi;
            o.count = im.npx;
            stats[img] = o;
        }
    }
}

template <int SRC>
__device__ __forceinline__ void tm_pass2_tile(const DevImage &im, int64_t tile, Coef k,
                                              TmArgs tm, Curve cv)
{
    constexpr int G = kStatsPxPerThread / group_px(SRC);
    constexpr int NV = kStatsPxPerThread;
    const TileRef t = tile_ref(im, tile, kStatsChunkPx);
    float lv[NV];
    bool valid[NV];
    tile_lum<SRC, G>(im, t, k, lv, valid);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const float x2 = hw_log2(fmaf(lv[i], im.unit, tm.eps));
        lv[i] = hw_rcp(1.0f + hw_exp2(cv.a * (x2 - cv.mu2)));
    }
    tile_store<SRC, G>(im, t, t.dst, im.dst_dtype, lv, 1.0f, 255.0f);
}

__global__ __launch_bounds__(kBlock) void k_tm_pass2(const DevImage *__restrict__ table,
                                                     const int64_t *__restrict__ tile_end,
                                                     int nimg, int64_t total_tiles, TmArgs tm,
                                                     const Curve *__restrict__ curves)
{
    for (int64_t tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
        const int i = find_image(tile_end, nimg, tile);
        const DevImage im = table[i];
        const Curve cv = curves[i];
        const int64_t lt = tile - im.tile_begin;
        if (im.src_dtype == 0)
            tm_pass2_tile<0>(im, lt, im.k, tm, cv);
        else if (im.src_dtype == 1)
            tm_pass2_tile<1>(im, lt, im.k, tm, cv);
        else
            tm_pass2_tile<2>(im, lt, im.k, tm, cv);
    }
}

// ------------------------------------------------------------ launchers

static unsigned grid_of(int64_t ntiles, int64_t grid)
{
    int64_t g = grid > 0 && grid < ntiles ? grid : ntiles;
    if (g > 0x7fffffff)
        g = 0x7fffffff;
    return (unsigned)(g > 0 ? g : 1);
}

hipError_t launch_decolor_single(const DevImage &im, int groups, int64_t grid,
                                 hipStream_t s)
{
    const int64_t ntiles = im.ntiles;
    const unsigned g = grid_of(ntiles, grid);
#define DC_LAUNCH_SINGLE(S, GG)                                                                   \
    hipLaunchKernelGGL((k_decolor_single<S, GG>), dim3(g), dim3(kBlock), 0, s, im, ntiles)
    switch (im.src_dtype * 8 + groups) {
    case 0 * 8 + 1: DC_LAUNCH_SINGLE(0, 1); break;
    case 0 * 8 + 2: DC_LAUNCH_SINGLE(0, 2); break;
    case 0 * 8 + 4: DC_LAUNCH_SINGLE(0, 4); break;
    case 1 * 8 + 1: DC_LAUNCH_SINGLE(1, 1); break;
    case 1 * 8 + 2: DC_LAUNCH_SINGLE(1, 2); break;
    case 1 * 8 + 4: DC_LAUNCH_SINGLE(1, 4); break;
    case 2 * 8 + 1: DC_LAUNCH_SINGLE(2, 1); break;
    case 2 * 8 + 2: DC_LAUNCH_SINGLE(2, 2); break;
    case 2 * 8 + 4: DC_LAUNCH_SINGLE(2, 4); break;
    default: return hipErrorInvalidValue;
    }
#undef DC_LAUNCH_SINGLE
    return hipGetLastError();
}

hipError_t launch_decolor_table(const DevImage *table, const int64_t *tile_end, int nimg,
                                int64_t total_tiles, int mixed_src, int src_dtype,
                                int groups, int64_t grid, hipStream_t s)
{
    const unsigned g = grid_of(total_tiles, grid);
#define DC_LAUNCH_TABLE(S, GG, M)                                                                 \
    hipLaunchKernelGGL((k_decolor_table<S, GG, M>), dim3(g), dim3(kBlock), 0, s, table, tile_end,  \
                       nimg, total_tiles)
    if (mixed_src) {
        switch (groups) {
        case 1: DC_LAUNCH_TABLE(0, 1, true); break;
        case 2: DC_LAUNCH_TABLE(0, 2, true); break;
        case 4: DC_LAUNCH_TABLE(0, 4, true); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (src_dtype * 8 + groups) {
        case 0 * 8 + 1: DC_LAUNCH_TABLE(0, 1, false); break;
        case 0 * 8 + 2: DC_LAUNCH_TABLE(0, 2, false); break;
        case 0 * 8 + 4: DC_LAUNCH_TABLE(0, 4, false); break;
        case 1 * 8 + 1: DC_LAUNCH_TABLE(1, 1, false); break;
        case 1 * 8 + 2: DC_LAUNCH_TABLE(1, 2, false); break;
        case 1 * 8 + 4: DC_LAUNCH_TABLE(1, 4, false); break;
        case 2 * 8 + 1: DC_LAUNCH_TABLE(2, 1, false); break;
        case 2 * 8 + 2: DC_LAUNCH_TABLE(2, 2, false); break;
        case 2 * 8 + 4: DC_LAUNCH_TABLE(2, 4, false); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef DC_LAUNCH_TABLE
    return hipGetLastError();
}

hipError_t launch_tm_pass1(const DevImage *table, const int64_t *tile_end, int nimg,
                           int64_t total_tiles, TmArgs tm, Part *parts, hipStream_t s)
{
    hipLaunchKernelGGL(k_tm_pass1, dim3(grid_of(total_tiles, 0)), dim3(kBlock), 0, s, table,
                       tile_end, nimg, total_tiles, tm, parts);
    return hipGetLastError();
}

hipError_t launch_tm_finalize(const DevImage *table, int nimg, const int64_t *tile_end,
                              TmArgs tm, const Part *parts, Curve *curves, StatsOut *stats,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_tm_finalize, dim3(nimg), dim3(kBlock), 0, s, table, tile_end, tm, parts,
                       curves, stats);
    return hipGetLastError();
}

hipError_t launch_tm_pass2(const DevImage *table, const int64_t *tile_end, int nimg,
                           int64_t total_tiles, TmArgs tm, const Curve *curves,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_tm_pass2, dim3(grid_of(total_tiles, 0)), dim3(kBlock), 0, s, table,
                       tile_end, nimg, total_tiles, tm, curves);
    return hipGetLastError();
}

} // namespace dc
