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

// Output encodings. F32 stores v (times fscale when SF); F16 stores the
// round-to-nearest-even binary16 of the same; U8 stores v (times u8scale when
// SU) converted by v_cvt_pk_u8_f32, which rounds to nearest with ties to even
// and saturates to [0, 255] (NaN gives 0).
struct Enc {
    float fscale;
    float u8scale;
};

template <bool SU>
__device__ __forceinline__ unsigned pack_u8x4(float a, float b, float c, float d, float s)
{
    if constexpr (SU) {
        a *= s;
        b *= s;
        c *= s;
        d *= s;
    }
    unsigned w = __builtin_amdgcn_cvt_pk_u8_f32(a, 0, 0u);
    w = __builtin_amdgcn_cvt_pk_u8_f32(b, 1, w);
    w = __builtin_amdgcn_cvt_pk_u8_f32(c, 2, w);
    return __builtin_amdgcn_cvt_pk_u8_f32(d, 3, w);
}

__device__ __forceinline__ unsigned pack_f16x2(float a, float b)
{
    const unsigned short ha = __builtin_bit_cast(unsigned short, (_Float16)a);
    const unsigned short hb = __builtin_bit_cast(unsigned short, (_Float16)b);
    return (unsigned)ha | ((unsigned)hb << 16);
}

// Stores GPX consecutive values at pixel index px of a 1-channel row.
template <int GPX, bool SF, bool SU>
__device__ __forceinline__ void store_group(uint8_t *base, int dtype, int64_t px,
                                            const float (&v)[GPX], Enc e)
{
    if (dtype == 0) {
        unsigned w[GPX / 4];
#pragma unroll
        for (int i = 0; i < GPX / 4; ++i)
            w[i] = pack_u8x4<SU>(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3], e.u8scale);
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
            w[i] = SF ? pack_f16x2(v[2 * i] * e.fscale, v[2 * i + 1] * e.fscale)
                      : pack_f16x2(v[2 * i], v[2 * i + 1]);
        uint8_t *p = base + 2 * px;
        if constexpr (GPX == 4) {
            *gpw<u32x2>(p) = u32x2{w[0], w[1]};
        } else {
#pragma unroll
            for (int i = 0; i < GPX / 8; ++i)
                gpw<u32x4>(p)[i] = u32x4{w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]};
        }
    } else {
        uint8_t *p = base + 4 * px;
#pragma unroll
        for (int i = 0; i < GPX / 4; ++i) {
            float a = v[4 * i], b = v[4 * i + 1], c = v[4 * i + 2], d = v[4 * i + 3];
            if constexpr (SF) {
                a *= e.fscale;
                b *= e.fscale;
                c *= e.fscale;
                d *= e.fscale;
            }
            gpw<u32x4>(p)[i] = u32x4{__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                     __builtin_bit_cast(unsigned, c), __builtin_bit_cast(unsigned, d)};
        }
    }
}

template <bool SF, bool SU>
__device__ __forceinline__ void store_px(uint8_t *base, int dtype, int64_t px, float v, Enc e)
{
    if (dtype == 0)
        gpw<uint8_t>(base)[px] = (uint8_t)__builtin_amdgcn_cvt_pk_u8_f32(SU ? v * e.u8scale : v, 0, 0u);
    else if (dtype == 1)
        gpw<_Float16>(base)[px] = (_Float16)(SF ? v * e.fscale : v);
    else
        gpw<float>(base)[px] = SF ? v * e.fscale : v;
}

// Encoding of Lhat from L (input units): 8-bit input carries L in code units,
// so FP outputs scale by 1/255 and the 8-bit output takes L as is; float input
// carries Lhat, so only the 8-bit output scales (by 255).
template <int SRC>
struct LumEnc {
    static constexpr bool SF = SRC == 0;
    static constexpr bool SU = SRC != 0;
};

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
// pixels, or the same count of single pixels on the per-pixel walk). lv holds L
// in input units; valid marks pixels inside the segment. In both walks the
// valid slots of a thread form a prefix, and slot 0 of lane 0 of a wave holds
// the wave's first pixel.
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

// Writes per-pixel values v (laid out as tile_lum produced them) to one output.
template <int SRC, int G, bool SF, bool SU>
__device__ __forceinline__ void tile_store(const DevImage &im, const TileRef &t, uint8_t *out,
                                           int dtype, const float (&v)[G * group_px(SRC)], Enc e)
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
                store_group<GPX, SF, SU>(out, dtype, gp, vv, e);
            } else {
#pragma unroll
                for (int i = 0; i < GPX; ++i)
                    if (gp + i < t.n)
                        store_px<SF, SU>(out, dtype, gp + i, v[g * GPX + i], e);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < G * GPX; ++j) {
            const int64_t p = t.px0 + (int64_t)j * kBlock + tid;
            if (p < t.n)
                store_px<SF, SU>(out, dtype, p, v[j], e);
        }
    }
}

// Visits the global tiles of a persistent block (blockIdx.x, blockIdx.x +
// gridDim.x, ...) with the index of the image that owns each. tile_end is the
// inclusive prefix sum of the images' tile counts; tiles only grow, so the
// owner is found once by binary search and then advanced in place.
template <typename F>
__device__ __forceinline__ void for_each_tile(const int64_t *__restrict__ tile_end, int nimg,
                                              int64_t total_tiles, F &&f)
{
    int64_t tile = blockIdx.x;
    if (tile >= total_tiles)
        return;
    int lo = 0, hi = nimg - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tile_end[mid] > tile)
            hi = mid;
        else
            lo = mid + 1;
    }
    int i = lo;
    for (; tile < total_tiles; tile += gridDim.x) {
        while (tile_end[i] <= tile)
            ++i;
        f(i, tile);
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
__device__ __forceinline__ void decolor_tile(const DevImage &im, int64_t tile)
{
    constexpr int GPX = group_px(SRC);
    constexpr int ES = elem_size(SRC);
    constexpr bool SF = LumEnc<SRC>::SF, SU = LumEnc<SRC>::SU;
    const TileRef t = tile_ref(im, tile, (int64_t)kBlock * G * GPX);
    const Enc e{im.unit, 255.0f};
    const Coef k = im.k;
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
                store_group<GPX, SF, SU>(t.dst, im.dst_dtype, gp, v, e);
                if (t.dst2)
                    store_group<GPX, SF, SU>(t.dst2, im.dst2_dtype, gp, v, e);
            } else {
                for (int64_t p = gp; p < t.n && p < gp + GPX; ++p) {
                    float R, G_, B;
                    load_px<SRC>(t.src + p * 3 * ES, R, G_, B);
                    const float v = lum<SRC>(R, G_, B, k);
                    store_px<SF, SU>(t.dst, im.dst_dtype, p, v, e);
                    if (t.dst2)
                        store_px<SF, SU>(t.dst2, im.dst2_dtype, p, v, e);
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
                store_px<SF, SU>(t.dst, im.dst_dtype, p, v, e);
                if (t.dst2)
                    store_px<SF, SU>(t.dst2, im.dst2_dtype, p, v, e);
            }
        }
    }
}

template <int SRC, int G>
__global__ __launch_bounds__(kBlock) void k_decolor_single(DevImage im, int64_t ntiles)
{
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        decolor_tile<SRC, G>(im, tile);
}

// One launch over the tiles of many images. MIXED = the input element type
// varies per image (a uniform branch per tile); otherwise it is SRC.
template <int SRC, int G, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_decolor_table(const DevImage *__restrict__ table,
                                                          const int64_t *__restrict__ tile_end,
                                                          int nimg, int64_t total_tiles)
{
    for_each_tile(tile_end, nimg, total_tiles, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        const int64_t lt = tile - im.tile_begin;
        if constexpr (MIXED) {
            // Tile sizes are per image: G groups of its own group width.
            if (im.src_dtype == 0)
                decolor_tile<0, G>(im, lt);
            else if (im.src_dtype == 1)
                decolor_tile<1, G>(im, lt);
            else
                decolor_tile<2, G>(im, lt);
        } else {
            decolor_tile<SRC, G>(im, lt);
        }
    });
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

// x2 = log2(Lhat + eps) from L in input units. Both passes use this one
// expression, so a pixel gets the same x2 in the statistics and in the curve.
__device__ __forceinline__ float xlog2(float l, float unit, float eps)
{
    return hw_log2(fmaf(l, unit, eps));
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// Statistics pass over one tile of kStatsChunkPx pixels (16 per thread). Each
// wave reduces its 1024 pixels to one partial with no workgroup barrier: sums
// of d = x2 - K and d^2, shifted by K = x2 of the wave's first pixel (so a
// flat image gives exactly mean = K, M2 = 0), count and the extremes of L.
// Chunks are fixed slices of each image, so the partials, and the statistics
// merged from them in a fixed order, never depend on the other images of the
// call or on the launch shape.
template <int SRC>
__device__ __forceinline__ void tm_pass1_tile(const DevImage &im, int64_t tile, TmArgs tm,
                                              Part *__restrict__ parts)
{
    constexpr int G = kStatsPxPerThread / group_px(SRC);
    constexpr int NV = kStatsPxPerThread;
    const TileRef t = tile_ref(im, tile, kStatsChunkPx);
    float lv[NV];
    bool valid[NV];
    tile_lum<SRC, G>(im, t, im.k, lv, valid);
    if (t.dst2)
        tile_store<SRC, G, LumEnc<SRC>::SF, LumEnc<SRC>::SU>(im, t, t.dst2, im.dst2_dtype, lv,
                                                            Enc{im.unit, 255.0f});
    float x[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i)
        x[i] = xlog2(lv[i], im.unit, tm.eps);
    const float K = __builtin_bit_cast(
        float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x[0])));
    float s = 0.0f, q = 0.0f, lo = lv[0], hi = lv[0];
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i)
        cnt += valid[i] ? 1 : 0;
    if (cnt == NV) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const float d = x[i] - K;
            s += d;
            q = fmaf(d, d, q);
            lo = fminf(lo, lv[i]);
            hi = fmaxf(hi, lv[i]);
        }
    } else if (cnt > 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const float d = valid[i] ? x[i] - K : 0.0f;
            const float l = valid[i] ? lv[i] : lv[0];
            s += d;
            q = fmaf(d, d, q);
            lo = fminf(lo, l);
            hi = fmaxf(hi, l);
        }
    } else {
        lo = __builtin_inff();
        hi = -__builtin_inff();
    }
    s = wave_sum(s);
    q = wave_sum(q);
    const float n = wave_sum((float)cnt);
    lo = wave_min(lo);
    hi = wave_max(hi);
    const int lane = threadIdx.x & 63;
    if (lane == 0) {
        Part p = part_empty();
        if (n > 0.0f) {
            const float m = s / n;
            p = Part{n, K + m, fmaxf(fmaf(-s, m, q), 0.0f), lo * im.unit, hi * im.unit};
        }
        parts[im.chunk_begin + tile * kWavesPerBlock + (threadIdx.x >> 6)] = p;
    }
}

__global__ __launch_bounds__(kBlock) void k_tm_pass1(const DevImage *__restrict__ table,
                                                     const int64_t *__restrict__ tile_end,
                                                     int nimg, int64_t total_tiles, TmArgs tm,
                                                     Part *__restrict__ parts)
{
    for_each_tile(tile_end, nimg, total_tiles, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        const int64_t lt = tile - im.tile_begin;
        if (im.src_dtype == 0)
            tm_pass1_tile<0>(im, lt, tm, parts);
        else if (im.src_dtype == 1)
            tm_pass1_tile<1>(im, lt, tm, parts);
        else
            tm_pass1_tile<2>(im, lt, tm, parts);
    });
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
    const int64_t nch = (tile_end[img] - im.tile_begin) * kWavesPerBlock;
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
__device__ __forceinline__ void tm_pass2_tile(const DevImage &im, int64_t tile, TmArgs tm, Curve cv)
{
    constexpr int G = kStatsPxPerThread / group_px(SRC);
    constexpr int NV = kStatsPxPerThread;
    const TileRef t = tile_ref(im, tile, kStatsChunkPx);
    float lv[NV];
    bool valid[NV];
    tile_lum<SRC, G>(im, t, im.k, lv, valid);
#pragma unroll
    for (int i = 0; i < NV; ++i)
        lv[i] = hw_rcp(1.0f + hw_exp2(cv.a * (xlog2(lv[i], im.unit, tm.eps) - cv.mu2)));
    tile_store<SRC, G, false, true>(im, t, t.dst, im.dst_dtype, lv, Enc{1.0f, 255.0f});
}

__global__ __launch_bounds__(kBlock) void k_tm_pass2(const DevImage *__restrict__ table,
                                                     const int64_t *__restrict__ tile_end,
                                                     int nimg, int64_t total_tiles, TmArgs tm,
                                                     const Curve *__restrict__ curves)
{
    for_each_tile(tile_end, nimg, total_tiles, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        const Curve cv = curves[i];
        const int64_t lt = tile - im.tile_begin;
        if (im.src_dtype == 0)
            tm_pass2_tile<0>(im, lt, tm, cv);
        else if (im.src_dtype == 1)
            tm_pass2_tile<1>(im, lt, tm, cv);
        else
            tm_pass2_tile<2>(im, lt, tm, cv);
    });
}

// ------------------------------------------------------------ launchers

static unsigned grid_of(int64_t ntiles, int64_t grid)
{
    int64_t g = grid > 0 && grid < ntiles ? grid : ntiles;
    if (g > 0x7fffffff)
        g = 0x7fffffff;
    return (unsigned)(g > 0 ? g : 1);
}

hipError_t launch_decolor_single(const DevImage &im, int groups, int64_t grid, hipStream_t s)
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
                                int64_t total_tiles, int mixed_src, int src_dtype, int groups,
                                int64_t grid, hipStream_t s)
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
                           int64_t total_tiles, TmArgs tm, Part *parts, int64_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_tm_pass1, dim3(grid_of(total_tiles, grid)), dim3(kBlock), 0, s, table,
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
                           int64_t total_tiles, TmArgs tm, const Curve *curves, int64_t grid,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_tm_pass2, dim3(grid_of(total_tiles, grid)), dim3(kBlock), 0, s, table,
                       tile_end, nimg, total_tiles, tm, curves);
    return hipGetLastError();
}

} // namespace dc
