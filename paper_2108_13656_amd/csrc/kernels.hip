// HIP kernels (gfx950) of the colour-temperature decolorization, Eqs. (1)-(6)
// of Ambalathankandy et al. (arXiv 2108.13656, Sec. II-B), and of the tone
// mapping built on its luminance: the global map (Sec. III-B.1, read as a
// centred sigmoid in the log domain, slope normalised by the image's standard
// deviation) with gray or re-coloured output, and the local map (Sec. III-B.2,
// smoothed local histogram equalisation on a tile grid). Also the comparator
// gray channels (rgb2gray Y, V of HSV, CIE L*) on the same data path.
//
// The work is an elementwise stream bounded by HBM bandwidth, so there is no
// MFMA here: each lane owns 12-byte work units of interleaved RGB (4 px of u8,
// 2 of f16, 1 of f32), loaded with one dwordx3 each so that a wave's lanes read
// contiguous memory, decodes them in registers, evaluates the luminance in FP32
// with the hardware square-root / reciprocal-square-root / reciprocal
// instructions, and writes its outputs with 1-16 byte stores.
#include "dc_internal.h"

#include <mutex>

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

// A float channel as every kernel reads it: NaN and negatives as lo, values
// above hi as hi. hi is the input format's ceiling: 65504, the largest finite
// binary16 (so +Inf reads as 65504), or 1e18, the top of the supported binary32
// range (+Inf included). NaN goes to lo because max returns its non-NaN operand.
__device__ __forceinline__ float chan_clamp(float v, float lo, float hi)
{
    return fminf(fmaxf(v, lo), hi);
}
template <int SRC>
__host__ __device__ constexpr float chan_max()
{
    return SRC == 1 ? 65504.0f : 1e18f;
}

// L for binary16 input: the division-free form of lum_code on the decoded
// values (the same four constants), finished as sqrt(Y) / S. Binary16 spans
// 6e-8 .. 65504, so Y stays between about 1e-30 and 5e20 and no intermediate
// leaves the FP32 normal range; NaN and negative channels read as 0 and +Inf
// as 65504 (chan_clamp). Blue reads as at least 1e-30, which keeps
// S > 0 without a clamp of its own and changes no result: binary16 has no
// value below 6e-8 but 0, and every term of 1e-30 either underflows to 0
// (B^2, C^2) or is absorbed (in S, G + B), so a black pixel still gives
// sqrt(0) * (1 / 1e-30) = 0.
__device__ __forceinline__ float lum_half(float R, float G, float B, Coef k)
{
    R = chan_clamp(R, 0.0f, chan_max<1>());
    G = chan_clamp(G, 0.0f, chan_max<1>());
    B = chan_clamp(B, 1e-30f, chan_max<1>());
    const float rr = R * R, gg = G * G;
    const float Q = hw_sqrt(fmaf(B, B, fmaf(R, R, gg)));          // sqrt(3) * Eq. (1)
    const float Lgr3 = hw_sqrt(fmaf(k.cr, rr, k.cg * gg));        // sqrt(3) * Eq. (3)
    const float rg = R + G;
    const float S = rg + B;
    const float A = fmaf(R, Lgr3, (G + B) * Q);                   // sqrt(3) S * Eq. (4)
    const float C = B * fmaf(1.73205080756887729f, rg, Q);        // sqrt(3) S * Eq. (5)
    const float Y = fmaf(k.ck * A, A, k.cc * (C * C));            // S^2 * Eq. (6)^2
    return hw_sqrt(Y) * hw_rcp(S);
}

// L for linear float input. The pixel is first normalised by S, so every
// intermediate lies in [0, 1] whatever the radiance scale (binary16 spans
// 6e-8 .. 65504), and L = S * L(r, g, b) by degree-1 homogeneity. NaN and
// negative channels read as 0, values above 1e18 as 1e18 (chan_clamp).
__device__ __forceinline__ float lum_linear(float R, float G, float B, Coef k)
{
    R = chan_clamp(R, 0.0f, chan_max<2>());
    G = chan_clamp(G, 0.0f, chan_max<2>());
    B = chan_clamp(B, 0.0f, chan_max<2>());
    const float S = (R + G) + B;
    const float inv = hw_rcp(fmaxf(S, 1e-30f));
    const float r = R * inv, g = G * inv, b = B * inv;
    const float rr = r * r, gg = g * g;
    const float lw = hw_sqrt(fmaf(b, b, fmaf(r, r, gg)) * (1.0f / 3.0f)); // Eq. (1)
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
    else if constexpr (SRC == 1)
        return lum_half(R, G, B, k);
    else
        return lum_linear(R, G, B, k);
}

// ------------------------------------------------------------ memory

// Buffer resources for the packed walk's loads: word 3 selects 32-bit data
// with no swizzle (the raw form on gfx9-class chips), the record count is set
// to its maximum so no range check ever clips a load, and the cache-policy bit
// 2 marks a load nontemporal (streaming), as __builtin_nontemporal_load does.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kBufferNontemporal = 2;

// Image pointers come from descriptors in memory, so the compiler cannot tell
// they are global; these casts give global_load/global_store instead of flat.
// The pointee types carry 1-byte alignment: on the row walk a unit's address
// follows the image's pitch and offset, not the unit's size, and the target's
// unaligned access mode (which the compiler assumes for gfx950 under ROCm)
// serves such accesses with the same dwordx3 / dwordx4 instructions.
#define DC_GLOBAL __attribute__((address_space(1)))
template <typename T>
struct Unaligned {
    typedef T type __attribute__((aligned(1)));
};
template <typename T>
__device__ __forceinline__ const DC_GLOBAL typename Unaligned<T>::type *gp(const void *p)
{
    return (const DC_GLOBAL typename Unaligned<T>::type *)p;
}
template <typename T>
__device__ __forceinline__ DC_GLOBAL typename Unaligned<T>::type *gpw(void *p)
{
    return (DC_GLOBAL typename Unaligned<T>::type *)p;
}

// Unit stores of the outputs are nontemporal: every output byte is written
// once and not read again by the kernel that writes it, so streaming stores
// keep output lines from displacing input lines in L2 and the last-level
// cache and leave less dirty data for the next pass to write back (2-5 %
// faster per pass on MI355X, measured on the 16 x 4096^2 tone map and the
// 64-frame video batch).
template <typename T>
__device__ __forceinline__ void put(DC_GLOBAL typename Unaligned<T>::type *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// ------------------------------------------------------------ decode
//
// Work unit: 12 bytes of interleaved RGB per lane, loaded with one dwordx3
// (4 pixels of u8, 2 of f16, 1 of f32). Lanes of a wave take consecutive
// units, so every load instruction reads 768 contiguous bytes and every store
// instruction writes contiguous bytes too; a thread holds U units of a tile,
// all loads issued before any arithmetic.

__host__ __device__ constexpr int unit_px(int src_dtype)
{
    return src_dtype == 0 ? 4 : (src_dtype == 1 ? 2 : 1);
}

__device__ __forceinline__ float half_lo(unsigned w)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
}
__device__ __forceinline__ float half_hi(unsigned w)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}

// Element e (channel value number e) of a 12-byte unit held as 3 dwords.
template <int SRC>
__device__ __forceinline__ float chan(const unsigned (&w)[3], int e)
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

// One unit: three dwords from any element-aligned address (a single dwordx3;
// the target serves unaligned dword accesses).
// The loads are nontemporal (NT): a pass reads each input byte once, and an
// input that a later pass reads again (the tone map's curve pass) is, at the
// batch sizes that matter, far larger than the caches. Streaming loads leave
// L2 to the small shared data (descriptors, partials, curves) and made the
// tone map's curve pass about 6 % faster on MI355X. A tile-table
// decolorization that reads one input for several images (weights per image
// on outputs of differing layouts) keeps plain loads for it, so the repeats
// hit in cache; the weight-sweep kernel reads its shared input once.
template <bool NT = true>
__device__ __forceinline__ void load_unit(const uint8_t *p, unsigned (&w)[3])
{
    const auto *q = gp<unsigned>(p);
    if constexpr (NT) {
        w[0] = __builtin_nontemporal_load(&q[0]);
        w[1] = __builtin_nontemporal_load(&q[1]);
        w[2] = __builtin_nontemporal_load(&q[2]);
    } else {
        w[0] = q[0];
        w[1] = q[1];
        w[2] = q[2];
    }
}

template <int SRC>
__device__ __forceinline__ void load_px(const uint8_t *p, float &R, float &G, float &B)
{
    if constexpr (SRC == 0) {
        const auto *b = gp<uint8_t>(p);
        R = b[0];
        G = b[1];
        B = b[2];
    } else if constexpr (SRC == 1) {
        const auto *h = gp<_Float16>(p);
        R = (float)h[0];
        G = (float)h[1];
        B = (float)h[2];
    } else {
        const auto *f = gp<float>(p);
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
__device__ __forceinline__ unsigned u8_of(float v, float s, int byte, unsigned acc)
{
    return __builtin_amdgcn_cvt_pk_u8_f32(SU ? v * s : v, byte, acc);
}

__device__ __forceinline__ unsigned pack_f16x2(float a, float b)
{
    const unsigned short ha = __builtin_bit_cast(unsigned short, (_Float16)a);
    const unsigned short hb = __builtin_bit_cast(unsigned short, (_Float16)b);
    return (unsigned)ha | ((unsigned)hb << 16);
}

// Stores the PPU values of one unit at pixel index lp of a 1-channel row
// whose pixel 0 is at base.
template <int PPU, bool SF, bool SU>
__device__ __forceinline__ void store_unit(uint8_t *base, int dtype, uint32_t lp,
                                           const float (&v)[PPU], Enc e)
{
    if (dtype == 0) {
        unsigned w = 0;
#pragma unroll
        for (int i = 0; i < PPU; ++i)
            w = u8_of<SU>(v[i], e.u8scale, i, w);
        uint8_t *p = base + lp;
        if constexpr (PPU == 4)
            put(gpw<unsigned>(p), w);
        else if constexpr (PPU == 2)
            put(gpw<unsigned short>(p), (unsigned short)w);
        else
            put(gpw<uint8_t>(p), (uint8_t)w);
    } else if (dtype == 1) {
        float a[PPU];
#pragma unroll
        for (int i = 0; i < PPU; ++i)
            a[i] = SF ? v[i] * e.fscale : v[i];
        uint8_t *p = base + 2 * lp;
        if constexpr (PPU == 4)
            put(gpw<u32x2>(p), u32x2{pack_f16x2(a[0], a[1]), pack_f16x2(a[2], a[3])});
        else if constexpr (PPU == 2)
            put(gpw<unsigned>(p), pack_f16x2(a[0], a[1]));
        else
            put(gpw<_Float16>(p), (_Float16)a[0]);
    } else {
        unsigned b[PPU];
#pragma unroll
        for (int i = 0; i < PPU; ++i)
            b[i] = __builtin_bit_cast(unsigned, SF ? v[i] * e.fscale : v[i]);
        uint8_t *p = base + 4 * lp;
        if constexpr (PPU == 4)
            put(gpw<u32x4>(p), u32x4{b[0], b[1], b[2], b[3]});
        else if constexpr (PPU == 2)
            put(gpw<u32x2>(p), u32x2{b[0], b[1]});
        else
            put(gpw<unsigned>(p), b[0]);
    }
}

template <bool SF, bool SU>
__device__ __forceinline__ void store_px(uint8_t *base, int dtype, uint32_t lp, float v, Enc e)
{
    if (dtype == 0)
        gpw<uint8_t>(base)[lp] = (uint8_t)u8_of<SU>(v, e.u8scale, 0, 0u);
    else if (dtype == 1)
        gpw<_Float16>(base)[lp] = (_Float16)(SF ? v * e.fscale : v);
    else
        gpw<float>(base)[lp] = SF ? v * e.fscale : v;
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

// One tile: base pointers at the tile's first pixel (uniform across the
// workgroup) and how many pixels of its segment remain from there. A packed
// image is one segment of W * H pixels. A pitched image on the row walk is
// tiled the same way, over its W * H pixels in row-major order: tile-local
// pixel p lies q(p) rows below the tile's first pixel, at byte offset
// p * bpp + q(p) * gap from it (gap = pitch - W * bpp, the row's padding),
// q(p) = floor((col0 + p) / W) = mulhi(col0 + p, magic) with col0 the first
// pixel's column and magic = ceil(2^32 / W), exact for the widths the runtime
// gives this walk. Offsets within a tile fit in 32 bits.
struct TileRef {
    const uint8_t *src;
    uint8_t *dst;
    uint8_t *dst2;
    int64_t rem;
    uint32_t col0, magic, width, gs, gd, gd2;
};

// DST_CH = channels per pixel of dst (3 for the re-coloured tone map).
template <int DST_CH = 1>
__device__ __forceinline__ TileRef tile_ref(const DevImage &im, int64_t tile, int64_t tile_px)
{
    TileRef t;
    const int64_t es = 3 * elem_size(im.src_dtype), ed = DST_CH * elem_size(im.dst_dtype);
    const int64_t e2 = im.dst2 ? elem_size(im.dst2_dtype) : 0;
    t.col0 = 0;
    t.magic = im.magic;
    t.width = (uint32_t)im.width;
    t.gs = im.gap_src;
    t.gd = im.gap_dst;
    t.gd2 = im.gap_dst2;
    if (im.walk == kWalkRows) {
        const int64_t px0 = tile * tile_px;
        const int64_t row0 = (int64_t)((uint64_t)px0 / (uint64_t)t.width);
        const int64_t col0 = px0 - row0 * (int64_t)t.width;
        t.col0 = (uint32_t)col0;
        t.src = im.src + row0 * im.src_seg_stride + col0 * es;
        t.dst = im.dst + row0 * im.dst_seg_stride + col0 * ed;
        t.dst2 = im.dst2 ? im.dst2 + row0 * im.dst2_seg_stride + col0 * e2 : nullptr;
        t.rem = im.seg_len - px0;
        return t;
    }
    const int64_t seg = tile / im.tiles_per_seg;
    const int64_t ts = tile - seg * im.tiles_per_seg;
    const int64_t px0 = ts * tile_px;
    const int64_t segs = im.walk == kWalkScalar ? seg : 0; // packed: one segment
    t.src = im.src + segs * im.src_seg_stride + px0 * es;
    t.dst = im.dst + segs * im.dst_seg_stride + px0 * ed;
    t.dst2 = im.dst2 ? im.dst2 + segs * im.dst2_seg_stride + px0 * e2 : nullptr;
    t.rem = im.seg_len - px0;
    return t;
}

// Tile-local pixel of slot (u, j) of this thread: unit u covers pixels
// (u * kBlock + tid) * PPU + j on the vector walks; the per-pixel walk uses
// (u * PPU + j) * kBlock + tid. Either way the slots a thread holds are in
// increasing pixel order, so its valid slots form a prefix, and slot 0 of lane
// 0 of a wave is the wave's first pixel.
template <int PPU>
__device__ __forceinline__ uint32_t slot_lp(bool vec, int u, int j)
{
    const uint32_t tid = threadIdx.x;
    return vec ? (uint32_t)(u * kBlock + tid) * PPU + j : (uint32_t)(u * PPU + j) * kBlock + tid;
}

// Rows below the tile's first pixel of tile-local pixel p (0 off the row walk).
template <bool ROWS>
__device__ __forceinline__ uint32_t row_q(const TileRef &t, uint32_t p)
{
    if constexpr (ROWS)
        return __umulhi(t.col0 + p, t.magic);
    else
        return 0u;
}

// Where the unit of PPU pixels from tile-local pixel lp lies: q of its first
// pixel, and whether a row break falls inside it (its pixels are then not
// contiguous; only when W is not a multiple of PPU).
struct UnitPos {
    uint32_t q;
    bool split;
};
template <int PPU, bool ROWS>
__device__ __forceinline__ UnitPos unit_pos(const TileRef &t, uint32_t lp)
{
    UnitPos u{row_q<ROWS>(t, lp), false};
    if constexpr (ROWS && PPU > 1)
        u.split = (t.width & (PPU - 1)) != 0 && row_q<ROWS>(t, lp + PPU - 1) != u.q;
    return u;
}

// Element e (channel value number e) of a unit held as 3 dwords, set to the
// element's bits.
template <int SRC>
__device__ __forceinline__ void set_elem(unsigned (&w)[3], int e, unsigned bits)
{
    if constexpr (SRC == 0) {
        const int sh = 8 * (e & 3);
        w[e >> 2] = (w[e >> 2] & ~(0xffu << sh)) | (bits << sh);
    } else if constexpr (SRC == 1) {
        const int sh = 16 * (e & 1);
        w[e >> 1] = (w[e >> 1] & ~(0xffffu << sh)) | (bits << sh);
    } else {
        w[e] = bits;
    }
}

// Loads the unit from tile-local pixel lp: one dwordx3 at its first pixel.
// A unit that a row break splits gets the same load first (its 12 bytes run
// from that pixel through the row's end and padding into the next row, all
// inside the image: a next row exists, and the row walk has W >= 4), then
// patch_unit reads each pixel past the break from the next row.
template <int SRC, bool ROWS, bool NT = true>
__device__ __forceinline__ void load_unit_at(const TileRef &t, uint32_t lp, UnitPos up,
                                             unsigned (&w)[3])
{
    load_unit<NT>(t.src + lp * (3 * elem_size(SRC)) + __umul24(up.q, t.gs), w);
}

template <int SRC, bool ROWS>
__device__ __forceinline__ void patch_unit(const TileRef &t, uint32_t lp, UnitPos up,
                                           unsigned (&w)[3])
{
    constexpr int PPU = unit_px(SRC);
    constexpr int ES = elem_size(SRC);
    if constexpr (ROWS && PPU > 1) {
        if (up.split) {
#pragma unroll
            for (int j = 1; j < PPU; ++j) {
                const uint32_t qj = row_q<ROWS>(t, lp + j);
                if (qj != up.q) {
                    const uint8_t *p = t.src + (lp + j) * (3 * ES) + __umul24(qj, t.gs);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        if constexpr (SRC == 0)
                            set_elem<SRC>(w, 3 * j + c, gp<uint8_t>(p)[c]);
                        else
                            set_elem<SRC>(w, 3 * j + c, gp<unsigned short>(p)[c]);
                    }
                }
            }
        }
    }
}

// Positions and loads of a thread's U units of a full tile, all issued before
// any arithmetic; each unit is patched (patch_unit) where it is consumed, so
// the rare reloads of split units do not hold registers across the others.
template <int SRC, int U, bool ROWS, bool NT = true>
__device__ __forceinline__ void load_units(const TileRef &t, unsigned (&w)[U][3],
                                           UnitPos (&up)[U])
{
    constexpr int PPU = unit_px(SRC);
    if constexpr (!ROWS) {
        // Packed walk (4-byte aligned tile base, which the runtime guarantees
        // for this walk): unit u of lane x lies u * kBlock + x units from the
        // tile's first byte. Buffer loads through a resource on that byte take
        // the lane offset from one register and u's offset from a scalar one,
        // so the loads cost no per-lane address arithmetic. The three dword
        // loads of a unit are merged into one dwordx3.
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc((void *)t.src, (short)0, -1, kBufferWord3);
        uint32_t off = threadIdx.x * 12u;
        asm("" : "+v"(off)); // an opaque sum, so the 4 and 8 fold into the loads' offsets
        constexpr int aux = NT ? kBufferNontemporal : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int so = u * (kBlock * 12);
            up[u] = UnitPos{0u, false};
            w[u][0] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, off, so, aux);
            w[u][1] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, off + 4u, so, aux);
            w[u][2] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, off + 8u, so, aux);
        }
        // Keeps every load above the callers' stores: the compiler may not
        // prove that a store misses the input, and a load sunk below one
        // would wait for it, and for the loads before it, one unit at a time.
        asm volatile("" ::: "memory");
        return;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        up[u] = unit_pos<PPU, ROWS>(t, slot_lp<PPU>(true, u, 0));
        load_unit_at<SRC, ROWS, NT>(t, slot_lp<PPU>(true, u, 0), up[u], w[u]);
    }
}


// Luminance of all U * PPU pixels a thread owns in a FULL tile on a vector
// walk (every slot inside the segment): all U loads are issued first. lv holds
// L in input units; up the units' positions (for the stores).
template <int SRC, int U, bool ROWS>
__device__ __forceinline__ void tile_lum_full(const TileRef &t, Coef k,
                                              float (&lv)[U * unit_px(SRC)], UnitPos (&up)[U])
{
    constexpr int PPU = unit_px(SRC);
    unsigned w[U][3];
    load_units<SRC, U, ROWS>(t, w, up);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        patch_unit<SRC, ROWS>(t, slot_lp<PPU>(true, u, 0), up[u], w[u]);
#pragma unroll
        for (int j = 0; j < PPU; ++j)
            lv[u * PPU + j] = lum<SRC>(chan<SRC>(w[u], 3 * j), chan<SRC>(w[u], 3 * j + 1),
                                       chan<SRC>(w[u], 3 * j + 2), k);
    }
}

// Stores the PPU values of the unit from tile-local pixel lp to an output
// whose tile base is `out` with row padding `gap`: one store, or pixel by
// pixel for a unit split by a row break.
template <int PPU, bool SF, bool SU, bool ROWS>
__device__ __forceinline__ void store_unit_at(const TileRef &t, uint8_t *out, uint32_t gap,
                                              int dtype, uint32_t lp, UnitPos up,
                                              const float (&v)[PPU], Enc e)
{
    if (!up.split) {
        store_unit<PPU, SF, SU>(out + __umul24(up.q, gap), dtype, lp, v, e);
        return;
    }
#pragma unroll
    for (int j = 0; j < PPU; ++j)
        store_px<SF, SU>(out + __umul24(row_q<ROWS>(t, lp + j), gap), dtype, lp + j, v[j], e);
}

// Writes the per-slot values of a full tile (laid out as tile_lum_full
// produced them) to one output.
template <int SRC, int U, bool SF, bool SU, bool ROWS>
__device__ __forceinline__ void tile_store_full(const TileRef &t, uint8_t *out, uint32_t gap,
                                                int dtype, const float (&v)[U * unit_px(SRC)],
                                                const UnitPos (&up)[U], Enc e)
{
    constexpr int PPU = unit_px(SRC);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        float vv[PPU];
#pragma unroll
        for (int j = 0; j < PPU; ++j)
            vv[j] = v[u * PPU + j];
        store_unit_at<PPU, SF, SU, ROWS>(t, out, gap, dtype, slot_lp<PPU>(true, u, 0), up[u], vv,
                                         e);
    }
}

// L (input units) of tile-local pixel p, loaded channel by channel.
template <int SRC, bool ROWS>
__device__ __forceinline__ float lum_at(const TileRef &t, uint32_t p, Coef k)
{
    float R, G_, B;
    load_px<SRC>(t.src + p * (3 * elem_size(SRC)) + __umul24(row_q<ROWS>(t, p), t.gs), R, G_, B);
    return lum<SRC>(R, G_, B, k);
}

// L (input units) of the pixel at p, loaded channel by channel.
template <int SRC>
__device__ __forceinline__ void lum_at_px(const uint8_t *p, Coef k, float &l)
{
    float R, G_, B;
    load_px<SRC>(p, R, G_, B);
    l = lum<SRC>(R, G_, B, k);
}

// Visits global tiles t0 + blockIdx.x, t0 + blockIdx.x + gridDim.x, ... below
// t1 with the index of the image that owns each, searching images img0 ..
// img0 + nimg - 1. tile_end is the inclusive prefix sum of the images' tile
// counts; tiles only grow, so the owner is found once by binary search and
// then advanced in place.
template <typename F>
__device__ __forceinline__ void for_each_tile(const int64_t *__restrict__ tile_end, int img0,
                                              int nimg, int64_t t0, int64_t t1, F &&f)
{
    int64_t tile = t0 + blockIdx.x;
    if (tile >= t1)
        return;
    int lo = img0, hi = img0 + nimg - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tile_end[mid] > tile)
            hi = mid;
        else
            lo = mid + 1;
    }
    int i = lo;
    for (; tile < t1; tile += gridDim.x) {
        while (tile_end[i] <= tile)
            ++i;
        f(i, tile);
    }
}

// ------------------------------------------------------- decolorization

// Decolorization of one tile of kBlock * U units. On a full tile every load of
// the thread's U units is issued first, then each unit is evaluated and stored
// while later loads are still in flight; a partial tile (the segment's end) and
// the per-pixel walk go pixel by pixel with bounds checks.
template <int SRC, int U, bool ROWS>
__device__ __forceinline__ void decolor_tile(const DevImage &im, int64_t tile)
{
    constexpr int PPU = unit_px(SRC);
    constexpr int64_t TILE = (int64_t)kBlock * U * PPU;
    constexpr bool SF = LumEnc<SRC>::SF, SU = LumEnc<SRC>::SU;
    const TileRef t = tile_ref(im, tile, TILE);
    const Enc e{im.unit, 255.0f};
    const Coef k = im.k;
    const bool vec = im.walk != kWalkScalar;
    if (vec && t.rem >= TILE) {
        unsigned w[U][3];
        UnitPos up[U];
        if (im.shared_src)
            load_units<SRC, U, ROWS, false>(t, w, up);
        else
            load_units<SRC, U, ROWS>(t, w, up);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            patch_unit<SRC, ROWS>(t, slot_lp<PPU>(true, u, 0), up[u], w[u]);
            float v[PPU];
#pragma unroll
            for (int j = 0; j < PPU; ++j)
                v[j] = lum<SRC>(chan<SRC>(w[u], 3 * j), chan<SRC>(w[u], 3 * j + 1),
                                chan<SRC>(w[u], 3 * j + 2), k);
            const uint32_t lp = slot_lp<PPU>(true, u, 0);
            store_unit_at<PPU, SF, SU, ROWS>(t, t.dst, t.gd, im.dst_dtype, lp, up[u], v, e);
            if (t.dst2)
                store_unit_at<PPU, SF, SU, ROWS>(t, t.dst2, t.gd2, im.dst2_dtype, lp, up[u], v, e);
        }
        return;
    }
    const uint32_t rem = (uint32_t)(t.rem < TILE ? t.rem : TILE);
#pragma unroll 1
    for (int s = 0; s < U * PPU; ++s) {
        const uint32_t p = slot_lp<PPU>(vec, s / PPU, s % PPU);
        if (p < rem) {
            const float v = lum_at<SRC, ROWS>(t, p, k);
            const uint32_t q = row_q<ROWS>(t, p);
            store_px<SF, SU>(t.dst + __umul24(q, t.gd), im.dst_dtype, p, v, e);
            if (t.dst2)
                store_px<SF, SU>(t.dst2 + __umul24(q, t.gd2), im.dst2_dtype, p, v, e);
        }
    }
}

// Kernel template argument G = 48-byte groups per thread = 4 units.
// ROWS = the image is on the row walk (a launch covers images of one kind).
template <int SRC, int G, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_decolor_single(DevImage im, int64_t ntiles)
{
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        decolor_tile<SRC, 4 * G, ROWS>(im, tile);
}

// One launch over the tiles [t0, t1) of images img0 .. img0 + nimg - 1.
// MIXED = the input element type varies per image (a uniform branch per
// tile); otherwise it is SRC. ROWS = every image of the range is on the row
// walk (the runtime sorts a table so that row-walk images form one range).
template <int SRC, int G, bool MIXED, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_decolor_table(const DevImage *__restrict__ table,
                                                          const int64_t *__restrict__ tile_end,
                                                          int img0, int nimg, int64_t t0,
                                                          int64_t t1)
{
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        const int64_t lt = tile - im.tile_begin;
        if constexpr (MIXED) {
            // Tile sizes are per image: 4G units of its own unit width.
            if (im.src_dtype == 0)
                decolor_tile<0, 4 * G, ROWS>(im, lt);
            else if (im.src_dtype == 1)
                decolor_tile<1, 4 * G, ROWS>(im, lt);
            else
                decolor_tile<2, 4 * G, ROWS>(im, lt);
        } else {
            decolor_tile<SRC, 4 * G, ROWS>(im, lt);
        }
    });
}

// ------------------------------------------------------------ weight sweep

// The weight sweep (Fig. 4's explorer): n outputs of one input, output j with
// its own (beta_R, beta_k). Every image of the table shares the input and the
// geometry of image 0 (the runtime checks this), so a thread loads its units
// once and evaluates Eqs. (1)-(6) for each pair from the same decoded pixels;
// the terms that do not depend on the weights are loop-invariant in the pair
// loop and leave it, so each further pair costs only the weight-dependent part.
// Each output is the same expression of the same inputs as a single call, so
// the results are bit-identical to dc_decolorize with that pair.
template <int SRC, int U, bool ROWS>
__device__ __forceinline__ void sweep_tile(const DevImage *__restrict__ table, int i0, int i1,
                                           int64_t tile)
{
    constexpr int PPU = unit_px(SRC);
    constexpr int ES = elem_size(SRC);
    constexpr int64_t TILE = (int64_t)kBlock * U * PPU;
    constexpr bool SF = LumEnc<SRC>::SF, SU = LumEnc<SRC>::SU;
    const DevImage im = table[0];
    const TileRef t = tile_ref(im, tile, TILE);
    const int64_t dst_off = t.dst - im.dst; // the tile's output offset, the same in every image
    const Enc e{im.unit, 255.0f};
    const bool vec = im.walk != kWalkScalar;
    if (vec && t.rem >= TILE) {
        unsigned w[U][3];
        UnitPos up[U];
        load_units<SRC, U, ROWS>(t, w, up);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            patch_unit<SRC, ROWS>(t, slot_lp<PPU>(true, u, 0), up[u], w[u]);
            float R[PPU], G[PPU], B[PPU];
#pragma unroll
            for (int j = 0; j < PPU; ++j) {
                R[j] = chan<SRC>(w[u], 3 * j);
                G[j] = chan<SRC>(w[u], 3 * j + 1);
                B[j] = chan<SRC>(w[u], 3 * j + 2);
            }
            const uint32_t lp = slot_lp<PPU>(true, u, 0);
#pragma unroll 1
            for (int i = i0; i < i1; ++i) {
                const Coef k = table[i].k;
                float v[PPU];
#pragma unroll
                for (int j = 0; j < PPU; ++j)
                    v[j] = lum<SRC>(R[j], G[j], B[j], k);
                store_unit_at<PPU, SF, SU, ROWS>(t, table[i].dst + dst_off, t.gd, im.dst_dtype, lp,
                                                 up[u], v, e);
            }
        }
        return;
    }
    const uint32_t rem = (uint32_t)(t.rem < TILE ? t.rem : TILE);
#pragma unroll 1
    for (int sl = 0; sl < U * PPU; ++sl) {
        const uint32_t p = slot_lp<PPU>(vec, sl / PPU, sl % PPU);
        if (p < rem) {
            const uint32_t q = row_q<ROWS>(t, p);
            float R, G, B;
            load_px<SRC>(t.src + p * (3 * ES) + __umul24(q, t.gs), R, G, B);
#pragma unroll 1
            for (int i = i0; i < i1; ++i)
                store_px<SF, SU>(table[i].dst + dst_off + __umul24(q, t.gd), im.dst_dtype, p,
                                 lum<SRC>(R, G, B, table[i].k), e);
        }
    }
}

// Work item w = (chunk c, tile t) with w = c * ntiles + t: pairs
// [c * per, min(n, (c + 1) * per)) of tile t. Splitting the pairs into chunks
// keeps the launch wide on small images; each chunk reads the tile again.
template <int SRC, int G, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_sweep(const DevImage *__restrict__ table, int n,
                                                  int per, int64_t ntiles, int64_t nwork)
{
    for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int64_t c = w / ntiles;
        const int i0 = (int)c * per;
        const int i1 = n - i0 < per ? n : i0 + per;
        sweep_tile<SRC, 4 * G, ROWS>(table, i0, i1, w - c * ntiles);
    }
}

// ---------------------------------------------------- comparator channels

// Gray channels the paper compares its L with, evaluated on the same data
// path (Table I's same-machine comparison, on the GPU): CH 1 = the rgb2gray
// weighted sum quoted in Sec. I, CH 2 = V of HSV, CH 3 = CIE 1976 L* / 100
// built on that Y with white Y_n = 1 (cube root as exp2(log2(y) / 3)).
// Inputs are scaled to normalised units first; float channels read as
// chan_clamp leaves them (NaN and negatives 0, past the format's ceiling the
// ceiling).
template <int SRC, int CH>
__device__ __forceinline__ float comparator_px(float R, float G, float B, float unit)
{
    if constexpr (SRC != 0) {
        R = chan_clamp(R, 0.0f, chan_max<SRC>());
        G = chan_clamp(G, 0.0f, chan_max<SRC>());
        B = chan_clamp(B, 0.0f, chan_max<SRC>());
    }
    R *= unit;
    G *= unit;
    B *= unit;
    if constexpr (CH == 2) {
        return fmaxf(R, fmaxf(G, B));
    } else {
        const float y = fmaf(0.2989f, R, fmaf(0.5870f, G, 0.1140f * B));
        if constexpr (CH == 1)
            return y;
        const float knee = 0.008856451679035631f; // (6/29)^3
        const float f = y > knee ? hw_exp2(hw_log2(y) * (1.0f / 3.0f))
                                 : fmaf(y, 7.787037037037037f, 0.13793103448275862f);
        return fmaf(1.16f, f, -0.16f);
    }
}

// One tile of a comparator channel (4 units per thread), same walks and
// encodings as the decolorization; values are already normalised.
template <int SRC, int CH, bool ROWS>
__device__ __forceinline__ void channel_tile(const DevImage &im, int64_t tile)
{
    constexpr int U = 4;
    constexpr int PPU = unit_px(SRC);
    constexpr int ES = elem_size(SRC);
    constexpr int64_t TILE = (int64_t)kBlock * U * PPU;
    const TileRef t = tile_ref(im, tile, TILE);
    const Enc e{1.0f, 255.0f};
    const bool vec = im.walk != kWalkScalar;
    if (vec && t.rem >= TILE) {
        unsigned w[U][3];
        UnitPos up[U];
        load_units<SRC, U, ROWS>(t, w, up);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            patch_unit<SRC, ROWS>(t, slot_lp<PPU>(true, u, 0), up[u], w[u]);
            float v[PPU];
#pragma unroll
            for (int j = 0; j < PPU; ++j)
                v[j] = comparator_px<SRC, CH>(chan<SRC>(w[u], 3 * j), chan<SRC>(w[u], 3 * j + 1),
                                         chan<SRC>(w[u], 3 * j + 2), im.unit);
            const uint32_t lp = slot_lp<PPU>(true, u, 0);
            store_unit_at<PPU, false, true, ROWS>(t, t.dst, t.gd, im.dst_dtype, lp, up[u], v, e);
            if (t.dst2)
                store_unit_at<PPU, false, true, ROWS>(t, t.dst2, t.gd2, im.dst2_dtype, lp, up[u], v,
                                                      e);
        }
        return;
    }
    const uint32_t rem = (uint32_t)(t.rem < TILE ? t.rem : TILE);
#pragma unroll 1
    for (int s = 0; s < U * PPU; ++s) {
        const uint32_t p = slot_lp<PPU>(vec, s / PPU, s % PPU);
        if (p < rem) {
            const uint32_t q = row_q<ROWS>(t, p);
            float R, G_, B;
            load_px<SRC>(t.src + p * (3 * ES) + __umul24(q, t.gs), R, G_, B);
            const float v = comparator_px<SRC, CH>(R, G_, B, im.unit);
            store_px<false, true>(t.dst + __umul24(q, t.gd), im.dst_dtype, p, v, e);
            if (t.dst2)
                store_px<false, true>(t.dst2 + __umul24(q, t.gd2), im.dst2_dtype, p, v, e);
        }
    }
}

template <int SRC, int CH, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_channel_table(const DevImage *__restrict__ table,
                                                          const int64_t *__restrict__ tile_end,
                                                          int img0, int nimg, int64_t t0,
                                                          int64_t t1)
{
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        channel_tile<SRC, CH, ROWS>(im, tile - im.tile_begin);
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

// Wave-wide reductions with DPP row permutes (no LDS round trip): two quad
// swaps, a half-row and a row mirror leave every lane of a 16-lane row with
// the row's result; row_bcast:15 then folds row 0 into row 1 and row 2 into
// row 3, and row_bcast:31 rows 0-1 into rows 2-3, so lane 63 holds the result
// over all 64 lanes, which readlane returns as a uniform value. Lanes of rows a
// broadcast step leaves alone take the operation's identity.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_from(int identity, int v)
{
    return __builtin_amdgcn_update_dpp(identity, v, CTRL, ROW_MASK, 0xf, false);
}
constexpr int kDppQuad1032 = 0xb1, kDppQuad2301 = 0x4e, kDppRowHalfMirror = 0x141,
              kDppRowMirror = 0x140, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

__device__ __forceinline__ float wave_sum(float v)
{
    // Rows that a broadcast step leaves alone add +0 (only lane 63 is read).
    constexpr int id = 0;
    auto add = [](float a, int b) { return a + __builtin_bit_cast(float, b); };
    v = add(v, dpp_from<kDppQuad1032>(id, __builtin_bit_cast(int, v)));
    v = add(v, dpp_from<kDppQuad2301>(id, __builtin_bit_cast(int, v)));
    v = add(v, dpp_from<kDppRowHalfMirror>(id, __builtin_bit_cast(int, v)));
    v = add(v, dpp_from<kDppRowMirror>(id, __builtin_bit_cast(int, v)));
    v = add(v, dpp_from<kDppRowBcast15, 0xa>(id, __builtin_bit_cast(int, v)));
    v = add(v, dpp_from<kDppRowBcast31, 0xc>(id, __builtin_bit_cast(int, v)));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Extremes of values that are never NaN and never -0 (luminance, or the
// infinities that stand for no pixel): for such floats the order of their bits
// as signed integers is their numeric order, so integer min / max take the
// place of the float ones (which would first quiet possible signalling NaNs).
__device__ __forceinline__ float wave_min(float v)
{
    int x = __builtin_bit_cast(int, v);
    constexpr int id = 0x7fffffff;
    x = min(x, dpp_from<kDppQuad1032>(id, x));
    x = min(x, dpp_from<kDppQuad2301>(id, x));
    x = min(x, dpp_from<kDppRowHalfMirror>(id, x));
    x = min(x, dpp_from<kDppRowMirror>(id, x));
    x = min(x, dpp_from<kDppRowBcast15, 0xa>(id, x));
    x = min(x, dpp_from<kDppRowBcast31, 0xc>(id, x));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(x, 63));
}
__device__ __forceinline__ float wave_max(float v)
{
    int x = __builtin_bit_cast(int, v);
    constexpr int id = (int)0x80000000u;
    x = max(x, dpp_from<kDppQuad1032>(id, x));
    x = max(x, dpp_from<kDppQuad2301>(id, x));
    x = max(x, dpp_from<kDppRowHalfMirror>(id, x));
    x = max(x, dpp_from<kDppRowMirror>(id, x));
    x = max(x, dpp_from<kDppRowBcast15, 0xa>(id, x));
    x = max(x, dpp_from<kDppRowBcast31, 0xc>(id, x));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(x, 63));
}

// Statistics pass over one tile of kStatsChunkPx pixels (16 per thread). Each
// wave reduces its 1024 pixels to one partial with no workgroup barrier: sums
// of d = x2 - K and d^2, shifted by K = x2 of the wave's first pixel (so a
// flat image gives exactly mean = K, M2 = 0), count and the extremes of L.
// Chunks are fixed slices of each image, so the partials, and the statistics
// merged from them in a fixed order, never depend on the other images of the
// call or on the launch shape.
template <int SRC, bool ROWS>
__device__ __forceinline__ void tm_pass1_tile(const DevImage &im, int64_t tile, TmArgs tm,
                                              WavePart *__restrict__ parts)
{
    constexpr int PPU = unit_px(SRC);
    constexpr int U = kStatsPxPerThread / PPU;
    constexpr int NV = kStatsPxPerThread;
    constexpr bool SF = LumEnc<SRC>::SF, SU = LumEnc<SRC>::SU;
    const TileRef t = tile_ref(im, tile, kStatsChunkPx);
    const Enc e{im.unit, 255.0f};
    const bool vec = im.walk != kWalkScalar;
    float K, s = 0.0f, q = 0.0f, cnt, lo = __builtin_inff(), hi = -__builtin_inff();
    const bool full = vec && t.rem >= kStatsChunkPx;
    if (full) {
        float lv[NV];
        UnitPos up[U];
        tile_lum_full<SRC, U, ROWS>(t, im.k, lv, up);
        if (t.dst2)
            tile_store_full<SRC, U, SF, SU, ROWS>(t, t.dst2, t.gd2, im.dst2_dtype, lv, up, e);
        float x[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            x[i] = xlog2(lv[i], im.unit, tm.eps);
        K = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x[0])));
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const float d = x[i] - K;
            s += d;
            q = fmaf(d, d, q);
            lo = fminf(lo, lv[i]);
            hi = fmaxf(hi, lv[i]);
        }
        cnt = (float)NV;
    } else {
        // Partial tile or per-pixel walk: one pixel at a time. Slot 0 of lane
        // 0 is the wave's first pixel, valid whenever any pixel of the wave is.
        const uint32_t rem = (uint32_t)(t.rem < kStatsChunkPx ? t.rem : kStatsChunkPx);
        const uint32_t p0 = slot_lp<PPU>(vec, 0, 0);
        const float l0 = p0 < rem ? lum_at<SRC, ROWS>(t, p0, im.k) : 0.0f;
        K = __builtin_bit_cast(
            float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, xlog2(l0, im.unit, tm.eps))));
        cnt = 0.0f;
#pragma unroll 1
        for (int i = 0; i < NV; ++i) {
            const uint32_t p = slot_lp<PPU>(vec, i / PPU, i % PPU);
            if (p < rem) {
                const float l = lum_at<SRC, ROWS>(t, p, im.k);
                if (t.dst2)
                    store_px<SF, SU>(t.dst2 + __umul24(row_q<ROWS>(t, p), t.gd2), im.dst2_dtype, p, l, e);
                const float d = xlog2(l, im.unit, tm.eps) - K;
                s += d;
                q = fmaf(d, d, q);
                lo = fminf(lo, l);
                hi = fmaxf(hi, l);
                cnt += 1.0f;
            }
        }
    }
    s = wave_sum(s);
    q = wave_sum(q);
    const float n = full ? (float)(64 * NV) : wave_sum(cnt); // a full tile fills every lane
    lo = wave_min(lo + 0.0f); // + 0 turns a -0 into +0
    hi = wave_max(hi + 0.0f);
    if ((threadIdx.x & 63) == 0)
        parts[im.chunk_begin + tile * kWavesPerBlock + (threadIdx.x >> 6)] =
            WavePart{n, K, s, q, lo, hi};
}

// Tone-map kernels cover tiles [t0, t1) of images img0 .. img0 + nimg - 1, so
// one launch can span every image of a call or a single image. MIXED = the
// input element type varies per image; otherwise it is SRC (one instantiation
// per type keeps the register count of the uniform case low).
template <int SRC, bool MIXED, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_tm_pass1(const DevImage *__restrict__ table,
                                                     const int64_t *__restrict__ tile_end,
                                                     int img0, int nimg, int64_t t0, int64_t t1,
                                                     TmArgs tm, WavePart *__restrict__ parts)
{
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        const int64_t lt = tile - im.tile_begin;
        if constexpr (MIXED) {
            if (im.src_dtype == 0)
                tm_pass1_tile<0, ROWS>(im, lt, tm, parts);
            else if (im.src_dtype == 1)
                tm_pass1_tile<1, ROWS>(im, lt, tm, parts);
            else
                tm_pass1_tile<2, ROWS>(im, lt, tm, parts);
        } else {
            tm_pass1_tile<SRC, ROWS>(im, lt, tm, parts);
        }
    });
}

// The binary16 statistics pass of uniform batches off the row walk, held to 80 VGPRs: its body
// fits them without spilling, and the sixth wave per SIMD that this allows
// hides more of the load latency (about 3 % faster on MI355X; the other
// instantiations would spill under the same limit).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_tm_pass1_f16(
    const DevImage *__restrict__ table, const int64_t *__restrict__ tile_end, int img0, int nimg,
    int64_t t0, int64_t t1, TmArgs tm, WavePart *__restrict__ parts)
{
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        tm_pass1_tile<1, false>(im, tile - im.tile_begin, tm, parts);
    });
}

// A wave's raw partial as a Part: mean = K + s / n, m2 = q - s (s / n)
// (never below 0), extremes in Lhat units.
__device__ __forceinline__ Part part_of(const WavePart &w, float unit)
{
    if (!(w.n > 0.0f))
        return part_empty();
    const float m = w.s / w.n;
    return Part{w.n, w.K + m, fmaxf(fmaf(-w.s, m, w.q), 0.0f), w.lo * unit, w.hi * unit};
}

// Level 1 of the statistics combine for group g (global numbering) of image
// im: the workgroup merges the fixed group of up to kBlock consecutive wave
// partials g - grp_begin of the image (one per thread, loaded in parallel) with
// a fixed LDS tree, and thread 0 writes one group partial. Every thread of the
// workgroup takes part; sh is kBlock entries of LDS.
// DEVICE = the group partial is read by another workgroup of this launch:
// it is stored field by field at device scope (written through to the point
// where every L2 of the chip sees it).
template <bool DEVICE = false>
__device__ __forceinline__ void combine_group(const DevImage &im, int64_t g,
                                              const WavePart *__restrict__ parts,
                                              Part *__restrict__ parts2, Part *sh)
{
    const int64_t nparts = im.ntiles * kWavesPerBlock;
    const int64_t c = (g - im.grp_begin) * kBlock + threadIdx.x;
    const int tid = threadIdx.x;
    sh[tid] = c < nparts ? part_of(parts[im.chunk_begin + c], im.unit) : part_empty();
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (tid < s)
            sh[tid] = merge(sh[tid], sh[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        if constexpr (DEVICE) {
            float *f = &parts2[g].n;
            const Part r = sh[0];
            __hip_atomic_store(f + 0, r.n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(f + 1, r.mean, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(f + 2, r.m2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(f + 3, r.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(f + 4, r.hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            parts2[g] = sh[0];
        }
    }
}

// Level 1 as a kernel: block g merges group g0 + g.
__global__ __launch_bounds__(kBlock) void k_tm_combine(const DevImage *__restrict__ table,
                                                       const int64_t *__restrict__ grp_end,
                                                       int img0, int nimg, int64_t g0,
                                                       const WavePart *__restrict__ parts,
                                                       Part *__restrict__ parts2)
{
    __shared__ Part sh[kBlock];
    const int64_t g = g0 + blockIdx.x;
    int lo = img0, hi = img0 + nimg - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (grp_end[mid] > g)
            hi = mid;
        else
            lo = mid + 1;
    }
    const DevImage im = table[lo];
    combine_group(im, g, parts, parts2, sh);
}

// Level 2 for image number img of the table: the workgroup merges the image's
// group partials in a fixed order, then thread 0 writes the curve
// coefficients (and, when asked, the statistics for the caller). Every thread
// takes part; sh is kBlock entries of LDS.
// A group partial written by another workgroup of the same launch, read
// field by field at device scope (coherent across the chip's L2s).
__device__ __forceinline__ Part load_part_device(const Part *p)
{
    const float *f = &p->n;
    Part r;
    r.n = __hip_atomic_load(f + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r.mean = __hip_atomic_load(f + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r.m2 = __hip_atomic_load(f + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r.lo = __hip_atomic_load(f + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r.hi = __hip_atomic_load(f + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return r;
}

// DEVICE = the group partials come from other workgroups of this launch.
template <bool DEVICE = false>
__device__ __forceinline__ void finalize_image(const DevImage &im, int img, TmArgs tm,
                                              const Part *__restrict__ parts2,
                                              Curve *__restrict__ curves,
                                              StatsOut *__restrict__ stats, Part *sh)
{
    const int tid = threadIdx.x;
    Part a = part_empty();
    for (int64_t c = tid; c < im.ngrp; c += kBlock)
        a = merge(a, DEVICE ? load_part_device(&parts2[im.grp_begin + c])
                            : parts2[im.grp_begin + c]);
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
            // The table may be reordered by input type; stats follow the
            // caller's image order.
            StatsOut o;
            o.log_mean = tot.mean * ln2;
            o.log_std = sigma2 * ln2;
            o.l_min = tot.lo;
            o.l_max = tot.hi;
            o.count = im.npx;
            stats[im.image] = o;
        }
    }
}

// Level 2 as a kernel: one workgroup per image, images img0 + blockIdx.x.
__global__ __launch_bounds__(kBlock) void k_tm_finalize(const DevImage *__restrict__ table,
                                                        int img0, TmArgs tm,
                                                        const Part *__restrict__ parts2,
                                                        Curve *__restrict__ curves,
                                                        StatsOut *__restrict__ stats)
{
    __shared__ Part sh[kBlock];
    const int img = img0 + blockIdx.x;
    const DevImage im = table[img];
    finalize_image(im, img, tm, parts2, curves, stats, sh);
}

// Both levels of the combine in one launch: block g0 + blockIdx.x merges its
// group (level 1, as k_tm_combine) and publishes the group partial, and the
// block that completes an image's groups merges them (level 2, as
// k_tm_finalize) and resets the image's counter to 0 for the next use. The
// merge trees are those of the two-kernel form, so the results are the same
// bits; counters holds one word per table image, zero when the launch starts.
// Publication: the partial is stored at device scope (its stores written
// through), the workgroup waits until those stores have completed, and only
// then counts its group with a device-scope atomic; the last counter reads the
// partials with device-scope loads after that atomic has returned. No L2
// write-back is needed, since nothing else of this launch is read across
// workgroups (a release fence per workgroup, which writes the L2 back, costs
// ~20 us over the 1024 groups of 16 x 4096^2 images).
__global__ __launch_bounds__(kBlock) void k_tm_combine_finalize(
    const DevImage *__restrict__ table, const int64_t *__restrict__ grp_end, int img0, int nimg,
    int64_t g0, TmArgs tm, const WavePart *__restrict__ parts, Part *__restrict__ parts2,
    unsigned *__restrict__ counters, Curve *__restrict__ curves, StatsOut *__restrict__ stats)
{
    __shared__ Part sh[kBlock];
    __shared__ int last;
    const int64_t g = g0 + blockIdx.x;
    int lo = img0, hi = img0 + nimg - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (grp_end[mid] > g)
            hi = mid;
        else
            lo = mid + 1;
    }
    const DevImage im = table[lo];
    combine_group<true>(im, g, parts, parts2, sh);
    if (threadIdx.x == 0) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0); // the partial's stores have completed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        last = __hip_atomic_fetch_add(&counters[lo], 1u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) == (unsigned)(im.ngrp - 1);
    }
    __syncthreads();
    if (!last)
        return;
    finalize_image<true>(im, lo, tm, parts2, curves, stats, sh);
    if (threadIdx.x == 0)
        counters[lo] = 0u;
}

// T = 1 / (1 + exp2(a (x2 - mu2))) of one pixel.
__device__ __forceinline__ float curve(float l, float unit, TmArgs tm, Curve cv)
{
    return hw_rcp(1.0f + hw_exp2(cv.a * (xlog2(l, unit, tm.eps) - cv.mu2)));
}

template <int SRC, bool ROWS>
__device__ __forceinline__ void tm_pass2_tile(const DevImage &im, int64_t tile, TmArgs tm, Curve cv)
{
    constexpr int PPU = unit_px(SRC);
    constexpr int U = kStatsPxPerThread / PPU;
    constexpr int NV = kStatsPxPerThread;
    const TileRef t = tile_ref(im, tile, kStatsChunkPx);
    const Enc e{1.0f, 255.0f};
    const bool vec = im.walk != kWalkScalar;
    if (vec && t.rem >= kStatsChunkPx) {
        float lv[NV];
        UnitPos up[U];
        tile_lum_full<SRC, U, ROWS>(t, im.k, lv, up);
#pragma unroll
        for (int i = 0; i < NV; ++i)
            lv[i] = curve(lv[i], im.unit, tm, cv);
        tile_store_full<SRC, U, false, true, ROWS>(t, t.dst, t.gd, im.dst_dtype, lv, up, e);
        return;
    }
    const uint32_t rem = (uint32_t)(t.rem < kStatsChunkPx ? t.rem : kStatsChunkPx);
#pragma unroll 1
    for (int i = 0; i < NV; ++i) {
        const uint32_t p = slot_lp<PPU>(vec, i / PPU, i % PPU);
        if (p < rem)
            store_px<false, true>(t.dst + __umul24(row_q<ROWS>(t, p), t.gd), im.dst_dtype, p,
                                  curve(lum_at<SRC, ROWS>(t, p, im.k), im.unit, tm, cv), e);
    }
}

template <int SRC, bool MIXED, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_tm_pass2(const DevImage *__restrict__ table,
                                                     const int64_t *__restrict__ tile_end,
                                                     int img0, int nimg, int64_t t0, int64_t t1,
                                                     TmArgs tm, const Curve *__restrict__ curves)
{
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        const Curve cv = curves[i];
        const int64_t lt = tile - im.tile_begin;
        if constexpr (MIXED) {
            if (im.src_dtype == 0)
                tm_pass2_tile<0, ROWS>(im, lt, tm, cv);
            else if (im.src_dtype == 1)
                tm_pass2_tile<1, ROWS>(im, lt, tm, cv);
            else
                tm_pass2_tile<2, ROWS>(im, lt, tm, cv);
        } else {
            tm_pass2_tile<SRC, ROWS>(im, lt, tm, cv);
        }
    });
}

// ------------------------------------------------- colour re-synthesis

// Colour output of the tone map for one pixel: every channel C becomes
// T (C / L)^s, clamped to at most 1, with C and L in the input's units (their
// ratio is unit-free); E is the curve's exponential, T = 1 / (1 + E). A pixel
// with no colour to carry (L at most 1e-6 S: black, or the degenerate weights
// 0) becomes grey T; the 8-bit form's L of a black pixel is about 1e-7 (its
// tiny addends), hence the extra 1e-6 there. The ratio is formed first, so its
// logarithm stays small for ordinary colours and the power is accurate:
//   kColourGrey  (s = 0): T everywhere;
//   kColourRatio (s = 1): C k + g, k = T / L and g = 0, or k = 0 and g = T for
//                         a grey pixel (one reciprocal for T and 1/L together);
//   kColourPow   (other s): exp2(s log2(C / L + g) + log2 T) with 1/L taken as
//                         0 and g = 1 for a grey pixel (ratio 1, so T), g = 0
//                         otherwise; log2 T = -log2(1 + E), finite where T
//                         underflows.
// U8: the values are wanted as 8-bit codes, so they come out times 255 (folded
// into k, or into the exponent as log2 255) and the saturating 8-bit
// conversion does the clamp at 255; other outputs are clamped at 1 here.
// Whether a pixel has no colour to carry (the grey case of colour_px), from
// the raw channels and its L.
template <int SRC>
__device__ __forceinline__ bool colour_grey(float R, float G, float B, float l)
{
    if constexpr (SRC != 0) {
        R = chan_clamp(R, 0.0f, chan_max<SRC>());
        G = chan_clamp(G, 0.0f, chan_max<SRC>());
        B = chan_clamp(B, 0.0f, chan_max<SRC>());
    }
    const float S = (R + G) + B;
    return !(l > fmaf(S, 1e-6f, SRC == 0 ? 1e-6f : 0.0f));
}

// ANYGREY = false: the caller has found that no pixel of this unit, in any
// lane of the wave, is grey, so the selects between the grey and the coloured
// form are left out; the coloured form's values are the same bits either way.
template <int SRC, int MODE, bool U8, bool ANYGREY = true>
__device__ __forceinline__ void colour_px(float R, float G, float B, float l, float E, float s,
                                          float *o)
{
    constexpr float kOut = U8 ? 255.0f : 1.0f;
    if constexpr (MODE == kColourGrey) {
        o[0] = o[1] = o[2] = hw_rcp(1.0f + E) * kOut;
        return;
    }
    const bool grey = ANYGREY && colour_grey<SRC>(R, G, B, l);
    if constexpr (SRC != 0) {
        R = chan_clamp(R, 0.0f, chan_max<SRC>());
        G = chan_clamp(G, 0.0f, chan_max<SRC>());
        B = chan_clamp(B, 0.0f, chan_max<SRC>());
    }
    const float C[3] = {R, G, B};
    if constexpr (MODE == kColourRatio) {
        const float lc = fmaxf(l, 1e-30f);
        const float k = hw_rcp((1.0f + E) * lc);
        const float ko = grey ? 0.0f : k * kOut;
        const float g = grey ? k * lc * kOut : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float v = fmaf(C[c], ko, g);
            o[c] = U8 ? v : fminf(v, 1.0f);
        }
    } else {
        constexpr float kLogOut = U8 ? 7.99435343685885793f : 0.0f; // log2(255)
        const float lT = kLogOut - hw_log2(1.0f + E);
        const float il = grey ? 0.0f : hw_rcp(l);
        const float g = grey ? 1.0f : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = fmaf(s, hw_log2(fmaf(C[c], il, g)), lT);
            o[c] = hw_exp2(U8 ? e : fminf(e, 0.0f));
        }
    }
}

// Stores the 3 * PPU channel values of one unit (PPU pixels) at pixel lp of
// an interleaved RGB row whose pixel 0 is at base (any element alignment; the
// target serves unaligned dword accesses). 8-bit values arrive times 255 and
// are converted by the saturating v_cvt_pk_u8_f32.
template <int PPU>
__device__ __forceinline__ void store_rgb_unit(uint8_t *base, int dtype, uint32_t lp,
                                               const float (&o)[3 * PPU])
{
    if (dtype == 0) {
        uint8_t *p = base + 3 * lp;
        if constexpr (PPU == 4) {
            unsigned w[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                w[j] = 0u;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    w[j] = u8_of<false>(o[4 * j + i], 1.0f, i, w[j]);
            }
            auto *q = gpw<unsigned>(p);
            put(&q[0], w[0]);
            put(&q[1], w[1]);
            put(&q[2], w[2]);
        } else if constexpr (PPU == 2) {
            auto *q = gpw<unsigned short>(p);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                put(&q[j], (unsigned short)u8_of<false>(o[2 * j + 1], 1.0f, 1,
                                                        u8_of<false>(o[2 * j], 1.0f, 0, 0u)));
        } else {
            auto *q = gpw<uint8_t>(p);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                put(&q[j], (uint8_t)u8_of<false>(o[j], 1.0f, 0, 0u));
        }
    } else if (dtype == 1) {
        uint8_t *p = base + 6 * lp;
        if constexpr (PPU == 4) {
            auto *q = gpw<u32x2>(p);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                put(&q[j], u32x2{pack_f16x2(o[4 * j], o[4 * j + 1]),
                                 pack_f16x2(o[4 * j + 2], o[4 * j + 3])});
        } else if constexpr (PPU == 2) {
            auto *q = gpw<unsigned>(p);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                put(&q[j], pack_f16x2(o[2 * j], o[2 * j + 1]));
        } else {
            auto *q = gpw<_Float16>(p);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                put(&q[j], (_Float16)o[j]);
        }
    } else {
        uint8_t *p = base + 12 * lp;
        unsigned b[3 * PPU];
#pragma unroll
        for (int i = 0; i < 3 * PPU; ++i)
            b[i] = __builtin_bit_cast(unsigned, o[i]);
        if constexpr (PPU == 4) {
            auto *q = gpw<u32x4>(p);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                put(&q[j], u32x4{b[4 * j], b[4 * j + 1], b[4 * j + 2], b[4 * j + 3]});
        } else if constexpr (PPU == 2) {
            auto *q = gpw<u32x2>(p);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                put(&q[j], u32x2{b[2 * j], b[2 * j + 1]});
        } else {
            auto *q = gpw<unsigned>(p);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                put(&q[j], b[j]);
        }
    }
}

// Colour curve pass with 8-bit RGB output over a full packed tile of binary16
// input, each lane taking two adjacent units (4 pixels): their 12 bytes of
// RGB codes go out in one dwordx3, so every store instruction of a wave
// writes 768 contiguous bytes and no line leaves L2 partly written (a lane's
// single unit has 6 bytes of output, which took a dword and a short store
// whose lines the two instructions each covered only in part). Loads: the
// pair's 24 bytes as buffer loads from the tile's first byte (the packed
// walk's 4-byte aligned base). Per pixel, the same expressions as the unit
// form, so the same bits.
template <int SRC, int MODE>
__device__ __forceinline__ void tm_colour_pairs(const DevImage &im, const TileRef &t, TmArgs tm,
                                                Curve cv)
{
    constexpr int NP = kStatsPxPerThread / 4; // pairs of units per lane
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void *)t.src, (short)0, -1, kBufferWord3);
    uint32_t off = threadIdx.x * 24u;
    asm("" : "+v"(off)); // an opaque sum, so the constant offsets fold into the loads
    unsigned w[NP][2][3];
#pragma unroll
    for (int v = 0; v < NP; ++v) {
        const int so = v * (kBlock * 24);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                w[v][h][c] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(
                    r, off + 12u * h + 4u * c, so, kBufferNontemporal);
    }
    asm volatile("" ::: "memory"); // loads stay above the stores that follow
#pragma unroll
    for (int v = 0; v < NP; ++v) {
        float o[12], l[4], E[4];
        bool grey = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned(&u)[3] = w[v][j >> 1];
            const int b = 3 * (j & 1);
            const float R = chan<SRC>(u, b), G = chan<SRC>(u, b + 1), B = chan<SRC>(u, b + 2);
            l[j] = lum<SRC>(R, G, B, im.k);
            E[j] = hw_exp2(cv.a * (xlog2(l[j], im.unit, tm.eps) - cv.mu2));
            grey = grey || colour_grey<SRC>(R, G, B, l[j]);
        }
        if (MODE == kColourGrey || __builtin_amdgcn_ballot_w64(grey) == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const unsigned(&u)[3] = w[v][j >> 1];
                const int b = 3 * (j & 1);
                colour_px<SRC, MODE, true, false>(chan<SRC>(u, b), chan<SRC>(u, b + 1),
                                                  chan<SRC>(u, b + 2), l[j], E[j],
                                                  tm.saturation, &o[3 * j]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const unsigned(&u)[3] = w[v][j >> 1];
                const int b = 3 * (j & 1);
                colour_px<SRC, MODE, true, true>(chan<SRC>(u, b), chan<SRC>(u, b + 1),
                                                 chan<SRC>(u, b + 2), l[j], E[j], tm.saturation,
                                                 &o[3 * j]);
            }
        }
        store_rgb_unit<4>(t.dst, 0, (uint32_t)(v * kBlock + threadIdx.x) * 4u, o);
    }
}

// Curve pass with colour output over one statistics tile: the same units,
// tiles and curve as tm_pass2_tile, and 3 output channels per pixel. U8 =
// the image's dst is 8-bit (a uniform choice per image).
template <int SRC, int MODE, bool U8, bool ROWS>
__device__ __forceinline__ void tm_colour_tile(const DevImage &im, int64_t tile, TmArgs tm,
                                               Curve cv)
{
    constexpr int PPU = unit_px(SRC);
    constexpr int U = kStatsPxPerThread / PPU;
    constexpr int ES = elem_size(SRC);
    const TileRef t = tile_ref<3>(im, tile, kStatsChunkPx);
    const Enc e{1.0f, 1.0f};
    const int dt = U8 ? 0 : im.dst_dtype;
    const bool vec = im.walk != kWalkScalar;
    if constexpr (U8 && PPU == 2 && !ROWS) {
        if (vec && t.rem >= kStatsChunkPx) {
            tm_colour_pairs<SRC, MODE>(im, t, tm, cv);
            return;
        }
    }
    if (vec && t.rem >= kStatsChunkPx) {
        unsigned w[U][3];
        UnitPos up[U];
        load_units<SRC, U, ROWS>(t, w, up);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            patch_unit<SRC, ROWS>(t, slot_lp<PPU>(true, u, 0), up[u], w[u]);
            float o[3 * PPU], l[PPU], E[PPU];
            bool grey = false;
#pragma unroll
            for (int j = 0; j < PPU; ++j) {
                const float R = chan<SRC>(w[u], 3 * j), G = chan<SRC>(w[u], 3 * j + 1),
                            B = chan<SRC>(w[u], 3 * j + 2);
                l[j] = lum<SRC>(R, G, B, im.k);
                E[j] = hw_exp2(cv.a * (xlog2(l[j], im.unit, tm.eps) - cv.mu2));
                grey = grey || colour_grey<SRC>(R, G, B, l[j]);
            }
            // A grey pixel (black, mostly) anywhere in the wave's unit takes the
            // form with the grey selects; other units skip them.
            if (MODE == kColourGrey || __builtin_amdgcn_ballot_w64(grey) == 0) {
#pragma unroll
                for (int j = 0; j < PPU; ++j)
                    colour_px<SRC, MODE, U8, false>(chan<SRC>(w[u], 3 * j),
                                                    chan<SRC>(w[u], 3 * j + 1),
                                                    chan<SRC>(w[u], 3 * j + 2), l[j], E[j],
                                                    tm.saturation, &o[3 * j]);
            } else {
#pragma unroll
                for (int j = 0; j < PPU; ++j)
                    colour_px<SRC, MODE, U8, true>(chan<SRC>(w[u], 3 * j),
                                                   chan<SRC>(w[u], 3 * j + 1),
                                                   chan<SRC>(w[u], 3 * j + 2), l[j], E[j],
                                                   tm.saturation, &o[3 * j]);
            }
            const uint32_t lp = slot_lp<PPU>(true, u, 0);
            if (!up[u].split) {
                store_rgb_unit<PPU>(t.dst + __umul24(up[u].q, t.gd), dt, lp, o);
            } else {
                // a unit split by a row break: each pixel into its own row
#pragma unroll
                for (int j = 0; j < PPU; ++j)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        store_px<false, false>(t.dst + __umul24(row_q<ROWS>(t, lp + j), t.gd), dt,
                                               3 * (lp + j) + c, o[3 * j + c], e);
            }
        }
        return;
    }
    const uint32_t rem = (uint32_t)(t.rem < kStatsChunkPx ? t.rem : kStatsChunkPx);
#pragma unroll 1
    for (int i = 0; i < kStatsPxPerThread; ++i) {
        const uint32_t p = slot_lp<PPU>(vec, i / PPU, i % PPU);
        if (p < rem) {
            const uint32_t q = row_q<ROWS>(t, p);
            float R, G, B;
            load_px<SRC>(t.src + p * (3 * ES) + __umul24(q, t.gs), R, G, B);
            const float l = lum<SRC>(R, G, B, im.k);
            const float E = hw_exp2(cv.a * (xlog2(l, im.unit, tm.eps) - cv.mu2));
            float o[3];
            colour_px<SRC, MODE, U8>(R, G, B, l, E, tm.saturation, o);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                store_px<false, false>(t.dst + __umul24(q, t.gd), dt, 3 * p + c, o[c], e);
        }
    }
}

template <int SRC, int MODE, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_tm_colour(const DevImage *__restrict__ table,
                                                      const int64_t *__restrict__ tile_end,
                                                      int img0, int nimg, int64_t t0, int64_t t1,
                                                      TmArgs tm, const Curve *__restrict__ curves)
{
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        if (im.dst_dtype == 0)
            tm_colour_tile<SRC, MODE, true, ROWS>(im, tile - im.tile_begin, tm, curves[i]);
        else
            tm_colour_tile<SRC, MODE, false, ROWS>(im, tile - im.tile_begin, tm, curves[i]);
    });
}

// ----------------------------------------------------- local tone map

// The local tone map (Sec. III-B.2, smoothed local histogram equalisation)
// walks each image in square tiles of kLtmTile x kLtmTile pixels, one tile per
// workgroup visit: 64 rows of 64 / PPU work units. Thread t, pass i takes row
// i * (kBlock / UPR) + t / UPR and unit t % UPR of it (UPR = units per tile
// row), so a wave's lanes cover whole row segments and slot 0 of lane 0 is
// the wave's first pixel in the tile; each row segment of a pass is contiguous
// in memory.
struct LtmRef {
    const uint8_t *src; // tile's pixel (0, 0)
    uint8_t *dst;
    uint8_t *dst2;
    int64_t sp, dp, d2p; // row pitches
    int bw, bh;          // tile width and height inside the image
    int tx, ty, nx, ny;  // tile coordinates and grid size
    bool vec;            // full-width tile on a 16-byte aligned walk
};

__device__ __forceinline__ LtmRef ltm_ref(const DevImage &im, int64_t tile)
{
    LtmRef r;
    r.nx = (int)im.tiles_per_seg;
    r.ny = (int)(im.ntiles / im.tiles_per_seg);
    r.ty = (int)(tile / r.nx);
    r.tx = (int)(tile - (int64_t)r.ty * r.nx);
    const int64_t x0 = (int64_t)r.tx * kLtmTile, y0 = (int64_t)r.ty * kLtmTile;
    r.bw = (int)min((int64_t)kLtmTile, (int64_t)im.width - x0);
    r.bh = (int)min((int64_t)kLtmTile, (int64_t)im.height - y0);
    r.sp = im.src_seg_stride;
    r.dp = im.dst_seg_stride;
    r.d2p = im.dst2_seg_stride;
    r.src = im.src + y0 * r.sp + x0 * 3 * elem_size(im.src_dtype);
    r.dst = im.dst + y0 * r.dp + x0 * elem_size(im.dst_dtype);
    r.dst2 = im.dst2 ? im.dst2 + y0 * r.d2p + x0 * elem_size(im.dst2_dtype) : nullptr;
    r.vec = im.walk != kWalkScalar && r.bw == kLtmTile;
    return r;
}

// Row and first column (within the tile) of slot (pass i, unit pixel q).
template <int PPU>
__device__ __forceinline__ void ltm_slot(int i, int q, int &row, int &col)
{
    constexpr int UPR = kLtmTile / PPU;
    constexpr int RPP = kBlock / UPR;
    const int t = threadIdx.x;
    row = i * RPP + t / UPR;
    col = (t % UPR) * PPU + q;
}

// Bin position u of x2 = log2(Lhat + eps): 2 bins per stop, bin centres at
// integers, bin 0 centred half a bin above log2(eps), so u = 2 (x2 - lo2) -
// 0.5 with lo2 = log2(eps); u0 = -(2 lo2 + 0.5) is the per-tile constant of
// ltm_u0. u is clamped to [0, kLtmBins - 1), just below the last centre, so
// its bin k = floor(u) <= kLtmBins - 2 and fraction f = u - k come from one
// conversion and one fract; the clamp moves a pixel past the last centre by
// less than 2^-18 of a bin.
__device__ __forceinline__ float ltm_u0(float lo2) { return -fmaf(2.0f, lo2, 0.5f); }
__device__ __forceinline__ float ltm_u(float x2, float u0)
{
    const float u = fmaf(2.0f, x2, u0);
    return fminf(fmaxf(u, 0.0f), 0x1.f7fffcp+5f); // 63 - 2^-18
}
__device__ __forceinline__ int ltm_bin(float u) { return (int)u; }
__device__ __forceinline__ float ltm_frac(float u) { return __builtin_amdgcn_fractf(u); }

// Statistics pass of the local tone map over one tile: the global statistics
// partial of each wave (as tm_pass1_tile) and the tile's soft histogram of u
// (mass 1 - f to bin k, f to bin k + 1, in units of 2^-19, integer LDS atomics,
// so the histogram does not depend on the order of the adds). When the image's
// output is FP32 the pass also parks x2 = log2(Lhat + eps) there, for the
// curve pass to read instead of the input (im.staged).
template <int SRC>
__device__ __forceinline__ void ltm_pass1_tile(const DevImage &im, int64_t tile, TmArgs tm,
                                               WavePart *__restrict__ parts,
                                               unsigned *__restrict__ hist, unsigned *lds_hist)
{
    constexpr int PPU = unit_px(SRC);
    constexpr int U = kStatsPxPerThread / PPU;
    constexpr int ES = elem_size(SRC);
    constexpr bool SF = LumEnc<SRC>::SF, SU = LumEnc<SRC>::SU;
    const LtmRef r = ltm_ref(im, tile);
    const Enc e{im.unit, 255.0f};
    const float u0 = ltm_u0(hw_log2(tm.eps));
    if (threadIdx.x < kLtmBins)
        lds_hist[threadIdx.x] = 0u;
    __syncthreads();
    float K = 0.0f, s = 0.0f, q = 0.0f, cnt = 0.0f, lo = __builtin_inff(), hi = -__builtin_inff();
    {
        int row0, col0;
        ltm_slot<PPU>(0, 0, row0, col0);
        float l0 = 0.0f;
        if (row0 < r.bh && col0 < r.bw)
            lum_at_px<SRC>(r.src + row0 * r.sp + col0 * 3 * ES, im.k, l0);
        K = __builtin_bit_cast(
            float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, xlog2(l0, im.unit, tm.eps))));
    }
    const bool staged = im.staged != 0;
    // one pixel into the statistics and the histogram (the caller counts it)
    auto add = [&](float l) {
        const float x2 = xlog2(l, im.unit, tm.eps);
        const float d = x2 - K;
        s += d;
        q = fmaf(d, d, q);
        lo = fminf(lo, l);
        hi = fmaxf(hi, l);
        const float u = ltm_u(x2, u0);
        const int k = ltm_bin(u);
        const unsigned whi = (unsigned)fmaf(ltm_frac(u), (float)kLtmOne, 0.5f);
        atomicAdd(&lds_hist[k], kLtmOne - whi);
        atomicAdd(&lds_hist[k + 1], whi);
        return x2;
    };
    if (r.vec) {
        // all of the thread's unit loads first, then the arithmetic
        // rows past the image's end (bottom tiles) load the last row again, so
        // every load is unconditional and all of them are in flight together
        unsigned w[U][3];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int row, col;
            ltm_slot<PPU>(i, 0, row, col);
            load_unit(r.src + min(row, r.bh - 1) * r.sp + col * 3 * ES, w[i]);
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int row, col;
            ltm_slot<PPU>(i, 0, row, col);
            if (row < r.bh) {
                float v[PPU], x[PPU];
#pragma unroll
                for (int j = 0; j < PPU; ++j) {
                    v[j] = lum<SRC>(chan<SRC>(w[i], 3 * j), chan<SRC>(w[i], 3 * j + 1),
                                    chan<SRC>(w[i], 3 * j + 2), im.k);
                    x[j] = add(v[j]);
                }
                cnt += (float)PPU;
                if (r.dst2)
                    store_unit<PPU, SF, SU>(r.dst2 + row * r.d2p, im.dst2_dtype, col, v, e);
                if (staged)
                    store_unit<PPU, false, false>(r.dst + row * r.dp, 2, col, x, e);
            }
        }
    } else {
#pragma unroll 1
        for (int sl = 0; sl < kStatsPxPerThread; ++sl) {
            int row, col;
            ltm_slot<PPU>(sl / PPU, sl % PPU, row, col);
            if (row < r.bh && col < r.bw) {
                float l;
                lum_at_px<SRC>(r.src + row * r.sp + col * 3 * ES, im.k, l);
                const float x2 = add(l);
                cnt += 1.0f;
                if (r.dst2)
                    store_px<SF, SU>(r.dst2 + row * r.d2p, im.dst2_dtype, col, l, e);
                if (staged)
                    store_px<false, false>(r.dst + row * r.dp, 2, col, x2, e);
            }
        }
    }
    s = wave_sum(s);
    q = wave_sum(q);
    const float n = wave_sum(cnt);
    lo = wave_min(lo + 0.0f); // + 0 turns a -0 into +0
    hi = wave_max(hi + 0.0f);
    if ((threadIdx.x & 63) == 0)
        parts[im.chunk_begin + tile * kWavesPerBlock + (threadIdx.x >> 6)] =
            WavePart{n, K, s, q, lo, hi};
    __syncthreads();
    if (threadIdx.x < kLtmBins)
        hist[(im.tile_begin + tile) * kLtmBins + threadIdx.x] = lds_hist[threadIdx.x];
    __syncthreads();
}

template <int SRC>
__global__ __launch_bounds__(kBlock) void k_ltm_pass1(const DevImage *__restrict__ table,
                                                      const int64_t *__restrict__ tile_end,
                                                      int img0, int nimg, int64_t t0, int64_t t1,
                                                      TmArgs tm, WavePart *__restrict__ parts,
                                                      unsigned *__restrict__ hist)
{
    __shared__ unsigned lds_hist[kLtmBins];
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        ltm_pass1_tile<SRC>(im, tile - im.tile_begin, tm, parts, hist, lds_hist);
    });
}

// Per tile: the 3 x 3 smoothing of the neighbouring tiles' histograms with
// weights (1, 2, 1) x (1, 2, 1) (tiles outside the grid left out), the prefix
// sums over the bins, and the quadratic of each bin interval,
//   F(k + f) = [P(k) + H(k)/2 + H(k) f + (H(k+1) - H(k)) f^2 / 2] / M,
// which is the triangle-smoothed cumulative distribution exactly. One wave per
// tile, lane b = bin b; integer sums in double (exact below 2^53).
__global__ __launch_bounds__(64) void k_ltm_tables(const DevImage *__restrict__ table,
                                                   const int64_t *__restrict__ tile_end, int nimg,
                                                   const unsigned *__restrict__ hist,
                                                   LtmCoef *__restrict__ coef)
{
    const int64_t g = blockIdx.x;
    int lo = 0, hi = nimg - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tile_end[mid] > g)
            hi = mid;
        else
            lo = mid + 1;
    }
    const DevImage im = table[lo];
    const int nx = (int)im.tiles_per_seg, ny = (int)(im.ntiles / im.tiles_per_seg);
    const int64_t lt = g - im.tile_begin;
    const int ty = (int)(lt / nx), tx = (int)(lt - (int64_t)ty * nx);
    const int b = threadIdx.x;
    double h = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
        const int sy = ty + dy;
        if (sy < 0 || sy >= ny)
            continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int sx = tx + dx;
            if (sx < 0 || sx >= nx)
                continue;
            const double w = (dx == 0 ? 2.0 : 1.0) * (dy == 0 ? 2.0 : 1.0);
            h += w * (double)hist[(im.tile_begin + (int64_t)sy * nx + sx) * kLtmBins + b];
        }
    }
    // inclusive scan over the 64 lanes, then the exclusive prefix and total
    double incl = h;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double v = __shfl_up(incl, off, 64);
        if (b >= off)
            incl += v;
    }
    const double total = __shfl(incl, 63, 64);
    const double prefix = incl - h;
    const double next = __shfl_down(h, 1, 64);
    const double inv = 1.0 / total;
    LtmCoef c;
    c.a = (float)((prefix + 0.5 * h) * inv);
    c.b = (float)(h * inv);
    c.c = b < kLtmBins - 1 ? (float)(0.5 * (next - h) * inv) : 0.0f;
    c.pad = 0.0f;
    coef[g * kLtmBins + b] = c;
}

// First corner index in the 3 x 3 tile neighbourhood (the second is the next
// one) and the weight of the second corner along one axis, for tile-local
// coordinate p of tile t in a grid of n: the pixel lies between the centres of
// tiles t - 1 and t (p < 32) or t and t + 1, at distance (p + 1/2) / 64 -/+ 1/2
// from the first (exact in FP32); at the grid's edges it takes tile t alone
// (weight 0 on the second corner, which then may lie outside the grid).
__device__ __forceinline__ void ltm_axis(int p, int t, int n, int &c0, float &w)
{
    const bool lower = p < kLtmTile / 2;
    const bool edge = lower ? t == 0 : t == n - 1;
    c0 = (lower && !edge) ? 0 : 1;
    w = edge ? 0.0f : fmaf((float)p + 0.5f, 1.0f / kLtmTile, lower ? 0.5f : -0.5f);
}

// A bin's quadratic as staged in LDS: 3 words, so consecutive bins are 3
// banks apart and lanes looking up different bins rarely share a bank.
struct LtmLds {
    float a, b, c;
};

// Stages the curve tables of tile (tx, ty)'s 3 x 3 neighbourhood in LDS
// (entries of tiles outside the grid are left unset and never read).
__device__ __forceinline__ void ltm_stage(const DevImage &im, const LtmRef &r,
                                          const LtmCoef *__restrict__ coef, LtmLds *lds)
{
    for (int idx = threadIdx.x; idx < 9 * kLtmBins; idx += kBlock) {
        const int nb = idx / kLtmBins, bin = idx - nb * kLtmBins;
        const int sx = r.tx + nb % 3 - 1, sy = r.ty + nb / 3 - 1;
        if (sx >= 0 && sx < r.nx && sy >= 0 && sy < r.ny) {
            const LtmCoef c = coef[(im.tile_begin + (int64_t)sy * r.nx + sx) * kLtmBins + bin];
            lds[idx] = LtmLds{c.a, c.b, c.c};
        } else {
            // read only with weight 0 at the grid's edges: any finite value
            lds[idx] = LtmLds{0.0f, 0.0f, 0.0f};
        }
    }
    __syncthreads();
}

// T of one pixel from its x2 = log2(Lhat + eps): the global curve T_g, the
// bilinear blend T_l of the four corner tiles' curves at u, and
// T = T_g + strength (T_l - T_g). cy0/wy: the row's axis; cx0/wx: the
// column's.
__device__ __forceinline__ float ltm_value(float x2, float u0, TmArgs tm, Curve cv,
                                           const LtmLds *lds, int cx0, float wx, int cy0, float wy)
{
    const float tg = hw_rcp(1.0f + hw_exp2(cv.a * (x2 - cv.mu2)));
    const float u = ltm_u(x2, u0);
    const int k = ltm_bin(u);
    const float f = ltm_frac(u);
    // the four corners' entries for bin k sit at fixed distances from the
    // first one, so a single address serves all four LDS reads
    const LtmLds *c = lds + (cy0 * 3 + cx0) * kLtmBins + k;
    auto F = [&](const LtmLds &e) { return fmaf(f, fmaf(f, e.c, e.b), e.a); };
    const float f00 = F(c[0]), f10 = F(c[kLtmBins]), f01 = F(c[3 * kLtmBins]),
                f11 = F(c[4 * kLtmBins]);
    const float top = fmaf(wx, f10 - f00, f00);
    const float bot = fmaf(wx, f11 - f01, f01);
    const float tl = fmaf(wy, bot - top, top);
    return fmaf(tm.strength, tl - tg, tg);
}

// Curve pass of the local tone map over one tile, recomputing L from the
// input: the 3 x 3 neighbourhood's curve tables are staged in LDS, then every
// pixel gets ltm_value. Tile centres sit at 64 t + 32 pixels.
template <int SRC>
__device__ __forceinline__ void ltm_pass2_tile(const DevImage &im, int64_t tile, TmArgs tm,
                                               Curve cv, const LtmCoef *__restrict__ coef,
                                               LtmLds *lds)
{
    constexpr int PPU = unit_px(SRC);
    constexpr int U = kStatsPxPerThread / PPU;
    constexpr int ES = elem_size(SRC);
    const LtmRef r = ltm_ref(im, tile);
    const Enc e{1.0f, 255.0f};
    const float u0 = ltm_u0(hw_log2(tm.eps));
    if (r.vec) {
        // rows past the image's end (bottom tiles) load the last row again, so
        // every load is unconditional and all of them are in flight together,
        // also while the curve tables are being staged
        unsigned w[U][3];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int row, col;
            ltm_slot<PPU>(i, 0, row, col);
            load_unit(r.src + min(row, r.bh - 1) * r.sp + col * 3 * ES, w[i]);
        }
        ltm_stage(im, r, coef, lds);
        int col0, row0;
        ltm_slot<PPU>(0, 0, row0, col0);
        int cx0[PPU];
        float wx[PPU];
#pragma unroll
        for (int j = 0; j < PPU; ++j)
            ltm_axis(col0 + j, r.tx, r.nx, cx0[j], wx[j]);
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int row, col;
            ltm_slot<PPU>(i, 0, row, col);
            if (row < r.bh) {
                int cy0;
                float wy;
                ltm_axis(row, r.ty, r.ny, cy0, wy);
                float v[PPU];
#pragma unroll
                for (int j = 0; j < PPU; ++j) {
                    const float l = lum<SRC>(chan<SRC>(w[i], 3 * j), chan<SRC>(w[i], 3 * j + 1),
                                             chan<SRC>(w[i], 3 * j + 2), im.k);
                    v[j] = ltm_value(xlog2(l, im.unit, tm.eps), u0, tm, cv, lds, cx0[j], wx[j],
                                     cy0, wy);
                }
                store_unit<PPU, false, true>(r.dst + row * r.dp, im.dst_dtype, col, v, e);
            }
        }
    } else {
        ltm_stage(im, r, coef, lds);
#pragma unroll 1
        for (int sl = 0; sl < kStatsPxPerThread; ++sl) {
            int row, col;
            ltm_slot<PPU>(sl / PPU, sl % PPU, row, col);
            if (row < r.bh && col < r.bw) {
                float l;
                lum_at_px<SRC>(r.src + row * r.sp + col * 3 * ES, im.k, l);
                int cx0, cy0;
                float wx, wy;
                ltm_axis(col, r.tx, r.nx, cx0, wx);
                ltm_axis(row, r.ty, r.ny, cy0, wy);
                store_px<false, true>(r.dst + row * r.dp, im.dst_dtype, col,
                                      ltm_value(xlog2(l, im.unit, tm.eps), u0, tm, cv, lds, cx0,
                                                wx, cy0, wy),
                                      e);
            }
        }
    }
    __syncthreads();
}

// Curve pass over one tile of an image whose FP32 output holds x2 from the
// statistics pass: reads x2 (4 pixels per 16-byte unit) and overwrites it with
// T; the input is not touched.
__device__ __forceinline__ void ltm_pass2_staged_tile(const DevImage &im, int64_t tile, TmArgs tm,
                                                      Curve cv, const LtmCoef *__restrict__ coef,
                                                      LtmLds *lds)
{
    constexpr int PPU = 4;
    constexpr int U = kStatsPxPerThread / PPU;
    const LtmRef r = ltm_ref(im, tile);
    const float u0 = ltm_u0(hw_log2(tm.eps));
    if (r.vec) {
        float w[U][PPU];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int row, col;
            ltm_slot<PPU>(i, 0, row, col);
            const u32x4 t = *gp<u32x4>(r.dst + min(row, r.bh - 1) * r.dp + col * 4);
            // Elements go through plain scalars first: hipcc's
            // __builtin_bit_cast applied directly to a vector element (t.y)
            // reads element 0.
            const unsigned e[PPU] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int j = 0; j < PPU; ++j)
                w[i][j] = __builtin_bit_cast(float, e[j]);
        }
        ltm_stage(im, r, coef, lds);
        int col0, row0;
        ltm_slot<PPU>(0, 0, row0, col0);
        int cx0[PPU];
        float wx[PPU];
#pragma unroll
        for (int j = 0; j < PPU; ++j)
            ltm_axis(col0 + j, r.tx, r.nx, cx0[j], wx[j]);
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int row, col;
            ltm_slot<PPU>(i, 0, row, col);
            if (row < r.bh) {
                int cy0;
                float wy;
                ltm_axis(row, r.ty, r.ny, cy0, wy);
                unsigned o[PPU];
#pragma unroll
                for (int j = 0; j < PPU; ++j)
                    o[j] = __builtin_bit_cast(unsigned, ltm_value(w[i][j], u0, tm, cv, lds, cx0[j],
                                                                  wx[j], cy0, wy));
                put(gpw<u32x4>(r.dst + row * r.dp + col * 4), u32x4{o[0], o[1], o[2], o[3]});
            }
        }
    } else {
        ltm_stage(im, r, coef, lds);
#pragma unroll 1
        for (int sl = 0; sl < kStatsPxPerThread; ++sl) {
            int row, col;
            ltm_slot<PPU>(sl / PPU, sl % PPU, row, col);
            if (row < r.bh && col < r.bw) {
                auto *p = gpw<float>(r.dst + row * r.dp) + col;
                int cx0, cy0;
                float wx, wy;
                ltm_axis(col, r.tx, r.nx, cx0, wx);
                ltm_axis(row, r.ty, r.ny, cy0, wy);
                *p = ltm_value(*p, u0, tm, cv, lds, cx0, wx, cy0, wy);
            }
        }
    }
    __syncthreads();
}

// Colour output of one pixel from a tone-mapped T (the local map's blend):
// every channel T (C / L)^s clamped to at most 1, grey T where there is no
// colour to carry, in the same three modes and 8-bit scaling as colour_px
// (which takes the global curve's exponential instead of T); ANYGREY as
// there.
template <int SRC, int MODE, bool U8, bool ANYGREY = true>
__device__ __forceinline__ void colour_of_t(float R, float G, float B, float l, float T, float s,
                                            float *o)
{
    constexpr float kOut = U8 ? 255.0f : 1.0f;
    if constexpr (MODE == kColourGrey) {
        o[0] = o[1] = o[2] = T * kOut;
        return;
    }
    const bool grey = ANYGREY && colour_grey<SRC>(R, G, B, l);
    if constexpr (SRC != 0) {
        R = chan_clamp(R, 0.0f, chan_max<SRC>());
        G = chan_clamp(G, 0.0f, chan_max<SRC>());
        B = chan_clamp(B, 0.0f, chan_max<SRC>());
    }
    const float C[3] = {R, G, B};
    const float il = grey ? 0.0f : hw_rcp(fmaxf(l, 1e-30f));
    if constexpr (MODE == kColourRatio) {
        const float ko = T * il * kOut;
        const float g = grey ? T * kOut : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float v = fmaf(C[c], ko, g);
            o[c] = U8 ? v : fminf(v, 1.0f);
        }
    } else {
        constexpr float kLogOut = U8 ? 7.99435343685885793f : 0.0f; // log2(255)
        const float lT = hw_log2(T) + kLogOut;
        const float g = grey ? 1.0f : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = fmaf(s, hw_log2(fmaf(C[c], il, g)), lT);
            o[c] = hw_exp2(U8 ? e : fminf(e, 0.0f));
        }
    }
}

// Curve pass of the local tone map with colour output over one tile: reads
// the input (the colour needs it), T as ltm_pass2_tile, 3 channels per pixel.
template <int SRC, int MODE, bool U8>
__device__ __forceinline__ void ltm_colour_tile(const DevImage &im, int64_t tile, TmArgs tm,
                                                Curve cv, const LtmCoef *__restrict__ coef,
                                                LtmLds *lds)
{
    constexpr int PPU = unit_px(SRC);
    constexpr int U = kStatsPxPerThread / PPU;
    constexpr int ES = elem_size(SRC);
    const LtmRef r = ltm_ref(im, tile);
    const Enc e{1.0f, 1.0f};
    const float u0 = ltm_u0(hw_log2(tm.eps));
    const int dt = U8 ? 0 : im.dst_dtype;
    uint8_t *dst = im.dst + (int64_t)r.ty * kLtmTile * r.dp +
                   (int64_t)r.tx * kLtmTile * 3 * elem_size(im.dst_dtype);
    if (r.vec) {
        unsigned w[U][3];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int row, col;
            ltm_slot<PPU>(i, 0, row, col);
            load_unit(r.src + min(row, r.bh - 1) * r.sp + col * 3 * ES, w[i]);
        }
        ltm_stage(im, r, coef, lds);
        int col0, row0;
        ltm_slot<PPU>(0, 0, row0, col0);
        int cx0[PPU];
        float wx[PPU];
#pragma unroll
        for (int j = 0; j < PPU; ++j)
            ltm_axis(col0 + j, r.tx, r.nx, cx0[j], wx[j]);
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int row, col;
            ltm_slot<PPU>(i, 0, row, col);
            if (row < r.bh) {
                int cy0;
                float wy;
                ltm_axis(row, r.ty, r.ny, cy0, wy);
                float o[3 * PPU], l[PPU], T[PPU];
                bool grey = false;
#pragma unroll
                for (int j = 0; j < PPU; ++j) {
                    const float R = chan<SRC>(w[i], 3 * j), G = chan<SRC>(w[i], 3 * j + 1),
                                B = chan<SRC>(w[i], 3 * j + 2);
                    l[j] = lum<SRC>(R, G, B, im.k);
                    T[j] = ltm_value(xlog2(l[j], im.unit, tm.eps), u0, tm, cv, lds, cx0[j], wx[j],
                                     cy0, wy);
                    grey = grey || colour_grey<SRC>(R, G, B, l[j]);
                }
                // as in the global map: units of grey-free waves skip the selects
                if (MODE == kColourGrey || __builtin_amdgcn_ballot_w64(grey) == 0) {
#pragma unroll
                    for (int j = 0; j < PPU; ++j)
                        colour_of_t<SRC, MODE, U8, false>(
                            chan<SRC>(w[i], 3 * j), chan<SRC>(w[i], 3 * j + 1),
                            chan<SRC>(w[i], 3 * j + 2), l[j], T[j], tm.saturation, &o[3 * j]);
                } else {
#pragma unroll
                    for (int j = 0; j < PPU; ++j)
                        colour_of_t<SRC, MODE, U8, true>(
                            chan<SRC>(w[i], 3 * j), chan<SRC>(w[i], 3 * j + 1),
                            chan<SRC>(w[i], 3 * j + 2), l[j], T[j], tm.saturation, &o[3 * j]);
                }
                store_rgb_unit<PPU>(dst + row * r.dp, dt, col, o);
            }
        }
    } else {
        ltm_stage(im, r, coef, lds);
#pragma unroll 1
        for (int sl = 0; sl < kStatsPxPerThread; ++sl) {
            int row, col;
            ltm_slot<PPU>(sl / PPU, sl % PPU, row, col);
            if (row < r.bh && col < r.bw) {
                float R, G, B;
                load_px<SRC>(r.src + row * r.sp + col * 3 * ES, R, G, B);
                const float l = lum<SRC>(R, G, B, im.k);
                int cx0, cy0;
                float wx, wy;
                ltm_axis(col, r.tx, r.nx, cx0, wx);
                ltm_axis(row, r.ty, r.ny, cy0, wy);
                const float T = ltm_value(xlog2(l, im.unit, tm.eps), u0, tm, cv, lds, cx0, wx,
                                          cy0, wy);
                float o[3];
                colour_of_t<SRC, MODE, U8>(R, G, B, l, T, tm.saturation, o);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    store_px<false, false>(dst + row * r.dp, dt, 3 * col + c, o[c], e);
            }
        }
    }
    __syncthreads();
}

template <int SRC, int MODE>
__global__ __launch_bounds__(kBlock) void k_ltm_colour(const DevImage *__restrict__ table,
                                                       const int64_t *__restrict__ tile_end,
                                                       int img0, int nimg, int64_t t0, int64_t t1,
                                                       TmArgs tm, const Curve *__restrict__ curves,
                                                       const LtmCoef *__restrict__ coef)
{
    __shared__ LtmLds lds[9 * kLtmBins];
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        if (im.dst_dtype == 0)
            ltm_colour_tile<SRC, MODE, true>(im, tile - im.tile_begin, tm, curves[i], coef, lds);
        else
            ltm_colour_tile<SRC, MODE, false>(im, tile - im.tile_begin, tm, curves[i], coef, lds);
    });
}

// SRC 3 = the staged form (FP32 output holding x2), whatever the input type.
template <int SRC>
__global__ __launch_bounds__(kBlock) void k_ltm_pass2(const DevImage *__restrict__ table,
                                                      const int64_t *__restrict__ tile_end,
                                                      int img0, int nimg, int64_t t0, int64_t t1,
                                                      TmArgs tm, const Curve *__restrict__ curves,
                                                      const LtmCoef *__restrict__ coef)
{
    __shared__ LtmLds lds[9 * kLtmBins];
    for_each_tile(tile_end, img0, nimg, t0, t1, [&](int i, int64_t tile) {
        const DevImage im = table[i];
        if constexpr (SRC == 3)
            ltm_pass2_staged_tile(im, tile - im.tile_begin, tm, curves[i], coef, lds);
        else
            ltm_pass2_tile<SRC>(im, tile - im.tile_begin, tm, curves[i], coef, lds);
    });
}

// ------------------------------------------------------------ row copy

// Copies `rows` rows of row_bytes each from src (row pitch src_pitch; for the
// server, a pinned host buffer the GPU reads across PCIe) to dst (row pitch
// dst_pitch): workgroup (x, y) moves 16-byte pieces x * 256 + tid of row y,
// the unaligned pieces and the row's last bytes included (the target serves
// unaligned dword accesses); the grid is (ceil(row_bytes / 4096), rows).
__global__ __launch_bounds__(kBlock) void k_copy_rows(uint8_t *__restrict__ dst, int64_t dst_pitch,
                                                      const uint8_t *__restrict__ src,
                                                      int64_t src_pitch, int64_t row_bytes)
{
    const int64_t y = blockIdx.y;
    const int64_t off = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 16;
    if (off >= row_bytes)
        return;
    const uint8_t *s = src + y * src_pitch + off;
    uint8_t *d = dst + y * dst_pitch + off;
    if (off + 16 <= row_bytes) {
        *gpw<u32x4>(d) = *gp<u32x4>(s);
    } else {
        for (int64_t i = 0; off + i < row_bytes; ++i)
            *gpw<uint8_t>(d + i) = *gp<uint8_t>(s + i);
    }
}

// ------------------------------------------------------------ scratch

// Workspace of dc_tonemap_global_noalloc: one per device, held until the
// process ends, shared by every such call on the device (calls that overlap on
// one device race on it). Host code never passes this name to a kernel: in
// host code it is a stand-in, not a device address; scratch_address gives the
// real one.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void **p)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[dev] = a;
    }
    *p = addr[dev];
    return hipSuccess;
}

// ------------------------------------------------------------ launchers

static unsigned grid_of(int64_t ntiles, int64_t grid)
{
    int64_t g = grid > 0 && grid < ntiles ? grid : ntiles;
    if (g > 0x7fffffff)
        g = 0x7fffffff;
    return (unsigned)(g > 0 ? g : 1);
}

// Launches the row-walk or the other instantiation of a kernel template:
// DC_BY_ROWS(M, args) expands M(args, true) or M(args, false) by the runtime
// flag `rows`.
#define DC_BY_ROWS(M, ...)                                                                        \
    do {                                                                                          \
        if (rows)                                                                                 \
            M(__VA_ARGS__, true);                                                                 \
        else                                                                                      \
            M(__VA_ARGS__, false);                                                                \
    } while (0)

hipError_t launch_decolor_single(const DevImage &im, int groups, int64_t grid, hipStream_t s)
{
    const int64_t ntiles = im.ntiles;
    const unsigned g = grid_of(ntiles, grid);
    const bool rows = im.walk == kWalkRows;
#define DC_LAUNCH_SINGLE(S, GG, R)                                                                \
    hipLaunchKernelGGL((k_decolor_single<S, GG, R>), dim3(g), dim3(kBlock), 0, s, im, ntiles)
    switch (im.src_dtype * 8 + groups) {
    case 0 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_SINGLE, 0, 1); break;
    case 0 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_SINGLE, 0, 2); break;
    case 0 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_SINGLE, 0, 4); break;
    case 1 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_SINGLE, 1, 1); break;
    case 1 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_SINGLE, 1, 2); break;
    case 1 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_SINGLE, 1, 4); break;
    case 2 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_SINGLE, 2, 1); break;
    case 2 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_SINGLE, 2, 2); break;
    case 2 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_SINGLE, 2, 4); break;
    default: return hipErrorInvalidValue;
    }
#undef DC_LAUNCH_SINGLE
    return hipGetLastError();
}

hipError_t launch_decolor_table(const DevImage *table, const int64_t *tile_end, int img0,
                                int nimg, int64_t t0, int64_t t1, int mixed_src, int src_dtype,
                                int groups, int rows, int64_t grid, hipStream_t s)
{
    const unsigned g = grid_of(t1 - t0, grid);
#define DC_LAUNCH_TABLE(S, GG, M, R)                                                              \
    hipLaunchKernelGGL((k_decolor_table<S, GG, M, R>), dim3(g), dim3(kBlock), 0, s, table,         \
                       tile_end, img0, nimg, t0, t1)
    if (mixed_src) {
        switch (groups) {
        case 1: DC_BY_ROWS(DC_LAUNCH_TABLE, 0, 1, true); break;
        case 2: DC_BY_ROWS(DC_LAUNCH_TABLE, 0, 2, true); break;
        case 4: DC_BY_ROWS(DC_LAUNCH_TABLE, 0, 4, true); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (src_dtype * 8 + groups) {
        case 0 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_TABLE, 0, 1, false); break;
        case 0 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_TABLE, 0, 2, false); break;
        case 0 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_TABLE, 0, 4, false); break;
        case 1 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_TABLE, 1, 1, false); break;
        case 1 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_TABLE, 1, 2, false); break;
        case 1 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_TABLE, 1, 4, false); break;
        case 2 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_TABLE, 2, 1, false); break;
        case 2 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_TABLE, 2, 2, false); break;
        case 2 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_TABLE, 2, 4, false); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef DC_LAUNCH_TABLE
    return hipGetLastError();
}

hipError_t launch_sweep(const DevImage *table, int n, int per, int64_t ntiles, int src_dtype,
                        int groups, int rows, int64_t grid, hipStream_t s)
{
    if (n < 1 || per < 1 || ntiles < 1)
        return hipErrorInvalidValue;
    const int64_t nwork = ntiles * ((n + per - 1) / per);
    const unsigned g = grid_of(nwork, grid);
#define DC_LAUNCH_SWEEP(S, GG, R)                                                                 \
    hipLaunchKernelGGL((k_sweep<S, GG, R>), dim3(g), dim3(kBlock), 0, s, table, n, per, ntiles,  \
                       nwork)
    switch (src_dtype * 8 + groups) {
    case 0 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_SWEEP, 0, 1); break;
    case 0 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_SWEEP, 0, 2); break;
    case 0 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_SWEEP, 0, 4); break;
    case 1 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_SWEEP, 1, 1); break;
    case 1 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_SWEEP, 1, 2); break;
    case 1 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_SWEEP, 1, 4); break;
    case 2 * 8 + 1: DC_BY_ROWS(DC_LAUNCH_SWEEP, 2, 1); break;
    case 2 * 8 + 2: DC_BY_ROWS(DC_LAUNCH_SWEEP, 2, 2); break;
    case 2 * 8 + 4: DC_BY_ROWS(DC_LAUNCH_SWEEP, 2, 4); break;
    default: return hipErrorInvalidValue;
    }
#undef DC_LAUNCH_SWEEP
    return hipGetLastError();
}

hipError_t launch_channel(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                          int64_t t0, int64_t t1, int src_dtype, int channel, int rows,
                          int64_t grid, hipStream_t s)
{
    const dim3 g(grid_of(t1 - t0, grid));
#define DC_LAUNCH_CH(S, C, R)                                                                     \
    hipLaunchKernelGGL((k_channel_table<S, C, R>), g, dim3(kBlock), 0, s, table, tile_end, img0,   \
                       nimg, t0, t1)
    switch (src_dtype * 4 + channel) {
    case 0 * 4 + 1: DC_BY_ROWS(DC_LAUNCH_CH, 0, 1); break;
    case 0 * 4 + 2: DC_BY_ROWS(DC_LAUNCH_CH, 0, 2); break;
    case 0 * 4 + 3: DC_BY_ROWS(DC_LAUNCH_CH, 0, 3); break;
    case 1 * 4 + 1: DC_BY_ROWS(DC_LAUNCH_CH, 1, 1); break;
    case 1 * 4 + 2: DC_BY_ROWS(DC_LAUNCH_CH, 1, 2); break;
    case 1 * 4 + 3: DC_BY_ROWS(DC_LAUNCH_CH, 1, 3); break;
    case 2 * 4 + 1: DC_BY_ROWS(DC_LAUNCH_CH, 2, 1); break;
    case 2 * 4 + 2: DC_BY_ROWS(DC_LAUNCH_CH, 2, 2); break;
    case 2 * 4 + 3: DC_BY_ROWS(DC_LAUNCH_CH, 2, 3); break;
    default: return hipErrorInvalidValue;
    }
#undef DC_LAUNCH_CH
    return hipGetLastError();
}

hipError_t launch_tm_pass1(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                           int64_t t0, int64_t t1, int mixed_src, int src_dtype, int rows,
                           TmArgs tm, WavePart *parts, int64_t grid, hipStream_t s)
{
    const dim3 g(grid_of(t1 - t0, grid));
#define DC_LAUNCH_P1(S, M, R)                                                                     \
    hipLaunchKernelGGL((k_tm_pass1<S, M, R>), g, dim3(kBlock), 0, s, table, tile_end, img0, nimg,  \
                       t0, t1, tm, parts)
    if (mixed_src)
        DC_BY_ROWS(DC_LAUNCH_P1, 0, true);
    else if (src_dtype == 0)
        DC_BY_ROWS(DC_LAUNCH_P1, 0, false);
    else if (src_dtype == 1 && !rows)
        hipLaunchKernelGGL(k_tm_pass1_f16, g, dim3(kBlock), 0, s, table, tile_end, img0, nimg, t0,
                           t1, tm, parts);
    else if (src_dtype == 1)
        DC_LAUNCH_P1(1, false, true);
    else
        DC_BY_ROWS(DC_LAUNCH_P1, 2, false);
#undef DC_LAUNCH_P1
    return hipGetLastError();
}

hipError_t launch_tm_combine(const DevImage *table, const int64_t *grp_end, int img0, int nimg,
                             int64_t g0, int64_t g1, const WavePart *parts, Part *parts2,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_tm_combine, dim3((unsigned)(g1 - g0)), dim3(kBlock), 0, s, table, grp_end,
                       img0, nimg, g0, parts, parts2);
    return hipGetLastError();
}

hipError_t launch_copy_rows(void *dst, int64_t dst_pitch, const void *src, int64_t src_pitch,
                            int64_t row_bytes, int rows, hipStream_t s)
{
    if (rows < 1 || row_bytes < 1)
        return hipSuccess;
    const int64_t gx = (row_bytes + (int64_t)kBlock * 16 - 1) / ((int64_t)kBlock * 16);
    if (gx > 0x7fffffff)
        return hipErrorInvalidValue;
    // the grid's y extent is at most 65535: rows go in chunks of that many
    for (int r0 = 0; r0 < rows; r0 += 65535) {
        const int n = rows - r0 < 65535 ? rows - r0 : 65535;
        hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)gx, (unsigned)n), dim3(kBlock), 0, s,
                           (uint8_t *)dst + (int64_t)r0 * dst_pitch, dst_pitch,
                           (const uint8_t *)src + (int64_t)r0 * src_pitch, src_pitch, row_bytes);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_tm_combine_finalize(const DevImage *table, const int64_t *grp_end, int img0,
                                      int nimg, int64_t g0, int64_t g1, TmArgs tm,
                                      const WavePart *parts, Part *parts2, unsigned *counters,
                                      Curve *curves, StatsOut *stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_tm_combine_finalize, dim3((unsigned)(g1 - g0)), dim3(kBlock), 0, s, table,
                       grp_end, img0, nimg, g0, tm, parts, parts2, counters, curves, stats);
    return hipGetLastError();
}

hipError_t launch_tm_finalize(const DevImage *table, int img0, int nimg, TmArgs tm,
                              const Part *parts2, Curve *curves, StatsOut *stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_tm_finalize, dim3(nimg), dim3(kBlock), 0, s, table, img0, tm, parts2,
                       curves, stats);
    return hipGetLastError();
}

hipError_t launch_tm_colour(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                            int64_t t0, int64_t t1, int src_dtype, int mode, int rows, TmArgs tm,
                            const Curve *curves, int64_t grid, hipStream_t s)
{
    const dim3 g(grid_of(t1 - t0, grid));
#define DC_LAUNCH_COL(S, M, R)                                                                    \
    hipLaunchKernelGGL((k_tm_colour<S, M, R>), g, dim3(kBlock), 0, s, table, tile_end, img0,       \
                       nimg, t0, t1, tm, curves)
    switch (src_dtype * 4 + mode) {
    case 0 * 4 + kColourGrey: DC_BY_ROWS(DC_LAUNCH_COL, 0, kColourGrey); break;
    case 0 * 4 + kColourRatio: DC_BY_ROWS(DC_LAUNCH_COL, 0, kColourRatio); break;
    case 0 * 4 + kColourPow: DC_BY_ROWS(DC_LAUNCH_COL, 0, kColourPow); break;
    case 1 * 4 + kColourGrey: DC_BY_ROWS(DC_LAUNCH_COL, 1, kColourGrey); break;
    case 1 * 4 + kColourRatio: DC_BY_ROWS(DC_LAUNCH_COL, 1, kColourRatio); break;
    case 1 * 4 + kColourPow: DC_BY_ROWS(DC_LAUNCH_COL, 1, kColourPow); break;
    case 2 * 4 + kColourGrey: DC_BY_ROWS(DC_LAUNCH_COL, 2, kColourGrey); break;
    case 2 * 4 + kColourRatio: DC_BY_ROWS(DC_LAUNCH_COL, 2, kColourRatio); break;
    case 2 * 4 + kColourPow: DC_BY_ROWS(DC_LAUNCH_COL, 2, kColourPow); break;
    default: return hipErrorInvalidValue;
    }
#undef DC_LAUNCH_COL
    return hipGetLastError();
}

hipError_t launch_ltm_pass1(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                            int64_t t0, int64_t t1, int src_dtype, TmArgs tm, WavePart *parts,
                            unsigned *hist, int64_t grid, hipStream_t s)
{
    const dim3 g(grid_of(t1 - t0, grid));
#define DC_LAUNCH_L1(S)                                                                           \
    hipLaunchKernelGGL((k_ltm_pass1<S>), g, dim3(kBlock), 0, s, table, tile_end, img0, nimg, t0,  \
                       t1, tm, parts, hist)
    if (src_dtype == 0)
        DC_LAUNCH_L1(0);
    else if (src_dtype == 1)
        DC_LAUNCH_L1(1);
    else
        DC_LAUNCH_L1(2);
#undef DC_LAUNCH_L1
    return hipGetLastError();
}

hipError_t launch_ltm_tables(const DevImage *table, const int64_t *tile_end, int nimg,
                             int64_t total_tiles, const unsigned *hist, LtmCoef *coef,
                             hipStream_t s)
{
    if (total_tiles <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_ltm_tables, dim3((unsigned)total_tiles), dim3(64), 0, s, table, tile_end,
                       nimg, hist, coef);
    return hipGetLastError();
}

hipError_t launch_ltm_pass2(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                            int64_t t0, int64_t t1, int src_dtype, TmArgs tm, const Curve *curves,
                            const LtmCoef *coef, int64_t grid, hipStream_t s)
{
    const dim3 g(grid_of(t1 - t0, grid));
#define DC_LAUNCH_L2(S)                                                                           \
    hipLaunchKernelGGL((k_ltm_pass2<S>), g, dim3(kBlock), 0, s, table, tile_end, img0, nimg, t0,  \
                       t1, tm, curves, coef)
    if (src_dtype == 0)
        DC_LAUNCH_L2(0);
    else if (src_dtype == 1)
        DC_LAUNCH_L2(1);
    else if (src_dtype == 2)
        DC_LAUNCH_L2(2);
    else
        DC_LAUNCH_L2(3);
#undef DC_LAUNCH_L2
    return hipGetLastError();
}

hipError_t launch_ltm_colour(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                             int64_t t0, int64_t t1, int src_dtype, int mode, TmArgs tm,
                             const Curve *curves, const LtmCoef *coef, hipStream_t s)
{
    const dim3 g(grid_of(t1 - t0, 0));
#define DC_LAUNCH_LC(S, M)                                                                        \
    hipLaunchKernelGGL((k_ltm_colour<S, M>), g, dim3(kBlock), 0, s, table, tile_end, img0, nimg,   \
                       t0, t1, tm, curves, coef)
    switch (src_dtype * 4 + mode) {
    case 0 * 4 + kColourGrey: DC_LAUNCH_LC(0, kColourGrey); break;
    case 0 * 4 + kColourRatio: DC_LAUNCH_LC(0, kColourRatio); break;
    case 0 * 4 + kColourPow: DC_LAUNCH_LC(0, kColourPow); break;
    case 1 * 4 + kColourGrey: DC_LAUNCH_LC(1, kColourGrey); break;
    case 1 * 4 + kColourRatio: DC_LAUNCH_LC(1, kColourRatio); break;
    case 1 * 4 + kColourPow: DC_LAUNCH_LC(1, kColourPow); break;
    case 2 * 4 + kColourGrey: DC_LAUNCH_LC(2, kColourGrey); break;
    case 2 * 4 + kColourRatio: DC_LAUNCH_LC(2, kColourRatio); break;
    case 2 * 4 + kColourPow: DC_LAUNCH_LC(2, kColourPow); break;
    default: return hipErrorInvalidValue;
    }
#undef DC_LAUNCH_LC
    return hipGetLastError();
}

hipError_t launch_tm_pass2(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                           int64_t t0, int64_t t1, int mixed_src, int src_dtype, int rows,
                           TmArgs tm, const Curve *curves, int64_t grid, hipStream_t s)
{
    const dim3 g(grid_of(t1 - t0, grid));
#define DC_LAUNCH_P2(S, M, R)                                                                     \
    hipLaunchKernelGGL((k_tm_pass2<S, M, R>), g, dim3(kBlock), 0, s, table, tile_end, img0, nimg,  \
                       t0, t1, tm, curves)
    if (mixed_src)
        DC_BY_ROWS(DC_LAUNCH_P2, 0, true);
    else if (src_dtype == 0)
        DC_BY_ROWS(DC_LAUNCH_P2, 0, false);
    else if (src_dtype == 1)
        DC_BY_ROWS(DC_LAUNCH_P2, 1, false);
    else
        DC_BY_ROWS(DC_LAUNCH_P2, 2, false);
#undef DC_LAUNCH_P2
    return hipGetLastError();
}

} // namespace dc
