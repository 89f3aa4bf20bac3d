// Internal types shared by the HIP kernels (kernels.hip) and the host runtime
// (runtime.cpp). Not part of the public ABI (include/decolor.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dc {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kGroupBytes = 48;      // input bytes per vector group: 3 x 16 B
constexpr int kStatsPxPerThread = 16; // pixels per thread in a statistics chunk
constexpr int64_t kStatsChunkPx = (int64_t)kBlock * kStatsPxPerThread; // 4096 px per tile
constexpr int kWavesPerBlock = kBlock / 64; // statistics partials per tone-map tile

// Local tone map: square tiles of kLtmTile pixels (one workgroup's 4096-pixel
// statistics chunk each), kLtmBins soft bins of log2 luminance, 2 per stop
// from log2(eps), histogram masses in fixed point (kLtmOne per pixel).
constexpr int kLtmTile = 64;
constexpr int kLtmBins = 64;
constexpr unsigned kLtmOne = 1u << 19;

// Pixels per vector group for each input element type (48 B of RGB).
__host__ __device__ constexpr int group_px(int src_dtype)
{
    return src_dtype == 0 ? 16 : (src_dtype == 1 ? 8 : 4);
}

__host__ __device__ constexpr int elem_size(int dtype)
{
    return dtype == 0 ? 1 : (dtype == 1 ? 2 : 4);
}

// How an image is walked.
enum Walk : int32_t {
    kWalkPacked = 0, // one segment of W*H pixels from a 4-byte aligned start, vector
                     // units loaded with buffer loads
    kWalkRows = 1,   // pitched rows, or packed rows from an unaligned start (all gaps
                     // 0): tiled as one segment of W*H pixels in row-major order,
                     // vector units placed across the row breaks (magic, gaps)
    kWalkScalar = 2, // H segments of W pixels, one pixel at a time
};

// The row walk needs q = floor(x / W) = mulhi(x, ceil(2^32 / W)) to be exact
// for x < W + the largest tile (16384 px), i.e. W (W + 16384) < 2^32, and the
// rows' padding to fit the 32-bit offsets within a tile; wider images or
// wider padding take the per-pixel walk.
constexpr int32_t kRowWalkMaxWidth = 46000;
constexpr int64_t kRowWalkMaxGap = (int64_t)1 << 18;

// Per-pixel coefficients of Eqs. (3) and (6), in the scaling the input's
// per-pixel form expects (see lum_code / lum_half / lum_linear).
struct Coef {
    float cr; // beta_R        (x3 for 8-bit and binary16 input)
    float cg; // 1 - beta_R    (x3 for 8-bit and binary16 input)
    float ck; // beta_k        (/3 for 8-bit and binary16 input)
    float cc; // 1 - beta_k    (/3 for 8-bit and binary16 input)
};

// Device-side descriptor of one image, built by the host runtime.
struct DevImage {
    const uint8_t *src;
    uint8_t *dst;
    uint8_t *dst2;
    int64_t src_seg_stride; // bytes between segment starts (row pitch, or 0 when packed)
    int64_t dst_seg_stride;
    int64_t dst2_seg_stride;
    int64_t seg_len;        // pixels per segment
    int64_t tiles_per_seg;  // tiles of the launch's tile size per segment
    int64_t tile_begin;     // first global tile of this image (batched launches)
    int64_t chunk_begin;    // first statistics partial of this image (tone map)
    int64_t ntiles;         // tiles of this image
    int64_t npx;            // pixels, width * height
    int64_t grp_begin;      // first level-2 statistics partial of this image
    int64_t ngrp;           // level-2 partials: ceil(ntiles * kWavesPerBlock / kBlock)
    int32_t src_dtype;
    int32_t dst_dtype;
    int32_t dst2_dtype;     // -1 = none
    int32_t walk;
    int32_t image;          // index within the call
    int32_t rgb_out;        // tone map: dst holds 3 channels (re-coloured RGB)
    int32_t width;          // pixels per row (local tone map's 2-D tile walk)
    int32_t height;         // rows
    int32_t staged;         // local tone map: the FP32 dst carries x2 between passes
    int32_t shared_src;     // decolorization: another image of the call reads the same input
    float unit;             // Lhat = L * unit (1/255 for 8-bit input)
    Coef k;                 // per-pixel constants for this image's input type
    // Row walk: ceil(2^32 / width), and each buffer's row padding in bytes
    // (pitch minus the row's bytes).
    uint32_t magic;
    uint32_t gap_src;
    uint32_t gap_dst;
    uint32_t gap_dst2;
};

// Statistics partial of one chunk, in log2 units: count, mean and sum of
// squared deviations of x2 = log2(Lhat + eps) (Chan et al. merge), and the
// extremes of Lhat.
struct Part {
    float n, mean, m2, lo, hi;
};

// What a wave of a statistics pass writes for its 1024 pixels: the count, the
// shift K (x2 of the wave's first pixel), the sums of d = x2 - K and d^2, and
// the extremes of L in input units. The combine turns it into a Part (mean =
// K + s / n, m2 = q - s^2 / n, extremes times the image's unit), so the
// statistics pass spends no division or scaling per wave.
struct WavePart {
    float n, K, s, q, lo, hi;
};

// Per-image curve of the tone map: T = 1 / (1 + exp2(a * (x2 - mu2))).
struct Curve {
    float a, mu2;
};

struct TmArgs {
    float eps;
    float contrast;
    float sigma_floor;
    float saturation; // exponent s of the colour output
    float strength;   // local tone map: weight of the local curve
};

// Local tone map: one tile's curve as a quadratic per bin interval k:
// F(k + f) = a + f (b + f c), f in [0, 1].
struct LtmCoef {
    float a, b, c, pad;
};

// Colour output modes: s = 0 (grey T), s = 1 (ratio kept), any other s.
enum ColourMode : int { kColourGrey = 0, kColourRatio = 1, kColourPow = 2 };

// Output statistics, laid out as dc_stats.
struct StatsOut {
    float log_mean, log_std, l_min, l_max;
    int64_t count;
};

// The tone map's fixed device scratch (kernels.hip), used by the entry point
// that allocates nothing: descriptor table, tile and group prefixes, wave and
// group partials and curves of one call, laid out as a ring slot would hold
// them. kScratchBytes bounds one call: at most kScratchMaxImages images and
// about 340 Mpx (24 B of wave partials per 1024 px).
constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr int kScratchMaxImages = 1024;
constexpr int kMaxDevices = 64;
// Device address of the scratch array on the current device (looked up once
// per device with hipGetSymbolAddress, then cached).
hipError_t scratch_address(void **p);

// Kernel launchers (kernels.hip). All return the hipError_t of the launch.
// `rows` = every image of the launch is on the row walk (kWalkRows); a launch
// never mixes row-walk images with others.
hipError_t launch_decolor_single(const DevImage &im, int groups, int64_t grid, hipStream_t s);
// n images sharing the input and geometry of table[0] (ntiles tiles each):
// each workgroup reads a tile once for up to `per` of the images.
hipError_t launch_sweep(const DevImage *table, int n, int per, int64_t ntiles, int src_dtype,
                        int groups, int rows, int64_t grid, hipStream_t s);
hipError_t launch_decolor_table(const DevImage *table, const int64_t *tile_end, int img0,
                                int nimg, int64_t t0, int64_t t1, int mixed_src, int src_dtype,
                                int groups, int rows, int64_t grid, hipStream_t s);
hipError_t launch_channel(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                          int64_t t0, int64_t t1, int src_dtype, int channel, int rows,
                          int64_t grid, hipStream_t s);
hipError_t launch_tm_pass1(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                           int64_t t0, int64_t t1, int mixed_src, int src_dtype, int rows,
                           TmArgs tm, WavePart *parts, int64_t grid, hipStream_t s);
hipError_t launch_tm_combine(const DevImage *table, const int64_t *grp_end, int img0, int nimg,
                             int64_t g0, int64_t g1, const WavePart *parts, Part *parts2,
                             hipStream_t s);
hipError_t launch_tm_finalize(const DevImage *table, int img0, int nimg, TmArgs tm,
                              const Part *parts2, Curve *curves, StatsOut *stats, hipStream_t s);
// Copies rows x row_bytes from src (pitch src_pitch; may be pinned host memory)
// to dst (pitch dst_pitch).
hipError_t launch_copy_rows(void *dst, int64_t dst_pitch, const void *src, int64_t src_pitch,
                            int64_t row_bytes, int rows, hipStream_t s);
// Both combine levels in one launch over groups [g0, g1) of images img0 ..
// img0 + nimg - 1; counters: one word per table image, zero at the start and
// left zero.
hipError_t launch_tm_combine_finalize(const DevImage *table, const int64_t *grp_end, int img0,
                                      int nimg, int64_t g0, int64_t g1, TmArgs tm,
                                      const WavePart *parts, Part *parts2, unsigned *counters,
                                      Curve *curves, StatsOut *stats, hipStream_t s);
hipError_t launch_tm_colour(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                            int64_t t0, int64_t t1, int src_dtype, int mode, int rows, TmArgs tm,
                            const Curve *curves, int64_t grid, hipStream_t s);
hipError_t launch_ltm_pass1(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                            int64_t t0, int64_t t1, int src_dtype, TmArgs tm, WavePart *parts,
                            unsigned *hist, int64_t grid, hipStream_t s);
hipError_t launch_ltm_tables(const DevImage *table, const int64_t *tile_end, int nimg,
                             int64_t total_tiles, const unsigned *hist, LtmCoef *coef,
                             hipStream_t s);
// src_dtype 3 selects the staged curve pass (FP32 dst holding x2).
hipError_t launch_ltm_pass2(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                            int64_t t0, int64_t t1, int src_dtype, TmArgs tm, const Curve *curves,
                            const LtmCoef *coef, int64_t grid, hipStream_t s);
hipError_t launch_ltm_colour(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                             int64_t t0, int64_t t1, int src_dtype, int mode, TmArgs tm,
                             const Curve *curves, const LtmCoef *coef, hipStream_t s);
hipError_t launch_tm_pass2(const DevImage *table, const int64_t *tile_end, int img0, int nimg,
                           int64_t t0, int64_t t1, int mixed_src, int src_dtype, int rows,
                           TmArgs tm, const Curve *curves, int64_t grid, hipStream_t s);

} // namespace dc
