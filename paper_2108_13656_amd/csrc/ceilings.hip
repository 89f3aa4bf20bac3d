// Memory ceilings of the MI355X for the access patterns of the hot path,
// measured with plain streaming kernels that do no arithmetic: what HBM
// sustains for a read-only stream (the statistics pass), a write-only stream,
// and mixed streams at the read:write ratios of the passes (6:4 for the curve
// pass on binary16 input with an FP32 output, 3:5 for 8-bit video with 8-bit
// and FP32 outputs, 1:1 for a copy). Built as its own library
// (libdc_ceilings.so) for the benchmark; the decolorization library does not
// use it. It also times the two-pass schedules of the tone map with no
// arithmetic: the batch order (read every image, then read every image again
// and write its output) and a lagged order (each image re-read one image
// later, while its lines may still be in the last-level cache), to show what
// the traffic of each order costs on its own; and the same for a schedule that
// parks a 4-byte per-pixel intermediate between the passes (first pass: read
// the input, write the intermediate; second pass: read it back, write the
// output) in batch and lagged order.
//
// Workgroups walk fixed tiles of both buffers (all of a thread's loads issued
// before its stores), and loads and stores are nontemporal like the product
// kernels' unit loads and stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Reads nr vectors of src and writes nw vectors of dst in tiles: tile j is
// the VR * 256 vectors of src from j * VR * 256 on and the VW * 256 vectors of
// dst from j * VW * 256 on, so the two streams advance at the ratio VR:VW
// throughout the pass. A workgroup takes tiles j = blockIdx.x, + gridDim.x, ...
// (one tile each when the grid covers them); thread x loads vectors
// k * 256 + x of its tile (k < VR) before it stores any, so each load and
// store instruction of a wave touches 1 KiB of contiguous memory. sink
// receives a value only if the data XORs to a constant no input holds, which
// keeps the loads alive.
template <int VR, int VW>
__global__ __launch_bounds__(256) void k_stream(const u32x4 *__restrict__ src, int64_t nr,
                                                u32x4 *__restrict__ dst, int64_t nw,
                                                int64_t ntiles, unsigned *__restrict__ sink)
{
    unsigned acc = 0;
    for (int64_t j = blockIdx.x; j < ntiles; j += gridDim.x) {
        u32x4 v[VR > 0 ? VR : 1];
#pragma unroll
        for (int k = 0; k < VR; ++k) {
            const int64_t i = (j * VR + k) * 256 + threadIdx.x;
            v[k] = i < nr ? __builtin_nontemporal_load(src + i) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < VR; ++k)
            acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            const int64_t i = (j * VW + k) * 256 + threadIdx.x;
            if (i < nw)
                __builtin_nontemporal_store(u32x4{acc, (unsigned)i, acc, (unsigned)k}, dst + i);
        }
    }
    if (acc == 0x5ca1ab1eu)
        sink[0] = acc;
}

// The same tiled stream with the hot path's access sizes: each load reads a
// 12-byte unit (one dwordx3, as the kernels' units of 4 u8, 2 binary16 or 1
// binary32 pixels) and each store writes 8 bytes (two FP32 outputs, as the
// curve pass stores a binary16 unit's T). Tile j: VR * 256 units of src from
// j * VR * 256 on, VW * 256 8-byte words of dst from j * VW * 256 on.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <int VR, int VW>
__global__ __launch_bounds__(256) void k_stream12(const unsigned *__restrict__ src, int64_t nr,
                                                  u32x2 *__restrict__ dst, int64_t nw,
                                                  int64_t ntiles, unsigned *__restrict__ sink)
{
    unsigned acc = 0;
    for (int64_t j = blockIdx.x; j < ntiles; j += gridDim.x) {
        unsigned v[VR > 0 ? VR : 1][3];
#pragma unroll
        for (int k = 0; k < VR; ++k) {
            const int64_t i = (j * VR + k) * 256 + threadIdx.x;
            if (i < nr) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    v[k][c] = __builtin_nontemporal_load(src + 3 * i + c);
            } else {
                v[k][0] = v[k][1] = v[k][2] = 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < VR; ++k)
            acc ^= v[k][0] ^ v[k][1] ^ v[k][2];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            const int64_t i = (j * VW + k) * 256 + threadIdx.x;
            if (i < nw)
                __builtin_nontemporal_store(u32x2{acc, (unsigned)i}, dst + i);
        }
    }
    if (acc == 0x5ca1ab1eu)
        sink[0] = acc;
}

// One stage of a lagged two-pass schedule over images of tpi tiles (a tile:
// 6 x 256 vectors of input, 4 x 256 of output, the byte ratio of binary16 RGB
// to FP32 gray): item 2j reads tile j of image s (plain loads, so the lines
// may stay in the last-level cache), item 2j + 1 reads tile j of image s - 1
// again (nontemporal) and writes that tile's output. Stage 0 has only the
// first kind, stage nimg only the second.
__global__ __launch_bounds__(256) void k_stage(const u32x4 *__restrict__ in, u32x4 *__restrict__ out,
                                               int s, int nimg, int64_t tpi,
                                               unsigned *__restrict__ sink)
{
    const bool has1 = s < nimg, has2 = s >= 1;
    const int64_t items = (has1 ? tpi : 0) + (has2 ? tpi : 0);
    unsigned acc = 0;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const bool first = has1 && has2 ? (it & 1) == 0 : has1;
        const int64_t j = has1 && has2 ? it >> 1 : it;
        const int img = first ? s : s - 1;
        const u32x4 *src = in + ((int64_t)img * tpi + j) * 6 * 256 + threadIdx.x;
        u32x4 v[6];
        if (first) {
#pragma unroll
            for (int k = 0; k < 6; ++k)
                v[k] = src[k * 256];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k)
                v[k] = __builtin_nontemporal_load(src + k * 256);
            u32x4 *dst = out + ((int64_t)img * tpi + j) * 4 * 256 + threadIdx.x;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                __builtin_nontemporal_store(v[k] ^ v[k + 2], dst + k * 256);
        }
    }
    if (acc == 0x5ca1ab1eu)
        sink[0] = acc;
}

// One stage of a lagged schedule that parks a 4-byte per-pixel intermediate
// between the passes instead of re-reading the input: item 2j reads tile j of
// image s (6 x 256 vectors, nontemporal) and writes its intermediate (4 x 256
// vectors, plain stores, so the lines may stay in the last-level cache); item
// 2j + 1 reads the intermediate of tile j of image s - 1 back (plain loads) and
// writes that tile's output (4 x 256 vectors, nontemporal). Stage 0 has only
// the first kind, stage nimg only the second.
__global__ __launch_bounds__(256) void k_stage_parked(const u32x4 *__restrict__ in,
                                                      u32x4 *__restrict__ mid,
                                                      u32x4 *__restrict__ out, int s, int nimg,
                                                      int64_t tpi, unsigned *__restrict__ sink)
{
    const bool has1 = s < nimg, has2 = s >= 1;
    const int64_t items = (has1 ? tpi : 0) + (has2 ? tpi : 0);
    unsigned acc = 0;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const bool first = has1 && has2 ? (it & 1) == 0 : has1;
        const int64_t j = has1 && has2 ? it >> 1 : it;
        const int img = first ? s : s - 1;
        const int64_t t = (int64_t)img * tpi + j;
        if (first) {
            const u32x4 *src = in + t * 6 * 256 + threadIdx.x;
            u32x4 v[6];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                v[k] = __builtin_nontemporal_load(src + k * 256);
            u32x4 *dst = mid + t * 4 * 256 + threadIdx.x;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                dst[k * 256] = v[k] ^ v[k + 2];
        } else {
            const u32x4 *src = mid + t * 4 * 256 + threadIdx.x;
            u32x4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                v[k] = src[k * 256];
            u32x4 *dst = out + t * 4 * 256 + threadIdx.x;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                __builtin_nontemporal_store(v[k] ^ u32x4{1u, 2u, 3u, 4u}, dst + k * 256);
            acc ^= v[0].x;
        }
    }
    if (acc == 0x5ca1ab1eu)
        sink[0] = acc;
}

} // namespace

extern "C" {

// Enqueues one pass that reads src_bytes of src and writes dst_bytes of dst
// (sizes rounded down to 16 bytes; both pointers 16-byte aligned), as
// `reads` : `writes` 16-byte vectors per thread and tile, one of (8, 0),
// (0, 8), (6, 4), (3, 5), (4, 4); a stream with 0 vectors per tile is skipped.
// The tile count follows the longer stream at that ratio, so give sizes in the
// same ratio for a pass that mixes reads and writes throughout. grid = number
// of 256-thread workgroups, or 0 for one workgroup per tile. sink is a device
// word. Returns the hipError_t of the launch.
int dcx_stream(const void *src, int64_t src_bytes, void *dst, int64_t dst_bytes, int reads,
               int writes, int grid, void *sink, void *stream)
{
    const int64_t nr = reads > 0 ? src_bytes / 16 : 0, nw = writes > 0 ? dst_bytes / 16 : 0;
    const int64_t tr = reads > 0 ? (nr + reads * 256 - 1) / (reads * 256) : 0;
    const int64_t tw = writes > 0 ? (nw + writes * 256 - 1) / (writes * 256) : 0;
    const int64_t ntiles = tr > tw ? tr : tw;
    const u32x4 *s = (const u32x4 *)src;
    u32x4 *d = (u32x4 *)dst;
    unsigned *k = (unsigned *)sink;
    hipStream_t st = (hipStream_t)stream;
    if (grid < 0 || ntiles < 1 || ntiles > 0x7fffffff)
        return (int)hipErrorInvalidValue;
    const unsigned g = (unsigned)(grid > 0 && grid < ntiles ? grid : ntiles);
#define DCX_LAUNCH(R, W) \
    hipLaunchKernelGGL((k_stream<R, W>), dim3(g), dim3(256), 0, st, s, nr, d, nw, ntiles, k)
    switch (reads * 16 + writes) {
    case 8 * 16 + 0: DCX_LAUNCH(8, 0); break;
    case 0 * 16 + 8: DCX_LAUNCH(0, 8); break;
    case 6 * 16 + 4: DCX_LAUNCH(6, 4); break;
    case 3 * 16 + 5: DCX_LAUNCH(3, 5); break;
    case 4 * 16 + 4: DCX_LAUNCH(4, 4); break;
    default: return (int)hipErrorInvalidValue;
    }
#undef DCX_LAUNCH
    return (int)hipGetLastError();
}

// As dcx_stream with 12-byte loads and 8-byte stores (the hot path's unit
// sizes): src_bytes / 12 units read and dst_bytes / 8 words written, as
// `reads` : `writes` per thread and tile, one of (8, 0), (6, 6) (the curve
// pass's 12 : 8 bytes), (0, 8). src 4-byte and dst 8-byte aligned.
int dcx_stream12(const void *src, int64_t src_bytes, void *dst, int64_t dst_bytes, int reads,
                 int writes, int grid, void *sink, void *stream)
{
    const int64_t nr = reads > 0 ? src_bytes / 12 : 0, nw = writes > 0 ? dst_bytes / 8 : 0;
    const int64_t tr = reads > 0 ? (nr + reads * 256 - 1) / (reads * 256) : 0;
    const int64_t tw = writes > 0 ? (nw + writes * 256 - 1) / (writes * 256) : 0;
    const int64_t ntiles = tr > tw ? tr : tw;
    if (grid < 0 || ntiles < 1 || ntiles > 0x7fffffff)
        return (int)hipErrorInvalidValue;
    const unsigned g = (unsigned)(grid > 0 && grid < ntiles ? grid : ntiles);
    const unsigned *s = (const unsigned *)src;
    u32x2 *d = (u32x2 *)dst;
    unsigned *k = (unsigned *)sink;
    hipStream_t st = (hipStream_t)stream;
#define DCX_LAUNCH12(R, W) \
    hipLaunchKernelGGL((k_stream12<R, W>), dim3(g), dim3(256), 0, st, s, nr, d, nw, ntiles, k)
    switch (reads * 16 + writes) {
    case 8 * 16 + 0: DCX_LAUNCH12(8, 0); break;
    case 6 * 16 + 6: DCX_LAUNCH12(6, 6); break;
    case 0 * 16 + 8: DCX_LAUNCH12(0, 8); break;
    default: return (int)hipErrorInvalidValue;
    }
#undef DCX_LAUNCH12
    return (int)hipGetLastError();
}

// Enqueues stage s (0 <= s <= nimg) of the lagged two-pass schedule over nimg
// images of tpi tiles each: in holds nimg * tpi * 24 KiB, out nimg * tpi *
// 16 KiB (16-byte aligned). grid = workgroups, or 0 for one per item.
int dcx_stage(const void *in, void *out, int s, int nimg, int64_t tpi, int grid, void *sink,
              void *stream)
{
    if (s < 0 || s > nimg || nimg < 1 || tpi < 1 || grid < 0)
        return (int)hipErrorInvalidValue;
    const int64_t items = (s < nimg ? tpi : 0) + (s >= 1 ? tpi : 0);
    if (items > 0x7fffffff)
        return (int)hipErrorInvalidValue;
    const unsigned g = (unsigned)(grid > 0 && grid < items ? grid : items);
    hipLaunchKernelGGL(k_stage, dim3(g), dim3(256), 0, (hipStream_t)stream, (const u32x4 *)in,
                       (u32x4 *)out, s, nimg, tpi, (unsigned *)sink);
    return (int)hipGetLastError();
}

// Enqueues stage s (0 <= s <= nimg) of the lagged parked schedule over nimg
// images of tpi tiles each: in holds nimg * tpi * 24 KiB, mid and out
// nimg * tpi * 16 KiB each (16-byte aligned). grid = workgroups, or 0 for one
// per item.
int dcx_stage_parked(const void *in, void *mid, void *out, int s, int nimg, int64_t tpi,
                     int grid, void *sink, void *stream)
{
    if (s < 0 || s > nimg || nimg < 1 || tpi < 1 || grid < 0)
        return (int)hipErrorInvalidValue;
    const int64_t items = (s < nimg ? tpi : 0) + (s >= 1 ? tpi : 0);
    if (items > 0x7fffffff)
        return (int)hipErrorInvalidValue;
    const unsigned g = (unsigned)(grid > 0 && grid < items ? grid : items);
    hipLaunchKernelGGL(k_stage_parked, dim3(g), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4 *)in, (u32x4 *)mid, (u32x4 *)out, s, nimg, tpi,
                       (unsigned *)sink);
    return (int)hipGetLastError();
}

} // extern "C"
