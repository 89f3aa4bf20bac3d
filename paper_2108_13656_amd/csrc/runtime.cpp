// Host runtime behind include/decolor.h: argument validation, the context and
// its workspace ring, the per-image walk classification and tile tables, the
// launch sequences of the compute entry points (decolorization, weight sweep,
// comparator channels, global and local tone map), plans with HIP-graph
// capture, the autotuner and the continuous-batching server.
#include "../../include/decolor.h"
#include "dc_internal.h"
#include "serve_policy.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

namespace {

thread_local std::string g_last_error;

// Environment switches, read once: DC_LOG_LEVEL (0 = silent, the default;
// 1 = every failing call prints its message to stderr; 2 = also the
// autotuner's choices and server creation), DC_AUTOTUNE (0 = dc_autotune keeps
// the shapes in place without measuring; anything else, or unset, tunes).
int env_int(const char *name, int fallback)
{
    const char *v = std::getenv(name);
    if (!v || !*v)
        return fallback;
    char *end = nullptr;
    const long x = std::strtol(v, &end, 10);
    return end && *end == '\0' ? (int)x : fallback;
}

int log_level()
{
    static const int level = env_int("DC_LOG_LEVEL", 0);
    return level;
}

bool autotune_enabled()
{
    static const bool on = env_int("DC_AUTOTUNE", 1) != 0;
    return on;
}

void log_msg(int level, const std::string &msg)
{
    if (log_level() >= level)
        std::fprintf(stderr, "[decolor] %s\n", msg.c_str());
}

int fail(int status, const std::string &msg)
{
    g_last_error = msg;
    log_msg(1, "error " + std::to_string(status) + ": " + msg);
    return status;
}

// A named host range around an entry point or a server step, visible to
// `rocprofv3 --marker-trace` next to the kernels it enqueues (a no-op cost
// when no tracer is attached).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePush(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Runs the body of an entry point so that no C++ exception crosses the C
// interface: a failed host allocation becomes DC_ERR_NO_MEMORY, a size beyond
// the host containers' limits DC_ERR_INVALID_ARG.
template <class F>
int guarded(F &&body) noexcept
{
    auto note = [](int status, const char *msg) noexcept {
        try {
            g_last_error = msg;
        } catch (...) {
            g_last_error.clear();
        }
        return status;
    };
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return note(DC_ERR_NO_MEMORY, "host memory allocation failed");
    } catch (const std::length_error &) {
        return note(DC_ERR_INVALID_ARG, "sizes exceed what the host containers hold");
    } catch (...) {
        return note(DC_ERR_INVALID_ARG, "unexpected host exception");
    }
}

bool dtype_ok(int32_t d) { return d == DC_U8 || d == DC_F16 || d == DC_F32; }

struct Range {
    uintptr_t lo, hi; // [lo, hi)
    int image;
    int kind; // 0 src, 1 dst, 2 dst2
};

const char *kind_name(int k) { return k == 0 ? "src" : (k == 1 ? "dst" : "dst2"); }

// Byte extent of a 2-D buffer: (height - 1) rows of pitch plus one row. Returns
// false on int64 overflow.
bool extent(const void *base, int64_t pitch, int64_t row_bytes, int32_t height, Range &r)
{
    const __int128 span = (__int128)pitch * (height - 1) + row_bytes;
    if (span > (__int128)INT64_MAX)
        return false;
    const __int128 hi = (__int128)(uintptr_t)base + span;
    if (hi > (__int128)UINTPTR_MAX)
        return false;
    r.lo = (uintptr_t)base;
    r.hi = (uintptr_t)hi;
    return true;
}

int validate_params(const dc_params *p)
{
    if (!p)
        return DC_OK;
    const float b[2] = {p->beta_r, p->beta_k};
    for (float v : b)
        if (!std::isfinite(v) || v < 0.0f || v > 1.0f)
            return fail(DC_ERR_INVALID_ARG, "beta_r and beta_k must be finite and in [0, 1]");
    return DC_OK;
}

int validate_tm(const dc_tm_params *tm)
{
    if (!tm)
        return DC_OK;
    const float v[3] = {tm->eps, tm->contrast, tm->sigma_floor};
    for (float x : v)
        if (!std::isfinite(x) || !(x > 0.0f))
            return fail(DC_ERR_INVALID_ARG, "eps, contrast and sigma_floor must be finite and > 0");
    if (!(tm->saturation >= 0.0f && tm->saturation <= 2.0f))
        return fail(DC_ERR_INVALID_ARG, "saturation must be in [0, 2]");
    if (!(tm->local_strength >= 0.0f && tm->local_strength <= 1.0f))
        return fail(DC_ERR_INVALID_ARG, "local_strength must be in [0, 1]");
    return DC_OK;
}

// Checks of the input half of a descriptor; fills its byte extent. at is the
// descriptor's label for messages (anything convertible to std::string).
template <class Label>
int check_src(const dc_image &m, const Label &at, Range &r)
{
    if (!m.src)
        return fail(DC_ERR_INVALID_ARG, "src must not be NULL" + std::string(at));
    if (m.width < 1 || m.height < 1)
        return fail(DC_ERR_INVALID_ARG, "width and height must be >= 1" + std::string(at));
    if (!dtype_ok(m.src_dtype))
        return fail(DC_ERR_INVALID_ARG, "src_dtype must be DC_U8, DC_F16 or DC_F32" + std::string(at));
    const int64_t es = dc::elem_size(m.src_dtype);
    const int64_t row_in = 3 * es * (int64_t)m.width;
    if (m.src_pitch < row_in)
        return fail(DC_ERR_INVALID_ARG, "src_pitch is smaller than 3 * width * element size" + std::string(at));
    if ((uintptr_t)m.src % es || m.src_pitch % es)
        return fail(DC_ERR_INVALID_ARG, "src and src_pitch must be multiples of the element size" + std::string(at));
    if (!extent(m.src, m.src_pitch, row_in, m.height, r))
        return fail(DC_ERR_INVALID_ARG, "src extent overflows" + std::string(at));
    return DC_OK;
}

// allowed: the dc_image flags this call accepts (DC_IMG_RGB_OUT for the tone
// map, DC_IMG_HOST_SRC for server requests); other known flags are
// DC_ERR_UNSUPPORTED, unknown bits DC_ERR_INVALID_ARG.
// outs_buf and ins_buf, when given, are the work lists (cleared here; with
// enough capacity reserved the check makes no host allocation on success).
int validate_images(const dc_image *imgs, int32_t n, int32_t allowed,
                    std::vector<Range> *outs_buf = nullptr, std::vector<Range> *ins_buf = nullptr)
{
    if (n < 0)
        return fail(DC_ERR_INVALID_ARG, "n must be >= 0");
    if (n > 0 && !imgs)
        return fail(DC_ERR_INVALID_ARG, "image list is NULL");
    std::vector<Range> outs_own, ins_own;
    std::vector<Range> &outs = outs_buf ? *outs_buf : outs_own;
    std::vector<Range> &ins = ins_buf ? *ins_buf : ins_own;
    outs.clear();
    ins.clear();
    outs.reserve((size_t)n * 2);
    ins.reserve((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const dc_image &m = imgs[i];
        // The image's label, built only for a message.
        struct At {
            int32_t i;
            operator std::string() const { return " (image " + std::to_string(i) + ")"; }
        } const at{i};
        if (!m.src || !m.dst)
            return fail(DC_ERR_INVALID_ARG, "src and dst must not be NULL" + std::string(at));
        if (m.width < 1 || m.height < 1)
            return fail(DC_ERR_INVALID_ARG, "width and height must be >= 1" + std::string(at));
        if (m.flags & ~(DC_IMG_RGB_OUT | DC_IMG_HOST_SRC))
            return fail(DC_ERR_INVALID_ARG, "unknown flags" + std::string(at));
        if ((m.flags & DC_IMG_RGB_OUT) && !(allowed & DC_IMG_RGB_OUT))
            return fail(DC_ERR_UNSUPPORTED, "DC_IMG_RGB_OUT applies to the tone map only" + std::string(at));
        if ((m.flags & DC_IMG_HOST_SRC) && !(allowed & DC_IMG_HOST_SRC))
            return fail(DC_ERR_UNSUPPORTED, "DC_IMG_HOST_SRC applies to server requests only" + std::string(at));
        if (!dtype_ok(m.src_dtype) || !dtype_ok(m.dst_dtype))
            return fail(DC_ERR_INVALID_ARG, "src_dtype and dst_dtype must be DC_U8, DC_F16 or DC_F32" + std::string(at));
        if (m.dst2_dtype == DC_NONE) {
            if (m.dst2)
                return fail(DC_ERR_INVALID_ARG, "dst2 must be NULL when dst2_dtype is DC_NONE" + std::string(at));
        } else {
            if (!dtype_ok(m.dst2_dtype))
                return fail(DC_ERR_INVALID_ARG, "dst2_dtype must be DC_NONE, DC_U8, DC_F16 or DC_F32" + std::string(at));
            if (!m.dst2)
                return fail(DC_ERR_INVALID_ARG, "dst2 is NULL but dst2_dtype is set" + std::string(at));
        }
        Range r;
        const int src_rc = check_src(m, at, r);
        if (src_rc != DC_OK)
            return src_rc;
        r.image = i;
        r.kind = 0;
        ins.push_back(r);
        const void *op[2] = {m.dst, m.dst2};
        const int64_t pitch[2] = {m.dst_pitch, m.dst2_pitch};
        const int32_t dt[2] = {m.dst_dtype, m.dst2_dtype};
        for (int o = 0; o < 2; ++o) {
            if (!op[o])
                continue;
            const int64_t eo = dc::elem_size(dt[o]);
            const int64_t ch = (o == 0 && (m.flags & DC_IMG_RGB_OUT)) ? 3 : 1;
            const int64_t row = ch * eo * (int64_t)m.width;
            if (pitch[o] < row)
                return fail(DC_ERR_INVALID_ARG, std::string(kind_name(o + 1)) +
                                                    "_pitch is smaller than its row bytes" + std::string(at));
            if ((uintptr_t)op[o] % eo || pitch[o] % eo)
                return fail(DC_ERR_INVALID_ARG, std::string(kind_name(o + 1)) +
                                                    " and its pitch must be multiples of the element size" + std::string(at));
            if (!extent(op[o], pitch[o], row, m.height, r))
                return fail(DC_ERR_INVALID_ARG, std::string(kind_name(o + 1)) + " extent overflows" + std::string(at));
            r.image = i;
            r.kind = o + 1;
            outs.push_back(r);
        }
    }
    // No output may overlap another output or any input (inputs may be shared).
    auto by_lo = [](const Range &a, const Range &b) { return a.lo < b.lo; };
    std::sort(outs.begin(), outs.end(), by_lo);
    for (size_t j = 1; j < outs.size(); ++j)
        if (outs[j].lo < outs[j - 1].hi)
            return fail(DC_ERR_ALIAS, std::string(kind_name(outs[j].kind)) + " of image " +
                                          std::to_string(outs[j].image) + " overlaps " +
                                          kind_name(outs[j - 1].kind) + " of image " +
                                          std::to_string(outs[j - 1].image));
    for (const Range &in : ins) {
        // The output with the largest lo below in.hi is the only candidate
        // that can overlap, since outputs are disjoint and sorted.
        auto it = std::lower_bound(outs.begin(), outs.end(), Range{in.hi, 0, 0, 0}, by_lo);
        if (it != outs.begin()) {
            const Range &o = *(it - 1);
            if (o.hi > in.lo)
                return fail(DC_ERR_ALIAS, std::string(kind_name(o.kind)) + " of image " +
                                              std::to_string(o.image) + " overlaps src of image " +
                                              std::to_string(in.image));
        }
    }
    return DC_OK;
}

// Constants of the per-pixel forms. The division-free form (8-bit and
// binary16 input) carries sqrt(3) S scaling (cr, cg scaled by 3; ck, cc by
// 1/3); the normalised form (binary32 input) uses the plain weights. Computed
// in double, rounded once.
dc::Coef coef_of(const dc_params *p, int src_dtype)
{
    const double br = p ? p->beta_r : 0.55, bk = p ? p->beta_k : 0.80;
    if (src_dtype != DC_F32)
        return dc::Coef{(float)(3.0 * br), (float)(3.0 * (1.0 - br)), (float)(bk / 3.0),
                        (float)((1.0 - bk) / 3.0)};
    return dc::Coef{(float)br, (float)(1.0 - br), (float)bk, (float)(1.0 - bk)};
}

dc::TmArgs tm_of(const dc_tm_params *tm)
{
    return tm ? dc::TmArgs{tm->eps, tm->contrast, tm->sigma_floor, tm->saturation,
                           tm->local_strength}
              : dc::TmArgs{1e-4f, 2.0f, 1e-3f, 1.0f, 0.5f};
}

// Walk of an image for the tile-table kernels: packed rows are one segment
// (the packed walk from a 4-byte aligned start, else the row walk with zero
// gaps); pitched rows take the row walk unless the width or the padding is past
// what its 32-bit arithmetic covers (or W < 4, where a unit split by a row
// break could reach past the next row), then one segment per row, pixel by
// pixel.
int walk_of(const dc_image &m)
{
    const int64_t W = m.width, H = m.height;
    const int64_t es = dc::elem_size(m.src_dtype);
    const int64_t e1 = dc::elem_size(m.dst_dtype) * ((m.flags & DC_IMG_RGB_OUT) ? 3 : 1);
    const int64_t e2 = m.dst2 ? dc::elem_size(m.dst2_dtype) : 0;
    const int64_t gs = m.src_pitch - 3 * es * W, gd = m.dst_pitch - e1 * W;
    const int64_t g2 = m.dst2 ? m.dst2_pitch - e2 * W : 0;
    // The packed walk's unit loads are buffer loads from each tile's first
    // byte, which must be 4-byte aligned: tiles start at multiples of 12 bytes
    // from the image's first byte, so that byte must be. Packed rows at an
    // unaligned start take the row walk with zero gaps, whose tiles, units and
    // addresses are the packed walk's (every row offset q * gap is 0, and a
    // unit across a row break is contiguous), so the results are the same
    // bits, for any width.
    const bool aligned = ((uintptr_t)m.src & 3u) == 0;
    if (H == 1 || (gs == 0 && gd == 0 && g2 == 0))
        return aligned ? dc::kWalkPacked : dc::kWalkRows;
    if (W >= 4 && W <= dc::kRowWalkMaxWidth && gs < dc::kRowWalkMaxGap &&
        gd < dc::kRowWalkMaxGap && g2 < dc::kRowWalkMaxGap)
        return dc::kWalkRows;
    return dc::kWalkScalar;
}

// Walk classification and tile count of one image for tiles of tile_px pixels.
dc::DevImage describe(const dc_image &m, int index, int64_t tile_px, const dc_params *params)
{
    dc::DevImage d;
    std::memset(&d, 0, sizeof(d));
    d.src = (const uint8_t *)m.src;
    d.dst = (uint8_t *)m.dst;
    d.dst2 = (uint8_t *)m.dst2;
    d.src_dtype = m.src_dtype;
    d.dst_dtype = m.dst_dtype;
    d.dst2_dtype = m.dst2 ? m.dst2_dtype : DC_NONE;
    d.image = index;
    d.rgb_out = (m.flags & DC_IMG_RGB_OUT) ? 1 : 0;
    d.unit = m.src_dtype == DC_U8 ? (float)(1.0 / 255.0) : 1.0f;
    d.npx = (int64_t)m.width * m.height;
    d.width = m.width;
    d.height = m.height;
    d.k = coef_of(params, m.src_dtype);

    const int64_t W = m.width, H = m.height;
    const int64_t es = dc::elem_size(m.src_dtype);
    const int64_t e1 = dc::elem_size(m.dst_dtype) * (d.rgb_out ? 3 : 1); // dst bytes per pixel
    const int64_t e2 = m.dst2 ? dc::elem_size(m.dst2_dtype) : 0;
    const int64_t gs = m.src_pitch - 3 * es * W, gd = m.dst_pitch - e1 * W;
    const int64_t g2 = m.dst2 ? m.dst2_pitch - e2 * W : 0;
    // Any element-aligned base takes the vector units (the target serves
    // unaligned dword accesses). Packed rows are one segment; pitched rows are
    // tiled the same way over W * H pixels, with the row breaks placed per unit
    // (the row walk), or else one segment per row (walk_of).
    const int walk = walk_of(m);
    const bool packed = walk == dc::kWalkPacked, rows = walk == dc::kWalkRows;
    d.src_seg_stride = m.src_pitch;
    d.dst_seg_stride = m.dst_pitch;
    d.dst2_seg_stride = m.dst2 ? m.dst2_pitch : 0;
    int64_t nseg;
    if (packed || rows) {
        d.walk = packed ? dc::kWalkPacked : dc::kWalkRows;
        d.seg_len = W * H;
        nseg = 1;
        if (!packed) {
            d.magic = (uint32_t)(((uint64_t)1 << 32) / (uint64_t)W +
                                 (((uint64_t)1 << 32) % (uint64_t)W != 0));
            // One row, or rows without padding: every row offset is 0 (the
            // pitch of a single row is never used).
            const bool nogap = H == 1 || (gs == 0 && gd == 0 && g2 == 0);
            d.gap_src = nogap ? 0u : (uint32_t)gs;
            d.gap_dst = nogap ? 0u : (uint32_t)gd;
            d.gap_dst2 = nogap ? 0u : (uint32_t)g2;
        }
    } else {
        d.walk = dc::kWalkScalar;
        d.seg_len = W;
        nseg = H;
    }
    d.tiles_per_seg = (d.seg_len + tile_px - 1) / tile_px;
    d.ntiles = d.tiles_per_seg * nseg;
    return d;
}

// Local tone map: a grid of kLtmTile-square tiles per image, walked row by
// row inside a tile. Unit loads need 4-byte aligned rows; unit stores of the
// outputs the same 16-byte alignment as the other walks, else per pixel.
dc::DevImage describe_local(const dc_image &m, int index, const dc_params *params)
{
    dc::DevImage d = describe(m, index, dc::kStatsChunkPx, params);
    const int64_t W = m.width, H = m.height;
    const int64_t nx = (W + dc::kLtmTile - 1) / dc::kLtmTile;
    const int64_t ny = (H + dc::kLtmTile - 1) / dc::kLtmTile;
    d.width = m.width;
    d.height = m.height;
    d.seg_len = W;
    d.tiles_per_seg = nx;
    d.ntiles = nx * ny;
    d.src_seg_stride = m.src_pitch;
    d.dst_seg_stride = m.dst_pitch;
    d.dst2_seg_stride = m.dst2 ? m.dst2_pitch : 0;
    const bool src4 = (uintptr_t)m.src % 4 == 0 && m.src_pitch % 4 == 0;
    const bool out16 = (uintptr_t)m.dst % 16 == 0 && m.dst_pitch % 16 == 0 &&
                       (!m.dst2 || ((uintptr_t)m.dst2 % 16 == 0 && m.dst2_pitch % 16 == 0));
    d.walk = (src4 && out16) ? dc::kWalkRows : dc::kWalkScalar;
    d.staged = (m.dst_dtype == DC_F32 && !(m.flags & DC_IMG_RGB_OUT)) ? 1 : 0;
    return d;
}

} // namespace

// ------------------------------------------------------------------ context

// Launch shapes. groups = vector groups per thread in a decolorization tile
// (per input type, and one value for batches that mix input types); *_gpc =
// persistent workgroups per compute unit (0 = one workgroup per tile).
// Defaults are the shapes the autotuner picked on MI355X for the 64-frame
// video batch (u8) and the 16 x 4096^2 binary16 tone map.
struct Tune {
    int groups[3] = {1, 2, 2};
    int mixed_groups = 1;
    int decolor_gpc = 0;
    int mixed_gpc = 0;
    int pass1_gpc = 16;
    int pass2_gpc = 0;
    int tm_pipeline = 0; // m >= 1: the tone map in groups of m images on two streams
};

namespace {
struct NoAlloc;
}

struct dc_ctx {
    static constexpr int kSlots = 16;
    struct Slot {
        void *host = nullptr;  // pinned staging of the descriptor table
        size_t host_cap = 0;
        void *dev = nullptr;   // device table, tile ends, partials, curves
        size_t dev_cap = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
    };
    int device = 0;
    int num_cu = 256;
    Tune tune;
    // Second stream and fork/join events of the per-image tone-map pipeline.
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> fork;
    Slot slots[kSlots];
    int next = 0;
    // Measurement hooks: timing events recorded around each kernel.
    static constexpr int kMaxEvents = 8;
    bool profiling = false;
    hipEvent_t prof[kMaxEvents] = {};
    int prof_used = 0;
    // dc_tonemap_global_noalloc: the device address of the fixed scratch array
    // on this context's device, and the host state set up for it here.
    void *scratch = nullptr;
    NoAlloc *na = nullptr;
};

namespace {

int hip_fail(hipError_t e, const char *what)
{
    return fail(DC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Records timing event i on the stream when profiling is on.
void mark(dc_ctx *ctx, bool on, int i, hipStream_t s)
{
    if (!on || !ctx->profiling || i >= dc_ctx::kMaxEvents)
        return;
    if (i == 0)
        ctx->prof_used = 0;
    if (hipEventRecord(ctx->prof[i], s) == hipSuccess)
        ctx->prof_used = i + 1;
}

int ensure_prof_events(dc_ctx *ctx)
{
    if (ctx->prof[0])
        return DC_OK;
    for (auto &e : ctx->prof) {
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess)
            return fail(DC_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(err));
    }
    return DC_OK;
}

int64_t grid_blocks(const dc_ctx *ctx, int gpc) { return gpc > 0 ? (int64_t)gpc * ctx->num_cu : 0; }

// Host image of a launch: descriptors, tile prefix and the launch shape that
// the tile sizes were built for.
struct HostTable {
    std::vector<dc::DevImage> d;
    std::vector<int64_t> tile_end;
    std::vector<int64_t> grp_end; // tone map: inclusive prefix of level-2 partial counts
    int64_t total_tiles = 0;
    int64_t total_grps = 0;
    bool mixed = false;
    int src0 = 0;
    int groups = 2;  // decolorization only
    bool tonemap = false; // statistics workspace (global and local tone map)
    bool local = false;   // local tone map: histograms and curve tables too
    // Tone map and channels: the table is stably sorted by input type (then
    // gray before colour output); runs[k] = {first image, end image, type,
    // colour output} of each run, so each pass launches its per-type kernel
    // once per run.
    // Every table is sorted so that images on the row walk form runs of their
    // own (rows = 1): a launch covers images of one walk kind.
    struct Run {
        int img0, img1, src, rgb, staged, rows;
    };
    std::vector<Run> runs;
    std::vector<int32_t> order; // build_table's sort permutation (kept for its capacity)
    // Reserves room for n images, so that build_table makes no host
    // allocation for a call of up to n images.
    void reserve(size_t n)
    {
        d.reserve(n);
        tile_end.reserve(n);
        grp_end.reserve(n);
        runs.reserve(n);
        order.reserve(n);
    }
};

// kind of table: decolorization (tiles of the tuned group count), tone map
// (fixed 4096-pixel tiles, sorted by input type) or comparator channel (one
// 48-byte group per thread, sorted by input type).
enum TableKind { kTabDecolor = 0, kTabTonemap = 1, kTabChannel = 2, kTabLocal = 3 };

// per_image, when not NULL, holds one dc_params per image (in the caller's
// order) and overrides params.
void build_table(const dc_image *imgs, int32_t n, const dc_params *params, TableKind kind,
                 const Tune &tune, HostTable &h, const dc_params *per_image = nullptr)
{
    const bool tonemap = kind == kTabTonemap || kind == kTabLocal;
    h.d.resize((size_t)n);
    h.tile_end.resize((size_t)n);
    h.grp_end.resize((size_t)n);
    h.tonemap = tonemap;
    h.local = kind == kTabLocal;
    h.src0 = n > 0 ? imgs[0].src_dtype : 0;
    h.mixed = false;
    for (int32_t i = 0; i < n; ++i)
        h.mixed |= imgs[i].src_dtype != h.src0;
    h.groups = h.mixed ? tune.mixed_groups : tune.groups[h.src0];
    std::vector<int32_t> &order = h.order;
    order.resize((size_t)n);
    for (int32_t i = 0; i < n; ++i)
        order[i] = i;
    // A stable order by (walk, input type, output kind) for the tone map and
    // the channels, by walk alone for decolorization: the caller's index
    // breaks ties, so std::sort (which needs no temporary buffer) gives it.
    // The local tone map has its own 2-D walk and ignores the row walk.
    auto rows_of = [&](int32_t i) { return kind != kTabLocal && walk_of(imgs[i]) == dc::kWalkRows; };
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const bool wa = rows_of(a), wb = rows_of(b);
        if (wa != wb)
            return wb;
        if (kind == kTabDecolor)
            return a < b;
        // then input type, then colour output, then (local tone map) FP32 staging
        auto key = [&](const dc_image &m) {
            const int rgb = (m.flags & DC_IMG_RGB_OUT) ? 2 : 0;
            return kind == kTabLocal ? (rgb ? rgb : (m.dst_dtype == DC_F32 ? 1 : 0)) : rgb;
        };
        const int ra = key(imgs[a]), rb = key(imgs[b]);
        if (imgs[a].src_dtype != imgs[b].src_dtype)
            return imgs[a].src_dtype < imgs[b].src_dtype;
        return ra != rb ? ra < rb : a < b;
    });
    h.runs.clear();
    int64_t total = 0;
    for (int32_t i = 0; i < n; ++i) {
        const dc_image &m = imgs[order[i]];
        const int64_t tile_px =
            tonemap ? dc::kStatsChunkPx
                    : (int64_t)dc::kBlock * (kind == kTabChannel ? 1 : h.groups) *
                          dc::group_px(m.src_dtype);
        const dc_params *pp = per_image ? &per_image[order[i]] : params;
        h.d[i] = kind == kTabLocal ? describe_local(m, order[i], pp)
                                   : describe(m, order[i], tile_px, pp);
        const int rgb = h.d[i].rgb_out, staged = h.d[i].staged;
        const int rows = kind != kTabLocal && h.d[i].walk == dc::kWalkRows;
        // decolorization runs split on the walk only (one launch handles mixed types)
        const int src = kind == kTabDecolor ? -1 : m.src_dtype;
        if (h.runs.empty() || h.runs.back().src != src || h.runs.back().rgb != rgb ||
            h.runs.back().staged != staged || h.runs.back().rows != rows)
            h.runs.push_back(HostTable::Run{i, i + 1, src, rgb, staged, rows});
        else
            h.runs.back().img1 = i + 1;
        h.d[i].tile_begin = total;
        h.d[i].chunk_begin = total * dc::kWavesPerBlock; // tone map: one partial per wave
        total += h.d[i].ntiles;
        h.tile_end[i] = total;
    }
    h.total_tiles = total;
    if (kind == kTabDecolor) {
        // inputs read for more than one image of the call keep cached loads
        std::vector<std::pair<const uint8_t *, int32_t>> srcs((size_t)n);
        for (int32_t i = 0; i < n; ++i)
            srcs[i] = {h.d[i].src, i};
        std::sort(srcs.begin(), srcs.end());
        for (int32_t i = 0; i + 1 < n; ++i)
            if (srcs[i].first == srcs[i + 1].first)
                h.d[srcs[i].second].shared_src = h.d[srcs[i + 1].second].shared_src = 1;
    }
    int64_t grps = 0;
    for (int32_t i = 0; i < n; ++i) {
        h.d[i].grp_begin = grps;
        h.d[i].ngrp = (h.d[i].ntiles * dc::kWavesPerBlock + dc::kBlock - 1) / dc::kBlock;
        grps += h.d[i].ngrp;
        h.grp_end[i] = grps;
    }
    h.total_grps = tonemap ? grps : 0;
}

// Byte layout of the device copy: table | tile ends | group ends (uploaded)
// then the workspace: wave partials | group partials | curves, and for the
// local tone map tile histograms | tile curve tables.
struct Layout {
    size_t table, ends, gends, counters, parts, parts2, curves, hist, coef, upload, total;
};

// The tone map's per-image combine counters are part of the upload, written
// as zeros with the table, so a staged call starts from zero whatever the
// slot held before; the combine leaves them zero again (plans upload once).
Layout layout_of(const HostTable &h)
{
    const size_t n = h.d.size();
    Layout l;
    l.table = 0;
    l.ends = align_up(sizeof(dc::DevImage) * n, 256);
    l.gends = l.ends + align_up(sizeof(int64_t) * n, 256);
    l.counters = l.gends + align_up(sizeof(int64_t) * n, 256);
    l.parts = l.counters + (h.tonemap ? align_up(sizeof(unsigned) * n, 256) : 0);
    l.upload = l.parts;
    l.parts2 = l.parts + (h.tonemap ? align_up(sizeof(dc::WavePart) * (size_t)h.total_tiles *
                                                   dc::kWavesPerBlock, 256) : 0);
    l.curves = l.parts2 + (h.tonemap ? align_up(sizeof(dc::Part) * (size_t)h.total_grps, 256) : 0);
    l.hist = l.curves + (h.tonemap ? align_up(sizeof(dc::Curve) * n, 256) : 0);
    const size_t nt = h.local ? (size_t)h.total_tiles : 0;
    l.coef = l.hist + align_up(sizeof(unsigned) * dc::kLtmBins * nt, 256);
    l.total = l.coef + align_up(sizeof(dc::LtmCoef) * dc::kLtmBins * nt, 256);
    return l;
}

void write_upload(const HostTable &h, const Layout &l, char *dst)
{
    std::memcpy(dst + l.table, h.d.data(), sizeof(dc::DevImage) * h.d.size());
    std::memcpy(dst + l.ends, h.tile_end.data(), sizeof(int64_t) * h.tile_end.size());
    std::memcpy(dst + l.gends, h.grp_end.data(), sizeof(int64_t) * h.grp_end.size());
    std::memset(dst + l.counters, 0, l.parts - l.counters);
}

static_assert(DC_NOALLOC_SCRATCH_BYTES == dc::kScratchBytes, "scratch size in the ABI header");
static_assert(DC_NOALLOC_MAX_IMAGES == dc::kScratchMaxImages, "scratch image limit in the ABI header");

// Host state of dc_tonemap_global_noalloc, set up by dc_create so that the
// entry point allocates nothing: the argument check's work lists and the table
// builder's arrays reserved for kScratchMaxImages images, and pinned staging
// for the descriptor upload with the event of its last copy.
struct NoAlloc {
    HostTable h;
    std::vector<Range> outs, ins;
    void *host = nullptr;
    size_t host_cap = 0;
    hipEvent_t copied = nullptr;
    bool pending = false;
};

// Bytes of the largest upload (table, tile ends, group ends, counters) of a call.
size_t noalloc_upload_cap()
{
    const size_t n = dc::kScratchMaxImages;
    return align_up(sizeof(dc::DevImage) * n, 256) + 2 * align_up(sizeof(int64_t) * n, 256) +
           align_up(sizeof(unsigned) * n, 256);
}

struct DevBufs {
    const dc::DevImage *table;
    const int64_t *tile_end;
    const int64_t *grp_end;
    unsigned *counters;
    dc::WavePart *parts;
    dc::Part *parts2;
    dc::Curve *curves;
    unsigned *hist;
    dc::LtmCoef *coef;
};

DevBufs bufs_of(void *dev, const Layout &l)
{
    char *p = (char *)dev;
    return DevBufs{(const dc::DevImage *)(p + l.table), (const int64_t *)(p + l.ends),
                   (const int64_t *)(p + l.gends), (unsigned *)(p + l.counters),
                   (dc::WavePart *)(p + l.parts),
                   (dc::Part *)(p + l.parts2), (dc::Curve *)(p + l.curves),
                   (unsigned *)(p + l.hist), (dc::LtmCoef *)(p + l.coef)};
}

// Kernel sequence of a decolorization launch over a staged table.
int enqueue_decolor(dc_ctx *ctx, const HostTable &h, const DevBufs &b, const Tune &t,
                    hipStream_t st, bool marks)
{
    mark(ctx, marks, 0, st);
    hipError_t e = hipSuccess;
    for (const auto &r : h.runs) {
        const int64_t t0 = h.d[r.img0].tile_begin, t1 = h.tile_end[r.img1 - 1];
        if (e == hipSuccess)
            e = dc::launch_decolor_table(b.table, b.tile_end, r.img0, r.img1 - r.img0, t0, t1,
                                         h.mixed, h.src0, h.groups, r.rows,
                                         grid_blocks(ctx, h.mixed ? t.mixed_gpc : t.decolor_gpc),
                                         st);
    }
    if (e != hipSuccess)
        return hip_fail(e, "decolorize launch");
    mark(ctx, marks, 1, st);
    return DC_OK;
}

// Weight sweep: when every image of a per-image-weights call reads the same
// input with the same geometry and output type (and has no second output),
// one pass over the input serves all of them. Returns the pairs per work item
// (the pairs split into chunks only as far as needed for about four
// workgroups per CU), or 0 when the table is not a sweep.
int sweep_per(const dc_ctx *ctx, const HostTable &h)
{
    const int n = (int)h.d.size();
    if (n < 2 || h.mixed)
        return 0;
    const dc::DevImage &a = h.d[0];
    for (const dc::DevImage &m : h.d)
        if (m.src != a.src || m.dst2 || m.dst_dtype != a.dst_dtype || m.walk != a.walk ||
            m.seg_len != a.seg_len || m.tiles_per_seg != a.tiles_per_seg ||
            m.ntiles != a.ntiles || m.src_seg_stride != a.src_seg_stride ||
            m.dst_seg_stride != a.dst_seg_stride)
            return 0;
    const int64_t want = 4 * (int64_t)ctx->num_cu;
    int64_t chunks = (want + a.ntiles - 1) / a.ntiles;
    chunks = chunks < 1 ? 1 : (chunks > n ? n : chunks);
    return (int)((n + chunks - 1) / chunks);
}

// Events for the grouped pipeline: fork[i] marks "statistics pass of group i
// done" on the main stream; fork[n] marks "side stream done".
int ensure_fork(dc_ctx *ctx, size_t n)
{
    if (!ctx->side) {
        hipError_t e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
        if (e != hipSuccess)
            return hip_fail(e, "hipStreamCreate");
    }
    while (ctx->fork.size() < n + 1) {
        hipEvent_t ev = nullptr;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess)
            return hip_fail(e, "hipEventCreate");
        ctx->fork.push_back(ev);
    }
    return DC_OK;
}

// Colour mode of a saturation: s = 0 grey, s = 1 ratio, anything else power.
int colour_mode(float saturation)
{
    return saturation == 0.0f ? dc::kColourGrey
                              : (saturation == 1.0f ? dc::kColourRatio : dc::kColourPow);
}

// Curve pass over tiles [t0, t1) of images img0 .. img0 + nimg - 1, all of
// input type src and all with (rgb) or without colour output.
hipError_t launch_curve(const DevBufs &b, int img0, int nimg, int64_t t0, int64_t t1, int src,
                        int rgb, int rows, dc::TmArgs a, int64_t grid, hipStream_t st)
{
    if (!rgb)
        return dc::launch_tm_pass2(b.table, b.tile_end, img0, nimg, t0, t1, 0, src, rows, a,
                                   b.curves, grid, st);
    return dc::launch_tm_colour(b.table, b.tile_end, img0, nimg, t0, t1, src,
                                colour_mode(a.saturation), rows, a, b.curves, grid, st);
}

// Kernel sequence of a tone map over a staged table. t.tm_pipeline = 0: the
// statistics pass over every image, the two-level combine, then the curve pass
// over every image. t.tm_pipeline = m >= 1: the images go in groups of m (runs
// of one input type and output kind split into chunks of m); a group's
// statistics pass runs on the caller's stream and its combine and curve pass
// on a second stream, so the curve pass of one group overlaps the statistics
// pass of the next (the VALU-bound statistics pass beside the memory-bound
// curve pass). Every schedule computes the same values: each kernel's
// per-image work is fixed.
// one_launch_combine: both combine levels in one kernel (one launch fewer,
// for the server's small latency-bound batches; the two-kernel form is faster
// on the device for large calls). Both give the same bits.
int enqueue_tonemap(dc_ctx *ctx, const HostTable &h, const DevBufs &b, const Tune &t,
                    dc::TmArgs a, dc::StatsOut *stats, hipStream_t st, bool marks,
                    bool one_launch_combine = false)
{
    const int n = (int)h.d.size();
    const int64_t g1 = grid_blocks(ctx, t.pass1_gpc), g2 = grid_blocks(ctx, t.pass2_gpc);
    hipError_t e = hipSuccess;
    if (!t.tm_pipeline || n == 0) {
        mark(ctx, marks, 0, st);
        for (const auto &r : h.runs) {
            const int64_t t0 = h.d[r.img0].tile_begin, t1 = h.tile_end[r.img1 - 1];
            if (e == hipSuccess)
                e = dc::launch_tm_pass1(b.table, b.tile_end, r.img0, r.img1 - r.img0, t0, t1, 0,
                                        r.src, r.rows, a, b.parts, g1, st);
        }
        mark(ctx, marks, 1, st);
        if (one_launch_combine) {
            if (e == hipSuccess)
                e = dc::launch_tm_combine_finalize(b.table, b.grp_end, 0, n, 0, h.total_grps, a,
                                                   b.parts, b.parts2, b.counters, b.curves, stats,
                                                   st);
        } else {
            if (e == hipSuccess)
                e = dc::launch_tm_combine(b.table, b.grp_end, 0, n, 0, h.total_grps, b.parts,
                                          b.parts2, st);
            if (e == hipSuccess)
                e = dc::launch_tm_finalize(b.table, 0, n, a, b.parts2, b.curves, stats, st);
        }
        mark(ctx, marks, 2, st);
        for (const auto &r : h.runs) {
            const int64_t t0 = h.d[r.img0].tile_begin, t1 = h.tile_end[r.img1 - 1];
            if (e == hipSuccess)
                e = launch_curve(b, r.img0, r.img1 - r.img0, t0, t1, r.src, r.rgb, r.rows, a, g2,
                                 st);
        }
        mark(ctx, marks, 3, st);
        if (e != hipSuccess)
            return hip_fail(e, "tonemap launch");
        return DC_OK;
    }
    const int m = t.tm_pipeline;
    size_t chunks = 0;
    for (const auto &r : h.runs)
        chunks += (size_t)((r.img1 - r.img0 + m - 1) / m);
    int rc = ensure_fork(ctx, chunks);
    if (rc != DC_OK)
        return rc;
    mark(ctx, marks, 0, st);
    size_t c = 0;
    for (const auto &r : h.runs) {
        for (int i0 = r.img0; i0 < r.img1 && e == hipSuccess; i0 += m, ++c) {
            const int k = std::min(m, r.img1 - i0);
            const int64_t t0 = h.d[i0].tile_begin, t1 = h.tile_end[i0 + k - 1];
            e = dc::launch_tm_pass1(b.table, b.tile_end, i0, k, t0, t1, 0, r.src, r.rows, a,
                                    b.parts, g1, st);
            if (e == hipSuccess)
                e = hipEventRecord(ctx->fork[c], st);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(ctx->side, ctx->fork[c], 0);
            if (e == hipSuccess)
                e = dc::launch_tm_combine(b.table, b.grp_end, i0, k, h.d[i0].grp_begin,
                                          h.grp_end[i0 + k - 1], b.parts, b.parts2, ctx->side);
            if (e == hipSuccess)
                e = dc::launch_tm_finalize(b.table, i0, k, a, b.parts2, b.curves, stats, ctx->side);
            if (e == hipSuccess)
                e = launch_curve(b, i0, k, t0, t1, r.src, r.rgb, r.rows, a, g2, ctx->side);
        }
    }
    if (e == hipSuccess)
        e = hipEventRecord(ctx->fork[chunks], ctx->side);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(st, ctx->fork[chunks], 0);
    mark(ctx, marks, 1, st);
    if (e != hipSuccess)
        return hip_fail(e, "tonemap pipeline launch");
    return DC_OK;
}

// Kernel sequence of the local tone map over a staged table: per input-type
// run the statistics-and-histogram pass over 64 x 64 tiles, the two-level
// statistics combine, the per-tile curve tables, then per run the curve pass
// (for images with an FP32 output, the form that reads back the x2 the first
// pass parked in that output instead of the input). One workgroup per tile.
int enqueue_local(dc_ctx *ctx, const HostTable &h, const DevBufs &b, dc::TmArgs a,
                  dc::StatsOut *stats, hipStream_t st, bool marks)
{
    const int n = (int)h.d.size();
    hipError_t e = hipSuccess;
    mark(ctx, marks, 0, st);
    for (const auto &r : h.runs) {
        const int64_t t0 = h.d[r.img0].tile_begin, t1 = h.tile_end[r.img1 - 1];
        if (e == hipSuccess)
            e = dc::launch_ltm_pass1(b.table, b.tile_end, r.img0, r.img1 - r.img0, t0, t1, r.src, a,
                                     b.parts, b.hist, 0, st);
    }
    mark(ctx, marks, 1, st);
    if (e == hipSuccess)
        e = dc::launch_tm_combine(b.table, b.grp_end, 0, n, 0, h.total_grps, b.parts, b.parts2, st);
    if (e == hipSuccess)
        e = dc::launch_tm_finalize(b.table, 0, n, a, b.parts2, b.curves, stats, st);
    if (e == hipSuccess)
        e = dc::launch_ltm_tables(b.table, b.tile_end, n, h.total_tiles, b.hist, b.coef, st);
    mark(ctx, marks, 2, st);
    for (const auto &r : h.runs) {
        const int64_t t0 = h.d[r.img0].tile_begin, t1 = h.tile_end[r.img1 - 1];
        if (e == hipSuccess)
            e = r.rgb ? dc::launch_ltm_colour(b.table, b.tile_end, r.img0, r.img1 - r.img0, t0,
                                              t1, r.src, colour_mode(a.saturation), a, b.curves,
                                              b.coef, st)
                      : dc::launch_ltm_pass2(b.table, b.tile_end, r.img0, r.img1 - r.img0, t0, t1,
                                             r.staged ? 3 : r.src, a, b.curves, b.coef, 0, st);
    }
    mark(ctx, marks, 3, st);
    if (e != hipSuccess)
        return hip_fail(e, "local tone map launch");
    return DC_OK;
}

// Takes the next workspace slot, waiting for the work that last used it, and
// makes sure it can hold host_bytes of staging and dev_bytes on the device.
int acquire_slot(dc_ctx *ctx, size_t host_bytes, size_t dev_bytes, dc_ctx::Slot **out)
{
    dc_ctx::Slot &s = ctx->slots[ctx->next];
    ctx->next = (ctx->next + 1) % dc_ctx::kSlots;
    if (s.pending) {
        if (hipEventSynchronize(s.done) != hipSuccess)
            return fail(DC_ERR_HIP, "hipEventSynchronize failed on a workspace slot");
        s.pending = false;
    }
    if (s.host_cap < host_bytes) {
        if (s.host)
            (void)hipHostFree(s.host);
        s.host = nullptr;
        s.host_cap = 0;
        const size_t cap = std::max(host_bytes + host_bytes / 2, (size_t)4096);
        if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess)
            return fail(DC_ERR_NO_MEMORY, "pinned staging allocation failed");
        s.host_cap = cap;
    }
    if (s.dev_cap < dev_bytes) {
        if (s.dev)
            (void)hipFree(s.dev);
        s.dev = nullptr;
        s.dev_cap = 0;
        const size_t cap = std::max(dev_bytes + dev_bytes / 2, (size_t)65536);
        if (hipMalloc(&s.dev, cap) != hipSuccess)
            return fail(DC_ERR_NO_MEMORY, "device workspace allocation failed");
        s.dev_cap = cap;
    }
    *out = &s;
    return DC_OK;
}

int release_slot(dc_ctx::Slot *s, hipStream_t stream)
{
    if (hipEventRecord(s->done, stream) != hipSuccess)
        return fail(DC_ERR_HIP, "hipEventRecord failed");
    s->pending = true;
    return DC_OK;
}

// Holds a staged slot until the call's work is enqueued: finish() records the
// slot's completion event after the last kernel; an early return after a
// failure records it too (in the destructor), because the upload, and maybe
// some kernels, are already queued and still read the slot, so the next call
// that takes the slot must wait for them.
struct SlotHold {
    dc_ctx::Slot *slot;
    hipStream_t st;
    int finish()
    {
        dc_ctx::Slot *s = slot;
        slot = nullptr;
        return release_slot(s, st);
    }
    ~SlotHold()
    {
        if (slot)
            (void)release_slot(slot, st);
    }
};

// Stages a table in the next ring slot and copies it to the device on `st`.
int stage(dc_ctx *ctx, const HostTable &h, hipStream_t st, dc_ctx::Slot **slot, DevBufs *b)
{
    const Layout l = layout_of(h);
    int rc = acquire_slot(ctx, l.upload, l.total, slot);
    if (rc != DC_OK)
        return rc;
    write_upload(h, l, (char *)(*slot)->host);
    hipError_t e = hipMemcpyAsync((*slot)->dev, (*slot)->host, l.upload, hipMemcpyHostToDevice, st);
    if (e != hipSuccess)
        return hip_fail(e, "descriptor upload");
    *b = bufs_of((*slot)->dev, l);
    return DC_OK;
}

int check_ctx(dc_ctx *ctx)
{
    if (!ctx)
        return fail(DC_ERR_INVALID_ARG, "context is NULL");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    // The launch checks read the thread's last HIP error: drop one that an
    // earlier call left behind (a failed allocation, say), so that this call
    // reports only its own.
    (void)hipGetLastError();
    return DC_OK;
}

bool tune_ok(const dc_tuning &t)
{
    auto g_ok = [](int g) { return g == 1 || g == 2 || g == 4; };
    auto c_ok = [](int c) { return c >= 0 && c <= 64; };
    return g_ok(t.groups[0]) && g_ok(t.groups[1]) && g_ok(t.groups[2]) && g_ok(t.mixed_groups) &&
           c_ok(t.decolor_grid_per_cu) && c_ok(t.mixed_grid_per_cu) && c_ok(t.pass1_grid_per_cu) &&
           c_ok(t.pass2_grid_per_cu) && t.tonemap_pipeline >= 0 && t.tonemap_pipeline <= 1024;
}

dc_tuning to_public(const Tune &t)
{
    dc_tuning o;
    for (int i = 0; i < 3; ++i)
        o.groups[i] = t.groups[i];
    o.mixed_groups = t.mixed_groups;
    o.decolor_grid_per_cu = t.decolor_gpc;
    o.mixed_grid_per_cu = t.mixed_gpc;
    o.pass1_grid_per_cu = t.pass1_gpc;
    o.pass2_grid_per_cu = t.pass2_gpc;
    o.tonemap_pipeline = t.tm_pipeline;
    return o;
}

Tune from_public(const dc_tuning &o)
{
    Tune t;
    for (int i = 0; i < 3; ++i)
        t.groups[i] = o.groups[i];
    t.mixed_groups = o.mixed_groups;
    t.decolor_gpc = o.decolor_grid_per_cu;
    t.mixed_gpc = o.mixed_grid_per_cu;
    t.pass1_gpc = o.pass1_grid_per_cu;
    t.pass2_gpc = o.pass2_grid_per_cu;
    t.tm_pipeline = o.tonemap_pipeline;
    return t;
}

} // namespace

// ------------------------------------------------------------------ plans

struct dc_plan {
    dc_ctx *ctx = nullptr;
    int32_t kind = DC_PLAN_DECOLORIZE;
    HostTable h;
    Tune tune;
    void *dev = nullptr;
    DevBufs b{};
    dc::TmArgs tm{};
    dc::StatsOut *stats = nullptr;
    bool graph = false;
    hipGraphExec_t exec = nullptr;
};

namespace {

int plan_enqueue(dc_plan *p, hipStream_t st, bool marks)
{
    if (p->kind == DC_PLAN_TONEMAP)
        return enqueue_tonemap(p->ctx, p->h, p->b, p->tune, p->tm, p->stats, st, marks);
    if (p->kind == DC_PLAN_LOCAL)
        return enqueue_local(p->ctx, p->h, p->b, p->tm, p->stats, st, marks);
    return enqueue_decolor(p->ctx, p->h, p->b, p->tune, st, marks);
}

void plan_free(dc_plan *p)
{
    if (!p)
        return;
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->dev)
        (void)hipFree(p->dev);
    delete p;
}

// Builds a plan with a given launch shape (used by dc_plan_create and the tuner).
int plan_build(dc_ctx *ctx, int32_t kind, const dc_image *imgs, int32_t n, const dc_params *params,
               const dc_tm_params *tm, dc_stats *stats, int32_t flags, const Tune &tune,
               dc_plan **out)
{
    dc_plan *p = new (std::nothrow) dc_plan();
    if (!p)
        return fail(DC_ERR_NO_MEMORY, "plan allocation failed");
    p->ctx = ctx;
    p->kind = kind;
    p->tune = tune;
    p->tm = tm_of(tm);
    p->stats = (dc::StatsOut *)stats;
    p->graph = (flags & DC_PLAN_GRAPH) != 0;
    build_table(imgs, n, params,
                kind == DC_PLAN_TONEMAP ? kTabTonemap
                                        : (kind == DC_PLAN_LOCAL ? kTabLocal : kTabDecolor),
                tune, p->h);
    const Layout l = layout_of(p->h);
    std::vector<char> up(l.upload);
    write_upload(p->h, l, up.data());
    hipError_t e = hipMalloc(&p->dev, l.total);
    if (e != hipSuccess) {
        plan_free(p);
        return fail(DC_ERR_NO_MEMORY, "plan workspace allocation failed");
    }
    e = hipMemcpy(p->dev, up.data(), l.upload, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "plan upload");
    }
    p->b = bufs_of(p->dev, l);
    *out = p;
    return DC_OK;
}

// Per-interval durations of `reps` timed runs of a plan after one warm-up.
int time_plan(dc_plan *p, hipStream_t st, int reps, std::vector<float> *per_interval)
{
    dc_ctx *ctx = p->ctx;
    const int ev = ensure_prof_events(ctx);
    if (ev != DC_OK)
        return ev;
    const bool was = ctx->profiling;
    ctx->profiling = true;
    const int nint = (p->kind == DC_PLAN_TONEMAP && !p->tune.tm_pipeline) || p->kind == DC_PLAN_LOCAL
                         ? 3
                         : 1;
    std::vector<std::vector<float>> samples(nint);
    for (int r = 0; r < reps + 1; ++r) {
        int rc = plan_enqueue(p, st, true);
        if (rc != DC_OK) {
            ctx->profiling = was;
            return rc;
        }
        if (hipEventSynchronize(ctx->prof[nint]) != hipSuccess) {
            ctx->profiling = was;
            return fail(DC_ERR_HIP, "tuner timing failed");
        }
        if (r == 0)
            continue; // warm-up
        for (int i = 0; i < nint; ++i) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ctx->prof[i], ctx->prof[i + 1]);
            samples[i].push_back(ms);
        }
    }
    ctx->profiling = was;
    // The fastest run of each interval: the least disturbed measurement.
    per_interval->assign(nint, 0.0f);
    for (int i = 0; i < nint; ++i)
        (*per_interval)[i] = *std::min_element(samples[i].begin(), samples[i].end());
    return DC_OK;
}

} // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int dc_version(void) { return DC_ABI_VERSION; }

const char *dc_status_string(int status)
{
    switch (status) {
    case DC_OK: return "ok";
    case DC_ERR_INVALID_ARG: return "invalid argument";
    case DC_ERR_UNSUPPORTED: return "unsupported";
    case DC_ERR_ALIAS: return "output overlaps an input or another output";
    case DC_ERR_NO_MEMORY: return "out of memory";
    case DC_ERR_HIP: return "HIP runtime error";
    case DC_ERR_NO_DEVICE: return "no usable device";
    case DC_ERR_CANCELLED: return "cancelled";
    default: return "unknown status";
    }
}

const char *dc_last_error_message(void) { return g_last_error.c_str(); }

int dc_validate(const dc_image *imgs, int32_t n, const dc_params *params, const dc_tm_params *tm)
{
    return guarded([&]() -> int {
        g_last_error.clear();
        int rc = validate_params(params);
        if (rc == DC_OK)
            rc = validate_tm(tm);
        if (rc == DC_OK)
            rc = validate_images(imgs, n, tm != nullptr ? DC_IMG_RGB_OUT : 0);
        return rc;
    });
}

int dc_create(dc_ctx **out, int device)
{
    return guarded([&]() -> int {
        g_last_error.clear();
        if (!out)
            return fail(DC_ERR_INVALID_ARG, "ctx out-pointer is NULL");
        *out = nullptr;
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
            return fail(DC_ERR_NO_DEVICE, "no HIP device is visible");
        if (device < 0 || device >= count)
            return fail(DC_ERR_NO_DEVICE, "device index out of range");
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess)
            return hip_fail(e, "hipSetDevice");
        dc_ctx *ctx = new (std::nothrow) dc_ctx();
        if (!ctx)
            return fail(DC_ERR_NO_MEMORY, "context allocation failed");
        ctx->device = device;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
            cus > 0)
            ctx->num_cu = cus;
        for (auto &s : ctx->slots) {
            e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
            if (e != hipSuccess) {
                dc_destroy(ctx);
                return hip_fail(e, "hipEventCreate");
            }
        }
        // Set-up of dc_tonemap_global_noalloc: the scratch array's address on
        // this device, reserved host lists, pinned staging and its event.
        e = dc::scratch_address(&ctx->scratch);
        if (e != hipSuccess) {
            dc_destroy(ctx);
            return hip_fail(e, "hipGetSymbolAddress of the scratch array");
        }
        ctx->na = new (std::nothrow) NoAlloc();
        if (!ctx->na) {
            dc_destroy(ctx);
            return fail(DC_ERR_NO_MEMORY, "context allocation failed");
        }
        ctx->na->h.reserve(dc::kScratchMaxImages);
        ctx->na->outs.reserve(2 * (size_t)dc::kScratchMaxImages);
        ctx->na->ins.reserve(dc::kScratchMaxImages);
        const size_t cap = noalloc_upload_cap();
        if (hipHostMalloc(&ctx->na->host, cap, hipHostMallocDefault) != hipSuccess) {
            ctx->na->host = nullptr;
            dc_destroy(ctx);
            return fail(DC_ERR_NO_MEMORY, "pinned staging allocation failed");
        }
        ctx->na->host_cap = cap;
        e = hipEventCreateWithFlags(&ctx->na->copied, hipEventDisableTiming);
        if (e != hipSuccess) {
            dc_destroy(ctx);
            return hip_fail(e, "hipEventCreate");
        }
        *out = ctx;
        return DC_OK;
    });
}

int dc_destroy(dc_ctx *ctx)
{
    return guarded([&]() -> int {
        if (!ctx)
            return DC_OK;
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &s : ctx->slots) {
            if (s.host)
                (void)hipHostFree(s.host);
            if (s.dev)
                (void)hipFree(s.dev);
            if (s.done)
                (void)hipEventDestroy(s.done);
        }
        for (auto &e : ctx->prof)
            if (e)
                (void)hipEventDestroy(e);
        for (auto &e : ctx->fork)
            (void)hipEventDestroy(e);
        if (ctx->side)
            (void)hipStreamDestroy(ctx->side);
        if (ctx->na) {
            if (ctx->na->host)
                (void)hipHostFree(ctx->na->host);
            if (ctx->na->copied)
                (void)hipEventDestroy(ctx->na->copied);
            delete ctx->na;
        }
        delete ctx;
        return DC_OK;
    });
}

int dc_get_tuning(dc_ctx *ctx, dc_tuning *out)
{
    return guarded([&]() -> int {
        g_last_error.clear();
        if (!ctx || !out)
            return fail(DC_ERR_INVALID_ARG, "context or output is NULL");
        *out = to_public(ctx->tune);
        return DC_OK;
    });
}

int dc_set_tuning(dc_ctx *ctx, const dc_tuning *t)
{
    return guarded([&]() -> int {
        g_last_error.clear();
        if (!ctx || !t)
            return fail(DC_ERR_INVALID_ARG, "context or tuning is NULL");
        if (!tune_ok(*t))
            return fail(DC_ERR_INVALID_ARG, "groups must be 1, 2 or 4, grids per CU in [0, 64] and "
                                            "tonemap_pipeline in [0, 1024]");
        ctx->tune = from_public(*t);
        return DC_OK;
    });
}

int dc_set_profiling(dc_ctx *ctx, int on)
{
    return guarded([&]() -> int {
        g_last_error.clear();
        if (!ctx)
            return fail(DC_ERR_INVALID_ARG, "context is NULL");
        if (on) {
            (void)hipSetDevice(ctx->device);
            const int rc = ensure_prof_events(ctx);
            if (rc != DC_OK)
                return rc;
        }
        ctx->profiling = on != 0;
        ctx->prof_used = 0;
        return DC_OK;
    });
}

int dc_last_timings(dc_ctx *ctx, float *ms, int32_t cap)
{
    return guarded([&]() -> int {
        g_last_error.clear();
        if (!ctx || (!ms && cap > 0) || cap < 0)
            return fail(DC_ERR_INVALID_ARG, "bad context or output array");
        if (ctx->prof_used < 2)
            return 0;
        hipError_t e = hipEventSynchronize(ctx->prof[ctx->prof_used - 1]);
        if (e != hipSuccess)
            return hip_fail(e, "hipEventSynchronize");
        int n = 0;
        for (int i = 0; i + 1 < ctx->prof_used && n < cap; ++i, ++n) {
            e = hipEventElapsedTime(&ms[n], ctx->prof[i], ctx->prof[i + 1]);
            if (e != hipSuccess)
                return hip_fail(e, "hipEventElapsedTime");
        }
        return n;
    });
}

int dc_decolorize(dc_ctx *ctx, const dc_image *img, const dc_params *params, void *stream)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_decolorize");
        g_last_error.clear();
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        if (!img)
            return fail(DC_ERR_INVALID_ARG, "image is NULL");
        rc = dc_validate(img, 1, params, nullptr);
        if (rc != DC_OK)
            return rc;
        const int g = ctx->tune.groups[img->src_dtype];
        const dc::DevImage d =
            describe(*img, 0, (int64_t)dc::kBlock * g * dc::group_px(img->src_dtype), params);
        const hipStream_t st = (hipStream_t)stream;
        mark(ctx, true, 0, st);
        hipError_t e = dc::launch_decolor_single(d, g, grid_blocks(ctx, ctx->tune.decolor_gpc), st);
        if (e != hipSuccess)
            return hip_fail(e, "decolorize launch");
        mark(ctx, true, 1, st);
        return DC_OK;
    });
}

int dc_decolorize_batch(dc_ctx *ctx, const dc_image *imgs, int32_t n, const dc_params *params,
                        void *stream)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_decolorize_batch");
        g_last_error.clear();
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        rc = dc_validate(imgs, n, params, nullptr);
        if (rc != DC_OK || n == 0)
            return rc;
        const hipStream_t st = (hipStream_t)stream;
        HostTable h;
        build_table(imgs, n, params, kTabDecolor, ctx->tune, h);
        dc_ctx::Slot *slot = nullptr;
        DevBufs b;
        rc = stage(ctx, h, st, &slot, &b);
        if (rc != DC_OK)
            return rc;
        SlotHold hold{slot, st};
        rc = enqueue_decolor(ctx, h, b, ctx->tune, st, true);
        if (rc != DC_OK)
            return rc;
        return hold.finish();
    });
}

int dc_decolorize_batch_betas(dc_ctx *ctx, const dc_image *imgs, int32_t n,
                              const dc_params *betas, void *stream)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_decolorize_batch_betas");
        g_last_error.clear();
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        if (betas)
            for (int32_t i = 0; i < n && rc == DC_OK; ++i)
                rc = validate_params(&betas[i]);
        if (rc == DC_OK)
            rc = dc_validate(imgs, n, nullptr, nullptr);
        if (rc != DC_OK || n == 0)
            return rc;
        const hipStream_t st = (hipStream_t)stream;
        HostTable h;
        build_table(imgs, n, nullptr, kTabDecolor, ctx->tune, h, betas);
        dc_ctx::Slot *slot = nullptr;
        DevBufs b;
        rc = stage(ctx, h, st, &slot, &b);
        if (rc != DC_OK)
            return rc;
        SlotHold hold{slot, st};
        const int per = sweep_per(ctx, h);
        if (per > 0) {
            mark(ctx, true, 0, st);
            const hipError_t e =
                dc::launch_sweep(b.table, n, per, h.d[0].ntiles, h.src0, h.groups,
                                 h.d[0].walk == dc::kWalkRows,
                                 grid_blocks(ctx, ctx->tune.decolor_gpc), st);
            if (e != hipSuccess)
                return hip_fail(e, "sweep launch");
            mark(ctx, true, 1, st);
        } else {
            rc = enqueue_decolor(ctx, h, b, ctx->tune, st, true);
            if (rc != DC_OK)
                return rc;
        }
        return hold.finish();
    });
}

int dc_tonemap_global(dc_ctx *ctx, const dc_image *imgs, int32_t n, const dc_params *params,
                      const dc_tm_params *tm, dc_stats *stats, void *stream)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_tonemap_global");
        g_last_error.clear();
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        rc = dc_validate(imgs, n, params, tm);
        if (rc != DC_OK || n == 0)
            return rc;
        const hipStream_t st = (hipStream_t)stream;
        HostTable h;
        build_table(imgs, n, params, kTabTonemap, ctx->tune, h);
        dc_ctx::Slot *slot = nullptr;
        DevBufs b;
        rc = stage(ctx, h, st, &slot, &b);
        if (rc != DC_OK)
            return rc;
        SlotHold hold{slot, st};
        rc = enqueue_tonemap(ctx, h, b, ctx->tune, tm_of(tm), (dc::StatsOut *)stats, st, true);
        if (rc != DC_OK)
            return rc;
        return hold.finish();
    });
}

int dc_tonemap_global_noalloc(dc_ctx *ctx, const dc_image *imgs, int32_t n,
                              const dc_params *params, const dc_tm_params *tm, dc_stats *stats,
                              void *stream)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_tonemap_global_noalloc");
        g_last_error.clear();
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        if (n > dc::kScratchMaxImages)
            return fail(DC_ERR_INVALID_ARG, "dc_tonemap_global_noalloc takes at most " +
                                                std::to_string(dc::kScratchMaxImages) +
                                                " images per call");
        NoAlloc &na = *ctx->na;
        rc = validate_params(params);
        if (rc == DC_OK)
            rc = validate_tm(tm);
        if (rc == DC_OK)
            rc = validate_images(imgs, n, DC_IMG_RGB_OUT, &na.outs, &na.ins);
        if (rc != DC_OK || n == 0)
            return rc;
        const hipStream_t st = (hipStream_t)stream;
        // The per-image pipeline would need a second stream and events made
        // on first use, so this entry point always takes the batch schedule.
        Tune tune = ctx->tune;
        tune.tm_pipeline = 0;
        build_table(imgs, n, params, kTabTonemap, tune, na.h);
        const Layout l = layout_of(na.h);
        if (l.total > dc::kScratchBytes)
            return fail(DC_ERR_INVALID_ARG,
                        "the call needs " + std::to_string(l.total) +
                            " bytes of workspace; dc_tonemap_global_noalloc has a fixed " +
                            std::to_string(dc::kScratchBytes) +
                            "-byte scratch (about 340 Mpx per call)");
        if (na.pending) {
            // The previous call's upload still reads the staging.
            if (hipEventSynchronize(na.copied) != hipSuccess)
                return fail(DC_ERR_HIP, "hipEventSynchronize failed on the scratch upload");
            na.pending = false;
        }
        write_upload(na.h, l, (char *)na.host);
        hipError_t e = hipMemcpyAsync(ctx->scratch, na.host, l.upload, hipMemcpyHostToDevice, st);
        if (e != hipSuccess)
            return hip_fail(e, "descriptor upload to the scratch");
        e = hipEventRecord(na.copied, st);
        if (e != hipSuccess)
            return hip_fail(e, "hipEventRecord");
        na.pending = true;
        return enqueue_tonemap(ctx, na.h, bufs_of(ctx->scratch, l), tune, tm_of(tm),
                               (dc::StatsOut *)stats, st, true);
    });
}

int dc_tonemap_local(dc_ctx *ctx, const dc_image *imgs, int32_t n, const dc_params *params,
                     const dc_tm_params *tm, dc_stats *stats, void *stream)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_tonemap_local");
        g_last_error.clear();
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        rc = dc_validate(imgs, n, params, tm);
        if (rc != DC_OK || n == 0)
            return rc;
        const hipStream_t st = (hipStream_t)stream;
        HostTable h;
        build_table(imgs, n, params, kTabLocal, ctx->tune, h);
        dc_ctx::Slot *slot = nullptr;
        DevBufs b;
        rc = stage(ctx, h, st, &slot, &b);
        if (rc != DC_OK)
            return rc;
        SlotHold hold{slot, st};
        rc = enqueue_local(ctx, h, b, tm_of(tm), (dc::StatsOut *)stats, st, true);
        if (rc != DC_OK)
            return rc;
        return hold.finish();
    });
}

int dc_channel_batch(dc_ctx *ctx, const dc_image *imgs, int32_t n, int32_t channel, void *stream)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_channel_batch");
        g_last_error.clear();
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        if (channel < DC_CH_Y601 || channel > DC_CH_CIELAB_L)
            return fail(DC_ERR_INVALID_ARG, "channel must be DC_CH_Y601, DC_CH_HSV_V or DC_CH_CIELAB_L");
        rc = dc_validate(imgs, n, nullptr, nullptr);
        if (rc != DC_OK || n == 0)
            return rc;
        const hipStream_t st = (hipStream_t)stream;
        HostTable h;
        build_table(imgs, n, nullptr, kTabChannel, ctx->tune, h);
        dc_ctx::Slot *slot = nullptr;
        DevBufs b;
        rc = stage(ctx, h, st, &slot, &b);
        if (rc != DC_OK)
            return rc;
        SlotHold hold{slot, st};
        mark(ctx, true, 0, st);
        hipError_t e = hipSuccess;
        for (const auto &r : h.runs) {
            if (e == hipSuccess)
                e = dc::launch_channel(b.table, b.tile_end, r.img0, r.img1 - r.img0,
                                       h.d[r.img0].tile_begin, h.tile_end[r.img1 - 1], r.src, channel,
                                       r.rows, 0, st);
        }
        if (e != hipSuccess)
            return hip_fail(e, "channel launch");
        mark(ctx, true, 1, st);
        return hold.finish();
    });
}

int dc_plan_create(dc_ctx *ctx, int32_t kind, const dc_image *imgs, int32_t n,
                   const dc_params *params, const dc_tm_params *tm, dc_stats *stats, int32_t flags,
                   dc_plan **plan)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_plan_create");
        g_last_error.clear();
        if (!plan)
            return fail(DC_ERR_INVALID_ARG, "plan out-pointer is NULL");
        *plan = nullptr;
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        if (kind != DC_PLAN_DECOLORIZE && kind != DC_PLAN_TONEMAP && kind != DC_PLAN_LOCAL)
            return fail(DC_ERR_INVALID_ARG,
                        "kind must be DC_PLAN_DECOLORIZE, DC_PLAN_TONEMAP or DC_PLAN_LOCAL");
        if (flags & ~DC_PLAN_GRAPH)
            return fail(DC_ERR_INVALID_ARG, "unknown plan flags");
        if (n < 1)
            return fail(DC_ERR_INVALID_ARG, "a plan needs at least one image");
        if (kind == DC_PLAN_DECOLORIZE && (tm || stats))
            return fail(DC_ERR_INVALID_ARG, "tm and stats apply to tone-map plans only");
        rc = dc_validate(imgs, n, params, kind == DC_PLAN_DECOLORIZE ? nullptr : tm);
        if (rc != DC_OK)
            return rc;
        return plan_build(ctx, kind, imgs, n, params, tm, stats, flags, ctx->tune, plan);
    });
}

int dc_plan_run(dc_plan *p, void *stream)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_plan_run");
        g_last_error.clear();
        if (!p)
            return fail(DC_ERR_INVALID_ARG, "plan is NULL");
        int rc = check_ctx(p->ctx);
        if (rc != DC_OK)
            return rc;
        const hipStream_t st = (hipStream_t)stream;
        if (!p->graph)
            return plan_enqueue(p, st, true);
        if (!st)
            return fail(DC_ERR_INVALID_ARG, "graph plans need a non-null stream");
        if (!p->exec) {
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess)
                return hip_fail(e, "hipStreamBeginCapture");
            rc = plan_enqueue(p, st, false);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(st, &g);
            if (rc != DC_OK) {
                if (g)
                    (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess)
                return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                p->exec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
        }
        hipError_t e = hipGraphLaunch(p->exec, st);
        if (e != hipSuccess)
            return hip_fail(e, "hipGraphLaunch");
        return DC_OK;
    });
}

int dc_plan_destroy(dc_plan *p)
{
    return guarded([&]() -> int {
        if (!p)
            return DC_OK;
        (void)hipSetDevice(p->ctx->device);
        (void)hipDeviceSynchronize();
        plan_free(p);
        return DC_OK;
    });
}

int dc_autotune(dc_ctx *ctx, int32_t kind, const dc_image *imgs, int32_t n,
                const dc_params *params, const dc_tm_params *tm, void *stream, dc_tuning *chosen)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_autotune");
        g_last_error.clear();
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        if (kind != DC_PLAN_DECOLORIZE && kind != DC_PLAN_TONEMAP)
            return fail(DC_ERR_INVALID_ARG, "kind must be DC_PLAN_DECOLORIZE or DC_PLAN_TONEMAP");
        if (n < 1)
            return fail(DC_ERR_INVALID_ARG, "tuning needs at least one image");
        rc = dc_validate(imgs, n, params, kind == DC_PLAN_TONEMAP ? tm : nullptr);
        if (rc != DC_OK)
            return rc;
        if (!autotune_enabled()) {
            log_msg(2, "DC_AUTOTUNE=0: launch shapes kept as they are");
            if (chosen)
                *chosen = to_public(ctx->tune);
            return DC_OK;
        }
        const hipStream_t st = (hipStream_t)stream;
        const int gpcs[] = {0, 1, 2, 4, 8, 16};
        const int reps = 10;
        // A candidate replaces the current choice only when it is faster by more
        // than this factor, so run-to-run noise does not flip between shapes whose
        // times are within it; the current shapes are measured first.
        const float margin = 0.98f;
        Tune best = ctx->tune;
        std::vector<float> ms;
        auto run = [&](const Tune &t, std::vector<float> *out) -> int {
            dc_plan *p = nullptr;
            int r = plan_build(ctx, kind, imgs, n, params, tm, nullptr, 0, t, &p);
            if (r == DC_OK)
                r = time_plan(p, st, reps, out);
            if (p) {
                (void)hipStreamSynchronize(st);
                plan_free(p);
            }
            return r;
        };
        if (kind == DC_PLAN_DECOLORIZE) {
            bool mixed = false;
            for (int32_t i = 1; i < n; ++i)
                mixed |= imgs[i].src_dtype != imgs[0].src_dtype;
            rc = run(ctx->tune, &ms);
            if (rc != DC_OK)
                return rc;
            float best_ms = ms[0];
            for (int g : {1, 2, 4}) {
                for (int c : gpcs) {
                    Tune t = ctx->tune;
                    if (mixed) {
                        t.mixed_groups = g;
                        t.mixed_gpc = c;
                    } else {
                        t.groups[imgs[0].src_dtype] = g;
                        t.decolor_gpc = c;
                    }
                    rc = run(t, &ms);
                    if (rc != DC_OK)
                        return rc;
                    if (ms[0] < margin * best_ms) {
                        best_ms = ms[0];
                        best = t;
                    }
                }
            }
        } else {
            Tune cur = ctx->tune;
            cur.tm_pipeline = 0;
            rc = run(cur, &ms);
            if (rc != DC_OK)
                return rc;
            float b1 = ms[0], b2 = ms[2];
            for (int c : gpcs) {
                Tune t = ctx->tune;
                t.tm_pipeline = 0;
                t.pass1_gpc = c;
                t.pass2_gpc = c;
                rc = run(t, &ms);
                if (rc != DC_OK)
                    return rc;
                if (ms[0] < margin * b1) {
                    b1 = ms[0];
                    best.pass1_gpc = c;
                }
                if (ms[2] < margin * b2) {
                    b2 = ms[2];
                    best.pass2_gpc = c;
                }
            }
            // Whole-sequence time of the two schedules with the chosen grids.
            float whole[2];
            for (int pl = 0; pl < 2; ++pl) {
                Tune t = best;
                t.tm_pipeline = pl;
                rc = run(t, &ms);
                if (rc != DC_OK)
                    return rc;
                whole[pl] = 0.0f;
                for (float m : ms)
                    whole[pl] += m;
            }
            best.tm_pipeline = whole[1] < margin * whole[0] ? 1 : 0;
        }
        ctx->tune = best;
        if (chosen)
            *chosen = to_public(best);
        if (log_level() >= 2)
            log_msg(2, std::string("autotune ") + (kind == DC_PLAN_TONEMAP ? "tone map" : "decolorize") +
                           ": groups " + std::to_string(best.groups[0]) + "/" +
                           std::to_string(best.groups[1]) + "/" + std::to_string(best.groups[2]) +
                           " mixed " + std::to_string(best.mixed_groups) + ", grids per CU " +
                           std::to_string(best.decolor_gpc) + "/" + std::to_string(best.mixed_gpc) +
                           ", passes " + std::to_string(best.pass1_gpc) + "/" +
                           std::to_string(best.pass2_gpc) + ", pipeline " +
                           std::to_string(best.tm_pipeline));
        return DC_OK;
    });
}

} // extern "C"

// ------------------------------------------------------------------ serving

// Continuous-batching server. Requests wait in FIFO order; a request is
// admitted when its output fits the server's device-memory arena (first fit,
// 256-byte granules, coalescing free list); whenever one of the launch lanes
// (each its own stream) is idle, every admitted request (up to max_batch)
// goes into one tone-map launch on that lane; a lane whose completion event
// has fired retires its requests and frees their memory, which admits more.
// Each image's result does not depend on the batch it lands in.
struct dc_server {
    struct Req {
        dc_request r;
        double t_submit = 0, t_admit = 0, t_launch = 0;
        size_t off = 0, bytes = 0; // budget block: [input copy | output]
        size_t in_bytes = 0;       // bytes of the input copy (host inputs)
        bool owned = false;
    };
    struct Lane {
        hipStream_t s = nullptr;
        hipEvent_t done = nullptr;
        std::vector<Req> batch;
        bool busy = false;
        // per-launch host buffers, kept for their capacity
        std::vector<dc_image> imgs;
        HostTable h;
    };
    dc_ctx *ctx = nullptr;
    dc_server_config cfg{};
    char *arena = nullptr;
    dc::Arena blocks; // offsets into `arena`
    std::deque<Req> waiting, admitted;
    std::vector<Lane> lanes;
    std::vector<dc_completion> done;
    std::chrono::steady_clock::time_point t0;
    int64_t in_system = 0;
    // host time spent enqueueing lane launches, and their number
    double launch_host_s = 0.0;
    int64_t launches = 0;
};

namespace {

double server_now(const dc_server *sv)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - sv->t0).count();
}

// Bytes of a server-allocated output. Rows are packed (pitch = row bytes), so a
// packed input keeps the packed vector walk; blocks start on 256-byte granules.
size_t out_bytes(const dc_image &m, int64_t *pitch)
{
    const int64_t ch = (m.flags & DC_IMG_RGB_OUT) ? 3 : 1;
    *pitch = ch * dc::elem_size(m.dst_dtype) * m.width;
    return dc::granules((size_t)*pitch * (size_t)m.height);
}

// Bytes of the device copy of a host input (rows packed), granule-rounded.
size_t in_bytes(const dc_image &m, int64_t *pitch)
{
    *pitch = 3 * dc::elem_size(m.src_dtype) * m.width;
    return dc::granules((size_t)*pitch * (size_t)m.height);
}

void complete(dc_server *sv, const dc_server::Req &q, int status, int batch, double t_done)
{
    dc_completion c;
    c.id = q.r.id;
    c.status = status;
    c.batch_size = batch;
    c.t_submit = q.t_submit;
    c.t_admit = q.t_admit;
    c.t_launch = q.t_launch;
    c.t_done = t_done;
    sv->done.push_back(c);
    --sv->in_system;
}

// A launch on a lane failed: its requests complete with that status and give
// their memory back, so none of them is later reported as done by a batch it
// never ran in. Copies or kernels already enqueued on the lane may still write
// that memory, so the lane is drained first.
int fail_lane(dc_server *sv, dc_server::Lane &ln, int status)
{
    (void)hipStreamSynchronize(ln.s);
    const double t = server_now(sv);
    for (auto &r : ln.batch) {
        if (r.owned)
            sv->blocks.release(r.off, r.bytes);
        complete(sv, r, status, 0, t);
    }
    ln.batch.clear();
    ln.busy = false;
    return status;
}

int server_step(dc_server *sv)
{
    // 1. retire finished launches
    for (auto &ln : sv->lanes) {
        if (!ln.busy)
            continue;
        const hipError_t q = hipEventQuery(ln.done);
        if (q == hipErrorNotReady)
            continue;
        if (q != hipSuccess)
            return hip_fail(q, "server launch failed");
        const double t = server_now(sv);
        for (auto &r : ln.batch) {
            if (r.owned)
                sv->blocks.release(r.off, r.bytes);
            complete(sv, r, DC_OK, (int)ln.batch.size(), t);
        }
        ln.batch.clear();
        ln.busy = false;
    }
    // 2. admit in FIFO order while input copies and outputs fit
    const double t_admit = server_now(sv);
    dc::admit_fifo(
        sv->waiting, sv->admitted, sv->blocks,
        [](const dc_server::Req &q) -> size_t {
            // a device input with a caller output takes no budget
            int64_t pitch = 0;
            const bool host = (q.r.img.flags & DC_IMG_HOST_SRC) != 0;
            return (host ? in_bytes(q.r.img, &pitch) : 0) +
                   (q.r.img.dst ? 0 : out_bytes(q.r.img, &pitch));
        },
        [&](dc_server::Req &q, size_t off, size_t bytes) {
            q.t_admit = t_admit;
            if (!bytes)
                return;
            int64_t in_pitch = 0, out_pitch = 0;
            const size_t ib =
                (q.r.img.flags & DC_IMG_HOST_SRC) ? in_bytes(q.r.img, &in_pitch) : 0;
            q.off = off;
            q.bytes = bytes;
            q.in_bytes = ib;
            q.owned = true;
            if (!q.r.img.dst) {
                (void)out_bytes(q.r.img, &out_pitch);
                q.r.img.dst = sv->arena + off + ib;
                q.r.img.dst_pitch = out_pitch;
            }
        },
        [&](const dc_server::Req &q) { complete(sv, q, DC_ERR_NO_MEMORY, 0, server_now(sv)); });
    // 3. launch admitted work on idle lanes
    for (auto &ln : sv->lanes) {
        if (sv->admitted.empty())
            break;
        if (ln.busy)
            continue;
        TraceRange trace("dc_server_launch");
        const auto t_begin = std::chrono::steady_clock::now();
        const size_t k = std::min<size_t>(sv->admitted.size(), (size_t)sv->cfg.max_batch);
        std::vector<dc_image> &imgs = ln.imgs;
        imgs.resize(k);
        const double t = server_now(sv);
        for (size_t i = 0; i < k; ++i) {
            ln.batch.push_back(sv->admitted.front());
            sv->admitted.pop_front();
            dc_server::Req &q = ln.batch.back();
            q.t_launch = t;
            imgs[i] = q.r.img;
            if (q.r.img.flags & DC_IMG_HOST_SRC) {
                // the input's device copy, packed, at the start of its block
                int64_t pitch = 0;
                (void)in_bytes(q.r.img, &pitch);
                char *d = sv->arena + q.off;
                const size_t rows = (size_t)q.r.img.height;
                // one linear copy when the host rows are packed too; pitched
                // host rows are gathered by a kernel reading the pinned rows
                // across PCIe (hipMemcpy2DAsync moved only ~1.4 GB/s here)
                const hipError_t ce =
                    q.r.img.src_pitch == pitch
                        ? hipMemcpyAsync(d, q.r.img.src, (size_t)pitch * rows,
                                         hipMemcpyHostToDevice, ln.s)
                        : dc::launch_copy_rows(d, pitch, q.r.img.src, q.r.img.src_pitch, pitch,
                                               (int)rows, ln.s);
                if (ce != hipSuccess)
                    return fail_lane(sv, ln, hip_fail(ce, "host input copy"));
                imgs[i].src = d;
                imgs[i].src_pitch = pitch;
                imgs[i].flags &= ~DC_IMG_HOST_SRC;
            }
        }
        HostTable &h = ln.h;
        {
            TraceRange tr("dc_server_launch_table");
            build_table(imgs.data(), (int32_t)k, &sv->cfg.params, kTabTonemap, sv->ctx->tune, h);
        }
        dc_ctx::Slot *slot = nullptr;
        DevBufs b;
        int rc;
        {
            TraceRange tr("dc_server_launch_upload");
            rc = stage(sv->ctx, h, ln.s, &slot, &b);
        }
        if (rc != DC_OK)
            return fail_lane(sv, ln, rc);
        SlotHold hold{slot, ln.s};
        {
            TraceRange tr("dc_server_launch_kernels");
            rc = enqueue_tonemap(sv->ctx, h, b, sv->ctx->tune, tm_of(&sv->cfg.tm), nullptr, ln.s,
                                 false, true);
        }
        if (rc == DC_OK)
            rc = hold.finish();
        if (rc != DC_OK)
            return fail_lane(sv, ln, rc);
        const hipError_t e = hipEventRecord(ln.done, ln.s);
        if (e != hipSuccess)
            return fail_lane(sv, ln, hip_fail(e, "hipEventRecord"));
        ln.busy = true;
        sv->launch_host_s +=
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count();
        ++sv->launches;
    }
    return DC_OK;
}

} // namespace

extern "C" {

int dc_server_create(dc_ctx *ctx, const dc_server_config *cfg, dc_server **out)
{
    return guarded([&]() -> int {
        g_last_error.clear();
        if (!out)
            return fail(DC_ERR_INVALID_ARG, "server out-pointer is NULL");
        *out = nullptr;
        int rc = check_ctx(ctx);
        if (rc != DC_OK)
            return rc;
        if (!cfg || cfg->budget_bytes <= 0 || cfg->max_batch < 1 || cfg->max_inflight < 1 ||
            cfg->max_inflight > 8 || cfg->flags != 0)
            return fail(DC_ERR_INVALID_ARG,
                        "budget_bytes > 0, max_batch >= 1, max_inflight in [1, 8] and flags 0 are required");
        rc = validate_params(&cfg->params);
        if (rc == DC_OK)
            rc = validate_tm(&cfg->tm);
        if (rc != DC_OK)
            return rc;
        dc_server *sv = new (std::nothrow) dc_server();
        if (!sv)
            return fail(DC_ERR_NO_MEMORY, "server allocation failed");
        sv->ctx = ctx;
        sv->cfg = *cfg;
        const size_t arena_bytes = (size_t)cfg->budget_bytes / dc::kGranule * dc::kGranule;
        if (hipMalloc((void **)&sv->arena, arena_bytes) != hipSuccess) {
            delete sv;
            return fail(DC_ERR_NO_MEMORY, "server arena allocation failed");
        }
        sv->blocks.reset(arena_bytes);
        sv->lanes.resize((size_t)cfg->max_inflight);
        for (auto &ln : sv->lanes) {
            if (hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess) {
                dc_server_destroy(sv);
                return fail(DC_ERR_HIP, "server stream or event creation failed");
            }
        }
        sv->t0 = std::chrono::steady_clock::now();
        *out = sv;
        return DC_OK;
    });
}

int dc_server_destroy(dc_server *sv)
{
    return guarded([&]() -> int {
        if (!sv)
            return DC_OK;
        (void)hipSetDevice(sv->ctx->device);
        for (auto &ln : sv->lanes) {
            if (ln.s) {
                (void)hipStreamSynchronize(ln.s);
                (void)hipStreamDestroy(ln.s);
            }
            if (ln.done)
                (void)hipEventDestroy(ln.done);
        }
        if (sv->arena)
            (void)hipFree(sv->arena);
        delete sv;
        return DC_OK;
    });
}

int dc_server_host_stats(dc_server *sv, double *launch_seconds, int64_t *launches)
{
    if (!sv)
        return fail(DC_ERR_INVALID_ARG, "server is NULL");
    if (launch_seconds)
        *launch_seconds = sv->launch_host_s;
    if (launches)
        *launches = sv->launches;
    return DC_OK;
}

double dc_server_clock(dc_server *sv) { return sv ? server_now(sv) : 0.0; }

int dc_server_submit(dc_server *sv, const dc_request *reqs, int32_t n, double t_submit)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_server_submit");
        g_last_error.clear();
        if (!sv || n < 0 || (n > 0 && !reqs))
            return fail(DC_ERR_INVALID_ARG, "bad server or request list");
        for (int32_t i = 0; i < n; ++i) {
            const dc_image &m = reqs[i].img;
            const std::string at = " (request " + std::to_string(reqs[i].id) + ")";
            Range r;
            int rc = check_src(m, at, r);
            if (rc != DC_OK)
                return rc;
            if (!dtype_ok(m.dst_dtype) || m.dst2 || m.dst2_dtype != DC_NONE ||
                (m.flags & ~(DC_IMG_RGB_OUT | DC_IMG_HOST_SRC)))
                return fail(DC_ERR_INVALID_ARG, "dst_dtype must be set; dst2 must be absent; flags "
                                                "DC_IMG_RGB_OUT and DC_IMG_HOST_SRC only" + at);
            if (m.dst) {
                rc = validate_images(&m, 1, DC_IMG_RGB_OUT | DC_IMG_HOST_SRC);
                if (rc != DC_OK)
                    return rc;
            }
        }
        const double t = t_submit >= 0.0 ? t_submit : server_now(sv);
        for (int32_t i = 0; i < n; ++i) {
            dc_server::Req q;
            q.r = reqs[i];
            q.t_submit = t;
            sv->waiting.push_back(q);
            ++sv->in_system;
        }
        return DC_OK;
    });
}

int dc_server_step(dc_server *sv)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_server_step");
        g_last_error.clear();
        if (!sv)
            return fail(DC_ERR_INVALID_ARG, "server is NULL");
        int rc = check_ctx(sv->ctx);
        if (rc == DC_OK)
            rc = server_step(sv);
        return rc != DC_OK ? rc : (int)std::min<int64_t>(sv->in_system, 0x7fffffff);
    });
}

int dc_server_poll(dc_server *sv, dc_completion *out, int32_t cap)
{
    return guarded([&]() -> int {
        g_last_error.clear();
        if (!sv || cap < 0 || (cap > 0 && !out))
            return fail(DC_ERR_INVALID_ARG, "bad server or output array");
        const int32_t n = (int32_t)std::min<size_t>(sv->done.size(), (size_t)cap);
        std::copy(sv->done.begin(), sv->done.begin() + n, out);
        sv->done.erase(sv->done.begin(), sv->done.begin() + n);
        return n;
    });
}

int dc_server_cancel(dc_server *sv, int64_t id)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_server_cancel");
        g_last_error.clear();
        if (!sv)
            return fail(DC_ERR_INVALID_ARG, "server is NULL");
        const bool hit = dc::cancel_queued(
            sv->waiting, sv->admitted, sv->blocks,
            [id](const dc_server::Req &q) { return q.r.id == id; },
            [](const dc_server::Req &q) {
                return std::pair<size_t, size_t>(q.off, q.owned ? q.bytes : 0);
            },
            [&](const dc_server::Req &q) {
                complete(sv, q, DC_ERR_CANCELLED, 0, server_now(sv));
            });
        return hit ? 1 : 0;
    });
}

int dc_server_replay(dc_server *sv, const dc_request *reqs, const double *arrival_s, int32_t n,
                     dc_completion *out)
{
    return guarded([&]() -> int {
        TraceRange trace("dc_server_replay");
        g_last_error.clear();
        if (!sv || n < 0 || (n > 0 && (!reqs || !arrival_s || !out)))
            return fail(DC_ERR_INVALID_ARG, "bad replay arguments");
        for (int32_t i = 1; i < n; ++i)
            if (!(arrival_s[i] >= arrival_s[i - 1]))
                return fail(DC_ERR_INVALID_ARG, "arrival times must be non-decreasing");
        int rc = check_ctx(sv->ctx);
        if (rc != DC_OK)
            return rc;
        const double base = server_now(sv);
        int32_t next = 0, got = 0;
        while (got < n) {
            const double now = server_now(sv) - base;
            int32_t k = next;
            while (k < n && arrival_s[k] <= now)
                ++k;
            for (int32_t i = next; i < k; ++i) {
                rc = dc_server_submit(sv, &reqs[i], 1, base + arrival_s[i]);
                if (rc != DC_OK)
                    return rc;
            }
            next = k;
            rc = server_step(sv);
            if (rc != DC_OK)
                return rc;
            const int32_t m = dc_server_poll(sv, out + got, n - got);
            got += m;
        }
        return DC_OK;
    });
}

} // extern "C"

static_assert(sizeof(dc_stats) == sizeof(dc::StatsOut), "dc_stats layout");
static_assert(sizeof(dc_image) == 72, "dc_image layout");
