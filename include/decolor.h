/*
 * decolor.h - C ABI of the MI355X (gfx950) colour-temperature decolorization
 * library.
 *
 * The method: Ambalathankandy et al., "A color temperature-based high-speed
 * decolorization: an empirical approach for tone mapping applications"
 * (arXiv 2108.13656).
 *   - Decolorization, Sec. II-B, Eqs. (1)-(6): per pixel,
 *       L_white = sqrt((R^2 + G^2 + B^2) / 3)                       (1)
 *       L_b     = B                                                  (2)
 *       L_gr    = sqrt(beta_R R^2 + (1 - beta_R) G^2)                (3)
 *       L_warm  = R/S L_gr + (1 - R/S) L_white,  S = R + G + B        (4)
 *       L_cool  = (1 - B/S) L_b + B/S L_white                         (5)
 *       L       = sqrt(beta_k L_warm^2 + (1 - beta_k) L_cool^2)      (6)
 *     with beta_R = 0.55, beta_k = 0.8 (the values chosen after Eq. (6)).
 *   - Global tone mapping on L, Sec. III-B.1: the paper names a centred
 *     sigmoid tone curve; this library reads it as
 *       x = ln(Lhat + eps) over all pixels of one image,
 *       mu = mean(x), sigma = population standard deviation of x,
 *       T  = 1 / (1 + exp(-contrast (x - mu) / max(sigma, sigma_floor))).
 *     The paper shows its tone-mapped results in colour without a formula;
 *     the colour output (DC_IMG_RGB_OUT) is read as the ratio re-colouring
 *       C_out = min(1, T (C / Lhat)^s)   for C = R, G, B (normalised units),
 *     saturation s >= 0; a pixel with Lhat == 0 becomes grey T. With s = 1
 *     the channel ratios are kept and the output's Eqs. (1)-(6) luminance is
 *     T wherever no channel was clamped.
 *
 * Units. 8-bit inputs are code values 0..255 (no gamma linearisation); binary16
 * and binary32 inputs are linear values as stored. Lhat, the "normalised"
 * luminance, is L / 255 for 8-bit input and L itself for float input. A black
 * pixel (R + G + B == 0) has L = 0; NaN and negative channels read as 0. Float
 * inputs are meant to lie in [0, 1e18]; values below 1e-30 may be flushed.
 *
 * Output encodings (dst, dst2): DC_F32 = the value as float; DC_F16 = binary16,
 * round to nearest even; DC_U8 = min(255, floor(255 v + 0.5)) with v clamped
 * to >= 0, where v is Lhat for decolorization and T for tone mapping.
 *
 * Memory. Every image pointer (src, dst, dst2) is a DEVICE pointer on the
 * context's device, owned by the caller, and must stay valid until the work
 * enqueued on `stream` has completed. Images are interleaved HWC RGB (3
 * channels, R first) with a row pitch in bytes; outputs are one channel with
 * their own row pitch. Host arrays passed to a call (dc_image lists, params)
 * are read before the call returns and may be freed at once. The context owns
 * its workspace (descriptor tables, statistics partials) and frees it in
 * dc_destroy. Every pixel is read and written with 12-byte vector units
 * (4 8-bit, 2 binary16 or 1 binary32 pixels) whatever the alignment of its
 * element: rows whose pitch exceeds their bytes (crops, padding) are tiled
 * like their packed copy, for widths of 4 to 46000 pixels and row padding
 * below 256 KiB; images past those limits are walked pixel by pixel, still
 * correct but slower.
 *
 * Streams. `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * All compute calls are asynchronous with respect to the host.
 *
 * Errors. Calls return DC_OK (0) or a negative DC_ERR_* code. Arguments are
 * validated before anything is enqueued; a batch is all-or-nothing. Nothing
 * aborts and no C++ exception crosses this interface. dc_last_error_message()
 * gives a thread-local description of the last failure.
 *
 * Threads. A context is not thread-safe: use one per host thread, or
 * serialise the calls that use it (its plans' and servers' calls included),
 * as the Python binding does with one lock per device context.
 */
#ifndef DECOLOR_H
#define DECOLOR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DC_ABI_VERSION 1

/* Status codes. */
#define DC_OK 0
#define DC_ERR_INVALID_ARG (-1) /* null pointer, bad size, pitch, dtype or parameter */
#define DC_ERR_UNSUPPORTED (-2) /* a combination the library does not implement */
#define DC_ERR_ALIAS (-3)       /* an output overlaps an input or another output */
#define DC_ERR_NO_MEMORY (-4)   /* a device or host allocation failed */
#define DC_ERR_HIP (-5)         /* a HIP runtime call failed */
#define DC_ERR_NO_DEVICE (-6)   /* no usable GPU, or the device index is out of range */
#define DC_ERR_CANCELLED (-7)   /* serving: the request was cancelled before its launch */

/* Element types. DC_NONE marks an absent optional output. */
#define DC_NONE (-1)
#define DC_U8 0
#define DC_F16 1
#define DC_F32 2

/* Eq. (3) and Eq. (6) weights. Each must be finite and in [0, 1] (the paper
 * uses the open interval (0.5, 1); the blends stay convex on all of [0, 1]). */
typedef struct dc_params {
    float beta_r; /* default 0.55 */
    float beta_k; /* default 0.80 */
} dc_params;

/* Tone-curve parameters (Sec. III-B.1 reading above). eps > 0 keeps the
 * logarithm finite on black pixels; contrast > 0 is the slope in units of the
 * image's standard deviation; sigma_floor > 0 bounds the slope on flat images;
 * saturation in [0, 2] is the exponent s of the colour output (used only by
 * images flagged DC_IMG_RGB_OUT); local_strength in [0, 1] is the weight of the
 * local curve in dc_tonemap_local (0 gives the global tone map). Note that a
 * zero-filled struct asks for s = 0 (grey) and strength 0. */
typedef struct dc_tm_params {
    float eps;            /* default 1e-4 */
    float contrast;       /* default 2.0  */
    float sigma_floor;    /* default 1e-3 */
    float saturation;     /* default 1.0  */
    float local_strength; /* default 0.5  */
} dc_tm_params;

/* One image. width, height >= 1. src_pitch >= 3 * width * sizeof(src element);
 * dst_pitch >= width * sizeof(dst element); dst2 (optional, NULL with
 * dst2_dtype = DC_NONE) likewise. Outputs must not overlap the input or each
 * other. flags is 0, or DC_IMG_RGB_OUT in a tone-map call (dc_tonemap_global,
 * dc_tonemap_local, their plans, server requests): dst then receives the re-coloured
 * interleaved RGB (3 channels, R first, dst_pitch >= 3 * width * sizeof(dst
 * element)) instead of the gray T; dst2 keeps its meaning. Other calls reject
 * the flag with DC_ERR_UNSUPPORTED; unknown bits are DC_ERR_INVALID_ARG. */
#define DC_IMG_RGB_OUT 1
/* Server requests only: img.src is a HOST pointer (pinned memory, e.g. from
 * hipHostMalloc, for an asynchronous copy). The server copies the image into
 * its device budget on the launch lane's stream before the kernels. */
#define DC_IMG_HOST_SRC 2
typedef struct dc_image {
    const void *src; /* device, interleaved RGB, row y at src + y * src_pitch */
    void *dst;       /* device, 1 channel */
    void *dst2;      /* device, 1 channel, or NULL */
    int64_t src_pitch;
    int64_t dst_pitch;
    int64_t dst2_pitch;
    int32_t width;
    int32_t height;
    int32_t src_dtype;  /* DC_U8, DC_F16 or DC_F32 */
    int32_t dst_dtype;  /* DC_U8, DC_F16 or DC_F32 */
    int32_t dst2_dtype; /* DC_NONE, DC_U8, DC_F16 or DC_F32 */
    int32_t flags;      /* 0 or DC_IMG_RGB_OUT */
} dc_image;

/* Per-image statistics of the global tone map (FP32 accumulation). */
typedef struct dc_stats {
    float log_mean; /* mu: mean of ln(Lhat + eps) */
    float log_std;  /* sigma: population standard deviation of ln(Lhat + eps) */
    float l_min;    /* smallest Lhat */
    float l_max;    /* largest Lhat */
    int64_t count;  /* pixels, width * height */
} dc_stats;

typedef struct dc_ctx dc_ctx;

/* Creates a context bound to HIP device `device` (it becomes current on the
 * calling thread). *ctx receives the handle. Errors: DC_ERR_INVALID_ARG (ctx
 * NULL), DC_ERR_NO_DEVICE, DC_ERR_NO_MEMORY, DC_ERR_HIP. */
int dc_create(dc_ctx **ctx, int device);

/* Synchronises the device and frees the context's workspace. NULL is a no-op. */
int dc_destroy(dc_ctx *ctx);

/* Host-only argument check, the same one every compute call runs first; it
 * touches no GPU and needs no context. tm may be NULL when no tone map is
 * meant. Returns DC_OK or the error the compute call would return. */
int dc_validate(const dc_image *imgs, int32_t n, const dc_params *params,
                const dc_tm_params *tm);

/* Decolorization of one image, Sec. II-B, Eqs. (1)-(6): writes Lhat of every
 * pixel to img->dst (and img->dst2 if set), each in its own encoding. params
 * NULL means the defaults. One pass over the input, one over each output. */
int dc_decolorize(dc_ctx *ctx, const dc_image *img, const dc_params *params, void *stream);

/* Decolorization of n images of any sizes and element types in one persistent
 * launch over a device tile table (Sec. II-B, Eqs. (1)-(6) per pixel). imgs is
 * a HOST array of n descriptors; n == 0 is a no-op. The result of every image
 * is bit-identical to dc_decolorize on that image alone. */
int dc_decolorize_batch(dc_ctx *ctx, const dc_image *imgs, int32_t n, const dc_params *params,
                        void *stream);

/* As dc_decolorize_batch, but image i uses its own weights betas[i] (a HOST
 * array of n dc_params; NULL means the defaults for all). This is the
 * weight-sweep explorer of Fig. 4, which plots how beta_R and beta_k bias L
 * along colour ramps: a sweep of one image over many (beta_R, beta_k) pairs is
 * n descriptors sharing one src with n outputs, all in one launch. When every
 * descriptor has the same src, size, src_pitch, dst_dtype and dst_pitch and
 * no dst2, the launch reads each
 * input tile once for all the pairs (the weight-independent terms of Eqs.
 * (1)-(6) are evaluated once per pixel); otherwise it is the tile table of
 * dc_decolorize_batch. Every weight must be finite and in [0, 1]. Results are
 * bit-identical to dc_decolorize of each image with its weights either way. */
int dc_decolorize_batch_betas(dc_ctx *ctx, const dc_image *imgs, int32_t n,
                              const dc_params *betas, void *stream);

/* Global tone map (Sec. III-B.1 reading above) of n images: per image, one
 * statistics pass fused with the decolorization (Eqs. (1)-(6)), a fixed-order
 * combine of per-chunk partials, and a curve pass that recomputes L and writes
 * T to dst, or the re-coloured RGB for images flagged DC_IMG_RGB_OUT (and
 * Lhat to dst2 if set). imgs is a HOST array; tm NULL means the
 * defaults; stats, if not NULL, is a DEVICE array of n dc_stats that receives
 * each image's statistics. Results of an image do not depend on which other
 * images share the call. */
int dc_tonemap_global(dc_ctx *ctx, const dc_image *imgs, int32_t n, const dc_params *params,
                      const dc_tm_params *tm, dc_stats *stats, void *stream);

/* For callers that cannot allocate (code that must not call hipMalloc or
 * allocate host memory per call: tight serving loops, harnesses that forbid
 * it): dc_tonemap_global with the same arguments and bit-identical results,
 * but the call allocates nothing, on the device or the host. Its workspace
 * (descriptor table, statistics partials, curves) is one fixed device array of
 * DC_NOALLOC_SCRATCH_BYTES per device, held until the process ends and shared
 * by every call of this entry point on that device: it keeps the last call's
 * contents (every call rewrites what it reads), and calls that overlap on one
 * device (on other streams, contexts or threads) race on it, so serialise
 * them. The descriptor table goes up from pinned staging that dc_create sets
 * aside; a call first waits for the previous call's upload (not its kernels).
 * Limits: n <= DC_NOALLOC_MAX_IMAGES and about 340 Mpx per call (24 bytes of
 * partials per 1024 pixels plus the table must fit the array); a larger call
 * returns DC_ERR_INVALID_ARG before any work. It always runs the batch
 * schedule (statistics pass over every image, combine, curve pass). Errors
 * otherwise as dc_tonemap_global. */
#define DC_NOALLOC_SCRATCH_BYTES (8 << 20)
#define DC_NOALLOC_MAX_IMAGES 1024
int dc_tonemap_global_noalloc(dc_ctx *ctx, const dc_image *imgs, int32_t n,
                              const dc_params *params, const dc_tm_params *tm, dc_stats *stats,
                              void *stream);

/* Local tone map (Sec. III-B.2: tone curves from smoothed local cumulative
 * histograms, the paper's choice for its local operator; it defers the
 * algorithm to its cited O(1) design). Reading, per image:
 *   u = clamp(2 log2((Lhat + eps) / eps) - 0.5, 0, 63): position on 64 bins of
 *       log2 luminance, 2 per stop, bin centres at integers;
 *   each 64 x 64-pixel tile (edge tiles smaller) collects a soft histogram
 *       (mass 1 - f on bin floor(u), f on the next; f the fraction);
 *   each tile's histogram is smoothed over its 3 x 3 tile neighbourhood with
 *       weights (1, 2, 1) x (1, 2, 1), and its curve F_t is the cumulative
 *       distribution of those masses spread by the unit triangle kernel;
 *   T_l bilinearly interpolates, at the pixel's u, the curves of the four
 *       tile centres around the pixel (centres at 64 t + 32, clamped at the
 *       grid's edges);
 *   T = (1 - local_strength) T_g + local_strength T_l, with T_g the global
 *       curve above (statistics as dc_tonemap_global, written to stats).
 * Images flagged DC_IMG_RGB_OUT get the same colour output as the global map
 * with this T: min(1, T (C / Lhat)^s) per channel. Histograms hold integer
 * masses (2^-19 per pixel), so results do not depend on the order of the
 * additions. Otherwise as dc_tonemap_global. */
int dc_tonemap_local(dc_ctx *ctx, const dc_image *imgs, int32_t n, const dc_params *params,
                     const dc_tm_params *tm, dc_stats *stats, void *stream);

/* Comparator gray channels on the same data path, for side-by-side
 * comparison with Eqs. (1)-(6) on the same GPU (the paper's run-time table
 * compares its method with CIELAB L on one CPU; Sec. I quotes the rgb2gray
 * weights; Sec. III-B.1 tone-maps Y and V as well):
 *   DC_CH_Y601:     0.2989 R + 0.5870 G + 0.1140 B
 *   DC_CH_HSV_V:    max(R, G, B)
 *   DC_CH_CIELAB_L: CIE 1976 L* / 100 on that Y with white Y_n = 1
 * on normalised inputs (8-bit / 255), written to dst (and dst2) in the same
 * encodings as dc_decolorize. imgs is a HOST array; n == 0 is a no-op. */
#define DC_CH_Y601 1
#define DC_CH_HSV_V 2
#define DC_CH_CIELAB_L 3
int dc_channel_batch(dc_ctx *ctx, const dc_image *imgs, int32_t n, int32_t channel, void *stream);

/* ---------------------------------------------------------------- plans
 * A plan freezes one call's images, parameters and launch shape: the
 * descriptor table is built, validated and copied to the device once, and
 * every dc_plan_run enqueues only the kernels. This is the batched launch of
 * dc_decolorize_batch (kind DC_PLAN_DECOLORIZE), the three-kernel tone map
 * of dc_tonemap_global (kind DC_PLAN_TONEMAP) or the local tone map of
 * dc_tonemap_local (kind DC_PLAN_LOCAL) for callers that process the
 * same buffers repeatedly (video pipelines, serving slots). The buffers named
 * by the plan must outlive it. With DC_PLAN_GRAPH the first run captures the
 * kernels into a HIP graph on `stream` (which must not be NULL) and every run
 * replays that graph. Results equal those of the corresponding direct call.
 * A plan may run on any stream of its context's device, but runs of one plan
 * must not overlap (they share its statistics workspace). */
typedef struct dc_plan dc_plan;
#define DC_PLAN_DECOLORIZE 0
#define DC_PLAN_TONEMAP 1
#define DC_PLAN_LOCAL 2
#define DC_PLAN_GRAPH 1 /* flag */

/* imgs: HOST array of n >= 1 descriptors; tm and stats (DEVICE, n entries)
 * only for the tone-map kinds; flags 0 or DC_PLAN_GRAPH. Allocates the plan's
 * device workspace and waits for its upload. Errors as dc_tonemap_global. */
int dc_plan_create(dc_ctx *ctx, int32_t kind, const dc_image *imgs, int32_t n,
                   const dc_params *params, const dc_tm_params *tm, dc_stats *stats,
                   int32_t flags, dc_plan **plan);
int dc_plan_run(dc_plan *plan, void *stream);
/* Synchronises the device and frees the plan. NULL is a no-op. */
int dc_plan_destroy(dc_plan *plan);

/* --------------------------------------------------------------- tuning
 * Launch shapes used by later calls and plans of a context. groups: vector
 * groups (48 input bytes each) per thread in a decolorization tile, 1, 2 or 4,
 * per input type (index DC_U8, DC_F16, DC_F32) and for batches mixing input
 * types; *_grid_per_cu: persistent workgroups per compute unit, 0..64, where
 * 0 launches one workgroup per tile; tonemap_pipeline m >= 1 runs the tone map
 * in groups of m images with the curve pass of one group on a second stream
 * beside the statistics pass of the next (the autotuner compares m = 0 and 1).
 * The tone map's statistics chunks are fixed
 * (1024 pixels per partial, merged in a fixed tree), so no setting changes any
 * result bit. The local tone map always runs one workgroup per 64 x 64 tile and
 * is not tuned. */
typedef struct dc_tuning {
    int32_t groups[3];
    int32_t mixed_groups;
    int32_t decolor_grid_per_cu;  /* batches of one input type */
    int32_t mixed_grid_per_cu;    /* batches mixing input types */
    int32_t pass1_grid_per_cu;
    int32_t pass2_grid_per_cu;
    int32_t tonemap_pipeline; /* 0: each pass over all images; m >= 1: groups of m images,
                                 a group's curve pass beside the next group's statistics pass
                                 on a second stream */
} dc_tuning;

int dc_get_tuning(dc_ctx *ctx, dc_tuning *out);
int dc_set_tuning(dc_ctx *ctx, const dc_tuning *tuning);

/* Autotuner: times every candidate launch shape (groups 1/2/4 x grids per CU
 * 0/1/2/4/8/16 for kind DC_PLAN_DECOLORIZE; grids per CU for each tone-map
 * pass, then the two schedules, for DC_PLAN_TONEMAP) on the given images with
 * HIP events on `stream` (fastest of 10 runs after a warm-up), keeps the best
 * in the context (the fields of the given batch's class only; the shapes in
 * place are measured first and a candidate replaces them only when it is more
 * than 2 % faster, so timing noise does not flip between equal shapes) and
 * writes it to *chosen (if not NULL). The candidate runs write the images'
 * outputs. Synchronises `stream`. kind DC_PLAN_LOCAL is not tuned
 * (DC_ERR_INVALID_ARG). With the environment variable DC_AUTOTUNE=0 the call
 * measures nothing and keeps (and reports) the shapes in place.
 *
 * Environment: DC_LOG_LEVEL=1 makes every failing call print its message
 * (dc_last_error_message) to stderr; DC_LOG_LEVEL=2 also prints the
 * autotuner's choices. Both variables are read once per process. */
int dc_autotune(dc_ctx *ctx, int32_t kind, const dc_image *imgs, int32_t n,
                const dc_params *params, const dc_tm_params *tm, void *stream,
                dc_tuning *chosen);

/* -------------------------------------------------------------- serving
 * Continuous-batching server for the global tone map of single-image requests
 * of any size and element type (each request: decolorization + statistics +
 * curve). Requests wait in FIFO order and are admitted when their output (and,
 * for host inputs, the input's device copy) fits the server's device-memory
 * budget (a first-fit arena allocated once at
 * creation); whenever one of max_inflight launch lanes (each its own stream) is
 * idle, every admitted request, up to max_batch, goes into one launch on it;
 * when a launch's completion event fires its requests complete and their
 * memory returns to the budget, admitting more. Work of different lanes
 * overlaps on the device. Each request's result is bit-identical to
 * dc_tonemap_global on that image alone (the statistics of an image never
 * depend on its batch). Not thread-safe; one host thread drives a server. */
typedef struct dc_server dc_server;

typedef struct dc_server_config {
    int64_t budget_bytes;  /* device bytes for server-allocated outputs and input copies, > 0 */
    int32_t max_batch;     /* images per launch, >= 1 */
    int32_t max_inflight;  /* launch lanes, 1..8 */
    int32_t flags;         /* reserved, 0 */
    dc_params params;      /* Eqs. (3), (6) weights */
    dc_tm_params tm;       /* tone curve */
} dc_server_config;

/* One request. img.src (DEVICE, or HOST with DC_IMG_HOST_SRC), size,
 * src_dtype and dst_dtype as in dc_image; dst2 must be NULL (dst2_dtype
 * DC_NONE); flags may hold DC_IMG_RGB_OUT and DC_IMG_HOST_SRC. With img.dst
 * NULL the server allocates the output (rows packed) from its budget and frees
 * it when the request completes (the output is not kept); with img.dst set
 * (caller memory, dst_pitch given) the output stays there and takes no budget.
 * A host input takes budget for its device copy (rows packed) until the
 * request completes; the host memory must stay valid until then. Packed host
 * rows (src_pitch = 3 * width * element size) go over in one linear copy;
 * pitched ones take hipMemcpy2DAsync, which is much slower. */
typedef struct dc_request {
    int64_t id;
    dc_image img;
} dc_request;

/* A finished request. Times are seconds on the server clock (dc_server_clock):
 * submitted (for replays: the scheduled arrival), admitted, launched, and the
 * step that saw its launch complete. status is DC_OK; DC_ERR_NO_MEMORY for a
 * request whose output is larger than the whole budget (rejected at once);
 * DC_ERR_CANCELLED for a request cancelled before its launch (t_launch is 0
 * for a request that never launched; t_admit too if it was never admitted); or,
 * when enqueueing its launch failed, that failure's status (the step that saw
 * it returns it too, after waiting for the lane and freeing the batch's
 * memory). */
typedef struct dc_completion {
    int64_t id;
    int32_t status;
    int32_t batch_size;
    double t_submit, t_admit, t_launch, t_done;
} dc_completion;

int dc_server_create(dc_ctx *ctx, const dc_server_config *cfg, dc_server **server);
/* Waits for the server's lanes and frees its arena. NULL is a no-op. */
int dc_server_destroy(dc_server *server);
/* Queues n HOST request descriptors (copied); t_submit < 0 means now. Each is
 * checked like dc_validate (its input part, and its output when given). */
int dc_server_submit(dc_server *server, const dc_request *reqs, int32_t n, double t_submit);
/* Non-blocking: retires finished launches, admits what fits, launches on idle
 * lanes. Returns the number of requests still queued or running (>= 0), or
 * a negative status. */
int dc_server_step(dc_server *server);
/* Moves up to cap completions (oldest first) into out (HOST); returns the count. */
int dc_server_poll(dc_server *server, dc_completion *out, int32_t cap);
/* Cancels request `id` if it has not been launched yet (it is still waiting,
 * or admitted but not yet in a launch): it completes at once with status
 * DC_ERR_CANCELLED and its memory returns to the budget. Returns 1 when a
 * request was cancelled, 0 when no queued request has that id (unknown,
 * already launched or already complete), or a negative status. With several
 * queued requests of one id, the oldest is cancelled. */
int dc_server_cancel(dc_server *server, int64_t id);
double dc_server_clock(dc_server *server);
/* Host cost of the server's launches since it was created: the seconds spent
 * enqueueing lane launches (descriptor table, upload and kernels of each
 * batch) and how many there were. Either pointer may be NULL. Errors:
 * DC_ERR_INVALID_ARG for a NULL server. */
int dc_server_host_stats(dc_server *server, double *launch_seconds, int64_t *launches);
/* Trace replay: submits reqs[i] when arrival_s[i] (seconds from the call,
 * non-decreasing) has passed, stepping the server in a busy loop until all n
 * have completed; out (HOST, n entries) receives the completions in the
 * order they finished. */
int dc_server_replay(dc_server *server, const dc_request *reqs, const double *arrival_s,
                     int32_t n, dc_completion *out);

/* Measurement hooks (instrumentation, not part of the method). With on != 0,
 * every later compute call on ctx records timing events on its stream before
 * and after each kernel it launches: decolorize, decolorize_batch,
 * decolorize_batch_betas and channel_batch record one interval (their one
 * kernel, or run of kernels); tonemap_global records three (the statistics
 * pass, the two-level combine, the curve pass), or one (the whole sequence)
 * when the two-stream schedule is selected; tonemap_local records three (the
 * statistics-and-histogram pass, the combine with the curve tables, the curve
 * pass). dc_last_timings waits for the
 * last such call to finish and writes up to cap interval lengths in
 * milliseconds to ms (host array); it returns how many it wrote, or a negative
 * status. Only the most recent call's intervals are kept. */
int dc_set_profiling(dc_ctx *ctx, int on);
int dc_last_timings(dc_ctx *ctx, float *ms, int32_t cap);

/* Static description of a status code. */
const char *dc_status_string(int status);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *dc_last_error_message(void);

/* DC_ABI_VERSION of the built library. */
int dc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DECOLOR_H */
