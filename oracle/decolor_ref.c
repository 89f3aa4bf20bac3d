/*
 * FP64 CPU oracle for the colour-temperature decolorization and its global
 * tone-mapping application.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may call, link or load
 * this file: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it, to decide whether the GPU results are right and to time
 * a plain CPU implementation beside them. It shares no code, header, table or
 * constant with the HIP kernels.
 *
 * What it computes (Ambalathankandy et al., "A color temperature-based
 * high-speed decolorization", arXiv 2108.13656):
 *   - Sec. II-B, Eqs. (1)-(6): the per-pixel luminance L from (R, G, B) with the
 *     two weights beta_R (warm bias of red over green, Eq. 3) and beta_k (warm
 *     over cool, Eq. 6); defaults beta_R = 0.55, beta_k = 0.8 (end of Sec. II-B).
 *   - Sec. III-B.1: a global tone curve applied to L. The paper only says the
 *     curve is a centred sigmoid for contrast enhancement; the statistics and the
 *     curve below are this project's reading of that sentence:
 *         x = ln(Lhat + eps) for every pixel of the image,
 *         mu = mean(x), sigma = population standard deviation of x,
 *         T = 1 / (1 + exp(-c (x - mu) / max(sigma, sigma_floor))).
 *
 * Readings where the paper is silent:
 *   - u8 inputs are code values 0..255, no gamma linearisation; f16 and f32
 *     inputs are the stored values.  "Normalised units" Lhat = L / 255 for u8
 *     input and Lhat = L for float input (L is degree-1 homogeneous, so the
 *     scale only fixes the unit of the output).
 *   - A black pixel (R + G + B == 0) has L = 0, the limit of Eqs. (4)-(6).
 *   - NaN and negative channel values are read as 0. A binary16 channel of
 *     +Inf reads as 65504, the format's largest finite value; a binary32
 *     channel above 1e18 (+Inf included) reads as 1e18, the top of the range
 *     the library accepts for linear input.
 *   - beta_R and beta_k may be anywhere in the closed interval [0, 1].
 *   - u8 encode rounds half up and clamps: min(255, floor(255 Lhat + 0.5)).
 *   - f16 encode is IEEE binary16 round-to-nearest-even.
 *
 * Arithmetic is plain IEEE double with the C library's sqrt, log and exp; build
 * with -O2 -fno-fast-math -ffp-contract=off so that nothing is fused or
 * reordered.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { REF_U8 = 0, REF_F16 = 1, REF_F32 = 2 };

/* ---------------------------------------------------------------- binary16 */

/* IEEE 754 binary16 to double, from the format's definition: 1 sign bit,
 * 5 exponent bits (bias 15), 10 fraction bits; exponent 0 encodes zero and
 * subnormals (fraction * 2^-24), exponent 31 encodes infinities and NaNs. */
double ref_half_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 31;
    int f = h & 1023;
    double v;
    if (e == 0)
        v = ldexp((double)f, -24);
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = ldexp(1024.0 + f, e - 25);
    return sign ? -v : v;
}

/* double to binary16 with round-to-nearest, ties to even. Magnitudes at or
 * above 65520 (the midpoint between the largest finite half and 2^16) become
 * infinity. */
uint16_t ref_double_to_half(double x)
{
    uint16_t sign = 0;
    if (isnan(x))
        return 0x7e00;
    if (signbit(x)) {
        sign = 0x8000;
        x = -x;
    }
    if (x >= 65520.0)
        return sign | 0x7c00;
    if (x == 0.0)
        return sign;
    int e2;
    frexp(x, &e2);            /* x = m * 2^e2, m in [0.5, 1) */
    int exp_unb = e2 - 1;     /* x = m' * 2^exp_unb, m' in [1, 2) */
    /* Spacing of representable halves near x: 2^(exp_unb - 10) for normals,
     * 2^-24 for subnormals. Round x / spacing to the nearest integer, ties to
     * even (x / spacing is exact: spacing is a power of two). */
    int q_exp = exp_unb < -14 ? -24 : exp_unb - 10;
    double scaled = ldexp(x, -q_exp);
    double fl = floor(scaled);
    double rem = scaled - fl;
    double k = fl;
    if (rem > 0.5 || (rem == 0.5 && fmod(fl, 2.0) != 0.0))
        k = fl + 1.0;
    double r = ldexp(k, q_exp); /* the rounded value, exactly */
    if (r >= 65520.0)
        return sign | 0x7c00;
    /* Re-encode r, which is exactly representable. */
    if (r < ldexp(1.0, -14)) {
        return sign | (uint16_t)(r * ldexp(1.0, 24));
    }
    int er;
    double mr = frexp(r, &er); /* r = mr * 2^er, mr in [0.5,1) */
    int biased = er - 1 + 15;
    uint16_t frac = (uint16_t)((mr * 2.0 - 1.0) * 1024.0);
    return sign | (uint16_t)(biased << 10) | frac;
}

/* ------------------------------------------------------------- Eqs. (1)-(6) */

static double sanitise(double v)
{
    /* NaN and negative values read as 0 (NaN fails the comparison). */
    return (v > 0.0) ? v : 0.0;
}

/* Luminance L of one pixel, Sec. II-B, Eqs. (1)-(6), evaluated in the paper's
 * order and notation. Output in the units of the input. */
double ref_decolor_px(double R, double G, double B, double beta_r, double beta_k)
{
    R = sanitise(R);
    G = sanitise(G);
    B = sanitise(B);
    double S = R + G + B;
    if (S == 0.0)
        return 0.0; /* black: limit of Eqs. (4)-(6) */

    double L_white = sqrt((R * R + G * G + B * B) / 3.0);            /* Eq. (1) */
    double L_b = B;                                                   /* Eq. (2) */
    double L_gr = sqrt(beta_r * R * R + (1.0 - beta_r) * G * G);      /* Eq. (3) */
    double wr = R / S;
    double wb = B / S;
    double L_warm = wr * L_gr + (1.0 - wr) * L_white;                 /* Eq. (4) */
    double L_cool = (1.0 - wb) * L_b + wb * L_white;                  /* Eq. (5) */
    return sqrt(beta_k * L_warm * L_warm + (1.0 - beta_k) * L_cool * L_cool); /* Eq. (6) */
}

/* All four intermediate luminances of one pixel (for tests that inspect the
 * individual equations): out = {L_white, L_gr, L_warm, L_cool, L}. */
void ref_decolor_px_terms(double R, double G, double B, double beta_r, double beta_k,
                          double *out)
{
    R = sanitise(R);
    G = sanitise(G);
    B = sanitise(B);
    double S = R + G + B;
    double L_white = sqrt((R * R + G * G + B * B) / 3.0);
    double L_gr = sqrt(beta_r * R * R + (1.0 - beta_r) * G * G);
    double L_warm = 0.0, L_cool = 0.0;
    if (S != 0.0) {
        double wr = R / S, wb = B / S;
        L_warm = wr * L_gr + (1.0 - wr) * L_white;
        L_cool = (1.0 - wb) * B + wb * L_white;
    }
    out[0] = L_white;
    out[1] = L_gr;
    out[2] = L_warm;
    out[3] = L_cool;
    out[4] = ref_decolor_px(R, G, B, beta_r, beta_k);
}

/* ------------------------------------------------- comparator channels */

/* Gray channels the paper compares its L with, in normalised units (inputs
 * already divided by 255 for 8-bit data):
 *   kind 1: Gray = 0.2989 R + 0.5870 G + 0.1140 B, the weighted sum of the
 *           MATLAB rgb2gray function quoted in Sec. I;
 *   kind 2: V of HSV = max(R, G, B) (Sec. III-B.1, Fig. GTMO);
 *   kind 3: CIE 1976 L* / 100 with Y = the kind-1 gray of the normalised
 *           values (the paper notes CIELAB L builds on the Y of YCbCr) and white
 *           Y_n = 1: 116 f(Y) - 16 with f(t) = t^(1/3) above (6/29)^3 and
 *           t / (3 (6/29)^2) + 4/29 below it.
 * NaN and negative channels read as 0. */
double ref_comparator_px(double r, double g, double b, int kind)
{
    r = sanitise(r);
    g = sanitise(g);
    b = sanitise(b);
    double y = 0.2989 * r + 0.5870 * g + 0.1140 * b;
    if (kind == 1)
        return y;
    if (kind == 2)
        return r > g ? (r > b ? r : b) : (g > b ? g : b);
    const double d = 6.0 / 29.0;
    double f = y > d * d * d ? cbrt(y) : y / (3.0 * d * d) + 4.0 / 29.0;
    return (116.0 * f - 16.0) / 100.0;
}

static double load_channel(const unsigned char *p, int dtype, int c);

/* A comparator channel of every pixel of an interleaved HWC image, in
 * normalised units (row-major, packed out). Returns 0, or -1 on a bad
 * argument. */
int ref_comparator_image(const void *src, int dtype, int W, int H, int64_t pitch_bytes, int kind,
                         double *out)
{
    if (!src || !out || W < 0 || H < 0 || dtype < 0 || dtype > 2 || kind < 1 || kind > 3)
        return -1;
    int es = dtype == REF_U8 ? 1 : dtype == REF_F16 ? 2 : 4;
    if (pitch_bytes < (int64_t)3 * es * W)
        return -1;
    double unit = dtype == REF_U8 ? 255.0 : 1.0;
    for (int y = 0; y < H; ++y) {
        const unsigned char *row = (const unsigned char *)src + (int64_t)y * pitch_bytes;
        for (int x = 0; x < W; ++x) {
            const unsigned char *p = row + (int64_t)3 * es * x;
            double r = load_channel(p, dtype, 0);
            double g = load_channel(p, dtype, 1);
            double b = load_channel(p, dtype, 2);
            out[(int64_t)y * W + x] = ref_comparator_px(r / unit, g / unit, b / unit, kind);
        }
    }
    return 0;
}

/* --------------------------------------------------------------- encoders */

/* Normalised Lhat -> 8-bit code: round half up, clamp to [0, 255]. */
uint8_t ref_encode_u8(double lhat)
{
    double v = floor(255.0 * sanitise(lhat) + 0.5);
    return (uint8_t)(v > 255.0 ? 255.0 : v);
}

void ref_encode_u8_array(const double *lhat, int64_t n, uint8_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = ref_encode_u8(lhat[i]);
}

void ref_encode_f16_array(const double *v, int64_t n, uint16_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = ref_double_to_half(v[i]);
}

void ref_decode_f16_array(const uint16_t *h, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = ref_half_to_double(h[i]);
}

/* ------------------------------------------------------------ whole images */

/* Upper end of a float channel: +Inf in binary16 reads as 65504 (the largest
 * finite binary16), anything above 1e18 in binary32 as 1e18 (the top of the
 * supported range). NaN passes through (sanitise reads it as 0). */
static double cap_channel(double v, int dtype)
{
    const double hi = dtype == REF_F16 ? 65504.0 : 1e18;
    return v > hi ? hi : v;
}

static double load_channel(const unsigned char *p, int dtype, int c)
{
    switch (dtype) {
    case REF_U8:
        return (double)p[c];
    case REF_F16: {
        uint16_t h;
        memcpy(&h, p + 2 * c, 2);
        return cap_channel(ref_half_to_double(h), REF_F16);
    }
    default: {
        float f;
        memcpy(&f, p + 4 * c, 4);
        return cap_channel((double)f, REF_F32);
    }
    }
}

static int dtype_size(int dtype)
{
    return dtype == REF_U8 ? 1 : dtype == REF_F16 ? 2 : 4;
}

typedef struct {
    const unsigned char *src;
    int dtype, W;
    int64_t pitch;
    double beta_r, beta_k;
    double *out;
    int row0, row1;
} rows_job;

static void decolor_rows(const rows_job *j)
{
    int es = dtype_size(j->dtype);
    double unit = j->dtype == REF_U8 ? 255.0 : 1.0;
    for (int y = j->row0; y < j->row1; ++y) {
        const unsigned char *row = j->src + (int64_t)y * j->pitch;
        for (int x = 0; x < j->W; ++x) {
            const unsigned char *p = row + (int64_t)3 * es * x;
            double R = load_channel(p, j->dtype, 0);
            double G = load_channel(p, j->dtype, 1);
            double B = load_channel(p, j->dtype, 2);
            j->out[(int64_t)y * j->W + x] = ref_decolor_px(R, G, B, j->beta_r, j->beta_k) / unit;
        }
    }
}

static void *decolor_rows_thread(void *arg)
{
    decolor_rows((const rows_job *)arg);
    return NULL;
}

/* Normalised luminance Lhat of every pixel of an interleaved HWC RGB image.
 * src: host pointer, row y starts at src + y * pitch_bytes; out: W*H doubles,
 * row-major and packed. nthreads <= 1 runs on the calling thread; otherwise the
 * rows are split into nthreads contiguous bands. Returns 0, or -1 on a bad
 * argument. */
int ref_decolorize_image(const void *src, int dtype, int W, int H, int64_t pitch_bytes,
                         double beta_r, double beta_k, double *out, int nthreads)
{
    if (!src || !out || W < 0 || H < 0 || dtype < 0 || dtype > 2)
        return -1;
    if (pitch_bytes < (int64_t)3 * dtype_size(dtype) * W)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > H)
        nthreads = H > 0 ? H : 1;
    rows_job *jobs = (rows_job *)calloc((size_t)nthreads, sizeof(rows_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return -1;
    }
    for (int t = 0; t < nthreads; ++t) {
        rows_job j = {(const unsigned char *)src, dtype, W, pitch_bytes, beta_r, beta_k, out,
                      (int)((int64_t)H * t / nthreads), (int)((int64_t)H * (t + 1) / nthreads)};
        jobs[t] = j;
    }
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&tids[t], NULL, decolor_rows_thread, &jobs[t]);
    decolor_rows(&jobs[0]);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(tids[t], NULL);
    free(jobs);
    free(tids);
    return 0;
}

/* L in code units for every 24-bit colour: out[(R << 16) | (G << 8) | B]. */
void ref_all_colours(double beta_r, double beta_k, double *out)
{
    for (int r = 0; r < 256; ++r)
        for (int g = 0; g < 256; ++g)
            for (int b = 0; b < 256; ++b)
                out[(r << 16) | (g << 8) | b] = ref_decolor_px(r, g, b, beta_r, beta_k);
}

/* ---------------------------------------------------- global tone mapping */

/* Statistics of x = ln(Lhat + eps) over all n pixels of one image, two passes
 * in double: stats = {mu, sigma, min Lhat, max Lhat}. n == 0 gives zeros. */
void ref_tonemap_stats(const double *lhat, int64_t n, double eps, double *stats)
{
    if (n <= 0) {
        stats[0] = stats[1] = stats[2] = stats[3] = 0.0;
        return;
    }
    double sum = 0.0, mn = lhat[0], mx = lhat[0];
    for (int64_t i = 0; i < n; ++i) {
        sum += log(lhat[i] + eps);
        if (lhat[i] < mn)
            mn = lhat[i];
        if (lhat[i] > mx)
            mx = lhat[i];
    }
    double mu = sum / (double)n;
    double ss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = log(lhat[i] + eps) - mu;
        ss += d * d;
    }
    stats[0] = mu;
    stats[1] = sqrt(ss / (double)n);
    stats[2] = mn;
    stats[3] = mx;
}

/* The same statistics over a multiset of values: value lhat[i] occurs count[i]
 * times (count[i] >= 0), so an image can be given as the histogram of its
 * colours. The total count is the number of pixels; values with count 0 take
 * no part, also not in the extremes. */
void ref_tonemap_stats_counted(const double *lhat, const int64_t *count, int64_t n, double eps,
                               double *stats)
{
    double total = 0.0, sum = 0.0, mn = INFINITY, mx = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        if (count[i] <= 0)
            continue;
        total += (double)count[i];
        sum += (double)count[i] * log(lhat[i] + eps);
        if (lhat[i] < mn)
            mn = lhat[i];
        if (lhat[i] > mx)
            mx = lhat[i];
    }
    if (total == 0.0) {
        stats[0] = stats[1] = stats[2] = stats[3] = 0.0;
        return;
    }
    double mu = sum / total;
    double ss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (count[i] <= 0)
            continue;
        double d = log(lhat[i] + eps) - mu;
        ss += (double)count[i] * d * d;
    }
    stats[0] = mu;
    stats[1] = sqrt(ss / total);
    stats[2] = mn;
    stats[3] = mx;
}

/* The centred sigmoid on one pixel, given the image's mu and sigma. */
double ref_tonemap_curve(double lhat, double eps, double contrast, double mu, double sigma,
                         double sigma_floor)
{
    double s = sigma > sigma_floor ? sigma : sigma_floor;
    double x = log(lhat + eps);
    return 1.0 / (1.0 + exp(-contrast * (x - mu) / s));
}

void ref_tonemap_curve_array(const double *lhat, int64_t n, double eps, double contrast,
                             double mu, double sigma, double sigma_floor, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = ref_tonemap_curve(lhat[i], eps, contrast, mu, sigma, sigma_floor);
}

/* Whole global tone map of one image: decolorize (threaded over rows), the
 * statistics (single thread), then the curve. lhat_out (W*H, may be NULL)
 * receives the normalised luminance, t_out (W*H) the curve value, stats the
 * four figures of ref_tonemap_stats. Returns 0, or -1 on a bad argument or
 * allocation failure. */
int ref_tonemap_image(const void *src, int dtype, int W, int H, int64_t pitch_bytes,
                      double beta_r, double beta_k, double eps, double contrast,
                      double sigma_floor, double *lhat_out, double *t_out, double *stats,
                      int nthreads)
{
    int64_t n = (int64_t)W * H;
    double *lhat = lhat_out;
    if (!t_out || !stats)
        return -1;
    if (!lhat) {
        lhat = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        if (!lhat)
            return -1;
    }
    int rc = ref_decolorize_image(src, dtype, W, H, pitch_bytes, beta_r, beta_k, lhat, nthreads);
    if (rc == 0) {
        ref_tonemap_stats(lhat, n, eps, stats);
        ref_tonemap_curve_array(lhat, n, eps, contrast, stats[0], stats[1], sigma_floor, t_out);
    }
    if (!lhat_out)
        free(lhat);
    return rc;
}

/* ------------------------------------------------- colour re-synthesis */

/* Colour output of the global tone map. Sec. III-B.1 shows its tone-mapped
 * results in colour but gives no re-colouring formula; the reading used here
 * is the classic ratio re-colouring of a tone-mapped luminance: each channel
 * C of the pixel, in the same normalised units as Lhat, becomes
 *     C_out = min(1, T (C / Lhat)^s),
 * with saturation exponent s >= 0 and 0^0 = 1. With s = 1 every channel ratio
 * is kept and, Eqs. (1)-(6) being homogeneous of degree 1, the luminance of the
 * unclamped output is T itself; s = 0 gives the grey T. A pixel with
 * Lhat == 0 has no defined ratio and becomes grey T. NaN and negative channel
 * values read as 0, as in the luminance. */
double ref_colour_channel(double c, double lhat, double t, double s)
{
    c = sanitise(c);
    if (!(lhat > 0.0))
        return t;
    double v = t * pow(c / lhat, s);
    return v < 1.0 ? v : 1.0;
}

/* The colour output of any tone map: every channel of every pixel
 * re-coloured by ref_colour_channel from the image's Lhat and tone-mapped T
 * (W*H doubles each, row-major) into rgb_out (W*H*3, channels interleaved).
 * Returns 0, or -1 on a bad argument. */
int ref_recolour_image(const void *src, int dtype, int W, int H, int64_t pitch_bytes,
                       const double *lhat, const double *t, double saturation, double *rgb_out)
{
    if (!src || !lhat || !t || !rgb_out || W < 0 || H < 0 || dtype < 0 || dtype > 2 ||
        !(saturation >= 0.0))
        return -1;
    int es = dtype_size(dtype);
    double unit = dtype == REF_U8 ? 255.0 : 1.0;
    for (int y = 0; y < H; ++y) {
        const unsigned char *row = (const unsigned char *)src + (int64_t)y * pitch_bytes;
        for (int x = 0; x < W; ++x) {
            const unsigned char *p = row + (int64_t)3 * es * x;
            int64_t i = (int64_t)y * W + x;
            for (int c = 0; c < 3; ++c)
                rgb_out[3 * i + c] = ref_colour_channel(load_channel(p, dtype, c) / unit, lhat[i],
                                                        t[i], saturation);
        }
    }
    return 0;
}

/* Colour global tone map of one image: T, Lhat and the statistics as
 * ref_tonemap_image, then the re-coloured RGB of every pixel into rgb_out
 * (W*H*3 doubles, row-major, channels interleaved). lhat_out may be NULL.
 * Returns 0, or -1 on a bad argument or allocation failure. */
int ref_tonemap_colour_image(const void *src, int dtype, int W, int H, int64_t pitch_bytes,
                             double beta_r, double beta_k, double eps, double contrast,
                             double sigma_floor, double saturation, double *lhat_out,
                             double *t_out, double *rgb_out, double *stats, int nthreads)
{
    int64_t n = (int64_t)W * H;
    double *lhat = lhat_out;
    if (!t_out || !rgb_out || !stats || !(saturation >= 0.0))
        return -1;
    if (!lhat) {
        lhat = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        if (!lhat)
            return -1;
    }
    int rc = ref_tonemap_image(src, dtype, W, H, pitch_bytes, beta_r, beta_k, eps, contrast,
                               sigma_floor, lhat, t_out, stats, nthreads);
    if (rc == 0)
        rc = ref_recolour_image(src, dtype, W, H, pitch_bytes, lhat, t_out, saturation, rgb_out);
    if (!lhat_out)
        free(lhat);
    return rc;
}

/* ------------------------------------------------------ local tone mapping */

/* Local tone map on the luminance, Sec. III-B.2. The paper builds it on
 * smoothed local histogram equalisation (tone curves from local cumulative
 * histograms, as in its cited O(1) design) and gives no equations; the
 * reading used here, step by step:
 *   1. Lhat, the global statistics and the global curve T_g of every pixel,
 *      exactly as ref_tonemap_image.
 *   2. The pixel's position on a fixed log2 scale of 64 bins, 2 per stop,
 *      starting at eps: u = clamp(2 log2((Lhat + eps) / eps) - 0.5, 0, 63),
 *      so bin centres are the integers 0..63.
 *   3. Histograms on a grid of 64 x 64-pixel tiles (edge tiles may be
 *      smaller): each pixel puts mass 1 - f on bin k and f on bin k + 1,
 *      k = min(floor(u), 62), f = u - k (linear soft binning).
 *   4. Spatial smoothing: H_t = sum over the 3 x 3 neighbouring tiles t' of
 *      w(dx) w(dy) h_t', w(0) = 2, w(+-1) = 1, tiles outside the grid absent.
 *   5. The tile's tone curve is the cumulative distribution of its smoothed
 *      histogram with every bin's mass spread by the unit triangle kernel:
 *      F_t(u) = sum_b H_t(b) R(u - b) / sum_b H_t(b), R the integral of the
 *      triangle max(0, 1 - |x|).
 *   6. The pixel's local value interpolates the curves of the four tile
 *      centres around it bilinearly (tile t's centre at 64 t + 32 pixels,
 *      clamped at the grid's edges): T_l.
 *   7. Output T = (1 - strength) T_g + strength T_l.
 * Returns 0, or -1 on a bad argument or allocation failure. */

#define REF_LTM_TILE 64
#define REF_LTM_BINS 64

static double ltm_u(double lhat, double eps)
{
    double u = 2.0 * log2((lhat + eps) / eps) - 0.5;
    if (!(u > 0.0))
        return 0.0;
    return u < REF_LTM_BINS - 1 ? u : (double)(REF_LTM_BINS - 1);
}

/* Integral of the unit triangle kernel, from -inf to x. */
static double ltm_tri_cdf(double x)
{
    if (x <= -1.0)
        return 0.0;
    if (x <= 0.0)
        return 0.5 * (1.0 + x) * (1.0 + x);
    if (x <= 1.0)
        return 1.0 - 0.5 * (1.0 - x) * (1.0 - x);
    return 1.0;
}

/* sample: NULL, or nsample pixel indices (y * W + x) at which alone T is
 * evaluated into t_out[0 .. nsample) (steps 1 to 4 still cover every pixel). */
int ref_tonemap_local_image(const void *src, int dtype, int W, int H, int64_t pitch_bytes,
                            double beta_r, double beta_k, double eps, double contrast,
                            double sigma_floor, double strength, double *t_out, double *stats,
                            int nthreads, const int64_t *sample, int64_t nsample)
{
    if (!t_out || !stats || W < 1 || H < 1 || !(strength >= 0.0 && strength <= 1.0))
        return -1;
    const int64_t n = (int64_t)W * H;
    const int nx = (W + REF_LTM_TILE - 1) / REF_LTM_TILE, ny = (H + REF_LTM_TILE - 1) / REF_LTM_TILE;
    double *lhat = (double *)malloc((size_t)n * sizeof(double));
    double *tg = (double *)malloc((size_t)n * sizeof(double));
    double *hist = (double *)calloc((size_t)nx * ny * REF_LTM_BINS, sizeof(double));
    double *smooth = (double *)calloc((size_t)nx * ny * REF_LTM_BINS, sizeof(double));
    int rc = -1;
    if (!lhat || !tg || !hist || !smooth)
        goto done;
    /* step 1 */
    rc = ref_tonemap_image(src, dtype, W, H, pitch_bytes, beta_r, beta_k, eps, contrast,
                           sigma_floor, lhat, tg, stats, nthreads);
    if (rc != 0)
        goto done;
    /* steps 2 and 3 */
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double u = ltm_u(lhat[(int64_t)y * W + x], eps);
            int k = (int)floor(u);
            if (k > REF_LTM_BINS - 2)
                k = REF_LTM_BINS - 2;
            double f = u - k;
            double *h = hist + ((int64_t)(y / REF_LTM_TILE) * nx + x / REF_LTM_TILE) * REF_LTM_BINS;
            h[k] += 1.0 - f;
            h[k + 1] += f;
        }
    /* step 4 */
    for (int ty = 0; ty < ny; ++ty)
        for (int tx = 0; tx < nx; ++tx) {
            double *s = smooth + ((int64_t)ty * nx + tx) * REF_LTM_BINS;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int sx = tx + dx, sy = ty + dy;
                    if (sx < 0 || sx >= nx || sy < 0 || sy >= ny)
                        continue;
                    double w = (dx == 0 ? 2.0 : 1.0) * (dy == 0 ? 2.0 : 1.0);
                    const double *h = hist + ((int64_t)sy * nx + sx) * REF_LTM_BINS;
                    for (int b = 0; b < REF_LTM_BINS; ++b)
                        s[b] += w * h[b];
                }
        }
    /* steps 5 to 7 */
    for (int64_t j = 0; j < (sample ? nsample : n); ++j) {
        const int64_t pix = sample ? sample[j] : j;
        if (pix < 0 || pix >= n) {
            rc = -1;
            goto done;
        }
        const int y = (int)(pix / W), x = (int)(pix % W);
        double gy = (y + 0.5) / REF_LTM_TILE - 0.5;
        int ty0 = (int)floor(gy);
        double fy = gy - ty0;
        if (ty0 < 0) {
            ty0 = 0;
            fy = 0.0;
        }
        if (ty0 >= ny - 1) {
            ty0 = ny - 1;
            fy = 0.0;
        }
        int ty1 = ty0 + 1 < ny ? ty0 + 1 : ny - 1;
        {
            double gx = (x + 0.5) / REF_LTM_TILE - 0.5;
            int tx0 = (int)floor(gx);
            double fx = gx - tx0;
            if (tx0 < 0) {
                tx0 = 0;
                fx = 0.0;
            }
            if (tx0 >= nx - 1) {
                tx0 = nx - 1;
                fx = 0.0;
            }
            int tx1 = tx0 + 1 < nx ? tx0 + 1 : nx - 1;
            int64_t i = (int64_t)y * W + x;
            double u = ltm_u(lhat[i], eps);
            const int tyy[4] = {ty0, ty0, ty1, ty1}, txx[4] = {tx0, tx1, tx0, tx1};
            const double wt[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
            double tl = 0.0;
            for (int c = 0; c < 4; ++c) {
                const double *s = smooth + ((int64_t)tyy[c] * nx + txx[c]) * REF_LTM_BINS;
                double num = 0.0, den = 0.0;
                for (int b = 0; b < REF_LTM_BINS; ++b) {
                    num += s[b] * ltm_tri_cdf(u - b);
                    den += s[b];
                }
                tl += wt[c] * (num / den);
            }
            t_out[j] = (1.0 - strength) * tg[i] + strength * tl;
        }
    }
done:
    free(lhat);
    free(tg);
    free(hist);
    free(smooth);
    return rc;
}
