/*
 * afr_oracle.c -- plain, slow FP64 reference for temporally adaptive reconstruction from a deep
 * buffer of space-time samples (Dayal, Woolley, Watson, Luebke: "Adaptive Frameless Rendering").
 *
 * TEST INFRASTRUCTURE. This file is the checker, not the product: only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it. It shares no code, header, table or constant
 * generator with the GPU library, and the GPU library never calls it.
 *
 * Everything is double precision, single-threaded, with no blocking, fusion or reordering beyond
 * what each definition states. Where the paper is silent or garbled, the reading used is stated at
 * the function that needs it.
 *
 * Layouts (all row-major, C order):
 *   slot planes  [H][W][K]   slot 0 is the newest sample of a pixel, count[p] slots are filled
 *   count        [H][W]      uint8
 *   src          [H][W][K]   stream index of the sample in each slot, -1 when empty
 *   stats        [OR_NSTAT][Ty][Tx]   per statistics tile
 *   rgb          [3][H][W],  aux [2][H][W] = (E_max, W')
 *
 * Parity status: every function here is pinned by the tests listed in its comment, except where a
 * comment says "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads: the per-row (or per-tile-row) loops below run under OpenMP when the file is built with
 * -fopenmp. Every output element is computed by one thread in the same operation order as with a
 * single thread, so results do not depend on the thread count. */
#ifdef _OPENMP
#include <omp.h>
#endif

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

enum {
    OR_GX = 0, OR_GY, OR_GT, OR_VOL, OR_VAR, OR_LMEAN, OR_EX2, OR_EY2, OR_SX2, OR_SY2, OR_KT2,
    OR_NSTAT
};

typedef struct {
    double sigma;     /* spatial width scale (not in the paper; scales e_x, e_y)              */
    double tau;       /* temporal sensitivity (not in the paper; scales G_t)                  */
    double alpha;     /* age-weight rate per ms: exp(-alpha * age), Sec. 4 (3.47 per second)  */
    double e_min;     /* smooth lower clamp of the spatial std, px                            */
    double e_max;     /* smooth upper clamp scale of the spatial std, px (INFINITY = none)    */
    double g_floor;   /* quadrature floor of spatial gradients, 1/px                          */
    double dt_floor;  /* floor of the new/old age separation, ms                              */
    double age_floor; /* floor of the mean tile age in the density estimate, ms               */
    double t_now;     /* reconstruction time, ms                                              */
    int radius;       /* gather radius R: Chebyshev block of (2R+1)^2 pixels                  */
    int tile;         /* statistics tile edge B_g, px                                         */
} or_params;

typedef struct {
    int width, height, k, fp16;
    double t_ref;                    /* stream reference time (float32-representable), ms     */
    double *ox, *oy, *ta, *r, *g, *b; /* [H][W][K]; ta = t (FP32 mode) or age_ref (FP16 mode) */
    uint8_t *count;                  /* [H][W] */
    int32_t *src;                    /* [H][W][K] */
} or_buffer;

/* ------------------------------------------------------------------------------------------------
 * IEEE 754 binary16 round-to-nearest-even, written from the format's definition: 11 significant
 * bits, normal exponents -14..15, subnormal quantum 2^-24, largest finite 65504. The input is scaled
 * by the binary16 quantum of its binade (an exact power-of-two scaling), rounded to an integer with
 * ties to even, and scaled back. Pinned against NumPy's float32 -> float16 conversion.
 * --------------------------------------------------------------------------------------------- */
double or_f16_round(double v)
{
    if (isnan(v) || isinf(v) || v == 0.0)
        return v;
    double a = fabs(v);
    int e;
    frexp(a, &e);                 /* a = f * 2^e with f in [0.5, 1): binade exponent is e - 1 */
    int q = (e - 1) - 10;         /* quantum exponent for 11 significant bits                   */
    if (q < -24)
        q = -24;                  /* subnormal range: fixed quantum 2^-24                       */
    double m = nearbyint(ldexp(a, -q)); /* default rounding mode: nearest, ties to even          */
    double r = ldexp(m, q);
    if (r > 65504.0)
        r = INFINITY;
    return copysign(r, v);
}

/* ------------------------------------------------------------------------------------------------
 * Build the per-pixel deep buffer (Sec. 4: each pixel holds a queue; a new sample enters at the
 * front and, when the queue is full, the sample at the back leaves; Sec. 5.2: the reconstructor's
 * samples arrive as one time-ordered stream).
 *
 * Valid samples: all six fields finite, 0 <= x < W, 0 <= y < H, t <= t_ref; in FP16 mode the
 * rounded age and colours must also be finite. Others are dropped and counted.
 * Arrival order is ascending (t, stream index): a later sample with an equal time counts as newer.
 * Stored per slot: ox = x - floor(x), oy = y - floor(y), ta = t (FP32 mode) or
 * age_ref = f16(fp32(t_ref - t)) (FP16 mode), and the colour (rounded to binary16 in FP16 mode).
 *
 * This replays the queue insertion literally. Pinned against a sort-and-take-top-K brute force and
 * against the counting invariants (count = min(K, arrivals); K >= occupancy keeps every sample).
 *
 * Reprojection (Sec. 6.2: the reconstructor redraws its samples for the current view; here with the
 * optional per-sample velocity of Sec. 4, taken in image space). When vx, vy are given, a sample's
 * position is advanced to the buffer's reference time before everything above:
 *   x' = x + vx * (t_ref - t), y' = y + vy * (t_ref - t)
 * in binary32 with three separate roundings (subtraction, product, sum; no fused multiply-add), so
 * the home pixel is an exact function of the stored inputs. Validity and the stored offsets use
 * x', y'. Pinned by: zero velocity equals the plain build; a sample displaced by whole pixels lands
 * on the expected pixel with unchanged offsets; samples moved outside the image are dropped.
 * --------------------------------------------------------------------------------------------- */
typedef struct { float t; int64_t i; } or_key;

static int or_key_cmp(const void *pa, const void *pb)
{
    const or_key *a = (const or_key *)pa, *b = (const or_key *)pb;
    if (a->t < b->t) return -1;
    if (a->t > b->t) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

int or_build(int64_t n, const float *x_in, const float *y_in, const float *t, const float *r,
             const float *g, const float *b, const float *vx, const float *vy, or_buffer *out,
             int64_t *dropped)
{
    const int W = out->width, H = out->height, K = out->k;
    if (W <= 0 || H <= 0 || K < 1 || K > 255 || n < 0)
        return 1;
    const size_t HW = (size_t)W * H, HWK = HW * K;
    const float t_ref = (float)out->t_ref;
#pragma omp parallel for schedule(static)
    for (size_t s = 0; s < HWK; ++s) {
        out->ox[s] = out->oy[s] = out->ta[s] = out->r[s] = out->g[s] = out->b[s] = 0.0;
        out->src[s] = -1;
    }
    memset(out->count, 0, HW);

    or_key *keys = (or_key *)malloc(sizeof(or_key) * (size_t)(n > 0 ? n : 1));
    if (!keys)
        return 4;
    /* positions at the reference time (reprojection), or the stored positions */
    const float *x = x_in, *y = y_in;
    float *xa = NULL, *ya = NULL;
    if (vx && vy && n > 0) {
        xa = (float *)malloc(sizeof(float) * (size_t)n);
        ya = (float *)malloc(sizeof(float) * (size_t)n);
        if (!xa || !ya) {
            free(keys);
            free(xa);
            free(ya);
            return 4;
        }
        for (int64_t i = 0; i < n; ++i) {
            volatile float d = t_ref - t[i];     /* each operation rounded on its own */
            volatile float px = vx[i] * d, py = vy[i] * d;
            xa[i] = x_in[i] + px;
            ya[i] = y_in[i] + py;
        }
        x = xa;
        y = ya;
    }
    /* which samples are kept: decided per sample (in parallel), then collected in stream order */
    unsigned char *keep = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
    if (!keep) {
        free(keys);
        free(xa);
        free(ya);
        return 4;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int ok = isfinite(x[i]) && isfinite(y[i]) && isfinite(t[i]) && isfinite(r[i]) &&
                 isfinite(g[i]) && isfinite(b[i]);
        ok = ok && x[i] >= 0.0f && x[i] < (float)W && y[i] >= 0.0f && y[i] < (float)H;
        ok = ok && t[i] <= t_ref;
        if (ok && out->fp16) {
            float age = t_ref - t[i];
            ok = isfinite(or_f16_round(age)) && isfinite(or_f16_round(r[i])) &&
                 isfinite(or_f16_round(g[i])) && isfinite(or_f16_round(b[i]));
        }
        keep[i] = (unsigned char)ok;
    }
    int64_t nv = 0, nd = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (keep[i]) {
            keys[nv].t = t[i];
            keys[nv].i = i;
            ++nv;
        } else {
            ++nd;
        }
    }
    free(keep);
    qsort(keys, (size_t)nv, sizeof(or_key), or_key_cmp);

    /* Queues of different pixels are independent: each thread takes a band of rows and inserts,
     * in sorted order, the samples that land in it. */
#pragma omp parallel
    {
#ifdef _OPENMP
    const int nth = omp_get_num_threads(), th = omp_get_thread_num();
#else
    const int nth = 1, th = 0;
#endif
    const int row0 = (int)((int64_t)H * th / nth), row1 = (int)((int64_t)H * (th + 1) / nth);
    for (int64_t a = 0; a < nv; ++a) {
        const int64_t i = keys[a].i;
        const double fx = floor((double)x[i]), fy = floor((double)y[i]);
        if (fy < row0 || fy >= row1)
            continue;
        const size_t p = (size_t)fy * W + (size_t)fx;
        const size_t base = p * K;
        int c = out->count[p];
        int last = c < K ? c : K - 1;         /* the back sample leaves when the queue is full */
        for (int k = last; k >= 1; --k) {
            out->ox[base + k] = out->ox[base + k - 1];
            out->oy[base + k] = out->oy[base + k - 1];
            out->ta[base + k] = out->ta[base + k - 1];
            out->r[base + k] = out->r[base + k - 1];
            out->g[base + k] = out->g[base + k - 1];
            out->b[base + k] = out->b[base + k - 1];
            out->src[base + k] = out->src[base + k - 1];
        }
        double vox = (double)x[i] - fx, voy = (double)y[i] - fy;
        if (out->fp16) {
            float age = t_ref - t[i];             /* binary32 subtraction, then binary16 */
            out->ox[base] = or_f16_round(vox);
            out->oy[base] = or_f16_round(voy);
            out->ta[base] = or_f16_round((double)age);
            out->r[base] = or_f16_round(r[i]);
            out->g[base] = or_f16_round(g[i]);
            out->b[base] = or_f16_round(b[i]);
        } else {
            out->ox[base] = vox;
            out->oy[base] = voy;
            out->ta[base] = (double)t[i];
            out->r[base] = r[i];
            out->g[base] = g[i];
            out->b[base] = b[i];
        }
        out->src[base] = (int32_t)i;
        out->count[p] = (uint8_t)(c < K ? c + 1 : K);
    }
    }
    free(keys);
    free(xa);
    free(ya);
    if (dropped)
        *dropped = nd;
    return 0;
}

/* Age of a slot at the reconstruction time. FP32 mode stores the time itself; FP16 mode stores the
 * age relative to t_ref, so the age at t_now adds (t_now - t_ref). */
static double slot_age(const or_buffer *buf, const or_params *p, size_t s)
{
    return buf->fp16 ? (p->t_now - buf->t_ref) + buf->ta[s] : p->t_now - buf->ta[s];
}

/* Luminance of linear RGB. The paper says only "luminance" (Sec. 4); the Rec. 709 weights are the
 * reading used here. */
static double luminance(double r, double g, double b)
{
    return 0.2126 * r + 0.7152 * g + 0.0722 * b;
}

/* ------------------------------------------------------------------------------------------------
 * Per-pixel statistics and gradients (Sec. 4 variance weights, Sec. 4.1 crosshair gradients).
 *
 *   omega = exp(-alpha * age)                       age weight, Sec. 4 (e^{-3.47 a})
 *   Omega_p = sum omega,  Lbar_p = sum omega L / Omega_p           (n_p >= 1)
 *   Temporal gradient (n_p >= 2): slots ranked newest first are split at h = ceil(n_p / 2) into a
 *   "new" half (rank < h) and an "old" half; with unweighted means of L and age over each half,
 *       G_t(p) = |L_new - L_old| / max(a_old - a_new, dt_floor).
 *   This is the crosshair's |L(t) - L(t0)| / (t - t0) of Sec. 4.1 with "same sub-pixel spot"
 *   relaxed to "same pixel", since scattered samples have no collocated pairs (a reading).
 *   Spatial gradient: G_x(p) is the mean of |Lbar_p - Lbar_q| over q = p -/+ x_hat inside the image
 *   with n_q >= 1 (the crosshair's average of one-sided differences at 1 px spacing); G_y alike.
 *
 * Undefined values are written as NaN. Pinned by closed forms: linear luminance ramps give the
 * ramp slopes, L = c t at fixed positions gives |c|, constant colour gives zero.
 * --------------------------------------------------------------------------------------------- */
int or_pixel_stats(const or_buffer *buf, const or_params *p, double *lbar, double *omega,
                   double *gx, double *gy, double *gt)
{
    const int W = buf->width, H = buf->height, K = buf->k;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t px = (size_t)j * W + i;
            const int n = buf->count[px];
            lbar[px] = omega[px] = gt[px] = NAN;
            if (n == 0)
                continue;
            double sw = 0.0, swl = 0.0;
            for (int k = 0; k < n; ++k) {
                const size_t s = px * K + k;
                const double L = luminance(buf->r[s], buf->g[s], buf->b[s]);
                const double w = exp(-p->alpha * slot_age(buf, p, s));
                sw += w;
                swl += w * L;
            }
            omega[px] = sw;
            lbar[px] = swl / sw;
            if (n >= 2) {
                const int h = (n + 1) / 2;
                double ln = 0.0, lo = 0.0, an = 0.0, ao = 0.0;
                for (int k = 0; k < n; ++k) {
                    const size_t s = px * K + k;
                    const double L = luminance(buf->r[s], buf->g[s], buf->b[s]);
                    const double a = slot_age(buf, p, s);
                    if (k < h) { ln += L; an += a; }
                    else       { lo += L; ao += a; }
                }
                ln /= h; an /= h;
                lo /= (n - h); ao /= (n - h);
                gt[px] = fabs(ln - lo) / fmax(ao - an, p->dt_floor);
            }
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t px = (size_t)j * W + i;
            gx[px] = gy[px] = NAN;
            if (buf->count[px] == 0)
                continue;
            double sx = 0.0, sy = 0.0;
            int nx = 0, ny = 0;
            if (i > 0 && buf->count[px - 1] > 0)     { sx += fabs(lbar[px] - lbar[px - 1]); ++nx; }
            if (i + 1 < W && buf->count[px + 1] > 0) { sx += fabs(lbar[px] - lbar[px + 1]); ++nx; }
            if (j > 0 && buf->count[px - W] > 0)     { sy += fabs(lbar[px] - lbar[px - W]); ++ny; }
            if (j + 1 < H && buf->count[px + W] > 0) { sy += fabs(lbar[px] - lbar[px + W]); ++ny; }
            if (nx) gx[px] = sx / nx;
            if (ny) gy[px] = sy / ny;
        }
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Filter extents from gradients and sample volume (Sec. 5.1):
 *   e_x G_x = e_y G_y = e_t G_t  and  e_x e_y e_t = V  give
 *   e_x = cbrt(V G_y G_t / G_x^2), e_y = cbrt(V G_x G_t / G_y^2), e_t = cbrt(V G_x G_y / G_t^2).
 * (The printed volume equation names e_z; it is read as e_t.) Here G_t is scaled by tau, spatial
 * gradients get a quadrature floor, and the temporal Gaussian is written with k_t = 1 / e_t:
 *   ex2 = e_x^2, ey2 = e_y^2, kt2 = 1 / e_t^2 = cbrt(u^2 / (V Gx Gy))^2 with u = tau G_t.
 * When u == 0 (static content) the limit is ex2 = ey2 = kt2 = 0: every age weighs the same and the
 * spatial width sits at its floor. Spatial stds get a smooth clamp,
 *   sx2 = e_min^2 + z e_max^2 / (e_max^2 + z),  z = sigma^2 ex2   (sx2 = e_min^2 + z if e_max = inf),
 * which is C-infinity in sigma and tau. Extents are standard deviations with support constant 1
 * (the paper says "proportional"; a reading). A tile with a temporal gradient but no buffered
 * samples (V = +inf, u > 0: crosshair gradients over an empty tile) takes the formula's limit as V
 * grows: ex2 = ey2 = +inf, so the clamped width is its ceiling e_min^2 + e_max^2 (+inf without a
 * clamp), and kt2 = 0 (a reading; the paper does not treat the case). Estimates need g_floor > 0:
 * with a zero floor a flat tile divides by a zero gradient. Pinned by the paper's own constraints
 * in a test mode (g_floor = e_min = 0, e_max = inf, sigma = tau = 1), by unit covariance and by the
 * large-V limit.
 * --------------------------------------------------------------------------------------------- */
void or_extents(double gx, double gy, double gt, double vol, const or_params *p, double *out5)
{
    const double hx = sqrt(gx * gx + p->g_floor * p->g_floor);
    const double hy = sqrt(gy * gy + p->g_floor * p->g_floor);
    const double u = p->tau * gt;
    double ex2 = 0.0, ey2 = 0.0, kt2 = 0.0;
    if (u != 0.0) {
        const double cx = cbrt(vol * hy * u / (hx * hx));
        const double cy = cbrt(vol * hx * u / (hy * hy));
        const double ck = cbrt(u * u / (vol * hx * hy));
        ex2 = cx * cx;
        ey2 = cy * cy;
        kt2 = ck * ck;
    }
    const double zx = p->sigma * p->sigma * ex2, zy = p->sigma * p->sigma * ey2;
    const double em2 = p->e_max * p->e_max, en2 = p->e_min * p->e_min;
    double sx2, sy2;
    if (isinf(p->e_max)) {
        sx2 = en2 + zx;
        sy2 = en2 + zy;
    } else {
        sx2 = en2 + (isinf(zx) ? em2 : zx * em2 / (em2 + zx));
        sy2 = en2 + (isinf(zy) ? em2 : zy * em2 / (em2 + zy));
    }
    out5[0] = ex2;
    out5[1] = ey2;
    out5[2] = sx2;
    out5[3] = sy2;
    out5[4] = kt2;
}

/* ------------------------------------------------------------------------------------------------
 * Per-tile statistics (Sec. 4 tile variation, Sec. 4.1 age-weighted gradient averaging, Sec. 5.1
 * sample volume). Tiles are fixed B_g x B_g squares (the paper's adaptive K-D tiles belong to its
 * sampler; a reading), clipped at the image border.
 *   G_*(T) = sum Omega_p G_*(p) / sum Omega_p over the tile pixels where G_*(p) is defined, else 0.
 *   n_T = total slots, abar_T = mean slot age, R_l = n_T / (A_T * 2 max(abar_T, age_floor)) in
 *   samples per px^2 ms (for uniform arrival over a span D, 2 abar = D), V = 1 / R_l; an empty tile
 *   has V = +inf (it has no defined gradient, so its extents are the u == 0 limit anyway).
 *   L_m = sum omega L / sum omega and v_T = sum omega (L - L_m)^2 / sum omega over the tile's
 *   slots, computed in two passes.
 * Pinned by closed forms: age grids give V, two-valued luminance gives v_T, ramps give gradients.
 * --------------------------------------------------------------------------------------------- */
int or_estimate(const or_buffer *buf, const or_params *p, double *stats)
{
    const int W = buf->width, H = buf->height, K = buf->k, B = p->tile;
    if (B < 1 || W < 1 || H < 1 || !(p->g_floor > 0.0))
        return 1;
    const int Tx = (W + B - 1) / B, Ty = (H + B - 1) / B;
    const size_t HW = (size_t)W * H, NT = (size_t)Tx * Ty;
    double *lbar = (double *)malloc(sizeof(double) * HW * 5);
    if (!lbar)
        return 4;
    double *omega = lbar + HW, *gx = lbar + 2 * HW, *gy = lbar + 3 * HW, *gt = lbar + 4 * HW;
    or_pixel_stats(buf, p, lbar, omega, gx, gy, gt);

#pragma omp parallel for schedule(dynamic, 1)
    for (int ty = 0; ty < Ty; ++ty)
        for (int tx = 0; tx < Tx; ++tx) {
            const size_t T = (size_t)ty * Tx + tx;
            const int i0 = tx * B, i1 = (tx + 1) * B < W ? (tx + 1) * B : W;
            const int j0 = ty * B, j1 = (ty + 1) * B < H ? (ty + 1) * B : H;
            double num[3] = {0, 0, 0}, den[3] = {0, 0, 0};
            double n_t = 0.0, sum_age = 0.0, sw = 0.0, swl = 0.0;
            for (int j = j0; j < j1; ++j)
                for (int i = i0; i < i1; ++i) {
                    const size_t px = (size_t)j * W + i;
                    const double *gp[3] = {gx, gy, gt};
                    for (int c = 0; c < 3; ++c)
                        if (!isnan(gp[c][px])) {
                            num[c] += omega[px] * gp[c][px];
                            den[c] += omega[px];
                        }
                    for (int k = 0; k < buf->count[px]; ++k) {
                        const size_t s = px * K + k;
                        const double a = slot_age(buf, p, s);
                        const double L = luminance(buf->r[s], buf->g[s], buf->b[s]);
                        const double w = exp(-p->alpha * a);
                        n_t += 1.0;
                        sum_age += a;
                        sw += w;
                        swl += w * L;
                    }
                }
            double lm = 0.0, var = 0.0;
            if (n_t > 0.0) {
                lm = swl / sw;
                double acc = 0.0;
                for (int j = j0; j < j1; ++j)
                    for (int i = i0; i < i1; ++i) {
                        const size_t px = (size_t)j * W + i;
                        for (int k = 0; k < buf->count[px]; ++k) {
                            const size_t s = px * K + k;
                            const double L = luminance(buf->r[s], buf->g[s], buf->b[s]);
                            const double w = exp(-p->alpha * slot_age(buf, p, s));
                            acc += w * (L - lm) * (L - lm);
                        }
                    }
                var = acc / sw;
            }
            const double area = (double)(i1 - i0) * (j1 - j0);
            double vol = INFINITY;
            if (n_t > 0.0) {
                const double abar = sum_age / n_t;
                const double rate = n_t / (area * 2.0 * fmax(abar, p->age_floor));
                vol = 1.0 / rate;
            }
            double g3[3];
            for (int c = 0; c < 3; ++c)
                g3[c] = den[c] > 0.0 ? num[c] / den[c] : 0.0;
            double e5[5];
            or_extents(g3[0], g3[1], g3[2], vol, p, e5);
            stats[OR_GX * NT + T] = g3[0];
            stats[OR_GY * NT + T] = g3[1];
            stats[OR_GT * NT + T] = g3[2];
            stats[OR_VOL * NT + T] = vol;
            stats[OR_VAR * NT + T] = var;
            stats[OR_LMEAN * NT + T] = lm;
            stats[OR_EX2 * NT + T] = e5[0];
            stats[OR_EY2 * NT + T] = e5[1];
            stats[OR_SX2 * NT + T] = e5[2];
            stats[OR_SY2 * NT + T] = e5[3];
            stats[OR_KT2 * NT + T] = e5[4];
        }
    free(lbar);
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Crosshair gradients (Sec. 4.1). A crosshair is a centre sample at (x, y, t), four samples taken at
 * the same instant one pixel away, (x -/+ 1, y, t) and (x, y -/+ 1, t), and an earlier sample taken
 * at the same sub-pixel spot, (x, y, t0). Each is given here as an index into the sample stream
 * (-1 or any index outside the stream: absent). With L the luminance of a sample:
 *   horizontal gradient  the mean of |L_c - L_n| over the present horizontal neighbours n (the
 *                        paper's |L - L_{x+-1}| / 2 read as the average of the two one-sided
 *                        differences, as for the scattered estimator); likewise vertical;
 *   temporal gradient    |L_c - L_old| / max(t - t0, dt_floor), defined when t0 < t.
 * A neighbour or old sample whose luminance is not finite counts as absent; an undefined gradient
 * is written as -1 (every defined one is >= 0). A crosshair whose centre is absent or has a
 * non-finite luminance gets a NaN position, so that the queue build drops it.
 *
 * Each record carries the centre's position and time; the sampler pushes it into the per-pixel
 * queue of its deep buffer (Sec. 4.1), which or_build models with the gradients in the colour
 * fields. Pinned by: a static luminance ramp gives the ramp slopes and a zero temporal gradient;
 * L = c t at a fixed spot gives |c|; missing neighbours and a later "old" sample are skipped.
 * --------------------------------------------------------------------------------------------- */
static int or_index_ok(int32_t i, int64_t n) { return i >= 0 && (int64_t)i < n; }

int or_crosshair_records(int64_t ns, const float *x, const float *y, const float *t, const float *r,
                         const float *g, const float *b, int64_t nx, const int32_t *centre,
                         const int32_t *xm, const int32_t *xp, const int32_t *ym,
                         const int32_t *yp, const int32_t *old, double dt_floor, float *cx,
                         float *cy, float *ct, double *gx, double *gy, double *gt)
{
    for (int64_t i = 0; i < nx; ++i) {
        const int32_t c = centre[i];
        gx[i] = gy[i] = gt[i] = -1.0;
        double Lc = NAN;
        if (or_index_ok(c, ns))
            Lc = luminance(r[c], g[c], b[c]);
        if (!isfinite(Lc)) {
            cx[i] = cy[i] = ct[i] = NAN;
            continue;
        }
        cx[i] = x[c];
        cy[i] = y[c];
        ct[i] = t[c];
        const int32_t *hn[2] = {xm, xp}, *vn[2] = {ym, yp};
        double sum = 0.0;
        int cnt = 0;
        for (int q = 0; q < 2; ++q) {
            const int32_t j = hn[q][i];
            if (!or_index_ok(j, ns))
                continue;
            const double L = luminance(r[j], g[j], b[j]);
            if (isfinite(L)) { sum += fabs(Lc - L); ++cnt; }
        }
        if (cnt)
            gx[i] = sum / cnt;
        sum = 0.0;
        cnt = 0;
        for (int q = 0; q < 2; ++q) {
            const int32_t j = vn[q][i];
            if (!or_index_ok(j, ns))
                continue;
            const double L = luminance(r[j], g[j], b[j]);
            if (isfinite(L)) { sum += fabs(Lc - L); ++cnt; }
        }
        if (cnt)
            gy[i] = sum / cnt;
        const int32_t o = old[i];
        if (or_index_ok(o, ns)) {
            const double L0 = luminance(r[o], g[o], b[o]);
            const double t1 = t[c], t0 = t[o];
            if (isfinite(L0) && isfinite(t0) && isfinite(t1) && t0 < t1)
                gt[i] = fabs(Lc - L0) / fmax(t1 - t0, dt_floor);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Tile gradients from a crosshair queue buffer (Sec. 4.1: sample gradients are averaged with the
 * same age weights as the colour variation of Sec. 4). xbuf holds, per pixel, the newest crosshair
 * records (FP32 mode: ta is the crosshair time, r/g/b its three gradients, -1 where undefined).
 *   G_*(T) = sum omega g / sum omega over the tile's records with a defined g, else 0,
 *   omega = exp(-alpha (t_now - t)).
 * The volume, variance and mean luminance planes of `stats` (from the sample buffer) are kept; the
 * three gradient planes are replaced and the extents recomputed from them and stats' volume.
 * Pinned by closed forms on constructed queues (equal gradients give that gradient for any ages,
 * two records give the exp-weighted mean, undefined records are skipped).
 * --------------------------------------------------------------------------------------------- */
int or_crosshair_tiles(const or_buffer *xbuf, const or_params *p, double *stats)
{
    const int W = xbuf->width, H = xbuf->height, K = xbuf->k, B = p->tile;
    if (B < 1 || W < 1 || H < 1 || xbuf->fp16 || !(p->g_floor > 0.0))
        return 1;
    const int Tx = (W + B - 1) / B, Ty = (H + B - 1) / B;
    const size_t NT = (size_t)Tx * Ty;
#pragma omp parallel for schedule(dynamic, 1)
    for (int ty = 0; ty < Ty; ++ty)
        for (int tx = 0; tx < Tx; ++tx) {
            const size_t T = (size_t)ty * Tx + tx;
            const int i0 = tx * B, i1 = (tx + 1) * B < W ? (tx + 1) * B : W;
            const int j0 = ty * B, j1 = (ty + 1) * B < H ? (ty + 1) * B : H;
            double num[3] = {0, 0, 0}, den[3] = {0, 0, 0};
            for (int j = j0; j < j1; ++j)
                for (int i = i0; i < i1; ++i) {
                    const size_t px = (size_t)j * W + i;
                    for (int k = 0; k < xbuf->count[px]; ++k) {
                        const size_t s = px * K + k;
                        const double w = exp(-p->alpha * (p->t_now - xbuf->ta[s]));
                        const double gv[3] = {xbuf->r[s], xbuf->g[s], xbuf->b[s]};
                        for (int c = 0; c < 3; ++c)
                            if (gv[c] >= 0.0) {
                                num[c] += w * gv[c];
                                den[c] += w;
                            }
                    }
                }
            double g3[3], e5[5];
            for (int c = 0; c < 3; ++c)
                g3[c] = den[c] > 0.0 ? num[c] / den[c] : 0.0;
            or_extents(g3[0], g3[1], g3[2], stats[OR_VOL * NT + T], p, e5);
            stats[OR_GX * NT + T] = g3[0];
            stats[OR_GY * NT + T] = g3[1];
            stats[OR_GT * NT + T] = g3[2];
            stats[OR_EX2 * NT + T] = e5[0];
            stats[OR_EY2 * NT + T] = e5[1];
            stats[OR_SX2 * NT + T] = e5[2];
            stats[OR_SY2 * NT + T] = e5[3];
            stats[OR_KT2 * NT + T] = e5[4];
        }
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Gather reconstruction (Sec. 5.2: per pixel, the normalised weighted average of nearby samples;
 * Sec. 5.1: Gaussian filter, axis-aligned in x, y and t, shaped per tile).
 * For pixel p = (i, j) in tile T, every filled slot s of every pixel q with |q_x - i| <= R and
 * |q_y - j| <= R inside the image contributes with exponent
 *   E_s = -1/2 (dx^2 / sx2 + dy^2 / sy2 + a^2 kt2),
 *   dx = (q_x + ox) - (i + 1/2),  dy = (q_y + oy) - (j + 1/2),  a = slot age at t_now,
 * using T's sx2, sy2, kt2 (the temporal Gaussian is one-sided in age, centred at t_now, since all
 * samples lie in the past). C_p = sum exp(E_s - E_max) c_s / W',  W' = sum exp(E_s - E_max); the
 * shift by E_max = max_s E_s only keeps the terms representable: C_p = sum w c / sum w.
 * A block with no slots gives C_p = 0, E_max = 0, W' = 0. Support truncation is the integer block
 * (the paper's epsilon cut-off / splat size is replaced by a fixed radius; a reading).
 * Pinned by: constant colour, convexity, tau = 0 against an independent spatial Gaussian gather,
 * one-sample blocks, newest-sample limit (traditional frameless, Sec. 5), linearity, mirror and
 * shift covariance, hand-computed tiny cases.
 * --------------------------------------------------------------------------------------------- */
static int block_bounds(int c, int R, int N, int *lo, int *hi)
{
    *lo = c - R < 0 ? 0 : c - R;
    *hi = c + R > N - 1 ? N - 1 : c + R;
    return *hi >= *lo;
}

int or_reconstruct(const or_buffer *buf, const double *stats, const or_params *p, double *rgb,
                   double *aux)
{
    const int W = buf->width, H = buf->height, K = buf->k, B = p->tile, R = p->radius;
    if (B < 1 || R < 0)
        return 1;
    const int Tx = (W + B - 1) / B, Ty = (H + B - 1) / B;
    const size_t HW = (size_t)W * H, NT = (size_t)Tx * Ty;
    for (size_t T = 0; T < NT; ++T)
        if (!(stats[OR_SX2 * NT + T] > 0.0) || !(stats[OR_SY2 * NT + T] > 0.0) ||
            !(stats[OR_KT2 * NT + T] >= 0.0))
            return 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t px = (size_t)j * W + i;
            const size_t T = (size_t)(j / B) * Tx + (i / B);
            const double sx2 = stats[OR_SX2 * NT + T], sy2 = stats[OR_SY2 * NT + T];
            const double kt2 = stats[OR_KT2 * NT + T];
            int qx0, qx1, qy0, qy1;
            block_bounds(i, R, W, &qx0, &qx1);
            block_bounds(j, R, H, &qy0, &qy1);
            double emax = -INFINITY;
            int any = 0;
            for (int qy = qy0; qy <= qy1; ++qy)
                for (int qx = qx0; qx <= qx1; ++qx) {
                    const size_t q = (size_t)qy * W + qx;
                    for (int k = 0; k < buf->count[q]; ++k) {
                        const size_t s = q * K + k;
                        const double dx = (qx + buf->ox[s]) - (i + 0.5);
                        const double dy = (qy + buf->oy[s]) - (j + 0.5);
                        const double a = slot_age(buf, p, s);
                        const double E = -0.5 * (dx * dx / sx2 + dy * dy / sy2 + a * a * kt2);
                        if (E > emax) emax = E;
                        any = 1;
                    }
                }
            double wsum = 0.0, cr = 0.0, cg = 0.0, cb = 0.0;
            if (any) {
                for (int qy = qy0; qy <= qy1; ++qy)
                    for (int qx = qx0; qx <= qx1; ++qx) {
                        const size_t q = (size_t)qy * W + qx;
                        for (int k = 0; k < buf->count[q]; ++k) {
                            const size_t s = q * K + k;
                            const double dx = (qx + buf->ox[s]) - (i + 0.5);
                            const double dy = (qy + buf->oy[s]) - (j + 0.5);
                            const double a = slot_age(buf, p, s);
                            const double E = -0.5 * (dx * dx / sx2 + dy * dy / sy2 + a * a * kt2);
                            const double w = exp(E - emax);
                            wsum += w;
                            cr += w * buf->r[s];
                            cg += w * buf->g[s];
                            cb += w * buf->b[s];
                        }
                    }
                rgb[px] = cr / wsum;
                rgb[HW + px] = cg / wsum;
                rgb[2 * HW + px] = cb / wsum;
                aux[px] = emax;
                aux[HW + px] = wsum;
            } else {
                rgb[px] = rgb[HW + px] = rgb[2 * HW + px] = 0.0;
                aux[px] = 0.0;
                aux[HW + px] = 0.0;
            }
        }
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Adjoint of the reconstruction (not in the paper: gradients for fitting sigma and tau).
 * With pi_s(p) = exp(E_s - E_max) / W' and g(p, ch) = dl/dC(p, ch), tile statistics held fixed:
 *   dl/dc_{s,ch} = sum_p g(p, ch) pi_s(p)
 *   dl/dtheta    = sum_p sum_ch g(p, ch) sum_s pi_s(p) (c_{s,ch} - C_{p,ch}) dE_s/dtheta
 *   dE/dtheta    = 1/2 (dx^2 dsx2/dtheta / sx2^2 + dy^2 dsy2/dtheta / sy2^2) - 1/2 a^2 dkt2/dtheta
 * From the extents: z = sigma^2 ex2, dsx2/dz = e_max^4 / (e_max^2 + z)^2 (1 without a clamp),
 * dz/dsigma = 2 sigma ex2, dz/dtau = sigma^2 (2/3) ex2 / tau, dkt2/dtau = (4/3) kt2 / tau,
 * dkt2/dsigma = 0; at the large-V limit (ex2 = +inf) the width is constant in sigma and tau, so
 * those derivatives are 0. Requires tau > 0. Everything (E, E_max, W', C) is recomputed here.
 * Pinned by FP64 central finite differences of or_reconstruct and by the adjoint identity
 * <J v, u> = <v, J^T u>.
 * --------------------------------------------------------------------------------------------- */
int or_backward(const or_buffer *buf, const double *stats, const or_params *p,
                const double *grad_rgb, double *grad_slot, double *grad_params)
{
    const int W = buf->width, H = buf->height, K = buf->k, B = p->tile, R = p->radius;
    if (B < 1 || R < 0 || !(p->tau > 0.0))
        return 1;
    const int Tx = (W + B - 1) / B, Ty = (H + B - 1) / B;
    const size_t HW = (size_t)W * H, NT = (size_t)Tx * Ty, HWK = HW * K;
    for (size_t s = 0; s < 3 * HWK; ++s)
        grad_slot[s] = 0.0;
    double g_sigma = 0.0, g_tau = 0.0;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t px = (size_t)j * W + i;
            const size_t T = (size_t)(j / B) * Tx + (i / B);
            const double sx2 = stats[OR_SX2 * NT + T], sy2 = stats[OR_SY2 * NT + T];
            const double kt2 = stats[OR_KT2 * NT + T];
            const double ex2 = stats[OR_EX2 * NT + T], ey2 = stats[OR_EY2 * NT + T];
            if (!(sx2 > 0.0) || !(sy2 > 0.0))
                return 2;
            const double zx = p->sigma * p->sigma * ex2, zy = p->sigma * p->sigma * ey2;
            double dsx_dz = 1.0, dsy_dz = 1.0;
            if (!isinf(p->e_max)) {
                const double em2 = p->e_max * p->e_max;
                dsx_dz = em2 * em2 / ((em2 + zx) * (em2 + zx));
                dsy_dz = em2 * em2 / ((em2 + zy) * (em2 + zy));
            }
            const double dsx_dsig = isinf(ex2) ? 0.0 : dsx_dz * 2.0 * p->sigma * ex2;
            const double dsy_dsig = isinf(ey2) ? 0.0 : dsy_dz * 2.0 * p->sigma * ey2;
            const double dsx_dtau =
                isinf(ex2) ? 0.0 : dsx_dz * p->sigma * p->sigma * (2.0 / 3.0) * ex2 / p->tau;
            const double dsy_dtau =
                isinf(ey2) ? 0.0 : dsy_dz * p->sigma * p->sigma * (2.0 / 3.0) * ey2 / p->tau;
            const double dkt_dtau = (4.0 / 3.0) * kt2 / p->tau;

            int qx0, qx1, qy0, qy1;
            block_bounds(i, R, W, &qx0, &qx1);
            block_bounds(j, R, H, &qy0, &qy1);
            double emax = -INFINITY;
            int any = 0;
            for (int qy = qy0; qy <= qy1; ++qy)
                for (int qx = qx0; qx <= qx1; ++qx) {
                    const size_t q = (size_t)qy * W + qx;
                    for (int k = 0; k < buf->count[q]; ++k) {
                        const size_t s = q * K + k;
                        const double dx = (qx + buf->ox[s]) - (i + 0.5);
                        const double dy = (qy + buf->oy[s]) - (j + 0.5);
                        const double a = slot_age(buf, p, s);
                        const double E = -0.5 * (dx * dx / sx2 + dy * dy / sy2 + a * a * kt2);
                        if (E > emax) emax = E;
                        any = 1;
                    }
                }
            if (!any)
                continue;
            double wsum = 0.0, C[3] = {0, 0, 0};
            for (int qy = qy0; qy <= qy1; ++qy)
                for (int qx = qx0; qx <= qx1; ++qx) {
                    const size_t q = (size_t)qy * W + qx;
                    for (int k = 0; k < buf->count[q]; ++k) {
                        const size_t s = q * K + k;
                        const double dx = (qx + buf->ox[s]) - (i + 0.5);
                        const double dy = (qy + buf->oy[s]) - (j + 0.5);
                        const double a = slot_age(buf, p, s);
                        const double E = -0.5 * (dx * dx / sx2 + dy * dy / sy2 + a * a * kt2);
                        const double w = exp(E - emax);
                        wsum += w;
                        C[0] += w * buf->r[s];
                        C[1] += w * buf->g[s];
                        C[2] += w * buf->b[s];
                    }
                }
            for (int c = 0; c < 3; ++c)
                C[c] /= wsum;
            const double g0 = grad_rgb[px], g1 = grad_rgb[HW + px], g2 = grad_rgb[2 * HW + px];
            for (int qy = qy0; qy <= qy1; ++qy)
                for (int qx = qx0; qx <= qx1; ++qx) {
                    const size_t q = (size_t)qy * W + qx;
                    for (int k = 0; k < buf->count[q]; ++k) {
                        const size_t s = q * K + k;
                        const double dx = (qx + buf->ox[s]) - (i + 0.5);
                        const double dy = (qy + buf->oy[s]) - (j + 0.5);
                        const double a = slot_age(buf, p, s);
                        const double E = -0.5 * (dx * dx / sx2 + dy * dy / sy2 + a * a * kt2);
                        const double pi = exp(E - emax) / wsum;
                        grad_slot[s] += g0 * pi;
                        grad_slot[HWK + s] += g1 * pi;
                        grad_slot[2 * HWK + s] += g2 * pi;
                        const double h = g0 * (buf->r[s] - C[0]) + g1 * (buf->g[s] - C[1]) +
                                         g2 * (buf->b[s] - C[2]);
                        const double dsig = 0.5 * (dx * dx * dsx_dsig / (sx2 * sx2) +
                                                   dy * dy * dsy_dsig / (sy2 * sy2));
                        const double dtau = 0.5 * (dx * dx * dsx_dtau / (sx2 * sx2) +
                                                   dy * dy * dsy_dtau / (sy2 * sy2)) -
                                            0.5 * a * a * dkt_dtau;
                        g_sigma += pi * h * dsig;
                        g_tau += pi * h * dtau;
                    }
                }
        }
    grad_params[0] = g_sigma;
    grad_params[1] = g_tau;
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Scatter reconstruction (Sec. 5.2: every buffered sample is splatted onto the image and adds its
 * filter-weighted colour and its weight to each pixel its splat covers; the image is the ratio of
 * the two sums). A sample of home pixel q = (q_x, q_y) with offsets (ox, oy) and splat size
 * size[q] (Sec. 6.2: all samples of a region share the region's splat size) covers pixel p when
 *   |d_x| <= h and |d_y| <= h,  d_x = ((q_x - p_x) - 1/2) + ox,  d_y likewise,  h = min(size, max)/2
 * with d and h evaluated in binary32 (an integer decision, so it is taken in the precision of the
 * GPU form). Its exponent at p uses p's tile parameters, as the fragment program of Sec. 5.2 reads
 * the tile texture at the fragment:
 *   E = -1/2 (d_x^2 / sx2 + d_y^2 / sy2 + a^2 kt2).
 * Per pixel, C_p = sum exp(E - E_max) c / W', W' = sum exp(E - E_max), aux = (E_max, W'), as for the
 * gather; a pixel no splat covers is 0 with aux (0, 0). The coverage map records, per pixel, the
 * number n of splats that covered it and their mean size (0 if n = 0): sizes are counted in
 * units of 1/256 px (round(256 size), exact for the sizes or_splat_sizes makes), the integer sum
 * of units is exact, and the mean is (float(units) / n) / 256 in binary32.
 * The two passes (maxima, then sums) follow the splat loop over samples.
 * Pinned by: with size 2R + 1 and offsets inside (0, 1) the covered set is the gather's block and
 * the image equals or_reconstruct; a lone sample paints exactly its footprint with its colour;
 * coverage counts on regular sample grids have closed forms.
 * --------------------------------------------------------------------------------------------- */
static int or_covers(int q, int p, double o, float h, double *d)
{
    volatile float dq = (float)(q - p) - 0.5f;
    volatile float df = dq + (float)o;
    *d = df;
    return fabsf(df) <= h;
}

int or_scatter(const or_buffer *buf, const double *stats, const or_params *p, const float *size,
               float max_size, double *rgb, double *aux, float *cov_n, float *cov_size)
{
    const int W = buf->width, H = buf->height, K = buf->k, B = p->tile;
    if (B < 1 || !(max_size > 0.0f))
        return 1;
    const int Tx = (W + B - 1) / B, Ty = (H + B - 1) / B;
    const size_t HW = (size_t)W * H, NT = (size_t)Tx * Ty;
    double *emax = (double *)malloc(sizeof(double) * HW * 5);
    int64_t *units = (int64_t *)malloc(sizeof(int64_t) * HW);
    if (!emax || !units) {
        free(emax);
        free(units);
        return 4;
    }
    double *ws = emax + HW, *cr = emax + 2 * HW, *cg = emax + 3 * HW, *cb = emax + 4 * HW;
    for (size_t i = 0; i < HW; ++i) {
        emax[i] = -INFINITY;
        ws[i] = cr[i] = cg[i] = cb[i] = 0.0;
        units[i] = 0;
        cov_n[i] = 0.0f;
    }
    const int reach = (int)ceil(0.5 * max_size + 0.5) + 1;
    for (int pass = 0; pass < 2; ++pass)
        for (int qy = 0; qy < H; ++qy)
            for (int qx = 0; qx < W; ++qx) {
                const size_t q = (size_t)qy * W + qx;
                const float sz = fminf(size[q], max_size);
                volatile float h = 0.5f * sz;
                for (int k = 0; k < buf->count[q]; ++k) {
                    const size_t s = q * K + k;
                    const double a = slot_age(buf, p, s);
                    for (int py = qy - reach; py <= qy + reach; ++py) {
                        double dy;
                        if (py < 0 || py >= H || !or_covers(qy, py, buf->oy[s], h, &dy))
                            continue;
                        for (int px = qx - reach; px <= qx + reach; ++px) {
                            double dx;
                            if (px < 0 || px >= W || !or_covers(qx, px, buf->ox[s], h, &dx))
                                continue;
                            const size_t o = (size_t)py * W + px;
                            const size_t T = (size_t)(py / B) * Tx + (px / B);
                            const double sx2 = stats[OR_SX2 * NT + T];
                            const double sy2 = stats[OR_SY2 * NT + T];
                            const double kt2 = stats[OR_KT2 * NT + T];
                            /* the exponent from the exact offsets, not the binary32 test values */
                            const double ex = (qx - px - 0.5) + buf->ox[s];
                            const double ey = (qy - py - 0.5) + buf->oy[s];
                            const double E = -0.5 * (ex * ex / sx2 + ey * ey / sy2 + a * a * kt2);
                            if (pass == 0) {
                                if (E > emax[o]) emax[o] = E;
                                cov_n[o] += 1.0f;
                                units[o] += (int64_t)rintf(256.0f * sz);
                            } else {
                                const double w = exp(E - emax[o]);
                                ws[o] += w;
                                cr[o] += w * buf->r[s];
                                cg[o] += w * buf->g[s];
                                cb[o] += w * buf->b[s];
                            }
                        }
                    }
                }
            }
    for (size_t i = 0; i < HW; ++i) {
        if (cov_n[i] > 0.0f) {
            rgb[i] = cr[i] / ws[i];
            rgb[HW + i] = cg[i] / ws[i];
            rgb[2 * HW + i] = cb[i] / ws[i];
            aux[i] = emax[i];
            aux[HW + i] = ws[i];
            volatile float m = (float)units[i] / cov_n[i];
            cov_size[i] = m * 0.00390625f;
        } else {
            rgb[i] = rgb[HW + i] = rgb[2 * HW + i] = 0.0;
            aux[i] = aux[HW + i] = 0.0;
            cov_size[i] = 0.0f;
        }
    }
    free(emax);
    free(units);
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Adaptive splat size (Sec. 6.2). The splat size of pixel q for the next image is the mean size of
 * the splats that reached q in the previous image, multiplied by `grow` where fewer than n_low
 * splats reached it (undersampled: grow fast) and by `shrink` where more than n_high did
 * (oversampled: shrink gradually); with no splat at all, or no previous image, the base is
 * `size_default`. The result is clamped to [size_min, size_max] and rounded to a multiple of
 * 1/256 px (ties to even), all in binary32, so that sizes are exact and coverage sums of them too.
 * Pinned by the rule's cases (n = 0, n < n_low, n_low <= n <= n_high, n > n_high, the clamps).
 * --------------------------------------------------------------------------------------------- */
typedef struct {
    float size_default, size_min, size_max, grow, shrink;
    int n_low, n_high;
} or_splat;

void or_splat_sizes(int W, int H, const float *cov_n, const float *cov_size, const or_splat *sp,
                    float *size)
{
    for (size_t i = 0; i < (size_t)W * H; ++i) {
        volatile float v = sp->size_default;
        if (cov_n && cov_size) {
            const float n = cov_n[i];
            if (n > 0.0f)
                v = cov_size[i];
            if (n < (float)sp->n_low)
                v = v * sp->grow;
            else if (n > (float)sp->n_high)
                v = v * sp->shrink;
        }
        v = fminf(fmaxf(v, sp->size_min), sp->size_max);
        volatile float u = v * 256.0f;
        size[i] = rintf(u) * 0.00390625f;
    }
}

/* ------------------------------------------------------------------------------------------------
 * Sampler feedback statistics (Sec. 4, 4.1, 6.1). Inputs: the sampler's deep buffer (per-pixel
 * queues of depth b, Sec. 4) and its tile statistics from or_estimate (which hold the age-weighted
 * luminance variance v_T of Sec. 4 and the tile gradients of Sec. 4.1). Per tile T of s_T pixels:
 *   |T| = samples in T's block, empty_T = s_T b - |T|;
 *   mean empty per tile e = (w h b - |buffer|) / |tiles|;
 *   u_T = 1 - min(1, m e / empty_T)            (undersampling, Sec. 6.1; read with the mean empty
 *                                               count per tile in the numerator; 0 when empty_T = 0)
 *   E_T = s_T (kappa v_T / sum v + lambda u_T / sum u)   (tile error, Sec. 6.1, without the
 *                                               occlusion term, which needs occlusion rays; a term
 *                                               whose sum is 0 contributes 0)
 * Gain control (Sec. 4.1): with dC/ds the mean over tiles of (G_x + G_y) / 2, dC/dt the mean of G_t
 * and T the mean over non-empty tiles of their mean sample age, the tile width that balances
 * dC/ds S = i dC/dt T is S = i (dC/dt) T / (dC/ds), and the target tile count is w h / S^2
 * (S = 0 and +inf tiles when dC/dt = 0: static content is tiled as finely as possible; S = +inf and
 * 0 tiles when dC/ds = 0 < dC/dt).
 * glob receives: sum v, sum u, e, dC/ds, dC/dt, T, S, target tile count.
 * Pinned by hand-computed u and E on two-tile buffers, the normalisations (sum E_T / s_T over tiles
 * is kappa + lambda when both sums are positive) and a constructed gain-control case.
 * --------------------------------------------------------------------------------------------- */
typedef struct {
    double kappa, lambda, m, gain;
} or_sampler;

int or_sampler_stats(const or_buffer *buf, const double *stats, const or_params *p,
                     const or_sampler *sp, double *E, double *u, double *glob)
{
    const int W = buf->width, H = buf->height, K = buf->k, B = p->tile;
    if (B < 1)
        return 1;
    const int Tx = (W + B - 1) / B, Ty = (H + B - 1) / B;
    const size_t NT = (size_t)Tx * Ty;
    double *empty = (double *)malloc(sizeof(double) * NT);
    if (!empty)
        return 4;
    double n_all = 0.0, sum_v = 0.0, sum_gs = 0.0, sum_gt = 0.0, sum_age = 0.0, n_aged = 0.0;
    for (int ty = 0; ty < Ty; ++ty)
        for (int tx = 0; tx < Tx; ++tx) {
            const size_t T = (size_t)ty * Tx + tx;
            const int i0 = tx * B, i1 = (tx + 1) * B < W ? (tx + 1) * B : W;
            const int j0 = ty * B, j1 = (ty + 1) * B < H ? (ty + 1) * B : H;
            double n_t = 0.0, a_t = 0.0;
            for (int j = j0; j < j1; ++j)
                for (int i = i0; i < i1; ++i) {
                    const size_t px = (size_t)j * W + i;
                    for (int k = 0; k < buf->count[px]; ++k) {
                        n_t += 1.0;
                        a_t += slot_age(buf, p, px * K + k);
                    }
                }
            empty[T] = (double)(i1 - i0) * (j1 - j0) * K - n_t;
            n_all += n_t;
            if (n_t > 0.0) {
                sum_age += a_t / n_t;
                n_aged += 1.0;
            }
            sum_v += stats[OR_VAR * NT + T];
            sum_gs += 0.5 * (stats[OR_GX * NT + T] + stats[OR_GY * NT + T]);
            sum_gt += stats[OR_GT * NT + T];
        }
    const double e = ((double)W * H * K - n_all) / (double)NT;
    double sum_u = 0.0;
    for (size_t T = 0; T < NT; ++T) {
        u[T] = empty[T] > 0.0 ? 1.0 - fmin(1.0, sp->m * e / empty[T]) : 0.0;
        sum_u += u[T];
    }
    for (int ty = 0; ty < Ty; ++ty)
        for (int tx = 0; tx < Tx; ++tx) {
            const size_t T = (size_t)ty * Tx + tx;
            const int bw = (tx + 1) * B < W ? B : W - tx * B;
            const int bh = (ty + 1) * B < H ? B : H - ty * B;
            double v = 0.0;
            if (sum_v > 0.0)
                v += sp->kappa * stats[OR_VAR * NT + T] / sum_v;
            if (sum_u > 0.0)
                v += sp->lambda * u[T] / sum_u;
            E[T] = (double)bw * bh * v;
        }
    const double dcds = sum_gs / (double)NT, dcdt = sum_gt / (double)NT;
    const double tbar = n_aged > 0.0 ? sum_age / n_aged : 0.0;
    double S, target;
    if (dcdt == 0.0) { /* static content: the finest tiling */
        S = 0.0;
        target = INFINITY;
    } else if (dcds == 0.0) {
        S = INFINITY;
        target = 0.0;
    } else {
        S = sp->gain * dcdt * tbar / dcds;
        target = S > 0.0 ? (double)W * H / (S * S) : INFINITY;
    }
    const double g[8] = {sum_v, sum_u, e, dcds, dcdt, tbar, S, target};
    memcpy(glob, g, sizeof(g));
    free(empty);
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Tile selection for the next samples (Sec. 4: the sampler picks a tile at random and a uniform
 * spot inside it; with fixed tiles, a tile is picked with probability proportional to its error
 * E_T, which biases sampling as the paper's equal-error adaptive tiles do under uniform choice).
 * Integer weights make the choice exact: q_T = floor(E_T / E_max * 2^24) computed in FP64 from the
 * binary32 E_T (E_T that is negative or not finite counts as 0; when no tile is positive every q_T
 * is 1); with Q = sum q_T, draw k takes r = rnd[k] >> 8 and picks the tile T with
 * cum_T <= (r Q) >> 24 < cum_T + q_T. Its spot is x = x0 + u1 bw, y = y0 + u2 bh in binary32 with
 * u1 = (rnd[n + k] >> 8) 2^-24 and u2 = (rnd[2n + k] >> 8) 2^-24, (x0, y0) the tile corner and
 * (bw, bh) its clipped size; a spot that rounds onto the far edge is moved to the float below it.
 * At most 65536 tiles, so that r Q stays below 2^64.
 * Pinned by hand-computed draws on two tiles, frequencies on many draws and uniform E.
 * --------------------------------------------------------------------------------------------- */
int or_sampler_select(int W, int H, int B, const float *E, int64_t n, const uint32_t *rnd,
                      float *x, float *y, int32_t *tile)
{
    if (B < 1 || W < 1 || H < 1)
        return 1;
    const int Tx = (W + B - 1) / B, Ty = (H + B - 1) / B;
    const size_t NT = (size_t)Tx * Ty;
    if (NT > 65536) /* keeps r Q below 2^64 */
        return 1;
    uint64_t *cum = (uint64_t *)malloc(sizeof(uint64_t) * (NT + 1));
    if (!cum)
        return 4;
    double emax = 0.0;
    for (size_t T = 0; T < NT; ++T)
        if (isfinite(E[T]) && E[T] > emax)
            emax = E[T];
    cum[0] = 0;
    for (size_t T = 0; T < NT; ++T) {
        uint64_t q = 1;
        if (emax > 0.0)
            q = (isfinite(E[T]) && E[T] > 0.0f) ? (uint64_t)floor((double)E[T] / emax * 16777216.0)
                                                : 0;
        cum[T + 1] = cum[T] + q;
    }
    const uint64_t Q = cum[NT];
    for (int64_t k = 0; k < n; ++k) {
        const uint64_t target = ((uint64_t)(rnd[k] >> 8) * Q) >> 24;
        size_t lo = 0, hi = NT; /* the T with cum[T] <= target < cum[T + 1] */
        while (hi - lo > 1) {
            const size_t mid = (lo + hi) / 2;
            if (cum[mid] <= target) lo = mid;
            else hi = mid;
        }
        const int tx = (int)(lo % Tx), ty = (int)(lo / Tx);
        const int x0 = tx * B, y0 = ty * B;
        const int bw = x0 + B < W ? B : W - x0, bh = y0 + B < H ? B : H - y0;
        volatile float u1 = (float)(rnd[n + k] >> 8) * 5.9604644775390625e-8f;
        volatile float u2 = (float)(rnd[2 * n + k] >> 8) * 5.9604644775390625e-8f;
        volatile float ox = u1 * (float)bw, oy = u2 * (float)bh;
        volatile float xs = (float)x0 + ox, ys = (float)y0 + oy;
        const float xe = (float)(x0 + bw), ye = (float)(y0 + bh);
        x[k] = xs < xe ? xs : nextafterf(xe, 0.0f);
        y[k] = ys < ye ? ys : nextafterf(ye, 0.0f);
        if (tile)
            tile[k] = (int32_t)lo;
    }
    free(cum);
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Equal-error tiles (Sec. 4: the sampler's tiles each hold about the same colour variation and are
 * picked uniformly, so small tiles form over edges and motion; Sec. 4.1: gain control sets how many
 * tiles there are). The adaptive K-D tree itself is not built; its effect is reproduced over the
 * fixed statistics tiles: the tiles are put in Morton (Z-curve) order, the curve is cut into N
 * parts of equal error, and each part is picked with probability 1/N, a uniform spot inside it.
 * Exactly:
 *   q_T = integer error weights as in or_sampler_select, C_m = sum of q over the first m tiles on
 *   the curve, Q = C_nt; tile m starts in part p_m = min(N - 1, floor(C_m N / Q));
 *   a part that tiles start in is the run of those tiles, and spreads its 1/N over them by area;
 *   a part no tile starts in lies inside the error of the tile before it on the curve, which takes
 *   its whole 1/N.
 * The output weight of tile T (proportional to its probability; the factor 1/N is dropped) is
 *   P_T = s_T / A(run of p_T) + (number of parts strictly between p_T and the next tile's part,
 *         or up to N for the last tile),
 * in FP64 from integers, stored as float. With Q = 0 every P_T is s_T (uniform by area). N is the
 * gain-control target tile count rounded and clamped to [1, tiles], or an explicit count.
 * Pinned by: N = 1 is uniform by area; equal errors with N = tiles give every tile weight 1; a
 * single tile holding all the error takes N - 2 whole parts; the weights sum to N.
 * --------------------------------------------------------------------------------------------- */
static uint32_t or_spread_bits(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 16; ++b)
        r |= ((v >> b) & 1u) << (2 * b);
    return r;
}

typedef struct { uint32_t code; int32_t tile; } or_morton;

static int or_morton_cmp(const void *a, const void *b)
{
    const uint32_t x = ((const or_morton *)a)->code, y = ((const or_morton *)b)->code;
    return (x > y) - (x < y);
}

int or_sampler_tile_weights(int W, int H, int B, const float *E, double target, int n_override,
                            float *P)
{
    if (B < 1 || W < 1 || H < 1)
        return 1;
    const int Tx = (W + B - 1) / B, Ty = (H + B - 1) / B;
    const int NT = Tx * Ty;
    if (NT > 65536)
        return 1;
    int N = n_override;
    if (N <= 0) {
        double r = isnan(target) ? 1.0 : nearbyint(target);
        N = r < 1.0 ? 1 : (r > NT ? NT : (int)r);
    }
    if (N > NT)
        N = NT;
    or_morton *ord = (or_morton *)malloc(sizeof(or_morton) * NT);
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (NT + 1));
    int64_t *A = (int64_t *)malloc(sizeof(int64_t) * (NT + 1));
    int64_t *part = (int64_t *)malloc(sizeof(int64_t) * NT);
    if (!ord || !C || !A || !part) {
        free(ord); free(C); free(A); free(part);
        return 4;
    }
    for (int ty = 0; ty < Ty; ++ty)
        for (int tx = 0; tx < Tx; ++tx) {
            ord[ty * Tx + tx].code = or_spread_bits((uint32_t)tx) | (or_spread_bits((uint32_t)ty) << 1);
            ord[ty * Tx + tx].tile = ty * Tx + tx;
        }
    qsort(ord, NT, sizeof(or_morton), or_morton_cmp);
    double emax = 0.0;
    for (int T = 0; T < NT; ++T)
        if (isfinite(E[T]) && E[T] > emax)
            emax = E[T];
    C[0] = 0;
    A[0] = 0;
    for (int m = 0; m < NT; ++m) {
        const int T = ord[m].tile, tx = T % Tx, ty = T / Tx;
        const int bw = (tx + 1) * B < W ? B : W - tx * B, bh = (ty + 1) * B < H ? B : H - ty * B;
        uint64_t q = 0;
        if (emax > 0.0 && isfinite(E[T]) && E[T] > 0.0f)
            q = (uint64_t)floor((double)E[T] / emax * 16777216.0);
        C[m + 1] = C[m] + q;
        A[m + 1] = A[m] + (int64_t)bw * bh;
    }
    const uint64_t Q = C[NT];
    for (int m = 0; m < NT; ++m) {
        const uint64_t p = Q ? C[m] * (uint64_t)N / Q : 0;
        part[m] = p < (uint64_t)N - 1 ? (int64_t)p : N - 1;
    }
    for (int m = 0; m < NT; ++m) {
        const int T = ord[m].tile;
        const double s = (double)(A[m + 1] - A[m]);
        if (Q == 0) {
            P[T] = (float)s;
            continue;
        }
        int lo = m, hi = m + 1; /* the run of tiles starting in the same part */
        while (lo > 0 && part[lo - 1] == part[m]) --lo;
        while (hi < NT && part[hi] == part[m]) ++hi;
        const int64_t next = m + 1 < NT ? part[m + 1] : N;
        const int64_t extra = next - part[m] - 1 > 0 ? next - part[m] - 1 : 0;
        P[T] = (float)(s / (double)(A[hi] - A[lo]) + (double)extra);
    }
    free(ord); free(C); free(A); free(part);
    return 0;
}
