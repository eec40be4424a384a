/*
 * afr.h -- C ABI of libafr: temporally adaptive reconstruction of an image from a temporally deep
 * buffer of space-time samples, on AMD Instinct MI355X (gfx950).
 *
 * Method: Dayal, Woolley, Watson, Luebke, "Adaptive Frameless Rendering".
 *   - samples stream from a sampler into a reconstructor (Sec. 4.2, Sec. 5.2);
 *   - each pixel keeps a short queue of its newest samples (Sec. 4);
 *   - local colour gradients in space and time and the local sample density shape an axis-aligned
 *     Gaussian space-time filter per tile (Sec. 4.1, Sec. 5.1);
 *   - each pixel is the normalised weighted average of nearby samples (Sec. 5.2).
 *
 * Conventions shared by every call
 *   Memory      All array arguments are DEVICE pointers owned by the caller (for example PyTorch
 *               tensors); structs themselves live in host memory. The library never allocates device
 *               memory: calls that need scratch space take a caller-provided workspace whose size is
 *               given by the matching *_workspace_bytes query.
 *   Layout      Per-slot planes are [K][H][W] (row-major, slot-major: plane k holds every pixel's
 *               k-th newest sample, slot 0 is the newest). Images are planar [C][H][W]. Tile statistics
 *               are planar [AFR_NSTAT][tiles_y][tiles_x].
 *   Units       Positions in pixels (pixel (i, j) covers [i, i+1) x [j, j+1)), time in milliseconds.
 *   Streams     Every call enqueues asynchronous work on the given HIP stream (0 = null stream) and
 *               returns without synchronising. Calls are re-entrant; calls on different streams that
 *               share output or workspace memory race.
 *   Errors      Arguments are validated on the host before anything is launched: an invalid call
 *               returns AFR_E_INVALID or AFR_E_RANGE and enqueues nothing. A failed launch returns
 *               AFR_E_DEVICE. Faults inside kernels surface at the caller's next synchronisation.
 *               No C++ exception crosses this interface. Every output is fully overwritten, so a call
 *               can be re-issued after an error.
 */
#ifndef AFR_H
#define AFR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum afr_status {
    AFR_OK = 0,
    AFR_E_INVALID = 1,      /* NULL pointer, inconsistent sizes or layout                       */
    AFR_E_RANGE = 2,        /* a size or parameter outside its documented range                 */
    AFR_E_DEVICE = 3,       /* a HIP launch or runtime call failed                              */
    AFR_E_NOMEM = 4,        /* the caller's workspace is smaller than the query returned        */
    AFR_E_UNSUPPORTED = 5   /* a valid request that this library does not implement             */
} afr_status;

/* Storage precision of a deep buffer. Arithmetic is FP32 (FP64 in the statistics) either way. */
typedef enum afr_precision {
    AFR_FP32 = 0,           /* ox, oy, t, r, g, b stored as float; tage holds the time t        */
    AFR_FP16 = 1            /* stored as IEEE binary16 (round to nearest even); tage holds the   */
                            /* age relative to t_ref, age_ref = t_ref - t, so recent samples get */
                            /* the finest quantisation; slots are 12-byte records (see below)    */
} afr_precision;

/* A stream of samples (Sec. 4.2: the sampler streams every sample to the reconstructor). Device
 * SoA float32 arrays of length n: sub-pixel position (x, y), time t in ms, and linear RGB colour. The
 * order of the stream does not matter: samples are ranked by the key (t, index).
 *
 * vx, vy (optional, both or neither; NULL = no reprojection): image-space velocity in px/ms of the
 * surface each sample hit (the optional per-sample velocity of Sec. 4). When given, the build
 * reprojects (Sec. 6.2) every sample to the buffer's reference time before binning it:
 *   x' = x + vx * (t_ref - t),  y' = y + vy * (t_ref - t)
 * in binary32 with each of the subtraction, product and sum rounded on its own (no fused
 * multiply-add), and x', y' replace x, y everywhere below (home pixel, validity, stored offsets). */
typedef struct afr_samples {
    const float *x, *y, *t, *r, *g, *b;
    int64_t n;
    const float *vx, *vy;
} afr_samples;

/* Per-pixel deep buffer (Sec. 4): pixel p keeps count[p] <= K slots, newest first. For every filled
 * slot: ox = x - floor(x), oy = y - floor(y) in [0, 1], tage (see afr_precision) and the colour.
 * Empty slots hold zeros. src (optional, may be NULL) receives the stream index of each slot or -1;
 * it maps slot gradients back to stream samples.
 *
 * Slot s = k H W + y W + x (slot plane k of pixel (x, y)) is stored
 *   AFR_FP32: in six planes, field f of slot s at ((float *)f)[s];
 *   AFR_FP16: as a 12-byte record of six binary16 values in the order (ox, oy, r, g, b, age_ref),
 *             records [K][H][W] one after another starting at ox (4-byte aligned); the six field
 *             pointers address the first record's fields, so oy = ox + 1, r = ox + 2, g = ox + 3,
 *             b = ox + 4, tage = ox + 5 as binary16 pointers, and field f of slot s is at
 *             ((binary16 *)f)[6 s]. One 12-byte load fetches a whole slot; any other
 *             arrangement of the six pointers is AFR_E_INVALID. */
typedef struct afr_deep_buffer {
    int32_t width, height;  /* pixels, >= 1                                                     */
    int32_t k;              /* slots per pixel, 1..255                                           */
    int32_t precision;      /* afr_precision                                                     */
    float t_ref;            /* stream reference time: samples with t > t_ref are dropped         */
    void *ox, *oy, *tage, *r, *g, *b; /* fields, laid out as above                               */
    uint8_t *count;         /* [H][W]                                                            */
    int32_t *src;           /* [K][H][W] or NULL                                                 */
} afr_deep_buffer;

/* Per-tile statistics, planes of float [tiles_y][tiles_x] in this order. */
enum {
    AFR_STAT_GX = 0,  /* age-weighted mean horizontal luminance gradient, 1/px   (Sec. 4.1)      */
    AFR_STAT_GY,      /* age-weighted mean vertical luminance gradient, 1/px     (Sec. 4.1)      */
    AFR_STAT_GT,      /* age-weighted mean temporal luminance gradient, 1/ms     (Sec. 4.1)      */
    AFR_STAT_VOL,     /* space-time volume per sample V = 1/R_l, px^2 ms; +inf if empty (5.1)    */
    AFR_STAT_VAR,     /* age-weighted luminance variance of the tile              (Sec. 4)       */
    AFR_STAT_LMEAN,   /* age-weighted mean luminance of the tile                  (Sec. 4)       */
    AFR_STAT_EX2,     /* e_x^2 before width scaling and clamping, px^2            (Sec. 5.1)     */
    AFR_STAT_EY2,     /* e_y^2 before width scaling and clamping, px^2            (Sec. 5.1)     */
    AFR_STAT_SX2,     /* horizontal filter variance used by the gather, px^2                     */
    AFR_STAT_SY2,     /* vertical filter variance used by the gather, px^2                       */
    AFR_STAT_KT2,     /* temporal filter rate squared 1/e_t^2, 1/ms^2             (Sec. 5.1)     */
    AFR_NSTAT
};

typedef struct afr_tile_stats {
    int32_t tile;               /* tile edge B_g in px; must equal afr_params.tile               */
    int32_t tiles_x, tiles_y;   /* ceil(width / tile), ceil(height / tile)                       */
    float *data;                /* [AFR_NSTAT][tiles_y][tiles_x]                                 */
} afr_tile_stats;

/* Filter constants. Defaults in brackets. */
typedef struct afr_params {
    float sigma;       /* spatial width scale [1.0]; >= 0                                        */
    float tau;         /* temporal sensitivity, scales G_t [0.5]; >= 0 (> 0 for the backward)    */
    float alpha;       /* age-weight rate, per ms [3.47e-3]: exp(-3.47 a) with a in s (Sec. 4)   */
    float e_min;       /* spatial std floor, px [0.5]; > 0                                       */
    float e_max;       /* spatial std clamp scale, px [1.0]; > 0 or +inf                         */
    float g_floor;     /* quadrature floor of spatial gradients, 1/px [1e-3]; > 0                */
    float dt_floor;    /* floor of the new/old age separation, ms [1e-3]; > 0                    */
    float age_floor;   /* floor of the mean age in the density estimate, ms [1e-3]; > 0          */
    int32_t radius;    /* gather radius R: Chebyshev block of (2R+1)^2 pixels [2]; 0..4          */
    int32_t tile;      /* statistics tile edge B_g, px [8]; 1..16                                */
    float t_now;       /* reconstruction time, ms; >= the buffer's t_ref                         */
} afr_params;

/* Human-readable name of a status code. */
const char *afr_status_string(afr_status status);

/* Library version string. */
const char *afr_version(void);

/* ---------------------------------------------------------------------------------------------
 * Deep-buffer build (Sec. 4 per-pixel queues fed by the Sec. 4.2 / 5.2 sample stream).
 *
 * Bins every valid sample to its home pixel (floor(x), floor(y)) and keeps, per pixel, the
 * min(K, arrivals) samples with the largest key (t, stream index), newest in slot 0: the state the
 * paper's queue reaches when the stream is inserted in time order (a later sample with an equal time
 * counts as newer). A sample is valid when all six fields are finite, 0 <= x < width,
 * 0 <= y < height and t <= out->t_ref; in FP16 mode its age and colours must also round to finite
 * binary16 values. Invalid samples are dropped, not errors.
 *
 *   s            device sample stream; n < 2^31; AFR_E_INVALID if exactly one of vx, vy is NULL
 *   out          geometry, precision, t_ref and destination planes (all overwritten)
 *   ws, ws_bytes device workspace of at least afr_build_workspace_bytes(n, width, height, k) bytes
 *   dropped_dev  optional device int64: receives the number of dropped samples
 * ------------------------------------------------------------------------------------------- */
size_t afr_build_workspace_bytes(int64_t n, int32_t width, int32_t height, int32_t k);
afr_status afr_build_deep_buffer(const afr_samples *s, afr_deep_buffer *out, void *ws,
                                 size_t ws_bytes, int64_t *dropped_dev, hipStream_t stream);

/* The same build with per-stage timing: stage_end[0 .. afr_build_stage_count()-1] are caller-owned
 * events (created by the caller) that are recorded on `stream` after the bin-count, offset-scan,
 * record-scatter and per-pixel-select stages, in that order, so that each stage's duration is the
 * time between consecutive events (the first measured from an event the caller records before the
 * call). Results are identical to afr_build_deep_buffer. AFR_E_INVALID if stage_end or any of its
 * events is NULL. */
int32_t afr_build_stage_count(void);
afr_status afr_build_deep_buffer_staged(const afr_samples *s, afr_deep_buffer *out, void *ws,
                                        size_t ws_bytes, int64_t *dropped_dev, hipStream_t stream,
                                        hipEvent_t *stage_end);

/* ---------------------------------------------------------------------------------------------
 * Gradient, density and filter-extent estimation per tile (Sec. 4, 4.1, 5.1).
 *
 * Per pixel: luminance L (Rec. 709 weights), age weight w = exp(-alpha a), age-weighted mean Lbar.
 * Age weights are evaluated over the FP64 exponent range (relative precision about 2e-7 down to
 * w = 2^-1022, ages of about 200 s at the default alpha); a pixel whose samples are all older than
 * that has no weight and its mean, like the FP64 definition's, is undefined (NaN).
 * Spatial gradient: mean |Lbar_p - Lbar_q| over the filled 4-neighbours in x (resp. y). Temporal
 * gradient: slots split by rank into a newer and an older half, |L_new - L_old| divided by
 * max(a_old - a_new, dt_floor). Per tile: age-weighted means of the three gradients over the pixels
 * where they are defined (0 otherwise), V = A * 2 max(mean age, age_floor) / n, the age-weighted
 * luminance mean and variance, and the extents: with Gx' = sqrt(Gx^2 + g_floor^2) (same for y) and
 * u = tau Gt, ex2 = cbrt(V Gy' u / Gx'^2)^2, ey2 = cbrt(V Gx' u / Gy'^2)^2,
 * kt2 = cbrt(u^2 / (V Gx' Gy'))^2 (all 0 when u = 0), then
 * sx2 = e_min^2 + z e_max^2 / (e_max^2 + z), z = sigma^2 ex2 (likewise sy2). A tile with u > 0 and
 * no buffered samples (V = +inf; crosshair gradients over an empty tile) takes the large-V limit:
 * ex2 = ey2 = +inf, sx2 = sy2 = e_min^2 + e_max^2 (+inf when e_max is), kt2 = 0.
 *
 *   buf   a built deep buffer; out->data receives every statistic plane (overwritten)
 * ------------------------------------------------------------------------------------------- */
afr_status afr_estimate_gradients(const afr_deep_buffer *buf, const afr_params *params,
                                  afr_tile_stats *out, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Scatter form (Sec. 5.2) with adaptive splat size (Sec. 6.2).
 *
 * Every filled slot s of pixel q is a splat: a square of edge size[q] (px) centred on the sample,
 * covering output pixel p when |d_x| <= h and |d_y| <= h, with
 *   d_x = ((q_x - p_x) - 1/2) + ox_s,  d_y = ((q_y - p_y) - 1/2) + oy_s,  h = min(size[q], max_size)/2
 * evaluated in binary32 (all samples of a pixel share its splat size, as the samples of a region do
 * in the paper). At p the splat has exponent E = -1/2 (d_x^2 / sx2 + d_y^2 / sy2 + a^2 kt2) with p's
 * tile parameters, and C_p = sum exp(E - E_max) c / W', W' = sum exp(E - E_max) over the covering
 * splats; aux = (E_max, W'); a pixel no splat covers is 0 with aux (0, 0). With size 2R + 1 every
 * sample whose offsets lie strictly inside (0, 1) covers exactly the pixels whose gather block
 * holds it, so the image equals afr_reconstruct's. The coverage map holds, per pixel, the number n
 * of covering splats and their mean size (0 if none), taken as (float(sum of round(256 size)) / n)
 * / 256 in binary32. Colour sums are accumulated with atomics: their last bits may differ from run
 * to run; footprints, counts and mean sizes are exact.
 * ------------------------------------------------------------------------------------------- */
typedef struct afr_splat_params {
    float size_default;  /* size without a previous image, or where no splat arrived, px [5]      */
    float size_min, size_max;  /* clamp of the sizes, px [1, 16]; 0 < min <= default <= max <= 64 */
    float grow;          /* factor where fewer than n_low splats arrived [4]; >= 1                  */
    float shrink;        /* factor where more than n_high splats arrived [0.7]; in (0, 1]          */
    int32_t n_low, n_high; /* [4, 32]; 0 <= n_low <= n_high                                        */
} afr_splat_params;

/* Splat sizes for the next image from this image's coverage map (Sec. 6.2): the mean size of the
 * splats that reached the pixel (size_default where none did), times grow where n < n_low or
 * shrink where n > n_high, clamped to [size_min, size_max] and rounded to a multiple of 1/256 px
 * (binary32, ties to even).
 *   coverage  device [2][H][W] (n, mean size) from afr_reconstruct_scatter, or NULL: the first image
 *   size      device [H][W] output */
afr_status afr_splat_sizes(int32_t width, int32_t height, const float *coverage,
                           const afr_splat_params *params, float *size, hipStream_t stream);

/*   size      device [H][W] splat edge per source pixel, px (values above max_size count as max_size)
 *   max_size  largest splat edge, px, in (0, 64]; it bounds how far a splat reaches
 *   rgb       device [3][H][W];  aux  device [2][H][W] or NULL;  coverage  device [2][H][W] or NULL */
afr_status afr_reconstruct_scatter(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                   const afr_params *params, const float *size, float max_size,
                                   float *rgb, float *aux, float *coverage, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Sampler feedback (Sec. 4, 4.1, 6.1): per-tile statistics the sampler steers by, computed from its
 * own deep buffer (per-pixel queues of depth b; Sec. 4 uses b = 4) and that buffer's tile statistics
 * from afr_estimate_gradients. Per tile T of s_T pixels:
 *   |T| = samples in T, empty_T = s_T b - |T|, e = (w h b - |buffer|) / tiles (mean empty per tile),
 *   u_T = 1 - min(1, m e / empty_T)  (0 when empty_T = 0)              undersampling (Sec. 6.1)
 *   E_T = s_T (kappa v_T / sum v + lambda u_T / sum u)                  tile error (Sec. 6.1)
 * with v_T the tile's age-weighted luminance variance (Sec. 4); a share whose sum is 0 adds 0; the
 * occlusion share of the paper needs occlusion rays and is left out. Gain control (Sec. 4.1): with
 * dC/ds the mean over tiles of (G_x + G_y) / 2, dC/dt the mean of G_t and T the mean over non-empty
 * tiles of their mean sample age, S = gain dC/dt T / dC/ds balances dC/ds S = gain dC/dt T, and the
 * target tile count is w h / S^2 (S = 0 and inf tiles when dC/dt = 0: static content is tiled as
 * finely as possible; S = inf and 0 tiles when dC/ds = 0 < dC/dt). All sums are FP64 in a fixed
 * order.
 * ------------------------------------------------------------------------------------------- */
typedef struct afr_sampler_params {
    float kappa;   /* weight of the variation share [0.7]; kappa, lambda >= 0, kappa + lambda <= 1 */
    float lambda;  /* weight of the undersampling share [0.3]                                      */
    float m;       /* undersampling factor m >= 0 [2]                                              */
    float gain;    /* gain constant i > 0 [4]                                                      */
} afr_sampler_params;

/* Workspace for afr_sampler_stats and afr_sampler_select on `tiles` tiles. */
size_t afr_sampler_workspace_bytes(int32_t tiles);

/*   buf, stats  the sampler's buffer and its statistics (stats->tile == params->tile)
 *   E, u        device [tiles_y][tiles_x] float outputs
 *   globals     device double[8]: sum v, sum u, e, dC/ds, dC/dt, T, S, target tile count */
afr_status afr_sampler_stats(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                             const afr_params *params, const afr_sampler_params *sp, float *E,
                             float *u, double *globals, void *ws, size_t ws_bytes,
                             hipStream_t stream);

/* Equal-error tiles (Sec. 4: the sampler's tiles hold about equal colour variation and are picked
 * uniformly; Sec. 4.1: gain control sets their number). The adaptive K-D tiling is not built; its
 * effect is reproduced over the fixed tiles: on the Z-curve (Morton order) over the tile grid, the
 * integer error weights q_T of afr_sampler_select are summed (C_m over the first m tiles, total Q),
 * tile m starts in part p_m = min(N - 1, floor(C_m N / Q)), and each of the N parts is worth 1/N:
 * a part that tiles start in spreads it over them by area, a part no tile starts in gives it to the
 * tile before it on the curve. Output, per tile, proportional to its probability:
 *   P_T = s_T / (area of the tiles starting in p_T) + (parts strictly between p_T and the next
 *         tile's part, or up to N after the last tile)
 * in FP64 from integers, stored as float; P_T = s_T when Q = 0. Feeding P to afr_sampler_select
 * draws from these tiles.
 *   E         device [tiles_y][tiles_x] float tile errors (at most 65536 tiles)
 *   globals   device double[8] from afr_sampler_stats: N = the target tile count rounded to
 *             nearest and clamped to [1, tiles] (1 if NaN); may be NULL when n_parts > 0
 *   n_parts   N itself when > 0 (clamped to the tile count)
 *   weights   device [tiles_y][tiles_x] float output */
afr_status afr_sampler_tile_weights(int32_t width, int32_t height, int32_t tile, const float *E,
                                    const double *globals, int32_t n_parts, float *weights,
                                    void *ws, size_t ws_bytes, hipStream_t stream);

/* Spots for the next n samples (Sec. 4: a tile at random, then a uniform spot in it). With fixed
 * tiles a tile is drawn with probability proportional to E_T, which biases sampling as the paper's
 * equal-error adaptive tiles do under a uniform choice. The choice is exact integer arithmetic:
 * q_T = floor(E_T / E_max 2^24) in FP64 (E_T negative or not finite: 0; all q_T = 1 when no E_T is
 * positive), Q = sum q_T, and draw k takes r = rnd[k] >> 8 and the tile T with
 * cum_T <= (r Q) >> 24 < cum_T + q_T. Its spot is x = x0 + u1 bw, y = y0 + u2 bh in binary32, with
 * u1 = (rnd[n + k] >> 8) 2^-24, u2 = (rnd[2n + k] >> 8) 2^-24, (x0, y0) the tile's corner and
 * (bw, bh) its size clipped to the image; a spot that rounds onto the far edge takes the float below.
 *   E        device [tiles_y][tiles_x] float (tiles of edge `tile` over width x height), at most 65536
 *   rnd      device uint32 [3 n], random bits supplied by the caller
 *   x, y     device float [n] outputs; tile_out optional device int32 [n] (the chosen tile) */
afr_status afr_sampler_select(int32_t width, int32_t height, int32_t tile, const float *E,
                              int64_t n, const uint32_t *rnd, float *x, float *y, int32_t *tile_out,
                              void *ws, size_t ws_bytes, hipStream_t stream);

/* afr_sampler_select for callers that cannot allocate device memory (code under HIP graph capture,
 * tight per-frame serving loops, harnesses that forbid allocation): the same draws, bit for bit, with
 * no workspace argument. The prefix of tile weights lives in a library-owned device array of
 * 65 537 64-bit entries (512 KiB, the largest tile count the selection accepts plus one), one per GPU,
 * held until the process ends. The call allocates nothing and frees nothing. Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (on different streams) race. More than
 * 65 536 tiles is AFR_E_RANGE, as for afr_sampler_select. The first call on a device looks up the
 * array's device address (hipGetSymbolAddress) and keeps it; that lookup is not capturable, so make
 * one call on each device before capturing. */
afr_status afr_sampler_select_noalloc(int32_t width, int32_t height, int32_t tile, const float *E,
                                      int64_t n, const uint32_t *rnd, float *x, float *y,
                                      int32_t *tile_out, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * RMS error against a reference image (the per-frame error the evaluation of Sec. 7 reports, and the
 * loss the filter parameters sigma and tau are fit on) and its gradient, for chaining into
 * afr_reconstruct_backward.
 *   loss = scale * sqrt(sum_i (img_i - ref_i)^2 / n),  grad_i = scale * (img_i - ref_i) / (n * rms)
 * (grad 0 when rms is 0). Sums are FP64 in a fixed order, so results do not change between runs.
 *   img, ref   device float [n] (any layout, the same for both)
 *   loss       optional device double: receives the loss
 *   grad       optional device float [n]: receives the gradient
 *   ws         device workspace of afr_rms_workspace_bytes() bytes
 * ------------------------------------------------------------------------------------------- */
size_t afr_rms_workspace_bytes(void);
afr_status afr_rms_loss(const float *img, const float *ref, int64_t n, double scale, double *loss,
                        float *grad, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Crosshair gradients (Sec. 4.1, 4.2). A crosshair is a centre sample at (x, y, t), the four samples
 * taken at the same instant one pixel away, (x -/+ 1, y, t) and (x, y -/+ 1, t), and an earlier
 * sample taken at the same sub-pixel spot, (x, y, t0). afr_crosshairs gives each as a device int32
 * index into a sample stream; -1 (or any index outside the stream) marks an absent sample.
 * ------------------------------------------------------------------------------------------- */
typedef struct afr_crosshairs {
    const int32_t *centre;   /* [n] centre sample                                                 */
    const int32_t *xm, *xp;  /* [n] neighbours at x - 1 and x + 1                                 */
    const int32_t *ym, *yp;  /* [n] neighbours at y - 1 and y + 1                                 */
    const int32_t *old;      /* [n] the earlier sample at the centre's sub-pixel spot             */
    int64_t n;               /* number of crosshairs, < 2^31                                      */
} afr_crosshairs;

/* The sampler's crosshair queues. Per crosshair, with L the luminance of a sample (Rec. 709):
 *   gx = mean of |L_c - L_n| over the present horizontal neighbours with finite L (else -1),
 *   gy likewise over the vertical ones,
 *   gt = |L_c - L_old| / max(t - t0, params->dt_floor) when the old sample is present, its L and
 *        time are finite and t0 < t (else -1),
 * computed in FP64 and stored as float. Each crosshair record (the centre's x, y, t and the three
 * gradients) is pushed into the queue of the centre's pixel exactly as afr_build_deep_buffer pushes
 * samples: `out` receives, per pixel, the newest min(K, arrivals) records, with the gradients in the
 * r, g, b planes (gx, gy, gt) and the centre time in tage. A crosshair whose centre is absent or has a
 * non-finite luminance, or whose record is invalid by the build's rule, is dropped.
 *
 *   s, xh        device sample stream (velocities ignored) and crosshairs
 *   params       only dt_floor is used (validated like afr_estimate_gradients, without t_now)
 *   out          AFR_FP32 only (AFR_E_UNSUPPORTED otherwise); geometry, K and t_ref as for a build
 *   ws, ws_bytes device workspace of at least afr_crosshair_workspace_bytes(xh->n, width, height)
 *   dropped_dev  optional device int64: receives the number of dropped crosshairs
 */
size_t afr_crosshair_workspace_bytes(int64_t n, int32_t width, int32_t height);
afr_status afr_build_crosshair_buffer(const afr_samples *s, const afr_crosshairs *xh,
                                      const afr_params *params, afr_deep_buffer *out, void *ws,
                                      size_t ws_bytes, int64_t *dropped_dev, hipStream_t stream);

/* Tile statistics with crosshair gradients: everything afr_estimate_gradients computes from `buf`,
 * then the three gradient planes replaced by the age-weighted means over the tile's crosshair
 * records in `xbuf` (Sec. 4.1 with the age weights of Sec. 4),
 *   G(T) = sum omega g / sum omega over the records with g >= 0 (0 if none),
 *   omega = exp(-alpha (t_now - t)),
 * and the extents recomputed from them and the tile's volume V (as stored in out, float). xbuf must
 * be an AFR_FP32 buffer of buf's width and height made by afr_build_crosshair_buffer, with
 * params->t_now >= xbuf->t_ref. */
afr_status afr_estimate_gradients_crosshair(const afr_deep_buffer *buf,
                                            const afr_deep_buffer *xbuf,
                                            const afr_params *params, afr_tile_stats *out,
                                            hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Adaptive space-time gather (Sec. 5.1 Gaussian filter, Sec. 5.2 normalised weighted average).
 *
 * Pixel p = (i, j) in tile T gathers every filled slot s of the pixels q with |q_x - i| <= R and
 * |q_y - j| <= R inside the image, with E_s = -1/2 (dx^2/sx2 + dy^2/sy2 + a^2 kt2),
 * dx = q_x + ox - (i + 1/2), dy = q_y + oy - (j + 1/2), a = t_now - t, using T's statistics:
 *   C_p = sum_s exp(E_s - E_max) c_s / W',  W' = sum_s exp(E_s - E_max),  E_max = max_s E_s.
 * A pixel whose block holds no slot gets C_p = 0, E_max = 0, W' = 0.
 *
 *   rgb   [3][H][W] float output
 *   aux   [2][H][W] float output (E_max, W'), or NULL; the backward needs it
 * afr_reconstruct runs the LDS-tiled separable form; afr_reconstruct_plain runs the direct form
 * (one thread per pixel, one exponential per pair). Both compute the same quantity.
 * ------------------------------------------------------------------------------------------- */
afr_status afr_reconstruct(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                           const afr_params *params, float *rgb, float *aux, hipStream_t stream);
afr_status afr_reconstruct_plain(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                 const afr_params *params, float *rgb, float *aux,
                                 hipStream_t stream);

/* Statistics and gather in one launch: the same result as afr_estimate_gradients (into stats)
 * followed by afr_reconstruct, bit for bit, with the deep buffer read by one kernel per group of
 * tiles that first reduces the group's statistics and then gathers it (8 px tiles; other tile sizes
 * run the two steps one after the other).
 *   stats  receives every statistic plane (overwritten), as afr_estimate_gradients
 *   rgb    [3][H][W] float output;  aux  [2][H][W] float output or NULL */
afr_status afr_forward(const afr_deep_buffer *buf, const afr_params *params, afr_tile_stats *stats,
                       float *rgb, float *aux, hipStream_t stream);

/* afr_reconstruct with an explicit launch shape: tiles_per_wave (1, 2 or 4; 0 = the library's choice)
 * statistics tiles side by side are processed by one workgroup, one 64-lane wave per tile (R >= 3
 * allows at most 2). The shape changes only how work is spread over waves: every pixel sums the same
 * terms in the same order, so all shapes give bit-identical output. Used by the tuner; shapes the
 * kernel does not support for the given radius fall back to a supported one. */
afr_status afr_reconstruct_launch(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                  const afr_params *params, int32_t tiles_per_wave, float *rgb,
                                  float *aux, hipStream_t stream);

/* Launch-shape tuner for afr_reconstruct: times every supported tiles_per_wave on these inputs
 * (writes rgb; blocking: synchronises the stream), records the fastest for the buffer class
 * (width, height, K, precision, radius) in a process-wide, thread-safe table that afr_reconstruct
 * and afr_reconstruct_launch(..., 0, ...) consult, and reports it. */
afr_status afr_reconstruct_tune(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                const afr_params *params, float *rgb, int32_t *best_tiles_per_wave,
                                float *best_ms, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Adjoint of afr_reconstruct with the tile statistics held fixed (they are inputs of the gather,
 * as the paper's tile information is, Sec. 4.2). With pi_s(p) = exp(E_s - E_max)/W':
 *   grad_slot[ch][s] = sum_p grad_rgb[ch][p] pi_s(p)
 *   grad_params[0]   = dl/dsigma, grad_params[1] = dl/dtau, through sx2, sy2 and kt2.
 * The per-pair weights are recomputed, not stored. Requires tau > 0. Deterministic: no floating-
 * point atomics; reductions run in a fixed order.
 *
 *   rgb, aux   outputs of the forward call on the same inputs
 *   grad_rgb   [3][H][W] dl/dC
 *   grad_slot  [3][K][H][W] float output (empty slots get 0)
 *   grad_params 2 floats, device
 *   ws         at least afr_backward_workspace_bytes(width, height, k, radius) bytes
 * ------------------------------------------------------------------------------------------- */
size_t afr_backward_workspace_bytes(int32_t width, int32_t height, int32_t k, int32_t radius);
afr_status afr_reconstruct_backward(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                    const afr_params *params, const float *rgb, const float *aux,
                                    const float *grad_rgb, float *grad_slot, float *grad_params,
                                    void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Batched reconstruction: many independent estimate + gather pipelines of uneven size in one
 * launch. Work items are (item, group of tiles_per_wave tiles), one workgroup each, numbered with
 * the larger items first; each work item estimates its own tiles' statistics and then gathers them,
 * so items never wait on each other. Outputs are bit-identical to afr_estimate_gradients followed
 * by afr_reconstruct on each item, for every tiles_per_wave.
 *
 * Restrictions: every item uses 8 px statistics tiles, the same radius and the same precision;
 * other batches return AFR_E_UNSUPPORTED. Items must not share output memory. At most 2^24 work
 * items in all (AFR_E_RANGE).
 * ------------------------------------------------------------------------------------------- */
typedef struct afr_batch_item {
    afr_deep_buffer buf;   /* a built deep buffer                                               */
    afr_tile_stats stats;  /* receives the item's statistics                                    */
    afr_params params;     /* per item (t_now, sigma, tau, ...); radius and tile shared         */
    float *rgb;            /* [3][H][W] output                                                  */
    float *aux;            /* [2][H][W] output or NULL                                          */
} afr_batch_item;

typedef struct afr_batch afr_batch; /* opaque host-side plan */

/* Device workspace for a batch of n items (item table, first work item of each item). */
size_t afr_batch_workspace_bytes(int32_t n_items);

/* Validates the items, orders them by work, uploads the item table to ws (a blocking host-to-device
 * copy) and returns a host-side plan. Not capturable; call once per batch layout. tiles_per_wave:
 * 1, 2 or 4, or 0 for the library default. The items' device memory must stay valid while the plan
 * is used; ws must not be shared with another plan. */
afr_status afr_batch_create(const afr_batch_item *items, int32_t n_items, int32_t tiles_per_wave,
                            void *ws, size_t ws_bytes, afr_batch **plan);

/* Enqueues the whole batch (one kernel launch) on the stream. Performs no host
 * synchronisation, allocation, memset or copy, so it can be captured into a HIP graph and replayed;
 * replays of one plan must not overlap. */
afr_status afr_batch_run(const afr_batch *plan, hipStream_t stream);

/* Times every supported tiles_per_wave on the plan (blocking: synchronises the stream), keeps the
 * fastest in the plan, and reports it. The outputs are overwritten by the timing runs. */
afr_status afr_batch_tune(afr_batch *plan, hipStream_t stream, int32_t *best_tiles_per_wave,
                          float *best_ms);

/* Current launch shape of a plan. */
int32_t afr_batch_tiles_per_wave(const afr_batch *plan);

void afr_batch_destroy(afr_batch *plan);

/* The whole batch in one call, without a plan: the same validation and result as afr_batch_create
 * followed by afr_batch_run, bit for bit, with the item table written to the workspace by small
 * kernels that carry it in their arguments. The call enqueues only kernels (no allocation, host
 * synchronisation, copy or memset), so it can be captured into a HIP graph with the items' values
 * at capture time; a replay writes those values again.
 *   items, n   as afr_batch_create (host memory, read during the call only)
 *   tune       tiles_per_wave: 1, 2 or 4, or 0 for the library's choice (the shape afr_batch_tune
 *              last found fastest for this precision and radius in this process, else the
 *              default); ws, ws_bytes: device workspace of afr_batch_workspace_bytes(n) bytes, which
 *              must not be in use by another batch while the call's kernels run
 * Errors: as afr_batch_create; AFR_E_INVALID for a NULL tune or workspace, AFR_E_NOMEM for a small
 * one. */
typedef struct afr_tune {
    int32_t tiles_per_wave;
    void *ws;
    size_t ws_bytes;
} afr_tune;
afr_status afr_batch_reconstruct(const afr_batch_item *items, int32_t n, const afr_tune *tune,
                                 hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* AFR_H */
