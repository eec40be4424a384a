// C ABI entry points of libafr: synchronous argument validation, workspace carving, and launches on
// the caller's stream. No entry point allocates device memory or synchronises.
#include <cmath>

#include "afr_internal.h"

namespace {

using namespace afr;

afr_status from_hip(hipError_t e) { return e == hipSuccess ? AFR_OK : AFR_E_DEVICE; }

#define AFR_TRY(expr)                         \
    do {                                      \
        const afr_status _st = (expr);        \
        if (_st != AFR_OK) return _st;        \
    } while (0)

}  // namespace

extern "C" {

const char *afr_status_string(afr_status s) {
    switch (s) {
        case AFR_OK: return "ok";
        case AFR_E_INVALID: return "invalid argument";
        case AFR_E_RANGE: return "argument out of range";
        case AFR_E_DEVICE: return "device error";
        case AFR_E_NOMEM: return "workspace too small";
        case AFR_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *afr_version(void) { return "afr 0.1.0 gfx950"; }

size_t afr_build_workspace_bytes(int64_t n, int32_t width, int32_t height, int32_t k) {
    (void)k;
    if (n < 0 || width < 1 || height < 1) return 0;
    return build_ws_bytes(n, width, height);
}

static afr_status build_checked(const afr_samples *s, afr_deep_buffer *out, void *ws,
                                size_t ws_bytes, int64_t *dropped_dev, hipStream_t stream,
                                hipEvent_t *stage_end) {
    AFR_TRY(check_buffer(out));
    if (!s || s->n < 0) return AFR_E_INVALID;
    if (s->n >= (int64_t(1) << 31)) return AFR_E_RANGE;
    if (s->n > 0 && (!s->x || !s->y || !s->t || !s->r || !s->g || !s->b)) return AFR_E_INVALID;
    if (!s->vx != !s->vy) return AFR_E_INVALID;
    if (!ws) return AFR_E_INVALID;
    if (!build_supported(out->width, out->height)) return AFR_E_UNSUPPORTED;
    if (ws_bytes < build_ws_bytes(s->n, out->width, out->height)) return AFR_E_NOMEM;
    const BuildWs w = build_ws_carve(ws, s->n, out->width, out->height);
    unsigned long long *dropped =
        dropped_dev ? reinterpret_cast<unsigned long long *>(dropped_dev) : w.dropped_internal;
    return from_hip(launch_build(*s, *out, w, dropped, stream, stage_end));
}

afr_status afr_build_deep_buffer(const afr_samples *s, afr_deep_buffer *out, void *ws,
                                 size_t ws_bytes, int64_t *dropped_dev, hipStream_t stream) {
    return build_checked(s, out, ws, ws_bytes, dropped_dev, stream, nullptr);
}

int32_t afr_build_stage_count(void) { return kBuildStages; }

afr_status afr_build_deep_buffer_staged(const afr_samples *s, afr_deep_buffer *out, void *ws,
                                        size_t ws_bytes, int64_t *dropped_dev, hipStream_t stream,
                                        hipEvent_t *stage_end) {
    if (!stage_end) return AFR_E_INVALID;
    for (int i = 0; i < kBuildStages; ++i)
        if (!stage_end[i]) return AFR_E_INVALID;
    return build_checked(s, out, ws, ws_bytes, dropped_dev, stream, stage_end);
}

size_t afr_rms_workspace_bytes(void) { return rms_ws_bytes(); }

afr_status afr_rms_loss(const float *img, const float *ref, int64_t n, double scale, double *loss,
                        float *grad, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || !ws) return AFR_E_INVALID;
    if (n > 0 && (!img || !ref)) return AFR_E_INVALID;
    if (!std::isfinite(scale)) return AFR_E_RANGE;
    if (ws_bytes < rms_ws_bytes()) return AFR_E_NOMEM;
    return from_hip(launch_rms_loss(img, ref, n, scale, loss, grad, ws, stream));
}

size_t afr_sampler_workspace_bytes(int32_t tiles) {
    if (tiles < 1) return 0;
    return sampler_ws_bytes(tiles);
}

afr_status afr_sampler_stats(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                             const afr_params *params, const afr_sampler_params *sp, float *E,
                             float *u, double *globals, void *ws, size_t ws_bytes,
                             hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(stats, buf, params));
    if (!sp || !E || !u || !globals || !ws) return AFR_E_INVALID;
    const float vals[] = {sp->kappa, sp->lambda, sp->m, sp->gain};
    for (float v : vals)
        if (!finite(v)) return AFR_E_RANGE;
    if (sp->kappa < 0.0f || sp->lambda < 0.0f || sp->kappa + sp->lambda > 1.0f) return AFR_E_RANGE;
    if (sp->m < 0.0f || !(sp->gain > 0.0f)) return AFR_E_RANGE;
    const int64_t nt = (int64_t)stats->tiles_x * stats->tiles_y;
    if (nt > (int64_t(1) << 30)) return AFR_E_RANGE;
    if (ws_bytes < sampler_ws_bytes((int32_t)nt)) return AFR_E_NOMEM;
    return from_hip(launch_sampler_stats(*buf, *stats, *params, *sp, E, u, globals, ws, stream));
}

afr_status afr_sampler_tile_weights(int32_t width, int32_t height, int32_t tile, const float *E,
                                    const double *globals, int32_t n_parts, float *weights,
                                    void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!E || !weights || !ws) return AFR_E_INVALID;
    if (n_parts <= 0 && !globals) return AFR_E_INVALID;
    if (width < 1 || height < 1 || tile < 1) return AFR_E_RANGE;
    const int64_t nt = (int64_t)((width + tile - 1) / tile) * ((height + tile - 1) / tile);
    if (nt > kMaxSamplerTiles) return AFR_E_RANGE;
    if (ws_bytes < sampler_ws_bytes((int32_t)nt)) return AFR_E_NOMEM;
    return from_hip(launch_sampler_tile_weights(width, height, tile, E, globals, n_parts, weights,
                                                ws, stream));
}

afr_status afr_sampler_select(int32_t width, int32_t height, int32_t tile, const float *E,
                              int64_t n, const uint32_t *rnd, float *x, float *y, int32_t *tile_out,
                              void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!E || !ws || n < 0) return AFR_E_INVALID;
    if (n > 0 && (!rnd || !x || !y)) return AFR_E_INVALID;
    if (width < 1 || height < 1 || tile < 1) return AFR_E_RANGE;
    const int64_t nt = (int64_t)((width + tile - 1) / tile) * ((height + tile - 1) / tile);
    if (nt > kMaxSamplerTiles || n >= (int64_t(1) << 31)) return AFR_E_RANGE;
    if (ws_bytes < sampler_ws_bytes((int32_t)nt)) return AFR_E_NOMEM;
    return from_hip(launch_sampler_select(width, height, tile, E, n, rnd, x, y, tile_out, ws,
                                          stream));
}

afr_status afr_sampler_select_noalloc(int32_t width, int32_t height, int32_t tile, const float *E,
                                      int64_t n, const uint32_t *rnd, float *x, float *y,
                                      int32_t *tile_out, hipStream_t stream) {
    if (!E || n < 0) return AFR_E_INVALID;
    if (n > 0 && (!rnd || !x || !y)) return AFR_E_INVALID;
    if (width < 1 || height < 1 || tile < 1) return AFR_E_RANGE;
    const int64_t nt = (int64_t)((width + tile - 1) / tile) * ((height + tile - 1) / tile);
    if (nt > kMaxSamplerTiles || n >= (int64_t(1) << 31)) return AFR_E_RANGE;
    return from_hip(launch_sampler_select_noalloc(width, height, tile, E, n, rnd, x, y, tile_out,
                                                  stream));
}

afr_status afr_splat_sizes(int32_t width, int32_t height, const float *coverage,
                           const afr_splat_params *sp, float *size, hipStream_t stream) {
    if (!sp || !size) return AFR_E_INVALID;
    if (width < 1 || height < 1 || (int64_t)width * height >= (int64_t(1) << 29)) return AFR_E_RANGE;
    const float vals[] = {sp->size_default, sp->size_min, sp->size_max, sp->grow, sp->shrink};
    for (float v : vals)
        if (!finite(v)) return AFR_E_RANGE;
    if (!(sp->size_min > 0.0f) || sp->size_default < sp->size_min ||
        sp->size_max < sp->size_default || sp->size_max > kMaxSplat)
        return AFR_E_RANGE;
    if (sp->grow < 1.0f || !(sp->shrink > 0.0f) || sp->shrink > 1.0f) return AFR_E_RANGE;
    if (sp->n_low < 0 || sp->n_high < sp->n_low) return AFR_E_RANGE;
    return from_hip(launch_splat_sizes(width, height, coverage, *sp, size, stream));
}

afr_status afr_reconstruct_scatter(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                   const afr_params *params, const float *size, float max_size,
                                   float *rgb, float *aux, float *coverage, hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(stats, buf, params));
    if (!size || !rgb) return AFR_E_INVALID;
    if (!finite(max_size) || !(max_size > 0.0f) || max_size > kMaxSplat) return AFR_E_RANGE;
    return from_hip(launch_scatter(*buf, *stats, *params, size, max_size, rgb, aux, coverage,
                                   stream));
}

size_t afr_crosshair_workspace_bytes(int64_t n, int32_t width, int32_t height) {
    if (n < 0 || width < 1 || height < 1) return 0;
    return crosshair_ws_bytes(n, width, height);
}

afr_status afr_build_crosshair_buffer(const afr_samples *s, const afr_crosshairs *xh,
                                      const afr_params *params, afr_deep_buffer *out, void *ws,
                                      size_t ws_bytes, int64_t *dropped_dev, hipStream_t stream) {
    AFR_TRY(check_buffer(out));
    AFR_TRY(check_params(params, nullptr));
    if (!s || s->n < 0 || !xh || xh->n < 0) return AFR_E_INVALID;
    if (s->n >= (int64_t(1) << 31) || xh->n >= (int64_t(1) << 31)) return AFR_E_RANGE;
    if (s->n > 0 && (!s->x || !s->y || !s->t || !s->r || !s->g || !s->b)) return AFR_E_INVALID;
    if (xh->n > 0 && (!xh->centre || !xh->xm || !xh->xp || !xh->ym || !xh->yp || !xh->old))
        return AFR_E_INVALID;
    if (!ws) return AFR_E_INVALID;
    if (out->precision != AFR_FP32) return AFR_E_UNSUPPORTED;
    if (!build_supported(out->width, out->height)) return AFR_E_UNSUPPORTED;
    if (ws_bytes < crosshair_ws_bytes(xh->n, out->width, out->height)) return AFR_E_NOMEM;
    return from_hip(launch_crosshair_build(*s, *xh, *params, *out, ws,
                                           reinterpret_cast<unsigned long long *>(dropped_dev),
                                           stream));
}

afr_status afr_estimate_gradients_crosshair(const afr_deep_buffer *buf,
                                            const afr_deep_buffer *xbuf,
                                            const afr_params *params, afr_tile_stats *out,
                                            hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_buffer(xbuf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_params(params, xbuf));
    AFR_TRY(check_stats(out, buf, params));
    if (xbuf->precision != AFR_FP32) return AFR_E_UNSUPPORTED;
    if (xbuf->width != buf->width || xbuf->height != buf->height) return AFR_E_INVALID;
    return from_hip(launch_crosshair_estimate(*buf, *xbuf, *params, *out, stream));
}

afr_status afr_estimate_gradients(const afr_deep_buffer *buf, const afr_params *params,
                                  afr_tile_stats *out, hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(out, buf, params));
    return from_hip(launch_estimate(*buf, *params, *out, stream));
}

afr_status afr_reconstruct(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                           const afr_params *params, float *rgb, float *aux, hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(stats, buf, params));
    if (!rgb) return AFR_E_INVALID;
    const int tuned = tuned_tiles_per_wave(*buf, params->radius);
    return from_hip(launch_reconstruct_tiled(*buf, *stats, *params,
                                             tuned ? tuned : default_tiles_per_group(params->radius),
                                             rgb, aux, stream));
}

afr_status afr_forward(const afr_deep_buffer *buf, const afr_params *params, afr_tile_stats *stats,
                       float *rgb, float *aux, hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(stats, buf, params));
    if (!rgb) return AFR_E_INVALID;
    const int tuned = tuned_tiles_per_wave(*buf, params->radius);
    return from_hip(launch_forward(*buf, *params, *stats,
                                   tuned ? tuned : default_tiles_per_group(params->radius), rgb, aux,
                                   stream));
}

afr_status afr_reconstruct_tune(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                const afr_params *params, float *rgb, int32_t *best_tiles_per_wave,
                                float *best_ms, hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(stats, buf, params));
    if (!rgb) return AFR_E_INVALID;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return AFR_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return AFR_E_DEVICE;
    }
    int best = 0;
    float best_t = 1e30f;
    afr_status st = AFR_OK;
    const int shapes[3] = {1, 2, 4};
    for (int s = 0; s < 3 && st == AFR_OK; ++s) {
        if (shapes[s] > default_tiles_per_group(params->radius)) continue;
        constexpr int kReps = 5;
        st = from_hip(launch_reconstruct_tiled(*buf, *stats, *params, shapes[s], rgb, nullptr, stream));
        if (st == AFR_OK && hipEventRecord(e0, stream) != hipSuccess) st = AFR_E_DEVICE;
        for (int r = 0; r < kReps && st == AFR_OK; ++r)
            st = from_hip(launch_reconstruct_tiled(*buf, *stats, *params, shapes[s], rgb, nullptr,
                                                   stream));
        float ms = 0.0f;
        if (st == AFR_OK && (hipEventRecord(e1, stream) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = AFR_E_DEVICE;
        if (st == AFR_OK && ms / kReps < best_t) {
            best_t = ms / kReps;
            best = shapes[s];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != AFR_OK) return st;
    record_tiles_per_wave(*buf, params->radius, best);
    if (best_tiles_per_wave) *best_tiles_per_wave = best;
    if (best_ms) *best_ms = best_t;
    return AFR_OK;
}

afr_status afr_reconstruct_launch(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                  const afr_params *params, int32_t tiles_per_wave, float *rgb,
                                  float *aux, hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(stats, buf, params));
    if (!rgb) return AFR_E_INVALID;
    if (tiles_per_wave < 0 || tiles_per_wave > 4) return AFR_E_RANGE;
    const int tuned = tuned_tiles_per_wave(*buf, params->radius);
    const int tpw = tiles_per_wave == 0
                        ? (tuned ? tuned : default_tiles_per_group(params->radius))
                        : tiles_per_wave;
    return from_hip(launch_reconstruct_tiled(*buf, *stats, *params, tpw, rgb, aux, stream));
}

afr_status afr_reconstruct_plain(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                 const afr_params *params, float *rgb, float *aux,
                                 hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(stats, buf, params));
    if (!rgb) return AFR_E_INVALID;
    return from_hip(launch_reconstruct_plain(*buf, *stats, *params, rgb, aux, stream));
}

size_t afr_backward_workspace_bytes(int32_t width, int32_t height, int32_t k, int32_t radius) {
    if (width < 1 || height < 1 || k < 1 || k > 255 || radius < 0 || radius > kMaxRadius) return 0;
    return backward_ws_bytes(width, height, k, radius);
}

afr_status afr_reconstruct_backward(const afr_deep_buffer *buf, const afr_tile_stats *stats,
                                    const afr_params *params, const float *rgb, const float *aux,
                                    const float *grad_rgb, float *grad_slot, float *grad_params,
                                    void *ws, size_t ws_bytes, hipStream_t stream) {
    AFR_TRY(check_buffer(buf));
    AFR_TRY(check_params(params, buf));
    AFR_TRY(check_stats(stats, buf, params));
    if (!(params->tau > 0.0f)) return AFR_E_RANGE;
    if (!rgb || !aux || !grad_rgb || !grad_slot || !grad_params || !ws) return AFR_E_INVALID;
    if (ws_bytes < backward_ws_bytes(buf->width, buf->height, buf->k, params->radius))
        return AFR_E_NOMEM;
    return from_hip(launch_backward(*buf, *stats, *params, rgb, aux, grad_rgb, grad_slot,
                                    grad_params, ws, stream));
}

}  // extern "C"
