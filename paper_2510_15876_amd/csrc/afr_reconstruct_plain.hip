// Direct gather (Sec. 5.2 normalised weighted average with the Sec. 5.1 Gaussian space-time filter).
//
// One thread per output pixel, global loads, one exponential per (slot, pixel) pair and two passes
// over the (2R+1)^2 block: the first finds E_max, the second accumulates exp(E - E_max) and the
// weighted colours. This is the baseline form that the LDS-tiled kernel is measured against.
#include "afr_internal.h"

namespace afr {
namespace {

struct RecParams {
    float t_now, dt_ref;
    int radius;
};

template <typename S>
__global__ __launch_bounds__(256) void k_reconstruct_plain(BufView<S> v, RecParams p, TileGeom tg,
                                                           const float *__restrict__ stats,
                                                           float *__restrict__ rgb,
                                                           float *__restrict__ aux) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= v.width || j >= v.height) return;
    const int W = v.width, H = v.height, R = p.radius;
    const size_t hw = (size_t)W * H;
    const int T = (j / tg.tile) * tg.tiles_x + i / tg.tile;
    const float cx = 0.5f / stats[AFR_STAT_SX2 * tg.nt + T];
    const float cy = 0.5f / stats[AFR_STAT_SY2 * tg.nt + T];
    const float ct = 0.5f * stats[AFR_STAT_KT2 * tg.nt + T];
    const int qx0 = max(0, i - R), qx1 = min(W - 1, i + R);
    const int qy0 = max(0, j - R), qy1 = min(H - 1, j + R);

    float emax = -INFINITY;
    for (int qy = qy0; qy <= qy1; ++qy)
        for (int qx = qx0; qx <= qx1; ++qx) {
            const size_t q = (size_t)qy * W + qx;
            const int n = v.count[q];
            const float bx = (float)(qx - i) - 0.5f, by = (float)(qy - j) - 0.5f;
            for (int k = 0; k < n; ++k) {
                const size_t s = (size_t)k * hw + q;
                const float dx = bx + Codec<S>::dec(fld(v.ox, s));
                const float dy = by + Codec<S>::dec(fld(v.oy, s));
                const float a = Codec<S>::age(fld(v.ta, s), p.t_now, p.dt_ref);
                const float e = -(dx * dx * cx + dy * dy * cy + a * a * ct);
                emax = fmaxf(emax, e);
            }
        }
    const size_t px = (size_t)j * W + i;
    if (emax == -INFINITY) {  // no slot in the block
        rgb[px] = rgb[hw + px] = rgb[2 * hw + px] = 0.0f;
        if (aux) aux[px] = aux[hw + px] = 0.0f;
        return;
    }
    float ws = 0.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    for (int qy = qy0; qy <= qy1; ++qy)
        for (int qx = qx0; qx <= qx1; ++qx) {
            const size_t q = (size_t)qy * W + qx;
            const int n = v.count[q];
            const float bx = (float)(qx - i) - 0.5f, by = (float)(qy - j) - 0.5f;
            for (int k = 0; k < n; ++k) {
                const size_t s = (size_t)k * hw + q;
                const float dx = bx + Codec<S>::dec(fld(v.ox, s));
                const float dy = by + Codec<S>::dec(fld(v.oy, s));
                const float a = Codec<S>::age(fld(v.ta, s), p.t_now, p.dt_ref);
                const float e = -(dx * dx * cx + dy * dy * cy + a * a * ct);
                const float w = expf(e - emax);
                ws += w;
                cr += w * Codec<S>::dec(fld(v.r, s));
                cg += w * Codec<S>::dec(fld(v.g, s));
                cb += w * Codec<S>::dec(fld(v.b, s));
            }
        }
    const float inv = 1.0f / ws;
    rgb[px] = cr * inv;
    rgb[hw + px] = cg * inv;
    rgb[2 * hw + px] = cb * inv;
    if (aux) {
        aux[px] = emax;
        aux[hw + px] = ws;
    }
}

}  // namespace

hipError_t launch_reconstruct_plain(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                    const afr_params &prm, float *rgb, float *aux,
                                    hipStream_t st) {
    const RecParams p{prm.t_now, prm.t_now - buf.t_ref, prm.radius};
    const dim3 block(64, 4);
    const dim3 grid((buf.width + 63) / 64, (buf.height + 3) / 4);
    const TileGeom tg = geom_of(stats);
    if (buf.precision == AFR_FP16)
        k_reconstruct_plain<__half><<<grid, block, 0, st>>>(view_of<__half>(buf), p, tg, stats.data,
                                                            rgb, aux);
    else
        k_reconstruct_plain<float><<<grid, block, 0, st>>>(view_of<float>(buf), p, tg, stats.data,
                                                           rgb, aux);
    return hipGetLastError();
}

}  // namespace afr
