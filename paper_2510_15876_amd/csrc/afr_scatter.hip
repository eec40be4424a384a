// Scatter form of the reconstruction (Sec. 5.2) with adaptive splat size (Sec. 6.2).
//
// The paper's GPU reconstructor draws every buffered sample as a point splat and lets blending
// accumulate the filter-weighted colour and the weight of every covered pixel. Here the splats are
// binned by output tile instead of rasterised: one 256-thread workgroup per 16 x 16 tile takes the
// samples of the source pixels whose splats can reach the tile, and each thread splats its samples
// into per-pixel LDS accumulators with LDS atomics. Two passes over the same samples keep the sums
// in range, as the two-pass gather does: the first records each pixel's largest exponent (as the
// smallest Q = -E, an unsigned minimum of its bits), the coverage count and the splat-size sum; the
// second adds exp(E - E_max) and its colour-weighted terms. LDS float atomics make the last bits of
// the sums depend on arrival order; coverage counts, size sums and footprints are exact.
//
//   k_splat_sizes  per pixel: the next image's splat size from this image's coverage map
//   k_scatter      per 16 x 16 output tile: the two splat passes, then colour, aux and coverage
#include <cmath>

#include "afr_internal.h"

namespace afr {
namespace {

constexpr int kSTile = 16;                 // output tile edge
constexpr int kSThreads = kSTile * kSTile;  // one thread per output pixel in the final step

struct SplatRule {
    float size_default, size_min, size_max, grow, shrink;
    int32_t n_low, n_high;
};

__global__ __launch_bounds__(256) void k_splat_sizes(const float *__restrict__ cov_n,
                                                      const float *__restrict__ cov_size,
                                                      SplatRule r, int hw, float *size) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= hw) return;
    float v = r.size_default;
    if (cov_n) {
        const float n = cov_n[i];
        if (n > 0.0f) v = cov_size[i];
        if (n < (float)r.n_low) v = v * r.grow;
        else if (n > (float)r.n_high) v = v * r.shrink;
    }
    v = fminf(fmaxf(v, r.size_min), r.size_max);
    size[i] = rintf(v * 256.0f) * 0.00390625f;
}

struct ScatterParams {
    float t_now, dt_ref, max_size;
    int reach;  // largest |q - p| a splat of size max_size can span
};

// Signed offset from pixel p's centre to a sample of pixel q with offset o, in binary32 (the
// footprint test compares it with the half-width).
__device__ inline float splat_offset(int q, int p, float o) {
#pragma clang fp contract(off)
    return ((float)(q - p) - 0.5f) + o;
}

__device__ inline float splat_q(float dx, float dy, float a, float4 pr) {
#pragma clang fp contract(off)
    return 0.5f * (dx * dx * pr.x + dy * dy * pr.y + a * a * pr.z);
}

template <typename S>
__global__ __launch_bounds__(kSThreads) void k_scatter(BufView<S> v, ScatterParams p, TileGeom tg,
                                                       const float *__restrict__ stats,
                                                       const float *__restrict__ size,
                                                       float *__restrict__ rgb,
                                                       float *__restrict__ aux,
                                                       float *__restrict__ cov, int gx) {
    __shared__ unsigned qmin[kSThreads];
    __shared__ float accw[kSThreads], accr[kSThreads], accg[kSThreads], accb[kSThreads];
    __shared__ unsigned ncov[kSThreads], units[kSThreads];
    __shared__ float4 prm[kSThreads];  // (1/sx2, 1/sy2, kt2) of each output pixel's tile
    const int W = v.width, H = v.height;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (bid % gx) * kSTile, y0 = (bid / gx) * kSTile;
    const int e = threadIdx.x;
    const int px = x0 + (e % kSTile), py = y0 + (e / kSTile);
    qmin[e] = 0x7f800000u;  // +inf
    accw[e] = accr[e] = accg[e] = accb[e] = 0.0f;
    ncov[e] = units[e] = 0u;
    if (px < W && py < H) {
        const int T = (py / tg.tile) * tg.tiles_x + px / tg.tile;
        prm[e] = make_float4(1.0f / stats[AFR_STAT_SX2 * tg.nt + T],
                             1.0f / stats[AFR_STAT_SY2 * tg.nt + T], stats[AFR_STAT_KT2 * tg.nt + T],
                             0.0f);
    } else {
        prm[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    const int qx0 = max(0, x0 - p.reach), qx1 = min(W - 1, x0 + kSTile - 1 + p.reach);
    const int qy0 = max(0, y0 - p.reach), qy1 = min(H - 1, y0 + kSTile - 1 + p.reach);
    const int tx1 = min(W - 1, x0 + kSTile - 1), ty1 = min(H - 1, y0 + kSTile - 1);
    const int rw = qx1 - qx0 + 1, nreg = rw * (qy1 - qy0 + 1);
    const size_t plane = (size_t)W * H;
    for (int pass = 0; pass < 2; ++pass) {
        for (int r = e; r < nreg; r += kSThreads) {
            const int qx = qx0 + r % rw, qy = qy0 + r / rw;
            const size_t q = (size_t)qy * W + qx;
            const int n = v.count[q];
            if (n == 0) continue;
            const float sz = fminf(size[q], p.max_size);
            const float h = 0.5f * sz;
            if (!(h >= 0.0f)) continue;
            const unsigned su = (unsigned)rintf(256.0f * sz);
            const int ax0 = max(x0, qx - p.reach), ax1 = min(tx1, qx + p.reach);
            const int ay0 = max(y0, qy - p.reach), ay1 = min(ty1, qy + p.reach);
            if (ax0 > ax1 || ay0 > ay1) continue;
            for (int k = 0; k < n; ++k) {
                const size_t s = (size_t)k * plane + q;
                const float ox = Codec<S>::dec(fld(v.ox, s)), oy = Codec<S>::dec(fld(v.oy, s));
                const float a = Codec<S>::age(fld(v.ta, s), p.t_now, p.dt_ref);
                float cr = 0.0f, cg = 0.0f, cb = 0.0f;
                if (pass == 1) {
                    cr = Codec<S>::dec(fld(v.r, s));
                    cg = Codec<S>::dec(fld(v.g, s));
                    cb = Codec<S>::dec(fld(v.b, s));
                }
                for (int yy = ay0; yy <= ay1; ++yy) {
                    const float dy = splat_offset(qy, yy, oy);
                    if (!(fabsf(dy) <= h)) continue;
                    for (int xx = ax0; xx <= ax1; ++xx) {
                        const float dx = splat_offset(qx, xx, ox);
                        if (!(fabsf(dx) <= h)) continue;
                        const int pe = (yy - y0) * kSTile + (xx - x0);
                        const float Q = splat_q(dx, dy, a, prm[pe]);
                        if (pass == 0) {
                            atomicMin(&qmin[pe], __float_as_uint(Q));
                            atomicAdd(&ncov[pe], 1u);
                            atomicAdd(&units[pe], su);
                        } else {
                            const float w = expf(__uint_as_float(qmin[pe]) - Q);
                            atomicAdd(&accw[pe], w);
                            atomicAdd(&accr[pe], w * cr);
                            atomicAdd(&accg[pe], w * cg);
                            atomicAdd(&accb[pe], w * cb);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (px >= W || py >= H) return;
    const size_t o = (size_t)py * W + px;
    const unsigned n = ncov[e];
    if (n > 0) {
        const float ws = accw[e];
        rgb[o] = accr[e] / ws;
        rgb[plane + o] = accg[e] / ws;
        rgb[2 * plane + o] = accb[e] / ws;
        if (aux) {
            aux[o] = -__uint_as_float(qmin[e]);
            aux[plane + o] = ws;
        }
    } else {
        rgb[o] = rgb[plane + o] = rgb[2 * plane + o] = 0.0f;
        if (aux) aux[o] = aux[plane + o] = 0.0f;
    }
    if (cov) {
        cov[o] = (float)n;
        cov[plane + o] = n > 0 ? ((float)units[e] / (float)n) * 0.00390625f : 0.0f;
    }
}

}  // namespace

int splat_reach(float max_size) { return (int)std::ceil(0.5f * max_size + 0.5f); }

hipError_t launch_splat_sizes(int32_t w, int32_t h, const float *coverage,
                              const afr_splat_params &sp, float *size, hipStream_t st) {
    const SplatRule r{sp.size_default, sp.size_min, sp.size_max, sp.grow, sp.shrink, sp.n_low,
                      sp.n_high};
    const int hw = w * h;
    k_splat_sizes<<<(hw + 255) / 256, 256, 0, st>>>(coverage, coverage ? coverage + hw : nullptr, r,
                                                   hw, size);
    return hipGetLastError();
}

hipError_t launch_scatter(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                          const afr_params &prm, const float *size, float max_size, float *rgb,
                          float *aux, float *coverage, hipStream_t st) {
    const TileGeom tg = geom_of(stats);
    const ScatterParams p{prm.t_now, prm.t_now - buf.t_ref, max_size, splat_reach(max_size)};
    const int gx = (buf.width + kSTile - 1) / kSTile, gy = (buf.height + kSTile - 1) / kSTile;
    if (buf.precision == AFR_FP16)
        k_scatter<__half><<<gx * gy, kSThreads, 0, st>>>(view_of<__half>(buf), p, tg, stats.data,
                                                         size, rgb, aux, coverage, gx);
    else
        k_scatter<float><<<gx * gy, kSThreads, 0, st>>>(view_of<float>(buf), p, tg, stats.data, size,
                                                        rgb, aux, coverage, gx);
    return hipGetLastError();
}

}  // namespace afr
