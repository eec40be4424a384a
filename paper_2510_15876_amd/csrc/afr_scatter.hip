// Scatter form of the reconstruction (Sec. 5.2) with adaptive splat size (Sec. 6.2).
//
// The paper's GPU reconstructor draws every buffered sample as a point splat and lets blending
// accumulate the filter-weighted colour and the weight of every covered pixel. Here each output
// pixel collects the splats that cover it instead: one 256-thread workgroup per 16 x 16 output
// tile, one thread per output pixel, walking the source pixels whose splats can reach it in a fixed
// order (source row, then column, relative to the pixel; slots in rank order) and applying the
// same binary32 footprint test to each of their samples. Nothing is added by more than one thread,
// so every sum has a fixed order and the image is identical from run to run. Two walks keep the
// sums in range, as the two-pass gather does: the first finds the pixel's largest exponent (as the
// smallest Q = -E), its coverage count and splat-size sum; the second adds exp(E - E_max) and its
// colour-weighted terms, one binary32 partial per source pixel added into binary64 totals.
//
// With splats up to 16 px (reach <= 9) the tile's source region, 34 x 34 pixels, has its splat
// sizes and slot counts staged in LDS, and the walk is limited to the reach of the region's
// largest splat; larger splats read them from global memory.
//
//   k_splat_sizes  per pixel: the next image's splat size from this image's coverage map
//   k_scatter      per 16 x 16 output tile: the two walks, then colour, aux and coverage
#include <cmath>

#include "afr_internal.h"

namespace afr {
namespace {

constexpr int kSTile = 16;                 // output tile edge
constexpr int kSThreads = kSTile * kSTile;  // one thread per output pixel
constexpr int kStageReach = 9;              // splats up to 16 px: sizes and counts staged in LDS
constexpr int kStageEdge = kSTile + 2 * kStageReach;

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

// One slot's geometry (offsets, age) and colour.
struct SlotRec {
    float ox, oy, a, r, g, b;
};
template <bool COLOUR>
__device__ inline SlotRec load_rec(const BufView<__half> &v, size_t s, const ScatterParams &p) {
    // the 12-byte record (ox | oy, r | g, b | age_ref)
    const unsigned *w = reinterpret_cast<const unsigned *>(v.ox) + 3 * s;
    const unsigned w0 = w[0], w2 = w[2];
    SlotRec d;
    d.ox = __half2float(__ushort_as_half((unsigned short)(w0 & 0xffffu)));
    d.oy = __half2float(__ushort_as_half((unsigned short)(w0 >> 16)));
    d.a = p.dt_ref + __half2float(__ushort_as_half((unsigned short)(w2 >> 16)));
    d.r = d.g = d.b = 0.0f;
    if (COLOUR) {
        const unsigned w1 = w[1];
        d.r = __half2float(__ushort_as_half((unsigned short)(w1 & 0xffffu)));
        d.g = __half2float(__ushort_as_half((unsigned short)(w1 >> 16)));
        d.b = __half2float(__ushort_as_half((unsigned short)(w2 & 0xffffu)));
    }
    return d;
}
template <bool COLOUR>
__device__ inline SlotRec load_rec(const BufView<float> &v, size_t s, const ScatterParams &p) {
    SlotRec d;
    d.ox = v.ox[s];
    d.oy = v.oy[s];
    d.a = p.t_now - v.ta[s];
    d.r = d.g = d.b = 0.0f;
    if (COLOUR) {
        d.r = v.r[s];
        d.g = v.g[s];
        d.b = v.b[s];
    }
    return d;
}

// Splat size (min(size, max_size)) and slot count of source pixel q; a negative size (or one
// that is not a number once clamped) covers nothing.
struct SrcPix {
    float sz;
    int n;
};
__device__ inline SrcPix src_pix(const float *size, const uint8_t *count, size_t q, float max_size) {
    SrcPix s;
    s.sz = fminf(size[q], max_size);
    s.n = s.sz >= 0.0f ? (int)count[q] : 0;
    return s;
}

template <typename S, bool STAGED>
__global__ __launch_bounds__(kSThreads) void k_scatter(BufView<S> v, ScatterParams p, TileGeom tg,
                                                       const float *__restrict__ stats,
                                                       const float *__restrict__ size,
                                                       float *__restrict__ rgb,
                                                       float *__restrict__ aux,
                                                       float *__restrict__ cov, int gx) {
    constexpr int NS = STAGED ? kStageEdge * kStageEdge : 1;
    __shared__ float s_sz[NS];
    __shared__ unsigned char s_n[NS];
    __shared__ unsigned s_hmax;
    const int W = v.width, H = v.height;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (bid % gx) * kSTile, y0 = (bid / gx) * kSTile;
    const int e = threadIdx.x;
    const int px = x0 + (e % kSTile), py = y0 + (e / kSTile);
    const size_t plane = (size_t)W * H;

    // ---- the walk's reach: the largest splat of the staged region, else max_size --------------
    int re = p.reach;
    if (STAGED) {
        if (e == 0) s_hmax = 0u;
        __syncthreads();
        unsigned hm = 0u;
        for (int r = e; r < NS; r += kSThreads) {
            const int qx = x0 - kStageReach + r % kStageEdge, qy = y0 - kStageReach + r / kStageEdge;
            SrcPix sp{0.0f, 0};
            if (qx >= 0 && qx < W && qy >= 0 && qy < H)
                sp = src_pix(size, v.count, (size_t)qy * W + qx, p.max_size);
            s_sz[r] = sp.sz;
            s_n[r] = (unsigned char)sp.n;
            if (sp.n > 0) hm = max(hm, __float_as_uint(sp.sz));  // sizes >= 0: bit order is order
        }
        if (hm) atomicMax(&s_hmax, hm);
        __syncthreads();
        // q can cover p only if |q - p| <= h + 1/2, h = sz / 2
        re = min(re, (int)floorf(0.5f * __uint_as_float(s_hmax) + 0.5f));
    }
    if (px >= W || py >= H) return;  // no barrier follows

    const int T = (py / tg.tile) * tg.tiles_x + px / tg.tile;
    const float isx = 1.0f / stats[AFR_STAT_SX2 * tg.nt + T];
    const float isy = 1.0f / stats[AFR_STAT_SY2 * tg.nt + T];
    const float kt2 = stats[AFR_STAT_KT2 * tg.nt + T];
    const float4 pr = make_float4(isx, isy, kt2, 0.0f);
    const int dy0 = max(-re, -py), dy1 = min(re, H - 1 - py);
    const int dx0 = max(-re, -px), dx1 = min(re, W - 1 - px);

    auto source = [&](int qx, int qy) -> SrcPix {
        if (STAGED) {
            const int r = (qy - y0 + kStageReach) * kStageEdge + (qx - x0 + kStageReach);
            return SrcPix{s_sz[r], (int)s_n[r]};
        }
        return src_pix(size, v.count, (size_t)qy * W + qx, p.max_size);
    };

    // ---- walk 1: largest exponent, coverage count, size units ------------------------------------
    float qmin = INFINITY;
    unsigned ncov = 0u;
    unsigned long long units = 0ull;  // sizes in 1/256 px, summed exactly
    for (int dy = dy0; dy <= dy1; ++dy) {
        const int qy = py + dy;
        for (int dx = dx0; dx <= dx1; ++dx) {
            const int qx = px + dx;
            const SrcPix sp = source(qx, qy);
            const float h = 0.5f * sp.sz;
            if (sp.n == 0 || (float)abs(dx) - 0.5f > h || (float)abs(dy) - 0.5f > h) continue;
            const unsigned long long su = (unsigned long long)rintf(256.0f * sp.sz);
            const size_t q = (size_t)qy * W + qx;
            for (int k = 0; k < sp.n; ++k) {
                const SlotRec d = load_rec<false>(v, (size_t)k * plane + q, p);
                const float fy = splat_offset(qy, py, d.oy), fx = splat_offset(qx, px, d.ox);
                if (fabsf(fy) <= h && fabsf(fx) <= h) {
                    qmin = fminf(qmin, splat_q(fx, fy, d.a, pr));
                    ++ncov;
                    units += su;
                }
            }
        }
    }
    // ---- walk 2: the weights exp(E - E_max) and the weighted colours -----------------------------
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (ncov > 0u) {
        for (int dy = dy0; dy <= dy1; ++dy) {
            const int qy = py + dy;
            for (int dx = dx0; dx <= dx1; ++dx) {
                const int qx = px + dx;
                const SrcPix sp = source(qx, qy);
                const float h = 0.5f * sp.sz;
                if (sp.n == 0 || (float)abs(dx) - 0.5f > h || (float)abs(dy) - 0.5f > h) continue;
                const size_t q = (size_t)qy * W + qx;
                float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int k = 0; k < sp.n; ++k) {
                    const SlotRec d = load_rec<true>(v, (size_t)k * plane + q, p);
                    const float fy = splat_offset(qy, py, d.oy), fx = splat_offset(qx, px, d.ox);
                    if (fabsf(fy) <= h && fabsf(fx) <= h) {
                        const float w = expf(qmin - splat_q(fx, fy, d.a, pr));
                        part[0] += w;
                        part[1] = fmaf(w, d.r, part[1]);
                        part[2] = fmaf(w, d.g, part[2]);
                        part[3] = fmaf(w, d.b, part[3]);
                    }
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += (double)part[c];
            }
        }
    }
    const size_t o = (size_t)py * W + px;
    if (ncov > 0u) {
        const double inv = 1.0 / acc[0];
        rgb[o] = (float)(acc[1] * inv);
        rgb[plane + o] = (float)(acc[2] * inv);
        rgb[2 * plane + o] = (float)(acc[3] * inv);
        if (aux) {
            aux[o] = -qmin;
            aux[plane + o] = (float)acc[0];
        }
    } else {
        rgb[o] = rgb[plane + o] = rgb[2 * plane + o] = 0.0f;
        if (aux) aux[o] = aux[plane + o] = 0.0f;
    }
    if (cov) {
        cov[o] = (float)ncov;
        cov[plane + o] = ncov > 0u ? ((float)units / (float)ncov) * 0.00390625f : 0.0f;
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
    const bool staged = p.reach <= kStageReach;
    if (buf.precision == AFR_FP16) {
        if (staged)
            k_scatter<__half, true><<<gx * gy, kSThreads, 0, st>>>(
                view_of<__half>(buf), p, tg, stats.data, size, rgb, aux, coverage, gx);
        else
            k_scatter<__half, false><<<gx * gy, kSThreads, 0, st>>>(
                view_of<__half>(buf), p, tg, stats.data, size, rgb, aux, coverage, gx);
    } else {
        if (staged)
            k_scatter<float, true><<<gx * gy, kSThreads, 0, st>>>(
                view_of<float>(buf), p, tg, stats.data, size, rgb, aux, coverage, gx);
        else
            k_scatter<float, false><<<gx * gy, kSThreads, 0, st>>>(
                view_of<float>(buf), p, tg, stats.data, size, rgb, aux, coverage, gx);
    }
    return hipGetLastError();
}

}  // namespace afr
