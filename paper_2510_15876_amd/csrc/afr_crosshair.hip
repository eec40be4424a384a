// Crosshair gradient estimator (Sec. 4.1): the sampler measures gradients on crosshairs (a centre
// sample, four samples one pixel away at the same instant, and an earlier sample at the same
// sub-pixel spot), pushes each crosshair into the per-pixel queue of its deep buffer, and averages
// the queued gradients per tile with the age weights of Sec. 4.
//
//   k_xh_records  one thread per crosshair: gathers its samples' colours from the stream, forms the
//                 three gradients in FP64 and writes a record (centre x, y, t; gx, gy, gt) with -1
//                 marking an undefined gradient and a NaN position for a crosshair without a usable
//                 centre. Records then go through the deep-buffer build (afr_build.hip) unchanged:
//                 the crosshair queue is a deep buffer whose colour planes hold the gradients.
//   k_xh_tiles    one wave per tile: per-lane FP64 sums of omega g and omega over the queued records
//                 of the lane's pixels, a fixed butterfly across the wave, then the extents from the
//                 new gradients and the tile's sample volume (estimated from the sample buffer).
#include "afr_tile_estimate.h"

namespace afr {
namespace {

constexpr int kRecThreads = 256;

struct XhRecords {
    float *x, *y, *t, *gx, *gy, *gt;
};

__device__ inline bool index_ok(int32_t i, int64_t n) { return i >= 0 && (int64_t)i < n; }

__device__ inline double sample_luminance(const afr_samples &s, int32_t i) {
#pragma clang fp contract(off)
    return est::kLumR * (double)s.r[i] + est::kLumG * (double)s.g[i] + est::kLumB * (double)s.b[i];
}

// Mean of |Lc - L_n| over the present neighbours with a finite luminance; -1 if there is none.
__device__ inline double pair_gradient(const afr_samples &s, double lc, int32_t a, int32_t b) {
#pragma clang fp contract(off)
    double sum = 0.0;
    int cnt = 0;
    if (index_ok(a, s.n)) {
        const double l = sample_luminance(s, a);
        if (isfinite(l)) {
            sum += fabs(lc - l);
            ++cnt;
        }
    }
    if (index_ok(b, s.n)) {
        const double l = sample_luminance(s, b);
        if (isfinite(l)) {
            sum += fabs(lc - l);
            ++cnt;
        }
    }
    return cnt ? sum / (double)cnt : -1.0;
}

__global__ __launch_bounds__(kRecThreads) void k_xh_records(afr_samples s, afr_crosshairs xh,
                                                             double dt_floor, XhRecords out) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kRecThreads + threadIdx.x;
    if (i >= xh.n) return;
    const int32_t c = xh.centre[i];
    const double lc = index_ok(c, s.n) ? sample_luminance(s, c) : (double)NAN;
    if (!isfinite(lc)) {  // no usable centre: the build drops the record
        out.x[i] = out.y[i] = out.t[i] = NAN;
        out.gx[i] = out.gy[i] = out.gt[i] = -1.0f;
        return;
    }
    const float tc = s.t[c];
    out.x[i] = s.x[c];
    out.y[i] = s.y[c];
    out.t[i] = tc;
    out.gx[i] = (float)pair_gradient(s, lc, xh.xm[i], xh.xp[i]);
    out.gy[i] = (float)pair_gradient(s, lc, xh.ym[i], xh.yp[i]);
    double gt = -1.0;
    const int32_t o = xh.old[i];
    if (index_ok(o, s.n)) {
        const double l0 = sample_luminance(s, o);
        const double t1 = tc, t0 = s.t[o];
        if (isfinite(l0) && isfinite(t0) && isfinite(t1) && t0 < t1)
            gt = fabs(lc - l0) / fmax(t1 - t0, dt_floor);
    }
    out.gt[i] = (float)gt;
}

struct XhAcc {
    double gx, wx, gy, wy, gt, wt;
};

__global__ __launch_bounds__(kWave) void k_xh_tiles(BufView<float> x, est::EstParams p, TileGeom tg,
                                                     float *stats) {
#pragma clang fp contract(off)
    const int T = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = T % tg.tiles_x, ty = T / tg.tiles_x;
    const int B = tg.tile;
    const int i0 = tx * B, j0 = ty * B;
    const int bw = min(B, x.width - i0), bh = min(B, x.height - j0);
    const size_t plane = (size_t)x.width * x.height;
    XhAcc a{0, 0, 0, 0, 0, 0};
    for (int e = threadIdx.x; e < bw * bh; e += kWave) {
        const size_t px = (size_t)(j0 + e / bw) * x.width + i0 + e % bw;
        const int n = x.count[px];
        for (int k = 0; k < n; ++k) {
            const size_t s = (size_t)k * plane + px;
            const double w = exp(-p.alpha * (p.t_now - (double)x.ta[s]));
            const double gx = x.r[s], gy = x.g[s], gt = x.b[s];
            if (gx >= 0.0) {
                a.gx += w * gx;
                a.wx += w;
            }
            if (gy >= 0.0) {
                a.gy += w * gy;
                a.wy += w;
            }
            if (gt >= 0.0) {
                a.gt += w * gt;
                a.wt += w;
            }
        }
    }
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) {
        a.gx += __shfl_xor(a.gx, m, kWave);
        a.wx += __shfl_xor(a.wx, m, kWave);
        a.gy += __shfl_xor(a.gy, m, kWave);
        a.wy += __shfl_xor(a.wy, m, kWave);
        a.gt += __shfl_xor(a.gt, m, kWave);
        a.wt += __shfl_xor(a.wt, m, kWave);
    }
    if (threadIdx.x != 0) return;
    const double gx = a.wx > 0.0 ? a.gx / a.wx : 0.0;
    const double gy = a.wy > 0.0 ? a.gy / a.wy : 0.0;
    const double gt = a.wt > 0.0 ? a.gt / a.wt : 0.0;
    const int nt = tg.nt;
    const double vol = stats[AFR_STAT_VOL * nt + T];
    double ex2, ey2, sx2, sy2, kt2;
    est::extents(gx, gy, gt, vol, p, ex2, ey2, sx2, sy2, kt2);
    stats[AFR_STAT_GX * nt + T] = (float)gx;
    stats[AFR_STAT_GY * nt + T] = (float)gy;
    stats[AFR_STAT_GT * nt + T] = (float)gt;
    stats[AFR_STAT_EX2 * nt + T] = (float)ex2;
    stats[AFR_STAT_EY2 * nt + T] = (float)ey2;
    stats[AFR_STAT_SX2 * nt + T] = (float)sx2;
    stats[AFR_STAT_SY2 * nt + T] = (float)sy2;
    stats[AFR_STAT_KT2 * nt + T] = (float)kt2;
}

}  // namespace

size_t crosshair_ws_bytes(int64_t n, int32_t w, int32_t h) {
    return 6 * align_up((size_t)(n > 0 ? n : 1) * sizeof(float)) + build_ws_bytes(n, w, h);
}

hipError_t launch_crosshair_build(const afr_samples &s, const afr_crosshairs &xh,
                                  const afr_params &prm, const afr_deep_buffer &out, void *ws,
                                  unsigned long long *dropped_or_null, hipStream_t st) {
    const size_t arr = align_up((size_t)(xh.n > 0 ? xh.n : 1) * sizeof(float));
    char *p = static_cast<char *>(ws);
    XhRecords rec;
    float **f[6] = {&rec.x, &rec.y, &rec.t, &rec.gx, &rec.gy, &rec.gt};
    for (int i = 0; i < 6; ++i) *f[i] = reinterpret_cast<float *>(p + i * arr);
    void *bws = p + 6 * arr;
    const BuildWs w = build_ws_carve(bws, xh.n, out.width, out.height);
    if (xh.n > 0) {
        const int64_t nb = (xh.n + kRecThreads - 1) / kRecThreads;
        k_xh_records<<<(unsigned)nb, kRecThreads, 0, st>>>(s, xh, (double)prm.dt_floor, rec);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    afr_samples r{};
    r.x = rec.x;
    r.y = rec.y;
    r.t = rec.t;
    r.r = rec.gx;
    r.g = rec.gy;
    r.b = rec.gt;
    r.n = xh.n;
    return launch_build(r, out, w, dropped_or_null ? dropped_or_null : w.dropped_internal, st,
                        nullptr);
}

hipError_t launch_crosshair_estimate(const afr_deep_buffer &buf, const afr_deep_buffer &xbuf,
                                     const afr_params &prm, const afr_tile_stats &out,
                                     hipStream_t st) {
    hipError_t e = launch_estimate(buf, prm, out, st);
    if (e != hipSuccess) return e;
    const TileGeom tg = geom_of(out);
    k_xh_tiles<<<tg.nt, kWave, 0, st>>>(view_of<float>(xbuf), est_params(xbuf, prm), tg, out.data);
    return hipGetLastError();
}

}  // namespace afr
