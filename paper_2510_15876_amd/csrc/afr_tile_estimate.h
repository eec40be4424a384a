// Per-tile statistics (Sec. 4, 4.1, 5.1) as a device routine shared by afr_estimate_gradients and the
// batched persistent kernel: one 64-lane wave evaluates one statistics tile.
//
// Phase 1 visits every pixel of the tile and its one-pixel halo once, reading the pixel's slots a
// single time and accumulating in FP64: the age-weighted mean luminance (needed by the neighbours'
// spatial differences), the weighted second moment, the new-half / old-half means that give the
// temporal difference quotient, and the age sum. Results go to LDS. Phase 2 gives each tile pixel
// its spatial gradients from the LDS neighbours and folds all per-pixel terms into one accumulator
// per lane; lanes are combined by a fixed-shape butterfly within the wave and in wave order across
// waves, so the statistics are deterministic. Luminance variance merges per-pixel (weight, mean, M2)
// triples with the pairwise form of Welford's update.
//
// FP64 here is a precision choice: spatial gradients are differences of neighbouring means, and in
// flat regions FP32 rounding of those means would move the filter widths by ~1e-4 relative. The
// work is small next to the gather (one pass over the slots, FP64 FMA is full rate on CDNA).
#pragma once
#include "afr_internal.h"

namespace afr {
namespace est {

struct EstParams {
    double alpha, t_now, dt_ref, dt_floor, age_floor, g_floor, sigma, tau, e_min, e_max;
};

// Rec. 709 luminance weights of linear RGB.
constexpr double kLumR = 0.2126, kLumG = 0.7152, kLumB = 0.0722;

struct Acc {
    double gx, wx, gy, wy, gt, wt;  // sums of Omega_p G(p) and Omega_p over defined pixels
    double n, sa;                   // slot count and age sum
    double w, mean, m2;             // age-weighted luminance: weight, mean, sum of squared deviations
};

__device__ inline Acc acc_zero() { return Acc{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}; }

__device__ inline Acc acc_combine(const Acc &a, const Acc &b) {
    Acc c;
    c.gx = a.gx + b.gx;
    c.wx = a.wx + b.wx;
    c.gy = a.gy + b.gy;
    c.wy = a.wy + b.wy;
    c.gt = a.gt + b.gt;
    c.wt = a.wt + b.wt;
    c.n = a.n + b.n;
    c.sa = a.sa + b.sa;
    if (b.w == 0.0) {
        c.w = a.w;
        c.mean = a.mean;
        c.m2 = a.m2;
    } else if (a.w == 0.0) {
        c.w = b.w;
        c.mean = b.mean;
        c.m2 = b.m2;
    } else {
        c.w = a.w + b.w;
        const double d = b.mean - a.mean;
        c.mean = a.mean + d * (b.w / c.w);
        c.m2 = a.m2 + b.m2 + d * d * (a.w * b.w / c.w);
    }
    return c;
}

__device__ inline double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, kWave); }

__device__ inline Acc acc_shfl_xor(const Acc &a, int m) {
    Acc o;
    o.gx = shfl_xor_d(a.gx, m);
    o.wx = shfl_xor_d(a.wx, m);
    o.gy = shfl_xor_d(a.gy, m);
    o.wy = shfl_xor_d(a.wy, m);
    o.gt = shfl_xor_d(a.gt, m);
    o.wt = shfl_xor_d(a.wt, m);
    o.n = shfl_xor_d(a.n, m);
    o.sa = shfl_xor_d(a.sa, m);
    o.w = shfl_xor_d(a.w, m);
    o.mean = shfl_xor_d(a.mean, m);
    o.m2 = shfl_xor_d(a.m2, m);
    return o;
}

// Filter extents from tile gradients and volume; see afr_estimate_gradients in afr.h.
__device__ inline void extents(double gx, double gy, double gt, double vol, const EstParams &p,
                               double &ex2, double &ey2, double &sx2, double &sy2, double &kt2) {
    const double hx = sqrt(gx * gx + p.g_floor * p.g_floor);
    const double hy = sqrt(gy * gy + p.g_floor * p.g_floor);
    const double u = p.tau * gt;
    ex2 = ey2 = kt2 = 0.0;
    if (u != 0.0) {
        const double cx = cbrt(vol * hy * u / (hx * hx));
        const double cy = cbrt(vol * hx * u / (hy * hy));
        const double ck = cbrt(u * u / (vol * hx * hy));
        ex2 = cx * cx;
        ey2 = cy * cy;
        kt2 = ck * ck;
    }
    const double zx = p.sigma * p.sigma * ex2, zy = p.sigma * p.sigma * ey2;
    const double n2 = p.e_min * p.e_min;
    if (isinf(p.e_max)) {
        sx2 = n2 + zx;
        sy2 = n2 + zy;
    } else {
        const double m2 = p.e_max * p.e_max;
        sx2 = n2 + zx * m2 / (m2 + zx);
        sy2 = n2 + zy * m2 / (m2 + zy);
    }
}

// LDS scratch of one tile evaluation for tiles of edge <= TB (the tile and its one-pixel halo).
template <int TB>
struct Smem {
    static constexpr int kHalo = (TB + 2) * (TB + 2);
    double lbar[kHalo], om[kHalo], gt[kHalo], sa[kHalo], m2[kHalo];
    int n[kHalo];
    Acc wave[256 / kWave];
};

// Evaluates tile T (edge tg.tile <= TB) with the calling workgroup (blockDim.x threads, a multiple
// of 64, <= 256, with 2 * blockDim.x >= (tile + 2)^2) and writes its statistics. If tparams is not NULL, thread 0 also stores (sx2, sy2, kt2) there (LDS),
// visible to the workgroup after the caller's next barrier.
template <typename S, int TB>
__device__ void estimate_tile(const BufView<S> &v, const EstParams &p, const TileGeom &tg, int T,
                              float *stats, Smem<TB> &sm, float *tparams) {
    double *s_lbar = sm.lbar, *s_om = sm.om, *s_gt = sm.gt, *s_sa = sm.sa, *s_m2 = sm.m2;
    int *s_n = sm.n;
    Acc *s_wave = sm.wave;
    const int B = tg.tile;
    const int i0 = (T % tg.tiles_x) * B, j0 = (T / tg.tiles_x) * B;
    const int bw = min(B, v.width - i0), bh = min(B, v.height - j0);
    const int rw = bw + 2, rh = bh + 2;
    const size_t hw = (size_t)v.width * v.height;

    // Phase 1: per-pixel moments over the tile and its one-pixel halo. Each lane takes up to
    // kItems pixels of the region; the slot planes are visited in chunks of kChunk, and every load
    // of a chunk (all items, all planes of the chunk) is issued before any of them is used, so a
    // lane waits for memory once per chunk instead of once per slot. Per pixel the slots are still
    // added in rank order, so the sums do not depend on the chunking.
    constexpr int kItems = 2, kChunk = 8;
    const int nh = rw * rh;
    int px_[kItems], n_[kItems];
    int kmax = 0;
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int h = threadIdx.x + it * blockDim.x;
        const int x = i0 - 1 + h % rw, y = j0 - 1 + h / rw;
        const bool live = h < nh && x >= 0 && x < v.width && y >= 0 && y < v.height;
        px_[it] = live ? y * v.width + x : 0;
        n_[it] = live ? v.count[px_[it]] : 0;
        kmax = max(kmax, n_[it]);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, kWave));
    const size_t bytes = hw * sizeof(S);
    double s0[kItems], s1[kItems], s2[kItems], ln[kItems], lo[kItems], an[kItems], ao[kItems],
        sa_[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it)
        s0[it] = s1[it] = s2[it] = ln[it] = lo[it] = an[it] = ao[it] = sa_[it] = 0.0;
    for (int k0 = 0; k0 < kmax; k0 += kChunk) {
        S cr[kChunk][kItems], cg[kChunk][kItems], cb[kChunk][kItems], ct[kChunk][kItems];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            const int k = min(k0 + j, v.k - 1);  // planes past K are never used
            const size_t base = (size_t)k * hw;
            const auto rr = plane_rsrc(v.r + base, bytes), rg = plane_rsrc(v.g + base, bytes);
            const auto rb = plane_rsrc(v.b + base, bytes), rt = plane_rsrc(v.ta + base, bytes);
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                const unsigned off = (unsigned)px_[it] * (unsigned)sizeof(S);
                cr[j][it] = plane_load<S>(rr, off);
                cg[j][it] = plane_load<S>(rg, off);
                cb[j][it] = plane_load<S>(rb, off);
                ct[j][it] = plane_load<S>(rt, off);
            }
        }
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            const int k = k0 + j;
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                if (k < n_[it]) {
                    const double L = kLumR * (double)Codec<S>::dec(cr[j][it]) +
                                     kLumG * (double)Codec<S>::dec(cg[j][it]) +
                                     kLumB * (double)Codec<S>::dec(cb[j][it]);
                    const double a = Codec<S>::age64(ct[j][it], p.t_now, p.dt_ref);
                    const double w = (double)expf((float)(-p.alpha * a));
                    s0[it] += w;
                    s1[it] += w * L;
                    s2[it] += w * L * L;
                    sa_[it] += a;
                    if (k < (n_[it] + 1) / 2) {
                        ln[it] += L;
                        an[it] += a;
                    } else {
                        lo[it] += L;
                        ao[it] += a;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int h = threadIdx.x + it * blockDim.x;
        if (h >= nh) continue;
        const int n = n_[it];
        double om = 0.0, lb = 0.0, gt = -1.0, m2 = 0.0;
        if (n > 0) {
            om = s0[it];
            lb = s1[it] / s0[it];
            m2 = fmax(s2[it] - s1[it] * lb, 0.0);
        }
        if (n >= 2) {
            const int half = (n + 1) / 2;
            const double dn = half, dd = n - half;
            gt = fabs(ln[it] / dn - lo[it] / dd) / fmax(ao[it] / dd - an[it] / dn, p.dt_floor);
        }
        s_n[h] = n;
        s_om[h] = om;
        s_lbar[h] = lb;
        s_gt[h] = gt;
        s_sa[h] = sa_[it];
        s_m2[h] = m2;
    }
    __syncthreads();

    // Phase 2: per tile pixel, spatial gradients from LDS neighbours, then fold into Acc.
    Acc acc = acc_zero();
    for (int e = threadIdx.x; e < bw * bh; e += blockDim.x) {
        const int h = (e / bw + 1) * rw + (e % bw + 1);
        const int n = s_n[h];
        if (n == 0) continue;
        const double lb = s_lbar[h], om = s_om[h];
        double sx = 0.0, sy = 0.0;
        int nx = 0, ny = 0;
        if (s_n[h - 1]) { sx += fabs(lb - s_lbar[h - 1]); ++nx; }
        if (s_n[h + 1]) { sx += fabs(lb - s_lbar[h + 1]); ++nx; }
        if (s_n[h - rw]) { sy += fabs(lb - s_lbar[h - rw]); ++ny; }
        if (s_n[h + rw]) { sy += fabs(lb - s_lbar[h + rw]); ++ny; }
        Acc a = acc_zero();
        if (nx) { a.gx = om * (sx / nx); a.wx = om; }
        if (ny) { a.gy = om * (sy / ny); a.wy = om; }
        if (s_gt[h] >= 0.0) { a.gt = om * s_gt[h]; a.wt = om; }
        a.n = n;
        a.sa = s_sa[h];
        a.w = om;
        a.mean = lb;
        a.m2 = s_m2[h];
        acc = acc_combine(acc, a);
    }
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) acc = acc_combine(acc, acc_shfl_xor(acc, m));
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) s_wave[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
    Acc t = s_wave[0];
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) t = acc_combine(t, s_wave[w]);

    const double gx = t.wx > 0.0 ? t.gx / t.wx : 0.0;
    const double gy = t.wy > 0.0 ? t.gy / t.wy : 0.0;
    const double gt = t.wt > 0.0 ? t.gt / t.wt : 0.0;
    const double area = (double)bw * bh;
    const double vol = t.n > 0.0 ? area * 2.0 * fmax(t.sa / t.n, p.age_floor) / t.n : INFINITY;
    const double var = t.w > 0.0 ? t.m2 / t.w : 0.0;
    const double lmean = t.w > 0.0 ? t.mean : 0.0;
    double ex2, ey2, sx2, sy2, kt2;
    extents(gx, gy, gt, vol, p, ex2, ey2, sx2, sy2, kt2);
    const int nt = tg.nt;
    stats[AFR_STAT_GX * nt + T] = (float)gx;
    stats[AFR_STAT_GY * nt + T] = (float)gy;
    stats[AFR_STAT_GT * nt + T] = (float)gt;
    stats[AFR_STAT_VOL * nt + T] = (float)vol;
    stats[AFR_STAT_VAR * nt + T] = (float)var;
    stats[AFR_STAT_LMEAN * nt + T] = (float)lmean;
    stats[AFR_STAT_EX2 * nt + T] = (float)ex2;
    stats[AFR_STAT_EY2 * nt + T] = (float)ey2;
    stats[AFR_STAT_SX2 * nt + T] = (float)sx2;
    stats[AFR_STAT_SY2 * nt + T] = (float)sy2;
    stats[AFR_STAT_KT2 * nt + T] = (float)kt2;
    if (tparams) {
        tparams[0] = (float)sx2;
        tparams[1] = (float)sy2;
        tparams[2] = (float)kt2;
    }
    }
    __syncthreads();  // the LDS scratch may be reused by the caller after this point
}

}  // namespace est

// Estimator constants of a call (defined with afr_estimate_gradients).
est::EstParams est_params(const afr_deep_buffer &buf, const afr_params &prm);

}  // namespace afr
