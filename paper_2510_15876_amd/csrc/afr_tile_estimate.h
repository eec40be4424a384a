// Per-tile statistics (Sec. 4, 4.1, 5.1): device routines shared by afr_estimate_gradients and the
// batched persistent kernel.
//
// Phase 1 visits every pixel of a region (tiles plus a one-pixel halo) once, reading the pixel's
// slots a single time in rank order and accumulating in FP64: the age-weighted mean luminance
// (needed by the neighbours' spatial differences), the weighted second moment, the new-half /
// old-half means that give the temporal difference quotient, and the age sum. Results go to LDS.
// Phase 2 gives each tile pixel its spatial gradients from the LDS neighbours and reduces a tile
// with 16 lanes of one wave (so that a wave reduces four tiles at once): lane g folds the pixels
// e = g, g + 16, ... in increasing order, and the 16 partial accumulators are combined by a fixed
// tree (g with g + 8, then + 4, + 2, + 1, the lower first). Luminance variance merges per-pixel
// (weight, mean, M2) triples with the pairwise form of Welford's update.
//
// Two drivers share these routines: a strip kernel (afr_estimate_gradients, tiles of edge <= 8)
// where a workgroup covers a 32-pixel-wide strip of tiles, so that each wave reads whole image rows
// per slot plane, and a per-tile routine (tiles up to 16 px, and the batched kernel). Floating-point
// contraction is off in every routine here, so a pixel's moments and a tile's reduction round the
// same way in either driver and the statistics are identical bit for bit.
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
#pragma clang fp contract(off)
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
        // pairwise (Chan et al.) form of Welford's update, one division
        c.w = a.w + b.w;
        const double r = 1.0 / c.w;
        const double d = b.mean - a.mean;
        c.mean = a.mean + d * (b.w * r);
        c.m2 = a.m2 + b.m2 + d * d * (a.w * b.w * r);
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

// The accumulator of lane src, in every lane.
__device__ inline Acc acc_shfl(const Acc &a, int src) {
    Acc o;
    o.gx = __shfl(a.gx, src, kWave);
    o.wx = __shfl(a.wx, src, kWave);
    o.gy = __shfl(a.gy, src, kWave);
    o.wy = __shfl(a.wy, src, kWave);
    o.gt = __shfl(a.gt, src, kWave);
    o.wt = __shfl(a.wt, src, kWave);
    o.n = __shfl(a.n, src, kWave);
    o.sa = __shfl(a.sa, src, kWave);
    o.w = __shfl(a.w, src, kWave);
    o.mean = __shfl(a.mean, src, kWave);
    o.m2 = __shfl(a.m2, src, kWave);
    return o;
}

// Filter extents from tile gradients and volume; see afr_estimate_gradients in afr.h. V = +inf with
// u > 0 (a tile with crosshair gradients but no buffered samples) gives ex2 = ey2 = +inf and takes
// the clamp's limit, the ceiling e_min^2 + e_max^2, and kt2 = 0.
__device__ inline void extents(double gx, double gy, double gt, double vol, const EstParams &p,
                               double &ex2, double &ey2, double &sx2, double &sy2, double &kt2) {
#pragma clang fp contract(off)
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
        sx2 = n2 + (isinf(zx) ? m2 : zx * m2 / (m2 + zx));
        sy2 = n2 + (isinf(zy) ? m2 : zy * m2 / (m2 + zy));
    }
}

// ---- per-pixel moments (phase 1) ---------------------------------------------------------------

struct PixAcc {
    double s0, s1, s2, ln, lo, an, sa;  // ln, lo: luminance of the newer and older half; an: newer ages
};

__device__ inline PixAcc pix_zero() { return PixAcc{0, 0, 0, 0, 0, 0, 0}; }

// Age weight e^{-alpha a} (Sec. 4) over the FP64 exponent range: with x = alpha a log2(e) = n + f,
// n an integer and f in [0, 1), the weight is 2^-f (float32, within 2 ulp) scaled exactly by 2^-n.
// A float32 exponential of -alpha a would reach zero past about 30 s of age at alpha = 3.47 / s
// (leaving a pixel whose samples are all that old with no weight); this form holds the weight's
// relative precision down to 2^-1022 (ages of about 200 s).
__device__ inline double age_weight(double alpha, double a) {
#pragma clang fp contract(off)
    const double x = alpha * a * 1.4426950408889634;
    const double n = floor(x);
    const int e = (int)fmin(fmax(-n, -2000.0), 2000.0);  // -n, clamped
    // n - x lies in (-1, 0]: the hardware exponential needs no range handling there
    return ldexp((double)__builtin_amdgcn_exp2f((float)(n - x)), e);
}

// Adds slot k (rank order) of a pixel with n slots: colour (r, g, b) and stored age field ta. The
// older half's age sum is the total minus the newer half's (pix_store); the luminance sums of both
// halves are kept, so that a pixel whose samples share one luminance has a temporal difference of
// exactly zero.
template <typename S>
__device__ inline void pix_add(PixAcc &m, const EstParams &p, S r, S g, S b, S ta, int k, int n) {
#pragma clang fp contract(off)
    const double L = fma(kLumB, (double)Codec<S>::dec(b),
                         fma(kLumG, (double)Codec<S>::dec(g), kLumR * (double)Codec<S>::dec(r)));
    const double a = Codec<S>::age64(ta, p.t_now, p.dt_ref);
    const double w = age_weight(p.alpha, a);
    const double wl = w * L;
    m.s0 += w;
    m.s1 += wl;
    m.s2 = fma(wl, L, m.s2);
    m.sa += a;
    // the half is chosen by exact 0/1 multipliers: fma(1, x, s) = s + x and fma(0, x, s) = s (the
    // sums start at +0 and are never -0), three fused multiply-adds instead of selects and adds
    const bool newer = k < (n + 1) / 2;
    const double in_new = newer ? 1.0 : 0.0, in_old = newer ? 0.0 : 1.0;
    m.ln = fma(in_new, L, m.ln);
    m.lo = fma(in_old, L, m.lo);
    m.an = fma(in_new, a, m.an);
}

// Region scratch: per-pixel (count, Omega, mean luminance, temporal gradient or -1, age sum, M2)
// in LDS, row-major with a given pitch.
struct Region {
    double *lbar, *om, *gt, *sa, *m2;
    int *n;
};

__device__ inline void pix_store(const Region &rg, int h, const PixAcc &m, int n, double dt_floor) {
#pragma clang fp contract(off)
    double om = 0.0, lb = 0.0, gt = -1.0, m2 = 0.0;
    if (n > 0) {
        om = m.s0;
        lb = m.s1 / m.s0;
        m2 = fmax(m.s2 - m.s1 * lb, 0.0);
    }
    if (n >= 2) {
        const int half = (n + 1) / 2;
        const double dn = half, dd = n - half;
        gt = fabs(m.ln / dn - m.lo / dd) / fmax((m.sa - m.an) / dd - m.an / dn, dt_floor);
    }
    rg.n[h] = n;
    rg.om[h] = om;
    rg.lbar[h] = lb;
    rg.gt[h] = gt;
    rg.sa[h] = m.sa;
    rg.m2[h] = m2;
}

// ---- per-tile reduction (phase 2) ---------------------------------------------------------------

// Accumulator of region pixel h (pitch rp) with its spatial gradients from the four neighbours.
__device__ inline Acc pixel_acc(const Region &rg, int h, int rp) {
#pragma clang fp contract(off)
    Acc a = acc_zero();
    const int n = rg.n[h];
    if (n == 0) return a;
    const double lb = rg.lbar[h], om = rg.om[h];
    double sx = 0.0, sy = 0.0;
    int nx = 0, ny = 0;
    if (rg.n[h - 1]) { sx += fabs(lb - rg.lbar[h - 1]); ++nx; }
    if (rg.n[h + 1]) { sx += fabs(lb - rg.lbar[h + 1]); ++nx; }
    if (rg.n[h - rp]) { sy += fabs(lb - rg.lbar[h - rp]); ++ny; }
    if (rg.n[h + rp]) { sy += fabs(lb - rg.lbar[h + rp]); ++ny; }
    if (nx) { a.gx = om * (sx / nx); a.wx = om; }
    if (ny) { a.gy = om * (sy / ny); a.wy = om; }
    if (rg.gt[h] >= 0.0) { a.gt = om * rg.gt[h]; a.wt = om; }
    a.n = n;
    a.sa = rg.sa[h];
    a.w = om;
    a.mean = lb;
    a.m2 = rg.m2[h];
    return a;
}

// Lanes that reduce one tile: an aligned segment of a wave.
constexpr int kGroups = 16;

// Reduces a bw x bh tile whose top-left region pixel is h0 with the calling lane's 16-lane segment
// (g = lane mod 16): group g folds the pixels e = g, g + 16, ... in increasing order, then the
// groups are combined by the tree g + 8, g + 4, g + 2, g + 1 (the lower group first). Every lane
// of the wave must call this together (the segments may reduce different tiles); every lane of a
// segment receives its tile's sum.
__device__ inline Acc segment_tile_acc(const Region &rg, int h0, int rp, int bw, int bh, int lane) {
#pragma clang fp contract(off)
    Acc acc = acc_zero();
    for (int e = lane % kGroups; e < bw * bh; e += kGroups)
        acc = acc_combine(acc, pixel_acc(rg, h0 + (e / bw) * rp + e % bw, rp));
    // A lane g < m of the segment combines its value with lane g + m's, which holds the tree over
    // its own subtree after the previous level; lanes g >= m compute values that are never read.
#pragma unroll
    for (int m = kGroups / 2; m > 0; m >>= 1) acc = acc_combine(acc, acc_shfl_xor(acc, m));
    return acc_shfl(acc, lane & ~(kGroups - 1));
}

// Tile statistics from the tile's accumulator, evaluated by the 16 lanes of a segment (every lane
// of the wave calls it; `write` false for segments without a tile): lanes g = 0, 1, 2 of the
// segment take the three cube roots of the extents at once (the same operations as extents()), and
// lane 0 of the segment writes the stats planes and, if tparams is not NULL, (sx2, sy2, kt2) to
// tparams.
__device__ inline void tile_finish(const Acc &t, const EstParams &p, const TileGeom &tg, int T,
                                   int bw, int bh, float *stats, float *tparams, int lane,
                                   bool write) {
#pragma clang fp contract(off)
    const int g = lane % kGroups, base = lane - g;
    const double gx = t.wx > 0.0 ? t.gx / t.wx : 0.0;
    const double gy = t.wy > 0.0 ? t.gy / t.wy : 0.0;
    const double gt = t.wt > 0.0 ? t.gt / t.wt : 0.0;
    const double area = (double)bw * bh;
    const double vol = t.n > 0.0 ? area * 2.0 * fmax(t.sa / t.n, p.age_floor) / t.n : INFINITY;
    const double var = t.w > 0.0 ? t.m2 / t.w : 0.0;
    const double lmean = t.w > 0.0 ? t.mean : 0.0;
    const double hx = sqrt(gx * gx + p.g_floor * p.g_floor);
    const double hy = sqrt(gy * gy + p.g_floor * p.g_floor);
    const double u = p.tau * gt;
    double ex2 = 0.0, ey2 = 0.0, kt2 = 0.0;
    {  // every lane takes part in the shuffles; u is uniform over a segment
        const double num = g == 0 ? vol * hy * u : (g == 1 ? vol * hx * u : u * u);
        const double den = g == 0 ? hx * hx : (g == 1 ? hy * hy : vol * hx * hy);
        const double c = u != 0.0 && g < 3 ? cbrt(num / den) : 0.0;
        const double cx = __shfl(c, base, kWave), cy = __shfl(c, base + 1, kWave);
        const double ck = __shfl(c, base + 2, kWave);
        if (u != 0.0) {
            ex2 = cx * cx;
            ey2 = cy * cy;
            kt2 = ck * ck;
        }
    }
    const double zx = p.sigma * p.sigma * ex2, zy = p.sigma * p.sigma * ey2;
    const double n2 = p.e_min * p.e_min;
    double sx2, sy2;
    if (isinf(p.e_max)) {
        sx2 = n2 + zx;
        sy2 = n2 + zy;
    } else {
        const double m2 = p.e_max * p.e_max;
        sx2 = n2 + (isinf(zx) ? m2 : zx * m2 / (m2 + zx));
        sy2 = n2 + (isinf(zy) ? m2 : zy * m2 / (m2 + zy));
    }
    if (g != 0 || !write) return;
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

// Holds a loaded value in place: an empty asm statement that consumes (and nominally rewrites) it.
// A slot's fields are used only under the test k < n, so without this the compiler sinks each load
// into its test and the lane then waits for memory once per slot; placed after the last load of a
// chunk it keeps every load of the chunk ahead of the first wait.
__device__ inline void hold(unsigned &w) { asm volatile("" : "+v"(w)); }

// Phase 1 over the region pixels h = threadIdx.x + it * blockDim.x (it < ITEMS, h < nh) of a region
// with origin (x0, y0) and pitch rp: the slot planes are visited in chunks of KC, and every load of
// a chunk (all items, all planes of the chunk) is issued before any is used, so a lane waits for
// memory once per chunk. Per pixel the slots are still added in rank order.
template <typename S, int ITEMS, int KC>
__device__ inline void region_moments(const BufView<S> &v, const EstParams &p, const Region &rg,
                                      int x0, int y0, int rp, int nh) {
    const size_t hw = (size_t)v.width * v.height;
    int px_[ITEMS], n_[ITEMS];
    int kmax = 0;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int h = threadIdx.x + it * blockDim.x;
        const int x = x0 + h % rp, y = y0 + h / rp;
        const bool live = h < nh && x >= 0 && x < v.width && y >= 0 && y < v.height;
        px_[it] = live ? y * v.width + x : 0;
        n_[it] = live ? v.count[px_[it]] : 0;
        kmax = max(kmax, n_[it]);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, kWave));
    PixAcc m[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) m[it] = pix_zero();
    // raw 32-bit words of each slot: binary16 (r | g, b | age_ref), binary32 (r, g, b, t)
    constexpr int NW = std::is_same<S, __half>::value ? 2 : 4;
    using Chunk = unsigned[KC][ITEMS][NW];
    auto load = [&](Chunk &raw, int k0) {
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int k = min(k0 + j, v.k - 1);  // planes past K are never used
            if constexpr (std::is_same<S, __half>::value) {
                const size_t bytes = hw * Slots<__half>::kBytes;
                const auto rs = plane_rsrc(v.ox + (size_t)k * hw * Slots<__half>::kStride, bytes);
#pragma unroll
                for (int it = 0; it < ITEMS; ++it) {
                    const unsigned off = (unsigned)px_[it] * Slots<__half>::kBytes + 4u;
                    const uint2 w = load_u32x2(rs, off);
                    raw[j][it][0] = w.x;
                    raw[j][it][1] = w.y;
                }
            } else {
                const size_t base = (size_t)k * hw, bytes = hw * sizeof(S);
                const auto rr = plane_rsrc(v.r + base, bytes), rg_ = plane_rsrc(v.g + base, bytes);
                const auto rb = plane_rsrc(v.b + base, bytes), rt = plane_rsrc(v.ta + base, bytes);
#pragma unroll
                for (int it = 0; it < ITEMS; ++it) {
                    const unsigned off = (unsigned)px_[it] * (unsigned)sizeof(S);
                    raw[j][it][0] = __builtin_amdgcn_raw_buffer_load_b32(rr, off, 0, 0);
                    raw[j][it][1] = __builtin_amdgcn_raw_buffer_load_b32(rg_, off, 0, 0);
                    raw[j][it][2] = __builtin_amdgcn_raw_buffer_load_b32(rb, off, 0, 0);
                    raw[j][it][3] = __builtin_amdgcn_raw_buffer_load_b32(rt, off, 0, 0);
                }
            }
        }
    };
    auto consume = [&](Chunk &raw, int k0) {
#pragma unroll
        for (int j = 0; j < KC; ++j)
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
#pragma unroll
                for (int f = 0; f < NW; ++f) hold(raw[j][it][f]);
#pragma unroll
        for (int j = 0; j < KC; ++j)
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) {
                if (k0 + j >= n_[it]) continue;
                S cr, cg, cb, ct;
                if constexpr (std::is_same<S, __half>::value) {
                    cr = __ushort_as_half((unsigned short)(raw[j][it][0] & 0xffffu));
                    cg = __ushort_as_half((unsigned short)(raw[j][it][0] >> 16));
                    cb = __ushort_as_half((unsigned short)(raw[j][it][1] & 0xffffu));
                    ct = __ushort_as_half((unsigned short)(raw[j][it][1] >> 16));
                } else {
                    cr = __uint_as_float(raw[j][it][0]);
                    cg = __uint_as_float(raw[j][it][1]);
                    cb = __uint_as_float(raw[j][it][2]);
                    ct = __uint_as_float(raw[j][it][3]);
                }
                pix_add<S>(m[it], p, cr, cg, cb, ct, k0 + j, n_[it]);
            }
    };
    // two chunks in flight: the next chunk's loads are issued before the current one is consumed
    Chunk ca, cb;
    if (kmax > 0) load(ca, 0);
    for (int k0 = 0; k0 < kmax; k0 += 2 * KC) {
        load(cb, k0 + KC);
        consume(ca, k0);
        load(ca, k0 + 2 * KC);
        consume(cb, k0 + KC);
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int h = threadIdx.x + it * blockDim.x;
        if (h < nh) pix_store(rg, h, m[it], n_[it], p.dt_floor);
    }
}

// ---- per-tile driver ----------------------------------------------------------------------------

// LDS scratch of one tile evaluation for tiles of edge <= TB (the tile and its one-pixel halo).
template <int TB>
struct Smem {
    static constexpr int kHalo = (TB + 2) * (TB + 2);
    double lbar[kHalo], om[kHalo], gt[kHalo], sa[kHalo], m2[kHalo];
    int n[kHalo];
};

// Evaluates tile T (edge tg.tile <= TB) with the calling workgroup (blockDim.x threads, a multiple
// of 64, <= 256, with 2 * blockDim.x >= (tile + 2)^2) and writes its statistics. If tparams is not
// NULL, thread 0 also stores (sx2, sy2, kt2) there (LDS), visible to the workgroup after the
// caller's next barrier.
template <typename S, int TB>
__device__ void estimate_tile(const BufView<S> &v, const EstParams &p, const TileGeom &tg, int T,
                              float *stats, Smem<TB> &sm, float *tparams) {
    const Region rg{sm.lbar, sm.om, sm.gt, sm.sa, sm.m2, sm.n};
    const int B = tg.tile;
    const int i0 = (T % tg.tiles_x) * B, j0 = (T / tg.tiles_x) * B;
    const int bw = min(B, v.width - i0), bh = min(B, v.height - j0);
    const int rw = bw + 2, rh = bh + 2;
    // four slot planes per load chunk: the batched kernel, which runs this routine and the gather in
    // one wave, keeps its register count (and so its waves per SIMD) down (3.86 -> 3.77 ms per batch)
    region_moments<S, 2, 4>(v, p, rg, i0 - 1, j0 - 1, rw, rw * rh);
    __syncthreads();
    if (threadIdx.x < kWave) {  // the first wave; its first segment's result is written
        const int lane = threadIdx.x;
        const Acc t = segment_tile_acc(rg, rw + 1, rw, bw, bh, lane);
        tile_finish(t, p, tg, T, bw, bh, stats, tparams, lane, lane < kGroups);
    }
    __syncthreads();  // the LDS scratch may be reused by the caller after this point
}

// ---- strip driver (tiles of edge <= 8) ----------------------------------------------------------

// A strip of TILES 8 px tiles (fewer when tiles are smaller: 8 TILES pixels wide) of one tile row,
// evaluated by a workgroup of 64 TILES threads. The region is the strip plus a one-pixel halo.
template <int TILES>
struct Strip {
    static constexpr int THREADS = 64 * TILES;
    static constexpr int W = 8 * TILES;                             // pixels
    static constexpr int REGION = (W + 2) * (8 + 2);                // region pixels
    static constexpr int ITEMS = (REGION + THREADS - 1) / THREADS;  // per thread
};

template <int TILES>
struct StripSmem {
    static constexpr int N = Strip<TILES>::REGION;
    double lbar[N], om[N], gt[N], sa[N], m2[N];
    int n[N];
};

// Tiles per strip and strips per tile row for tile edge B <= 8.
__host__ __device__ inline int strip_tiles(int B, int tiles) { return 8 * tiles / B; }

// Evaluates the tiles tx0 .. tx0 + strip_tiles(B, TILES) - 1 of tile row ty with a 64 TILES-thread
// workgroup. Tile t of the strip is reduced by segment t mod 4 of wave (t / 4) mod TILES, in the
// per-tile routine's order, so the statistics do not depend on TILES or on which wave reduces a
// tile. If tparams is not NULL (LDS), the (sx2, sy2, kt2) of tile tx0 + t are also stored at
// tparams + 3 t, visible after the caller's next barrier.
template <typename S, int TILES>
__device__ void estimate_strip(const BufView<S> &v, const EstParams &p, const TileGeom &tg, int tx0,
                               int ty, float *stats, StripSmem<TILES> &sm, float *tparams) {
    using ST = Strip<TILES>;
    const Region rg{sm.lbar, sm.om, sm.gt, sm.sa, sm.m2, sm.n};
    const int B = tg.tile;
    const int ntile = min(strip_tiles(B, TILES), tg.tiles_x - tx0);
    const int i0 = tx0 * B, j0 = ty * B;
    const int sw = min(ntile * B, v.width - i0), sh = min(B, v.height - j0);
    const int rp = sw + 2;
    region_moments<S, ST::ITEMS, (std::is_same<S, __half>::value ? 4 : 2)>(v, p, rg, i0 - 1, j0 - 1, rp, rp * (sh + 2));
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    constexpr int kSeg = kWave / kGroups;  // tiles per wave and round
    for (int t0 = wid * kSeg; t0 < ntile; t0 += TILES * kSeg) {  // uniform over the wave
        const int t = t0 + lane / kGroups;
        const bool has = t < ntile;
        const int tt = has ? t : t0;  // a segment without a tile repeats the round's first (unused)
        const int bw = min(B, v.width - (i0 + tt * B)), bh = sh;
        const Acc acc = segment_tile_acc(rg, rp + 1 + tt * B, rp, bw, bh, lane);
        tile_finish(acc, p, tg, ty * tg.tiles_x + tx0 + tt, bw, bh, stats,
                    tparams ? tparams + 3 * tt : nullptr, lane, has);
    }
}

}  // namespace est

// Estimator constants of a call (defined with afr_estimate_gradients).
est::EstParams est_params(const afr_deep_buffer &buf, const afr_params &prm);

}  // namespace afr
