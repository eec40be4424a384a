// LDS-tiled separable gather (Sec. 5.1 Gaussian space-time filter, Sec. 5.2 normalised average),
// as a device routine shared by afr_reconstruct and the batched persistent kernel.
//
// The filter is an axis-aligned Gaussian whose widths are constant over a statistics tile, so for an
// output pixel (i, j) of tile T and a slot s of source pixel q = (i + m, j + n) the weight factors:
//   w = X_T(s, m) * Y_T(s, n) * Tm_T(s),
//   X = exp(-(m + ox - 1/2)^2 / (2 sx2)), Y = exp(-(n + oy - 1/2)^2 / (2 sy2)),
//   Tm = exp(-(a^2 - a_ref^2) kt2 / 2).
// For each slot plane k the wave first evaluates, for every source pixel of each tile's
// (8+2R) x (8+2R) region, the 2R+1 values of X and of Y (three exponentials per axis with the
// Gaussian recurrence X(m+1) = X(m) * rho * exp(-(2m+1)/(2 sx2)), rho = exp(-(ox - 1/2)/sx2)) and
// P = Tm * (1, r, g, b), and stores them in LDS. Each lane then owns four output pixels of one tile
// column and adds (X * Y) * P into four 4-channel accumulators: one multiply and four FMAs per
// (slot, pixel) pair, with every LDS index resolved at compile time.
//
// Shift: a_ref is the smallest slot-0 age over the tile's source region (slot 0 is each pixel's
// newest sample), so every Tm <= 1; the pixel's largest weight is at least exp(-(2R+1)^2 / (8 e_min^2))
// times the tile-relative temporal factor of its newest sample. A pixel whose weight sum still
// falls below 1e-30 (its block's samples are all far older than the region's newest) is recomputed
// exactly by the direct two-pass form. aux receives (m, W) with m = -a_ref^2 kt2 / 2 and
// W = sum exp(E - m), which is what the adjoint needs.
//
// Accumulation order per pixel is fixed (slot plane, then source row, then source column), so the
// result does not depend on launch shape. Workgroups are assigned so that each XCD's L2 holds a
// contiguous band of the image (neighbouring workgroups share halo rows).
#pragma once
#include "afr_internal.h"

namespace afr {
namespace gat {

constexpr float kLog2e = 1.4426950408889634f;
constexpr int kB = 8;  // statistics tile edge handled by this kernel

struct TiledParams {
    float t_now, dt_ref;
};

// LDS of one group evaluation.
template <int R, int TPW>
struct Smem {
    static constexpr int RW = 8 + 2 * R, NP = RW * RW, PS = NP + 5, NM = 2 * R + 1;
    float4 P[TPW * PS];
    float X[TPW * NM * PS];
    float Y[TPW * NM * PS];
};

// Exact two-pass evaluation of one pixel (the direct form), used when the shared shift underflows.
template <typename S>
__device__ void direct_pixel(const BufView<S> &v, const TiledParams &p, int R, int i, int j,
                             float cx, float cy, float ct, float *rgb, float *aux) {
    const int W = v.width, H = v.height;
    const size_t hw = (size_t)W * H;
    const int qx0 = max(0, i - R), qx1 = min(W - 1, i + R);
    const int qy0 = max(0, j - R), qy1 = min(H - 1, j + R);
    float emax = -INFINITY;
    for (int qy = qy0; qy <= qy1; ++qy)
        for (int qx = qx0; qx <= qx1; ++qx) {
            const size_t q = (size_t)qy * W + qx;
            const float bx = (float)(qx - i) - 0.5f, by = (float)(qy - j) - 0.5f;
            for (int k = 0; k < v.count[q]; ++k) {
                const size_t s = (size_t)k * hw + q;
                const float dx = bx + Codec<S>::dec(v.ox[s]);
                const float dy = by + Codec<S>::dec(v.oy[s]);
                const float a = Codec<S>::age(v.ta[s], p.t_now, p.dt_ref);
                emax = fmaxf(emax, -(dx * dx * cx + dy * dy * cy + a * a * ct));
            }
        }
    const size_t px = (size_t)j * W + i;
    float ws = 0.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    if (emax != -INFINITY) {
        for (int qy = qy0; qy <= qy1; ++qy)
            for (int qx = qx0; qx <= qx1; ++qx) {
                const size_t q = (size_t)qy * W + qx;
                const float bx = (float)(qx - i) - 0.5f, by = (float)(qy - j) - 0.5f;
                for (int k = 0; k < v.count[q]; ++k) {
                    const size_t s = (size_t)k * hw + q;
                    const float dx = bx + Codec<S>::dec(v.ox[s]);
                    const float dy = by + Codec<S>::dec(v.oy[s]);
                    const float a = Codec<S>::age(v.ta[s], p.t_now, p.dt_ref);
                    const float w = expf(-(dx * dx * cx + dy * dy * cy + a * a * ct) - emax);
                    ws += w;
                    cr += w * Codec<S>::dec(v.r[s]);
                    cg += w * Codec<S>::dec(v.g[s]);
                    cb += w * Codec<S>::dec(v.b[s]);
                }
            }
    }
    const float inv = ws > 0.0f ? 1.0f / ws : 0.0f;
    rgb[px] = cr * inv;
    rgb[hw + px] = cg * inv;
    rgb[2 * hw + px] = cb * inv;
    if (aux) {
        aux[px] = emax == -INFINITY ? 0.0f : emax;
        aux[hw + px] = ws;
    }
}

// Minimum / maximum over aligned groups of G lanes (G a power of two <= 64).
template <int G>
__device__ inline float group_min(float v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ inline int wave_max_int(int v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

// Workgroups are dealt round-robin to the 8 XCDs (physical id b runs on XCD b % 8). Give XCD x the
// logical ids x*per .. x*per+per-1 so that each XCD's L2 serves a contiguous band of the image and
// the halo rows neighbouring workgroups share stay in one L2. The last nblocks % 8 ids map to
// themselves, so the mapping is a bijection for every grid size.
__device__ inline int xcd_remap(int b, int nblocks) {
    constexpr int kXcd = 8;
    const int per = nblocks / kXcd;
    const int x = b % kXcd, local = b / kXcd;
    return local < per ? x * per + local : b;
}

// One wave per TPW horizontally adjacent tiles; LPT = 64 / TPW lanes per tile, each lane owning
// ROWS = 8 * 8 / LPT output rows of one tile column. TPW only changes how work is spread over lanes;
// every pixel sums the same terms in the same order, so the output is identical for every TPW.
// Gathers the tiles tx0 .. tx0+TPW-1 of tile row ty with one 64-lane wave (the calling workgroup).
// tparam (LDS) must hold each tile's (sx2, sy2, kt2) and be visible to all lanes on entry.
template <typename S, int R, int TPW>
__device__ void gather_group(const BufView<S> &v, const TiledParams &p, const TileGeom &tg, int tx0,
                             int ty, Smem<R, TPW> &sm, const float *tparam,
                             float *__restrict__ rgb, float *__restrict__ aux) {
    constexpr int LPT = kWave / TPW;        // lanes per tile
    constexpr int ROWS = kB * kB / LPT;     // output rows per lane
    constexpr int RW = kB + 2 * R;          // source region edge per tile
    constexpr int NP = RW * RW;             // source pixels per tile
    constexpr int PS = NP + 5;              // padded plane stride (spreads tiles over LDS banks)
    constexpr int NM = 2 * R + 1;           // offsets per axis
    constexpr int ITEMS = (NP + LPT - 1) / LPT;
    float4 *sP = sm.P;
    float *sX = sm.X, *sY = sm.Y;

    const int W = v.width, H = v.height;
    const size_t hw = (size_t)W * H;
    const int lane = threadIdx.x;
    const int my_t = lane / LPT, sub = lane % LPT;
    const int my_c = sub % kB, my_h = sub / kB;
    const int tcol = tx0 + my_t;
    const int qx_org = tcol * kB - R, qy_org = ty * kB - R;

    // This lane's tile constants (log2 units) and the Gaussian recurrence factors
    // g[m] = exp2(-(2(m - R) + 1) c): X(m+1) = X(m) * rho * g[m], starting from the smallest X(-R).
    const float sx2 = tparam[3 * my_t], sy2 = tparam[3 * my_t + 1];
    const float kt2 = tparam[3 * my_t + 2];
    const float cx2 = kLog2e * (0.5f / sx2), cy2 = kLog2e * (0.5f / sy2);
    const float ct2 = kLog2e * (0.5f * kt2);
    float gxm[NM], gym[NM];
#pragma unroll
    for (int m = 0; m < 2 * R; ++m) {
        gxm[m] = exp2f(-(float)(2 * (m - R) + 1) * cx2);
        gym[m] = exp2f(-(float)(2 * (m - R) + 1) * cy2);
    }

    // Items: this lane's source pixels of its tile region; address and depth are loop invariant.
    int iq[ITEMS], icnt[ITEMS];
    float amin = INFINITY;
    int kmax = 0;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int pix = sub + it * LPT;
        const int qx = qx_org + pix % RW, qy = qy_org + pix / RW;
        iq[it] = 0;
        icnt[it] = 0;
        if (pix < NP && qx >= 0 && qx < W && qy >= 0 && qy < H) {
            iq[it] = qy * W + qx;
            icnt[it] = v.count[iq[it]];
        }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        kmax = max(kmax, icnt[it]);
        // slot 0 is each pixel's newest sample: the region's smallest age is among them
        if (icnt[it] > 0) amin = fminf(amin, Codec<S>::age(v.ta[iq[it]], p.t_now, p.dt_ref));
    }
    kmax = wave_max_int(kmax);
    amin = group_min<LPT>(amin);
    if (amin == INFINITY) amin = 0.0f;  // empty region: any shift works

    // Two-level sum: each slot plane's <= (2R+1)^2 terms go into a partial, and the partials of
    // the K planes are added with Kahan compensation.
    float acc[ROWS][4], cmp[ROWS][4];
#pragma unroll
    for (int u = 0; u < ROWS; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[u][c] = cmp[u][c] = 0.0f;

    // Raw slot data of one plane, prefetched one plane ahead.
    S rox[ITEMS], roy[ITEMS], rta[ITEMS], rr[ITEMS], rg[ITEMS], rb[ITEMS];
    auto load_plane = [&](int k) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const size_t s = (size_t)min(k, v.k - 1) * hw + iq[it];
            rox[it] = v.ox[s];
            roy[it] = v.oy[s];
            rta[it] = v.ta[s];
            rr[it] = v.r[s];
            rg[it] = v.g[s];
            rb[it] = v.b[s];
        }
    };
    if (kmax > 0) load_plane(0);

    float4 *tP = sP + my_t * PS;
    float *tX = sX + my_t * NM * PS;
    float *tY = sY + my_t * NM * PS;
    for (int k = 0; k < kmax; ++k) {
        // Separable factors of plane k for this tile's source region.
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int pix = sub + it * LPT;
            if (pix < NP) {
                float4 P = make_float4(0.f, 0.f, 0.f, 0.f);
                float X[NM], Y[NM];
#pragma unroll
                for (int m = 0; m < NM; ++m) X[m] = Y[m] = 0.0f;
                if (k < icnt[it]) {
                    const float dx = Codec<S>::dec(rox[it]) - 0.5f;
                    const float dy = Codec<S>::dec(roy[it]) - 0.5f;
                    const float a = Codec<S>::age(rta[it], p.t_now, p.dt_ref);
                    const float tm = exp2f(-((a - amin) * (a + amin)) * ct2);
                    P = make_float4(tm, tm * Codec<S>::dec(rr[it]), tm * Codec<S>::dec(rg[it]),
                                    tm * Codec<S>::dec(rb[it]));
                    // X[m] = exp2(-((m - R) + dx)^2 cx2), upward from the smallest value X[0]
                    const float ex = dx - (float)R, ey = dy - (float)R;
                    X[0] = exp2f(-ex * ex * cx2);
                    Y[0] = exp2f(-ey * ey * cy2);
                    if (R > 0) {
                        const float rhox = exp2f(-2.0f * dx * cx2), rhoy = exp2f(-2.0f * dy * cy2);
#pragma unroll
                        for (int m = 0; m < 2 * R; ++m) {
                            X[m + 1] = X[m] * rhox * gxm[m];
                            Y[m + 1] = Y[m] * rhoy * gym[m];
                        }
                    }
                }
                tP[pix] = P;
#pragma unroll
                for (int m = 0; m < NM; ++m) {
                    tX[m * PS + pix] = X[m];
                    tY[m * PS + pix] = Y[m];
                }
            }
        }
        if (k + 1 < kmax) load_plane(k + 1);  // in flight while plane k is accumulated
        __syncthreads();
        // Lane owns rows my_h*ROWS + u of column my_c. Source row (region coordinates)
        // my_h*ROWS + vv, source column my_c + w; offsets m = w - R, n = vv - u - R.
        float part[ROWS][4];
#pragma unroll
        for (int u = 0; u < ROWS; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) part[u][c] = 0.0f;
#pragma unroll
        for (int vv = 0; vv < ROWS + 2 * R; ++vv) {
#pragma unroll
            for (int w = 0; w < NM; ++w) {
                const int pix = (my_h * ROWS + vv) * RW + my_c + w;
                const float4 P = tP[pix];
                const float x = tX[w * PS + pix];
#pragma unroll
                for (int u = 0; u < ROWS; ++u) {
                    const int nn = vv - u;  // n + R
                    if (nn >= 0 && nn <= 2 * R) {
                        const float wgt = x * tY[nn * PS + pix];
                        part[u][0] += wgt * P.x;
                        part[u][1] += wgt * P.y;
                        part[u][2] += wgt * P.z;
                        part[u][3] += wgt * P.w;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < ROWS; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float y = part[u][c] - cmp[u][c];
                const float t = acc[u][c] + y;
                cmp[u][c] = (t - acc[u][c]) - y;
                acc[u][c] = t;
            }
        __syncthreads();
    }

    const int i = tcol * kB + my_c;
    if (tcol >= tg.tiles_x || i >= W) return;  // no barrier follows
    const float ctn = 0.5f * kt2;
    const float shift = -(amin * amin) * ctn;
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int j = ty * kB + my_h * ROWS + u;
        if (j >= H) continue;
        const size_t px = (size_t)j * W + i;
        const float ws = acc[u][0];
        if (ws >= 1e-30f) {
            const float inv = 1.0f / ws;
            rgb[px] = acc[u][1] * inv;
            rgb[hw + px] = acc[u][2] * inv;
            rgb[2 * hw + px] = acc[u][3] * inv;
            if (aux) {
                aux[px] = shift;
                aux[hw + px] = ws;
            }
        } else {
            direct_pixel<S>(v, p, R, i, j, 0.5f / sx2, 0.5f / sy2, ctn, rgb, aux);
        }
    }
}

}  // namespace gat
}  // namespace afr
