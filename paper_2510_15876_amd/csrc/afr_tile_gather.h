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
// P = Tm * (1, r, g, b), and stores them in LDS. Each lane then owns ROWS output pixels of one tile
// column and adds (X * Y) * P into 4-channel accumulators: one multiply and four FMAs per
// (slot, pixel) pair, with every LDS index resolved at compile time.
// With binary16 storage the temporal factor goes into Y instead (Y' = Y * Tm, its exponent added to
// that of Y(-R) before the recurrence) and the colours stay in LDS as the stored binary16 values, which
// the FMAs take as operands directly (mixed-precision FMA): the same arithmetic count per pair from 16
// instead of 24 bytes of LDS reads. The recurrences start from the smallest value of the row, which
// must not underflow: tiles narrower than that bound (and, for the folded Y', than a tighter one)
// evaluate each value from its own exponential instead (see xrec, yrec).
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
#include <type_traits>

#include "afr_internal.h"

namespace afr {
namespace gat {

constexpr float kLog2e = 1.4426950408889634f;

// 2^x by the hardware instruction: results below the smallest normal flush to zero (such weights
// are < 2^-126 of the largest and cannot move a normalised sum).
__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
constexpr int kB = 8;  // statistics tile edge handled by this kernel

struct TiledParams {
    float t_now, dt_ref;
};

// LDS of one group evaluation. P: one float4 per source pixel of each tile's region (row pitch RW);
// with binary16 storage the same array holds each source pixel's three colours as they are stored
// (one uint2: r | g << 16, b), at the same positions in uint2 units.
// XY: per tile and region row, the 2R+1 offsets m one after another (pitch XP), each with the row's X
// values in columns [0, RW) and its Y values in columns [RW, 2 RW): X(row, col, m) at
// row * RP + m * XP + col with RP = (2R+1) XP. A lane's X and Y reads of one source row then lie
// within a few hundred bytes, so they pair into two-address reads with little address arithmetic,
// and RP modulo 64 is an odd multiple of 8 at every R, so an 8 x 8 block of lanes reading
// (row + h, col + c) hits 64 distinct banks. Tiles are XYS apart with XYS = 8 (mod 64), which puts
// the lane blocks of up to four tiles on disjoint banks.
template <int R>
struct XYLayout {
    static constexpr int RW = 8 + 2 * R, NM = 2 * R + 1;
    static constexpr int XP = (2 * RW <= 24) ? 24 : 40;
    static constexpr int RP = NM * XP;                                  // one region row
    static constexpr int XYS = (RW * RP + 55) / 64 * 64 + 8;            // one tile
};
// P: with one tile per wave, (P.x, P.y) and (P.z, P.w) of region (row, col) are float2s at
// row * XP + col and row * XP + RW + col, so the 64-bit reads of an 8 x 8 lane block hit distinct
// banks; with more tiles per wave, one float4 per pixel with row pitch RW and tile pitch PS.
template <int R, int TPW>
struct Smem {
    static constexpr int RW = 8 + 2 * R, NP = RW * RW, PS = NP + 5;
    static constexpr int NP4 = TPW == 1 ? RW * XYLayout<R>::XP / 2 : TPW * PS;
    float4 P[NP4];
    float XY[TPW * XYLayout<R>::XYS];
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
    constexpr int XP = XYLayout<R>::XP, RP = XYLayout<R>::RP;
    constexpr bool kMix = std::is_same<S, __half>::value;  // colours kept as binary16 in LDS
    float4 *sP = sm.P;

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
        gxm[m] = fast_exp2(-(float)(2 * (m - R) + 1) * cx2);
        gym[m] = fast_exp2(-(float)(2 * (m - R) + 1) * cy2);
    }
    // The recurrence needs its starting value X(-R) >= 2^-(R+1/2)^2 c to stay in float32's normal
    // range: (R + 1/2)^2 c <= 120. With binary16 storage Y'(-R) also carries Tm: a Y'(-R) below the
    // subnormal range then drops the source's other Y' values too, which are at most
    // 2^((R+1/2)^2 cy2) times larger, so the folded recurrence is kept to (R + 1/2)^2 cy2 <= 20
    // (lost weights < 2^-129 of the region reference, below every normalised pixel's resolution). The
    // default width floor (0.5 px) gives 18 at R = 2. Narrower tiles take one exponential per value.
    constexpr float kR2 = (R + 0.5f) * (R + 0.5f);
    const bool xrec = kR2 * cx2 <= 120.0f;
    const bool yrec = kR2 * cy2 <= (kMix ? 20.0f : 120.0f);

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

    // Raw slot data of one plane, prefetched one plane ahead: buffer loads with the plane's base in
    // scalar registers and this lane's loop-invariant byte offset.
    unsigned ioff[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) ioff[it] = (unsigned)iq[it] * (unsigned)sizeof(S);
    S rox[ITEMS], roy[ITEMS], rta[ITEMS], rr[ITEMS], rg[ITEMS], rb[ITEMS];
    auto load_plane = [&](int k) {
        const size_t base = (size_t)k * hw, bytes = hw * sizeof(S);
        const auto rox_ = plane_rsrc(v.ox + base, bytes), roy_ = plane_rsrc(v.oy + base, bytes);
        const auto rta_ = plane_rsrc(v.ta + base, bytes), rr_ = plane_rsrc(v.r + base, bytes);
        const auto rg_ = plane_rsrc(v.g + base, bytes), rb_ = plane_rsrc(v.b + base, bytes);
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            rox[it] = plane_load<S>(rox_, ioff[it]);
            roy[it] = plane_load<S>(roy_, ioff[it]);
            rta[it] = plane_load<S>(rta_, ioff[it]);
            rr[it] = plane_load<S>(rr_, ioff[it]);
            rg[it] = plane_load<S>(rg_, ioff[it]);
            rb[it] = plane_load<S>(rb_, ioff[it]);
        }
    };
    if (kmax > 0) load_plane(0);

    float4 *tP = sP + my_t * PS;
    float2 *tPP = reinterpret_cast<float2 *>(sP);  // split layout (one tile per wave)
    // binary16 colours: row pitch XP (one tile per wave) or the tile's plane of PS entries
    uint2 *tC = reinterpret_cast<uint2 *>(sP) + (TPW == 1 ? 0 : my_t * PS);
    float *tX = sm.XY + my_t * XYLayout<R>::XYS;  // X of region (row, col, m) at row * RP + m * XP + col
    float *tY = tX + RW;                          // Y at row * RP + m * XP + RW + col
    // Separable factors of plane k for this tile's source region. A slot beyond its pixel's count
    // (or a pixel outside the image) gets P = 0 and finite dummy factors. REC: the recurrences (the
    // tile allows them, the usual case); otherwise every factor from its own exponential.
    auto factors = [&](int k, auto rec_c) {
        constexpr bool REC = decltype(rec_c)::value;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int pix = sub + it * LPT;
            if (pix < NP) {
                const bool on = k < icnt[it];
                const float dx = on ? Codec<S>::dec(rox[it]) - 0.5f : 0.0f;
                const float dy = on ? Codec<S>::dec(roy[it]) - 0.5f : 0.0f;
                const float a = on ? Codec<S>::age(rta[it], p.t_now, p.dt_ref) : amin;
                const float lt = -((a - amin) * (a + amin)) * ct2;  // log2 Tm
                // binary16 storage: Y'(m) = Y(m) Tm, 0 for an empty slot; with the recurrence Tm's
                // exponent joins Y(0)'s, evaluated 2^32 up and scaled back so that it keeps
                // subnormal values (see the top of the file)
                const float lt_on = on ? lt : -INFINITY;
                // X[m] = exp2(-((m - R) + dx)^2 cx2): upward from the smallest value X[0] by the
                // recurrence, or each from its own exponential
                float X[NM], Y[NM];
                if constexpr (REC) {
                    const float ex = dx - (float)R, ey = dy - (float)R;
                    X[0] = fast_exp2(-ex * ex * cx2);
                    Y[0] = kMix ? fast_exp2(-ey * ey * cy2 + lt_on + 32.0f) * 0x1p-32f
                                : fast_exp2(-ey * ey * cy2);
                    if (R > 0) {
                        const float rhox = fast_exp2(-2.0f * dx * cx2);
                        const float rhoy = fast_exp2(-2.0f * dy * cy2);
#pragma unroll
                        for (int m = 0; m < 2 * R; ++m) {
                            X[m + 1] = X[m] * rhox * gxm[m];
                            Y[m + 1] = Y[m] * rhoy * gym[m];
                        }
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < NM; ++m) {
                        const float ex = dx + (float)(m - R), ey = dy + (float)(m - R);
                        X[m] = fast_exp2(-ex * ex * cx2);
                        Y[m] = fast_exp2(-ey * ey * cy2 + (kMix ? lt_on : 0.0f));
                    }
                }
                const int xy = (pix / RW) * XP + pix % RW;
                const int xyt = (pix / RW) * RP + pix % RW;
                if constexpr (kMix) {
                    // an empty slot's colours are written as 0 (its Y' is 0)
                    const unsigned c0 = on ? ((unsigned)__half_as_ushort(rr[it]) |
                                              ((unsigned)__half_as_ushort(rg[it]) << 16))
                                           : 0u;
                    const unsigned c1 = on ? (unsigned)__half_as_ushort(rb[it]) : 0u;
                    tC[TPW == 1 ? xy : pix] = make_uint2(c0, c1);
                } else {
                    const float tm = fast_exp2(lt);
                    const float4 P =
                        on ? make_float4(tm, tm * Codec<S>::dec(rr[it]),
                                         tm * Codec<S>::dec(rg[it]), tm * Codec<S>::dec(rb[it]))
                           : make_float4(0.f, 0.f, 0.f, 0.f);
                    if constexpr (TPW == 1) {
                        tPP[xy] = make_float2(P.x, P.y);
                        tPP[xy + RW] = make_float2(P.z, P.w);
                    } else {
                        tP[pix] = P;
                    }
                }
#pragma unroll
                for (int m = 0; m < NM; ++m) {
                    tX[xyt + m * XP] = X[m];
                    tY[xyt + m * XP] = Y[m];
                }
            }
        }
    };
    // The choice is the tile's own, so a tile evaluates the same way whichever tiles share its wave.
    // When every tile of the wave allows the recurrences (the usual case) one branch-free instruction
    // stream runs; a wave holding tiles of both kinds runs each form on its own lanes.
    const bool rec_t = xrec && yrec;
    const bool rec = __all(rec_t);  // uniform over the wave
    for (int k = 0; k < kmax; ++k) {
        if (rec)
            factors(k, std::true_type{});
        else if (TPW > 1 && rec_t)
            factors(k, std::true_type{});
        else
            factors(k, std::false_type{});
        __syncthreads();
        // Plane k+1 is loaded in the same scheduling region as plane k's accumulation (no branch
        // around it: after the last plane it reloads plane K-1, unused), so the accumulation
        // covers the load latency.
        load_plane(min(k + 1, v.k - 1));
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
                const int xy = (my_h * ROWS + vv) * XP + my_c + w;
                const int xyt = (my_h * ROWS + vv) * RP + my_c + w;
                const float x = tX[xyt + w * XP];
                if constexpr (kMix) {
                    const uint2 cw = tC[TPW == 1 ? xy : pix];
                    const __half2 rg2 = __halves2half2(__ushort_as_half((unsigned short)cw.x),
                                                       __ushort_as_half((unsigned short)(cw.x >> 16)));
                    const __half bh = __ushort_as_half((unsigned short)cw.y);
#pragma unroll
                    for (int u = 0; u < ROWS; ++u) {
                        const int nn = vv - u;  // n + R
                        if (nn >= 0 && nn <= 2 * R) {
                            const float wgt = x * tY[xyt + nn * XP];  // X * Y * Tm
                            part[u][0] += wgt;
                            part[u][1] = fmaf(wgt, __low2float(rg2), part[u][1]);
                            part[u][2] = fmaf(wgt, __high2float(rg2), part[u][2]);
                            part[u][3] = fmaf(wgt, __half2float(bh), part[u][3]);
                        }
                    }
                } else {
                    float4 P;
                    if constexpr (TPW == 1) {
                        const float2 a = tPP[xy], b = tPP[xy + RW];
                        P = make_float4(a.x, a.y, b.x, b.y);
                    } else {
                        P = tP[pix];
                    }
#pragma unroll
                    for (int u = 0; u < ROWS; ++u) {
                        const int nn = vv - u;  // n + R
                        if (nn >= 0 && nn <= 2 * R) {
                            const float wgt = x * tY[xyt + nn * XP];
                            part[u][0] += wgt * P.x;
                            part[u][1] += wgt * P.y;
                            part[u][2] += wgt * P.z;
                            part[u][3] += wgt * P.w;
                        }
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
