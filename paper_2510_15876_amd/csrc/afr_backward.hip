// Adjoint of the gather with the tile statistics held fixed (gradients for fitting sigma and tau and
// for the sample colours; not part of the paper, which only runs the forward filter).
//
// With pi_s(p) = exp(E_s(p) - m_p) / W_p (m_p, W_p from the forward's aux output):
//   colour gradient   dl/dc_{s,ch} = sum_p g(p,ch) pi_s(p)
//   filter parameters dl/dtheta    = sum_p sum_s pi_s(p) h_s(p) dE_s(p)/dtheta,
//                     h_s(p) = sum_ch g(p,ch) (c_{s,ch} - C_{p,ch})
// Per-pair weights are recomputed from the buffer, never stored, and nothing uses floating-point
// atomics: every sum runs in a fixed order.
//
// Tiled form (8 px statistics tiles, the layout of the tiled gather). The weight of slot s for pixel
// p of tile T factors as X_T(s, m) Y_T(s, n) Tm_T(s) (see afr_gather.h), and with
//   s_p = exp(shift_T - m_p) / W_p,  g'_p = g(p, .) s_p,  k'_p = (g(p, .) . C_p) s_p
// the two sums become, per pair, w = X Y Tm:
//   colour gradient of s += w g'_p,    parameter terms += w (g'_p . c_s - k'_p) dE/dtheta,
// where dE/dtheta is dx^2 and dy^2 times per-tile coefficients plus a^2 times one (for tau).
//   k_bwd_prep   per tile: the tile's shift (the gather's: smallest slot-0 age of the region),
//                g'_p and k'_p per pixel. A pixel the forward had to evaluate directly (its shifted
//                weights underflow: shift_T - m_p > 60) is flagged and its parameter terms are
//                computed exactly here.
//   k_bwd_tile   per tile: each lane owns source slots of the tile's region, evaluates their factors
//                once per plane and visits the tile pixels in reach; it writes the slot's colour-
//                gradient partial for this tile and folds the parameter terms per lane.
//   k_bwd_slots  per slot: adds the partials of the (at most four) tiles whose region holds it, in
//                tile order, plus exact terms from flagged pixels in reach.
//   k_reduce_params  sums the per-tile parameter partials in tile order.
// Other tile sizes use the direct form: k_bwd_pixel (pixel-parallel: g/W per pixel and the
// parameter terms) and k_bwd_sample (slot-parallel gather of the colour gradients).
#include <algorithm>

#include "afr_internal.h"

namespace afr {
namespace {

constexpr int kBX = 64, kBY = 4;

struct BwdParams {
    float t_now, dt_ref;
    int radius;
    double sigma, tau, e_max;
};

// Per-tile coefficients: E = -(dx^2 cx + dy^2 cy + a^2 ct);
// dE/dsigma = dx^2 fxs + dy^2 fys;  dE/dtau = dx^2 fxt + dy^2 fyt - a^2 fkt.
struct TileCoef {
    float cx, cy, ct;
    float fxs, fys, fxt, fyt, fkt;
};

__device__ inline TileCoef tile_coef(const float *stats, int nt, int T, const BwdParams &p) {
    const double sx2 = stats[AFR_STAT_SX2 * nt + T], sy2 = stats[AFR_STAT_SY2 * nt + T];
    const double kt2 = stats[AFR_STAT_KT2 * nt + T];
    const double ex2 = stats[AFR_STAT_EX2 * nt + T], ey2 = stats[AFR_STAT_EY2 * nt + T];
    const double zx = p.sigma * p.sigma * ex2, zy = p.sigma * p.sigma * ey2;
    double dx_dz = 1.0, dy_dz = 1.0;
    if (!isinf(p.e_max)) {
        const double m2 = p.e_max * p.e_max;
        dx_dz = m2 * m2 / ((m2 + zx) * (m2 + zx));
        dy_dz = m2 * m2 / ((m2 + zy) * (m2 + zy));
    }
    // at the large-V limit (ex2 = +inf) the width is its ceiling, constant in sigma and tau
    const bool fx = !isinf(ex2), fy = !isinf(ey2);
    const double dsx_ds = fx ? dx_dz * 2.0 * p.sigma * ex2 : 0.0;
    const double dsy_ds = fy ? dy_dz * 2.0 * p.sigma * ey2 : 0.0;
    const double dsx_dt = fx ? dx_dz * p.sigma * p.sigma * (2.0 / 3.0) * ex2 / p.tau : 0.0;
    const double dsy_dt = fy ? dy_dz * p.sigma * p.sigma * (2.0 / 3.0) * ey2 / p.tau : 0.0;
    const double dkt_dt = (4.0 / 3.0) * kt2 / p.tau;
    TileCoef c;
    // the exponent coefficients use the forward kernels' float expressions bit for bit
    c.cx = 0.5f / stats[AFR_STAT_SX2 * nt + T];
    c.cy = 0.5f / stats[AFR_STAT_SY2 * nt + T];
    c.ct = 0.5f * stats[AFR_STAT_KT2 * nt + T];
    c.fxs = (float)(0.5 * dsx_ds / (sx2 * sx2));
    c.fys = (float)(0.5 * dsy_ds / (sy2 * sy2));
    c.fxt = (float)(0.5 * dsx_dt / (sx2 * sx2));
    c.fyt = (float)(0.5 * dsy_dt / (sy2 * sy2));
    c.fkt = (float)(0.5 * dkt_dt);
    return c;
}

template <typename S>
__global__ __launch_bounds__(kBX *kBY) void k_bwd_pixel(BufView<S> v, BwdParams p, TileGeom tg,
                                                        const float *__restrict__ stats,
                                                        const float *__restrict__ rgb,
                                                        const float *__restrict__ aux,
                                                        const float *__restrict__ grad,
                                                        float *__restrict__ gw,
                                                        double *__restrict__ partial) {
    __shared__ double s_red[2][kBX * kBY / kWave];
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int W = v.width, H = v.height, R = p.radius;
    const size_t hw = (size_t)W * H;
    double d_sig = 0.0, d_tau = 0.0;
    if (i < W && j < H) {
        const size_t px = (size_t)j * W + i;
        const float m = aux[px], wsum = aux[hw + px];
        if (wsum > 0.0f) {
            const float inv = 1.0f / wsum;
            const float g0 = grad[px], g1 = grad[hw + px], g2 = grad[2 * hw + px];
            const float C0 = rgb[px], C1 = rgb[hw + px], C2 = rgb[2 * hw + px];
            gw[px] = g0 * inv;
            gw[hw + px] = g1 * inv;
            gw[2 * hw + px] = g2 * inv;
            const int T = (j / tg.tile) * tg.tiles_x + i / tg.tile;
            const TileCoef c = tile_coef(stats, tg.nt, T, p);
            float ax = 0.0f, ay = 0.0f, at = 0.0f;
            const int qx0 = max(0, i - R), qx1 = min(W - 1, i + R);
            const int qy0 = max(0, j - R), qy1 = min(H - 1, j + R);
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
                        const float e = -(dx * dx * c.cx + dy * dy * c.cy + a * a * c.ct);
                        const float pi = expf(e - m) * inv;
                        const float h = g0 * (Codec<S>::dec(fld(v.r, s)) - C0) +
                                        g1 * (Codec<S>::dec(fld(v.g, s)) - C1) +
                                        g2 * (Codec<S>::dec(fld(v.b, s)) - C2);
                        const float ph = pi * h;
                        ax += ph * dx * dx;
                        ay += ph * dy * dy;
                        at += ph * a * a;
                    }
                }
            d_sig = (double)ax * c.fxs + (double)ay * c.fys;
            d_tau = (double)ax * c.fxt + (double)ay * c.fyt - (double)at * c.fkt;
        } else {
            gw[px] = gw[hw + px] = gw[2 * hw + px] = 0.0f;
        }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        d_sig += __shfl_xor(d_sig, o, kWave);
        d_tau += __shfl_xor(d_tau, o, kWave);
    }
    const int t = threadIdx.y * kBX + threadIdx.x;
    if ((t & (kWave - 1)) == 0) {
        s_red[0][t / kWave] = d_sig;
        s_red[1][t / kWave] = d_tau;
    }
    __syncthreads();
    if (t == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kBX * kBY / kWave; ++w) {
            a += s_red[0][w];
            b += s_red[1][w];
        }
        const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        partial[2 * blk] = a;
        partial[2 * blk + 1] = b;
    }
}

template <typename S>
__global__ __launch_bounds__(kBX *kBY) void k_bwd_sample(BufView<S> v, BwdParams p, TileGeom tg,
                                                         const float *__restrict__ stats,
                                                         const float *__restrict__ aux,
                                                         const float *__restrict__ gw,
                                                         float *__restrict__ gslot) {
    const int qx = blockIdx.x * kBX + threadIdx.x;
    const int qy = blockIdx.y * kBY + threadIdx.y;
    const int W = v.width, H = v.height, K = v.k, R = p.radius;
    if (qx >= W || qy >= H) return;
    const size_t hw = (size_t)W * H, hwk = hw * K;
    const size_t q = (size_t)qy * W + qx;
    const int n = v.count[q];
    const int px0 = max(0, qx - R), px1 = min(W - 1, qx + R);
    const int py0 = max(0, qy - R), py1 = min(H - 1, qy + R);
    for (int k = 0; k < K; ++k) {
        const size_t s = (size_t)k * hw + q;
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
        if (k < n) {
            const float ox = Codec<S>::dec(fld(v.ox, s)), oy = Codec<S>::dec(fld(v.oy, s));
            const float a = Codec<S>::age(fld(v.ta, s), p.t_now, p.dt_ref);
            for (int py = py0; py <= py1; ++py)
                for (int px = px0; px <= px1; ++px) {
                    const size_t pp = (size_t)py * W + px;
                    const float wsum = aux[hw + pp];
                    if (!(wsum > 0.0f)) continue;
                    const int T = (py / tg.tile) * tg.tiles_x + px / tg.tile;
                    const float cx = 0.5f / stats[AFR_STAT_SX2 * tg.nt + T];
                    const float cy = 0.5f / stats[AFR_STAT_SY2 * tg.nt + T];
                    const float ct = 0.5f * stats[AFR_STAT_KT2 * tg.nt + T];
                    const float dx = ((float)(qx - px) - 0.5f) + ox;
                    const float dy = ((float)(qy - py) - 0.5f) + oy;
                    const float e = -(dx * dx * cx + dy * dy * cy + a * a * ct);
                    const float w = expf(e - aux[pp]);
                    s0 += gw[pp] * w;
                    s1 += gw[hw + pp] * w;
                    s2 += gw[2 * hw + pp] * w;
                }
        }
        gslot[s] = s0;
        gslot[hwk + s] = s1;
        gslot[2 * hwk + s] = s2;
    }
}

// ---- tiled adjoint (8 px statistics tiles) -------------------------------------------------------

constexpr int kTB = 8;                  // statistics tile edge of the tiled form
constexpr float kLog2eB = 1.4426950408889634f;
constexpr float kDirectExp = 60.0f;     // shift - m beyond which a pixel is evaluated directly

template <int R>
struct RegionGeom {
    static constexpr int RW = kTB + 2 * R, NP = RW * RW, NM = 2 * R + 1;
    static constexpr int ITEMS = (NP + kWave - 1) / kWave;
};

struct TiledWs {
    float4 *gk;           // [H][W] (g'_0, g'_1, g'_2, k'); zero for excluded pixels
    unsigned char *flag;  // [H][W] 1 where the pixel is evaluated directly
    float *amin;          // [nt] the tile's age reference (smallest slot-0 age of its region)
    int *nflag;           // [nt] flagged pixels of the tile
    double *pp;           // [2 nt][2] parameter partials: prep (flagged pixels), then tile
    float *part;          // [nt][K][3][NP] colour-gradient partials of each tile's region slots
};

template <int R>
size_t tiled_ws_bytes(int32_t w, int32_t h, int32_t k) {
    const size_t hw = (size_t)w * h;
    const size_t nt = (size_t)((w + kTB - 1) / kTB) * ((h + kTB - 1) / kTB);
    return align_up(hw * sizeof(float4)) + align_up(hw) + align_up(nt * 4) + align_up(nt * 4) +
           align_up(nt * 4 * 8) + align_up(nt * (size_t)k * 3 * RegionGeom<R>::NP * 4);
}

size_t tiled_ws_bytes_r(int32_t w, int32_t h, int32_t k, int r) {
    switch (r) {
        case 0: return tiled_ws_bytes<0>(w, h, k);
        case 1: return tiled_ws_bytes<1>(w, h, k);
        case 2: return tiled_ws_bytes<2>(w, h, k);
        case 3: return tiled_ws_bytes<3>(w, h, k);
        default: return tiled_ws_bytes<4>(w, h, k);
    }
}

template <int R>
TiledWs tiled_ws_carve(void *ws, int32_t w, int32_t h, int32_t k) {
    const size_t hw = (size_t)w * h;
    const size_t nt = (size_t)((w + kTB - 1) / kTB) * ((h + kTB - 1) / kTB);
    char *p = static_cast<char *>(ws);
    TiledWs o;
    o.gk = reinterpret_cast<float4 *>(p);
    p += align_up(hw * sizeof(float4));
    o.flag = reinterpret_cast<unsigned char *>(p);
    p += align_up(hw);
    o.amin = reinterpret_cast<float *>(p);
    p += align_up(nt * 4);
    o.nflag = reinterpret_cast<int *>(p);
    p += align_up(nt * 4);
    o.pp = reinterpret_cast<double *>(p);
    p += align_up(nt * 4 * 8);
    o.part = reinterpret_cast<float *>(p);
    return o;
}

__device__ inline float wave_min_f(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ inline int wave_sum_i(int v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Exact parameter terms of pixel (i, j) (the direct form), accumulated in float per pixel.
template <typename S>
__device__ inline void direct_param_terms(const BufView<S> &v, const BwdParams &p, const TileCoef &c,
                                          int i, int j, float m, float inv, float g0, float g1,
                                          float g2, float C0, float C1, float C2, double &d_sig,
                                          double &d_tau) {
    const int W = v.width, H = v.height, R = p.radius;
    const size_t hw = (size_t)W * H;
    double ax = 0.0, ay = 0.0, at = 0.0;  // the terms cancel (sum of pi h is zero): double sums
    const int qx0 = max(0, i - R), qx1 = min(W - 1, i + R);
    const int qy0 = max(0, j - R), qy1 = min(H - 1, j + R);
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
                const float e = -(dx * dx * c.cx + dy * dy * c.cy + a * a * c.ct);
                const float pi = expf(e - m) * inv;
                const float h = g0 * (Codec<S>::dec(fld(v.r, s)) - C0) +
                                g1 * (Codec<S>::dec(fld(v.g, s)) - C1) +
                                g2 * (Codec<S>::dec(fld(v.b, s)) - C2);
                const double ph = (double)(pi * h);
                ax += ph * (double)(dx * dx);
                ay += ph * (double)(dy * dy);
                at += ph * (double)(a * a);
            }
        }
    d_sig = ax * c.fxs + ay * c.fys;
    d_tau = ax * c.fxt + ay * c.fyt - at * c.fkt;
}

template <typename S, int R>
__global__ __launch_bounds__(kWave) void k_bwd_prep(BufView<S> v, BwdParams p, TileGeom tg,
                                                    const float *__restrict__ stats,
                                                    const float *__restrict__ rgb,
                                                    const float *__restrict__ aux,
                                                    const float *__restrict__ grad, TiledWs ws) {
    using G = RegionGeom<R>;
    const int T = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = T % tg.tiles_x, ty = T / tg.tiles_x;
    const int W = v.width, H = v.height, lane = threadIdx.x;
    const size_t hw = (size_t)W * H;
    const float kt2 = stats[AFR_STAT_KT2 * tg.nt + T];
    // the gather's age reference: smallest slot-0 age over the tile's source region
    float amin = INFINITY;
#pragma unroll
    for (int it = 0; it < G::ITEMS; ++it) {
        const int pix = lane + it * kWave;
        const int qx = tx * kTB - R + pix % G::RW, qy = ty * kTB - R + pix / G::RW;
        if (pix < G::NP && qx >= 0 && qx < W && qy >= 0 && qy < H) {
            const size_t q = (size_t)qy * W + qx;
            if (v.count[q] > 0) amin = fminf(amin, Codec<S>::age(fld(v.ta, q), p.t_now, p.dt_ref));
        }
    }
    amin = wave_min_f(amin);
    if (amin == INFINITY) amin = 0.0f;
    const float shift = -(amin * amin) * (0.5f * kt2);
    const int i = tx * kTB + lane % kTB, j = ty * kTB + lane / kTB;
    double d_sig = 0.0, d_tau = 0.0;
    int flagged = 0;
    if (i < W && j < H) {
        const size_t px = (size_t)j * W + i;
        const float m = aux[px], wsum = aux[hw + px];
        float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
        unsigned char f = 0;
        if (wsum > 0.0f) {
            const float g0 = grad[px], g1 = grad[hw + px], g2 = grad[2 * hw + px];
            const float C0 = rgb[px], C1 = rgb[hw + px], C2 = rgb[2 * hw + px];
            const float e = shift - m;
            if (e <= kDirectExp) {
                const float sc = expf(e) / wsum;
                o = make_float4(g0 * sc, g1 * sc, g2 * sc, (g0 * C0 + g1 * C1 + g2 * C2) * sc);
            } else {
                f = 1;
                flagged = 1;
                const TileCoef c = tile_coef(stats, tg.nt, T, p);
                direct_param_terms<S>(v, p, c, i, j, m, 1.0f / wsum, g0, g1, g2, C0, C1, C2, d_sig,
                                      d_tau);
            }
        }
        ws.gk[px] = o;
        ws.flag[px] = f;
    }
    d_sig = wave_sum_d(d_sig);
    d_tau = wave_sum_d(d_tau);
    flagged = wave_sum_i(flagged);
    if (lane == 0) {
        ws.amin[T] = amin;
        ws.nflag[T] = flagged;
        ws.pp[2 * T] = d_sig;
        ws.pp[2 * T + 1] = d_tau;
    }
}

// One thread per source slot of the tile's region (ITEMS waves per tile). Waves run their own
// plane loops (no barrier inside); their parameter sums are combined in wave order at the end.
template <typename S, int R>
__global__ __launch_bounds__(RegionGeom<R>::ITEMS *kWave) void k_bwd_tile(
    BufView<S> v, BwdParams p, TileGeom tg, const float *__restrict__ stats, TiledWs ws) {
    using G = RegionGeom<R>;
    constexpr int RW = G::RW, NP = G::NP, NM = G::NM, NW = G::ITEMS;
    // (g', k') of the tile's pixels on a grid padded by 2R zeros on every side (tile-local rows and
    // columns -2R .. 8 + 2R - 1): a slot reads its 2R+1 x 2R+1 pixels at fixed offsets, and pixels
    // outside the tile (or the image) contribute nothing without a test. Rows are GP entries apart
    // with GP = RW (mod 16): the lanes of a wave (slots in row-major order, RW per region row) then
    // read consecutive 16-byte entries as far as the LDS banks are concerned, without conflicts.
    constexpr int GW = kTB + 4 * R;
    constexpr int GP = GW + ((RW - GW) % 16 + 16) % 16;
    __shared__ float4 s_gk[GW * GP];
    __shared__ double s_red[2][NW];
    const int T = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = T % tg.tiles_x, ty = T / tg.tiles_x;
    const int W = v.width, H = v.height, K = v.k;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const size_t hw = (size_t)W * H;
    for (int e = tid; e < GW * GP; e += NW * kWave) {
        const int li = e % GP - 2 * R, lj = e / GP - 2 * R;
        const int i = tx * kTB + li, j = ty * kTB + lj;
        const bool inside = li >= 0 && li < kTB && lj >= 0 && lj < kTB && i < W && j < H;
        s_gk[e] = inside ? ws.gk[(size_t)j * W + i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const float sx2 = stats[AFR_STAT_SX2 * tg.nt + T], sy2 = stats[AFR_STAT_SY2 * tg.nt + T];
    const float kt2 = stats[AFR_STAT_KT2 * tg.nt + T];
    const float cx2 = kLog2eB * (0.5f / sx2), cy2 = kLog2eB * (0.5f / sy2);
    const float ct2 = kLog2eB * (0.5f * kt2);
    const float amin = ws.amin[T];
    float gxm[NM];
#pragma unroll
    for (int m = 0; m < 2 * R; ++m) gxm[m] = __builtin_amdgcn_exp2f(-(float)(2 * (m - R) + 1) * cx2);
    float gym[2 * R > 0 ? 2 * R : 1];
    gym[0] = 1.0f;
#pragma unroll
    for (int n = 0; n < 2 * R; ++n) gym[n] = __builtin_amdgcn_exp2f(-(float)(2 * (n - R) + 1) * cy2);
    // Recurrences start from the smallest value of a row and need it in float32's range: Y(-R) >=
    // 2^-(R+1/2)^2 cy2 normal, (R + 1/2)^2 cy2 <= 120; X(-R) carries Tm, and a product below the
    // subnormal range would drop the larger X values too (at most 2^((R+1/2)^2 cx2) times larger), so
    // the X recurrence is kept to (R + 1/2)^2 cx2 <= 20. Narrower tiles evaluate every value directly.
    constexpr float kR2 = (R + 0.5f) * (R + 0.5f);
    const bool xrec = kR2 * cx2 <= 20.0f, yrec = kR2 * cy2 <= 120.0f;
    // Row offsets n with a pixel of the tile for some slot of this wave: a slot in region row r
    // reaches tile rows r - n in [0, 8) only. The wave's slots span region rows r_lo .. r_hi, so
    // rows outside [max(0, r_lo - 7), min(2R, r_hi)] add exact zeros for every lane and are skipped.
    const int r_lo = (wid * kWave) / RW, r_hi = min(NP - 1, wid * kWave + kWave - 1) / RW;
    const int n_lo = max(0, r_lo - (kTB - 1)), n_hi = min(2 * R, r_hi);
    const int pix = tid;
    const int rr_ = pix / RW, cc = pix % RW;
    // the slot's pixel at row offset n, column offset m is s_gk[(rr_ - n + 2R) GP + cc - m + 2R];
    // lanes past the region read from the origin (their weights are 0)
    const float4 *gk0 = s_gk + (pix < NP ? rr_ * GP + cc : 0);
    const int qx = tx * kTB - R + cc, qy = ty * kTB - R + rr_;
    const bool in = pix < NP && qx >= 0 && qx < W && qy >= 0 && qy < H;
    const unsigned q = in ? (unsigned)(qy * W + qx) : 0u;
    const unsigned ioff = q * (unsigned)(sizeof(S) * Slots<S>::kStride);
    const int icnt = in ? v.count[q] : 0;
    int kmax = icnt;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, kWave));
    __syncthreads();  // s_gk visible
    S rox, roy, rta, rr, rg, rb;
    auto load_plane = [&](int k) {
        // a binary16 slot is a 12-byte record: each field's descriptor starts at its field of the
        // plane's first record and steps by the record size
        const size_t base = (size_t)k * hw * Slots<S>::kStride;
        const size_t bytes = hw * sizeof(S) * Slots<S>::kStride;
        rox = plane_load<S>(plane_rsrc(v.ox + base, bytes), ioff);
        roy = plane_load<S>(plane_rsrc(v.oy + base, bytes), ioff);
        rta = plane_load<S>(plane_rsrc(v.ta + base, bytes), ioff);
        rr = plane_load<S>(plane_rsrc(v.r + base, bytes), ioff);
        rg = plane_load<S>(plane_rsrc(v.g + base, bytes), ioff);
        rb = plane_load<S>(plane_rsrc(v.b + base, bytes), ioff);
    };
    if (kmax > 0) load_plane(0);
    // parameter terms: float within one row of pixels, double across rows (the terms cancel: the
    // pi-weighted sum of h over a pixel's slots is zero)
    double Sx = 0.0, Sy = 0.0, Sa = 0.0;
    for (int k = 0; k < kmax; ++k) {
        const bool on = k < icnt;
        const float dx = on ? Codec<S>::dec(rox) - 0.5f : 0.0f;
        const float dy = on ? Codec<S>::dec(roy) - 0.5f : 0.0f;
        const float a = on ? Codec<S>::age(rta, p.t_now, p.dt_ref) : amin;
        const float cr = on ? Codec<S>::dec(rr) : 0.0f;
        const float cg = on ? Codec<S>::dec(rg) : 0.0f;
        const float cb = on ? Codec<S>::dec(rb) : 0.0f;
        load_plane(min(k + 1, K - 1));  // in flight during this plane's pairs
        const float da2 = (a - amin) * (a + amin);  // a^2 - amin^2 >= 0
        const float tm = on ? __builtin_amdgcn_exp2f(-da2 * ct2) : 0.0f;
        // X for the 2R+1 column offsets (times the temporal factor), kept in registers; the rows
        // are visited one at a time with Y advanced by its recurrence.
        float X[NM], dx2[NM];
        const float ex = dx - (float)R;
        if (xrec) {
            X[0] = __builtin_amdgcn_exp2f(-ex * ex * cx2) * tm;
            if (R > 0) {
                const float rhox = __builtin_amdgcn_exp2f(-2.0f * dx * cx2);
#pragma unroll
                for (int m = 0; m < 2 * R; ++m) X[m + 1] = X[m] * rhox * gxm[m];
            }
        } else {
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                const float e = dx + (float)(m - R);
                X[m] = __builtin_amdgcn_exp2f(-e * e * cx2) * tm;
            }
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const float ux = (float)(m - R) + dx;
            dx2[m] = ux * ux;
        }
        // Y for the 2R+1 row offsets, by the recurrence from the first row this wave needs or by
        // one exponential each, before the rows are visited, so that the rows form one unrolled
        // sequence whose LDS reads the compiler can issue ahead of the previous row's arithmetic.
        float Y[NM];
        {
            const float rhoy = __builtin_amdgcn_exp2f(-2.0f * dy * cy2);
            const float ey0 = dy + (float)(n_lo - R);
            float yv = __builtin_amdgcn_exp2f(-ey0 * ey0 * cy2);
#pragma unroll
            for (int n = 0; n < NM; ++n) {
                if (yrec) {
                    Y[n] = yv;  // valid from n_lo on; rows before it are not visited
                    if (n >= n_lo) yv *= rhoy * gym[n < 2 * R ? n : 0];
                } else {
                    const float e = dy + (float)(n - R);
                    Y[n] = __builtin_amdgcn_exp2f(-e * e * cy2);
                }
            }
        }
        // The a^2 factor of the tau terms enters as a^2 - amin^2: for every pixel the pi-weighted sum
        // of h over its slots is zero, so a constant offset of a^2 changes nothing but the
        // rounding, and this one keeps the factor small wherever a weight is not negligible.
        const float a2 = da2;
        float gr = 0.0f, gg = 0.0f, gb = 0.0f;
#pragma unroll
        for (int n = 0; n < NM; ++n) {
            if (n < n_lo || n > n_hi) continue;  // uniform over the wave
            const float uy = (float)(n - R) + dy;
            const float dyn2 = uy * uy;
            const float4 *grow = gk0 + (2 * R - n) * GP + 2 * R;
            float rx = 0.0f, rh = 0.0f;  // sums of hwt dx^2 and of hwt over the row
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                const float w = X[m] * Y[n];
                const float4 g4 = grow[-m];
                gr += w * g4.x;
                gg += w * g4.y;
                gb += w * g4.z;
                const float hwt = w * (g4.x * cr + g4.y * cg + g4.z * cb - g4.w);
                rx += hwt * dx2[m];
                rh += hwt;
            }
            Sx += (double)rx;
            Sy += (double)rh * dyn2;
            Sa += (double)rh * a2;
        }
        if (on) {
            float *pt = ws.part + ((size_t)T * K + k) * 3 * NP + pix;
            pt[0] = gr;
            pt[NP] = gg;
            pt[2 * NP] = gb;
        }
    }
    const TileCoef c = tile_coef(stats, tg.nt, T, p);
    double d_sig = Sx * c.fxs + Sy * c.fys;
    double d_tau = Sx * c.fxt + Sy * c.fyt - Sa * c.fkt;
    d_sig = wave_sum_d(d_sig);
    d_tau = wave_sum_d(d_tau);
    if (lane == 0) {
        s_red[0][wid] = d_sig;
        s_red[1][wid] = d_tau;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < NW; ++w) {
            a += s_red[0][w];
            b += s_red[1][w];
        }
        ws.pp[2 * (tg.nt + T)] = a;
        ws.pp[2 * (tg.nt + T) + 1] = b;
    }
}

template <typename S, int R>
__global__ __launch_bounds__(kBX *kBY) void k_bwd_slots(BufView<S> v, BwdParams p, TileGeom tg,
                                                        const float *__restrict__ stats,
                                                        const float *__restrict__ aux,
                                                        const float *__restrict__ grad,
                                                        TiledWs ws, float *__restrict__ gslot) {
    using G = RegionGeom<R>;
    constexpr int RW = G::RW, NP = G::NP;
    const int qx = blockIdx.x * kBX + threadIdx.x;
    const int qy = blockIdx.y * kBY + threadIdx.y;
    const int W = v.width, H = v.height, K = v.k;
    if (qx >= W || qy >= H) return;
    const size_t hw = (size_t)W * H, hwk = hw * K;
    const size_t q = (size_t)qy * W + qx;
    const int n = v.count[q];
    // tiles whose source region holds q, in tile order, and whether any has flagged pixels
    int tl[4], off[4], nt_ = 0;
    bool anyflag = false;
    const int tqx = qx / kTB, tqy = qy / kTB;
    for (int yy = max(0, tqy - 1); yy <= min(tg.tiles_y - 1, tqy + 1); ++yy)
        for (int xx = max(0, tqx - 1); xx <= min(tg.tiles_x - 1, tqx + 1); ++xx) {
            const int rx = qx - (xx * kTB - R), ry = qy - (yy * kTB - R);
            if (rx >= 0 && rx < RW && ry >= 0 && ry < RW && nt_ < 4) {
                tl[nt_] = yy * tg.tiles_x + xx;
                off[nt_] = ry * RW + rx;
                anyflag = anyflag || ws.nflag[tl[nt_]] > 0;
                ++nt_;
            }
        }
    for (int k = 0; k < K; ++k) {
        const size_t s = (size_t)k * hw + q;
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
        if (k < n) {
            for (int t = 0; t < nt_; ++t) {
                const float *pt = ws.part + ((size_t)tl[t] * K + k) * 3 * NP + off[t];
                s0 += pt[0];
                s1 += pt[NP];
                s2 += pt[2 * NP];
            }
            if (anyflag) {  // exact terms from pixels evaluated directly
                const float ox = Codec<S>::dec(fld(v.ox, s)), oy = Codec<S>::dec(fld(v.oy, s));
                const float a = Codec<S>::age(fld(v.ta, s), p.t_now, p.dt_ref);
                for (int py = max(0, qy - R); py <= min(H - 1, qy + R); ++py)
                    for (int px = max(0, qx - R); px <= min(W - 1, qx + R); ++px) {
                        const size_t pp = (size_t)py * W + px;
                        if (!ws.flag[pp]) continue;
                        const int T = (py / kTB) * tg.tiles_x + px / kTB;
                        const float cx = 0.5f / stats[AFR_STAT_SX2 * tg.nt + T];
                        const float cy = 0.5f / stats[AFR_STAT_SY2 * tg.nt + T];
                        const float ct = 0.5f * stats[AFR_STAT_KT2 * tg.nt + T];
                        const float dx = ((float)(qx - px) - 0.5f) + ox;
                        const float dy = ((float)(qy - py) - 0.5f) + oy;
                        const float e = -(dx * dx * cx + dy * dy * cy + a * a * ct);
                        const float w = expf(e - aux[pp]) / aux[hw + pp];
                        s0 += grad[pp] * w;
                        s1 += grad[hw + pp] * w;
                        s2 += grad[2 * hw + pp] * w;
                    }
            }
        }
        gslot[s] = s0;
        gslot[hwk + s] = s1;
        gslot[2 * hwk + s] = s2;
    }
}

// Sums nb (sigma, tau) partials in a fixed order: thread t adds entries t, t + 256, ... in index
// order (loads issued eight at a time), then a fixed tree over the threads.
__global__ __launch_bounds__(256) void k_reduce_params(const double *__restrict__ partial, int nb,
                                                       float *__restrict__ out) {
    __shared__ double s[2][256];
    double a = 0.0, b = 0.0;
    constexpr int kU = 8;
    int i = threadIdx.x;
    for (; i + (kU - 1) * 256 < nb; i += kU * 256) {
        double va[kU], vb[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            va[u] = partial[2 * (i + u * 256)];
            vb[u] = partial[2 * (i + u * 256) + 1];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            a += va[u];
            b += vb[u];
        }
    }
    for (; i < nb; i += 256) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (float)s[0][0];
        out[1] = (float)s[1][0];
    }
}

inline dim3 pixel_grid(int w, int h) { return dim3((w + kBX - 1) / kBX, (h + kBY - 1) / kBY); }

template <typename S>
hipError_t launch_bwd_typed(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                            const BwdParams &p, const float *rgb, const float *aux,
                            const float *grad, float *gslot, float *gparams, void *ws,
                            hipStream_t st) {
    const BufView<S> v = view_of<S>(buf);
    const TileGeom tg = geom_of(stats);
    const dim3 grid = pixel_grid(buf.width, buf.height), block(kBX, kBY);
    const size_t hw = (size_t)buf.width * buf.height;
    float *gw = static_cast<float *>(ws);
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + align_up(3 * hw * 4));
    k_bwd_pixel<S><<<grid, block, 0, st>>>(v, p, tg, stats.data, rgb, aux, grad, gw, partial);
    k_bwd_sample<S><<<grid, block, 0, st>>>(v, p, tg, stats.data, aux, gw, gslot);
    k_reduce_params<<<1, 256, 0, st>>>(partial, (int)(grid.x * grid.y), gparams);
    return hipGetLastError();
}

template <typename S, int R>
hipError_t launch_bwd_tiled(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                            const BwdParams &p, const float *rgb, const float *aux,
                            const float *grad, float *gslot, float *gparams, void *ws,
                            hipStream_t st) {
    const BufView<S> v = view_of<S>(buf);
    const TileGeom tg = geom_of(stats);
    const TiledWs w = tiled_ws_carve<R>(ws, buf.width, buf.height, buf.k);
    k_bwd_prep<S, R><<<tg.nt, kWave, 0, st>>>(v, p, tg, stats.data, rgb, aux, grad, w);
    k_bwd_tile<S, R><<<tg.nt, RegionGeom<R>::ITEMS * kWave, 0, st>>>(v, p, tg, stats.data, w);
    k_bwd_slots<S, R><<<pixel_grid(buf.width, buf.height), dim3(kBX, kBY), 0, st>>>(
        v, p, tg, stats.data, aux, grad, w, gslot);
    k_reduce_params<<<1, 256, 0, st>>>(w.pp, 2 * tg.nt, gparams);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_bwd_tiled_r(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                              const BwdParams &p, const float *rgb, const float *aux,
                              const float *grad, float *gslot, float *gparams, void *ws,
                              hipStream_t st) {
    switch (p.radius) {
        case 0: return launch_bwd_tiled<S, 0>(buf, stats, p, rgb, aux, grad, gslot, gparams, ws, st);
        case 1: return launch_bwd_tiled<S, 1>(buf, stats, p, rgb, aux, grad, gslot, gparams, ws, st);
        case 2: return launch_bwd_tiled<S, 2>(buf, stats, p, rgb, aux, grad, gslot, gparams, ws, st);
        case 3: return launch_bwd_tiled<S, 3>(buf, stats, p, rgb, aux, grad, gslot, gparams, ws, st);
        default: return launch_bwd_tiled<S, 4>(buf, stats, p, rgb, aux, grad, gslot, gparams, ws, st);
    }
}

}  // namespace

size_t backward_ws_bytes(int32_t w, int32_t h, int32_t k, int32_t radius) {
    const size_t hw = (size_t)w * h;
    const dim3 g = pixel_grid(w, h);
    const size_t direct = align_up(3 * hw * 4) + align_up((size_t)g.x * g.y * 2 * 8);
    return std::max(direct, tiled_ws_bytes_r(w, h, k, radius));
}

hipError_t launch_backward(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                           const afr_params &prm, const float *rgb, const float *aux,
                           const float *grad_rgb, float *grad_slot, float *grad_params, void *ws,
                           hipStream_t st) {
    BwdParams p;
    p.t_now = prm.t_now;
    p.dt_ref = prm.t_now - buf.t_ref;
    p.radius = prm.radius;
    p.sigma = prm.sigma;
    p.tau = prm.tau;
    p.e_max = prm.e_max;
    if (stats.tile == kTB) {  // tiled form
        if (buf.precision == AFR_FP16)
            return launch_bwd_tiled_r<__half>(buf, stats, p, rgb, aux, grad_rgb, grad_slot,
                                              grad_params, ws, st);
        return launch_bwd_tiled_r<float>(buf, stats, p, rgb, aux, grad_rgb, grad_slot, grad_params,
                                         ws, st);
    }
    if (buf.precision == AFR_FP16)
        return launch_bwd_typed<__half>(buf, stats, p, rgb, aux, grad_rgb, grad_slot, grad_params,
                                        ws, st);
    return launch_bwd_typed<float>(buf, stats, p, rgb, aux, grad_rgb, grad_slot, grad_params, ws,
                                   st);
}

}  // namespace afr
