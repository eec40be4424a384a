// Adjoint of the gather with the tile statistics held fixed (gradients for fitting sigma and tau and
// for the sample colours; not part of the paper, which only runs the forward filter).
//
// With pi_s(p) = exp(E_s(p) - m_p) / W_p (m_p, W_p from the forward's aux output):
//   colour gradient   dl/dc_{s,ch} = sum_p g(p,ch) pi_s(p)
//   filter parameters dl/dtheta    = sum_p sum_s pi_s(p) h_s(p) dE_s(p)/dtheta,
//                     h_s(p) = sum_ch g(p,ch) (c_{s,ch} - C_{p,ch})
// Pass 1 (k_bwd_pixel) is pixel-parallel: it stores g/W per pixel and reduces the parameter terms
// per workgroup in FP64. Pass 2 (k_bwd_sample) is slot-parallel: each slot gathers from the pixels
// whose block contains it, so no atomics are needed. Pass 3 sums the workgroup partials in a fixed
// order. Per-pair weights are recomputed from the buffer, never stored.
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
    const double dsx_ds = dx_dz * 2.0 * p.sigma * ex2, dsy_ds = dy_dz * 2.0 * p.sigma * ey2;
    const double dsx_dt = dx_dz * p.sigma * p.sigma * (2.0 / 3.0) * ex2 / p.tau;
    const double dsy_dt = dy_dz * p.sigma * p.sigma * (2.0 / 3.0) * ey2 / p.tau;
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
                        const float dx = bx + Codec<S>::dec(v.ox[s]);
                        const float dy = by + Codec<S>::dec(v.oy[s]);
                        const float a = Codec<S>::age(v.ta[s], p.t_now, p.dt_ref);
                        const float e = -(dx * dx * c.cx + dy * dy * c.cy + a * a * c.ct);
                        const float pi = expf(e - m) * inv;
                        const float h = g0 * (Codec<S>::dec(v.r[s]) - C0) +
                                        g1 * (Codec<S>::dec(v.g[s]) - C1) +
                                        g2 * (Codec<S>::dec(v.b[s]) - C2);
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
            const float ox = Codec<S>::dec(v.ox[s]), oy = Codec<S>::dec(v.oy[s]);
            const float a = Codec<S>::age(v.ta[s], p.t_now, p.dt_ref);
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

__global__ __launch_bounds__(256) void k_reduce_params(const double *__restrict__ partial, int nb,
                                                       float *__restrict__ out) {
    __shared__ double s[2][256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
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

}  // namespace

size_t backward_ws_bytes(int32_t w, int32_t h) {
    const size_t hw = (size_t)w * h;
    const dim3 g = pixel_grid(w, h);
    return align_up(3 * hw * 4) + align_up((size_t)g.x * g.y * 2 * 8);
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
    if (buf.precision == AFR_FP16)
        return launch_bwd_typed<__half>(buf, stats, p, rgb, aux, grad_rgb, grad_slot, grad_params,
                                        ws, st);
    return launch_bwd_typed<float>(buf, stats, p, rgb, aux, grad_rgb, grad_slot, grad_params, ws,
                                   st);
}

}  // namespace afr
