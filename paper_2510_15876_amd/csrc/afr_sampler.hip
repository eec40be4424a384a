// Sampler feedback statistics (Sec. 4, 4.1, 6.1) and error-proportional tile selection.
//
//   k_smp_tiles    one wave per tile of the sampler's buffer: the tile's sample count and mean
//                  sample age (FP64), plus its variation and mean gradients from the statistics
//   k_smp_global   one workgroup: fixed-order FP64 reductions over tiles (sample total, variation,
//                  gradients, ages), then each tile's undersampling u_T, their sum, each tile's error
//                  E_T and the gain-control figures
//   k_smp_weights  one workgroup: integer tile weights q_T = floor(E_T / E_max 2^24) and their
//                  exclusive prefix sum (exact, so independent of the scan's order)
//   k_smp_draw     one thread per new sample: the tile whose weight interval holds the draw (binary
//                  search over the prefix sums) and a uniform spot inside it, in binary32
#include <mutex>

#include "afr_internal.h"

namespace afr {
namespace {

constexpr int kGThreads = 1024;

struct TilePart {
    double empty, age, v, gs, gt;  // empty slots; mean age (or -1 if the tile holds no sample)
};

template <typename S>
__global__ __launch_bounds__(kWave) void k_smp_tiles(BufView<S> v, double t_now, double dt_ref,
                                                     TileGeom tg, const float *__restrict__ stats,
                                                     TilePart *part) {
    const int T = blockIdx.x;
    const int tx = T % tg.tiles_x, ty = T / tg.tiles_x, B = tg.tile;
    const int i0 = tx * B, j0 = ty * B;
    const int bw = min(B, v.width - i0), bh = min(B, v.height - j0);
    const size_t plane = (size_t)v.width * v.height;
    double n = 0.0, a = 0.0;
    for (int e = threadIdx.x; e < bw * bh; e += kWave) {
        const size_t px = (size_t)(j0 + e / bw) * v.width + i0 + e % bw;
        const int c = v.count[px];
        for (int k = 0; k < c; ++k) {
            n += 1.0;
            a += Codec<S>::age64(fld(v.ta, (size_t)k * plane + px), t_now, dt_ref);
        }
    }
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) {
        n += __shfl_xor(n, m, kWave);
        a += __shfl_xor(a, m, kWave);
    }
    if (threadIdx.x != 0) return;
    const int nt = tg.nt;
    TilePart p;
    p.empty = (double)bw * bh * v.k - n;
    p.age = n > 0.0 ? a / n : -1.0;
    p.v = stats[AFR_STAT_VAR * nt + T];
    p.gs = 0.5 * ((double)stats[AFR_STAT_GX * nt + T] + (double)stats[AFR_STAT_GY * nt + T]);
    p.gt = stats[AFR_STAT_GT * nt + T];
    part[T] = p;
}

// Sum of one double per thread over the workgroup in a fixed order; the result is valid in every
// thread.
__device__ inline double block_sum(double x, double *sh) {
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) x += __shfl_xor(x, m, kWave);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) sh[w] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kGThreads / kWave; ++i) t += sh[i];
    return t;
}

struct SmpParams {
    double kappa, lambda, m, gain;
};

__global__ __launch_bounds__(kGThreads) void k_smp_global(const TilePart *__restrict__ part,
                                                           TileGeom tg, int W, int H, int K,
                                                           SmpParams sp, float *E, float *u,
                                                           double *glob) {
    __shared__ double sh[kGThreads / kWave];
    const int nt = tg.nt;
    double empty = 0.0, sv = 0.0, sgs = 0.0, sgt = 0.0, sage = 0.0, naged = 0.0;
    for (int T = threadIdx.x; T < nt; T += kGThreads) {
        const TilePart p = part[T];
        empty += p.empty;
        sv += p.v;
        sgs += p.gs;
        sgt += p.gt;
        if (p.age >= 0.0) {
            sage += p.age;
            naged += 1.0;
        }
    }
    empty = block_sum(empty, sh);
    sv = block_sum(sv, sh);
    sgs = block_sum(sgs, sh);
    sgt = block_sum(sgt, sh);
    sage = block_sum(sage, sh);
    naged = block_sum(naged, sh);
    const double e = empty / (double)nt;  // empty slots are exact integers in FP64
    double su = 0.0;
    for (int T = threadIdx.x; T < nt; T += kGThreads) {
        const double et = part[T].empty;
        const double ut = et > 0.0 ? 1.0 - fmin(1.0, sp.m * e / et) : 0.0;
        u[T] = (float)ut;
        su += ut;
    }
    su = block_sum(su, sh);
    for (int T = threadIdx.x; T < nt; T += kGThreads) {
        const int tx = T % tg.tiles_x, ty = T / tg.tiles_x;
        const int bw = min(tg.tile, W - tx * tg.tile), bh = min(tg.tile, H - ty * tg.tile);
        const double et = part[T].empty;
        const double ut = et > 0.0 ? 1.0 - fmin(1.0, sp.m * e / et) : 0.0;
        double x = 0.0;
        if (sv > 0.0) x += sp.kappa * part[T].v / sv;
        if (su > 0.0) x += sp.lambda * ut / su;
        E[T] = (float)((double)bw * bh * x);
    }
    if (threadIdx.x == 0) {
        const double dcds = sgs / (double)nt, dcdt = sgt / (double)nt;
        const double tbar = naged > 0.0 ? sage / naged : 0.0;
        double S, target;
        if (dcdt == 0.0) {  // static content: the finest tiling
            S = 0.0;
            target = INFINITY;
        } else if (dcds == 0.0) {
            S = INFINITY;
            target = 0.0;
        } else {
            S = sp.gain * dcdt * tbar / dcds;
            target = S > 0.0 ? (double)W * H / (S * S) : INFINITY;
        }
        glob[0] = sv;
        glob[1] = su;
        glob[2] = e;
        glob[3] = dcds;
        glob[4] = dcdt;
        glob[5] = tbar;
        glob[6] = S;
        glob[7] = target;
    }
    (void)K;
}

__global__ __launch_bounds__(kGThreads) void k_smp_weights(const float *__restrict__ E, int nt,
                                                            unsigned long long *cum) {
    __shared__ float smax[kGThreads / kWave];
    __shared__ unsigned long long ssum[kGThreads / kWave];
    // largest positive finite error (exact: a maximum)
    float m = 0.0f;
    for (int T = threadIdx.x; T < nt; T += kGThreads) {
        const float x = E[T];
        if (isfinite(x) && x > m) m = x;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, kWave));
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == 0) smax[w] = m;
    __syncthreads();
    m = 0.0f;
    for (int i = 0; i < kGThreads / kWave; ++i) m = fmaxf(m, smax[i]);
    const double emax = m;
    // each thread owns a contiguous run of tiles; runs are scanned in thread order
    const int per = (nt + kGThreads - 1) / kGThreads;
    const int t0 = min(nt, threadIdx.x * per), t1 = min(nt, t0 + per);
    auto weight = [&](int T) -> unsigned long long {
        if (!(emax > 0.0)) return 1ull;
        const float x = E[T];
        return (isfinite(x) && x > 0.0f) ? (unsigned long long)floor((double)x / emax * 16777216.0)
                                         : 0ull;
    };
    unsigned long long run = 0;
    for (int T = t0; T < t1; ++T) run += weight(T);
    // exclusive scan of the run totals across the workgroup
    unsigned long long incl = run;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const unsigned long long n = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += n;
    }
    if (lane == kWave - 1) ssum[w] = incl;
    __syncthreads();
    unsigned long long base = incl - run;
    for (int i = 0; i < w; ++i) base += ssum[i];
    for (int T = t0; T < t1; ++T) {
        cum[T] = base;
        base += weight(T);
    }
    if (threadIdx.x == kGThreads - 1) cum[nt] = base;
}

struct DrawGeom {
    int W, H, B, tiles_x, nt;
};

__global__ __launch_bounds__(256) void k_smp_draw(const unsigned long long *__restrict__ cum,
                                                   DrawGeom g, const uint32_t *__restrict__ rnd,
                                                   int64_t n, float *x, float *y, int32_t *tile) {
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const unsigned long long Q = cum[g.nt];
    const unsigned long long target = ((unsigned long long)(rnd[k] >> 8) * Q) >> 24;
    int lo = 0, hi = g.nt;  // the T with cum[T] <= target < cum[T + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] <= target) lo = mid;
        else hi = mid;
    }
    const int tx = lo % g.tiles_x, ty = lo / g.tiles_x;
    const int x0 = tx * g.B, y0 = ty * g.B;
    const int bw = min(g.B, g.W - x0), bh = min(g.B, g.H - y0);
    const float u1 = (float)(rnd[n + k] >> 8) * 5.9604644775390625e-8f;
    const float u2 = (float)(rnd[2 * n + k] >> 8) * 5.9604644775390625e-8f;
    const float xs = (float)x0 + u1 * (float)bw, ys = (float)y0 + u2 * (float)bh;
    const float xe = (float)(x0 + bw), ye = (float)(y0 + bh);
    x[k] = xs < xe ? xs : __uint_as_float(__float_as_uint(xe) - 1u);
    y[k] = ys < ye ? ys : __uint_as_float(__float_as_uint(ye) - 1u);
    if (tile) tile[k] = lo;
}

// ---- equal-error tiles along the Z-curve ---------------------------------------------------------

__device__ inline uint32_t spread_bits(uint32_t v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Position of tile (tx, ty) on the Z-curve over a tiles_x x tiles_y grid: the number of tiles
// whose code is smaller. For each set bit of the code, the codes that agree above it and have a 0
// there fix the high bits of x and of y and leave the low ones free; their count inside the grid
// is a product of two clamped ranges.
__device__ inline int z_rank(int tx, int ty, int tiles_x, int tiles_y) {
    const uint32_t c = spread_bits(tx) | (spread_bits(ty) << 1);
    long long rank = 0;
    for (int i = 31; i >= 0; --i) {
        if (!((c >> i) & 1u)) continue;
        const int fx = (i + 1) / 2, fy = i / 2;  // free low bits of x and y below position i
        // fixed high bits: those of c above i, with bit i cleared
        const uint32_t hi = (c >> i) & ~1u;
        uint32_t px = 0, py = 0;
        for (int b = 0; b < 32; ++b) {
            const int pos = i + b;
            if (pos > 31) break;
            const uint32_t bit = (hi >> b) & 1u;
            if (pos % 2 == 0) px |= bit << (pos / 2 - fx);
            else py |= bit << ((pos - 1) / 2 - fy);
        }
        const long long nx = min(max((long long)tiles_x - ((long long)px << fx), 0ll), 1ll << fx);
        const long long ny = min(max((long long)tiles_y - ((long long)py << fy), 0ll), 1ll << fy);
        rank += nx * ny;
    }
    return (int)rank;
}

struct WeightsGeom {
    int W, H, B, tiles_x, tiles_y, nt;
};

__global__ __launch_bounds__(256) void k_smp_zorder(WeightsGeom g, int32_t *perm) {
    const int T = blockIdx.x * 256 + threadIdx.x;
    if (T >= g.nt) return;
    perm[z_rank(T % g.tiles_x, T / g.tiles_x, g.tiles_x, g.tiles_y)] = T;
}

__device__ inline int tile_area(int T, const WeightsGeom &g) {
    const int tx = T % g.tiles_x, ty = T / g.tiles_x;
    return min(g.B, g.W - tx * g.B) * min(g.B, g.H - ty * g.B);
}

// Exclusive prefix sums along the curve of the integer error weights (C) and of the tile areas (A).
__global__ __launch_bounds__(kGThreads) void k_smp_zscan(const float *__restrict__ E,
                                                          const int32_t *__restrict__ perm,
                                                          WeightsGeom g, unsigned long long *C,
                                                          long long *A) {
    __shared__ float smax[kGThreads / kWave];
    __shared__ unsigned long long sq[kGThreads / kWave];
    __shared__ long long sa[kGThreads / kWave];
    const int nt = g.nt;
    float m = 0.0f;
    for (int T = threadIdx.x; T < nt; T += kGThreads) {
        const float x = E[T];
        if (isfinite(x) && x > m) m = x;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, kWave));
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == 0) smax[w] = m;
    __syncthreads();
    m = 0.0f;
    for (int i = 0; i < kGThreads / kWave; ++i) m = fmaxf(m, smax[i]);
    const double emax = m;
    auto weight = [&](int T) -> unsigned long long {
        const float x = E[T];
        return (emax > 0.0 && isfinite(x) && x > 0.0f)
                   ? (unsigned long long)floor((double)x / emax * 16777216.0)
                   : 0ull;
    };
    const int per = (nt + kGThreads - 1) / kGThreads;
    const int m0 = min(nt, threadIdx.x * per), m1 = min(nt, m0 + per);
    unsigned long long rq = 0;
    long long ra = 0;
    for (int i = m0; i < m1; ++i) {
        rq += weight(perm[i]);
        ra += tile_area(perm[i], g);
    }
    unsigned long long iq = rq;
    long long ia = ra;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const unsigned long long nq = __shfl_up(iq, o, kWave);
        const long long na = __shfl_up(ia, o, kWave);
        if (lane >= o) {
            iq += nq;
            ia += na;
        }
    }
    if (lane == kWave - 1) {
        sq[w] = iq;
        sa[w] = ia;
    }
    __syncthreads();
    unsigned long long bq = iq - rq;
    long long ba = ia - ra;
    for (int i = 0; i < w; ++i) {
        bq += sq[i];
        ba += sa[i];
    }
    for (int i = m0; i < m1; ++i) {
        C[i] = bq;
        A[i] = ba;
        bq += weight(perm[i]);
        ba += tile_area(perm[i], g);
    }
    if (threadIdx.x == kGThreads - 1) {
        C[nt] = bq;
        A[nt] = ba;
    }
}

__device__ inline int parts_of(const double *glob, int n_parts, int nt) {
    int N = n_parts;
    if (N <= 0) {
        const double t = glob[7];
        const double r = isnan(t) ? 1.0 : rint(t);
        N = r < 1.0 ? 1 : (r > (double)nt ? nt : (int)r);
    }
    return min(N, nt);
}

__global__ __launch_bounds__(256) void k_smp_zparts(const unsigned long long *__restrict__ C,
                                                    WeightsGeom g, const double *glob, int n_parts,
                                                    int32_t *part) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= g.nt) return;
    const int N = parts_of(glob, n_parts, g.nt);
    const unsigned long long Q = C[g.nt];
    const unsigned long long p = Q ? C[m] * (unsigned long long)N / Q : 0ull;
    part[m] = p < (unsigned long long)(N - 1) ? (int)p : N - 1;
}

__global__ __launch_bounds__(256) void k_smp_zweights(const int32_t *__restrict__ perm,
                                                      const unsigned long long *__restrict__ C,
                                                      const long long *__restrict__ A,
                                                      const int32_t *__restrict__ part,
                                                      WeightsGeom g, const double *glob,
                                                      int n_parts, float *P) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= g.nt) return;
    const int T = perm[m];
    const double s = (double)(A[m + 1] - A[m]);
    if (C[g.nt] == 0ull) {
        P[T] = (float)s;
        return;
    }
    const int pm = part[m];
    int lo = 0, hi = m;  // first position of this part: part[lo] == pm, lo <= m
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (part[mid] < pm) lo = mid + 1;
        else hi = mid;
    }
    int lo2 = m + 1, hi2 = g.nt;  // first position after this part
    while (lo2 < hi2) {
        const int mid = (lo2 + hi2) >> 1;
        if (part[mid] <= pm) lo2 = mid + 1;
        else hi2 = mid;
    }
    const int N = parts_of(glob, n_parts, g.nt);
    const int next = m + 1 < g.nt ? part[m + 1] : N;
    const int extra = max(0, next - pm - 1);
    P[T] = (float)(s / (double)(A[lo2] - A[lo]) + (double)extra);
}

}  // namespace

size_t sampler_ws_bytes(int32_t tiles) {
    const size_t nt = (size_t)tiles;
    return align_up(nt * sizeof(TilePart)) + align_up((nt + 1) * 8) +  // stats parts, select prefix
           align_up(nt * 4) + 2 * align_up((nt + 1) * 8) + align_up(nt * 4);  // Z-curve order, C, A, parts
}

hipError_t launch_sampler_tile_weights(int32_t w, int32_t h, int32_t tile, const float *E,
                                       const double *glob, int32_t n_parts, float *P, void *ws,
                                       hipStream_t st) {
    const int tiles_x = (w + tile - 1) / tile, tiles_y = (h + tile - 1) / tile;
    const int nt = tiles_x * tiles_y;
    char *p = static_cast<char *>(ws) + align_up((size_t)nt * sizeof(TilePart)) +
              align_up((size_t)(nt + 1) * 8);
    int32_t *perm = reinterpret_cast<int32_t *>(p);
    p += align_up((size_t)nt * 4);
    unsigned long long *C = reinterpret_cast<unsigned long long *>(p);
    p += align_up((size_t)(nt + 1) * 8);
    long long *A = reinterpret_cast<long long *>(p);
    p += align_up((size_t)(nt + 1) * 8);
    int32_t *part = reinterpret_cast<int32_t *>(p);
    const WeightsGeom g{w, h, tile, tiles_x, tiles_y, nt};
    const int nb = (nt + 255) / 256;
    k_smp_zorder<<<nb, 256, 0, st>>>(g, perm);
    k_smp_zscan<<<1, kGThreads, 0, st>>>(E, perm, g, C, A);
    k_smp_zparts<<<nb, 256, 0, st>>>(C, g, glob, n_parts, part);
    k_smp_zweights<<<nb, 256, 0, st>>>(perm, C, A, part, g, glob, n_parts, P);
    return hipGetLastError();
}

hipError_t launch_sampler_stats(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                const afr_params &prm, const afr_sampler_params &sp, float *E,
                                float *u, double *glob, void *ws, hipStream_t st) {
    const TileGeom tg = geom_of(stats);
    TilePart *part = static_cast<TilePart *>(ws);
    const double t_now = prm.t_now, dt_ref = (double)prm.t_now - (double)buf.t_ref;
    if (buf.precision == AFR_FP16)
        k_smp_tiles<__half><<<tg.nt, kWave, 0, st>>>(view_of<__half>(buf), t_now, dt_ref, tg,
                                                     stats.data, part);
    else
        k_smp_tiles<float><<<tg.nt, kWave, 0, st>>>(view_of<float>(buf), t_now, dt_ref, tg,
                                                    stats.data, part);
    const SmpParams p{sp.kappa, sp.lambda, sp.m, sp.gain};
    k_smp_global<<<1, kGThreads, 0, st>>>(part, tg, buf.width, buf.height, buf.k, p, E, u, glob);
    return hipGetLastError();
}

// ---- spot selection without a caller workspace --------------------------------------------------
// The prefix of tile weights lives in a file-scope device array instead of the caller's workspace:
// one per GPU, held until the process ends, shared by every call on that GPU (calls that overlap on
// one GPU race). k_smp_weights rewrites all of its nt + 1 entries on every call, so nothing in it
// has to start at zero. In host code `scratch` names a host-side stand-in, not the device array: its
// device address comes from hipGetSymbolAddress, looked up once per device with that device current
// and kept per device.
static __device__ __align__(256) unsigned long long scratch[kMaxSamplerTiles + 1];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this device's scratch array (looked up on the first call on the device).
hipError_t sampler_scratch(unsigned long long **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<unsigned long long *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_sampler_select_noalloc(int32_t w, int32_t h, int32_t tile, const float *E,
                                         int64_t n, const uint32_t *rnd, float *x, float *y,
                                         int32_t *tile_out, hipStream_t st) {
    unsigned long long *cum = nullptr;
    const hipError_t e = sampler_scratch(&cum);
    if (e != hipSuccess) return e;
    const int tiles_x = (w + tile - 1) / tile, tiles_y = (h + tile - 1) / tile;
    const int nt = tiles_x * tiles_y;  // <= kMaxSamplerTiles, checked by the caller
    k_smp_weights<<<1, kGThreads, 0, st>>>(E, nt, cum);
    if (n > 0) {
        const DrawGeom g{w, h, tile, tiles_x, nt};
        k_smp_draw<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(cum, g, rnd, n, x, y, tile_out);
    }
    return hipGetLastError();
}

hipError_t launch_sampler_select(int32_t w, int32_t h, int32_t tile, const float *E, int64_t n,
                                 const uint32_t *rnd, float *x, float *y, int32_t *tile_out,
                                 void *ws, hipStream_t st) {
    const int tiles_x = (w + tile - 1) / tile, tiles_y = (h + tile - 1) / tile;
    const int nt = tiles_x * tiles_y;
    unsigned long long *cum = reinterpret_cast<unsigned long long *>(
        static_cast<char *>(ws) + align_up((size_t)nt * sizeof(TilePart)));
    k_smp_weights<<<1, kGThreads, 0, st>>>(E, nt, cum);
    if (n > 0) {
        const DrawGeom g{w, h, tile, tiles_x, nt};
        k_smp_draw<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(cum, g, rnd, n, x, y, tile_out);
    }
    return hipGetLastError();
}

}  // namespace afr
