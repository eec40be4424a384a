// LDS-tiled separable gather (Sec. 5.1 Gaussian space-time filter, Sec. 5.2 normalised average): the
// device routine behind afr_reconstruct, the fused forward and the batched persistent kernel.
//
// The filter is an axis-aligned Gaussian whose widths are constant over a statistics tile, so for an
// output pixel (i, j) of tile T and a slot s of the source pixel q = (i + m, j + n) the weight factors:
//   w = X(s, m) Y(s, n) Tm(s),   X = 2^(-(m + d)^2 cx),  Y = 2^(-(n + e)^2 cy),
//   Tm = 2^(-(a^2 - a_ref^2) ct),  d = ox - 1/2, e = oy - 1/2,
// with cx = log2(e) / (2 sx2), cy = log2(e) / (2 sy2), ct = log2(e) kt2 / 2 from T's statistics.
//
// Work split. A workgroup of TPG waves handles TPG horizontally adjacent tiles of one tile row; wave t
// owns tile t and each of its lanes one output pixel. For every slot plane the workgroup first
// evaluates, for every source pixel of each tile's (8+2R)^2 region, a table of 2(2R+1) factors and the
// slot's colour (the factor stage: TPG (8+2R)^2 evaluations spread evenly over all lanes of the
// workgroup), then every lane adds its pixel's (2R+1)^2 terms (the pair stage): one multiply and four
// fused multiply-adds per (slot, pixel) pair, every LDS index a compile-time offset from the lane's
// base. With binary16 storage the colours stay in LDS as the stored halves and feed mixed-precision
// FMAs.
//
// Factor stage (recurrence form): with u = d - R the table holds
//   Xr(m) = X(m) / X(-R)             (Xr(-R) = 1),
//   Yr(n) = X(-R) Y(n) Tm,
// so that Xr(m) Yr(n) = w. Yr(-R) is one exponential, 2^(-u^2 cx - v^2 cy - (a^2 - a_ref^2) ct)
// (v = e - R), evaluated 2^32 up and scaled back so that it keeps subnormal values; the ratios
// X(m+1)/X(m) = 2^(-(2(u + m + R) + 1) cx) start from one exponential and advance by the tile
// constant qx = 2^(-2 cx) (likewise for Y). Three exponentials per evaluation in all. Starting at the
// smallest value, the recurrences amplify the absolute rounding of a subnormal start by at most
// 2^((R+1/2)^2 (cx + cy)); tiles allow them when that exponent is <= 40 (the default width floor of
// 0.5 px gives 36 at R = 2), so every weight carries an absolute error below 2^-110. Narrower tiles
// (caller-supplied statistics) take the direct form, one exponential per value, normalised at m = 0:
// Xr(m) = 2^(-m (m + 2d) cx) <= 1, Yr(n) = X(0) Y(n) Tm.
//
// Shift: a_ref is the smallest slot-0 age over the tile's source region (slot 0 is each pixel's
// newest sample), so every Tm <= 1. A pixel whose weight sum falls below 2^-80 (its block's samples
// are all far older than the region's newest) is recomputed exactly by the direct two-pass form, so
// the weights' absolute errors stay below 2^-30 of every normalised sum. aux receives (m, W) with
// m = -a_ref^2 kt2 / 2 and W = sum exp(E - m), which is what the adjoint needs.
//
// Loads: each evaluation's slot of the next plane is fetched while the current plane's pairs are
// added (one 12-byte load for a binary16 slot record, six 4-byte loads for binary32 planes). The
// evaluations of a workgroup are dealt to consecutive lanes in table order; lanes past the last one
// evaluate nothing useful and write a dummy entry of their own, so that the common case runs without
// per-lane branches.
//
// Accumulation: each slot plane's (2R+1)^2 terms (source row, then column) go into a binary32
// partial, and the partials of the K planes are added in plane order in binary64. Planes beyond a
// tile's own occupancy add exact zeros. Every pixel sums the same terms in the same order for any
// TPG, so the output does not depend on the launch shape.
//
// LDS layout: entry e of a tile pair's region table sits at row r, column c of a row of PITCH entries
// holding both tiles' rows side by side (tile 2p at [0, RW), 2p + 1 at [RW, 2 RW)); each factor is an
// array over entries, colours a third array. PITCH = 24 (R <= 2) or 40 makes the 8 x 8 lanes of a wave
// read 64 distinct banks for the factors and, per half wave, distinct bank pairs for the binary16
// colours; the factor stage writes consecutive entries from consecutive lanes.
#pragma once
#include <type_traits>

#include "afr_internal.h"

namespace afr {
namespace gat {

constexpr float kLog2e = 1.4426950408889634f;
constexpr int kB = 8;                    // statistics tile edge handled by this routine
constexpr double kTinySum = 0x1p-80;     // weight sums below this take the direct form
constexpr float kRecBound = 40.0f;       // (R + 1/2)^2 (cx + cy) above this: direct factors

struct TiledParams {
    float t_now, dt_ref;
};

// Per-tile constants of one workgroup.
struct TileConst {
    float cx, qx, cy, qy;  // log2 inverse half-variances, recurrence steps 2^(-2c)
    float ct, lt0;         // temporal rate; ct a_ref^2 (+32 for the recurrence form)
    float shift;           // aux shift -a_ref^2 kt2 / 2 (natural log units)
    int rec;               // recurrence form allowed
};

template <int R, int TPG>
struct Layout {
    static constexpr int RW = kB + 2 * R;                 // region edge
    static constexpr int NM = 2 * R + 1;                  // offsets per axis
    static constexpr int NP = RW * RW;                    // region pixels per tile
    static constexpr int PITCH = (2 * RW <= 24) ? 24 : 40;
    static constexpr int PAIRS = (TPG + 1) / 2;           // tile pairs
    static constexpr int PAIR_ENTRIES = RW * PITCH;
    static constexpr int NE = (PAIRS * PAIR_ENTRIES + 63) / 64 * 64;  // entries per array
    static constexpr int NED = NE + 64;  // plus one dummy entry per lane for idle evaluations
    static constexpr int NEVAL = TPG * NP;                // evaluations per plane
    static constexpr int THREADS = 64 * TPG;
    static constexpr int ROUNDS = (NEVAL + THREADS - 1) / THREADS;
};

template <typename S>
struct ColourWord;  // one slot's colour as held in LDS
template <>
struct ColourWord<__half> {
    using T = uint2;  // (r | g << 16, b)
};
template <>
struct ColourWord<float> {
    using T = float4;  // (r, g, b, 0)
};

template <typename S, int R, int TPG>
struct Smem {
    using L = Layout<R, TPG>;
    float XY[2 * L::NM][L::NED];  // Xr(m) at [m + R], Yr(n) at [NM + n + R]
    typename ColourWord<S>::T col[L::NED];
    TileConst tc[TPG];
    unsigned amin_bits[TPG];
    int kmax;
};

// Exact two-pass evaluation of one pixel (the direct form), used when the shared shift underflows.
// cx, cy, ct are the natural-log coefficients 1/(2 sx2), 1/(2 sy2), kt2/2.
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
                const float dx = bx + Codec<S>::dec(fld(v.ox, s));
                const float dy = by + Codec<S>::dec(fld(v.oy, s));
                const float a = Codec<S>::age(fld(v.ta, s), p.t_now, p.dt_ref);
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
                    const float dx = bx + Codec<S>::dec(fld(v.ox, s));
                    const float dy = by + Codec<S>::dec(fld(v.oy, s));
                    const float a = Codec<S>::age(fld(v.ta, s), p.t_now, p.dt_ref);
                    const float w = expf(-(dx * dx * cx + dy * dy * cy + a * a * ct) - emax);
                    ws += w;
                    cr += w * Codec<S>::dec(fld(v.r, s));
                    cg += w * Codec<S>::dec(fld(v.g, s));
                    cb += w * Codec<S>::dec(fld(v.b, s));
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

// Raw stored fields of one slot: the binary16 record as its three 32-bit words (ox | oy, r | g,
// b | age_ref), which are already the colour word the LDS table holds; binary32 fields one per
// register. The prefetch of the next plane lands here and is first touched by the next factor
// stage.
template <typename S>
struct RawSlot;
template <>
struct RawSlot<__half> {
    uint3 w;
};
template <>
struct RawSlot<float> {
    float ox, oy, ta, r, g, b;
};

__device__ inline void load_slot(RawSlot<__half> &d, const BufView<__half> &v, size_t plane,
                                 size_t hw, unsigned px) {
    const auto rs = plane_rsrc(v.ox + plane * hw * Slots<__half>::kStride, hw * Slots<__half>::kBytes);
    d.w = load_u32x3(rs, px * (unsigned)Slots<__half>::kBytes);
}
__device__ inline void load_slot(RawSlot<float> &d, const BufView<float> &v, size_t plane,
                                 size_t hw, unsigned px) {
    const size_t base = plane * hw, bytes = hw * sizeof(float);
    const unsigned off = px * (unsigned)sizeof(float);
    d.ox = plane_load<float>(plane_rsrc(v.ox + base, bytes), off);
    d.oy = plane_load<float>(plane_rsrc(v.oy + base, bytes), off);
    d.ta = plane_load<float>(plane_rsrc(v.ta + base, bytes), off);
    d.r = plane_load<float>(plane_rsrc(v.r + base, bytes), off);
    d.g = plane_load<float>(plane_rsrc(v.g + base, bytes), off);
    d.b = plane_load<float>(plane_rsrc(v.b + base, bytes), off);
}

__device__ inline float half_lo(unsigned w) { return __half2float(__ushort_as_half((unsigned short)(w & 0xffffu))); }
__device__ inline float half_hi(unsigned w) { return __half2float(__ushort_as_half((unsigned short)(w >> 16))); }

// Position offsets and colour of a slot, all 0 for an empty slot (or a pixel outside the image) so
// that every factor stays finite whatever the buffer holds there.
__device__ inline float slot_ox(const RawSlot<__half> &d, bool on) { return on ? half_lo(d.w.x) : 0.0f; }
__device__ inline float slot_oy(const RawSlot<__half> &d, bool on) { return on ? half_hi(d.w.x) : 0.0f; }
__device__ inline float slot_age(const RawSlot<__half> &d, const TiledParams &p) {
    return p.dt_ref + half_hi(d.w.z);
}
__device__ inline uint2 slot_colour(const RawSlot<__half> &d, bool on) {
    return make_uint2(on ? d.w.y : 0u, on ? d.w.z : 0u);  // (r | g, b | age): b is the low half
}
__device__ inline float slot_ox(const RawSlot<float> &d, bool on) { return on ? d.ox : 0.0f; }
__device__ inline float slot_oy(const RawSlot<float> &d, bool on) { return on ? d.oy : 0.0f; }
__device__ inline float slot_age(const RawSlot<float> &d, const TiledParams &p) {
    return p.t_now - d.ta;
}
__device__ inline float4 slot_colour(const RawSlot<float> &d, bool on) {
    return on ? make_float4(d.r, d.g, d.b, 0.0f) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Adds one pair's weight and colour to a pixel's plane partial.
__device__ inline void add_pair(float (&part)[4], float w, const uint2 &c) {
    part[0] += w;
    part[1] = fmaf(w, __low2float(__builtin_bit_cast(__half2, c.x)), part[1]);
    part[2] = fmaf(w, __high2float(__builtin_bit_cast(__half2, c.x)), part[2]);
    part[3] = fmaf(w, __low2float(__builtin_bit_cast(__half2, c.y)), part[3]);
}
__device__ inline void add_pair(float (&part)[4], float w, const float4 &c) {
    part[0] += w;
    part[1] = fmaf(w, c.x, part[1]);
    part[2] = fmaf(w, c.y, part[2]);
    part[3] = fmaf(w, c.z, part[3]);
}

// Gathers the tiles tx0 .. tx0+TPG-1 of tile row ty with a workgroup of 64 TPG threads (wave t owns
// tile tx0 + t). tparam (LDS or global, visible to every thread on entry) holds each tile's
// (sx2, sy2, kt2); a tile at or beyond tiles_x is skipped. The caller must not touch sm until the
// workgroup has passed a barrier after this routine returns.
template <typename S, int R, int TPG>
__device__ void gather_strip(const BufView<S> &v, const TiledParams &p, const TileGeom &tg, int tx0,
                             int ty, Smem<S, R, TPG> &sm, const float *tparam,
                             float *__restrict__ rgb, float *__restrict__ aux) {
    using L = Layout<R, TPG>;
    constexpr int RW = L::RW, NM = L::NM, PITCH = L::PITCH, ROUNDS = L::ROUNDS;
    using ColT = typename ColourWord<S>::T;

    const int W = v.width, H = v.height;
    const size_t hw = (size_t)W * H;
    const int tid = threadIdx.x;

    // ---- per-tile constants --------------------------------------------------------------------
    if (tid < TPG) {
        const float sx2 = tparam[3 * tid], sy2 = tparam[3 * tid + 1], kt2 = tparam[3 * tid + 2];
        TileConst c;
        c.cx = kLog2e * (0.5f / sx2);
        c.cy = kLog2e * (0.5f / sy2);
        c.ct = kLog2e * (0.5f * kt2);
        c.qx = __builtin_amdgcn_exp2f(-2.0f * c.cx);
        c.qy = __builtin_amdgcn_exp2f(-2.0f * c.cy);
        c.rec = (R + 0.5f) * (R + 0.5f) * (c.cx + c.cy) <= kRecBound;
        c.lt0 = 0.0f;
        c.shift = 0.0f;
        sm.tc[tid] = c;
        sm.amin_bits[tid] = 0x7f800000u;  // +inf
    }
    if (tid == 0) sm.kmax = 0;

    // ---- this thread's evaluations: entry, tile, source pixel ------------------------------------
    // Evaluation e = it * THREADS + tid covers entry e of the tables (consecutive lanes write
    // consecutive entries), for tile t and region pixel (r, c).
    int ent[ROUNDS], til[ROUNDS], cnt[ROUNDS];
    unsigned pix[ROUNDS];
    bool vld[ROUNDS];
#pragma unroll
    for (int it = 0; it < ROUNDS; ++it) {
        const int e = it * L::THREADS + tid;
        int t = 0, r = 0, c = 0, entry = 0;
        if (TPG == 1) {
            r = e / RW;
            c = e % RW;
            entry = r * PITCH + c;
        } else {
            const int pr = e / (2 * L::NP), rem = e % (2 * L::NP);
            r = rem / (2 * RW);
            const int cc = rem % (2 * RW);
            t = 2 * pr + (cc >= RW ? 1 : 0);
            c = cc >= RW ? cc - RW : cc;
            entry = pr * L::PAIR_ENTRIES + r * PITCH + cc;
        }
        const int qx = (tx0 + t) * kB - R + c, qy = ty * kB - R + r;
        const bool live = e < L::NEVAL && tx0 + t < tg.tiles_x && qx >= 0 && qx < W && qy >= 0 &&
                          qy < H;
        const int iq = live ? qy * W + qx : 0;
        vld[it] = e < L::NEVAL;
        ent[it] = e < L::NEVAL ? entry : L::NE + tid % kWave;  // idle: the lane's dummy entry
        til[it] = min(t, TPG - 1);  // (an evaluation past the last one has no tile)
        cnt[it] = live ? v.count[iq] : 0;
        pix[it] = (unsigned)iq;
    }
    // plane 0 of every evaluation, then the region's smallest slot-0 age and deepest pixel
    RawSlot<S> raw[ROUNDS];
#pragma unroll
    for (int it = 0; it < ROUNDS; ++it) load_slot(raw[it], v, 0, hw, pix[it]);
    __syncthreads();  // tile constants and counters initialised
    int kmy = 0;
#pragma unroll
    for (int it = 0; it < ROUNDS; ++it) {
        kmy = max(kmy, cnt[it]);
        if (cnt[it] > 0) {
            const float a = fmaxf(slot_age(raw[it], p), 0.0f);
            atomicMin(&sm.amin_bits[til[it]], __float_as_uint(a));
        }
    }
    if (kmy > 0) atomicMax(&sm.kmax, kmy);
    __syncthreads();
    if (tid < TPG) {
        TileConst &c = sm.tc[tid];
        float amin = __uint_as_float(sm.amin_bits[tid]);
        if (!(amin < INFINITY)) amin = 0.0f;  // empty region: any shift works
        c.lt0 = c.ct * (amin * amin) + (c.rec ? 32.0f : 0.0f);
        c.shift = -(amin * amin) * (0.5f * tparam[3 * tid + 2]);
    }
    __syncthreads();
    const int kmax = sm.kmax;
    TileConst tcs[ROUNDS];
#pragma unroll
    for (int it = 0; it < ROUNDS; ++it) tcs[it] = sm.tc[til[it]];

    // ---- output pixel of this lane -----------------------------------------------------------------
    const int wave = tid / kWave, lane = tid % kWave;
    const int pj = lane / kB, pi = lane % kB;
    const int base = (wave / 2) * L::PAIR_ENTRIES + pj * PITCH + (wave & 1) * RW + pi;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};

    // Factor stage of plane k for evaluation it (raw data d). REC: the recurrence form.
    auto factor = [&](int it, int k, const RawSlot<S> &d, auto rec_c) {
        constexpr bool REC = decltype(rec_c)::value;
        const TileConst &tc = tcs[it];
        const bool on = k < cnt[it];
        float X[NM], Y[NM];
        const float age = slot_age(d, p);
        if constexpr (REC) {
            const float u = slot_ox(d, on) - (R + 0.5f), w = slot_oy(d, on) - (R + 0.5f);
            float z = fmaf(-tc.ct, age * age, tc.lt0);
            z = fmaf(-(u * tc.cx), u, z);
            z = fmaf(-(w * tc.cy), w, z);
            z = on ? z : -INFINITY;
            Y[0] = __builtin_amdgcn_exp2f(z) * 0x1p-32f;
            X[0] = 1.0f;
            if (R > 0) {
                float rx = __builtin_amdgcn_exp2f(fmaf(u, -2.0f * tc.cx, -tc.cx));
                float ry = __builtin_amdgcn_exp2f(fmaf(w, -2.0f * tc.cy, -tc.cy));
                X[1] = rx;
                Y[1] = Y[0] * ry;
#pragma unroll
                for (int m = 2; m < NM; ++m) {
                    rx *= tc.qx;
                    ry *= tc.qy;
                    X[m] = X[m - 1] * rx;
                    Y[m] = Y[m - 1] * ry;
                }
            }
        } else {
            const float dx = slot_ox(d, on) - 0.5f, dy = slot_oy(d, on) - 0.5f;
            float z0 = fmaf(-tc.ct, age * age, tc.lt0);
            z0 = fmaf(-(dx * tc.cx), dx, z0);
            z0 = on ? z0 : -INFINITY;
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                const float fm = (float)(m - R);
                X[m] = __builtin_amdgcn_exp2f(-(fm * fmaf(2.0f, dx, fm)) * tc.cx);
                const float ey = dy + fm;
                Y[m] = __builtin_amdgcn_exp2f(fmaf(-(ey * tc.cy), ey, z0));
            }
        }
        const int e = ent[it];
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            sm.XY[m][e] = X[m];
            sm.XY[NM + m][e] = Y[m];
        }
        sm.col[e] = slot_colour(d, on);
    };
    // One plane: factor stage, barrier, prefetch of plane k + 1 into the registers just consumed,
    // pair stage, barrier. The prefetch sits in the same scheduling region as the pair stage (no
    // branch around it: past the last plane it reloads plane K-1, unused), so the pairs cover its
    // latency.
    auto plane = [&](int k, RawSlot<S>(&rs)[ROUNDS]) {
#pragma unroll
        for (int it = 0; it < ROUNDS; ++it) {
            // wave-uniform choices keep the common case free of per-lane branches; an idle lane
            // writes its dummy entry
            if (!__any(vld[it])) continue;
            if (__all(tcs[it].rec != 0) || tcs[it].rec)
                factor(it, k, rs[it], std::true_type{});
            else
                factor(it, k, rs[it], std::false_type{});
        }
        __syncthreads();
        {
            const int nk = min(k + 1, v.k - 1);
#pragma unroll
            for (int it = 0; it < ROUNDS; ++it) load_slot(rs[it], v, nk, hw, pix[it]);
        }
        // pair stage: source row n, then column m
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int n = 0; n < NM; ++n)
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                const int e = base + n * PITCH + m;
                const float w = sm.XY[m][e] * sm.XY[NM + n][e];
                const ColT c = sm.col[e];
                add_pair(part, w, c);
            }
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += (double)part[c];
        __syncthreads();
    };
    for (int k = 0; k < kmax; ++k) plane(k, raw);

    // ---- output --------------------------------------------------------------------------------
    const int tcol = tx0 + wave;
    const int i = tcol * kB + pi, j = ty * kB + pj;
    if (tcol >= tg.tiles_x || i >= W || j >= H) return;  // no barrier follows
    const size_t px = (size_t)j * W + i;
    const double ws = acc[0];
    if (ws >= kTinySum) {
        const double inv = 1.0 / ws;
        rgb[px] = (float)(acc[1] * inv);
        rgb[hw + px] = (float)(acc[2] * inv);
        rgb[2 * hw + px] = (float)(acc[3] * inv);
        if (aux) {
            aux[px] = sm.tc[wave].shift;
            aux[hw + px] = (float)ws;
        }
    } else {
        const float sx2 = tparam[3 * wave], sy2 = tparam[3 * wave + 1], kt2 = tparam[3 * wave + 2];
        direct_pixel<S>(v, p, R, i, j, 0.5f / sx2, 0.5f / sy2, 0.5f * kt2, rgb, aux);
    }
}

}  // namespace gat
}  // namespace afr
