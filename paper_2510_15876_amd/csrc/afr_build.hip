// Deep-buffer build: bin the sample stream to home pixels and keep each pixel's K newest samples.
//
// The paper's reconstructor receives samples as one stream (Sec. 4.2, Sec. 5.2) and each pixel keeps
// a queue of its newest samples (Sec. 4). Replaying queue insertions one sample at a time is serial
// per pixel; the same final state is the top-K by key (t, stream index) of the samples binned to the
// pixel, which this file computes with a counting sort:
//   1. k_build_clear   zero the per-pixel arrival counters and the dropped counter
//   2. k_build_count   validate each sample, count arrivals per home pixel (integer atomics)
//   3. scan            exclusive prefix sum of the counts -> bucket offsets
//   4. k_build_scatter write (time, index) keys into each pixel's bucket (order inside is arbitrary)
//   5. k_build_select  per pixel: register top-K over its bucket, then gather and store the slots
// Every decision is integer or an exact comparison of stored float32 inputs, so the result is
// bit-exact and independent of launch shape and atomic order.
#include "afr_internal.h"

namespace afr {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;

struct ValidCtx {
    int32_t w, h;
    float t_ref;
    int32_t fp16;
};

// Validity rule shared by the count and scatter passes (they must agree sample by sample).
__device__ inline bool sample_valid(float x, float y, float t, float r, float g, float b,
                                    const ValidCtx &c) {
    bool ok = isfinite(x) && isfinite(y) && isfinite(t) && isfinite(r) && isfinite(g) && isfinite(b);
    ok = ok && x >= 0.0f && x < (float)c.w && y >= 0.0f && y < (float)c.h && t <= c.t_ref;
    if (ok && c.fp16) {
        // binary16 round-to-nearest-even overflows to infinity exactly when |v| >= 65520
        const float age = c.t_ref - t;
        ok = age < 65520.0f && fabsf(r) < 65520.0f && fabsf(g) < 65520.0f && fabsf(b) < 65520.0f;
    }
    return ok;
}

__device__ inline int wave_sum_int(int v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__global__ void k_build_clear(int32_t *cnt, int32_t hw, unsigned long long *dropped) {
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < hw; i += stride) cnt[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *dropped = 0ull;
}

__global__ void k_build_count(afr_samples s, ValidCtx c, int32_t *cnt,
                              unsigned long long *dropped) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride) {
        const float x = s.x[i], y = s.y[i];
        if (sample_valid(x, y, s.t[i], s.r[i], s.g[i], s.b[i], c)) {
            const int p = (int)floorf(y) * c.w + (int)floorf(x);
            atomicAdd(&cnt[p], 1);
        } else {
            ++bad;
        }
    }
    bad = wave_sum_int(bad);  // every lane reaches this point: no early exit above
    if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicAdd(dropped, (unsigned long long)bad);
}

// Block-wide exclusive scan of one int per thread (blockDim = kScanThreads).
__device__ inline int block_exclusive_scan(int v, int &total) {
    __shared__ int wave_tot[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int n = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += n;
    }
    if (lane == kWave - 1) wave_tot[wid] = incl;
    __syncthreads();
    int base = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wid) base += wave_tot[w];
        total += wave_tot[w];
    }
    __syncthreads();
    return base + incl - v;
}

// Per-block exclusive scan of cnt into off; block totals into bsum.
__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const int32_t *cnt, int32_t hw,
                                                             int32_t *off, int32_t *bsum) {
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) {
        v[e] = (base + e < hw) ? cnt[base + e] : 0;
        sum += v[e];
    }
    int total;
    int run = block_exclusive_scan(sum, total);
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) {
        if (base + e < hw) off[base + e] = run;
        run += v[e];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the block sums in place (one block, chunked), bsum[nb] = grand total.
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int32_t *bsum, int32_t nb) {
    int carry = 0;
    for (int c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int i = c0 + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int total;
        const int ex = block_exclusive_scan(v, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t *off, int32_t hw,
                                                          const int32_t *bsum, int32_t nb) {
    const int base = blockIdx.x * kScanBlock;
    const int add = bsum[blockIdx.x];
    for (int e = threadIdx.x; e < kScanBlock; e += kScanThreads)
        if (base + e < hw) off[base + e] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) off[hw] = bsum[nb];
}

// Order key of a sample: the float time mapped to an unsigned integer with the same order (-0 is
// folded onto +0 so that equal times tie), in the high word; the stream index in the low word. A
// larger key is a newer sample; 0 is below every valid key and marks an empty list entry.
__device__ inline unsigned long long order_key(float t, int i) {
    if (t == 0.0f) t = 0.0f;
    const unsigned u = __float_as_uint(t);
    const unsigned k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)k << 32) | (unsigned)i;
}

__device__ inline int key_index(unsigned long long key) { return (int)(unsigned)(key & 0xffffffffu); }

__global__ void k_build_scatter(afr_samples s, ValidCtx c, const int32_t *off, int32_t *cnt,
                                unsigned long long *bucket) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride) {
        const float x = s.x[i], y = s.y[i], t = s.t[i];
        if (!sample_valid(x, y, t, s.r[i], s.g[i], s.b[i], c)) continue;
        const int p = (int)floorf(y) * c.w + (int)floorf(x);
        const int pos = off[p] + atomicSub(&cnt[p], 1) - 1;
        bucket[pos] = order_key(t, (int)i);
    }
}


template <typename S>
__device__ inline void store_slot(const afr_samples &s, const afr_deep_buffer &out, size_t o,
                                  int i) {
    S *ox = static_cast<S *>(out.ox), *oy = static_cast<S *>(out.oy);
    S *ta = static_cast<S *>(out.tage), *r = static_cast<S *>(out.r);
    S *g = static_cast<S *>(out.g), *b = static_cast<S *>(out.b);
    if (i >= 0) {
        const float x = s.x[i], y = s.y[i];
        ox[o] = Codec<S>::enc(x - floorf(x));
        oy[o] = Codec<S>::enc(y - floorf(y));
        ta[o] = Codec<S>::enc_time(s.t[i], out.t_ref);
        r[o] = Codec<S>::enc(s.r[i]);
        g[o] = Codec<S>::enc(s.g[i]);
        b[o] = Codec<S>::enc(s.b[i]);
    } else {
        ox[o] = oy[o] = ta[o] = r[o] = g[o] = b[o] = Codec<S>::enc(0.0f);
    }
    if (out.src) out.src[o] = i;
}

template <typename S, int KMAX>
__global__ void k_build_select(afr_samples s, afr_deep_buffer out, const int32_t *off,
                               const unsigned long long *bucket) {
    const int hw = out.width * out.height;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= hw) return;
    const int K = out.k;
    const int b0 = off[p], b1 = off[p + 1];
    unsigned long long top[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) top[k] = 0ull;
    for (int e = b0; e < b1; ++e) {
        // insertion into a descending register list: one unsigned compare and two selects per
        // entry, so every lane runs the same instruction stream
        unsigned long long c = bucket[e];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const unsigned long long a = top[k];
            const bool gt = c > a;
            top[k] = gt ? c : a;
            c = gt ? a : c;
        }
    }
    const int n = min(b1 - b0, K);
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < K) store_slot<S>(s, out, (size_t)k * hw + p, k < n ? key_index(top[k]) : -1);
    out.count[p] = (uint8_t)n;
}

// Depths above 64: rank by repeated maximum scans over the bucket (O(arrivals * K), no lists).
template <typename S>
__global__ void k_build_select_scan(afr_samples s, afr_deep_buffer out, const int32_t *off,
                                    const unsigned long long *bucket) {
    const int hw = out.width * out.height;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= hw) return;
    const int K = out.k;
    const int b0 = off[p], b1 = off[p + 1];
    const int n = min(b1 - b0, K);
    unsigned long long prev = ~0ull;
    for (int k = 0; k < K; ++k) {
        unsigned long long best = 0ull;
        if (k < n) {
            for (int e = b0; e < b1; ++e) {
                const unsigned long long c = bucket[e];
                best = (c < prev && c > best) ? c : best;
            }
            prev = best;
        }
        store_slot<S>(s, out, (size_t)k * hw + p, k < n ? key_index(best) : -1);
    }
    out.count[p] = (uint8_t)n;
}

template <typename S>
hipError_t launch_select(const afr_samples &s, const afr_deep_buffer &out, const BuildWs &ws,
                         hipStream_t st) {
    const int hw = out.width * out.height;
    const int threads = 256, blocks = (hw + threads - 1) / threads;
    if (out.k <= 4)
        k_build_select<S, 4><<<blocks, threads, 0, st>>>(s, out, ws.off, ws.bucket);
    else if (out.k <= 8)
        k_build_select<S, 8><<<blocks, threads, 0, st>>>(s, out, ws.off, ws.bucket);
    else if (out.k <= 16)
        k_build_select<S, 16><<<blocks, threads, 0, st>>>(s, out, ws.off, ws.bucket);
    else if (out.k <= 32)
        k_build_select<S, 32><<<blocks, threads, 0, st>>>(s, out, ws.off, ws.bucket);
    else if (out.k <= 64)
        k_build_select<S, 64><<<blocks, threads, 0, st>>>(s, out, ws.off, ws.bucket);
    else
        k_build_select_scan<S><<<blocks, threads, 0, st>>>(s, out, ws.off, ws.bucket);
    return hipGetLastError();
}

}  // namespace

size_t build_ws_bytes(int64_t n, int32_t w, int32_t h) {
    const size_t hw = (size_t)w * h;
    const size_t nb = (hw + kScanBlock - 1) / kScanBlock;
    return align_up(hw * 4) + align_up((hw + 1) * 4) + align_up((nb + 1) * 4) +
           align_up((size_t)(n > 0 ? n : 1) * 8) + align_up(8);
}

BuildWs build_ws_carve(void *ws, int64_t n, int32_t w, int32_t h) {
    const size_t hw = (size_t)w * h;
    const size_t nb = (hw + kScanBlock - 1) / kScanBlock;
    char *p = static_cast<char *>(ws);
    BuildWs o;
    o.cnt = reinterpret_cast<int32_t *>(p);
    p += align_up(hw * 4);
    o.off = reinterpret_cast<int32_t *>(p);
    p += align_up((hw + 1) * 4);
    o.bsum = reinterpret_cast<int32_t *>(p);
    p += align_up((nb + 1) * 4);
    o.bucket = reinterpret_cast<unsigned long long *>(p);
    p += align_up((size_t)(n > 0 ? n : 1) * 8);
    o.dropped_internal = reinterpret_cast<unsigned long long *>(p);
    return o;
}

hipError_t launch_build(const afr_samples &s, const afr_deep_buffer &out, const BuildWs &ws,
                        unsigned long long *dropped, hipStream_t st) {
    const int hw = out.width * out.height;
    const ValidCtx c{out.width, out.height, out.t_ref, out.precision == AFR_FP16 ? 1 : 0};
    const int nb = (hw + kScanBlock - 1) / kScanBlock;
    const int sblocks = (int)std::min<int64_t>((s.n + 255) / 256, 8192);
    k_build_clear<<<std::max(1, std::min((hw + 255) / 256, 4096)), 256, 0, st>>>(ws.cnt, hw, dropped);
    if (s.n > 0) k_build_count<<<std::max(1, sblocks), 256, 0, st>>>(s, c, ws.cnt, dropped);
    k_scan_blocks<<<nb, kScanThreads, 0, st>>>(ws.cnt, hw, ws.off, ws.bsum);
    k_scan_sums<<<1, kScanThreads, 0, st>>>(ws.bsum, nb);
    k_scan_add<<<nb, kScanThreads, 0, st>>>(ws.off, hw, ws.bsum, nb);
    if (s.n > 0) k_build_scatter<<<std::max(1, sblocks), 256, 0, st>>>(s, c, ws.off, ws.cnt, ws.bucket);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return out.precision == AFR_FP16 ? launch_select<__half>(s, out, ws, st)
                                     : launch_select<float>(s, out, ws, st);
}

}  // namespace afr
