// Deep-buffer build: bin the sample stream to home pixels and keep each pixel's K newest samples.
//
// The paper's reconstructor receives samples as one stream (Sec. 4.2, Sec. 5.2) and each pixel keeps
// a queue of its newest samples (Sec. 4). Replaying queue insertions one sample at a time is serial
// per pixel; the same final state is the top-K by key (t, stream index) of the samples binned to the
// pixel, which this file computes with a counting sort:
//   1. k_build_clear   zero the per-pixel arrival counters and the dropped counter
//   2. k_build_count   read x, y; samples inside the image take an arrival rank in their home pixel
//                      (the return value of an integer atomic), others are dropped
//   3. scan            exclusive prefix sum of the counts -> bucket offsets
//   4. k_build_scatter read the whole sample and write one 32-byte record (order key, ox, oy, t, r,
//                      g, b) to bucket[offset + rank]; a sample that fails the remaining validity
//                      checks writes key 0 and is dropped (no atomics in this pass)
//   5. k_build_select  per pixel: register top-K over its contiguous records, then store the slots
// Every decision is integer or an exact comparison of stored float32 inputs, so the result is
// bit-exact and independent of launch shape and atomic order (the rank only orders a bucket).
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

// Validity: the position decides the home pixel (checked in the count pass); time, colour and the
// binary16 range are checked in the scatter pass. Together they are the rule of afr.h.
__device__ inline bool position_valid(float x, float y, const ValidCtx &c) {
    return isfinite(x) && isfinite(y) && x >= 0.0f && x < (float)c.w && y >= 0.0f && y < (float)c.h;
}

__device__ inline bool payload_valid(float t, float r, float g, float b, const ValidCtx &c) {
    bool ok = isfinite(t) && isfinite(r) && isfinite(g) && isfinite(b) && t <= c.t_ref;
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

__global__ void k_build_count(afr_samples s, ValidCtx c, int32_t *cnt, int32_t *rank,
                              unsigned long long *dropped) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride) {
        const float x = s.x[i], y = s.y[i];
        int rk = -1;
        if (position_valid(x, y, c)) {
            const int p = (int)floorf(y) * c.w + (int)floorf(x);
            rk = atomicAdd(&cnt[p], 1);
        } else {
            ++bad;
        }
        rank[i] = rk;
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

// One bucket record per sample routed to a pixel: order key (0 = invalid) and the stored fields.
struct alignas(16) Record {
    unsigned long long key;
    float ox, oy, t, r, g, b;
};
static_assert(sizeof(Record) == 32, "bucket record is 32 bytes");

__global__ void k_build_scatter(afr_samples s, ValidCtx c, const int32_t *off, const int32_t *rank,
                                Record *bucket, unsigned long long *dropped) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride) {
        const int rk = rank[i];
        if (rk < 0) continue;
        const float x = s.x[i], y = s.y[i], t = s.t[i], r = s.r[i], g = s.g[i], b = s.b[i];
        const float fx = floorf(x), fy = floorf(y);
        const int p = (int)fy * c.w + (int)fx;
        Record rec;
        const bool ok = payload_valid(t, r, g, b, c);
        bad += ok ? 0 : 1;
        rec.key = ok ? order_key(t, (int)i) : 0ull;
        rec.ox = x - fx;
        rec.oy = y - fy;
        rec.t = t;
        rec.r = r;
        rec.g = g;
        rec.b = b;
        bucket[off[p] + rk] = rec;
    }
    bad = wave_sum_int(bad);
    if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicAdd(dropped, (unsigned long long)bad);
}

template <typename S>
__device__ inline void store_slot(const afr_deep_buffer &out, size_t o, const Record *rec) {
    S *ox = static_cast<S *>(out.ox), *oy = static_cast<S *>(out.oy);
    S *ta = static_cast<S *>(out.tage), *r = static_cast<S *>(out.r);
    S *g = static_cast<S *>(out.g), *b = static_cast<S *>(out.b);
    if (rec) {
        const Record e = *rec;
        ox[o] = Codec<S>::enc(e.ox);
        oy[o] = Codec<S>::enc(e.oy);
        ta[o] = Codec<S>::enc_time(e.t, out.t_ref);
        r[o] = Codec<S>::enc(e.r);
        g[o] = Codec<S>::enc(e.g);
        b[o] = Codec<S>::enc(e.b);
        if (out.src) out.src[o] = key_index(e.key);
    } else {
        ox[o] = oy[o] = ta[o] = r[o] = g[o] = b[o] = Codec<S>::enc(0.0f);
        if (out.src) out.src[o] = -1;
    }
}

template <typename S, int KMAX>
__global__ void k_build_select(afr_deep_buffer out, const int32_t *off, const Record *bucket) {
    const int hw = out.width * out.height;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= hw) return;
    const int K = out.k;
    const int b0 = off[p], b1 = off[p + 1];
    unsigned long long top[KMAX];
    int pos[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        top[k] = 0ull;
        pos[k] = -1;
    }
    int nvalid = 0;
    for (int e = b0; e < b1; ++e) {
        // insertion into a descending register list: one unsigned compare and selects per entry,
        // so every lane runs the same instruction stream
        unsigned long long c = bucket[e].key;
        int ce = e;
        nvalid += c != 0ull;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const unsigned long long a = top[k];
            const int ae = pos[k];
            const bool gt = c > a;
            top[k] = gt ? c : a;
            pos[k] = gt ? ce : ae;
            c = gt ? a : c;
            ce = gt ? ae : ce;
        }
    }
    const int n = min(nvalid, K);
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < K) store_slot<S>(out, (size_t)k * hw + p, k < n ? bucket + pos[k] : nullptr);
    out.count[p] = (uint8_t)n;
}

// Depths above 64: rank by repeated maximum scans over the records (O(arrivals * K), no lists).
template <typename S>
__global__ void k_build_select_scan(afr_deep_buffer out, const int32_t *off, const Record *bucket) {
    const int hw = out.width * out.height;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= hw) return;
    const int K = out.k;
    const int b0 = off[p], b1 = off[p + 1];
    int nvalid = 0;
    for (int e = b0; e < b1; ++e) nvalid += bucket[e].key != 0ull;
    const int n = min(nvalid, K);
    unsigned long long prev = ~0ull;
    for (int k = 0; k < K; ++k) {
        unsigned long long best = 0ull;
        int be = -1;
        if (k < n) {
            for (int e = b0; e < b1; ++e) {
                const unsigned long long c = bucket[e].key;
                const bool take = c < prev && c > best;
                best = take ? c : best;
                be = take ? e : be;
            }
            prev = best;
        }
        store_slot<S>(out, (size_t)k * hw + p, k < n ? bucket + be : nullptr);
    }
    out.count[p] = (uint8_t)n;
}

template <typename S>
hipError_t launch_select(const afr_deep_buffer &out, const BuildWs &ws, hipStream_t st) {
    const Record *bucket = static_cast<const Record *>(ws.bucket);
    const int hw = out.width * out.height;
    const int threads = 256, blocks = (hw + threads - 1) / threads;
    if (out.k <= 4)
        k_build_select<S, 4><<<blocks, threads, 0, st>>>(out, ws.off, bucket);
    else if (out.k <= 8)
        k_build_select<S, 8><<<blocks, threads, 0, st>>>(out, ws.off, bucket);
    else if (out.k <= 16)
        k_build_select<S, 16><<<blocks, threads, 0, st>>>(out, ws.off, bucket);
    else if (out.k <= 32)
        k_build_select<S, 32><<<blocks, threads, 0, st>>>(out, ws.off, bucket);
    else if (out.k <= 64)
        k_build_select<S, 64><<<blocks, threads, 0, st>>>(out, ws.off, bucket);
    else
        k_build_select_scan<S><<<blocks, threads, 0, st>>>(out, ws.off, bucket);
    return hipGetLastError();
}

}  // namespace

size_t build_ws_bytes(int64_t n, int32_t w, int32_t h) {
    const size_t hw = (size_t)w * h;
    const size_t nb = (hw + kScanBlock - 1) / kScanBlock;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return align_up(hw * 4) + align_up((hw + 1) * 4) + align_up((nb + 1) * 4) + align_up(nn * 4) +
           align_up(nn * sizeof(Record)) + align_up(8);
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
    const size_t nn = (size_t)(n > 0 ? n : 1);
    o.bsum = reinterpret_cast<int32_t *>(p);
    p += align_up((nb + 1) * 4);
    o.rank = reinterpret_cast<int32_t *>(p);
    p += align_up(nn * 4);
    o.bucket = p;
    p += align_up(nn * sizeof(Record));
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
    if (s.n > 0) k_build_count<<<std::max(1, sblocks), 256, 0, st>>>(s, c, ws.cnt, ws.rank, dropped);
    k_scan_blocks<<<nb, kScanThreads, 0, st>>>(ws.cnt, hw, ws.off, ws.bsum);
    k_scan_sums<<<1, kScanThreads, 0, st>>>(ws.bsum, nb);
    k_scan_add<<<nb, kScanThreads, 0, st>>>(ws.off, hw, ws.bsum, nb);
    Record *bucket = static_cast<Record *>(ws.bucket);
    if (s.n > 0)
        k_build_scatter<<<std::max(1, sblocks), 256, 0, st>>>(s, c, ws.off, ws.rank, bucket, dropped);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return out.precision == AFR_FP16 ? launch_select<__half>(out, ws, st)
                                     : launch_select<float>(out, ws, st);
}

}  // namespace afr
