// Deep-buffer build: bin the sample stream to home pixels and keep each pixel's K newest samples.
//
// The paper's reconstructor receives samples as one stream (Sec. 4.2, Sec. 5.2) and each pixel keeps
// a queue of its newest samples (Sec. 4). Replaying queue insertions one sample at a time is serial
// per pixel; the same final state is the top-K by key (t, stream index) of the samples binned to the
// pixel. This file computes it with a two-level partition that keeps random accesses in LDS and L2:
//   1. k_bin_count    per chunk of the stream: LDS histogram over bins of 64 x 4 px;
//                     samples outside the image are dropped here (after reprojection to the
//                     reference time when the stream carries velocities; the scatter repeats it)
//   2. k_scan_rows    per bin: exclusive prefix sum of its row of (bin, chunk) counts, in place,
//                     and the bin's total; a record's position in the bucket is the sum of the
//                     totals of the bins before its own (each consumer adds those up itself) plus
//                     its chunk's offset in the row
//   3. k_bin_scatter  per chunk: coalesced loads of every field, an LDS counting sort by bin, and
//                     32-byte records (order key, x, y, t, r, g, b) staged in LDS in bin order, a
//                     window at a time, so that consecutive lanes store consecutive records of a
//                     bin's run (for a binary16 buffer the payload is stored already encoded, 8
//                     bytes); invalid time or colour writes key 0
//   4. k_bin_select   per bin: its records' keys are counting-sorted by pixel into an LDS list
//                     (in one sweep that holds the keys in registers when the bin fits the list,
//                     else in passes over groups of rows), each pixel takes a register top-K over
//                     its keys, and the selected records are stored to the slot planes
// Chunks are dealt to XCDs in contiguous runs, so that the table entries of neighbouring chunks
// (adjacent in the bin-major table) and the ends of their runs in each bin meet in one L2.
// Every decision is integer or an exact comparison of stored float32 inputs, so the result is
// bit-exact and independent of launch shape and atomic order (atomics only order records inside a
// group that is sorted by key afterwards).
#include <type_traits>

#include "afr_internal.h"

namespace afr {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;
constexpr int kChunkThreads = 512;  // two 512-thread scatter workgroups share a CU, so one loads
                                    // while the other sorts and stores
// Samples per thread (PER) of the count and scatter kernels, chosen per launch (pick_per): a chunk
// is kChunkThreads * PER samples.
constexpr int kPerMin = 6, kPerMax = 10;
constexpr int kWin = 2048;  // records staged in LDS per scatter window (64 KiB, binary16: 48 KiB)
constexpr int kBinW = 64;                          // bin width, px (a power of two)
static_assert((kBinW & (kBinW - 1)) == 0, "bin width is a power of two");
constexpr int kMaxBins = 4096;                     // LDS capacity of the per-chunk bin tables
constexpr int kMaxBinPx = 2048;                    // pixels per bin (rows grow from 4 to 32)
constexpr int kListCap = 5120;                     // records sorted in LDS per select pass
// Select workgroup: 512 threads while the per-pixel top-K stays small (KMAX <= 16; the sweep and the
// LDS sort then have twice the waves to overlap, at the same LDS per bin), else 256 (register lists
// of 32 or 64 keys need the registers).
template <int KMAX>
constexpr int sel_threads() { return KMAX <= 16 ? 512 : 256; }

struct ValidCtx {
    int32_t w, h;
    float t_ref;
    int32_t fp16;
};

// Bins of bw x bh pixels, bw = kBinW and bh a power of two (bh = 1 << sbh).
struct BinGeom {
    int32_t bw, bh, sbh, nbx, nby, nb;
};

// Validity: the position decides the home pixel (checked when binning); time, colour and the
// binary16 range are checked when the record is written. Together they are the rule of afr.h.
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

// Sum of one int per thread over the workgroup (blockDim.x = NT), valid in thread 0.
template <int NT>
__device__ inline int block_sum_int(int v) {
    __shared__ int wsum[NT / kWave];
    v = wave_sum_int(v);
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = v;
    __syncthreads();
    int t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / kWave; ++w) t += wsum[w];
    return t;
}

// Reprojection to the reference time (Sec. 6.2 with the per-sample velocity of Sec. 4): each of the
// subtraction, product and sum is rounded on its own, so the home pixel is an exact function of the
// stored inputs. A non-finite time or velocity makes the position non-finite, which drops the sample.
__device__ inline void advect(float &x, float &y, float t, float vx, float vy, float t_ref) {
    const float d = __fsub_rn(t_ref, t);
    x = __fadd_rn(x, __fmul_rn(vx, d));
    y = __fadd_rn(y, __fmul_rn(vy, d));
}

// Bin of a position inside the image (x, y >= 0): shifts, since both bin edges are powers of two.
__device__ inline int bin_of(float x, float y, const BinGeom &g) {
    return (int)((unsigned)floorf(y) >> g.sbh) * g.nbx + (int)((unsigned)floorf(x) / kBinW);
}

// Order key of a sample: the float time mapped to an unsigned integer with the same order (-0 is
// folded onto +0 so that equal times tie), in the high word; the stream index in the low word. A
// larger key is a newer sample; 0 is below every valid key and marks an invalid record.
__device__ inline unsigned long long order_key(float t, int i) {
    if (t == 0.0f) t = 0.0f;
    const unsigned u = __float_as_uint(t);
    const unsigned k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)k << 32) | (unsigned)i;
}

__device__ inline int key_index(unsigned long long key) { return (int)(unsigned)(key & 0xffffffffu); }

// MOTION: the stream carries velocities and positions are reprojected first.
template <bool MOTION, int kChunkPer>
__global__ __launch_bounds__(kChunkThreads) void k_bin_count(afr_samples s, ValidCtx c, BinGeom g,
                                                             int32_t *ht, int nchunks,
                                                             int32_t *bad_tab) {
    constexpr int kChunk = kChunkThreads * kChunkPer;
    __shared__ int hist[kMaxBins];
    for (int b = threadIdx.x; b < g.nb; b += kChunkThreads) hist[b] = 0;
    const int chunk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)chunk * kChunk;
    float xs[kChunkPer], ys[kChunkPer];
    float ts[MOTION ? kChunkPer : 1], us[MOTION ? kChunkPer : 1], vs[MOTION ? kChunkPer : 1];
#pragma unroll
    for (int j = 0; j < kChunkPer; ++j) {  // all loads first
        const int64_t i = min(base + (int64_t)j * kChunkThreads + threadIdx.x, s.n - 1);
        xs[j] = s.x[i];
        ys[j] = s.y[i];
        if constexpr (MOTION) {
            ts[j] = s.t[i];
            us[j] = s.vx[i];
            vs[j] = s.vy[i];
        }
    }
    if constexpr (MOTION) {
#pragma unroll
        for (int j = 0; j < kChunkPer; ++j) advect(xs[j], ys[j], ts[j], us[j], vs[j], c.t_ref);
    }
    __syncthreads();
    int bad = 0;
#pragma unroll
    for (int j = 0; j < kChunkPer; ++j) {
        if (base + (int64_t)j * kChunkThreads + threadIdx.x >= s.n) continue;
        if (position_valid(xs[j], ys[j], c)) atomicAdd(&hist[bin_of(xs[j], ys[j], g)], 1);
        else ++bad;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < g.nb; b += kChunkThreads)
        ht[(size_t)b * nchunks + chunk] = hist[b];
    bad = block_sum_int<kChunkThreads>(bad);
    if (threadIdx.x == 0) bad_tab[chunk] = bad;  // samples outside the image
}

// Block-wide exclusive scan of one int per thread (blockDim = NT).
template <int NT>
__device__ inline int block_exclusive_scan(int v, int &total) {
    __shared__ int wave_tot[NT / kWave];
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
    for (int w = 0; w < NT / kWave; ++w) {
        if (w < wid) base += wave_tot[w];
        total += wave_tot[w];
    }
    __syncthreads();
    return base + incl - v;
}

// Exclusive scan of n ints in LDS into out (may alias), by a block of NT threads; returns the total.
template <int NT>
__device__ inline int block_scan_lds(const int *in, int *out, int n) {
    int carry = 0;
    for (int c0 = 0; c0 < n; c0 += NT) {
        const int q = c0 + threadIdx.x;
        const int v = q < n ? in[q] : 0;
        int total;
        const int ex = block_exclusive_scan<NT>(v, total);
        if (q < n) out[q] = carry + ex;
        carry += total;
    }
    return carry;
}

// One workgroup per bin: exclusive scan of the bin's row of the bin-major (bin, chunk) count table
// in place, and the bin's total into tot[bin].
__global__ __launch_bounds__(kScanThreads) void k_scan_rows(int32_t *tab, int nchunks, int32_t *tot) {
    const int b = blockIdx.x;
    int32_t *row = tab + (size_t)b * nchunks;
    int carry = 0;
    for (int c0 = 0; c0 < nchunks; c0 += kScanBlock) {
        const int base = c0 + threadIdx.x * kScanItems;
        int v[kScanItems];
        int sum = 0;
#pragma unroll
        for (int e = 0; e < kScanItems; ++e) {
            v[e] = base + e < nchunks ? row[base + e] : 0;
            sum += v[e];
        }
        int total;
        int run = carry + block_exclusive_scan<kScanThreads>(sum, total);
#pragma unroll
        for (int e = 0; e < kScanItems; ++e) {
            if (base + e < nchunks) row[base + e] = run;
            run += v[e];
        }
        carry += total;
    }
    if (threadIdx.x == 0) tot[b] = carry;
}

// Position in the bucket of bin b's first record: the totals of the bins before it, summed by the
// calling workgroup (NT threads) in a fixed order; valid in every thread.
template <int NT>
__device__ inline int bin_start(const int32_t *tot, int b) {
    __shared__ int s_start;
    __syncthreads();  // an earlier block_sum_int of the caller has been read out
    int v = 0;
    for (int i = threadIdx.x; i < b; i += NT) v += tot[i];
    v = block_sum_int<NT>(v);
    if (threadIdx.x == 0) s_start = v;
    __syncthreads();
    return s_start;
}

struct alignas(16) Record {
    unsigned long long key;
    float x, y, t, r, g, b;
};
static_assert(sizeof(Record) == 32, "staged record is 32 bytes");

// The bucket holds each record in two arrays: (key, x, y), 16 bytes, read by the selection's sweep,
// and the payload, read only for the records a pixel keeps: (t, r, g, b) as float4 for a binary32
// buffer, or already encoded as four binary16 values (age, r | g, b) in 8 bytes for a binary16 one.
struct alignas(16) KeyXY {
    unsigned long long key;
    float x, y;
};
static_assert(sizeof(KeyXY) == 16, "record half is 16 bytes");
struct Bucket {
    KeyXY *a;
    float4 *b;  // binary32 payload
    uint2 *h;   // binary16 payload (same memory as b)
};
struct BinRecs {
    const KeyXY *a;
    const float4 *b;
    const uint2 *h;
};

__device__ inline unsigned pack_half2(__half lo, __half hi) {
    return (unsigned)__half_as_ushort(lo) | ((unsigned)__half_as_ushort(hi) << 16);
}

// LDS: the per-bin table [nb] (counts, then offsets in the chunk's sorted order, then the global
// position minus that offset) and the staged records [kWin], whose key array first holds the bins'
// first positions in the bucket (an exclusive scan of the bin totals); a staged record's bin, and
// so its destination, is recomputed from its own x, y. H: binary16 buffer, whose payload is encoded to its
// four halves as soon as the record is loaded, so the record holds fewer registers and is staged in
// 24 instead of 32 bytes.
template <bool MOTION, int kChunkPer, bool H>
__global__ __launch_bounds__(kChunkThreads, 4) void k_bin_scatter(afr_samples s, ValidCtx c, BinGeom g,
                                                               const int32_t *ot,
                                                               const int32_t *tot, int nchunks,
                                                               Bucket bucket, int32_t *bad_tab) {
    constexpr int kChunk = kChunkThreads * kChunkPer;
    extern __shared__ uint4 scat_lds[];  // 16-byte aligned for the staged records
    int *scat_sm = reinterpret_cast<int *>(scat_lds);
    int *tab = scat_sm;  // [nb]
    // staged records as three arrays [kWin] (keys, positions, payloads): a lane's scattered write
    // of one 8- or 16-byte field meets fewer bank conflicts than a 32-byte record's, and the store
    // loop reads each array in order
    unsigned long long *skey = reinterpret_cast<unsigned long long *>(scat_sm + ((g.nb + 3) & ~3));
    // the bins' first positions [nb] live in the key array until the records are staged
    static_assert(kWin * sizeof(unsigned long long) >= kMaxBins * sizeof(int), "room for [nb]");
    int *bstart = reinterpret_cast<int *>(skey);
    float2 *sxy = reinterpret_cast<float2 *>(skey + kWin);
    float4 *spl = reinterpret_cast<float4 *>(sxy + kWin);  // binary32 payload
    uint2 *sph = reinterpret_cast<uint2 *>(sxy + kWin);    // binary16 payload
    for (int b = threadIdx.x; b < g.nb; b += kChunkThreads) {
        tab[b] = 0;
        bstart[b] = tot[b];
    }
    const int chunk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)chunk * kChunk;
    Record rec[kChunkPer];
#pragma unroll
    for (int j = 0; j < kChunkPer; ++j) {  // coalesced loads of every field
        const int64_t i = min(base + (int64_t)j * kChunkThreads + threadIdx.x, s.n - 1);
        rec[j].x = s.x[i];
        rec[j].y = s.y[i];
        rec[j].t = s.t[i];
        rec[j].r = s.r[i];
        rec[j].g = s.g[i];
        rec[j].b = s.b[i];
        if constexpr (MOTION) advect(rec[j].x, rec[j].y, rec[j].t, s.vx[i], s.vy[i], c.t_ref);
    }
    __syncthreads();
    // while the samples arrive: the first bucket position of each bin (fewer values are live here
    // than after the histogram, which keeps two workgroups per CU within the registers)
    block_scan_lds<kChunkThreads>(bstart, bstart, g.nb);
    int bin[kChunkPer], sp[kChunkPer];
    uint2 hp[H ? kChunkPer : 1];
    int bad = 0;
#pragma unroll
    for (int j = 0; j < kChunkPer; ++j) {
        const int64_t i = base + (int64_t)j * kChunkThreads + threadIdx.x;
        const bool in = i < s.n && position_valid(rec[j].x, rec[j].y, c);
        const bool ok = in && payload_valid(rec[j].t, rec[j].r, rec[j].g, rec[j].b, c);
        bad += (in && !ok) ? 1 : 0;
        rec[j].key = ok ? order_key(rec[j].t, (int)i) : 0ull;
        bin[j] = in ? bin_of(rec[j].x, rec[j].y, g) : -1;
        sp[j] = in ? atomicAdd(&tab[bin[j]], 1) : 0;  // rank inside the bin
        if constexpr (H)  // the binary16 slot record's last two words: (r, g), (b, age_ref)
            hp[j] = make_uint2(pack_half2(Codec<__half>::enc(rec[j].r), Codec<__half>::enc(rec[j].g)),
                               pack_half2(Codec<__half>::enc(rec[j].b),
                                          Codec<__half>::enc_time(rec[j].t, c.t_ref)));
    }
    __syncthreads();
    const int nvalid = block_scan_lds<kChunkThreads>(tab, tab, g.nb);  // bin offsets, in place
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kChunkPer; ++j)
        if (bin[j] >= 0) sp[j] += tab[bin[j]];  // position in the chunk's bin-sorted order
    __syncthreads();
    for (int b = threadIdx.x; b < g.nb; b += kChunkThreads)
        tab[b] = bstart[b] + ot[(size_t)b * nchunks + chunk] - tab[b];
    __syncthreads();
    for (int w0 = 0; w0 < nvalid; w0 += kWin) {
#pragma unroll
        for (int j = 0; j < kChunkPer; ++j) {
            const int q = sp[j] - w0;
            if (bin[j] >= 0 && q >= 0 && q < kWin) {
                skey[q] = rec[j].key;
                sxy[q] = make_float2(rec[j].x, rec[j].y);
                if constexpr (H)
                    sph[q] = hp[j];
                else
                    spl[q] = make_float4(rec[j].t, rec[j].r, rec[j].g, rec[j].b);
            }
        }
        __syncthreads();
        const int nw = min(kWin, nvalid - w0);
        for (int q = threadIdx.x; q < nw; q += kChunkThreads) {
            const float2 xy = sxy[q];
            const int d = tab[bin_of(xy.x, xy.y, g)] + w0 + q;
            bucket.a[d] = KeyXY{skey[q], xy.x, xy.y};
            if constexpr (H)
                bucket.h[d] = sph[q];
            else
                bucket.b[d] = spl[q];
        }
        __syncthreads();
    }
    bad = block_sum_int<kChunkThreads>(bad);
    if (threadIdx.x == 0) bad_tab[nchunks + chunk] = bad;  // invalid time or colour
}

// Stores a record (key, x, y | t, r, g, b) or, when e < 0, an empty slot at slot-plane offset o.
template <typename S>
__device__ inline void store_record(const afr_deep_buffer &out, size_t o, int e, const KeyXY &a,
                                    const float4 &c) {
    if constexpr (std::is_same<S, __half>::value) {  // one 12-byte slot record
        uint3 w = make_uint3(0u, 0u, 0u);
        if (e >= 0) {
            w.x = (unsigned)__half_as_ushort(Codec<__half>::enc(a.x - floorf(a.x))) |
                  ((unsigned)__half_as_ushort(Codec<__half>::enc(a.y - floorf(a.y))) << 16);
            w.y = (unsigned)__half_as_ushort(Codec<__half>::enc(c.y)) |
                  ((unsigned)__half_as_ushort(Codec<__half>::enc(c.z)) << 16);
            w.z = (unsigned)__half_as_ushort(Codec<__half>::enc(c.w)) |
                  ((unsigned)__half_as_ushort(Codec<__half>::enc_time(c.x, out.t_ref)) << 16);
        }
        reinterpret_cast<uint3 *>(out.ox)[o] = w;
    } else {
        S *ox = static_cast<S *>(out.ox), *oy = static_cast<S *>(out.oy);
        S *ta = static_cast<S *>(out.tage), *r = static_cast<S *>(out.r);
        S *g = static_cast<S *>(out.g), *b = static_cast<S *>(out.b);
        if (e >= 0) {
            ox[o] = Codec<S>::enc(a.x - floorf(a.x));
            oy[o] = Codec<S>::enc(a.y - floorf(a.y));
            ta[o] = Codec<S>::enc_time(c.x, out.t_ref);
            r[o] = Codec<S>::enc(c.y);
            g[o] = Codec<S>::enc(c.z);
            b[o] = Codec<S>::enc(c.w);
        } else {
            ox[o] = oy[o] = ta[o] = r[o] = g[o] = b[o] = Codec<S>::enc(0.0f);
        }
    }
    if (out.src) out.src[o] = e >= 0 ? key_index(a.key) : -1;
}

// Binary16 mode: the select keeps each listed record's encoded offsets (ox | oy << 16) in LDS, so
// that a kept record's fetch reads only its (t, r, g, b) half.
template <typename S>
constexpr bool kOxyInList = std::is_same<S, __half>::value;

__device__ inline unsigned encode_oxy(float x, float y) {
    return (unsigned)__half_as_ushort(Codec<__half>::enc(x - floorf(x))) |
           ((unsigned)__half_as_ushort(Codec<__half>::enc(y - floorf(y))) << 16);
}

// Stores a kept binary16 slot record from its encoded offsets, stream index and encoded payload.
__device__ inline void store_record_oxy(const afr_deep_buffer &out, size_t o, unsigned oxy, int src,
                                        const uint2 &h) {
    reinterpret_cast<uint3 *>(out.ox)[o] = make_uint3(oxy, h.x, h.y);
    if (out.src) out.src[o] = src;
}

// Stores record e of the bin (or an empty slot when e < 0) at slot-plane offset o.
template <typename S>
__device__ inline void store_slot(const afr_deep_buffer &out, size_t o, const BinRecs &rs, int e) {
    KeyXY a{0ull, 0.0f, 0.0f};
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (kOxyInList<S>) {
        if (e >= 0) {
            a = rs.a[e];
            store_record_oxy(out, o, encode_oxy(a.x, a.y), key_index(a.key), rs.h[e]);
            return;
        }
    } else if (e >= 0) {
        a = rs.a[e];
        c = rs.b[e];
    }
    store_record<S>(out, o, e, a, c);
}

// LDS slot of list entry l: one pad entry after every 16, so that the lanes of a wave, which read
// their pixels' lists at a stride of about 16 entries when pixels hold about 16 records, spread over
// the LDS banks instead of meeting in two.
constexpr int kListSlots = kListCap + kListCap / 16;
__device__ inline int swz(int l) { return l + (l >> 4); }

// Top-K of one pixel over its entries [l0, l1) of the LDS key list. KMAX <= 64: a pixel with at
// most KMAX entries sorts them in registers with a bitonic network; one with more inserts each into
// a descending register list (one unsigned compare and selects per entry and position). Larger K:
// repeated maximum scans. The selected records are then loaded together. [h0, h1): the slots this
// call stores (the whole list by default; h0 a multiple of 4 for KMAX <= 64), the pixel's count with
// slot 0.
template <typename S, int KMAX>
__device__ inline void select_pixel(const afr_deep_buffer &out, size_t p, size_t hw,
                                    const BinRecs &recs, const unsigned long long *keys,
                                    const unsigned short *pos, const unsigned *oxy, int l0, int l1,
                                    int h0 = 0, int h1 = KMAX) {
    const int K = out.k;
    int nvalid = 0;
    if constexpr (KMAX <= 64) {
        unsigned long long top[KMAX];
        int tp[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            top[k] = 0ull;
            tp[k] = 0;
        }
        if (l1 - l0 <= KMAX) {
            // All candidates fit the register list: load them (0 pads) and sort descending with a
            // bitonic network, KMAX/2 log2(KMAX) (log2(KMAX) + 1) / 2 compare-exchanges instead of
            // KMAX per candidate. Valid keys are distinct (they hold the stream index), so the
            // order is the same as the insertion's.
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int l = l0 + k;
                top[k] = l < l1 ? keys[swz(l)] : 0ull;
                tp[k] = l;
                nvalid += top[k] != 0ull;
            }
#pragma unroll
            for (int size = 2; size <= KMAX; size <<= 1)
#pragma unroll
                for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
                    for (int i = 0; i < KMAX; ++i) {
                        const int j = i ^ stride;
                        if (j > i) {
                            // descending blocks where bit `size` of i is clear, ascending otherwise,
                            // so that the last merge leaves the whole list descending
                            const unsigned long long a = top[i], b = top[j];
                            const bool sw = (i & size) == 0 ? a < b : a > b;
                            const int ea = tp[i], eb = tp[j];
                            top[i] = sw ? b : a;
                            top[j] = sw ? a : b;
                            tp[i] = sw ? eb : ea;
                            tp[j] = sw ? ea : eb;
                        }
                    }
        } else {
            for (int l = l0; l < l1; ++l) {
                unsigned long long c = keys[swz(l)];
                int ce = l;  // list index of the candidate
                nvalid += c != 0ull;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    const unsigned long long a = top[k];
                    const int ae = tp[k];
                    const bool gt = c > a;
                    top[k] = gt ? c : a;
                    tp[k] = gt ? ce : ae;
                    c = gt ? a : c;
                    ce = gt ? ae : ce;
                }
            }
        }
        const int n = min(nvalid, K);
        // The kept records are fetched four at a time, all loads before the stores, so that a
        // lane waits for memory once per group instead of once per slot.
        constexpr int kG = KMAX < 4 ? KMAX : 4;
#pragma unroll
        for (int k0 = 0; k0 < KMAX; k0 += kG) {
            if (k0 < h0 || k0 >= h1) continue;
            KeyXY a[kG];
            float4 c[kG];
            uint2 h[kOxyInList<S> ? kG : 1];
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                a[j] = KeyXY{0ull, 0.0f, 0.0f};
                c[j] = make_float4(0.f, 0.f, 0.f, 0.f);
                if constexpr (kOxyInList<S>) h[j] = make_uint2(0u, 0u);
                if (k0 + j < n) {
                    const int e = pos[swz(tp[k0 + j])];
                    if constexpr (kOxyInList<S>) {
                        h[j] = recs.h[e];
                    } else {
                        a[j] = recs.a[e];
                        c[j] = recs.b[e];
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                if (k0 + j >= K) continue;
                const size_t o = (size_t)(k0 + j) * hw + p;
                if constexpr (kOxyInList<S>) {
                    if (k0 + j < n) store_record_oxy(out, o, oxy[swz(tp[k0 + j])], key_index(top[k0 + j]), h[j]);
                    else store_record<S>(out, o, -1, a[j], c[j]);
                } else {
                    store_record<S>(out, o, k0 + j < n ? 0 : -1, a[j], c[j]);
                }
            }
        }
        if (h0 == 0) out.count[p] = (uint8_t)n;
    } else {
        for (int l = l0; l < l1; ++l) nvalid += keys[swz(l)] != 0ull;
        const int n = min(nvalid, K);
        unsigned long long prev = ~0ull;
        for (int k = 0; k < K; ++k) {
            unsigned long long best = 0ull;
            int be = 0;
            if (k < n) {
                for (int l = l0; l < l1; ++l) {
                    const unsigned long long c = keys[swz(l)];
                    const bool take = c < prev && c > best;
                    best = take ? c : best;
                    be = take ? (int)pos[swz(l)] : be;
                }
                prev = best;
            }
            store_slot<S>(out, (size_t)k * hw + p, recs, k < n ? be : -1);
        }
        out.count[p] = (uint8_t)n;
    }
}

// Same selection straight from the bin's records, for passes whose records exceed the LDS list.
template <typename S>
__device__ inline void select_pixel_scan(const afr_deep_buffer &out, size_t p, size_t hw,
                                         const BinRecs &recs, int nrec, int px, int py) {
    const int K = out.k;
    auto mine = [&](int e) {
        return (int)floorf(recs.a[e].x) == px && (int)floorf(recs.a[e].y) == py;
    };
    int nvalid = 0;
    for (int e = 0; e < nrec; ++e) nvalid += mine(e) && recs.a[e].key != 0ull;
    const int n = min(nvalid, K);
    unsigned long long prev = ~0ull;
    for (int k = 0; k < K; ++k) {
        unsigned long long best = 0ull;
        int be = 0;
        if (k < n) {
            for (int e = 0; e < nrec; ++e) {
                const unsigned long long c = recs.a[e].key;
                const bool take = mine(e) && c < prev && c > best;
                best = take ? c : best;
                be = take ? e : be;
            }
            prev = best;
        }
        store_slot<S>(out, (size_t)k * hw + p, recs, k < n ? be : -1);
    }
    out.count[p] = (uint8_t)n;
}

// Key, x and y of a record in one 16-byte load.
__device__ inline KeyXY load_key_xy(const KeyXY *r) { return *r; }

// One workgroup per bin. LDS: per-pixel offsets [npx + 1], then the key list (u64), the records'
// positions in the bin (u16) and, for binary16 buffers, their encoded offsets (u32), each with
// kListSlots entries (kListCap records plus the pads of swz).
template <typename S, int KMAX>
__global__ __launch_bounds__(sel_threads<KMAX>()) void k_bin_select(afr_deep_buffer out, BinGeom g,
                                                            const int32_t *tot, int nchunks,
                                                            Bucket bucket, const int32_t *bad_tab,
                                                            unsigned long long *dropped) {
    constexpr int kSelThreads = sel_threads<KMAX>(), kSelPer = kListCap / kSelThreads;
    extern __shared__ uint4 sel_lds[];  // 16-byte aligned for the key list
    int *sel_sm = reinterpret_cast<int *>(sel_lds);
    if (blockIdx.x == 0) {  // dropped samples: the per-chunk counts of the count and scatter passes
        int v = 0;
        for (int i = threadIdx.x; i < 2 * nchunks; i += kSelThreads) v += bad_tab[i];
        v = block_sum_int<kSelThreads>(v);
        if (threadIdx.x == 0) *dropped = (unsigned long long)v;
    }
    const int npx = g.bw * g.bh;
    int *poff = sel_sm;  // [npx + 1]
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(sel_sm + ((npx + 2) & ~1));
    unsigned short *pos = reinterpret_cast<unsigned short *>(keys + kListSlots);
    unsigned *oxy = reinterpret_cast<unsigned *>(pos + kListSlots);  // binary16 only
    const int b = blockIdx.x;
    const int s0 = bin_start<kSelThreads>(tot, b);
    const int nrec = tot[b];
    const BinRecs recs{bucket.a + s0, bucket.b + s0, bucket.h + s0};
    const int bx0 = (b % g.nbx) * kBinW, by0 = (b / g.nbx) * g.bh;
    const int W = out.width, H = out.height;
    const size_t hw = (size_t)W * H;
    const int rows = min(g.bh, H - by0);
    auto local_id = [&](float x, float y) {
        return ((int)floorf(y) - by0) * kBinW + ((int)floorf(x) - bx0);
    };
    for (int q = threadIdx.x; q <= npx; q += kSelThreads) poff[q] = 0;
    __syncthreads();
    if (nrec <= kListCap) {
        // One sweep: each thread keeps its records' keys, pixels and ranks in registers.
        unsigned long long kk[kSelPer];
        int id[kSelPer], rk[kSelPer];
        unsigned ox[kOxyInList<S> ? kSelPer : 1];
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) {
            const int e = j * kSelThreads + threadIdx.x;
            if (e < nrec) {
                const KeyXY r = load_key_xy(recs.a + e);
                kk[j] = r.key;
                id[j] = local_id(r.x, r.y);
                rk[j] = atomicAdd(&poff[id[j]], 1);
                if constexpr (kOxyInList<S>) ox[j] = encode_oxy(r.x, r.y);
            }
        }
        __syncthreads();
        const int total = block_scan_lds<kSelThreads>(poff, poff, npx);
        if (threadIdx.x == 0) poff[npx] = total;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) {
            const int e = j * kSelThreads + threadIdx.x;
            if (e < nrec) {
                const int l = poff[id[j]] + rk[j];
                keys[swz(l)] = kk[j];
                pos[swz(l)] = (unsigned short)e;
                if constexpr (kOxyInList<S>) oxy[swz(l)] = ox[j];
            }
        }
        __syncthreads();
        // Binary32 records with 4 < K <= 16: two threads per pixel (the two halves of the workgroup,
        // so each wave stays on one half) sort the same list and store half of the slots each,
        // which halves the chain of 32-byte record fetches per thread.
        constexpr int kHalves = (KMAX >= 8 && KMAX <= 16 && !kOxyInList<S>) ? 2 : 1;
        const int nq = rows * kBinW;
        for (int t = threadIdx.x; t < kHalves * nq; t += kSelThreads) {
            const int q = t % nq, hh = t / nq;
            const int px = bx0 + q % kBinW, py = by0 + q / kBinW;
            if (px < W)
                select_pixel<S, KMAX>(out, (size_t)py * W + px, hw, recs, keys, pos, oxy, poff[q],
                                      poff[q + 1], hh * (KMAX / kHalves),
                                      (hh + 1) * (KMAX / kHalves));
        }
        return;
    }
    // Larger bins: count per pixel, then passes over groups of whole rows whose records fit the
    // list. During a pass's fill the offsets of its pixels advance to their ends, so a pixel's
    // list is [end of the previous pixel, own end). A single row beyond the list (or a bin beyond
    // u16 positions) takes the direct scan.
    for (int e = threadIdx.x; e < nrec; e += kSelThreads) {
        const KeyXY r = load_key_xy(recs.a + e);
        atomicAdd(&poff[local_id(r.x, r.y)], 1);
    }
    __syncthreads();
    const int total = block_scan_lds<kSelThreads>(poff, poff, npx);
    if (threadIdx.x == 0) poff[npx] = total;
    __syncthreads();
    for (int r0 = 0; r0 < rows;) {
        int r1 = r0 + 1;
        while (r1 < rows && poff[(r1 + 1) * kBinW] - poff[r0 * kBinW] <= kListCap) ++r1;
        const int q0 = r0 * kBinW, q1 = r1 * kBinW;
        const int lo = poff[q0], hi = poff[q1];
        __syncthreads();  // every thread has read the bounds before the fill moves them
        if (hi - lo <= kListCap && nrec <= 65536) {
            for (int e = threadIdx.x; e < nrec; e += kSelThreads) {
                const KeyXY r = load_key_xy(recs.a + e);
                const int q = local_id(r.x, r.y);
                if (q >= q0 && q < q1) {
                    const int l = atomicAdd(&poff[q], 1) - lo;
                    keys[swz(l)] = r.key;
                    pos[swz(l)] = (unsigned short)e;
                    if constexpr (kOxyInList<S>) oxy[swz(l)] = encode_oxy(r.x, r.y);
                }
            }
            __syncthreads();
            for (int q = q0 + threadIdx.x; q < q1; q += kSelThreads) {
                const int px = bx0 + q % kBinW, py = by0 + q / kBinW;
                if (px < W)
                    select_pixel<S, KMAX>(out, (size_t)py * W + px, hw, recs, keys, pos, oxy,
                                          q == q0 ? 0 : poff[q - 1] - lo, poff[q] - lo);
            }
        } else {
            for (int q = q0 + threadIdx.x; q < q1; q += kSelThreads) {
                const int px = bx0 + q % kBinW, py = by0 + q / kBinW;
                if (px < W) select_pixel_scan<S>(out, (size_t)py * W + px, hw, recs, nrec, px, py);
            }
        }
        __syncthreads();  // the list is rewritten by the next pass
        r0 = r1;
    }
}

template <typename S>
size_t select_shmem(const BinGeom &g) {
    return (size_t)((g.bw * g.bh + 2) & ~1) * sizeof(int) +
           kListSlots * (sizeof(unsigned long long) + sizeof(unsigned short) +
                         (kOxyInList<S> ? sizeof(unsigned) : 0));
}

template <typename S>
hipError_t launch_select(const afr_deep_buffer &out, const BinGeom &g, const int32_t *tot,
                         int nchunks, Bucket bucket, const int32_t *bad_tab,
                         unsigned long long *dropped, hipStream_t st) {
    const size_t shmem = select_shmem<S>(g);
    const dim3 grid(g.nb);
    auto go = [&](auto kmax_c) {
        constexpr int KM = decltype(kmax_c)::value;
        k_bin_select<S, KM><<<grid, dim3(sel_threads<KM>()), shmem, st>>>(out, g, tot, nchunks,
                                                                        bucket, bad_tab, dropped);
    };
    if (out.k <= 4) go(std::integral_constant<int, 4>{});
    else if (out.k <= 8) go(std::integral_constant<int, 8>{});
    else if (out.k <= 16) go(std::integral_constant<int, 16>{});
    else if (out.k <= 32) go(std::integral_constant<int, 32>{});
    else if (out.k <= 64) go(std::integral_constant<int, 64>{});
    else go(std::integral_constant<int, 256>{});
    return hipGetLastError();
}

__global__ void k_fill_zero(int32_t *p, int64_t len) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0;
}

BinGeom bin_geom(int32_t w, int32_t h) {
    BinGeom g;
    g.bw = kBinW;
    g.nbx = (w + g.bw - 1) / g.bw;
    g.bh = 4;
    g.sbh = 2;
    while ((size_t)g.nbx * ((h + g.bh - 1) / g.bh) > (size_t)kMaxBins && g.bw * g.bh < kMaxBinPx) {
        g.bh *= 2;
        ++g.sbh;
    }
    g.nby = (h + g.bh - 1) / g.bh;
    g.nb = g.nbx * g.nby;
    return g;
}

int64_t n_chunks(int64_t n, int per) {
    const int64_t chunk = (int64_t)kChunkThreads * per;
    return std::max<int64_t>(1, (n + chunk - 1) / chunk);
}

// Samples per thread for a launch over n samples. Two scatter workgroups are resident per CU, so the
// chunks run in ceil(chunks / (2 CUs)) rounds, and a round takes time in proportion to the chunk
// size; a partial last round costs a whole one. Take the size with the least rounds x size (the
// larger on a tie: a shorter offset table). The result never depends on the chunk size.
int pick_per(int64_t n) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    const int64_t slots = 2 * (int64_t)cus;
    int best = 8;
    int64_t best_cost = INT64_MAX;
    for (int per = kPerMin; per <= kPerMax; per += 2) {
        const int64_t cost = ((n_chunks(n, per) + slots - 1) / slots) * per;
        if (cost <= best_cost) {
            best_cost = cost;
            best = per;
        }
    }
    return best;
}

}  // namespace

bool build_supported(int32_t w, int32_t h) { return bin_geom(w, h).nb <= kMaxBins; }

// Workspace tables are sized for the smallest chunk (the most chunks) a launch can choose.
size_t build_ws_bytes(int64_t n, int32_t w, int32_t h) {
    const BinGeom g = bin_geom(w, h);
    const int64_t len = (int64_t)g.nb * n_chunks(n, kPerMin);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return align_up((size_t)(len + 1) * 4) + align_up((size_t)(g.nb + 1) * 4) +
           align_up((size_t)2 * n_chunks(n, kPerMin) * 4) + 2 * align_up(nn * sizeof(KeyXY)) +
           align_up(8);
}

BuildWs build_ws_carve(void *ws, int64_t n, int32_t w, int32_t h) {
    const BinGeom g = bin_geom(w, h);
    const int64_t len = (int64_t)g.nb * n_chunks(n, kPerMin);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    char *p = static_cast<char *>(ws);
    BuildWs o;
    o.offsets = reinterpret_cast<int32_t *>(p);
    p += align_up((size_t)(len + 1) * 4);
    o.bsum = reinterpret_cast<int32_t *>(p);
    p += align_up((size_t)(g.nb + 1) * 4);
    o.bad = reinterpret_cast<int32_t *>(p);
    p += align_up((size_t)2 * n_chunks(n, kPerMin) * 4);
    o.bucket = p;
    p += 2 * align_up(nn * sizeof(KeyXY));
    o.dropped_internal = reinterpret_cast<unsigned long long *>(p);
    return o;
}

hipError_t launch_build(const afr_samples &s, const afr_deep_buffer &out, const BuildWs &ws,
                        unsigned long long *dropped, hipStream_t st, hipEvent_t *stage_end) {
    auto mark = [&](int i) { return stage_end ? hipEventRecord(stage_end[i], st) : hipSuccess; };
    const ValidCtx c{out.width, out.height, out.t_ref, out.precision == AFR_FP16 ? 1 : 0};
    const BinGeom g = bin_geom(out.width, out.height);
    const int per = pick_per(s.n);
    const int64_t nch = n_chunks(s.n, per);
    const int64_t len = (int64_t)g.nb * nch;
    const size_t half = align_up((size_t)(s.n > 0 ? s.n : 1) * sizeof(KeyXY));
    char *pay = static_cast<char *>(ws.bucket) + half;
    const Bucket bucket{static_cast<KeyXY *>(ws.bucket), reinterpret_cast<float4 *>(pay),
                        reinterpret_cast<uint2 *>(pay)};
    // count and scatter with PER samples per thread, with or without reprojection
    auto chunked = [&](auto per_c, bool count) {
        constexpr int P = decltype(per_c)::value;
        const bool H = out.precision == AFR_FP16;
        const size_t shmem = count ? 0
                                   : (size_t)((g.nb + 3) & ~3) * sizeof(int) +
                                         kWin * (H ? sizeof(KeyXY) + sizeof(uint2) : sizeof(Record));
        if (count && s.vx)
            k_bin_count<true, P><<<(int)nch, kChunkThreads, 0, st>>>(s, c, g, ws.offsets, (int)nch,
                                                                     ws.bad);
        else if (count)
            k_bin_count<false, P><<<(int)nch, kChunkThreads, 0, st>>>(s, c, g, ws.offsets,
                                                                      (int)nch, ws.bad);
        else if (s.vx && H)
            k_bin_scatter<true, P, true><<<(int)nch, kChunkThreads, shmem, st>>>(
                s, c, g, ws.offsets, ws.bsum, (int)nch, bucket, ws.bad);
        else if (s.vx)
            k_bin_scatter<true, P, false><<<(int)nch, kChunkThreads, shmem, st>>>(
                s, c, g, ws.offsets, ws.bsum, (int)nch, bucket, ws.bad);
        else if (H)
            k_bin_scatter<false, P, true><<<(int)nch, kChunkThreads, shmem, st>>>(
                s, c, g, ws.offsets, ws.bsum, (int)nch, bucket, ws.bad);
        else
            k_bin_scatter<false, P, false><<<(int)nch, kChunkThreads, shmem, st>>>(
                s, c, g, ws.offsets, ws.bsum, (int)nch, bucket, ws.bad);
    };
    auto launch_chunked = [&](bool count) {
        if (per == 6) chunked(std::integral_constant<int, 6>{}, count);
        else if (per == 10) chunked(std::integral_constant<int, 10>{}, count);
        else chunked(std::integral_constant<int, 8>{}, count);
    };
    if (s.n > 0) {
        launch_chunked(true);
    } else {  // no samples: every (bin, chunk) count of the single empty chunk is zero, none dropped
        k_fill_zero<<<std::max(1, std::min((int)((len + 255) / 256), 1024)), 256, 0, st>>>(ws.offsets,
                                                                                       len);
        k_fill_zero<<<1, 256, 0, st>>>(ws.bad, 2 * nch);
    }
    hipError_t e = mark(0);
    if (e != hipSuccess) return e;
    k_scan_rows<<<g.nb, kScanThreads, 0, st>>>(ws.offsets, (int)nch, ws.bsum);
    if ((e = mark(1)) != hipSuccess) return e;
    if (s.n > 0) launch_chunked(false);
    if ((e = hipGetLastError()) != hipSuccess || (e = mark(2)) != hipSuccess) return e;
    e = out.precision == AFR_FP16
            ? launch_select<__half>(out, g, ws.bsum, (int)nch, bucket, ws.bad, dropped, st)
            : launch_select<float>(out, g, ws.bsum, (int)nch, bucket, ws.bad, dropped, st);
    return e != hipSuccess ? e : mark(3);
}

}  // namespace afr
