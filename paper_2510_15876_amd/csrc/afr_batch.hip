// Batched reconstruction in one launch, and the launch-shape tuner.
//
// A work item is (batch item, group of TPG statistics tiles in one tile row). One workgroup per work
// item first evaluates the statistics of its own tiles (est::estimate_strip, the code of
// afr_estimate_gradients) and then gathers them (gat::gather_strip, the code of afr_reconstruct), so
// no work item depends on another and nothing spins. Work items are numbered with the larger batch
// items first and dealt to workgroups in that order, in short runs per XCD (not one contiguous
// range per XCD, which would leave the XCDs holding the large items to finish last), so a run is
// one kernel launch and nothing else: capturable and replayable. (A persistent grid taking items
// from a counter needed 128 registers and four waves per SIMD; one item per workgroup fits in 96
// and five: 2.69 -> 2.1-2.2 ms for the 64-item batch.)
#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <type_traits>
#include <vector>

#include "afr_gather.h"
#include "afr_tile_estimate.h"

namespace afr {
namespace {

struct DevItem {
    const void *ox, *oy, *ta, *r, *g, *b;
    const uint8_t *count;
    int32_t width, height, k;
    float t_ref;
    TileGeom tg;
    float *stats, *rgb, *aux;
    est::EstParams ep;
    gat::TiledParams tp;
};

constexpr int kShapes[3] = {1, 2, 4};

template <typename S>
__device__ inline BufView<S> item_view(const DevItem &d) {
    BufView<S> v;
    v.ox = static_cast<const S *>(d.ox);
    v.oy = static_cast<const S *>(d.oy);
    v.ta = static_cast<const S *>(d.ta);
    v.r = static_cast<const S *>(d.r);
    v.g = static_cast<const S *>(d.g);
    v.b = static_cast<const S *>(d.b);
    v.count = d.count;
    v.width = d.width;
    v.height = d.height;
    v.k = d.k;
    v.t_ref = d.t_ref;
    return v;
}

// Waves per SIMD the batch kernel is compiled for, as the fused single-frame kernel: five with
// binary16 storage at R <= 2 (at most 96 VGPRs), four with binary32, unbounded at larger radii.
template <typename S, int R>
constexpr int batch_waves() { return R <= 2 ? (std::is_same<S, __half>::value ? 5 : 4) : 1; }

template <typename S, int R, int TPG>
__global__ __launch_bounds__(64 * TPG, (batch_waves<S, R>())) void k_batch(const DevItem *__restrict__ items, int n,
                                                   const int *__restrict__ first) {
    constexpr size_t kEst = sizeof(est::StripSmem<TPG>), kGat = sizeof(gat::Smem<S, R, TPG>);
    __shared__ __align__(16) unsigned char raw[kEst > kGat ? kEst : kGat];
    __shared__ float tparam[3 * TPG];
    est::StripSmem<TPG> &esm = *reinterpret_cast<est::StripSmem<TPG> *>(raw);
    gat::Smem<S, R, TPG> &gsm = *reinterpret_cast<gat::Smem<S, R, TPG> *>(raw);
    {
        // The work item (the grid is exactly first[n] workgroups). Workgroups are dealt to the eight
        // XCDs in turn; within each group of 64, XCD x takes the 8 consecutive items from 8x, so
        // neighbouring tile groups (which share halo rows) meet in one L2 while every XCD still
        // moves through the list, large items to small, with the others (2.16 -> 2.11 ms).
        const int bid = (int)blockIdx.x, g64 = bid / 64;
        const int w = (g64 + 1) * 64 <= (int)gridDim.x ? g64 * 64 + (bid % 8) * 8 + (bid / 8) % 8
                                                         : bid;
        int lo = 0, hi = n - 1;  // the item b with first[b] <= w < first[b + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (first[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        const DevItem &d = items[lo];
        const BufView<S> v = item_view<S>(d);
        const int gx = (d.tg.tiles_x + TPG - 1) / TPG;
        const int local = w - first[lo];
        const int tx0 = (local % gx) * TPG, ty = local / gx;
        if (threadIdx.x < TPG && tx0 + (int)threadIdx.x >= d.tg.tiles_x) {  // no such tile
            tparam[3 * threadIdx.x] = 1.0f;
            tparam[3 * threadIdx.x + 1] = 1.0f;
            tparam[3 * threadIdx.x + 2] = 0.0f;
        }
        est::estimate_strip<S, TPG>(v, d.ep, d.tg, tx0, ty, d.stats, esm, tparam);
        __syncthreads();
        gat::gather_strip<S, R, TPG>(v, d.tp, d.tg, tx0, ty, gsm, tparam, d.rgb, d.aux);
    }
}

using KernelFn = void (*)(const DevItem *, int, const int *);

template <typename S, int R>
KernelFn kernel_for(int tpw) {
    if (tpw == 4 && R <= 2) return k_batch<S, R, (R <= 2 ? 4 : 2)>;
    if (tpw >= 2) return k_batch<S, R, 2>;
    return k_batch<S, R, 1>;
}

template <typename S>
KernelFn kernel_for_r(int R, int tpw) {
    switch (R) {
        case 0: return kernel_for<S, 0>(tpw);
        case 1: return kernel_for<S, 1>(tpw);
        case 2: return kernel_for<S, 2>(tpw);
        case 3: return kernel_for<S, 3>(tpw);
        default: return kernel_for<S, 4>(tpw);
    }
}

KernelFn batch_kernel(int precision, int R, int tpw) {
    return precision == AFR_FP16 ? kernel_for_r<__half>(R, tpw) : kernel_for_r<float>(R, tpw);
}

int shape_index(int tpw) { return tpw == 1 ? 0 : (tpw == 2 ? 1 : 2); }

bool shape_supported(int tpw, int R) { return tpw == 1 || tpw == 2 || (tpw == 4 && R <= 2); }

size_t table_bytes(int n) { return align_up((size_t)n * sizeof(DevItem)); }
size_t first_bytes(int n) { return align_up((size_t)(n + 1) * sizeof(int)); }

// Host image of a validated batch: the item table in work order (larger items first, so that the
// last items taken are the smallest, which evens the tail) and, per launch shape, the first work
// item of every batch item (with the total at [n]).
struct HostPlan {
    int n = 0, precision = 0, radius = 0, tpw = 0;
    std::vector<DevItem> table;
    std::vector<int> first[3];
};

afr_status make_host_plan(const afr_batch_item *items, int32_t n, int32_t tiles_per_wave,
                          int default_tpw, HostPlan &hp) {
    if (tiles_per_wave != 0 && tiles_per_wave != 1 && tiles_per_wave != 2 && tiles_per_wave != 4)
        return AFR_E_RANGE;
    const int R = items[0].params.radius, prec = items[0].buf.precision;
    for (int i = 0; i < n; ++i) {
        const afr_batch_item &it = items[i];
        afr_status st = check_buffer(&it.buf);
        if (st == AFR_OK) st = check_params(&it.params, &it.buf);
        if (st == AFR_OK) st = check_stats(&it.stats, &it.buf, &it.params);
        if (st != AFR_OK) return st;
        if (!it.rgb) return AFR_E_INVALID;
        if (it.params.tile != 8 || it.params.radius != R || it.buf.precision != prec)
            return AFR_E_UNSUPPORTED;
    }
    const int tpw = tiles_per_wave == 0 ? default_tpw : tiles_per_wave;
    if (!shape_supported(tpw, R)) return AFR_E_RANGE;
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const double wa = (double)items[a].buf.width * items[a].buf.height * items[a].buf.k;
        const double wb = (double)items[b].buf.width * items[b].buf.height * items[b].buf.k;
        return wa > wb;
    });
    hp.n = n;
    hp.precision = prec;
    hp.radius = R;
    hp.tpw = tpw;
    hp.table.assign(n, DevItem{});
    for (int s = 0; s < 3; ++s) hp.first[s].assign(n + 1, 0);
    for (int j = 0; j < n; ++j) {
        const afr_batch_item &it = items[order[j]];
        DevItem &d = hp.table[j];
        d.ox = it.buf.ox;
        d.oy = it.buf.oy;
        d.ta = it.buf.tage;
        d.r = it.buf.r;
        d.g = it.buf.g;
        d.b = it.buf.b;
        d.count = it.buf.count;
        d.width = it.buf.width;
        d.height = it.buf.height;
        d.k = it.buf.k;
        d.t_ref = it.buf.t_ref;
        d.tg = geom_of(it.stats);
        d.stats = it.stats.data;
        d.rgb = it.rgb;
        d.aux = it.aux;
        d.ep = est_params(it.buf, it.params);
        d.tp = gat::TiledParams{it.params.t_now, it.params.t_now - it.buf.t_ref};
        for (int s = 0; s < 3; ++s) {
            const int gx = (d.tg.tiles_x + kShapes[s] - 1) / kShapes[s];
            const int64_t next = (int64_t)hp.first[s][j] + (int64_t)gx * d.tg.tiles_y;
            if (next >= (int64_t(1) << 24)) return AFR_E_RANGE;  // one workgroup per work item
            hp.first[s][j + 1] = (int)next;
        }
    }
    return AFR_OK;
}

// Launch shape that afr_batch_tune last found fastest, per (precision, radius).
std::mutex g_btune_mu;
std::map<std::pair<int, int>, int> g_btune;

// Writes words to device memory from a kernel's arguments (passed by value, so the launch can be
// captured into a graph with the data in it).
constexpr int kArgWords = 480;
struct WordBlock {
    uint32_t w[kArgWords];
};
__global__ void k_put_words(uint32_t *__restrict__ dst, WordBlock b, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = b.w[i];
}

hipError_t put_bytes(void *dst, const void *src, size_t bytes, hipStream_t st) {
    static_assert(sizeof(DevItem) % 4 == 0, "the item table is whole words");
    const uint32_t *w = static_cast<const uint32_t *>(src);
    uint32_t *d = static_cast<uint32_t *>(dst);
    const size_t nw = bytes / 4;
    for (size_t o = 0; o < nw; o += kArgWords) {
        WordBlock b;
        const int m = (int)std::min<size_t>(kArgWords, nw - o);
        std::copy(w + o, w + o + m, b.w);
        k_put_words<<<1, 256, 0, st>>>(d + o, b, m);
    }
    return hipGetLastError();
}

// ---- single-frame tuner cache: (width, height, k, precision, radius) -> tiles per wave ---------
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int>, int> g_tune;

}  // namespace

int tuned_tiles_per_wave(const afr_deep_buffer &b, int radius) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(std::make_tuple(b.width, b.height, b.k, b.precision, radius));
    return it == g_tune.end() ? 0 : it->second;
}

void record_tiles_per_wave(const afr_deep_buffer &b, int radius, int tpw) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[std::make_tuple(b.width, b.height, b.k, b.precision, radius)] = tpw;
}

}  // namespace afr

struct afr_batch {
    int n = 0;
    int precision = 0, radius = 0;
    int tpw = 2;
    int total[3] = {0, 0, 0};  // work items (workgroups) per launch shape
    afr::DevItem *d_items = nullptr;
    int *d_first[3] = {nullptr, nullptr, nullptr};
};

using namespace afr;

extern "C" {

size_t afr_batch_workspace_bytes(int32_t n) {
    if (n < 1) return 0;
    return table_bytes(n) + 3 * first_bytes(n);
}

afr_status afr_batch_create(const afr_batch_item *items, int32_t n, int32_t tiles_per_wave,
                            void *ws, size_t ws_bytes, afr_batch **plan) {
    if (!items || n < 1 || !ws || !plan) return AFR_E_INVALID;
    *plan = nullptr;
    if (ws_bytes < afr_batch_workspace_bytes(n)) return AFR_E_NOMEM;
    HostPlan hp;
    const afr_status st = make_host_plan(items, n, tiles_per_wave,
                                         items[0].params.radius <= 2 ? 4 : 2, hp);
    if (st != AFR_OK) return st;
    char *p = static_cast<char *>(ws);
    afr_batch *b = new (std::nothrow) afr_batch;
    if (!b) return AFR_E_NOMEM;
    b->n = n;
    b->precision = hp.precision;
    b->radius = hp.radius;
    b->tpw = hp.tpw;
    b->d_items = reinterpret_cast<DevItem *>(p);
    p += table_bytes(n);
    for (int s = 0; s < 3; ++s) {
        b->d_first[s] = reinterpret_cast<int *>(p);
        p += first_bytes(n);
        b->total[s] = hp.first[s][n];
    }
    hipError_t e = hipMemcpy(b->d_items, hp.table.data(), n * sizeof(DevItem), hipMemcpyHostToDevice);
    for (int s = 0; s < 3 && e == hipSuccess; ++s)
        e = hipMemcpy(b->d_first[s], hp.first[s].data(), (n + 1) * sizeof(int),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete b;
        return AFR_E_DEVICE;
    }
    *plan = b;
    return AFR_OK;
}

afr_status afr_batch_reconstruct(const afr_batch_item *items, int32_t n, const afr_tune *tune,
                                 hipStream_t stream) {
    if (!items || n < 1 || !tune || !tune->ws) return AFR_E_INVALID;
    if (tune->ws_bytes < afr_batch_workspace_bytes(n)) return AFR_E_NOMEM;
    int def = items[0].params.radius <= 2 ? 4 : 2;
    {
        std::lock_guard<std::mutex> lock(g_btune_mu);
        const auto it = g_btune.find({items[0].buf.precision, items[0].params.radius});
        if (it != g_btune.end()) def = it->second;
    }
    HostPlan hp;
    const afr_status st = make_host_plan(items, n, tune->tiles_per_wave, def, hp);
    if (st != AFR_OK) return st;
    const int s = shape_index(hp.tpw);
    const int total = hp.first[s][n];
    char *p = static_cast<char *>(tune->ws);
    DevItem *d_items = reinterpret_cast<DevItem *>(p);
    p += table_bytes(n);
    int *d_first = reinterpret_cast<int *>(p);  // this shape's first items only
    hipError_t e = put_bytes(d_items, hp.table.data(), n * sizeof(DevItem), stream);
    if (e == hipSuccess) e = put_bytes(d_first, hp.first[s].data(), (n + 1) * sizeof(int), stream);
    if (e != hipSuccess) return AFR_E_DEVICE;
    if (total == 0) return AFR_OK;  // no tiles at all
    KernelFn fn = batch_kernel(hp.precision, hp.radius, hp.tpw);
    hipLaunchKernelGGL(fn, dim3(total), dim3(kWave * hp.tpw), 0, stream, d_items, n, d_first);
    return hipGetLastError() == hipSuccess ? AFR_OK : AFR_E_DEVICE;
}

afr_status afr_batch_run(const afr_batch *b, hipStream_t stream) {
    if (!b) return AFR_E_INVALID;
    const int s = shape_index(b->tpw);
    if (b->total[s] == 0) return AFR_OK;  // no tiles at all
    KernelFn fn = batch_kernel(b->precision, b->radius, b->tpw);
    hipLaunchKernelGGL(fn, dim3(b->total[s]), dim3(kWave * b->tpw), 0, stream, b->d_items, b->n,
                       b->d_first[s]);
    return hipGetLastError() == hipSuccess ? AFR_OK : AFR_E_DEVICE;
}

afr_status afr_batch_tune(afr_batch *b, hipStream_t stream, int32_t *best_tpw, float *best_ms) {
    if (!b) return AFR_E_INVALID;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return AFR_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return AFR_E_DEVICE;
    }
    const int keep = b->tpw;
    int best = keep;
    float best_t = 1e30f;
    afr_status st = AFR_OK;
    for (int s = 0; s < 3 && st == AFR_OK; ++s) {
        if (!shape_supported(kShapes[s], b->radius)) continue;
        b->tpw = kShapes[s];
        st = afr_batch_run(b, stream);  // warm-up
        constexpr int kReps = 3;
        if (st == AFR_OK && hipEventRecord(e0, stream) != hipSuccess) st = AFR_E_DEVICE;
        for (int r = 0; r < kReps && st == AFR_OK; ++r) st = afr_batch_run(b, stream);
        float ms = 0.0f;
        if (st == AFR_OK && (hipEventRecord(e1, stream) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = AFR_E_DEVICE;
        if (st == AFR_OK && ms / kReps < best_t) {
            best_t = ms / kReps;
            best = kShapes[s];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tpw = st == AFR_OK ? best : keep;
    if (st == AFR_OK) {
        std::lock_guard<std::mutex> lock(g_btune_mu);
        g_btune[{b->precision, b->radius}] = best;
    }
    if (st == AFR_OK) {
        if (best_tpw) *best_tpw = best;
        if (best_ms) *best_ms = best_t;
    }
    return st;
}

int32_t afr_batch_tiles_per_wave(const afr_batch *b) { return b ? b->tpw : 0; }

void afr_batch_destroy(afr_batch *b) { delete b; }

}  // extern "C"
