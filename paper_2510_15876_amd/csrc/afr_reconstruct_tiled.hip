// afr_reconstruct and afr_forward: one workgroup of TPG waves per group of TPG horizontally adjacent
// statistics tiles (see afr_gather.h). afr_forward first evaluates the group's tile statistics with
// the strip estimator of afr_estimate_gradients (afr_tile_estimate.h) and hands their filter widths
// to the gather through LDS, so one launch reads the deep buffer for both steps. Workgroups are
// assigned so that each XCD's L2 serves a contiguous band of the image.
#include <type_traits>

#include "afr_gather.h"
#include "afr_tile_estimate.h"

namespace afr {
namespace {

// Largest group the static LDS allows at a radius (tables of R >= 3 regions take two tiles at most).
constexpr int max_group(int R) { return R <= 2 ? 4 : 2; }

// Waves per SIMD the kernels are compiled for. Four tiles per workgroup at R <= 2 with binary16
// storage: five (at most 96 VGPRs), so that five workgroups share a CU (their LDS, 30 KiB each, fits)
// and the 1200 workgroups of a 640x480 image run in one round; the fused kernel, which unbounded
// took 104 VGPRs (four waves, two rounds), fits without spills (forward 82 -> 77 us when bounded).
// Binary32 storage: four (at most 128 VGPRs), one round for 1024 workgroups (512x512).
template <typename S, int R>
constexpr int waves_per_simd() { return R <= 2 ? (std::is_same<S, __half>::value ? 5 : 4) : 1; }

template <typename S, int R, int TPG>
__global__ __launch_bounds__(64 * TPG, (waves_per_simd<S, R>())) void k_gather(
    BufView<S> v, gat::TiledParams p, TileGeom tg, const float *__restrict__ stats,
    float *__restrict__ rgb, float *__restrict__ aux, int gx) {
    __shared__ gat::Smem<S, R, TPG> sm;
    __shared__ float tparam[3 * TPG];
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx0 = (bid % gx) * TPG, ty = bid / gx;
    if (threadIdx.x < 3 * TPG) {
        const int t = threadIdx.x / 3, f = threadIdx.x % 3;
        const int T = ty * tg.tiles_x + min(tx0 + t, tg.tiles_x - 1);
        const int plane = f == 0 ? AFR_STAT_SX2 : (f == 1 ? AFR_STAT_SY2 : AFR_STAT_KT2);
        tparam[threadIdx.x] = stats[plane * tg.nt + T];
    }
    __syncthreads();
    gat::gather_strip<S, R, TPG>(v, p, tg, tx0, ty, sm, tparam, rgb, aux);
}

// Statistics, then the gather, of one group of TPG tiles (8 px tiles only).
template <typename S, int R, int TPG>
__global__ __launch_bounds__(64 * TPG, (waves_per_simd<S, R>())) void k_forward(
    BufView<S> v, est::EstParams ep, gat::TiledParams p, TileGeom tg, float *__restrict__ stats,
    float *__restrict__ rgb, float *__restrict__ aux, int gx) {
    constexpr size_t kEst = sizeof(est::StripSmem<TPG>), kGat = sizeof(gat::Smem<S, R, TPG>);
    __shared__ __align__(16) unsigned char raw[kEst > kGat ? kEst : kGat];
    __shared__ float tparam[3 * TPG];
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx0 = (bid % gx) * TPG, ty = bid / gx;
    if (threadIdx.x < TPG && tx0 + (int)threadIdx.x >= tg.tiles_x) {  // no such tile: any widths
        tparam[3 * threadIdx.x] = 1.0f;
        tparam[3 * threadIdx.x + 1] = 1.0f;
        tparam[3 * threadIdx.x + 2] = 0.0f;
    }
    est::estimate_strip<S, TPG>(v, ep, tg, tx0, ty, stats,
                                *reinterpret_cast<est::StripSmem<TPG> *>(raw), tparam);
    __syncthreads();
    gat::gather_strip<S, R, TPG>(v, p, tg, tx0, ty, *reinterpret_cast<gat::Smem<S, R, TPG> *>(raw),
                                 tparam, rgb, aux);
}

template <typename S, int R, int TPG>
hipError_t launch_rt(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                     const gat::TiledParams &p, const est::EstParams *ep, float *rgb, float *aux,
                     hipStream_t st) {
    const TileGeom tg = geom_of(stats);
    const int gx = (tg.tiles_x + TPG - 1) / TPG;
    const int nblocks = gx * tg.tiles_y;
    if (ep)
        k_forward<S, R, TPG><<<nblocks, 64 * TPG, 0, st>>>(view_of<S>(buf), *ep, p, tg, stats.data,
                                                           rgb, aux, gx);
    else
        k_gather<S, R, TPG><<<nblocks, 64 * TPG, 0, st>>>(view_of<S>(buf), p, tg, stats.data, rgb,
                                                          aux, gx);
    return hipGetLastError();
}

template <typename S, int R>
hipError_t launch_r(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                    const gat::TiledParams &p, const est::EstParams *ep, int tpg, float *rgb,
                    float *aux, hipStream_t st) {
    constexpr int G = max_group(R);
    if (tpg >= 4 && G >= 4) return launch_rt<S, R, G>(buf, stats, p, ep, rgb, aux, st);
    if (tpg >= 2) return launch_rt<S, R, 2>(buf, stats, p, ep, rgb, aux, st);
    return launch_rt<S, R, 1>(buf, stats, p, ep, rgb, aux, st);
}

template <typename S>
hipError_t launch_s(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                    const gat::TiledParams &p, const est::EstParams *ep, int R, int tpg,
                    float *rgb, float *aux, hipStream_t st) {
    switch (R) {
        case 0: return launch_r<S, 0>(buf, stats, p, ep, tpg, rgb, aux, st);
        case 1: return launch_r<S, 1>(buf, stats, p, ep, tpg, rgb, aux, st);
        case 2: return launch_r<S, 2>(buf, stats, p, ep, tpg, rgb, aux, st);
        case 3: return launch_r<S, 3>(buf, stats, p, ep, tpg, rgb, aux, st);
        default: return launch_r<S, 4>(buf, stats, p, ep, tpg, rgb, aux, st);
    }
}

}  // namespace

int default_tiles_per_group(int radius) { return max_group(radius); }

hipError_t launch_reconstruct_tiled(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                    const afr_params &prm, int tiles_per_group, float *rgb,
                                    float *aux, hipStream_t st) {
    // The tiled form is specialised for 8 px statistics tiles; other tile sizes take the direct form.
    if (stats.tile != 8) return launch_reconstruct_plain(buf, stats, prm, rgb, aux, st);
    const gat::TiledParams p{prm.t_now, prm.t_now - buf.t_ref};
    if (buf.precision == AFR_FP16)
        return launch_s<__half>(buf, stats, p, nullptr, prm.radius, tiles_per_group, rgb, aux, st);
    return launch_s<float>(buf, stats, p, nullptr, prm.radius, tiles_per_group, rgb, aux, st);
}

hipError_t launch_forward(const afr_deep_buffer &buf, const afr_params &prm,
                          const afr_tile_stats &stats, int tiles_per_group, float *rgb, float *aux,
                          hipStream_t st) {
    if (stats.tile != 8) {  // other tile sizes: the two separate steps
        const hipError_t e = launch_estimate(buf, prm, stats, st);
        if (e != hipSuccess) return e;
        return launch_reconstruct_plain(buf, stats, prm, rgb, aux, st);
    }
    const gat::TiledParams p{prm.t_now, prm.t_now - buf.t_ref};
    const est::EstParams ep = est_params(buf, prm);
    if (buf.precision == AFR_FP16)
        return launch_s<__half>(buf, stats, p, &ep, prm.radius, tiles_per_group, rgb, aux, st);
    return launch_s<float>(buf, stats, p, &ep, prm.radius, tiles_per_group, rgb, aux, st);
}

}  // namespace afr
