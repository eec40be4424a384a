// afr_reconstruct: one 64-lane workgroup per group of tiles_per_wave statistics tiles
// (see afr_tile_gather.h). Workgroups are assigned so that each XCD's L2 serves a contiguous band of
// the image.
#include "afr_tile_gather.h"

namespace afr {
namespace {

// One tile per wave at R <= 2 keeps five waves per SIMD (at most 96 VGPRs): the LDS of 19 such
// workgroups fits a CU, enough for every tile of a 640x480 image to be resident at once.
template <typename S, int R, int TPW>
__global__ __launch_bounds__(kWave, (TPW == 1 && R <= 2) ? 5 : 1) void k_reconstruct_tiled(
    BufView<S> v, gat::TiledParams p, TileGeom tg, const float *__restrict__ stats,
    float *__restrict__ rgb, float *__restrict__ aux, int gx) {
    __shared__ gat::Smem<R, TPW> sm;
    __shared__ float tparam[3 * TPW];
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx0 = (bid % gx) * TPW, ty = bid / gx;
    if (threadIdx.x < 3 * TPW) {
        const int t = threadIdx.x / 3, f = threadIdx.x % 3;
        const int T = ty * tg.tiles_x + min(tx0 + t, tg.tiles_x - 1);
        const int plane = f == 0 ? AFR_STAT_SX2 : (f == 1 ? AFR_STAT_SY2 : AFR_STAT_KT2);
        tparam[threadIdx.x] = stats[plane * tg.nt + T];
    }
    __syncthreads();
    gat::gather_group<S, R, TPW>(v, p, tg, tx0, ty, sm, tparam, rgb, aux);
}

template <typename S, int R, int TPW>
hipError_t launch_rt(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                     const gat::TiledParams &p, float *rgb, float *aux, hipStream_t st) {
    const TileGeom tg = geom_of(stats);
    const int gx = (tg.tiles_x + TPW - 1) / TPW;
    const int nblocks = gx * tg.tiles_y;
    k_reconstruct_tiled<S, R, TPW><<<nblocks, kWave, 0, st>>>(view_of<S>(buf), p, tg, stats.data,
                                                               rgb, aux, gx);
    return hipGetLastError();
}

template <typename S, int R>
hipError_t launch_r(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                    const gat::TiledParams &p, int tpw, float *rgb, float *aux, hipStream_t st) {
    // Four tiles per wave would exceed the static LDS budget at R = 4.
    if (tpw >= 4 && R <= 3) return launch_rt<S, R, (R <= 3 ? 4 : 2)>(buf, stats, p, rgb, aux, st);
    if (tpw >= 2) return launch_rt<S, R, 2>(buf, stats, p, rgb, aux, st);
    return launch_rt<S, R, 1>(buf, stats, p, rgb, aux, st);
}

template <typename S>
hipError_t launch_s(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                    const gat::TiledParams &p, int R, int tpw, float *rgb, float *aux,
                    hipStream_t st) {
    switch (R) {
        case 0: return launch_r<S, 0>(buf, stats, p, tpw, rgb, aux, st);
        case 1: return launch_r<S, 1>(buf, stats, p, tpw, rgb, aux, st);
        case 2: return launch_r<S, 2>(buf, stats, p, tpw, rgb, aux, st);
        case 3: return launch_r<S, 3>(buf, stats, p, tpw, rgb, aux, st);
        default: return launch_r<S, 4>(buf, stats, p, tpw, rgb, aux, st);
    }
}

}  // namespace

hipError_t launch_reconstruct_tiled(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                    const afr_params &prm, int tiles_per_wave, float *rgb,
                                    float *aux, hipStream_t st) {
    // The tiled form is specialised for 8 px statistics tiles; other tile sizes take the direct form.
    if (stats.tile != 8) return launch_reconstruct_plain(buf, stats, prm, rgb, aux, st);
    const gat::TiledParams p{prm.t_now, prm.t_now - buf.t_ref};
    if (buf.precision == AFR_FP16)
        return launch_s<__half>(buf, stats, p, prm.radius, tiles_per_wave, rgb, aux, st);
    return launch_s<float>(buf, stats, p, prm.radius, tiles_per_wave, rgb, aux, st);
}

}  // namespace afr
