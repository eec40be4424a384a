// afr_estimate_gradients (see afr_tile_estimate.h): for tiles of edge <= 8 one 256-thread workgroup
// per 32-pixel-wide strip of tiles, else one workgroup per tile. Workgroups are dealt to XCDs in
// contiguous bands so that the one-pixel halos neighbouring workgroups share hit one L2.
#include "afr_tile_estimate.h"

namespace afr {
namespace {

template <typename S, int TB>
__global__ __launch_bounds__(TB <= 8 ? 64 : 256) void k_estimate(BufView<S> v, est::EstParams p,
                                                                 TileGeom tg, float *stats) {
    __shared__ est::Smem<TB> sm;
    est::estimate_tile<S, TB>(v, p, tg, xcd_remap(blockIdx.x, gridDim.x), stats, sm, nullptr);
}

// Five waves per SIMD (at most 96 VGPRs): a 640 x 480 image's 1200 strips are then all resident at
// once; two slot planes per load chunk keep the moments within that budget.
template <typename S>
__global__ __launch_bounds__(est::Strip<4>::THREADS, 5) void k_estimate_strip(BufView<S> v,
                                                                             est::EstParams p,
                                                                             TileGeom tg, int sx,
                                                                             float *stats) {
    __shared__ est::StripSmem<4> sm;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    est::estimate_strip<S, 4>(v, p, tg, (b % sx) * est::strip_tiles(tg.tile, 4), b / sx, stats, sm,
                              nullptr);
}

}  // namespace

est::EstParams est_params(const afr_deep_buffer &buf, const afr_params &prm) {
    est::EstParams p;
    p.alpha = prm.alpha;
    p.t_now = prm.t_now;
    p.dt_ref = (double)prm.t_now - (double)buf.t_ref;
    p.dt_floor = prm.dt_floor;
    p.age_floor = prm.age_floor;
    p.g_floor = prm.g_floor;
    p.sigma = prm.sigma;
    p.tau = prm.tau;
    p.e_min = prm.e_min;
    p.e_max = prm.e_max;
    return p;
}

hipError_t launch_estimate(const afr_deep_buffer &buf, const afr_params &prm,
                           const afr_tile_stats &out, hipStream_t stream) {
    const est::EstParams p = est_params(buf, prm);
    const TileGeom tg = geom_of(out);
    if (tg.tile <= 8) {  // strips of 32 px
        const int st = est::strip_tiles(tg.tile, 4);
        const int sx = (tg.tiles_x + st - 1) / st;
        const int grid = sx * tg.tiles_y;
        if (buf.precision == AFR_FP16)
            k_estimate_strip<__half><<<grid, est::Strip<4>::THREADS, 0, stream>>>(
                view_of<__half>(buf), p, tg, sx, out.data);
        else
            k_estimate_strip<float><<<grid, est::Strip<4>::THREADS, 0, stream>>>(
                view_of<float>(buf), p, tg, sx, out.data);
    } else if (buf.precision == AFR_FP16) {
        k_estimate<__half, kMaxTile><<<tg.nt, 256, 0, stream>>>(view_of<__half>(buf), p, tg, out.data);
    } else {
        k_estimate<float, kMaxTile><<<tg.nt, 256, 0, stream>>>(view_of<float>(buf), p, tg, out.data);
    }
    return hipGetLastError();
}

}  // namespace afr
