// afr_estimate_gradients: one workgroup per statistics tile (see afr_tile_estimate.h), tiles dealt
// to XCDs in contiguous bands so that the one-pixel halos neighbouring tiles share hit one L2.
#include "afr_tile_estimate.h"

namespace afr {
namespace {

template <typename S, int TB>
__global__ __launch_bounds__(TB <= 8 ? 64 : 256) void k_estimate(BufView<S> v, est::EstParams p,
                                                                 TileGeom tg, float *stats) {
    __shared__ est::Smem<TB> sm;
    est::estimate_tile<S, TB>(v, p, tg, xcd_remap(blockIdx.x, gridDim.x), stats, sm, nullptr);
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
                           const afr_tile_stats &out, hipStream_t st) {
    const est::EstParams p = est_params(buf, prm);
    const TileGeom tg = geom_of(out);
    const bool small = tg.tile <= 8;  // one wave per tile, scratch for a 10 x 10 halo region
    if (buf.precision == AFR_FP16) {
        if (small) k_estimate<__half, 8><<<tg.nt, 64, 0, st>>>(view_of<__half>(buf), p, tg, out.data);
        else k_estimate<__half, kMaxTile><<<tg.nt, 256, 0, st>>>(view_of<__half>(buf), p, tg, out.data);
    } else {
        if (small) k_estimate<float, 8><<<tg.nt, 64, 0, st>>>(view_of<float>(buf), p, tg, out.data);
        else k_estimate<float, kMaxTile><<<tg.nt, 256, 0, st>>>(view_of<float>(buf), p, tg, out.data);
    }
    return hipGetLastError();
}

}  // namespace afr
