// afr_estimate_gradients: one workgroup per statistics tile (see afr_tile_estimate.h).
#include "afr_tile_estimate.h"

namespace afr {
namespace {

template <typename S>
__global__ __launch_bounds__(256) void k_estimate(BufView<S> v, est::EstParams p, TileGeom tg,
                                                  float *stats) {
    __shared__ est::Smem sm;
    est::estimate_tile<S>(v, p, tg, blockIdx.x, stats, sm, nullptr);
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
    const int threads = tg.tile <= 8 ? 64 : 256;
    if (buf.precision == AFR_FP16)
        k_estimate<__half><<<tg.nt, threads, 0, st>>>(view_of<__half>(buf), p, tg, out.data);
    else
        k_estimate<float><<<tg.nt, threads, 0, st>>>(view_of<float>(buf), p, tg, out.data);
    return hipGetLastError();
}

}  // namespace afr
