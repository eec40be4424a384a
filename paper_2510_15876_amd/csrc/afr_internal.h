// Internal declarations of libafr: device views of the public structs, storage codecs and the
// host-side launchers that each kernel translation unit exports to the API layer.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "afr.h"

namespace afr {

constexpr int kWave = 64;
constexpr int kMaxTile = 16;
constexpr int kMaxRadius = 4;

// ---- storage codecs ---------------------------------------------------------------------------
// FP32 buffers store the sample time t; FP16 buffers store age_ref = t_ref - t as binary16.
template <typename S>
struct Codec;

template <>
struct Codec<float> {
    __device__ static float dec(float v) { return v; }
    __device__ static float enc(float v) { return v; }
    // age at t_now of a stored time value
    __device__ static float age(float tv, float t_now, float /*dt_ref*/) { return t_now - tv; }
    __device__ static double age64(float tv, double t_now, double /*dt_ref*/) {
        return t_now - (double)tv;
    }
    // value stored for a sample time (fp32 mode keeps the time itself)
    __device__ static float enc_time(float t, float /*t_ref*/) { return t; }
};

template <>
struct Codec<__half> {
    __device__ static float dec(__half v) { return __half2float(v); }
    __device__ static __half enc(float v) { return __float2half_rn(v); }
    __device__ static float age(__half tv, float /*t_now*/, float dt_ref) {
        return dt_ref + __half2float(tv);
    }
    __device__ static double age64(__half tv, double /*t_now*/, double dt_ref) {
        return dt_ref + (double)__half2float(tv);
    }
    __device__ static __half enc_time(float t, float t_ref) { return __float2half_rn(t_ref - t); }
};

// ---- device views -----------------------------------------------------------------------------
template <typename S>
struct BufView {
    const S *ox, *oy, *ta, *r, *g, *b;
    const uint8_t *count;
    int32_t width, height, k;
    float t_ref;
};

template <typename S>
inline BufView<S> view_of(const afr_deep_buffer &d) {
    BufView<S> v;
    v.ox = static_cast<const S *>(d.ox);
    v.oy = static_cast<const S *>(d.oy);
    v.ta = static_cast<const S *>(d.tage);
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

// Layout of the tile statistics and of the gather geometry, as seen by the kernels.
struct TileGeom {
    int32_t tile, tiles_x, tiles_y;
    int32_t nt;  // tiles_x * tiles_y (plane stride)
};

inline TileGeom geom_of(const afr_tile_stats &s) {
    return TileGeom{s.tile, s.tiles_x, s.tiles_y, s.tiles_x * s.tiles_y};
}

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// ---- launchers (each returns hipGetLastError() of its launches) ---------------------------------
struct BuildWs {
    int32_t *cnt;       // [HW]       arrivals per pixel
    int32_t *off;       // [HW + 1]   bucket offsets (exclusive scan of cnt)
    int32_t *bsum;      // [nblk + 1] scan block sums
    int32_t *rank;      // [n]        arrival rank of each sample in its home pixel, -1 if dropped
    void *bucket;       // [n]        32-byte records grouped by home pixel
    unsigned long long *dropped_internal;
};
size_t build_ws_bytes(int64_t n, int32_t w, int32_t h);
BuildWs build_ws_carve(void *ws, int64_t n, int32_t w, int32_t h);
hipError_t launch_build(const afr_samples &s, const afr_deep_buffer &out, const BuildWs &ws,
                        unsigned long long *dropped, hipStream_t st);

hipError_t launch_estimate(const afr_deep_buffer &buf, const afr_params &p, const afr_tile_stats &out,
                           hipStream_t st);

hipError_t launch_reconstruct_plain(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                    const afr_params &p, float *rgb, float *aux, hipStream_t st);
// tiles_per_wave: launch shape of the tiled gather (1, 2 or 4); it does not change the result.
hipError_t launch_reconstruct_tiled(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                    const afr_params &p, int tiles_per_wave, float *rgb, float *aux,
                                    hipStream_t st);

size_t backward_ws_bytes(int32_t w, int32_t h);
hipError_t launch_backward(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                           const afr_params &p, const float *rgb, const float *aux,
                           const float *grad_rgb, float *grad_slot, float *grad_params, void *ws,
                           hipStream_t st);

}  // namespace afr
