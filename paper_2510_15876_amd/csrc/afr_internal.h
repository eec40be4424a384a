// Internal declarations of libafr: device views of the public structs, storage codecs and the
// host-side launchers that each kernel translation unit exports to the API layer.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
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

// Slot layout: binary32 buffers keep each field in its own [K][H][W] plane; binary16 buffers keep
// each slot as one 12-byte record (ox, oy, r, g, b, age_ref), so the field pointers step by six
// elements from slot to slot.
template <typename S>
struct Slots;
template <>
struct Slots<float> {
    static constexpr int kStride = 1;
};
template <>
struct Slots<__half> {
    static constexpr int kStride = 6;
    static constexpr int kBytes = 12;
};

// Field value of slot s (slot plane k of pixel q: s = k W H + q) through its field pointer.
template <typename S>
__device__ inline S fld(const S *f, size_t s) {
    return f[s * Slots<S>::kStride];
}

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

// ---- host-side argument validation shared by the entry points ----------------------------------
inline bool finite(float v) { return std::isfinite(v); }


inline afr_status check_buffer(const afr_deep_buffer *b) {
    if (!b) return AFR_E_INVALID;
    if (b->width < 1 || b->height < 1) return AFR_E_RANGE;
    if (b->k < 1 || b->k > 255) return AFR_E_RANGE;
    if (b->precision != AFR_FP32 && b->precision != AFR_FP16) return AFR_E_RANGE;
    // every flat slot index must fit in int32 arithmetic on the device, and the buffer-resource
    // loads address one slot plane with 32-bit byte offsets: a plane stays below 2^31 bytes
    if ((int64_t)b->width * b->height * b->k >= (int64_t(1) << 31)) return AFR_E_RANGE;
    const int64_t slot_bytes = b->precision == AFR_FP16 ? 12 : 4;
    if ((int64_t)b->width * b->height * slot_bytes >= (int64_t(1) << 31)) return AFR_E_RANGE;
    if (!finite(b->t_ref)) return AFR_E_RANGE;
    if (!b->ox || !b->oy || !b->tage || !b->r || !b->g || !b->b || !b->count) return AFR_E_INVALID;
    if (b->precision == AFR_FP16) {  // one array of 12-byte records, fields at 2-byte steps
        const char *o = static_cast<const char *>(b->ox);
        if (reinterpret_cast<uintptr_t>(o) % 4 != 0 || static_cast<const char *>(b->oy) != o + 2 ||
            static_cast<const char *>(b->r) != o + 4 || static_cast<const char *>(b->g) != o + 6 ||
            static_cast<const char *>(b->b) != o + 8 || static_cast<const char *>(b->tage) != o + 10)
            return AFR_E_INVALID;
    }
    return AFR_OK;
}

inline afr_status check_params(const afr_params *p, const afr_deep_buffer *b) {
    if (!p) return AFR_E_INVALID;
    const float vals[] = {p->sigma, p->tau, p->alpha, p->e_min, p->g_floor, p->dt_floor,
                          p->age_floor, p->t_now};
    for (float v : vals)
        if (!finite(v)) return AFR_E_RANGE;
    if (p->sigma < 0.0f || p->tau < 0.0f || p->alpha < 0.0f || !(p->g_floor > 0.0f)) return AFR_E_RANGE;
    if (!(p->e_min > 0.0f) || !(p->e_max > 0.0f) || std::isnan(p->e_max)) return AFR_E_RANGE;
    if (!(p->dt_floor > 0.0f) || !(p->age_floor > 0.0f)) return AFR_E_RANGE;
    if (p->radius < 0 || p->radius > kMaxRadius) return AFR_E_RANGE;
    if (p->tile < 1 || p->tile > kMaxTile) return AFR_E_RANGE;
    if (b && !(p->t_now >= b->t_ref)) return AFR_E_RANGE;
    return AFR_OK;
}

inline afr_status check_stats(const afr_tile_stats *s, const afr_deep_buffer *b, const afr_params *p) {
    if (!s || !s->data) return AFR_E_INVALID;
    if (s->tile != p->tile) return AFR_E_INVALID;
    if (s->tiles_x != (b->width + s->tile - 1) / s->tile ||
        s->tiles_y != (b->height + s->tile - 1) / s->tile)
        return AFR_E_INVALID;
    return AFR_OK;
}

// Launch shape chosen by afr_reconstruct_tune for a buffer class (0 when none was recorded).
int tuned_tiles_per_wave(const afr_deep_buffer &b, int radius);
void record_tiles_per_wave(const afr_deep_buffer &b, int radius, int tpw);

// ---- launchers (each returns hipGetLastError() of its launches) ---------------------------------
struct BuildWs {
    int32_t *offsets;   // [bins * chunks + 1] (bin, chunk) counts, then each bin row's exclusive scan
    int32_t *bsum;      // [bins] record count of each bin
    int32_t *bad;       // [2 * chunks] dropped samples per chunk (outside the image; invalid payload)
    void *bucket;       // [n] records grouped by bin, as two 16-byte halves in two arrays
    unsigned long long *dropped_internal;
};
// Buffer-resource loads of one slot plane: the descriptor (SGPRs) holds the plane's base address
// and byte size, each lane passes only a 32-bit byte offset, and a load at or past the size returns
// zero instead of touching memory. Plane sizes are < 2^31 bytes (check_buffer enforces it).
constexpr int kBufferWord3 = 0x00020000;  // gfx9 family: raw (untyped) 32-bit data
__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kBufferWord3);
}
template <typename S>
__device__ inline S plane_load(__amdgpu_buffer_rsrc_t r, unsigned byte_off);
template <>
__device__ inline float plane_load<float>(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
template <>
__device__ inline __half plane_load<__half>(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    return __ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, byte_off, 0, 0));
}

// Two and three consecutive 32-bit words (4-byte aligned offset) through the same descriptor.
__device__ inline uint2 load_u32x2(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
    return make_uint2(v[0], v[1]);
}
__device__ inline uint3 load_u32x3(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, byte_off, 0, 0);
    return make_uint3(v[0], v[1], v[2]);
}

// Workgroups are dealt round-robin to the 8 XCDs (physical id b runs on XCD b % 8). Give XCD x the
// logical ids x*per .. x*per+per-1 so that each XCD's L2 serves a contiguous band of the image and
// the halo rows neighbouring workgroups share stay in one L2. The last nblocks % 8 ids map to
// themselves, so the mapping is a bijection for every grid size.
__device__ inline int xcd_remap(int b, int nblocks) {
    constexpr int kXcd = 8;
    const int per = nblocks / kXcd;
    const int x = b % kXcd, local = b / kXcd;
    return local < per ? x * per + local : b;
}

// Images whose bin table fits the build's LDS tables (up to 4096 bins of 64 x 32 px, ~8.4 M pixels).
bool build_supported(int32_t w, int32_t h);
size_t build_ws_bytes(int64_t n, int32_t w, int32_t h);
BuildWs build_ws_carve(void *ws, int64_t n, int32_t w, int32_t h);
// stage_end (nullable) receives, in order, an event record after the count, scan, scatter and
// select kernels (kBuildStages events).
constexpr int kBuildStages = 4;
hipError_t launch_build(const afr_samples &s, const afr_deep_buffer &out, const BuildWs &ws,
                        unsigned long long *dropped, hipStream_t st, hipEvent_t *stage_end);

hipError_t launch_estimate(const afr_deep_buffer &buf, const afr_params &p, const afr_tile_stats &out,
                           hipStream_t st);

hipError_t launch_reconstruct_plain(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                    const afr_params &p, float *rgb, float *aux, hipStream_t st);
// tiles_per_group: launch shape of the tiled gather (1, 2 or 4 tiles, one wave each, per workgroup;
// R >= 3 takes at most 2); it does not change the result.
hipError_t launch_reconstruct_tiled(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                    const afr_params &p, int tiles_per_group, float *rgb,
                                    float *aux, hipStream_t st);
// Statistics and gather of each tile group in one launch (8 px tiles; other sizes run the two steps).
hipError_t launch_forward(const afr_deep_buffer &buf, const afr_params &p,
                          const afr_tile_stats &stats, int tiles_per_group, float *rgb, float *aux,
                          hipStream_t st);
// The library's default group for a radius (the largest the LDS allows).
int default_tiles_per_group(int radius);

size_t crosshair_ws_bytes(int64_t n, int32_t w, int32_t h);
hipError_t launch_crosshair_build(const afr_samples &s, const afr_crosshairs &xh,
                                  const afr_params &prm, const afr_deep_buffer &out, void *ws,
                                  unsigned long long *dropped_or_null, hipStream_t st);
hipError_t launch_crosshair_estimate(const afr_deep_buffer &buf, const afr_deep_buffer &xbuf,
                                     const afr_params &prm, const afr_tile_stats &out,
                                     hipStream_t st);

constexpr float kMaxSplat = 64.0f;  // largest splat edge the scatter form accepts, px
int splat_reach(float max_size);
hipError_t launch_splat_sizes(int32_t w, int32_t h, const float *coverage,
                              const afr_splat_params &sp, float *size, hipStream_t st);
hipError_t launch_scatter(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                          const afr_params &prm, const float *size, float max_size, float *rgb,
                          float *aux, float *coverage, hipStream_t st);

constexpr int kMaxSamplerTiles = 65536;  // keeps the selection's draw times total below 2^64
size_t sampler_ws_bytes(int32_t tiles);
hipError_t launch_sampler_stats(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                                const afr_params &prm, const afr_sampler_params &sp, float *E,
                                float *u, double *glob, void *ws, hipStream_t st);
hipError_t launch_sampler_tile_weights(int32_t w, int32_t h, int32_t tile, const float *E,
                                       const double *glob, int32_t n_parts, float *P, void *ws,
                                       hipStream_t st);
hipError_t launch_sampler_select(int32_t w, int32_t h, int32_t tile, const float *E, int64_t n,
                                 const uint32_t *rnd, float *x, float *y, int32_t *tile_out,
                                 void *ws, hipStream_t st);
// The same selection with its prefix in a library-owned device array (no workspace, no allocation).
hipError_t launch_sampler_select_noalloc(int32_t w, int32_t h, int32_t tile, const float *E,
                                         int64_t n, const uint32_t *rnd, float *x, float *y,
                                         int32_t *tile_out, hipStream_t st);

size_t rms_ws_bytes();
hipError_t launch_rms_loss(const float *img, const float *ref, int64_t n, double scale,
                           double *loss, float *grad, void *ws, hipStream_t st);

size_t backward_ws_bytes(int32_t w, int32_t h, int32_t k, int32_t radius);
hipError_t launch_backward(const afr_deep_buffer &buf, const afr_tile_stats &stats,
                           const afr_params &p, const float *rgb, const float *aux,
                           const float *grad_rgb, float *grad_slot, float *grad_params, void *ws,
                           hipStream_t st);

}  // namespace afr
