// RMS error of a reconstructed image against a reference, and its gradient: the loss on which the
// filter parameters are fit (one term per frame), in two small kernels.
//
//   k_rms_part   a fixed grid of workgroups, each summing (img - ref)^2 over a grid-stride range in
//                FP64 and reducing in a fixed order: one partial per workgroup
//   k_rms_out    a fixed grid of workgroups, each adding the partials in the same fixed order (so
//                every workgroup holds the same rms = sqrt(sum / n)); workgroup 0 writes the loss,
//                scale * rms, and all of them the gradient scale * (img - ref) / (n * rms) over a
//                grid-stride range (0 when rms is 0)
// Every sum has a fixed order, so the loss and the gradient do not change from run to run.
#include <algorithm>

#include "afr_internal.h"

namespace afr {
namespace {

constexpr int kLossThreads = 256;
constexpr int kLossBlocks = 1024;

__device__ inline double block_sum_d(double v, double *sh) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kLossThreads / kWave; ++i) t += sh[i];
    return t;
}

__global__ __launch_bounds__(kLossThreads) void k_rms_part(const float *__restrict__ img,
                                                            const float *__restrict__ ref, int64_t n,
                                                            double *part) {
    __shared__ double sh[kLossThreads / kWave];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kLossThreads;
    for (int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; i < n; i += stride) {
        const double d = (double)img[i] - (double)ref[i];
        s += d * d;
    }
    s = block_sum_d(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// loss (if not NULL) = scale * rms; grad (if not NULL) per element
__global__ __launch_bounds__(kLossThreads) void k_rms_out(const double *__restrict__ part, int nb,
                                                           const float *__restrict__ img,
                                                           const float *__restrict__ ref, int64_t n,
                                                           double scale, double *loss,
                                                           float *grad) {
    __shared__ double sh[kLossThreads / kWave];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kLossThreads) s += part[i];
    s = block_sum_d(s, sh);
    const double rms = n > 0 ? sqrt(s / (double)n) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) loss[0] = scale * rms;
    if (!grad) return;
    const int64_t stride = (int64_t)gridDim.x * kLossThreads;
    for (int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; i < n; i += stride) {
        const double d = (double)img[i] - (double)ref[i];
        grad[i] = rms > 0.0 ? (float)(scale * d / ((double)n * rms)) : 0.0f;
    }
}

}  // namespace

size_t rms_ws_bytes() { return align_up(kLossBlocks * sizeof(double)); }

hipError_t launch_rms_loss(const float *img, const float *ref, int64_t n, double scale,
                           double *loss, float *grad, void *ws, hipStream_t st) {
    double *part = static_cast<double *>(ws);
    const int64_t blocks = std::max<int64_t>(1, (n + kLossThreads - 1) / kLossThreads);
    const int nb = (int)std::min<int64_t>(kLossBlocks, blocks);
    k_rms_part<<<nb, kLossThreads, 0, st>>>(img, ref, n, part);
    const int ng = grad ? (int)std::min<int64_t>(kLossBlocks, blocks) : 1;
    k_rms_out<<<ng, kLossThreads, 0, st>>>(part, nb, img, ref, n, scale, loss, grad);
    return hipGetLastError();
}

}  // namespace afr
