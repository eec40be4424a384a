// RMS error of a reconstructed image against a reference, and its gradient: the loss on which the
// filter parameters are fit (one term per frame), fused into three small kernels.
//
//   k_rms_part   a fixed grid of workgroups, each summing (img - ref)^2 over a grid-stride range in
//                FP64 and reducing in a fixed order: one partial per workgroup
//   k_rms_final  one workgroup: the partials in a fixed order, then scale * sqrt(sum / n)
//   k_rms_grad   per element: scale * (img - ref) / (n * rms), 0 when rms is 0
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

// out[0] = rms; loss (if not NULL) = scale * rms
__global__ __launch_bounds__(kLossThreads) void k_rms_final(const double *__restrict__ part, int nb,
                                                             int64_t n, double scale, double *out,
                                                             double *loss) {
    __shared__ double sh[kLossThreads / kWave];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kLossThreads) s += part[i];
    s = block_sum_d(s, sh);
    if (threadIdx.x == 0) {
        const double rms = n > 0 ? sqrt(s / (double)n) : 0.0;
        out[0] = rms;
        if (loss) loss[0] = scale * rms;
    }
}

__global__ __launch_bounds__(kLossThreads) void k_rms_grad(const float *__restrict__ img,
                                                            const float *__restrict__ ref, int64_t n,
                                                            double scale,
                                                            const double *__restrict__ out,
                                                            float *grad) {
    const int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
    if (i >= n) return;
    const double rms = out[0];
    const double d = (double)img[i] - (double)ref[i];
    grad[i] = rms > 0.0 ? (float)(scale * d / ((double)n * rms)) : 0.0f;
}

}  // namespace

size_t rms_ws_bytes() { return align_up(kLossBlocks * sizeof(double)) + align_up(sizeof(double)); }

hipError_t launch_rms_loss(const float *img, const float *ref, int64_t n, double scale,
                           double *loss, float *grad, void *ws, hipStream_t st) {
    double *part = static_cast<double *>(ws);
    double *out = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                             align_up(kLossBlocks * sizeof(double)));
    const int nb = (int)std::min<int64_t>(kLossBlocks, std::max<int64_t>(1, (n + kLossThreads - 1) /
                                                                                 kLossThreads));
    k_rms_part<<<nb, kLossThreads, 0, st>>>(img, ref, n, part);
    k_rms_final<<<1, kLossThreads, 0, st>>>(part, nb, n, scale, out, loss);
    if (grad && n > 0)
        k_rms_grad<<<(unsigned)((n + kLossThreads - 1) / kLossThreads), kLossThreads, 0, st>>>(
            img, ref, n, scale, out, grad);
    return hipGetLastError();
}

}  // namespace afr
