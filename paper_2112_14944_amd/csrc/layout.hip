// PDist (Eq. eq:pprdist), its backward, and the O(k^2) stress layout kernels
// (Eq. eq:loss; the appendix's stress majorization in Jacobi form).
#include <math.h>

#include "layout_core.hpp"

namespace pprviz {

// Delta from a k x k DPPR block, 64x64 output tiles.  The transposed tile is
// staged through LDS so both reads are coalesced.  z_ij and z_ji are the same
// FP32 sum (addition commutes), so the result is exactly symmetric.
__global__ __launch_bounds__(256) void pdist_kernel(const float* __restrict__ pid, int32_t k, int64_t n_clamp,
                                                    float* __restrict__ delta) {
    const float hi = pdist_hi(n_clamp);
    __shared__ float tt[64][65];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.y * 64;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    // tt[jj][ii] = pid[j0+jj][i0+ii]
    for (int jj = w; jj < 64; jj += 4) {
        const int64_t j = j0 + jj, i = i0 + lane;
        tt[jj][lane] = (j < k && i < k) ? pid[j * k + i] : 0.f;
    }
    __syncthreads();
    for (int ii = w; ii < 64; ii += 4) {
        const int64_t i = i0 + ii, j = j0 + lane;
        if (i >= k || j >= k) continue;
        const float z = pid[i * k + j] + tt[lane][ii];
        delta[i * k + j] = (i == j) ? 0.f : pdist_value(z, hi);
    }
}

__global__ __launch_bounds__(256) void pdist_backward_kernel(const float* __restrict__ pid,
                                                             const float* __restrict__ gdelta, int32_t k,
                                                             int64_t n_clamp, float* __restrict__ gpid) {
    const float hi = pdist_hi(n_clamp);
    __shared__ float tt[64][65];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.y * 64;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    for (int jj = w; jj < 64; jj += 4) {
        const int64_t j = j0 + jj, i = i0 + lane;
        tt[jj][lane] = (j < k && i < k) ? pid[j * k + i] : 0.f;
    }
    __syncthreads();
    for (int ii = w; ii < 64; ii += 4) {
        const int64_t i = i0 + ii, j = j0 + lane;
        if (i >= k || j >= k) continue;
        const float z = pid[i * k + j] + tt[lane][ii];
        gpid[i * k + j] = (i == j) ? 0.f : gdelta[i * k + j] * pdist_dz(z, hi);
    }
}

template <int MODE>
static void launch_layout(const float* delta, int32_t k, const float* x, float* xout, double* part, float scale,
                          float* gx, float* gd, hipStream_t s) {
    const unsigned blocks = (unsigned)((k + kLayoutRowsPerBlock - 1) / kLayoutRowsPerBlock);
    hipLaunchKernelGGL((layout_rows_kernel<MODE>), dim3(blocks), dim3(256), 0, s, delta, (int64_t)k, k,
                       reinterpret_cast<const float2*>(x), reinterpret_cast<float2*>(xout), part, scale,
                       reinterpret_cast<float2*>(gx), gd);
}

static unsigned layout_blocks(int32_t k) {
    return (unsigned)((k + kLayoutRowsPerBlock - 1) / kLayoutRowsPerBlock);
}

}  // namespace pprviz

using namespace pprviz;

extern "C" {

ppr_status pdist(const float* dppr, int32_t k, int64_t n_clamp, float* delta, void* stream) {
    if (dppr == nullptr || delta == nullptr || k < 1 || n_clamp < 1 || dppr == delta) return PPR_EINVAL;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    dim3 grid((k + 63) / 64, (k + 63) / 64);
    hipLaunchKernelGGL(pdist_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream), dppr, k, n_clamp, delta);
    return launch_status();
}

ppr_status pdist_backward(const float* dppr, const float* grad_delta, int32_t k, int64_t n_clamp,
                          float* grad_dppr, void* stream) {
    if (!dppr || !grad_delta || !grad_dppr || k < 1 || n_clamp < 1) return PPR_EINVAL;
    if (grad_dppr == dppr || grad_dppr == grad_delta) return PPR_EINVAL;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    dim3 grid((k + 63) / 64, (k + 63) / 64);
    hipLaunchKernelGGL(pdist_backward_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream), dppr,
                       grad_delta, k, n_clamp, grad_dppr);
    return launch_status();
}

size_t layout_workspace(int32_t k) {
    if (k < 1) return 0;
    return align_up(sizeof(double) * (size_t)layout_blocks(k));
}

ppr_status stress_eval(const float* delta, int32_t k, const float* x, double* stress_out, void* ws,
                       size_t ws_bytes, void* stream) {
    if (!delta || !x || !stress_out || k < 1) return PPR_EINVAL;
    if (ws == nullptr || ws_bytes < layout_workspace(k)) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(ws);
    launch_layout<kLayoutStress>(delta, k, x, nullptr, part, 1.f, nullptr, nullptr, s);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, part, (int64_t)layout_blocks(k), stress_out);
    return launch_status();
}

ppr_status layout_step(const float* delta, int32_t k, const float* x_in, float* x_out, double* stress_out,
                       void* ws, size_t ws_bytes, void* stream) {
    if (!delta || !x_in || !x_out || k < 1 || x_in == x_out) return PPR_EINVAL;
    if (stress_out && (ws == nullptr || ws_bytes < layout_workspace(k))) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(ws);
    if (stress_out) {
        launch_layout<kLayoutStepStress>(delta, k, x_in, x_out, part, 1.f, nullptr, nullptr, s);
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, part, (int64_t)layout_blocks(k),
                           stress_out);
    } else {
        launch_layout<kLayoutStep>(delta, k, x_in, x_out, nullptr, 1.f, nullptr, nullptr, s);
    }
    return launch_status();
}

ppr_status stress_backward(const float* delta, int32_t k, const float* x, float grad_scale, float* grad_x,
                           float* grad_delta, void* stream) {
    if (!delta || !x || k < 1 || (!grad_x && !grad_delta)) return PPR_EINVAL;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (grad_delta)
        launch_layout<kLayoutGradBoth>(delta, k, x, nullptr, nullptr, grad_scale, grad_x, grad_delta, s);
    else
        launch_layout<kLayoutGradX>(delta, k, x, nullptr, nullptr, grad_scale, grad_x, nullptr, s);
    return launch_status();
}

}  // extern "C"
