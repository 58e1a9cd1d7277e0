// Device-side PDist formula and the pairwise layout / stress / gradient row
// kernels, shared by the single-layout entry points and the batched path.
#pragma once

#include "common.hpp"

namespace pprviz {

// Upper clamp 2 ln n of Eq. eq:pprdist, evaluated in FP64 and rounded once.
__device__ __forceinline__ float pdist_hi(int64_t n_clamp) { return (float)(2.0 * log((double)n_clamp)); }

// Eq. eq:pprdist: min(max(1 - ln z, 2), 2 ln n); an unreachable pair (z <= 0)
// takes the upper bound.  NaN stays NaN.
__device__ __forceinline__ float pdist_value(float z, float hi) {
    if (z != z) return z;
    if (!(z > 0.f)) return hi;
    const float raw = 1.0f - logf(z);
    return fminf(fmaxf(raw, 2.0f), hi);
}

// dDelta/dz: -1/z strictly inside the clamp range, 0 on or beyond the kinks.
__device__ __forceinline__ float pdist_dz(float z, float hi) {
    if (!(z > 0.f)) return 0.f;
    const float raw = 1.0f - logf(z);
    return (raw > 2.0f && raw < hi) ? -1.0f / z : 0.0f;
}

enum {
    kLayoutStep = 0,        // x_out only
    kLayoutStepStress = 1,  // x_out and stress partials of x_in
    kLayoutStress = 2,      // stress partials only
    kLayoutGradX = 3,       // dL/dX
    kLayoutGradBoth = 4,    // dL/dX (optional) and dL/dDelta
};

constexpr int kLayoutRowsPerWave = 4;
constexpr int kLayoutRowsPerBlock = 4 * kLayoutRowsPerWave;

// Pairwise work of 4 consecutive rows i (one wave) against all j of a
// k-node layout.  Lanes stride over j, so each row of Delta is read
// coalesced and each X_j load serves 4 rows.
//   step:   X+_i = (sum_j w X_j + c (X_i - X_j)) / sum_j w,
//           w = Delta^-2, c = w Delta / d = Delta^-1 d^-1  (Jacobi sweep of
//           L^w X = L^Y Y; a coincident pair has d = 0 and adds only w X_j)
//   stress: sum_{j != i} (1 - d/Delta)^2, halved per unordered pair
//   grad:   dL/dX_i = sum_j 2 w (d - Delta) (X_i - X_j)/d,
//           dL/dDelta_ij = 2 (1 - d/Delta) d / Delta^2
// Returns this wave's stress contribution (lane 0 holds the wave total).
template <int MODE>
__device__ __forceinline__ double layout_rows(const float* __restrict__ delta, int64_t ld, int32_t k,
                                              const float2* __restrict__ x, int row_begin,
                                              float2* __restrict__ xout, float scale,
                                              float2* __restrict__ gx, float* __restrict__ gd) {
    constexpr bool STEP = (MODE == kLayoutStep || MODE == kLayoutStepStress);
    constexpr bool STRESS = (MODE == kLayoutStepStress || MODE == kLayoutStress);
    constexpr bool GRAD = (MODE == kLayoutGradX || MODE == kLayoutGradBoth);
    const int lane = threadIdx.x & 63;
    float2 xi[kLayoutRowsPerWave];
    bool ok[kLayoutRowsPerWave];
    float ax[kLayoutRowsPerWave], ay[kLayoutRowsPerWave], aw[kLayoutRowsPerWave], as[kLayoutRowsPerWave];
#pragma unroll
    for (int r = 0; r < kLayoutRowsPerWave; ++r) {
        const int i = row_begin + r;
        ok[r] = i < k;
        xi[r] = ok[r] ? x[i] : make_float2(0.f, 0.f);
        ax[r] = ay[r] = aw[r] = as[r] = 0.f;
    }
    for (int j = lane; j < k; j += kWave) {
        const float2 xj = x[j];
#pragma unroll
        for (int r = 0; r < kLayoutRowsPerWave; ++r) {
            if (!ok[r]) continue;
            const int i = row_begin + r;
            const float D = delta[(int64_t)i * ld + j];
            const bool off = (j != i);
            const float dx = xi[r].x - xj.x;
            const float dy = xi[r].y - xj.y;
            const float r2 = fmaf(dx, dx, dy * dy);
            const float rs = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
            const float inv = off ? __builtin_amdgcn_rcpf(D) : 0.f;
            const float w = inv * inv;
            if (STEP) {
                const float c = inv * rs;
                ax[r] = fmaf(w, xj.x, fmaf(c, dx, ax[r]));
                ay[r] = fmaf(w, xj.y, fmaf(c, dy, ay[r]));
                aw[r] += w;
            }
            if (STRESS || GRAD) {
                const float d = r2 * rs;
                const float t = fmaf(-d, inv, 1.0f);
                if (STRESS) as[r] = off ? fmaf(t, t, as[r]) : as[r];
                if (GRAD) {
                    const float g = 2.0f * (d - D) * w * rs;
                    ax[r] = fmaf(g, dx, ax[r]);
                    ay[r] = fmaf(g, dy, ay[r]);
                    if (MODE == kLayoutGradBoth) gd[(int64_t)i * ld + j] = off ? scale * 2.0f * t * d * w : 0.f;
                }
            }
        }
    }
    double st = 0.0;
#pragma unroll
    for (int r = 0; r < kLayoutRowsPerWave; ++r) {
        if (!ok[r]) continue;  // wave-uniform
        const int i = row_begin + r;
        if (STEP || GRAD) {
            const float sx = wave_sum(ax[r]);
            const float sy = wave_sum(ay[r]);
            if (STEP) {
                const float sw = wave_sum(aw[r]);
                if (lane == 0) xout[i] = sw > 0.f ? make_float2(sx / sw, sy / sw) : xi[r];
            } else if (gx && lane == 0) {
                gx[i] = make_float2(scale * sx, scale * sy);
            }
        }
        if (STRESS) st += wave_sum((double)as[r]);
    }
    return 0.5 * st;
}

// One block = 16 rows (4 waves x 4 rows) of one k-node layout.
template <int MODE>
__global__ __launch_bounds__(256) void layout_rows_kernel(const float* __restrict__ delta, int64_t ld, int32_t k,
                                                          const float2* __restrict__ x, float2* __restrict__ xout,
                                                          double* __restrict__ part, float scale,
                                                          float2* __restrict__ gx, float* __restrict__ gd) {
    __shared__ double red[4];
    const int wave = threadIdx.x >> 6;
    const int row_begin = blockIdx.x * kLayoutRowsPerBlock + wave * kLayoutRowsPerWave;
    const double st = layout_rows<MODE>(delta, ld, k, x, row_begin, xout, scale, gx, gd);
    if (MODE == kLayoutStepStress || MODE == kLayoutStress) {
        if ((threadIdx.x & 63) == 0) red[wave] = st;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// out[0] = sum of part[0..m) in a fixed order (single block).
static __global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ part, int64_t m,
                                                           double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace pprviz
