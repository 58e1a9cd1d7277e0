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
    kLayoutWsum = 5,        // per-row sum_j Delta_ij^-2 (the diagonal of L^w)
};

// Added to every squared distance before the reciprocal square root, so that
// a coincident pair (and the diagonal) gets a finite 1/d; its direction term
// c * (X_i - X_j) is then exactly zero because X_i - X_j is.  For squared
// distances above ~2e-23 the term is below half an ulp and changes nothing
// beyond the rounding of the sum itself.
constexpr float kMinSq = 1e-30f;

constexpr int kLayoutRowsPerWave = 4;
constexpr int kLayoutRowsPerBlock = 4 * kLayoutRowsPerWave;

// Work of one pair (i, j), accumulated into the row's running sums (see
// layout_rows for the formulas).
template <int MODE, bool INV>
__device__ __forceinline__ void layout_pair(float Dv, bool off, float2 xi, float2 xj, float& ax, float& ay,
                                            float& aw, float& as, float scale, float* gd_ij) {
    constexpr bool STEP = (MODE == kLayoutStep || MODE == kLayoutStepStress);
    constexpr bool STRESS = (MODE == kLayoutStepStress || MODE == kLayoutStress);
    constexpr bool GRAD = (MODE == kLayoutGradX || MODE == kLayoutGradBoth);
    constexpr bool WSUM = (MODE == kLayoutWsum);
    constexpr bool acc_w = WSUM || (STEP && !INV);
    const float inv = INV ? Dv : (off ? __builtin_amdgcn_rcpf(Dv) : 0.f);
    const float w = inv * inv;
    if (acc_w) aw += w;
    if (WSUM) return;
    const float dx = xi.x - xj.x;
    const float dy = xi.y - xj.y;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, kMinSq));
    const float rs = __builtin_amdgcn_rsqf(r2);
    if (STEP) {
        const float c = inv * rs;
        ax = fmaf(w, xj.x, fmaf(c, dx, ax));
        ay = fmaf(w, xj.y, fmaf(c, dy, ay));
    }
    if (STRESS || GRAD) {
        const float d = r2 * rs;
        const float t = fmaf(-d, inv, 1.0f);
        if (STRESS) as = off ? fmaf(t, t, as) : as;
        if (GRAD) {
            const float g = 2.0f * (d - Dv) * w * rs;
            ax = fmaf(g, dx, ax);
            ay = fmaf(g, dy, ay);
            if (MODE == kLayoutGradBoth) *gd_ij = off ? scale * 2.0f * t * d * w : 0.f;
        }
    }
}

// Pairwise work of 4 consecutive rows i (one wave) against all j of a
// k-node layout.  Lanes stride over j, so each row of Delta is read
// coalesced and each X_j load serves 4 rows.
//   step:   X+_i = (sum_j w X_j + c (X_i - X_j)) / sum_j w,
//           w = Delta^-2, c = w Delta / d = Delta^-1 d^-1  (Jacobi sweep of
//           L^w X = L^Y Y; a coincident pair adds only w X_j)
//   stress: sum_{j != i} (1 - d/Delta)^2, halved per unordered pair
//   grad:   dL/dX_i = sum_j 2 w (d - Delta) (X_i - X_j)/d,
//           dL/dDelta_ij = 2 (1 - d/Delta) d / Delta^2
// INV: `delta` holds 1/Delta with a zero diagonal (precomputed once for many
// sweeps) instead of Delta.  wsum: per-row sum_j w written by the kLayoutWsum
// pass (same summation order); a step with INV reads it from there, a step
// without INV accumulates it itself.
// Full groups of 4 rows take a branch-free path that issues the loads of 4
// columns (16 Delta values, 4 positions) before their arithmetic.
// Returns this wave's stress contribution (lane 0 holds the wave total).
template <int MODE, bool INV>
__device__ __forceinline__ double layout_rows(const float* __restrict__ delta, int64_t ld, int32_t k,
                                              const float2* __restrict__ x, int row_begin,
                                              float2* __restrict__ xout, float scale,
                                              float2* __restrict__ gx, float* __restrict__ gd,
                                              float* __restrict__ wsum) {
    constexpr int R = kLayoutRowsPerWave;
    constexpr bool STEP = (MODE == kLayoutStep || MODE == kLayoutStepStress);
    constexpr bool STRESS = (MODE == kLayoutStepStress || MODE == kLayoutStress);
    constexpr bool GRAD = (MODE == kLayoutGradX || MODE == kLayoutGradBoth);
    constexpr bool WSUM = (MODE == kLayoutWsum);
    static_assert(!(INV && GRAD), "the gradient needs Delta itself");
    const int lane = threadIdx.x & 63;
    float2 xi[R];
    bool ok[R];
    float ax[R], ay[R], aw[R], as[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = row_begin + r;
        ok[r] = i < k;
        xi[r] = ok[r] ? x[i] : make_float2(0.f, 0.f);
        ax[r] = ay[r] = aw[r] = as[r] = 0.f;
    }
    int j = lane;
    if (row_begin + R <= k) {
        const float* __restrict__ drow = delta + (int64_t)row_begin * ld;
        for (; j + 3 * kWave < k; j += 4 * kWave) {
            float2 xv[4];
            float dv[4][R];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[u] = x[j + u * kWave];
#pragma unroll
                for (int r = 0; r < R; ++r) dv[u][r] = drow[(int64_t)r * ld + j + u * kWave];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int jj = j + u * kWave;
                    layout_pair<MODE, INV>(dv[u][r], jj != row_begin + r, xi[r], xv[u], ax[r], ay[r], aw[r], as[r], scale,
                                           GRAD ? gd + (int64_t)(row_begin + r) * ld + jj : nullptr);
                }
            }
        }
    }
    for (; j < k; j += kWave) {
        const float2 xj = x[j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int i = row_begin + r;
            layout_pair<MODE, INV>(delta[(int64_t)i * ld + j], j != i, xi[r], xj, ax[r], ay[r], aw[r], as[r],
                                   scale, GRAD ? gd + (int64_t)i * ld + j : nullptr);
        }
    }
    double st = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;  // wave-uniform
        const int i = row_begin + r;
        if (WSUM) {
            const float sw = wave_sum(aw[r]);
            if (lane == 0) wsum[i] = sw;
        }
        if (STEP || GRAD) {
            const float sx = wave_sum(ax[r]);
            const float sy = wave_sum(ay[r]);
            if (STEP) {
                const float sw = INV ? wsum[i] : wave_sum(aw[r]);
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
    const double st = layout_rows<MODE, false>(delta, ld, k, x, row_begin, xout, scale, gx, gd, nullptr);
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
