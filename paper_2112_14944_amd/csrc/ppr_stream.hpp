// Power iteration for graphs too large for the LDS-resident tile kernel: the
// node-major iterate lives in HBM (ping-pong buffers) and each push is one
// launch.  A wave owns one row per pass and its 64 lanes are 64 consecutive
// source columns, so every gathered neighbour row is one contiguous 256-byte
// read and the arc list is wave-uniform (scalar loads).
//
// The same step serves the adjoint solve of the weight gradient:
//     A_{k+1} = Gb + (1-alpha) P^T A_k      (Gb = D G, forcing term)
// which gathers over the same neighbours with the same coefficients.
#pragma once

#include "common.hpp"

namespace pprviz {

inline int64_t stream_ld(int64_t ncols) { return (ncols + 63) / 64 * 64; }
constexpr int kStreamResidRows = 4096;
inline int64_t stream_resid_chunks(int64_t n) { return (n + kStreamResidRows - 1) / kStreamResidRows; }

struct StreamArgs {
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const float* weight;
    const float* invd;
    const float* deg;
    int32_t n;
    int32_t ncols;        // valid columns (sources / adjoint right-hand sides)
    int64_t ld;           // leading dimension of the iterate (multiple of 64)
    float alpha;
    const int32_t* src;   // forward: source node of column s (nullptr: column s = node s)
    const float* forcing; // adjoint: G [n][ld_forcing] (Gb = deg[v] * G[v][s]); nullptr = forward
    int64_t ld_forcing;
};

constexpr int kStreamRowsPerWave = 4;
constexpr int kStreamRowsPerBlock = 4 * kStreamRowsPerWave;

// MODE 0: forward (forcing alpha at the source row); MODE 1: adjoint.
template <int MODE, bool WEIGHTED, bool FINAL>
__global__ __launch_bounds__(256) void stream_step_kernel(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ weight, const float* __restrict__ invd, const float* __restrict__ deg,
    const int32_t* __restrict__ src, const float* __restrict__ forcing, int64_t ld_forcing, int32_t n,
    int32_t ncols, int64_t ld, float alpha, const float* __restrict__ yin, float* __restrict__ yout) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.y * 64 + lane;
    const bool valid = col < ncols;
    int my_src = -1;
    if (MODE == 0 && valid) my_src = src ? src[col] : (int)col;
    const float oma = 1.0f - alpha;
    const int v0 = blockIdx.x * kStreamRowsPerBlock + wave * kStreamRowsPerWave;
    for (int r = 0; r < kStreamRowsPerWave; ++r) {
        const int v = __builtin_amdgcn_readfirstlane(v0 + r);
        if (v >= n) return;
        const int rs = row_ptr[v];
        const int re = row_ptr[v + 1];
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        if (rs == re) a0 = yin[(int64_t)v * ld + col];
        int e = rs;
        for (; e + 8 <= re; e += 8) {
            const int64_t u0 = col_idx[e + 0], u1 = col_idx[e + 1], u2 = col_idx[e + 2], u3 = col_idx[e + 3];
            const int64_t u4 = col_idx[e + 4], u5 = col_idx[e + 5], u6 = col_idx[e + 6], u7 = col_idx[e + 7];
            const float y0 = yin[u0 * ld + col], y1 = yin[u1 * ld + col], y2 = yin[u2 * ld + col],
                        y3 = yin[u3 * ld + col];
            const float y4 = yin[u4 * ld + col], y5 = yin[u5 * ld + col], y6 = yin[u6 * ld + col],
                        y7 = yin[u7 * ld + col];
            if (WEIGHTED) {
                a0 = fmaf(weight[e + 0], y0, a0);
                a1 = fmaf(weight[e + 1], y1, a1);
                a2 = fmaf(weight[e + 2], y2, a2);
                a3 = fmaf(weight[e + 3], y3, a3);
                a0 = fmaf(weight[e + 4], y4, a0);
                a1 = fmaf(weight[e + 5], y5, a1);
                a2 = fmaf(weight[e + 6], y6, a2);
                a3 = fmaf(weight[e + 7], y7, a3);
            } else {
                a0 += y0;
                a1 += y1;
                a2 += y2;
                a3 += y3;
                a0 += y4;
                a1 += y5;
                a2 += y6;
                a3 += y7;
            }
        }
        for (; e < re; ++e) {
            const int64_t u = col_idx[e];
            const float y = yin[u * ld + col];
            if (WEIGHTED) a0 = fmaf(weight[e], y, a0); else a0 += y;
        }
        float x = (a0 + a1) + (a2 + a3);
        if (MODE == 0) {
            x += (v == my_src) ? alpha : 0.0f;
        } else {
            x += valid ? deg[v] * forcing[(int64_t)v * ld_forcing + col] : 0.0f;
        }
        yout[(int64_t)v * ld + col] = FINAL ? x : x * oma * invd[v];
    }
}

// Y_0 for the forward iteration: zero everywhere but the source rows.
static __global__ void stream_init_forward_kernel(const int32_t* __restrict__ src, const float* __restrict__ invd,
                                           int32_t ncols, int64_t ld, float alpha, int final_,
                                           float* __restrict__ y) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ncols) return;
    int v = src ? src[s] : s;
    y[(int64_t)v * ld + s] = final_ ? alpha : alpha * (1.0f - alpha) * invd[v];
}

// Y_0 = (1-alpha)/d * Gb for the adjoint (Gb = d * G), or Gb itself when final.
static __global__ void stream_init_adjoint_kernel(const float* __restrict__ forcing, int64_t ld_forcing,
                                           const float* __restrict__ deg, const float* __restrict__ invd,
                                           int32_t n, int32_t ncols, int64_t ld, float alpha, int final_,
                                           float* __restrict__ y) {
    const int64_t col = (int64_t)blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;
    float g = col < ncols ? deg[v] * forcing[v * ld_forcing + col] : 0.0f;
    y[v * ld + col] = final_ ? g : g * (1.0f - alpha) * invd[v];
}

// out[s][j] = X[tgt[j]][s] (and d(src_s) times it), 64x64 tiles through LDS.
static __global__ __launch_bounds__(256) void stream_transpose_kernel(
    const float* __restrict__ x, int64_t ld, int32_t ncols, const int32_t* __restrict__ src,
    const int32_t* __restrict__ tgt, int32_t n_tgt, const float* __restrict__ deg,
    float* __restrict__ ppr_out, float* __restrict__ dppr_out, int64_t ld_out) {
    __shared__ float tile[64][65];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int64_t s0 = (int64_t)blockIdx.y * 64;
    for (int jj = w; jj < 64; jj += 4) {
        const int64_t j = j0 + jj;
        float val = 0.f;
        if (j < n_tgt) {
            const int64_t tn = tgt ? tgt[j] : j;
            val = x[tn * ld + s0 + lane];
        }
        tile[jj][lane] = val;
    }
    __syncthreads();
    for (int ss = w; ss < 64; ss += 4) {
        const int64_t s = s0 + ss;
        if (s >= ncols) break;
        const int64_t j = j0 + lane;
        if (j >= n_tgt) continue;
        const float val = tile[lane][ss];
        if (ppr_out) ppr_out[s * ld_out + j] = val;
        if (dppr_out) {
            const int sn = src ? src[s] : (int)s;
            dppr_out[s * ld_out + j] = val * deg[sn];
        }
    }
}

// Column sums of X over row chunks in FP64 (first pass of the residual).
static __global__ __launch_bounds__(256) void stream_colsum_kernel(const float* __restrict__ x, int32_t n, int64_t ld,
                                                            double* __restrict__ part) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.y * 64 + lane;
    const int64_t r0 = (int64_t)blockIdx.x * kStreamResidRows;
    const int64_t r1 = min((int64_t)n, r0 + kStreamResidRows);
    double s = 0.0;
    for (int64_t r = r0 + w; r < r1; r += 4) s += (double)x[r * ld + col];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0) part[(int64_t)blockIdx.x * ld + col] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

static __global__ void stream_resid_kernel(const double* __restrict__ part, int64_t chunks, int64_t ld, int32_t ncols,
                                    double* __restrict__ resid) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ncols) return;
    double t = 0.0;
    for (int64_t c = 0; c < chunks; ++c) t += part[c * ld + s];
    resid[s] = 1.0 - t;
}

template <int MODE, bool FINAL>
inline void stream_launch_step(const StreamArgs& a, const float* yin, float* yout, hipStream_t s) {
    dim3 grid((unsigned)((a.n + kStreamRowsPerBlock - 1) / kStreamRowsPerBlock), (unsigned)(a.ld / 64));
    if (a.weight)
        hipLaunchKernelGGL((stream_step_kernel<MODE, true, FINAL>), grid, dim3(256), 0, s, a.row_ptr, a.col_idx,
                           a.weight, a.invd, a.deg, a.src, a.forcing, a.ld_forcing, a.n, a.ncols, a.ld, a.alpha,
                           yin, yout);
    else
        hipLaunchKernelGGL((stream_step_kernel<MODE, false, FINAL>), grid, dim3(256), 0, s, a.row_ptr, a.col_idx,
                           a.weight, a.invd, a.deg, a.src, a.forcing, a.ld_forcing, a.n, a.ncols, a.ld, a.alpha,
                           yin, yout);
}

// T pushes (forward, a.forcing == nullptr) or T adjoint terms; returns the
// buffer that holds the final unscaled iterate.
inline const float* stream_power_iteration(const StreamArgs& a, int T, float* ya, float* yb, hipStream_t s) {
    const int64_t total = (int64_t)a.n * a.ld;
    const bool adj = a.forcing != nullptr;
    fill<float>(ya, 0.0f, total, s);
    if (T <= 0) return ya;
    if (adj) {
        dim3 grid((unsigned)((a.n + 3) / 4), (unsigned)(a.ld / 64));
        hipLaunchKernelGGL(stream_init_adjoint_kernel, grid, dim3(256), 0, s, a.forcing, a.ld_forcing, a.deg,
                           a.invd, a.n, a.ncols, a.ld, a.alpha, T == 1 ? 1 : 0, ya);
    } else {
        hipLaunchKernelGGL(stream_init_forward_kernel, dim3((a.ncols + 255) / 256), dim3(256), 0, s, a.src,
                           a.invd, a.ncols, a.ld, a.alpha, T == 1 ? 1 : 0, ya);
    }
    float* in = ya;
    float* out = yb;
    for (int it = 1; it < T; ++it) {
        const bool fin = (it == T - 1);
        if (adj) {
            if (fin) stream_launch_step<1, true>(a, in, out, s); else stream_launch_step<1, false>(a, in, out, s);
        } else {
            if (fin) stream_launch_step<0, true>(a, in, out, s); else stream_launch_step<0, false>(a, in, out, s);
        }
        float* t = in;
        in = out;
        out = t;
    }
    return in;
}

inline void stream_write_outputs(const float* x, const StreamArgs& a, const int32_t* tgt, int32_t n_tgt,
                                 float* ppr_out, float* dppr_out, hipStream_t s) {
    if (!ppr_out && !dppr_out) return;
    dim3 grid((unsigned)((n_tgt + 63) / 64), (unsigned)((a.ncols + 63) / 64));
    hipLaunchKernelGGL(stream_transpose_kernel, grid, dim3(256), 0, s, x, a.ld, a.ncols, a.src, tgt, n_tgt, a.deg,
                       ppr_out, dppr_out, (int64_t)n_tgt);
}

inline void stream_residuals(const float* x, const StreamArgs& a, double* part, double* resid, hipStream_t s) {
    const int64_t chunks = stream_resid_chunks(a.n);
    dim3 grid((unsigned)chunks, (unsigned)(a.ld / 64));
    hipLaunchKernelGGL(stream_colsum_kernel, grid, dim3(256), 0, s, x, a.n, a.ld, part);
    hipLaunchKernelGGL(stream_resid_kernel, dim3((a.ncols + 255) / 256), dim3(256), 0, s, part, chunks, a.ld,
                       a.ncols, resid);
}

}  // namespace pprviz
