// Exact stress-majorization step (the appendix's Guttman transform):
//     L^w X+ = L^Y(Y) Y,   X+ = (L^w)^+ L^Y(Y) Y,
// with L^w_ij = -Delta_ij^-2 and L^Y_ij = -1 / (Delta_ij ||Y_i - Y_j||) off the
// diagonal (0 for a coincident pair) and the negated row sums on it.  L^w is
// singular (L^w 1 = 0); the right-hand side sums to zero, and conjugate
// gradients started from the centred Y stay in the centred subspace, so they
// converge to the pseudo-inverse solution, the minimiser with zero centroid.
//
// The x and y coordinates are two independent systems with the same matrix;
// they run side by side with their own CG scalars.  Per iteration:
//   apply:      Ap_i = sum_j w_ij (p_i - p_j), and p . Ap, one pass over Delta
//   update:     alpha = r.r / p.Ap;  x += alpha p;  r -= alpha Ap;  r.r
//   direction:  beta = r.r(new) / r.r(old);  p = r + beta p;  stop test
// Every dot product is summed in FP64 from per-block partials in a fixed
// order, so the iterates do not depend on scheduling.  The host launches the
// iterations in batches (8, then doubling) and reads the stop flag after each;
// kernels launched after the flag is set return at once.  The apply is the
// pairwise row sweep of the Jacobi step (4 rows per wave, lanes striding
// over j, 4 columns of loads in flight); it reads Delta once, 4 k^2 bytes.
#include <math.h>

#include <algorithm>

#include "layout_core.hpp"
#include "ppr_core.hpp"

namespace pprviz {

namespace {

enum { kCgRhs = 0, kCgApply = 1 };
constexpr int kCgRows = kLayoutRowsPerBlock;  // rows per block of the pairwise kernels
constexpr int kCgVec = 256;                   // entries per block of the vector kernels

struct CgState {
    double mean[2];
    double bb[2];      // |b|^2 per coordinate
    double rr[2][2];   // |r|^2 per coordinate, by iteration parity
    int32_t done;
    int32_t iters;
};

struct CgWs {
    CgState* st;
    float2* r;
    float2* p;
    float2* ap;
    double* part_rows;  // [row blocks][4]
    double* part_vec;   // [vector blocks][2]
};

inline int64_t cg_row_blocks(int32_t k) { return (k + kCgRows - 1) / kCgRows; }
inline int64_t cg_vec_blocks(int32_t k) { return (k + kCgVec - 1) / kCgVec; }

template <typename Cursor>
void cg_ws_layout(Cursor& c, int32_t k, CgWs* w) {
    CgWs t{};
    t.st = c.template take<CgState>(1);
    t.r = c.template take<float2>((size_t)k);
    t.p = c.template take<float2>((size_t)k);
    t.ap = c.template take<float2>((size_t)k);
    t.part_rows = c.template take<double>((size_t)cg_row_blocks(k) * 4);
    t.part_vec = c.template take<double>((size_t)cg_vec_blocks(k) * 2);
    if (w) *w = t;
}

// Sum of part[0 .. m) with stride `stride` starting at `off`, by one block in
// a fixed order (strided per thread, then a tree); every thread gets it.
__device__ double block_sum(const double* __restrict__ part, int64_t m, int stride, int off) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) s += part[i * stride + off];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// Mean of the positions (one block, FP64).
__global__ __launch_bounds__(256) void cg_mean_kernel(const float2* __restrict__ x, int32_t k,
                                                      CgState* __restrict__ st) {
    __shared__ double rx[256], ry[256];
    double sx = 0.0, sy = 0.0;
    for (int i = threadIdx.x; i < k; i += 256) {
        sx += (double)x[i].x;
        sy += (double)x[i].y;
    }
    rx[threadIdx.x] = sx;
    ry[threadIdx.x] = sy;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rx[threadIdx.x] += rx[threadIdx.x + o];
            ry[threadIdx.x] += ry[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->mean[0] = rx[0] / k;
        st->mean[1] = ry[0] / k;
        st->done = 0;
        st->iters = 0;
    }
}

// x0 = Y - mean(Y), the warm start.
__global__ void cg_center_kernel(const float2* __restrict__ y, int32_t k, const CgState* __restrict__ st,
                                 float2* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    x[i] = make_float2((float)((double)y[i].x - st->mean[0]), (float)((double)y[i].y - st->mean[1]));
}

// Pairwise pass of 16 rows per block.
//  kCgRhs (x = Y):   b_i = sum_j c_ij (Y_i - Y_j), c = 1/(Delta d) (0 when
//                    coincident), and r_i = b_i - sum_j w_ij (Y_i - Y_j), which
//                    is b - L^w x0 because L^w annihilates the mean; writes
//                    r and p = r; partials |b|^2, |r|^2 per coordinate.
//  kCgApply (x = p): Ap_i = sum_j w_ij (p_i - p_j); partials p . Ap.
template <int MODE>
__global__ __launch_bounds__(256) void cg_rows_kernel(const float* __restrict__ delta, int32_t k,
                                                      const float2* __restrict__ x, float2* __restrict__ out_a,
                                                      float2* __restrict__ out_b, double* __restrict__ part,
                                                      const CgState* __restrict__ st) {
    if (st->done) return;
    constexpr int R = kLayoutRowsPerWave;
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row_begin = blockIdx.x * kCgRows + wave * R;
    float2 xi[R];
    bool ok[R];
    float bx[R], by[R], lx[R], ly[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = row_begin + r;
        ok[r] = i < k;
        xi[r] = ok[r] ? x[i] : make_float2(0.f, 0.f);
        bx[r] = by[r] = lx[r] = ly[r] = 0.f;
    }
    auto pair = [&](int r, float Dv, bool off, float2 xj) {
        const float inv = off ? __builtin_amdgcn_rcpf(Dv) : 0.f;
        const float w = inv * inv;
        const float dx = xi[r].x - xj.x;
        const float dy = xi[r].y - xj.y;
        lx[r] = fmaf(w, dx, lx[r]);
        ly[r] = fmaf(w, dy, ly[r]);
        if (MODE == kCgRhs) {
            const float rs = __builtin_amdgcn_rsqf(fmaf(dx, dx, fmaf(dy, dy, kMinSq)));
            const float c = inv * rs;
            bx[r] = fmaf(c, dx, bx[r]);
            by[r] = fmaf(c, dy, by[r]);
        }
    };
    int j = lane;
    if (row_begin + R <= k) {
        const float* __restrict__ drow = delta + (int64_t)row_begin * k;
        for (; j + 3 * kWave < k; j += 4 * kWave) {
            float2 xv[4];
            float dv[4][R];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[u] = x[j + u * kWave];
#pragma unroll
                for (int r = 0; r < R; ++r) dv[u][r] = drow[(int64_t)r * k + j + u * kWave];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int r = 0; r < R; ++r) pair(r, dv[u][r], j + u * kWave != row_begin + r, xv[u]);
        }
    }
    for (; j < k; j += kWave) {
        const float2 xj = x[j];
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (ok[r]) pair(r, delta[(int64_t)(row_begin + r) * k + j], j != row_begin + r, xj);
    }
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;  // wave-uniform
        const int i = row_begin + r;
        const float sx = wave_sum(lx[r]);
        const float sy = wave_sum(ly[r]);
        if (MODE == kCgRhs) {
            const float tx = wave_sum(bx[r]);
            const float ty = wave_sum(by[r]);
            const float2 rv = make_float2(tx - sx, ty - sy);
            if (lane == 0) {
                out_a[i] = rv;
                out_b[i] = rv;
            }
            d0 += (double)tx * tx;
            d1 += (double)ty * ty;
            d2 += (double)rv.x * rv.x;
            d3 += (double)rv.y * rv.y;
        } else {
            if (lane == 0) out_a[i] = make_float2(sx, sy);
            d0 += (double)xi[r].x * sx;
            d1 += (double)xi[r].y * sy;
        }
    }
    if (lane == 0) {
        red[wave][0] = d0;
        red[wave][1] = d1;
        red[wave][2] = d2;
        red[wave][3] = d3;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        part[(int64_t)blockIdx.x * 4 + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    }
}

// After the right-hand side: |b|^2 and |r|^2 into the state (one block); the
// rounds stop at once when both residuals already meet the tolerance.
__global__ __launch_bounds__(256) void cg_init_kernel(const double* __restrict__ part, int64_t blocks, double tol2,
                                                      CgState* __restrict__ st) {
    const double b0 = block_sum(part, blocks, 4, 0);
    const double b1 = block_sum(part, blocks, 4, 1);
    const double r0 = block_sum(part, blocks, 4, 2);
    const double r1 = block_sum(part, blocks, 4, 3);
    if (threadIdx.x == 0) {
        st->bb[0] = b0;
        st->bb[1] = b1;
        st->rr[0][0] = r0;
        st->rr[0][1] = r1;
        st->done = (r0 <= tol2 * b0 && r1 <= tol2 * b1) ? 1 : 0;
    }
}

// x += alpha p, r -= alpha Ap for this block's entries; partial |r|^2.
__global__ __launch_bounds__(256) void cg_update_kernel(int32_t k, int32_t it, const double* __restrict__ part_rows,
                                                        int64_t row_blocks, const float2* __restrict__ p,
                                                        const float2* __restrict__ ap, float2* __restrict__ x,
                                                        float2* __restrict__ r, double* __restrict__ part_vec,
                                                        CgState* __restrict__ st) {
    if (st->done) return;
    const double pap0 = block_sum(part_rows, row_blocks, 4, 0);
    const double pap1 = block_sum(part_rows, row_blocks, 4, 1);
    const double* rr = st->rr[it & 1];
    const float a0 = pap0 > 0.0 ? (float)(rr[0] / pap0) : 0.f;
    const float a1 = pap1 > 0.0 ? (float)(rr[1] / pap1) : 0.f;
    const int i = blockIdx.x * kCgVec + threadIdx.x;
    double s0 = 0.0, s1 = 0.0;
    if (i < k) {
        const float2 pv = p[i], av = ap[i];
        float2 xv = x[i], rv = r[i];
        xv.x = fmaf(a0, pv.x, xv.x);
        xv.y = fmaf(a1, pv.y, xv.y);
        rv.x = fmaf(-a0, av.x, rv.x);
        rv.y = fmaf(-a1, av.y, rv.y);
        x[i] = xv;
        r[i] = rv;
        s0 = (double)rv.x * rv.x;
        s1 = (double)rv.y * rv.y;
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_vec[(int64_t)blockIdx.x * 2 + 0] = red[0][0];
        part_vec[(int64_t)blockIdx.x * 2 + 1] = red[1][0];
    }
}

// p = r + beta p; block 0 records |r|^2 for the next iteration, counts the
// iteration and sets the stop flag.
__global__ __launch_bounds__(256) void cg_direction_kernel(int32_t k, int32_t it, const double* __restrict__ part_vec,
                                                           int64_t vec_blocks, double tol2,
                                                           const float2* __restrict__ r, float2* __restrict__ p,
                                                           CgState* __restrict__ st) {
    if (st->done) return;
    const double n0 = block_sum(part_vec, vec_blocks, 2, 0);
    const double n1 = block_sum(part_vec, vec_blocks, 2, 1);
    const double* rr = st->rr[it & 1];
    const float b0 = rr[0] > 0.0 ? (float)(n0 / rr[0]) : 0.f;
    const float b1 = rr[1] > 0.0 ? (float)(n1 / rr[1]) : 0.f;
    const int i = blockIdx.x * kCgVec + threadIdx.x;
    if (i < k) {
        const float2 rv = r[i];
        float2 pv = p[i];
        pv.x = fmaf(b0, pv.x, rv.x);
        pv.y = fmaf(b1, pv.y, rv.y);
        p[i] = pv;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr[(it + 1) & 1][0] = n0;
        st->rr[(it + 1) & 1][1] = n1;
        st->iters = it + 1;
        if (n0 <= tol2 * st->bb[0] && n1 <= tol2 * st->bb[1]) st->done = 1;
    }
}


// ---------------------------------------------------------------- batch form
// The exact step for every subgraph of a batch in one launch: one block of
// 1024 threads per subgraph runs the whole CG above with its vectors in LDS
// (Y, x, r, p, Ap: 40 bytes per node, 92 KB at the largest subgraph).  Rows
// are dealt to the 16 waves round-robin; each row's pair sums use the same
// per-lane order and wave tree as cg_rows_kernel, the dot products are FP64
// wave trees whose 16 wave sums are added in wave order.
constexpr int kCgBatchMaxN = Res<16>::NMAX;  // the batch's largest subgraph (2304, the resident PPR tile's limit)
constexpr int kCgBatchThreads = 1024;
constexpr int kCgBatchWaves = kCgBatchThreads / kWave;

// Fixed-order block sum of two FP64 values per thread; every thread gets both.
__device__ __forceinline__ void cg_batch_sum2(double& a, double& b, double (*red)[kCgBatchWaves]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();  // the previous sum's readers are done with red
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
    }
    __syncthreads();
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < kCgBatchWaves; ++w) {
        s0 += red[0][w];
        s1 += red[1][w];
    }
    a = s0;
    b = s1;
}

// Row pass over subgraph rows with v = Y (RHS: b_i and r_i = b_i - (L^w Y)_i,
// written to r and p; FP64 |b|^2 and |r|^2 per coordinate) or v = p (APPLY:
// Ap_i; FP64 p . Ap).  d0..d3 hold this lane's share of the dot products.
template <int MODE>
__device__ __forceinline__ void cg_batch_rows(const float* __restrict__ delta, int32_t k, const float2* v,
                                             float2* ra, float2* rb, double& d0, double& d1, double& d2,
                                             double& d3) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // two rows per wave at a time (i and i + 16), sharing each column's
    // position load; 2 x 8 row segments of Delta in flight per wave
    for (int i0 = wave; i0 < k; i0 += 2 * kCgBatchWaves) {
        const int i1 = i0 + kCgBatchWaves;
        const bool has1 = i1 < k;  // uniform in the wave
        const float2 xi[2] = {v[i0], has1 ? v[i1] : make_float2(0.f, 0.f)};
        const float* __restrict__ drow[2] = {delta + (int64_t)i0 * k, delta + (int64_t)(has1 ? i1 : i0) * k};
        float lx[2] = {0.f, 0.f}, ly[2] = {0.f, 0.f}, bx[2] = {0.f, 0.f}, by[2] = {0.f, 0.f};
        auto pair = [&](int r, int i, int j, float Dv, float2 xj) {
            const float inv = j != i ? __builtin_amdgcn_rcpf(Dv) : 0.f;
            const float w = inv * inv;
            const float dx = xi[r].x - xj.x;
            const float dy = xi[r].y - xj.y;
            lx[r] = fmaf(w, dx, lx[r]);
            ly[r] = fmaf(w, dy, ly[r]);
            if (MODE == kCgRhs) {
                const float rs = __builtin_amdgcn_rsqf(fmaf(dx, dx, fmaf(dy, dy, kMinSq)));
                const float c = inv * rs;
                bx[r] = fmaf(c, dx, bx[r]);
                by[r] = fmaf(c, dy, by[r]);
            }
        };
        int j = lane;
        for (; j + 7 * kWave < k; j += 8 * kWave) {
            float dv[2][8];
            float2 xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                dv[0][u] = drow[0][j + u * kWave];
                dv[1][u] = drow[1][j + u * kWave];
                xv[u] = v[j + u * kWave];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                pair(0, i0, j + u * kWave, dv[0][u], xv[u]);
                pair(1, i1, j + u * kWave, dv[1][u], xv[u]);
            }
        }
        for (; j < k; j += kWave) {
            const float2 xj = v[j];
            pair(0, i0, j, drow[0][j], xj);
            pair(1, i1, j, drow[1][j], xj);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            if (r == 1 && !has1) break;
            const int i = r == 0 ? i0 : i1;
            const float sx = wave_sum(lx[r]);
            const float sy = wave_sum(ly[r]);
            if (MODE == kCgRhs) {
                const float tx = wave_sum(bx[r]);
                const float ty = wave_sum(by[r]);
                const float2 rv = make_float2(tx - sx, ty - sy);
                if (lane == 0) {
                    ra[i] = rv;
                    rb[i] = rv;
                    d0 += (double)tx * tx;
                    d1 += (double)ty * ty;
                    d2 += (double)rv.x * rv.x;
                    d3 += (double)rv.y * rv.y;
                }
            } else if (lane == 0) {
                ra[i] = make_float2(sx, sy);
                d0 += (double)xi[r].x * sx;
                d1 += (double)xi[r].y * sy;
            }
        }
    }
}

__global__ __launch_bounds__(kCgBatchThreads) void cg_batch_kernel(const int64_t* __restrict__ node_off,
                                                                   const int64_t* __restrict__ mat_off,
                                                                   const float* __restrict__ delta_pool,
                                                                   const float2* __restrict__ x_in,
                                                                   float2* __restrict__ x_out, double tol2,
                                                                   int32_t max_iter, int32_t* __restrict__ iters_out,
                                                                   int32_t* __restrict__ conv_out) {
    __shared__ float2 Y[kCgBatchMaxN], X[kCgBatchMaxN], Rv[kCgBatchMaxN], P[kCgBatchMaxN], AP[kCgBatchMaxN];
    __shared__ double red[2][kCgBatchWaves];
    const int g = blockIdx.x;
    const int64_t base = node_off[g];
    const int64_t kk = node_off[g + 1] - base;
    if (kk < 1 || kk > kCgBatchMaxN) {  // uniform in the block
        if (threadIdx.x == 0) {
            if (iters_out) iters_out[g] = -1;
            if (conv_out) conv_out[g] = 0;
        }
        return;
    }
    const int k = (int)kk;
    const float* __restrict__ delta = delta_pool + mat_off[g];
    // centred start x0 = Y - mean(Y), mean in FP64
    double mx = 0.0, my = 0.0;
    for (int i = threadIdx.x; i < k; i += kCgBatchThreads) {
        const float2 y = x_in[base + i];
        Y[i] = y;
        mx += (double)y.x;
        my += (double)y.y;
    }
    cg_batch_sum2(mx, my, red);
    mx /= k;
    my /= k;
    for (int i = threadIdx.x; i < k; i += kCgBatchThreads)
        X[i] = make_float2((float)((double)Y[i].x - mx), (float)((double)Y[i].y - my));
    __syncthreads();
    double b0 = 0.0, b1 = 0.0, r0 = 0.0, r1 = 0.0;
    cg_batch_rows<kCgRhs>(delta, k, Y, Rv, P, b0, b1, r0, r1);
    cg_batch_sum2(b0, b1, red);
    cg_batch_sum2(r0, r1, red);
    bool done = r0 <= tol2 * b0 && r1 <= tol2 * b1;
    int it = 0;
    for (; !done && it < max_iter; ++it) {
        double p0 = 0.0, p1 = 0.0, unused0 = 0.0, unused1 = 0.0;
        cg_batch_rows<kCgApply>(delta, k, P, AP, nullptr, p0, p1, unused0, unused1);
        cg_batch_sum2(p0, p1, red);  // its barriers also order the Ap writes before the reads below
        const float a0 = p0 > 0.0 ? (float)(r0 / p0) : 0.f;
        const float a1 = p1 > 0.0 ? (float)(r1 / p1) : 0.f;
        double n0 = 0.0, n1 = 0.0;
        for (int i = threadIdx.x; i < k; i += kCgBatchThreads) {
            const float2 pv = P[i], av = AP[i];
            float2 xv = X[i], rv = Rv[i];
            xv.x = fmaf(a0, pv.x, xv.x);
            xv.y = fmaf(a1, pv.y, xv.y);
            rv.x = fmaf(-a0, av.x, rv.x);
            rv.y = fmaf(-a1, av.y, rv.y);
            X[i] = xv;
            Rv[i] = rv;
            n0 += (double)rv.x * rv.x;
            n1 += (double)rv.y * rv.y;
        }
        cg_batch_sum2(n0, n1, red);
        const float e0 = r0 > 0.0 ? (float)(n0 / r0) : 0.f;
        const float e1 = r1 > 0.0 ? (float)(n1 / r1) : 0.f;
        for (int i = threadIdx.x; i < k; i += kCgBatchThreads) {
            const float2 rv = Rv[i];
            float2 pv = P[i];
            pv.x = fmaf(e0, pv.x, rv.x);
            pv.y = fmaf(e1, pv.y, rv.y);
            P[i] = pv;
        }
        __syncthreads();  // p complete before the next apply
        r0 = n0;
        r1 = n1;
        done = n0 <= tol2 * b0 && n1 <= tol2 * b1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += kCgBatchThreads) x_out[base + i] = X[i];
    if (threadIdx.x == 0) {
        if (iters_out) iters_out[g] = it;
        if (conv_out) conv_out[g] = done ? 1 : 0;
    }
}

}  // namespace

}  // namespace pprviz

using namespace pprviz;

extern "C" {

size_t layout_exact_workspace(int32_t k) {
    if (k < 1) return 0;
    WsSize c;
    cg_ws_layout(c, k, nullptr);
    return c.used;
}

ppr_status layout_step_exact(const float* delta, int32_t k, const float* x_in, float* x_out, double cg_tol,
                             int32_t cg_max_iter, int32_t* cg_iters_out, void* ws, size_t ws_bytes, void* stream) {
    if (!delta || !x_in || !x_out || k < 1 || x_in == x_out) return PPR_EINVAL;
    if (!(cg_tol >= 0.0) || !std::isfinite(cg_tol) || cg_max_iter < 0) return PPR_EINVAL;
    if ((int64_t)k * k > ((int64_t)1 << 40)) return PPR_EUNSUPPORTED;
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    CgWs w;
    cg_ws_layout(cur, k, &w);
    if (ws == nullptr || cur.used > ws_bytes) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float2* y = reinterpret_cast<const float2*>(x_in);
    float2* x = reinterpret_cast<float2*>(x_out);
    const double tol2 = cg_tol * cg_tol;
    const int64_t rb = cg_row_blocks(k), vb = cg_vec_blocks(k);

    hipLaunchKernelGGL(cg_mean_kernel, dim3(1), dim3(256), 0, s, y, k, w.st);
    hipLaunchKernelGGL(cg_center_kernel, dim3((unsigned)vb), dim3(kCgVec), 0, s, y, k, w.st, x);
    hipLaunchKernelGGL((cg_rows_kernel<kCgRhs>), dim3((unsigned)rb), dim3(256), 0, s, delta, k, y, w.r, w.p,
                       w.part_rows, w.st);
    hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(256), 0, s, w.part_rows, rb, tol2, w.st);

    // Iterations in growing batches; between batches the host reads the
    // stop flag.  Kernels launched after the flag is set return at once.
    int32_t launched = 0, batch = 8;
    CgState hs{};
    while (true) {
        const int32_t end = std::min(cg_max_iter, launched + batch);
        for (int32_t it = launched; it < end; ++it) {
            hipLaunchKernelGGL((cg_rows_kernel<kCgApply>), dim3((unsigned)rb), dim3(256), 0, s, delta, k, w.p, w.ap,
                               nullptr, w.part_rows, w.st);
            hipLaunchKernelGGL(cg_update_kernel, dim3((unsigned)vb), dim3(kCgVec), 0, s, k, it, w.part_rows, rb, w.p,
                               w.ap, x, w.r, w.part_vec, w.st);
            hipLaunchKernelGGL(cg_direction_kernel, dim3((unsigned)vb), dim3(kCgVec), 0, s, k, it, w.part_vec, vb,
                               tol2, w.r, w.p, w.st);
        }
        launched = end;
        if (launch_status() != PPR_OK) return PPR_EHIP;
        PPRVIZ_HIP_TRY(hipMemcpyAsync(&hs, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        PPRVIZ_HIP_TRY(hipStreamSynchronize(s));
        if (hs.done || launched >= cg_max_iter) break;
        batch = std::min(batch * 2, 128);
    }
    if (cg_iters_out) *cg_iters_out = hs.iters;
    return hs.done ? PPR_OK : PPR_ENOCONV;
}


ppr_status pprviz_batch_step_exact(const ppr_batch* b, const float* delta_pool, const float* x_in, float* x_out,
                                   double cg_tol, int32_t cg_max_iter, int32_t* iters_out, int32_t* converged_out,
                                   void* stream) {
    if (b == nullptr || b->n_graphs < 1 || b->n_nodes < 1 || !b->node_off || !b->mat_off) return PPR_EINVAL;
    if (!delta_pool || !x_in || !x_out || x_in == x_out) return PPR_EINVAL;
    if (!(cg_tol >= 0.0) || !std::isfinite(cg_tol) || cg_max_iter < 0) return PPR_EINVAL;
    if (b->max_n < 1) return PPR_EINVAL;
    if (b->max_n > kCgBatchMaxN) return PPR_EUNSUPPORTED;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipLaunchKernelGGL(cg_batch_kernel, dim3((unsigned)b->n_graphs), dim3(kCgBatchThreads), 0,
                       static_cast<hipStream_t>(stream), b->node_off, b->mat_off, delta_pool,
                       reinterpret_cast<const float2*>(x_in), reinterpret_cast<float2*>(x_out), cg_tol * cg_tol,
                       cg_max_iter, iters_out, converged_out);
    return launch_status();
}

}  // extern "C"
