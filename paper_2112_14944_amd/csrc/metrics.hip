// Aesthetic metrics of a layout (Section 2.1): node distribution,
// ND(X) = sum_{i<j} 1 / ||X_i - X_j||^2 (Definition def:node-distri), and the
// uniform length coefficient variance ULCV(X) = l_sigma / l_mu of the edge
// lengths (Definition def:edge-var, population deviation).
//
// ND is one pass over the pairs i < j: 4 rows per wave, lanes striding over
// j > i, each lane adding its terms in FP64; per-block partials are added in
// a fixed order.  ULCV sums l and l^2 over the arcs of the symmetric CSR (each
// edge twice, which leaves mean and deviation unchanged), one node per lane,
// also in FP64 with fixed-order partials.
#include <math.h>

#include <algorithm>

#include "internal.hpp"

namespace pprviz {

namespace {

constexpr int kNdRows = 16;   // rows per block (4 waves x 4 rows)
constexpr int kUlNodes = 256; // nodes per block of the ULCV pass

inline int64_t nd_blocks(int32_t k) { return (k + kNdRows - 1) / kNdRows; }
inline int64_t ul_blocks(int32_t k) { return (k + kUlNodes - 1) / kUlNodes; }

__global__ __launch_bounds__(256) void nd_kernel(const float2* __restrict__ x, int32_t k, double* __restrict__ part) {
    __shared__ double red[4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    double s = 0.0;
    for (int r = 0; r < 4; ++r) {
        const int i = blockIdx.x * kNdRows + wave * 4 + r;
        if (i >= k) break;  // wave-uniform
        const float2 xi = x[i];
        for (int j = i + 1 + lane; j < k; j += kWave) {
            const float2 xj = x[j];
            const double dx = (double)xi.x - xj.x;
            const double dy = (double)xi.y - xj.y;
            s += 1.0 / (dx * dx + dy * dy);  // a coincident pair gives +inf
        }
    }
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// part[b][0] = sum of arc lengths, part[b][1] = sum of squares, block b's nodes.
__global__ __launch_bounds__(256) void ulcv_kernel(const float2* __restrict__ x, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, int32_t k,
                                                   double* __restrict__ part) {
    __shared__ double r1[256], r2[256];
    const int v = blockIdx.x * kUlNodes + threadIdx.x;
    double s1 = 0.0, s2 = 0.0;
    if (v < k) {
        const float2 xv = x[v];
        for (int e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const float2 xu = x[col_idx[e]];
            const double dx = (double)xv.x - xu.x;
            const double dy = (double)xv.y - xu.y;
            const double l2 = dx * dx + dy * dy;
            s1 += sqrt(l2);
            s2 += l2;
        }
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[(int64_t)blockIdx.x * 2] = r1[0];
        part[(int64_t)blockIdx.x * 2 + 1] = r2[0];
    }
}

// out[0] = ND; out[1] = ULCV from the arc sums (nnz arcs), NaN when undefined.
__global__ __launch_bounds__(256) void metrics_finish_kernel(const double* __restrict__ nd_part, int64_t nd_n,
                                                             const double* __restrict__ ul_part, int64_t ul_n,
                                                             int64_t nnz, double* __restrict__ out) {
    __shared__ double a[256], b[256], c[256];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = threadIdx.x; i < nd_n; i += 256) s0 += nd_part[i];
    for (int64_t i = threadIdx.x; i < ul_n; i += 256) {
        s1 += ul_part[i * 2];
        s2 += ul_part[i * 2 + 1];
    }
    a[threadIdx.x] = s0;
    b[threadIdx.x] = s1;
    c[threadIdx.x] = s2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            a[threadIdx.x] += a[threadIdx.x + o];
            b[threadIdx.x] += b[threadIdx.x + o];
            c[threadIdx.x] += c[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = a[0];
        double u = NAN;
        if (nnz > 0) {
            const double mu = b[0] / (double)nnz;
            const double var = fmax(c[0] / (double)nnz - mu * mu, 0.0);
            if (mu > 0.0) u = sqrt(var) / mu;
        }
        out[1] = u;
    }
}

struct MetricsWs {
    double* nd_part;
    double* ul_part;
    double* out;
};

template <typename Cursor>
void metrics_ws_layout(Cursor& c, int32_t k, MetricsWs* w) {
    MetricsWs t{};
    t.nd_part = c.template take<double>((size_t)nd_blocks(k));
    t.ul_part = c.template take<double>((size_t)ul_blocks(k) * 2);
    t.out = c.template take<double>(2);
    if (w) *w = t;
}

}  // namespace

}  // namespace pprviz

using namespace pprviz;

extern "C" {

size_t layout_metrics_workspace(int32_t k) {
    if (k < 1) return 0;
    WsSize c;
    metrics_ws_layout(c, k, nullptr);
    return c.used;
}

ppr_status layout_metrics(const float* x, int32_t k, const ppr_csr* g, double* nd_out, double* ulcv_out, void* ws,
                          size_t ws_bytes, void* stream) {
    if (x == nullptr || k < 1 || (nd_out == nullptr && ulcv_out == nullptr)) return PPR_EINVAL;
    if (ulcv_out) {
        const ppr_status st = validate_csr(g);
        if (st != PPR_OK) return st;
        if (g->n != k) return PPR_EINVAL;
    }
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    MetricsWs w;
    metrics_ws_layout(cur, k, &w);
    if (ws == nullptr || cur.used > ws_bytes) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float2* xv = reinterpret_cast<const float2*>(x);
    const int64_t nb = nd_out ? nd_blocks(k) : 0;
    const int64_t ub = ulcv_out ? ul_blocks(k) : 0;
    if (nb) hipLaunchKernelGGL(nd_kernel, dim3((unsigned)nb), dim3(256), 0, s, xv, k, w.nd_part);
    if (ub)
        hipLaunchKernelGGL(ulcv_kernel, dim3((unsigned)ub), dim3(256), 0, s, xv, g->row_ptr, g->col_idx, k,
                           w.ul_part);
    hipLaunchKernelGGL(metrics_finish_kernel, dim3(1), dim3(256), 0, s, w.nd_part, nb, w.ul_part, ub,
                       ulcv_out ? g->nnz : (int64_t)0, w.out);
    if (launch_status() != PPR_OK) return PPR_EHIP;
    double out[2];
    PPRVIZ_HIP_TRY(hipMemcpyAsync(out, w.out, sizeof(out), hipMemcpyDeviceToHost, s));
    PPRVIZ_HIP_TRY(hipStreamSynchronize(s));
    if (nd_out) *nd_out = out[0];
    if (ulcv_out) *ulcv_out = out[1];
    return PPR_OK;
}

}  // extern "C"
