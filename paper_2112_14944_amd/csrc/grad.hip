// Gradient of a loss on the all-pairs DPPR with respect to the edge weights.
//
// Chain rule through the walk of Section 3.1 and Definition def:pprdist
// (rows = sources, Q = (1-alpha) P = (1-alpha) D^-1 W, pi_hat = alpha sum Q^j):
//   Gb = D G                       G = dLoss/dpi_d, pi_d = D pi_hat
//   A  = sum_{j<T} (Q^T)^j Gb      adjoint of pi = alpha (I - Q)^-1, truncated
//                                  like the T-push forward
//   dQ[u][v] = <A[u,:], pi_hat[v,:]>
//   g(u->v)  = (1-alpha)/d_u (dQ[u][v] - sum_b P_ub dQ[u][b]) + sum_t G[u][t] pi_hat[u][t]
//   dLoss/dw_{u,v} = g(u->v) + g(v->u)   (one weight shared by both arcs)
// The adjoint gathers over the same neighbours with the same coefficients as
// the forward push, so it reuses the streaming step with a dense forcing term.
#include "internal.hpp"

namespace pprviz {

// One wave per arc: dq[e] = <A[u, :], pi[v, :]>, A in the slab layout of
// the streaming iterate, pi row-major n x n.
__global__ __launch_bounds__(256) void arc_dot_kernel(const int32_t* __restrict__ row_of_arc,
                                                      const int32_t* __restrict__ col_idx, int64_t nnz,
                                                      const float* __restrict__ A,
                                                      const float* __restrict__ pi, int32_t n,
                                                      double* __restrict__ dq) {
    const int lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= nnz) return;
    const int64_t u = row_of_arc[e];
    const int64_t v = col_idx[e];
    const float* p = pi + v * (int64_t)n;
    double s = 0.0;
    for (int t = lane; t < n; t += 64) s = fma((double)A[sidx(u, t, n)], (double)p[t], s);
    s = wave_sum(s);
    if (lane == 0) dq[e] = s;
}

// dd[u] = sum_t G[u][t] pi[u][t]
__global__ __launch_bounds__(256) void row_dot_kernel(const float* __restrict__ G, const float* __restrict__ pi,
                                                      int32_t n, double* __restrict__ dd) {
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u >= n) return;
    double s = 0.0;
    for (int t = lane; t < n; t += 64) s = fma((double)G[u * n + t], (double)pi[u * n + t], s);
    s = wave_sum(s);
    if (lane == 0) dd[u] = s;
}

__global__ void row_of_arc_kernel(const int32_t* __restrict__ row_ptr, int32_t n, int32_t* __restrict__ row_of_arc) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    for (int e = row_ptr[u]; e < row_ptr[u + 1]; ++e) row_of_arc[e] = (int32_t)u;
}

// g(u->v) per arc; one thread per row.
__global__ void arc_grad_kernel(const int32_t* __restrict__ row_ptr, const float* __restrict__ weight,
                                const float* __restrict__ deg, const double* __restrict__ dq,
                                const double* __restrict__ dd, int32_t n, float alpha, double* __restrict__ g) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int rs = row_ptr[u], re = row_ptr[u + 1];
    if (rs == re) return;
    const double d = deg[u];
    double row = 0.0;
    for (int e = rs; e < re; ++e) row += (weight ? (double)weight[e] : 1.0) / d * dq[e];
    const double f = (1.0 - (double)alpha) / d;
    for (int e = rs; e < re; ++e) g[e] = f * (dq[e] - row) + dd[u];
}

// Edge gradient: the arc's own term plus that of its reverse arc, found by
// binary search in the (sorted) neighbour list of the other endpoint.
__global__ void edge_sum_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                                const int32_t* __restrict__ row_of_arc, int64_t nnz, const double* __restrict__ g,
                                float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int u = row_of_arc[e];
    const int v = col_idx[e];
    int lo = row_ptr[v], hi = row_ptr[v + 1] - 1;
    int rev = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = col_idx[mid];
        if (c == u) {
            rev = mid;
            break;
        }
        if (c < u) lo = mid + 1; else hi = mid - 1;
    }
    out[e] = (float)(g[e] + (rev >= 0 ? g[rev] : 0.0));
}

struct BwdWs {
    PprWs f;  // forward recompute (any kernel) plus the streaming buffers of the adjoint
    float* pi;
    double* dq;
    double* dd;
    double* g;
    int32_t* row_of_arc;
};

template <typename Cursor>
static void bwd_layout(Cursor& c, int n, int64_t nnz, bool weighted, bool recompute, BwdWs* w) {
    BwdWs t;
    ppr_ws_layout(c, n, nnz, weighted, n, &t.f, true);
    t.pi = recompute ? c.template take<float>((size_t)n * n) : nullptr;
    t.dq = c.template take<double>((size_t)std::max<int64_t>(nnz, 1));
    t.dd = c.template take<double>(n);
    t.g = c.template take<double>((size_t)std::max<int64_t>(nnz, 1));
    t.row_of_arc = c.template take<int32_t>((size_t)std::max<int64_t>(nnz, 1));
    if (w) *w = t;
}

}  // namespace pprviz

using namespace pprviz;

extern "C" {

size_t ppr_backward_workspace(const ppr_csr* g, int recompute) {
    if (g == nullptr || g->n < 1 || g->nnz < 0) return 0;
    WsSize c;
    bwd_layout(c, g->n, g->nnz, g->weight != nullptr, recompute != 0, nullptr);
    return c.used;
}

ppr_status ppr_matrix_backward(const ppr_csr* g, float alpha, int32_t T, const float* ppr,
                               const float* grad_dppr, float* grad_arc, void* ws, size_t ws_bytes,
                               void* stream) {
    ppr_status st = validate_csr(g);
    if (st != PPR_OK) return st;
    if (!(alpha > 0.0f && alpha < 1.0f) || T < 0 || grad_dppr == nullptr || (g->nnz > 0 && grad_arc == nullptr))
        return PPR_EINVAL;
    if ((int64_t)g->n * g->n > ((int64_t)1 << 36) || g->n > kStreamMaxN) return PPR_EUNSUPPORTED;
    const bool recompute = (ppr == nullptr);
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    BwdWs w;
    bwd_layout(cur, g->n, g->nnz, g->weight != nullptr, recompute, &w);
    if (ws == nullptr || cur.used > ws_bytes) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    if (g->nnz == 0) return PPR_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = g->n;
    const PprWs& f = w.f;
    launch_degree(g->row_ptr, g->weight, n, f.deg, f.invd, s);
    const float* pi = ppr;
    if (recompute) {
        ppr_forward(g, nullptr, n, nullptr, n, alpha, T, w.pi, nullptr, f.deg, f.invd, nullptr, f, s);
        pi = w.pi;
    }
    stream_row_order(g->row_ptr, n, f.hist, f.rows, s);
    StreamArgs sa;
    sa.rows = f.rows;
    sa.row_ptr = g->row_ptr;
    sa.col_idx = g->col_idx;
    sa.weight = g->weight;
    sa.invd = f.invd;
    sa.deg = f.deg;
    sa.n = n;
    sa.ncols = n;
    sa.ld = stream_ld(n);
    sa.alpha = alpha;
    sa.src = nullptr;
    sa.forcing = grad_dppr;
    sa.ld_forcing = n;
    const float* A = stream_power_iteration(sa, T, f.ya, f.yb, s);
    hipLaunchKernelGGL(row_of_arc_kernel, dim3((n + 255) / 256), dim3(256), 0, s, g->row_ptr, n, w.row_of_arc);
    hipLaunchKernelGGL(arc_dot_kernel, dim3((unsigned)((g->nnz + 3) / 4)), dim3(256), 0, s, w.row_of_arc, g->col_idx,
                       g->nnz, A, pi, n, w.dq);
    hipLaunchKernelGGL(row_dot_kernel, dim3((n + 3) / 4), dim3(256), 0, s, grad_dppr, pi, n, w.dd);
    hipLaunchKernelGGL(arc_grad_kernel, dim3((n + 255) / 256), dim3(256), 0, s, g->row_ptr, g->weight, f.deg, w.dq,
                       w.dd, n, alpha, w.g);
    hipLaunchKernelGGL(edge_sum_kernel, dim3((unsigned)((g->nnz + 255) / 256)), dim3(256), 0, s, g->row_ptr,
                       g->col_idx, w.row_of_arc, g->nnz, w.g, grad_arc);
    return launch_status();
}

}  // extern "C"
