// Single-graph multi-source PPR / DPPR (ppr_matrix) and shared helpers.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "ppr_core.hpp"
#include "internal.hpp"

namespace pprviz {

__global__ void degree_kernel(const int32_t* __restrict__ row_ptr, const float* __restrict__ weight,
                              int64_t n, float* __restrict__ deg, float* __restrict__ invd) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int rs = row_ptr[v], re = row_ptr[v + 1];
    float d;
    if (weight) {
        float s = 0.f;
        for (int e = rs; e < re; ++e) s += weight[e];
        d = s;
    } else {
        d = (float)(re - rs);
    }
    deg[v] = d;
    invd[v] = (re > rs && d > 0.f) ? 1.0f / d : 1.0f;
}

// Row table of the resident tile: rows sorted by degree, longest first, ties
// by row id; one block per graph.  rs/re locate the row in the tile's arc
// copy, where global row v starts at row_ptr[v] + kArcRowPad v (room to pad
// each row, see bank_order_kernel).
__global__ __launch_bounds__(256) void row_table_kernel(const int32_t* __restrict__ row_ptr,
                                                       const int64_t* __restrict__ node_off, int32_t n_single,
                                                       RowEnt* __restrict__ table) {
    constexpr int kMaxRows = 4096;
    __shared__ uint32_t key[kMaxRows];
    const int g = blockIdx.x;
    const int64_t base = node_off ? node_off[g] : 0;
    const int n = node_off ? (int)(node_off[g + 1] - base) : n_single;
    if (n <= 0 || n > kMaxRows) return;  // larger graphs never use the resident tile
    int P = 1;
    while (P < n) P <<= 1;
    for (int i = threadIdx.x; i < P; i += 256) {
        if (i < n) {
            const int d = min(row_ptr[base + i + 1] - row_ptr[base + i], 4095);
            key[i] = ((uint32_t)(4095 - d) << 12) | (uint32_t)i;
        } else {
            key[i] = 0xFFFFFFFFu;
        }
    }
    __syncthreads();
    // bitonic sort, ascending key = descending degree, ties by row id
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += 256) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint32_t x = key[i], y = key[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        key[i] = y;
                        key[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int p = threadIdx.x; p < n; p += 256) {
        const int v = (int)(key[p] & 4095u);
        const int64_t gv = base + v;
        const int rs = row_ptr[gv] + kArcRowPad * (int)gv;
        table[base + p] = RowEnt{rs, rs + (row_ptr[gv + 1] - row_ptr[gv]), v, 0};
    }
}

// Copy of the arcs for the resident tile, one thread per row slot of all
// graphs, with each row's arcs dealt by LDS bank class.  In the tile, the four
// quads of a 16-lane LDS pass read the rows of four consecutive slot
// positions, arc position m of each at the same instruction, and a row u of a
// 16- (32-) column tile starts in bank group u mod 4 (u mod 2).  Position m of
// the row in slot p therefore takes an arc of class (m + p) mod 4 (mod 2)
// while that class lasts, so the four reads of a pass fall in different bank
// groups.  Only the order of each row's arcs changes (and with it the order of
// the FP32 sum).  The copy holds each arc's LDS byte offset in the tile,
// (u - first node) * 4 COLS, not its node id, and each row with arcs is
// padded with the offset of the tile's zero row to at least 16 arcs and to a
// multiple of 8, so the tile's chunks (a full 16-arc chunk first, then full
// chunks and a last one of 16 or 8) need no bound checks.
__global__ __launch_bounds__(256) void bank_order_kernel(const int32_t* __restrict__ col_idx,
                                                        const float* __restrict__ weight,
                                                        const int64_t* __restrict__ node_off, int32_t n_graphs,
                                                        int64_t n_slots, const RowEnt* __restrict__ table,
                                                        int32_t* __restrict__ col_out, float* __restrict__ w_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_slots) return;
    int g = 0;
    if (node_off) {  // graph of slot i: largest g with node_off[g] <= i
        int lo = 0, hi = n_graphs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (node_off[mid] <= i) lo = mid; else hi = mid - 1;
        }
        g = lo;
    }
    const int64_t base = node_off ? node_off[g] : 0;
    const int n = node_off ? (int)(node_off[g + 1] - base) : (int)n_slots;
    const int p = (int)(i - base);
    const int cols = res_cols_for(n);
    const int M = cols == 16 ? 4 : (cols == 32 ? 2 : 1);  // bank classes
    const int stride = (cols > 0 ? cols : 16) * 4;        // LDS bytes per row
    const RowEnt r = table[i];
    const int shift = kArcRowPad * (int)(base + r.v);  // copy position - CSR position
    const int rs = r.rs - shift, re = r.re - shift;
    const int deg = re - rs;
    const int pad_end = r.rs + (deg == 0 ? 0 : max(16, (deg + 7) / 8 * 8));
    for (int m = r.re; m < pad_end; ++m) {
        col_out[m] = n * stride;
        if (w_out) w_out[m] = 0.f;
    }
    if (M == 1) {
        for (int e = rs; e < re; ++e) {
            col_out[e + shift] = (int)(col_idx[e] - base) * stride;
            if (w_out) w_out[e + shift] = weight[e];
        }
        return;
    }
    // next[c]: next arc of class c in the original order (re when none)
    int next[4];
    for (int c = 0; c < 4; ++c) {
        int e = rs;
        while (e < re && (int)((col_idx[e] - base) & (M - 1)) != c) ++e;
        next[c] = c < M ? e : re;
    }
    for (int m = rs; m < re; ++m) {
        int c = (m - rs + p) & (M - 1);
        for (int t = 0; t < M && next[c] >= re; ++t) c = (c + 1) & (M - 1);
        const int e = next[c];
        col_out[m + shift] = (int)(col_idx[e] - base) * stride;
        if (w_out) w_out[m + shift] = weight[e];
        int f = e + 1;
        while (f < re && (int)((col_idx[f] - base) & (M - 1)) != c) ++f;
        next[c] = f;
    }
}

void launch_row_table(const int32_t* row_ptr, const int32_t* col_idx, const float* weight,
                      const int64_t* node_off, int32_t n_single, int32_t blocks, int64_t n_slots, RowEnt* table,
                      int32_t* col_out, float* w_out, hipStream_t s) {
    hipLaunchKernelGGL(row_table_kernel, dim3(blocks), dim3(256), 0, s, row_ptr, node_off, n_single, table);
    hipLaunchKernelGGL(bank_order_kernel, dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, s, col_idx, weight,
                       node_off, blocks, n_slots, table, col_out, w_out);
}

template <int COLS, bool WEIGHTED>
__global__ __launch_bounds__(kResThreads) void ppr_resident_kernel(ResArgs a, int32_t n, int32_t n_src,
                                                                 int32_t n_tgt) {
    __shared__ ResLds L;
    TileTask t;
    t.n = n;
    t.s0 = blockIdx.x * COLS;
    t.ncols = min(COLS, n_src - t.s0);
    t.n_tgt = n_tgt;
    t.base = 0;
    t.out_off = 0;
    t.ld = n_tgt;
    res_tile<COLS, WEIGHTED>(t, a, L);
}

void launch_degree(const int32_t* row_ptr, const float* weight, int64_t n, float* deg, float* invd,
                   hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(degree_kernel, dim3((unsigned)blocks), dim3(256), 0, s, row_ptr, weight, n, deg, invd);
}

template <int COLS>
static void launch_resident(bool weighted, const ResArgs& a, int n, int n_src, int n_tgt, hipStream_t s) {
    dim3 grid((n_src + COLS - 1) / COLS);
    if (weighted)
        hipLaunchKernelGGL((ppr_resident_kernel<COLS, true>), grid, dim3(kResThreads), 0, s, a, n, n_src, n_tgt);
    else
        hipLaunchKernelGGL((ppr_resident_kernel<COLS, false>), grid, dim3(kResThreads), 0, s, a, n, n_src, n_tgt);
}

ppr_status validate_csr(const ppr_csr* g) {
    if (g == nullptr || g->n < 1 || g->nnz < 0 || g->nnz >= (int64_t)INT32_MAX) return PPR_EINVAL;
    if (g->row_ptr == nullptr || (g->nnz > 0 && g->col_idx == nullptr)) return PPR_EINVAL;
    return PPR_OK;
}

bool use_resident(int n) { return res_cols_for(n) != 0; }

// T pushes from every source; deg/invd must already hold the degrees.  Three
// kernels by size: the LDS-resident tile (n <= 2304), the mid-size kernel
// with the iterate columns in LDS (n <= 40831), and the streaming SpMM with
// the iterate in HBM.
void ppr_forward(const ppr_csr* g, const int32_t* src, int32_t n_src, const int32_t* tgt, int32_t n_tgt,
                 float alpha, int32_t T, float* ppr_out, float* dppr_out, const float* deg, const float* invd,
                 double* resid, const PprWs& w, hipStream_t s) {
    const int n = g->n;
    if (use_resident(n)) {
        launch_row_table(g->row_ptr, g->col_idx, g->weight, nullptr, n, 1, n, w.rows, w.col_r,
                         g->weight ? w.w_r : nullptr, s);
        ResArgs a;
        a.rows = w.rows;
        a.row_ptr = g->row_ptr;
        a.col_idx = w.col_r;
        a.weight = g->weight ? w.w_r : nullptr;
        a.invd = invd;
        a.deg = deg;
        a.src = src;
        a.tgt = tgt;
        a.alpha = alpha;
        a.T = T;
        a.ppr_out = ppr_out;
        a.dppr_out = dppr_out;
        a.resid = resid;
        const bool wt = g->weight != nullptr;
        switch (res_cols_for(n)) {
            case 64: launch_resident<64>(wt, a, n, n_src, n_tgt, s); break;
            case 32: launch_resident<32>(wt, a, n, n_src, n_tgt, s); break;
            default: launch_resident<16>(wt, a, n, n_src, n_tgt, s); break;
        }
    } else if (mid_cols_for(n) != 0) {
        mid_forward(g, src, n_src, tgt, n_tgt, alpha, T, ppr_out, dppr_out, deg, invd, resid, w.mid, s);
    } else {
        stream_row_order(g->row_ptr, n, w.hist, w.rows, s);
        StreamArgs sa;
        sa.rows = w.rows;
        sa.row_ptr = g->row_ptr;
        sa.col_idx = g->col_idx;
        sa.weight = g->weight;
        sa.invd = invd;
        sa.deg = deg;
        sa.n = n;
        sa.ncols = n_src;
        sa.ld = stream_ld(n_src);
        sa.alpha = alpha;
        sa.src = src;
        sa.forcing = nullptr;
        sa.ld_forcing = 0;
        const float* x = stream_power_iteration(sa, T, w.ya, w.yb, s);
        stream_write_outputs(x, sa, tgt, n_tgt, ppr_out, dppr_out, s);
        if (resid) stream_residuals(x, sa, w.part, resid, s);
    }
}


// Scratch memory of ppr_matrix_noalloc: a fixed device array, one copy per
// GPU, that replaces the caller's workspace for callers that cannot allocate
// (graph capture, tight serving loops).  Host code never passes the array's
// name to a kernel: scratch_address resolves it once per device, with that
// device current, and keeps the device address.
constexpr size_t kScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;

static ppr_status scratch_address(hipStream_t s, void** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    if (s != nullptr) {
        hipDevice_t d = 0;
        PPRVIZ_HIP_TRY(hipStreamGetDevice(s, &d));
        dev = (int)d;
    } else {
        PPRVIZ_HIP_TRY(hipGetDevice(&dev));
    }
    if (dev < 0 || dev >= kMaxDevices) return PPR_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        int cur = 0;
        PPRVIZ_HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) PPRVIZ_HIP_TRY(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) PPRVIZ_HIP_TRY(hipSetDevice(cur));
        if (e != hipSuccess || p == nullptr) return PPR_EHIP;
        addr[dev] = p;
    }
    *out = addr[dev];
    return PPR_OK;
}

// ppr_matrix with the workspace given (the caller's, or this GPU's scratch).
static ppr_status ppr_matrix_impl(const ppr_csr* g, const int32_t* src, int32_t n_src, const int32_t* tgt,
                                  int32_t n_tgt, float alpha, double tol_l1, int32_t max_iter, float* ppr_out,
                                  float* dppr_out, double* resid_out, int32_t* iters_out, void* ws,
                                  size_t ws_bytes, void* stream, bool scratch_ws) {
    ppr_status st = validate_csr(g);
    if (st != PPR_OK) return st;
    if (n_src < 0 || n_tgt < 0 || (n_src > 0 && src == nullptr)) return PPR_EINVAL;
    if (tgt == nullptr && n_tgt != g->n) return PPR_EINVAL;
    if (!(alpha > 0.0f && alpha < 1.0f) || max_iter < 0) return PPR_EINVAL;
    if ((int64_t)n_src * (int64_t)std::max(n_tgt, 1) > ((int64_t)1 << 40)) return PPR_EUNSUPPORTED;
    if (g->n > kStreamMaxN) return PPR_EUNSUPPORTED;
    int32_t T = 0, conv = 1;
    st = pprviz_pushes_for_tolerance(alpha, tol_l1, max_iter, &T, &conv);
    if (st != PPR_OK) return st;
    if (iters_out) *iters_out = T;
    if (n_src == 0) return conv ? PPR_OK : PPR_ENOCONV;
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    PprWs w;
    ppr_ws_layout(cur, g->n, g->nnz, g->weight != nullptr, n_src, &w);
    if (ws == nullptr || cur.used > ws_bytes) return scratch_ws ? PPR_EUNSUPPORTED : PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = g->n;
    launch_degree(g->row_ptr, g->weight, n, w.deg, w.invd, s);

    ppr_forward(g, src, n_src, tgt, n_tgt, alpha, T, ppr_out, dppr_out, w.deg, w.invd, w.resid, w, s);
    st = launch_status();
    if (st != PPR_OK) return st;
    if (resid_out) {
        PPRVIZ_HIP_TRY(hipMemcpyAsync(resid_out, w.resid, sizeof(double) * n_src, hipMemcpyDeviceToHost, s));
        PPRVIZ_HIP_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < n_src; ++i)
            if (!isfinite(resid_out[i])) return PPR_ENONFINITE;
    }
    return conv ? PPR_OK : PPR_ENOCONV;
}

}  // namespace pprviz

using namespace pprviz;

extern "C" {

const char* pprviz_version(void) { return "pprviz-gfx950 1.0"; }

const char* pprviz_status_string(int status) {
    switch (status) {
        case PPR_OK: return "ok";
        case PPR_EINVAL: return "invalid argument";
        case PPR_ENOCONV: return "iteration cap reached before the residual tolerance";
        case PPR_EWORKSPACE: return "workspace missing or too small";
        case PPR_EHIP: return "HIP runtime error";
        case PPR_ENONFINITE: return "non-finite result";
        case PPR_EUNSUPPORTED: return "size not supported by this build";
        default: return "unknown status";
    }
}

ppr_status pprviz_pushes_for_tolerance(float alpha, double tol, int32_t max_iter, int32_t* pushes,
                                       int32_t* converged) {
    if (!(alpha > 0.0f && alpha < 1.0f) || max_iter < 0 || pushes == nullptr) return PPR_EINVAL;
    const double q = 1.0 - (double)alpha;
    int32_t T;
    int32_t conv = 1;
    if (!(tol > 0.0)) {
        T = max_iter;
    } else if (tol >= 1.0) {
        T = 0;
    } else {
        double t = ceil(log(tol) / log(q));
        if (t < 0) t = 0;
        if (t > 2.0e9) t = 2.0e9;
        int64_t ti = (int64_t)t;
        while (ti > 0 && pow(q, (double)(ti - 1)) <= tol) --ti;
        while (pow(q, (double)ti) > tol) ++ti;
        if (ti > max_iter) {
            T = max_iter;
            conv = 0;
        } else {
            T = (int32_t)ti;
        }
    }
    *pushes = T;
    if (converged) *converged = conv;
    return PPR_OK;
}


size_t ppr_matrix_workspace(const ppr_csr* g, int32_t n_src, int32_t n_tgt) {
    (void)n_tgt;
    if (g == nullptr || g->n < 1 || n_src < 0) return 0;
    WsSize c;
    ppr_ws_layout(c, g->n, g->nnz, g->weight != nullptr, n_src, nullptr);
    return c.used;
}

ppr_status ppr_matrix(const ppr_csr* g, const int32_t* src, int32_t n_src, const int32_t* tgt,
                      int32_t n_tgt, float alpha, double tol_l1, int32_t max_iter, float* ppr_out,
                      float* dppr_out, double* resid_out, int32_t* iters_out, void* ws, size_t ws_bytes,
                      void* stream) {
    return ppr_matrix_impl(g, src, n_src, tgt, n_tgt, alpha, tol_l1, max_iter, ppr_out, dppr_out, resid_out,
                           iters_out, ws, ws_bytes, stream, false);
}

size_t ppr_matrix_noalloc_max_scratch(void) { return kScratchBytes; }

ppr_status ppr_matrix_noalloc(const ppr_csr* g, const int32_t* src, int32_t n_src, const int32_t* tgt,
                              int32_t n_tgt, float alpha, double tol_l1, int32_t max_iter, float* ppr_out,
                              float* dppr_out, double* resid_out, int32_t* iters_out, void* stream) {
    // The workspace bound is checked before the scratch address is looked up,
    // so an oversized request fails without touching the device.
    ppr_status st = validate_csr(g);
    if (st != PPR_OK) return st;
    if (n_src < 0) return PPR_EINVAL;
    if (ppr_matrix_workspace(g, n_src, n_tgt) > kScratchBytes) return PPR_EUNSUPPORTED;
    void* scr = nullptr;
    st = scratch_address(static_cast<hipStream_t>(stream), &scr);
    if (st != PPR_OK) return st;
    return ppr_matrix_impl(g, src, n_src, tgt, n_tgt, alpha, tol_l1, max_iter, ppr_out, dppr_out, resid_out,
                           iters_out, scr, kScratchBytes, stream, true);
}

}  // extern "C"
