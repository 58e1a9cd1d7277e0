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

// Slot table and arc copy of the resident tile (group layout, see
// ppr_core.hpp), one block per graph.
//  1. Rows sorted by degree, longest first, ties by row id (bitonic sort of
//     4096 keys in LDS; a graph of the resident tile has at most 2304 rows).
//  2. Group g's length: its longest row (at least 1: a row without arcs gets
//     its self arc) in 8-arc halves; chunk offsets by a prefix sum in sorted
//     order.
//  3. Arcs are dealt by LDS bank class.  One LDS cycle of the tile's
//     16-byte reads serves M rows at once (M = 4, 2, 1 for 16, 32, 64
//     columns: 64 bytes of each of 4 rows, 128 of 2, 256 of 1;
//     res_conflict_set names them), and row u starts in bank class u mod M.
//     One thread takes such a set of M rows and fills their positions m = 0,
//     1, ... together: each row takes, among the classes no other row has
//     taken at m, the one it holds most arcs of; a row with no such arc pads
//     with the zero row of a free class (the tile has one zero row per class)
//     as long as it can still fit its arcs, and otherwise takes a
//     conflicting class.  Only the order of each row's arcs changes (and
//     with it the order of the FP32 sum).  The copy holds each arc's LDS byte
//     offset in the tile, (u - first node) * 4 COLS, not its node id.
// A graph whose padded groups exceed its reserved region (possible only with
// repeated arcs, when a row is longer than n) gets one half chunk per row
// holding the row's own offset and a NaN scale, so that its outputs are NaN.
// The rows of a group whose LDS reads are served in the same cycles.  A
// 16-byte LDS read by a wave is served 16 lanes at a time, lanes grouped by
// lane bit 5 and the parity of lane bits 2..4 (a probe of the patterns
// across the 16 quads of a wave: quads {0,3,5,6} share cycles, as do
// {1,2,4,7} and the same sets plus 8).  With 16 columns a quad is a row,
// so those quad sets are the row sets; with 32 columns quads 2r and 2r+1
// read the two halves of row r, and the rows whose halves meet in one
// cycle set are {0,3} and {1,2} (and plus 4); with 64 columns one row fills
// a cycle set.
__device__ __forceinline__ void res_conflict_set(int M, int j, int rr[4]) {
    if (M == 4) {
        const int h = (j >> 1) * 8;
        const bool odd = (j & 1) != 0;
        rr[0] = h + (odd ? 1 : 0);
        rr[1] = h + (odd ? 2 : 3);
        rr[2] = h + (odd ? 4 : 5);
        rr[3] = h + (odd ? 7 : 6);
    } else if (M == 2) {
        const int h = (j >> 1) * 4;
        rr[0] = h + ((j & 1) ? 1 : 0);
        rr[1] = h + ((j & 1) ? 2 : 3);
        rr[2] = rr[3] = 0;
    } else {
        rr[0] = j;
        rr[1] = rr[2] = rr[3] = 0;
    }
}

// One set of M rows of a group (res_conflict_set), dealt together.
struct ResDealSet {
    int L;          // positions every row of the set fills (the group's length)
    int words;      // entries per row over all its chunks
    int32_t* ca;    // the group's chunk 0 in the arc copy
    float* wa;      // same for the weights, or nullptr
    int GW, n, stride;
    int64_t base;
    bool over;      // NaN layout: each row holds only its own offset
    const int32_t* row_ptr;
    const int32_t* sorted;  // each row's arcs as LDS offsets, grouped by class (CSR order within a class)
    const float* wsorted;   // their weights, or nullptr
    const int32_t (*cstart)[4];  // per row: first arc of each class within its group of sorted
};

// Fills the set's rows position by position.  At position m the rows choose
// in the order m, m+1, ... (mod M); each takes the free class it holds most
// arcs of, pads with the zero row of a free class when it has none and can
// still fit its arcs, and otherwise takes its largest class (a conflict).
// Rows without arcs hold their own offset first; v[i] < 0 marks a dummy slot.
template <int M>
__device__ __forceinline__ void res_deal_set(const ResDealSet& d, const int rr[4], const int v[4]) {
    auto at = [&](int m) { return (int64_t)(m >> 4) * 16 * d.GW + (m & 15); };
    auto zero_row = [&](int c) { return (d.n + (((c - d.n) % M) + M) % M) * d.stride; };
    auto put = [&](int i, int m, int off, float w) {
        d.ca[16 * rr[i] + at(m)] = off;
        if (d.wa) d.wa[16 * rr[i] + at(m)] = w;
    };
    int cnt[M][M], cur[M][M], rem[M], re[M];
    bool fixed[M];  // rows written outside the deal (own offset first, or dummies)
#pragma unroll
    for (int i = 0; i < M; ++i) {
        rem[i] = 0;
        re[i] = 0;
        fixed[i] = false;
#pragma unroll
        for (int c = 0; c < M; ++c) cnt[i][c] = cur[i][c] = 0;
        if (v[i] < 0) continue;
        const int rs = d.row_ptr[d.base + v[i]];
        re[i] = d.row_ptr[d.base + v[i] + 1];
        if (d.over || re[i] == rs) {
            put(i, 0, v[i] * d.stride, 1.f);
            for (int m = 1; m < d.words; ++m) put(i, m, d.n * d.stride, 0.f);
            fixed[i] = true;
            continue;
        }
        rem[i] = re[i] - rs;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const int c0 = d.cstart[v[i]][c];
            const int c1 = c + 1 < M ? d.cstart[v[i]][c + 1] : re[i] - rs;
            cnt[i][c] = c1 - c0;
            cur[i][c] = rs + c0;
        }
    }
    for (int mb = 0; mb < d.L; mb += M) {
#pragma unroll
        for (int s = 0; s < M; ++s) {
            const int m = mb + s;
            uint32_t taken = 0, placed = 0;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int i = (s + k) % M;
                if (fixed[i] || rem[i] == 0) continue;
                int pick = -1, pany = -1, pickv = 0, panyv = 0;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    const int x = cnt[i][c];
                    if (x > panyv) {
                        pany = c;
                        panyv = x;
                    }
                    if (!(taken >> c & 1u) && x > pickv) {
                        pick = c;
                        pickv = x;
                    }
                }
                placed |= 1u << i;
                if (pick < 0 && rem[i] < d.L - m && taken != (1u << M) - 1u) {
                    const int c = __builtin_ctz(~taken);
                    taken |= 1u << c;
                    put(i, m, zero_row(c), 0.f);
                    continue;
                }
                if (pick < 0) pick = pany;
                taken |= 1u << pick;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    if (c != pick) continue;
                    const int e = cur[i][c]++;
                    put(i, m, d.sorted[e], d.wsorted ? d.wsorted[e] : 0.f);
                    --cnt[i][c];
                }
                --rem[i];
            }
            // rows already done, and dummy slots: zero rows of free classes
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (fixed[i] || (placed >> i & 1u)) continue;
                const int c = taken == (1u << M) - 1u ? 0 : __builtin_ctz(~taken);
                taken |= 1u << c;
                put(i, m, zero_row(c), 0.f);
            }
        }
    }
    // entries past L up to the end of the last chunk (never read)
#pragma unroll
    for (int i = 0; i < M; ++i) {
        if (fixed[i]) continue;
        for (int m = d.L; m < d.words; ++m) put(i, m, d.n * d.stride, 0.f);
    }
}

__global__ __launch_bounds__(256) void res_layout_kernel(const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col_idx,
                                                        const float* __restrict__ weight,
                                                        const float* __restrict__ invd,
                                                        const int64_t* __restrict__ node_off, int32_t n_single,
                                                        ResSlot* __restrict__ slots, int32_t* __restrict__ arcs,
                                                        float* __restrict__ warcs, int32_t* __restrict__ sorted,
                                                        float* __restrict__ wsorted) {
    constexpr int kMaxRows = 4096;
    __shared__ uint32_t key[kMaxRows];
    __shared__ int32_t cstart[Res<16>::NMAX][4];
    __shared__ int64_t goff[kResMaxGroups + 1];
    __shared__ int32_t ghalves[kResMaxGroups];
    const int g = blockIdx.x;
    const int64_t base = node_off ? node_off[g] : 0;
    const int n = node_off ? (int)(node_off[g + 1] - base) : n_single;
    const int cols = n > 0 ? res_cols_for(n) : 0;
    if (cols == 0) return;  // larger graphs never use the resident tile
    const int GW = 256 / cols;                            // group size, Res<cols>::RPW
    const int M = cols == 16 ? 4 : (cols == 32 ? 2 : 1);  // bank classes = rows per LDS pass
    const int stride = cols * 4;                          // LDS bytes per row
    TileTask tb;
    res_graph_bases(base, row_ptr[base], row_ptr[base + n], g, n, tb);

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
    // each row's arcs as LDS offsets, grouped by bank class (CSR order within
    // a class), and where each class starts
    for (int v = threadIdx.x; v < n; v += 256) {
        const int rs = row_ptr[base + v], re = row_ptr[base + v + 1];
        int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        for (int e = rs; e < re; ++e) {
            const int c = (int)((col_idx[e] - base) & (M - 1));
            c0 += c == 0;
            c1 += c == 1;
            c2 += c == 2;
            c3 += c == 3;
        }
        int pos[4] = {rs, rs + c0, rs + c0 + c1, rs + c0 + c1 + c2};
        cstart[v][0] = 0;
        cstart[v][1] = c0;
        cstart[v][2] = c0 + c1;
        cstart[v][3] = c0 + c1 + c2;
        for (int e = rs; e < re; ++e) {
            const int u = (int)(col_idx[e] - base);
            const int c = u & (M - 1);
            const int at = c == 0 ? pos[0]++ : (c == 1 ? pos[1]++ : (c == 2 ? pos[2]++ : pos[3]++));
            sorted[at] = u * stride;
            if (wsorted) wsorted[at] = weight[e];
        }
    }
    const int ng = (n + GW - 1) / GW;
    for (int gi = threadIdx.x; gi < ng; gi += 256) {
        int dmax = 1;
        for (int r = 0; r < GW; ++r) {
            const int p = gi * GW + r;
            if (p < n) {
                const int64_t gv = base + (int)(key[p] & 4095u);
                dmax = max(dmax, row_ptr[gv + 1] - row_ptr[gv]);
            }
        }
        const int h = (int)(((int64_t)dmax + 7) / 8);
        ghalves[gi] = h;
        goff[gi + 1] = (int64_t)((h + 1) / 2) * 16 * GW;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        goff[0] = 0;
        for (int gi = 0; gi < ng; ++gi) goff[gi + 1] += goff[gi];
    }
    __syncthreads();
    const bool over = goff[ng] > (int64_t)tb.cwords;
    // slot table
    for (int p = threadIdx.x; p < ng * GW; p += 256) {
        const int gi = p / GW;
        const int r = p - gi * GW;
        const int h = over ? 1 : ghalves[gi];
        const int64_t o = over ? (int64_t)gi * 16 * GW + 16 * r : goff[gi] + 16 * r;
        int v = n;
        float iv = 0.f;
        if (p < n) {
            v = (int)(key[p] & 4095u);
            iv = over ? __int_as_float(0x7fc00000) : invd[base + v];
        }
        slots[tb.tbase + p] = ResSlot{(int32_t)o, h, v, iv};
    }
    // arcs: one thread per set of M rows of a group whose reads share LDS
    // cycles (4 sets per group)
    for (int t = threadIdx.x; t < ng * 4; t += 256) {
        const int gi = t >> 2;
        ResDealSet d;
        d.L = over ? 8 : ghalves[gi] * 8;
        d.words = over ? 16 : (ghalves[gi] + 1) / 2 * 16;
        d.ca = arcs + tb.cbase + (over ? (int64_t)gi * 16 * GW : goff[gi]);
        d.wa = warcs ? warcs + tb.cbase + (over ? (int64_t)gi * 16 * GW : goff[gi]) : nullptr;
        d.GW = GW;
        d.n = n;
        d.stride = stride;
        d.base = base;
        d.over = over;
        d.row_ptr = row_ptr;
        d.sorted = sorted;
        d.wsorted = weight ? wsorted : nullptr;
        d.cstart = cstart;
        int rr[4];
        res_conflict_set(M, t & 3, rr);
        int v[4];
        for (int i = 0; i < 4; ++i) {
            const int p = gi * GW + rr[i];
            v[i] = (i < M && p < n) ? (int)(key[p] & 4095u) : -1;
        }
        if (M == 4) res_deal_set<4>(d, rr, v);
        else if (M == 2) res_deal_set<2>(d, rr, v);
        else res_deal_set<1>(d, rr, v);
    }
}


void launch_res_layout(const int32_t* row_ptr, const int32_t* col_idx, const float* weight, const float* invd,
                       const int64_t* node_off, int32_t n_single, int32_t blocks, ResSlot* slots, int32_t* arcs,
                       float* warcs, int32_t* sorted, float* wsorted, hipStream_t s) {
    hipLaunchKernelGGL(res_layout_kernel, dim3(blocks), dim3(256), 0, s, row_ptr, col_idx, weight, invd, node_off,
                       n_single, slots, arcs, warcs, sorted, wsorted);
}

template <int COLS, bool WEIGHTED>
__global__ __launch_bounds__(kResThreads) void ppr_resident_kernel(ResArgs a, int32_t n, int64_t nnz,
                                                                 int32_t n_src, int32_t n_tgt) {
    __shared__ ResLds L;
    TileTask t;
    t.n = n;
    t.s0 = blockIdx.x * COLS;
    t.ncols = min(COLS, n_src - t.s0);
    t.n_tgt = n_tgt;
    t.base = 0;
    t.out_off = 0;
    t.ld = n_tgt;
    res_graph_bases(0, 0, nnz, 0, n, t);
    res_tile<COLS, WEIGHTED>(t, a, L);
}

void launch_degree(const int32_t* row_ptr, const float* weight, int64_t n, float* deg, float* invd,
                   hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(degree_kernel, dim3((unsigned)blocks), dim3(256), 0, s, row_ptr, weight, n, deg, invd);
}

template <int COLS>
static void launch_resident(bool weighted, const ResArgs& a, int n, int64_t nnz, int n_src, int n_tgt,
                            hipStream_t s) {
    dim3 grid((n_src + COLS - 1) / COLS);
    if (weighted)
        hipLaunchKernelGGL((ppr_resident_kernel<COLS, true>), grid, dim3(kResThreads), 0, s, a, n, nnz, n_src, n_tgt);
    else
        hipLaunchKernelGGL((ppr_resident_kernel<COLS, false>), grid, dim3(kResThreads), 0, s, a, n, nnz, n_src,
                           n_tgt);
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
        launch_res_layout(g->row_ptr, g->col_idx, g->weight, invd, nullptr, n, 1, w.slots, w.col_r,
                          g->weight ? w.w_r : nullptr, w.sorted_r, g->weight ? w.sorted_w : nullptr, s);
        ResArgs a;
        a.slots = w.slots;
        a.arcs = w.col_r;
        a.warcs = g->weight ? w.w_r : nullptr;
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
            case 64: launch_resident<64>(wt, a, n, g->nnz, n_src, n_tgt, s); break;
            case 32: launch_resident<32>(wt, a, n, g->nnz, n_src, n_tgt, s); break;
            default: launch_resident<16>(wt, a, n, g->nnz, n_src, n_tgt, s); break;
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
