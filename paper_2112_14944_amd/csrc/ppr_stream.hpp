// Power iteration for graphs too large to keep any source column of the
// iterate in LDS (more than 40831 nodes): the iterate lives in HBM (ping-pong
// buffers, column slabs of 32 sources) and each push is one launch.  A wave
// takes 8 rows side by side, so every gathered neighbour row is one
// contiguous 128-byte read (details at stream_step_kernel).
//
// The same step serves the adjoint solve of the weight gradient:
//     A_{k+1} = Gb + (1-alpha) P^T A_k      (Gb = D G, forcing term)
// which gathers over the same neighbours with the same coefficients.
#pragma once

#include "ppr_core.hpp"

namespace pprviz {

inline int64_t stream_ld(int64_t ncols) { return (ncols + 63) / 64 * 64; }
constexpr int kStreamResidRows = 4096;
inline int64_t stream_resid_chunks(int64_t n) { return (n + kStreamResidRows - 1) / kStreamResidRows; }

// Iterate layout: column slabs of 32 columns, each slab stored node-major
// and contiguous (n rows of 128 bytes), slab after slab; ld columns in all
// (ld a multiple of 64), so a buffer holds n * ld floats.
constexpr int kSlab = 32;
constexpr int kSlabVec = kSlab / 4;             // float4 per slab row
constexpr int kArcsPerLoad = kWave / kSlabVec;  // arcs one wave load covers

__host__ __device__ __forceinline__ int64_t sidx(int64_t v, int64_t col, int64_t n) {
    return ((col / kSlab) * n + v) * kSlab + (col % kSlab);
}

struct StreamArgs {
    const RowEnt* rows;   // rows by non-increasing degree (stream_row_order)
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const float* weight;
    const float* invd;
    const float* deg;
    int32_t n;
    int32_t ncols;        // valid columns (sources / adjoint right-hand sides)
    int64_t ld;           // columns held (multiple of 64)
    float alpha;
    const int32_t* src;   // forward: source node of column s (nullptr: column s = node s)
    const float* forcing; // adjoint: G [n][ld_forcing] (Gb = deg[v] * G[v][s]); nullptr = forward
    int64_t ld_forcing;
};

constexpr int kStreamRowsPerWave = kWave / kSlabVec;  // 8 rows side by side
constexpr int kStreamRowsPerBlock = 4 * kStreamRowsPerWave;
constexpr int kXcds = 8;
// A slab of the iterate that fits this budget stays in one XCD's L2 (4 MB)
// next to the arc stream while that XCD sweeps it.
constexpr int64_t kStreamSlabBudget = 3 << 20;
constexpr int kDegKeys = 4096;
// Slab gathers use 32-bit byte offsets: n * 128 must stay below 2^31.
constexpr int32_t kStreamMaxN = 1 << 24;  // degree classes of the row order (exact below 4095)

// Launch shape of one push: `slabs` column slabs, each swept by `row_blocks`
// blocks of 32 rows.
struct StreamGrid {
    int32_t row_blocks;
    int32_t slabs;
    int32_t full_rounds;  // rounds of 8 slabs run one per XCD (0: none)
};

// Block -> (slab, row block).  Workgroups go to the 8 XCDs round-robin by
// linear id, so blocks b, b + 8, b + 16, ... share one XCD.  In each of the
// first full_rounds rounds every XCD sweeps all rows of a slab of its own, so
// the neighbour rows it gathers are served by its own L2.  The remaining
// slabs are taken one after another by all XCDs together (for large n that
// keeps one slab at a time in the shared last-level cache).  The grid has
// exactly slabs * row_blocks blocks and the map is a bijection onto the pairs.
__device__ __forceinline__ void stream_block_map(const StreamGrid& g, int& slab, int& rb) {
    const int b = blockIdx.x;
    const int full_blocks = g.full_rounds * kXcds * g.row_blocks;
    if (b < full_blocks) {
        const int local = b / kXcds;
        slab = (local / g.row_blocks) * kXcds + b % kXcds;
        rb = local % g.row_blocks;
    } else {
        const int local = b - full_blocks;
        slab = g.full_rounds * kXcds + local / g.row_blocks;
        rb = local % g.row_blocks;
    }
}

// Row order by degree, largest first: a counting sort over KEYS degree
// classes (degrees from KEYS - 1 up share the first class), so that the 8
// rows a streaming-step wave takes side by side have (nearly) equal arc
// counts.  The order within a class is whatever the atomics give; it only
// decides which rows share a wave, never a sum.  This histogram with one
// global atomic per row serves the mid-size kernel's 65536 exact classes
// (which do not fit in LDS; it has a stable scatter of its own); the
// streaming row order below counts per block in LDS.
template <int KEYS>
static __global__ void stream_deg_hist_kernel(const int32_t* __restrict__ row_ptr, int32_t n,
                                              int32_t* __restrict__ hist) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int d = min(row_ptr[v + 1] - row_ptr[v], KEYS - 1);
    atomicAdd(&hist[KEYS - 1 - d], 1);
}

// Exclusive prefix sum of the KEYS class counts, in place (one block).
template <int KEYS>
static __global__ __launch_bounds__(1024) void stream_deg_scan_kernel(int32_t* __restrict__ hist) {
    constexpr int kPer = KEYS / 1024;
    static_assert(KEYS % 1024 == 0, "keys");
    __shared__ int32_t part[1024];
    const int t0 = threadIdx.x * kPer;
    int32_t t = 0;
    for (int i = 0; i < kPer; ++i) t += hist[t0 + i];
    part[threadIdx.x] = t;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t x = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - t;
    for (int i = 0; i < kPer; ++i) {
        const int32_t h = hist[t0 + i];
        hist[t0 + i] = run;
        run += h;
    }
}

// Streaming row order: the class counts are kept per block in LDS.  A block
// counts its kOrderNodes rows there and adds each nonzero class count to the
// global histogram once, then reserves one range per class with one atomic
// and hands out positions inside it from LDS.  With a few hundred rows per
// degree class in a block, this takes the global atomics on the few classes
// of common degrees down from one per row to one per block and class.
constexpr int kOrderNodes = 2048;

template <int KEYS>
static __global__ __launch_bounds__(1024) void stream_deg_hist_lds_kernel(const int32_t* __restrict__ row_ptr,
                                                                          int32_t n, int32_t* __restrict__ hist) {
    __shared__ int32_t cnt[KEYS];
    for (int i = threadIdx.x; i < KEYS; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * kOrderNodes;
    const int64_t e = min((int64_t)n, b + kOrderNodes);
    for (int64_t v = b + threadIdx.x; v < e; v += blockDim.x) {
        const int d = min(row_ptr[v + 1] - row_ptr[v], KEYS - 1);
        atomicAdd(&cnt[KEYS - 1 - d], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < KEYS; i += blockDim.x)
        if (cnt[i]) atomicAdd(&hist[i], cnt[i]);
}

template <int KEYS>
static __global__ __launch_bounds__(1024) void stream_deg_scatter_lds_kernel(const int32_t* __restrict__ row_ptr,
                                                                             int32_t n, int32_t* __restrict__ cursor,
                                                                             RowEnt* __restrict__ rows) {
    __shared__ int32_t cnt[KEYS];
    for (int i = threadIdx.x; i < KEYS; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * kOrderNodes;
    const int64_t e = min((int64_t)n, b + kOrderNodes);
    for (int64_t v = b + threadIdx.x; v < e; v += blockDim.x) {
        const int d = min(row_ptr[v + 1] - row_ptr[v], KEYS - 1);
        atomicAdd(&cnt[KEYS - 1 - d], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < KEYS; i += blockDim.x)
        if (cnt[i]) cnt[i] = atomicAdd(&cursor[i], cnt[i]);
    __syncthreads();
    for (int64_t v = b + threadIdx.x; v < e; v += blockDim.x) {
        const int rs = row_ptr[v], re = row_ptr[v + 1];
        const int d = min(re - rs, KEYS - 1);
        const int pos = atomicAdd(&cnt[KEYS - 1 - d], 1);
        rows[pos] = RowEnt{rs, re, (int32_t)v, 0};
    }
}

template <int KEYS = kDegKeys>
inline void stream_row_order(const int32_t* row_ptr, int32_t n, int32_t* hist, RowEnt* rows, hipStream_t s) {
    static_assert(KEYS * 4 <= 32768, "per-block class counts must fit in LDS");
    fill<int32_t>(hist, 0, KEYS, s);
    const unsigned blocks = (unsigned)((n + kOrderNodes - 1) / kOrderNodes);
    hipLaunchKernelGGL(stream_deg_hist_lds_kernel<KEYS>, dim3(blocks), dim3(1024), 0, s, row_ptr, n, hist);
    hipLaunchKernelGGL(stream_deg_scan_kernel<KEYS>, dim3(1), dim3(1024), 0, s, hist);
    hipLaunchKernelGGL(stream_deg_scatter_lds_kernel<KEYS>, dim3(blocks), dim3(1024), 0, s, row_ptr, n, hist,
                       rows);
}

__device__ __forceinline__ void f4_acc(float4& a, float4 y) {
    a.x += y.x;
    a.y += y.y;
    a.z += y.z;
    a.w += y.w;
}

__device__ __forceinline__ void f4_fma(float4& a, float w, float4 y) {
    a.x = fmaf(w, y.x, a.x);
    a.y = fmaf(w, y.y, a.y);
    a.z = fmaf(w, y.z, a.z);
    a.w = fmaf(w, y.w, a.w);
}

// Gather of one 16-byte piece of a slab row through a buffer resource: an
// offset past the slab (a padded arc slot) reads zeros and touches no memory.
__device__ __forceinline__ float4 slab_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_float4(__int_as_float(v[0]), __int_as_float(v[1]), __int_as_float(v[2]), __int_as_float(v[3]));
}

// Sum over the arcs of this lane's row of w_vu * Y[u][4 columns of piece
// qoff] (w = 1 without weights).  The 8 lanes of a row read 8 arc indices at
// once, coalesced, and pass them round with ds_bpermute; each lane then adds
// its row's neighbours in arc order, so a row's sum does not depend on which
// rows share its wave.  Every lane of the wave must call it (dg = 0 for a
// lane without a row).
// FLAGGED: only neighbours u with flags[u] != 0 are read (the others count
// as zero rows), and `got` is set when the row has such a neighbour.
// STEP: arcs a lane group advances per pass; 8 when each group owns a row,
// 64 when the wave's 8 groups share one row (group g then passes its row's
// arcs from 8g on, and the caller adds the groups' sums).
template <bool WEIGHTED, bool FLAGGED = false, int STEP = kSlabVec>
__device__ __forceinline__ float4 slab_gather(__amdgpu_buffer_rsrc_t rin, const int32_t* __restrict__ col_idx,
                                              const float* __restrict__ weight, int rs, int dg, int lane,
                                              uint32_t qoff, const uint8_t* __restrict__ flags = nullptr,
                                              int* got = nullptr) {
    const int q = lane % kSlabVec;
    int dmax = dg;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o, kWave));
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int any = 0;
    const int lead = (lane & ~(kSlabVec - 1)) * 4;  // ds_bpermute address of the group's first lane
    // Software pipeline over the passes: arc indices are loaded two passes
    // ahead, weights and push flags one pass ahead, so that a long row's
    // pass waits only on its own gathers.
    int idx_cur = q < dg ? col_idx[rs + q] : -1;
    int idx_next = STEP + q < dg ? col_idx[rs + STEP + q] : -1;
    float wl_cur = 0.f;
    if (WEIGHTED) wl_cur = q < dg ? weight[rs + q] : 0.f;
    bool on_cur = true;
    if (FLAGGED) on_cur = idx_cur >= 0 && flags[idx_cur] != 0;
    for (int k0 = 0; k0 < dmax; k0 += STEP) {
        int idx = idx_cur;
        const float wl = wl_cur;
        const bool on = on_cur;
        const int idx_after = k0 + 2 * STEP + q < dg ? col_idx[rs + k0 + 2 * STEP + q] : -1;
        if (WEIGHTED) wl_cur = k0 + STEP + q < dg ? weight[rs + k0 + STEP + q] : 0.f;
        if (FLAGGED) {
            on_cur = idx_next >= 0 && flags[idx_next] != 0;
            idx = on ? idx : -1;
            any |= on ? 1 : 0;
        }
        idx_cur = idx_next;
        idx_next = idx_after;
        float4 y[kSlabVec];
#pragma unroll
        for (int j = 0; j < kSlabVec; ++j) {
            const int u = __builtin_amdgcn_ds_bpermute(lead + 4 * j, idx);
            y[j] = slab_load(rin, ((uint32_t)u << 7) | qoff);
        }
#pragma unroll
        for (int j = 0; j < kSlabVec; ++j) {
            if (WEIGHTED) {
                const float w = __int_as_float(__builtin_amdgcn_ds_bpermute(lead + 4 * j, __float_as_int(wl)));
                f4_fma(acc, w, y[j]);
            } else {
                f4_acc(acc, y[j]);
            }
        }
    }
    if (FLAGGED) {
        // OR over the 8 lanes of the row
#pragma unroll
        for (int o = 1; o < kSlabVec; o <<= 1) any |= __shfl_xor(any, o, kWave);
        *got = any;
    }
    return acc;
}

// One push (MODE 0: forward, forcing alpha at each column's source row;
// MODE 1: adjoint, forcing deg[v] * G[v][col]).  A wave takes 8 rows of the
// degree order side by side within one slab: lane = 8 * g + q, where g picks
// the row and q 4 of the slab's 32 columns (one 16-byte load per arc, summed
// by slab_gather).
template <int MODE, bool WEIGHTED, bool FINAL>
__global__ __launch_bounds__(256) void stream_step_kernel(
    const RowEnt* __restrict__ rows, const int32_t* __restrict__ col_idx,
    const float* __restrict__ weight, const float* __restrict__ invd, const float* __restrict__ deg,
    const int32_t* __restrict__ src, const float* __restrict__ forcing, int64_t ld_forcing, int32_t n,
    int32_t ncols, float alpha, StreamGrid grid, const float* __restrict__ yin, float* __restrict__ yout) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int q = lane % kSlabVec;
    int slab, rb;
    stream_block_map(grid, slab, rb);
    const int64_t slab_off = (int64_t)slab * n * kSlab;
    const uint32_t slab_bytes = (uint32_t)n * (kSlab * 4);
    const __amdgpu_buffer_rsrc_t rin =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(yin + slab_off), 0, (int)slab_bytes, 0x00020000);
    const int ri = rb * kStreamRowsPerBlock + wave * kStreamRowsPerWave + lane / kSlabVec;
    const bool has_row = ri < n;
    int rs = 0, dg = 0, v = 0;
    if (has_row) {
        const RowEnt e = load_row(as_global(rows), ri);
        rs = e.rs;
        dg = e.re - e.rs;
        v = e.v;
    }
    const uint32_t qoff = (uint32_t)q * 16u;
    float4 acc = slab_gather<WEIGHTED>(rin, col_idx, weight, rs, dg, lane, qoff);
    if (has_row && dg == 0) acc = slab_load(rin, ((uint32_t)v << 7) | qoff);
    if (!has_row) return;
    const int col0 = slab * kSlab + q * 4;
    float x[4] = {acc.x, acc.y, acc.z, acc.w};
    const float sv = FINAL ? 1.0f : (1.0f - alpha) * invd[v];
    const float dv = MODE == 1 ? deg[v] : 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int col = col0 + c;
        if (MODE == 0) {
            if (col < ncols && v == (src ? src[col] : col)) x[c] += alpha;
        } else {
            x[c] += col < ncols ? dv * forcing[(int64_t)v * ld_forcing + col] : 0.0f;
        }
        x[c] = FINAL ? x[c] : x[c] * sv;
    }
    float4* o4 = reinterpret_cast<float4*>(yout + slab_off);
    o4[(int64_t)v * kSlabVec + q] = make_float4(x[0], x[1], x[2], x[3]);
}

// Y_0 for the forward iteration: zero everywhere but the source rows.
static __global__ void stream_init_forward_kernel(const int32_t* __restrict__ src, const float* __restrict__ invd,
                                           int32_t n, int32_t ncols, float alpha, int final_,
                                           float* __restrict__ y) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ncols) return;
    int v = src ? src[s] : s;
    y[sidx(v, s, n)] = final_ ? alpha : alpha * (1.0f - alpha) * invd[v];
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
    y[sidx(v, col, n)] = final_ ? g : g * (1.0f - alpha) * invd[v];
}

// out[s][j] = X[tgt[j]][s] (and d(src_s) times it), 64x64 tiles through LDS.
static __global__ __launch_bounds__(256) void stream_transpose_kernel(
    const float* __restrict__ x, int32_t n, int32_t ncols, const int32_t* __restrict__ src,
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
            val = x[sidx(tn, s0 + lane, n)];
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
    for (int64_t r = r0 + w; r < r1; r += 4) s += (double)x[sidx(r, col, n)];
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
    StreamGrid g;
    g.row_blocks = (a.n + kStreamRowsPerBlock - 1) / kStreamRowsPerBlock;
    g.slabs = (int32_t)(a.ld / kSlab);
    g.full_rounds = ((int64_t)a.n * kSlab * 4 <= kStreamSlabBudget) ? g.slabs / kXcds : 0;
    const dim3 grid((unsigned)((int64_t)g.row_blocks * g.slabs));
    if (a.weight)
        hipLaunchKernelGGL((stream_step_kernel<MODE, true, FINAL>), grid, dim3(256), 0, s, a.rows, a.col_idx,
                           a.weight, a.invd, a.deg, a.src, a.forcing, a.ld_forcing, a.n, a.ncols, a.alpha, g, yin,
                           yout);
    else
        hipLaunchKernelGGL((stream_step_kernel<MODE, false, FINAL>), grid, dim3(256), 0, s, a.rows, a.col_idx,
                           a.weight, a.invd, a.deg, a.src, a.forcing, a.ld_forcing, a.n, a.ncols, a.alpha, g, yin,
                           yout);
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
                           a.invd, a.n, a.ncols, a.alpha, T == 1 ? 1 : 0, ya);
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
    hipLaunchKernelGGL(stream_transpose_kernel, grid, dim3(256), 0, s, x, a.n, a.ncols, a.src, tgt, n_tgt, a.deg,
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
