// Multi-source PPR power iteration kernels (device side), shared by the
// single-graph entry points and the batched persistent kernel.
//
// Section 3.1 of the paper defines pi(s, t) through a random walk with restart;
// Section 3.3 computes it near-exactly by power iteration, whose synchronous
// form pushes every node at once (the push of Eq. eq:fwd-invariant).  Here the
// iterate is X_t = pi_hat after t+1 pushes, stored node-major (row v holds
// pi_hat(s, v) for the sources s of a tile, one lane per source):
//     X_0 = alpha E,   X_{t+1}[v, s] = alpha [v == src_s] + (1-alpha) sum_u P[u, v] X_t[u, s].
// Each step gathers over the in-neighbours u of v, which for an undirected
// graph are its CSR neighbours.  The kernels keep Y[u, s] = (1-alpha) X[u, s] /
// d(u) instead of X, so that a unit-weight gather is a plain sum and a
// weighted one a single FMA per arc; a node without arcs keeps its own mass
// (implicit self-loop, Y = (1-alpha) X).
#pragma once

#include "common.hpp"

namespace pprviz {

// 1024 threads (16 waves, 4 per SIMD) leave each wave 128 VGPRs.
constexpr int kResThreads = 1024;
constexpr int kResWaves = kResThreads / kWave;
constexpr int kArcPad = 16;  // padding entries after the tile's arc array (chunk loads read ahead)
constexpr int kArcRowPad = 16;  // room per row in the tile's arc copy for padding the row
constexpr int kResMaxK = 9;  // rows per lane (4 columns each) held in registers across a step

// Tile geometry.  Lanes work in quads: a quad owns 16 columns of one row, each
// lane 4 consecutive columns read with one 16-byte LDS load per arc, and the
// quad's arcs are broadcast inside the quad with DPP quad_perm.  A row of a
// COLS-wide tile takes COLS/16 quads.
template <int COLS>
struct Res {
    static constexpr int QPR = COLS / 16;                  // quads per row
    static constexpr int RPW = 16 / QPR;                   // rows per wave per pass
    static constexpr int RPP = kResWaves * RPW;            // rows per block pass
    static constexpr int NMAX = RPP * kResMaxK;            // largest graph for this tile width
    static constexpr int STRIDE = COLS * 4;                // bytes per LDS row
};

// LDS floats for one resident tile: n rows plus one zero row, times COLS; the
// maximum over the three tile widths (577*64, 1153*32, 2305*16).
constexpr int kResLdsFloats = 36928;
static_assert((Res<64>::NMAX + 1) * 64 <= kResLdsFloats, "lds");
static_assert((Res<32>::NMAX + 1) * 32 <= kResLdsFloats, "lds");
static_assert((Res<16>::NMAX + 1) * 16 <= kResLdsFloats, "lds");

__host__ __device__ inline int res_cols_for(int n) {
    return n <= Res<64>::NMAX ? 64 : (n <= Res<32>::NMAX ? 32 : (n <= Res<16>::NMAX ? 16 : 0));
}

// One source tile of one graph.
struct TileTask {
    int32_t n;        // node count of the graph
    int32_t s0;       // first source index of the tile
    int32_t ncols;    // sources in the tile (<= COLS)
    int32_t n_tgt;    // output columns
    int64_t base;     // global id of the graph's node 0
    int64_t out_off;  // offset of output row 0
    int64_t ld;       // output leading dimension
};

// Row table entry: a row of the resident tile's slot order.
struct __attribute__((aligned(16))) RowEnt {
    int32_t rs;   // first arc
    int32_t re;   // one past the last arc
    int32_t v;    // row id (local to its graph)
    int32_t pad;
};

__device__ __forceinline__ RowEnt load_row(gcptr<RowEnt> p, int64_t i) {
    RowEnt e;
    e.rs = p[i].rs;
    e.re = p[i].re;
    e.v = p[i].v;
    e.pad = 0;
    return e;
}

struct ResArgs {
    const RowEnt* rows;      // per graph, rows in slot order (row_table_kernel)
    const int32_t* row_ptr;  // global CSR row pointers
    const int32_t* col_idx;  // arc copy (bank_order_kernel): LDS byte offset of the neighbour's row, rows padded
    const float* weight;     // arc weights, or nullptr
    const float* invd;       // per global node: 1/d, or 1 for a node without arcs
    const float* deg;        // per global node: weighted degree d
    const int32_t* src;      // source local ids by source index, or nullptr (source i = node i)
    const int32_t* tgt;      // target local ids, or nullptr (targets = nodes 0..n_tgt-1)
    float alpha;
    int32_t T;               // pushes
    float* ppr_out;          // nullable
    float* dppr_out;         // nullable
    double* resid;           // nullable, indexed by source index
};

// Broadcast lane J of every quad to the whole quad (DPP quad_perm [J,J,J,J]).
template <int J>
__device__ __forceinline__ int quad_bcast(int v) {
    return __builtin_amdgcn_update_dpp(0, v, J * 0x55, 0xf, 0xf, false);
}
template <int J>
__device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), J * 0x55, 0xf, 0xf, false));
}

__device__ __forceinline__ float4 lds_load4(const float* lds, int byte_off) {
    return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(lds) + byte_off);
}

// One chunk of 16 arcs (NH = 2 halves) or 8 arcs (NH = 1) of a quad's row:
// arc 4L + W sits in lane L, word W (a0..a3 hold LDS byte offsets of the
// neighbours' rows, the zero row past the row's end), so the arcs are summed
// in row order.  Eight 16-byte reads are issued before their adds.
template <bool WEIGHTED, int NH>
__device__ __forceinline__ void gather_chunk(const float* __restrict__ lds, int a0, int a1, int a2, int a3,
                                             float w0, float w1, float w2, float w3, int cbyte, float4& acc) {
#define PPRVIZ_RD(M, A) y[(M) & 7] = lds_load4(lds, quad_bcast<(M) / 4>(A) + cbyte);
#define PPRVIZ_ACC(M, W)                                          \
    if (WEIGHTED) {                                               \
        const float ww = quad_bcast<(M) / 4>(W);                  \
        acc.x = fmaf(ww, y[(M) & 7].x, acc.x);                    \
        acc.y = fmaf(ww, y[(M) & 7].y, acc.y);                    \
        acc.z = fmaf(ww, y[(M) & 7].z, acc.z);                    \
        acc.w = fmaf(ww, y[(M) & 7].w, acc.w);                    \
    } else {                                                      \
        acc.x += y[(M) & 7].x;                                    \
        acc.y += y[(M) & 7].y;                                    \
        acc.z += y[(M) & 7].z;                                    \
        acc.w += y[(M) & 7].w;                                    \
    }
    float4 y[8];
    PPRVIZ_RD(0, a0) PPRVIZ_RD(1, a1) PPRVIZ_RD(2, a2) PPRVIZ_RD(3, a3)
    PPRVIZ_RD(4, a0) PPRVIZ_RD(5, a1) PPRVIZ_RD(6, a2) PPRVIZ_RD(7, a3)
    __builtin_amdgcn_sched_barrier(0);
    PPRVIZ_ACC(0, w0) PPRVIZ_ACC(1, w1) PPRVIZ_ACC(2, w2) PPRVIZ_ACC(3, w3)
    PPRVIZ_ACC(4, w0) PPRVIZ_ACC(5, w1) PPRVIZ_ACC(6, w2) PPRVIZ_ACC(7, w3)
    if (NH == 1) return;
    __builtin_amdgcn_sched_barrier(0);
    PPRVIZ_RD(8, a0) PPRVIZ_RD(9, a1) PPRVIZ_RD(10, a2) PPRVIZ_RD(11, a3)
    PPRVIZ_RD(12, a0) PPRVIZ_RD(13, a1) PPRVIZ_RD(14, a2) PPRVIZ_RD(15, a3)
    __builtin_amdgcn_sched_barrier(0);
    PPRVIZ_ACC(8, w0) PPRVIZ_ACC(9, w1) PPRVIZ_ACC(10, w2) PPRVIZ_ACC(11, w3)
    PPRVIZ_ACC(12, w0) PPRVIZ_ACC(13, w1) PPRVIZ_ACC(14, w2) PPRVIZ_ACC(15, w3)
#undef PPRVIZ_RD
#undef PPRVIZ_ACC
}

// Keeps a value opaque to the optimizer, so that per-row loads and addresses
// are recomputed inside each step instead of being hoisted out of the step
// loop (where 18 rows' worth of them would no longer fit in registers).
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ int opaque_s32(int v) {
    v = __builtin_amdgcn_readfirstlane(v);
    asm volatile("" : "+s"(v));
    return v;
}
__device__ __forceinline__ int64_t opaque_s(int64_t v) {
    int lo = __builtin_amdgcn_readfirstlane((int)v);
    int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// LDS of one resident tile: the iterate Y (n rows of COLS floats and a zero
// row) followed by the n per-node factors (1-alpha)/d.
struct ResLds {
    float y[kResLdsFloats];
    float scale[Res<16>::NMAX];
};

// Loads one 16-arc chunk of a quad's row (arcs e0 + 4i + q for i = 0..3).
// Rows of the arc copy are padded with the zero row's offset to at least 16
// arcs and to a multiple of 8, and a later chunk with at most 8 arcs left
// uses only lanes 0 and 1, so every arc the gather uses is a real arc or the
// zero row: no bound checks.
template <bool WEIGHTED>
__device__ __forceinline__ void load_chunk(gcptr<int32_t> pc, gcptr<float> pw, int e0, int q, int& r0, int& r1,
                                           int& r2, int& r3, float& w0, float& w1, float& w2, float& w3) {
    // lane q takes the 4 consecutive arcs e0 + 4q .. e0 + 4q + 3; the arc
    // array is padded by 16 entries, so the loads need no guard
    const int e = e0 + 4 * q;
    r0 = pc[e];
    r1 = pc[e + 1];
    r2 = pc[e + 2];
    r3 = pc[e + 3];
    if (WEIGHTED) {
        w0 = pw[e];
        w1 = pw[e + 1];
        w2 = pw[e + 2];
        w3 = pw[e + 3];
    }
}

// All T pushes for one source tile with the tile's iterate resident in LDS.
// Each lane keeps its rows' new values (4 columns per row) in registers
// between the two barriers of a step.
template <int COLS, bool WEIGHTED>
__device__ __forceinline__ void res_tile(const TileTask& t, const ResArgs& a, ResLds& L) {
    constexpr int QPR = Res<COLS>::QPR;
    constexpr int RPW = Res<COLS>::RPW;
    constexpr int RPP = Res<COLS>::RPP;
    constexpr int STRIDE = Res<COLS>::STRIDE;
    float* __restrict__ lds = L.y;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int quad = lane >> 2;
    const int q = lane & 3;
    const int rsub = quad / QPR;                 // row slot of the quad in the wave
    const int col0 = (quad % QPR) * 16 + q * 4;  // first of the lane's 4 columns
    const int cbyte = col0 * 4;
    const int n = t.n;
    const int64_t base = t.base;
    const float alpha = a.alpha;
    const float oma = 1.0f - alpha;
    const gcptr<int32_t> rp = as_global(a.row_ptr);
    const gcptr<int32_t> pc = as_global(a.col_idx);
    const gcptr<float> pw = as_global(a.weight);
    const gcptr<int32_t> srcp = as_global(a.src);

    // local source node of each of the lane's 4 columns (-1 outside the tile)
    int msrc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = col0 + i;
        msrc[i] = c < t.ncols ? (a.src ? srcp[t.s0 + c] : t.s0 + c) : -1;
    }

    for (int i = tid; i < (n + 1) * COLS; i += kResThreads) lds[i] = 0.f;
    for (int i = tid; i < n; i += kResThreads) L.scale[i] = oma * as_global(a.invd)[base + i];
    __syncthreads();
    if (tid < t.ncols && a.T >= 2) {
        int s = a.src ? srcp[t.s0 + tid] : t.s0 + tid;
        lds[s * COLS + tid] = alpha * L.scale[s];
    }
    __syncthreads();

    float4 xr[kResMaxK];
    int vs[kResMaxK];  // row id of each slot
    const int row0 = wave * RPW + rsub;  // slot of pass k is row0 + k * RPP
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) {
        const int slot = row0 + k * RPP;
        const int v = slot < n ? as_global(a.rows)[base + slot].v : -1;
        vs[k] = v;
        const bool on = a.T >= 1;
        xr[k] = make_float4(on && v == msrc[0] ? alpha : 0.f, on && v == msrc[1] ? alpha : 0.f,
                            on && v == msrc[2] ? alpha : 0.f, on && v == msrc[3] ? alpha : 0.f);
    }

    const gcptr<RowEnt> rows = as_global(a.rows);
    for (int it = 1; it < a.T; ++it) {
        const int r0 = opaque(row0);
        const int64_t b = opaque_s(base);
        const int n = opaque_s32(t.n);
        // Rows are visited in slot order (degree-sorted, so the rows that
        // share a pass have similar length).  Row-level software pipeline:
        // the first chunk of slot k+1 and the table entry of slot k+2 are
        // loaded while slot k is summed.
        RowEnt e1 = {0, 0, 0, 0}, e2 = {0, 0, 0, 0};
        if (r0 < n) e1 = load_row(rows, b + r0);
        if (r0 + RPP < n) e2 = load_row(rows, b + r0 + RPP);
        int p0 = 0, p1 = 0, p2 = 0, p3 = 0;
        float pw0 = 0.f, pw1 = 0.f, pw2 = 0.f, pw3 = 0.f;
        load_chunk<WEIGHTED>(pc, pw, e1.rs, q, p0, p1, p2, p3, pw0, pw1, pw2, pw3);
#pragma unroll
        for (int k = 0; k < kResMaxK; ++k) {
            if (k * RPP < n) {
                const int slot = r0 + k * RPP;
                const int rs = e1.rs, re = e1.re, v = e1.v;
                const int c0 = p0, c1 = p1, c2 = p2, c3 = p3;
                const float cw0 = pw0, cw1 = pw1, cw2 = pw2, cw3 = pw3;
                e1 = e2;
                if (k + 1 < kResMaxK && slot + RPP < n)
                    load_chunk<WEIGHTED>(pc, pw, e1.rs, q, p0, p1, p2, p3, pw0, pw1, pw2, pw3);
                if (k + 2 < kResMaxK && slot + 2 * RPP < n) e2 = load_row(rows, b + slot + 2 * RPP);
                if (slot < n) {
                    vs[k] = v;
                    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (rs == re) acc = lds_load4(lds, v * STRIDE + cbyte);
                    if (rs < re) {
                        gather_chunk<WEIGHTED, 2>(lds, c0, c1, c2, c3, cw0, cw1, cw2, cw3, cbyte, acc);
                    }
                    // further chunks of rows longer than 16 arcs; a tail of
                    // at most 8 arcs takes a half chunk
#pragma nounroll
                    for (int e0 = rs + 16; e0 < re; e0 += 16) {
                        int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
                        float dw0 = 0.f, dw1 = 0.f, dw2 = 0.f, dw3 = 0.f;
                        load_chunk<WEIGHTED>(pc, pw, e0, q, d0, d1, d2, d3, dw0, dw1, dw2, dw3);
                        if (re - e0 > 8) {
                            gather_chunk<WEIGHTED, 2>(lds, d0, d1, d2, d3, dw0, dw1, dw2, dw3, cbyte, acc);
                        } else {
                            gather_chunk<WEIGHTED, 1>(lds, d0, d1, d2, d3, dw0, dw1, dw2, dw3, cbyte, acc);
                        }
                    }
                    acc.x += v == msrc[0] ? alpha : 0.f;
                    acc.y += v == msrc[1] ? alpha : 0.f;
                    acc.z += v == msrc[2] ? alpha : 0.f;
                    acc.w += v == msrc[3] ? alpha : 0.f;
                    xr[k] = acc;
                }
            }
        }
        // the slots' scales (constant for the tile) are read before the
        // barrier, all at once, instead of one LDS round trip per slot after it
        float sc[kResMaxK];
#pragma unroll
        for (int k = 0; k < kResMaxK; ++k) sc[k] = L.scale[max(vs[k], 0)];
        __syncthreads();
        const int r1 = opaque(row0);
        const int n1 = opaque_s32(t.n);
#pragma unroll
        for (int k = 0; k < kResMaxK; ++k) {
            if (k * RPP < n1) {
                const int slot = r1 + k * RPP;
                if (slot < n1) {
                    const int v = vs[k];
                    *reinterpret_cast<float4*>(reinterpret_cast<char*>(lds) + v * STRIDE + cbyte) =
                        make_float4(xr[k].x * sc[k], xr[k].y * sc[k], xr[k].z * sc[k], xr[k].w * sc[k]);
                }
            }
        }
        __syncthreads();
    }

    // Epilogue.  FP64 residual 1 - sum_v pi_hat(s, v): per-column partial sums
    // go through the (no longer needed) iterate area; then the unscaled
    // iterate is written column-swizzled so that the transposed read below is
    // conflict-free.
    double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) {
        const int slot = row0 + k * RPP;
        if (k * RPP < n && slot < n) {
            part[0] += (double)xr[k].x;
            part[1] += (double)xr[k].y;
            part[2] += (double)xr[k].z;
            part[3] += (double)xr[k].w;
        }
    }
    // lanes holding the same columns: same (quad % QPR, q), other row slots
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int o = 4 * QPR; o < kWave; o <<= 1) part[i] += __shfl_xor(part[i], o, kWave);
    }
    double* red = reinterpret_cast<double*>(lds);
    __syncthreads();
    if (rsub == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wave * COLS + col0 + i] = part[i];
    }
    __syncthreads();
    if (tid < t.ncols && a.resid) {
        double s = 0.0;
        for (int w = 0; w < kResWaves; ++w) s += red[w * COLS + tid];
        as_global_w(a.resid)[t.s0 + tid] = 1.0 - s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) {
        const int slot = row0 + k * RPP;
        if (k * RPP < n && slot < n) {
            const int v = vs[k];
            const int sw = v & (COLS - 1);
            lds[v * COLS + ((col0 + 0) ^ sw)] = xr[k].x;
            lds[v * COLS + ((col0 + 1) ^ sw)] = xr[k].y;
            lds[v * COLS + ((col0 + 2) ^ sw)] = xr[k].z;
            lds[v * COLS + ((col0 + 3) ^ sw)] = xr[k].w;
        }
    }
    __syncthreads();
    if (a.ppr_out || a.dppr_out) {
        for (int ci = 0; ci < t.ncols; ++ci) {
            const int s_local = a.src ? srcp[t.s0 + ci] : t.s0 + ci;
            const float dsc = as_global(a.deg)[base + s_local];
            const int64_t row = t.out_off + (int64_t)(t.s0 + ci) * t.ld;
            for (int j = tid; j < t.n_tgt; j += kResThreads) {
                const int tn = a.tgt ? as_global(a.tgt)[j] : j;
                const float x = lds[tn * COLS + (ci ^ (tn & (COLS - 1)))];
                if (a.ppr_out) as_global_w(a.ppr_out)[row + j] = x;
                if (a.dppr_out) as_global_w(a.dppr_out)[row + j] = x * dsc;
            }
        }
    }
    __syncthreads();
}

// Slot order of the rows of each graph for the resident tile: rows sorted by
// degree, longest first (ties by row id); one block per graph.  node_off ==
// nullptr means a single graph of n_single nodes.
__global__ void row_table_kernel(const int32_t* __restrict__ row_ptr, const int64_t* __restrict__ node_off,
                                 int32_t n_single, RowEnt* __restrict__ table);

// Degree and inverse degree of every node (the d of Definition def:pprdist is
// the out-degree; with weights, the sum of the node's arc weights).
__global__ void degree_kernel(const int32_t* __restrict__ row_ptr, const float* __restrict__ weight,
                              int64_t n, float* __restrict__ deg, float* __restrict__ invd);

}  // namespace pprviz
