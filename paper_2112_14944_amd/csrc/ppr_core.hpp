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

constexpr int kResThreads = 1024;
constexpr int kResWaves = kResThreads / kWave;
constexpr int kResMaxK = 36;  // rows per lane held in registers across a step

template <int COLS>
struct Res {
    static constexpr int RPW = kWave / COLS;               // rows per wave per pass
    static constexpr int RPP = kResWaves * RPW;            // rows per block pass
    static constexpr int NMAX = RPP * kResMaxK;            // largest graph for this tile width
    static constexpr int STRIDE = COLS * 4;                // bytes per LDS row
};

// LDS floats for one resident tile: (NMAX + 1 dummy zero row) * COLS, max over
// the three tile widths (577*64, 1153*32, 2305*16).
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

struct ResArgs {
    const int32_t* row_ptr;  // global CSR row pointers
    const int32_t* col_idx;  // global node ids
    const float* weight;     // arc weights or nullptr
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

// Sum of Y[u][c] over 16 arcs whose LDS row offsets (bytes) sit in the 16
// lanes of each DPP row; lanes past the row's end point at the zero row.
template <bool WEIGHTED>
__device__ __forceinline__ float gather16(const float* __restrict__ lds, int off, float w, int c4) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#define PPRVIZ_G(J, ACC)                                                   \
    {                                                                      \
        int o = row_bcast<J>(off);                                         \
        float x = lds_load(lds, o + c4);                                   \
        if (WEIGHTED) ACC = fmaf(row_bcast<J>(w), x, ACC); else ACC += x; \
    }
    PPRVIZ_G(0, s0) PPRVIZ_G(1, s1) PPRVIZ_G(2, s2) PPRVIZ_G(3, s3)
    PPRVIZ_G(4, s0) PPRVIZ_G(5, s1) PPRVIZ_G(6, s2) PPRVIZ_G(7, s3)
    PPRVIZ_G(8, s0) PPRVIZ_G(9, s1) PPRVIZ_G(10, s2) PPRVIZ_G(11, s3)
    PPRVIZ_G(12, s0) PPRVIZ_G(13, s1) PPRVIZ_G(14, s2) PPRVIZ_G(15, s3)
#undef PPRVIZ_G
    return (s0 + s1) + (s2 + s3);
}

// Keeps a value opaque to the optimizer, so that per-row loads and addresses
// are recomputed inside each step instead of being hoisted out of the step
// loop (where 36 rows' worth of them would no longer fit in registers).
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ int64_t opaque_s(int64_t v) {
    int lo = __builtin_amdgcn_readfirstlane((int)v);
    int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// LDS of one resident tile: the iterate Y (n+1 rows of COLS floats, the last
// row all zero) followed by the n per-node factors (1-alpha)/d.
struct ResLds {
    float y[kResLdsFloats];
    float scale[Res<16>::NMAX];
};

// All T pushes for one source tile with the tile's iterate resident in LDS.
// Block = 1024 threads; lane c = lane % COLS is the tile column (source), a
// wave covers 64/COLS rows per pass, and each lane keeps its rows' new values
// in registers between the two barriers of a step.
template <int COLS, bool WEIGHTED>
__device__ void res_tile(const TileTask& t, const ResArgs& a, ResLds& L) {
    constexpr int RPW = Res<COLS>::RPW;
    constexpr int RPP = Res<COLS>::RPP;
    constexpr int STRIDE = Res<COLS>::STRIDE;
    float* __restrict__ lds = L.y;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int c = lane % COLS;
    const int rsub = lane / COLS;
    const int c4 = c * 4;
    const int l16 = lane & 15;
    const int n = t.n;
    const int64_t base = t.base;
    const float alpha = a.alpha;
    const float oma = 1.0f - alpha;
    const int dummy = n * STRIDE;

    int my_src = -1;
    if (c < t.ncols) my_src = a.src ? a.src[t.s0 + c] : t.s0 + c;

    for (int i = tid; i < (n + 1) * COLS; i += kResThreads) lds[i] = 0.f;
    for (int i = tid; i < n; i += kResThreads) L.scale[i] = oma * a.invd[base + i];
    __syncthreads();
    if (tid < t.ncols && a.T >= 2) {
        int s = a.src ? a.src[t.s0 + tid] : t.s0 + tid;
        lds[s * COLS + tid] = alpha * L.scale[s];
    }
    __syncthreads();

    float xr[kResMaxK];
    const int row0 = wave * RPW + rsub;  // row of pass k is row0 + k * RPP
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) xr[k] = (a.T >= 1 && row0 + k * RPP == my_src) ? alpha : 0.f;

    for (int it = 1; it < a.T; ++it) {
        const int r0 = opaque(row0);
        const int64_t b = opaque_s(base);
#pragma unroll
        for (int k = 0; k < kResMaxK; ++k) {
            if (k * RPP < n) {
                const int v = r0 + k * RPP;
                if (v < n) {
                    const int rs = a.row_ptr[b + v];
                    const int re = a.row_ptr[b + v + 1];
                    float acc = 0.f;
                    if (rs == re) acc = lds[v * COLS + c];
                    for (int e0 = rs; e0 < re; e0 += 16) {
                        const int e = e0 + l16;
                        int off = dummy;
                        float w = 0.f;
                        if (e < re) {
                            off = (int)(a.col_idx[e] - b) * STRIDE;
                            if (WEIGHTED) w = a.weight[e];
                        }
                        acc += gather16<WEIGHTED>(lds, off, w, c4);
                    }
                    xr[k] = acc + (v == my_src ? alpha : 0.f);
                }
            }
        }
        __syncthreads();
        const int r1 = opaque(row0);
#pragma unroll
        for (int k = 0; k < kResMaxK; ++k) {
            if (k * RPP < n) {
                const int v = r1 + k * RPP;
                if (v < n) lds[v * COLS + c] = xr[k] * L.scale[v];
            }
        }
        __syncthreads();
    }

    // Epilogue.  FP64 residual 1 - sum_v pi_hat(s, v): per-wave partials go
    // to the (no longer needed) iterate area, then the unscaled iterate is
    // written column-swizzled so that the transposed read below is
    // conflict-free.
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) {
        const int v = row0 + k * RPP;
        if (k * RPP < n && v < n) part += (double)xr[k];
    }
#pragma unroll
    for (int o = COLS; o < kWave; o <<= 1) part += __shfl_xor(part, o, kWave);
    double* red = reinterpret_cast<double*>(lds);
    __syncthreads();
    if (rsub == 0) red[wave * kWave + c] = part;
    __syncthreads();
    if (tid < t.ncols && a.resid) {
        double s = 0.0;
        for (int w = 0; w < kResWaves; ++w) s += red[w * kWave + tid];
        a.resid[t.s0 + tid] = 1.0 - s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) {
        const int v = row0 + k * RPP;
        if (k * RPP < n && v < n) lds[v * COLS + (c ^ (v & (COLS - 1)))] = xr[k];
    }
    __syncthreads();
    if (a.ppr_out || a.dppr_out) {
        for (int ci = 0; ci < t.ncols; ++ci) {
            const int s_local = a.src ? a.src[t.s0 + ci] : t.s0 + ci;
            const float dsc = a.deg[base + s_local];
            const int64_t row = t.out_off + (int64_t)(t.s0 + ci) * t.ld;
            for (int j = tid; j < t.n_tgt; j += kResThreads) {
                const int tn = a.tgt ? a.tgt[j] : j;
                const float x = lds[tn * COLS + (ci ^ (tn & (COLS - 1)))];
                if (a.ppr_out) a.ppr_out[row + j] = x;
                if (a.dppr_out) a.dppr_out[row + j] = x * dsc;
            }
        }
    }
    __syncthreads();
}

// Degree and inverse degree of every node (the d of Definition def:pprdist is
// the out-degree; with weights, the sum of the node's arc weights).
__global__ void degree_kernel(const int32_t* __restrict__ row_ptr, const float* __restrict__ weight,
                              int64_t n, float* __restrict__ deg, float* __restrict__ invd);

}  // namespace pprviz
