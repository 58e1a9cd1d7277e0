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
constexpr int kResMaxK = 9;  // passes (row groups per wave) held in registers across a step

// Tile geometry.  Lanes work in quads: a quad owns 16 columns of one row, each
// lane 4 consecutive columns read with one 16-byte LDS load per arc, and the
// quad's arcs are broadcast inside the quad with DPP quad_perm.  A row of a
// COLS-wide tile takes COLS/16 quads; a wave takes RPW rows side by side (a
// group) per pass.
template <int COLS>
struct Res {
    static constexpr int QPR = COLS / 16;                  // quads per row
    static constexpr int RPW = 16 / QPR;                   // rows per wave per pass (group size)
    static constexpr int RPP = kResWaves * RPW;            // rows per block pass
    static constexpr int NMAX = RPP * kResMaxK;            // largest graph for this tile width
    static constexpr int STRIDE = COLS * 4;                // bytes per LDS row
};

// LDS floats for one resident tile: n rows plus one zero row per LDS bank
// class (4, 2, 1 for 16, 32, 64 columns: 64 floats in every case), times
// COLS; the maximum over the three tile widths (577*64, 1154*32, 2308*16).
constexpr int kResZeroFloats = 64;
constexpr int kResLdsFloats = 36928;
static_assert(Res<64>::NMAX * 64 + kResZeroFloats <= kResLdsFloats, "lds");
static_assert(Res<32>::NMAX * 32 + kResZeroFloats <= kResLdsFloats, "lds");
static_assert(Res<16>::NMAX * 16 + kResZeroFloats <= kResLdsFloats, "lds");

__host__ __device__ inline int res_cols_for(int n) {
    return n <= Res<64>::NMAX ? 64 : (n <= Res<32>::NMAX ? 32 : (n <= Res<16>::NMAX ? 16 : 0));
}

// Group layout of the resident tile (res_layout_kernel).  The slots of a
// graph are its rows in degree order, longest first; slots g*RPW .. g*RPW +
// RPW - 1 form group g, the rows one wave sums side by side in one pass.
// Every row of a group is padded (with the tile's zero row) to the length of
// the group's longest row, rounded up to 8 arcs, so all lanes of a pass run
// the same number of 16-arc chunks (the last one half full when the count of
// 8-arc halves is odd) under scalar control.  The group's arcs are stored
// chunk-major: entry j of chunk c of the group's row r sits at
//     off(g) + 16 RPW c + 16 r + j,
// so a lane's 4 arcs of a chunk are one 16-byte load at a lane-constant
// offset plus a scalar one.  A row without arcs gets one arc to itself (its
// own mass stays put, the self-loop convention).  Padding reads one of the
// tile's zero rows (one per LDS bank class, rows n .. n + 64/COLS - 1).
// Slots past the last row (the end of the last group) are dummies: every arc
// is a zero row and the row they write back is zero row n itself, with
// zeros.
constexpr int kResTabPad = 16;        // slot-table entries per graph beyond its n rows
constexpr int kResArcPerNode = 32;    // arc-copy entries per node beyond its arcs
constexpr int kResArcPerGraph = 256;  // and per graph
constexpr int kResMaxGroups = Res<16>::NMAX / Res<16>::RPW;
static_assert(Res<32>::NMAX / Res<32>::RPW == kResMaxGroups && Res<64>::NMAX / Res<64>::RPW == kResMaxGroups,
              "groups");

// Arc-copy entries reserved for a graph of n nodes and nnz arcs.  With the
// rows sorted longest first, group g >= 1 is padded to a length no longer
// than any row of group g - 1, so the padded groups hold at most
// RPW * dmax + nnz + n entries (the n for the self arcs), plus at most 15 per
// row for rounding to whole chunks: below nnz + 32 n + 256 whenever dmax <= n
// (no repeated arcs).  A graph that needs more (repeated arcs) gets a
// minimal layout and NaN scales, so its outputs are NaN.
__host__ __device__ inline int64_t res_arc_words(int64_t nnz, int64_t n) {
    return nnz + kResArcPerNode * n + kResArcPerGraph;
}

// Slot-table entry of the resident tile.
struct __attribute__((aligned(16))) ResSlot {
    int32_t off;     // arc-copy entry of the slot's row, chunk 0, relative to the graph's copy
    int32_t halves;  // 8-arc halves of every row of the slot's group (>= 1)
    int32_t v;       // row id (local to its graph); n for a dummy slot
    float invd;      // 1/d of the row (0 for a dummy slot)
};

// Row entry of the mid-size and streaming kernels' row orders.
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

// One source tile of one graph.
struct TileTask {
    int32_t n;        // node count of the graph
    int32_t s0;       // first source index of the tile
    int32_t ncols;    // sources in the tile (<= COLS)
    int32_t n_tgt;    // output columns
    int64_t base;     // global id of the graph's node 0
    int64_t out_off;  // offset of output row 0
    int64_t ld;       // output leading dimension
    int64_t tbase;    // first slot-table entry of the graph
    int64_t cbase;    // first arc-copy entry of the graph
    int32_t cwords;   // arc-copy entries of the graph (res_arc_words)
};

// Where graph g's slot table and arc copy start, for a graph whose nodes start
// at global id `base` and whose arcs start at CSR position e0.
__host__ __device__ inline void res_graph_bases(int64_t base, int64_t e0, int64_t e1, int64_t g, int32_t n,
                                                TileTask& t) {
    t.tbase = base + kResTabPad * g;
    t.cbase = e0 + kResArcPerNode * base + kResArcPerGraph * g;
    t.cwords = (int32_t)res_arc_words(e1 - e0, n);
}

struct ResArgs {
    const ResSlot* slots;    // per graph: slot table in group layout (res_layout_kernel)
    const int32_t* arcs;     // arc copy in group layout: LDS byte offset of each arc's neighbour row
    const float* warcs;      // arc weights in the same layout, or nullptr
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

// Keeps a value opaque to the optimizer, so that per-row loads and addresses
// are recomputed inside a loop instead of being hoisted out of it (where many
// rows' worth of them would no longer fit in registers).
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

// A pointer or count the caller knows to be wave-uniform, moved to scalar
// registers (a buffer resource built from values in vector registers is
// otherwise taken lane by lane, one load per distinct value).
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

// 16-byte load through a buffer resource (offsets in bytes; soff must be
// wave-uniform).
__device__ __forceinline__ int4 buf_load_i4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    return make_int4((int)v[0], (int)v[1], (int)v[2], (int)v[3]);
}
// A group's arc start and length: its first slot entry, the same for all
// lanes.
__device__ __forceinline__ int2 grp_load(__amdgpu_buffer_rsrc_t r, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, 0, (int)soff, 0);
    return make_int2((int)v[0], (int)v[1]);
}
__device__ __forceinline__ float4 buf_load_f4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    return make_float4(__int_as_float(v[0]), __int_as_float(v[1]), __int_as_float(v[2]), __int_as_float(v[3]));
}

// One chunk of 16 arcs of a quad's row (8 when `half`, a wave-uniform flag):
// arc 4L + W sits in lane L, word W (a.x..a.w hold LDS byte offsets of the
// neighbours' rows, the zero row past the row's end), so the arcs are summed
// in row order.  Eight 16-byte reads are issued before their adds.
template <bool WEIGHTED>
__device__ __forceinline__ void gather_chunk(const float* __restrict__ lds, int4 a, float4 w, int cbyte, bool half,
                                             float4& acc) {
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
    PPRVIZ_RD(0, a.x) PPRVIZ_RD(1, a.y) PPRVIZ_RD(2, a.z) PPRVIZ_RD(3, a.w)
    PPRVIZ_RD(4, a.x) PPRVIZ_RD(5, a.y) PPRVIZ_RD(6, a.z) PPRVIZ_RD(7, a.w)
    __builtin_amdgcn_sched_barrier(0);
    PPRVIZ_ACC(0, w.x) PPRVIZ_ACC(1, w.y) PPRVIZ_ACC(2, w.z) PPRVIZ_ACC(3, w.w)
    PPRVIZ_ACC(4, w.x) PPRVIZ_ACC(5, w.y) PPRVIZ_ACC(6, w.z) PPRVIZ_ACC(7, w.w)
    if (half) return;
    __builtin_amdgcn_sched_barrier(0);
    PPRVIZ_RD(8, a.x) PPRVIZ_RD(9, a.y) PPRVIZ_RD(10, a.z) PPRVIZ_RD(11, a.w)
    PPRVIZ_RD(12, a.x) PPRVIZ_RD(13, a.y) PPRVIZ_RD(14, a.z) PPRVIZ_RD(15, a.w)
    __builtin_amdgcn_sched_barrier(0);
    PPRVIZ_ACC(8, w.x) PPRVIZ_ACC(9, w.y) PPRVIZ_ACC(10, w.z) PPRVIZ_ACC(11, w.w)
    PPRVIZ_ACC(12, w.x) PPRVIZ_ACC(13, w.y) PPRVIZ_ACC(14, w.z) PPRVIZ_ACC(15, w.w)
#undef PPRVIZ_RD
#undef PPRVIZ_ACC
}

// LDS of one resident tile: the iterate Y (n rows of COLS floats and the zero
// rows).
struct ResLds {
    float y[kResLdsFloats];
};

constexpr int kBufFlags = 0x00020000;  // buffer resource word 3: 32-bit data, no swizzle

// All T pushes for one source tile with the tile's iterate resident in LDS.
// Each lane keeps its rows' new values (4 columns per row) in registers
// between the two barriers of a step.  Pass k of wave w sums group
// w + 16 k of the slot table; all control flow inside a step is wave-uniform.
template <int COLS, bool WEIGHTED>
__device__ __forceinline__ void res_tile(const TileTask& t, const ResArgs& a, ResLds& L) {
    constexpr int QPR = Res<COLS>::QPR;
    constexpr int RPW = Res<COLS>::RPW;
    constexpr int STRIDE = Res<COLS>::STRIDE;
    constexpr uint32_t kChunkBytes = 64u * RPW;  // one 16-arc chunk of a group
    constexpr uint32_t kGroupBytes = 16u * RPW;  // one group's slot entries
    float* __restrict__ lds = L.y;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int quad = lane >> 2;
    const int q = lane & 3;
    const int rsub = quad / QPR;                 // row of the quad in its group
    const int col0 = (quad % QPR) * 16 + q * 4;  // first of the lane's 4 columns
    const int cbyte = col0 * 4;
    const int n = __builtin_amdgcn_readfirstlane(t.n);
    const int ngroups = (n + RPW - 1) / RPW;
    const int cbytes = __builtin_amdgcn_readfirstlane(t.cwords) * 4;
    const float alpha = a.alpha;
    const float oma = 1.0f - alpha;
    const gcptr<int32_t> srcp = as_global(a.src);
    const __amdgpu_buffer_rsrc_t tab = __builtin_amdgcn_make_buffer_rsrc(
        uniform_ptr(const_cast<ResSlot*>(a.slots + t.tbase)), 0, ngroups * (int)kGroupBytes, kBufFlags);
    const __amdgpu_buffer_rsrc_t arc =
        __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(const_cast<int32_t*>(a.arcs + t.cbase)), 0, cbytes, kBufFlags);
    __amdgpu_buffer_rsrc_t warc = arc;
    if (WEIGHTED)
        warc = __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(const_cast<float*>(a.warcs + t.cbase)), 0, cbytes,
                                                 kBufFlags);
    const uint32_t tvoff = (uint32_t)rsub * 16u;                // the lane's slot entry within its group
    const uint32_t lane_arc = (uint32_t)rsub * 64u + q * 16u;  // the lane's 4 arcs within a chunk

    // local source node of each of the lane's 4 columns (-1 outside the tile)
    int msrc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = col0 + i;
        msrc[i] = c < t.ncols ? (a.src ? srcp[t.s0 + c] : t.s0 + c) : -1;
    }

    // Per pass: the LDS byte address the row's 4 columns are stored to, the
    // row's scale (1 - alpha)/d, and which of the lane's columns have the
    // row as their source (4 bits per pass).
    int vaddr[kResMaxK];
    float sc[kResMaxK];
    float4 xr[kResMaxK];
    uint32_t sbits_lo = 0, sbits_hi = 0;
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) {
        vaddr[k] = n * STRIDE + cbyte;
        sc[k] = 0.f;
        xr[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        if ((wave + kResWaves * k) * RPW < n) {
            const int4 e = buf_load_i4(tab, tvoff, (uint32_t)(wave + kResWaves * k) * kGroupBytes);
            vaddr[k] = e.z * STRIDE + cbyte;
            sc[k] = oma * __int_as_float(e.w);
            const uint32_t bits = (e.z == msrc[0] ? 1u : 0u) | (e.z == msrc[1] ? 2u : 0u) |
                                  (e.z == msrc[2] ? 4u : 0u) | (e.z == msrc[3] ? 8u : 0u);
            if (k < 8) sbits_lo |= bits << (4 * k); else sbits_hi |= bits << (4 * (k - 8));
            if (a.T >= 1)
                xr[k] = make_float4(bits & 1u ? alpha : 0.f, bits & 2u ? alpha : 0.f, bits & 4u ? alpha : 0.f,
                                    bits & 8u ? alpha : 0.f);
        }
    }
    // Y_0 = scale * X_0: every row is written by the lanes of its slot; the
    // zero rows are cleared (dummy slots write zeros into the first as well)
    for (int i = tid; i < kResZeroFloats; i += kResThreads) lds[n * COLS + i] = 0.f;
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) {
        if ((wave + kResWaves * k) * RPW < n)
            *reinterpret_cast<float4*>(reinterpret_cast<char*>(lds) + vaddr[k]) =
                make_float4(xr[k].x * sc[k], xr[k].y * sc[k], xr[k].z * sc[k], xr[k].w * sc[k]);
    }
    __syncthreads();

    for (int it = 1; it < a.T; ++it) {
        // Chunk-level software pipeline: the arcs of the next chunk (of this
        // pass, else the first of the next pass) are loaded while the current
        // chunk is summed, alternating between two register sets.  A lane's 4
        // arcs of any chunk sit at the lane-constant offset lane_arc from the
        // chunk's start, so every arc load takes a scalar offset: the group's
        // start g4 (bytes) plus the chunk's.  A group's start and length are
        // loaded two passes ahead of their use.
        int4 A = make_int4(0, 0, 0, 0), B = A;
        float4 WA = make_float4(0.f, 0.f, 0.f, 0.f), WB = WA;
        int2 e1 = make_int2(0, 1);
        uint32_t g4 = 0;
        int h = 1;
        if (wave * RPW < n) {
            const int2 e0 = grp_load(tab, (uint32_t)wave * kGroupBytes);
            if ((wave + kResWaves) * RPW < n) e1 = grp_load(tab, (uint32_t)(wave + kResWaves) * kGroupBytes);
            g4 = (uint32_t)__builtin_amdgcn_readfirstlane(e0.x) * 4u;
            h = __builtin_amdgcn_readfirstlane(e0.y);
            A = buf_load_i4(arc, lane_arc, g4);
            if (WEIGHTED) WA = buf_load_f4(warc, lane_arc, g4);
        }
        // the source bits are re-read each step, so that their tests stay in
        // vector registers instead of being hoisted into scalar masks
        const uint32_t sl = (uint32_t)opaque((int)sbits_lo);
        const uint32_t sh = (uint32_t)opaque((int)sbits_hi);
#pragma unroll
        for (int k = 0; k < kResMaxK; ++k) {
            const int gk = wave + kResWaves * k;
            if (gk * RPW < n) {
                const bool nxt = k + 1 < kResMaxK && (gk + kResWaves) * RPW < n;
                int2 e2 = make_int2(0, 1);
                if (k + 2 < kResMaxK && (gk + 2 * kResWaves) * RPW < n)
                    e2 = grp_load(tab, (uint32_t)(gk + 2 * kResWaves) * kGroupBytes);
                // next pass's start (this pass's own when there is none: the
                // last prefetch then reloads a chunk already read)
                const uint32_t g4n = nxt ? (uint32_t)__builtin_amdgcn_readfirstlane(e1.x) * 4u : g4;
                const int hn = __builtin_amdgcn_readfirstlane(e1.y);
                const int nch = (h + 1) >> 1;
                const bool odd = (h & 1) != 0;
                float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
                // chunks in pairs: A holds chunk c, B chunk c + 1
                for (int c = 0;; c += 2) {
                    const bool has1 = c + 1 < nch;
                    const uint32_t s1 = has1 ? g4 + (uint32_t)(c + 1) * kChunkBytes : g4n;
                    B = buf_load_i4(arc, lane_arc, s1);
                    if (WEIGHTED) WB = buf_load_f4(warc, lane_arc, s1);
                    gather_chunk<WEIGHTED>(lds, A, WA, cbyte, !has1 && odd, acc);
                    if (!has1) {
                        A = B;  // the next pass's first chunk
                        WA = WB;
                        break;
                    }
                    const bool has2 = c + 2 < nch;
                    const uint32_t s2 = has2 ? g4 + (uint32_t)(c + 2) * kChunkBytes : g4n;
                    A = buf_load_i4(arc, lane_arc, s2);
                    if (WEIGHTED) WA = buf_load_f4(warc, lane_arc, s2);
                    gather_chunk<WEIGHTED>(lds, B, WB, cbyte, !has2 && odd, acc);
                    if (!has2) break;
                }
                const uint32_t sb = (k < 8 ? sl >> (4 * k) : sh >> (4 * (k - 8))) & 15u;
                if (sb) {
                    acc.x += (sb & 1u) ? alpha : 0.f;
                    acc.y += (sb & 2u) ? alpha : 0.f;
                    acc.z += (sb & 4u) ? alpha : 0.f;
                    acc.w += (sb & 8u) ? alpha : 0.f;
                }
                xr[k] = acc;
                g4 = g4n;
                h = hn;
                e1 = e2;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kResMaxK; ++k) {
            if ((wave + kResWaves * k) * RPW < n)
                *reinterpret_cast<float4*>(reinterpret_cast<char*>(lds) + vaddr[k]) =
                    make_float4(xr[k].x * sc[k], xr[k].y * sc[k], xr[k].z * sc[k], xr[k].w * sc[k]);
        }
        __syncthreads();
    }

    // Epilogue.  FP64 residual 1 - sum_v pi_hat(s, v): per-column partial sums
    // go through the (no longer needed) iterate area; then the unscaled
    // iterate is written column-swizzled so that the transposed read below is
    // conflict-free.  Dummy slots hold zeros and add nothing.
    double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kResMaxK; ++k) {
        if ((wave + kResWaves * k) * RPW < n) {
            part[0] += (double)xr[k].x;
            part[1] += (double)xr[k].y;
            part[2] += (double)xr[k].z;
            part[3] += (double)xr[k].w;
        }
    }
    // lanes holding the same columns: same (quad % QPR, q), other rows
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
        if ((wave + kResWaves * k) * RPW < n) {
            const int v = (vaddr[k] - cbyte) / STRIDE;
            const int sw = v & (COLS - 1);
            lds[v * COLS + ((col0 + 0) ^ sw)] = xr[k].x;
            lds[v * COLS + ((col0 + 1) ^ sw)] = xr[k].y;
            lds[v * COLS + ((col0 + 2) ^ sw)] = xr[k].z;
            lds[v * COLS + ((col0 + 3) ^ sw)] = xr[k].w;
        }
    }
    __syncthreads();
    const int64_t base = t.base;
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

// Slot table and arc copy of the resident tile in group layout (see above),
// one block per graph; node_off == nullptr means a single graph of n_single
// nodes.  Needs the inverse degrees.
__global__ void res_layout_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                                  const float* __restrict__ weight, const float* __restrict__ invd,
                                  const int64_t* __restrict__ node_off, int32_t n_single, ResSlot* __restrict__ slots,
                                  int32_t* __restrict__ arcs, float* __restrict__ warcs);

// Degree and inverse degree of every node (the d of Definition def:pprdist is
// the out-degree; with weights, the sum of the node's arc weights).
__global__ void degree_kernel(const int32_t* __restrict__ row_ptr, const float* __restrict__ weight,
                              int64_t n, float* __restrict__ deg, float* __restrict__ invd);

}  // namespace pprviz
