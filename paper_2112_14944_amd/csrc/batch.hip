// Batched path: thousands of independent subgraphs (standing in for the
// supernodes of the paper's multi-level hierarchy, Section 2.2) each taken
// through all-pairs PPR -> DPPR -> PDist -> Jacobi stress layout, with no
// host round trip.  Planning happens on the device, so the whole sequence can
// be captured into one HIP graph.
//
//  plan      one block: counting sort of the subgraphs by size (largest first,
//            the longest-processing-time order), per-subgraph prefix sums of
//            PPR tiles, PDist tiles and layout row blocks.
//  ppr       persistent kernel, one 1024-thread block per CU; blocks pop
//            (subgraph, source tile) tasks from an atomic counter in LPT order
//            and run the LDS-resident power iteration of ppr_core.hpp.
//  pdist     grid-stride over (subgraph, 64x64 tile) items.
//  layout    per-node sums of Delta^-2 (one pair-tile pass), then
//            stress_iters sweeps, each a pair-tile pass over the 64x64 tiles
//            of one triangle of every subgraph plus a pass that combines the
//            partial blocks; then one stress pass of the final layout.
#include <math.h>

#include <algorithm>

#include "internal.hpp"
#include "layout_core.hpp"
#include "ppr_core.hpp"

namespace pprviz {

constexpr int kBatchMaxN = Res<16>::NMAX;  // 2304
constexpr int kPlanThreads = 1024;

// One layout task (up to kStripGroup strips of a super-row) with everything
// its wave needs to start, so that a task costs one scalar load of its record
// before its 1/Delta stream starts.
struct __attribute__((aligned(16))) StripRec {
    int32_t k;     // subgraph size
    int32_t sj;    // S << 16 | J0
    int64_t node;  // first node of the subgraph (positions)
    int64_t iv;    // offset of its 1/Delta block
    int64_t pb;    // offset of its partial blocks
};

struct BatchPlan {
    int32_t* order;      // [G] subgraph ids, largest first
    int64_t* tile_pre;   // [G+1] prefix of PPR tiles in LPT order
    int64_t* pd_pre;     // [G+1] prefix of 64x64 PDist tile pairs (I <= J; subgraph order)
    int64_t* rb_pre;     // [G+1] prefix of 16-row layout blocks (subgraph order)
    int32_t* pd_graph;   // subgraph of each PDist tile item
    int32_t* rb_graph;   // subgraph of each layout row-block item
    int64_t* pt_pre;     // [G+1] prefix of the layout sweeps' tasks (256 rows x up to 256 columns)
    StripRec* strip_tab; // [pt_pre[G]] layout tasks, largest first
    int64_t* rt_pre;     // [G+1] prefix of 64-row tiles (sweep finalize items)
    int32_t* rt_graph;   // subgraph of each 64-row tile
    int64_t* pb_pre;     // [G+1] prefix of the partial blocks, T*T*64 floats per subgraph
    int64_t* iv_pre;     // [G+1] prefix of the 1/Delta pool, k rows of inv_ld(k) floats per subgraph
    int32_t* counter;    // [4] PPR task queue heads, one per tile width; layout task queue head
    int32_t* cls_pos;    // [4] first LPT position of the 16-, 32- and 64-column classes, then G
};

__device__ __forceinline__ int graph_n(const int64_t* node_off, int g) {
    return (int)(node_off[g + 1] - node_off[g]);
}

// Largest i with pre[i] <= item, for a non-decreasing prefix array of size m+1.
__device__ __forceinline__ int find_segment(const int64_t* __restrict__ pre, int m, int64_t item) {
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// PPR tiles of an n-node subgraph (0 for a size the resident kernel cannot
// hold; the host rejects such batches before launch).
__device__ __forceinline__ int64_t tiles_of(int n) {
    const int cols = res_cols_for(n);
    return cols == 0 ? 0 : (n + cols - 1) / cols;
}

constexpr int kPlanPrefixes = 7;

// Row stride of a subgraph's block in the 1/Delta pool: rows start on a
// 128-byte boundary, so the 256-byte row segments a pair tile reads span two
// cache lines, not three.
__host__ __device__ __forceinline__ int64_t inv_ld(int k) { return ((int64_t)k + 31) / 32 * 32; }

__device__ __forceinline__ int64_t* plan_prefix(const BatchPlan& p, int which) {
    switch (which) {
        case 0: return p.tile_pre;
        case 1: return p.pd_pre;
        case 2: return p.rb_pre;
        case 3: return p.pt_pre;
        case 4: return p.rt_pre;
        case 5: return p.pb_pre;
        default: return p.iv_pre;
    }
}

// Items of an n-node subgraph for each prefix of the plan.
__device__ __forceinline__ int64_t plan_count(int which, int n) {
    const int64_t T = (n + kPT - 1) / kPT;
    switch (which) {
        case 0: return tiles_of(n);                                          // PPR source tiles
        case 1: return T * (T + 1) / 2;                                      // PDist 64x64 tile pairs
        case 2: return (n + kLayoutRowsPerBlock - 1) / kLayoutRowsPerBlock;  // stress row blocks
        case 3: return strip_task_count(T);                                  // layout tasks (S, J0)
        case 4: return T;                                                    // 64-row tiles
        case 5: return T * T * kPT;                                          // partial-block floats
        default: return (int64_t)n * inv_ld(n);                              // 1/Delta pool floats
    }
}

// Size class of a task for the largest-first order: its pair count (live
// rows times columns of each of its strips, at most 256 x 256) in steps of
// 64, largest first.
constexpr int kStripClasses = kStripGroup * kStripBlocks * kPT * kPT / 64;

__device__ __forceinline__ int strip_class(int k, int T, int S, int J0) {
    int pairs = 0;
    for (int J = J0; J < min(T, J0 + kStripGroup); ++J) {
        const int d = J - kStripBlocks * S;
        const int nl = min(kStripBlocks, min(T - kStripBlocks * S, d + 1));
        const int rows = min(nl * kPT, k - kStripBlocks * S * kPT);
        const int cols = min(kPT, k - J * kPT);
        pairs += rows * cols;
    }
    return (kStripGroup * kStripBlocks * kPT * kPT - pairs) / 64;
}

__global__ __launch_bounds__(kPlanThreads) void batch_plan_kernel(const int64_t* __restrict__ node_off, int32_t G,
                                                                  BatchPlan p) {
    __shared__ int32_t hist[kBatchMaxN + 2];
    __shared__ int64_t scan_tmp[kPlanThreads];
    const int tid = threadIdx.x;
    for (int i = tid; i < kBatchMaxN + 2; i += kPlanThreads) hist[i] = 0;
    __syncthreads();
    for (int g = tid; g < G; g += kPlanThreads) atomicAdd(&hist[min(graph_n(node_off, g), kBatchMaxN + 1)], 1);
    __syncthreads();
    // exclusive prefix over sizes in descending order: start[size]
    if (tid == 0) {
        int32_t run = 0;
        for (int sz = kBatchMaxN + 1; sz >= 0; --sz) {
            const int32_t c = hist[sz];
            hist[sz] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int g = tid; g < G; g += kPlanThreads) {
        const int pos = atomicAdd(&hist[min(graph_n(node_off, g), kBatchMaxN + 1)], 1);
        p.order[pos] = g;
    }
    __syncthreads();
    __threadfence_block();
    // prefix sums (sequential chunks per thread, then a block scan): PPR
    // tiles in LPT order; PDist tiles, stress row blocks, layout pair tiles,
    // 64-row tiles and partial-block floats in subgraph order
    for (int which = 0; which < kPlanPrefixes; ++which) {
        int64_t* out = plan_prefix(p, which);
        const int per = (G + kPlanThreads - 1) / kPlanThreads;
        const int a = tid * per, b = min(G, a + per);
        int64_t loc = 0;
        for (int i = a; i < b; ++i) loc += plan_count(which, graph_n(node_off, which == 0 ? p.order[i] : i));
        scan_tmp[tid] = loc;
        __syncthreads();
        if (tid == 0) {
            int64_t run = 0;
            for (int i = 0; i < kPlanThreads; ++i) {
                const int64_t c = scan_tmp[i];
                scan_tmp[i] = run;
                run += c;
            }
        }
        __syncthreads();
        int64_t run = scan_tmp[tid];
        for (int i = a; i < b; ++i) {
            out[i] = run;
            run += plan_count(which, graph_n(node_off, which == 0 ? p.order[i] : i));
        }
        if (tid == kPlanThreads - 1) out[G] = run;
        __syncthreads();
    }
    // item -> subgraph maps (one load per item instead of a binary search)
    for (int g = tid; g < G; g += kPlanThreads) {
        for (int64_t i = p.pd_pre[g]; i < p.pd_pre[g + 1]; ++i) p.pd_graph[i] = g;
        for (int64_t i = p.rb_pre[g]; i < p.rb_pre[g + 1]; ++i) p.rb_graph[i] = g;
    }
    for (int g = tid; g < G; g += kPlanThreads) {
        for (int64_t i = p.rt_pre[g]; i < p.rt_pre[g + 1]; ++i) p.rt_graph[i] = g;
    }
    // Layout tasks of every subgraph, by size largest first (a counting sort
    // over size classes of 64 pairs), so that the sweeps' queue hands out the
    // largest first.  Which wave runs a task never changes a sum: each task
    // writes its own partial slots.
    __shared__ int32_t scls[kStripClasses];
    for (int i = tid; i < kStripClasses; i += kPlanThreads) scls[i] = 0;
    __syncthreads();
    for (int g = tid; g < G; g += kPlanThreads) {
        const int k = graph_n(node_off, g);
        const int T = (k + kPT - 1) / kPT;
        const int ns = (int)strip_task_count(T);
        for (int t = 0; t < ns; ++t) {
            int S, J0;
            strip_task_sj(t, T, S, J0);
            atomicAdd(&scls[strip_class(k, T, S, J0)], 1);
        }
    }
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int c = 0; c < kStripClasses; ++c) {
            const int32_t n = scls[c];
            scls[c] = run;
            run += n;
        }
    }
    __syncthreads();
    for (int g = tid; g < G; g += kPlanThreads) {
        const int k = graph_n(node_off, g);
        const int T = (k + kPT - 1) / kPT;
        const int ns = (int)strip_task_count(T);
        for (int t = 0; t < ns; ++t) {
            int S, J0;
            strip_task_sj(t, T, S, J0);
            const int pos = atomicAdd(&scls[strip_class(k, T, S, J0)], 1);
            StripRec r;
            r.k = k;
            r.sj = (S << 16) | J0;
            r.node = node_off[g];
            r.iv = p.iv_pre[g];
            r.pb = p.pb_pre[g];
            p.strip_tab[pos] = r;
        }
    }
    // Sizes are sorted descending, so each tile width owns a contiguous range
    // of positions: n > Res<32>::NMAX (16 columns), then n > Res<64>::NMAX
    // (32 columns), then the rest (64 columns).
    __shared__ int32_t cls_cnt[2];
    if (tid < 2) cls_cnt[tid] = 0;
    __syncthreads();
    for (int g = tid; g < G; g += kPlanThreads) {
        const int n = graph_n(node_off, g);
        if (n > Res<32>::NMAX) atomicAdd(&cls_cnt[0], 1);
        else if (n > Res<64>::NMAX) atomicAdd(&cls_cnt[1], 1);
    }
    __syncthreads();
    if (tid == 0) {
        p.counter[0] = p.counter[1] = p.counter[2] = p.counter[3] = 0;
        p.cls_pos[0] = 0;
        p.cls_pos[1] = cls_cnt[0];
        p.cls_pos[2] = cls_cnt[0] + cls_cnt[1];
        p.cls_pos[3] = G;
    }
}

struct BatchArgs {
    const int64_t* node_off;
    const int64_t* mat_off;
    const int32_t* row_ptr;
    int32_t G;
    ResArgs r;  // graph-global fields; src/tgt null (all pairs), ppr_out null
};

// Persistent kernel for the subgraphs of one tile width: blocks pop task ids
// of the class's range (LPT order) until it is exhausted.
template <int COLS, int CLS>
__global__ __launch_bounds__(kResThreads) void batch_ppr_kernel(BatchArgs b, BatchPlan p) {
    __shared__ ResLds L;
    __shared__ int32_t task_sh;
    const int p0 = p.cls_pos[CLS];
    const int p1 = p.cls_pos[CLS + 1];
    if (p0 >= p1) return;
    const int64_t first = p.tile_pre[p0];
    const int64_t last = p.tile_pre[p1];
    for (;;) {
        if (threadIdx.x == 0) task_sh = atomicAdd(&p.counter[CLS], 1);
        __syncthreads();
        const int64_t task = first + __builtin_amdgcn_readfirstlane(task_sh);
        __syncthreads();
        if (task >= last) return;
        const int pos = p0 + find_segment(p.tile_pre + p0, p1 - p0, task);
        const int g = p.order[pos];
        const int64_t tile = task - p.tile_pre[pos];
        const int n = graph_n(b.node_off, g);
        TileTask t;
        t.n = n;
        t.s0 = (int)(tile * COLS);
        t.ncols = min(COLS, n - t.s0);
        t.n_tgt = n;
        t.base = b.node_off[g];
        t.out_off = b.mat_off[g];
        t.ld = n;
        res_graph_bases(t.base, b.row_ptr[t.base], b.row_ptr[t.base + n], g, n, t);
        res_tile<COLS, false>(t, b.r, L);
    }
}

// PDist of every subgraph by 64x64 tile pairs (I, J), I <= J: both tiles of
// pi_d, (I, J) and (J, I), are read once into LDS, and Eq. eq:pprdist's
// symmetric z = pi_d(i, j) + pi_d(j, i) gives both tiles of Delta (the same
// sum in the same order as an element-wise evaluation, so the result is
// bit-identical to the single-graph kernel's); also writes 1/Delta (zero
// diagonal) for the layout sweeps, with the same reciprocal the
// single-layout kernel evaluates per pair.
constexpr int kPdistThreads = 512;

__global__ __launch_bounds__(kPdistThreads) void batch_pdist_kernel(const int64_t* __restrict__ node_off,
                                                          const int64_t* __restrict__ mat_off, int32_t G,
                                                          const int64_t* __restrict__ pd_pre,
                                                          const int32_t* __restrict__ pd_graph,
                                                          const float* __restrict__ pid, float* __restrict__ delta,
                                                          const int64_t* __restrict__ iv_pre, float* __restrict__ inv) {
    __shared__ float ta[64][65], tb[64][65];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t total = pd_pre[G];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int g = pd_graph[item];
        const int k = graph_n(node_off, g);
        const int nt = (k + 63) / 64;
        // item -> (I, J), I <= J, row by row over the upper triangle of tiles
        int I = 0;
        int64_t rem = item - pd_pre[g];
        while (rem >= nt - I) {
            rem -= nt - I;
            ++I;
        }
        const int J = I + (int)rem;
        const int64_t i0 = (int64_t)I * 64, j0 = (int64_t)J * 64;
        const float* P = pid + mat_off[g];
        float* D = delta + mat_off[g];
        float* V = inv + iv_pre[g];
        const int64_t ldv = inv_ld(k);
        const float hi = pdist_hi(k);
        __syncthreads();
        // ta = tile (I, J) of pi_d, tb = tile (J, I)
        for (int rr = w; rr < 64; rr += kPdistThreads / 64) {
            ta[rr][lane] = (i0 + rr < k && j0 + lane < k) ? P[(i0 + rr) * k + j0 + lane] : 0.f;
            if (I != J) tb[rr][lane] = (j0 + rr < k && i0 + lane < k) ? P[(j0 + rr) * k + i0 + lane] : 0.f;
        }
        __syncthreads();
        // tile (I, J): z(i, j) = pi_d(i, j) + pi_d(j, i)
        for (int rr = w; rr < 64; rr += kPdistThreads / 64) {
            const int64_t i = i0 + rr, j = j0 + lane;
            if (i >= k || j >= ldv) continue;
            if (j >= k) {
                // row padding of 1/Delta: zeros, which the strips read as absent pairs
                V[i * ldv + j] = 0.f;
                continue;
            }
            const float z = ta[rr][lane] + (I != J ? tb[lane][rr] : ta[lane][rr]);
            const float dv = (i == j) ? 0.f : pdist_value(z, hi);
            D[i * k + j] = dv;
            V[i * ldv + j] = (i == j) ? 0.f : __builtin_amdgcn_rcpf(dv);
        }
        if (I == J) continue;
        // tile (J, I): z(j, i) = pi_d(j, i) + pi_d(i, j)
        for (int rr = w; rr < 64; rr += kPdistThreads / 64) {
            const int64_t j = j0 + rr, i = i0 + lane;
            if (i >= k || j >= k) continue;
            const float z = tb[rr][lane] + ta[lane][rr];
            const float dv = pdist_value(z, hi);
            D[j * k + i] = dv;
            V[j * ldv + i] = __builtin_amdgcn_rcpf(dv);
        }
    }
}

// Row kernels over (subgraph, 16 rows) items, grid-stride: pre is the
// per-subgraph prefix of the item list and item_graph its subgraph map.
// Used for the stress of the final layout, whose per-item partials are then
// summed per subgraph in item order.
template <int MODE>
__global__ __launch_bounds__(256) void batch_layout_kernel(const int64_t* __restrict__ node_off,
                                                           const int64_t* __restrict__ mat_off, int32_t G,
                                                           const int64_t* __restrict__ pre,
                                                           const int32_t* __restrict__ item_graph,
                                                           const int64_t* __restrict__ iv_pre,
                                                           const float* __restrict__ inv,
                                                           const float2* __restrict__ x, float2* __restrict__ xout,
                                                           float* __restrict__ wsum, double* __restrict__ part) {
    __shared__ double red[4];
    const int wave = threadIdx.x >> 6;
    const int64_t total = pre[G];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int g = item_graph[item];
        const int k = graph_n(node_off, g);
        const int64_t rb = item - pre[g];
        const int64_t nb = node_off[g];
        const int row_begin = (int)(rb * kLayoutRowsPerBlock) + wave * kLayoutRowsPerWave;
        const double st = layout_rows<MODE, true>(inv + iv_pre[g], inv_ld(k), k, x + nb, row_begin,
                                                  xout ? xout + nb : nullptr, 1.f, nullptr, nullptr,
                                                  wsum ? wsum + nb : nullptr);
        if (MODE == kLayoutStress) {
            if ((threadIdx.x & 63) == 0) red[wave] = st;
            __syncthreads();
            if (threadIdx.x == 0) part[item] = (red[0] + red[1]) + (red[2] + red[3]);
            __syncthreads();
        }
    }
}

// Task pass over every subgraph (see strip_task): wave w of the grid starts
// with task w of the plan's largest-first table, then takes the next task
// nobody has taken from the queue head (zeroed by the plan kernel and by
// every finalize launch), so that the waves finish together.  The next
// index is claimed at the start of a task and read at its end.
template <int MODE>
__global__ __launch_bounds__(256) void batch_pair_kernel(const int64_t* __restrict__ pt_pre, int32_t G,
                                                         const StripRec* __restrict__ strip_tab,
                                                         const float* __restrict__ inv,
                                                         const float2* __restrict__ x, float* __restrict__ px,
                                                         float* __restrict__ py, int32_t* __restrict__ queue) {
    __shared__ StripLds<MODE> lds[4];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int total = (int)pt_pre[G];
    const int W = (int)gridDim.x * 4;
    int item = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wave);
    if (item >= total) return;
    StripPend pend = strip_pend_none(px);
    // lane 0 takes the queue's next index; the other lanes' increments go
    // outside the resource, so that no branch (and no early wait) surrounds it
    const __amdgpu_buffer_rsrc_t qr = __builtin_amdgcn_make_buffer_rsrc(queue, 0, 4, 0x00020000);
    const int qoff = lane == 0 ? 0 : (int)kStripOutside;
    while (true) {
        const StripRec cur = strip_tab[item];
        const int claim = __builtin_amdgcn_raw_ptr_buffer_atomic_add_i32(1, qr, qoff, 0, 0);
        const int k = __builtin_amdgcn_readfirstlane(cur.k);
        const int sj = __builtin_amdgcn_readfirstlane(cur.sj);
        const int T = (k + kPT - 1) / kPT;
        strip_task<MODE>(inv + cur.iv, inv_ld(k), k, x + cur.node, sj >> 16, sj & 0xffff, T, px + cur.pb,
                         py + cur.pb, lds[wave], pend);
        item = W + __builtin_amdgcn_readfirstlane(claim);
        if (item >= total) break;
    }
    strip_pend_issue<MODE>(pend);
}

// Combine the partial blocks: one wave per 64-row block of a subgraph.
template <int MODE>
__global__ __launch_bounds__(256) void batch_pair_finalize_kernel(const int64_t* __restrict__ node_off, int32_t G,
                                                                  const int64_t* __restrict__ rt_pre,
                                                                  const int32_t* __restrict__ rt_graph,
                                                                  const int64_t* __restrict__ pb_pre,
                                                                  const float* __restrict__ px,
                                                                  const float* __restrict__ py,
                                                                  const float2* __restrict__ x,
                                                                  float2* __restrict__ xout,
                                                                  float* __restrict__ wsum,
                                                                  int32_t* __restrict__ queue) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t total = rt_pre[G];
    // the next task pass starts its queue at zero (its launch follows this one)
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0;
    for (int64_t item = (int64_t)blockIdx.x * 4 + wave; item < total; item += (int64_t)gridDim.x * 4) {
        const int g = rt_graph[item];
        const int k = graph_n(node_off, g);
        const int T = (k + kPT - 1) / kPT;
        const int i = (int)(item - rt_pre[g]) * kPT + lane;
        if (i >= k) continue;
        const int64_t nb = node_off[g];
        const int64_t pb = pb_pre[g];
        strip_finalize<MODE>(i, T, px + pb, py + pb, x + nb, xout ? xout + nb : nullptr, wsum + nb);
    }
}

// stress_out[g] = sum of its row-block partials, in order.
__global__ void batch_stress_sum_kernel(const int64_t* __restrict__ rb_pre, int32_t G, const double* __restrict__ part,
                                        double* __restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    double s = 0.0;
    for (int64_t i = rb_pre[g]; i < rb_pre[g + 1]; ++i) s += part[i];
    out[g] = s;
}

__global__ void copy_kernel(const float* __restrict__ a, float* __restrict__ b, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) b[i] = a[i];
}

struct BatchWs {
    ResSlot* slots;  // resident-tile slot tables (res_layout_kernel)
    int32_t* col_r;  // arc copies in group layout
    int32_t* sorted_r;  // arcs grouped by LDS bank class (layout staging)
    float* deg;
    float* invd;
    float* inv;   // 1/Delta pool (zero diagonal)
    float* wsum;  // per node sum_j Delta^-2
    float* xtmp;
    double* part;
    float* px;  // strip partial blocks of the sweeps (x, y; the weight pass uses px)
    float* py;
    BatchPlan plan;
};

template <typename Cursor>
static void batch_layout_ws(Cursor& c, const ppr_batch* b, BatchWs* w) {
    BatchWs t;
    t.slots = c.template take<ResSlot>((size_t)(b->n_nodes + (int64_t)kResTabPad * b->n_graphs));
    t.col_r = c.template take<int32_t>(
        (size_t)(b->nnz + (int64_t)kResArcPerNode * b->n_nodes + (int64_t)kResArcPerGraph * b->n_graphs));
    t.sorted_r = c.template take<int32_t>((size_t)std::max<int64_t>(b->nnz, 1));
    t.deg = c.template take<float>((size_t)b->n_nodes);
    t.invd = c.template take<float>((size_t)b->n_nodes);
    // 1/Delta pool with rows padded to 32 floats: sum_g k (k + 31) <= pool + 31 n_nodes
    t.inv = c.template take<float>((size_t)(b->pool_size + 31 * b->n_nodes + 32));
    t.wsum = c.template take<float>((size_t)b->n_nodes);
    t.xtmp = c.template take<float>((size_t)b->n_nodes * 2);
    // row blocks: sum over g of ceil(n_g/16) <= n_nodes/16 + G
    t.part = c.template take<double>((size_t)(b->n_nodes / kLayoutRowsPerBlock + b->n_graphs + 1));
    // partial blocks: sum_g ceil(n_g/64)^2 * 64 <= (pool/4096 + n_nodes/32 + G) * 64 floats
    const size_t pblk = (size_t)(b->pool_size / 4096 + b->n_nodes / 32 + b->n_graphs + 1) * kPT;
    t.px = c.template take<float>(pblk);
    t.py = c.template take<float>(pblk);
    t.plan.order = c.template take<int32_t>((size_t)b->n_graphs);
    t.plan.tile_pre = c.template take<int64_t>((size_t)b->n_graphs + 1);
    t.plan.pd_pre = c.template take<int64_t>((size_t)b->n_graphs + 1);
    t.plan.rb_pre = c.template take<int64_t>((size_t)b->n_graphs + 1);
    // item counts: sum_g ceil(n_g/64)^2 <= pool/4096 + n_nodes/32 + G, and
    // sum_g ceil(n_g/16) <= n_nodes/16 + G
    t.plan.pd_graph = c.template take<int32_t>((size_t)(b->pool_size / 4096 + b->n_nodes / 32 + b->n_graphs + 1));
    t.plan.rb_graph = c.template take<int32_t>((size_t)(b->n_nodes / kLayoutRowsPerBlock + b->n_graphs + 1));
    // tasks: sum_g strip_task_count(T) <= sum_g T(T+1)/2 <= pool/8192 + 3 n_nodes/128 + G;
    // 64-row tiles <= n_nodes/64 + G
    t.plan.pt_pre = c.template take<int64_t>((size_t)b->n_graphs + 1);
    t.plan.strip_tab = c.template take<StripRec>((size_t)(b->pool_size / 8192 + 3 * b->n_nodes / 128 + b->n_graphs + 1));
    t.plan.rt_pre = c.template take<int64_t>((size_t)b->n_graphs + 1);
    t.plan.rt_graph = c.template take<int32_t>((size_t)(b->n_nodes / kPT + b->n_graphs + 1));
    t.plan.pb_pre = c.template take<int64_t>((size_t)b->n_graphs + 1);
    t.plan.iv_pre = c.template take<int64_t>((size_t)b->n_graphs + 1);

    t.plan.counter = c.template take<int32_t>(64);
    t.plan.cls_pos = c.template take<int32_t>(64);
    if (w) *w = t;
}

static int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

// Blocks of the pair-tile kernel that one CU holds at once (the static tile
// deal assumes every block of the grid is resident).
template <int MODE>
static int pair_blocks_per_cu() {
    static const int nb = [] {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, batch_pair_kernel<MODE>, 256, 0) != hipSuccess || v < 1)
            v = 4;
        return v;
    }();
    return nb;
}

static ppr_status batch_validate(const ppr_batch* b, float alpha, int32_t max_iter, int32_t stress_iters,
                                 const float* x0, float* x_out, float* dppr_pool, float* delta_pool) {
    if (b == nullptr || b->n_graphs < 1 || b->n_nodes < 1 || b->nnz < 0 || b->nnz >= (int64_t)INT32_MAX)
        return PPR_EINVAL;
    if (!b->node_off || !b->row_ptr || (b->nnz > 0 && !b->col_idx) || !b->mat_off) return PPR_EINVAL;
    if (!(alpha > 0.0f && alpha < 1.0f) || max_iter < 0 || stress_iters < 0) return PPR_EINVAL;
    if (!x0 || !x_out || x0 == x_out || !dppr_pool || !delta_pool) return PPR_EINVAL;
    if (b->max_n < 1 || b->pool_size < b->n_nodes) return PPR_EINVAL;
    if (b->max_n > kBatchMaxN) return PPR_EUNSUPPORTED;
    return PPR_OK;
}

// Enqueues the batched pipeline.  With `ev` (5 events) the stage boundaries
// are recorded: [0] start, [1] after planning, [2] after PPR, [3] after PDist,
// [4] after the layout sweeps and the final stress pass.
static ppr_status batch_enqueue(const ppr_batch* b, float alpha, int32_t T, int32_t stress_iters, const float* x0,
                                float* x_out, float* dppr_pool, float* delta_pool, double* stress_out,
                                const BatchWs& w, hipStream_t s, hipEvent_t* ev = nullptr) {
    const int G = b->n_graphs;
    if (ev) PPRVIZ_HIP_TRY(hipEventRecord(ev[0], s));
    launch_degree(b->row_ptr, nullptr, b->n_nodes, w.deg, w.invd, s);
    launch_res_layout(b->row_ptr, b->col_idx, nullptr, w.invd, b->node_off, 0, G, w.slots, w.col_r, nullptr,
                      w.sorted_r, nullptr, s);
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, b->node_off, G, w.plan);
    if (ev) PPRVIZ_HIP_TRY(hipEventRecord(ev[1], s));

    BatchArgs ba;
    ba.node_off = b->node_off;
    ba.mat_off = b->mat_off;
    ba.row_ptr = b->row_ptr;
    ba.G = G;
    ba.r.slots = w.slots;
    ba.r.arcs = w.col_r;
    ba.r.warcs = nullptr;
    ba.r.deg = w.deg;
    ba.r.src = nullptr;
    ba.r.tgt = nullptr;
    ba.r.alpha = alpha;
    ba.r.T = T;
    ba.r.ppr_out = nullptr;
    ba.r.dppr_out = dppr_pool;
    ba.r.resid = nullptr;
    const int cus = device_cu_count();
    hipLaunchKernelGGL((batch_ppr_kernel<16, 0>), dim3(cus), dim3(kResThreads), 0, s, ba, w.plan);
    hipLaunchKernelGGL((batch_ppr_kernel<32, 1>), dim3(cus), dim3(kResThreads), 0, s, ba, w.plan);
    hipLaunchKernelGGL((batch_ppr_kernel<64, 2>), dim3(cus), dim3(kResThreads), 0, s, ba, w.plan);
    if (ev) PPRVIZ_HIP_TRY(hipEventRecord(ev[2], s));

    const unsigned grid = (unsigned)cus * 8;
    hipLaunchKernelGGL(batch_pdist_kernel, dim3(grid), dim3(kPdistThreads), 0, s, b->node_off, b->mat_off, G, w.plan.pd_pre,
                       w.plan.pd_graph, dppr_pool, delta_pool, w.plan.iv_pre, w.inv);
    const unsigned pgrid = (unsigned)cus * pair_blocks_per_cu<kPairStep>();
    const unsigned wgrid = (unsigned)cus * pair_blocks_per_cu<kPairW>();
    const unsigned fgrid = (unsigned)cus * 8;
    // per-node weight sums, from the pair tiles in the order the sweeps use
    hipLaunchKernelGGL((batch_pair_kernel<kPairW>), dim3(wgrid), dim3(256), 0, s, w.plan.pt_pre, G, w.plan.strip_tab,
                       w.inv, reinterpret_cast<const float2*>(x0), w.px, w.py, w.plan.counter + 3);
    hipLaunchKernelGGL((batch_pair_finalize_kernel<kPairW>), dim3(fgrid), dim3(256), 0, s, b->node_off, G,
                       w.plan.rt_pre, w.plan.rt_graph, w.plan.pb_pre, w.px, w.py,
                       reinterpret_cast<const float2*>(x0), nullptr, w.wsum, w.plan.counter + 3);
    if (ev) PPRVIZ_HIP_TRY(hipEventRecord(ev[3], s));

    // Jacobi sweeps, ping-pong so that the last one lands in x_out.
    const float2* cur = reinterpret_cast<const float2*>(x0);
    float2* bufs[2] = {reinterpret_cast<float2*>(x_out), reinterpret_cast<float2*>(w.xtmp)};
    int next = (stress_iters % 2 == 1) ? 0 : 1;
    if (stress_iters == 0) {
        hipLaunchKernelGGL(copy_kernel, dim3(1024), dim3(256), 0, s, x0, x_out, b->n_nodes * 2);
        cur = reinterpret_cast<const float2*>(x_out);
    }
    for (int it = 0; it < stress_iters; ++it) {
        float2* out = bufs[next];
        hipLaunchKernelGGL((batch_pair_kernel<kPairStep>), dim3(pgrid), dim3(256), 0, s, w.plan.pt_pre, G,
                           w.plan.strip_tab, w.inv, cur, w.px, w.py, w.plan.counter + 3);
        hipLaunchKernelGGL((batch_pair_finalize_kernel<kPairStep>), dim3(fgrid), dim3(256), 0, s, b->node_off, G,
                           w.plan.rt_pre, w.plan.rt_graph, w.plan.pb_pre, w.px, w.py, cur, out, w.wsum,
                           w.plan.counter + 3);
        cur = out;
        next ^= 1;
    }
    if (stress_out) {
        hipLaunchKernelGGL((batch_layout_kernel<kLayoutStress>), dim3(grid), dim3(256), 0, s, b->node_off, b->mat_off,
                           G, w.plan.rb_pre, w.plan.rb_graph, w.plan.iv_pre, w.inv, cur, nullptr, nullptr, w.part);
        hipLaunchKernelGGL(batch_stress_sum_kernel, dim3((G + 255) / 256), dim3(256), 0, s, w.plan.rb_pre, G, w.part,
                           stress_out);
    }
    if (ev) PPRVIZ_HIP_TRY(hipEventRecord(ev[4], s));
    return launch_status();
}

}  // namespace pprviz

using namespace pprviz;

struct pprviz_batch_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int32_t pprviz_batch_max_n(void) { return kBatchMaxN; }

size_t pprviz_batch_workspace(const ppr_batch* b) {
    if (b == nullptr || b->n_graphs < 1 || b->n_nodes < 1) return 0;
    WsSize c;
    batch_layout_ws(c, b, nullptr);
    return c.used;
}

ppr_status pprviz_batch(const ppr_batch* b, float alpha, double tol_l1, int32_t max_iter, int32_t stress_iters,
                        const float* x0, float* x_out, float* dppr_pool, float* delta_pool, double* stress_out,
                        void* ws, size_t ws_bytes, void* stream) {
    ppr_status st = batch_validate(b, alpha, max_iter, stress_iters, x0, x_out, dppr_pool, delta_pool);
    if (st != PPR_OK) return st;
    int32_t T = 0, conv = 1;
    st = pprviz_pushes_for_tolerance(alpha, tol_l1, max_iter, &T, &conv);
    if (st != PPR_OK) return st;
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    BatchWs w;
    batch_layout_ws(cur, b, &w);
    if (ws == nullptr || cur.used > ws_bytes) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    st = batch_enqueue(b, alpha, T, stress_iters, x0, x_out, dppr_pool, delta_pool, stress_out, w,
                       static_cast<hipStream_t>(stream));
    if (st != PPR_OK) return st;
    return conv ? PPR_OK : PPR_ENOCONV;
}

ppr_status pprviz_batch_profile(const ppr_batch* b, float alpha, double tol_l1, int32_t max_iter,
                                int32_t stress_iters, const float* x0, float* x_out, float* dppr_pool,
                                float* delta_pool, double* stress_out, void* ws, size_t ws_bytes, void* stream,
                                double* stage_ms) {
    if (stage_ms == nullptr) return PPR_EINVAL;
    ppr_status st = batch_validate(b, alpha, max_iter, stress_iters, x0, x_out, dppr_pool, delta_pool);
    if (st != PPR_OK) return st;
    int32_t T = 0, conv = 1;
    st = pprviz_pushes_for_tolerance(alpha, tol_l1, max_iter, &T, &conv);
    if (st != PPR_OK) return st;
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    BatchWs w;
    batch_layout_ws(cur, b, &w);
    if (ws == nullptr || cur.used > ws_bytes) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev[5] = {};
    for (int i = 0; i < 5; ++i) {
        if (hipEventCreate(&ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
            return PPR_EHIP;
        }
    }
    st = batch_enqueue(b, alpha, T, stress_iters, x0, x_out, dppr_pool, delta_pool, stress_out, w, s, ev);
    if (st == PPR_OK && hipEventSynchronize(ev[4]) != hipSuccess) st = PPR_EHIP;
    if (st == PPR_OK) {
        for (int i = 0; i < 4; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) st = PPR_EHIP;
            stage_ms[i] = ms;
        }
    }
    for (int i = 0; i < 5; ++i) (void)hipEventDestroy(ev[i]);
    if (st != PPR_OK) return st;
    return conv ? PPR_OK : PPR_ENOCONV;
}

ppr_status pprviz_batch_plan_create(const ppr_batch* b, float alpha, double tol_l1, int32_t max_iter,
                                    int32_t stress_iters, const float* x0, float* x_out, float* dppr_pool,
                                    float* delta_pool, double* stress_out, void* ws, size_t ws_bytes, void* stream,
                                    pprviz_batch_plan** plan) {
    (void)stream;
    if (plan == nullptr) return PPR_EINVAL;
    *plan = nullptr;
    ppr_status st = batch_validate(b, alpha, max_iter, stress_iters, x0, x_out, dppr_pool, delta_pool);
    if (st != PPR_OK) return st;
    int32_t T = 0, conv = 1;
    st = pprviz_pushes_for_tolerance(alpha, tol_l1, max_iter, &T, &conv);
    if (st != PPR_OK) return st;
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    BatchWs w;
    batch_layout_ws(cur, b, &w);
    if (ws == nullptr || cur.used > ws_bytes) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t cs = nullptr;
    PPRVIZ_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = batch_enqueue(b, alpha, T, stress_iters, x0, x_out, dppr_pool, delta_pool, stress_out, w, cs);
        e = hipStreamEndCapture(cs, &graph);
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || st != PPR_OK || graph == nullptr) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != PPR_OK ? st : PPR_EHIP;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return PPR_EHIP;
    }
    auto* p = new (std::nothrow) pprviz_batch_plan;
    if (p == nullptr) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return PPR_EHIP;
    }
    p->graph = graph;
    p->exec = exec;
    *plan = p;
    return conv ? PPR_OK : PPR_ENOCONV;
}

ppr_status pprviz_batch_plan_launch(pprviz_batch_plan* plan, void* stream) {
    if (plan == nullptr || plan->exec == nullptr) return PPR_EINVAL;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    PPRVIZ_HIP_TRY(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    return PPR_OK;
}

void pprviz_batch_plan_destroy(pprviz_batch_plan* plan) {
    if (plan == nullptr) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
}

}  // extern "C"
