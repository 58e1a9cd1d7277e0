// Level-l DPPR between the k children of a supernode by Group Forward-Push
// (Section 4.2, Algorithm alg:fwdpushsn), run for all k source supernodes at
// once in synchronous rounds.
//
// Column i of the iterate belongs to source supernode V_i.  Its residue
// starts at d(v) / |F(V_i)| on each leaf v of V_i.  In a round, every (node,
// column) pair whose residue r exceeds d(v) * r_max pushes it: alpha * r is
// added to the node's estimate, r / d(v) is what each neighbour u later
// receives times (1 - alpha) w_uv, and the pair's residue becomes 0; what a
// node receives during a round waits for the next round.  Each push is one
// of the paper's push operations (applied to the residue held at the start
// of the round), so the invariant of Lemma lem:fwdpushag and, once no pair
// exceeds its threshold, the error bound of Lemma lem:fpsn-correct hold for
// the result.  The level-l value is the estimate summed over the leaves of
// the target supernode and divided by their count (Definition def:spprdeg).
//
// The round is the streaming power-iteration step with a thresholded
// epilogue: iterate columns in slabs of 32 (node-major within a slab), rows
// by degree, 8 rows side by side per wave, neighbour rows gathered as 128-byte
// pieces.  Each round flags, per slab and node, the rows that pushed, and the
// next round reads only flagged neighbours and skips rows that received
// nothing.  On large grids, in the late rounds, in which few pairs still push,
// the pushing rows also mark the heads of their arcs (when no block of the
// round before pushed along more than half its arcs or kGfpMarkArcs,
// kGfpMarkArcsWide for blocks of wide rows), and the next round skips the
// unmarked rows without reading their arcs; a round that is over that cap
// anywhere leaves the next one to the flags alone.  In the dense rounds of
// large grids (every block of the round before pushed along at least 7/8 of
// its arcs), the rows that do not push write zero sends, and the round after,
// if dense as well, gathers every neighbour without reading push flags.  Round
// t sets a device flag when it pushed anything; round t + 1 exits at once when
// round t pushed nothing, and the host reads the flag every few rounds to stop
// launching.
//
// The same rounds run the Group Backward-Push (Algorithm alg:bwdpushsn):
// column c is target supernode col_set[c], residues start at 1 / |F(V_j)|,
// each column has its own absolute threshold (Eq. eq:brmax), what arrives at
// v is scaled by 1 / d(v), and a push adds alpha d(v) r to the estimate.
// Tau-Push (Algorithm alg:taupush) runs the forward rounds from every
// source, picks the targets whose DNPR (Eq. eq:dnpr-dnppr) exceeds tau on
// the device, and overwrites their columns with the backward rounds.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace pprviz {

namespace {

constexpr int kGfpChunk = 2048;  // leaves per block of the aggregation
constexpr int kGfpInfo = 4;      // [0] bad leaf lists, [1] largest leaf set, [2] wide rows
// Rows with more arcs than this are gathered by a whole wave (8 lane groups
// on one row) instead of one 8-lane group: the longest row then takes 64
// arcs per pass instead of 8, which keeps it from outlasting the rest of a
// round.
constexpr int kGfpWideDeg = 256;
static_assert(kGfpWideDeg + 2 <= kDegKeys, "wide rows must have degree classes of their own");
// A block whose pushing rows hold more arcs than this, or more than half of
// the block's arcs, in a round is over the mark cap: it writes no receive
// marks for the next round and stops the marks of the round after.
constexpr int kGfpMarkArcs = 2048;
// The cap for blocks of wide rows (one row per wave, each wave marking its
// own row's arcs 256 at a time).
constexpr int kGfpMarkArcsWide = 8192;
// Rounds write and use receive marks only when their grid holds more than
// this many blocks (4 x the 2048 blocks of 256 threads that 256 CUs keep
// resident): a round whose blocks all fit at once is bound by one block's
// latency, which the marks lengthen, and its flag scan is short anyway.
constexpr int64_t kGfpMarkMinBlocks = 8192;

struct GfpWs {
    RowEnt* rows;
    int32_t* hist;
    float* deg;
    float* invd;
    float* resid;      // residue kept by each (node, column), slab layout
    float* est;        // estimate per (node, column), slab layout
    float* send[2];    // r / d of the pairs that pushed, by round parity
    uint8_t* flag[2];  // per slab and node: pushed in that round, by round parity
    uint8_t* recv[2];  // per slab and node: marked by a pushing neighbour, by round parity
    int32_t* active;   // 1 when the round pushed anything
    int32_t* over;     // 1 when a block of the round was over the mark cap
    int32_t* sparse;   // 1 when a block of the round pushed along fewer than 7/8 of its arcs
    int32_t* info;
    double* part;      // aggregation partials [k][chunks][ld]
    int32_t* col_set;  // backward: the target supernode of each column
    float* th_col;     // backward: the residue threshold of each column (ld entries)
    double* set_mean;  // mean leaf degree of each supernode (Tau-Push)
    int32_t* count;    // number of targets Tau-Push refines backward
};

inline int64_t gfp_ld(int32_t k) { return (int64_t)(k + kSlab - 1) / kSlab * kSlab; }
inline int64_t gfp_chunks(int32_t n) { return ((int64_t)n + kGfpChunk - 1) / kGfpChunk; }
// 32-bit words of one receive-mark buffer (a byte per slab and node)
inline int64_t gfp_recv_words(int32_t n, int64_t ld) { return ((int64_t)n * (ld / kSlab) + 3) / 4; }

template <typename Cursor>
void gfp_ws_layout(Cursor& c, int32_t n, int32_t k, int32_t max_rounds, GfpWs* w) {
    const int64_t ld = gfp_ld(k);
    GfpWs t{};
    t.rows = c.template take<RowEnt>((size_t)n);
    t.hist = c.template take<int32_t>(kDegKeys);
    t.deg = c.template take<float>((size_t)n);
    t.invd = c.template take<float>((size_t)n);
    t.resid = c.template take<float>((size_t)(n * ld));
    t.est = c.template take<float>((size_t)(n * ld));
    t.send[0] = c.template take<float>((size_t)(n * ld));
    t.send[1] = c.template take<float>((size_t)(n * ld));
    t.flag[0] = c.template take<uint8_t>((size_t)(n * (ld / kSlab)));
    t.flag[1] = c.template take<uint8_t>((size_t)(n * (ld / kSlab)));
    // both mark buffers in one piece of whole words, cleared by one fill
    uint8_t* recv = reinterpret_cast<uint8_t*>(c.template take<uint32_t>((size_t)(2 * gfp_recv_words(n, ld))));
    t.recv[0] = recv;
    t.recv[1] = recv ? recv + 4 * gfp_recv_words(n, ld) : nullptr;
    t.active = c.template take<int32_t>((size_t)std::max(max_rounds, 1));
    t.over = c.template take<int32_t>((size_t)std::max(max_rounds, 1));
    t.sparse = c.template take<int32_t>((size_t)std::max(max_rounds, 1));
    t.info = c.template take<int32_t>(kGfpInfo);
    t.part = c.template take<double>((size_t)(k * gfp_chunks(n) * ld));
    t.col_set = c.template take<int32_t>((size_t)k);
    t.th_col = c.template take<float>((size_t)ld);
    t.set_mean = c.template take<double>((size_t)k);
    t.count = c.template take<int32_t>(1);
    if (w) *w = t;
}

// Leaf lists: leaf_ptr[0] = 0, leaf_ptr[k] = n_leaves, every set of 1 .. n
// leaves.  info[0] becomes nonzero on any violation; info[1] is the largest
// set.
__global__ void gfp_check_ptr_kernel(const int32_t* __restrict__ leaf_ptr, int32_t k, int64_t n_leaves, int32_t n,
                                     int32_t* __restrict__ info) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > k) return;
    if (i == 0 && leaf_ptr[0] != 0) atomicOr(&info[0], 1);
    if (i == k) {
        if ((int64_t)leaf_ptr[k] != n_leaves) atomicOr(&info[0], 1);
        return;
    }
    const int64_t sz = (int64_t)leaf_ptr[i + 1] - leaf_ptr[i];
    if (sz < 1 || sz > n) atomicOr(&info[0], 1);
    else atomicMax(&info[1], (int32_t)sz);
}

// Leaf ids in [0, n); reads leaf_idx only when the pointers passed the check
// (they then bound every index to [0, n_leaves)).
__global__ void gfp_check_idx_kernel(const int32_t* __restrict__ leaf_idx, int64_t n_leaves, int32_t n,
                                     int32_t* __restrict__ info) {
    if (info[0] != 0) return;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; p < n_leaves; p += stride) {
        const int32_t v = leaf_idx[p];
        if (v < 0 || v >= n) atomicOr(&info[0], 2);
    }
}

// Rows with more than kGfpWideDeg arcs: after the scatter of the degree
// order, hist[c] is the end of class c (classes run from the largest degree
// down), so the end of the class of degree kGfpWideDeg + 1 counts them.
__global__ void gfp_wide_count_kernel(const int32_t* __restrict__ hist, int32_t* __restrict__ info) {
    info[2] = hist[kDegKeys - 2 - kGfpWideDeg];
}

// Initial residues of column c, supernode i = col_set[c] (c itself when
// col_set is null): forward d(v) / |F(V_i)|, backward 1 / |F(V_i)|, at each
// leaf v of V_i.  A leaf listed twice in one set receives its share twice.
// Blocks (c, *) take the leaves of that set, 256 at a time.
__global__ void gfp_seed_kernel(const int32_t* __restrict__ leaf_ptr, const int32_t* __restrict__ leaf_idx,
                                const float* __restrict__ deg, int32_t n, const int32_t* __restrict__ col_set,
                                int backward, float* __restrict__ resid) {
    const int c = blockIdx.x;
    const int i = col_set ? col_set[c] : c;
    const int b = leaf_ptr[i], e = leaf_ptr[i + 1];
    for (int p = b + (int)blockIdx.y * 256 + (int)threadIdx.x; p < e; p += (int)gridDim.y * 256) {
        const int32_t v = leaf_idx[p];
        atomicAdd(&resid[sidx(v, c, n)], (backward ? 1.0f : deg[v]) / (float)(e - b));
    }
}

// Mean leaf degree of each supernode, in FP64 (one block per set).
__global__ __launch_bounds__(256) void gfp_set_mean_kernel(const int32_t* __restrict__ leaf_ptr,
                                                           const int32_t* __restrict__ leaf_idx,
                                                           const float* __restrict__ deg,
                                                           double* __restrict__ set_mean) {
    __shared__ double red[256];
    const int i = blockIdx.x;
    const int b = leaf_ptr[i], e = leaf_ptr[i + 1];
    double s = 0.0;
    for (int p = b + (int)threadIdx.x; p < e; p += 256) s += (double)deg[leaf_idx[p]];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) set_mean[i] = red[0] / (double)(e - b);
}

// Tau-Push's choice of targets (one block of 1024): on an undirected graph
// the DNPR of Eq. eq:dnpr-dnppr is tau_j = (mean leaf degree of V_j) / m,
// since the DPPR column sums are the degrees; every V_j with tau_j > tau is
// listed, in increasing j, with its backward threshold of Eq. eq:brmax,
// eps delta over the largest mean leaf degree among the other supernodes.
__global__ __launch_bounds__(1024) void tau_select_kernel(const double* __restrict__ set_mean, int32_t k, double m,
                                                          double tau, double eps_delta,
                                                          int32_t* __restrict__ col_set, float* __restrict__ th_col,
                                                          int32_t* __restrict__ count) {
    __shared__ double top[1024][2];
    __shared__ int arg[1024];
    __shared__ int scan[1024];
    // largest and second largest mean (ties: the lower index is the largest)
    double m1 = -1.0, m2 = -1.0;
    int a1 = -1;
    for (int j = threadIdx.x; j < k; j += 1024) {
        const double x = set_mean[j];
        if (x > m1) {
            m2 = m1;
            m1 = x;
            a1 = j;
        } else if (x > m2) {
            m2 = x;
        }
    }
    top[threadIdx.x][0] = m1;
    top[threadIdx.x][1] = m2;
    arg[threadIdx.x] = a1;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double x1 = top[threadIdx.x][0], x2 = top[threadIdx.x][1];
            const double y1 = top[threadIdx.x + o][0], y2 = top[threadIdx.x + o][1];
            const int ax = arg[threadIdx.x], ay = arg[threadIdx.x + o];
            const bool xfirst = x1 > y1 || (x1 == y1 && ax >= 0 && (ay < 0 || ax < ay));
            top[threadIdx.x][0] = xfirst ? x1 : y1;
            arg[threadIdx.x] = xfirst ? ax : ay;
            top[threadIdx.x][1] = xfirst ? fmax(x2, y1) : fmax(y2, x1);
        }
        __syncthreads();
    }
    const double best = top[0][0], second = top[0][1];
    const int best_j = arg[0];
    int base = 0;
    for (int j0 = 0; j0 < k; j0 += 1024) {
        const int j = j0 + (int)threadIdx.x;
        // with a single supernode there is no other one for Eq. eq:brmax:
        // its column keeps the forward value
        const bool pick = k > 1 && j < k && set_mean[j] / m > tau;
        scan[threadIdx.x] = pick ? 1 : 0;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int x = (int)threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
            __syncthreads();
            scan[threadIdx.x] += x;
            __syncthreads();
        }
        if (pick) {
            const int pos = base + scan[threadIdx.x] - 1;
            const double other = (j == best_j) ? second : best;
            col_set[pos] = j;
            th_col[pos] = other > 0.0 ? (float)(eps_delta / other) : 3.0e38f;
        }
        base += scan[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

// Backward run of the standalone entry: columns take the caller's targets and
// thresholds; info[0] flags a target outside [0, k).
__global__ void gbp_columns_kernel(const int32_t* __restrict__ targets, const float* __restrict__ rb_max,
                                   int32_t n_targets, int32_t k, int32_t* __restrict__ col_set,
                                   float* __restrict__ th_col, int32_t* __restrict__ info) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_targets) return;
    const int32_t j = targets[c];
    if (j < 0 || j >= k) {
        atomicOr(&info[0], 4);
        col_set[c] = 0;
    } else {
        col_set[c] = j;
    }
    th_col[c] = rb_max[c];
}

struct GfpRound {
    const RowEnt* rows;
    const int32_t* col_idx;
    const float* weight;
    const float* deg;
    const float* invd;
    float* resid;
    float* est;
    const float* send_in;   // what the previous round pushed (GATHER)
    float* send_out;        // what this round pushes (SELECT)
    const uint8_t* flag_in; // which nodes pushed in the previous round, per slab (GATHER)
    uint8_t* flag_out;      // which nodes push in this round, per slab (SELECT)
    uint8_t* recv_in;       // marks written by round p, taken and cleared here (GATHER)
    uint8_t* recv_out;      // marks for the next round (SELECT)
    const float* th_col;    // backward: the threshold of each column
    int32_t* active;        // active[t] = 1 when round t pushed anything
    int32_t* over;          // over[t] = 1 when some block of round t was over the mark cap
    int32_t* sparse;        // sparse[t] = 1 when some block of round t pushed along < 7/8 of its arcs
    int32_t n;
    int32_t wide;           // rows 0 .. wide-1 of the degree order have > kGfpWideDeg arcs
    int32_t wide_blocks;    // blocks of 4 wide rows (one per wave), ahead of the rest
    float alpha;
    float r_max;
    int32_t t;              // this round (SELECT)
    int32_t p;              // the round whose sends are gathered (GATHER)
};

// One round.  GATHER: add (1 - alpha) sum_u w_vu send_in[u] to the kept
// residue (rounds t >= 1, and the closing delivery after a round cap),
// reading only neighbours flagged as having pushed; a row with no such
// neighbour keeps its residue, which the previous round left at or below
// its threshold, and is skipped.  SELECT: push every pair over its
// threshold (rounds t >= 0) and flag the rows that pushed.
// BACKWARD (Algorithm alg:bwdpushsn, in the same rounds): the residue
// arriving at v is (1 - alpha) / d(v) sum_u w_vu send[u] with send = r of the
// pairs that pushed, the threshold is the column's own, and a push adds
// alpha d(v) r to the estimate.
template <bool WEIGHTED, bool GATHER, bool SELECT, bool BACKWARD, bool MARKS>
__global__ __launch_bounds__(256) void gfp_round_kernel(GfpRound a, StreamGrid grid) {
    if (a.t > 0 && a.active[a.t - 1] == 0) return;  // the previous round pushed nothing
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int q = lane % kSlabVec;
    int slab, rb;
    stream_block_map(grid, slab, rb);
    const int n = a.n;
    const int64_t slab_off = (int64_t)slab * n * kSlab;
    const int grp = lane / kSlabVec;
    const bool wide = rb < a.wide_blocks;  // uniform in the block
    const int ri = wide ? rb * 4 + wave
                        : a.wide + (rb - a.wide_blocks) * kStreamRowsPerBlock + wave * kStreamRowsPerWave + grp;
    const bool has_row = ri < (wide ? a.wide : n);
    const int64_t flag_off = (int64_t)slab * n;
    // the previous round's cap flag, read early (it decides the marks below)
    const bool may_mark = SELECT && MARKS && a.t >= 1 && a.over[a.t - 1] == 0;
    // After a round that was dense in every block, this round also writes
    // zeros for the rows that do not push, so that the next round can gather
    // every neighbour without reading push flags (a zero piece adds +0.0 to a
    // sum of non-negative terms, so the result does not change).
    const bool zero_fill = SELECT && MARKS && a.t >= 1 && a.sparse[a.t - 1] == 0;
    const bool flagless = GATHER && MARKS && a.p >= 1 && a.sparse[a.p - 1] == 0 && a.sparse[a.p] == 0;
    int rs = 0, dg = 0, v = 0;
    if (has_row) {
        const RowEnt e = load_row(as_global(a.rows), ri);
        rs = e.rs;
        dg = e.re - e.rs;
        v = e.v;
    }
    const uint32_t qoff = (uint32_t)q * 16u;
    const int deg_row = dg;
    if (GATHER && MARKS && a.p >= 1 && a.over[a.p - 1] == 0) {
        // Round p marked the heads of its pushing rows' arcs (no block of
        // round p - 1 was over the cap): take this row's mark and clear it
        // for reuse.  When no block of round p was over the cap either, the
        // marks are complete and, the arcs being symmetric, a row without one
        // has no pushing neighbour.
        const uint8_t mark = has_row ? a.recv_in[flag_off + v] : 0;
        if (mark && (wide ? lane == 0 : q == 0)) a.recv_in[flag_off + v] = 0;
        if (mark == 0 && a.over[a.p] == 0) dg = 0;
    }
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int got = 1;
    if (GATHER) {
        const uint32_t slab_bytes = (uint32_t)n * (kSlab * 4);
        const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(a.send_in + slab_off), 0, (int)slab_bytes, 0x00020000);
        if (wide) {
            if (flagless)
                acc = slab_gather<WEIGHTED, false, kWave>(rin, a.col_idx, a.weight, rs + kSlabVec * grp,
                                                          max(dg - kSlabVec * grp, 0), lane, qoff);
            else
                acc = slab_gather<WEIGHTED, true, kWave>(rin, a.col_idx, a.weight, rs + kSlabVec * grp,
                                                         max(dg - kSlabVec * grp, 0), lane, qoff,
                                                         a.flag_in + flag_off, &got);
            // add the 8 groups' sums (a fixed tree) into every group
#pragma unroll
            for (int o = kSlabVec; o < kWave; o <<= 1) {
                acc.x += __shfl_xor(acc.x, o, kWave);
                acc.y += __shfl_xor(acc.y, o, kWave);
                acc.z += __shfl_xor(acc.z, o, kWave);
                acc.w += __shfl_xor(acc.w, o, kWave);
                got |= __shfl_xor(got, o, kWave);
            }
        } else if (flagless) {
            acc = slab_gather<WEIGHTED, false>(rin, a.col_idx, a.weight, rs, dg, lane, qoff);
        } else {
            acc = slab_gather<WEIGHTED, true>(rin, a.col_idx, a.weight, rs, dg, lane, qoff, a.flag_in + flag_off,
                                              &got);
        }
    }
    // a wide row is finished by its first lane group
    const bool owner = has_row && (!wide || grp == 0);
    int pushed = 0;
    if (owner && got) {
        const int64_t off = slab_off + (int64_t)v * kSlab + q * 4;
        float4* r4 = reinterpret_cast<float4*>(a.resid + off);
        float r[4] = {r4->x, r4->y, r4->z, r4->w};
        if (GATHER) {
            const float keep = BACKWARD ? (1.0f - a.alpha) * a.invd[v] : 1.0f - a.alpha;
            r[0] += keep * acc.x;
            r[1] += keep * acc.y;
            r[2] += keep * acc.z;
            r[3] += keep * acc.w;
        }
        if (SELECT) {
            const float dv = a.deg[v];
            float th[4];
            if (BACKWARD) {
                const float4 t4 = *reinterpret_cast<const float4*>(a.th_col + slab * kSlab + q * 4);
                th[0] = t4.x;
                th[1] = t4.y;
                th[2] = t4.z;
                th[3] = t4.w;
            } else {
                th[0] = th[1] = th[2] = th[3] = dv * a.r_max;
            }
            const float id = a.invd[v];
            float s[4], add[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bool on = r[c] > th[c];
                pushed += on ? 1 : 0;
                s[c] = on ? (BACKWARD ? r[c] : r[c] * id) : 0.f;
                add[c] = on ? (BACKWARD ? a.alpha * dv * r[c] : a.alpha * r[c]) : 0.f;
                r[c] = on ? 0.f : r[c];
            }
            // what a row sends is read only when the row is flagged, i.e.
            // when one of its 8 lanes pushed: the others write their zeros
            // only then
            int row_any = pushed;
#pragma unroll
            for (int o = 1; o < kSlabVec; o <<= 1) row_any |= __shfl_xor(row_any, o, kWave);
            if (row_any) *reinterpret_cast<float4*>(a.send_out + off) = make_float4(s[0], s[1], s[2], s[3]);
            if (pushed) {
                float4* e4 = reinterpret_cast<float4*>(a.est + off);
                float4 ev = *e4;
                ev.x += add[0];
                ev.y += add[1];
                ev.z += add[2];
                ev.w += add[3];
                *e4 = ev;
            }
        }
        *r4 = make_float4(r[0], r[1], r[2], r[3]);
    }
    if (SELECT) {
        // flag the row when any of its 32 columns pushed (OR over its 8 lanes)
        int row_pushed = pushed;
#pragma unroll
        for (int o = 1; o < kSlabVec; o <<= 1) row_pushed |= __shfl_xor(row_pushed, o, kWave);
        if (owner && q == 0) a.flag_out[flag_off + v] = row_pushed ? 1 : 0;
        if (zero_fill && owner && !row_pushed)
            *reinterpret_cast<float4*>(a.send_out + slab_off + (int64_t)v * kSlab + q * 4) =
                make_float4(0.f, 0.f, 0.f, 0.f);
        __shared__ int block_pushed;
        __shared__ int block_arcs;  // arcs of the block's pushing rows
        __shared__ int block_all;   // arcs of all the block's rows
        if (threadIdx.x == 0) {
            block_pushed = 0;
            if (MARKS) {
                block_arcs = 0;
                block_all = 0;
            }
        }
        __syncthreads();
        if (pushed) block_pushed = 1;
        if (MARKS && owner && q == 0) {
            atomicAdd(&block_all, deg_row);
            if (row_pushed) atomicAdd(&block_arcs, deg_row);
        }
        __syncthreads();
        if (threadIdx.x == 0 && block_pushed) a.active[a.t] = 1;
        if (MARKS) {
            const int arcs = block_arcs;
            const bool over = arcs > min(wide ? kGfpMarkArcsWide : kGfpMarkArcs, block_all / 2);
            if (threadIdx.x == 0 && over) a.over[a.t] = 1;
            if (threadIdx.x == 0 && 8 * (int64_t)arcs < 7 * (int64_t)block_all) a.sparse[a.t] = 1;
            // Mark the heads of the pushing rows' arcs for the next round, when
            // the previous round was under the cap everywhere (a round that
            // follows a dense one is likely dense too, and its marks would go
            // unused).
            if (may_mark && arcs > 0 && !over && has_row) {
                if (wide) {
                    // the first lane group owns the row; the whole wave marks
                    if (__shfl(row_pushed, 0, kWave))
                        for (int j0 = 0; j0 < deg_row; j0 += 4 * kWave) {
                            int u[4];
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int j = j0 + r * kWave + lane;
                                u[r] = j < deg_row ? a.col_idx[rs + j] : -1;
                            }
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                if ((unsigned)u[r] < (unsigned)n) a.recv_out[flag_off + u[r]] = 1;
                        }
                } else if (row_pushed) {
                    for (int j = q; j < deg_row; j += kSlabVec) {
                        const int u = a.col_idx[rs + j];
                        if ((unsigned)u < (unsigned)n) a.recv_out[flag_off + u] = 1;
                    }
                }
            }
        }
    }
}

// Aggregation partials: part[j][chunk][col] = sum of est[v][col] over the
// chunk's leaves v of F(V_j), in FP64.  8 groups of 32 lanes take every 8th
// leaf; the groups' sums are added in a fixed order.
__global__ __launch_bounds__(256) void gfp_aggregate_kernel(const float* __restrict__ est, int32_t n, int64_t ld,
                                                            const int32_t* __restrict__ leaf_ptr,
                                                            const int32_t* __restrict__ leaf_idx, int64_t chunks,
                                                            double* __restrict__ part) {
    __shared__ double red[8][kSlab];
    const int j = blockIdx.x;
    const int64_t ch = blockIdx.y;
    const int c = threadIdx.x % kSlab;
    const int g = threadIdx.x / kSlab;
    const int64_t b = (int64_t)leaf_ptr[j] + ch * kGfpChunk;
    const int64_t e = min((int64_t)leaf_ptr[j + 1], b + kGfpChunk);
    for (int64_t slab = 0; slab < ld / kSlab; ++slab) {
        const float* x = est + slab * n * kSlab;
        // four leaves in flight per lane, added in leaf order
        double s = 0.0;
        int64_t p = b + g;
        for (; p + 24 < e; p += 32) {
            const int32_t v0 = leaf_idx[p], v1 = leaf_idx[p + 8], v2 = leaf_idx[p + 16], v3 = leaf_idx[p + 24];
            const float x0 = x[(int64_t)v0 * kSlab + c], x1 = x[(int64_t)v1 * kSlab + c];
            const float x2 = x[(int64_t)v2 * kSlab + c], x3 = x[(int64_t)v3 * kSlab + c];
            s += (double)x0;
            s += (double)x1;
            s += (double)x2;
            s += (double)x3;
        }
        for (; p < e; p += 8) s += (double)x[(int64_t)leaf_idx[p] * kSlab + c];
        red[g][c] = s;
        __syncthreads();
        if (g == 0) {
            double t = 0.0;
#pragma unroll
            for (int h = 0; h < 8; ++h) t += red[h][c];
            part[((int64_t)j * chunks + ch) * ld + slab * kSlab + c] = t;
        }
        __syncthreads();
    }
}

// Forward (col_set null, k columns): out[i][j] = (sum over chunks of
// part[j][chunk][i]) / |F(V_j)|, the estimates of source column i summed over
// the leaves of target V_j.  Backward: out[i][col_set[c]] = (sum over chunks
// of part[i][chunk][c]) / |F(V_i)|, the estimates of target column c summed
// over the leaves of source V_i.
__global__ void gfp_finish_kernel(const double* __restrict__ part, const int32_t* __restrict__ leaf_ptr, int32_t k,
                                  int64_t chunks, int64_t ld, int32_t ncols, const int32_t* __restrict__ col_set,
                                  float* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)k * ncols) return;
    int set, col;
    int64_t o;
    if (col_set == nullptr) {
        col = (int)(idx / k);
        set = (int)(idx % k);
        o = idx;
    } else {
        set = (int)(idx / ncols);
        col = (int)(idx % ncols);
        o = (int64_t)set * k + col_set[col];
    }
    const int64_t size = (int64_t)leaf_ptr[set + 1] - leaf_ptr[set];
    const int64_t used = (size + kGfpChunk - 1) / kGfpChunk;
    double t = 0.0;
    for (int64_t ch = 0; ch < used; ++ch) t += part[((int64_t)set * chunks + ch) * ld + col];
    out[o] = (float)(t / (double)size);
}

// out[i][v] = x[v][i] for i < k (slab layout -> row-major [k][n]), 64 x 64
// tiles through LDS.
__global__ __launch_bounds__(256) void gfp_transpose_kernel(const float* __restrict__ x, int32_t n, int32_t k,
                                                            float* __restrict__ out) {
    __shared__ float tile[64][65];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int64_t c0 = (int64_t)blockIdx.y * 64;
    for (int vv = w; vv < 64; vv += 4) {
        const int64_t v = v0 + vv, c = c0 + lane;
        tile[vv][lane] = (v < n && c < k) ? x[sidx(v, c, n)] : 0.f;
    }
    __syncthreads();
    for (int cc = w; cc < 64; cc += 4) {
        const int64_t c = c0 + cc, v = v0 + lane;
        if (c < k && v < n) out[c * n + v] = tile[lane][cc];
    }
}

StreamGrid gfp_grid(int32_t n, int32_t wide, int64_t ld) {
    StreamGrid g;
    g.row_blocks = (wide + 3) / 4 + (n - wide + kStreamRowsPerBlock - 1) / kStreamRowsPerBlock;
    g.slabs = (int32_t)(ld / kSlab);
    g.full_rounds = ((int64_t)n * kSlab * 4 <= kStreamSlabBudget) ? g.slabs / kXcds : 0;
    return g;
}

template <bool GATHER, bool SELECT, bool MARKS>
void gfp_launch_round(bool weighted, bool backward, const GfpRound& a, const StreamGrid& g, hipStream_t s) {
    const dim3 grid((unsigned)((int64_t)g.row_blocks * g.slabs));
    if (backward) {
        if (weighted)
            hipLaunchKernelGGL((gfp_round_kernel<true, GATHER, SELECT, true, MARKS>), grid, dim3(256), 0, s, a, g);
        else
            hipLaunchKernelGGL((gfp_round_kernel<false, GATHER, SELECT, true, MARKS>), grid, dim3(256), 0, s, a, g);
    } else {
        if (weighted)
            hipLaunchKernelGGL((gfp_round_kernel<true, GATHER, SELECT, false, MARKS>), grid, dim3(256), 0, s, a, g);
        else
            hipLaunchKernelGGL((gfp_round_kernel<false, GATHER, SELECT, false, MARKS>), grid, dim3(256), 0, s, a,
                               g);
    }
}

template <bool GATHER, bool SELECT>
void gfp_launch_round(bool weighted, bool backward, bool marks, const GfpRound& a, const StreamGrid& g,
                      hipStream_t s) {
    if (marks)
        gfp_launch_round<GATHER, SELECT, true>(weighted, backward, a, g, s);
    else
        gfp_launch_round<GATHER, SELECT, false>(weighted, backward, a, g, s);
}

ppr_status read_i32(const int32_t* dev, int32_t* host, size_t count, hipStream_t s) {
    PPRVIZ_HIP_TRY(hipMemcpyAsync(host, dev, sizeof(int32_t) * count, hipMemcpyDeviceToHost, s));
    PPRVIZ_HIP_TRY(hipStreamSynchronize(s));
    return PPR_OK;
}

struct GfpArgs {
    const ppr_csr* g;
    const int32_t* leaf_ptr;
    const int32_t* leaf_idx;
    int32_t k;
    int64_t n_leaves;
    float alpha;
    int32_t max_rounds;
};

ppr_status gfp_validate(const GfpArgs& A, size_t ws_bytes, void* ws, GfpWs* w) {
    ppr_status st = validate_csr(A.g);
    if (st != PPR_OK) return st;
    if (A.k < 1 || A.leaf_ptr == nullptr || A.leaf_idx == nullptr) return PPR_EINVAL;
    if (A.n_leaves < A.k || A.n_leaves > (int64_t)A.k * A.g->n || A.n_leaves >= (int64_t)INT32_MAX)
        return PPR_EINVAL;
    if (!(A.alpha > 0.0f && A.alpha < 1.0f) || A.max_rounds < 1) return PPR_EINVAL;
    if (A.g->n > kStreamMaxN) return PPR_EUNSUPPORTED;
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    gfp_ws_layout(cur, A.g->n, A.k, A.max_rounds, w);
    if (ws == nullptr || cur.used > ws_bytes) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    return PPR_OK;
}

// Checks the leaf lists (and the backward targets, when given), builds the
// degrees and the degree row order, and reads back the check results, the
// largest leaf set and the count of wide rows.  Nothing else is enqueued.
ppr_status gfp_prepare(const GfpArgs& A, const GfpWs& w, const int32_t* targets, const float* rb_max,
                       int32_t n_targets, int32_t info[kGfpInfo], hipStream_t s) {
    const int32_t n = A.g->n;
    fill<int32_t>(w.info, 0, kGfpInfo, s);
    hipLaunchKernelGGL(gfp_check_ptr_kernel, dim3((unsigned)((A.k + 256) / 256)), dim3(256), 0, s, A.leaf_ptr,
                       A.k, A.n_leaves, n, w.info);
    hipLaunchKernelGGL(gfp_check_idx_kernel, dim3((unsigned)std::min<int64_t>((A.n_leaves + 255) / 256, 4096)),
                       dim3(256), 0, s, A.leaf_idx, A.n_leaves, n, w.info);
    if (targets) {
        fill<float>(w.th_col, 3.0e38f, gfp_ld(A.k), s);
        hipLaunchKernelGGL(gbp_columns_kernel, dim3((unsigned)((n_targets + 255) / 256)), dim3(256), 0, s, targets,
                           rb_max, n_targets, A.k, w.col_set, w.th_col, w.info);
    }
    // Row order by degree; the rows with more than kGfpWideDeg arcs come
    // first, and their count is read back with the check results.
    launch_degree(A.g->row_ptr, A.g->weight, n, w.deg, w.invd, s);
    stream_row_order(A.g->row_ptr, n, w.hist, w.rows, s);
    hipLaunchKernelGGL(gfp_wide_count_kernel, dim3(1), dim3(1), 0, s, w.hist, w.info);
    ppr_status st = launch_status();
    if (st != PPR_OK) return st;
    if ((st = read_i32(w.info, info, kGfpInfo, s)) != PPR_OK) return st;
    return info[0] != 0 ? PPR_EINVAL : PPR_OK;
}

// One direction of pushes in rounds, from seeding to the k x k output.
// Forward: k columns, column i the source supernode V_i, threshold
// d(v) * r_max.  Backward: ncols columns, column c the target supernode
// col_set[c] with threshold th_col[c] (both already in the workspace); only
// the target columns of out are written.
ppr_status gfp_run(const GfpArgs& A, const GfpWs& w, const int32_t info[kGfpInfo], bool backward, int32_t ncols,
                   float r_max, float* dppr_out, float* est_out, float* resid_out, int32_t* rounds_out,
                   bool* capped_out, hipStream_t s) {
    const int32_t n = A.g->n;
    const int32_t k = A.k;
    const int64_t ld = gfp_ld(ncols);
    const int32_t wide = info[2];
    ppr_status st;
    fill<float>(w.resid, 0.f, n * ld, s);
    fill<float>(w.est, 0.f, n * ld, s);
    fill<int32_t>(w.active, 0, A.max_rounds, s);
    const StreamGrid grid = gfp_grid(n, wide, ld);
    const bool marks = (int64_t)grid.row_blocks * grid.slabs > kGfpMarkMinBlocks;
    if (marks) {
        fill<int32_t>(w.over, 0, A.max_rounds, s);
        fill<int32_t>(w.sparse, 0, A.max_rounds, s);
        fill<uint32_t>(reinterpret_cast<uint32_t*>(w.recv[0]), 0u, 2 * gfp_recv_words(n, ld), s);
    }
    hipLaunchKernelGGL(gfp_seed_kernel, dim3((unsigned)ncols, (unsigned)std::min(4096, (info[1] + 255) / 256)),
                       dim3(256), 0, s, A.leaf_ptr, A.leaf_idx, w.deg, n, backward ? w.col_set : nullptr,
                       backward ? 1 : 0, w.resid);

    const bool weighted = A.g->weight != nullptr;
    GfpRound a;
    a.rows = w.rows;
    a.col_idx = A.g->col_idx;
    a.weight = A.g->weight;
    a.deg = w.deg;
    a.invd = w.invd;
    a.resid = w.resid;
    a.est = w.est;
    a.active = w.active;
    a.over = w.over;
    a.sparse = w.sparse;
    a.th_col = w.th_col;
    a.n = n;
    a.wide = wide;
    a.wide_blocks = (wide + 3) / 4;
    a.alpha = A.alpha;
    a.r_max = r_max;
    a.t = 0;
    a.p = -1;
    a.send_in = nullptr;
    a.send_out = w.send[0];
    a.flag_in = nullptr;
    a.flag_out = w.flag[0];
    a.recv_in = nullptr;
    a.recv_out = w.recv[0];
    gfp_launch_round<false, true>(weighted, backward, marks, a, grid, s);

    // Rounds 1 .. max_rounds - 1 in growing batches; after each batch the
    // host reads the last round's flag and stops when it is clear.
    int32_t launched = 1, last = -1, batch = 4;
    while (true) {
        if ((st = launch_status()) != PPR_OK) return st;
        if ((st = read_i32(w.active + launched - 1, &last, 1, s)) != PPR_OK) return st;
        if (last == 0 || launched == A.max_rounds) break;
        const int32_t end = std::min(A.max_rounds, launched + batch);
        for (int32_t t = launched; t < end; ++t) {
            a.t = t;
            a.p = t - 1;
            a.send_in = w.send[(t - 1) & 1];
            a.send_out = w.send[t & 1];
            a.flag_in = w.flag[(t - 1) & 1];
            a.flag_out = w.flag[t & 1];
            a.recv_in = w.recv[(t - 1) & 1];
            a.recv_out = w.recv[t & 1];
            gfp_launch_round<true, true>(weighted, backward, marks, a, grid, s);
        }
        launched = end;
        batch = std::min(batch * 2, 64);
    }
    // Rounds run: up to and including the first that pushed nothing.
    std::vector<int32_t> counts((size_t)launched);
    if ((st = read_i32(w.active, counts.data(), (size_t)launched, s)) != PPR_OK) return st;
    int32_t rounds = launched;
    for (int32_t t = 0; t < launched; ++t)
        if (counts[(size_t)t] == 0) {
            rounds = t + 1;
            break;
        }
    const bool capped = counts[(size_t)rounds - 1] != 0;
    if (capped) {
        // deliver what the last round sent, so that the residues and the
        // estimates satisfy the invariant
        a.t = 0;
        a.p = rounds - 1;
        a.send_in = w.send[(rounds - 1) & 1];
        a.send_out = nullptr;
        a.flag_in = w.flag[(rounds - 1) & 1];
        a.flag_out = nullptr;
        a.recv_in = w.recv[(rounds - 1) & 1];
        a.recv_out = nullptr;
        gfp_launch_round<true, false>(weighted, backward, marks, a, grid, s);
    }

    const int64_t chunks = gfp_chunks(n);
    const int64_t used = ((int64_t)info[1] + kGfpChunk - 1) / kGfpChunk;
    hipLaunchKernelGGL(gfp_aggregate_kernel, dim3((unsigned)k, (unsigned)used), dim3(256), 0, s, w.est, n, ld,
                       A.leaf_ptr, A.leaf_idx, chunks, w.part);
    hipLaunchKernelGGL(gfp_finish_kernel, dim3((unsigned)(((int64_t)k * ncols + 255) / 256)), dim3(256), 0, s,
                       w.part, A.leaf_ptr, k, chunks, ld, ncols, backward ? w.col_set : nullptr, dppr_out);
    const dim3 tgrid((unsigned)((n + 63) / 64), (unsigned)((ncols + 63) / 64));
    if (est_out) hipLaunchKernelGGL(gfp_transpose_kernel, tgrid, dim3(256), 0, s, w.est, n, ncols, est_out);
    if (resid_out) hipLaunchKernelGGL(gfp_transpose_kernel, tgrid, dim3(256), 0, s, w.resid, n, ncols, resid_out);
    if ((st = launch_status()) != PPR_OK) return st;
    if (rounds_out) *rounds_out = rounds;
    if (capped_out) *capped_out = capped;
    return PPR_OK;
}

}  // namespace

}  // namespace pprviz

using namespace pprviz;

extern "C" {

size_t gfp_workspace(const ppr_csr* g, int32_t k, int32_t max_rounds) {
    if (g == nullptr || g->n < 1 || k < 1 || max_rounds < 1) return 0;
    WsSize c;
    gfp_ws_layout(c, g->n, k, max_rounds, nullptr);
    return c.used;
}

ppr_status gfp_level_dppr(const ppr_csr* g, const int32_t* leaf_ptr, const int32_t* leaf_idx, int32_t k,
                          int64_t n_leaves, float alpha, double r_max, int32_t max_rounds, float* dppr_out,
                          float* est_out, float* resid_out, int32_t* rounds_out, void* ws, size_t ws_bytes,
                          void* stream) {
    if (!(r_max >= 0.0) || !std::isfinite(r_max) || dppr_out == nullptr) return PPR_EINVAL;
    const GfpArgs A{g, leaf_ptr, leaf_idx, k, n_leaves, alpha, max_rounds};
    GfpWs w;
    ppr_status st = gfp_validate(A, ws_bytes, ws, &w);
    if (st != PPR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t info[kGfpInfo] = {0, 0, 0, 0};
    if ((st = gfp_prepare(A, w, nullptr, nullptr, 0, info, s)) != PPR_OK) return st;
    bool capped = false;
    st = gfp_run(A, w, info, false, k, (float)r_max, dppr_out, est_out, resid_out, rounds_out, &capped, s);
    if (st != PPR_OK) return st;
    return capped ? PPR_ENOCONV : PPR_OK;
}

ppr_status gbp_level_dppr(const ppr_csr* g, const int32_t* leaf_ptr, const int32_t* leaf_idx, int32_t k,
                          int64_t n_leaves, const int32_t* targets, int32_t n_targets, const float* rb_max,
                          float alpha, int32_t max_rounds, float* dppr_out, float* est_out, float* resid_out,
                          int32_t* rounds_out, void* ws, size_t ws_bytes, void* stream) {
    if (targets == nullptr || rb_max == nullptr || n_targets < 1 || n_targets > k || dppr_out == nullptr)
        return PPR_EINVAL;
    const GfpArgs A{g, leaf_ptr, leaf_idx, k, n_leaves, alpha, max_rounds};
    GfpWs w;
    ppr_status st = gfp_validate(A, ws_bytes, ws, &w);
    if (st != PPR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t info[kGfpInfo] = {0, 0, 0, 0};
    if ((st = gfp_prepare(A, w, targets, rb_max, n_targets, info, s)) != PPR_OK) return st;
    bool capped = false;
    st = gfp_run(A, w, info, true, n_targets, 0.f, dppr_out, est_out, resid_out, rounds_out, &capped, s);
    if (st != PPR_OK) return st;
    return capped ? PPR_ENOCONV : PPR_OK;
}

ppr_status tau_push_level_dppr(const ppr_csr* g, const int32_t* leaf_ptr, const int32_t* leaf_idx, int32_t k,
                               int64_t n_leaves, float alpha, double eps, double delta, double tau,
                               int32_t max_rounds, float* dppr_out, int32_t* n_backward_out, int32_t* rounds_out,
                               void* ws, size_t ws_bytes, void* stream) {
    if (!(eps > 0.0) || !(delta > 0.0) || !std::isfinite(eps) || !std::isfinite(delta) || !std::isfinite(tau) ||
        dppr_out == nullptr)
        return PPR_EINVAL;
    const GfpArgs A{g, leaf_ptr, leaf_idx, k, n_leaves, alpha, max_rounds};
    GfpWs w;
    ppr_status st = gfp_validate(A, ws_bytes, ws, &w);
    if (st != PPR_OK) return st;
    if (g->nnz < 1) return PPR_EINVAL;  // m = 0 leaves Eq. eq:rmax undefined
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t info[kGfpInfo] = {0, 0, 0, 0};
    if ((st = gfp_prepare(A, w, nullptr, nullptr, 0, info, s)) != PPR_OK) return st;
    // Algorithm alg:taupush: tau = 1 / sqrt(k n) unless given, r_max by
    // Eq. eq:rmax with m = nnz (each undirected edge is two arcs)
    const double m = (double)g->nnz;
    const double t = tau > 0.0 ? tau : 1.0 / std::sqrt((double)k * (double)g->n);
    const double r_max = eps * delta / (m * t);
    bool capped_f = false, capped_b = false;
    int32_t rounds[2] = {0, 0};
    st = gfp_run(A, w, info, false, k, (float)r_max, dppr_out, nullptr, nullptr, &rounds[0], &capped_f, s);
    if (st != PPR_OK) return st;
    // targets with DNPR above tau, refined by the backward pushes
    fill<float>(w.th_col, 3.0e38f, gfp_ld(k), s);
    hipLaunchKernelGGL(gfp_set_mean_kernel, dim3((unsigned)k), dim3(256), 0, s, leaf_ptr, leaf_idx, w.deg,
                       w.set_mean);
    hipLaunchKernelGGL(tau_select_kernel, dim3(1), dim3(1024), 0, s, w.set_mean, k, m, t, eps * delta, w.col_set,
                       w.th_col, w.count);
    if ((st = launch_status()) != PPR_OK) return st;
    int32_t nb = 0;
    if ((st = read_i32(w.count, &nb, 1, s)) != PPR_OK) return st;
    if (nb > 0) {
        st = gfp_run(A, w, info, true, nb, 0.f, dppr_out, nullptr, nullptr, &rounds[1], &capped_b, s);
        if (st != PPR_OK) return st;
    }
    if (n_backward_out) *n_backward_out = nb;
    if (rounds_out) {
        rounds_out[0] = rounds[0];
        rounds_out[1] = rounds[1];
    }
    return (capped_f || capped_b) ? PPR_ENOCONV : PPR_OK;
}

}  // extern "C"
