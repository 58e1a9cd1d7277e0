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
// nothing, so the late rounds, in which few pairs still push, cost little
// more than reading the arcs.  Round t sets a device flag when it pushed
// anything; round t + 1 exits at once when round t pushed nothing, and the
// host reads the flag every few rounds to stop launching.
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

struct GfpWs {
    RowEnt* rows;
    int32_t* hist;
    float* deg;
    float* invd;
    float* resid;      // residue kept by each (node, column), slab layout
    float* est;        // estimate per (node, column), slab layout
    float* send[2];    // r / d of the pairs that pushed, by round parity
    uint8_t* flag[2];  // per slab and node: pushed in that round, by round parity
    int32_t* active;   // 1 when the round pushed anything
    int32_t* info;
    double* part;      // aggregation partials [k][chunks][ld]
};

inline int64_t gfp_ld(int32_t k) { return (int64_t)(k + kSlab - 1) / kSlab * kSlab; }
inline int64_t gfp_chunks(int32_t n) { return ((int64_t)n + kGfpChunk - 1) / kGfpChunk; }

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
    t.active = c.template take<int32_t>((size_t)std::max(max_rounds, 1));
    t.info = c.template take<int32_t>(kGfpInfo);
    t.part = c.template take<double>((size_t)(k * gfp_chunks(n) * ld));
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

// Initial residues: d(v) / |F(V_i)| in column i at each leaf v of V_i.  A
// leaf listed twice in one set receives its share twice.
// Blocks (i, *) take the leaves of set i, 256 at a time.
__global__ void gfp_seed_kernel(const int32_t* __restrict__ leaf_ptr, const int32_t* __restrict__ leaf_idx,
                                const float* __restrict__ deg, int32_t n, float* __restrict__ resid) {
    const int i = blockIdx.x;
    const int b = leaf_ptr[i], e = leaf_ptr[i + 1];
    for (int p = b + (int)blockIdx.y * 256 + (int)threadIdx.x; p < e; p += (int)gridDim.y * 256) {
        const int32_t v = leaf_idx[p];
        atomicAdd(&resid[sidx(v, i, n)], deg[v] / (float)(e - b));
    }
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
    int32_t* active;        // active[t] = 1 when round t pushed anything
    int32_t n;
    int32_t wide;           // rows 0 .. wide-1 of the degree order have > kGfpWideDeg arcs
    int32_t wide_blocks;    // blocks of 4 wide rows (one per wave), ahead of the rest
    float alpha;
    float r_max;
    int32_t t;
};

// One round.  GATHER: add (1 - alpha) sum_u w_vu send_in[u] to the kept
// residue (rounds t >= 1, and the closing delivery after a round cap),
// reading only neighbours flagged as having pushed; a row with no such
// neighbour keeps its residue, which the previous round left at or below
// its threshold, and is skipped.  SELECT: push every pair over its
// threshold (rounds t >= 0) and flag the rows that pushed.
template <bool WEIGHTED, bool GATHER, bool SELECT>
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
    int rs = 0, dg = 0, v = 0;
    if (has_row) {
        const RowEnt e = load_row(as_global(a.rows), ri);
        rs = e.rs;
        dg = e.re - e.rs;
        v = e.v;
    }
    const uint32_t qoff = (uint32_t)q * 16u;
    const int64_t flag_off = (int64_t)slab * n;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int got = 1;
    if (GATHER) {
        const uint32_t slab_bytes = (uint32_t)n * (kSlab * 4);
        const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(a.send_in + slab_off), 0, (int)slab_bytes, 0x00020000);
        if (wide) {
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
            const float keep = 1.0f - a.alpha;
            r[0] += keep * acc.x;
            r[1] += keep * acc.y;
            r[2] += keep * acc.z;
            r[3] += keep * acc.w;
        }
        if (SELECT) {
            const float th = a.deg[v] * a.r_max;
            const float id = a.invd[v];
            float s[4], add[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bool on = r[c] > th;
                pushed += on ? 1 : 0;
                s[c] = on ? r[c] * id : 0.f;
                add[c] = on ? a.alpha * r[c] : 0.f;
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
        __shared__ int block_pushed;
        if (threadIdx.x == 0) block_pushed = 0;
        __syncthreads();
        if (pushed) block_pushed = 1;
        __syncthreads();
        if (threadIdx.x == 0 && block_pushed) a.active[a.t] = 1;
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

// out[i][j] = (sum over chunks of part[j][chunk][i]) / |F(V_j)|.
__global__ void gfp_finish_kernel(const double* __restrict__ part, const int32_t* __restrict__ leaf_ptr, int32_t k,
                                  int64_t chunks, int64_t ld, float* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)k * k) return;
    const int i = (int)(idx / k), j = (int)(idx % k);
    const int64_t size = (int64_t)leaf_ptr[j + 1] - leaf_ptr[j];
    const int64_t used = (size + kGfpChunk - 1) / kGfpChunk;
    double t = 0.0;
    for (int64_t ch = 0; ch < used; ++ch) t += part[((int64_t)j * chunks + ch) * ld + i];
    out[idx] = (float)(t / (double)size);
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

template <bool GATHER, bool SELECT>
void gfp_launch_round(bool weighted, const GfpRound& a, const StreamGrid& g, hipStream_t s) {
    const dim3 grid((unsigned)((int64_t)g.row_blocks * g.slabs));
    if (weighted)
        hipLaunchKernelGGL((gfp_round_kernel<true, GATHER, SELECT>), grid, dim3(256), 0, s, a, g);
    else
        hipLaunchKernelGGL((gfp_round_kernel<false, GATHER, SELECT>), grid, dim3(256), 0, s, a, g);
}

ppr_status read_i32(const int32_t* dev, int32_t* host, size_t count, hipStream_t s) {
    PPRVIZ_HIP_TRY(hipMemcpyAsync(host, dev, sizeof(int32_t) * count, hipMemcpyDeviceToHost, s));
    PPRVIZ_HIP_TRY(hipStreamSynchronize(s));
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
    ppr_status st = validate_csr(g);
    if (st != PPR_OK) return st;
    if (k < 1 || leaf_ptr == nullptr || leaf_idx == nullptr || dppr_out == nullptr) return PPR_EINVAL;
    if (n_leaves < k || n_leaves > (int64_t)k * g->n || n_leaves >= (int64_t)INT32_MAX) return PPR_EINVAL;
    if (!(alpha > 0.0f && alpha < 1.0f) || !(r_max >= 0.0) || !std::isfinite(r_max) || max_rounds < 1)
        return PPR_EINVAL;
    if (g->n > kStreamMaxN) return PPR_EUNSUPPORTED;
    WsCursor cur{static_cast<char*>(ws), ws_bytes};
    GfpWs w;
    gfp_ws_layout(cur, g->n, k, max_rounds, &w);
    if (ws == nullptr || cur.used > ws_bytes) return PPR_EWORKSPACE;
    if (pending_error() != PPR_OK) return PPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t n = g->n;
    const int64_t ld = gfp_ld(k);

    // Leaf lists first: no output is written unless they are valid.
    int32_t info[kGfpInfo] = {0, 0, 0, 0};
    fill<int32_t>(w.info, 0, kGfpInfo, s);
    hipLaunchKernelGGL(gfp_check_ptr_kernel, dim3((unsigned)((k + 256) / 256)), dim3(256), 0, s, leaf_ptr, k,
                       n_leaves, n, w.info);
    hipLaunchKernelGGL(gfp_check_idx_kernel, dim3((unsigned)std::min<int64_t>((n_leaves + 255) / 256, 4096)),
                       dim3(256), 0, s, leaf_idx, n_leaves, n, w.info);
    // Row order by degree; the rows with more than kGfpWideDeg arcs come
    // first, and their count is read back with the check results.
    launch_degree(g->row_ptr, g->weight, n, w.deg, w.invd, s);
    stream_row_order(g->row_ptr, n, w.hist, w.rows, s);
    hipLaunchKernelGGL(gfp_wide_count_kernel, dim3(1), dim3(1), 0, s, w.hist, w.info);
    if ((st = launch_status()) != PPR_OK) return st;
    if ((st = read_i32(w.info, info, kGfpInfo, s)) != PPR_OK) return st;
    if (info[0] != 0) return PPR_EINVAL;
    const int32_t wide = info[2];

    fill<float>(w.resid, 0.f, n * ld, s);
    fill<float>(w.est, 0.f, n * ld, s);
    fill<int32_t>(w.active, 0, max_rounds, s);
    hipLaunchKernelGGL(gfp_seed_kernel, dim3((unsigned)k, (unsigned)std::min(4096, (info[1] + 255) / 256)),
                       dim3(256), 0, s,
                       leaf_ptr, leaf_idx, w.deg, n, w.resid);

    const bool weighted = g->weight != nullptr;
    const StreamGrid grid = gfp_grid(n, wide, ld);
    GfpRound a;
    a.rows = w.rows;
    a.col_idx = g->col_idx;
    a.weight = g->weight;
    a.deg = w.deg;
    a.invd = w.invd;
    a.resid = w.resid;
    a.est = w.est;
    a.active = w.active;
    a.n = n;
    a.wide = wide;
    a.wide_blocks = (wide + 3) / 4;
    a.alpha = alpha;
    a.r_max = (float)r_max;
    a.t = 0;
    a.send_in = nullptr;
    a.send_out = w.send[0];
    a.flag_in = nullptr;
    a.flag_out = w.flag[0];
    gfp_launch_round<false, true>(weighted, a, grid, s);

    // Rounds 1 .. max_rounds - 1 in growing batches; after each batch the
    // host reads the last round's count and stops when it is zero.
    int32_t launched = 1, last = -1, batch = 4;
    while (true) {
        if ((st = launch_status()) != PPR_OK) return st;
        if ((st = read_i32(w.active + launched - 1, &last, 1, s)) != PPR_OK) return st;
        if (last == 0 || launched == max_rounds) break;
        const int32_t end = std::min(max_rounds, launched + batch);
        for (int32_t t = launched; t < end; ++t) {
            a.t = t;
            a.send_in = w.send[(t - 1) & 1];
            a.send_out = w.send[t & 1];
            a.flag_in = w.flag[(t - 1) & 1];
            a.flag_out = w.flag[t & 1];
            gfp_launch_round<true, true>(weighted, a, grid, s);
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
        a.send_in = w.send[(rounds - 1) & 1];
        a.send_out = nullptr;
        a.flag_in = w.flag[(rounds - 1) & 1];
        a.flag_out = nullptr;
        gfp_launch_round<true, false>(weighted, a, grid, s);
    }

    const int64_t chunks = gfp_chunks(n);
    const int64_t used = ((int64_t)info[1] + kGfpChunk - 1) / kGfpChunk;
    hipLaunchKernelGGL(gfp_aggregate_kernel, dim3((unsigned)k, (unsigned)used), dim3(256), 0, s, w.est, n, ld,
                       leaf_ptr, leaf_idx, chunks, w.part);
    hipLaunchKernelGGL(gfp_finish_kernel, dim3((unsigned)(((int64_t)k * k + 255) / 256)), dim3(256), 0, s, w.part,
                       leaf_ptr, k, chunks, ld, dppr_out);
    const dim3 tgrid((unsigned)((n + 63) / 64), (unsigned)((k + 63) / 64));
    if (est_out) hipLaunchKernelGGL(gfp_transpose_kernel, tgrid, dim3(256), 0, s, w.est, n, k, est_out);
    if (resid_out) hipLaunchKernelGGL(gfp_transpose_kernel, tgrid, dim3(256), 0, s, w.resid, n, k, resid_out);
    if ((st = launch_status()) != PPR_OK) return st;
    if (rounds_out) *rounds_out = rounds;
    return capped ? PPR_ENOCONV : PPR_OK;
}

}  // extern "C"
