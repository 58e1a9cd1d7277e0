// Power iteration for mid-size graphs: too large for the LDS-resident tile,
// small enough that C = 4, 2 or 1 source columns of the iterate for every
// node fit in one CU's 160 KB of LDS (up to 40831 nodes).
//
// A block owns C sources and keeps Y = (1-alpha) X / d of its columns in LDS
// for all T pushes, so the iterate never goes to HBM: each push only streams
// the arc list, which all blocks share through L2.  The push is the same
// synchronous update as in the other kernels (Section 3.3's power iteration):
//     X_{t+1}[v] = alpha [v == s] + sum_{u in N(v)} w_vu Y_t[u].
//
// Preparation (once per call, on the device):
//  - rows are sorted by degree, largest first, ties by id (stable scatter);
//  - rows longer than a wave's fair share are cut into parts whose partial
//    sums are added back in a fixed order (mid_split_kernel);
//  - the rows are cut into slices of 64, one row per lane, so the rows of a
//    slice have nearly equal arc counts, and the slices are dealt to the
//    block's 16 waves longest first (mid_plan_kernel);
//  - the arcs of a slice are stored lane-interleaved (a sliced-ELL layout):
//    group g of the slice holds arcs 4g .. 4g+3 of each of its 64 rows, 4
//    16-bit entries per lane, so one 8-byte load per lane reads 4 arcs of its
//    row and a wave load is one contiguous 512-byte segment.  An entry is the
//    LDS float index u * C of the neighbour's row; rows shorter than the
//    slice point at a zero row.  Within a row, arcs are placed by LDS bank
//    class so that the lanes of one LDS pass read different banks
//    (mid_fill_kernel).  Each wave's slices are stored one after another, so
//    a wave reads one contiguous stream per push.
// A lane keeps the sums of its KS rows in registers until every wave has
// finished gathering, then writes them back (synchronous update).
#pragma once

#include "ppr_core.hpp"
#include "ppr_stream.hpp"

namespace pprviz {

constexpr int kMidThreads = 1024;
constexpr int kMidWaves = kMidThreads / kWave;
constexpr int kMidLdsFloats = 40832;  // 160 KB less the residual reduction scratch
constexpr int kMidSlotCap = 48;       // slot table stride per wave (largest KS)
constexpr int kMidGroup = 256;        // stream entries per group: 64 lanes x 4 arcs
constexpr int kMidPrefetch = 2;       // groups each lane reads ahead
constexpr int kMidKeys = 65536;       // exact degree classes of the row order
constexpr int kMidMaxParts = 1024;    // parts of split rows: they fill at most the first 16 slices

// Columns per block for an n-node graph (0: not a mid-size graph).
__host__ __device__ inline int mid_cols_for(int n) {
    if (res_cols_for(n) != 0) return 0;
    if ((int64_t)(n + 1) * 4 <= kMidLdsFloats) return 4;
    if ((int64_t)(n + 1) * 2 <= kMidLdsFloats) return 2;
    if ((int64_t)(n + 1) <= kMidLdsFloats) return 1;
    return 0;
}

// Row slots per lane: 16 waves x KS slots hold every slice of the largest
// graph of that width (160, 320, 639 slices) with 20% to spare for the deal.
__host__ __device__ constexpr int mid_slots(int C) { return C == 4 ? 12 : (C == 2 ? 24 : 48); }

__host__ __device__ inline int64_t mid_slices(int n) { return (n + 63) / 64; }

// Bound on the stream's groups.  With rows sorted by degree, slice i >= 1 is
// no wider than the smallest row of slice i-1, so 64 * width(i) is at most
// the arc count of slice i-1; the first slice adds at most 64 * (largest
// degree), and rounding up to whole groups at most 256 entries per slice.
// The parts of split rows fill at most 16 more slices, each at most as wide
// as the largest degree.  The largest degree is at most n when no row lists
// a neighbour twice; a graph that breaks the bound is flagged by the plan and
// gets NaN outputs.
inline int64_t mid_stream_groups(int n, int64_t nnz) {
    const int64_t maxdeg = nnz < (int64_t)n ? nnz : (int64_t)n;
    return (64 * 17 * (maxdeg + 4) + nnz + kMidGroup * mid_slices(n + kMidMaxParts) + kMidGroup - 1) / kMidGroup +
           kMidPrefetch;
}

// Plan (int32 words): group counts of each wave's slots, the first group of
// each wave's stream, the overflow flag, the row count after splitting and
// the number of split rows.
constexpr int kPlanStart = kMidWaves * kMidSlotCap;
constexpr int kPlanFlag = kPlanStart + kMidWaves;
constexpr int kPlanRows = kPlanFlag + 1;
constexpr int kPlanHubs = kPlanRows + 1;
constexpr int kPlanInts = kPlanHubs + 1;

// Split of long rows.  A slice is as wide as its longest row, so a slice of
// rows with hundreds of arcs gives its wave far more work than the others in
// each push, and its deal (one wave per slice pass, below) takes as long.
// Rows longer than D arcs are therefore cut into parts of D arcs (the last
// part shorter), each part a row of its own, placed ahead of all other rows
// so that they fill the first (at most 16) slices, which the deal gives to
// slot 0 of waves 0..15.  After slot 0, a part's lane writes its sum to a
// partial slot in LDS just past the iterate; after the push's barrier, one
// lane per split row adds the partials in part order (a fixed order) in
// FP64, so that a row of thousands of arcs is summed no less accurately than
// a short one, and writes the row.  D starts at half a wave's mean share of
// the arcs and doubles until the parts fit the spare LDS after the iterate
// and the first 16 slices; nothing is split when the longest row fits in a
// wave's mean share.

// One block.  Chooses D, writes the row list after splitting (parts first,
// tagged with their partial index + 1), one combine entry per split row
// (LDS byte address of the row, scale, LDS byte address of its first
// partial, part count), and clears the slot-0 partial targets.
static __global__ __launch_bounds__(1024) void mid_split_kernel(const RowEnt* __restrict__ rows, int32_t n,
                                                               int64_t nnz, int32_t C, float alpha,
                                                               const float* __restrict__ invd,
                                                               int32_t* __restrict__ plan, RowEnt* __restrict__ vrows,
                                                               int4* __restrict__ comb,
                                                               int32_t* __restrict__ part_dst,
                                                               int32_t* __restrict__ rowpos) {
    __shared__ int32_t hub_pb[kMidMaxParts];
    __shared__ int64_t sD;
    __shared__ int32_t sH, sP;
    const int tid = threadIdx.x;
    if (tid == 0) {
        // target part length: half a wave's mean share of the arcs (16 waves)
        const int64_t groups = (nnz * 11 / 10 + kMidGroup - 1) / kMidGroup;
        int64_t D = 4 * max((int64_t)2, (groups + 2 * kMidWaves - 1) / (2 * kMidWaves));
        // no split when the widest slice is no wider than a wave's mean share:
        // the deal already balances such slices
        const int64_t maxdeg = rows[0].re - rows[0].rs;
        if ((maxdeg + 3) / 4 <= groups / kMidWaves) D = INT64_MAX / 4;
        const int cap = min(kMidMaxParts, (kMidLdsFloats - (n + 1) * C) / C);
        int H = 0, P = 0;
        for (;;) {
            H = 0;
            P = 0;
            while (H < n && (int64_t)(rows[H].re - rows[H].rs) > D && P <= cap) {
                P += (int)(((int64_t)(rows[H].re - rows[H].rs) + D - 1) / D);
                ++H;
            }
            if (P <= cap && (H == n || (int64_t)(rows[H].re - rows[H].rs) <= D)) break;
            D *= 2;
        }
        int pb = 0;
        for (int h = 0; h < H; ++h) {
            hub_pb[h] = pb;
            pb += (int)(((int64_t)(rows[h].re - rows[h].rs) + D - 1) / D);
        }
        sD = D;
        sH = H;
        sP = P;
        plan[kPlanRows] = P + n - H;
        plan[kPlanHubs] = H;
    }
    __syncthreads();
    const int64_t D = sD;
    const int H = sH, P = sP;
    const int part0 = (n + 1) * C * 4;  // LDS byte address of partial slot 0
    for (int h = tid; h < H; h += 1024) {
        const RowEnt e = rows[h];
        const int m = (int)(((int64_t)(e.re - e.rs) + D - 1) / D);
        const int pb = hub_pb[h];
        for (int j = 0; j < m; ++j) {
            const int a = e.rs + (int)(j * D);
            const int b = (int)min((int64_t)e.re, (int64_t)e.rs + (j + 1) * D);
            vrows[pb + j] = RowEnt{a, b, e.v, pb + j + 1};
        }
        comb[h] = make_int4(e.v * C * 4, __float_as_int((1.0f - alpha) * invd[e.v]), part0 + pb * C * 4, m);
        rowpos[e.v] = -1;
    }
    for (int i = H + tid; i < n; i += 1024) {
        const RowEnt e = rows[i];
        vrows[P + i - H] = RowEnt{e.rs, e.re, e.v, 0};
    }
    for (int i = tid; i < kMidWaves * kWave; i += 1024) part_dst[i] = -1;
}

// Stable scatter of the rows into degree order (one block): rows go in
// chunks of 1024 ids; each chunk is sorted by (class, id) in LDS, and a row's
// place is its class's running cursor plus its rank among the chunk's rows of
// that class.  Ties in degree thus keep id order, which makes the slices, the
// arc deal below and with it every FP32 sum independent of scheduling.
// cursor: exclusive prefix sums of the class counts (stream_deg_scan_kernel).
static __global__ __launch_bounds__(1024) void mid_row_order_kernel(const int32_t* __restrict__ row_ptr, int32_t n,
                                                                   int32_t* __restrict__ cursor,
                                                                   RowEnt* __restrict__ rows) {
    __shared__ uint32_t key[1024];
    __shared__ int32_t run_start[1024];
    __shared__ int32_t base_of[1024];
    const int tid = threadIdx.x;
    for (int c0 = 0; c0 < n; c0 += 1024) {
        const int v = c0 + tid;
        uint32_t k = 0xFFFFFFFFu;
        if (v < n) {
            const int d = min(row_ptr[v + 1] - row_ptr[v], kMidKeys - 1);
            k = ((uint32_t)(kMidKeys - 1 - d) << 16) | (uint32_t)tid;
        }
        key[tid] = k;
        __syncthreads();
        for (int w = 2; w <= 1024; w <<= 1) {
            for (int j = w >> 1; j > 0; j >>= 1) {
                const int ixj = tid ^ j;
                if (ixj > tid) {
                    const uint32_t x = key[tid], y = key[ixj];
                    if ((x > y) == ((tid & w) == 0)) {
                        key[tid] = y;
                        key[ixj] = x;
                    }
                }
                __syncthreads();
            }
        }
        const uint32_t me = key[tid];
        const bool live = me != 0xFFFFFFFFu;
        const uint32_t cls = me >> 16;
        const bool first = tid == 0 || (key[tid - 1] >> 16) != cls;
        run_start[tid] = first ? tid : 0;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {  // prefix max: start of each class run
            const int x = tid >= o ? run_start[tid - o] : 0;
            __syncthreads();
            run_start[tid] = max(run_start[tid], x);
            __syncthreads();
        }
        const bool last = tid == 1023 || key[tid + 1] == 0xFFFFFFFFu || (key[tid + 1] >> 16) != cls;
        const int rs = run_start[tid];
        // the last row of each run advances its class cursor (an L2 atomic,
        // so later chunks never see a stale cached value) and hands the old
        // value to the run through LDS
        if (live && last) base_of[rs] = atomicAdd(&cursor[cls], tid - rs + 1);
        __syncthreads();
        if (live) {
            const int u = c0 + (int)(me & 0xFFFFu);
            rows[base_of[rs] + (tid - rs)] = RowEnt{row_ptr[u], row_ptr[u + 1], u, 0};
        }
        __syncthreads();
    }
}

// One block, over the rows after splitting.  Slice widths (in groups), then
// the longest-first deal of the slices to waves (wave 0; lanes 0..15 hold the
// waves' loads and slot counts; slices 0..15 go to slot 0 of waves 0..15,
// as all loads start at 0 and ties go to the lowest wave), then the stream
// offsets.
static __global__ __launch_bounds__(1024) void mid_plan_kernel(const RowEnt* __restrict__ rows,
                                                              int32_t ks, int64_t cap_groups,
                                                              int32_t* __restrict__ plan,
                                                              int32_t* __restrict__ slice_goff,
                                                              int32_t* __restrict__ slice_slot) {
    constexpr int kSlots = kMidWaves * kMidSlotCap;
    __shared__ int32_t width[kSlots];
    __shared__ int32_t slot_slice[kSlots];
    __shared__ int32_t cnt[kMidWaves];
    __shared__ int32_t flag;
    const int tid = threadIdx.x;
    const int n = plan[kPlanRows];  // rows after splitting
    const int nsl = (n + 63) / 64;
    for (int i = tid; i < kSlots; i += 1024) slot_slice[i] = -1;
    for (int i = tid; i < nsl; i += 1024) {
        int m = 1;
        for (int l = 0; l < 64; ++l) {
            const int r = i * 64 + l;
            if (r < n) m = max(m, rows[r].re - rows[r].rs);
        }
        width[i] = (m + 3) / 4;
    }
    __syncthreads();
    if (tid < kWave) {
        const int lane = tid;
        int64_t load = 0;
        int c = 0;
        for (int i = 0; i < nsl; ++i) {
            unsigned long long key =
                (lane < kMidWaves && c < ks) ? ((unsigned long long)load << 4) | (unsigned)lane : ~0ull;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long other = __shfl_xor(key, o, kWave);
                key = other < key ? other : key;
            }
            if (lane == (int)(key & 15ull)) {
                slot_slice[lane * kMidSlotCap + c] = i;
                ++c;
                load += width[i];
            }
        }
        if (lane < kMidWaves) cnt[lane] = c;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t off = 0;
        for (int w = 0; w < kMidWaves; ++w) {
            plan[kPlanStart + w] = (int32_t)(off < INT32_MAX ? off : 0);
            for (int p = 0; p < cnt[w]; ++p) {
                const int sl = slot_slice[w * kMidSlotCap + p];
                slice_goff[sl] = (int32_t)(off < INT32_MAX ? off : 0);
                slice_slot[sl] = w * kMidSlotCap + p;
                off += width[sl];
            }
        }
        flag = off + kMidPrefetch > cap_groups ? 1 : 0;
        plan[kPlanFlag] = flag;
    }
    __syncthreads();
    for (int i = tid; i < kSlots; i += 1024) {
        const int sl = slot_slice[i];
        plan[i] = (sl >= 0 && !flag) ? width[sl] : 0;
    }
}

// One wave per LDS pass of a slice (C waves per slice, M = 64 / C rows
// each): the arc stream of its rows, as LDS float indices
// u * C (weights alongside), padded with the zero row n * C; a row without
// arcs gets one arc to itself of weight 1 (the implicit self-loop).  Also the
// rows' LDS byte addresses (u * 4 C) and scales (1-alpha)/d in their slot's table.
//
// Arcs are dealt to stream positions by LDS bank class.  Row u of the tile
// starts at bank (u * C) mod 64, so its class is u mod M, M = 64 / C, and one
// LDS pass of the gather serves M lanes (256 bytes).  For each position k and
// each pass, the pass's lanes that still have arcs choose in turn (starting
// at a lane that moves with k) an arc from a class used least so far in that
// pass (0, 1, 2 or more times; the zero row read by finished lanes counts
// once), ties broken from a preferred class that moves with lane and k.  Each
// row's arcs are first bucketed by class in a scratch copy.  Only the order
// of each row's FP32 sum depends on the deal, and the deal depends only on
// the graph.
static __global__ __launch_bounds__(64) void mid_fill_kernel(
    const RowEnt* __restrict__ rows, const int32_t* __restrict__ col_idx, const float* __restrict__ weight,
    const float* __restrict__ invd, int32_t n, int32_t C, float alpha, const int32_t* __restrict__ plan,
    const int32_t* __restrict__ slice_goff, const int32_t* __restrict__ slice_slot, int32_t* __restrict__ tmp_u,
    float* __restrict__ tmp_w, uint16_t* __restrict__ sell, float* __restrict__ sellw, int2* __restrict__ vtab,
    int32_t* __restrict__ part_dst, int32_t* __restrict__ rowpos) {
    __shared__ int32_t beg[kWave][kWave];  // per lane and class: first bucketed arc
    __shared__ int32_t pos[kWave][kWave];  // per lane and class: one past the last remaining arc
    const int lane = threadIdx.x;
    if (plan[kPlanFlag] != 0) return;
    const int nv = plan[kPlanRows];  // rows after splitting
    const int M = kWave / C;
    const int passes = kWave / M;
    const int64_t sl = blockIdx.x / passes;
    if (sl >= mid_slices(nv)) return;
    const int q0 = (int)(blockIdx.x % passes) * M;  // first slice lane of this pass
    const int q = q0 + lane;                         // this lane's position in the slice
    const uint64_t full = M == 64 ? ~0ull : ((1ull << M) - 1);
    const int slot = slice_slot[sl];
    const int64_t goff = slice_goff[sl];
    const int W = 4 * plan[slot];
    const int64_t i = sl * 64 + q;
    int v = -1, rs = 0, re = 0, tag = 0;
    if (lane < M && i < nv) {
        const RowEnt e = rows[i];
        v = e.v;
        rs = e.rs;
        re = e.re;
        tag = e.pad;
    }
    const bool self = v >= 0 && re == rs;
    // bucket the row's arcs by class
    for (int c = 0; c < M; ++c) pos[lane][c] = 0;
    if (v >= 0)
        for (int e = rs; e < re; ++e) ++pos[lane][col_idx[e] & (M - 1)];
    uint64_t avail = 0;
    int run = 0;
    for (int c = 0; c < M; ++c) {
        const int k = pos[lane][c];
        beg[lane][c] = run;
        pos[lane][c] = run;
        if (k > 0) avail |= 1ull << c;
        run += k;
    }
    if (v >= 0)
        for (int e = rs; e < re; ++e) {
            const int u = col_idx[e];
            const int at = pos[lane][u & (M - 1)]++;
            tmp_u[rs + at] = u;
            if (weight) tmp_w[rs + at] = weight[e];
        }
    if (self) avail = 1ull << (v & (M - 1));
    const int zc = n & (M - 1);
    const uint32_t zero = (uint32_t)n * (uint32_t)C;
    uint2* d = reinterpret_cast<uint2*>(sell) + goff * 64 + q;
    float4* dw = sellw ? reinterpret_cast<float4*>(sellw) + goff * 64 + q : nullptr;
    uint32_t pk[4];
    float pw[4];
    // the deal runs on the scalar unit: every value below except my_c and
    // avail is wave-uniform (readfirstlane keeps the compiler from moving it
    // to vector registers)
    const int Mm1 = __builtin_amdgcn_readfirstlane(M - 1);
    const uint64_t fullS = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(full >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)full);
    const int zcS = __builtin_amdgcn_readfirstlane(zc);
    for (int k = 0; k < W; ++k) {
        int my_c = -1;
        const uint64_t live = __ballot(avail != 0);  // lanes with arcs left
        const int rot = k & Mm1;
        {
            uint64_t z = fullS, o = 0, t = 0;
            const uint64_t pm = live & fullS;
            if (pm != fullS) {  // some lane of the pass reads the zero row
                z &= ~(1ull << zcS);
                o |= 1ull << zcS;
            }
            // the pass's lanes with arcs left, in turn from lane rot
            uint64_t rest = rot == 0 ? pm : (((pm >> rot) | (pm << (Mm1 + 1 - rot))) & fullS);
            while (rest != 0) {
                const int b = __builtin_ctzll(rest);
                rest &= rest - 1;
                const int L = __builtin_amdgcn_readfirstlane((b + rot) & Mm1);
                const uint64_t a =
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(avail >> 32), L) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)avail, L);
                uint64_t m = a & z;
                if (m == 0) m = a & o;
                if (m == 0) m = a & t;
                if (m == 0) m = a;
                const int sh = (7 * (q0 + L) + 3 * k) & Mm1;
                const uint64_t r = sh == 0 ? m : (((m >> sh) | (m << (Mm1 + 1 - sh))) & fullS);
                const int c = __builtin_amdgcn_readfirstlane((__builtin_ctzll(r) + sh) & Mm1);
                my_c = lane == L ? c : my_c;
                const uint64_t bit = 1ull << c;
                if (z & bit) {
                    z &= ~bit;
                    o |= bit;
                } else if (o & bit) {
                    o &= ~bit;
                    t |= bit;
                } else {
                    t &= ~bit;
                }
            }
        }
        uint32_t u = zero;
        float w = 0.f;
        if (my_c >= 0) {
            if (self) {
                u = (uint32_t)v * (uint32_t)C;
                w = 1.f;
                avail = 0;
            } else {
                const int at = --pos[lane][my_c];
                if (at == beg[lane][my_c]) avail &= ~(1ull << my_c);
                u = (uint32_t)tmp_u[rs + at] * (uint32_t)C;
                w = weight ? tmp_w[rs + at] : 1.f;
            }
        }
        pk[k & 3] = u;
        pw[k & 3] = w;
        if ((k & 3) == 3 && lane < M) {
            d[(int64_t)(k >> 2) * 64] = make_uint2(pk[0] | (pk[1] << 16), pk[2] | (pk[3] << 16));
            if (dw) dw[(int64_t)(k >> 2) * 64] = make_float4(pw[0], pw[1], pw[2], pw[3]);
        }
    }
    if (lane < M) {
        // a part of a split row is written through its partial slot, not here
        vtab[(int64_t)slot * 64 + q] = (v >= 0 && tag == 0)
                                           ? make_int2(v * C * 4, __float_as_int((1.0f - alpha) * invd[v]))
                                           : make_int2(-1, 0);
        if (tag > 0 && slot % kMidSlotCap == 0)
            part_dst[(slot / kMidSlotCap) * kWave + q] = (n + 1) * C * 4 + (tag - 1) * C * 4;
        if (v >= 0 && tag == 0) rowpos[v] = slot * 64 + q;
    }
}

struct MidArgs {
    const int32_t* plan;
    const int32_t* rowpos;    // per node: its slot and lane, -1 when split
    const int32_t* part_dst;  // per wave and lane: LDS byte address of its slot-0 partial, or -1
    const int4* comb;         // per split row: row address, scale, first partial address, parts
    const uint16_t* sell;
    const float* sellw;  // nullptr: unit weights
    const int2* vtab;
    const float* invd;
    const float* deg;
    const int32_t* src;  // nullptr: column s is node s
    const int32_t* tgt;  // nullptr: all nodes
    int32_t n;
    int32_t n_src;
    int32_t n_tgt;
    int32_t T;
    float alpha;
    float* ppr_out;
    float* dppr_out;
    double* resid;
};

// acc += w * Y[idx .. idx + C) (w = 1: plain sum).
template <int C, bool WEIGHTED>
__device__ __forceinline__ void mid_arc(const float* L, uint32_t idx, float w, float (&acc)[C]) {
    if constexpr (C == 4) {
        const float4 y = *reinterpret_cast<const float4*>(L + idx);
        if (WEIGHTED) {
            acc[0] = fmaf(w, y.x, acc[0]);
            acc[1] = fmaf(w, y.y, acc[1]);
            acc[2] = fmaf(w, y.z, acc[2]);
            acc[3] = fmaf(w, y.w, acc[3]);
        } else {
            acc[0] += y.x;
            acc[1] += y.y;
            acc[2] += y.z;
            acc[3] += y.w;
        }
    } else if constexpr (C == 2) {
        const float2 y = *reinterpret_cast<const float2*>(L + idx);
        if (WEIGHTED) {
            acc[0] = fmaf(w, y.x, acc[0]);
            acc[1] = fmaf(w, y.y, acc[1]);
        } else {
            acc[0] += y.x;
            acc[1] += y.y;
        }
    } else {
        const float y = L[idx];
        acc[0] = WEIGHTED ? fmaf(w, y, acc[0]) : acc[0] + y;
    }
}

template <int C, bool WEIGHTED>
__global__ __launch_bounds__(kMidThreads) void ppr_mid_kernel(MidArgs a) {
    constexpr int KS = mid_slots(C);
    __shared__ __attribute__((aligned(16))) float L[kMidLdsFloats];
    __shared__ double red[kMidWaves][4];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int n = a.n;
    const int T = a.T;
    const float alpha = a.alpha;
    const int s0 = blockIdx.x * C;
    int sn[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sn[c] = s0 + c < a.n_src ? (a.src ? a.src[s0 + c] : s0 + c) : -1;
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    int sa[C];  // LDS byte address of each source's row (-8: no source)
#pragma unroll
    for (int c = 0; c < C; ++c) sa[c] = sn[c] >= 0 ? sn[c] * C * 4 : -8;
    // slot and lane holding each source's row (-1: none, or a split row,
    // which its combining lane handles)
    int sslot[C], slane[C];  // slot of this wave (-1: another wave's or none) and lane
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int sp = __builtin_amdgcn_readfirstlane(sn[c] >= 0 ? a.rowpos[sn[c]] : -1);
        sslot[c] = (sp >= 0 && (sp >> 6) / kMidSlotCap == wvu) ? (sp >> 6) % kMidSlotCap : -1;
        slane[c] = sp & 63;
    }

    if (a.plan[kPlanFlag] != 0) {  // stream bound exceeded (repeated arcs): no result
        const float nan = __int_as_float(0x7fc00000);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (sn[c] < 0) break;
            const int64_t row = (int64_t)(s0 + c) * a.n_tgt;
            for (int j = tid; j < a.n_tgt; j += kMidThreads) {
                if (a.ppr_out) a.ppr_out[row + j] = nan;
                if (a.dppr_out) a.dppr_out[row + j] = nan;
            }
            if (a.resid && tid == 0) a.resid[s0 + c] = (double)nan;
        }
        return;
    }

    for (int i = tid; i < (n + 1) * C; i += kMidThreads) L[i] = 0.f;
    __syncthreads();
    // X after the first push is alpha at each source; the buffer holds Y of
    // it, or X itself when that push is the last
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (tid == c && T >= 1 && sn[c] >= 0)
            L[sn[c] * C + c] = T == 1 ? alpha : alpha * (1.0f - alpha) * a.invd[sn[c]];
    __syncthreads();

    const int gtab = lane < KS ? a.plan[wv * kMidSlotCap + lane] : 0;
    const int pdst = a.part_dst[tid];  // slot-0 partial target of this lane (parts of split rows)
    int4 cmb = make_int4(-1, 0, 0, 0);  // split row this lane combines, if any
    if (tid < a.plan[kPlanHubs]) cmb = a.comb[tid];
    const int64_t start = a.plan[kPlanStart + wv];
    using f4v = float __attribute__((ext_vector_type(4)));
    const gcptr<uint64_t> sbase = as_global(reinterpret_cast<const uint64_t*>(a.sell)) + start * 64 + lane;
    const gcptr<f4v> wbase = WEIGHTED ? as_global(reinterpret_cast<const f4v*>(a.sellw)) + start * 64 + lane : nullptr;
    // slot table of this wave: a scalar base per 8 slots plus the lane's
    // byte offset, so that its addresses take no vector registers
    const int64_t vt_wave = (int64_t)reinterpret_cast<uintptr_t>(a.vtab) + (int64_t)wvu * kMidSlotCap * 64 * 8;

    float acc[KS][C];
    for (int it = 1; it < T; ++it) {
        // ring of the next kMidPrefetch groups of this wave's stream (it runs
        // on across slot boundaries: the wave's slices are stored in order)
        constexpr int D = kMidPrefetch;
        gcptr<uint64_t> sp = sbase + D * 64;
        uint64_t q[D];
#pragma unroll
        for (int j = 0; j < D; ++j) q[j] = sbase[j * 64];
        gcptr<f4v> wp = nullptr;
        f4v r[D];
#pragma unroll
        for (int j = 0; j < D; ++j) r[j] = f4v{1.f, 1.f, 1.f, 1.f};
        if (WEIGHTED) {
            wp = wbase + D * 64;
#pragma unroll
            for (int j = 0; j < D; ++j) r[j] = wbase[j * 64];
        }
#pragma unroll
        for (int p = 0; p < KS; ++p) {
#pragma unroll
            for (int c = 0; c < C; ++c) acc[p][c] = 0.f;
            const int gp = __builtin_amdgcn_readlane(gtab, p);
            for (int i = 0; i < gp; ++i) {
                const uint64_t cur = q[0];
#pragma unroll
                for (int j = 0; j + 1 < D; ++j) q[j] = q[j + 1];
                q[D - 1] = *sp;
                sp += 64;
                f4v cw = r[0];
                if (WEIGHTED) {
#pragma unroll
                    for (int j = 0; j + 1 < D; ++j) r[j] = r[j + 1];
                    r[D - 1] = *wp;
                    wp += 64;
                }
                const uint32_t lo = (uint32_t)cur, hi = (uint32_t)(cur >> 32);
                mid_arc<C, WEIGHTED>(L, lo & 0xffffu, cw.x, acc[p]);
                mid_arc<C, WEIGHTED>(L, lo >> 16, cw.y, acc[p]);
                mid_arc<C, WEIGHTED>(L, hi & 0xffffu, cw.z, acc[p]);
                mid_arc<C, WEIGHTED>(L, hi >> 16, cw.w, acc[p]);
            }
            if (p == 0 && pdst >= 0) {  // a part of a split row: its sum goes to its partial slot
                float* dst = reinterpret_cast<float*>(reinterpret_cast<char*>(L) + pdst);
#pragma unroll
                for (int c = 0; c < C; ++c) dst[c] = acc[0][c];
            }
        }
        // write-back: the slot table (LDS byte address of the row, scale
        // (1-alpha)/d) is read in batches of 8 slots, each batch loaded one
        // batch ahead; the first batch is in flight across the barrier
        const bool fin = it == T - 1;
        const uint32_t lane8 = (uint32_t)opaque(lane * 8);
        constexpr int NB = (KS + 7) / 8;
        uint64_t e[2][8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < KS)
                e[0][j] = *reinterpret_cast<gcptr<uint64_t>>(reinterpret_cast<gcptr<char>>(opaque_s(vt_wave)) +
                                                             lane8 + j * 512);
        __syncthreads();
#pragma unroll
        for (int bt = 0; bt < NB; ++bt) {
            if (bt + 1 < NB) {
                const int64_t vsb = opaque_s(vt_wave + (int64_t)(bt + 1) * 8 * 512);
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if ((bt + 1) * 8 + j < KS)
                        e[(bt + 1) & 1][j] =
                            *reinterpret_cast<gcptr<uint64_t>>(reinterpret_cast<gcptr<char>>(vsb) + lane8 + j * 512);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int p = bt * 8 + j;
                if (p < KS && __builtin_amdgcn_readlane(gtab, p) > 0) {
                    // the restart term alpha at the block's source rows: a
                    // wave-uniform test of the slot, then the one lane
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        if (opaque_s32(sslot[c]) == p)
                            if (lane == slane[c]) acc[p][c] += alpha;
                    const int addr = (int)(uint32_t)e[bt & 1][j];
                    if (addr >= 0) {
                        const float sc = fin ? 1.0f : __int_as_float((int)(uint32_t)(e[bt & 1][j] >> 32));
                        float* dst = reinterpret_cast<float*>(reinterpret_cast<char*>(L) + addr);
#pragma unroll
                        for (int c = 0; c < C; ++c) dst[c] = acc[p][c] * sc;
                    }
                }
            }
        }
        if (cmb.x >= 0) {  // split row: its parts' partial sums in part order, in FP64
            double x[C];
#pragma unroll
            for (int c = 0; c < C; ++c) x[c] = 0.0;
            const float* pp = reinterpret_cast<const float*>(reinterpret_cast<const char*>(L) + cmb.z);
            for (int j = 0; j < cmb.w; ++j)
#pragma unroll
                for (int c = 0; c < C; ++c) x[c] += (double)pp[j * C + c];
            const float sc = fin ? 1.0f : __int_as_float(cmb.y);
            float* dst = reinterpret_cast<float*>(reinterpret_cast<char*>(L) + cmb.x);
#pragma unroll
            for (int c = 0; c < C; ++c) dst[c] = ((float)x[c] + (cmb.x == sa[c] ? alpha : 0.f)) * sc;
        }
        __syncthreads();
    }

    // X is now in LDS (zero when T = 0).  FP64 residual 1 - sum_v X[v, s] in
    // a fixed order: rows strided over threads, then waves in order.
    double part[C];
#pragma unroll
    for (int c = 0; c < C; ++c) part[c] = 0.0;
    for (int v = tid; v < n; v += kMidThreads)
#pragma unroll
        for (int c = 0; c < C; ++c) part[c] += (double)L[v * C + c];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        part[c] = wave_sum(part[c]);
        if (lane == 0) red[wv][c] = part[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (tid == c && sn[c] >= 0 && a.resid) {
            double t = 0.0;
            for (int w = 0; w < kMidWaves; ++w) t += red[w][c];
            a.resid[s0 + c] = 1.0 - t;
        }
    }
    // outputs: row s of pi_hat / DPPR over the targets, coalesced
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (sn[c] < 0) break;
        const int64_t row = (int64_t)(s0 + c) * a.n_tgt;
        const float ds = a.dppr_out ? a.deg[sn[c]] : 0.f;
        for (int j = tid; j < a.n_tgt; j += kMidThreads) {
            const int t = a.tgt ? a.tgt[j] : j;
            const float x = L[t * C + c];
            if (a.ppr_out) a.ppr_out[row + j] = x;
            if (a.dppr_out) a.dppr_out[row + j] = x * ds;
        }
    }
}

// Graph-side preparation (row order, plan, arc stream) and the launch.
struct MidWs {
    RowEnt* rows;
    int32_t* hist;        // kMidKeys
    int32_t* plan;        // kPlanInts
    int32_t* slice_goff;  // mid_slices(n)
    int32_t* slice_slot;  // mid_slices(n)
    int2* vtab;           // kMidWaves * kMidSlotCap * 64: (LDS byte address of the row, scale)
    uint16_t* sell;       // mid_stream_groups * kMidGroup
    float* sellw;         // same, weighted graphs only
    int32_t* tmp_u;       // nnz: arcs bucketed by bank class
    float* tmp_w;         // nnz, weighted graphs only
    RowEnt* vrows;        // n + kMidMaxParts: rows after splitting long rows
    int4* comb;           // kMidMaxParts: one entry per split row
    int32_t* part_dst;    // kMidWaves * 64: slot-0 partial targets
    int32_t* rowpos;      // n: (wave * kMidSlotCap + slot) * 64 + lane of each row, -1 for split rows
};

template <int C, bool W>
inline void mid_launch(const MidArgs& a, hipStream_t s) {
    const unsigned blocks = (unsigned)((a.n_src + C - 1) / C);
    hipLaunchKernelGGL((ppr_mid_kernel<C, W>), dim3(blocks), dim3(kMidThreads), 0, s, a);
}

inline void mid_forward(const ppr_csr* g, const int32_t* src, int32_t n_src, const int32_t* tgt, int32_t n_tgt,
                        float alpha, int32_t T, float* ppr_out, float* dppr_out, const float* deg,
                        const float* invd, double* resid, const MidWs& w, hipStream_t s) {
    const int n = g->n;
    const int C = mid_cols_for(n);
    const bool weighted = g->weight != nullptr;
    fill<int32_t>(w.hist, 0, kMidKeys, s);
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(stream_deg_hist_kernel<kMidKeys>, dim3(nb), dim3(256), 0, s, g->row_ptr, n, w.hist);
    hipLaunchKernelGGL(stream_deg_scan_kernel<kMidKeys>, dim3(1), dim3(1024), 0, s, w.hist);
    hipLaunchKernelGGL(mid_row_order_kernel, dim3(1), dim3(1024), 0, s, g->row_ptr, n, w.hist, w.rows);
    hipLaunchKernelGGL(mid_split_kernel, dim3(1), dim3(1024), 0, s, w.rows, n, g->nnz, C, alpha, invd, w.plan,
                       w.vrows, w.comb, w.part_dst, w.rowpos);
    hipLaunchKernelGGL(mid_plan_kernel, dim3(1), dim3(1024), 0, s, w.vrows, mid_slots(C),
                       mid_stream_groups(n, g->nnz), w.plan, w.slice_goff, w.slice_slot);
    hipLaunchKernelGGL(mid_fill_kernel, dim3((unsigned)(mid_slices(n + kMidMaxParts) * C)), dim3(64), 0, s,
                       w.vrows, g->col_idx, g->weight, invd, n, C, alpha, w.plan, w.slice_goff, w.slice_slot,
                       w.tmp_u, weighted ? w.tmp_w : nullptr, w.sell, weighted ? w.sellw : nullptr, w.vtab,
                       w.part_dst, w.rowpos);
    MidArgs a;
    a.plan = w.plan;
    a.part_dst = w.part_dst;
    a.rowpos = w.rowpos;
    a.comb = w.comb;
    a.sell = w.sell;
    a.sellw = weighted ? w.sellw : nullptr;
    a.vtab = w.vtab;
    a.invd = invd;
    a.deg = deg;
    a.src = src;
    a.tgt = tgt;
    a.n = n;
    a.n_src = n_src;
    a.n_tgt = n_tgt;
    a.T = T;
    a.alpha = alpha;
    a.ppr_out = ppr_out;
    a.dppr_out = dppr_out;
    a.resid = resid;
    if (C == 4) {
        if (weighted) mid_launch<4, true>(a, s); else mid_launch<4, false>(a, s);
    } else if (C == 2) {
        if (weighted) mid_launch<2, true>(a, s); else mid_launch<2, false>(a, s);
    } else {
        if (weighted) mid_launch<1, true>(a, s); else mid_launch<1, false>(a, s);
    }
}

}  // namespace pprviz
