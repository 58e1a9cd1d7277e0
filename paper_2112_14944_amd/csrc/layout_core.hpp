// Device-side PDist formula and the pairwise layout / stress / gradient row
// kernels, shared by the single-layout entry points and the batched path.
#pragma once

#include "common.hpp"

namespace pprviz {

// Upper clamp 2 ln n of Eq. eq:pprdist, evaluated in FP64 and rounded once.
__device__ __forceinline__ float pdist_hi(int64_t n_clamp) { return (float)(2.0 * log((double)n_clamp)); }

// Eq. eq:pprdist: min(max(1 - ln z, 2), 2 ln n); an unreachable pair (z <= 0)
// takes the upper bound.  NaN stays NaN.
__device__ __forceinline__ float pdist_value(float z, float hi) {
    if (z != z) return z;
    if (!(z > 0.f)) return hi;
    const float raw = 1.0f - logf(z);
    return fminf(fmaxf(raw, 2.0f), hi);
}

// dDelta/dz: -1/z strictly inside the clamp range, 0 on or beyond the kinks.
__device__ __forceinline__ float pdist_dz(float z, float hi) {
    if (!(z > 0.f)) return 0.f;
    const float raw = 1.0f - logf(z);
    return (raw > 2.0f && raw < hi) ? -1.0f / z : 0.0f;
}

enum {
    kLayoutStep = 0,        // x_out only
    kLayoutStepStress = 1,  // x_out and stress partials of x_in
    kLayoutStress = 2,      // stress partials only
    kLayoutGradX = 3,       // dL/dX
    kLayoutGradBoth = 4,    // dL/dX (optional) and dL/dDelta
    kLayoutWsum = 5,        // per-row sum_j Delta_ij^-2 (the diagonal of L^w)
};

// Added to every squared distance before the reciprocal square root, so that
// a coincident pair (and the diagonal) gets a finite 1/d; its direction term
// c * (X_i - X_j) is then exactly zero because X_i - X_j is.  For squared
// distances above ~2e-23 the term is below half an ulp and changes nothing
// beyond the rounding of the sum itself.
constexpr float kMinSq = 1e-30f;

constexpr int kLayoutRowsPerWave = 4;
constexpr int kLayoutRowsPerBlock = 4 * kLayoutRowsPerWave;

// Work of one pair (i, j), accumulated into the row's running sums (see
// layout_rows for the formulas).
template <int MODE, bool INV>
__device__ __forceinline__ void layout_pair(float Dv, bool off, float2 xi, float2 xj, float& ax, float& ay,
                                            float& aw, float& as, float scale, float* gd_ij) {
    constexpr bool STEP = (MODE == kLayoutStep || MODE == kLayoutStepStress);
    constexpr bool STRESS = (MODE == kLayoutStepStress || MODE == kLayoutStress);
    constexpr bool GRAD = (MODE == kLayoutGradX || MODE == kLayoutGradBoth);
    constexpr bool WSUM = (MODE == kLayoutWsum);
    constexpr bool acc_w = WSUM || (STEP && !INV);
    const float inv = INV ? Dv : (off ? __builtin_amdgcn_rcpf(Dv) : 0.f);
    const float w = inv * inv;
    if (acc_w) aw += w;
    if (WSUM) return;
    const float dx = xi.x - xj.x;
    const float dy = xi.y - xj.y;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, kMinSq));
    const float rs = __builtin_amdgcn_rsqf(r2);
    if (STEP) {
        const float c = inv * rs;
        ax = fmaf(w, xj.x, fmaf(c, dx, ax));
        ay = fmaf(w, xj.y, fmaf(c, dy, ay));
    }
    if (STRESS || GRAD) {
        const float d = r2 * rs;
        const float t = fmaf(-d, inv, 1.0f);
        if (STRESS) as = off ? fmaf(t, t, as) : as;
        if (GRAD) {
            const float g = 2.0f * (d - Dv) * w * rs;
            ax = fmaf(g, dx, ax);
            ay = fmaf(g, dy, ay);
            if (MODE == kLayoutGradBoth) *gd_ij = off ? scale * 2.0f * t * d * w : 0.f;
        }
    }
}

// Pairwise work of 4 consecutive rows i (one wave) against all j of a
// k-node layout.  Lanes stride over j, so each row of Delta is read
// coalesced and each X_j load serves 4 rows.
//   step:   X+_i = (sum_j w X_j + c (X_i - X_j)) / sum_j w,
//           w = Delta^-2, c = w Delta / d = Delta^-1 d^-1  (Jacobi sweep of
//           L^w X = L^Y Y; a coincident pair adds only w X_j)
//   stress: sum_{j != i} (1 - d/Delta)^2, halved per unordered pair
//   grad:   dL/dX_i = sum_j 2 w (d - Delta) (X_i - X_j)/d,
//           dL/dDelta_ij = 2 (1 - d/Delta) d / Delta^2
// INV: `delta` holds 1/Delta with a zero diagonal (precomputed once for many
// sweeps) instead of Delta.  wsum: per-row sum_j w written by the kLayoutWsum
// pass (same summation order); a step with INV reads it from there, a step
// without INV accumulates it itself.
// Full groups of 4 rows take a branch-free path that issues the loads of 4
// columns (16 Delta values, 4 positions) before their arithmetic.
// Returns this wave's stress contribution (lane 0 holds the wave total).
template <int MODE, bool INV>
__device__ __forceinline__ double layout_rows(const float* __restrict__ delta, int64_t ld, int32_t k,
                                              const float2* __restrict__ x, int row_begin,
                                              float2* __restrict__ xout, float scale,
                                              float2* __restrict__ gx, float* __restrict__ gd,
                                              float* __restrict__ wsum) {
    constexpr int R = kLayoutRowsPerWave;
    constexpr bool STEP = (MODE == kLayoutStep || MODE == kLayoutStepStress);
    constexpr bool STRESS = (MODE == kLayoutStepStress || MODE == kLayoutStress);
    constexpr bool GRAD = (MODE == kLayoutGradX || MODE == kLayoutGradBoth);
    constexpr bool WSUM = (MODE == kLayoutWsum);
    static_assert(!(INV && GRAD), "the gradient needs Delta itself");
    const int lane = threadIdx.x & 63;
    float2 xi[R];
    bool ok[R];
    float ax[R], ay[R], aw[R], as[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = row_begin + r;
        ok[r] = i < k;
        xi[r] = ok[r] ? x[i] : make_float2(0.f, 0.f);
        ax[r] = ay[r] = aw[r] = as[r] = 0.f;
    }
    int j = lane;
    if (row_begin + R <= k) {
        const float* __restrict__ drow = delta + (int64_t)row_begin * ld;
        for (; j + 3 * kWave < k; j += 4 * kWave) {
            float2 xv[4];
            float dv[4][R];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[u] = x[j + u * kWave];
#pragma unroll
                for (int r = 0; r < R; ++r) dv[u][r] = drow[(int64_t)r * ld + j + u * kWave];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int jj = j + u * kWave;
                    layout_pair<MODE, INV>(dv[u][r], jj != row_begin + r, xi[r], xv[u], ax[r], ay[r], aw[r], as[r], scale,
                                           GRAD ? gd + (int64_t)(row_begin + r) * ld + jj : nullptr);
                }
            }
        }
    }
    for (; j < k; j += kWave) {
        const float2 xj = x[j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int i = row_begin + r;
            layout_pair<MODE, INV>(delta[(int64_t)i * ld + j], j != i, xi[r], xj, ax[r], ay[r], aw[r], as[r],
                                   scale, GRAD ? gd + (int64_t)i * ld + j : nullptr);
        }
    }
    double st = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;  // wave-uniform
        const int i = row_begin + r;
        if (WSUM) {
            const float sw = wave_sum(aw[r]);
            if (lane == 0) wsum[i] = sw;
        }
        if (STEP || GRAD) {
            const float sx = wave_sum(ax[r]);
            const float sy = wave_sum(ay[r]);
            if (STEP) {
                const float sw = INV ? wsum[i] : wave_sum(aw[r]);
                if (lane == 0) xout[i] = sw > 0.f ? make_float2(sx / sw, sy / sw) : xi[r];
            } else if (gx && lane == 0) {
                gx[i] = make_float2(scale * sx, scale * sy);
            }
        }
        if (STRESS) st += wave_sum((double)as[r]);
    }
    return 0.5 * st;
}

// One block = 16 rows (4 waves x 4 rows) of one k-node layout.
template <int MODE>
__global__ __launch_bounds__(256) void layout_rows_kernel(const float* __restrict__ delta, int64_t ld, int32_t k,
                                                          const float2* __restrict__ x, float2* __restrict__ xout,
                                                          double* __restrict__ part, float scale,
                                                          float2* __restrict__ gx, float* __restrict__ gd) {
    __shared__ double red[4];
    const int wave = threadIdx.x >> 6;
    const int row_begin = blockIdx.x * kLayoutRowsPerBlock + wave * kLayoutRowsPerWave;
    const double st = layout_rows<MODE, false>(delta, ld, k, x, row_begin, xout, scale, gx, gd, nullptr);
    if (MODE == kLayoutStepStress || MODE == kLayoutStress) {
        if ((threadIdx.x & 63) == 0) red[wave] = st;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// ---------------------------------------------------------------------------
// Strip Jacobi sweep of the batch.  Delta is symmetric, so each unordered
// pair {i, j} is evaluated once and feeds both rows.  The sweep formula of
// layout_rows, X+_i = (sum_j w X_j + c (X_i - X_j)) / sum_j w with
// w = Delta^-2 and c = 1 / (Delta d), is X_i + sum_j g (X_i - X_j) / sum_j w
// with g = c - w, so a pair adds g (X_i - X_j) to row i and its negative to
// row j, and the combine step adds X_i and divides by the precomputed weight
// sum.  A pair with 1/Delta = 0 (the diagonal) has g = 0, and a coincident
// pair has X_i - X_j = 0, so neither adds anything.
//
// A strip (S, J) is the 256 rows of super-row S, as four 64-row blocks
// A = 4 S + r, against the 64 columns of block J (J >= 4 S).  Lane l holds
// the four consecutive rows 256 S + 4 l .. + 3 (all in block 4 S + l / 16),
// and the wave walks the columns j, reading 1/Delta[j][i] for its four rows
// with one 16-byte load (together one contiguous 1 KB piece of row j).  Row
// block A takes every pair with the columns when A < J and feeds both ends,
// its ordered pairs only when A == J (the diagonal block: rows only, each
// pair seen from both ends), and nothing when A > J (the strip of J's
// super-row has those pairs).  Column sums of 8 columns at a time go through
// a small LDS block, where 8 lanes per column add 8 lanes' partials each and
// three lane exchanges finish the column.
//
// A task is up to kStripGroup consecutive strips of one super-row, J0 = 4 S +
// kStripGroup m .. J0 + nJ - 1: row sums stay in registers across its column
// blocks, so a row's partial is written once per task, not once per strip
// (the sweep is bound by its 1/Delta stream, and writes interleaved with that
// stream cost far more read bandwidth than their bytes).
//
// Partials, 64 floats per slot and component in a [T][T] grid per subgraph:
// row block A's sum over a task's columns goes to slot (A, max(A, J0)) (the
// diagonal task J0 = 4 S into (A, A), the others into (A, J0) with J0 > A);
// column block J's sum over super-row S goes to (J, S), written only for
// J > 4 S (where some row block lies left of J).  Row slots have a second
// index >= A and column slots one < A / 4 + 1 <= A, so the two never meet.
// strip_finalize adds a node's slots in one fixed order, so the result does
// not depend on which wave ran which task.
constexpr int kPT = 64;
constexpr int kStripBlocks = 4;
constexpr int kPTChunk = 8;     // columns per LDS column exchange
constexpr int kStripGroup = 4;  // column blocks per task

// Tasks of a subgraph with T column blocks: super-row S (of U = ceil(T / 4))
// holds U - S of them.
__host__ __device__ __forceinline__ int64_t strip_task_count(int64_t T) {
    const int64_t U = (T + kStripBlocks - 1) / kStripBlocks;
    return U * (U + 1) / 2;
}

// Task index t of a T-block subgraph -> (S, J0).
__device__ __forceinline__ void strip_task_sj(int t, int T, int& S, int& J0) {
    const int U = (T + kStripBlocks - 1) / kStripBlocks;
    int s = 0;
    while (t >= U - s) {
        t -= U - s;
        ++s;
    }
    S = s;
    J0 = kStripBlocks * s + kStripGroup * t;
}

enum { kPairStep = 0, kPairW = 1 };

// LDS of one wave for the column sums of one 8-column chunk.
template <int MODE>
struct StripLds;
template <>
struct StripLds<kPairStep> {
    float2 v[kPTChunk][kWave];
};
template <>
struct StripLds<kPairW> {
    float v[kPTChunk][kWave];
};

// Byte offset past every subgraph block of the 1/Delta pool: a buffer load
// there returns 0 and touches no memory.
constexpr uint32_t kStripOutside = 0x80000000u;

// What the column exchange of a task needs.
struct StripCtx {
    int lane, S, T, cc, cp;
    __amdgpu_buffer_rsrc_t prx, pry;  // the subgraph's partial blocks ([T][T][64] floats each)
};

typedef unsigned int StripU4 __attribute__((ext_vector_type(4)));

// s_waitcnt immediate that waits until at most N vector memory operations
// are outstanding and leaves the export and LDS/scalar counters alone
// (vmcnt in bits 3:0 and 15:14, expcnt 6:4 = 7, lgkmcnt 11:8 = 15).
template <int N>
constexpr int kWaitVmcnt = (N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8);

// A task's row partials, stored by the next task of the same wave once that
// task's loads are in flight.  Loads and stores retire in one ordered count,
// so a store issued at the end of a task would hold up the first wait of the
// next one until the write is acknowledged.
struct StripPend {
    StripU4 vx, vy;
    __amdgpu_buffer_rsrc_t rx, ry;
    int off;  // byte offset in the partial blocks; kStripOutside: nothing to store
};

// Nothing pending: stores through empty resources.
__device__ __forceinline__ StripPend strip_pend_none(float* __restrict__ any) {
    StripPend p;
    p.vx = p.vy = StripU4{0u, 0u, 0u, 0u};
    p.rx = p.ry = __builtin_amdgcn_make_buffer_rsrc(any, 0, 0, 0x00020000);
    p.off = (int)kStripOutside;
    return p;
}

template <int MODE>
__device__ __forceinline__ void strip_pend_issue(const StripPend& p) {
    __builtin_amdgcn_raw_buffer_store_b128(p.vx, p.rx, p.off, 0, 0);
    if (MODE == kPairStep) __builtin_amdgcn_raw_buffer_store_b128(p.vy, p.ry, p.off, 0, 0);
}

// Buffer resources over the partial blocks, so that a store from an idle
// lane goes outside them instead of behind a branch.
template <int MODE>
__device__ __forceinline__ void strip_part_rsrc(StripCtx& t, float* __restrict__ px, float* __restrict__ py) {
    const int bytes = t.T * t.T * kPT * 4;
    t.prx = __builtin_amdgcn_make_buffer_rsrc(px, 0, bytes, 0x00020000);
    t.pry = __builtin_amdgcn_make_buffer_rsrc(MODE == kPairStep ? py : px, 0, bytes, 0x00020000);
}

// Column sums of one chunk (columns c .. c + 7 of block J, ncol of whose
// columns exist): lane (cc, cp) adds the partials of lanes 8 cp .. 8 cp + 7
// for column cc, starting at lane 8 cp + cp so that the 8 lanes of a column
// read 8 different bank groups, and three lane exchanges give every lane of
// the group the column total.  Lane l keeps the total of column l of the
// block (colx, coly), taken in the chunk that holds it, and the block's last
// chunk (jend) stores the 64 totals as one 256-byte row per component into
// slot (J, S), when J > 4 S (before that no row block lies left of J and the
// sums are zero): whole lines, since lines written piecemeal while the
// 1/Delta stream runs cost far more than their bytes.
template <int MODE>
__device__ __forceinline__ void strip_columns(const StripCtx& t, int J, int c, int ncol, bool jend, float& colx,
                                              float& coly, StripLds<MODE>& L) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    float sx = 0.f, sy = 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = t.cp * 8 + ((u + t.cp) & 7);
        if constexpr (MODE == kPairStep) {
            const float2 v = L.v[t.cc][r];
            sx += v.x;
            sy += v.y;
        } else {
            sx += L.v[t.cc][r];
        }
    }
    sx += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sx), 0xB1, 0xf, 0xf, false));
    sx += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sx), 0x4E, 0xf, 0xf, false));
    sx += __shfl_xor(sx, 4, kWave);
    if (MODE == kPairStep) {
        sy += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sy), 0xB1, 0xf, 0xf, false));
        sy += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sy), 0x4E, 0xf, 0xf, false));
        sy += __shfl_xor(sy, 4, kWave);
    }
    // column c + (l % 8) is held by lanes 8 (l % 8) .. + 7; lane l keeps it
    // when it is column l, i.e. in chunk l / 8 of the block
    const int src = 8 * (t.lane & 7);
    const bool mine = (t.lane >> 3) == (c >> 3);
    const float vx = __shfl(sx, src, kWave);
    colx = mine ? vx : colx;
    if (MODE == kPairStep) {
        const float vy = __shfl(sy, src, kWave);
        coly = mine ? vy : coly;
    }
    const bool wr = jend && t.lane < ncol && J > kStripBlocks * t.S;
    const int o = wr ? ((J * t.T + t.S) * kPT + t.lane) * 4 : (int)kStripOutside;
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(colx), t.prx, o, 0, 0);
    if (MODE == kPairStep) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(coly), t.pry, o, 0, 0);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// A task in 16-byte form: lane l owns rows 256 S + 4 l .. + 3 of row block
// A = 4 S + l / 16 and reads a column's four values with one 16-byte buffer
// load; the task's columns (64 J0 on, nJ blocks) are one sequence of 8-column
// chunks.  MASKED = false is a task whose 256 rows all lie in the subgraph
// and left of J0 and whose columns all exist (the bulk of every large
// subgraph).  MASKED = true is any other task: for column block J, lanes
// with A > J read zeros (offset outside the resource); lanes of the diagonal
// block A == J add to their own rows only, so their column terms are dropped
// at the exchange; columns past k read zeros through the scalar offset, and
// rows from k to the padded row length read the zeros written into the
// padding of the 1/Delta rows.
//
// No memory operation depends on a branch: the prefetch after the last
// chunk reads past the task's columns, which returns zeros without a memory
// access, and partial stores of idle lanes go outside their resource.  The
// compiler then waits for exactly the loads a chunk uses, with the next
// chunk's loads still in flight.
template <int MODE, bool MASKED>
__device__ __forceinline__ void strip_task_body(const float* __restrict__ m, int64_t ld, int32_t k,
                                                const float2* __restrict__ x, int S, int J0, int T,
                                                float* __restrict__ px, float* __restrict__ py, StripLds<MODE>& L,
                                                StripPend& pend) {
    constexpr int H = kPTChunk / 2;
    const int lane = threadIdx.x & 63;
    const int A = S * kStripBlocks + lane / 16;
    const int nJ = min(kStripGroup, T - J0);
    const int c0 = S * kStripBlocks * kPT;
    const int i0 = c0 + 4 * lane;
    const int j0 = J0 * kPT;
    // columns of the task that exist (at least one)
    const int ncol = MASKED ? min(kPT * nJ, k - j0) : kPT * nJ;
    // Positions of the lane's rows and of the task's columns (one float2 per
    // lane and column block), through a buffer resource over the subgraph's
    // k positions: rows and columns past k read zeros, and unlike plain loads
    // from a read-only pointer these stay in place relative to the task's
    // loads and stores (no load sits behind a branch, and the first wait
    // finds only them ahead of the 1/Delta loads).
    float2 xi[4];
    float2 xc[kStripGroup];
    if constexpr (MODE == kPairStep) {
        const __amdgpu_buffer_rsrc_t xr =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(x), 0, k * 8, 0x00020000);
        if constexpr (MASKED) {
            // clamped so that no load is partly outside the resource (and the
            // four cannot be fused into wider ones); rows past k take 0
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b64(xr, min(i0 + r, k - 1) * 8, 0, 0);
                const bool ok = i0 + r < k;
                xi[r] = make_float2(ok ? __uint_as_float(v[0]) : 0.f, ok ? __uint_as_float(v[1]) : 0.f);
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const StripU4 v = __builtin_amdgcn_raw_buffer_load_b128(xr, i0 * 8 + 16 * h, 0, 0);
                xi[2 * h] = make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
                xi[2 * h + 1] = make_float2(__uint_as_float(v[2]), __uint_as_float(v[3]));
            }
        }
#pragma unroll
        for (int b = 0; b < kStripGroup; ++b) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(xr, (j0 + b * kPT + lane) * 8, 0, 0);
            xc[b] = make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) xi[r] = make_float2(0.f, 0.f);
#pragma unroll
        for (int b = 0; b < kStripGroup; ++b) xc[b] = make_float2(0.f, 0.f);
    }
    asm volatile("" ::: "memory");  // the position loads go out before the task's
    StripCtx t;
    t.lane = lane;
    t.S = S;
    t.T = T;
    t.cc = lane >> 3;
    t.cp = lane & 7;
    strip_part_rsrc<MODE>(t, px, py);
    const __amdgpu_buffer_rsrc_t mr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(m + c0), 0, (int)(((int64_t)k * ld - c0) * 4), 0x00020000);
    const bool rowok = !MASKED || i0 < ld;
    // four loads of columns cg .. cg + 3 (one column block: 64 is a multiple of 4)
    auto load4 = [&](int cg, StripU4 (&v)[H]) {
        const int voff = (!MASKED || (rowok && A <= J0 + cg / kPT)) ? 16 * lane : (int)kStripOutside;
#pragma unroll
        for (int s = 0; s < H; ++s) {
            const int c = cg + s;
            const int soff = c < ncol ? (int)((int64_t)(j0 + c) * ld * 4) : (int)(kStripOutside >> 1);
            v[s] = __builtin_amdgcn_raw_buffer_load_b128(mr, voff, soff, 0);
        }
    };
    float ax[4] = {0.f, 0.f, 0.f, 0.f}, ay[4] = {0.f, 0.f, 0.f, 0.f};
    float colx = 0.f, coly = 0.f;  // total of column l of the current block (lane l)
    // The loop is entered with the memory operations outstanding in the order
    // its back edge leaves them: four loads of the first half-chunk, four of
    // the second, then as many stores as a chunk's column exchange makes (here
    // the previous task's row partials).  The compiler merges the two orders
    // when it places its waits; with the same order each wait covers only the
    // loads a column uses.
    StripU4 ha[H], hb[H];
    load4(0, ha);
    asm volatile("" ::: "memory");
    load4(H, hb);
    asm volatile("" ::: "memory");
    strip_pend_issue<MODE>(pend);
    // wait here for the positions only, so that they are not pending when the
    // loop is entered
    constexpr int kInFlight = 2 * H + (MODE == kPairStep ? 2 : 1);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt<kInFlight>);
    asm volatile("" ::: "memory");
    float2 xcol = xc[0];
    auto math = [&](const StripU4 (&v)[H], int cb, int s0, bool full) {
#pragma unroll
        for (int s = 0; s < H; ++s) {
            float cx = 0.f, cy = 0.f;
            float2 xj = make_float2(0.f, 0.f);
            if (MODE == kPairStep) {
                // the column's position from the lane that loaded it: no
                // memory access inside the loop besides the 1/Delta stream
                xj.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xcol.x), cb + s));
                xj.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xcol.y), cb + s));
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float inv = __uint_as_float(v[s][r]);
                const float w = inv * inv;
                if (MODE == kPairStep) {
                    const float dx = xi[r].x - xj.x;
                    const float dy = xi[r].y - xj.y;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, kMinSq));
                    const float g = fmaf(inv, __builtin_amdgcn_rsqf(r2), -w);
                    ax[r] = fmaf(g, dx, ax[r]);
                    ay[r] = fmaf(g, dy, ay[r]);
                    cx = fmaf(-g, dx, cx);
                    cy = fmaf(-g, dy, cy);
                } else {
                    ax[r] += w;
                    cx += w;
                }
            }
            if (MASKED) {
                cx = full ? cx : 0.f;
                cy = full ? cy : 0.f;
            }
            if constexpr (MODE == kPairStep) L.v[s0 + s][lane] = make_float2(cx, cy);
            else L.v[s0 + s][lane] = cx;
            // keep each column's accumulations in place: sinking them to the
            // end of the chunk would hold every pair's temporaries in registers
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                asm volatile("" : "+v"(ax[r]));
                if (MODE == kPairStep) asm volatile("" : "+v"(ay[r]));
            }
        }
    };
    // at least one chunk: a task always has a column
    const int nq = (ncol + kPTChunk - 1) / kPTChunk;
    int q = 0;
#pragma nounroll
    do {
        // the barriers keep each half-chunk's loads between the arithmetic
        // of the two halves, in the order the waits above assume
        const int cg = q * kPTChunk;
        const int J = J0 + cg / kPT;
        const int cb = cg % kPT;
        const bool full = A < J;
        math(ha, cb, 0, full);
        asm volatile("" ::: "memory");
        load4(cg + kPTChunk, ha);
        asm volatile("" ::: "memory");
        // the second half's values pass through here, so that its arithmetic
        // (and the wait for its loads) stays after the loads just issued
#pragma unroll
        for (int s = 0; s < H; ++s) asm volatile("" : "+v"(hb[s]));
        math(hb, cb + H, H, full);
        asm volatile("" ::: "memory");
        load4(cg + kPTChunk + H, hb);
        asm volatile("" ::: "memory");
        strip_columns<MODE>(t, J, cb, min(kPT, k - J * kPT), cb + kPTChunk == kPT || q + 1 == nq, colx, coly, L);
        // next column block: the positions of its columns
        if (MODE == kPairStep && kStripGroup > 1) {
            const bool nb = cb + kPTChunk == kPT;
#pragma unroll
            for (int b = 0; b + 1 < kStripGroup; ++b) {
                xc[b].x = nb ? xc[b + 1].x : xc[b].x;
                xc[b].y = nb ? xc[b + 1].y : xc[b].y;
            }
            xcol = xc[0];
        }
    } while (++q < nq);
    // rows 4 lane .. 4 lane + 3 of the task are rows a .. a + 3 of block A
    const int o = ((A * T + max(A, J0)) * kPT + (4 * lane) % kPT) * 4;
    pend.off = A < T ? o : (int)kStripOutside;
    pend.rx = t.prx;
    pend.ry = t.pry;
    pend.vx = StripU4{__float_as_uint(ax[0]), __float_as_uint(ax[1]), __float_as_uint(ax[2]), __float_as_uint(ax[3])};
    pend.vy = StripU4{__float_as_uint(ay[0]), __float_as_uint(ay[1]), __float_as_uint(ay[2]), __float_as_uint(ay[3])};
}

// One task (S, J0).  MODE kPairStep: the position sums g (X_i - X_j) into
// (px, py); kPairW: the weight sums w into px.  `m` is the subgraph's 1/Delta
// block (k rows of ld floats, zero diagonal, rows zero-padded to ld), px and
// py its partial blocks ([T][T][64] floats).  Stores the previous task's row
// partials from `pend` and leaves this task's there.
template <int MODE>
__device__ __forceinline__ void strip_task(const float* __restrict__ m, int64_t ld, int32_t k,
                                           const float2* __restrict__ x, int S, int J0, int T,
                                           float* __restrict__ px, float* __restrict__ py, StripLds<MODE>& L,
                                           StripPend& pend) {
    const int nJ = min(kStripGroup, T - J0);
    if (J0 >= kStripBlocks * S + kStripBlocks && (J0 + nJ) * kPT <= k)
        strip_task_body<MODE, false>(m, ld, k, x, S, J0, T, px, py, L, pend);
    else
        strip_task_body<MODE, true>(m, ld, k, x, S, J0, T, px, py, L, pend);
}

// Node i (row block A, super-row S = A / 4) of a k-node subgraph: add its
// partial slots in a fixed order, the column slots (A, S') for S' <
// ceil(A / 4), then the row slots (A, A) and (A, 4 S + kStripGroup m) for
// m >= 1.  MODE kPairW writes the weight sum; kPairStep writes
// X+_i = X_i + sum_j g (X_i - X_j) / sum_j w (X_i when the weight sum is 0).
template <int MODE>
__device__ __forceinline__ void strip_finalize(int i, int T, const float* __restrict__ px,
                                               const float* __restrict__ py, const float2* __restrict__ x,
                                               float2* __restrict__ xout, float* __restrict__ wsum) {
    const int A = i / kPT, a = i % kPT;
    const int64_t base = (int64_t)A * T * kPT + a;
    const int ncs = (A + kStripBlocks - 1) / kStripBlocks;
    float sx = 0.f, sy = 0.f;
    for (int B = 0; B < ncs; ++B) {
        const int64_t o = base + (int64_t)B * kPT;
        sx += px[o];
        if (MODE == kPairStep) sy += py[o];
    }
    for (int B = A; B < T; B = (B == A ? (A / kStripBlocks) * kStripBlocks + kStripGroup : B + kStripGroup)) {
        const int64_t o = base + (int64_t)B * kPT;
        sx += px[o];
        if (MODE == kPairStep) sy += py[o];
    }
    if (MODE == kPairW) {
        wsum[i] = sx;
        return;
    }
    const float sw = wsum[i];
    const float2 xi = x[i];
    xout[i] = sw > 0.f ? make_float2(xi.x + sx / sw, xi.y + sy / sw) : xi;
}

// out[0] = sum of part[0..m) in a fixed order (single block).
static __global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ part, int64_t m,
                                                           double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace pprviz
