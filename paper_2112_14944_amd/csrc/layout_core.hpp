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
// Pair-tile Jacobi sweep.  Delta is symmetric, so each unordered pair {i, j}
// is evaluated once and feeds both rows: with d = X_i - X_j,
//     row i gets   w X_j + c d        row j gets   w X_i - c d
// (the two terms of the sweep formula in layout_rows, seen from each end).
// The k x k matrix is cut into 64 x 64 tiles (I, J), I <= J.  One wave takes
// one tile: lane l is row i = 64 I + l, and the wave walks the 64 columns j
// of tile J one per step, reading Delta[j][i] (row j, so the 64 lanes read
// 256 contiguous bytes).  Row sums stay in the lane; the column sums of 8
// steps at a time go through a small LDS block, where 8 lanes per column add
// 8 rows each and three lane exchanges finish the column.  A diagonal tile
// (I == J) takes every ordered pair and feeds rows only.
//
// Each tile writes its sums to a partial block: P[I][J] holds what the rows
// of tile I received from the columns of tile J (and P[J][I] the reverse), so
// a node's total is the sum of its T blocks in block order, independent of
// which wave ran which tile.  pair_finalize combines them.
//
// Memory read per sweep: the tiles of one triangle (about half of Delta).
constexpr int kPT = 64;
constexpr int kPTChunk = 8;

// LDS of one wave for the column sums of one chunk, per row and column:
// (x, y) when positions are summed, w when weights are.
template <bool POS, bool WGT>
struct PairLds;
template <>
struct PairLds<true, false> {
    float2 xy[kPTChunk][kWave];
};
template <>
struct PairLds<true, true> {
    float2 xy[kPTChunk][kWave];
    float w[kPTChunk][kWave];
};
template <>
struct PairLds<false, true> {
    float w[kPTChunk][kWave];
};

enum { kPairStep = 0, kPairStepW = 1, kPairW = 2 };

// Upper-triangle tile index t -> (I, J), I <= J, row-major over J: t = J (J + 1) / 2 + I.
__device__ __forceinline__ void pair_tile_ij(int t, int& I, int& J) {
    int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    while (j * (j + 1) / 2 > t) --j;
    J = j;
    I = t - j * (j + 1) / 2;
}

// Per-tile state of one wave in pair_tile_body.
struct PairTileCtx {
    __amdgpu_buffer_rsrc_t mr;  // rows 64 I .. of the subgraph's matrix
    int lane, i, j0, ncol, I, J, T, cc, cp;
    bool row_ok;
    float2 xi;
};

// Loads of one 8-column chunk: m[j][i] for the lane's row and the chunk's
// columns (one coalesced 256-byte row segment per column), and X_j.  The
// matrix is read through a buffer resource whose base is row 64 I, with the
// column's offset as a scalar and the lane's as the one vector offset, so
// that no per-column addresses take vector registers.
template <bool POS, bool FULL>
__device__ __forceinline__ void pair_load(const PairTileCtx& t, int64_t ld,
                                          int32_t k, const float2* __restrict__ x, int q, float (&mv)[kPTChunk],
                                          float2 (&xj)[kPTChunk]) {
    const int jq = t.j0 + q * kPTChunk;
#pragma unroll
    for (int s = 0; s < kPTChunk; ++s) {
        const bool col_ok = FULL || (q * kPTChunk + s < t.ncol);
        mv[s] = (col_ok && t.row_ok) ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                           t.mr, t.lane * 4, (int)((int64_t)(jq + s) * ld * 4), 0))
                                     : 0.f;
        if (POS) xj[s] = x[FULL ? jq + s : min(jq + s, k - 1)];
    }
}

// Arithmetic of one chunk: row sums into (ax, ay, aw); for an off-diagonal
// tile the column terms go through LDS and each column's sum over the 64
// rows is written to the partial block P[J][I].
template <bool INV, int MODE, bool DIAG, bool FULL, typename Lds>
__device__ __forceinline__ void pair_chunk(const PairTileCtx& t, int q, const float (&mv)[kPTChunk],
                                           const float2 (&xj)[kPTChunk], float& ax, float& ay, float& aw,
                                           float* __restrict__ px, float* __restrict__ py, float* __restrict__ pw,
                                           Lds& L) {
    constexpr bool POS = (MODE != kPairW);
    constexpr bool WGT = (MODE != kPairStep);
    const int jq = t.j0 + q * kPTChunk;
#pragma unroll
    for (int s = 0; s < kPTChunk; ++s) {
        const int j = jq + s;
        float inv;
        if (INV) {
            inv = mv[s];
        } else {
            const bool col_ok = FULL || (q * kPTChunk + s < t.ncol);
            inv = (col_ok && t.row_ok && (!DIAG || j != t.i)) ? __builtin_amdgcn_rcpf(mv[s]) : 0.f;
        }
        const float w = inv * inv;
        float cx = 0.f, cy = 0.f;
        if (POS) {
            const float dx = t.xi.x - xj[s].x;
            const float dy = t.xi.y - xj[s].y;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, kMinSq));
            const float c = inv * __builtin_amdgcn_rsqf(r2);
            const float tx = c * dx;
            const float ty = c * dy;
            ax = fmaf(w, xj[s].x, ax) + tx;
            ay = fmaf(w, xj[s].y, ay) + ty;
            cx = fmaf(w, t.xi.x, -tx);
            cy = fmaf(w, t.xi.y, -ty);
        }
        if (WGT) aw += w;
        if (!DIAG) {
            if constexpr (POS) L.xy[s][t.lane] = make_float2(cx, cy);
            if constexpr (WGT) L.w[s][t.lane] = w;
        }
    }
    if (DIAG) return;
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    float sx = 0.f, sy = 0.f, sw = 0.f;
    // lane (cc, cp) adds rows cp*8 .. cp*8+7 of column cc, starting at row
    // cp*8 + cp so that the 8 lanes of a column read 8 different bank groups
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = t.cp * 8 + ((u + t.cp) & 7);
        if constexpr (POS) {
            const float2 v = L.xy[t.cc][r];
            sx += v.x;
            sy += v.y;
        }
        if constexpr (WGT) sw += L.w[t.cc][r];
    }
    if (POS) {
        sx += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sx), 0xB1, 0xf, 0xf, false));
        sy += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sy), 0xB1, 0xf, 0xf, false));
        sx += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sx), 0x4E, 0xf, 0xf, false));
        sy += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sy), 0x4E, 0xf, 0xf, false));
        sx += __shfl_xor(sx, 4, kWave);
        sy += __shfl_xor(sy, 4, kWave);
    }
    if (WGT) {
        sw += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sw), 0xB1, 0xf, 0xf, false));
        sw += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sw), 0x4E, 0xf, 0xf, false));
        sw += __shfl_xor(sw, 4, kWave);
    }
    const int jj = q * kPTChunk + t.cc;
    if (t.cp == 0 && (FULL || jj < t.ncol)) {
        const int64_t o = ((int64_t)t.J * t.T + t.I) * kPT + jj;
        if (POS) {
            px[o] = sx;
            py[o] = sy;
        }
        if (WGT) pw[o] = sw;
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// One 64 x 64 tile.  MODE kPairStep: position sums only (the weight sums come
// from a kPairW pass); kPairStepW: positions and weights; kPairW: weights
// only.  INV: `m` holds 1/Delta with a zero diagonal, else Delta.  px, py, pw
// are this subgraph's partial blocks ([T][T][64]).  DIAG: I == J.  FULL: all
// 64 columns of tile J exist (no column bound checks).  The loads of the next
// chunk are issued before the arithmetic of the current one (two register
// sets, used alternately).
template <bool INV, int MODE, bool DIAG, bool FULL, typename Lds>
__device__ __forceinline__ void pair_tile_body(const float* __restrict__ m, int64_t ld, int32_t k,
                                               const float2* __restrict__ x, int I, int J, int T,
                                               float* __restrict__ px, float* __restrict__ py,
                                               float* __restrict__ pw, Lds& L) {
    constexpr bool POS = (MODE != kPairW);
    PairTileCtx t;
    t.lane = threadIdx.x & 63;
    t.i = I * kPT + t.lane;
    t.row_ok = t.i < k;
    t.xi = t.row_ok ? x[t.i] : make_float2(0.f, 0.f);
    t.j0 = J * kPT;
    t.ncol = FULL ? kPT : min(kPT, k - t.j0);
    t.I = I;
    t.J = J;
    t.T = T;
    t.cc = t.lane >> 3;
    t.cp = t.lane & 7;
    t.mr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(m + (int64_t)I * kPT), 0,
                                             (int)((int64_t)k * ld * 4), 0x00020000);
    const int nq = (t.ncol + kPTChunk - 1) / kPTChunk;
    float ax = 0.f, ay = 0.f, aw = 0.f;
    float ma[kPTChunk], mb[kPTChunk];
    float2 xa[kPTChunk], xb[kPTChunk];
    pair_load<POS, FULL>(t, ld, k, x, 0, ma, xa);
    for (int q = 0; q < nq; q += 2) {
        if (q + 1 < nq) pair_load<POS, FULL>(t, ld, k, x, q + 1, mb, xb);
        pair_chunk<INV, MODE, DIAG, FULL>(t, q, ma, xa, ax, ay, aw, px, py, pw, L);
        if (q + 1 < nq) {
            if (q + 2 < nq) pair_load<POS, FULL>(t, ld, k, x, q + 2, ma, xa);
            pair_chunk<INV, MODE, DIAG, FULL>(t, q + 1, mb, xb, ax, ay, aw, px, py, pw, L);
        }
    }
    if (t.row_ok) {
        const int64_t o = ((int64_t)I * T + J) * kPT + t.lane;
        if (POS) {
            px[o] = ax;
            py[o] = ay;
        }
        if (MODE != kPairStep) pw[o] = aw;
    }
}

// LDS type of a pair-tile launch in mode MODE.
template <int MODE>
using PairLdsOf = PairLds<MODE != kPairW, MODE != kPairStep>;

template <bool INV, int MODE>
__device__ __forceinline__ void pair_tile(const float* __restrict__ m, int64_t ld, int32_t k,
                                          const float2* __restrict__ x, int I, int J, int T,
                                          float* __restrict__ px, float* __restrict__ py,
                                          float* __restrict__ pw, PairLdsOf<MODE>& L) {
    const bool full = (J + 1) * kPT <= k;
    if (I == J) {
        pair_tile_body<INV, MODE, true, false>(m, ld, k, x, I, J, T, px, py, pw, L);
    } else if (full) {
        pair_tile_body<INV, MODE, false, true>(m, ld, k, x, I, J, T, px, py, pw, L);
    } else {
        pair_tile_body<INV, MODE, false, false>(m, ld, k, x, I, J, T, px, py, pw, L);
    }
}

// Node i of a k-node subgraph: combine its T partial blocks in block order.
// MODE kPairW writes the weight sum; the step modes write X+_i (or X_i when
// the weight sum is zero), taking the weight sum from `wsum` (kPairStep) or
// from the partials (kPairStepW).
template <int MODE>
__device__ __forceinline__ void pair_finalize(int i, int T, const float* __restrict__ px,
                                              const float* __restrict__ py, const float* __restrict__ pw,
                                              const float2* __restrict__ x, float2* __restrict__ xout,
                                              float* __restrict__ wsum) {
    const int A = i / kPT, a = i % kPT;
    const int64_t base = (int64_t)A * T * kPT + a;
    float sx = 0.f, sy = 0.f, sw = 0.f;
    for (int B = 0; B < T; ++B) {
        const int64_t o = base + (int64_t)B * kPT;
        if (MODE != kPairW) {
            sx += px[o];
            sy += py[o];
        }
        if (MODE != kPairStep) sw += pw[o];
    }
    if (MODE == kPairW) {
        wsum[i] = sw;
        return;
    }
    if (MODE == kPairStep) sw = wsum[i];
    xout[i] = sw > 0.f ? make_float2(sx / sw, sy / sw) : x[i];
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
