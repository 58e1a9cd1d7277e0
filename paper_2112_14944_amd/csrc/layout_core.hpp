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
// row 64 A + l of every block, and the wave walks the 64 columns j, reading
// 1/Delta[j][i] for its four rows (one contiguous 1 KB piece of row j).  Row
// block A takes every pair with the columns when A < J and feeds both ends,
// its ordered pairs only when A == J (the diagonal block: rows only, each
// pair seen from both ends), and nothing when A > J (the strip of J's
// super-row has those pairs).  Which case holds is the same for the whole
// wave.  Row sums stay in the lane; the column sums of 8 columns at a time go
// through a small LDS block, where 8 lanes per column add 8 lanes' partials
// each and three lane exchanges finish the column.
//
// Partials: P[A][J] (64 floats per component) holds row block A's sum over
// the columns of block J (J >= A); P[J][S] (S < J / 4) holds column block
// J's sum over the rows of super-row S.  These slot ranges are disjoint, and
// strip_finalize adds a node's slots in one fixed order, so the result does
// not depend on which wave ran which strip.
constexpr int kPT = 64;
constexpr int kStripBlocks = 4;
constexpr int kPTChunk = 8;  // columns per LDS column exchange

// Strips of a subgraph with T column blocks: super-row S holds the strips
// J = 4 S .. T - 1.
__host__ __device__ __forceinline__ int64_t strip_count(int64_t T) {
    const int64_t S = (T + kStripBlocks - 1) / kStripBlocks;
    return T * S - 2 * S * (S - 1);
}

// Strip index t of a T-block subgraph -> (S, J).
__device__ __forceinline__ void strip_sj(int t, int T, int& S, int& J) {
    int s = 0;
    while (t >= T - kStripBlocks * s) {
        t -= T - kStripBlocks * s;
        ++s;
    }
    S = s;
    J = kStripBlocks * s + t;
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

// The live row blocks of a strip are a prefix: blocks 4 S .. 4 S + NL - 1,
// all taking full pairs except the last, which is the diagonal block J when
// DIAG.  Both are template parameters, so every branch on a block's role is
// resolved at compile time.
template <int NL, bool DIAG>
struct StripShape {
    static constexpr bool full(int r) { return r < NL - (DIAG ? 1 : 0); }
    static constexpr bool live(int r) { return r < NL; }
    static constexpr bool any_full = NL - (DIAG ? 1 : 0) > 0;
};

// Byte offset past every subgraph block of the 1/Delta pool: a buffer load
// there returns 0 and touches no memory.
constexpr uint32_t kStripOutside = 0x80000000u;

struct StripCtx {
    __amdgpu_buffer_rsrc_t mr;  // 1/Delta rows from column 256 S on
    int lane, S, J, T, j0, ncol, cc, cp;
    uint32_t voff[kStripBlocks];  // lane's byte offset in a row, kStripOutside for rows >= k
    float2 xi[kStripBlocks];
    float2 xcol;                  // X of column 64 J + lane (read out per column with readlane)
};

// Loads of NC columns for the strip's live row blocks; nval is
// the number of those columns that exist.  Rows and columns outside the
// subgraph read zeros through the buffer resource, so no load is predicated.
template <typename SH, bool FULLCOLS, int NC>
__device__ __forceinline__ void strip_load(const StripCtx& t, int64_t ld, int jq, int nval,
                                           float (&mv)[kStripBlocks][NC]) {
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const bool col_ok = FULLCOLS || s < nval;
        const int soff = col_ok ? (int)((int64_t)(jq + s) * ld * 4) : (int)(kStripOutside >> 1);
#pragma unroll
        for (int r = 0; r < kStripBlocks; ++r) {
            if (!SH::live(r)) continue;
            mv[r][s] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(t.mr, (int)t.voff[r], soff, 0));
        }
    }
}

// Arithmetic of NC columns; their column terms go to LDS slots s0 .. s0 + NC - 1.
template <int MODE, typename SH, bool FULLCOLS, int NC>
__device__ __forceinline__ void strip_cols_math(const StripCtx& t, const float2* __restrict__ x, int32_t k, int jq,
                                                int s0, const float (&mv)[kStripBlocks][NC],
                                                float (&ax)[kStripBlocks], float (&ay)[kStripBlocks],
                                                StripLds<MODE>& L) {
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        float cx = 0.f, cy = 0.f;
        float2 xj = make_float2(0.f, 0.f);
        if (MODE == kPairStep) {
            // the column's position from the lane that loaded it: no memory
            // access inside the loop besides the 1/Delta stream
            const int c = jq - t.j0 + s;
            xj.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t.xcol.x), c));
            xj.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t.xcol.y), c));
        }
#pragma unroll
        for (int r = 0; r < kStripBlocks; ++r) {
            if (!SH::live(r)) continue;
            const float inv = mv[r][s];
            const float w = inv * inv;
            if (MODE == kPairStep) {
                const float dx = t.xi[r].x - xj.x;
                const float dy = t.xi[r].y - xj.y;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, kMinSq));
                const float g = fmaf(inv, __builtin_amdgcn_rsqf(r2), -w);
                ax[r] = fmaf(g, dx, ax[r]);
                ay[r] = fmaf(g, dy, ay[r]);
                if (SH::full(r)) {
                    cx = fmaf(-g, dx, cx);
                    cy = fmaf(-g, dy, cy);
                }
            } else {
                ax[r] += w;
                if (SH::full(r)) cx += w;
            }
        }
        if constexpr (SH::any_full) {
            if constexpr (MODE == kPairStep) L.v[s0 + s][t.lane] = make_float2(cx, cy);
            else L.v[s0 + s][t.lane] = cx;
        }
        // keep each column's accumulations in place: sinking them to the end
        // of the chunk would hold every pair's temporaries in registers
#pragma unroll
        for (int r = 0; r < kStripBlocks; ++r) {
            if (!SH::live(r)) continue;
            asm volatile("" : "+v"(ax[r]));
            if (MODE == kPairStep) asm volatile("" : "+v"(ay[r]));
        }
    }
}

// Column sums of one chunk (8 columns at jq): lane (cc, cp) adds the partials
// of lanes 8 cp .. 8 cp + 7 for column cc, starting at lane 8 cp + cp so that
// the 8 lanes of a column read 8 different bank groups; the column total goes
// to slot P[J][S].
template <int MODE, bool FULLCOLS>
__device__ __forceinline__ void strip_columns(const StripCtx& t, int q, float* __restrict__ px,
                                              float* __restrict__ py, StripLds<MODE>& L) {
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
    const int jj = q * kPTChunk + t.cc;
    if (t.cp == 0 && (FULLCOLS || jj < t.ncol)) {
        const int64_t o = ((int64_t)t.J * t.T + t.S) * kPT + jj;
        px[o] = sx;
        if (MODE == kPairStep) py[o] = sy;
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// One strip.  MODE kPairStep: the position sums g (X_i - X_j) into (px, py);
// kPairW: the weight sums w into px.  `m` is the subgraph's 1/Delta block
// (k rows of ld floats, zero diagonal), px and py its partial blocks
// ([T][T][64] floats).  FULLCOLS: all 64 columns of block J exist.  Loads of
// the next group of columns are issued before the arithmetic of the current
// one.
template <int MODE, typename SH, bool FULLCOLS>
__device__ __forceinline__ void strip_body(const float* __restrict__ m, int64_t ld, int32_t k,
                                           const float2* __restrict__ x, int S, int J, int T,
                                           float* __restrict__ px, float* __restrict__ py, StripLds<MODE>& L) {
    StripCtx t;
    t.lane = threadIdx.x & 63;
    t.S = S;
    t.J = J;
    t.T = T;
    t.j0 = J * kPT;
    t.ncol = FULLCOLS ? kPT : min(kPT, k - t.j0);
    t.cc = t.lane >> 3;
    t.cp = t.lane & 7;
#pragma unroll
    for (int r = 0; r < kStripBlocks; ++r) {
        const int i = (kStripBlocks * S + r) * kPT + t.lane;
        const bool rok = SH::live(r) && i < k;
        t.voff[r] = rok ? (uint32_t)((r * kPT + t.lane) * 4) : kStripOutside;
        t.xi[r] = (MODE == kPairStep && rok) ? x[i] : make_float2(0.f, 0.f);
    }
    t.xcol = MODE == kPairStep ? x[min(t.j0 + t.lane, k - 1)] : make_float2(0.f, 0.f);
    const int64_t c0 = (int64_t)S * kStripBlocks * kPT;
    t.mr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(m + c0), 0, (int)(((int64_t)k * ld - c0) * 4),
                                             0x00020000);
    float ax[kStripBlocks], ay[kStripBlocks];
#pragma unroll
    for (int r = 0; r < kStripBlocks; ++r) ax[r] = ay[r] = 0.f;
    // two load groups of 4 columns per exchange chunk; each group's loads
    // are issued one group ahead of its arithmetic
    const int nq = (t.ncol + kPTChunk - 1) / kPTChunk;
    constexpr int H = kPTChunk / 2;
    float ha[kStripBlocks][H], hb[kStripBlocks][H];
    strip_load<SH, FULLCOLS, H>(t, ld, t.j0, t.ncol, ha);
    strip_load<SH, FULLCOLS, H>(t, ld, t.j0 + H, t.ncol - H, hb);
#pragma nounroll
    for (int q = 0; q < nq; ++q) {
        const int jq = t.j0 + q * kPTChunk;
        strip_cols_math<MODE, SH, FULLCOLS, H>(t, x, k, jq, 0, ha, ax, ay, L);
        if (q + 1 < nq) strip_load<SH, FULLCOLS, H>(t, ld, jq + kPTChunk, t.ncol - (q + 1) * kPTChunk, ha);
        strip_cols_math<MODE, SH, FULLCOLS, H>(t, x, k, jq + H, H, hb, ax, ay, L);
        if (q + 1 < nq)
            strip_load<SH, FULLCOLS, H>(t, ld, jq + kPTChunk + H, t.ncol - (q + 1) * kPTChunk - H, hb);
        if constexpr (SH::any_full) strip_columns<MODE, FULLCOLS>(t, q, px, py, L);
    }
#pragma unroll
    for (int r = 0; r < kStripBlocks; ++r) {
        if (!SH::live(r)) continue;
        const int A = kStripBlocks * S + r;
        const int64_t o = ((int64_t)A * T + J) * kPT + t.lane;
        px[o] = ax[r];
        if (MODE == kPairStep) py[o] = ay[r];
    }
}

// A strip whose 256 rows all lie in the subgraph and left of block J, and
// whose 64 columns all exist (the bulk of every large subgraph): lane l owns
// the four consecutive rows 256 S + 4 l .. + 3 and reads their 1/Delta values
// of a column with one 16-byte load, a quarter of the load instructions of
// strip_body.  Same pair terms, column exchange and partial slots.
template <int MODE>
__device__ __forceinline__ void strip_body_x4(const float* __restrict__ m, int64_t ld, int32_t k,
                                              const float2* __restrict__ x, int S, int J, int T,
                                              float* __restrict__ px, float* __restrict__ py,
                                              StripLds<MODE>& L) {
    constexpr int H = kPTChunk / 2;
    const int lane = threadIdx.x & 63;
    const int i0 = S * kStripBlocks * kPT + 4 * lane;
    float2 xi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) xi[r] = MODE == kPairStep ? x[i0 + r] : make_float2(0.f, 0.f);
    const int j0 = J * kPT;
    const float2 xcol = MODE == kPairStep ? x[j0 + lane] : make_float2(0.f, 0.f);
    const float* __restrict__ rowp = m + i0;
    StripCtx t;
    t.lane = lane;
    t.S = S;
    t.J = J;
    t.T = T;
    t.j0 = j0;
    t.ncol = kPT;
    t.cc = lane >> 3;
    t.cp = lane & 7;
    float ax[4] = {0.f, 0.f, 0.f, 0.f}, ay[4] = {0.f, 0.f, 0.f, 0.f};
    float4 ha[H], hb[H];
#pragma unroll
    for (int s = 0; s < H; ++s) {
        ha[s] = *reinterpret_cast<const float4*>(rowp + (int64_t)(j0 + s) * ld);
        hb[s] = *reinterpret_cast<const float4*>(rowp + (int64_t)(j0 + H + s) * ld);
    }
    auto math = [&](const float4 (&v)[H], int c0, int s0) {
#pragma unroll
        for (int s = 0; s < H; ++s) {
            float cx = 0.f, cy = 0.f;
            float2 xj = make_float2(0.f, 0.f);
            if (MODE == kPairStep) {
                xj.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xcol.x), c0 + s));
                xj.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xcol.y), c0 + s));
            }
            const float iv[4] = {v[s].x, v[s].y, v[s].z, v[s].w};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float inv = iv[r];
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
            if constexpr (MODE == kPairStep) L.v[s0 + s][lane] = make_float2(cx, cy);
            else L.v[s0 + s][lane] = cx;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                asm volatile("" : "+v"(ax[r]));
                if (MODE == kPairStep) asm volatile("" : "+v"(ay[r]));
            }
        }
    };
    constexpr int nq = kPT / kPTChunk;
#pragma nounroll
    for (int q = 0; q < nq; ++q) {
        const int c = q * kPTChunk;
        math(ha, c, 0);
        if (q + 1 < nq) {
#pragma unroll
            for (int s = 0; s < H; ++s)
                ha[s] = *reinterpret_cast<const float4*>(rowp + (int64_t)(j0 + c + kPTChunk + s) * ld);
        }
        math(hb, c + H, H);
        if (q + 1 < nq) {
#pragma unroll
            for (int s = 0; s < H; ++s)
                hb[s] = *reinterpret_cast<const float4*>(rowp + (int64_t)(j0 + c + kPTChunk + H + s) * ld);
        }
        strip_columns<MODE, true>(t, q, px, py, L);
    }
    // rows 4 lane .. 4 lane + 3 of the strip are rows a .. a + 3 of block A
    const int A = S * kStripBlocks + lane / 16;
    const int64_t o = ((int64_t)A * T + J) * kPT + (4 * lane) % kPT;
    *reinterpret_cast<float4*>(px + o) = make_float4(ax[0], ax[1], ax[2], ax[3]);
    if (MODE == kPairStep) *reinterpret_cast<float4*>(py + o) = make_float4(ay[0], ay[1], ay[2], ay[3]);
}

template <int MODE, int NL, bool DIAG>
__device__ __forceinline__ void strip_cols(const float* __restrict__ m, int64_t ld, int32_t k,
                                           const float2* __restrict__ x, int S, int J, int T,
                                           float* __restrict__ px, float* __restrict__ py, StripLds<MODE>& L) {
    if ((J + 1) * kPT <= k)
        strip_body<MODE, StripShape<NL, DIAG>, true>(m, ld, k, x, S, J, T, px, py, L);
    else
        strip_body<MODE, StripShape<NL, DIAG>, false>(m, ld, k, x, S, J, T, px, py, L);
}

// Dispatch on the strip's shape: NL = live row blocks (those below T and at
// or left of J), DIAG = block J is one of them.
template <int MODE>
__device__ __forceinline__ void strip(const float* __restrict__ m, int64_t ld, int32_t k,
                                      const float2* __restrict__ x, int S, int J, int T, float* __restrict__ px,
                                      float* __restrict__ py, StripLds<MODE>& L) {
    const int d = J - kStripBlocks * S;
    if (d >= kStripBlocks && (J + 1) * kPT <= k) {
        strip_body_x4<MODE>(m, ld, k, x, S, J, T, px, py, L);
        return;
    }
    const int nl = min(kStripBlocks, min(T - kStripBlocks * S, d + 1));
    const bool diag = d < kStripBlocks;
    switch (nl * 2 + (diag ? 1 : 0)) {
        case 3: strip_cols<MODE, 1, true>(m, ld, k, x, S, J, T, px, py, L); break;
        case 4: strip_cols<MODE, 2, false>(m, ld, k, x, S, J, T, px, py, L); break;
        case 5: strip_cols<MODE, 2, true>(m, ld, k, x, S, J, T, px, py, L); break;
        case 6: strip_cols<MODE, 3, false>(m, ld, k, x, S, J, T, px, py, L); break;
        case 7: strip_cols<MODE, 3, true>(m, ld, k, x, S, J, T, px, py, L); break;
        case 8: strip_cols<MODE, 4, false>(m, ld, k, x, S, J, T, px, py, L); break;
        case 9: strip_cols<MODE, 4, true>(m, ld, k, x, S, J, T, px, py, L); break;
        default: strip_cols<MODE, 1, false>(m, ld, k, x, S, J, T, px, py, L); break;
    }
}

// Node i (row block A) of a k-node subgraph: add its partial slots in a fixed
// order, the column slots S < ceil(A / 4) and then the row slots J >= A.
// MODE kPairW writes the weight sum; kPairStep writes
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
    for (int B = A; B < T; ++B) {
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
