// Host-side functions and workspace layouts shared between the library's
// translation units.
#pragma once

#include <algorithm>

#include "common.hpp"
#include "ppr_core.hpp"
#include "ppr_mid.hpp"
#include "ppr_stream.hpp"

namespace pprviz {

// Workspace of the forward PPR (ppr_matrix, and the recompute inside
// ppr_matrix_backward).  Only the buffers of the kernel that n selects are
// taken, unless the streaming buffers are asked for as well.
struct PprWs {
    RowEnt* rows;
    ResSlot* slots;  // resident tile: slot table
    float* deg;
    float* invd;
    double* resid;
    int32_t* col_r;  // resident tile: arc copy in group layout
    float* w_r;
    int32_t* sorted_r;  // resident tile: arcs grouped by LDS bank class (layout staging)
    float* sorted_w;
    MidWs mid;       // mid-size kernel: plan and arc stream
    float* ya;       // streaming SpMM: iterate ping-pong
    float* yb;
    double* part;
    int32_t* hist;
};

template <typename Cursor>
void ppr_ws_layout(Cursor& c, int n, int64_t nnz, bool weighted, int n_src, PprWs* w, bool with_stream = false) {
    PprWs t{};
    t.rows = c.template take<RowEnt>(n);
    t.deg = c.template take<float>(n);
    t.invd = c.template take<float>(n);
    t.resid = c.template take<double>(std::max(n_src, 1));
    const bool res = res_cols_for(n) != 0;
    const bool mid = mid_cols_for(n) != 0;
    if (res) {
        t.slots = c.template take<ResSlot>((size_t)n + kResTabPad);
        t.col_r = c.template take<int32_t>((size_t)res_arc_words(nnz, n));
        t.w_r = weighted ? c.template take<float>((size_t)res_arc_words(nnz, n)) : nullptr;
        t.sorted_r = c.template take<int32_t>((size_t)std::max<int64_t>(nnz, 1));
        t.sorted_w = weighted ? c.template take<float>((size_t)std::max<int64_t>(nnz, 1)) : nullptr;
    }
    if (mid) {
        const int64_t groups = mid_stream_groups(n, nnz);
        t.mid.rows = t.rows;
        t.mid.hist = c.template take<int32_t>(kMidKeys);
        t.mid.plan = c.template take<int32_t>(kPlanInts);
        t.mid.slice_goff = c.template take<int32_t>((size_t)mid_slices(n + kMidMaxParts));
        t.mid.slice_slot = c.template take<int32_t>((size_t)mid_slices(n + kMidMaxParts));
        t.mid.vrows = c.template take<RowEnt>((size_t)n + kMidMaxParts);
        t.mid.comb = c.template take<int4>(kMidMaxParts);
        t.mid.part_dst = c.template take<int32_t>(kMidWaves * kWave);
        t.mid.rowpos = c.template take<int32_t>(n);
        t.mid.vtab = c.template take<int2>((size_t)kMidWaves * kMidSlotCap * 64);
        t.mid.sell = c.template take<uint16_t>((size_t)(groups * kMidGroup));
        t.mid.sellw = weighted ? c.template take<float>((size_t)(groups * kMidGroup)) : nullptr;
        t.mid.tmp_u = c.template take<int32_t>((size_t)std::max<int64_t>(nnz, 1));
        t.mid.tmp_w = weighted ? c.template take<float>((size_t)std::max<int64_t>(nnz, 1)) : nullptr;
    }
    if ((!res && !mid) || with_stream) {
        const int64_t ldy = stream_ld(with_stream ? n : n_src);
        t.ya = c.template take<float>((size_t)n * ldy);
        t.yb = c.template take<float>((size_t)n * ldy);
        t.part = c.template take<double>((size_t)stream_resid_chunks(n) * ldy);
        t.hist = c.template take<int32_t>(kDegKeys);
    }
    if (w) *w = t;
}

ppr_status validate_csr(const ppr_csr* g);
bool use_resident(int n);
void launch_degree(const int32_t* row_ptr, const float* weight, int64_t n, float* deg, float* invd,
                   hipStream_t s);
void ppr_forward(const ppr_csr* g, const int32_t* src, int32_t n_src, const int32_t* tgt, int32_t n_tgt,
                 float alpha, int32_t T, float* ppr_out, float* dppr_out, const float* deg, const float* invd,
                 double* resid, const PprWs& w, hipStream_t s);
void launch_res_layout(const int32_t* row_ptr, const int32_t* col_idx, const float* weight, const float* invd,
                       const int64_t* node_off, int32_t n_single, int32_t blocks, ResSlot* slots, int32_t* arcs,
                       float* warcs, int32_t* sorted, float* wsorted, hipStream_t s);

}  // namespace pprviz
