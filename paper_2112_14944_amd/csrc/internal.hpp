// Host-side functions shared between the library's translation units.
#pragma once

#include "common.hpp"
#include "ppr_core.hpp"

namespace pprviz {

ppr_status validate_csr(const ppr_csr* g);
bool use_resident(int n);
void launch_degree(const int32_t* row_ptr, const float* weight, int64_t n, float* deg, float* invd,
                   hipStream_t s);
void ppr_forward(const ppr_csr* g, const int32_t* src, int32_t n_src, const int32_t* tgt, int32_t n_tgt,
                 float alpha, int32_t T, float* ppr_out, float* dppr_out, const float* deg, const float* invd,
                 double* resid, RowEnt* rows, int32_t* col_r, float* w_r, int32_t* hist, float* ya, float* yb,
                 double* part, hipStream_t s);
void launch_row_table(const int32_t* row_ptr, const int32_t* col_idx, const float* weight,
                      const int64_t* node_off, int32_t n_single, int32_t blocks, int64_t n_slots, RowEnt* table,
                      int32_t* col_out, float* w_out, hipStream_t s);

}  // namespace pprviz
