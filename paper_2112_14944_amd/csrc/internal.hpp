// Host-side functions shared between the library's translation units.
#pragma once

#include "common.hpp"

namespace pprviz {

ppr_status validate_csr(const ppr_csr* g);
bool use_resident(int n);
void launch_degree(const int32_t* row_ptr, const float* weight, int64_t n, float* deg, float* invd,
                   hipStream_t s);
void ppr_forward(const ppr_csr* g, const int32_t* src, int32_t n_src, const int32_t* tgt, int32_t n_tgt,
                 float alpha, int32_t T, float* ppr_out, float* dppr_out, const float* deg, const float* invd,
                 double* resid, float* ya, float* yb, double* part, hipStream_t s);

}  // namespace pprviz
