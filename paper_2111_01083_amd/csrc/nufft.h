// NUFFT-accelerated south/north factors (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "pfmm_internal.h"

namespace pfmm {
size_t nufft_workspace_bytes(const pfmm_plan_s* p, int64_t ns, int64_t nt);
// R side: south/north coefficients [n_dens][n_sn][ncw] (complex) into the
// workspace; *csn_out points at them.
int nufft_R(const pfmm_plan_s* p, int64_t ns, const double* sx, const double* sy, const double* dens,
            char* ws, hipStream_t st, const double** csn_out);
// L side: south/north field at the targets, [n_dens][NOUT][nt] into val
// (canonical frame), from the weighted coefficients w [n_dens][n_coef].
int nufft_L(const pfmm_plan_s* p, int64_t nt, const double* tx, const double* ty, const double* w,
            int n_coef, char* ws, hipStream_t st, const double** val_out, double* val);
}  // namespace pfmm
