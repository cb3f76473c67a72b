// NUFFT-accelerated south/north part (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "pfmm_internal.h"

namespace pfmm {
size_t nufft_workspace_bytes(const pfmm_plan_s* p, int64_t ns, int64_t nt);
// Adds nothing to the outputs itself: fills *val_out (inside ws) with the
// south/north field [n_dens][NOUT][nt] in the canonical frame.
int nufft_far(const pfmm_plan_s* p, int64_t ns, int64_t nt, const double* sx, const double* sy,
              const double* dens, const double* tx, const double* ty, char* ws, hipStream_t st,
              const double** val_out);
}  // namespace pfmm
