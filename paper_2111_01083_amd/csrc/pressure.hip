// Pressure of the periodic Stokeslet sum (Sec. 5.2, the pressurelet of eq.
// stokeslet; Thms. south_thm_stokes_pressure and west_thm_stokes_pressure).
// The Stokeslet's pressure is p = (1/2pi) r.f / r^2 = -f . grad G_L with
// G_L = -(1/2pi) log r, so the periodic pressure of forces f_j is
//   p(t) = -(d/dx u_L[f1] + d/dy u_L[f2])(t),   u_L[q] = sum_j G_L^per(t - s_j) q_j,
// the divergence of the periodic Laplace gradient with the force components
// as (neutral) charges. Each Stokes plan holds a Laplace plan of the same
// lattice, tolerance and options with twice the density vectors; its
// gradients (caller's frame) are contracted here. A divergence of a periodic
// field has zero cell mean, which fixes the pressure's free constant.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "pfmm.h"
#include "pfmm_internal.h"

namespace pfmm {
namespace {

constexpr int PR_BLOCK = 256;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// grad [2 nd][2][nt] (Laplace gradients of f1, f2 per density vector) -> p [nd][nt]
__global__ void pressure_kernel(const double* grad, int nd, int64_t nt, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  for (int v = 0; v < nd; ++v) {
    const double* g1 = grad + (size_t)(2 * v) * 2 * nt;       // gradient of u_L[f1]
    const double* g2 = grad + (size_t)(2 * v + 1) * 2 * nt;   // gradient of u_L[f2]
    out[(size_t)v * nt + i] = -(g1[i] + g2[nt + i]);
  }
}

struct PresLayout { size_t eval_bytes, grad, total; };

PresLayout pres_layout(pfmm_plan_s* lap, int64_t ns, int64_t nt, int nd) {
  PresLayout L;
  L.eval_bytes = align_up(pfmm_workspace_bytes(lap, ns, nt));
  L.grad = L.eval_bytes;
  L.total = L.grad + align_up(8 * (size_t)2 * nd * 2 * (lap->self_exclude ? ns : nt));
  return L;
}

}  // namespace
}  // namespace pfmm

using namespace pfmm;

extern "C" {

size_t pfmm_workspace_bytes_pressure(pfmm_plan_t p, int64_t ns, int64_t nt) {
  if (!p || !p->lap || ns < 0 || nt < 0 || ns > PFMM_MAX_POINTS || nt > PFMM_MAX_POINTS) return 0;
  return pres_layout(p->lap, ns, nt, p->n_dens).total;
}

int pfmm_eval_pressure(pfmm_plan_t p, int64_t ns, const double* src_xy, const double* dens, int64_t nt,
                       const double* trg_xy, double* out_pres, void* workspace, size_t ws_bytes,
                       void* hip_stream) {
  if (!p || !p->lap || ns < 0 || nt < 0 || ns > PFMM_MAX_POINTS || nt > PFMM_MAX_POINTS) return PFMM_EINVAL;
  if (p->self_exclude && nt != ns) return PFMM_EINVAL;
  if (nt == 0 || !out_pres) return PFMM_OK;
  if (ns > 0 && (!src_xy || !dens)) return PFMM_EINVAL;
  if (!p->self_exclude && !trg_xy) return PFMM_EINVAL;
  const PresLayout L = pres_layout(p->lap, ns, nt, p->n_dens);
  if (!workspace || ws_bytes < L.total || ((uintptr_t)workspace & 255)) return PFMM_EWORKSPACE;
  char* ws = (char*)workspace;
  double* grad = (double*)(ws + L.grad);
  // forces [nd][2][ns] are the Laplace plan's 2 nd charge vectors
  int rc = eval_core(p->lap, ns, src_xy, dens, nt, p->self_exclude ? src_xy : trg_xy, nullptr, grad, ws,
                     L.eval_bytes, hip_stream);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(pressure_kernel, dim3((unsigned)((nt + PR_BLOCK - 1) / PR_BLOCK)), dim3(PR_BLOCK), 0, st,
                     (const double*)grad, p->n_dens, nt, out_pres);
  return hipGetLastError() == hipSuccess ? PFMM_OK : PFMM_EHIP;
}

}  // extern "C"
