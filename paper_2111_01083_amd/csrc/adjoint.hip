// Adjoint of the potential at the sources (targets = sources, self terms
// excluded). For pot_i = sum_j K(x_i, x_j) q_j with the periodic kernel K
// symmetric (K(t, s) = K(s, t): G is even and the lattice is symmetric,
// Sec. 1 eq. psum) and a loss L with g = dL/dpot:
//   dL/dq_j = sum_i g_i K(x_i, x_j) = u[g](x_j)
//   dL/dx_j = g_j grad u[q](x_j) + q_j grad u[g](x_j)
// (Stokes: per velocity component, dL/dx_j = sum_a g_ja grad u_a[f] + f_ja grad u_a[g]).
// Both fields come from one evaluation with the two densities [q, g]; for
// Laplace and Stokes g is first made neutral (subtracting its mean), which
// is exact for any loss that does not see the free constant of the potential.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "pfmm.h"
#include "pfmm_internal.h"

namespace pfmm {
namespace {

constexpr int ADJ_BLOCK = 256;

__global__ __launch_bounds__(1024) void mean_kernel(const double* g, int64_t n, int nc, double* out) {
  __shared__ double red[1024];
  for (int c = 0; c < nc; ++c) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += g[(size_t)c * n + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = n > 0 ? red[0] / (double)n : 0.0;
    __syncthreads();
  }
}

__global__ void adj_prep_kernel(const double* q, const double* g, const double* mean, int proj, int64_t n,
                                int nc, double* dens2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nc; ++c) {
    dens2[(size_t)c * n + i] = q[(size_t)c * n + i];
    dens2[(size_t)(nc + c) * n + i] = g[(size_t)c * n + i] - (proj ? mean[c] : 0.0);
  }
}

// pot2 [2][npot][n], grad2 [2][ngrad][n] (density 0 = q, 1 = projected g)
__global__ void adj_assemble_kernel(const double* dens2, const double* pot2, const double* grad2, int64_t n,
                                    int stokes, double* out_dq, double* out_dxy) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!stokes) {
    const double q = dens2[i], g = dens2[n + i];
    if (out_dq) out_dq[i] = pot2[n + i];
    if (out_dxy)
      for (int c = 0; c < 2; ++c)
        out_dxy[(size_t)c * n + i] = g * grad2[(size_t)c * n + i] + q * grad2[(size_t)(2 + c) * n + i];
  } else {
    if (out_dq)
      for (int a = 0; a < 2; ++a) out_dq[(size_t)a * n + i] = pot2[(size_t)(2 + a) * n + i];
    if (out_dxy)
      for (int c = 0; c < 2; ++c) {
        double s = 0.0;
        for (int a = 0; a < 2; ++a) {
          const double f = dens2[(size_t)a * n + i], g = dens2[(size_t)(2 + a) * n + i];
          s += g * grad2[(size_t)(2 * a + c) * n + i] + f * grad2[(size_t)(4 + 2 * a + c) * n + i];
        }
        out_dxy[(size_t)c * n + i] = s;
      }
  }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct AdjLayout { size_t eval_bytes, dens2, pot2, grad2, mean, total; };

AdjLayout adj_layout(pfmm_plan_s* p, int64_t ns) {
  AdjLayout L;
  const int saved = p->n_dens;
  p->n_dens = 2;
  L.eval_bytes = align_up(pfmm_workspace_bytes(p, ns, ns));
  p->n_dens = saved;
  const int nc = p->kernel == PFMM_STOKES ? 2 : 1;
  const int npot = nc, ngrad = p->kernel == PFMM_STOKES ? 4 : 2;
  size_t off = L.eval_bytes;
  L.dens2 = off; off += align_up(8 * (size_t)2 * nc * ns);
  L.pot2 = off; off += align_up(8 * (size_t)2 * npot * ns);
  L.grad2 = off; off += align_up(8 * (size_t)2 * ngrad * ns);
  L.mean = off; off += 256;
  L.total = off;
  return L;
}

}  // namespace
}  // namespace pfmm

using namespace pfmm;

extern "C" {

size_t pfmm_workspace_bytes_adjoint(pfmm_plan_t p, int64_t ns) {
  if (!p || ns < 0 || ns > PFMM_MAX_POINTS) return 0;
  return adj_layout(p, ns).total;
}

int pfmm_eval_adjoint(pfmm_plan_t p, int64_t ns, const double* src_xy, const double* dens,
                      const double* g_pot, double* out_dq, double* out_dxy, void* workspace,
                      size_t ws_bytes, void* hip_stream) {
  if (!p || ns < 0 || ns > PFMM_MAX_POINTS) return PFMM_EINVAL;
  if (!p->self_exclude || p->n_dens != 1) return PFMM_EINVAL;
  if (ns == 0 || (!out_dq && !out_dxy)) return PFMM_OK;
  if (!src_xy || !dens || !g_pot) return PFMM_EINVAL;
  const AdjLayout L = adj_layout(p, ns);
  if (!workspace || ws_bytes < L.total || ((uintptr_t)workspace & 255)) return PFMM_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  char* ws = (char*)workspace;
  double* dens2 = (double*)(ws + L.dens2);
  double* pot2 = (double*)(ws + L.pot2);
  double* grad2 = (double*)(ws + L.grad2);
  double* mean = (double*)(ws + L.mean);
  const int stokes = p->kernel == PFMM_STOKES;
  const int nc = stokes ? 2 : 1;
  const int proj = p->kernel != PFMM_YUKAWA;
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(1024), 0, st, g_pot, ns, nc, mean);
  const int nb = (int)((ns + ADJ_BLOCK - 1) / ADJ_BLOCK);
  hipLaunchKernelGGL(adj_prep_kernel, dim3(nb), dim3(ADJ_BLOCK), 0, st, dens, g_pot, (const double*)mean, proj,
                     ns, nc, dens2);
  const int saved = p->n_dens;
  p->n_dens = 2;
  int rc = eval_core(p, ns, src_xy, dens2, ns, src_xy, pot2, grad2, ws, L.eval_bytes, hip_stream);
  p->n_dens = saved;
  if (rc) return rc;
  hipLaunchKernelGGL(adj_assemble_kernel, dim3(nb), dim3(ADJ_BLOCK), 0, st, (const double*)dens2,
                     (const double*)pot2, (const double*)grad2, ns, stokes, out_dq, out_dxy);
  return hipGetLastError() == hipSuccess ? PFMM_OK : PFMM_EHIP;
}

}  // extern "C"
