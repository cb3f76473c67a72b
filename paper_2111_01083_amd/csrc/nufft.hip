// NUFFT-accelerated south/north factors (Sec. 6.1, eqs. fastanterp and
// fastinterp, Fig. nufftgrids). For a large aspect ratio the 2M+1 south/north
// plane waves are applied through M_GL Gauss-Legendre lines in y:
//
//   R side: v_jk = gamma(y_j, k) q_j (barycentric weights, eq. baryweights);
//           spread v_jk along x onto a periodic grid of nf points per line
//           (exponential-of-semicircle kernel, LDS sub-grid, then global
//           atomics); FFT each line; divide by the kernel's Fourier transform:
//           f_k(m) = sum_j e^{-i alpha_m x_j} v_jk (type-1 NUFFT, eq. nufft1);
//           then c^S_m = sum_k e^{a_m ybar_k} f_k(m), c^N_m = sum_k e^{-a_m ybar_k} f_k(m).
//   L side: on each line the field of the weighted modes, e.g.
//           G_k(m) = w^S_m e^{-a_m ybar_k} + w^N_m e^{a_m ybar_k}, is divided by
//           the kernel transform, inverse-FFT'd (type-2 NUFFT, eq. nufft2) and
//           interpolated to x_l with the same kernel; the lines are combined
//           with gamma(y_l, k). Derivatives in x and y are carried as their own
//           line fields (i alpha_m G and d/dy of the line weights).
//
// x is wrapped modulo d (the south/north waves are d-periodic in x); the
// west/east part and the Laplace/Stokes m = 0 terms stay on the direct path.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"
#include "nufft.h"

namespace pfmm {

namespace {

constexpr int NU_BLOCK = 256;
constexpr int NU_SPREAD_CHUNK = 4096;   // sources per spreading block
constexpr int NU_LDS_DOUBLES = 8192;    // LDS sub-grid budget (64 KB)

struct NuTabs {
  const double* sn;      // south/north records
  const double* ybar;    // [m_gl]
  const double* bary;    // [m_gl]
  const double* deconv;  // [M + 1]
};

NuTabs tabs_of(const pfmm_plan_s* p) {
  NuTabs t;
  t.sn = p->d_tab;
  t.ybar = p->d_tab + (size_t)p->n_sn * SN_REC + (size_t)p->n_ew * EW_REC;
  t.bary = t.ybar + p->nu.m_gl;
  t.deconv = t.bary + p->nu.m_gl;
  return t;
}

// number of real line fields on each side
int r_fields(int kernel) { return kernel == PFMM_STOKES ? 2 : 1; }
int l_fields(int kernel) { return kernel == PFMM_STOKES ? 12 : 3; }

struct NuLayout {
  size_t grid_r, spec, csn, grid_l, total;
  int lines_per_group, n_groups;
};

NuLayout nu_layout(const pfmm_plan_s* p, int64_t ns, int64_t nt) {
  (void)ns; (void)nt;
  NuLayout L;
  const int nf = p->nu.nf, mgl = p->nu.m_gl, nd = p->n_dens;
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += (b + 255) & ~(size_t)255; return o; };
  L.grid_r = take(8 * (size_t)nd * r_fields(p->kernel) * mgl * nf);               // real spread grids
  L.spec = take(16 * (size_t)nd * r_fields(p->kernel) * mgl * nf);               // complex FFT buffers
  L.csn = take(16 * (size_t)nd * p->n_sn * coef_per_wave(p->kernel));            // south/north coefficients
  L.grid_l = take(16 * (size_t)nd * l_fields(p->kernel) * mgl * nf);             // L-side line buffers
  L.lines_per_group = std::max(1, std::min(mgl, NU_LDS_DOUBLES / nf));
  L.n_groups = (mgl + L.lines_per_group - 1) / L.lines_per_group;
  L.total = off;
  return L;
}

struct c2 { double r, i; };

// exponential of semicircle, phi(z) = exp(b (sqrt(1 - z^2) - 1)) on |z| <= 1
__device__ __forceinline__ double es_kernel(double z, double b) {
  const double t = 1.0 - z * z;
  return t > 0.0 ? exp(b * (sqrt(t) - 1.0)) : 0.0;
}

// barycentric weights gamma(y, k) for all lines (second form, eq. baryweights);
// MG > 0: n == MG lines known at compile time (the arrays stay in registers)
template <int MG>
__device__ __forceinline__ void bary_weights(double y, const double* ybar, const double* sig, int n, double* g) {
  constexpr int NA = MG > 0 ? MG : 32;
  const int m = MG > 0 ? MG : n;
  int hit = -1;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    if (k < m) {
      const double dy = y - ybar[k];
      if (dy == 0.0) hit = k;
      g[k] = sig[k] / (dy == 0.0 ? 1.0 : dy);
      s += g[k];
    }
  }
  const double is = 1.0 / s;
#pragma unroll
  for (int k = 0; k < NA; ++k)
    if (k < m) g[k] = hit >= 0 ? (k == hit ? 1.0 : 0.0) : g[k] * is;
}

// launch-time choices: lines MG in {8, 12, 16} (else 0 = any, up to 32) and
// the kernel support NP in {9, 13, 17} points (w + 1 <= NP)
inline int mg_class(int mgl) { return (mgl == 8 || mgl == 12 || mgl == 16) ? mgl : 0; }
inline int np_class(int w) { return w + 1 <= 9 ? 9 : (w + 1 <= 13 ? 13 : 17); }

struct SpreadArgs {
  int64_t ns;
  int nf, w, mgl, nfield, lines_per_group, n_dens;
  double d, b, inv_h;
  const double *sx, *sy, *dens;
  const double *ybar, *bary;
  double* grid;          // [dens][field][mgl][nf]
};

// grid (x: source chunk, y: line group, z: dens * field)
template <int MG, int NP>
__global__ __launch_bounds__(NU_BLOCK) void spread_kernel(SpreadArgs a) {
  constexpr int NA = MG > 0 ? MG : 32;
  __shared__ double sg[NU_LDS_DOUBLES];
  const int vf = blockIdx.z;
  const int v = vf / a.nfield, fld = vf % a.nfield;
  const int k0 = blockIdx.y * a.lines_per_group;
  const int nk = min(a.lines_per_group, a.mgl - k0);
  const int nf = a.nf;
  for (int t = threadIdx.x; t < nk * nf; t += NU_BLOCK) sg[t] = 0.0;
  __syncthreads();
  const double* q = a.dens + ((size_t)v * a.nfield + fld) * a.ns;
  const int64_t j0 = (int64_t)blockIdx.x * NU_SPREAD_CHUNK;
  const int64_t j1 = min(j0 + NU_SPREAD_CHUNK, a.ns);
  const double half_w = 0.5 * a.w;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += NU_BLOCK) {
    double gam[NA];
    bary_weights<MG>(a.sy[j], a.ybar, a.bary, a.mgl, gam);
    double x = a.sx[j];
    x -= a.d * rint(x / a.d);                       // wrap into [-d/2, d/2]
    const double g = (x + 0.5 * a.d) * a.inv_h;      // grid coordinate
    const int l0 = (int)ceil(g - half_w);
    const double qj = q[j];
#pragma unroll
    for (int t = 0; t < NP; ++t) {
      if (t > a.w) break;
      const int l = l0 + t;
      const double ph = es_kernel((l - g) / half_w, a.b);
      if (ph == 0.0) continue;
      const int lw = ((l % nf) + nf) % nf;
      const double val = qj * ph;
#pragma unroll
      for (int kk = 0; kk < NA; ++kk)
        if (kk >= k0 && kk < k0 + nk) atomicAdd(&sg[(kk - k0) * nf + lw], val * gam[kk]);
    }
  }
  __syncthreads();
  double* out = a.grid + ((size_t)vf * a.mgl + k0) * nf;
  for (int t = threadIdx.x; t < nk * nf; t += NU_BLOCK) {
    const double val = sg[t];
    if (val != 0.0) atomicAdd(&out[t], val);
  }
}

// In-LDS radix-2 FFT of length n (power of two), one transform per block.
// dir = -1: sum_l x_l e^{-2 pi i m l/n}; dir = +1: e^{+...} (no scaling).
// real_in: input is a real array [n] per transform (imaginary part zero).
__global__ __launch_bounds__(NU_BLOCK) void fft_kernel(const double* in_real, const c2* in_cplx, c2* out,
                                                       int n, int log2n, int dir) {
  extern __shared__ c2 buf[];
  const size_t off = (size_t)blockIdx.x * n;
  for (int i = threadIdx.x; i < n; i += NU_BLOCK) {
    const int r = (int)(__brev((unsigned)i) >> (32 - log2n));
    buf[r] = in_real ? c2{in_real[off + i], 0.0} : in_cplx[off + i];
  }
  __syncthreads();
  for (int s = 1; s <= log2n; ++s) {
    const int m = 1 << s, half = m >> 1;
    for (int b = threadIdx.x; b < n / 2; b += NU_BLOCK) {
      const int grp = b / half, j = b - grp * half;
      const int i0 = grp * m + j, i1 = i0 + half;
      double sn, cs;
      sincospi((double)(dir * 2 * j) / (double)m, &sn, &cs);
      const c2 u = buf[i0], v = buf[i1];
      const c2 t = {cs * v.r - sn * v.i, cs * v.i + sn * v.r};
      buf[i0] = {u.r + t.r, u.i + t.i};
      buf[i1] = {u.r - t.r, u.i - t.i};
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += NU_BLOCK) out[off + i] = buf[i];
}

struct CombineArgs {
  int kernel, n_sn, m_lo, mgl, nf, n_dens, ncw, nfield;
  NuTabs t;
  const c2* spec;        // [dens][field][mgl][nf]
  c2* csn;               // [dens][n_sn][ncw] (far_R partial layout, south/north slots)
};

// lines -> south/north coefficients (R side); thread per (mode, dens)
__global__ void combine_kernel(CombineArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (i >= a.n_sn) return;
  const int m = a.m_lo + i;
  const double aa = a.t.sn[i * SN_REC + 1];
  const double fac = ((m & 1) ? -1.0 : 1.0) * a.t.deconv[m];    // e^{i alpha_m d/2} / Phi(alpha_m)
  c2 acc[8];
  for (int c = 0; c < 8; ++c) acc[c] = {0, 0};
  for (int k = 0; k < a.mgl; ++k) {
    const double yb = a.t.ybar[k];
    const double ep = exp(aa * yb), em = 1.0 / ep;
    for (int f = 0; f < a.nfield; ++f) {
      const c2 s = a.spec[(((size_t)v * a.nfield + f) * a.mgl + k) * a.nf + m];
      const c2 fm = {fac * s.r, fac * s.i};
      if (a.kernel == PFMM_STOKES) {
        acc[f].r += ep * fm.r;           acc[f].i += ep * fm.i;            // c^S
        acc[2 + f].r += yb * ep * fm.r;  acc[2 + f].i += yb * ep * fm.i;   // e^S
        acc[4 + f].r += em * fm.r;       acc[4 + f].i += em * fm.i;        // c^N
        acc[6 + f].r += yb * em * fm.r;  acc[6 + f].i += yb * em * fm.i;   // e^N
      } else {
        acc[0].r += ep * fm.r; acc[0].i += ep * fm.i;
        acc[1].r += em * fm.r; acc[1].i += em * fm.i;
      }
    }
  }
  c2* o = a.csn + ((size_t)v * a.n_sn + i) * a.ncw;
  for (int c = 0; c < a.ncw; ++c) o[c] = acc[c];
}

struct LinesArgs {
  int kernel, n_sn, m_lo, mgl, nf, n_dens, ncw, n_coef;
  NuTabs t;
  const c2* w;           // [dens][n_coef] (south/north slots first)
  c2* grid;              // [dens][lfield][mgl][nf], zeroed beforehand
};

// weighted modes -> line spectra (L side); thread per (mode, line, dens)
__global__ void lines_kernel(LinesArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y, v = blockIdx.z;
  if (i >= a.n_sn) return;
  const int m = a.m_lo + i;
  const double al = a.t.sn[i * SN_REC], aa = a.t.sn[i * SN_REC + 1];
  const double fac = ((m & 1) ? -1.0 : 1.0) * a.t.deconv[m];    // e^{-i alpha_m d/2} / Phi
  const double yb = a.t.ybar[k];
  const double ep = exp(aa * yb), em = 1.0 / ep;
  const c2* ww = a.w + (size_t)v * a.n_coef + (size_t)i * a.ncw;
  const int nlf = a.kernel == PFMM_STOKES ? 12 : 3;
  auto put = [&](int f, c2 val) {
    a.grid[(((size_t)v * nlf + f) * a.mgl + k) * a.nf + m] = {fac * val.r, fac * val.i};
  };
  auto lin = [&](c2 s, c2 n, double cs, double cn) { return c2{cs * s.r + cn * n.r, cs * s.i + cn * n.i}; };
  auto mul_i = [&](c2 z, double s) { return c2{-s * z.i, s * z.r}; };   // i s z
  if (a.kernel == PFMM_STOKES) {
    for (int c = 0; c < 2; ++c) {
      const c2 P = lin(ww[c], ww[4 + c], em, ep), Q = lin(ww[2 + c], ww[6 + c], em, ep);
      put(c, P);                                   // P
      put(2 + c, Q);                               // Q
      put(4 + c, mul_i(P, al));                    // P_x
      put(6 + c, mul_i(Q, al));                    // Q_x
      put(8 + c, lin(ww[c], ww[4 + c], -aa * em, aa * ep));      // P_y
      put(10 + c, lin(ww[2 + c], ww[6 + c], -aa * em, aa * ep)); // Q_y
    }
  } else {
    const c2 G = lin(ww[0], ww[1], em, ep);
    put(0, G);
    put(1, mul_i(G, al));
    put(2, lin(ww[0], ww[1], -aa * em, aa * ep));
  }
}

struct InterpArgs {
  int64_t nt;
  int kernel, mgl, nf, w, n_dens;
  double d, b, inv_h;
  NuTabs t;
  const double *tx, *ty;
  const c2* grid;        // [dens][lfield][mgl][nf] after the inverse FFT
  double* val;           // [dens][NOUT][nt]
};

// One target per thread. The barycentric weight of line k is formed inside
// the line loop from the normalising sum (no per-thread weight array), the
// NP kernel values stay in registers, and the line fields go through LDS.
template <int NP, bool STOKES>
__global__ __launch_bounds__(NU_BLOCK) void interp_kernel(InterpArgs a) {
  constexpr int NLF = STOKES ? 12 : 3, NO = STOKES ? 6 : 3;
  __shared__ double sF[NLF][NU_BLOCK];
  const int64_t l = (int64_t)blockIdx.x * NU_BLOCK + threadIdx.x;
  if (l >= a.nt) return;                 // no block-wide barrier below
  const int tid = threadIdx.x;
  const double y = a.ty[l];
  // barycentric weights (second form): g_k = (sig_k / (y - ybar_k)) / sum_j sig_j / (y - ybar_j)
  int hit = -1;
  double ssum = 0.0;
  for (int k = 0; k < a.mgl; ++k) {
    const double dy = y - a.t.ybar[k];
    if (dy == 0.0) hit = k;
    ssum += a.t.bary[k] / (dy == 0.0 ? 1.0 : dy);
  }
  const double inv_s = 1.0 / ssum;
  double x = a.tx[l];
  x -= a.d * rint(x / a.d);
  const double g = (x + 0.5 * a.d) * a.inv_h;
  const double half_w = 0.5 * a.w;
  const int l0 = (int)ceil(g - half_w);
  double ph[NP];
  int idx[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    const int li = l0 + t;
    ph[t] = t <= a.w ? es_kernel((li - g) / half_w, a.b) : 0.0;
    idx[t] = ((li % a.nf) + a.nf) % a.nf;
  }
  for (int v = 0; v < a.n_dens; ++v) {
    for (int f = 0; f < NLF; ++f) {
      double s = 0.0;
      for (int k = 0; k < a.mgl; ++k) {
        const double gk = hit >= 0 ? (k == hit ? 1.0 : 0.0) : a.t.bary[k] / (y - a.t.ybar[k]) * inv_s;
        const c2* row = a.grid + (((size_t)v * NLF + f) * a.mgl + k) * a.nf;
        double r = 0.0;
#pragma unroll
        for (int t = 0; t < NP; ++t)
          if (t <= a.w) r += ph[t] * row[idx[t]].r;
        s += gk * r;
      }
      sF[f][tid] = s;
    }
    double* o = a.val + (size_t)v * NO * a.nt;
    if constexpr (STOKES) {
      // u = P - y Q; du/dx = P_x - y Q_x; du/dy = P_y - y Q_y - Q
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        o[(size_t)c * a.nt + l] = sF[c][tid] - y * sF[2 + c][tid];
        o[(size_t)(2 + 2 * c) * a.nt + l] = sF[4 + c][tid] - y * sF[6 + c][tid];
        o[(size_t)(3 + 2 * c) * a.nt + l] = sF[8 + c][tid] - y * sF[10 + c][tid] - sF[2 + c][tid];
      }
    } else {
      o[l] = sF[0][tid];
      o[a.nt + l] = sF[1][tid];
      o[2 * a.nt + l] = sF[2][tid];
    }
  }
}

// dispatch over the compile-time classes
template <int MG, int NP>
void launch_spread_np(dim3 g, const SpreadArgs& sa, hipStream_t st) {
  hipLaunchKernelGGL((spread_kernel<MG, NP>), g, dim3(NU_BLOCK), 0, st, sa);
}
template <int MG>
void launch_spread_mg(dim3 g, const SpreadArgs& sa, hipStream_t st) {
  switch (np_class(sa.w)) {
    case 9: launch_spread_np<MG, 9>(g, sa, st); break;
    case 13: launch_spread_np<MG, 13>(g, sa, st); break;
    default: launch_spread_np<MG, 17>(g, sa, st); break;
  }
}
void launch_spread(dim3 g, const SpreadArgs& sa, hipStream_t st) {
  switch (mg_class(sa.mgl)) {
    case 8: launch_spread_mg<8>(g, sa, st); break;
    case 12: launch_spread_mg<12>(g, sa, st); break;
    case 16: launch_spread_mg<16>(g, sa, st); break;
    default: launch_spread_mg<0>(g, sa, st); break;
  }
}
template <int NP>
void launch_interp_np(dim3 g, const InterpArgs& ia, hipStream_t st) {
  if (ia.kernel == PFMM_STOKES) hipLaunchKernelGGL((interp_kernel<NP, true>), g, dim3(NU_BLOCK), 0, st, ia);
  else hipLaunchKernelGGL((interp_kernel<NP, false>), g, dim3(NU_BLOCK), 0, st, ia);
}
void launch_interp(dim3 g, const InterpArgs& ia, hipStream_t st) {
  switch (np_class(ia.w)) {
    case 9: launch_interp_np<9>(g, ia, st); break;
    case 13: launch_interp_np<13>(g, ia, st); break;
    default: launch_interp_np<17>(g, ia, st); break;
  }
}

__global__ void zero_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

void zero(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
}

int ilog2(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }

}  // namespace

size_t nufft_workspace_bytes(const pfmm_plan_s* p, int64_t ns, int64_t nt) {
  return nu_layout(p, ns, nt).total;
}

int nufft_R(const pfmm_plan_s* p, int64_t ns, const double* sx, const double* sy, const double* dens,
            char* ws, hipStream_t st, const double** csn_out) {
  const NuLayout L = nu_layout(p, ns, 0);
  const NuTabs t = tabs_of(p);
  const int nf = p->nu.nf, mgl = p->nu.m_gl, nd = p->n_dens, nfr = r_fields(p->kernel);
  double* grid = (double*)(ws + L.grid_r);
  c2* spec = (c2*)(ws + L.spec);
  c2* csn = (c2*)(ws + L.csn);
  zero(grid, (int64_t)nd * nfr * mgl * nf, st);
  if (ns > 0) {
    SpreadArgs sa{};
    sa.ns = ns; sa.nf = nf; sa.w = p->nu.w; sa.mgl = mgl; sa.nfield = nfr;
    sa.lines_per_group = L.lines_per_group; sa.n_dens = nd;
    sa.d = p->geo.d; sa.b = p->nu.es_beta; sa.inv_h = nf / p->geo.d;
    sa.sx = sx; sa.sy = sy; sa.dens = dens; sa.ybar = t.ybar; sa.bary = t.bary; sa.grid = grid;
    dim3 g((unsigned)((ns + NU_SPREAD_CHUNK - 1) / NU_SPREAD_CHUNK), (unsigned)L.n_groups, (unsigned)(nd * nfr));
    launch_spread(g, sa, st);
  }
  const int nfft = nd * nfr * mgl;
  hipLaunchKernelGGL(fft_kernel, dim3(nfft), dim3(NU_BLOCK), nf * sizeof(c2), st, (const double*)grid,
                     (const c2*)nullptr, spec, nf, ilog2(nf), -1);
  CombineArgs ca{};
  ca.kernel = p->kernel; ca.n_sn = p->n_sn; ca.m_lo = p->m_lo; ca.mgl = mgl; ca.nf = nf; ca.n_dens = nd;
  ca.ncw = coef_per_wave(p->kernel); ca.nfield = nfr; ca.t = t; ca.spec = spec; ca.csn = csn;
  hipLaunchKernelGGL(combine_kernel, dim3((p->n_sn + 127) / 128, nd), dim3(128), 0, st, ca);
  *csn_out = (const double*)csn;
  return PFMM_OK;
}

int nufft_L(const pfmm_plan_s* p, int64_t nt, const double* tx, const double* ty, const double* w,
            int n_coef, char* ws, hipStream_t st, const double** val_out, double* val) {
  const NuLayout L = nu_layout(p, 0, nt);
  const NuTabs t = tabs_of(p);
  const int nf = p->nu.nf, mgl = p->nu.m_gl, nd = p->n_dens, nlf = l_fields(p->kernel);
  c2* grid = (c2*)(ws + L.grid_l);
  zero((double*)grid, 2 * (int64_t)nd * nlf * mgl * nf, st);
  LinesArgs la{};
  la.kernel = p->kernel; la.n_sn = p->n_sn; la.m_lo = p->m_lo; la.mgl = mgl; la.nf = nf; la.n_dens = nd;
  la.ncw = coef_per_wave(p->kernel); la.n_coef = n_coef; la.t = t; la.w = (const c2*)w; la.grid = grid;
  hipLaunchKernelGGL(lines_kernel, dim3((p->n_sn + 127) / 128, mgl, nd), dim3(128), 0, st, la);
  const int nfft = nd * nlf * mgl;
  hipLaunchKernelGGL(fft_kernel, dim3(nfft), dim3(NU_BLOCK), nf * sizeof(c2), st, (const double*)nullptr,
                     (const c2*)grid, grid, nf, ilog2(nf), +1);
  if (nt > 0) {
    InterpArgs ia{};
    ia.nt = nt; ia.kernel = p->kernel; ia.mgl = mgl; ia.nf = nf; ia.w = p->nu.w; ia.n_dens = nd;
    ia.d = p->geo.d; ia.b = p->nu.es_beta; ia.inv_h = nf / p->geo.d; ia.t = t; ia.tx = tx; ia.ty = ty;
    ia.grid = grid; ia.val = val;
    launch_interp(dim3((unsigned)((nt + NU_BLOCK - 1) / NU_BLOCK)), ia, st);
  }
  *val_out = val;
  return PFMM_OK;
}

}  // namespace pfmm
