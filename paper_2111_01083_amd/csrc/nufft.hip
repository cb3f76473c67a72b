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

#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "nufft.h"

namespace pfmm {

namespace {

typedef const __attribute__((address_space(4))) double cdouble;   // tables: scalar loads

constexpr int NU_BLOCK = 256;
constexpr int SP_BLOCK = 512;           // spreading block (8 wavefronts)
constexpr int SP_WAVES = SP_BLOCK / 64;
constexpr int NU_LDS_BYTES = 65536;     // LDS sub-grid budget of a spreading block
constexpr int FFT_LDS_MAX = 4096;       // longest line transformed inside one block's LDS

struct NuTabs {
  const double* sn;      // south/north records
  const double* ybar;    // [m_gl]
  const double* bary;    // [m_gl]
  const double* deconv;  // [M + 1]
  const double* poly;    // [ES_TAPS][ES_COEF] kernel polynomials
};

NuTabs tabs_of(const pfmm_plan_s* p) {
  NuTabs t;
  t.sn = p->d_tab;
  t.ybar = p->d_tab + (size_t)p->n_sn * SN_REC + (size_t)p->n_ew * EW_REC;
  t.bary = t.ybar + p->nu.m_gl;
  t.deconv = t.bary + p->nu.m_gl;
  t.poly = t.deconv + (p->M + 1);
  return t;
}

// number of real line fields on each side
int r_fields(int kernel) { return kernel == PFMM_STOKES ? 2 : 1; }
int l_fields(int kernel) { return kernel == PFMM_STOKES ? 12 : 3; }

struct NuLayout {
  size_t grid_r, spec, csn, grid_l, real_l, fft_tmp, total;
  int lines_per_group, n_groups;
  bool spread_direct;
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
  L.real_l = take(8 * (size_t)nd * l_fields(p->kernel) * mgl * nf);              // their real parts, [dens][line][nf][field]
  // four-step transforms of lines longer than one block's LDS: a scratch copy
  L.fft_tmp = nf > FFT_LDS_MAX ? take(16 * (size_t)nd * l_fields(p->kernel) * mgl * nf) : 0;
  // spreading sub-grid in LDS (FP64: the deconvolution amplifies the
  // rounding of the grid's high frequencies, so the sums stay in FP64)
  L.lines_per_group = std::max(1, std::min(mgl, (int)(NU_LDS_BYTES / 8) / nf));
  // a line longer than the LDS budget: spread straight into the global grid
  L.spread_direct = (size_t)nf * 8 > (size_t)NU_LDS_BYTES;
  if (L.spread_direct) L.lines_per_group = mgl;
  L.n_groups = (mgl + L.lines_per_group - 1) / L.lines_per_group;
  L.total = off;
  return L;
}

struct c2 { double r, i; };

// Kernel values at the taps of a point at grid coordinate g: l0 = ceil(g -
// w/2) is the first tap, and tap t (0..w) has value p_t(u), u = 2(l0 - g +
// w/2) - 1 (polynomials fitted by the planner to the exponential of
// semicircle exp(b (sqrt(1 - z^2) - 1)), z = (l0 + t - g)/(w/2)). Taps t > w
// are zero.
template <int NP>
__device__ __forceinline__ void es_taps(double g, int w, int deg, const double* poly, int& l0, double* ph) {
  const double half_w = 0.5 * w;
  const double l0d = ceil(g - half_w);
  l0 = (int)l0d;
  const double u = 2.0 * (l0d - g + half_w) - 1.0;
  const cdouble* c = (const cdouble*)poly;
#pragma unroll
  for (int t = 0; t < NP; ++t) ph[t] = c[t * ES_COEF + deg - 1];
  for (int k = deg - 2; k >= 0; --k) {
#pragma unroll
    for (int t = 0; t < NP; ++t) ph[t] = fma(ph[t], u, c[t * ES_COEF + k]);
  }
#pragma unroll
  for (int t = 0; t < NP; ++t)
    if (t > w) ph[t] = 0.0;
}

// 1/x in FP64 from the hardware estimate and two Newton steps
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// barycentric weights gamma(y, k) for all lines (second form, eq. baryweights);
// MG > 0: n == MG lines known at compile time (the arrays stay in registers)
template <int MG>
__device__ __forceinline__ void bary_weights(double y, const double* ybar, const double* sig, int n, double* g) {
  constexpr int NA = MG > 0 ? MG : 32;
  const int m = MG > 0 ? MG : n;
  const cdouble* yb = (const cdouble*)ybar;
  const cdouble* sg = (const cdouble*)sig;
  int hit = -1;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    if (k < m) {
      const double dy = y - yb[k];
      if (dy == 0.0) hit = k;
      g[k] = sg[k] * rcp64(dy == 0.0 ? 1.0 : dy);
      s += g[k];
    }
  }
  const double is = rcp64(s);
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
  int nf, w, deg, mgl, nfield, lines_per_group, n_dens;
  double d, inv_h;
  const double *sx, *sy, *dens;
  const double *ybar, *bary, *poly;
  double* grid;          // [dens][field][mgl][nf]
};

// grid (x: source slice, y: line group, z: dens * field). Lane l of every
// wavefront works in segment l of the source array (64 segments of
// S = ceil(n/64) sources): global wavefront gw of GW takes offsets gw,
// gw + GW, ... of each segment, so the 64 lanes of a wavefront hold points
// far apart in the input order (inputs stored cluster by cluster would
// otherwise put a wavefront's 64 LDS atomic adds on the same few grid
// cells), while the SP_WAVES wavefronts of a block read neighbouring words
// of the same cache lines. Each block accumulates its lines in LDS (FP64)
// and adds them to the global grid once (lines too long for the LDS budget:
// straight into the global grid).
template <int MG, int NP, bool DIRECT>
__global__ __launch_bounds__(SP_BLOCK) void spread_kernel(SpreadArgs a) {
  constexpr int NA = MG > 0 ? MG : 32;
  extern __shared__ __align__(16) char sp_smem[];
  const int vf = blockIdx.z;
  const int v = vf / a.nfield, fld = vf % a.nfield;
  const int k0 = blockIdx.y * a.lines_per_group;
  const int nk = min(a.lines_per_group, a.mgl - k0);
  const int nf = a.nf;
  double* out = a.grid + ((size_t)vf * a.mgl + k0) * nf;
  // DIRECT (lines longer than the LDS budget): atomics straight into the grid
  double* sg = DIRECT ? out : (double*)sp_smem;
  if (!DIRECT) {
    for (int t = threadIdx.x; t < nk * nf; t += SP_BLOCK) sg[t] = 0.0;
    __syncthreads();
  }
  const double* q = a.dens + ((size_t)v * a.nfield + fld) * a.ns;
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * SP_WAVES + (threadIdx.x >> 6);
  const int64_t GW = (int64_t)gridDim.x * SP_WAVES;
  const int64_t seg = (a.ns + 63) / 64;
  for (int64_t c = gw; c < seg; c += GW) {   // uniform over the wavefront
    const int64_t j = lane * seg + c;
    if (j < a.ns) {
      double gam[NA];
      bary_weights<MG>(a.sy[j], a.ybar, a.bary, a.mgl, gam);
      double x = a.sx[j];
      x -= a.d * rint(x / a.d);                       // wrap into [-d/2, d/2]
      const double g = (x + 0.5 * a.d) * a.inv_h;      // grid coordinate
      int l0;
      double ph[NP];
      es_taps<NP>(g, a.w, a.deg, a.poly, l0, ph);
      const double qj = q[j];
      int lw = ((l0 % nf) + nf) % nf;
#pragma unroll
      for (int t = 0; t < NP; ++t) {
        const double val = qj * ph[t];
#pragma unroll
        for (int kk = 0; kk < NA; ++kk)
          if (kk >= k0 && kk < k0 + nk) atomicAdd(&sg[(kk - k0) * nf + lw], val * gam[kk]);
        lw = lw + 1 == nf ? 0 : lw + 1;
      }
    }
  }
  if (DIRECT) return;
  __syncthreads();
  for (int t = threadIdx.x; t < nk * nf; t += SP_BLOCK) {
    const double val = sg[t];
    if (val != 0.0) atomicAdd(&out[t], val);
  }
}

// In-LDS radix-2 FFT of length n (power of two), one transform per block.
// dir = -1: sum_l x_l e^{-2 pi i m l/n}; dir = +1: e^{+...} (no scaling).
// real_in: input is a real array [n] per transform (imaginary part zero).
// real_out (optional): the real parts of transform b = (v * nfl + f) * mgl + k
// go to real_out[((v * mgl + k) * n + i) * nfl + f] (fields of a grid point
// side by side; FP32 when real32 is set), and out is not written.
__global__ __launch_bounds__(NU_BLOCK) void fft_kernel(const double* in_real, const c2* in_cplx, c2* out,
                                                       int n, int log2n, int dir, double* real_out, int nfl,
                                                       int mgl, int real32) {
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
  if (real_out) {
    const int b = blockIdx.x, k = b % mgl, vf = b / mgl, f = vf % nfl, v = vf / nfl;
    const size_t o0 = (((size_t)v * mgl + k) * n) * nfl + f;
    if (real32) {
      float* o = (float*)real_out + o0;
      for (int i = threadIdx.x; i < n; i += NU_BLOCK) o[(size_t)i * nfl] = (float)buf[i].r;
    } else {
      double* o = real_out + o0;
      for (int i = threadIdx.x; i < n; i += NU_BLOCK) o[(size_t)i * nfl] = buf[i].r;
    }
  } else {
    for (int i = threadIdx.x; i < n; i += NU_BLOCK) out[off + i] = buf[i];
  }
}

// Longer lines (n > FFT_LDS_MAX points): four-step transform n = n1 n2. With
// l = l1 + n1 l2 and k = k2 + n2 k1,
//   X[k] = sum_l1 w_n^{l1 k2} w_n1^{l1 k1} (sum_l2 x[l1 + n1 l2] w_n2^{l2 k2}),
// so pass 1 takes n1 transforms of length n2 (stride n1) and multiplies by
// the twiddles w_n^{l1 k2}, and pass 2 takes n2 transforms of length n1.
// One block per (transform, line): element i of transform b of line y is read
// at y * n + b * in_bs + i * in_es and written at y * n + b * out_bs + i * out_es;
// tw_n > 0 multiplies output k of transform b by e^{dir 2 pi i b k / tw_n}.
// real_out as in fft_kernel (pass 2 of the L side only).
__global__ __launch_bounds__(NU_BLOCK) void fft_pass_kernel(const double* in_real, const c2* in_cplx, c2* out,
                                                            int64_t n, int ns, int log2ns, int dir, int64_t in_bs,
                                                            int64_t in_es, int64_t out_bs, int64_t out_es,
                                                            int64_t tw_n, double* real_out, int nfl, int mgl,
                                                            int real32) {
  extern __shared__ c2 buf[];
  const int64_t b = blockIdx.x, y = blockIdx.y;
  const size_t line = (size_t)y * n;
  for (int i = threadIdx.x; i < ns; i += NU_BLOCK) {
    const int r = (int)(__brev((unsigned)i) >> (32 - log2ns));
    const size_t at = line + b * in_bs + (size_t)i * in_es;
    buf[r] = in_real ? c2{in_real[at], 0.0} : in_cplx[at];
  }
  __syncthreads();
  for (int s = 1; s <= log2ns; ++s) {
    const int m = 1 << s, half = m >> 1;
    for (int q = threadIdx.x; q < ns / 2; q += NU_BLOCK) {
      const int grp = q / half, j = q - grp * half;
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
  for (int i = threadIdx.x; i < ns; i += NU_BLOCK) {
    c2 v = buf[i];
    if (tw_n > 0) {
      const int64_t e = (b * (int64_t)i) % tw_n;          // exact phase index
      double sn, cs;
      sincospi((double)(dir * 2) * (double)e / (double)tw_n, &sn, &cs);
      v = {cs * v.r - sn * v.i, cs * v.i + sn * v.r};
    }
    const int64_t pos = b * out_bs + (int64_t)i * out_es;   // position within the line
    if (real_out) {
      const int k = (int)(y % mgl), vf = (int)(y / mgl), f = vf % nfl, vv = vf / nfl;
      const size_t o0 = ((((size_t)vv * mgl + k) * n) + pos) * nfl + f;
      if (real32) ((float*)real_out)[o0] = (float)v.r;
      else real_out[o0] = v.r;
    } else {
      out[line + pos] = v;
    }
  }
}

int ilog2i(int64_t n) { int l = 0; while (((int64_t)1 << l) < n) ++l; return l; }

// n-point transform of `lines` lines: in-LDS for n <= FFT_LDS_MAX, else the
// four-step form through tmp (lines * n complex). Output as for fft_kernel.
void line_fft(const double* in_real, const c2* in_cplx, c2* out, c2* tmp, int64_t n, int lines, int dir,
              double* real_out, int nfl, int mgl, int real32, hipStream_t st) {
  if (n <= FFT_LDS_MAX) {
    hipLaunchKernelGGL(fft_kernel, dim3(lines), dim3(NU_BLOCK), n * sizeof(c2), st, in_real, in_cplx, out, (int)n,
                       ilog2i(n), dir, real_out, nfl, mgl, real32);
    return;
  }
  const int L = ilog2i(n);
  const int64_t n2 = (int64_t)1 << (L / 2), n1 = n / n2;    // n1 >= n2, both <= FFT_LDS_MAX
  // pass 1: n1 transforms (l1) of length n2 over l2 (stride n1); tmp[l1 n2 + k2]
  hipLaunchKernelGGL(fft_pass_kernel, dim3((unsigned)n1, lines), dim3(NU_BLOCK), n2 * sizeof(c2), st, in_real,
                     in_cplx, tmp, n, (int)n2, ilog2i(n2), dir, (int64_t)1, n1, n2, (int64_t)1, n, (double*)nullptr,
                     1, 1, 0);
  // pass 2: n2 transforms (k2) of length n1 over l1 (stride n2); X[k2 + n2 k1]
  hipLaunchKernelGGL(fft_pass_kernel, dim3((unsigned)n2, lines), dim3(NU_BLOCK), n1 * sizeof(c2), st,
                     (const double*)nullptr, (const c2*)tmp, out, n, (int)n1, ilog2i(n1), dir, (int64_t)1, n2,
                     (int64_t)1, n2, (int64_t)0, real_out, nfl, mgl, real32);
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
  int kernel, mgl, nf, w, deg, n_dens;
  double d, inv_h;
  NuTabs t;
  const double *tx, *ty;
  const void* grid;      // real line fields [dens][mgl][nf][lfield] after the inverse FFT (FP32 or FP64)
  double* val;           // [dens][NOUT][nt]
};

// One target per thread (targets in binned order, so a wavefront's taps fall
// on nearby grid points): line weights and kernel taps in registers, then
// for every line the NLF fields of its w + 1 taps (side by side in memory;
// FP32 for mixed plans, whose line fields follow the inverse FFT with no
// further amplification, FP64 otherwise).
template <int MG, int NP, bool STOKES, typename gr_t>
__global__ __launch_bounds__(NU_BLOCK) void interp_kernel(InterpArgs a) {
  constexpr int NLF = STOKES ? 12 : 3, NO = STOKES ? 6 : 3;
  constexpr int NA = MG > 0 ? MG : 32;
  const int64_t l = (int64_t)blockIdx.x * NU_BLOCK + threadIdx.x;
  if (l >= a.nt) return;                 // no block-wide barrier below
  const double y = a.ty[l];
  double gam[NA];
  bary_weights<MG>(y, a.t.ybar, a.t.bary, a.mgl, gam);
  double x = a.tx[l];
  x -= a.d * rint(x / a.d);
  const double g = (x + 0.5 * a.d) * a.inv_h;
  int l0;
  double ph[NP];
  es_taps<NP>(g, a.w, a.deg, a.t.poly, l0, ph);
  const int nf = a.nf;
  const int lw0 = ((l0 % nf) + nf) % nf;
  const int mgl = MG > 0 ? MG : a.mgl;
  for (int v = 0; v < a.n_dens; ++v) {
    double F[NLF];
#pragma unroll
    for (int f = 0; f < NLF; ++f) F[f] = 0.0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      if (k >= mgl) break;
      const gr_t* row = (const gr_t*)a.grid + (((size_t)v * mgl + k) * nf) * NLF;
      double S[NLF];
#pragma unroll
      for (int f = 0; f < NLF; ++f) S[f] = 0.0;
      int lw = lw0;
#pragma unroll
      for (int t = 0; t < NP; ++t) {
        const gr_t* pt = row + (size_t)lw * NLF;
#pragma unroll
        for (int f = 0; f < NLF; ++f) S[f] = fma(ph[t], (double)pt[f], S[f]);
        lw = lw + 1 == nf ? 0 : lw + 1;
      }
#pragma unroll
      for (int f = 0; f < NLF; ++f) F[f] = fma(gam[k], S[f], F[f]);
    }
    double* o = a.val + (size_t)v * NO * a.nt;
    if constexpr (STOKES) {
      // u = P - y Q; du/dx = P_x - y Q_x; du/dy = P_y - y Q_y - Q
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        o[(size_t)c * a.nt + l] = F[c] - y * F[2 + c];
        o[(size_t)(2 + 2 * c) * a.nt + l] = F[4 + c] - y * F[6 + c];
        o[(size_t)(3 + 2 * c) * a.nt + l] = F[8 + c] - y * F[10 + c] - F[2 + c];
      }
    } else {
      o[l] = F[0];
      o[a.nt + l] = F[1];
      o[2 * a.nt + l] = F[2];
    }
  }
}

// dispatch over the compile-time classes
template <int MG, int NP>
void launch_spread_np(dim3 g, const SpreadArgs& sa, bool direct, hipStream_t st) {
  if (direct) {
    hipLaunchKernelGGL((spread_kernel<MG, NP, true>), g, dim3(SP_BLOCK), 0, st, sa);
  } else {
    const size_t lds = (size_t)sa.lines_per_group * sa.nf * 8;
    hipLaunchKernelGGL((spread_kernel<MG, NP, false>), g, dim3(SP_BLOCK), lds, st, sa);
  }
}
template <int MG>
void launch_spread_mg(dim3 g, const SpreadArgs& sa, bool direct, hipStream_t st) {
  switch (np_class(sa.w)) {
    case 9: launch_spread_np<MG, 9>(g, sa, direct, st); break;
    case 13: launch_spread_np<MG, 13>(g, sa, direct, st); break;
    default: launch_spread_np<MG, 17>(g, sa, direct, st); break;
  }
}
void launch_spread(dim3 g, const SpreadArgs& sa, bool direct, hipStream_t st) {
  switch (mg_class(sa.mgl)) {
    case 8: launch_spread_mg<8>(g, sa, direct, st); break;
    case 12: launch_spread_mg<12>(g, sa, direct, st); break;
    case 16: launch_spread_mg<16>(g, sa, direct, st); break;
    default: launch_spread_mg<0>(g, sa, direct, st); break;
  }
}
template <int MG, int NP, typename gr_t>
void launch_interp_np(dim3 g, const InterpArgs& ia, hipStream_t st) {
  if (ia.kernel == PFMM_STOKES) hipLaunchKernelGGL((interp_kernel<MG, NP, true, gr_t>), g, dim3(NU_BLOCK), 0, st, ia);
  else hipLaunchKernelGGL((interp_kernel<MG, NP, false, gr_t>), g, dim3(NU_BLOCK), 0, st, ia);
}
template <int MG, typename gr_t>
void launch_interp_mg(dim3 g, const InterpArgs& ia, hipStream_t st) {
  switch (np_class(ia.w)) {
    case 9: launch_interp_np<MG, 9, gr_t>(g, ia, st); break;
    case 13: launch_interp_np<MG, 13, gr_t>(g, ia, st); break;
    default: launch_interp_np<MG, 17, gr_t>(g, ia, st); break;
  }
}
template <typename gr_t>
void launch_interp_t(dim3 g, const InterpArgs& ia, hipStream_t st) {
  switch (mg_class(ia.mgl)) {
    case 8: launch_interp_mg<8, gr_t>(g, ia, st); break;
    case 12: launch_interp_mg<12, gr_t>(g, ia, st); break;
    case 16: launch_interp_mg<16, gr_t>(g, ia, st); break;
    default: launch_interp_mg<0, gr_t>(g, ia, st); break;
  }
}
void launch_interp(dim3 g, const InterpArgs& ia, bool mixed, hipStream_t st) {
  if (mixed) launch_interp_t<float>(g, ia, st);
  else launch_interp_t<double>(g, ia, st);
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
    sa.ns = ns; sa.nf = nf; sa.w = p->nu.w; sa.deg = p->nu.es_deg; sa.mgl = mgl; sa.nfield = nfr;
    sa.lines_per_group = L.lines_per_group; sa.n_dens = nd;
    sa.d = p->geo.d; sa.inv_h = nf / p->geo.d;
    sa.sx = sx; sa.sy = sy; sa.dens = dens; sa.ybar = t.ybar; sa.bary = t.bary; sa.poly = t.poly;
    sa.grid = grid;
    // about two blocks per compute unit in all, each slice of at least 4
    // sources per thread
    const int64_t yz = (int64_t)L.n_groups * nd * nfr;
    const int64_t by_work = (ns + 4 * SP_BLOCK - 1) / (4 * SP_BLOCK);
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>(by_work, (512 + yz - 1) / yz));
    dim3 g((unsigned)bx, (unsigned)L.n_groups, (unsigned)(nd * nfr));
    launch_spread(g, sa, L.spread_direct, st);
  }
  const int nfft = nd * nfr * mgl;
  line_fft((const double*)grid, (const c2*)nullptr, spec, (c2*)(ws + L.fft_tmp), nf, nfft, -1, (double*)nullptr,
           1, 1, 0, st);
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
  double* real_l = (double*)(ws + L.real_l);
  const bool mixed = p->precision == PFMM_MIXED;   // FP32 line fields (no deconvolution follows)
  line_fft((const double*)nullptr, (const c2*)grid, grid, (c2*)(ws + L.fft_tmp), nf, nfft, +1, real_l, nlf, mgl,
           mixed ? 1 : 0, st);
  if (nt > 0) {
    InterpArgs ia{};
    ia.nt = nt; ia.kernel = p->kernel; ia.mgl = mgl; ia.nf = nf; ia.w = p->nu.w; ia.deg = p->nu.es_deg;
    ia.n_dens = nd; ia.d = p->geo.d; ia.inv_h = nf / p->geo.d; ia.t = t; ia.tx = tx; ia.ty = ty;
    ia.grid = real_l; ia.val = val;
    launch_interp(dim3((unsigned)((nt + NU_BLOCK - 1) / NU_BLOCK)), ia, mixed, st);
  }
  *val_out = val;
  return PFMM_OK;
}

}  // namespace pfmm
