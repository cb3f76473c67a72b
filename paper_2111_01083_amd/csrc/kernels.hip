// Device kernels of the periodic evaluator (gfx950):
//   prep   -- rotate/wrap points into the canonical cell; FP64 (and, mixed, FP32) densities
//   near   -- direct sum over the cell and its nearest images (Def. 1)
//   far_R  -- sources -> plane-wave coefficients (R of P = L D R, Sec. 6)
//   far_D  -- chunk reduction and the diagonal weights D
//   far_L  -- plane waves -> targets; adds the near partials; user frame out
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_math.h"
#include "kernels.h"

namespace pfmm {

// ---------------------------------------------------------------------------
// prep
// ---------------------------------------------------------------------------
// read-only tables (plan tables): loads through the constant address space
// with a uniform index become scalar loads
typedef const __attribute__((address_space(4))) double cdouble;
typedef const __attribute__((address_space(4))) BatchCell cBatchCell;
__device__ __forceinline__ const cdouble* as_const(const double* p) { return (const cdouble*)p; }

__global__ void prep_points_kernel(PrepArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double x = a.xy[i], y = a.xy[a.ystride + i];
  double xc = a.rc * x - a.rs * y, yc = a.rs * x + a.rc * y;
  // lattice coordinates u2 = y/eta, u1 = (x - u2 xi)/d, then u <- u - rint(u)
  // (singly periodic: u1 only)
  double k2 = a.wrap_y ? rint(yc / a.eta) : 0.0;
  yc -= k2 * a.eta;
  xc -= k2 * a.xi;
  double k1 = rint((xc - (yc / a.eta) * a.xi) / a.d);
  xc -= k1 * a.d;
  a.cx[i] = xc;
  a.cy[i] = yc;
}

__global__ void prep_dens_kernel(PrepDensArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t is = a.in_stride;
  for (int v = 0; v < a.n_dens; ++v) {
    if (a.stokes) {
      const double* f = a.dens + (size_t)v * 2 * is;
      double f1 = f[i], f2 = f[is + i];
      double g1 = a.rc * f1 - a.rs * f2, g2 = a.rs * f1 + a.rc * f2;
      double* o = a.out64 + (size_t)v * 2 * a.n;
      o[i] = g1; o[a.n + i] = g2;
      if (a.out32) {
        float* o32 = a.out32 + (size_t)v * 2 * a.n;
        o32[i] = (float)g1; o32[a.n + i] = (float)g2;
      }
    } else {
      const double q = a.dens[(size_t)v * is + i];
      if (a.out64) a.out64[(size_t)v * a.n + i] = q;
      if (a.out32) a.out32[(size_t)v * a.n + i] = (float)q;
    }
  }
}

void launch_prep_points(const PrepArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  int nb = (int)((a.n + 255) / 256);
  hipLaunchKernelGGL(prep_points_kernel, dim3(nb), dim3(256), 0, s, a);
}
void launch_prep_dens(const PrepDensArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  int nb = (int)((a.n + 255) / 256);
  hipLaunchKernelGGL(prep_dens_kernel, dim3(nb), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// target binning: a counting sort of the targets into square-ish bins of
// about 64 points, so that the targets of one wavefront are spatially close
// and take the same branches (K0/K1 small/large argument) for a given source.
// Only the targets are permuted, so each target's sum over sources keeps its
// order and results do not depend on the permutation.
// ---------------------------------------------------------------------------
__global__ void fill_int_kernel(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_double_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}
__global__ void bin_count_kernel(SortArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  int bx, by;
  if (a.lattice) {
    const double u2 = a.y[i] / a.eta, u1 = (a.x[i] - a.xi * u2) / a.d;
    bx = (int)floor((u1 + 0.5) * a.nbx);
    by = (int)floor((u2 + 0.5) * a.nby);
  } else {
    bx = (int)floor((a.x[i] - a.x0) * a.inv_w);
    by = (int)floor((a.y[i] - a.y0) * a.inv_h);
  }
  bx = min(max(bx, 0), a.nbx - 1);
  by = min(max(by, 0), a.nby - 1);
  // boustrophedon rows (lattice boxes: plain rows)
  int key = by * a.nbx + ((by & 1) && !a.lattice ? (a.nbx - 1 - bx) : bx);
  if (!PFMM_NEAR_BIN) key = 0;
  a.key[i] = key;
  // lanes with equal (key, block) add once for all of them: clustered points
  // put most of a wavefront in one bin, whose counter would otherwise take
  // up to 64 serialized atomics (a few rounds, then one add per lane)
  const int64_t slot = (int64_t)key * a.nblk + i / a.bp;
  bool done = false;
  for (int round = 0; round < 4; ++round) {
    const unsigned long long pending = __ballot(!done);
    if (!pending) break;
    const int lead = __ffsll((long long)pending) - 1;
    const int64_t lead_slot = __shfl(slot, lead);
    const bool mine = !done && slot == lead_slot;
    const unsigned long long same = __ballot(mine);
    if (mine && (threadIdx.x & 63) == lead) atomicAdd(&a.cnt[slot], __popcll(same));
    done = done || mine;
  }
  if (!done) atomicAdd(&a.cnt[slot], 1);
}
// In-place exclusive scan of cnt[bin][block] in three passes: segment sums
// (one block per SCAN_SEG entries), a scan of the segment sums (one block),
// then each segment rescanned from its offset.
__device__ __forceinline__ int block_excl_scan256(int v, int* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int u = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += u;
    __syncthreads();
  }
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}
__global__ __launch_bounds__(256) void bin_segsum_kernel(SortArgs a, int64_t n) {
  __shared__ int sh[256];
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_SEG + threadIdx.x * (SCAN_SEG / 256);
  int s = 0;
  for (int k = 0; k < SCAN_SEG / 256; ++k) s += b0 + k < n ? a.cnt[b0 + k] : 0;
  const int ex = block_excl_scan256(s, sh);
  if (threadIdx.x == 255) a.seg[blockIdx.x] = ex + s;
}
__global__ __launch_bounds__(256) void bin_segscan_kernel(SortArgs a, int n_seg) {
  __shared__ int sh[256];
  const int per = (n_seg + 255) / 256;
  const int b0 = threadIdx.x * per;
  int s = 0;
  for (int k = 0; k < per; ++k) s += b0 + k < n_seg ? a.seg[b0 + k] : 0;
  int run = block_excl_scan256(s, sh);
  for (int k = 0; k < per; ++k)
    if (b0 + k < n_seg) { const int h = a.seg[b0 + k]; a.seg[b0 + k] = run; run += h; }
}
__global__ __launch_bounds__(256) void bin_scan_kernel(SortArgs a, int64_t n) {
  __shared__ int sh[256];
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_SEG + threadIdx.x * (SCAN_SEG / 256);
  int s = 0;
  for (int k = 0; k < SCAN_SEG / 256; ++k) s += b0 + k < n ? a.cnt[b0 + k] : 0;
  int run = block_excl_scan256(s, sh) + a.seg[blockIdx.x];
  for (int k = 0; k < SCAN_SEG / 256; ++k)
    if (b0 + k < n) { const int h = a.cnt[b0 + k]; a.cnt[b0 + k] = run; run += h; }
}
// Stable placement: block b owns points [b bp, (b+1) bp) and, for every bin,
// the range that the scan gave to its points; it walks its points in index
// order, 256 at a time, and ranks equal keys by thread index, so points of a
// bin end up in ascending original index (the binned order, and with it every
// summation order downstream, does not depend on scheduling).
__global__ __launch_bounds__(256) void bin_scatter_kernel(SortArgs a) {
  __shared__ int s_key[256];
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int64_t p0 = (int64_t)blk * a.bp, p1 = min(p0 + a.bp, a.n);
  for (int64_t base = p0; base < p1; base += 256) {
    const int64_t i = base + tid;
    const int key = i < p1 ? a.key[i] : -1;
    s_key[tid] = key;
    __syncthreads();
    int rank = 0;
    bool last = true;
    for (int u = 0; u < 256; ++u) {
      const bool eq = s_key[u] == key;
      rank += (eq && u < tid) ? 1 : 0;
      last = last && !(eq && u > tid);
    }
    const int64_t slot = (int64_t)key * a.nblk + blk;
    if (key >= 0) {
      const int64_t pos = a.cnt[slot] + rank;
      a.perm[pos] = (int)i;
      a.sx[pos] = a.x[i];
      a.sy[pos] = a.y[i];
    }
    __syncthreads();
    if (key >= 0 && last) a.cnt[slot] += rank + 1;
    __syncthreads();
  }
}

void launch_sort_targets(const SortArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  const int64_t nc = (int64_t)a.nbx * a.nby * a.nblk;
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, a.cnt, (int)nc, 0);
  const int g = (int)((a.n + 255) / 256);
  hipLaunchKernelGGL(bin_count_kernel, dim3(g), dim3(256), 0, s, a);
  const int n_seg = (int)((nc + SCAN_SEG - 1) / SCAN_SEG);
  hipLaunchKernelGGL(bin_segsum_kernel, dim3(n_seg), dim3(256), 0, s, a, nc);
  hipLaunchKernelGGL(bin_segscan_kernel, dim3(1), dim3(256), 0, s, a, n_seg);
  hipLaunchKernelGGL(bin_scan_kernel, dim3(n_seg), dim3(256), 0, s, a, nc);
  hipLaunchKernelGGL(bin_scatter_kernel, dim3(a.nblk), dim3(256), 0, s, a);
}

void launch_fill_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_double_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

// ---------------------------------------------------------------------------
// near field. Each thread owns one target (taken in binned order); sources
// stream through LDS in tiles of NEAR_TILE and every tile is reused for all
// image shifts, which are applied to the targets. Block (x, y) = (target
// tile, source split); split y writes partial sums to
// part[y][dens*NOUT + c][n_trg] (FP64) in binned target order.
//
// MIXED: pair arithmetic in FP32 except the coordinate difference, which is
// taken in FP64 (full rate on CDNA4, exact for close pairs) and rounded once
// to FP32, so dx carries half an FP32 ulp of |dx| even for the closest pairs.
// Laplace/Stokes coordinates are pre-scaled by sigma = 2^k (exact) so that log2 of a typical scaled r^2
// is near zero; the shift 2k per pair is removed in FP64 at the end. The log
// terms are accumulated in FP64 pair by pair (one FP64 fma each); the other
// terms are FP32 partial sums over NEAR_FLUSH sources of one image flushed
// into FP64 accumulators (the rounding error of a blocked FP32 sum grows like
// the block length).
//
// Accumulators per density:
//   Laplace/Yukawa (3): sum q g(r), sum q h(r) dx, sum q h(r) dy
//   Stokes (8), with F = 2f, lg = log r^2, a = dx/r^2, b = dy/r^2, c2 = a F1 + b F2:
//     sum lg F1, sum lg F2, sum c2 dx, sum c2 dy, sum c2, sum c2 a dx,
//     sum c2 a dy, sum (F2 a - F1 b)
//
// r = 0: Laplace/Stokes evaluate at r^2 + R2MIN (R2MIN = 2^-100, so log2 is
// exact for the self pair, the only pair with r = 0 in a self-excluding
// evaluation); its value lg(R2MIN) * density is removed exactly in FP64 at
// the end (the gradient terms vanish because dx = dy = 0; 1/R2MIN = 2^100 is
// still finite in FP32). Yukawa (and the FP64 path)
// zero the pair with a select. Exactly coincident distinct points are a
// singularity of the sum and are not supported.
// ---------------------------------------------------------------------------
template <int K> struct NAcc { static constexpr int v = 3; };
template <> struct NAcc<PFMM_STOKES> { static constexpr int v = 8; };

struct alignas(16) SrcPt { double x, y; };

// Bounding boxes for the screened-kernel cutoff: min/max over a wavefront
// (every lane gets the result) and the squared gap between two boxes.
__device__ __forceinline__ void wave_box(double& x0, double& x1, double& y0, double& y1) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    x0 = fmin(x0, __shfl_xor(x0, o)); x1 = fmax(x1, __shfl_xor(x1, o));
    y0 = fmin(y0, __shfl_xor(y0, o)); y1 = fmax(y1, __shfl_xor(y1, o));
  }
}

__device__ __forceinline__ double box_gap2(double ax0, double ax1, double ay0, double ay1, double bx0,
                                           double bx1, double by0, double by1) {
  const double gx = fmax(0.0, fmax(bx0 - ax1, ax0 - bx1));
  const double gy = fmax(0.0, fmax(by0 - ay1, ay0 - by1));
  return gx * gx + gy * gy;
}
constexpr double BOX_EMPTY = 1.0e300;   // min/max start of an empty box

// a wavefront-uniform double moved to scalar registers
__device__ __forceinline__ double uniform_d(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int K, bool MIXED, int ND, int NA, typename real>
__device__ __forceinline__ void near_pair(real dx, real dy, const real* qv, const double* qd, real (&p)[ND][NA],
                                          double (&acc)[ND][NA], real beta, real r2min) {
  if constexpr (K == PFMM_YUKAWA || !MIXED) {
    const real r2 = dx * dx + dy * dy;
    const bool ok = r2 > (real)0;
    const real r2s = ok ? r2 : (real)1;
    if constexpr (K == PFMM_YUKAWA) {
      real k0, k1x;
      if constexpr (MIXED) bessel_k01_f32_wave(beta * __builtin_amdgcn_sqrtf(r2s), k0, k1x);
      else bessel_k01_f64(beta * sqrt(r2s), k0, k1x);
      k0 = ok ? k0 : (real)0;
      const real gx = k1x * dx, gy = k1x * dy;   // dx = dy = 0 when !ok
#pragma unroll
      for (int v = 0; v < ND; ++v) {
        const real q = qv[v];
        p[v][0] += q * k0; p[v][1] += q * gx; p[v][2] += q * gy;
      }
      return;
    } else {
      real lg = log(r2s), inv = 1.0 / r2s;
      lg = ok ? lg : (real)0;
      inv = ok ? inv : (real)0;
      if constexpr (K == PFMM_LAPLACE) {
#pragma unroll
        for (int v = 0; v < ND; ++v) {
          const real sq = qv[v] * inv;
          p[v][0] += qv[v] * lg; p[v][1] += sq * dx; p[v][2] += sq * dy;
        }
      } else {
        const real ia = inv * dx, ib = inv * dy;
#pragma unroll
        for (int v = 0; v < ND; ++v) {
          const real F1 = qv[2 * v], F2 = qv[2 * v + 1];
          const real c2 = ia * F1 + ib * F2;
          const real t = c2 * ia;
          p[v][0] += lg * F1; p[v][1] += lg * F2;
          p[v][2] += c2 * dx; p[v][3] += c2 * dy;
          p[v][4] += c2; p[v][5] += t * dx; p[v][6] += t * dy;
          p[v][7] += F2 * ia - F1 * ib;
        }
      }
      return;
    }
  } else {
    // r^2 + R2MIN: exactly R2MIN for the self pair, below half an ulp of r^2
    // for every pair with scaled r^2 >= 2^-76
    const real r2s = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, r2min));
    const real lg = __builtin_amdgcn_logf(r2s);
    const real inv = __builtin_amdgcn_rcpf(r2s);
    // log terms go straight into the FP64 accumulators (their FP32 partial
    // sums would carry the largest rounding error of the pair sum)
    const double lgd = (double)lg;
    if constexpr (K == PFMM_LAPLACE) {
#pragma unroll
      for (int v = 0; v < ND; ++v) {
        const real sq = qv[v] * inv;
        acc[v][0] = __builtin_fma(qd[v], lgd, acc[v][0]);
        p[v][1] += sq * dx; p[v][2] += sq * dy;
      }
    } else {
      const real ia = inv * dx, ib = inv * dy;
#pragma unroll
      for (int v = 0; v < ND; ++v) {
        const real F1 = qv[2 * v], F2 = qv[2 * v + 1];
        const real c2 = ia * F1 + ib * F2;
        const real t = c2 * ia;
        acc[v][0] = __builtin_fma(qd[2 * v], lgd, acc[v][0]);
        acc[v][1] = __builtin_fma(qd[2 * v + 1], lgd, acc[v][1]);
        p[v][2] += c2 * dx; p[v][3] += c2 * dy;
        p[v][4] += c2; p[v][5] += t * dx; p[v][6] += t * dy;
        p[v][7] += F2 * ia - F1 * ib;
      }
    }
  }
}

// Accumulators of one target (see above) -> potential and gradient (NOUT
// values). MIXED Laplace/Stokes: logs are log2 and gradients are in
// coordinates scaled by sigma.
template <int K, bool MIXED>
__device__ __forceinline__ void near_outputs(const double* A, double* o, double beta, double sigma) {
  const double inv4pi = 1.0 / (4 * PI), inv2pi = 1.0 / (2 * PI);
  const double lscale = MIXED ? 0.69314718055994530942 : 1.0;  // log2 -> ln
  const double gscale = (MIXED && K != PFMM_YUKAWA) ? sigma : 1.0;
  if constexpr (K == PFMM_LAPLACE) {
    o[0] = -inv4pi * lscale * A[0];
    o[1] = -inv2pi * gscale * A[1];
    o[2] = -inv2pi * gscale * A[2];
  } else if constexpr (K == PFMM_YUKAWA) {
    o[0] = inv2pi * A[0];
    o[1] = -beta * beta * inv2pi * A[1];
    o[2] = -beta * beta * inv2pi * A[2];
  } else {
    // (F = 2f): u_i = (1/4pi)[-(1/2) sum lg f_i + sum c r_i],
    // du1/dx = -du2/dy = (1/4pi) sum (c - 2 c dx^2/r^2),
    // du1/dy = (1/4pi)[W - B], du2/dx = (1/4pi)[-W - B],
    // W = sum (f2 dx - f1 dy)/r^2, B = 2 sum c dx dy/r^2
    const double h = 0.5 * inv4pi;
    o[0] = h * (-0.5 * lscale * A[0] + A[2]);
    o[1] = h * (-0.5 * lscale * A[1] + A[3]);
    o[2] = h * gscale * (A[4] - 2 * A[5]);
    o[3] = h * gscale * (A[7] - 2 * A[6]);
    o[4] = h * gscale * (-A[7] - 2 * A[6]);
    o[5] = -o[2];
  }
}

// One block's share of the near field: targets [tile*NEAR_BLOCK, +NEAR_BLOCK)
// in binned order against sources of split `split`, ND densities from dens0.
// Used by the single-cell kernel (block = (tile, split)) and by the batched
// persistent kernel (block pulls (cell, tile, split) tasks).
template <int K, bool MIXED, int ND>
__device__ __forceinline__ void near_block(const NearArgs& a, int64_t tile, int64_t split, SrcPt* s_pt,
                                           typename std::conditional<MIXED, float, double>::type* s_q,
                                           double* s_qd) {
  using real = typename std::conditional<MIXED, float, double>::type;
  constexpr int NC = (K == PFMM_STOKES) ? 2 : 1;
  constexpr int NA = NAcc<K>::v;
  // accumulators [0, NLOG) (the log terms) are summed in FP64 pair by pair
  constexpr int NLOG = (MIXED && K != PFMM_YUKAWA) ? NC : 0;
  constexpr int NO = (K == PFMM_STOKES) ? 6 : 3;
  constexpr int QN = ND * NC;

  const int tid = threadIdx.x;
  const int64_t k = tile * NEAR_BLOCK + tid;
  const int64_t kk = k < a.n_trg ? k : a.n_trg - 1;
  const double tx = a.tx[kk], ty = a.ty[kk];
  const int orig = k < a.n_trg ? a.perm[kk] : -1;
  // diag: the block's own tile of sources (binned order, same points as the targets)
  const int64_t s0 = a.diag ? (tile * NEAR_BLOCK) / a.diag_len * a.diag_len : split * a.split_len;
  const int64_t s1 = min(s0 + (a.diag ? a.diag_len : a.split_len), a.n_src);

  double acc[ND][NA];
#pragma unroll
  for (int v = 0; v < ND; ++v)
#pragma unroll
    for (int c = 0; c < NA; ++c) acc[v][c] = 0.0;

  const real beta = (real)a.beta;
  const real r2min = (real)a.r2min;
  const real qscale = (K == PFMM_STOKES) ? (real)2 : (real)1;
  // screened kernel: boxes of the block's targets and of each source tile
  // (scaled coordinates); an image that keeps the tile beyond the cutoff
  // from every target is skipped (uniform over the block)
  const bool cut = K == PFMM_YUKAWA && a.rcut2 < 1.0e300;
  __shared__ double s_box[2][NEAR_BLOCK / 64][4];
  if (cut) {
    double x0 = tx * a.geo.sigma, x1 = x0, y0 = ty * a.geo.sigma, y1 = y0;
    wave_box(x0, x1, y0, y1);
    if ((tid & 63) == 0) { s_box[0][tid >> 6][0] = x0; s_box[0][tid >> 6][1] = x1; s_box[0][tid >> 6][2] = y0; s_box[0][tid >> 6][3] = y1; }
  }
  for (int64_t base = s0; base < s1; base += NEAR_TILE) {
    const int nt = (int)min((int64_t)NEAR_TILE, s1 - base);
    __syncthreads();
    if (cut) {
      const bool ok = tid < nt;
      const int64_t j = base + (ok ? tid : 0);
      double x0 = ok ? a.sx[j] * a.geo.sigma : BOX_EMPTY, x1 = ok ? x0 : -BOX_EMPTY;
      double y0 = ok ? a.sy[j] * a.geo.sigma : BOX_EMPTY, y1 = ok ? y0 : -BOX_EMPTY;
      wave_box(x0, x1, y0, y1);
      if ((tid & 63) == 0) { s_box[1][tid >> 6][0] = x0; s_box[1][tid >> 6][1] = x1; s_box[1][tid >> 6][2] = y0; s_box[1][tid >> 6][3] = y1; }
    }
    if (tid < nt) {
      const int64_t j = base + tid;
      s_pt[tid] = SrcPt{a.sx[j] * a.geo.sigma, a.sy[j] * a.geo.sigma};   // exact scaling
      if constexpr (MIXED) {
#pragma unroll
        for (int v = 0; v < QN; ++v) {
          const size_t at = (size_t)(a.dens0 * NC + v) * a.n_src + j;
          s_q[tid * QN + v] = qscale * a.q32[at];
          // log terms take the exact FP64 densities: their sum stays neutral,
          // so no net-charge term times the log of cell-size distances appears
          if constexpr (NLOG > 0) s_qd[tid * QN + v] = (double)qscale * a.q64[at];
        }
      } else {
#pragma unroll
        for (int v = 0; v < QN; ++v) s_q[tid * QN + v] = qscale * a.q64[(size_t)(a.dens0 * NC + v) * a.n_src + j];
      }
    }
    __syncthreads();
    double tb[4] = {BOX_EMPTY, -BOX_EMPTY, BOX_EMPTY, -BOX_EMPTY}, sb[4] = {BOX_EMPTY, -BOX_EMPTY, BOX_EMPTY, -BOX_EMPTY};
    if (cut) {
#pragma unroll
      for (int w = 0; w < NEAR_BLOCK / 64; ++w) {
        tb[0] = fmin(tb[0], s_box[0][w][0]); tb[1] = fmax(tb[1], s_box[0][w][1]);
        tb[2] = fmin(tb[2], s_box[0][w][2]); tb[3] = fmax(tb[3], s_box[0][w][3]);
        sb[0] = fmin(sb[0], s_box[1][w][0]); sb[1] = fmax(sb[1], s_box[1][w][1]);
        sb[2] = fmin(sb[2], s_box[1][w][2]); sb[3] = fmax(sb[3], s_box[1][w][3]);
      }
    }
    for (int im = 0; im < a.geo.n_images; ++im) {
      if (cut) {
        const double lx = as_const(a.imx)[im] * a.geo.sigma, ly = as_const(a.imy)[im] * a.geo.sigma;
        if (box_gap2(tb[0], tb[1], tb[2], tb[3], sb[0] + lx, sb[1] + lx, sb[2] + ly, sb[3] + ly) > a.rcut2) continue;
      }
      const double txi = (tx - as_const(a.imx)[im]) * a.geo.sigma, tyi = (ty - as_const(a.imy)[im]) * a.geo.sigma;
      for (int jb = 0; jb < nt; jb += NEAR_FLUSH) {
        real p[ND][NA];
#pragma unroll
        for (int v = 0; v < ND; ++v)
#pragma unroll
          for (int c = 0; c < NA; ++c) p[v][c] = 0;
        auto body = [&](int j) {
          const SrcPt sp = s_pt[j];
          real qv[QN];
          double qd[NLOG > 0 ? QN : 1];
#pragma unroll
          for (int v = 0; v < QN; ++v) qv[v] = s_q[j * QN + v];
          if constexpr (NLOG > 0) {
#pragma unroll
            for (int v = 0; v < QN; ++v) qd[v] = s_qd[j * QN + v];
          }
          // FP64 difference (exact for close pairs), rounded once to FP32 in mixed
          const real dx = (real)(txi - sp.x), dy = (real)(tyi - sp.y);
          near_pair<K, MIXED, ND, NA, real>(dx, dy, qv, qd, p, acc, beta, r2min);
        };
        if (jb + NEAR_FLUSH <= nt) {
#pragma unroll
          for (int jj = 0; jj < NEAR_FLUSH; ++jj) body(jb + jj);
        } else {
          for (int j = jb; j < nt; ++j) body(j);
        }
#pragma unroll
        for (int v = 0; v < ND; ++v)
#pragma unroll
          for (int c = NLOG; c < NA; ++c) acc[v][c] += (double)p[v][c];
      }
    }
  }
  if (orig < 0) return;
  double* dst = a.part + (size_t)split * a.part_stride;
  if constexpr (MIXED && K != PFMM_YUKAWA) {
    // the self pair was evaluated at the clamped r^2: remove its exact value
    const double lg_self = (double)__builtin_amdgcn_logf((float)a.r2min);
    const int64_t i = a.diag ? k : (int64_t)orig;   // index of the target's own source
    const bool self_here = a.self && i >= s0 && i < s1;
    // log2 of the scaled r^2 is log2 r^2 + lg_shift for every other pair of
    // the split: remove lg_shift * (images * sum of the split's densities - own)
    const double ls = (double)a.geo.lg_shift;
#pragma unroll
    for (int v = 0; v < ND; ++v) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int comp = (a.dens0 + v) * NC + c;
        const double own = self_here ? (double)qscale * a.q64[(size_t)comp * a.n_src + i] : 0.0;
        double corr = self_here ? lg_self * own : 0.0;
        if (a.qsum) corr += ls * ((double)a.geo.n_images * (double)qscale * a.qsum[(size_t)split * a.qsum_stride + comp] - own);
        acc[v][c] -= corr;
      }
    }
  }
#pragma unroll
  for (int v = 0; v < ND; ++v) {
    double o[NO];
    near_outputs<K, MIXED>(acc[v], o, a.beta, a.geo.sigma);
#pragma unroll
    for (int c = 0; c < NO; ++c) {
      double* d = &dst[(size_t)((a.dens0 + v) * NO + c) * a.n_trg + k];
      if (a.atomic_out) unsafeAtomicAdd(d, o[c]);
      else *d = o[c];
    }
  }
}

template <int K, bool MIXED, int ND>
__global__ __launch_bounds__(NEAR_BLOCK) void near_kernel(NearArgs a) {
  using real = typename std::conditional<MIXED, float, double>::type;
  constexpr int QN = ND * ((K == PFMM_STOKES) ? 2 : 1);
  constexpr int QD = (MIXED && K != PFMM_YUKAWA) ? NEAR_TILE * QN : 1;
  __shared__ SrcPt s_pt[NEAR_TILE];
  __shared__ real s_q[NEAR_TILE * QN];
  __shared__ double s_qd[QD];
  near_block<K, MIXED, ND>(a, blockIdx.x, blockIdx.y, s_pt, s_q, s_qd);
}

// ---------------------------------------------------------------------------
// Symmetric near field (targets == sources). The free-space kernel is even,
// G(-r) = G(r), so the pair (i, j, l) seen from i and the pair (j, i, -l)
// seen from j share r^2 and every transcendental; only the gradient changes
// sign. Block (a, c): the MU_BLOCK points of binned tile a (one per thread)
// against the sources of chunk c that come after tile a, for ND density
// vectors at once. Sources pass through LDS in sub-tiles of 64; in step st
// lane t pairs its point with source (t + st) mod 64, so within a wavefront
// every lane works on a different source and the source-side sums go to a
// per-wavefront LDS row without conflicts or atomics. The 9, 15 or 21 images of
// a pair are summed in registers first (density-free moments, below), then
// multiplied by both points' densities in FP64. Each sub-tile's source-side
// sums and, at the end, each thread's own sums are converted to outputs and
// added to acc with FP64 atomics (the order of these adds is not fixed, so
// repeated runs agree to FP64 rounding). MIXED takes the coordinate difference
// in FP64 and the per-image arithmetic in FP32; the log2 of a group of images
// is that of the FP32 product of their r^2 (the plan bounds the product's
// range), as accurate as per-image logs and a log, a conversion and the FP64
// fmas per image cheaper. Yukawa: per (wavefront, source sub-tile) bounding
// boxes skip the images beyond the screened cutoff and pick the shortest
// K0/K1 fits that hold for every pair of the image. No r = 0 guard is needed
// (no point meets itself here).
// ---------------------------------------------------------------------------
constexpr int MU_SUB = 64;


// The densities of a pair (i, j) are the same under every image, so the image
// loop only accumulates density-free moments of the kernel, and the densities
// multiply them once per pair. Moments (dx, dy = r under one image,
// inv = 1/r^2, ia = dx inv, ib = dy inv):
//   Laplace: [0] sum ia, [1] sum ib
//   Yukawa:  [0] sum K0(x), [1] sum k dx, [2] sum k dy, k = K1(x)/x
//   Stokes:  [0] sum ia, [1] sum ib, [2] C = sum (ia dx - ib dy), [3] sum ia dy,
//            [4] sum ia^2 dx, [5] sum ia^2 dy; then sum ia dx = (n + C)/2 and
//            sum ib dy = (n - C)/2 (dx^2 + dy^2 = r^2, n images), and
//            sum ib^2 dx = sum ia - sum ia^2 dx (ia^2 dx + ib^2 dx = ia; its
//            absolute error stays at the scale of the outputs it enters). The
//            terms of C (cos 2 theta of each image direction) largely cancel,
//            so its FP32 partial sums stay small: an FP32 emulation of a
//            15-image cell puts the velocity error at 4.9e-7 against 7.4e-7
//            for separate sums of dx^2/r^2 and dy^2/r^2.
// The log terms take the product P of r^2 over the images instead: one log
// per pair (FP64) or per image group (mixed, log2 of an FP32 product).
template <int K, bool MIXED>
constexpr int mu_moments() {
  return K == PFMM_STOKES ? 6 : (K == PFMM_YUKAWA ? 3 : 2);
}

// ARG (mixed Yukawa) tells what every lane's x = beta r is known to be:
// 0 any (series branch included), 1 x > 2 (large-argument fits), 2 x >= KF_X
// (the shorter far fits)
template <int K, bool MIXED, typename real, int ARG = 0>
__device__ __forceinline__ void mutual_image(real dx, real dy, real* m, real& P, real beta) {
  if constexpr (K == PFMM_YUKAWA) {
    const real r2 = dx * dx + dy * dy;
    real k0, k1x;
    if constexpr (MIXED && ARG == 2) bessel_k01_f32_far(beta * __builtin_amdgcn_sqrtf(r2), k0, k1x);
    else if constexpr (MIXED && ARG == 1) bessel_k01_f32_large(beta * __builtin_amdgcn_sqrtf(r2), k0, k1x);
    else if constexpr (MIXED) bessel_k01_f32_wave(beta * __builtin_amdgcn_sqrtf(r2), k0, k1x);
    else bessel_k01_f64(beta * sqrt(r2), k0, k1x);
    m[0] += k0; m[1] += k1x * dx; m[2] += k1x * dy;
  } else {
    real inv;
    if constexpr (MIXED) {
      const real r2 = __builtin_fmaf(dx, dx, dy * dy);
      P *= r2;
      inv = __builtin_amdgcn_rcpf(r2);
    } else {
      const real r2 = dx * dx + dy * dy;
      P *= r2;
      inv = 1.0 / r2;
    }
    if constexpr (K == PFMM_LAPLACE) {
      m[0] += inv * dx; m[1] += inv * dy;
    } else {
      const real ia = inv * dx, ib = inv * dy;
      m[0] += ia; m[1] += ib;
      m[2] += ia * dx; m[2] -= ib * dy; m[3] += ia * dy;
      const real ia2 = ia * ia;
      m[4] += ia2 * dx; m[5] += ia2 * dy;
    }
  }
}

// Adds a pair's contributions to both points' FP64 sums: pA for i (source j,
// densities qj), pB for j (source i, displacement -r: odd moments change
// sign). The moments are converted to FP64 once and multiplied by the FP64
// densities; lsum is the pair's log sum (Laplace/Stokes), nimg the number of
// images summed.
template <int K, int ND, typename real>
__device__ __forceinline__ void mutual_accumulate(const real* m, double lsum, double nimg, const double* qi,
                                                  const double* qj, double (*pA)[NAcc<K>::v], double* pB,
                                                  int pb_stride) {
  constexpr int NA = NAcc<K>::v;
  constexpr int NM = K == PFMM_STOKES ? 6 : (K == PFMM_YUKAWA ? 3 : 2);
  double d[NM];
#pragma unroll
  for (int c = 0; c < NM; ++c) d[c] = (double)m[c];
#pragma unroll
  for (int v = 0; v < ND; ++v) {
    double* b = pB + (size_t)v * NA * pb_stride;
    if constexpr (K == PFMM_YUKAWA) {
      pA[v][0] = fma(qj[v], d[0], pA[v][0]); pA[v][1] = fma(qj[v], d[1], pA[v][1]);
      pA[v][2] = fma(qj[v], d[2], pA[v][2]);
      b[0] = fma(qi[v], d[0], b[0]); b[pb_stride] = fma(-qi[v], d[1], b[pb_stride]);
      b[2 * pb_stride] = fma(-qi[v], d[2], b[2 * pb_stride]);
    } else if constexpr (K == PFMM_LAPLACE) {
      pA[v][0] = fma(qj[v], lsum, pA[v][0]); pA[v][1] = fma(qj[v], d[0], pA[v][1]);
      pA[v][2] = fma(qj[v], d[1], pA[v][2]);
      b[0] = fma(qi[v], lsum, b[0]); b[pb_stride] = fma(-qi[v], d[0], b[pb_stride]);
      b[2 * pb_stride] = fma(-qi[v], d[1], b[2 * pb_stride]);
    } else {
      // (0, 1) = sum lg F; (2..7) = sum c dx, sum c dy, sum c, sum c ia dx,
      // sum c ia dy, sum (F2 ia - F1 ib), c = ia F1 + ib F2 (F = 2f as stored)
      const double a1 = qj[2 * v], a2 = qj[2 * v + 1], b1 = qi[2 * v], b2 = qi[2 * v + 1];
      const double mxx = 0.5 * (nimg + d[2]), myy = 0.5 * (nimg - d[2]);   // sum ia dx, sum ib dy
      const double t7 = d[0] - d[4];                                         // sum ib^2 dx
      pA[v][0] = fma(a1, lsum, pA[v][0]); pA[v][1] = fma(a2, lsum, pA[v][1]);
      pA[v][2] = fma(a1, mxx, fma(a2, d[3], pA[v][2]));
      pA[v][3] = fma(a1, d[3], fma(a2, myy, pA[v][3]));
      pA[v][4] = fma(a1, d[0], fma(a2, d[1], pA[v][4]));
      pA[v][5] = fma(a1, d[4], fma(a2, d[5], pA[v][5]));
      pA[v][6] = fma(a1, d[5], fma(a2, t7, pA[v][6]));
      pA[v][7] = fma(a2, d[0], fma(-a1, d[1], pA[v][7]));
      const int s = pb_stride;
      b[0] = fma(b1, lsum, b[0]); b[s] = fma(b2, lsum, b[s]);
      b[2 * s] = fma(b1, mxx, fma(b2, d[3], b[2 * s]));
      b[3 * s] = fma(b1, d[3], fma(b2, myy, b[3 * s]));
      b[4 * s] = fma(-b1, d[0], fma(-b2, d[1], b[4 * s]));
      b[5 * s] = fma(-b1, d[4], fma(-b2, d[5], b[5 * s]));
      b[6 * s] = fma(-b1, d[5], fma(-b2, t7, b[6 * s]));
      b[7 * s] = fma(b1, d[1], fma(-b2, d[0], b[7 * s]));
    }
  }
}

// LDS bytes of one mutual_block (the same for both precisions: coordinates,
// densities and the source-side sums are FP64)
template <int K, bool MIXED, int ND>
constexpr size_t mutual_lds_bytes() {
  constexpr int QN = ND * ((K == PFMM_STOKES) ? 2 : 1);
  return 8 * (2 * MU_SUB) + 8 * (size_t)QN * MU_SUB + 8 * (size_t)(MU_BLOCK / 64) * ND * NAcc<K>::v * MU_SUB;
}

// One (tile, chunk) task of the symmetric near field for densities
// [a.dens0, a.dens0 + ND); smem: mutual_lds_bytes<K, MIXED, ND>() bytes,
// 16-byte aligned. Every thread of the block must call it.
// the per-task arrays of a symmetric near-field task (the rest of the
// arguments come from MutualArgs, in kernel arguments or in a batch record
// read through the constant address space)
struct MuTask {
  const double *x, *y, *q64;
  double* acc;
  int dens0;
};

template <int K, bool MIXED, int ND, typename MA>
__device__ __forceinline__ void mutual_block(const MA& a, const MuTask& p, int64_t tile, int64_t chunk, char* smem) {
  using real = typename std::conditional<MIXED, float, double>::type;
  constexpr int NC = (K == PFMM_STOKES) ? 2 : 1;
  constexpr int QN = ND * NC;
  constexpr int NA = NAcc<K>::v;
  constexpr int NO = (K == PFMM_STOKES) ? 6 : 3;
  constexpr int NLOG = (K != PFMM_YUKAWA) ? NC : 0;   // log terms: FP64 density times the pair's log sum
  constexpr int NW = MU_BLOCK / 64;
  double* s_x = (double*)smem;
  double* s_y = s_x + MU_SUB;
  double* s_qd = s_y + MU_SUB;                         // [QN][MU_SUB]
  double* s_acc = s_qd + QN * MU_SUB;                  // [NW][ND*NA][MU_SUB]

  const int64_t a0 = tile * MU_BLOCK;
  const int64_t a_end = min(a0 + (int64_t)MU_BLOCK, a.n);
  const int64_t b0 = max(chunk * a.chunk_len, a_end);
  const int64_t b1 = min((chunk + 1) * a.chunk_len, a.n);
  if (b0 >= b1) return;                                   // uniform over the block
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t k = a0 + tid;
  const bool act = k < a.n;
  const double sg = a.sigma;
  const double qscale = (K == PFMM_STOKES) ? 2.0 : 1.0;
  const size_t qoff = (size_t)p.dens0 * NC * a.n;
  // an inactive lane sits far from every point with zero density
  const double tx = act ? p.x[k] * sg : 1.0e4, ty = act ? p.y[k] * sg : 1.0e4;
  // screened kernel: box of this wavefront's points; per source sub-tile an
  // image mask (images whose shifted sub-tile comes within the cutoff)
  const bool cut = K == PFMM_YUKAWA && a.rcut2 < 1.0e300;
  __shared__ double s_box[4];
  double wx0 = act ? tx : BOX_EMPTY, wx1 = act ? tx : -BOX_EMPTY;
  double wy0 = act ? ty : BOX_EMPTY, wy1 = act ? ty : -BOX_EMPTY;
  if (cut) {
    wave_box(wx0, wx1, wy0, wy1);
    wx0 = uniform_d(wx0); wx1 = uniform_d(wx1); wy0 = uniform_d(wy0); wy1 = uniform_d(wy1);
  }
  double qid[QN];
#pragma unroll
  for (int c = 0; c < QN; ++c) qid[c] = act ? qscale * p.q64[qoff + (size_t)c * a.n + k] : 0.0;
  const real beta = (real)a.beta;
  const cdouble* imx = as_const(a.imx);
  const cdouble* imy = as_const(a.imy);
  // mixed Laplace with the 9 images in one log group (m0 = 1, the common
  // case): the image loop is unrolled and the shifts stay in scalar registers
  // for the whole task (6 % faster; Stokes measured 2.5 % slower this way)
  const bool nine = K == PFMM_LAPLACE && MIXED && a.n_images == 9 && a.n_lg == 1;
  double i9x[9], i9y[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) { i9x[q] = nine ? imx[q] : 0.0; i9y[q] = nine ? imy[q] : 0.0; }
  double accA[ND][NA];
#pragma unroll
  for (int v = 0; v < ND; ++v)
#pragma unroll
    for (int c = 0; c < NA; ++c) accA[v][c] = 0.0;

  for (int64_t sb = b0; sb < b1; sb += MU_SUB) {
    const int nsb = (int)min((int64_t)MU_SUB, b1 - sb);
    __syncthreads();
    if (tid < MU_SUB) {
      const bool ok = tid < nsb;
      const int64_t j = sb + tid;
      s_x[tid] = ok ? p.x[j] * sg : -1.0e4;               // padding: far away, zero density
      s_y[tid] = ok ? p.y[j] * sg : -1.0e4;
#pragma unroll
      for (int c = 0; c < QN; ++c) {
        s_qd[c * MU_SUB + tid] = ok ? qscale * p.q64[qoff + (size_t)c * a.n + j] : 0.0;
      }
      if (cut) {   // MU_SUB = one wavefront
        double x0 = ok ? s_x[tid] : BOX_EMPTY, x1 = ok ? s_x[tid] : -BOX_EMPTY;
        double y0 = ok ? s_y[tid] : BOX_EMPTY, y1 = ok ? s_y[tid] : -BOX_EMPTY;
        wave_box(x0, x1, y0, y1);
        if (tid == 0) { s_box[0] = x0; s_box[1] = x1; s_box[2] = y0; s_box[3] = y1; }
      }
    }
    double* my_acc = s_acc + (size_t)wv * ND * NA * MU_SUB;
#pragma unroll
    for (int c = 0; c < ND * NA; ++c) my_acc[c * MU_SUB + lane] = 0.0;
    __syncthreads();
    // mask: images within the cutoff; smask: images where some pair may have
    // beta r <= 2 (K0/K1 series); fmask: images where every pair has
    // beta r >= KF_X (far fits); the others take the large-argument fits
    const unsigned all = (1u << a.n_images) - 1u;   // n_images <= MAX_IMAGES < 32
    unsigned mask = all, smask = all, fmask = 0u;
    if (cut) {
      const double bx0 = s_box[0], bx1 = s_box[1], by0 = s_box[2], by1 = s_box[3];
      const double small2 = 4.0001 / (a.beta * a.beta);
      const double far2 = (KF_X * KF_X * 1.0001) / (a.beta * a.beta);
      mask = 0; smask = 0;
      for (int im = 0; im < a.n_images; ++im) {
        const double g2 = box_gap2(wx0, wx1, wy0, wy1, bx0 + imx[im], bx1 + imx[im], by0 + imy[im], by1 + imy[im]);
        if (g2 <= a.rcut2) mask |= 1u << im;
        if (g2 <= small2) smask |= 1u << im;
        if (g2 >= far2) fmask |= 1u << im;
      }
      mask = __builtin_amdgcn_readfirstlane(mask);
      smask = __builtin_amdgcn_readfirstlane(smask);
      fmask = __builtin_amdgcn_readfirstlane(fmask);
    }
    for (int st = 0; st < MU_SUB && mask; ++st) {
      const int b = (lane + st) & (MU_SUB - 1);
      const double d0x = tx - s_x[b], d0y = ty - s_y[b];
      double qjd[QN];
#pragma unroll
      for (int c = 0; c < QN; ++c) qjd[c] = s_qd[c * MU_SUB + b];
      real m[mu_moments<K, MIXED>()];
#pragma unroll
      for (int c = 0; c < mu_moments<K, MIXED>(); ++c) m[c] = 0;
      double lsum = 0.0;   // Laplace/Stokes: sum of log r^2 (mixed: log2) over the images
      double cx = 0.0, cy = 0.0;   // Stokes, several log groups: FP64 sums of m[2], m[3]
      bool flushed = false;        // uniform
      if constexpr (NLOG > 0 && !MIXED) {
        // FP64: one log of the product of all images' r^2 (no range issue)
        real P = 1;
        for (int im = 0; im < a.n_images; ++im) {
          const real dx = d0x - imx[im], dy = d0y - imy[im];
          mutual_image<K, MIXED, real>(dx, dy, m, P, beta);
        }
        lsum = log(fmin(P, 1.0e300));
      } else if constexpr (NLOG > 0) {
        if (nine) {
          real P = a.lg_p0[0];
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            const real dx = (real)(d0x - i9x[q]), dy = (real)(d0y - i9y[q]);
            mutual_image<K, MIXED, real>(dx, dy, m, P, beta);
          }
          lsum = (double)__builtin_amdgcn_logf(__builtin_fminf(P, 3.40282347e38f)) - a.lg_e0[0];
        } else {
        // one log2 per image group of the product of its r^2 (FP32); with
        // several groups (rows of 5 or 7 images) the Stokes sums of order
        // one (C, sum ia dy) move to FP64 after each group, so none of them
        // runs over more than a row in FP32 (the 1/r-scale sums stay in FP32)
        int im = 0;
        for (int g = 0; g < a.n_lg; ++g) {
          real P = a.lg_p0[g];
          for (const int ie = a.lg_end[g]; im < ie; ++im) {
            const real dx = (real)(d0x - imx[im]), dy = (real)(d0y - imy[im]);
            mutual_image<K, MIXED, real>(dx, dy, m, P, beta);
          }
          // padding sources (far away, zero density) may overflow P; the clamp
          // keeps 0 * log2(P) finite (valid pairs stay below 2^122)
          lsum += (double)__builtin_amdgcn_logf(__builtin_fminf(P, 3.40282347e38f)) - a.lg_e0[g];
          if (K == PFMM_STOKES && a.n_lg > 1) {   // the O(1) sums C and sum ia dy
            cx += (double)m[2]; cy += (double)m[3];
            m[2] = 0; m[3] = 0;
            flushed = true;
          }
        }
        }
      } else {
        real P = 1;
        // images with only far arguments, then only large ones (no series
        // branch), then the rest
        if constexpr (MIXED && K == PFMM_YUKAWA) {
          // each loop visits only the set bits of its mask
          for (unsigned mm = mask & fmask; mm; mm &= mm - 1) {
            const int im = __builtin_ctz(mm);
            const real dx = (real)(d0x - imx[im]), dy = (real)(d0y - imy[im]);
            mutual_image<K, MIXED, real, 2>(dx, dy, m, P, beta);
          }
          for (unsigned mm = mask & ~smask & ~fmask; mm; mm &= mm - 1) {
            const int im = __builtin_ctz(mm);
            const real dx = (real)(d0x - imx[im]), dy = (real)(d0y - imy[im]);
            mutual_image<K, MIXED, real, 1>(dx, dy, m, P, beta);
          }
        }
        const unsigned gmask = (MIXED && K == PFMM_YUKAWA) ? (mask & smask) : mask;
        for (unsigned mm = gmask; mm; mm &= mm - 1) {
          const int im = __builtin_ctz(mm);
          const real dx = (real)(d0x - imx[im]), dy = (real)(d0y - imy[im]);
          mutual_image<K, MIXED, real>(dx, dy, m, P, beta);
        }
      }
      double md[mu_moments<K, MIXED>()];
#pragma unroll
      for (int c = 0; c < mu_moments<K, MIXED>(); ++c) md[c] = (double)m[c];
      if (K == PFMM_STOKES && flushed) { md[2] += cx; md[3] += cy; }
      mutual_accumulate<K, ND, double>(md, lsum, (double)a.n_images, qid, qjd, accA, my_acc + b, MU_SUB);
    }
    __syncthreads();
    if (tid < nsb) {
#pragma unroll
      for (int v = 0; v < ND; ++v) {
        double A[NA], o[NO];
#pragma unroll
        for (int c = 0; c < NA; ++c) {
          double t = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) t += s_acc[((size_t)w * ND * NA + v * NA + c) * MU_SUB + tid];
          A[c] = t;
        }
        near_outputs<K, MIXED>(A, o, a.beta, sg);
#pragma unroll
        for (int c = 0; c < NO; ++c)
          unsafeAtomicAdd(&p.acc[((size_t)(p.dens0 + v) * NO + c) * a.n + sb + tid], o[c]);
      }
    }
  }
  if (act) {
#pragma unroll
    for (int v = 0; v < ND; ++v) {
      double o[NO];
      near_outputs<K, MIXED>(accA[v], o, a.beta, sg);
#pragma unroll
      for (int c = 0; c < NO; ++c) unsafeAtomicAdd(&p.acc[((size_t)(p.dens0 + v) * NO + c) * a.n + k], o[c]);
    }
  }
}

template <int K, bool MIXED, int ND>
// waves per SIMD of the mixed Yukawa kernel: at most 6 (its registers allow
// no more), which lets the compiler keep the K0/K1 polynomial constants in
// registers instead of rematerializing them per image; the other kernels are
// not capped (a cap of 6 measured 3 % slower for Laplace)
__global__ __launch_bounds__(MU_BLOCK)
__attribute__((amdgpu_waves_per_eu(MIXED ? 4 : 1, (MIXED && K == PFMM_YUKAWA) ? 6 : 8)))
void near_mutual_kernel(MutualArgs a) {
  __shared__ __align__(16) char smem[mutual_lds_bytes<K, MIXED, ND>()];
  const MuTask p{a.x, a.y, a.q64, a.acc, a.dens0};
  mutual_block<K, MIXED, ND>(a, p, blockIdx.x, blockIdx.y, smem);
}

// densities per pass of the symmetric kernel (register budget)
template <int K> struct MuGroup { static constexpr int v = 4; };
template <> struct MuGroup<PFMM_STOKES> { static constexpr int v = 2; };

void launch_near_mutual(int kernel, bool mixed, const MutualArgs& a, int n_dens, hipStream_t s) {
  if (a.n <= MU_BLOCK) return;                           // one tile: the diagonal pass has it all
  const unsigned tiles = (unsigned)((a.n + MU_BLOCK - 1) / MU_BLOCK);
  const unsigned chunks = (unsigned)((a.n + a.chunk_len - 1) / a.chunk_len);
  const dim3 grid(tiles, chunks);
  auto go = [&](auto kc, auto mc) {
    constexpr int K = decltype(kc)::value;
    constexpr bool M = decltype(mc)::value;
    constexpr int G = MuGroup<K>::v;
    MutualArgs b = a;
    int v = 0;
    for (; v + G <= n_dens; v += G) { b.dens0 = v; hipLaunchKernelGGL((near_mutual_kernel<K, M, G>), grid, dim3(MU_BLOCK), 0, s, b); }
    for (; v < n_dens; ++v) { b.dens0 = v; hipLaunchKernelGGL((near_mutual_kernel<K, M, 1>), grid, dim3(MU_BLOCK), 0, s, b); }
  };
  using L = std::integral_constant<int, PFMM_LAPLACE>;
  using Y = std::integral_constant<int, PFMM_YUKAWA>;
  using S = std::integral_constant<int, PFMM_STOKES>;
  switch (kernel * 2 + (mixed ? 1 : 0)) {
    case 0: go(L{}, std::false_type{}); break;
    case 1: go(L{}, std::true_type{}); break;
    case 2: go(Y{}, std::false_type{}); break;
    case 3: go(Y{}, std::true_type{}); break;
    case 4: go(S{}, std::false_type{}); break;
    case 5: go(S{}, std::true_type{}); break;
  }
}

// ---------------------------------------------------------------------------
// Batched near field: a persistent grid; each block takes tasks from an
// atomic counter until none are left (every block reaches the exit once the
// counter passes n_tasks). A one-sided cell has (target tile, source split)
// tasks; a symmetric cell (self targets) has its diagonal tile tasks, which
// write the partial row in a first launch, and its (tile, chunk) pair tasks,
// which add to it with FP64 atomics in a second launch.
// ---------------------------------------------------------------------------
template <int K> constexpr size_t near_lds_bytes(bool mixed) {
  return sizeof(SrcPt) * NEAR_TILE + (mixed ? 4 : 8) * NEAR_TILE * 8 + (mixed ? 8 * NEAR_TILE * 8 : 8);
}

template <int K, bool MIXED>
__device__ __forceinline__ void batch_near_task(const BatchCell& r, char* ws, long long local, char* smem) {
  using real = typename std::conditional<MIXED, float, double>::type;
  SrcPt* s_pt = (SrcPt*)smem;
  real* s_q = (real*)(smem + sizeof(SrcPt) * NEAR_TILE);
  double* s_qd = (double*)(smem + sizeof(SrcPt) * NEAR_TILE + sizeof(real) * NEAR_TILE * 8);
  NearArgs a = r.args;
  int64_t tile, split;
  if (r.mutual) {
    // diagonal task: the tile's own sources in binned order
    tile = local; split = 0;
    a.sx = (const double*)(ws + r.o_tx); a.sy = (const double*)(ws + r.o_ty);
    a.q64 = (const double*)(ws + r.o_qb64); a.q32 = (const float*)(ws + r.o_qb32);
    a.diag = 1; a.diag_len = MU_BLOCK;
  } else {
    tile = local % r.n_tiles; split = local / r.n_tiles;
    a.sx = (const double*)(ws + r.o_sx); a.sy = (const double*)(ws + r.o_sy);
    a.q64 = (const double*)(ws + r.o_q64); a.q32 = (const float*)(ws + r.o_q32);
  }
  a.tx = (const double*)(ws + r.o_tx); a.ty = (const double*)(ws + r.o_ty);
  a.perm = (const int*)(ws + r.o_perm); a.part = (double*)(ws + r.o_part);
  a.qsum = r.o_qsum ? (const double*)(ws + r.o_qsum) : nullptr;
  const int nd = r.n_dens;
  int v = 0;
  for (; v + 4 <= nd; v += 4) { a.dens0 = v; near_block<K, MIXED, 4>(a, tile, split, s_pt, s_q, s_qd); }
  for (; v < nd; ++v) { a.dens0 = v; near_block<K, MIXED, 1>(a, tile, split, s_pt, s_q, s_qd); }
}

// densities [d0, d1) in groups of ND
template <int K, bool MIXED, int ND>
__device__ __forceinline__ void batch_mutual_task(const cBatchCell& r, char* ws, long long local, int d0, int d1,
                                                  char* smem) {
  const int64_t tile = local % r.n_tiles, chunk = local / r.n_tiles;
  MuTask p{(const double*)(ws + r.o_tx), (const double*)(ws + r.o_ty), (const double*)(ws + r.o_qb64),
           (double*)(ws + r.o_part), 0};
  for (int v = d0; v + ND <= d1; v += ND) { p.dens0 = v; mutual_block<K, MIXED, ND>(r.margs, p, tile, chunk, smem); }
}

// one launch per kernel type and phase (phase 0: one-sided and diagonal
// tasks, which write the partial rows; phase 1: symmetric tasks, which add)
// (phase 1 is launched once per density group size ND, for densities
// [b.dens_begin, b.dens_end))
template <int K, bool MIXED, int PHASE, int ND>
__global__ __launch_bounds__(NEAR_BLOCK) void near_batch_kernel(BatchNearArgs b) {
  static_assert(MU_BLOCK == NEAR_BLOCK, "batched tasks share one block size");
  __shared__ __align__(16) char smem[PHASE ? mutual_lds_bytes<K, MIXED, ND>() : near_lds_bytes<K>(MIXED)];
  __shared__ long long s_task;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_task = (long long)atomicAdd(b.counter, 1ULL);
    __syncthreads();
    // the task index is uniform: keep it, the cell search and the cell record
    // in scalar registers (records read through the constant address space)
    const unsigned long long tu = (unsigned long long)s_task;
    const long long t = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(tu >> 32)) << 32) |
                                    __builtin_amdgcn_readfirstlane((unsigned)tu));
    if (t >= b.n_tasks) break;
    const cBatchCell* recs = (const cBatchCell*)b.recs;
    int c = 0;
    while (c + 1 < b.n_cells && (PHASE ? recs[c + 1].task0m : recs[c + 1].task0) <= t) ++c;
    if constexpr (PHASE) batch_mutual_task<K, MIXED, ND>(recs[c], b.ws, t - recs[c].task0m, b.dens_begin, b.dens_end, smem);
    else batch_near_task<K, MIXED>(*(const BatchCell*)&recs[c], b.ws, t - recs[c].task0, smem);
  }
}

__global__ void gather_dens_kernel(const double* src, const int* perm, int64_t n, int ncomp, double* d64,
                                   float* d32) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t i = perm[k];
  for (int c = 0; c < ncomp; ++c) {
    const double q = src[(size_t)c * n + i];
    d64[(size_t)c * n + k] = q;
    if (d32) d32[(size_t)c * n + k] = (float)q;
  }
}

void launch_gather_dens(const double* src, const int* perm, int64_t n, int ncomp, double* dst64, float* dst32,
                        hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_dens_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, perm, n, ncomp,
                     dst64, dst32);
}

// per-split sums of the FP64 densities, used to remove the log2 shift.
// Two passes in a fixed order: QSUM_PARTS blocks per split sum their share
// of the split, then one thread per (split, component) adds the parts.
__global__ __launch_bounds__(256) void qsum_part_kernel(QsumArgs a) {
  __shared__ double red[256];
  const int split = blockIdx.x / QSUM_PARTS, part = blockIdx.x % QSUM_PARTS;
  const int64_t s0 = (int64_t)split * a.split_len;
  const int64_t s1 = min(s0 + a.split_len, a.n_src);
  const int64_t per = (s1 - s0 + QSUM_PARTS - 1) / QSUM_PARTS;
  const int64_t p0 = min(s0 + part * per, s1), p1 = min(p0 + per, s1);
  const int comp = blockIdx.y;
  double s = 0.0;
  for (int64_t j = p0 + threadIdx.x; j < p1; j += 256) s += a.q64[(size_t)comp * a.n_src + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.qpart[((size_t)split * QSUM_PARTS + part) * a.ncomp + comp] = red[0];
}
__global__ void qsum_final_kernel(QsumArgs a, int n_splits) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_splits * a.ncomp) return;
  const int split = t / a.ncomp, comp = t % a.ncomp;
  double s = 0.0;
  for (int p = 0; p < QSUM_PARTS; ++p) s += a.qpart[((size_t)split * QSUM_PARTS + p) * a.ncomp + comp];
  a.qsum[(size_t)split * a.ncomp + comp] = s;
}

void launch_qsum(const QsumArgs& a, int n_splits, hipStream_t s) {
  if (a.n_src <= 0 || n_splits <= 0) return;
  hipLaunchKernelGGL(qsum_part_kernel, dim3(n_splits * QSUM_PARTS, a.ncomp), dim3(256), 0, s, a);
  const int n = n_splits * a.ncomp;
  hipLaunchKernelGGL(qsum_final_kernel, dim3((n + 63) / 64), dim3(64), 0, s, a, n_splits);
}

void launch_near_batch(int kernel, bool mixed, int phase, const BatchNearArgs& b, int grid, hipStream_t s) {
  if (b.n_tasks <= 0) return;
  auto go = [&](auto kc, auto mc) {
    constexpr int K = decltype(kc)::value;
    constexpr bool M = decltype(mc)::value;
    if (phase == 0) {
      hipLaunchKernelGGL((near_batch_kernel<K, M, 0, 1>), dim3(grid), dim3(NEAR_BLOCK), 0, s, b);
    } else {
      constexpr int G = MuGroup<K>::v;
      const int full = b.n_dens / G * G;
      BatchNearArgs c = b;
      if (full > 0) {
        c.dens_begin = 0; c.dens_end = full;
        hipLaunchKernelGGL((near_batch_kernel<K, M, 1, G>), dim3(grid), dim3(NEAR_BLOCK), 0, s, c);
      }
      if (full < b.n_dens) {
        c.dens_begin = full; c.dens_end = b.n_dens; c.counter = b.counter2;
        hipLaunchKernelGGL((near_batch_kernel<K, M, 1, 1>), dim3(grid), dim3(NEAR_BLOCK), 0, s, c);
      }
    }
  };
  using L = std::integral_constant<int, PFMM_LAPLACE>;
  using Y = std::integral_constant<int, PFMM_YUKAWA>;
  using S = std::integral_constant<int, PFMM_STOKES>;
  switch (kernel * 2 + (mixed ? 1 : 0)) {
    case 0: go(L{}, std::false_type{}); break;
    case 1: go(L{}, std::true_type{}); break;
    case 2: go(Y{}, std::false_type{}); break;
    case 3: go(Y{}, std::true_type{}); break;
    case 4: go(S{}, std::false_type{}); break;
    case 5: go(S{}, std::true_type{}); break;
  }
}

void launch_near(int kernel, bool mixed, int nd, const NearArgs& a, int n_splits, hipStream_t s) {
  if (a.n_trg <= 0 || a.n_src <= 0) return;
  NearArgs b = a;
  const dim3 grid((unsigned)((a.n_trg + NEAR_BLOCK - 1) / NEAR_BLOCK), (unsigned)n_splits);
  auto go = [&](auto kc, auto mc) {
    constexpr int K = decltype(kc)::value;
    constexpr bool M = decltype(mc)::value;
    int v = 0;
    for (; v + 4 <= nd; v += 4) { b.dens0 = v; hipLaunchKernelGGL((near_kernel<K, M, 4>), grid, dim3(NEAR_BLOCK), 0, s, b); }
    for (; v < nd; ++v) { b.dens0 = v; hipLaunchKernelGGL((near_kernel<K, M, 1>), grid, dim3(NEAR_BLOCK), 0, s, b); }
  };
  using L = std::integral_constant<int, PFMM_LAPLACE>;
  using Y = std::integral_constant<int, PFMM_YUKAWA>;
  using S = std::integral_constant<int, PFMM_STOKES>;
  using T = std::true_type;
  using F = std::false_type;
  switch (kernel * 2 + (mixed ? 1 : 0)) {
    case 0: go(L{}, F{}); break;
    case 1: go(L{}, T{}); break;
    case 2: go(Y{}, F{}); break;
    case 3: go(Y{}, T{}); break;
    case 4: go(S{}, F{}); break;
    case 5: go(S{}, T{}); break;
  }
}

// ---------------------------------------------------------------------------
// far R: one thread per plane wave (south/north mode or west/east node; the
// last wave index holds the y-moments of the Laplace/Stokes m = 0 term),
// summing over one chunk of sources staged in LDS. FP64 throughout.
//   south/north (Thm. south_thm, south_thm_lap, south_thm_s):
//     c^S = sum q e^{a y - i alpha x},  c^N = sum q e^{-a y - i alpha x}
//     Stokes also e^S = sum y f e^{a y - i alpha x} (and north alike)
//   west/east (Thm. west_thm, west_thm_lap, west_thm_s; Appendix A), with
//   (x, y) the source in the west/east frame:
//     c^W = sum q e^{kappa x - i lambda y}, c^E = sum q e^{-kappa x - i lambda y}
//     Laplace/Stokes use e^{...} - 1 (exact for neutral densities, and free of
//     the O(1) cancellation at small lambda); Stokes also e^W = sum x f e^{...}
//     (force components stay canonical; far_D rotates them)
// ---------------------------------------------------------------------------
constexpr int FAR_R_TILE = 512;

struct cplx { double r, i; };
typedef const __attribute__((address_space(4))) cplx ccplx;
// a complex value from a table read through the constant address space
__device__ __forceinline__ cplx cld(const ccplx* p) { return {p->r, p->i}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.r * s, a.i * s}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.r, -a.i}; }
__device__ __forceinline__ cplx cmuli(cplx a) { return {-a.i, a.r}; }  // i*a
// e^{a + i b} - 1 and e^{-a + i b} - 1 without cancellation for small |a|,
// |b|, sharing their transcendentals (e^{-a} - 1 = -(e^a - 1) e^{-a})
__device__ __forceinline__ void cexpm1_pair(double a, double b, cplx& plus, cplx& minus) {
  double sh, ch;
  sincos_pw(0.5 * b, sh, ch);
  const double s = 2.0 * sh * ch, cm1 = -2.0 * sh * sh;   // sin b, cos b - 1
  const double c = 1.0 + cm1;
  const double em = expm1_pw(a), e = em + 1.0, ie = recip_pw(e);
  plus = {em * c + cm1, e * s};
  minus = {-em * ie * c + cm1, ie * s};
}

// Block (x, y, z) = (mode group, source chunk, density group): thread
// (slice, lane) owns mode/node x * lanes + lane and every slices-th source of
// each LDS tile; each plane-wave factor serves the DG densities of the group;
// the slices' partial sums are added in a fixed order at the end.
template <int K, int DG>
__global__ __launch_bounds__(FAR_R_BLOCK) void far_R_kernel(FarRArgs a) {
  constexpr int NC = (K == PFMM_STOKES) ? 2 : 1;
  constexpr int NCW = (K == PFMM_STOKES) ? 8 : 2;
  constexpr int TILE_D = (2 + DG * NC) * FAR_R_TILE, RED_D = FAR_R_BLOCK * NCW * 2;
  __shared__ double smem[TILE_D > RED_D ? TILE_D : RED_D];
  double* s_x = smem;
  double* s_y = smem + FAR_R_TILE;
  double* s_qb = smem + 2 * FAR_R_TILE;   // [DG][NC][FAR_R_TILE]
  const int v0 = blockIdx.z * DG;
  const int nd = min(DG, a.n_dens - v0);
  const int64_t j0 = (int64_t)blockIdx.y * a.chunk_len;
  const int64_t j1 = min(j0 + a.chunk_len, a.n_src);
  const int lanes = a.lanes, n_slices = FAR_R_BLOCK / lanes;
  const int lane = threadIdx.x % lanes, slice = threadIdx.x / lanes;
  // with skip_sn the lanes start at the first west/east node (the NUFFT path
  // supplies the south/north coefficients and far_D ignores those slots here)
  const int w = (a.skip_sn ? a.n_sn : 0) + blockIdx.x * lanes + lane;
  const int n_w = a.n_sn + a.n_ew;
  const bool in_sn = w < a.n_sn;
  const bool is_sn = in_sn && !a.skip_sn, is_ew = !in_sn && w < n_w, is_mom = w == n_w;
  double par0 = 0, par1 = 0;
  if (is_sn || is_ew) { par0 = a.tab[is_sn ? w * SN_REC : a.n_sn * SN_REC + (w - a.n_sn) * EW_REC];
                        par1 = a.tab[(is_sn ? w * SN_REC : a.n_sn * SN_REC + (w - a.n_sn) * EW_REC) + 1]; }
  cplx acc[DG][NCW];
#pragma unroll
  for (int d = 0; d < DG; ++d)
#pragma unroll
    for (int c = 0; c < NCW; ++c) acc[d][c] = {0, 0};
  const double* dens = a.dens + (size_t)v0 * NC * a.n_src;
  for (int64_t base = j0; base < j1; base += FAR_R_TILE) {
    const int nt = (int)min((int64_t)FAR_R_TILE, j1 - base);
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += FAR_R_BLOCK) {
      s_x[t] = a.sx[base + t]; s_y[t] = a.sy[base + t];
#pragma unroll
      for (int d = 0; d < DG; ++d)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          s_qb[(d * NC + c) * FAR_R_TILE + t] = d < nd ? dens[(size_t)(d * NC + c) * a.n_src + base + t] : 0.0;
    }
    __syncthreads();
    if (is_sn) {
      const double al = par0, aa = par1;
      for (int t = slice; t < nt; t += n_slices) {
        const double x = s_x[t], y = s_y[t];
        double sn, cs;
        sincos_pw(al * x, sn, cs);
        const double ep = exp_pw(aa * y), em = recip_pw(ep);
        const cplx ph = {cs, -sn};
        const cplx ps = cscale(ph, ep), pn = cscale(ph, em);
#pragma unroll
        for (int d = 0; d < DG; ++d) {
          if constexpr (K == PFMM_STOKES) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const double f = s_qb[(d * NC + c) * FAR_R_TILE + t];
              acc[d][c] = cadd(acc[d][c], cscale(ps, f));
              acc[d][2 + c] = cadd(acc[d][2 + c], cscale(ps, f * y));
              acc[d][4 + c] = cadd(acc[d][4 + c], cscale(pn, f));
              acc[d][6 + c] = cadd(acc[d][6 + c], cscale(pn, f * y));
            }
          } else {
            const double q = s_qb[d * FAR_R_TILE + t];
            acc[d][0] = cadd(acc[d][0], cscale(ps, q));
            acc[d][1] = cadd(acc[d][1], cscale(pn, q));
          }
        }
      }
    } else if (is_ew) {
      const double lam = par0, kap = par1;
      for (int t = slice; t < nt; t += n_slices) {
        // west/east frame coordinates
        const double x = a.ew_c * s_x[t] - a.ew_s * s_y[t], y = a.ew_s * s_x[t] + a.ew_c * s_y[t];
        if constexpr (K == PFMM_YUKAWA) {
          double sn, cs;
          sincos_pw(lam * y, sn, cs);
          const double ep = exp_pw(kap * x), em = recip_pw(ep);
          const cplx pw = {ep * cs, -ep * sn}, pe = {em * cs, -em * sn};
#pragma unroll
          for (int d = 0; d < DG; ++d) {
            const double q = s_qb[d * FAR_R_TILE + t];
            acc[d][0] = cadd(acc[d][0], cscale(pw, q));
            acc[d][1] = cadd(acc[d][1], cscale(pe, q));
          }
        } else {
          cplx wm, emm;                                 // e^{lam(x - i y)} - 1, e^{-lam(x + i y)} - 1
          cexpm1_pair(lam * x, -lam * y, wm, emm);
          if constexpr (K == PFMM_LAPLACE) {
#pragma unroll
            for (int d = 0; d < DG; ++d) {
              const double q = s_qb[d * FAR_R_TILE + t];
              acc[d][0] = cadd(acc[d][0], cscale(wm, q));
              acc[d][1] = cadd(acc[d][1], cscale(emm, q));
            }
          } else {
            const cplx wf = {wm.r + 1.0, wm.i}, ef = {emm.r + 1.0, emm.i};
#pragma unroll
            for (int d = 0; d < DG; ++d)
#pragma unroll
              for (int c = 0; c < 2; ++c) {
                const double f = s_qb[(d * NC + c) * FAR_R_TILE + t];
                acc[d][c] = cadd(acc[d][c], cscale(wm, f));
                acc[d][2 + c] = cadd(acc[d][2 + c], cscale(wf, f * x));
                acc[d][4 + c] = cadd(acc[d][4 + c], cscale(emm, f));
                acc[d][6 + c] = cadd(acc[d][6 + c], cscale(ef, f * x));
              }
          }
        }
      }
    } else if (is_mom && K != PFMM_YUKAWA) {
      for (int t = slice; t < nt; t += n_slices) {
        const double y = s_y[t];
#pragma unroll
        for (int d = 0; d < DG; ++d) {
          const double q = s_qb[d * NC * FAR_R_TILE + t];
          acc[d][0].r += q * y;
          acc[d][0].i += q * y * y;
        }
      }
    }
  }
  // per density: slice partials -> LDS (reusing the tile), summed by slice 0
  // in a fixed order
  double* red = smem;   // [slice][lane][NCW] complex
#pragma unroll
  for (int d = 0; d < DG; ++d) {
    if (d >= nd) break;   // uniform over the block
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NCW; ++c) {
      red[((size_t)(slice * lanes + lane) * NCW + c) * 2] = acc[d][c].r;
      red[((size_t)(slice * lanes + lane) * NCW + c) * 2 + 1] = acc[d][c].i;
    }
    __syncthreads();
    if (slice == 0) {
      cplx tot[NCW];
#pragma unroll
      for (int c = 0; c < NCW; ++c) {
        double sr = 0, si = 0;
        for (int sl = 0; sl < n_slices; ++sl) {
          sr += red[((size_t)(sl * lanes + lane) * NCW + c) * 2];
          si += red[((size_t)(sl * lanes + lane) * NCW + c) * 2 + 1];
        }
        tot[c] = {sr, si};
      }
      double* out = a.part + ((size_t)blockIdx.y * a.n_dens + v0 + d) * a.n_coef * 2;
      if (in_sn || is_ew) {
#pragma unroll
        for (int c = 0; c < NCW; ++c) { out[2 * (w * NCW + c)] = tot[c].r; out[2 * (w * NCW + c) + 1] = tot[c].i; }
      } else if (is_mom) {
        out[2 * (n_w * NCW)] = tot[0].r;
        out[2 * (n_w * NCW) + 1] = tot[0].i;
      }
    }
  }
}

// chunk partials -> chunk 0, one block per complex entry (fixed order)
__global__ __launch_bounds__(256) void far_sum_kernel(double* part, int n_chunks, int64_t n_cplx) {
  __shared__ double red[2][256];
  const int64_t e = blockIdx.x;
  double sr = 0, si = 0;
  for (int ch = threadIdx.x; ch < n_chunks; ch += 256) {
    const double* q = part + ((size_t)ch * n_cplx + e) * 2;
    sr += q[0]; si += q[1];
  }
  red[0][threadIdx.x] = sr; red[1][threadIdx.x] = si;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { part[e * 2] = red[0][0]; part[e * 2 + 1] = red[1][0]; }
}

void launch_far_sum(double* part, int n_chunks, int64_t n_cplx, hipStream_t s) {
  if (n_cplx <= 0 || n_chunks <= 1) return;
  hipLaunchKernelGGL(far_sum_kernel, dim3((unsigned)n_cplx), dim3(256), 0, s, part, n_chunks, n_cplx);
}

void launch_far_R(const FarRArgs& a, int n_chunks, hipStream_t s) {
  const int n_w = a.n_sn + a.n_ew + 1 - (a.skip_sn ? a.n_sn : 0);
  const int dg = far_r_dgroup(a.kernel, a.n_dens);
  dim3 grid((unsigned)((n_w + a.lanes - 1) / a.lanes), (unsigned)n_chunks, (unsigned)((a.n_dens + dg - 1) / dg));
  switch (a.kernel * 8 + dg) {
    case PFMM_LAPLACE * 8 + 1: hipLaunchKernelGGL((far_R_kernel<PFMM_LAPLACE, 1>), grid, dim3(FAR_R_BLOCK), 0, s, a); break;
    case PFMM_LAPLACE * 8 + 4: hipLaunchKernelGGL((far_R_kernel<PFMM_LAPLACE, 4>), grid, dim3(FAR_R_BLOCK), 0, s, a); break;
    case PFMM_YUKAWA * 8 + 1: hipLaunchKernelGGL((far_R_kernel<PFMM_YUKAWA, 1>), grid, dim3(FAR_R_BLOCK), 0, s, a); break;
    case PFMM_YUKAWA * 8 + 4: hipLaunchKernelGGL((far_R_kernel<PFMM_YUKAWA, 4>), grid, dim3(FAR_R_BLOCK), 0, s, a); break;
    case PFMM_STOKES * 8 + 1: hipLaunchKernelGGL((far_R_kernel<PFMM_STOKES, 1>), grid, dim3(FAR_R_BLOCK), 0, s, a); break;
    default: hipLaunchKernelGGL((far_R_kernel<PFMM_STOKES, 2>), grid, dim3(FAR_R_BLOCK), 0, s, a); break;
  }
}

// ---------------------------------------------------------------------------
// far D: sum the chunk partials (fixed order) and apply the diagonal factors.
//   scalar south/north: w^S = D c^S, w^N = conj(D) c^N  (D = fac T/(2 d a))
//   scalar west/east:   tW = DW c^W, tE = DE c^E -> (tW + tE, tE - tW)
//   Stokes south/north (Thm. south_thm_s, re-derived; M_S = [[1,i],[i,-1]],
//     M_N = [[-1,i],[i,1]], D = fac T/(4d)):
//     A_S = D (c^S/a - eta tau M_S c^S + M_S e^S), B_S = D M_S c^S
//     A_N = conj(D)(c^N/a + eta conj(tau) M_N c^N + M_N e^N), B_N = conj(D) M_N c^N
//   Stokes west/east (Thm. west_thm_s, re-derived; in the west/east frame,
//     force components rotated into it first and the results rotated back;
//     M_W = [[-1,i],[i,1]], M_E = [[1,i],[i,-1]], pre = w R/(4 pi)):
//     A_W = pre((B/lam) c^W - dP B M_W c^W + B M_W e^W + xi' B' M_W c^W), X_W = pre B M_W c^W
//     A_E = conj(pre)((conj B/lam) c^E + conj(dP) conj(B) M_E c^E + conj(B) M_E e^E
//               - xi' conj(B') M_E c^E),  X_E = conj(pre) conj(B) M_E c^E
//     stored as (A_W + A_E, A_E - A_W, X_W + X_E, X_E - X_W)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mat_s(cplx c1, cplx c2, cplx& o1, cplx& o2) {  // [[1,i],[i,-1]]
  o1 = cadd(c1, cmuli(c2));
  o2 = csub(cmuli(c1), c2);
}
__device__ __forceinline__ void mat_n(cplx c1, cplx c2, cplx& o1, cplx& o2) {  // [[-1,i],[i,1]]
  o1 = cadd(cscale(c1, -1.0), cmuli(c2));
  o2 = cadd(cmuli(c1), c2);
}

__global__ void far_D_kernel(FarDArgs a) {
  const int n_w = a.n_sn + a.n_ew;
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (w > n_w) return;
  const int ncw = a.ncw;
  const int nsum = (w == n_w) ? 1 : ncw;
  const int c0 = w * ncw;
  cplx c[8];
  for (int k = 0; k < nsum; ++k) {
    double sr = 0, si = 0;
    const bool sn_extra = a.extra && w < a.n_sn;     // south/north from the NUFFT path only
    for (int ch = 0; ch < (sn_extra ? 0 : a.n_chunks); ++ch) {
      const double* p = a.part + (((size_t)ch * a.n_dens + v) * a.n_coef + c0 + k) * 2;
      sr += p[0]; si += p[1];
    }
    if (sn_extra) {
      const double* e = a.extra + (((size_t)v * a.n_sn + w) * ncw + k) * 2;
      sr += e[0]; si += e[1];
    }
    c[k] = {sr, si};
  }
  double* out = a.w + ((size_t)v * a.n_coef + c0) * 2;
  cplx o[8];
  if (w == n_w) {
    out[0] = c[0].r; out[1] = c[0].i;
    return;
  }
  if (w < a.n_sn) {
    const double* r = a.tab + (size_t)w * SN_REC;
    const double aa = r[1];
    const cplx D = {r[2], r[3]}, tau = {r[4], r[5]};
    if (a.kernel != PFMM_STOKES) {
      o[0] = cmul(D, c[0]);
      o[1] = cmul(cconj(D), c[1]);
    } else {
      cplx m1, m2, e1, e2;
      mat_s(c[0], c[1], m1, m2);          // M_S c^S
      mat_s(c[2], c[3], e1, e2);          // M_S e^S
      const cplx et = cscale(tau, a.eta);
      o[0] = cmul(D, cadd(csub(cscale(c[0], 1.0 / aa), cmul(et, m1)), e1));
      o[1] = cmul(D, cadd(csub(cscale(c[1], 1.0 / aa), cmul(et, m2)), e2));
      o[2] = cmul(D, m1);
      o[3] = cmul(D, m2);
      mat_n(c[4], c[5], m1, m2);          // M_N c^N
      mat_n(c[6], c[7], e1, e2);          // M_N e^N
      const cplx Dn = cconj(D), etn = cscale(cconj(tau), a.eta);
      o[4] = cmul(Dn, cadd(cadd(cscale(c[4], 1.0 / aa), cmul(etn, m1)), e1));
      o[5] = cmul(Dn, cadd(cadd(cscale(c[5], 1.0 / aa), cmul(etn, m2)), e2));
      o[6] = cmul(Dn, m1);
      o[7] = cmul(Dn, m2);
    }
  } else {
    const double* r = a.tab + (size_t)a.n_sn * SN_REC + (size_t)(w - a.n_sn) * EW_REC;
    if (a.kernel != PFMM_STOKES) {
      const cplx DW = {r[2], r[3]}, DE = {r[4], r[5]};
      const cplx tW = cmul(DW, c[0]), tE = cmul(DE, c[1]);
      o[0] = cadd(tW, tE);
      o[1] = csub(tE, tW);
    } else {
      const double lam = r[0];
      const cplx pre = {r[2], r[3]}, B = {r[4], r[5]}, Bp = {r[6], r[7]}, dP = {r[8], r[9]};
      const cplx Bc = cconj(B), Bpc = cconj(Bp), prec = cconj(pre), dPc = cconj(dP);
      // force components of the coefficients into the west/east frame
      const double ec = a.ew_c, es = a.ew_s;
      cplx cc[8];
      for (int q = 0; q < 8; q += 2) {
        cc[q] = csub(cscale(c[q], ec), cscale(c[q + 1], es));
        cc[q + 1] = cadd(cscale(c[q], es), cscale(c[q + 1], ec));
      }
      cplx mw1, mw2, ew1, ew2, me1, me2, ee1, ee2;
      mat_n(cc[0], cc[1], mw1, mw2);      // M_W c^W  (M_W = [[-1,i],[i,1]])
      mat_n(cc[2], cc[3], ew1, ew2);      // M_W e^W
      mat_s(cc[4], cc[5], me1, me2);      // M_E c^E  (M_E = [[1,i],[i,-1]])
      mat_s(cc[6], cc[7], ee1, ee2);      // M_E e^E
      const cplx mw[2] = {mw1, mw2}, ew[2] = {ew1, ew2}, me[2] = {me1, me2}, ee[2] = {ee1, ee2};
      for (int k = 0; k < 2; ++k) {
        cplx AW = cmul(B, cscale(cc[k], 1.0 / lam));
        AW = csub(AW, cmul(dP, cmul(B, mw[k])));
        AW = cadd(AW, cmul(B, ew[k]));
        AW = cadd(AW, cscale(cmul(Bp, mw[k]), a.xi));
        AW = cmul(AW, pre);
        const cplx XW = cmul(cmul(B, mw[k]), pre);
        cplx AE = cmul(Bc, cscale(cc[4 + k], 1.0 / lam));
        AE = cadd(AE, cmul(dPc, cmul(Bc, me[k])));
        AE = cadd(AE, cmul(Bc, ee[k]));
        AE = csub(AE, cscale(cmul(Bpc, me[k]), a.xi));
        AE = cmul(AE, prec);
        const cplx XE = cmul(cmul(Bc, me[k]), prec);
        o[k] = cadd(AW, AE);
        o[2 + k] = csub(AE, AW);
        o[4 + k] = cadd(XW, XE);
        o[6 + k] = csub(XE, XW);
      }
      // velocity components back to the canonical frame
      for (int q = 0; q < 8; q += 2) {
        const cplx v1 = o[q], v2 = o[q + 1];
        o[q] = cadd(cscale(v1, ec), cscale(v2, es));
        o[q + 1] = csub(cscale(v2, ec), cscale(v1, es));
      }
    }
  }
  for (int k = 0; k < ncw; ++k) { out[2 * k] = o[k].r; out[2 * k + 1] = o[k].i; }
}

void launch_far_D(const FarDArgs& a, hipStream_t s) {
  int n = a.n_sn + a.n_ew + 1;
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)a.n_dens);
  hipLaunchKernelGGL(far_D_kernel, grid, dim3(64), 0, s, a);
}

// ---------------------------------------------------------------------------
// far L (+ combine): per target (in binned order, like the near partials),
// sum the plane waves, add the near partials of every split in fixed order,
// rotate back to the user frame and write at the target's original index.
//   scalar south/north: u += Re[(w^S e^{-a y} + w^N e^{a y}) e^{i alpha x}]
//   scalar west/east:   u += Re[e^{i lam y}(cosh(kap x) S + sinh(kap x) D)]
//                       with (x, y) the target in the west/east frame
//   Laplace m = 0 (Thm. south_thm_lap and corollary, plus the zero-mean
//   constant):          u += -y P_y/(d eta) + sum q y^2/(2 d eta)
//   Stokes: the same waves times (A - y B) (south/north) or (A - x X)
//   (west/east); m = 0 acts on u1 only, like Laplace with q = f1.
// ---------------------------------------------------------------------------
// e^{i phase} and e^{+-expo} of one plane wave, in FP64 in both precisions:
// the far field is a sum of such waves that cancels much of the near part,
// so FP32 factors (about 1e-7 each) would show as a 1e-6 relative error of a
// Laplace or Stokes potential, at about 1 % of an evaluation's time
__device__ __forceinline__ void wave_factors(double phase, double expo, double& sn, double& cs, double& ep, double& em) {
  sincos_pw(phase, sn, cs);
  ep = exp_pw(expo);
  em = recip_pw(ep);
}

template <int K, int DG>
__global__ __launch_bounds__(256) void far_L_kernel(FarLArgs a) {
  constexpr int NO = (K == PFMM_STOKES) ? 6 : 3;
  constexpr int NCW = (K == PFMM_STOKES) ? 8 : 2;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // binned position
  if (k >= a.n_trg) return;
  const int64_t i = a.perm[k];                                          // original index
  const double x = a.tx[k], y = a.ty[k];
  const cdouble* sn_tab = as_const(a.tab);
  const cdouble* ew_tab = sn_tab + (size_t)a.n_sn * SN_REC;
  // densities in groups of DG: every plane-wave factor serves the group
  for (int v0 = 0; v0 < a.n_dens; v0 += DG) {
    const int nd = min(DG, a.n_dens - v0);
    ccplx* w0 = (ccplx*)as_const(a.w) + (size_t)v0 * a.n_coef;
    double o[DG][NO];
#pragma unroll
    for (int d = 0; d < DG; ++d)
#pragma unroll
      for (int c = 0; c < NO; ++c) o[d][c] = 0;
    if (!a.nufft) {
      for (int m = 0; m < a.n_sn; ++m) {
        const double al = sn_tab[m * SN_REC], aa = sn_tab[m * SN_REC + 1];
        double sn, cs, ep, em;
        wave_factors(al * x, aa * y, sn, cs, ep, em);
        const cplx ph = {cs, sn};
#pragma unroll
        for (int d = 0; d < DG; ++d) {
          if (d >= nd) break;
          ccplx* ww = w0 + (size_t)d * a.n_coef + m * NCW;
          if constexpr (K == PFMM_STOKES) {
            const cplx LS = cscale(ph, em), LN = cscale(ph, ep);
            for (int q = 0; q < 2; ++q) {
              const cplx w0q = cld(ww + q), w2q = cld(ww + 2 + q), w4q = cld(ww + 4 + q), w6q = cld(ww + 6 + q);
              const cplx uS = cmul(LS, csub(w0q, cscale(w2q, y)));
              const cplx uN = cmul(LN, csub(w4q, cscale(w6q, y)));
              const cplx u = cadd(uS, uN);
              o[d][q] += u.r;
              o[d][2 + 2 * q] += -al * u.i;                       // Re(i alpha u)
              const cplx dy = csub(cscale(uN, aa), cscale(uS, aa));
              o[d][3 + 2 * q] += dy.r - cmul(LS, w2q).r - cmul(LN, w6q).r;
            }
          } else {
            const cplx w0v = cld(ww + 0), w1v = cld(ww + 1);
            const cplx sv = cscale(w0v, em), nv = cscale(w1v, ep);
            const cplx u = cmul(cadd(sv, nv), ph);
            o[d][0] += u.r;
            o[d][1] += -al * u.i;
            o[d][2] += aa * cmul(csub(nv, sv), ph).r;
          }
        }
      }
    }
    // west/east waves in the west/east frame: the target's coordinates there,
    // and gradients taken along that frame's axes (rotated back below)
    const double xe = a.ew_c * x - a.ew_s * y, ye = a.ew_s * x + a.ew_c * y;
    double ge[DG][K == PFMM_STOKES ? 4 : 2];
#pragma unroll
    for (int d = 0; d < DG; ++d)
#pragma unroll
      for (int c = 0; c < (K == PFMM_STOKES ? 4 : 2); ++c) ge[d][c] = 0;
    for (int kk = 0; kk < a.n_ew; ++kk) {
      const double lam = ew_tab[kk * EW_REC], kap = ew_tab[kk * EW_REC + 1];
      double sn, cs, ep, em;
      wave_factors(lam * ye, kap * xe, sn, cs, ep, em);
      const double ch = 0.5 * (ep + em), sh = 0.5 * (ep - em);
      const cplx ph = {cs, sn};
#pragma unroll
      for (int d = 0; d < DG; ++d) {
        if (d >= nd) break;
        ccplx* ww = w0 + (size_t)d * a.n_coef + (a.n_sn + kk) * NCW;
        if constexpr (K == PFMM_STOKES) {
          for (int c = 0; c < 2; ++c) {
            const cplx wc = cld(ww + c), w2c = cld(ww + 2 + c), w4c = cld(ww + 4 + c), w6c = cld(ww + 6 + c);
            const cplx SA = csub(wc, cscale(w4c, xe));    // SigmaA - x SigmaX
            const cplx DA = csub(w2c, cscale(w6c, xe));   // DeltaA - x DeltaX
            const cplx U = cadd(cscale(SA, ch), cscale(DA, sh));
            const cplx u = cmul(ph, U);
            o[d][c] += u.r;
            cplx G = cadd(cscale(SA, kap * sh), cscale(DA, kap * ch));
            G = csub(G, cadd(cscale(w4c, ch), cscale(w6c, sh)));
            ge[d][2 * c] += cmul(ph, G).r;
            ge[d][2 * c + 1] += -lam * u.i;
          }
        } else {
          const cplx w0v = cld(ww + 0), w1v = cld(ww + 1);
          const cplx U = cadd(cscale(w0v, ch), cscale(w1v, sh));
          const cplx u = cmul(ph, U);
          o[d][0] += u.r;
          ge[d][0] += kap * cmul(ph, cadd(cscale(w0v, sh), cscale(w1v, ch))).r;
          ge[d][1] += -lam * u.i;
        }
      }
    }
    // d/dx = c d/dx' + s d/dy', d/dy = -s d/dx' + c d/dy'
#pragma unroll
    for (int d = 0; d < DG; ++d) {
      if constexpr (K == PFMM_STOKES) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          o[d][2 + 2 * c] += a.ew_c * ge[d][2 * c] + a.ew_s * ge[d][2 * c + 1];
          o[d][3 + 2 * c] += -a.ew_s * ge[d][2 * c] + a.ew_c * ge[d][2 * c + 1];
        }
      } else {
        o[d][1] += a.ew_c * ge[d][0] + a.ew_s * ge[d][1];
        o[d][2] += -a.ew_s * ge[d][0] + a.ew_c * ge[d][1];
      }
    }
#pragma unroll
    for (int d = 0; d < DG; ++d) {
      if (d >= nd) break;
      const int v = v0 + d;
      if (K != PFMM_YUKAWA && a.m0term) {
        const cplx mom = cld(w0 + (size_t)d * a.n_coef + (a.n_sn + a.n_ew) * NCW);
        const double de = a.d * a.eta;
        o[d][0] += -y * mom.r / de + mom.i / (2 * de);
        o[d][K == PFMM_STOKES ? 3 : 2] += -mom.r / de;
      }
      if (a.nufft) {
#pragma unroll
        for (int c = 0; c < NO; ++c) o[d][c] += a.nu_val[((size_t)v * NO + c) * a.n_trg + k];
      }
      for (int s = 0; s < a.n_splits; ++s) {
        const double* p = a.near_part + (size_t)s * a.part_stride;
#pragma unroll
        for (int c = 0; c < NO; ++c) o[d][c] += p[((size_t)v * NO + c) * a.n_trg + k];
      }
      // back to the user frame: user = R^T canonical
      const double rc = a.rc, rs = a.rs;
      if constexpr (K == PFMM_STOKES) {
        const double u1 = rc * o[d][0] + rs * o[d][1], u2 = -rs * o[d][0] + rc * o[d][1];
        // J_user = R^T J R,  J = [[o2, o3], [o4, o5]]
        const double j11 = o[d][2], j12 = o[d][3], j21 = o[d][4], j22 = o[d][5];
        const double t11 = rc * j11 + rs * j21, t12 = rc * j12 + rs * j22;   // R^T J
        const double t21 = -rs * j11 + rc * j21, t22 = -rs * j12 + rc * j22;
        const double g11 = t11 * rc + t12 * rs, g12 = -t11 * rs + t12 * rc; // (R^T J) R
        const double g21 = t21 * rc + t22 * rs, g22 = -t21 * rs + t22 * rc;
        const int64_t os = a.out_stride;
        if (a.out_pot) {
          a.out_pot[((size_t)v * 2) * os + i] = u1;
          a.out_pot[((size_t)v * 2 + 1) * os + i] = u2;
        }
        if (a.out_grad) {
          double* g = a.out_grad + (size_t)v * 4 * os;
          g[i] = g11; g[os + i] = g12; g[2 * os + i] = g21; g[3 * os + i] = g22;
        }
      } else {
        const int64_t os = a.out_stride;
        if (a.out_pot) a.out_pot[(size_t)v * os + i] = o[d][0];
        if (a.out_grad) {
          a.out_grad[((size_t)v * 2) * os + i] = rc * o[d][1] + rs * o[d][2];
          a.out_grad[((size_t)v * 2 + 1) * os + i] = -rs * o[d][1] + rc * o[d][2];
        }
      }
    }
  }
}

void launch_far_L(const FarLArgs& a, hipStream_t s) {
  if (a.n_trg <= 0) return;
  dim3 grid((unsigned)((a.n_trg + 255) / 256));
  // densities per pass: 1, or a group that shares every plane-wave factor
  const bool grp = a.n_dens > 1;
  switch (a.kernel * 2 + (grp ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((far_L_kernel<PFMM_LAPLACE, 1>), grid, dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((far_L_kernel<PFMM_LAPLACE, 4>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((far_L_kernel<PFMM_YUKAWA, 1>), grid, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((far_L_kernel<PFMM_YUKAWA, 4>), grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((far_L_kernel<PFMM_STOKES, 1>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((far_L_kernel<PFMM_STOKES, 2>), grid, dim3(256), 0, s, a); break;
  }
}

}  // namespace pfmm
