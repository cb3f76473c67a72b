// Near part by a fast multipole method whose expansions are Chebyshev
// interpolants, on a tree of boxes in lattice coordinates.
//
// The near part of the splitting (Sec. 1, Def. 1) is the free-space sum of
// the kernel over the sources of the cell and of its images m e1 + n e2,
// |m| <= m0, |n| <= 1, at targets in the cell. Sec. 7 evaluates it with a
// free-space FMM over all those sources and notes that the image cells hold
// the same sources, hence the same hierarchy of expansions. Here that is
// built in: the tree lives in lattice coordinates u (x = u1 e1 + u2 e2), so a
// box of an image cell is a box of the cell moved by whole lattice vectors and
// carries the cell box's expansion unchanged; only the cell's own boxes are
// stored, and the near region is a (2 m0 + 1) x 3 super-grid of them.
//
// Expansions: on a box with local coordinates s in [-1, 1]^2, P x P tensor
// Chebyshev points s_ab. The far field of the box's sources is represented by
// equivalent densities W_ab = sum_j q_j l_a(s1_j) l_b(s2_j) at those points
// (l_a: Lagrange basis), the field of distant boxes at a target box by its
// samples F_ab at the points, interpolated at the targets. Upward: W of a
// parent from its children by exact polynomial transfer (M2M); across: F of
// a box += kernel(point_ab - point_cd) W_cd over its interaction list (the
// children of the parent's neighbours that are not neighbours, M2L, the
// kernel sampled on the fly); downward: F of a child += the parent's F
// interpolated at the child's points (L2L); at the leaves: interpolation of
// F at every target plus the direct sum over the 3 x 3 neighbouring leaf
// boxes, images included (P2P). Each of the potential and the gradient
// components is interpolated as its own field, so the gradient needs no
// differentiation of an interpolant.
//
// Precision: W, F and every sum over boxes in FP64. MIXED: kernel samples in
// FP32 (M2L on displacements box centre to box centre taken in FP64 plus node
// offsets, partial sums over one row of P source points flushed to FP64; P2P
// on displacements taken in FP64 and rounded once, log terms added in FP64
// pair by pair, the others in FP32 over 16 sources).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "device_math.h"
#include "fmm.h"
#include "kernels.h"

namespace pfmm {

namespace {

struct Lvl {
  int n1, n2;       // boxes along e1, e2
  double h1, h2;    // lattice half-widths of a box
};
__device__ __forceinline__ Lvl level_of(const FmmTree& t, int l) {
  Lvl v;
  v.n1 = t.k1 << l;
  v.n2 = t.k2 << l;
  v.h1 = 0.5 / v.n1;
  v.h2 = 0.5 / v.n2;
  return v;
}
__device__ __forceinline__ int floordiv(int a, int b) { return a >= 0 ? a / b : -((b - 1 - a) / b); }
__device__ __forceinline__ int posmod(int a, int b) { const int r = a % b; return r < 0 ? r + b : r; }

// first and one-past-last sorted index of leaf box k
__device__ __forceinline__ int64_t leaf_begin(const int* cnt, int nblk, int64_t k) {
  return k ? cnt[k * nblk - 1] : 0;
}
__device__ __forceinline__ int64_t leaf_end(const int* cnt, int nblk, int64_t k) { return cnt[(k + 1) * nblk - 1]; }

// Chebyshev points of the first kind s_a = cos((2a+1) pi / 2P) and their
// barycentric weights (-1)^a sin((2a+1) pi / 2P)
__device__ void cheb_init(int P, double* s, double* w) {
  for (int a = threadIdx.x; a < P; a += blockDim.x) {
    const double th = (2 * a + 1) * PI / (2 * P);
    s[a] = cos(th);
    if (w) w[a] = (a & 1) ? -sin(th) : sin(th);
  }
}

// Lagrange basis of the P points at x (barycentric form): out[a * stride]
__device__ void lagrange(int P, const double* s, const double* w, double x, double* out, int stride) {
  double sum = 0.0;
  int hit = -1;
  for (int a = 0; a < P; ++a) {
    const double dd = x - s[a];
    if (dd == 0.0) hit = a;
    const double t = dd == 0.0 ? 0.0 : w[a] / dd;
    out[a * stride] = t;
    sum += t;
  }
  const double inv = 1.0 / sum;
  for (int a = 0; a < P; ++a) out[a * stride] = hit >= 0 ? (a == hit ? 1.0 : 0.0) : out[a * stride] * inv;
}

// transfer matrices T[h][a][a'] = l_a'((s_a + 2h - 1) / 2): parent basis at
// the points of child half h (0 lower, 1 upper) of each dimension
__device__ void transfer_init(int P, const double* s, const double* w, double* T) {
  for (int r = threadIdx.x; r < 2 * P; r += blockDim.x) {
    const int h = r / P, a = r % P;
    lagrange(P, s, w, 0.5 * (s[a] + 2 * h - 1), T + (size_t)r * P, 1);
  }
}

// a.cheb holds s [FMM_PMAX], w [FMM_PMAX] and T [2 P][P] (transfer_init's
// layout); each block copies what it needs into LDS (s, w, T may be null)
__device__ void cheb_load(const FmmArgs& a, int P, double* s, double* w, double* T) {
  for (int k = threadIdx.x; k < P; k += blockDim.x) {
    s[k] = a.cheb[k];
    if (w) w[k] = a.cheb[FMM_PMAX + k];
  }
  if (T)
    for (int k = threadIdx.x; k < 2 * P * P; k += blockDim.x) T[k] = a.cheb[2 * FMM_PMAX + k];
}

// Lagrange basis of the P points at x into registers (entries P.. are zero)
__device__ __forceinline__ void basis_regs(int P, const double* s, const double* w, double x,
                                           double (&l)[FMM_PMAX]) {
  double sum = 0.0;
  int hit = -1;
#pragma unroll
  for (int a = 0; a < FMM_PMAX; ++a) {
    double t = 0.0;
    if (a < P) {
      const double dd = x - s[a];
      if (dd == 0.0) hit = a;
      t = dd == 0.0 ? 0.0 : w[a] / dd;
    }
    l[a] = t;
    sum += t;
  }
  const double inv = 1.0 / sum;
#pragma unroll
  for (int a = 0; a < FMM_PMAX; ++a) l[a] = hit >= 0 ? (a == hit ? 1.0 : 0.0) : l[a] * inv;
}

template <int K> struct Fk {
  static constexpr int NC = K == PFMM_STOKES ? 2 : 1;    // density components
  static constexpr int NO = K == PFMM_STOKES ? 6 : 3;    // outputs
  static constexpr int NA = K == PFMM_STOKES ? 8 : 3;    // pair accumulators
};

// The kernel values of one pair from r^2: Yukawa K0(beta r) and
// K1(beta r)/(beta r); Laplace and Stokes log r^2 (log2 in FP32) and 1/r^2.
template <int K, typename real>
__device__ __forceinline__ void pair_vals(real r2, real beta, real& va, real& vb) {
  constexpr bool F32 = std::is_same<real, float>::value;
  if constexpr (K == PFMM_YUKAWA) {
    if constexpr (F32) {
      // t = (beta r / 2)^2: when every lane is on the series (x <= 2, the
      // common case of leaf pairs), no square root
      const float t = r2 * (0.25f * beta * beta);
      if (__all(t <= 1.0f)) bessel_k01_f32_series_t(t, va, vb);
      else bessel_k01_f32_split(beta * __builtin_amdgcn_sqrtf(r2), va, vb);
    } else {
      const double t = r2 * (0.25 * beta * beta);
      if (__all(t <= 1.0)) bessel_k01_f64_series_t(t, va, vb);
      else bessel_k01_f64(beta * sqrt(r2), va, vb);
    }
  } else if constexpr (F32) {
    va = __builtin_amdgcn_logf(r2);
    vb = __builtin_amdgcn_rcpf(r2);
  } else {
    va = log(r2);
    vb = recip_pw(r2);
  }
}

// The terms of one pair (values va, vb from pair_vals, displacement dx, dy =
// target - source, weights w0, w1) added to the accumulators; LOG64: without
// the log terms.
template <int K, bool LOG64, typename real>
__device__ __forceinline__ void pair_acc(real va, real vb, real dx, real dy, real w0, real w1, real* acc) {
  if constexpr (K == PFMM_STOKES) {
    const real ia = vb * dx, ib = vb * dy;
    const real c = ia * w0 + ib * w1;
    const real ca = c * ia;
    if constexpr (!LOG64) { acc[0] += va * w0; acc[1] += va * w1; }
    acc[2] += c * dx; acc[3] += c * dy; acc[4] += c;
    acc[5] += ca * dx; acc[6] += ca * dy;
    acc[7] += w1 * ia - w0 * ib;
  } else {
    if constexpr (K == PFMM_YUKAWA || !LOG64) acc[0] += w0 * va;
    const real g = w0 * vb;
    acc[1] += g * dx;
    acc[2] += g * dy;
  }
}

// One kernel sample (pair displacement dx, dy = target - source) with
// weights w0 (w1: second Stokes component) into the accumulators:
//   Laplace: sum w lg, sum w dx/r^2, sum w dy/r^2           (lg = log r^2; log2 in FP32)
//   Yukawa:  sum w K0(beta r), sum w K1(beta r)/(beta r) dx, ... dy
//   Stokes:  sum lg w1, sum lg w2, sum c dx, sum c dy, sum c, sum c ia dx,
//            sum c ia dy, sum (w2 ia - w1 ib);  ia = dx/r^2, ib = dy/r^2,
//            c = ia w1 + ib w2
// GUARD: r = 0 contributes nothing (the self pair).
// LOG64: the log terms are left out of acc and lg is returned instead (the
// caller adds them in FP64).
// r2_self replaces r^2 of a guarded pair (its log then equals the caller's
// log shift, and the shifted log term vanishes).
template <int K, bool GUARD, bool LOG64, typename real>
__device__ __forceinline__ void fmm_pair(real dx, real dy, real w0, real w1, real* acc, real beta, real& lg_out,
                                         real r2_self = (real)1) {
  constexpr bool F32 = std::is_same<real, float>::value;
  real r2 = F32 ? __builtin_fmaf(dx, dx, dy * dy) : dx * dx + dy * dy;
  if constexpr (GUARD) {
    const bool ok = r2 > (real)0;
    r2 = ok ? r2 : r2_self;
    w0 = ok ? w0 : (real)0;
    w1 = ok ? w1 : (real)0;
  }
  real va, vb;
  pair_vals<K, real>(r2, beta, va, vb);
  lg_out = K == PFMM_YUKAWA ? (real)0 : va;
  pair_acc<K, LOG64, real>(va, vb, dx, dy, w0, w1, acc);
}

// accumulators -> outputs (potential, gradient; Stokes u1, u2, du1/dx,
// du1/dy, du2/dx, du2/dy); lscale converts the log base to natural logs
template <int K>
__device__ __forceinline__ void fmm_outputs(const double* A, double* o, double beta, double lscale) {
  const double inv4pi = 1.0 / (4 * PI), inv2pi = 1.0 / (2 * PI);
  if constexpr (K == PFMM_LAPLACE) {
    o[0] = -inv4pi * lscale * A[0];
    o[1] = -inv2pi * A[1];
    o[2] = -inv2pi * A[2];
  } else if constexpr (K == PFMM_YUKAWA) {
    o[0] = inv2pi * A[0];
    o[1] = -beta * beta * inv2pi * A[1];
    o[2] = -beta * beta * inv2pi * A[2];
  } else {
    // u_i = (1/4pi) sum [-(1/2) log r^2 f_i + (r.f) r_i / r^2]
    o[0] = inv4pi * (-0.5 * lscale * A[0] + A[2]);
    o[1] = inv4pi * (-0.5 * lscale * A[1] + A[3]);
    o[2] = inv4pi * (A[4] - 2 * A[5]);
    o[3] = inv4pi * (A[7] - 2 * A[6]);
    o[4] = inv4pi * (-A[7] - 2 * A[6]);
    o[5] = -o[2];
  }
}

}  // namespace

// the tables of cheb_load, once per evaluation (one block)
__global__ __launch_bounds__(64) void fmm_cheb_kernel(FmmArgs a) {
  const int P = a.t.P;
  __shared__ double s_s[FMM_PMAX], s_w[FMM_PMAX];
  cheb_init(P, s_s, s_w);
  __syncthreads();
  for (int k = threadIdx.x; k < P; k += blockDim.x) { a.cheb[k] = s_s[k]; a.cheb[FMM_PMAX + k] = s_w[k]; }
  transfer_init(P, s_s, s_w, a.cheb + 2 * FMM_PMAX);
}

// ---------------------------------------------------------------------------
// P2M: equivalent densities of each leaf box (grid: leaf boxes x densities)
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(FMM_CHUNK) void fmm_p2m_kernel(FmmArgs a) {
  const FmmTree& t = a.t;
  const int P = t.P, P2 = P * P;
  const int box = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
  const Lvl lv = level_of(t, t.L);
  const int i = box % lv.n1, j = box / lv.n1;
  // basis values [a][point], rows FMM_CHUNK + 1 apart (odd: the rows that
  // the threads of a wavefront read at one point fall in distinct banks)
  constexpr int LDL = FMM_CHUNK + 1;
  __shared__ double s_s[FMM_PMAX], s_w[FMM_PMAX];
  __shared__ double s_l1[FMM_PMAX * LDL], s_l2[FMM_PMAX * LDL];
  __shared__ double s_q[NC][FMM_CHUNK];
  cheb_load(a, P, s_s, s_w, nullptr);
  const int64_t b0 = leaf_begin(a.scnt, a.snblk, box), b1 = leaf_end(a.scnt, a.snblk, box);
  double acc[4][NC];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[r][c] = 0.0;
  __syncthreads();
  for (int64_t c0 = b0; c0 < b1; c0 += FMM_CHUNK) {
    const int nch = (int)min((int64_t)FMM_CHUNK, b1 - c0);
    if (tid < nch) {
      const int64_t k = c0 + tid;
      const double u2 = a.sy[k] / t.eta, u1 = (a.sx[k] - t.xi * u2) / t.d;
      lagrange(P, s_s, s_w, 2.0 * ((u1 + 0.5) * lv.n1 - i) - 1.0, s_l1 + tid, LDL);
      lagrange(P, s_s, s_w, 2.0 * ((u2 + 0.5) * lv.n2 - j) - 1.0, s_l2 + tid, LDL);
#pragma unroll
      for (int c = 0; c < NC; ++c) s_q[c][tid] = a.sq[((size_t)v * NC + c) * a.n_src + k];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int node = tid + r * FMM_CHUNK;
      if (node < P2) {
        const double* l1 = s_l1 + (node / P) * LDL;
        const double* l2 = s_l2 + (node % P) * LDL;
        for (int jj = 0; jj < nch; ++jj) {
          const double g = l1[jj] * l2[jj];
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[r][c] = fma(s_q[c][jj], g, acc[r][c]);
        }
      }
    }
    __syncthreads();
  }
  const int64_t gb = t.box_off[t.L] + box;
  const int qn = a.n_dens * NC;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int node = tid + r * FMM_CHUNK;
    if (node < P2)
#pragma unroll
      for (int c = 0; c < NC; ++c) a.W[((size_t)gb * qn + v * NC + c) * P2 + node] = acc[r][c];
  }
  if (tid == 0 && v == 0) a.scount[gb] = (int)(b1 - b0);
  // the box's total density per component (the W sum over its points)
  __shared__ double s_red[FMM_CHUNK];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double x = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (tid + r * FMM_CHUNK < P2) x += acc[r][c];
    s_red[tid] = x;
    __syncthreads();
    for (int o = FMM_CHUNK / 2; o > 0; o >>= 1) {
      if (tid < o) s_red[tid] += s_red[tid + o];
      __syncthreads();
    }
    if (tid == 0) a.Q[(size_t)gb * qn + v * NC + c] = s_red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// M2M: equivalent densities of the boxes of level l from their children
// (grid: boxes of level l x density components)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fmm_m2m_kernel(FmmArgs a, int l, int qn) {
  const FmmTree& t = a.t;
  const int P = t.P, P2 = P * P;
  const int box = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const Lvl lv = level_of(t, l), lc = level_of(t, l + 1);
  const int i = box % lv.n1, j = box / lv.n1;
  __shared__ double s_s[FMM_PMAX], s_w[FMM_PMAX];
  __shared__ double s_T[2 * FMM_PMAX * FMM_PMAX], s_c[FMM_PMAX * FMM_PMAX], s_t[FMM_PMAX * FMM_PMAX];
  cheb_load(a, P, s_s, s_w, s_T);
  double acc[2] = {0.0, 0.0};
  int cnt = 0;
  for (int h = 0; h < 4; ++h) {
    const int hi = h & 1, hj = h >> 1;
    const int64_t cb = t.box_off[l + 1] + (int64_t)(2 * j + hj) * lc.n1 + 2 * i + hi;
    __syncthreads();
    for (int n = tid; n < P2; n += 256) s_c[n] = a.W[((size_t)cb * qn + c) * P2 + n];
    if (tid == 0) cnt += a.scount[cb];
    __syncthreads();
    // s_t[a][b'] = sum_b W_child[a][b] T[hj][b][b']
    for (int n = tid; n < P2; n += 256) {
      const int ra = n / P, bp = n % P;
      double s = 0.0;
      for (int b = 0; b < P; ++b) s = fma(s_c[ra * P + b], s_T[(hj * P + b) * P + bp], s);
      s_t[n] = s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int n = tid + 256 * r;
      if (n < P2) {
        const int ap = n / P, bp = n % P;
        double s = 0.0;
        for (int ra = 0; ra < P; ++ra) s = fma(s_T[(hi * P + ra) * P + ap], s_t[ra * P + bp], s);
        acc[r] += s;
      }
    }
  }
  const int64_t gb = t.box_off[l] + box;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int n = tid + 256 * r;
    if (n < P2) a.W[((size_t)gb * qn + c) * P2 + n] = acc[r];
  }
  if (tid == 0 && c == 0) a.scount[gb] = cnt;
  if (tid == 0) {
    double q = 0.0;
    for (int h = 0; h < 4; ++h) {
      const int64_t cb = t.box_off[l + 1] + (int64_t)(2 * j + (h >> 1)) * lc.n1 + 2 * i + (h & 1);
      q += a.Q[(size_t)cb * qn + c];
    }
    a.Q[(size_t)gb * qn + c] = q;
  }
}

// ---------------------------------------------------------------------------
// M2L: local fields of every box of every level from its interaction list
// (grid: all boxes x densities; block: one thread per Chebyshev point).
// Level 0 has no parent: its list is every non-neighbouring box of the
// super-grid.
// ---------------------------------------------------------------------------
template <typename real> struct alignas(4 * sizeof(real)) SrcNode { real ox, oy, w0, w1; };

// 2^k with 2^k times a box's width about 1/2 at level l: coordinate
// differences are scaled by it (exactly) so that the log2 of a typical M2L or
// neighbour pair's r^2 is near zero, and its FP32 value carries an absolute
// error of an ulp of a small number; the shift 2k is removed in FP64
__host__ __device__ inline int level_shift(const FmmTree& t, int l) {
  const double h = sqrt(t.d * t.eta / ((double)(t.k1 << l) * (double)(t.k2 << l)));
  return -(int)lround(log2(2.0 * h));
}

// MIXED: the FP32 kernel samples (the finest levels); FP64: the coarse levels
// of a mixed evaluation (their equivalent densities are sums over many
// sources, too large for FP32 log terms) and every level in FP64 mode. Boxes
// gb0 + blockIdx.x. Slices: block z = blockIdx.z takes the entries
// [z per, (z + 1) per) of its box's interaction list (listed in a fixed
// order); with one slice it writes F, else its partial field to
// Fp[z][box - gb0], summed in slice order by fmm_slice_sum_kernel.
template <int K, bool MIXED>
__global__ __launch_bounds__(512) void fmm_m2l_kernel(FmmArgs a, int64_t gb0, int64_t nbox, int per) {
  using real = typename std::conditional<MIXED, float, double>::type;
  constexpr int NC = Fk<K>::NC, NO = Fk<K>::NO, NA = Fk<K>::NA;
  constexpr bool SHIFT = MIXED && K != PFMM_YUKAWA;     // scaled coordinates, log2 shifted
  const FmmTree& t = a.t;
  const int P = t.P, P2 = P * P;
  const int64_t gb = gb0 + blockIdx.x;
  const int v = blockIdx.y, tid = threadIdx.x;
  int l = 0;
  while (l < t.L && gb >= t.box_off[l + 1]) ++l;
  const Lvl lv = level_of(t, l);
  const int box = (int)(gb - t.box_off[l]);
  const int i = box % lv.n1, j = box / lv.n1;
  __shared__ double s_s[FMM_PMAX];
  __shared__ SrcNode<real> s_src[FMM_PMAX * FMM_PMAX];
  __shared__ double s_wsum[8][NC];
  cheb_load(a, P, s_s, nullptr, nullptr);
  __syncthreads();
  const bool act = tid < P2;
  const int na = act ? tid / P : 0, nb = act ? tid % P : 0;
  const int ksh = SHIFT ? level_shift(t, l) : 0;
  const double sc = ldexp(1.0, ksh);
  // the point's offset from its box centre (the same for every box of the
  // level), scaled
  const double ox = sc * (t.d * lv.h1 * s_s[na] + t.xi * lv.h2 * s_s[nb]);
  const double oy = sc * (t.eta * lv.h2 * s_s[nb]);
  // circumradius of a box: half its longer diagonal
  const double rad = 0.5 * fmax(hypot(2 * t.d * lv.h1 + 2 * t.xi * lv.h2, 2 * t.eta * lv.h2),
                                hypot(-2 * t.d * lv.h1 + 2 * t.xi * lv.h2, 2 * t.eta * lv.h2));
  const int qn = a.n_dens * NC;
  const real beta = (real)(a.beta / sc);
  double acc[NA];
#pragma unroll
  for (int c = 0; c < NA; ++c) acc[c] = 0.0;
  double wtot[NC];                                      // sum of the visited equivalent densities
#pragma unroll
  for (int c = 0; c < NC; ++c) wtot[c] = 0.0;
  const int I0 = -t.m0 * lv.n1, I1 = (t.m0 + 1) * lv.n1, J0 = -lv.n2, J1 = 2 * lv.n2;

  const int e0 = (int)blockIdx.z * per, e1 = e0 + per;
  int e = 0;                                            // list position (uniform over the block)
  auto visit = [&](int I, int J) {
    const int pos = e++;
    if (pos < e0 || pos >= e1) return;
    const int64_t sg = t.box_off[l] + (int64_t)posmod(J, lv.n2) * lv.n1 + posmod(I, lv.n1);
    if (a.scount[sg] == 0) return;                      // uniform over the block
    // target centre minus source centre (lattice difference of the super-grid)
    const double du1 = (double)(i - I) / lv.n1, du2 = (double)(j - J) / lv.n2;
    const double Dx = t.d * du1 + t.xi * du2, Dy = t.eta * du2;
    if (sqrt(Dx * Dx + Dy * Dy) - 2 * rad > a.rcut) return;
    __syncthreads();
    double w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = act ? a.W[((size_t)sg * qn + v * NC + c) * P2 + tid] : 0.0;
    if (act) {
      SrcNode<real> sn;
      sn.ox = (real)ox;
      sn.oy = (real)oy;
      sn.w0 = (real)w[0];
      sn.w1 = NC > 1 ? (real)w[NC - 1] : (real)0;
      s_src[tid] = sn;
    }
    if constexpr (SHIFT) {
      // the box's total equivalent density (FP64), for the log shift
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double x = w[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if ((tid & 63) == 0) s_wsum[tid >> 6][c] = x;
      }
    }
    __syncthreads();
    if constexpr (SHIFT) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) wtot[c] += s_wsum[q][c];
    }
    if (act) {
      const real ex = (real)(sc * Dx + ox), ey = (real)(sc * Dy + oy);
      for (int r = 0; r < P; ++r) {
        real p[NA];
#pragma unroll
        for (int c = 0; c < NA; ++c) p[c] = (real)0;
        for (int c = 0; c < P; ++c) {
          const SrcNode<real> sn = s_src[r * P + c];
          real lg;
          fmm_pair<K, false, false, real>(ex - sn.ox, ey - sn.oy, sn.w0, sn.w1, p, beta, lg);
        }
#pragma unroll
        for (int c = 0; c < NA; ++c) acc[c] += (double)p[c];
      }
    }
  };

  if (l == 0) {
    for (int J = J0; J < J1; ++J)
      for (int I = I0; I < I1; ++I)
        if (abs(I - i) > 1 || abs(J - j) > 1) visit(I, J);
  } else {
    const int pi = i >> 1, pj = j >> 1;
    for (int qj = pj - 1; qj <= pj + 1; ++qj)
      for (int qi = pi - 1; qi <= pi + 1; ++qi)
        for (int h = 0; h < 4; ++h) {
          const int I = 2 * qi + (h & 1), J = 2 * qj + (h >> 1);
          if (I < I0 || I >= I1 || J < J0 || J >= J1) continue;
          if (abs(I - i) > 1 || abs(J - j) > 1) visit(I, J);
        }
  }
  if (act) {
    if constexpr (SHIFT) {
      // log2 of scaled r^2 = log2 r^2 + 2k; scaled gradient sums carry 2^-k
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] -= 2.0 * ksh * wtot[c];
      if constexpr (K == PFMM_LAPLACE) { acc[1] *= sc; acc[2] *= sc; }
      else { acc[4] *= sc; acc[5] *= sc; acc[6] *= sc; acc[7] *= sc; }
    }
    double o[NO];
    fmm_outputs<K>(acc, o, a.beta, MIXED ? 0.69314718055994530942 : 1.0);
#pragma unroll
    for (int c = 0; c < NO; ++c) {
      if (gridDim.z == 1) a.F[((size_t)gb * a.n_dens * NO + v * NO + c) * P2 + tid] = o[c];
      else a.Fp[(((size_t)blockIdx.z * nbox + (gb - gb0)) * a.n_dens * NO + v * NO + c) * P2 + tid] = o[c];
    }
  }
}

// ---------------------------------------------------------------------------
// Tabulated M2L on the matrix cores. For one level and one parity group of
// target boxes (boxes whose parents sit alike share their 27 list classes)
// the lists are a matrix product: F[:, b] += sum over classes c of
// T_c W[:, b + offset_c], with T_c the class's FP64 table (rows: output
// component and target point, NO P^2; columns: source point and component,
// NC P^2) and W the source boxes' equivalent densities. A block takes 64 rows
// (16 per wavefront) by 32 target boxes over the classes of one slice; per
// class it gathers the 32 source boxes' W columns into LDS, and each
// wavefront streams its 16 table rows from memory into FP64 MFMA 16x16x4
// products (two per step, 16 boxes each). Inputs, products and sums are
// FP64 throughout.
// ---------------------------------------------------------------------------
typedef double fmm_v4d __attribute__((ext_vector_type(4)));
constexpr int MM_ROWS = 64, MM_BOXES = 32;   // block tile: 4 wavefronts x 16 rows, 2 x 16 boxes
constexpr int MM_KC = 128;                   // source columns per LDS stage
constexpr int MM_LD = MM_KC + 1;             // LDS row of one box (odd: the 16 boxes of a read hit distinct banks)
constexpr int MM_KSTEP = 16;                 // table values in flight per lane (16 products of K = 4)

template <int K>
__global__ __launch_bounds__(256) void fmm_m2l_mfma_kernel(FmmArgs a, int l, int per, int n_nt) {
  constexpr int NC = Fk<K>::NC, NO = Fk<K>::NO;
  const FmmTree& t = a.t;
  const int P = t.P, P2 = P * P;
  const int NS = NC * P2, NSP = (NS + 3) & ~3, M = NO * P2;
  const Lvl lv = level_of(t, l);
  const int hn1 = lv.n1 / 2, hn2 = lv.n2 / 2, hn = hn1 * hn2;
  const int g = blockIdx.x / n_nt, nt = blockIdx.x % n_nt;
  const int pi = g & 1, pj = g >> 1;
  const int v = (int)blockIdx.z / FMM_TAB_SLICES, z = (int)blockIdx.z % FMM_TAB_SLICES;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = (int)blockIdx.y * MM_ROWS + wv * 16;
  const int qn = a.n_dens * NC;
  __shared__ double s_wm[MM_BOXES * MM_LD];
  const double rad = 0.5 * fmax(hypot(2 * t.d * lv.h1 + 2 * t.xi * lv.h2, 2 * t.eta * lv.h2),
                                hypot(-2 * t.d * lv.h1 + 2 * t.xi * lv.h2, 2 * t.eta * lv.h2));
  const double* tab = (const double*)(a.tab + a.tab_off[l]);
  // this lane's row of the table tile (A) and its step within K = 4
  const int arow = m0 + (lane & 15), kq = lane >> 4;
  const bool arow_ok = arow < M;
  fmm_v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  const int e0 = z * per, e1 = e0 + per;
  int e = 0;
  for (int dJ = -2 - pj; dJ <= 3 - pj; ++dJ)
    for (int dI = -2 - pi; dI <= 3 - pi; ++dI) {
      if (abs(dI) <= 1 && abs(dJ) <= 1) continue;
      const int pos = e++;
      if (pos < e0 || pos >= e1) continue;
      const double Dx = -(t.d * dI / lv.n1 + t.xi * dJ / lv.n2), Dy = -(t.eta * dJ / lv.n2);
      if (sqrt(Dx * Dx + Dy * Dy) - 2 * rad > a.rcut) continue;   // uniform over the block
      const int cls = (dJ + 3) * 7 + dI + 3;
      const double* tc = tab + (size_t)cls * NS * M;     // [source column][row]
      for (int c0 = 0; c0 < NSP; c0 += MM_KC) {
        const int kc = min(MM_KC, NSP - c0);             // a multiple of 4
        __syncthreads();
        // gather: the source box of target box j, columns c0 .. c0 + kc
        // (zero past NC P^2 and for boxes beyond the group)
        for (int q = tid; q < MM_BOXES * kc; q += 256) {
          const int j = q / kc, r = c0 + q % kc;
          const int idx = nt * MM_BOXES + j;
          double w = 0.0;
          if (idx < hn && r < NS) {
            const int bi = 2 * (idx % hn1) + pi, bj = 2 * (idx / hn1) + pj;
            const int64_t sg = t.box_off[l] + (int64_t)posmod(bj + dJ, lv.n2) * lv.n1 + posmod(bi + dI, lv.n1);
            w = a.W[((size_t)sg * qn + v * NC + r / P2) * P2 + r % P2];
          }
          s_wm[j * MM_LD + q % kc] = w;
        }
        __syncthreads();
        for (int k0 = 0; k0 < kc; k0 += 4 * MM_KSTEP) {
          double av[MM_KSTEP];
#pragma unroll
          for (int u = 0; u < MM_KSTEP; ++u) {
            const int col = c0 + k0 + 4 * u + kq;
            av[u] = (arow_ok && col < NS) ? tc[(size_t)col * M + arow] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < MM_KSTEP; ++u) {
            if (k0 + 4 * u < kc) {                         // uniform
              const int cl = k0 + 4 * u + kq;
              const double b0 = s_wm[(lane & 15) * MM_LD + cl];
              const double b1 = s_wm[(16 + (lane & 15)) * MM_LD + cl];
              acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b0, acc0, 0, 0, 0);
              acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b1, acc1, 0, 0, 0);
            }
          }
        }
      }
    }
  // the lane holds rows m0 + lane / 16 + 4 r of boxes lane % 16 (acc0) and
  // 16 + lane % 16 (acc1), the output layout of the 16x16x4 FP64 product
  // (checked on the GPU against a host product): slice z's partial fields
  const int64_t nbox = t.box_off[l + 1] - t.box_off[l];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int idx = nt * MM_BOXES + h * 16 + (lane & 15);
    if (idx >= hn) continue;
    const int bi = 2 * (idx % hn1) + pi, bj = 2 * (idx / hn1) + pj;
    const int64_t lb = (int64_t)bj * lv.n1 + bi;
    const fmm_v4d& ac = h ? acc1 : acc0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + kq + 4 * r;
      if (row < M) a.Fp[(((size_t)z * nbox + lb) * a.n_dens + v) * NO * P2 + row] = ac[r];
    }
  }
}

// F[f0 + k] = sum over slices z (in order) of Fp[z n + k], k < n (the
// local fields of a range of boxes, n doubles from element f0)
__global__ __launch_bounds__(256) void fmm_slice_sum_kernel(FmmArgs a, int64_t f0, int64_t n, int n_slices) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int z = 0; z < n_slices; ++z) s += a.Fp[(size_t)z * n + k];
  a.F[f0 + k] = s;
}

// ---------------------------------------------------------------------------
// M2L tables. Table of level l, class cls = (dJ + 3) 7 + dI + 3 (source box =
// target box + (dI, dJ)): entry [cls][sc][o][t] = output o at target point t
// of unit density on source point-component sc, FP64 (grid: classes x
// source point-components; a thread per target point).
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(512) void fmm_table_build_kernel(FmmArgs a, int l, double* tab) {
  constexpr int NC = Fk<K>::NC, NO = Fk<K>::NO, NA = Fk<K>::NA;
  const FmmTree& t = a.t;
  const int P = t.P, P2 = P * P;
  const int cls = blockIdx.x, sc = blockIdx.y, tp = threadIdx.x;
  const int dI = cls % 7 - 3, dJ = cls / 7 - 3;
  if ((abs(dI) <= 1 && abs(dJ) <= 1) || tp >= P2) return;
  const Lvl lv = level_of(t, l);
  const int c = sc / P2, sn = sc % P2;
  auto node = [&](int a_) { return cos((2 * a_ + 1) * PI / (2 * P)); };
  const double ta = node(tp / P), tb = node(tp % P), sa = node(sn / P), sb = node(sn % P);
  // target point minus source point: -(box offset) + the two points' offsets
  const double dx = -(t.d * dI / lv.n1 + t.xi * dJ / lv.n2) + t.d * lv.h1 * (ta - sa) + t.xi * lv.h2 * (tb - sb);
  const double dy = -(t.eta * dJ / lv.n2) + t.eta * lv.h2 * (tb - sb);
  double acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k] = 0.0;
  double lg;
  fmm_pair<K, false, false, double>(dx, dy, c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, acc, a.beta, lg);
  double o[NO];
  fmm_outputs<K>(acc, o, a.beta, 1.0);
#pragma unroll
  for (int k = 0; k < NO; ++k)
    tab[(((size_t)cls * NC * P2 + sc) * NO + k) * P2 + tp] = o[k];
}

// ---------------------------------------------------------------------------
// L2L: local fields of the boxes of level l + 1 += their parent's,
// interpolated (grid: boxes of level l + 1 x output components)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fmm_l2l_kernel(FmmArgs a, int l, int no_total) {
  const FmmTree& t = a.t;
  const int P = t.P, P2 = P * P;
  const int box = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const Lvl lc = level_of(t, l + 1), lp = level_of(t, l);
  const int i = box % lc.n1, j = box / lc.n1;
  const int hi = i & 1, hj = j & 1;
  __shared__ double s_s[FMM_PMAX], s_w[FMM_PMAX];
  __shared__ double s_T[2 * FMM_PMAX * FMM_PMAX], s_p[FMM_PMAX * FMM_PMAX], s_t[FMM_PMAX * FMM_PMAX];
  cheb_load(a, P, s_s, s_w, s_T);
  const int64_t pg = t.box_off[l] + (int64_t)(j >> 1) * lp.n1 + (i >> 1);
  const int64_t cg = t.box_off[l + 1] + box;
  for (int n = tid; n < P2; n += 256) s_p[n] = a.F[((size_t)pg * no_total + c) * P2 + n];
  __syncthreads();
  // s_t[a'][b] = sum_b' F_parent[a'][b'] T[hj][b][b']
  for (int n = tid; n < P2; n += 256) {
    const int ap = n / P, b = n % P;
    double s = 0.0;
    for (int bp = 0; bp < P; ++bp) s = fma(s_p[ap * P + bp], s_T[(hj * P + b) * P + bp], s);
    s_t[n] = s;
  }
  __syncthreads();
  for (int n = tid; n < P2; n += 256) {
    const int ra = n / P, b = n % P;
    double s = 0.0;
    for (int ap = 0; ap < P; ++ap) s = fma(s_T[(hi * P + ra) * P + ap], s_t[ap * P + b], s);
    a.F[((size_t)cg * no_total + c) * P2 + n] += s;
  }
}

// ---------------------------------------------------------------------------
// Leaves: the local field interpolated at each target plus the direct sum over
// the 3 x 3 neighbouring leaf boxes with their image shifts (grid: leaf boxes
// x densities; a box's targets in chunks of FMM_LEAF, one per thread). The
// three boxes of a neighbour row are consecutive in leaf-box order, so a row
// is one range of sources (two where it crosses the cell's edge, whose
// parts carry different image shifts), streamed through LDS.
// ---------------------------------------------------------------------------
// The local field F of leaf box (i, j) (LDS, [NO][P^2]) interpolated at the
// target (tx, ty): o[c] = sum_ab l_a(x1) l_b(x2) F[c][a P + b]
template <int NO>
__device__ __forceinline__ void leaf_local(const FmmTree& t, const Lvl& lv, int i, int j, const double* s_s,
                                           const double* s_w, const double* s_F, double tx, double ty, double* o) {
  const int P = t.P, P2 = P * P;
  const double u2 = ty / t.eta, u1 = (tx - t.xi * u2) / t.d;
  const double x1 = 2.0 * ((u1 + 0.5) * lv.n1 - i) - 1.0, x2 = 2.0 * ((u2 + 0.5) * lv.n2 - j) - 1.0;
  // basis in the second dimension in registers, the first on the fly
  double l2[FMM_PMAX];
  basis_regs(P, s_s, s_w, x2, l2);
  double sum1 = 0.0;
  int hit1 = -1;
  for (int ra = 0; ra < P; ++ra) {
    const double dd = x1 - s_s[ra];
    if (dd == 0.0) hit1 = ra;
    sum1 += dd == 0.0 ? 0.0 : s_w[ra] / dd;
  }
  const double inv1 = 1.0 / sum1;
  for (int ra = 0; ra < P; ++ra) {
    double row[NO];
#pragma unroll
    for (int c = 0; c < NO; ++c) row[c] = 0.0;
#pragma unroll
    for (int b = 0; b < FMM_PMAX; ++b)
      if (b < P)
#pragma unroll
        for (int c = 0; c < NO; ++c) row[c] = fma(l2[b], s_F[c * P2 + ra * P + b], row[c]);
    const double dd = x1 - s_s[ra];
    const double la = hit1 >= 0 ? (ra == hit1 ? 1.0 : 0.0) : s_w[ra] / dd * inv1;
#pragma unroll
    for (int c = 0; c < NO; ++c) o[c] = fma(la, row[c], o[c]);
  }
}

// The direct pairs of one LDS chunk of nch sources against this thread's
// target, 16 sources per FP32 partial sum (log terms pair by pair in FP64)
template <int K, bool MIXED, bool GUARD, int BS>
__device__ __forceinline__ void leaf_pairs(int nch, double tx, double ty, const double* s_x, const double* s_y,
                                           const double (*s_q)[BS], const float (*s_q32)[BS],
                                           double sc, int ksh,
                                           typename std::conditional<MIXED, float, double>::type beta,
                                           typename std::conditional<MIXED, float, double>::type r2_self,
                                           double* acc) {
  using real = typename std::conditional<MIXED, float, double>::type;
  constexpr int NC = Fk<K>::NC, NA = Fk<K>::NA;
  constexpr int NLOG = (K != PFMM_YUKAWA && MIXED) ? NC : 0;
  for (int j0 = 0; j0 < nch; j0 += 16) {
    const int j1 = min(nch, j0 + 16);
    real p[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) p[c] = (real)0;
    for (int jj = j0; jj < j1; ++jj) {
      const real dx = NLOG > 0 ? (real)(sc * (tx - s_x[jj])) : (real)(tx - s_x[jj]);
      const real dy = NLOG > 0 ? (real)(sc * (ty - s_y[jj])) : (real)(ty - s_y[jj]);
      real w0, w1;
      if constexpr (MIXED) { w0 = s_q32[0][jj]; w1 = NC > 1 ? s_q32[NC - 1][jj] : 0.0f; }
      else { w0 = s_q[0][jj]; w1 = NC > 1 ? s_q[NC - 1][jj] : 0.0; }
      real lg;
      fmm_pair<K, GUARD, (NLOG > 0), real>(dx, dy, w0, w1, p, beta, lg, r2_self);
      if constexpr (NLOG > 0) {   // log terms straight into FP64 (a guarded pair gives 0)
        const double lgs = (double)lg - 2.0 * ksh;
        acc[0] = fma(s_q[0][jj], lgs, acc[0]);
        if constexpr (NC > 1) acc[1] = fma(s_q[NC - 1][jj], lgs, acc[1]);
      }
    }
#pragma unroll
    for (int c = NLOG; c < NA; ++c) acc[c] += (double)p[c];
  }
}

template <int K, bool MIXED, int BS>
__global__ __launch_bounds__(BS) void fmm_leaf_kernel(FmmArgs a) {
  using real = typename std::conditional<MIXED, float, double>::type;
  constexpr int NC = Fk<K>::NC, NO = Fk<K>::NO, NA = Fk<K>::NA;
  constexpr int NLOG = (K != PFMM_YUKAWA && MIXED) ? NC : 0;   // log terms summed in FP64 per pair
  const FmmTree& t = a.t;
  const int P = t.P, P2 = P * P;
  const int box = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
  const Lvl lv = level_of(t, t.L);
  const int i = box % lv.n1, j = box / lv.n1;
  const int64_t gb = t.box_off[t.L] + box;
  const int64_t t0 = leaf_begin(a.tcnt, a.tnblk, box), t1 = leaf_end(a.tcnt, a.tnblk, box);
  if (t0 >= t1) return;                                   // uniform over the block
  __shared__ double s_s[FMM_PMAX], s_w[FMM_PMAX];
  __shared__ double s_F[6 * FMM_PMAX * FMM_PMAX];
  __shared__ double s_x[BS], s_y[BS], s_q[NC][BS];
  __shared__ float s_q32[NC][BS];
  cheb_load(a, P, s_s, s_w, nullptr);
  for (int n = tid; n < NO * P2; n += BS)
    s_F[n] = a.F[((size_t)gb * a.n_dens * NO + v * NO) * P2 + n];
  __syncthreads();
  const real beta = (real)a.beta;
  // mixed Laplace/Stokes: differences scaled by 2^k (as in the M2L) so that
  // the FP32 log2 of r^2 is near zero; its shift 2k is removed in FP64
  const int ksh = NLOG > 0 ? level_shift(t, t.L) : 0;
  const double sc = ldexp(1.0, ksh);
  // stand-in r^2 of a guarded (r = 0) pair: the log shift's (Laplace, Stokes),
  // or x = beta r = 1 (Yukawa: the series branch, as the other pairs of a
  // fine leaf)
  const real r2_self = K == PFMM_YUKAWA ? (real)(1.0 / (a.beta * a.beta)) : (real)ldexp(1.0, 2 * ksh);
  for (int64_t tc = t0; tc < t1; tc += BS) {
    const int64_t k = tc + tid;
    const bool act = k < t1;
    const double tx = act ? a.tx[k] : 0.0, ty = act ? a.ty[k] : 0.0;
    // interpolated local field
    double o[NO];
#pragma unroll
    for (int c = 0; c < NO; ++c) o[c] = 0.0;
    if (act) leaf_local<NO>(t, lv, i, j, s_s, s_w, s_F, tx, ty, o);
    // direct sum over the neighbouring leaf boxes, one row at a time
    double acc[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) acc[c] = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
      const int J = j + dj, n = floordiv(J, lv.n2), row = posmod(J, lv.n2);
      for (int q = 0; q < 3;) {
        // boxes I = i - 1 + q .. i - 1 + last of one image column m
        const int m = floordiv(i - 1 + q, lv.n1);
        int last = q;
        while (last < 2 && floordiv(i + last, lv.n1) == m) ++last;
        const int64_t kb0 = (int64_t)row * lv.n1 + posmod(i - 1 + q, lv.n1);
        const int64_t kb1 = (int64_t)row * lv.n1 + posmod(i - 1 + last, lv.n1);
        const bool own = dj == 0 && m == 0 && q <= 1 && last >= 1;
        q = last + 1;
        const double shx = m * t.d + n * t.xi, shy = n * t.eta;
        const int64_t s0 = leaf_begin(a.scnt, a.snblk, kb0), s1 = leaf_end(a.scnt, a.snblk, kb1);
        for (int64_t c0 = s0; c0 < s1; c0 += BS) {
          const int nch = (int)min((int64_t)BS, s1 - c0);
          __syncthreads();
          if (tid < nch) {
            s_x[tid] = a.sx[c0 + tid] + shx;
            s_y[tid] = a.sy[c0 + tid] + shy;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              const double q = a.sq[((size_t)v * NC + c) * a.n_src + c0 + tid];
              s_q[c][tid] = q;
              s_q32[c][tid] = (float)q;
            }
          }
          __syncthreads();
          // r = 0 (a target that is a source) can only occur in the piece
          // that holds the target's own box, unshifted
          if (own) leaf_pairs<K, MIXED, true, BS>(nch, tx, ty, s_x, s_y, s_q, s_q32, sc, ksh, beta, r2_self, acc);
          else leaf_pairs<K, MIXED, false, BS>(nch, tx, ty, s_x, s_y, s_q, s_q32, sc, ksh, beta, r2_self, acc);
        }
      }
    }
    if (act) {
      if constexpr (NLOG > 0) {
        if constexpr (K == PFMM_LAPLACE) { acc[1] *= sc; acc[2] *= sc; }
        else { acc[4] *= sc; acc[5] *= sc; acc[6] *= sc; acc[7] *= sc; }
      }
      double d[NO];
      fmm_outputs<K>(acc, d, a.beta, MIXED ? 0.69314718055994530942 : 1.0);
#pragma unroll
      for (int c = 0; c < NO; ++c) a.part[((size_t)v * NO + c) * a.n_trg + k] = o[c] + d[c];
    }
  }
}

// ---------------------------------------------------------------------------
// Symmetric leaves, for targets that are the sources (one array, one order).
// A box's direct sum is split into its own box (one-sided, as above) and its
// four forward neighbours: the row above (i - 1 .. i + 1) and the box to the
// right. A pair of the box and a forward neighbour is evaluated once for both
// ends: the sums at the box's points go into its result, the sums at the
// neighbour's points into M, one slot per direction in which a point sees
// the box (slots 0..2: the row below, i - 1 .. i + 1; slot 3: the box to the
// left), and fmm_leaf_sym_add adds a point's slots to its result in that
// order. Each point is written to one slot by one block, so no atomics are
// needed and the result is deterministic.
//
// The four forward boxes form one stream of sources (each with its image
// shift), cut into tiles of 64. A wavefront takes its 64 points against a tile
// in 64 steps, lane l pairing its point with source (l + s) mod 64 at step s:
// its own sums stay in the lane, the sums at the sources move one lane down
// per step (a wavefront rotation), so that source b's sum is always in the
// lane that pairs with b next, and after 64 steps it is back in lane b.
// Mixed: the moving sums are FP32 over 16 steps, then added to FP64 sums in
// lane b (one cross-lane read per 16 steps); the log terms move in FP64.
// ---------------------------------------------------------------------------
// the value held by lane l + 1 (lane 0's for lane 63): DPP wave_rol:1, every
// lane of the wavefront active
__device__ __forceinline__ float rot_next(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ double rot_next(double x) {
  const long long u = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffll), 0x134, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0x134, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}

// forward box f (0..2: the row above, i - 1 .. i + 1; 3: the box to the
// right): its lattice offset and the slot in which its points see this box
__device__ __forceinline__ void fwd_offset(int f, int& di, int& dj) {
  di = f < 3 ? f - 1 : 1;
  dj = f < 3 ? 1 : 0;
}
__device__ __forceinline__ int fwd_slot(int f) { return f < 3 ? 2 - f : 3; }

template <int K, bool MIXED, int BS>
__global__ __launch_bounds__(BS) void fmm_leaf_sym_kernel(FmmArgs a) {
  using real = typename std::conditional<MIXED, float, double>::type;
  constexpr int NC = Fk<K>::NC, NO = Fk<K>::NO, NA = Fk<K>::NA;
  constexpr int NLOG = (K != PFMM_YUKAWA && MIXED) ? NC : 0;   // log terms summed in FP64 per pair
  constexpr int NW = BS / 64;
  const FmmTree& t = a.t;
  const int P = t.P, P2 = P * P;
  const int box = blockIdx.x, v = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const Lvl lv = level_of(t, t.L);
  const int i = box % lv.n1, j = box / lv.n1;
  const int64_t gb = t.box_off[t.L] + box;
  const int64_t t0 = leaf_begin(a.tcnt, a.tnblk, box), t1 = leaf_end(a.tcnt, a.tnblk, box);
  if (t0 >= t1) return;                                   // uniform over the block
  __shared__ double s_s[FMM_PMAX], s_w[FMM_PMAX];
  __shared__ double s_F[NO * FMM_PMAX * FMM_PMAX];
  __shared__ double s_x[BS], s_y[BS], s_q[NC][BS];
  __shared__ float s_q32[NC][BS];
  __shared__ double s_col[NW][NA][64];
  __shared__ int64_t s_g0[FMM_SLOTS], s_len[FMM_SLOTS];
  __shared__ double s_shx[FMM_SLOTS], s_shy[FMM_SLOTS];
  cheb_load(a, P, s_s, s_w, nullptr);
  for (int n = tid; n < NO * P2; n += BS)
    s_F[n] = a.F[((size_t)gb * a.n_dens * NO + v * NO) * P2 + n];
  if (tid < FMM_SLOTS) {
    int di, dj;
    fwd_offset(tid, di, dj);
    const int I = i + di, J = j + dj;
    const int m = floordiv(I, lv.n1), n = floordiv(J, lv.n2);
    const int64_t B = (int64_t)posmod(J, lv.n2) * lv.n1 + posmod(I, lv.n1);
    s_g0[tid] = leaf_begin(a.scnt, a.snblk, B);
    s_len[tid] = leaf_end(a.scnt, a.snblk, B) - s_g0[tid];
    s_shx[tid] = m * t.d + n * t.xi;
    s_shy[tid] = n * t.eta;
  }
  __syncthreads();
  // the forward stream: boxes f = 0..3 one after the other
  int64_t b0[FMM_SLOTS + 1];
  b0[0] = 0;
#pragma unroll
  for (int f = 0; f < FMM_SLOTS; ++f) b0[f + 1] = b0[f] + s_len[f];
  const int64_t nf = b0[FMM_SLOTS];
  const real beta = (real)a.beta;
  const int ksh = NLOG > 0 ? level_shift(t, t.L) : 0;
  const double sc = ldexp(1.0, ksh);
  // stand-in r^2 of a guarded (r = 0) pair: the log shift's (Laplace, Stokes),
  // or x = beta r = 1 (Yukawa: the series branch, as the other pairs of a
  // fine leaf)
  const real r2_self = K == PFMM_YUKAWA ? (real)(1.0 / (a.beta * a.beta)) : (real)ldexp(1.0, 2 * ksh);
  const size_t qv = (size_t)v * NC * a.n_src;
  const double far = 1.0e3 * (t.d + fabs(t.xi) + t.eta);
  // pairs farther apart than a quarter of that involve padding (r^2 in the
  // scaled units of the differences); their stand-in r^2: the log shift's
  // (Laplace, Stokes) or (1 / beta)^2 (Yukawa: K0(1), K1(1))
  const real dead2 = (real)((0.25 * far * sc) * (0.25 * far * sc));
  const real r2_dead = r2_self;
  for (int64_t tc = t0; tc < t1; tc += BS) {
    const int64_t k = tc + tid;
    const bool act = k < t1;
    // a wavefront with no point of the box skips the pairs (its column sums
    // are zero)
    const bool idle = tc + 64 * wv >= t1;
    // an inactive lane sits far from every source (the forward stream lies
    // within two cells of the origin), with zero density
    const double tx = act ? a.tx[k] : far, ty = act ? a.ty[k] : far;
    double qa[NC];
    real qr[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      qa[c] = act ? a.sq[qv + (size_t)c * a.n_src + k] : 0.0;
      qr[c] = (real)qa[c];
    }
    double acc[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) acc[c] = 0.0;
    // own box, one-sided (r = 0 guarded)
    for (int64_t c0 = t0; c0 < t1; c0 += BS) {
      const int nch = (int)min((int64_t)BS, t1 - c0);
      __syncthreads();
      if (tid < nch) {
        s_x[tid] = a.sx[c0 + tid];
        s_y[tid] = a.sy[c0 + tid];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double q = a.sq[qv + (size_t)c * a.n_src + c0 + tid];
          s_q[c][tid] = q;
          s_q32[c][tid] = (float)q;
        }
      }
      __syncthreads();
      if (!idle) leaf_pairs<K, MIXED, true, BS>(nch, tx, ty, s_x, s_y, s_q, s_q32, sc, ksh, beta, r2_self, acc);
    }
    // forward stream, both ends of every pair
    for (int64_t c0 = 0; c0 < nf; c0 += BS) {
      const int nch = (int)min((int64_t)BS, nf - c0);
      const int nsub = (nch + 63) >> 6;
      __syncthreads();
      if (tid < nsub * 64) {
        const int64_t p = c0 + tid;
        const bool ok = tid < nch;
        const int f = (p >= b0[1]) + (p >= b0[2]) + (p >= b0[3]);
        const int64_t g = s_g0[f] + (p - b0[f]);
        // padding: far from every point (and from the inactive lanes), zero density
        s_x[tid] = ok ? a.sx[g] + s_shx[f] : -far;
        s_y[tid] = ok ? a.sy[g] + s_shy[f] : -far;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double q = ok ? a.sq[qv + (size_t)c * a.n_src + g] : 0.0;
          s_q[c][tid] = q;
          s_q32[c][tid] = (float)q;
        }
      }
      __syncthreads();
      for (int sub = 0; sub < nsub; ++sub) {
        const int base = sub * 64;
        double D[NA];                                      // sums at source base + lane (FP64)
#pragma unroll
        for (int c = 0; c < NA; ++c) D[c] = 0.0;
        if (!idle) {
          // lane l meets source (l + s) mod 64 of the tile at step s: it
          // holds that source's coordinates and densities, which move one
          // lane down per step together with the sums at the sources
          double xs = s_x[base + lane], ys = s_y[base + lane];
          real ws[NC];
          double wl[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            ws[c] = MIXED ? (real)s_q32[c][base + lane] : (real)s_q[c][base + lane];
            wl[c] = s_q[c][base + lane];
          }
          real pc[NA];                                     // moving sums at the sources
#pragma unroll
          for (int c = 0; c < NA; ++c) pc[c] = (real)0;
          for (int s16 = 0; s16 < 64; s16 += 16) {
            real pr[NA];                                   // this lane's sums over 16 sources
#pragma unroll
            for (int c = 0; c < NA; ++c) pr[c] = (real)0;
#pragma unroll 2
            for (int st = s16; st < s16 + 16; ++st) {
              const real dx = NLOG > 0 ? (real)(sc * (tx - xs)) : (real)(tx - xs);
              const real dy = NLOG > 0 ? (real)(sc * (ty - ys)) : (real)(ty - ys);
              real r2 = MIXED ? __builtin_fmaf(dx, dx, dy * dy) : dx * dx + dy * dy;
              // a pair with a padding source or an inactive lane (weight
              // zero, far away) is evaluated at a harmless r^2 instead (the
              // small-argument branch, log shift cancelled)
              r2 = r2 > dead2 ? r2_dead : r2;
              real va, vb;
              pair_vals<K, real>(r2, beta, va, vb);
              pair_acc<K, (NLOG > 0), real>(va, vb, dx, dy, ws[0], ws[NC - 1], pr);
              pair_acc<K, (NLOG > 0), real>(va, vb, -dx, -dy, qr[0], qr[NC - 1], pc);
              if constexpr (NLOG > 0) {
                const double lgs = (double)va - 2.0 * ksh;
                acc[0] = fma(wl[0], lgs, acc[0]);
                D[0] = fma(qa[0], lgs, D[0]);
                if constexpr (NC > 1) {
                  acc[1] = fma(wl[NC - 1], lgs, acc[1]);
                  D[1] = fma(qa[NC - 1], lgs, D[1]);
                }
#pragma unroll
                for (int c = 0; c < NLOG; ++c) D[c] = rot_next(D[c]);
              }
#pragma unroll
              for (int c = NLOG; c < NA; ++c) pc[c] = rot_next(pc[c]);
              xs = rot_next(xs);
              ys = rot_next(ys);
#pragma unroll
              for (int c = 0; c < NC; ++c) {
                ws[c] = rot_next(ws[c]);
                if constexpr (NLOG > 0) wl[c] = rot_next(wl[c]);
              }
            }
#pragma unroll
            for (int c = NLOG; c < NA; ++c) acc[c] += (double)pr[c];
            if constexpr (MIXED) {
              // the moving sum of source base + lane sits in lane - s16 - 16
              const int from = (lane - s16 - 16) & 63;
#pragma unroll
              for (int c = NLOG; c < NA; ++c) {
                D[c] += (double)__shfl(pc[c], from);
                pc[c] = 0.0f;
              }
            }
          }
          if constexpr (!MIXED) {
#pragma unroll
            for (int c = 0; c < NA; ++c) D[c] = (double)pc[c];
          }
        }
#pragma unroll
        for (int c = 0; c < NA; ++c) s_col[wv][c][lane] = D[c];
        __syncthreads();
        if (tid < 64 && base + tid < nch) {
          double A[NA];
#pragma unroll
          for (int c = 0; c < NA; ++c) {
            double x = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) x += s_col[w][c][tid];
            A[c] = x;
          }
          if constexpr (NLOG > 0) {
            if constexpr (K == PFMM_LAPLACE) { A[1] *= sc; A[2] *= sc; }
            else { A[4] *= sc; A[5] *= sc; A[6] *= sc; A[7] *= sc; }
          }
          double d[NO];
          fmm_outputs<K>(A, d, a.beta, MIXED ? 0.69314718055994530942 : 1.0);
          const int64_t p = c0 + base + tid;
          const int f = (p >= b0[1]) + (p >= b0[2]) + (p >= b0[3]);
          const int64_t g = s_g0[f] + (p - b0[f]);
          double* m = a.M + ((size_t)(fwd_slot(f) * a.n_dens + v) * NO) * a.n_trg + g;
          // a box with more points than the block visits the stream once per
          // chunk of them: the same thread adds to what it wrote before
#pragma unroll
          for (int c = 0; c < NO; ++c) m[(size_t)c * a.n_trg] = (tc == t0 ? 0.0 : m[(size_t)c * a.n_trg]) + d[c];
        }
        __syncthreads();
      }
    }
    if (act) {
      if constexpr (NLOG > 0) {
        if constexpr (K == PFMM_LAPLACE) { acc[1] *= sc; acc[2] *= sc; }
        else { acc[4] *= sc; acc[5] *= sc; acc[6] *= sc; acc[7] *= sc; }
      }
      double o[NO], d[NO];
#pragma unroll
      for (int c = 0; c < NO; ++c) o[c] = 0.0;
      leaf_local<NO>(t, lv, i, j, s_s, s_w, s_F, tx, ty, o);
      fmm_outputs<K>(acc, d, a.beta, MIXED ? 0.69314718055994530942 : 1.0);
#pragma unroll
      for (int c = 0; c < NO; ++c) a.part[((size_t)v * NO + c) * a.n_trg + k] = o[c] + d[c];
    }
  }
}

// adds to each point of a leaf box the slots written by its backward
// neighbours (grid: leaf boxes x densities); a slot whose neighbour box is
// empty was not written and is skipped
template <int NO>
__global__ __launch_bounds__(256) void fmm_leaf_sym_add(FmmArgs a) {
  const FmmTree& t = a.t;
  const int box = blockIdx.x, v = blockIdx.y;
  const Lvl lv = level_of(t, t.L);
  const int i = box % lv.n1, j = box / lv.n1;
  const int64_t t0 = leaf_begin(a.tcnt, a.tnblk, box), t1 = leaf_end(a.tcnt, a.tnblk, box);
  if (t0 >= t1) return;
  bool use[FMM_SLOTS];
#pragma unroll
  for (int f = 0; f < FMM_SLOTS; ++f) {
    // the box that sees this one in slot fwd_slot(f) lies at minus forward offset f
    int di, dj;
    fwd_offset(f, di, dj);
    const int64_t A = (int64_t)posmod(j - dj, lv.n2) * lv.n1 + posmod(i - di, lv.n1);
    use[fwd_slot(f)] = leaf_end(a.scnt, a.snblk, A) > leaf_begin(a.scnt, a.snblk, A);
  }
  for (int64_t k = t0 + threadIdx.x; k < t1; k += 256) {
#pragma unroll
    for (int c = 0; c < NO; ++c) {
      double* out = a.part + ((size_t)v * NO + c) * a.n_trg + k;
      double x = *out;
#pragma unroll
      for (int sl = 0; sl < FMM_SLOTS; ++sl)
        if (use[sl]) x += a.M[((size_t)(sl * a.n_dens + v) * NO + c) * a.n_trg + k];
      *out = x;
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int fmm_order(int kernel, int precision, double tol) {
  // interpolation error of the near part measured against its direct sum
  // (uniform points, hexagonal cell, the worst of the cells tried): about
  // 1.5e-6 (Laplace, Yukawa) and 1e-5 (Stokes) at P = 8, falling by 4.5 and
  // 3.7 per added point; P is taken so that it stays below tol / 10
  (void)precision;
  const double e8 = kernel == PFMM_STOKES ? 1.0e-5 : 1.5e-6;
  const double rate = kernel == PFMM_STOKES ? 3.7 : 4.5;
  const double need = std::log(e8 / (0.1 * tol)) / std::log(rate);
  int P = 8 + (int)std::ceil(std::max(need, -4.0));
  return std::min(std::max(P, 4), FMM_PMAX);
}

void fmm_tree(const pfmm_plan_s* p, int64_t ns, int64_t nt, FmmTree& t) {
  const Geometry& g = p->geo;
  t.P = p->fmm_order;
  t.d = g.d; t.xi = g.xi; t.eta = g.eta;
  t.m0 = p->m0;
  // top grid k1 x k2 with boxes about as long along e1 as along e2 (the
  // interpolation error grows with the boxes' aspect ratio): the fewest top
  // boxes whose sides differ by at most 10 %, else the closest with at most
  // 128 of them
  const double r = g.d / std::hypot(g.xi, g.eta);
  double best_dev = 1e300;
  t.k1 = t.k2 = 1;
  for (int n = 1; n <= 128; ++n)
    for (int k2 = 1; k2 <= n; ++k2) {
      if (n % k2) continue;
      const int k1 = n / k2;
      const double dev = std::fabs(std::log(r * k2 / k1));
      if (dev < best_dev - 1e-12) { best_dev = dev; t.k1 = k1; t.k2 = k2; }
    }
  for (int n = 1; n <= 128; ++n) {
    bool found = false;
    for (int k2 = 1; k2 <= n && !found; ++k2) {
      if (n % k2) continue;
      const int k1 = n / k2;
      if (std::fabs(std::log(r * k2 / k1)) <= std::log(1.1)) { t.k1 = k1; t.k2 = k2; found = true; }
    }
    if (found) break;
  }
  // leaf level: neighbour pairs 9 ns nt / boxes against node pairs 27 P^4
  // per box (level 0: every non-neighbour of the super-grid), a list point
  // pair weighted by its cost relative to a leaf pair, measured on MI355X at
  // N = 2e5: tabulated lists (Laplace, Yukawa) cost 0.24 (Laplace FP64),
  // 0.36 (Yukawa mixed) and 0.08 (Yukawa FP64, whose leaf pairs take the
  // FP64 Bessel sequences) of a leaf pair; sampled lists (Stokes, and mixed
  // Laplace with its FP64 coarse levels) about one
  const bool mixed = p->precision == PFMM_MIXED;
  const double wm = p->kernel == PFMM_YUKAWA ? (mixed ? 0.36 : 0.08)
                    : (p->kernel == PFMM_LAPLACE && !mixed) ? 0.24 : 1.0;
  // symmetric leaves: the own box one-sided, the four forward boxes once for
  // both ends; their time relative to one-sided leaves, measured the same way
  const double wl = !fmm_symmetric_leaves(p) ? 1.0
                    : p->kernel == PFMM_YUKAWA ? (mixed ? 0.70 : 0.56)
                    : p->kernel == PFMM_LAPLACE ? (mixed ? 0.84 : 0.59) : (mixed ? 1.16 : 0.66);
  const double P4 = wm / wl * std::pow((double)t.P, 4);
  const double top = (double)t.k1 * t.k2;
  const double lvl0 = top * std::max(0.0, 3.0 * (2 * t.m0 + 1) * top - 9.0) * P4;
  double best = 0;
  int bestL = 0;
  for (int L = 0; L <= FMM_MAX_LEVEL; ++L) {
    const double leaves = top * std::pow(4.0, L);
    if (leaves > 4.0e6) break;
    double m2l = lvl0;
    for (int l = 1; l <= L; ++l) m2l += 27.0 * top * std::pow(4.0, l) * P4;
    const double cost = 9.0 * (double)ns * (double)nt / leaves + m2l;
    if (L == 0 || cost < best) { best = cost; bestL = L; }
  }
  t.L = bestL;
  if (p->tune_fmm_level > 0) {
    t.L = p->tune_fmm_level;
    while (t.L > 0 && top * std::pow(4.0, t.L) > 4.0e6) --t.L;
  }
  int64_t off = 0;
  for (int l = 0; l <= t.L; ++l) {
    t.box_off[l] = off;
    off += ((int64_t)t.k1 << l) * ((int64_t)t.k2 << l);
  }
  t.box_off[t.L + 1] = off;
}

// The M2L launches: box ranges (level 0 apart from the others, whose lists
// are longer; FP64 levels apart from FP32 ones) and for each the number of
// slices its interaction lists are split into, so that a launch has about
// FMM_M2L_BLOCKS blocks per density. Level 0 of a 1 x 1 top grid has an
// empty list.
struct M2lPart {
  int64_t lo, hi;
  int maxlist, S, per;
  bool f32;
};
// mixed: FP32 samples on every level for Yukawa (no log terms: its coarse
// levels measured the same error in FP32), the two finest otherwise
static bool level_f32(const FmmTree& t, int kernel, bool mixed, int l) {
  return mixed && (kernel == PFMM_YUKAWA || l >= t.L - FMM_F32_LEVELS + 1);
}

// the sampled (not tabulated) M2L of boxes below b_end
// The sampled boxes are every box outside the tabulated range [t_lo, t_hi)
// (out: at most M2L_MAX_PARTS parts).
constexpr int M2L_MAX_PARTS = 8;
static int m2l_parts(const FmmTree& t, int kernel, bool mixed, M2lPart* out, int64_t t_lo, int64_t t_hi) {
  int l32 = 0;
  while (l32 <= t.L && !level_f32(t, kernel, mixed, l32)) ++l32;
  const int64_t end = fmm_boxes(t), split = t.box_off[l32];
  const int64_t top = t.box_off[1];
  const int list0 = (t.k1 * t.k2 > 1) ? 3 * (2 * t.m0 + 1) * t.k1 * t.k2 : 1;
  int n = 0;
  for (int f32 = 0; f32 < 2; ++f32) {
    const int64_t r0 = f32 ? split : 0, r1 = f32 ? end : split;
    // the range less the tabulated boxes: up to two pieces
    int64_t pc[2][2] = {{r0, r1}, {0, 0}};
    if (t_hi > t_lo && t_lo < r1 && t_hi > r0) {
      pc[0][1] = std::max(r0, t_lo);
      pc[1][0] = std::min(r1, t_hi);
      pc[1][1] = r1;
    }
    for (int q = 0; q < 4; ++q) {
      const int64_t b0 = pc[q >> 1][0], b1 = pc[q >> 1][1];
      const int part = q & 1;
      const int64_t lo = part == 0 ? b0 : std::max(b0, top), hi = part == 0 ? std::min(b1, top) : b1;
      if (hi <= lo) continue;
      M2lPart& m = out[n++];
      m.lo = lo; m.hi = hi; m.f32 = f32;
      m.maxlist = part == 0 ? list0 : 27;
      const int64_t nbox = hi - lo;
      m.S = (int)std::min<int64_t>(m.maxlist, std::max<int64_t>(1, FMM_M2L_BLOCKS / nbox));
      m.per = (m.maxlist + m.S - 1) / m.S;
      m.S = (m.maxlist + m.per - 1) / m.per;
    }
  }
  return n;
}

int64_t fmm_slice_doubles(const FmmTree& t, int kernel, bool mixed, int n_dens) {
  const int64_t per_box = (int64_t)n_dens * (kernel == PFMM_STOKES ? 6 : 3) * t.P * t.P;
  M2lPart parts[M2L_MAX_PARTS];
  const int n = m2l_parts(t, kernel, mixed, parts, 0, 0);
  int64_t need = 0;
  for (int k = 0; k < n; ++k)
    if (parts[k].S > 1) need = std::max(need, (int64_t)parts[k].S * (parts[k].hi - parts[k].lo) * per_box);
  // tabulated levels (fmm_table_layout's choice) write FMM_TAB_SLICES partial fields
  int64_t off[FMM_MAX_LEVEL + 1];
  if (fmm_table_layout(t, kernel, mixed, off) > 0)
    for (int l = 0; l <= t.L; ++l)
      if (off[l] >= 0) need = std::max(need, (int64_t)FMM_TAB_SLICES * (t.box_off[l + 1] - t.box_off[l]) * per_box);
  return need;
}

template <int K, bool MIXED>
static void m2l_launch(const FmmArgs& a, hipStream_t s, const M2lPart& m) {
  constexpr int NO = Fk<K>::NO;
  const FmmTree& t = a.t;
  const int threads = (t.P * t.P + 63) / 64 * 64;
  const int64_t per_box = (int64_t)a.n_dens * NO * t.P * t.P;
  const int64_t nbox = m.hi - m.lo;
  hipLaunchKernelGGL((fmm_m2l_kernel<K, MIXED>), dim3((unsigned)nbox, a.n_dens, m.S), dim3(threads), 0, s, a, m.lo,
                     nbox, m.per);
  if (m.S > 1) {
    const int64_t n = nbox * per_box;
    hipLaunchKernelGGL(fmm_slice_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, m.lo * per_box, n,
                       m.S);
  }
}

template <int K>
static void m2l_table_launch(const FmmArgs& a, hipStream_t s, int l) {
  constexpr int NO = Fk<K>::NO;
  const FmmTree& t = a.t;
  const int P2 = t.P * t.P;
  const int hn = (t.k1 << l) / 2 * ((t.k2 << l) / 2);
  const int n_nt = (hn + MM_BOXES - 1) / MM_BOXES, n_mt = (NO * P2 + MM_ROWS - 1) / MM_ROWS;
  const int per = 27 / FMM_TAB_SLICES;
  hipLaunchKernelGGL((fmm_m2l_mfma_kernel<K>), dim3(4 * n_nt, n_mt, FMM_TAB_SLICES * a.n_dens), dim3(256), 0, s, a, l,
                     per, n_nt);
  const int64_t per_box = (int64_t)a.n_dens * NO * P2;
  const int64_t n = (t.box_off[l + 1] - t.box_off[l]) * per_box;
  hipLaunchKernelGGL(fmm_slice_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                     t.box_off[l] * per_box, n, FMM_TAB_SLICES);
}

size_t fmm_table_layout(const FmmTree& t, int kernel, bool mixed, int64_t* off) {
  for (int l = 0; l <= FMM_MAX_LEVEL; ++l) off[l] = -1;
  const size_t P2 = (size_t)t.P * t.P;
  const size_t nc = kernel == PFMM_STOKES ? 2 : 1, no = kernel == PFMM_STOKES ? 6 : 3;
  size_t total = 0;
  // a contiguous range of levels, finest first; mixed Stokes keeps sampling
  // its FP32 levels (measured at N = 2e5: FP32 samples 0.55 ms for the two
  // finest levels against 0.95 ms of FP64 products), and tabulates the FP64
  // ones below them
  int top = t.L;
  if (kernel == PFMM_STOKES && mixed)
    while (top >= 1 && level_f32(t, kernel, mixed, top)) --top;
  for (int l = top; l >= 1; --l) {
    const int64_t boxes = ((int64_t)t.k1 << l) * ((int64_t)t.k2 << l);
    if (boxes < FMM_TAB_MIN_BOXES) break;
    const size_t bytes = (FMM_CLASSES * nc * P2 * no * P2 * 8 + 255) & ~(size_t)255;
    if (total + bytes > FMM_TAB_MAX_BYTES) break;
    off[l] = (int64_t)total;
    total += bytes;
  }
  return total;
}

void fmm_build_tables(int kernel, bool mixed, const FmmArgs& a, char* tab, hipStream_t s) {
  (void)mixed;
  const FmmTree& t = a.t;
  const int threads = (t.P * t.P + 63) / 64 * 64;
  const int nc = kernel == PFMM_STOKES ? 2 : 1;
  for (int l = 0; l <= t.L; ++l) {
    if (a.tab_off[l] < 0) continue;
    const dim3 grid(FMM_CLASSES, nc * t.P * t.P);
    double* base = (double*)(tab + a.tab_off[l]);
    if (kernel == PFMM_LAPLACE)
      hipLaunchKernelGGL((fmm_table_build_kernel<PFMM_LAPLACE>), grid, dim3(threads), 0, s, a, l, base);
    else if (kernel == PFMM_YUKAWA)
      hipLaunchKernelGGL((fmm_table_build_kernel<PFMM_YUKAWA>), grid, dim3(threads), 0, s, a, l, base);
    else
      hipLaunchKernelGGL((fmm_table_build_kernel<PFMM_STOKES>), grid, dim3(threads), 0, s, a, l, base);
  }
}

template <int K, bool MIXED>
static void launch_fmm_t(const FmmArgs& a, hipStream_t s, hipEvent_t* ev) {
  constexpr int NC = Fk<K>::NC, NO = Fk<K>::NO;
  const FmmTree& t = a.t;
  const int64_t nleaf = t.box_off[t.L + 1] - t.box_off[t.L];
  auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], s); };
  mark(0);
  hipLaunchKernelGGL(fmm_cheb_kernel, dim3(1), dim3(64), 0, s, a);
  hipLaunchKernelGGL(fmm_p2m_kernel<NC>, dim3((unsigned)nleaf, a.n_dens), dim3(FMM_CHUNK), 0, s, a);
  for (int l = t.L - 1; l >= 0; --l) {
    const int64_t nb = t.box_off[l + 1] - t.box_off[l];
    hipLaunchKernelGGL(fmm_m2m_kernel, dim3((unsigned)nb, a.n_dens * NC), dim3(256), 0, s, a, l, a.n_dens * NC);
  }
  mark(1);
  // tabulated levels: one contiguous range lt..lt1 - 1 (FP64 tables and
  // products); the others sampled
  int lt = 0, lt1 = 0;
  if (a.tab) {
    while (lt <= t.L && a.tab_off[lt] < 0) ++lt;
    lt1 = lt;
    while (lt1 <= t.L && a.tab_off[lt1] >= 0) ++lt1;
  }
  M2lPart parts[M2L_MAX_PARTS];
  const int np = m2l_parts(t, K, MIXED, parts, t.box_off[lt], t.box_off[lt1]);
  for (int k = 0; k < np; ++k)
    if (!parts[k].f32) m2l_launch<K, false>(a, s, parts[k]);
  for (int l = lt; l < lt1; ++l) m2l_table_launch<K>(a, s, l);
  mark(2);
  for (int k = 0; k < np; ++k)
    if (parts[k].f32) m2l_launch<K, true>(a, s, parts[k]);
  mark(3);
  for (int l = 0; l < t.L; ++l) {
    const int64_t nb = t.box_off[l + 2] - t.box_off[l + 1];
    hipLaunchKernelGGL(fmm_l2l_kernel, dim3((unsigned)nb, a.n_dens * NO), dim3(256), 0, s, a, l, a.n_dens * NO);
  }
  mark(4);
  // one thread per target: blocks sized to the mean leaf occupancy (a
  // leaf's targets beyond the block loop in further chunks)
  const double mean = (double)a.n_trg / (double)nleaf;
  const dim3 lg((unsigned)nleaf, a.n_dens);
  if (a.M) {
    if (mean <= 56) hipLaunchKernelGGL((fmm_leaf_sym_kernel<K, MIXED, 64>), lg, dim3(64), 0, s, a);
    else if (mean <= 112) hipLaunchKernelGGL((fmm_leaf_sym_kernel<K, MIXED, 128>), lg, dim3(128), 0, s, a);
    else hipLaunchKernelGGL((fmm_leaf_sym_kernel<K, MIXED, FMM_LEAF>), lg, dim3(FMM_LEAF), 0, s, a);
    hipLaunchKernelGGL((fmm_leaf_sym_add<Fk<K>::NO>), lg, dim3(256), 0, s, a);
  } else if (mean <= 56)
    hipLaunchKernelGGL((fmm_leaf_kernel<K, MIXED, 64>), dim3((unsigned)nleaf, a.n_dens), dim3(64), 0, s, a);
  else if (mean <= 112)
    hipLaunchKernelGGL((fmm_leaf_kernel<K, MIXED, 128>), dim3((unsigned)nleaf, a.n_dens), dim3(128), 0, s, a);
  else
    hipLaunchKernelGGL((fmm_leaf_kernel<K, MIXED, FMM_LEAF>), dim3((unsigned)nleaf, a.n_dens), dim3(FMM_LEAF), 0, s,
                       a);
  mark(5);
}

void launch_fmm(int kernel, bool mixed, const FmmArgs& a, hipStream_t s, hipEvent_t* ev) {
  if (a.n_trg <= 0) return;
  if (kernel == PFMM_LAPLACE)
    mixed ? launch_fmm_t<PFMM_LAPLACE, true>(a, s, ev) : launch_fmm_t<PFMM_LAPLACE, false>(a, s, ev);
  else if (kernel == PFMM_YUKAWA)
    mixed ? launch_fmm_t<PFMM_YUKAWA, true>(a, s, ev) : launch_fmm_t<PFMM_YUKAWA, false>(a, s, ev);
  else mixed ? launch_fmm_t<PFMM_STOKES, true>(a, s, ev) : launch_fmm_t<PFMM_STOKES, false>(a, s, ev);
}

}  // namespace pfmm
