// Kernel argument structs and launch helpers (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "pfmm_internal.h"

namespace pfmm {

constexpr int NEAR_BLOCK = 256;   // threads (= targets) per near-field block
constexpr int NEAR_TILE = 256;    // sources per LDS tile
#ifndef PFMM_NEAR_FLUSH
#define PFMM_NEAR_FLUSH 16
#endif
#ifndef PFMM_NEAR_TPT
#define PFMM_NEAR_TPT 1
#endif
#ifndef PFMM_NEAR_BIN
#define PFMM_NEAR_BIN 1
#endif
constexpr int NEAR_FLUSH = PFMM_NEAR_FLUSH;  // FP32 partial-sum length before an FP64 flush (mixed)
constexpr int NEAR_TPT = PFMM_NEAR_TPT;      // targets per thread (single-density launches)
constexpr double R2MIN_F32 = 8.673617379884035e-19;   // 2^-60: r^2 clamp of the mixed Laplace/Stokes pair
constexpr int FAR_CHUNK = 2048;   // sources per far_R block

struct PrepArgs {
  int64_t n;
  const double* xy;          // [2][n] user frame
  double rc, rs, d, xi, eta;
  double *cx, *cy;           // canonical FP64
  float *hx, *lx, *hy, *ly;  // two-float copies (NULL unless mixed)
};

struct PrepDensArgs {
  int64_t n;
  int n_dens, stokes;
  const double* dens;        // user densities
  double rc, rs;
  double* out64;             // Stokes: rotated forces
  float* out32;              // FP32 copy (mixed), NULL otherwise
};

struct NearArgs {
  Geometry geo;
  int64_t n_src, n_trg, split_len;
  const double *sx, *sy;                 // FP64 sources
  const float *sxh, *sxl, *syh, *syl;    // two-float sources
  const double* q64;                     // densities [n_dens][nc][n_src]
  const float* q32;
  int dens0;                             // first density of this launch
  const double *tx, *ty;                 // FP64 targets in binned order
  const int* perm;                       // binned position -> original target index
  int self;                              // targets are the sources (same indices)
  double beta, r2min;
  double* part;                          // [split][n_dens*NOUT][n_trg]
  size_t part_stride;                    // doubles per split
};

struct SortArgs {
  int64_t n;
  const double *x, *y;       // canonical targets
  double x0, y0, inv_w, inv_h;
  int nbx, nby;
  int *key, *hist, *cursor, *perm;
  double *sx, *sy;           // binned copies
};

struct FarRArgs {
  int kernel, n_sn, n_ew, ncw, n_coef, n_dens;
  int skip_sn;               // south/north slots come from the NUFFT path (write zeros)
  int64_t n_src;
  const double* tab;         // sn records | ew records
  const double *sx, *sy;     // canonical sources
  const double* dens;        // canonical densities [n_dens][nc][n_src]
  double* part;              // [chunk][n_dens][n_coef] complex (2 doubles)
};

struct FarDArgs {
  int kernel, n_sn, n_ew, ncw, n_coef, n_dens, n_chunks;
  double eta, xi;
  const double* tab;
  const double* part;
  const double* extra;       // NUFFT south/north coefficients [n_dens][n_sn][ncw] or NULL
  double* w;                 // [n_dens][n_coef] complex
};

struct FarLArgs {
  int kernel, n_sn, n_ew, ncw, n_coef, n_dens, n_splits, nufft;
  int64_t n_trg;
  double d, eta, rc, rs;
  const double* tab;
  const double* w;
  const double *tx, *ty;     // canonical targets
  const double* near_part;   // [split][n_dens*NOUT][n_trg]
  size_t part_stride;
  const double* nu_val;      // NUFFT path: interpolated south/north field [n_dens*NOUT][n_trg]
  double *out_pot, *out_grad;
};

// launchers (kernels.hip)
void launch_prep_points(const PrepArgs& a, hipStream_t s);
void launch_prep_dens(const PrepDensArgs& a, hipStream_t s);
void launch_near(int kernel, bool mixed, int nd, const NearArgs& a, int n_splits, hipStream_t s);
void launch_sort_targets(const SortArgs& a, hipStream_t s);
void launch_fill_zero(double* p, int64_t n, hipStream_t s);
void launch_far_R(const FarRArgs& a, int n_chunks, hipStream_t s);
void launch_far_D(const FarDArgs& a, hipStream_t s);
void launch_far_L(const FarLArgs& a, hipStream_t s);

inline int near_nout(int kernel) { return kernel == PFMM_STOKES ? 6 : 3; }

}  // namespace pfmm
