// Kernel argument structs and launch helpers (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "pfmm_internal.h"

namespace pfmm {

constexpr int NEAR_BLOCK = 256;   // threads (= targets) per near-field block
constexpr int NEAR_TILE = 256;    // sources per LDS tile
#ifndef PFMM_MU_BLOCK
#define PFMM_MU_BLOCK 256
#endif
constexpr int MU_BLOCK = PFMM_MU_BLOCK;   // points per block of the symmetric near field (multiple of 256)
#ifndef PFMM_NEAR_FLUSH
#define PFMM_NEAR_FLUSH 16
#endif
#ifndef PFMM_NEAR_BIN
#define PFMM_NEAR_BIN 1
#endif
constexpr int NEAR_FLUSH = PFMM_NEAR_FLUSH;  // FP32 partial-sum length before an FP64 flush (mixed)
constexpr double R2MIN_F32 = 7.888609052210118e-31;   // 2^-100: r^2 guard of the mixed Laplace/Stokes pair
constexpr int FAR_R_BLOCK = 256;  // threads per far_R block: mode lanes x source slices
// mode lanes of a far_R block for n_w1 modes/nodes (incl. the moment slot):
// the smallest power of two >= n_w1 in [32, 256]; the other 256/lanes
// thread slices split the block's sources
// densities per far_R block (one plane-wave factor serves all of them)
inline int far_r_dgroup(int kernel, int n_dens) {
  return n_dens == 1 ? 1 : (kernel == PFMM_STOKES ? 2 : 4);
}
inline int far_r_lanes(int n_w1) {
  int l = 32;
  while (l < n_w1 && l < FAR_R_BLOCK) l *= 2;
  return l;
}

struct PrepArgs {
  int64_t n, ystride;        // y coordinates at xy[ystride + i]
  const double* xy;          // [2][*] user frame
  double rc, rs, d, xi, eta;
  int wrap_y;                // 0: singly periodic (wrap along e1 only)
  double *cx, *cy;           // canonical FP64
};

struct PrepDensArgs {
  int64_t n, in_stride;      // user density rows are in_stride apart
  int n_dens, stokes;
  const double* dens;        // user densities
  double rc, rs;
  double* out64;             // contiguous FP64 copy (Stokes: rotated forces) or NULL
  float* out32;              // FP32 copy (mixed), NULL otherwise
};

struct NearArgs {
  Geometry geo;
  int64_t n_src, n_trg, split_len;
  const double *sx, *sy;                 // FP64 sources
  const double* q64;                     // densities [n_dens][nc][n_src]
  const float* q32;
  int dens0;                             // first density of this launch
  const double *tx, *ty;                 // FP64 targets in binned order
  const int* perm;                       // binned position -> original target index
  int self;                              // targets are the sources (same indices)
  double beta, r2min;
  double rcut2;                          // screened kernel: an image whose source tile lies
                                         // farther than sqrt(rcut2) from all targets of the
                                         // block is skipped (scaled units; huge: never)
  const double *imx, *imy;               // image shifts (device, n_images each)
  const double* qsum;                    // mixed Laplace/Stokes: per split, sum of the
                                         // densities [split][qsum_stride] (NULL: no log shift)
  int qsum_stride;                       // n_dens * nc
  int diag;                              // 1: block t sums only the sources of the diag_len-point
                                         // tile that holds its targets (sources in binned order,
  int64_t diag_len;                      // self index = binned)
  int atomic_out;                        // 1: add results to part with FP64 atomics
  double* part;                          // [split][n_dens*NOUT][n_trg]
  size_t part_stride;                    // doubles per split
};

struct QsumArgs {
  int64_t n_src, split_len;
  int ncomp;                             // n_dens * nc
  const double* q64;                     // [ncomp][n_src]
  double* qsum;                          // [split][ncomp]
  double* qpart;                         // scratch [split][QSUM_PARTS][ncomp]
};
constexpr int QSUM_PARTS = 64;           // blocks per split in the first pass

struct SortArgs {
  int64_t n;
  const double *x, *y;       // canonical targets
  double x0, y0, inv_w, inv_h;
  int nbx, nby;
  int nblk;                  // point blocks of bp consecutive indices (stable placement)
  int64_t bp;
  int *key, *cnt, *perm;     // cnt: [bin][block] counts, then their exclusive prefix
  int* seg;                  // scratch: one int per SCAN_SEG entries of cnt
  double *sx, *sy;           // binned copies
  int lattice;               // 1: bins are nbx x nby boxes in lattice coordinates of the
  double d, xi, eta;         //    canonical cell (u2 = y / eta, u1 = (x - xi u2) / d), row by row
};

constexpr int SCAN_SEG = 4096;   // entries of the bin-count table per scan block

struct FarRArgs {
  int kernel, n_sn, n_ew, ncw, n_coef, n_dens;
  int skip_sn;               // south/north slots come from the NUFFT path (not computed here)
  int64_t n_src, chunk_len;  // sources per block (grid y = source chunks)
  int lanes;                 // far_r_lanes(n_sn + n_ew + 1)
  const double* tab;         // sn records | ew records
  double ew_c, ew_s;         // canonical -> west/east frame rotation
  const double *sx, *sy;     // canonical sources
  const double* dens;        // canonical densities [n_dens][nc][n_src]
  double* part;              // [chunk][n_dens][n_coef] complex (2 doubles)
};

struct FarDArgs {
  int kernel, n_sn, n_ew, ncw, n_coef, n_dens, n_chunks;
  double eta;                // canonical eta (south/north)
  double xi;                 // xi' of the west/east frame
  double ew_c, ew_s;         // canonical -> west/east frame rotation
  const double* tab;
  const double* part;
  const double* extra;       // NUFFT south/north coefficients [n_dens][n_sn][ncw] or NULL
  double* w;                 // [n_dens][n_coef] complex
};

struct FarLArgs {
  int kernel, n_sn, n_ew, ncw, n_coef, n_dens, n_splits, nufft;
  int64_t n_trg;
  double d, eta, rc, rs;
  double ew_c, ew_s;         // canonical -> west/east frame rotation
  int m0term;                // Laplace/Stokes m = 0 south/north term (doubly periodic only)
  const double* tab;
  const double* w;
  const double *tx, *ty;     // canonical targets in binned order
  const int* perm;           // binned position -> original index
  const double* near_part;   // [split][n_dens*NOUT][n_trg] in binned order
  size_t part_stride;
  const double* nu_val;      // NUFFT path: south/north field [n_dens*NOUT][n_trg], binned order
  double *out_pot, *out_grad;
  int64_t out_stride;        // output rows are out_stride apart (n_trg for one cell)
};

// symmetric near field for targets == sources: block
// (c, a) evaluates every pair (target tile a, source j in chunk c with j past
// tile a) and all images once, for both points; results are added with FP64
// atomics to acc, which already holds the tiles' own (diagonal) sums
struct MutualArgs {
  int n_images;
  const double *imx, *imy;               // image shifts times sigma (device, n_images each)
  double sigma;                          // coordinate scale (mixed Laplace/Stokes)
  double rcut2;                          // screened kernel cutoff (as in NearArgs)
  int n_lg;                              // log groups of the images (mixed Laplace/Stokes)
  int lg_end[MAX_IMAGES];                // one past the last image of each group
  float lg_p0[MAX_IMAGES];               // 2^e0: start of each group's r^2 product
  double lg_e0[MAX_IMAGES];              // e0, removed from each group's log2
  int64_t n, chunk_len;
  const double *x, *y;                   // canonical points in binned order
  const double* q64;                     // binned densities [n_dens][nc][n]
  const float* q32;                      // binned FP32 densities (mixed)
  int dens0;                             // first density of this launch
  double beta;
  double* acc;                           // [n_dens][NOUT][n] in binned order
};

// one cell of a batched near-field launch; array offsets are byte offsets
// into the batch workspace
struct BatchCell {
  NearArgs args;             // sizes, geometry, beta, split length, flags
  int kernel, n_dens, n_tiles;
  long long task0;           // first task of this cell in the one-sided / diagonal launch
  long long task0m;          // first task of this cell in the symmetric launch
  int64_t o_sx, o_sy, o_q64, o_q32, o_tx, o_ty, o_perm, o_part, o_qsum;
  // symmetric near field (self targets): n_tiles diagonal tasks in the first
  // launch, n_tiles * n_chunks (tile, chunk) tasks in the second; margs
  // pointers are set per task
  int mutual, n_chunks;
  int64_t o_qb64, o_qb32;
  MutualArgs margs;
};

struct BatchNearArgs {
  const BatchCell* recs;     // device array [n_cells], task0 ascending
  int n_cells;
  long long n_tasks;
  char* ws;
  unsigned long long* counter;   // zeroed before the launch
  unsigned long long* counter2;  // second symmetric launch (remainder densities), zeroed
  int n_dens, dens_begin, dens_end;
};

// launchers (kernels.hip)
void launch_prep_points(const PrepArgs& a, hipStream_t s);
void launch_prep_dens(const PrepDensArgs& a, hipStream_t s);
void launch_near(int kernel, bool mixed, int nd, const NearArgs& a, int n_splits, hipStream_t s);
void launch_sort_targets(const SortArgs& a, hipStream_t s);
// phase 0: one-sided and diagonal tasks; phase 1: symmetric (tile, chunk) tasks
void launch_near_batch(int kernel, bool mixed, int phase, const BatchNearArgs& b, int grid, hipStream_t s);
void launch_qsum(const QsumArgs& a, int n_splits, hipStream_t s);
void launch_near_mutual(int kernel, bool mixed, const MutualArgs& a, int n_dens, hipStream_t s);
// dst[c][k] = src[c][perm[k]] for c < ncomp (binned copies of the densities)
void launch_gather_dens(const double* src, const int* perm, int64_t n, int ncomp, double* dst64,
                        float* dst32, hipStream_t s);
void launch_fill_zero(double* p, int64_t n, hipStream_t s);
void launch_far_R(const FarRArgs& a, int n_chunks, hipStream_t s);
// part[0][i] = sum over chunks of part[chunk][i], i < n_cplx (complex entries)
void launch_far_sum(double* part, int n_chunks, int64_t n_cplx, hipStream_t s);
void launch_far_D(const FarDArgs& a, hipStream_t s);
void launch_far_L(const FarLArgs& a, hipStream_t s);

inline int near_nout(int kernel) { return kernel == PFMM_STOKES ? 6 : 3; }

}  // namespace pfmm
