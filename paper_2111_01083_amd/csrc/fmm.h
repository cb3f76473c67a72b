// Interpolation FMM for the near part (internal; fmm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "pfmm_internal.h"

namespace pfmm {

constexpr int FMM_PMAX = 20;          // Chebyshev points per dimension, at most
constexpr int FMM_MAX_LEVEL = 11;     // deepest leaf level
constexpr int FMM_CHUNK = 128;        // points per LDS chunk (P2M)
constexpr int FMM_LEAF = 256;         // threads (targets) and LDS sources per chunk of the leaf kernel
#ifndef PFMM_FMM_F32_LEVELS
#define PFMM_FMM_F32_LEVELS 2
#endif
constexpr int FMM_F32_LEVELS = PFMM_FMM_F32_LEVELS;   // mixed: levels (the finest) whose M2L samples the kernel in FP32
constexpr int64_t FMM_M2L_BLOCKS = 8192;  // M2L blocks per density aimed at by splitting interaction lists
constexpr double FMM_AUTO_PAIRS = 4294967296.0;   // AUTO near mode: FMM from N_S N_T >= 2^32
constexpr int FMM_AUTO_TOP = 16;      // ... and top grids of at most this many boxes

// The tree: level l has (k1 << l) x (k2 << l) boxes over the cell in lattice
// coordinates u = (u1, u2) in [-1/2, 1/2)^2 (x = u1 e1 + u2 e2), stored row by
// row (box = j n1 + i) after the boxes of the coarser levels. The boxes of
// the image cells m e1 + n e2 are those of the cell shifted by whole cells,
// so only the cell's own boxes carry expansions.
struct FmmTree {
  int P, L, k1, k2, m0;
  double d, xi, eta;                  // canonical lattice e1 = (d, 0), e2 = (xi, eta)
  int64_t box_off[FMM_MAX_LEVEL + 2]; // first box of each level; box_off[L + 1] = total
};

struct FmmArgs {
  FmmTree t;
  int n_dens;
  double beta;
  double rcut;                        // screened kernel: box pairs farther apart are skipped
  int64_t n_src, n_trg;
  const double *sx, *sy;              // sources in leaf-box order (canonical)
  const double* sq;                   // their densities [n_dens][nc][n_src]
  const double *tx, *ty;              // targets in leaf-box order
  const int *scnt, *tcnt;             // sort tables: leaf box k ends at cnt[(k + 1) nblk - 1]
  int snblk, tnblk;
  int* scount;                        // sources per box, every level [n_box]
  double* W;                          // equivalent densities [n_box][n_dens * nc][P^2]
  double* F;                          // local fields [n_box][n_dens * NOUT][P^2]
  double* Fp;                         // M2L partial fields of list slices (fmm_slice_doubles)
  double* Q;                          // total density of each box [n_box][n_dens * nc]
  // tabulated M2L: per level, byte offset into tab of its FP64 kernel
  // samples (-1: sampled on the fly)
  const char* tab;
  int64_t tab_off[FMM_MAX_LEVEL + 1];
  double* part;                       // near part [n_dens * NOUT][n_trg], leaf-box target order
  // Chebyshev points, barycentric weights and transfer matrices of order P
  // (FMM_CHEB_DOUBLES), computed once per evaluation by the first launch
  double* cheb;
  // symmetric leaves (targets are the sources): the sums at the points of a
  // box's forward neighbours, [FMM_SLOTS][n_dens * NOUT][n_trg]; NULL: one-sided
  double* M;
};

constexpr int FMM_SLOTS = 4;          // directions of the backward neighbours of a leaf box
constexpr int FMM_CHEB_DOUBLES = 2 * FMM_PMAX + 2 * FMM_PMAX * FMM_PMAX;

// the tree for n points: k1 x k2 top boxes and the leaf level from a cost
// model (pairs of the leaf neighbour sums against the node pairs of the
// interaction lists)
void fmm_tree(const pfmm_plan_s* p, int64_t n_src, int64_t n_trg, FmmTree& t);
inline int64_t fmm_boxes(const FmmTree& t) { return t.box_off[t.L + 1]; }
// leaves evaluated symmetrically (targets are the sources): by default for
// every kernel but mixed Stokes, whose FP32 pair costs less than the terms of
// its reverse and their lane moves (measured on MI355X at N = 2e5: 1.16x the
// one-sided time; 0.56..0.84x for the others), or as the tuning asks
inline bool fmm_symmetric_leaves(const pfmm_plan_s* p) {
  if (!p->self_exclude || p->tune_fmm_leaves == 1) return false;
  return p->tune_fmm_leaves == 2 || p->kernel != PFMM_STOKES || p->precision != PFMM_MIXED;
}
// Chebyshev points per dimension for a kernel, precision and tolerance
int fmm_order(int kernel, int precision, double tol);
// doubles of M2L slice scratch (partial local fields) an evaluation needs
int64_t fmm_slice_doubles(const FmmTree& t, int kernel, bool mixed, int n_dens);

// Tabulated M2L: the kernel samples between the Chebyshev points of two
// boxes of one level depend only on their offset class (dI, dJ) in
// [-3, 3]^2 minus [-1, 1]^2, so a level with enough boxes keeps them in an
// FP64 table of FMM_CLASSES x (nc P^2) x NOUT x P^2 entries built once per
// plan and tree, and its lists become FP64 matrix products on the matrix
// cores. fmm_table_layout fills off (bytes per level, -1: not tabulated) and
// returns the total bytes (0: none); fmm_build_tables launches the builds on
// s.
constexpr int FMM_CLASSES = 49;            // 7 x 7 offsets (the inner 3 x 3 unused)
constexpr int64_t FMM_TAB_MIN_BOXES = 64;  // levels with fewer boxes sample on the fly
constexpr size_t FMM_TAB_MAX_BYTES = (size_t)1 << 30;
constexpr int FMM_TAB_SLICES = 9;          // slices of the 27 classes (3 each), summed in order
#ifndef PFMM_FMM_TABLE_STOKES
#define PFMM_FMM_TABLE_STOKES 1
#endif
size_t fmm_table_layout(const FmmTree& t, int kernel, bool mixed, int64_t* off);
void fmm_build_tables(int kernel, bool mixed, const FmmArgs& a, char* tab, hipStream_t s);
// ev: NULL, or 6 events recorded on s at the stage boundaries (start,
// upward done, FP64 interaction lists done, FP32 ones done, downward done,
// leaves done)
void launch_fmm(int kernel, bool mixed, const FmmArgs& a, hipStream_t s, hipEvent_t* ev = nullptr);

}  // namespace pfmm
