// Internal plan structure and table layouts shared by the host planner and
// the device kernels of libpfmm. Not part of the public ABI.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

#include "pfmm.h"

namespace pfmm {

constexpr double PI = 3.14159265358979323846;
constexpr int MAX_IMAGES = 21;   // (2 m0 + 1) * 3 with m0 <= 3

// Near-field image shifts and canonical lattice, passed to kernels by value.
struct Geometry {
  double d, xi, eta;             // canonical lattice e1 = (d,0), e2 = (xi,eta)
  double rc, rs;                 // canonical = R * user, R = [[rc,-rs],[rs,rc]]
  int n_images;
  double img_x[MAX_IMAGES], img_y[MAX_IMAGES];
  // mixed Laplace/Stokes near field: coordinates are scaled by sigma = 2^k
  // (exact) so that sigma^2 * cell area ~ 1, which keeps |log2 r^2| small for
  // most pairs; log2 r^2 is then shifted by lg_shift = 2k, removed in FP64
  double sigma;
  int lg_shift;
  // symmetric mixed near field: the r^2 values of a run of consecutive images
  // are multiplied in FP32 and share one log2. Group g covers images
  // [lg_end[g-1], lg_end[g]) and starts its product at 2^lg_e0[g]; the plan
  // bounds every partial product away from FP32 overflow and underflow
  int n_lg;
  int lg_end[MAX_IMAGES];
  int lg_e0[MAX_IMAGES];
};

// Per south/north mode record (doubles), mode index m = m_lo + i:
//   [0] alpha_m = 2 pi m / d        [1] a_m (chi_m for Yukawa, |alpha_m| otherwise)
//   [2] Dr  [3] Di : scalar kernels  fac * T_m / (2 d a_m),  T_m = e^{-2Q}/(1-e^{-Q})
//                    Stokes          fac * T_m / (4 d)
//   [4] tau_r [5] tau_i : Stokes (2 - e^{-Q})/(1 - e^{-Q}); unused otherwise
//   fac = 1 for m = 0, 2 otherwise (modes -m are conjugates for real densities)
constexpr int SN_REC = 6;
// Per west/east node record (doubles). The west/east waves live in the
// west/east frame: canonical coordinates rotated by (ew_c, ew_s), in which
// e1 = (dx', dy') and e2 = (xi', eta') (Appendix A; the identity frame has
// dx' = d, dy' = 0, xi' = xi, eta' = eta):
//   [0] lambda  [1] kappa (sqrt(lambda^2+beta^2) for Yukawa, lambda otherwise)
//   scalar kernels: [2..3] DW = w R B/(2 pi kappa)  [4..5] DE = w conj(R B)/(2 pi kappa)
//   Stokes:         [2..3] pre = w R/(4 pi)  [4..5] B  [6..7] B'  [8..9] dx' P
//   a = kappa dx' - i lambda dy',  R = e^{-p a}/(1-e^{-a}), p = m0+1,
//   B = e^{-kappa xi' + i lambda eta'} + e^{kappa xi' - i lambda eta'} + 1,
//   B' = -e^{-lambda xi' + i lambda eta'} + e^{lambda xi' - i lambda eta'},
//   P = (p - (p-1) e^{-a})/(1 - e^{-a})
constexpr int EW_REC = 12;

// complex coefficients per wave (mode or node) and density:
//   scalar kernels: 2 (south|west, north|east)
//   Stokes: 8 = {c(2), e(2)} for south|west, then north|east
inline int coef_per_wave(int kernel) { return kernel == PFMM_STOKES ? 8 : 2; }

struct NufftParams {
  int m_gl;        // Gauss-Legendre lines in y
  int nf;          // fine grid points per period d
  int w;           // spreading kernel width (grid points)
  double es_beta;  // exponential-of-semicircle kernel shape parameter
  int es_deg;      // degree of the per-tap polynomials of the kernel
};

// Spreading kernel as polynomials: tap t (0..w) of a point whose grid offset
// is f = l0 - g + w/2 in [0, 1) has value sum_k c[t][k] u^k, u = 2f - 1;
// stored as ES_TAPS x ES_COEF doubles (fixed size, zero-padded)
constexpr int NUFFT_MAX_GRID = 1 << 20;   // NUFFT fine-grid points per line (two passes of <= 1024-point FFTs)
constexpr int ES_TAPS = 17;
constexpr int ES_COEF = 20;

}  // namespace pfmm

struct pfmm_plan_s {
  int kernel, precision, far_mode, m0, n_dens, self_exclude, check_neutral, profile;
  int mutual;                  // near field by symmetric pair evaluation (self targets)
  int near_none;               // far part only (near images left out)
  int near_fmm;                // near part by the FMM: 0 never, 1 always (P2), 2 for large N (AUTO)
  int fmm_order;               // its Chebyshev points per box dimension
  int tune_fmm_level;          // its leaf level (0: cost model)
  int tune_fmm_leaves;         // targets = sources: 0 symmetric leaves where they pay, 1 one-sided, 2 symmetric
  // tabulated M2L kernel samples of the FMM (device), built for the tree
  // fmm_tab_key = {L, k1, k2, device}; rebuilt when an evaluation's tree differs
  void* fmm_tab = nullptr;
  size_t fmm_tab_bytes = 0;
  int fmm_tab_key[4] = {-1, -1, -1, -1};
  double beta, tol, eps;
  pfmm::Geometry geo;
  int M, m_lo, n_sn;           // south/north modes m = m_lo..M
  int n_ew;                    // west/east nodes
  // west/east frame (Appendix A): canonical -> [[ew_c, -ew_s], [ew_s, ew_c]];
  // rotated so that e2 is vertical (xi' = 0) when the canonical frame would
  // need a wider near region, else the identity
  int ew_rotated;
  double ew_c, ew_s, ew_dx, ew_dy, ew_xi, ew_eta;
  int ew_rows;                 // west/east rows: 3 (n = -1, 0, 1) or 1 (singly periodic)
  int periodic;                // 2: doubly periodic (P2), 1: singly periodic in e1 (P1)
  std::vector<double> sn_tab;  // n_sn * SN_REC
  std::vector<double> ew_tab;  // n_ew * EW_REC
  std::vector<double> ew_nodes, ew_weights;
  // NUFFT path
  int use_nufft;
  pfmm::NufftParams nu;
  int nu_grid;                     // 0: default NUFFT grid, 1: doubled grid (set_nufft_grid)
  int64_t tune_near;               // near-field blocks target (0: default)
  std::vector<double> gl_nodes;    // ybar_k on [-eta/2, eta/2]
  std::vector<double> gl_bary;     // barycentric weights sigma_k
  std::vector<double> nu_deconv;   // 1/phihat(m) for m = 0..M (real, even kernel)
  std::vector<double> nu_poly;     // ES_TAPS * ES_COEF kernel polynomial coefficients
  // device copies (per device, uploaded lazily)
  int dev_id;
  double* d_tab;               // sn_tab | ew_tab | gl_nodes | gl_bary | nu_deconv | nu_poly | images
  size_t tab_img;              // offset in d_tab of img_x, img_y, then both times sigma
  size_t tab_doubles;
  // profiling: event triples (start, near done, end) of evaluations not yet read
  std::vector<void*> prof_events;
  std::vector<void*> prof_fmm_events;   // FMM near part: 6 events per evaluation (stage boundaries)
  // Stokes plans: a Laplace plan of the same lattice and options with 2 n_dens
  // density vectors, whose gradients give the pressure (pressure.hip)
  pfmm_plan_s* lap = nullptr;
};

namespace pfmm {
// host planner (plan.cpp)
int build_plan(int kernel, const double* e1, const double* e2, double tol,
               const pfmm_opts* opts, pfmm_plan_s* p);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// one evaluation with the plan's current n_dens (capi.hip)
size_t cell_workspace(pfmm_plan_s* p, int64_t ns, int64_t nt, int64_t forced_split);
int set_nufft_grid(pfmm_plan_s* p, int grid);
int eval_core(pfmm_plan_s* p, int64_t ns, const double* src_xy, const double* dens, int64_t nt,
              const double* trg_xy, double* out_pot, double* out_grad, void* workspace,
              size_t ws_bytes, void* hip_stream, int no_alloc = 0);
}  // namespace pfmm
