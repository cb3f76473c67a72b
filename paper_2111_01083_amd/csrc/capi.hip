// C ABI entry points: plan lifetime, workspace layout and the launch
// sequence of one evaluation (prep -> near | far_R -> far_D -> far_L).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fmm.h"
#include "kernels.h"
#include "nufft.h"
#include "pfmm.h"
#include "pfmm_internal.h"

using namespace pfmm;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace carve-up for one cell; offsets in bytes from the workspace base.
struct Layout {
  size_t scx, scy, tcx, tcy, q32, dens_c, near_part, far_part, w, nufft, nu_val;
  size_t key, perm, stx, sty, cnt, seg;       // target binning
  int nblk;
  int64_t bp;
  size_t qsum, qpart;                         // per-split density sums (mixed Laplace/Stokes), scratch
  size_t qb64, qb32;                          // binned densities (symmetric near field)
  int mutual;                                 // symmetric near field in this evaluation
  int64_t mu_chunk;                           // its source chunk length
  int nbx, nby;
  double bin_w, bin_h;
  size_t total;
  int n_splits, n_chunks, n_coef;
  int64_t chunk_len;
  int64_t split_len;
  size_t part_stride;  // doubles per split
  // near part by the FMM: the tree, leaf-box order of the sources (their own
  // sort unless they are the targets), expansions and per-box source counts
  int fmm;
  FmmTree ft;
  size_t skey, sperm, scnt, sseg, ssx, ssy;
  int snblk;
  int64_t sbp;
  size_t fW, fF, fcount, fFp, fQ, fM, fcheb;
};

// point blocks of the counting sort for n points in nbins bins
static int64_t sort_blocks(int64_t nbins, int64_t n) {
  const int64_t base = std::min<int64_t>(std::min<int64_t>(256, std::max<int64_t>(1, (1 << 26) / nbins)),
                                         std::max<int64_t>(1, (n + 1023) / 1024));
  const int64_t one_pass = std::min<int64_t>(std::max<int64_t>(1, (n + 255) / 256),
                                             std::max<int64_t>(1, (1 << 21) / nbins));
  return std::max(base, one_pass);
}

void plan_layout(const pfmm_plan_s* p, int64_t ns, int64_t nt, Layout& L, int64_t forced_split = 0) {
  const bool mixed = p->precision == PFMM_MIXED;
  const int nc = p->kernel == PFMM_STOKES ? 2 : 1;
  const int no = near_nout(p->kernel);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
  L.scx = take(8 * ns);
  L.scy = take(8 * ns);
  if (p->self_exclude) { L.tcx = L.scx; L.tcy = L.scy; }
  else { L.tcx = take(8 * nt); L.tcy = take(8 * nt); }
  if (mixed) {
    L.q32 = take(4 * (size_t)p->n_dens * nc * ns);
  } else {
    L.q32 = 0;
  }
  L.dens_c = take(8 * (size_t)p->n_dens * nc * ns);   // contiguous FP64 densities (Stokes: rotated)
  // FMM near part: explicit, or AUTO for doubly periodic single cells with
  // many pairs (batched cells take the direct near field)
  L.fmm = (!p->near_none && p->periodic == 2 && forced_split == 0 && ns > 0 && nt > 0 &&
           (p->near_fmm == 1 || (p->near_fmm == 2 && (double)ns * (double)nt >= FMM_AUTO_PAIRS))) ? 1 : 0;
  if (L.fmm) {
    fmm_tree(p, ns, nt, L.ft);
    // AUTO: not for cells whose top grid needs many boxes (their level-0
    // interaction lists span the whole super-grid)
    if (p->near_fmm == 2 && L.ft.k1 * L.ft.k2 > FMM_AUTO_TOP) L.fmm = 0;
  }
  // target bins of about 64 points over the canonical cell's bounding box
  // (FMM: the leaf boxes, in lattice coordinates)
  {
    const double W = p->geo.d + std::fabs(p->geo.xi), H = p->geo.eta;
    const double nb = std::max(1.0, std::min((double)nt / 64.0, 4.0e6));
    const double h = std::sqrt(W * H / nb);
    L.nbx = std::max(1, (int)std::ceil(W / h));
    L.nby = std::max(1, (int)std::ceil(H / h));
    if (L.fmm) { L.nbx = L.ft.k1 << L.ft.L; L.nby = L.ft.k2 << L.ft.L; }
    L.bin_w = W / L.nbx;
    L.bin_h = H / L.nby;
    L.key = take(4 * nt); L.perm = take(4 * nt); L.stx = take(8 * nt); L.sty = take(8 * nt);
    // stable placement in blocks of bp consecutive points: at most 256
    // blocks, or more, down to one rank pass of 256 points per block, while
    // the count table stays within 2^21 entries
    const int64_t nbins = (int64_t)L.nbx * L.nby;
    L.nblk = (int)sort_blocks(nbins, nt);
    L.bp = std::max<int64_t>(1, (nt + L.nblk - 1) / L.nblk);
    L.cnt = take(4 * (size_t)L.nbx * L.nby * L.nblk);
    L.seg = take(4 * (((size_t)L.nbx * L.nby * L.nblk + SCAN_SEG - 1) / SCAN_SEG));
  }
  // source splits for the near field: aim for >= 2048 blocks in flight
  int64_t tiles = std::max<int64_t>(1, (nt + NEAR_BLOCK - 1) / NEAR_BLOCK);
  int64_t max_s = std::max<int64_t>(1, (ns + NEAR_TILE - 1) / NEAR_TILE);
  // blocks in flight: the tuned target, else 2048 (one-sided) / 8192 (symmetric)
  const int64_t target = p->tune_near > 0 ? p->tune_near : 0;
  int64_t S = std::min<int64_t>(std::min<int64_t>(((target ? target : 2048) + tiles - 1) / tiles, max_s), 64);
  S = std::max<int64_t>(S, 1);
  int64_t per = (ns + S - 1) / S;
  if (forced_split > 0) per = forced_split;
  // the symmetric near field needs targets == sources; its diagonal pass
  // writes a single partial row
  // (forced_split > 0: batched cell; its symmetric tasks use chunks of that length)
  L.mutual = (p->mutual && p->self_exclude && ns == nt && !L.fmm) ? 1 : 0;
  if (L.mutual || p->near_none || L.fmm) per = std::max<int64_t>(ns, 1);
  per = std::max<int64_t>(NEAR_TILE, (per + NEAR_TILE - 1) / NEAR_TILE * NEAR_TILE);
  L.split_len = per;
  L.n_splits = (int)std::max<int64_t>(1, (ns + per - 1) / per);
  L.part_stride = (size_t)p->n_dens * no * nt;
  L.qsum = (mixed && p->kernel != PFMM_YUKAWA && !L.fmm) ? take(8 * (size_t)L.n_splits * p->n_dens * nc) : 0;
  L.qpart = L.qsum ? take(8 * (size_t)L.n_splits * QSUM_PARTS * p->n_dens * nc) : 0;
  L.near_part = take(8 * L.part_stride * L.n_splits);
  L.qb64 = L.qb32 = 0;
  L.mu_chunk = 0;
  L.skey = L.sperm = L.scnt = L.sseg = L.ssx = L.ssy = L.fW = L.fF = L.fcount = L.fFp = L.fQ = L.fM = L.fcheb = 0;
  L.snblk = 0;
  L.sbp = 0;
  if (L.fmm) {
    // sources in leaf-box order: the sorted targets when they are the sources
    if (!p->self_exclude) {
      const int64_t nbins = (int64_t)L.nbx * L.nby;
      L.snblk = (int)sort_blocks(nbins, ns);
      L.sbp = std::max<int64_t>(1, (ns + L.snblk - 1) / L.snblk);
      L.skey = take(4 * ns); L.sperm = take(4 * ns); L.ssx = take(8 * ns); L.ssy = take(8 * ns);
      L.scnt = take(4 * (size_t)nbins * L.snblk);
      L.sseg = take(4 * (((size_t)nbins * L.snblk + SCAN_SEG - 1) / SCAN_SEG));
    }
    L.qb64 = take(8 * (size_t)p->n_dens * nc * ns);
    const size_t nbox = (size_t)fmm_boxes(L.ft), P2 = (size_t)L.ft.P * L.ft.P;
    L.fW = take(8 * nbox * p->n_dens * nc * P2);
    L.fF = take(8 * nbox * p->n_dens * no * P2);
    L.fcount = take(4 * nbox);
    L.fFp = take(8 * (size_t)fmm_slice_doubles(L.ft, p->kernel, mixed, p->n_dens));
    L.fQ = take(8 * nbox * p->n_dens * nc);
    if (fmm_symmetric_leaves(p)) L.fM = take(8 * (size_t)FMM_SLOTS * p->n_dens * no * nt);
    L.fcheb = take(8 * (size_t)FMM_CHEB_DOUBLES);
  }
  if (L.mutual) {
    L.qb64 = take(8 * (size_t)p->n_dens * nc * ns);
    L.qb32 = mixed ? take(4 * (size_t)p->n_dens * nc * ns) : 0;
    // about 8192 source chunks x target tiles in total (half of them empty)
    const int64_t tiles = std::max<int64_t>(1, (ns + MU_BLOCK - 1) / MU_BLOCK);
    const int64_t want = std::max<int64_t>(1, ((target ? target : 8192) * 256 / MU_BLOCK + tiles - 1) / tiles);
    int64_t cl = forced_split > 0 ? forced_split : std::max<int64_t>(1024, (ns + want - 1) / want);
    L.mu_chunk = (cl + 63) / 64 * 64;
  }
  L.n_coef = (p->n_sn + p->n_ew) * coef_per_wave(p->kernel) + 1;
  {
    // far_R: enough source chunks for about 1024 blocks (each block streams
    // its chunk once for all modes/nodes of its lanes)
    const int n_w1 = (p->use_nufft ? 0 : p->n_sn) + p->n_ew + 1, lanes = far_r_lanes(n_w1);
    const int64_t wblocks = (n_w1 + lanes - 1) / lanes;
    const int dg = far_r_dgroup(p->kernel, p->n_dens);
    const int64_t zb = (p->n_dens + dg - 1) / dg;
    const int64_t want = std::max<int64_t>(1, (1024 + wblocks * zb - 1) / (wblocks * zb));
    int64_t clen = std::max<int64_t>(256, (ns + want - 1) / want);
    clen = (clen + 255) / 256 * 256;
    L.chunk_len = clen;
    L.n_chunks = (int)std::max<int64_t>(1, (ns + clen - 1) / clen);
  }
  L.far_part = take(16 * (size_t)L.n_chunks * p->n_dens * L.n_coef);
  L.w = take(16 * (size_t)p->n_dens * L.n_coef);
  L.nufft = p->use_nufft ? take(nufft_workspace_bytes(p, ns, nt)) : 0;
  L.nu_val = p->use_nufft ? take(8 * L.part_stride) : 0;
  L.total = off;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? PFMM_OK : PFMM_EHIP; }

}  // namespace

extern "C" {

int pfmm_plan(int kernel, const double* e1, const double* e2, double tol, const pfmm_opts* opts,
              pfmm_plan_t* out) {
  if (!out) return PFMM_EINVAL;
  pfmm_plan_s* p = new (std::nothrow) pfmm_plan_s();
  if (!p) return PFMM_ENOMEM;
  int rc = build_plan(kernel, e1, e2, tol, opts, p);
  if (rc != PFMM_OK) { delete p; return rc; }
  if (kernel == PFMM_STOKES) {
    // the pressure's Laplace plan: same lattice and options, the force
    // components as 2 n_dens charge vectors, no checks or events of its own
    pfmm_opts lo{};
    lo.n_dens = 1;
    if (opts) lo = *opts;
    lo.n_dens = 2 * p->n_dens;
    lo.beta = 0.0;
    lo.check_neutral = 0;
    lo.profile = 0;
    pfmm_plan_s* lap = new (std::nothrow) pfmm_plan_s();
    if (!lap) { delete p; return PFMM_ENOMEM; }
    rc = build_plan(PFMM_LAPLACE, e1, e2, tol, &lo, lap);
    if (rc != PFMM_OK) { delete lap; delete p; return rc; }
    p->lap = lap;
  }
  *out = p;
  return PFMM_OK;
}

}  // extern "C"

// Near-field cutoff of the screened (Yukawa) kernel: a pair beyond r_c with
// e^{-beta r_c} = eps / 30 is dropped. For sources of uniform density the
// dropped part of a potential is about 1.25 e^{-beta r_c} of its norm
// (K0(x) ~ sqrt(pi / 2x) e^{-x}), i.e. 0.04 eps; the far field is truncated
// at eps the same way. Other kernels: no cutoff.
static double near_rcut2(const pfmm_plan_s* p) {
  if (p->kernel != PFMM_YUKAWA || !(p->beta > 0)) return 1.0e308;
  const double rc = std::log(30.0 / p->eps) / p->beta;
  return rc * rc;
}

// image groups of the symmetric mixed near field (one log2 per group)
static void set_log_groups(MutualArgs& m, const Geometry& g) {
  m.n_lg = g.n_lg;
  for (int i = 0; i < g.n_lg; ++i) {
    m.lg_end[i] = g.lg_end[i];
    m.lg_p0[i] = std::ldexp(1.0f, g.lg_e0[i]);
    m.lg_e0[i] = (double)g.lg_e0[i];
  }
}

// the plan's device table: sn | ew | GL nodes | barycentric weights |
// NUFFT deconvolution | kernel polynomials | images (plain, then times sigma)
static std::vector<double> plan_table(pfmm_plan_s* p) {
  std::vector<double> tab;
  tab.insert(tab.end(), p->sn_tab.begin(), p->sn_tab.end());
  tab.insert(tab.end(), p->ew_tab.begin(), p->ew_tab.end());
  tab.insert(tab.end(), p->gl_nodes.begin(), p->gl_nodes.end());
  tab.insert(tab.end(), p->gl_bary.begin(), p->gl_bary.end());
  tab.insert(tab.end(), p->nu_deconv.begin(), p->nu_deconv.end());
  tab.insert(tab.end(), p->nu_poly.begin(), p->nu_poly.end());
  p->tab_img = tab.size();
  const Geometry& g = p->geo;
  for (int s = 0; s < 2; ++s) {
    const double f = s ? g.sigma : 1.0;
    for (int i = 0; i < g.n_images; ++i) tab.push_back(g.img_x[i] * f);
    for (int i = 0; i < g.n_images; ++i) tab.push_back(g.img_y[i] * f);
  }
  tab.push_back(0.0);
  return tab;
}

// rewrite an uploaded table in place (same size; device pointers into it,
// e.g. in batch records, stay valid)
static int plan_refresh_device(pfmm_plan_s* p) {
  if (!p->d_tab) return PFMM_OK;
  std::vector<double> tab = plan_table(p);
  if (tab.size() != p->tab_doubles) return PFMM_EINVAL;
  return hipMemcpy(p->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess
             ? PFMM_OK : PFMM_EHIP;
}

// Fixed device workspace of pfmm_eval_static. Every device the library runs
// on holds its own copy for the life of the process. In host code `scratch`
// only names the symbol: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// passed to kernels.
static __device__ __align__(256) char scratch[PFMM_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of `scratch` on the current device
int static_workspace(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return PFMM_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PFMM_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PFMM_OK;
}
}  // namespace

extern "C" {

int pfmm_plan_upload(pfmm_plan_t p) {
  if (!p) return PFMM_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFMM_EHIP;
  if (p->d_tab && p->dev_id == dev) return PFMM_OK;
  std::vector<double> tab = plan_table(p);
  if (p->d_tab) { (void)hipFree(p->d_tab); p->d_tab = nullptr; }
  double* d = nullptr;
  if (hipMalloc(&d, tab.size() * sizeof(double)) != hipSuccess) return PFMM_ENOMEM;
  if (hipMemcpy(d, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return PFMM_EHIP;
  }
  p->d_tab = d;
  p->dev_id = dev;
  p->tab_doubles = tab.size();
  void* ws = nullptr;
  (void)static_workspace(&ws);   // set-up of pfmm_eval_static on this device (it retries and reports)
  return PFMM_OK;
}

int pfmm_plan_get_info(pfmm_plan_t p, pfmm_plan_info_t* info) {
  if (!p || !info) return PFMM_EINVAL;
  info->kernel = p->kernel;
  info->precision = p->precision;
  info->far_mode_used = p->far_mode;
  info->m0 = p->m0;
  info->n_dens = p->n_dens;
  info->self_exclude = p->self_exclude;
  info->d = p->geo.d; info->xi = p->geo.xi; info->eta = p->geo.eta;
  info->rot_cos = p->geo.rc; info->rot_sin = p->geo.rs;
  info->eps = p->eps;
  info->n_modes = p->n_sn > 0 ? p->M : 0;
  info->n_quad = p->n_ew;
  info->periodic = p->periodic;
  info->ew_rotated = p->ew_rotated; info->ew_cos = p->ew_c; info->ew_sin = p->ew_s;
  info->m_gl = p->nu.m_gl; info->nufft_nf = p->nu.nf; info->nufft_w = p->nu.w;
  info->n_images = p->geo.n_images;
  info->n_log_groups = p->geo.n_lg;
  info->fmm_order = (p->near_fmm && p->periodic == 2 && !p->near_none) ? p->fmm_order : 0;
  info->fmm_symmetric = (info->fmm_order > 0 && fmm_symmetric_leaves(p)) ? 1 : 0;
  return PFMM_OK;
}

int pfmm_plan_get_quadrature(pfmm_plan_t p, double* nodes, double* weights) {
  if (!p) return PFMM_EINVAL;
  if (nodes) std::copy(p->ew_nodes.begin(), p->ew_nodes.end(), nodes);
  if (weights) std::copy(p->ew_weights.begin(), p->ew_weights.end(), weights);
  return PFMM_OK;
}

int pfmm_plan_get_spread_kernel(pfmm_plan_t p, double* coef, int* deg, double* beta_es) {
  if (!p) return PFMM_EINVAL;
  if (coef) std::copy(p->nu_poly.begin(), p->nu_poly.end(), coef);
  if (deg) *deg = p->nu.es_deg;
  if (beta_es) *beta_es = p->nu.es_beta;
  return PFMM_OK;
}

int pfmm_plan_get_log_groups(pfmm_plan_t p, int* ends, int* e0) {
  if (!p) return PFMM_EINVAL;
  for (int g = 0; g < p->geo.n_lg; ++g) {
    if (ends) ends[g] = p->geo.lg_end[g];
    if (e0) e0[g] = p->geo.lg_e0[g];
  }
  return PFMM_OK;
}

size_t pfmm_workspace_bytes(pfmm_plan_t p, int64_t ns, int64_t nt) {
  if (!p || ns < 0 || nt < 0 || ns > PFMM_MAX_POINTS || nt > PFMM_MAX_POINTS) return 0;
  if (p->self_exclude) nt = ns;
  Layout L;
  plan_layout(p, ns, nt, L);
  return L.total;
}

int pfmm_eval(pfmm_plan_t p, int64_t ns, const double* src_xy, const double* dens, int64_t nt,
              const double* trg_xy, double* out_pot, double* out_grad, void* workspace,
              size_t ws_bytes, void* hip_stream) {
  return pfmm::eval_core(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, workspace, ws_bytes, hip_stream);
}

}  // extern "C"


extern "C" {

int pfmm_eval_static(pfmm_plan_t p, int64_t ns, const double* src_xy, const double* dens, int64_t nt,
                     const double* trg_xy, double* out_pot, double* out_grad, void* hip_stream) {
  if (!p || ns < 0 || nt < 0 || ns > PFMM_MAX_POINTS || nt > PFMM_MAX_POINTS) return PFMM_EINVAL;
  const size_t need = cell_workspace(p, ns, nt, 0);
  if (need > PFMM_STATIC_WORKSPACE_BYTES) return PFMM_EWORKSPACE;
  void* ws = nullptr;
  int rc = static_workspace(&ws);
  if (rc) return rc;
  return pfmm::eval_core(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, ws, PFMM_STATIC_WORKSPACE_BYTES,
                         hip_stream, 1);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One cell's evaluation as three phases (shared by pfmm_eval and the batch):
//   prep  -- canonical points, densities, binned targets
//   near  -- near-field partial sums (single launch per cell, or batched)
//   far   -- far_R (or NUFFT R) -> far_D -> (NUFFT L) -> far_L
// ---------------------------------------------------------------------------
namespace pfmm {

struct CellRun {
  pfmm_plan_s* p;
  int64_t ns, nt;
  Layout L;
  char* ws;
  int* perm;
};
static double* D_(const CellRun& r, size_t off) { return (double*)(r.ws + off); }

static void cell_prep(CellRun& r, const double* src_xy, int64_t src_stride, const double* dens,
                      int64_t dens_stride, const double* trg_xy, int64_t trg_stride, hipStream_t st) {
  pfmm_plan_s* p = r.p;
  const Layout& L = r.L;
  char* ws = r.ws;
  auto D = [&](size_t off) { return (double*)(ws + off); };
  auto F = [&](size_t off) { return (float*)(ws + off); };
  const Geometry& g = p->geo;
  const bool mixed = p->precision == PFMM_MIXED;
  PrepArgs pa{};
  pa.rc = g.rc; pa.rs = g.rs; pa.d = g.d; pa.xi = g.xi; pa.eta = g.eta; pa.wrap_y = p->periodic == 2;
  pa.n = r.ns; pa.ystride = src_stride; pa.xy = src_xy; pa.cx = D(L.scx); pa.cy = D(L.scy);
  launch_prep_points(pa, st);
  if (!p->self_exclude) {
    PrepArgs pt = pa;
    pt.n = r.nt; pt.ystride = trg_stride; pt.xy = trg_xy; pt.cx = D(L.tcx); pt.cy = D(L.tcy);
    launch_prep_points(pt, st);
  }
  PrepDensArgs pd{};
  pd.n = r.ns; pd.in_stride = dens_stride; pd.n_dens = p->n_dens; pd.stokes = p->kernel == PFMM_STOKES;
  pd.dens = dens; pd.rc = g.rc; pd.rs = g.rs;
  pd.out64 = D(L.dens_c);
  pd.out32 = mixed ? F(L.q32) : nullptr;
  launch_prep_dens(pd, st);
  if (L.qsum) {
    QsumArgs qa{};
    qa.n_src = r.ns; qa.split_len = L.split_len; qa.ncomp = p->n_dens * (p->kernel == PFMM_STOKES ? 2 : 1);
    qa.q64 = D(L.dens_c); qa.qsum = D(L.qsum); qa.qpart = D(L.qpart);
    launch_qsum(qa, L.n_splits, st);
  }
  SortArgs sa{};
  sa.n = r.nt; sa.x = D(L.tcx); sa.y = D(L.tcy);
  sa.x0 = -0.5 * (g.d + std::fabs(g.xi)); sa.y0 = -0.5 * g.eta;
  sa.inv_w = 1.0 / L.bin_w; sa.inv_h = 1.0 / L.bin_h; sa.nbx = L.nbx; sa.nby = L.nby;
  sa.key = (int*)(ws + L.key); sa.perm = (int*)(ws + L.perm);
  sa.cnt = (int*)(ws + L.cnt); sa.nblk = L.nblk; sa.bp = L.bp; sa.seg = (int*)(ws + L.seg);
  sa.sx = D(L.stx); sa.sy = D(L.sty);
  sa.lattice = L.fmm; sa.d = g.d; sa.xi = g.xi; sa.eta = g.eta;
  launch_sort_targets(sa, st);
  r.perm = sa.perm;
  const int ncomp = p->n_dens * (p->kernel == PFMM_STOKES ? 2 : 1);
  if (L.mutual)
    launch_gather_dens(D(L.dens_c), sa.perm, r.ns, ncomp, D(L.qb64), mixed ? F(L.qb32) : nullptr, st);
  if (L.fmm) {
    const int* sperm = sa.perm;
    if (!p->self_exclude) {
      SortArgs ss = sa;
      ss.n = r.ns; ss.x = D(L.scx); ss.y = D(L.scy);
      ss.key = (int*)(ws + L.skey); ss.perm = (int*)(ws + L.sperm);
      ss.cnt = (int*)(ws + L.scnt); ss.nblk = L.snblk; ss.bp = L.sbp; ss.seg = (int*)(ws + L.sseg);
      ss.sx = D(L.ssx); ss.sy = D(L.ssy);
      launch_sort_targets(ss, st);
      sperm = ss.perm;
    }
    launch_gather_dens(D(L.dens_c), sperm, r.ns, ncomp, D(L.qb64), nullptr, st);
  }
}

static NearArgs cell_near_args(const CellRun& r) {
  const pfmm_plan_s* p = r.p;
  const Layout& L = r.L;
  char* ws = r.ws;
  auto D = [&](size_t off) { return (double*)(ws + off); };
  auto F = [&](size_t off) { return (float*)(ws + off); };
  NearArgs na{};
  na.geo = p->geo;
  na.imx = p->d_tab + p->tab_img; na.imy = na.imx + p->geo.n_images;   // plan uploaded beforehand
  na.n_src = r.ns; na.n_trg = r.nt; na.split_len = L.split_len;
  na.sx = D(L.scx); na.sy = D(L.scy);
  if (p->precision == PFMM_MIXED) {
    na.q32 = F(L.q32);
  }
  na.q64 = D(L.dens_c);
  na.tx = D(L.stx); na.ty = D(L.sty); na.perm = (const int*)(ws + L.perm);
  na.self = p->self_exclude;
  na.beta = p->beta;
  na.r2min = R2MIN_F32;
  na.rcut2 = near_rcut2(p);
  na.qsum = L.qsum ? D(L.qsum) : nullptr;
  na.qsum_stride = p->n_dens * (p->kernel == PFMM_STOKES ? 2 : 1);
  na.part = D(L.near_part);
  na.part_stride = L.part_stride;
  return na;
}

static int cell_far(CellRun& r, double* out_pot, double* out_grad, int64_t out_stride, hipStream_t st) {
  pfmm_plan_s* p = r.p;
  const Layout& L = r.L;
  char* ws = r.ws;
  auto D = [&](size_t off) { return (double*)(ws + off); };
  const Geometry& g = p->geo;
  const int K = p->kernel;
  const int64_t ns = r.ns, nt = r.nt;
  const double* dens_c = D(L.dens_c);
  FarRArgs fr{};
  fr.kernel = K; fr.n_sn = p->n_sn; fr.n_ew = p->n_ew; fr.ncw = coef_per_wave(K);
  fr.n_coef = L.n_coef; fr.n_dens = p->n_dens; fr.n_src = ns; fr.tab = p->d_tab;
  fr.ew_c = p->ew_c; fr.ew_s = p->ew_s;
  fr.sx = D(L.scx); fr.sy = D(L.scy); fr.dens = dens_c; fr.part = D(L.far_part);
  fr.skip_sn = p->use_nufft; fr.chunk_len = L.chunk_len;
  fr.lanes = far_r_lanes((p->use_nufft ? 0 : p->n_sn) + p->n_ew + 1);
  const double* csn = nullptr;
  if (p->use_nufft) {
    int rc = nufft_R(p, ns, D(L.scx), D(L.scy), dens_c, ws + L.nufft, st, &csn);
    if (rc) return rc;
  }
  int d_chunks = 1;
  if (ns > 0) {
    launch_far_R(fr, L.n_chunks, st);
    d_chunks = L.n_chunks;
    if (L.n_chunks > 4) {
      launch_far_sum(fr.part, L.n_chunks, (int64_t)p->n_dens * L.n_coef, st);
      d_chunks = 1;
    }
  } else {
    launch_fill_zero(fr.part, 2 * (int64_t)p->n_dens * L.n_coef, st);
  }
  FarDArgs fd{};
  fd.kernel = K; fd.n_sn = p->n_sn; fd.n_ew = p->n_ew; fd.ncw = fr.ncw; fd.n_coef = L.n_coef;
  fd.n_dens = p->n_dens; fd.n_chunks = d_chunks; fd.eta = g.eta; fd.xi = p->ew_xi;
  fd.ew_c = p->ew_c; fd.ew_s = p->ew_s;
  fd.tab = p->d_tab; fd.part = fr.part; fd.extra = csn; fd.w = D(L.w);
  launch_far_D(fd, st);
  const double* nu_val = nullptr;
  if (p->use_nufft) {
    int rc = nufft_L(p, nt, D(L.stx), D(L.sty), D(L.w), L.n_coef, ws + L.nufft, st, &nu_val, D(L.nu_val));
    if (rc) return rc;
  }
  FarLArgs fl{};
  fl.kernel = K; fl.n_sn = p->n_sn; fl.n_ew = p->n_ew; fl.ncw = fr.ncw; fl.n_coef = L.n_coef;
  fl.n_dens = p->n_dens; fl.n_splits = ns > 0 ? L.n_splits : 1; fl.nufft = p->use_nufft; fl.n_trg = nt;
  fl.d = g.d; fl.eta = g.eta; fl.rc = g.rc; fl.rs = g.rs; fl.tab = p->d_tab; fl.w = D(L.w);
  fl.ew_c = p->ew_c; fl.ew_s = p->ew_s;
  fl.m0term = p->periodic == 2;
  fl.tx = D(L.stx); fl.ty = D(L.sty); fl.perm = (const int*)(ws + L.perm);
  fl.near_part = D(L.near_part); fl.part_stride = L.part_stride;
  fl.nu_val = nu_val; fl.out_pot = out_pot; fl.out_grad = out_grad; fl.out_stride = out_stride;
  launch_far_L(fl, st);
  return PFMM_OK;
}

size_t cell_workspace(pfmm_plan_s* p, int64_t ns, int64_t nt, int64_t forced_split) {
  Layout L;
  plan_layout(p, ns, p->self_exclude ? ns : nt, L, forced_split);
  return L.total;
}

int cell_setup(pfmm_plan_s* p, int64_t ns, int64_t nt, char* ws, int64_t forced_split, CellRun& r) {
  r.p = p; r.ns = ns; r.nt = nt; r.ws = ws; r.perm = nullptr;
  plan_layout(p, ns, nt, r.L, forced_split);
  return PFMM_OK;
}

}  // namespace pfmm

int pfmm::eval_core(pfmm_plan_t p, int64_t ns, const double* src_xy, const double* dens, int64_t nt,
                    const double* trg_xy, double* out_pot, double* out_grad, void* workspace,
                    size_t ws_bytes, void* hip_stream, int no_alloc) {
  if (!p || ns < 0 || nt < 0 || ns > PFMM_MAX_POINTS || nt > PFMM_MAX_POINTS) return PFMM_EINVAL;
  if (p->self_exclude && nt != ns) return PFMM_EINVAL;
  if (ns > 0 && (!src_xy || !dens)) return PFMM_EINVAL;
  if (nt > 0 && !p->self_exclude && !trg_xy) return PFMM_EINVAL;
  if (nt == 0 || (!out_pot && !out_grad)) return PFMM_OK;
  CellRun r;
  cell_setup(p, ns, nt, (char*)workspace, 0, r);
  if (!workspace || ws_bytes < r.L.total || ((uintptr_t)workspace & 255)) return PFMM_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = PFMM_OK;
  if (no_alloc) {
    // the static-workspace entry point: no upload, no host copy, no events
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PFMM_EHIP;
    if (!p->d_tab || p->dev_id != dev || p->check_neutral || p->profile) return PFMM_EINVAL;
  } else {
    rc = pfmm_plan_upload(p);
    if (rc) return rc;
  }
  const int nc = p->kernel == PFMM_STOKES ? 2 : 1;
  if (p->check_neutral && p->kernel != PFMM_YUKAWA && ns > 0) {
    std::vector<double> h((size_t)p->n_dens * nc * ns);
    if (hipStreamSynchronize(st) != hipSuccess) return PFMM_EHIP;
    if (hipMemcpy(h.data(), dens, h.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) return PFMM_EHIP;
    for (int v = 0; v < p->n_dens * nc; ++v) {
      double s = 0, a = 0;
      for (int64_t j = 0; j < ns; ++j) { s += h[(size_t)v * ns + j]; a += std::fabs(h[(size_t)v * ns + j]); }
      if (std::fabs(s) > 1e-12 * a) return PFMM_ENOT_NEUTRAL;
    }
  }
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  if (p->profile) {
    // timing only (read after a synchronisation): no system-scope fence,
    // which would write back and invalidate the caches the next kernels use
    for (int k = 0; k < 3; ++k)
      if (hipEventCreateWithFlags(&ev[k], hipEventDisableSystemFence) != hipSuccess) {
        for (int q = 0; q < k; ++q) (void)hipEventDestroy(ev[q]);
        return PFMM_EHIP;
      }
    p->prof_events.push_back(ev[0]); p->prof_events.push_back(ev[1]); p->prof_events.push_back(ev[2]);
  }
  cell_prep(r, src_xy, ns, dens, ns, trg_xy, nt, st);
  NearArgs na = cell_near_args(r);
  if (p->profile) (void)hipEventRecord(ev[0], st);
  if (p->near_none) {
    launch_fill_zero(na.part, (int64_t)r.L.part_stride, st);   // far part alone
  } else if (r.L.fmm) {
    const Layout& L = r.L;
    FmmArgs fa{};
    fa.t = L.ft;
    fa.n_dens = p->n_dens;
    fa.beta = p->beta;
    fa.rcut = p->kernel == PFMM_YUKAWA ? std::sqrt(near_rcut2(p)) : 1.0e300;
    fa.n_src = ns; fa.n_trg = nt;
    fa.tx = D_(r, L.stx); fa.ty = D_(r, L.sty);
    fa.tcnt = (const int*)(r.ws + L.cnt); fa.tnblk = L.nblk;
    if (p->self_exclude) {
      fa.sx = fa.tx; fa.sy = fa.ty; fa.scnt = fa.tcnt; fa.snblk = fa.tnblk;
    } else {
      fa.sx = D_(r, L.ssx); fa.sy = D_(r, L.ssy);
      fa.scnt = (const int*)(r.ws + L.scnt); fa.snblk = L.snblk;
    }
    fa.sq = D_(r, L.qb64);
    fa.scount = (int*)(r.ws + L.fcount);
    fa.W = D_(r, L.fW); fa.F = D_(r, L.fF); fa.Fp = D_(r, L.fFp); fa.Q = D_(r, L.fQ);
    // tabulated M2L: the plan keeps the tables of its last tree; another
    // tree rebuilds them (allocating: not in the allocation-free entry
    // point, which then samples every level)
    {
      const bool mixed = p->precision == PFMM_MIXED;
      const size_t tb = fmm_table_layout(L.ft, p->kernel, mixed, fa.tab_off);
      int dev = 0;
      (void)hipGetDevice(&dev);
      const int key[4] = {L.ft.L, L.ft.k1, L.ft.k2, dev};
      const bool have = p->fmm_tab && std::equal(key, key + 4, p->fmm_tab_key);
      if (tb > 0 && (have || !no_alloc)) {
        if (!have) {
          if (p->fmm_tab_bytes < tb || p->fmm_tab_key[3] != dev) {
            if (p->fmm_tab) (void)hipFree(p->fmm_tab);
            p->fmm_tab = nullptr;
            p->fmm_tab_bytes = 0;
            if (hipMalloc(&p->fmm_tab, tb) != hipSuccess) { p->fmm_tab = nullptr; return PFMM_EHIP; }
            p->fmm_tab_bytes = tb;
          }
          fa.tab = (const char*)p->fmm_tab;
          fmm_build_tables(p->kernel, mixed, fa, (char*)p->fmm_tab, st);
          std::copy(key, key + 4, p->fmm_tab_key);
        }
        fa.tab = (const char*)p->fmm_tab;
      } else {
        for (int l = 0; l <= FMM_MAX_LEVEL; ++l) fa.tab_off[l] = -1;
        fa.tab = nullptr;
      }
    }
    fa.part = na.part;
    fa.M = L.fM ? D_(r, L.fM) : nullptr;
    fa.cheb = D_(r, L.fcheb);
    hipEvent_t fev[6] = {};
    bool timed = false;
    if (p->profile) {
      timed = true;
      for (int k = 0; k < 6 && timed; ++k)
        if (hipEventCreateWithFlags(&fev[k], hipEventDisableSystemFence) != hipSuccess) {
          for (int q = 0; q < k; ++q) (void)hipEventDestroy(fev[q]);
          timed = false;
        }
      if (timed)
        for (int k = 0; k < 6; ++k) p->prof_fmm_events.push_back(fev[k]);
    }
    launch_fmm(p->kernel, p->precision == PFMM_MIXED, fa, st, timed ? fev : nullptr);
  } else if (ns > 0 && r.L.mutual) {
    // diagonal tiles (one-sided, writes the partial row), then every other
    // pair once for both of its points (atomic adds into the same row)
    const bool mixed = p->precision == PFMM_MIXED;
    NearArgs nd = na;
    nd.diag = 1;
    nd.diag_len = MU_BLOCK;
    nd.sx = D_(r, r.L.stx); nd.sy = D_(r, r.L.sty);
    nd.q64 = D_(r, r.L.qb64); nd.q32 = mixed ? (const float*)(r.ws + r.L.qb32) : nullptr;
    launch_near(p->kernel, mixed, p->n_dens, nd, 1, st);
    MutualArgs ma{};
    const Geometry& g = p->geo;
    ma.n_images = g.n_images;
    ma.imx = p->d_tab + p->tab_img + 2 * g.n_images; ma.imy = ma.imx + g.n_images;
    ma.sigma = g.sigma;
    ma.rcut2 = near_rcut2(p);
    set_log_groups(ma, g);
    ma.n = ns; ma.chunk_len = r.L.mu_chunk;
    ma.x = nd.sx; ma.y = nd.sy; ma.q64 = nd.q64; ma.q32 = nd.q32;
    ma.beta = p->beta;
    ma.acc = na.part;
    launch_near_mutual(p->kernel, mixed, ma, p->n_dens, st);
  } else if (ns > 0) {
    launch_near(p->kernel, p->precision == PFMM_MIXED, p->n_dens, na, r.L.n_splits, st);
  } else {
    launch_fill_zero(na.part, (int64_t)r.L.part_stride, st);
  }
  if (p->profile) (void)hipEventRecord(ev[1], st);
  rc = cell_far(r, out_pot, out_grad, nt, st);
  if (rc) return rc;
  if (p->profile) (void)hipEventRecord(ev[2], st);
  return hip_ok(hipGetLastError());
}

extern "C" {

int pfmm_plan_stage_times(pfmm_plan_t p, double* near_ms, double* total_ms, int* n_evals) {
  if (!p) return PFMM_EINVAL;
  double sn = 0, st = 0;
  int n = 0, rc = PFMM_OK;
  for (size_t k = 0; k + 2 < p->prof_events.size(); k += 3) {
    hipEvent_t a = (hipEvent_t)p->prof_events[k], b = (hipEvent_t)p->prof_events[k + 1];
    hipEvent_t c = (hipEvent_t)p->prof_events[k + 2];
    float t1 = 0, t2 = 0;
    if (hipEventSynchronize(c) != hipSuccess || hipEventElapsedTime(&t1, a, b) != hipSuccess ||
        hipEventElapsedTime(&t2, a, c) != hipSuccess)
      rc = PFMM_EHIP;
    sn += t1; st += t2; ++n;
    (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c);
  }
  p->prof_events.clear();
  if (near_ms) *near_ms = sn;
  if (total_ms) *total_ms = st;
  if (n_evals) *n_evals = n;
  return rc;
}

int pfmm_plan_fmm_stage_times(pfmm_plan_t p, double* stage_ms, int* n_evals) {
  if (!p) return PFMM_EINVAL;
  double acc[5] = {0, 0, 0, 0, 0};
  int n = 0, rc = PFMM_OK;
  for (size_t k = 0; k + 5 < p->prof_fmm_events.size(); k += 6) {
    hipEvent_t* e = (hipEvent_t*)&p->prof_fmm_events[k];
    if (hipEventSynchronize(e[5]) != hipSuccess) rc = PFMM_EHIP;
    for (int q = 0; q < 5; ++q) {
      float t = 0;
      if (hipEventElapsedTime(&t, e[q], e[q + 1]) != hipSuccess) rc = PFMM_EHIP;
      acc[q] += t;
    }
    for (int q = 0; q < 6; ++q) (void)hipEventDestroy(e[q]);
    ++n;
  }
  p->prof_fmm_events.clear();
  if (stage_ms) std::copy(acc, acc + 5, stage_ms);
  if (n_evals) *n_evals = n;
  return rc;
}

int pfmm_fmm_tree(pfmm_plan_t p, int64_t ns, int64_t nt, int* out) {
  if (!p || !out || ns < 0 || nt < 0 || ns > PFMM_MAX_POINTS || nt > PFMM_MAX_POINTS) return PFMM_EINVAL;
  Layout L;
  plan_layout(p, ns, p->self_exclude ? ns : nt, L);
  out[0] = L.fmm;
  out[1] = L.fmm ? L.ft.L : 0;
  out[2] = L.fmm ? L.ft.k1 : 0;
  out[3] = L.fmm ? L.ft.k2 : 0;
  out[4] = L.fmm ? L.ft.P : 0;
  return PFMM_OK;
}

void pfmm_destroy(pfmm_plan_t p) {
  if (!p) return;
  if (p->lap) pfmm_destroy(p->lap);
  for (void* e : p->prof_events) (void)hipEventDestroy((hipEvent_t)e);
  for (void* e : p->prof_fmm_events) (void)hipEventDestroy((hipEvent_t)e);
  if (p->fmm_tab) (void)hipFree(p->fmm_tab);
  if (p->d_tab) (void)hipFree(p->d_tab);
  delete p;
}

const char* pfmm_strerror(int code) {
  switch (code) {
    case PFMM_OK: return "success";
    case PFMM_EINVAL: return "invalid argument";
    case PFMM_EINVAL_LATTICE: return "lattice vectors not finite or linearly dependent";
    case PFMM_EINVAL_TOL: return "tolerance outside [1e-14, 1e-2]";
    case PFMM_EWORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case PFMM_EHIP: return "HIP runtime error";
    case PFMM_ENOT_NEUTRAL: return "densities are not neutral (Laplace/Stokes need zero net charge/force)";
    case PFMM_ENOMEM: return "out of memory for plan tables";
    default: return "unknown error";
  }
}

}  // extern "C"


// ---------------------------------------------------------------------------
// Autotuning: candidates timed with HIP events on the caller's inputs.
// ---------------------------------------------------------------------------
namespace {
// one warm-up and two timed evaluations; per-evaluation near and total ms
int time_eval(pfmm_plan_s* p, int64_t ns, const double* src_xy, const double* dens, int64_t nt, const double* trg_xy,
              double* out_pot, double* out_grad, void* ws, size_t ws_bytes, void* stream, double* near_ms,
              double* total_ms) {
  const int saved = p->profile;
  p->profile = 1;
  int rc = pfmm_plan_stage_times(p, nullptr, nullptr, nullptr);
  if (!rc) rc = eval_core(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, ws, ws_bytes, stream);
  if (!rc) rc = pfmm_plan_stage_times(p, nullptr, nullptr, nullptr);
  for (int k = 0; k < 2 && !rc; ++k)
    rc = eval_core(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, ws, ws_bytes, stream);
  double nm = 0, tm = 0;
  int cnt = 0;
  const int rc2 = pfmm_plan_stage_times(p, &nm, &tm, &cnt);
  p->profile = saved;
  if (rc) return rc;
  if (rc2) return rc2;
  *near_ms = nm / std::max(cnt, 1);
  *total_ms = tm / std::max(cnt, 1);
  return PFMM_OK;
}
}  // namespace

extern "C" {

int pfmm_plan_get_tuning(pfmm_plan_t p, pfmm_tuning_t* t) {
  if (!p || !t) return PFMM_EINVAL;
  t->near_blocks = p->tune_near;
  t->nufft_grid = p->nu_grid;
  t->fmm_level = p->tune_fmm_level;
  t->fmm_leaves = p->tune_fmm_leaves;
  return PFMM_OK;
}

int pfmm_plan_set_tuning(pfmm_plan_t p, const pfmm_tuning_t* t) {
  if (!p || !t || t->near_blocks < 0 || t->near_blocks > (1LL << 24)) return PFMM_EINVAL;
  if (t->fmm_level < 0 || t->fmm_level > FMM_MAX_LEVEL) return PFMM_EINVAL;
  if (t->fmm_leaves < 0 || t->fmm_leaves > 2) return PFMM_EINVAL;
  if (t->nufft_grid != p->nu_grid) {
    const int old = p->nu_grid;
    int rc = set_nufft_grid(p, t->nufft_grid);
    if (rc) { (void)set_nufft_grid(p, old); return rc; }
    rc = plan_refresh_device(p);
    if (rc) {   // keep the host tables on the grid the device still holds
      (void)set_nufft_grid(p, old);
      return rc;
    }
  }
  p->tune_near = t->near_blocks;
  p->tune_fmm_level = t->fmm_level;
  p->tune_fmm_leaves = t->fmm_leaves;
  return PFMM_OK;
}

int pfmm_autotune(pfmm_plan_t p, int64_t ns, const double* src_xy, const double* dens, int64_t nt,
                  const double* trg_xy, double* out_pot, double* out_grad, void* ws, size_t ws_bytes,
                  void* stream, pfmm_tune_report_t* report) {
  if (!p || ns <= 0 || nt <= 0 || (!out_pot && !out_grad)) return PFMM_EINVAL;
  pfmm_tuning_t cur{};
  pfmm_plan_get_tuning(p, &cur);
  double nm = 0, tm = 0;
  int rc = time_eval(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, ws, ws_bytes, stream, &nm, &tm);
  if (rc) return rc;
  const double start_ms = tm;
  int tried = 1;
  // near field: blocks in flight, or the FMM tree's leaf level
  Layout L0;
  plan_layout(p, ns, nt, L0);
  const bool mutual = p->mutual && p->self_exclude && ns == nt;
  const int64_t near_c[3] = {mutual ? 4096 : 1024, mutual ? 8192 : 2048, mutual ? 16384 : 4096};
  pfmm_tuning_t best = cur;
  double best_near = nm;
  const bool sym0 = fmm_symmetric_leaves(p);
  for (int k = 0; k < 3; ++k) {
    pfmm_tuning_t t = cur;
    if (L0.fmm) {
      if (k < 2) {
        t.fmm_level = L0.ft.L + (k ? 1 : -1);
        if (t.fmm_level < 1 || t.fmm_level > FMM_MAX_LEVEL) continue;
      } else {
        // targets = sources: the other leaf form (symmetric or one-sided)
        if (!p->self_exclude) break;
        t.fmm_leaves = sym0 ? 1 : 2;
      }
    } else {
      t.near_blocks = near_c[k];
      if (t.near_blocks == cur.near_blocks) continue;
    }
    if ((rc = pfmm_plan_set_tuning(p, &t))) return rc;
    if (cell_workspace(p, ns, nt, 0) > ws_bytes) continue;
    double n1, t1;
    if ((rc = time_eval(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, ws, ws_bytes, stream, &n1, &t1))) return rc;
    ++tried;
    if (n1 < best_near) { best_near = n1; best = t; }
  }
  if ((rc = pfmm_plan_set_tuning(p, &best))) return rc;
  cur = best;
  // NUFFT grid (the far part is the total minus the near field)
  if (p->use_nufft) {
    double n0, t0;
    if ((rc = time_eval(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, ws, ws_bytes, stream, &n0, &t0))) return rc;
    double best_far = t0 - n0;
    for (int g = 0; g < 2; ++g) {
      if (g == cur.nufft_grid) continue;
      pfmm_tuning_t t = cur;
      t.nufft_grid = g;
      if (pfmm_plan_set_tuning(p, &t) != PFMM_OK) continue;   // grid not available
      if (cell_workspace(p, ns, nt, 0) > ws_bytes) continue;
      double n1, t1;
      if ((rc = time_eval(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, ws, ws_bytes, stream, &n1, &t1))) return rc;
      ++tried;
      if (t1 - n1 < best_far) { best_far = t1 - n1; best = t; }
    }
    if ((rc = pfmm_plan_set_tuning(p, &best))) return rc;
  }
  // the outputs hold the result of the chosen tuning
  double nb, tb;
  if ((rc = time_eval(p, ns, src_xy, dens, nt, trg_xy, out_pot, out_grad, ws, ws_bytes, stream, &nb, &tb))) return rc;
  if (report) { report->n_tried = tried; report->default_ms = start_ms; report->best_ms = tb; }
  return PFMM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched evaluation: per-cell prep, one persistent near-field launch over the
// tasks (cell, target tile, source split) of every cell, per-cell far field.
// Optionally captured once into a hipGraph and replayed.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t BATCH_SPLIT = 8192;   // sources per near-field task
}

struct pfmm_batch_s {
  int n_cells, n_recs, n_dens, mixed, self_exclude, nc, use_graph;
  std::vector<pfmm_plan_s*> plans;
  std::vector<int64_t> soff, toff;
  std::vector<size_t> base;            // workspace offset of each cell
  size_t counter_off, total;
  // per kernel type: records [rec0, rec0 + n_recs), tasks of the one-sided /
  // diagonal launch and of the symmetric launch
  struct Group { int kernel, rec0, n_recs; long long n_tasks, n_tasks_m; int grid, grid_m; } groups[3];
  int n_groups;
  int64_t split;                        // sources per near-field task (chunk or split length)
  int grid_mult;                        // persistent blocks per compute unit
  std::vector<int> nu_grid;             // each plan's NUFFT grid when the layout was built
  BatchCell* d_recs;
  hipStream_t cap_stream;
  hipGraphExec_t exec;
  const void* cap_args[5];
  void* cap_ws;
};

// (Re)build a batch's workspace layout, task records and launch shapes for
// task length `split` and `grid_mult` persistent blocks per compute unit.
static int batch_build(pfmm_batch_s* b, int64_t split, int grid_mult) {
  const int n_cells = b->n_cells;
  // workspace: cells in order, then the task counter
  size_t off = 0;
  b->base.resize(n_cells);
  std::vector<CellRun> runs(n_cells);
  for (int c = 0; c < n_cells; ++c) {
    const int64_t ns = b->soff[c + 1] - b->soff[c], nt = b->toff[c + 1] - b->toff[c];
    b->base[c] = off;
    cell_setup(b->plans[c], ns, nt, nullptr, split, runs[c]);
    off += align_up(runs[c].L.total);
  }
  b->counter_off = off;
  b->total = off + 256;
  // task records, most expensive cells first
  std::vector<int> order(n_cells);
  for (int c = 0; c < n_cells; ++c) order[c] = c;
  auto cost = [&](int c) {
    return (double)(b->soff[c + 1] - b->soff[c]) * (double)(b->toff[c + 1] - b->toff[c]) * b->plans[c]->geo.n_images;
  };
  // one persistent launch per kernel type; within it, most expensive cells first
  std::stable_sort(order.begin(), order.end(), [&](int a, int bb) {
    if (b->plans[a]->kernel != b->plans[bb]->kernel) return b->plans[a]->kernel < b->plans[bb]->kernel;
    return cost(a) > cost(bb);
  });
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  std::vector<BatchCell> recs;
  long long task = 0, task_m = 0;
  b->n_groups = 0;
  auto close_group = [&]() {
    if (b->n_groups == 0) return;
    pfmm_batch_s::Group& gr = b->groups[b->n_groups - 1];
    gr.n_recs = (int)recs.size() - gr.rec0;
    gr.n_tasks = task;
    gr.n_tasks_m = task_m;
    gr.grid = (int)std::max<long long>(1, std::min<long long>(task, (long long)grid_mult * cus));
    gr.grid_m = (int)std::max<long long>(1, std::min<long long>(task_m, (long long)grid_mult * cus));
  };
  for (int c : order) {
    const CellRun& r = runs[c];
    if (r.ns == 0 || r.nt == 0) continue;
    if (b->n_groups == 0 || b->groups[b->n_groups - 1].kernel != b->plans[c]->kernel) {
      close_group();
      b->groups[b->n_groups++] = {b->plans[c]->kernel, (int)recs.size(), 0, 0, 0, 1, 1};
      task = 0; task_m = 0;
    }
    BatchCell bc{};
    CellRun rr = r;
    rr.ws = nullptr;
    bc.args = cell_near_args(rr);
    const size_t B = b->base[c];
    const Layout& L = r.L;
    const bool mixed = b->mixed;
    bc.o_sx = B + L.scx; bc.o_sy = B + L.scy;
    bc.o_q64 = B + L.dens_c; bc.o_q32 = mixed ? B + L.q32 : 0;
    bc.o_tx = B + L.stx; bc.o_ty = B + L.sty; bc.o_perm = B + L.perm; bc.o_part = B + L.near_part;
    bc.o_qsum = L.qsum ? B + L.qsum : 0;
    bc.kernel = b->plans[c]->kernel; bc.n_dens = b->n_dens;
    bc.n_tiles = (int)((r.nt + NEAR_BLOCK - 1) / NEAR_BLOCK);
    bc.task0 = task;
    bc.task0m = task_m;
    bc.mutual = L.mutual;
    if (L.mutual) {
      const Geometry& g = b->plans[c]->geo;
      MutualArgs& m = bc.margs;
      m.n_images = g.n_images;
      m.imx = b->plans[c]->d_tab + b->plans[c]->tab_img + 2 * g.n_images; m.imy = m.imx + g.n_images;
      m.sigma = g.sigma; m.rcut2 = near_rcut2(b->plans[c]); set_log_groups(m, g); m.n = r.ns; m.chunk_len = L.mu_chunk; m.beta = b->plans[c]->beta;
      bc.n_chunks = (int)((r.ns + L.mu_chunk - 1) / L.mu_chunk);
      bc.o_qb64 = B + L.qb64; bc.o_qb32 = mixed ? B + L.qb32 : 0;
      task += bc.n_tiles;
      task_m += (long long)bc.n_tiles * bc.n_chunks;
    } else {
      task += (long long)bc.n_tiles * L.n_splits;
    }
    recs.push_back(bc);
  }
  close_group();
  if (b->d_recs) { (void)hipFree(b->d_recs); b->d_recs = nullptr; }
  if (!recs.empty()) {
    if (hipMalloc(&b->d_recs, recs.size() * sizeof(BatchCell)) != hipSuccess) return PFMM_ENOMEM;
    if (hipMemcpy(b->d_recs, recs.data(), recs.size() * sizeof(BatchCell), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(b->d_recs); b->d_recs = nullptr; return PFMM_EHIP;
    }
  }
  b->n_recs = (int)recs.size();
  b->split = split; b->grid_mult = grid_mult;
  b->nu_grid.resize(n_cells);
  for (int c = 0; c < n_cells; ++c) b->nu_grid[c] = b->plans[c]->nu_grid;
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }   // task tables changed
  return PFMM_OK;
}

// A plan's NUFFT grid (pfmm_plan_set_tuning, pfmm_autotune) sets the size of
// its cell's NUFFT workspace and the launch shapes of its far field: when one
// changed since the layout was built, rebuild layout, task records and graph.
static int batch_refresh(pfmm_batch_s* b) {
  for (int c = 0; c < b->n_cells; ++c)
    if (b->plans[c]->nu_grid != b->nu_grid[c]) return batch_build(b, b->split, b->grid_mult);
  return PFMM_OK;
}

extern "C" {

int pfmm_batch_create(int n_cells, const pfmm_plan_t* plans, const int64_t* src_off, const int64_t* trg_off,
                      int use_graph, pfmm_batch_t* out) {
  if (n_cells <= 0 || !plans || !src_off || !out) return PFMM_EINVAL;
  pfmm_plan_s* p0 = plans[0];
  if (!p0) return PFMM_EINVAL;
  const int nc = p0->kernel == PFMM_STOKES ? 2 : 1;
  for (int c = 0; c < n_cells; ++c) {
    pfmm_plan_s* p = plans[c];
    // check_neutral needs a stream synchronisation, which a batch never does;
    // far-only plans have no near tasks; singly periodic cells are not batched
    if (!p || p->precision != p0->precision || p->n_dens != p0->n_dens || p->self_exclude != p0->self_exclude ||
        (p->kernel == PFMM_STOKES ? 2 : 1) != nc || p->check_neutral || p->near_none || p->periodic != 2 ||
        p->near_fmm == 1)
      return PFMM_EINVAL;
    if (src_off[c + 1] < src_off[c] || src_off[c + 1] - src_off[c] > PFMM_MAX_POINTS) return PFMM_EINVAL;
    if (!p0->self_exclude &&
        (!trg_off || trg_off[c + 1] < trg_off[c] || trg_off[c + 1] - trg_off[c] > PFMM_MAX_POINTS))
      return PFMM_EINVAL;
  }
  if (src_off[0] != 0 || (!p0->self_exclude && trg_off[0] != 0)) return PFMM_EINVAL;
  pfmm_batch_s* b = new (std::nothrow) pfmm_batch_s();
  if (!b) return PFMM_ENOMEM;
  b->n_cells = n_cells; b->n_dens = p0->n_dens; b->mixed = p0->precision == PFMM_MIXED;
  b->self_exclude = p0->self_exclude; b->nc = nc; b->use_graph = use_graph ? 1 : 0;
  b->plans.assign(plans, plans + n_cells);
  b->soff.assign(src_off, src_off + n_cells + 1);
  if (p0->self_exclude) b->toff = b->soff; else b->toff.assign(trg_off, trg_off + n_cells + 1);
  b->d_recs = nullptr; b->cap_stream = nullptr; b->exec = nullptr; b->cap_ws = nullptr;
  for (auto& a : b->cap_args) a = nullptr;
  for (int c = 0; c < n_cells; ++c) {
    int rc = pfmm_plan_upload(plans[c]);
    if (rc) { delete b; return rc; }
  }
  b->d_recs = nullptr;
  int rc = batch_build(b, BATCH_SPLIT, 4);
  if (rc) { delete b; return rc; }
  *out = b;
  return PFMM_OK;
}

size_t pfmm_batch_workspace_bytes(pfmm_batch_t b) {
  if (!b || batch_refresh(b) != PFMM_OK) return 0;
  return b->total;
}

}  // extern "C"

static int batch_launch(pfmm_batch_s* b, const double* src_xy, const double* dens, const double* trg_xy,
                        double* out_pot, double* out_grad, char* ws, hipStream_t st) {
  const int64_t S = b->soff[b->n_cells], T = b->toff[b->n_cells];
  std::vector<CellRun> runs(b->n_cells);
  for (int c = 0; c < b->n_cells; ++c) {
    const int64_t ns = b->soff[c + 1] - b->soff[c], nt = b->toff[c + 1] - b->toff[c];
    cell_setup(b->plans[c], ns, nt, ws + b->base[c], b->split, runs[c]);
    if (nt == 0) continue;
    cell_prep(runs[c], src_xy + b->soff[c], S, dens + b->soff[c], S,
              b->self_exclude ? nullptr : trg_xy + b->toff[c], T, st);
    if (ns == 0) launch_fill_zero((double*)(ws + b->base[c] + runs[c].L.near_part), (int64_t)runs[c].L.part_stride, st);
  }
  launch_fill_zero((double*)(ws + b->counter_off), 9, st);
  for (int gi = 0; gi < b->n_groups; ++gi) {
    const pfmm_batch_s::Group& gr = b->groups[gi];
    BatchNearArgs na{};
    na.recs = b->d_recs + gr.rec0;
    na.n_cells = gr.n_recs;
    na.ws = ws;
    na.n_dens = b->n_dens;
    na.n_tasks = gr.n_tasks;
    na.counter = (unsigned long long*)(ws + b->counter_off) + 3 * gi;
    launch_near_batch(gr.kernel, b->mixed, 0, na, gr.grid, st);
    na.n_tasks = gr.n_tasks_m;
    na.counter = (unsigned long long*)(ws + b->counter_off) + 3 * gi + 1;
    na.counter2 = (unsigned long long*)(ws + b->counter_off) + 3 * gi + 2;
    launch_near_batch(gr.kernel, b->mixed, 1, na, gr.grid_m, st);
  }
  for (int c = 0; c < b->n_cells; ++c) {
    if (runs[c].nt == 0) continue;
    int rc = cell_far(runs[c], out_pot ? out_pot + b->toff[c] : nullptr, out_grad ? out_grad + b->toff[c] : nullptr,
                      T, st);
    if (rc) return rc;
  }
  return hip_ok(hipGetLastError());
}

extern "C" {

int pfmm_eval_batch(pfmm_batch_t b, const double* src_xy, const double* dens, const double* trg_xy,
                    double* out_pot, double* out_grad, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!b) return PFMM_EINVAL;
  if (!src_xy || !dens || (!b->self_exclude && !trg_xy)) return PFMM_EINVAL;
  if (!out_pot && !out_grad) return PFMM_OK;
  int rc0 = batch_refresh(b);
  if (rc0) return rc0;
  if (!workspace || ws_bytes < b->total || ((uintptr_t)workspace & 255)) return PFMM_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  char* ws = (char*)workspace;
  if (!b->use_graph) return batch_launch(b, src_xy, dens, trg_xy, out_pot, out_grad, ws, st);
  const void* args[5] = {src_xy, dens, trg_xy, out_pot, out_grad};
  bool same = b->exec && b->cap_ws == workspace;
  for (int k = 0; k < 5 && same; ++k) same = args[k] == b->cap_args[k];
  if (!same) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return PFMM_EHIP;
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return PFMM_EHIP;
    int rc = batch_launch(b, src_xy, dens, trg_xy, out_pot, out_grad, ws, b->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
    if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess || !graph) return PFMM_EHIP;
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { b->exec = nullptr; return PFMM_EHIP; }
    for (int k = 0; k < 5; ++k) b->cap_args[k] = args[k];
    b->cap_ws = workspace;
  }
  return hip_ok(hipGraphLaunch(b->exec, st));
}

int pfmm_batch_autotune(pfmm_batch_t b, const double* src_xy, const double* dens, const double* trg_xy,
                        double* out_pot, double* out_grad, void* workspace, size_t ws_bytes, void* hip_stream,
                        pfmm_tune_report_t* report) {
  if (!b || !src_xy || !dens || (!b->self_exclude && !trg_xy) || (!out_pot && !out_grad)) return PFMM_EINVAL;
  if (!workspace || ((uintptr_t)workspace & 255)) return PFMM_EWORKSPACE;
  int rc0 = batch_refresh(b);
  if (rc0) return rc0;
  hipStream_t st = (hipStream_t)hip_stream;
  char* ws = (char*)workspace;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return PFMM_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return PFMM_EHIP; }
  // one warm-up and one timed eager launch sequence
  auto timed = [&](double* ms) -> int {
    int rc = batch_launch(b, src_xy, dens, trg_xy, out_pot, out_grad, ws, st);
    if (rc) return rc;
    if (hipEventRecord(e0, st) != hipSuccess) return PFMM_EHIP;
    rc = batch_launch(b, src_xy, dens, trg_xy, out_pot, out_grad, ws, st);
    if (rc) return rc;
    float t = 0;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
      return PFMM_EHIP;
    *ms = t;
    return PFMM_OK;
  };
  const int64_t split0 = b->split;
  const int mult0 = b->grid_mult;
  int rc = PFMM_OK, tried = 0;
  double start_ms = 0, best_ms = 0;
  int64_t best_split = split0;
  int best_mult = mult0;
  if (b->total <= ws_bytes) {
    rc = timed(&start_ms);
    ++tried;
    best_ms = start_ms;
  } else {
    best_ms = 1e300;
  }
  const int64_t splits[3] = {4096, 8192, 16384};
  const int mults[3] = {2, 4, 8};
  for (int i = 0; i < 3 && !rc; ++i)
    for (int j = 0; j < 3 && !rc; ++j) {
      if (splits[i] == split0 && mults[j] == mult0) continue;
      if ((rc = batch_build(b, splits[i], mults[j]))) break;
      if (b->total > ws_bytes) continue;
      double ms = 0;
      if ((rc = timed(&ms))) break;
      ++tried;
      if (ms < best_ms) { best_ms = ms; best_split = splits[i]; best_mult = mults[j]; }
    }
  if (!rc) rc = batch_build(b, best_split, best_mult);
  if (!rc && b->total > ws_bytes) rc = PFMM_EWORKSPACE;
  if (!rc) rc = batch_launch(b, src_xy, dens, trg_xy, out_pot, out_grad, ws, st);
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = PFMM_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!rc && report) { report->n_tried = tried; report->default_ms = start_ms; report->best_ms = best_ms; }
  return rc;
}
void pfmm_batch_destroy(pfmm_batch_t b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_recs) (void)hipFree(b->d_recs);
  delete b;
}

}  // extern "C"
