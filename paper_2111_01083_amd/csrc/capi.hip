// C ABI entry points: plan lifetime, workspace layout and the launch
// sequence of one evaluation (prep -> near | far_R -> far_D -> far_L).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"
#include "nufft.h"
#include "pfmm.h"
#include "pfmm_internal.h"

using namespace pfmm;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace carve-up for one cell; offsets in bytes from the workspace base.
struct Layout {
  size_t scx, scy, tcx, tcy, sxh, sxl, syh, syl, q32, dens_c, near_part, far_part, w, nufft, nu_val;
  size_t key, perm, stx, sty, hist, cursor;   // target binning
  int nbx, nby;
  double bin_w, bin_h;
  size_t total;
  int n_splits, n_chunks, n_coef;
  int64_t split_len;
  size_t part_stride;  // doubles per split
};

void plan_layout(const pfmm_plan_s* p, int64_t ns, int64_t nt, Layout& L) {
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
    L.sxh = take(4 * ns); L.sxl = take(4 * ns); L.syh = take(4 * ns); L.syl = take(4 * ns);
    L.q32 = take(4 * (size_t)p->n_dens * nc * ns);
  } else {
    L.sxh = L.sxl = L.syh = L.syl = L.q32 = 0;
  }
  L.dens_c = p->kernel == PFMM_STOKES ? take(8 * (size_t)p->n_dens * 2 * ns) : 0;
  // target bins of about 64 points over the canonical cell's bounding box
  {
    const double W = p->geo.d + std::fabs(p->geo.xi), H = p->geo.eta;
    const double nb = std::max(1.0, std::min((double)nt / 64.0, 4.0e6));
    const double h = std::sqrt(W * H / nb);
    L.nbx = std::max(1, (int)std::ceil(W / h));
    L.nby = std::max(1, (int)std::ceil(H / h));
    L.bin_w = W / L.nbx;
    L.bin_h = H / L.nby;
    L.key = take(4 * nt); L.perm = take(4 * nt); L.stx = take(8 * nt); L.sty = take(8 * nt);
    L.hist = take(4 * (size_t)L.nbx * L.nby); L.cursor = take(4 * (size_t)L.nbx * L.nby);
  }
  // source splits for the near field: aim for >= 2048 blocks in flight
  int64_t tiles = std::max<int64_t>(1, (nt + NEAR_BLOCK - 1) / NEAR_BLOCK);
  int64_t max_s = std::max<int64_t>(1, (ns + NEAR_TILE - 1) / NEAR_TILE);
  int64_t S = std::min<int64_t>(std::min<int64_t>((2048 + tiles - 1) / tiles, max_s), 64);
  S = std::max<int64_t>(S, 1);
  int64_t per = (ns + S - 1) / S;
  per = std::max<int64_t>(NEAR_TILE, (per + NEAR_TILE - 1) / NEAR_TILE * NEAR_TILE);
  L.split_len = per;
  L.n_splits = (int)std::max<int64_t>(1, (ns + per - 1) / per);
  L.part_stride = (size_t)p->n_dens * no * nt;
  L.near_part = take(8 * L.part_stride * L.n_splits);
  L.n_chunks = (int)std::max<int64_t>(1, (ns + FAR_CHUNK - 1) / FAR_CHUNK);
  L.n_coef = (p->n_sn + p->n_ew) * coef_per_wave(p->kernel) + 1;
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
  *out = p;
  return PFMM_OK;
}

int pfmm_plan_upload(pfmm_plan_t p) {
  if (!p) return PFMM_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFMM_EHIP;
  if (p->d_tab && p->dev_id == dev) return PFMM_OK;
  std::vector<double> tab;
  tab.insert(tab.end(), p->sn_tab.begin(), p->sn_tab.end());
  tab.insert(tab.end(), p->ew_tab.begin(), p->ew_tab.end());
  tab.insert(tab.end(), p->gl_nodes.begin(), p->gl_nodes.end());
  tab.insert(tab.end(), p->gl_bary.begin(), p->gl_bary.end());
  tab.insert(tab.end(), p->nu_deconv.begin(), p->nu_deconv.end());
  tab.push_back(0.0);
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
  info->n_modes = p->M;
  info->n_quad = p->n_ew;
  info->m_gl = p->nu.m_gl; info->nufft_nf = p->nu.nf; info->nufft_w = p->nu.w;
  info->n_images = p->geo.n_images;
  return PFMM_OK;
}

int pfmm_plan_get_quadrature(pfmm_plan_t p, double* nodes, double* weights) {
  if (!p) return PFMM_EINVAL;
  if (nodes) std::copy(p->ew_nodes.begin(), p->ew_nodes.end(), nodes);
  if (weights) std::copy(p->ew_weights.begin(), p->ew_weights.end(), weights);
  return PFMM_OK;
}

size_t pfmm_workspace_bytes(pfmm_plan_t p, int64_t ns, int64_t nt) {
  if (!p || ns < 0 || nt < 0) return 0;
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

int pfmm::eval_core(pfmm_plan_t p, int64_t ns, const double* src_xy, const double* dens, int64_t nt,
                    const double* trg_xy, double* out_pot, double* out_grad, void* workspace,
                    size_t ws_bytes, void* hip_stream) {
  if (!p || ns < 0 || nt < 0) return PFMM_EINVAL;
  if (p->self_exclude && nt != ns) return PFMM_EINVAL;
  if (ns > 0 && (!src_xy || !dens)) return PFMM_EINVAL;
  if (nt > 0 && !p->self_exclude && !trg_xy) return PFMM_EINVAL;
  if (nt == 0 || (!out_pot && !out_grad)) return PFMM_OK;
  Layout L;
  plan_layout(p, ns, nt, L);
  if (!workspace || ws_bytes < L.total || ((uintptr_t)workspace & 255)) return PFMM_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = pfmm_plan_upload(p);
  if (rc) return rc;
  const int K = p->kernel;
  const bool mixed = p->precision == PFMM_MIXED;
  const int nc = K == PFMM_STOKES ? 2 : 1;
  if (p->check_neutral && K != PFMM_YUKAWA && ns > 0) {
    std::vector<double> h((size_t)p->n_dens * nc * ns);
    if (hipStreamSynchronize(st) != hipSuccess) return PFMM_EHIP;
    if (hipMemcpy(h.data(), dens, h.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) return PFMM_EHIP;
    for (int v = 0; v < p->n_dens * nc; ++v) {
      double s = 0, a = 0;
      for (int64_t j = 0; j < ns; ++j) { s += h[(size_t)v * ns + j]; a += std::fabs(h[(size_t)v * ns + j]); }
      if (std::fabs(s) > 1e-12 * a) return PFMM_ENOT_NEUTRAL;
    }
  }
  char* ws = (char*)workspace;
  auto D = [&](size_t off) { return (double*)(ws + off); };
  auto F = [&](size_t off) { return (float*)(ws + off); };
  const Geometry& g = p->geo;

  // prep
  PrepArgs pa{};
  pa.rc = g.rc; pa.rs = g.rs; pa.d = g.d; pa.xi = g.xi; pa.eta = g.eta;
  pa.n = ns; pa.xy = src_xy; pa.cx = D(L.scx); pa.cy = D(L.scy);
  if (mixed) { pa.hx = F(L.sxh); pa.lx = F(L.sxl); pa.hy = F(L.syh); pa.ly = F(L.syl); }
  launch_prep_points(pa, st);
  if (!p->self_exclude) {
    PrepArgs pt = pa;
    pt.n = nt; pt.xy = trg_xy; pt.cx = D(L.tcx); pt.cy = D(L.tcy);
    pt.hx = pt.lx = pt.hy = pt.ly = nullptr;
    launch_prep_points(pt, st);
  }
  const double* dens_c = dens;
  if (K == PFMM_STOKES || mixed) {
    PrepDensArgs pd{};
    pd.n = ns; pd.n_dens = p->n_dens; pd.stokes = K == PFMM_STOKES; pd.dens = dens;
    pd.rc = g.rc; pd.rs = g.rs;
    pd.out64 = K == PFMM_STOKES ? D(L.dens_c) : nullptr;
    pd.out32 = mixed ? F(L.q32) : nullptr;
    launch_prep_dens(pd, st);
    if (K == PFMM_STOKES) dens_c = D(L.dens_c);
  }

  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  if (p->profile) {
    for (int k = 0; k < 3; ++k)
      if (hipEventCreate(&ev[k]) != hipSuccess) return PFMM_EHIP;
    p->prof_events.push_back(ev[0]); p->prof_events.push_back(ev[1]); p->prof_events.push_back(ev[2]);
  }

  // bin the targets (near-field work order)
  SortArgs sa{};
  sa.n = nt; sa.x = D(L.tcx); sa.y = D(L.tcy);
  sa.x0 = -0.5 * (g.d + std::fabs(g.xi)); sa.y0 = -0.5 * g.eta;
  sa.inv_w = 1.0 / L.bin_w; sa.inv_h = 1.0 / L.bin_h; sa.nbx = L.nbx; sa.nby = L.nby;
  sa.key = (int*)(ws + L.key); sa.perm = (int*)(ws + L.perm);
  sa.hist = (int*)(ws + L.hist); sa.cursor = (int*)(ws + L.cursor);
  sa.sx = D(L.stx); sa.sy = D(L.sty);
  launch_sort_targets(sa, st);

  // near field
  NearArgs na{};
  na.geo = g;
  na.n_src = ns; na.n_trg = nt; na.split_len = L.split_len;
  na.sx = D(L.scx); na.sy = D(L.scy);
  if (mixed) { na.sxh = F(L.sxh); na.sxl = F(L.sxl); na.syh = F(L.syh); na.syl = F(L.syl); na.q32 = F(L.q32); }
  na.q64 = dens_c;
  na.tx = D(L.stx); na.ty = D(L.sty); na.perm = sa.perm;
  na.self = p->self_exclude;
  na.beta = p->beta;
  na.r2min = R2MIN_F32;
  na.part = D(L.near_part);
  na.part_stride = L.part_stride;
  if (ns > 0) {
    if (p->profile) (void)hipEventRecord(ev[0], st);
    launch_near(K, mixed, p->n_dens, na, L.n_splits, st);
    if (p->profile) (void)hipEventRecord(ev[1], st);
  } else {
    launch_fill_zero(na.part, (int64_t)L.part_stride, st);
  }
  const int n_splits_used = ns > 0 ? L.n_splits : 1;

  // far field: R (direct plane waves, or NUFFT for south/north), D, L
  FarRArgs fr{};
  fr.kernel = K; fr.n_sn = p->n_sn; fr.n_ew = p->n_ew; fr.ncw = coef_per_wave(K);
  fr.n_coef = L.n_coef; fr.n_dens = p->n_dens; fr.n_src = ns; fr.tab = p->d_tab;
  fr.sx = D(L.scx); fr.sy = D(L.scy); fr.dens = dens_c; fr.part = D(L.far_part);
  fr.skip_sn = p->use_nufft;
  const double* csn = nullptr;
  if (p->use_nufft) {
    rc = nufft_R(p, ns, D(L.scx), D(L.scy), dens_c, ws + L.nufft, st, &csn);
    if (rc) return rc;
  }
  if (ns > 0) launch_far_R(fr, L.n_chunks, st);
  else launch_fill_zero(fr.part, 2 * (int64_t)p->n_dens * L.n_coef, st);
  FarDArgs fd{};
  fd.kernel = K; fd.n_sn = p->n_sn; fd.n_ew = p->n_ew; fd.ncw = fr.ncw; fd.n_coef = L.n_coef;
  fd.n_dens = p->n_dens; fd.n_chunks = ns > 0 ? L.n_chunks : 1; fd.eta = g.eta; fd.xi = g.xi;
  fd.tab = p->d_tab; fd.part = fr.part; fd.extra = csn; fd.w = D(L.w);
  launch_far_D(fd, st);
  const double* nu_val = nullptr;
  if (p->use_nufft) {
    rc = nufft_L(p, nt, D(L.tcx), D(L.tcy), D(L.w), L.n_coef, ws + L.nufft, st, &nu_val, D(L.nu_val));
    if (rc) return rc;
  }
  FarLArgs fl{};
  fl.kernel = K; fl.n_sn = p->n_sn; fl.n_ew = p->n_ew; fl.ncw = fr.ncw; fl.n_coef = L.n_coef;
  fl.n_dens = p->n_dens; fl.n_splits = n_splits_used; fl.nufft = p->use_nufft; fl.n_trg = nt;
  fl.d = g.d; fl.eta = g.eta; fl.rc = g.rc; fl.rs = g.rs; fl.tab = p->d_tab; fl.w = D(L.w);
  fl.tx = D(L.tcx); fl.ty = D(L.tcy); fl.near_part = D(L.near_part); fl.part_stride = L.part_stride;
  fl.nu_val = nu_val; fl.out_pot = out_pot; fl.out_grad = out_grad;
  launch_far_L(fl, st);
  if (p->profile) {
    if (ns == 0) { (void)hipEventRecord(ev[0], st); (void)hipEventRecord(ev[1], st); }
    (void)hipEventRecord(ev[2], st);
  }
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

void pfmm_destroy(pfmm_plan_t p) {
  if (!p) return;
  for (void* e : p->prof_events) (void)hipEventDestroy((hipEvent_t)e);
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
