// Host-side planning: lattice canonicalisation, truncation sizes, the
// west/east quadrature rule, the diagonal weights D of the low-rank
// factorisations, and NUFFT parameters. No device work happens here.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "pfmm_internal.h"
#include "fmm.h"

namespace pfmm {

using cd = std::complex<double>;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
static void legendre(int n, double t, double& pn, double& dpn) {
  double p0 = 1, p1 = t;
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
    p0 = p1; p1 = p2;
  }
  pn = (n == 0) ? 1.0 : p1;
  double pm = (n <= 1) ? 1.0 : p0;
  dpn = (n == 0) ? 0.0 : n * (t * pn - pm) / (t * t - 1);
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(PI * (i + 0.75) / (n + 0.5)), pn, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, pn, dp);
      double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 4e-16) break;
    }
    legendre(n, t, pn, dp);
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1 - t * t) * dp * dp);
  }
}

namespace {

// 1 - e^{-a} for complex a, without cancellation for small |a|
cd one_minus_exp(cd a) {
  const double sh = std::sin(0.5 * a.imag());
  const cd em1(std::expm1(-a.real()) * std::cos(a.imag()) - 2 * sh * sh, -std::exp(-a.real()) * std::sin(a.imag()));
  return -em1;
}

// Gauss-Lagrange reduction of a 2D lattice basis; returns b1 (shortest) and
// b2 with |b1| <= |b2| and |b1.b2| <= |b1|^2/2.
void reduce_basis(double b1[2], double b2[2]) {
  auto dot = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1]; };
  for (int it = 0; it < 200; ++it) {
    if (dot(b2, b2) < dot(b1, b1)) { std::swap(b1[0], b2[0]); std::swap(b1[1], b2[1]); }
    double mu = std::nearbyint(dot(b1, b2) / dot(b1, b1));
    if (mu == 0) break;
    b2[0] -= mu * b1[0]; b2[1] -= mu * b1[1];
  }
  if (dot(b2, b2) < dot(b1, b1)) { std::swap(b1[0], b2[0]); std::swap(b1[1], b2[1]); }
}

// Log groups of the symmetric mixed near field. The log terms of a pair sum
// log2 r^2 over the images l of the near region; the kernel multiplies the
// FP32 r^2 of a run of images and takes one log2 of the product. Bounds for
// a group (coordinates scaled by sigma; a pair difference d0 lies in
// {u e1 + v e2 : |u|, |v| < 1}, so |d0| < dmax):
//   every factor |d0 - l|^2 < (dmax + |l|)^2, and
//   with l* the group image nearest to d0, |d0 - l| >= |l - l*| / 2 for the
//   others, so the product without l*'s factor is >= prod min(1, |l - l*|^2/4).
// Starting the product at 2^e0 keeps every partial product below 2^124 and,
// for the closest image's r^2 down to 2^-100, above 2^-124; within that range
// e0 is chosen to bring a typical product near 1 (the FP32 log2 is then most
// accurate). The groups tried are all images (cells with 9 images), the rows
// of fixed n (images one period d apart; the kernel also moves its FP32
// image sums to FP64 after each group, which keeps 15- and 21-image cells
// accurate), and single images (always valid: the per-image log).
void plan_log_groups(pfmm::Geometry& g, int per_row) {
  const double s = g.sigma;
  const double dmax = s * std::max(std::hypot(g.d + g.xi, g.eta), std::hypot(g.d - g.xi, g.eta));
  const int sizes[3] = {g.n_images <= 9 ? g.n_images : per_row, per_row, 1};
  for (int gs : sizes) {
    if (gs < 1 || g.n_images % gs) continue;
    bool ok = true;
    int n_lg = 0;
    for (int g0 = 0; g0 < g.n_images && ok; g0 += gs) {
      double fmax = 0, gmin = 0;
      for (int i = g0; i < g0 + gs; ++i) {
        const double li = s * std::hypot(g.img_x[i], g.img_y[i]);
        fmax += std::max(0.0, 2 * std::log2(dmax + li));
      }
      for (int k = g0; k < g0 + gs; ++k) {
        double t = 0;
        for (int i = g0; i < g0 + gs; ++i) {
          if (i == k) continue;
          const double sep2 = s * s * (std::pow(g.img_x[i] - g.img_x[k], 2) + std::pow(g.img_y[i] - g.img_y[k], 2));
          t += std::min(0.0, std::log2(sep2 / 4));
        }
        gmin = std::min(gmin, t);
      }
      // need e0 + fmax <= 124 and -100 + e0 + gmin >= -124 (two bits of slack each)
      const double lo = std::ceil(-22 - gmin), hi = std::floor(122 - fmax);
      if (lo > hi) { ok = false; break; }
      // typical log2 of the product: mean over pair differences
      // d0 = u e1 + v e2, u, v in {-3/4, -1/4, 1/4, 3/4}
      double typ = 0;
      for (int iu = 0; iu < 4; ++iu)
        for (int iv = 0; iv < 4; ++iv) {
          const double u = -0.75 + 0.5 * iu, v = -0.75 + 0.5 * iv;
          const double x0 = s * (u * g.d + v * g.xi), y0 = s * (v * g.eta);
          for (int i = g0; i < g0 + gs; ++i)
            typ += std::log2(std::pow(x0 - s * g.img_x[i], 2) + std::pow(y0 - s * g.img_y[i], 2));
        }
      typ /= 16;
      g.lg_e0[n_lg] = (int)std::min(std::max(-std::nearbyint(typ), lo), hi);
      g.lg_end[n_lg] = g0 + gs;
      ++n_lg;
    }
    if (ok) { g.n_lg = n_lg; return; }
  }
  g.n_lg = g.n_images;   // unreachable: single images always qualify
  for (int i = 0; i < g.n_images; ++i) { g.lg_end[i] = i + 1; g.lg_e0[i] = 0; }
}

// West/east rule (Thm. west_thm and its Laplace/Stokes limits): the paper's
// generalized Gaussian tables are not published, so the rule is built here
// from Gauss-Legendre panels. The integrand decays like e^{-kappa X} with
// X >= Xmin = m0 d - 2|xi| (closest west/east image), oscillates like
// e^{i lambda Y} with |Y| <= 2 eta, and its factor 1/(1-e^{-kappa d}) has
// poles at kappa d = 2 pi i k, so panels are at most 2 min(pi/2eta, pi/d)
// wide; for Yukawa with small beta the branch point at lambda = i beta gets
// dyadic panels near 0 (same recipe as the singly periodic rule of Sec. 3).
void ew_rule(int kernel, double beta, double d, double xi, double eta, int m0, double eps,
             std::vector<double>& nodes, std::vector<double>& wts) {
  nodes.clear(); wts.clear();
  const double Xmin = m0 * d - 2 * std::fabs(xi);
  const double lk = (std::log(1.0 / eps) + 2.0) / Xmin;
  double L;
  if (kernel == PFMM_YUKAWA) {
    if (lk <= beta) return;  // whole west/east contribution below eps
    L = std::sqrt(lk * lk - beta * beta);
  } else {
    L = lk;
  }
  // 12/16/20 Gauss-Legendre points per panel reach eps for eps >= 1e-8 / 1e-12 / below
  const int np = eps >= 1e-8 ? 12 : (eps >= 1e-12 ? 16 : 20);
  const double h0 = 2.0 * std::min(PI / (2 * eta), PI / d);
  std::vector<double> edges{0.0};
  if (kernel == PFMM_YUKAWA && beta < h0) {
    double b = std::max(beta, 1e-300);
    edges.push_back(std::min(b, L));
    while (edges.back() * 2 < std::min(h0, L)) edges.push_back(edges.back() * 2);
  }
  double start = edges.back();
  if (start < L) {
    int n = std::max(1, (int)std::ceil((L - start) / h0));
    double h = (L - start) / n;
    for (int i = 1; i <= n; ++i) edges.push_back(start + i * h);
  }
  std::vector<double> gx, gw;
  gauss_legendre(np, gx, gw);
  for (size_t e = 0; e + 1 < edges.size(); ++e) {
    double a = edges[e], b = edges[e + 1];
    for (int i = 0; i < np; ++i) {
      nodes.push_back(0.5 * (b - a) * (gx[i] + 1) + a);
      wts.push_back(0.5 * (b - a) * gw[i]);
    }
  }
}

// West/east rule in a rotated frame (Appendix A, eq. k0west2): with e2
// vertical the closest west/east image is a full column dx' away, but the
// integrand e^{-kappa X} e^{i lambda Y} B R, R = e^{-p a}/(1 - e^{-a}),
// a = kappa dx' - i lambda dy', oscillates with |Y| up to |dy'| + eta' plus
// the frequencies of R (multiples of dy'), and R has near-poles where
// lambda dy' ~ 2 pi k while kappa dx' is small. The rule is built by
// adaptive bisection of Gauss-Legendre panels on [0, L]: a panel is kept
// when its np- and 2np-point sums of every sampled integrand (X and Y over
// their ranges) agree within eps times that sample's integral of |f|,
// prorated by the panel's length. Laplace/Stokes samples are multiplied by
// lambda/(1+lambda) (the combined west+east integrand is smooth at 0).
// rows = 3: the rows n = -1, 0, 1 of the doubly periodic split, |y
// offsets| up to Ym = |dy'| + eta'; rows = 1: the singly periodic split (one
// row, B = 1), |y offsets| up to the strip height Ym.
void ew_rule_adaptive(int kernel, double beta, double dx, double dy, double xi2, double eta2, int rows, double Ym,
                      int m0, double eps, std::vector<double>& nodes, std::vector<double>& wts) {
  nodes.clear(); wts.clear();
  const double Xmin = m0 * dx;
  const double lk = (std::log(1.0 / eps) + 2.0) / Xmin;
  double L;
  if (kernel == PFMM_YUKAWA) {
    if (lk <= beta) return;
    L = std::sqrt(lk * lk - beta * beta);
  } else {
    L = lk;
  }
  const int p0 = m0 + 1;
  std::vector<double> sx, sy;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 9; ++j) {
      sx.push_back(dx * (-0.999 + 0.4995 * i));
      sy.push_back(Ym * (-1.0 + 0.25 * j));
    }
  const size_t ns = sx.size();
  auto f = [&](double lam, std::vector<cd>& out) {
    const double kap = kernel == PFMM_YUKAWA ? std::sqrt(lam * lam + beta * beta) : lam;
    const cd a(kap * dx, -lam * dy);
    const cd R = std::exp(-double(p0) * a) / one_minus_exp(a);
    const cd B = rows == 1 ? cd(1.0) : std::exp(cd(-kap * xi2, lam * eta2)) + std::exp(cd(kap * xi2, -lam * eta2)) + 1.0;
    const double s = kernel == PFMM_YUKAWA ? 1.0 / kap : lam / (1.0 + lam);
    for (size_t k = 0; k < ns; ++k) out[k] = s * std::exp(cd(-kap * sx[k], lam * sy[k])) * R * B;
  };
  const int np = eps >= 1e-8 ? 12 : (eps >= 1e-12 ? 16 : 20);
  std::vector<double> g1x, g1w, g2x, g2w;
  gauss_legendre(np, g1x, g1w);
  gauss_legendre(2 * np, g2x, g2w);
  std::vector<cd> val(ns);
  auto panel = [&](double a0, double b0, int n, const std::vector<double>& gx, const std::vector<double>& gw,
                   std::vector<cd>& I, std::vector<double>* A) {
    I.assign(ns, cd(0.0));
    if (A) A->assign(ns, 0.0);
    for (int i = 0; i < n; ++i) {
      const double lam = 0.5 * (b0 - a0) * (gx[i] + 1) + a0, w = 0.5 * (b0 - a0) * gw[i];
      f(lam, val);
      for (size_t k = 0; k < ns; ++k) {
        I[k] += w * val[k];
        if (A) (*A)[k] += w * std::abs(val[k]);
      }
    }
  };
  // scale of each sample: integral of |f| on a fine uniform composite rule
  const double h0 = std::min(L, 2 * PI / (Ym + 2 * std::fabs(dy) + eta2));
  const int n0 = std::max(1, (int)std::ceil(L / h0));
  std::vector<double> scale(ns, 0.0), tmpA;
  std::vector<cd> I1, I2;
  for (int e = 0; e < n0; ++e) {
    panel(L * e / n0, L * (e + 1) / n0, 2 * np, g2x, g2w, I2, &tmpA);
    for (size_t k = 0; k < ns; ++k) scale[k] += tmpA[k];
  }
  std::vector<std::pair<double, double>> todo;
  for (int e = n0 - 1; e >= 0; --e) todo.push_back({L * e / n0, L * (e + 1) / n0});
  std::vector<std::pair<double, double>> done;
  while (!todo.empty() && done.size() + todo.size() < 4096) {
    auto [a0, b0] = todo.back();
    todo.pop_back();
    panel(a0, b0, np, g1x, g1w, I1, nullptr);
    panel(a0, b0, 2 * np, g2x, g2w, I2, nullptr);
    bool ok = true;
    for (size_t k = 0; k < ns && ok; ++k)
      ok = std::abs(I1[k] - I2[k]) <= 0.25 * eps * scale[k] * (b0 - a0) / L;
    if (ok || b0 - a0 < 1e-9 * L) done.push_back({a0, b0});
    else { todo.push_back({0.5 * (a0 + b0), b0}); todo.push_back({a0, 0.5 * (a0 + b0)}); }
  }
  for (auto& pr : todo) done.push_back(pr);
  std::sort(done.begin(), done.end());
  for (auto [a0, b0] : done)
    for (int i = 0; i < np; ++i) {
      nodes.push_back(0.5 * (b0 - a0) * (g1x[i] + 1) + a0);
      wts.push_back(0.5 * (b0 - a0) * g1w[i]);
    }
}

// Least-squares solve min ||A x - b|| (A m x n, m >= n, row-major, full
// column rank) by Householder QR; A and b are overwritten.
bool lstsq(std::vector<double>& A, std::vector<double>& b, int m, int n, std::vector<double>& x) {
  for (int k = 0; k < n; ++k) {
    double nrm = 0;
    for (int i = k; i < m; ++i) nrm += A[(size_t)i * n + k] * A[(size_t)i * n + k];
    nrm = std::sqrt(nrm);
    if (nrm == 0) return false;
    const double a0 = A[(size_t)k * n + k], alpha = a0 > 0 ? -nrm : nrm;
    std::vector<double> v(m, 0.0);
    v[k] = a0 - alpha;
    for (int i = k + 1; i < m; ++i) v[i] = A[(size_t)i * n + k];
    double vv = 0;
    for (int i = k; i < m; ++i) vv += v[i] * v[i];
    for (int j = k; j < n; ++j) {
      double t = 0;
      for (int i = k; i < m; ++i) t += v[i] * A[(size_t)i * n + j];
      t *= 2 / vv;
      for (int i = k; i < m; ++i) A[(size_t)i * n + j] -= t * v[i];
    }
    double t = 0;
    for (int i = k; i < m; ++i) t += v[i] * b[i];
    t *= 2 / vv;
    for (int i = k; i < m; ++i) b[i] -= t * v[i];
  }
  x.assign(n, 0.0);
  for (int k = n - 1; k >= 0; --k) {
    double t = b[k];
    for (int j = k + 1; j < n; ++j) t -= A[(size_t)k * n + j] * x[j];
    if (A[(size_t)k * n + k] == 0) return false;
    x[k] = t / A[(size_t)k * n + k];
  }
  return true;
}

// Compressed west/east rule (canonical frame). The rule only ever integrates
// combinations of the plane waves f(lambda) = e^{-kappa X} e^{i lambda Y}
// (times 1/kappa for Yukawa) with X >= Xmin and |Y| <= 2 eta (every west/east
// image of every pair, Thm. west_thm; the Laplace/Stokes forms are
// superpositions of these over X). Sampling that family on the panel rule's
// nodes, a column-pivoted QR of the weighted samples picks the nodes that
// span it to eps, and least squares fits their weights to reproduce the panel
// rule's integrals of every sample; the result is kept only if it also
// reproduces them on a second, interleaved sample set to eps/4 of the
// largest integral, else the panel rule stays. This is the node selection step of generalized Gaussian
// quadrature, without its final Newton refinement of the nodes.
void compress_rule(int kernel, double beta, double Xmin, double Ymax, double eps, std::vector<double>& nodes,
                   std::vector<double>& wts) {
  const int n = (int)nodes.size();
  if (n < 8) return;
  auto kap = [&](double lam) { return kernel == PFMM_YUKAWA ? std::sqrt(lam * lam + beta * beta) : lam; };
  auto family = [&](double xs0, double ys0, std::vector<double>& X, std::vector<double>& Y) {
    X.clear(); Y.clear();
    const double span = (std::log(1.0 / eps) + 4.0) / std::max(kap(nodes[0] > 0 ? nodes[0] : 1e-3), 1e-300);
    const double xmax = Xmin + std::min(span, 60.0 * Xmin + 60.0);
    for (int i = 0; i < 24; ++i) {
      const double t = (i + xs0) / 24.0;
      X.push_back(Xmin * std::pow(xmax / Xmin, t * t));   // denser near Xmin
    }
    for (int j = 0; j <= 32; ++j) Y.push_back(Ymax * (-1.0 + 2.0 * (j + ys0) / 32.5));
  };
  auto fill = [&](const std::vector<double>& X, const std::vector<double>& Y, const std::vector<int>& cols,
                  const std::vector<double>* w, std::vector<double>& M, std::vector<double>* ref) {
    const int m = 2 * (int)(X.size() * Y.size()), nc = (int)cols.size();
    M.assign((size_t)m * nc, 0.0);
    if (ref) ref->assign(m, 0.0);
    int r = 0;
    for (double x : X)
      for (double y : Y) {
        double sr = 0, si = 0;
        for (int c = 0; c < nc; ++c) {
          const double lam = nodes[cols[c]], k = kap(lam);
          const double a = std::exp(-k * x) / (kernel == PFMM_YUKAWA ? k : 1.0);
          const double fr = a * std::cos(lam * y), fi = a * std::sin(lam * y);
          const double sc = w ? (*w)[c] : 1.0;
          M[(size_t)r * nc + c] = fr * sc;
          M[(size_t)(r + 1) * nc + c] = fi * sc;
          if (ref) { sr += wts[cols[c]] * fr; si += wts[cols[c]] * fi; }
        }
        if (ref) { (*ref)[r] = sr; (*ref)[r + 1] = si; }
        r += 2;
      }
  };
  std::vector<int> all(n);
  for (int i = 0; i < n; ++i) all[i] = i;
  std::vector<double> X, Y, F, ref;
  family(0.0, 0.0, X, Y);
  std::vector<double> sw(n);
  for (int i = 0; i < n; ++i) sw[i] = std::sqrt(std::fabs(wts[i]));
  fill(X, Y, all, &sw, F, &ref);
  const int m = 2 * (int)(X.size() * Y.size());
  // column-pivoted Householder QR of F until the largest remaining column
  // norm drops below eps/20 of the largest initial one
  std::vector<double> cn(n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) cn[j] += F[(size_t)i * n + j] * F[(size_t)i * n + j];
  const double c0 = std::sqrt(*std::max_element(cn.begin(), cn.end()));
  std::vector<int> perm = all;
  int r = 0;
  for (; r < std::min(m, n); ++r) {
    int jm = r;
    for (int j = r; j < n; ++j) if (cn[j] > cn[jm]) jm = j;
    if (std::sqrt(cn[jm]) < 0.05 * eps * c0) break;
    if (jm != r) {
      std::swap(perm[r], perm[jm]); std::swap(cn[r], cn[jm]);
      for (int i = 0; i < m; ++i) std::swap(F[(size_t)i * n + r], F[(size_t)i * n + jm]);
    }
    double nrm = 0;
    for (int i = r; i < m; ++i) nrm += F[(size_t)i * n + r] * F[(size_t)i * n + r];
    nrm = std::sqrt(nrm);
    const double a0 = F[(size_t)r * n + r], alpha = a0 > 0 ? -nrm : nrm;
    std::vector<double> v(m, 0.0);
    v[r] = a0 - alpha;
    for (int i = r + 1; i < m; ++i) v[i] = F[(size_t)i * n + r];
    double vv = 0;
    for (int i = r; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0) break;
    for (int j = r; j < n; ++j) {
      double t = 0;
      for (int i = r; i < m; ++i) t += v[i] * F[(size_t)i * n + j];
      t *= 2 / vv;
      for (int i = r; i < m; ++i) F[(size_t)i * n + j] -= t * v[i];
    }
    for (int j = r + 1; j < n; ++j) {
      double t = 0;
      for (int i = r + 1; i < m; ++i) t += F[(size_t)i * n + j] * F[(size_t)i * n + j];
      cn[j] = t;
    }
  }
  if (r >= n) return;
  std::vector<int> sel(perm.begin(), perm.begin() + r);
  std::sort(sel.begin(), sel.end());
  // weights: least squares against the panel rule's integrals of the samples
  std::vector<double> A, b = ref, w;
  fill(X, Y, sel, nullptr, A, nullptr);
  if (!lstsq(A, b, m, r, w)) return;
  // check on an interleaved sample set
  std::vector<double> X2, Y2, A2, ref2;
  family(0.5, 0.5, X2, Y2);
  fill(X2, Y2, sel, nullptr, A2, nullptr);
  fill(X2, Y2, all, nullptr, F, &ref2);
  const int m2 = 2 * (int)(X2.size() * Y2.size());
  double scale = 0, err = 0;
  for (int i = 0; i < m2; i += 2) {
    double sr = 0, si = 0;
    for (int c = 0; c < r; ++c) { sr += A2[(size_t)i * r + c] * w[c]; si += A2[(size_t)(i + 1) * r + c] * w[c]; }
    err = std::max(err, std::hypot(sr - ref2[i], si - ref2[i + 1]));
    scale = std::max(scale, std::hypot(ref2[i], ref2[i + 1]));
  }
  if (!(err <= 0.25 * eps * scale)) return;
  std::vector<double> nn(r), ww(r);
  for (int c = 0; c < r; ++c) { nn[c] = nodes[sel[c]]; ww[c] = w[c]; }
  nodes.swap(nn);
  wts.swap(ww);
}

}  // namespace

// NUFFT grid and kernel (Sec. 6.1). grid 0: the smallest power of two
// n_f >= 2(2M+1) (oversampling s_o >= 2) with width w = ceil(log10(1/eps)) + 1;
// grid 1: twice that grid (s_o >= 4), one point narrower. The
// exponential-of-semicircle kernel phi(z) = exp(b(sqrt(1-z^2)-1)) takes
// b = 0.97 pi (1 - 1/(2 s_o)) w for the nominal s_o (2.29 w, resp. 2.67 w:
// the kernel's transform must be small beyond the alias band, which moves
// out as s_o grows); its Fourier transform on |z| <= 1, scaled to half-width
// s = w h/2, is computed here by Gauss-Legendre quadrature for the
// deconvolution: Phi(alpha) = (w/2) int phi(z) cos(alpha s z) dz.
int set_nufft_grid(pfmm_plan_s* p, int grid) {
  const int M = p->M;
  int w = (int)std::ceil(std::log10(1.0 / p->eps)) + 1;
  w = std::max(4, std::min(w, 16));
  int nf = 16;
  while (nf < 2 * (2 * M + 1) || nf < 2 * w) nf *= 2;
  if (grid == 1) {
    if (2 * nf > NUFFT_MAX_GRID) return PFMM_EINVAL;
    nf *= 2;
    w = std::max(4, w - 1);
  } else if (grid != 0) {
    return PFMM_EINVAL;
  }
  p->nu.w = w;
  p->nu.nf = nf;
  const double so = grid == 1 ? 4.0 : 2.0;
  p->nu.es_beta = 0.97 * PI * (1 - 1 / (2 * so)) * w;
  p->nu_grid = grid;
  // the kernel's taps as polynomials in u = 2f - 1 (least squares on 4x
  // oversampled Chebyshev points, Householder QR), so that a point's w + 1
  // kernel values cost one Horner pass instead of w + 1 exp and sqrt
  {
    const int D = std::min(ES_COEF, w + 4);
    p->nu.es_deg = D;
    p->nu_poly.assign((size_t)ES_TAPS * ES_COEF, 0.0);
    const int K = 4 * D;
    const double bb = p->nu.es_beta;
    for (int t = 0; t <= w; ++t) {
      std::vector<double> A((size_t)K * D), y(K);
      for (int i = 0; i < K; ++i) {
        const double u = std::cos(PI * (i + 0.5) / K), f = 0.5 * (u + 1);
        const double z = (t + f - 0.5 * w) / (0.5 * w);
        y[i] = std::fabs(z) < 1 ? std::exp(bb * (std::sqrt(1 - z * z) - 1)) : 0.0;
        double pw = 1;
        for (int k = 0; k < D; ++k) { A[(size_t)i * D + k] = pw; pw *= u; }
      }
      // Householder QR of A (K x D), then R c = Q^T y
      for (int k = 0; k < D; ++k) {
        double nrm = 0;
        for (int i = k; i < K; ++i) nrm += A[(size_t)i * D + k] * A[(size_t)i * D + k];
        nrm = std::sqrt(nrm);
        const double a0 = A[(size_t)k * D + k];
        const double alpha = a0 > 0 ? -nrm : nrm;
        std::vector<double> v(K, 0.0);
        v[k] = a0 - alpha;
        for (int i = k + 1; i < K; ++i) v[i] = A[(size_t)i * D + k];
        double vv = 0;
        for (int i = k; i < K; ++i) vv += v[i] * v[i];
        if (vv == 0) continue;
        for (int j = k; j < D; ++j) {
          double s2 = 0;
          for (int i = k; i < K; ++i) s2 += v[i] * A[(size_t)i * D + j];
          s2 *= 2 / vv;
          for (int i = k; i < K; ++i) A[(size_t)i * D + j] -= s2 * v[i];
        }
        double s2 = 0;
        for (int i = k; i < K; ++i) s2 += v[i] * y[i];
        s2 *= 2 / vv;
        for (int i = k; i < K; ++i) y[i] -= s2 * v[i];
      }
      double* c = &p->nu_poly[(size_t)t * ES_COEF];
      for (int k = D - 1; k >= 0; --k) {
        double s2 = y[k];
        for (int j = k + 1; j < D; ++j) s2 -= A[(size_t)k * D + j] * c[j];
        c[k] = s2 / A[(size_t)k * D + k];
      }
    }
  }
  p->nu_deconv.assign(M + 1, 0.0);
  std::vector<double> qx, qw;
  gauss_legendre(2 * w + 40, qx, qw);
  const double h = p->geo.d / nf, s = w * h / 2, b = p->nu.es_beta;
  for (int m = 0; m <= M; ++m) {
    const double al = 2 * PI * m / p->geo.d;
    double acc = 0;
    for (size_t i = 0; i < qx.size(); ++i)
      acc += qw[i] * std::exp(b * (std::sqrt(1 - qx[i] * qx[i]) - 1)) * std::cos(al * s * qx[i]);
    p->nu_deconv[m] = 1.0 / (0.5 * w * acc);
  }
  return PFMM_OK;
}

int build_plan(int kernel, const double* e1, const double* e2, double tol, const pfmm_opts* opts,
               pfmm_plan_s* p) {
  if (kernel < 0 || kernel > 2) return PFMM_EINVAL;
  if (!e1 || !e2) return PFMM_EINVAL;
  for (int i = 0; i < 2; ++i)
    if (!std::isfinite(e1[i]) || !std::isfinite(e2[i])) return PFMM_EINVAL_LATTICE;
  double det = e1[0] * e2[1] - e1[1] * e2[0];
  double scale = std::max(std::hypot(e1[0], e1[1]), std::hypot(e2[0], e2[1]));
  if (!(std::fabs(det) > 1e-12 * scale * scale)) return PFMM_EINVAL_LATTICE;
  if (!(tol >= 1e-14 && tol <= 1e-2)) return PFMM_EINVAL_TOL;

  pfmm_opts o{};
  o.n_dens = 1;
  if (opts) o = *opts;
  if (o.n_dens < 1 || o.n_dens > 64) return PFMM_EINVAL;
  if (kernel == PFMM_YUKAWA && !(o.beta > 0 && std::isfinite(o.beta))) return PFMM_EINVAL;
  if (o.precision != PFMM_FP64 && o.precision != PFMM_MIXED) return PFMM_EINVAL;
  if (o.far_mode < 0 || o.far_mode > 2) return PFMM_EINVAL;
  if (o.m0 < 0 || o.m0 > 3 || o.m_gl < 0 || o.m_gl > 32) return PFMM_EINVAL;
  if (o.periodic != 0 && o.periodic != 1 && o.periodic != 2) return PFMM_EINVAL;

  p->kernel = kernel;
  p->precision = o.precision;
  p->n_dens = o.n_dens;
  p->self_exclude = o.self_exclude ? 1 : 0;
  p->check_neutral = o.check_neutral ? 1 : 0;
  p->profile = o.profile ? 1 : 0;
  if (o.near_mode < 0 || o.near_mode > 4) return PFMM_EINVAL;
  if (o.near_mode == PFMM_NEAR_MUTUAL && !o.self_exclude) return PFMM_EINVAL;
  if (o.near_mode == PFMM_NEAR_FMM && o.periodic == 1) return PFMM_EINVAL;   // the FMM tree needs both periods
  p->near_none = o.near_mode == PFMM_NEAR_NONE ? 1 : 0;
  p->mutual = (o.near_mode != PFMM_NEAR_ONE_SIDED && !p->near_none && o.self_exclude) ? 1 : 0;
  p->near_fmm = o.near_mode == PFMM_NEAR_FMM ? 1 : (o.near_mode == PFMM_NEAR_AUTO ? 2 : 0);
  p->fmm_order = fmm_order(kernel, o.precision, tol);
  p->beta = kernel == PFMM_YUKAWA ? o.beta : 0.0;
  p->tol = tol;
  p->eps = tol / 10;

  // --- canonical lattice (Sec. 1): e1 = (d, 0) the longer reduced vector,
  // e2 = (xi, eta) with eta > 0 and |xi| <= d/2. Singly periodic (P1):
  // e1 is the period and is not reduced; the cell is the strip of width d
  // and height eta (the part of e2 across e1), xi = 0.
  const bool p1 = o.periodic == 1;
  double b1[2] = {e1[0], e1[1]}, b2[2] = {e2[0], e2[1]};
  if (!p1) reduce_basis(b1, b2);
  else { std::swap(b1[0], b2[0]); std::swap(b1[1], b2[1]); }
  const double d = std::hypot(b2[0], b2[1]);
  const double rc = b2[0] / d, rs = -b2[1] / d;  // R rotates b2 onto +x
  double xi = rc * b1[0] - rs * b1[1];
  double eta = rs * b1[0] + rc * b1[1];
  if (eta < 0) { xi = -xi; eta = -eta; }
  xi -= d * std::nearbyint(xi / d);
  if (p1) xi = 0.0;
  p->periodic = p1 ? 1 : 2;
  pfmm::Geometry& g = p->geo;
  g.d = d; g.xi = xi; g.eta = eta; g.rc = rc; g.rs = rs;

  // --- near region (Def. 1): m0 = 1 keeps the closest west/east image at
  // x-distance >= d - 2|xi| (Thm. west_thm proof); require that to be >= d/2.
  g.sigma = 1.0;
  g.lg_shift = 0;
  if (o.precision == PFMM_MIXED && kernel != PFMM_YUKAWA) {
    const int k = (int)std::lround(-0.5 * std::log2(d * eta));
    g.sigma = std::ldexp(1.0, k);
    g.lg_shift = 2 * k;
  }
  // west/east frame: the canonical one keeps the closest west/east image at
  // x-distance m0 d - 2|xi|, enough with m0 = 1 while |xi| <= d/4. Beyond
  // that the waves are taken along e2-perp instead (Appendix A): the closest
  // west/east image is then one full column, dx' = d eta/|e2|, away, and
  // m0 = 1 (9 near images) holds for every shear. An explicit m0 >= 2 keeps
  // the canonical frame.
  int m0 = 1;
  p->ew_rotated = 0;
  if (o.m0 > 0) m0 = o.m0;
  else if (!p1 && std::fabs(xi) > 0.25 * d) p->ew_rotated = 1;
  if (!p1 && o.m0 == 1 && std::fabs(xi) > 0.25 * d) p->ew_rotated = 1;
  p->m0 = m0;
  {
    const double l2 = std::hypot(xi, eta);
    if (p->ew_rotated) {
      p->ew_c = eta / l2; p->ew_s = xi / l2;
      p->ew_dx = d * eta / l2; p->ew_dy = d * xi / l2; p->ew_xi = 0.0; p->ew_eta = l2;
    } else {
      p->ew_c = 1.0; p->ew_s = 0.0;
      p->ew_dx = d; p->ew_dy = 0.0; p->ew_xi = xi; p->ew_eta = eta;
    }
    // the west/east rows: n = -1, 0, 1 (P2) or n = 0 alone (P1)
    p->ew_rows = p1 ? 1 : 3;
    if (p1) p->ew_eta = 0.0;
  }
  g.n_images = 0;
  for (int n = p1 ? 0 : -1; n <= (p1 ? 0 : 1); ++n)
    for (int m = -m0; m <= m0; ++m) {
      g.img_x[g.n_images] = m * d + n * xi;
      g.img_y[g.n_images] = n * eta;
      ++g.n_images;
    }
  plan_log_groups(g, 2 * m0 + 1);

  const double eps = p->eps;
  const double beta = p->beta;
  // --- south/north truncation (eq. mpk0s)
  int M = (int)std::ceil(d / (2 * PI * eta) * std::log(1.0 / ((1 - std::exp(-2 * PI * eta / d)) * eps)));
  M = std::max(M, 1);
  p->m_lo = kernel == PFMM_YUKAWA ? 0 : 1;
  if (p1) M = p->m_lo - 1;   // no south/north rows
  // for Yukawa, drop modes whose whole contribution e^{-chi_m eta} is below eps
  if (kernel == PFMM_YUKAWA) {
    while (M > 0) {
      double al = 2 * PI * M / d, chi = std::sqrt(al * al + beta * beta);
      if (chi * eta > std::log(1.0 / eps) + 3) --M; else break;
    }
  }
  p->M = M;
  p->n_sn = std::max(0, M - p->m_lo + 1);
  p->sn_tab.assign((size_t)p->n_sn * SN_REC, 0.0);
  for (int i = 0; i < p->n_sn; ++i) {
    int m = p->m_lo + i;
    double al = 2 * PI * m / d;
    double a = kernel == PFMM_YUKAWA ? std::sqrt(al * al + beta * beta) : std::fabs(al);
    cd Q(a * eta, -al * xi);
    cd eQ = std::exp(-Q);
    cd T = eQ * eQ / (1.0 - eQ);                  // sum_{p>=2} e^{-pQ}
    double fac = (m == 0) ? 1.0 : 2.0;
    cd D = (kernel == PFMM_STOKES) ? fac * T / (4 * d) : fac * T / (2 * d * a);
    cd tau = (2.0 - eQ) / (1.0 - eQ);
    double* r = &p->sn_tab[(size_t)i * SN_REC];
    r[0] = al; r[1] = a; r[2] = D.real(); r[3] = D.imag(); r[4] = tau.real(); r[5] = tau.imag();
  }

  // --- west/east rule and weights (in the west/east frame)
  if (p1)
    ew_rule_adaptive(kernel, beta, d, 0.0, 0.0, 0.0, 1, eta, m0, eps, p->ew_nodes, p->ew_weights);
  else if (p->ew_rotated)
    ew_rule_adaptive(kernel, beta, p->ew_dx, p->ew_dy, p->ew_xi, p->ew_eta, 3, std::fabs(p->ew_dy) + p->ew_eta, m0,
                     eps, p->ew_nodes, p->ew_weights);
  else {
    ew_rule(kernel, beta, d, xi, eta, m0, eps, p->ew_nodes, p->ew_weights);
    if (o.ew_rule != 1) compress_rule(kernel, beta, m0 * d - 2 * std::fabs(xi), 2 * eta, eps, p->ew_nodes, p->ew_weights);
  }
  p->n_ew = (int)p->ew_nodes.size();
  p->ew_tab.assign((size_t)p->n_ew * EW_REC, 0.0);
  const int pp = m0 + 1;
  for (int k = 0; k < p->n_ew; ++k) {
    double lam = p->ew_nodes[k], w = p->ew_weights[k];
    double kap = kernel == PFMM_YUKAWA ? std::sqrt(lam * lam + beta * beta) : lam;
    const cd a(kap * p->ew_dx, -lam * p->ew_dy);
    const cd ea = std::exp(-a), om = one_minus_exp(a);
    const cd R = std::exp(-double(pp) * a) / om;
    const double x2 = p->ew_xi, y2 = p->ew_eta;
    cd B = p1 ? cd(1.0) : std::exp(cd(-kap * x2, lam * y2)) + std::exp(cd(kap * x2, -lam * y2)) + 1.0;
    double* r = &p->ew_tab[(size_t)k * EW_REC];
    r[0] = lam; r[1] = kap;
    if (kernel == PFMM_STOKES) {
      cd Bp = p1 ? cd(0.0) : -std::exp(cd(-lam * x2, lam * y2)) + std::exp(cd(lam * x2, -lam * y2));
      cd P = (double(pp) - double(pp - 1) * ea) / om;
      cd pre = w * R / (4 * PI), dP = p->ew_dx * P;
      r[2] = pre.real(); r[3] = pre.imag(); r[4] = B.real(); r[5] = B.imag();
      r[6] = Bp.real(); r[7] = Bp.imag(); r[8] = dP.real(); r[9] = dP.imag();
    } else {
      cd DW = w * R * B / (2 * PI * kap), DE = std::conj(DW);
      r[2] = DW.real(); r[3] = DW.imag(); r[4] = DE.real(); r[5] = DE.imag();
    }
  }

  // --- far mode and NUFFT parameters (Sec. 6.1)
  // NUFFT needs a grid of at least twice the 2M+1 modes; lines up to 4096
  // points are transformed in one block's LDS, longer ones in two passes
  const bool nufft_fits = 2 * (2 * M + 1) <= NUFFT_MAX_GRID;
  int far = o.far_mode;
  if (p1 && far == PFMM_FAR_NUFFT) return PFMM_EINVAL;   // no south/north part to accelerate
  if (p1) far = PFMM_FAR_DIRECT;
  if (far == PFMM_FAR_AUTO) far = (2 * M + 1 >= 256 && nufft_fits) ? PFMM_FAR_NUFFT : PFMM_FAR_DIRECT;
  if (far == PFMM_FAR_NUFFT && !nufft_fits) return PFMM_EINVAL;
  p->far_mode = far;
  p->use_nufft = far == PFMM_FAR_NUFFT;
  int mgl = o.m_gl;
  if (mgl == 0) mgl = eps >= 1e-7 ? 8 : (eps >= 1e-10 ? 12 : 16);  // rho0^-M_GL, rho0 = 3+sqrt 8
  p->nu.m_gl = mgl;
  set_nufft_grid(p, 0);
  std::vector<double> tx, tw;
  gauss_legendre(mgl, tx, tw);
  p->gl_nodes.resize(mgl);
  p->gl_bary.resize(mgl);
  for (int k = 0; k < mgl; ++k) {
    p->gl_nodes[k] = 0.5 * eta * tx[k];
    double s = 1;
    for (int j = 0; j < mgl; ++j)
      if (j != k) s *= (tx[k] - tx[j]);
    p->gl_bary[k] = 1.0 / s;
  }

  p->dev_id = -1;
  p->d_tab = nullptr;
  p->tab_doubles = 0;
  return PFMM_OK;
}

}  // namespace pfmm
