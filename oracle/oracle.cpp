// FP64 CPU oracle for doubly periodic potentials and gradients.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
// calls this file; only the test suite, the smoke check and the benchmark's
// CPU-baseline leg do. It shares no code, header, table or constant with
// the GPU path.
//
// What it computes is the plain definition of the periodic sum (Sec. 1,
// eq. psum): for targets t_i and sources s_j with densities q_j in a cell
// of the lattice {m e1 + n e2},
//     u(t_i) = sum_j sum_{(m,n) in Z^2} G(t_i - s_j - m e1 - n e2) q_j
// and its gradient, with the term (j == i, m = n = 0) left out when the
// targets are the sources. The free-space kernels are
//     Laplace:   G = -(1/2pi) log r                       (Sec. 1)
//     Yukawa:    G = (1/2pi) K0(beta r)                   (Sec. 1)
//     Stokeslet: G = -(1/4pi)(log r I - r r^T / r^2)      (Sec. 5.2, eq. stokeslet)
//     modified Stokeslet (Brinkman): the operator of Sec. 5 eq. msgreen on
//                G_MB = -(K0(beta r) + log r)/(2 pi beta^2)
// The Laplace and Stokes sums converge only conditionally; they need
// sum_j q_j = 0 (Sec. 1 eq. chargeneutral) and are defined here as the
// periodic ("tin-foil") solution with zero mean over the cell, which is
// what the paper's construction gives once its free constant is fixed
// (Sec. 4 says the potential is unique up to a constant).
//
// Methods (none is the paper's method):
//   * Laplace: Ewald split with parameter alpha. Real space uses
//     (1/4pi) E1(alpha^2 r^2); reciprocal space uses
//     (1/|C|) sum_{k != 0} exp(-k^2/4alpha^2)/k^2 e^{ik.t} S(k).
//     Self term: -q_i (gamma + 2 ln alpha)/(4pi).
//   * Laplace cross-check: closed-form sum over rows parallel to e1
//     (sine-product formula per row), plus the uniform-field term that
//     makes the slab-ordered sum periodic and the constant that makes
//     the cell mean zero. Needs the canonical lattice e1 = (d, 0) and all
//     points in the strip |y| <= eta/2.
//   * Yukawa: direct lattice sum truncated at a radius past which the
//     K0 tail is below the requested tolerance.
//   * Stokes: Ewald with the Hasimoto split phi(k) = (1 + k^2/4a^2) e^{-k^2/4a^2}:
//     real space (1/4pi)[(E1(x)/2 - e^{-x}) I + e^{-x} r r^T/r^2], x = a^2 r^2;
//     reciprocal (1/|C|) sum_{k!=0} (I - k k^T/k^2) phi(k)/k^2 e^{ik.t} F(k);
//     self term -(1/4pi)((gamma + 2 ln a)/2 + 1) f_i.
//   * modified Stokes: G = [G_Y I - Hess G_Y / beta^2] + Hess G_L / beta^2
//     (G_L, G_Y the Laplace and Yukawa kernels above); the bracket by a
//     direct lattice sum, Hess G_L by an Ewald split (k != 0), so the cell
//     mean of u is the net force / (beta^2 |C|) and no neutrality is needed.
// Special functions come from the C++17 standard library (std::expint,
// std::cyl_bessel_k).
//
// Layouts: points are SoA, x[n] then y[n]. Outputs are written, not
// accumulated. Return 0 on success, negative on bad input.

#include <cmath>
#include <complex>
#include <vector>
#include <algorithm>
#include <cstdint>
#include <cstdio>

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double EULER_GAMMA = 0.57721566490153286061;

double E1(double x) { return -std::expint(-x); }

struct Lattice {
  double e1x, e1y, e2x, e2y;
  double area;             // |e1 x e2|
  double b1x, b1y, b2x, b2y; // reciprocal basis, b_i . e_j = 2 pi delta_ij
};

int make_lattice(const double* e1, const double* e2, Lattice* L) {
  L->e1x = e1[0]; L->e1y = e1[1]; L->e2x = e2[0]; L->e2y = e2[1];
  double det = e1[0] * e2[1] - e1[1] * e2[0];
  if (!(std::fabs(det) > 0) || !std::isfinite(det)) return -1;
  L->area = std::fabs(det);
  // b1 = 2 pi (e2y, -e2x)/det, b2 = 2 pi (-e1y, e1x)/det
  L->b1x = 2 * PI * e2[1] / det;  L->b1y = -2 * PI * e2[0] / det;
  L->b2x = -2 * PI * e1[1] / det; L->b2y = 2 * PI * e1[0] / det;
  return 0;
}

// Move r to its image closest to the origin in lattice coordinates
// (components in (-1/2, 1/2]); only used to keep the image enumeration short.
void lattice_reduce(const Lattice& L, double& rx, double& ry) {
  double u1 = (rx * L.b1x + ry * L.b1y) / (2 * PI);
  double u2 = (rx * L.b2x + ry * L.b2y) / (2 * PI);
  double k1 = std::nearbyint(u1), k2 = std::nearbyint(u2);
  rx -= k1 * L.e1x + k2 * L.e2x;
  ry -= k1 * L.e1y + k2 * L.e2y;
}

// All lattice vectors l with |l| <= R (R >= 0).
std::vector<double> lattice_ball(const Lattice& L, double R) {
  // distance between adjacent lattice lines of constant m is area/|e2|
  double h1 = L.area / std::hypot(L.e2x, L.e2y);
  double h2 = L.area / std::hypot(L.e1x, L.e1y);
  long M = (long)std::ceil(R / h1) + 1, N = (long)std::ceil(R / h2) + 1;
  std::vector<double> out;
  for (long m = -M; m <= M; ++m)
    for (long n = -N; n <= N; ++n) {
      double lx = m * L.e1x + n * L.e2x, ly = m * L.e1y + n * L.e2y;
      if (std::hypot(lx, ly) <= R) { out.push_back(lx); out.push_back(ly); }
    }
  return out;
}

// Reciprocal vectors k = h1 b1 + h2 b2 with 0 < |k| <= K.
std::vector<double> reciprocal_ball(const Lattice& L, double K) {
  // h1 = k.e1/(2 pi), h2 = k.e2/(2 pi), so |h_i| <= K |e_i| / (2 pi)
  long H1 = (long)std::ceil(K * std::hypot(L.e1x, L.e1y) / (2 * PI)) + 1;
  long H2 = (long)std::ceil(K * std::hypot(L.e2x, L.e2y) / (2 * PI)) + 1;
  std::vector<double> out;
  for (long a = -H1; a <= H1; ++a)
    for (long b = -H2; b <= H2; ++b) {
      if (a == 0 && b == 0) continue;
      double kx = a * L.b1x + b * L.b2x, ky = a * L.b1y + b * L.b2y;
      if (std::hypot(kx, ky) <= K) { out.push_back(kx); out.push_back(ky); }
    }
  return out;
}

double max_extent(const Lattice& L, const double* x, const double* y, int64_t n) {
  double m = 0;
  for (int64_t i = 0; i < n; ++i) {
    double rx = x[i], ry = y[i];
    lattice_reduce(L, rx, ry);
    m = std::max(m, std::hypot(rx, ry));
  }
  return m;
}

// Second and third derivatives of a radial function g(|x|) at x = (rx, ry),
// from the first three radial derivatives d1, d2, d3 of g at r = |x|:
//   H_ij  = b x_i x_j + a delta_ij,
//   T_ijk = c x_i x_j x_k + b (delta_ij x_k + delta_ik x_j + delta_jk x_i),
//   a = d1/r, b = (d2 - d1/r)/r^2, c = (d3 - 3 d2/r + 3 d1/r^2)/r^3.
void radial_derivs(double rx, double ry, double d1, double d2, double d3,
                   double H[2][2], double T[2][2][2]) {
  const double r2 = rx * rx + ry * ry, r = std::sqrt(r2);
  const double a = d1 / r, b = (d2 - d1 / r) / r2;
  const double c = (d3 - 3 * d2 / r + 3 * d1 / r2) / (r2 * r);
  const double x[2] = {rx, ry};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      H[i][j] = b * x[i] * x[j] + (i == j ? a : 0.0);
      for (int k = 0; k < 2; ++k)
        T[i][j][k] = c * x[i] * x[j] * x[k] +
                     b * ((i == j ? x[k] : 0.0) + (i == k ? x[j] : 0.0) + (j == k ? x[i] : 0.0));
    }
}

}  // namespace

extern "C" {

// Laplace, Ewald split. dens: q[ns]. out_pot[nt], out_grad[2][nt] (may be NULL).
// self_idx (may be NULL): self_idx[i] = j >= 0 means target i sits exactly on
// source j and the term (j, zero lattice vector) is left out; -1 = none.
// alpha <= 0 picks a default. tol sets both cut-offs.
int oracle_laplace_ewald(const double* e1, const double* e2, double alpha, double tol,
                         int64_t ns, const double* sx, const double* sy, const double* q,
                         int64_t nt, const double* tx, const double* ty, const int64_t* self_idx,
                         double* out_pot, double* out_grad) {
  Lattice L;
  if (make_lattice(e1, e2, &L)) return -1;
  if (!(tol > 0 && tol < 1)) return -3;
  if (alpha <= 0) {
    double nn = std::max<double>(1.0, (double)ns * nt / (double)(ns + nt));
    alpha = std::sqrt(PI * std::sqrt(nn) / L.area);
    alpha = std::max(alpha, 4.0 / std::sqrt(L.area));
  }
  const double xc = std::log(1.0 / tol) + 3.0;      // alpha^2 rc^2
  const double rc = std::sqrt(xc) / alpha;
  const double kc = 2.0 * alpha * std::sqrt(xc);
  // Differences t - s are reduced to the nearest image first, so |r0| <= 2*ext.
  double ext = std::max(max_extent(L, sx, sy, ns), max_extent(L, tx, ty, nt));
  std::vector<double> img = lattice_ball(L, rc + 2 * ext + 1e-12);
  std::vector<double> kv = reciprocal_ball(L, kc);
  const size_t nimg = img.size() / 2, nk = kv.size() / 2;

  // structure factor S(k) = sum_j q_j exp(-i k.s_j)
  std::vector<double> Sre(nk), Sim(nk), coef(nk);
#pragma omp parallel for schedule(dynamic, 4)
  for (long a = 0; a < (long)nk; ++a) {
    double kx = kv[2 * a], ky = kv[2 * a + 1];
    double re = 0, im = 0;
    for (int64_t j = 0; j < ns; ++j) {
      double ph = kx * sx[j] + ky * sy[j];
      re += q[j] * std::cos(ph);
      im -= q[j] * std::sin(ph);
    }
    Sre[a] = re; Sim[a] = im;
    double k2 = kx * kx + ky * ky;
    coef[a] = std::exp(-k2 / (4 * alpha * alpha)) / k2 / L.area;
  }
  const double a2 = alpha * alpha;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
  for (int64_t i = 0; i < nt; ++i) {
    double pot = 0, gx = 0, gy = 0;
    // real space
    for (int64_t j = 0; j < ns; ++j) {
      double r0x = tx[i] - sx[j], r0y = ty[i] - sy[j];
      double bx = r0x, by = r0y;
      lattice_reduce(L, bx, by);
      for (size_t l = 0; l < nimg; ++l) {
        double rx = bx - img[2 * l], ry = by - img[2 * l + 1];
        double r2 = rx * rx + ry * ry;
        if (r2 > rc * rc) continue;
        if (r2 == 0) {
          // target i sitting exactly on source self_idx[i]: that is the
          // excluded (j == i, zero lattice vector) term; any other r == 0 is an error
          if (!(self_idx && j == self_idx[i])) bad = 1;
          continue;
        }
        double x = a2 * r2;
        pot += q[j] * E1(x) / (4 * PI);
        double g = -q[j] * std::exp(-x) / (2 * PI * r2);
        gx += g * rx; gy += g * ry;
      }
    }
    // reciprocal space
    for (size_t a = 0; a < nk; ++a) {
      double kx = kv[2 * a], ky = kv[2 * a + 1];
      double ph = kx * tx[i] + ky * ty[i];
      double c = std::cos(ph), s = std::sin(ph);
      // e^{ik.t} S(k)
      double re = c * Sre[a] - s * Sim[a];
      double im = c * Sim[a] + s * Sre[a];
      pot += coef[a] * re;
      gx -= coef[a] * kx * im;
      gy -= coef[a] * ky * im;
    }
    if (self_idx && self_idx[i] >= 0) pot -= q[self_idx[i]] * (EULER_GAMMA + 2 * std::log(alpha)) / (4 * PI);
    if (out_pot) out_pot[i] = pot;
    if (out_grad) { out_grad[i] = gx; out_grad[nt + i] = gy; }
  }
  return bad ? -4 : 0;
}

// Laplace, closed-form row sums. Canonical lattice e1 = (d, 0), e2 = (xi, eta),
// every point with |y| <= eta/2 (checked). nrows: rows summed on each side of
// the target's own row (terms decay like exp(-2 pi n eta / d)).
int oracle_laplace_rowsum(double d, double xi, double eta, int nrows,
                          int64_t ns, const double* sx, const double* sy, const double* q,
                          int64_t nt, const double* tx, const double* ty, const int64_t* self_idx,
                          double* out_pot, double* out_grad) {
  if (!(d > 0 && eta > 0)) return -1;
  const double hh = 0.5 * eta * (1 + 1e-12);
  for (int64_t j = 0; j < ns; ++j) if (std::fabs(sy[j]) > hh) return -5;
  for (int64_t i = 0; i < nt; ++i) if (std::fabs(ty[i]) > hh) return -5;
  double Py = 0, Qyy = 0;
  for (int64_t j = 0; j < ns; ++j) { Py += q[j] * sy[j]; Qyy += q[j] * sy[j] * sy[j]; }
  const double kap = 2 * PI / d;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < nt; ++i) {
    double pot = 0, gx = 0, gy = 0;
    for (int64_t j = 0; j < ns; ++j) {
      for (int n = -nrows; n <= nrows; ++n) {
        double wx = tx[i] - sx[j] - n * xi, wy = ty[i] - sy[j] - n * eta;
        // row sum over m of -(1/2pi) log|w - m d| = -|wy|/(2d) - (1/2pi) log|1 - e^{i kap sg w}| + const
        double sg = (wy >= 0) ? 1.0 : -1.0;
        if (n == 0 && self_idx && j == self_idx[i]) {
          // the row through the target itself, without the m = 0 term:
          // sum_{m != 0} -(1/2pi) log|m d| is a constant (dropped by neutrality
          // together with the other constants of the row sums) ...
          // ... so the row contributes -(1/2pi) log( lim_{w->0} |1 - e^{i kap w}|/|w| ) = -(1/2pi) log(kap).
          pot += -q[j] * std::log(kap) / (2 * PI);
          continue;
        }
        // |1 - e^{i kap sg w}| with w = wx + i wy: e^{i kap sg w} = e^{-kap |wy|} e^{i kap sg wx}
        double rho = std::exp(-kap * std::fabs(wy));
        double c = std::cos(kap * sg * wx), s = std::sin(kap * sg * wx);
        double gre = 1 - rho * c, gim = -rho * s;  // g = 1 - e^{...}
        double mod2 = gre * gre + gim * gim;
        pot += q[j] * (-std::fabs(wy) / (2 * d) - std::log(mod2) / (4 * PI));
        // g'/g with g' = -i kap sg e^{...}
        double epre = rho * c, epim = rho * s;               // e^{...}
        double dre = kap * sg * epim, dim = -kap * sg * epre; // -i kap sg e
        // (dre + i dim)/(gre + i gim)
        double fre = (dre * gre + dim * gim) / mod2;
        double fim = (dim * gre - dre * gim) / mod2;
        // grad log|g| = (Re f, -Im f); term is -(1/2pi) log|g|
        gx += q[j] * (-fre / (2 * PI));
        gy += q[j] * (fim / (2 * PI) - sg / (2 * d));
      }
    }
    pot += -ty[i] * Py / (d * eta) + Qyy / (2 * d * eta);
    gy += -Py / (d * eta);
    if (out_pot) out_pot[i] = pot;
    if (out_grad) { out_grad[i] = gx; out_grad[nt + i] = gy; }
  }
  return 0;
}

// Yukawa G = (1/2pi) K0(beta r): direct lattice sum over all images within
// radius R chosen from the tail bound (see body). dens q[ns].
int oracle_yukawa_lattice(const double* e1, const double* e2, double beta, double tol,
                          int64_t ns, const double* sx, const double* sy, const double* q,
                          int64_t nt, const double* tx, const double* ty, const int64_t* self_idx,
                          double* out_pot, double* out_grad) {
  Lattice L;
  if (make_lattice(e1, e2, &L)) return -1;
  if (!(beta > 0) || !(tol > 0 && tol < 1)) return -3;
  // Tail: sum over images farther than R of K0(beta r)/(2pi) is bounded by
  // (1/|C|) int_{R-diam}^inf K0(beta rho) 2 pi rho drho / (2pi) <= K0-type
  // decay; R is grown until (1 + 2pi R/(beta |C|)) K0(beta R) < tol.
  double R = 1.0 / beta;
  while ((1 + 2 * PI * R / (beta * L.area)) * std::cyl_bessel_k(0.0, beta * R) > tol) R *= 1.1;
  double ext = std::max(max_extent(L, sx, sy, ns), max_extent(L, tx, ty, nt));
  std::vector<double> img = lattice_ball(L, R + 2 * ext + 1e-12);
  const size_t nimg = img.size() / 2;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
  for (int64_t i = 0; i < nt; ++i) {
    double pot = 0, gx = 0, gy = 0;
    for (int64_t j = 0; j < ns; ++j) {
      double bx = tx[i] - sx[j], by = ty[i] - sy[j];
      lattice_reduce(L, bx, by);
      for (size_t l = 0; l < nimg; ++l) {
        double rx = bx - img[2 * l], ry = by - img[2 * l + 1];
        double r2 = rx * rx + ry * ry;
        if (r2 > R * R) continue;
        if (r2 == 0) {
          // target i sitting exactly on source self_idx[i]: that is the
          // excluded (j == i, zero lattice vector) term; any other r == 0 is an error
          if (!(self_idx && j == self_idx[i])) bad = 1;
          continue;
        }
        double r = std::sqrt(r2);
        pot += q[j] * std::cyl_bessel_k(0.0, beta * r) / (2 * PI);
        double g = -q[j] * beta * std::cyl_bessel_k(1.0, beta * r) / (2 * PI * r);
        gx += g * rx; gy += g * ry;
      }
    }
    if (out_pot) out_pot[i] = pot;
    if (out_grad) { out_grad[i] = gx; out_grad[nt + i] = gy; }
  }
  return bad ? -4 : 0;
}

// Stokeslet (mu = 1), Ewald with the Hasimoto split. dens f[2][ns] (f1 then f2).
// out_vel[2][nt], out_grad[4][nt] = (du1/dx, du1/dy, du2/dx, du2/dy).
int oracle_stokes_ewald(const double* e1, const double* e2, double alpha, double tol,
                        int64_t ns, const double* sx, const double* sy, const double* f,
                        int64_t nt, const double* tx, const double* ty, const int64_t* self_idx,
                        double* out_vel, double* out_grad) {
  Lattice L;
  if (make_lattice(e1, e2, &L)) return -1;
  if (!(tol > 0 && tol < 1)) return -3;
  if (alpha <= 0) {
    double nn = std::max<double>(1.0, (double)ns * nt / (double)(ns + nt));
    alpha = std::sqrt(PI * std::sqrt(nn) / L.area);
    alpha = std::max(alpha, 4.0 / std::sqrt(L.area));
  }
  const double* f1 = f;
  const double* f2 = f + ns;
  const double lt = std::log(1.0 / tol);
  const double xc = lt + 3.0;
  const double rc = std::sqrt(xc) / alpha;
  const double kc = 2.0 * alpha * std::sqrt(lt + std::log(2.0 + lt) + 3.0);
  double ext = std::max(max_extent(L, sx, sy, ns), max_extent(L, tx, ty, nt));
  std::vector<double> img = lattice_ball(L, rc + 2 * ext + 1e-12);
  std::vector<double> kv = reciprocal_ball(L, kc);
  const size_t nimg = img.size() / 2, nk = kv.size() / 2;
  const double a2 = alpha * alpha;

  // F(k) = sum_j f_j exp(-i k.s_j) (two complex components), then the
  // Fourier multiplier (I - k k^T/k^2) phi(k)/(k^2 |C|) applied once per k.
  std::vector<double> Are(nk), Aim(nk), Bre(nk), Bim(nk);
#pragma omp parallel for schedule(dynamic, 4)
  for (long a = 0; a < (long)nk; ++a) {
    double kx = kv[2 * a], ky = kv[2 * a + 1];
    double F1r = 0, F1i = 0, F2r = 0, F2i = 0;
    for (int64_t j = 0; j < ns; ++j) {
      double ph = kx * sx[j] + ky * sy[j];
      double c = std::cos(ph), s = std::sin(ph);
      F1r += f1[j] * c; F1i -= f1[j] * s;
      F2r += f2[j] * c; F2i -= f2[j] * s;
    }
    double k2 = kx * kx + ky * ky;
    double phi = (1 + k2 / (4 * a2)) * std::exp(-k2 / (4 * a2));
    double s = phi / (k2 * L.area);
    double p11 = 1 - kx * kx / k2, p12 = -kx * ky / k2, p22 = 1 - ky * ky / k2;
    Are[a] = s * (p11 * F1r + p12 * F2r); Aim[a] = s * (p11 * F1i + p12 * F2i);
    Bre[a] = s * (p12 * F1r + p22 * F2r); Bim[a] = s * (p12 * F1i + p22 * F2i);
  }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
  for (int64_t i = 0; i < nt; ++i) {
    double u1 = 0, u2 = 0, g11 = 0, g12 = 0, g21 = 0, g22 = 0;  // gIJ = d u_I / d x_J
    for (int64_t j = 0; j < ns; ++j) {
      double bx = tx[i] - sx[j], by = ty[i] - sy[j];
      lattice_reduce(L, bx, by);
      for (size_t l = 0; l < nimg; ++l) {
        double rx = bx - img[2 * l], ry = by - img[2 * l + 1];
        double r2 = rx * rx + ry * ry;
        if (r2 > rc * rc) continue;
        if (r2 == 0) {
          // target i sitting exactly on source self_idx[i]: that is the
          // excluded (j == i, zero lattice vector) term; any other r == 0 is an error
          if (!(self_idx && j == self_idx[i])) bad = 1;
          continue;
        }
        double x = a2 * r2, ex = std::exp(-x), e1v = E1(x);
        double fx = f1[j], fy = f2[j];
        double rf = rx * fx + ry * fy;
        // G_r f = (1/4pi)[(E1/2 - e^{-x}) f + e^{-x} (r.f) r / r^2]
        double cI = 0.5 * e1v - ex;
        u1 += (cI * fx + ex * rf * rx / r2) / (4 * PI);
        u2 += (cI * fy + ex * rf * ry / r2) / (4 * PI);
        // d/dx_k of the above:
        //   d(cI)/dx_k = -e^{-x} r_k/r^2 + 2 a^2 e^{-x} r_k
        //   d(e^{-x} (r.f) r_i / r^2)/dx_k = -2a^2 r_k e^{-x} (r.f) r_i/r^2
        //        + e^{-x} [ f_k r_i + (r.f) delta_ik ]/r^2 - 2 e^{-x} (r.f) r_i r_k / r^4
        double r[2] = {rx, ry}, ff[2] = {fx, fy};
        double gg[2][2];
        for (int ii = 0; ii < 2; ++ii)
          for (int kk = 0; kk < 2; ++kk) {
            double dcI = -ex * r[kk] / r2 + 2 * a2 * ex * r[kk];
            double t = dcI * ff[ii];
            t += -2 * a2 * r[kk] * ex * rf * r[ii] / r2;
            t += ex * (ff[kk] * r[ii] + (ii == kk ? rf : 0.0)) / r2;
            t += -2 * ex * rf * r[ii] * r[kk] / (r2 * r2);
            gg[ii][kk] = t / (4 * PI);
          }
        g11 += gg[0][0]; g12 += gg[0][1]; g21 += gg[1][0]; g22 += gg[1][1];
      }
    }
    for (size_t a = 0; a < nk; ++a) {
      double kx = kv[2 * a], ky = kv[2 * a + 1];
      double ph = kx * tx[i] + ky * ty[i];
      double c = std::cos(ph), s = std::sin(ph);
      double Ar = c * Are[a] - s * Aim[a], Ai = c * Aim[a] + s * Are[a];
      double Br = c * Bre[a] - s * Bim[a], Bi = c * Bim[a] + s * Bre[a];
      u1 += Ar; u2 += Br;
      // Re(i k_l e^{ik.t} A) = -k_l Im(...)
      g11 -= kx * Ai; g12 -= ky * Ai; g21 -= kx * Bi; g22 -= ky * Bi;
    }
    if (self_idx && self_idx[i] >= 0) {
      double c = ((EULER_GAMMA + 2 * std::log(alpha)) / 2 + 1) / (4 * PI);
      u1 -= c * f1[self_idx[i]]; u2 -= c * f2[self_idx[i]];
    }
    if (out_vel) { out_vel[i] = u1; out_vel[nt + i] = u2; }
    if (out_grad) {
      out_grad[i] = g11; out_grad[nt + i] = g12; out_grad[2 * nt + i] = g21; out_grad[3 * nt + i] = g22;
    }
  }
  return bad ? -4 : 0;
}

// Modified Stokeslet (Sec. 5, eq. msgreen): the fundamental solution of
// (beta^2 - Laplacian) u + grad p = f delta, div u = 0, built from the
// modified biharmonic Green's function G_MB = -(K0(beta r) + log r)/(2 pi beta^2).
// With G_L = -(1/2pi) log r and G_Y = (1/2pi) K0(beta r), G_MB = (G_L - G_Y)/beta^2
// and Laplacian G_MB = -G_Y, so the Stokeslet splits as
//     G_MS = [G_Y I - (1/beta^2) Hess G_Y] + (1/beta^2) Hess G_L.
// The bracket decays like K0 and is summed directly over the lattice (as
// the Yukawa sum); the Hessian of G_L is summed by an Ewald split of G_L
// (real space (1/4pi) E1(alpha^2 r^2), reciprocal e^{-k^2/4alpha^2}/k^2,
// k != 0), i.e. it is the Hessian of the zero-mean periodic Laplace
// Green's function. Hence the cell mean of u is (sum_j f_j)/(beta^2 |C|),
// Brinkman flow with a periodic pressure; no neutrality is needed.
// dens f[2][ns]; out_vel[2][nt], out_grad[4][nt] = (du1/dx, du1/dy,
// du2/dx, du2/dy). A target on its own source leaves out that whole term.
int oracle_mstokes(const double* e1, const double* e2, double beta, double alpha, double tol,
                   int64_t ns, const double* sx, const double* sy, const double* f,
                   int64_t nt, const double* tx, const double* ty, const int64_t* self_idx,
                   double* out_vel, double* out_grad) {
  Lattice L;
  if (make_lattice(e1, e2, &L)) return -1;
  if (!(beta > 0) || !(tol > 0 && tol < 1)) return -3;
  if (alpha <= 0) {
    double nn = std::max<double>(1.0, (double)ns * nt / (double)(ns + nt));
    alpha = std::sqrt(PI * std::sqrt(nn) / L.area);
    alpha = std::max(alpha, 4.0 / std::sqrt(L.area));
  }
  const double* f1 = f;
  const double* f2 = f + ns;
  const double ib2 = 1.0 / (beta * beta);
  // screened part: every term is bounded by a multiple of K0(beta r) + K1(beta r)
  double R = 1.0 / beta;
  while ((1 + 2 * PI * R / (beta * L.area)) *
             (std::cyl_bessel_k(0.0, beta * R) + std::cyl_bessel_k(1.0, beta * R)) > tol)
    R *= 1.1;
  // Laplace Hessian: Ewald cut-offs as for the Stokes sum
  const double lt = std::log(1.0 / tol);
  const double rc = std::sqrt(lt + 3.0) / alpha;
  const double kc = 2.0 * alpha * std::sqrt(lt + std::log(2.0 + lt) + 3.0);
  double ext = std::max(max_extent(L, sx, sy, ns), max_extent(L, tx, ty, nt));
  std::vector<double> img = lattice_ball(L, std::max(R, rc) + 2 * ext + 1e-12);
  std::vector<double> kv = reciprocal_ball(L, kc);
  const size_t nimg = img.size() / 2, nk = kv.size() / 2;
  const double a2 = alpha * alpha;

  // reciprocal part: V_i(k) = (1/|C|) (-k_i k_j) e^{-k^2/4a^2}/k^2 F_j(k),
  // F(k) = sum_s f_s e^{-i k.s}
  std::vector<double> Vr(2 * nk), Vi(2 * nk);
#pragma omp parallel for schedule(dynamic, 4)
  for (long a = 0; a < (long)nk; ++a) {
    double kx = kv[2 * a], ky = kv[2 * a + 1];
    double F1r = 0, F1i = 0, F2r = 0, F2i = 0;
    for (int64_t j = 0; j < ns; ++j) {
      double ph = kx * sx[j] + ky * sy[j];
      double c = std::cos(ph), s = std::sin(ph);
      F1r += f1[j] * c; F1i -= f1[j] * s;
      F2r += f2[j] * c; F2i -= f2[j] * s;
    }
    double k2 = kx * kx + ky * ky;
    double w = -std::exp(-k2 / (4 * a2)) / (k2 * L.area);
    double kFr = kx * F1r + ky * F2r, kFi = kx * F1i + ky * F2i;
    Vr[2 * a] = w * kx * kFr; Vi[2 * a] = w * kx * kFi;
    Vr[2 * a + 1] = w * ky * kFr; Vi[2 * a + 1] = w * ky * kFi;
  }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
  for (int64_t i = 0; i < nt; ++i) {
    double u[2] = {0, 0}, g[2][2] = {{0, 0}, {0, 0}};   // g[i][k] = d u_i / d x_k
    for (int64_t j = 0; j < ns; ++j) {
      double bx = tx[i] - sx[j], by = ty[i] - sy[j];
      lattice_reduce(L, bx, by);
      const double ff[2] = {f1[j], f2[j]};
      for (size_t l = 0; l < nimg; ++l) {
        double rx = bx - img[2 * l], ry = by - img[2 * l + 1];
        double r2 = rx * rx + ry * ry;
        if (r2 > R * R && r2 > rc * rc) continue;
        if (r2 == 0) {
          if (!(self_idx && j == self_idx[i])) bad = 1;
          continue;
        }
        double r = std::sqrt(r2);
        double H[2][2], T[2][2][2];
        if (r2 <= R * R) {
          // G_Y I - Hess G_Y / beta^2 with the radial derivatives of
          // G_Y = K0(beta r)/2pi: d1 = -beta K1, d2 = beta^2 (K0 + K1/(beta r)),
          // d3 = -beta^3 K1 - beta^2 K0/r - 2 beta K1/r^2 (all over 2pi)
          double k0 = std::cyl_bessel_k(0.0, beta * r), k1 = std::cyl_bessel_k(1.0, beta * r);
          double d0 = k0 / (2 * PI), d1 = -beta * k1 / (2 * PI);
          double d2 = beta * beta * (k0 + k1 / (beta * r)) / (2 * PI);
          double d3 = (-beta * beta * beta * k1 - beta * beta * k0 / r - 2 * beta * k1 / r2) / (2 * PI);
          radial_derivs(rx, ry, d1, d2, d3, H, T);
          const double x[2] = {rx, ry};
          for (int p = 0; p < 2; ++p) {
            u[p] += d0 * ff[p] - ib2 * (H[p][0] * ff[0] + H[p][1] * ff[1]);
            for (int k = 0; k < 2; ++k)
              g[p][k] += d1 * x[k] / r * ff[p] - ib2 * (T[p][0][k] * ff[0] + T[p][1][k] * ff[1]);
          }
        }
        if (r2 <= rc * rc) {
          // Hess of (1/4pi) E1(a^2 r^2) / beta^2: d1 = -e^{-x}/(2pi r),
          // d2 = e^{-x} (2a^2 + 1/r^2)/2pi, d3 = -e^{-x} (4a^4 r + 2a^2/r + 2/r^3)/2pi
          double ex = std::exp(-a2 * r2);
          double d1 = -ex / (2 * PI * r);
          double d2 = ex * (2 * a2 + 1 / r2) / (2 * PI);
          double d3 = -ex * (4 * a2 * a2 * r + 2 * a2 / r + 2 / (r2 * r)) / (2 * PI);
          radial_derivs(rx, ry, d1, d2, d3, H, T);
          for (int p = 0; p < 2; ++p) {
            u[p] += ib2 * (H[p][0] * ff[0] + H[p][1] * ff[1]);
            for (int k = 0; k < 2; ++k) g[p][k] += ib2 * (T[p][0][k] * ff[0] + T[p][1][k] * ff[1]);
          }
        }
      }
    }
    for (size_t a = 0; a < nk; ++a) {
      double kx = kv[2 * a], ky = kv[2 * a + 1];
      double ph = kx * tx[i] + ky * ty[i];
      double c = std::cos(ph), s = std::sin(ph);
      for (int p = 0; p < 2; ++p) {
        double re = c * Vr[2 * a + p] - s * Vi[2 * a + p], im = c * Vi[2 * a + p] + s * Vr[2 * a + p];
        u[p] += ib2 * re;
        // d/dx_k of Re(e^{ik.t} V) = -k_k Im(e^{ik.t} V)
        g[p][0] -= ib2 * kx * im; g[p][1] -= ib2 * ky * im;
      }
    }
    if (self_idx && self_idx[i] >= 0) {
      // the reciprocal sum holds the smooth part of the left-out term:
      // G_L - (1/4pi) E1(a^2 r^2) = const - a^2 r^2/(4pi) + O(r^4), whose
      // Hessian at 0 is -(a^2/2pi) I (odd third derivatives vanish)
      const int64_t s = self_idx[i];
      u[0] += ib2 * a2 / (2 * PI) * f1[s];
      u[1] += ib2 * a2 / (2 * PI) * f2[s];
    }
    if (out_vel) { out_vel[i] = u[0]; out_vel[nt + i] = u[1]; }
    if (out_grad) {
      out_grad[i] = g[0][0]; out_grad[nt + i] = g[0][1];
      out_grad[2 * nt + i] = g[1][0]; out_grad[3 * nt + i] = g[1][1];
    }
  }
  return bad ? -4 : 0;
}

// Free-space (non-periodic) direct sums, used by tests that pin the
// oracle's periodic sums in limits where images do not matter.
// kernel: 0 Laplace, 1 Yukawa (beta), 2 Stokes, 3 modified Stokes (beta).
// Same layouts as above.
int oracle_free_space(int kernel, double beta, int64_t ns, const double* sx, const double* sy,
                      const double* dens, int64_t nt, const double* tx, const double* ty,
                      const int64_t* self_idx, double* out_pot, double* out_grad) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < nt; ++i) {
    double p0 = 0, p1 = 0, g[4] = {0, 0, 0, 0};
    for (int64_t j = 0; j < ns; ++j) {
      if (self_idx && j == self_idx[i]) continue;
      double rx = tx[i] - sx[j], ry = ty[i] - sy[j];
      double r2 = rx * rx + ry * ry, r = std::sqrt(r2);
      if (kernel == 0) {
        p0 += -dens[j] * std::log(r) / (2 * PI);
        g[0] += -dens[j] * rx / (2 * PI * r2); g[1] += -dens[j] * ry / (2 * PI * r2);
      } else if (kernel == 1) {
        p0 += dens[j] * std::cyl_bessel_k(0.0, beta * r) / (2 * PI);
        double gg = -dens[j] * beta * std::cyl_bessel_k(1.0, beta * r) / (2 * PI * r);
        g[0] += gg * rx; g[1] += gg * ry;
      } else if (kernel == 3) {
        // modified Stokeslet as the operator of eq. msgreen on
        // G_MB = -(K0(beta r) + log r)/(2 pi beta^2): [[-d_yy, d_xy], [d_xy, -d_xx]] G_MB
        double br = beta * r, k0 = std::cyl_bessel_k(0.0, br), k1 = std::cyl_bessel_k(1.0, br);
        double cm = -1.0 / (2 * PI * beta * beta);
        double d1 = cm * (-beta * k1 + 1 / r);
        double d2 = cm * (beta * beta * (k0 + k1 / br) - 1 / r2);
        double d3 = cm * (-beta * beta * beta * k1 - beta * beta * k0 / r - 2 * beta * k1 / r2 + 2 / (r2 * r));
        double H[2][2], T[2][2][2];
        radial_derivs(rx, ry, d1, d2, d3, H, T);
        double fx = dens[j], fy = dens[ns + j];
        p0 += -H[1][1] * fx + H[0][1] * fy;
        p1 += H[0][1] * fx - H[0][0] * fy;
        for (int k = 0; k < 2; ++k) {
          g[k] += -T[1][1][k] * fx + T[0][1][k] * fy;
          g[2 + k] += T[0][1][k] * fx - T[0][0][k] * fy;
        }
      } else {
        double fx = dens[j], fy = dens[ns + j], rf = rx * fx + ry * fy;
        double lr = std::log(r);
        p0 += (-lr * fx + rf * rx / r2) / (4 * PI);
        p1 += (-lr * fy + rf * ry / r2) / (4 * PI);
        double rr[2] = {rx, ry}, ff[2] = {fx, fy};
        for (int a = 0; a < 2; ++a)
          for (int k = 0; k < 2; ++k)
            g[2 * a + k] += (-rr[k] * ff[a] / r2 + (ff[k] * rr[a] + (a == k ? rf : 0.0)) / r2
                             - 2 * rf * rr[a] * rr[k] / (r2 * r2)) / (4 * PI);
      }
    }
    if (kernel >= 2) {
      if (out_pot) { out_pot[i] = p0; out_pot[nt + i] = p1; }
      if (out_grad) for (int c = 0; c < 4; ++c) out_grad[c * nt + i] = g[c];
    } else {
      if (out_pot) out_pot[i] = p0;
      if (out_grad) { out_grad[i] = g[0]; out_grad[nt + i] = g[1]; }
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Singly periodic sums (Sec. 1, the operator P1: periodic in e1 = (d, 0)
// only, images m e1 for m in Z; Sec. 3 eq. ksplitting1). Canonical frame:
// the period is along x; y is unbounded. The Laplace and Stokes sums need
// neutral densities and are taken as the limit of symmetric partial sums
// over |m| <= M (the form the paper's west + east split produces).
// ---------------------------------------------------------------------------

// Laplace, P1: the symmetric row sum in closed form (sine product):
//   sum_m -(1/2pi) log|w - m d| = -(1/2pi) log|2 sin(pi w / d)| + const
//                               = -|y|/(2d) - (1/2pi) log|1 - e^{i kap sg w}| + const,
// kap = 2 pi/d, sg = sign(y), w = x + i y; the constants cancel for neutral
// q. A target on its own source takes the row without m = 0:
// lim_{w->0} (log|2 sin(pi w/d)| - log|w|) = log(2 pi/d).
int oracle_laplace_p1(double d, int64_t ns, const double* sx, const double* sy, const double* q,
                      int64_t nt, const double* tx, const double* ty, const int64_t* self_idx,
                      double* out_pot, double* out_grad) {
  if (!(d > 0)) return -1;
  const double kap = 2 * PI / d;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < nt; ++i) {
    double pot = 0, gx = 0, gy = 0;
    for (int64_t j = 0; j < ns; ++j) {
      if (self_idx && j == self_idx[i]) {
        pot += -q[j] * std::log(kap) / (2 * PI);
        continue;
      }
      const double wx = tx[i] - sx[j], wy = ty[i] - sy[j];
      const double sg = (wy >= 0) ? 1.0 : -1.0;
      const double rho = std::exp(-kap * std::fabs(wy));
      const double c = std::cos(kap * sg * wx), s = std::sin(kap * sg * wx);
      // |1 - rho e^{i phi}|^2 = (1 - rho)^2 + 4 rho sin^2(phi/2) (no cancellation)
      const double sh = std::sin(0.5 * kap * sg * wx);
      const double mod2 = (1 - rho) * (1 - rho) + 4 * rho * sh * sh;
      pot += q[j] * (-std::fabs(wy) / (2 * d) - std::log(mod2) / (4 * PI));
      // gradient of log|g|, g = 1 - e^{i kap sg w}: (Re g'/g, -Im g'/g)
      const double gre = 1 - rho * c, gim = -rho * s;
      const double dre = kap * sg * rho * s, dim = -kap * sg * rho * c;
      const double fre = (dre * gre + dim * gim) / mod2;
      const double fim = (dim * gre - dre * gim) / mod2;
      gx += q[j] * (-fre / (2 * PI));
      gy += q[j] * (fim / (2 * PI) - sg / (2 * d));
    }
    if (out_pot) out_pot[i] = pot;
    if (out_grad) { out_grad[i] = gx; out_grad[nt + i] = gy; }
  }
  return 0;
}

// Yukawa, P1: direct sum over the images m d, |m| <= M, with M grown until
// the dropped tail, at most 2 sum_{m > M} K0(beta (m - 1) d) <= 2 K0(beta (M - 1) d)
// / (1 - e^{-beta d}), is below tol (all points have |x| <= d/2 after
// wrapping, so an image m is at least (|m| - 1) d away).
int oracle_yukawa_p1(double d, double beta, double tol, int64_t ns, const double* sx, const double* sy,
                     const double* q, int64_t nt, const double* tx, const double* ty, const int64_t* self_idx,
                     double* out_pot, double* out_grad) {
  if (!(d > 0) || !(beta > 0) || !(tol > 0 && tol < 1)) return -1;
  int M = 2;
  while (2 * std::cyl_bessel_k(0.0, beta * (M - 1) * d) / (-std::expm1(-beta * d)) > tol) ++M;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
  for (int64_t i = 0; i < nt; ++i) {
    double pot = 0, gx = 0, gy = 0;
    for (int64_t j = 0; j < ns; ++j) {
      double bx = tx[i] - sx[j];
      bx -= d * std::nearbyint(bx / d);
      const double by = ty[i] - sy[j];
      for (int m = -M; m <= M; ++m) {
        const double rx = bx - m * d, ry = by, r2 = rx * rx + ry * ry;
        if (r2 == 0) {
          if (!(self_idx && j == self_idx[i])) bad = 1;
          continue;
        }
        const double r = std::sqrt(r2);
        pot += q[j] * std::cyl_bessel_k(0.0, beta * r) / (2 * PI);
        const double g = -q[j] * beta * std::cyl_bessel_k(1.0, beta * r) / (2 * PI * r);
        gx += g * rx; gy += g * ry;
      }
    }
    if (out_pot) out_pot[i] = pot;
    if (out_grad) { out_grad[i] = gx; out_grad[nt + i] = gy; }
  }
  return bad ? -4 : 0;
}

// Stokeslet, P1, in complex form: with w = x + i y, F = f1 + i f2 and
// u = u1 + i u2, the free-space Stokeslet reads
//   u = (1/4pi) [ -log|w| F + (F + conj F)/2 + i y conj(F) / conj(w) ]
// (r r^T f / r^2 = (F + (w / conj w) conj F)/2 and w / conj w = 1 + 2 i y / conj w).
// Summed symmetrically over the images w - m d: log|w| gives the sine
// product as for Laplace, sum_m 1/(conj w - m d) = (pi/d) cot(pi conj(w)/d),
// and the constant terms vanish for sum F = 0, so
//   u = (1/4pi) sum_j [ -log|2 sin(pi w_j / d)| F_j + i y_j (pi/d) cot(pi conj(w_j)/d) conj(F_j) ]
// with w_j = t - s_j. A target on its own source takes the images m != 0:
// (1/4pi)(-log(2 pi/d) F_i - Re F_i) (the x-directed images give r r^T f / r^2
// = (f1, 0)), and no gradient (the images pair up as m, -m).
int oracle_stokes_p1(double d, int64_t ns, const double* sx, const double* sy, const double* f,
                     int64_t nt, const double* tx, const double* ty, const int64_t* self_idx,
                     double* out_vel, double* out_grad) {
  if (!(d > 0)) return -1;
  typedef std::complex<double> cd;
  const double kap = 2 * PI / d, pd = PI / d;
  const double* f1 = f;
  const double* f2 = f + ns;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < nt; ++i) {
    cd u(0, 0), ux(0, 0), uy(0, 0);
    for (int64_t j = 0; j < ns; ++j) {
      const cd F(f1[j], f2[j]);
      if (self_idx && j == self_idx[i]) {
        u += (-std::log(kap) * F - F.real()) / (4 * PI);
        continue;
      }
      const double wx = tx[i] - sx[j], wy = ty[i] - sy[j];
      const double sg = (wy >= 0) ? 1.0 : -1.0;
      // log|2 sin(pi w/d)| = |y| pi/d + log|1 - E|, E = e^{i kap sg w}, |E| <= 1
      const double rho = std::exp(-kap * std::fabs(wy));
      const double sh = std::sin(0.5 * kap * sg * wx);
      const double mod2 = (1 - rho) * (1 - rho) + 4 * rho * sh * sh;
      const double lsin = std::fabs(wy) * pd + 0.5 * std::log(mod2);
      const cd E = rho * cd(std::cos(kap * sg * wx), std::sin(kap * sg * wx));
      // cot(pi w/d) = i (E + 1)/(E - 1) for y >= 0; for y < 0 with E = e^{-i kap w}:
      // cot = -i (E + 1)/(E - 1)
      const cd cotw = sg * cd(0, 1) * (E + 1.0) / (E - 1.0);
      // cot(pi conj(w)/d) = conj(cot(pi w/d)); 1/sin^2 = 1 + cot^2
      const cd cotc = std::conj(cotw);
      const cd csc2c = 1.0 + cotc * cotc;
      const cd Fc = std::conj(F);
      u += (-lsin * F + cd(0, 1) * wy * pd * cotc * Fc) / (4 * PI);
      // d/dx log|2 sin| = Re(pd cot w), d/dy = -Im(pd cot w)
      const double lx = (pd * cotw).real(), ly = -(pd * cotw).imag();
      // d/dx cot(pi conj w/d) = -pd csc^2, d/dy = +i pd csc^2
      ux += (-lx * F + cd(0, 1) * wy * pd * (-pd * csc2c) * Fc) / (4 * PI);
      uy += (-ly * F + cd(0, 1) * pd * cotc * Fc + cd(0, 1) * wy * pd * (cd(0, 1) * pd * csc2c) * Fc) / (4 * PI);
    }
    if (out_vel) { out_vel[i] = u.real(); out_vel[nt + i] = u.imag(); }
    if (out_grad) {
      out_grad[i] = ux.real(); out_grad[nt + i] = uy.real();
      out_grad[2 * nt + i] = ux.imag(); out_grad[3 * nt + i] = uy.imag();
    }
  }
  return 0;
}

}  // extern "C"
