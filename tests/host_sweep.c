/* Host-side sweep of libpfmm's planning, query, sizing and tuning entry
 * points over many random cells and option sets: aspect ratios 1..1000,
 * rotated, unreduced, hexagonal and near-degenerate lattices; every kernel,
 * precision, far mode, near mode, m0, n_dens and line count; tolerances
 * 1e-14..1e-2 plus invalid ones. The first argument sets the number of
 * cases (3000 by default). Built and run under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py; no GPU work
 * is done. Exits non-zero at the first inconsistent result. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pfmm.h"

static const double TWO_PI = 6.283185307179586;

static double urand(unsigned long long* s) {
  *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(*s >> 11) / 9007199254740992.0;
}

#define FAIL(msg)                                         \
  do {                                                    \
    printf("iteration %d: %s\n", it, msg);                \
    return 1;                                             \
  } while (0)

int main(int argc, char** argv) {
  unsigned long long seed = 12345;
  const int n_it = argc > 1 ? atoi(argv[1]) : 3000;
  int made = 0, refused = 0, it;
  for (it = 0; it < n_it; ++it) {
    const int shape = it % 6;
    const double A = pow(10.0, 3.0 * urand(&seed));
    const double th = TWO_PI * urand(&seed);
    double a[2], b[2], e1[2], e2[2];
    double tol;
    pfmm_opts o;
    pfmm_plan_t p = NULL;
    pfmm_plan_info_t inf;
    pfmm_tuning_t t;
    double *x, *w;
    int ends[64], e0s[64], i, j, k, kernel, rc;
    const long long sizes[6] = {0, 1, 257, 100000, 3000000, PFMM_MAX_POINTS};

    a[0] = A; a[1] = 0; b[0] = (urand(&seed) - 0.5) * A; b[1] = 1;
    if (shape == 1) { a[0] = 1; b[0] = 0.5; b[1] = sqrt(3.0) / 2; }
    if (shape == 2) b[0] += 3 * a[0];                            /* unreduced basis */
    if (shape == 3) b[1] = 1e-13;                                /* degenerate */
    if (shape == 4) { a[0] = 1; b[0] = 0; b[1] = pow(10.0, -3.0 * urand(&seed)); }
    e1[0] = cos(th) * a[0] - sin(th) * a[1]; e1[1] = sin(th) * a[0] + cos(th) * a[1];
    e2[0] = cos(th) * b[0] - sin(th) * b[1]; e2[1] = sin(th) * b[0] + cos(th) * b[1];
    memset(&o, 0, sizeof o);
    kernel = it % 3;
    o.beta = pow(10.0, 4.0 * urand(&seed) - 2.0);
    o.precision = (it / 3) % 2;
    o.far_mode = (it / 6) % 3;
    o.m0 = (it / 18) % 4;
    o.n_dens = 1 + (it / 72) % 17;
    o.self_exclude = (it / 7) % 2;
    o.m_gl = ((it / 11) % 3) * 8;
    o.near_mode = o.self_exclude ? (it / 13) % 3 : (it / 13) % 2;
    if ((it / 5) % 4 == 0) o.near_mode = PFMM_NEAR_FMM;
    tol = pow(10.0, -2.0 - 12.0 * urand(&seed));
    if (it % 97 == 0) tol = 0.5;

    rc = pfmm_plan(kernel, e1, e2, tol, &o, &p);
    if (rc) {
      ++refused;
      if (p) FAIL("plan handle set on error");
      if (!pfmm_strerror(rc)) FAIL("no message for an error code");
      continue;
    }
    ++made;
    if (pfmm_plan_get_info(p, &inf)) FAIL("info");
    if (!(inf.d > 0 && inf.eta > 0 && fabs(inf.xi) <= 0.5 * inf.d * (1 + 1e-12))) FAIL("canonical lattice");
    if (inf.n_images != 3 * (2 * inf.m0 + 1)) FAIL("image count");
    if (o.near_mode == PFMM_NEAR_FMM && (inf.fmm_order < 4 || inf.fmm_order > 20)) FAIL("fmm order");
    x = malloc(sizeof(double) * (inf.n_quad + 1));
    w = malloc(sizeof(double) * (inf.n_quad + 1));
    if (pfmm_plan_get_quadrature(p, x, w)) FAIL("quadrature");
    for (k = 0; k < inf.n_quad; ++k)
      if (!isfinite(x[k]) || !isfinite(w[k]) || x[k] < 0) FAIL("quadrature values");
    free(x);
    free(w);
    if (inf.n_log_groups < 1 || inf.n_log_groups > 64 || pfmm_plan_get_log_groups(p, ends, e0s)) FAIL("log groups");
    if (ends[inf.n_log_groups - 1] != inf.n_images) FAIL("log groups cover the images");
    for (i = 0; i < 6; ++i)
      for (j = 0; j < 6; ++j)
        if (pfmm_workspace_bytes(p, sizes[i], sizes[j]) == 0) FAIL("workspace size");
    if (pfmm_workspace_bytes(p, PFMM_MAX_POINTS + 1, 10) != 0) FAIL("point limit");
    (void)pfmm_workspace_bytes_adjoint(p, 1000);
    if (pfmm_plan_get_tuning(p, &t)) FAIL("get tuning");
    t.nufft_grid = 1;
    t.near_blocks = 4096;
    (void)pfmm_plan_set_tuning(p, &t);   /* the doubled grid may be refused */
    t.nufft_grid = 0;
    t.fmm_leaves = (it / 3) % 3;
    if (pfmm_plan_set_tuning(p, &t)) FAIL("set tuning back");
    if (pfmm_workspace_bytes(p, 5000, 5000) == 0) FAIL("workspace after tuning");
    if (pfmm_eval(p, -1, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL) != PFMM_EINVAL) FAIL("eval argument check");
    pfmm_destroy(p);
  }
  printf("plans made %d, refused %d\n", made, refused);
  return made > n_it / 3 && refused > n_it / 30 ? 0 : 1;
}
