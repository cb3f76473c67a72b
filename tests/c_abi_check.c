/* Plain C99 caller of libpfmm's host-only entry points: checks that
 * include/pfmm.h is valid C and that planning, plan queries, workspace
 * sizing and argument errors work through the C ABI without a GPU.
 * Prints "sizeof <struct> <bytes>" lines for the Python binding's layout
 * check and "ok" at the end; exits non-zero at the first failed check. */
#include <stdio.h>
#include <string.h>

#include "pfmm.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main(void) {
  const double e1[2] = {1.1, 0.35}, e2[2] = {-0.2, 0.9};
  const double bad[2] = {2.2, 0.7};   /* parallel to e1 */
  pfmm_opts o;
  pfmm_plan_t plan = NULL;
  pfmm_plan_info_t info;
  pfmm_tuning_t tune;
  int k;

  printf("sizeof pfmm_opts %zu\n", sizeof(pfmm_opts));
  printf("sizeof pfmm_plan_info_t %zu\n", sizeof(pfmm_plan_info_t));
  printf("sizeof pfmm_tuning_t %zu\n", sizeof(pfmm_tuning_t));
  printf("sizeof pfmm_tune_report_t %zu\n", sizeof(pfmm_tune_report_t));

  /* default options (opts = NULL) */
  CHECK(pfmm_plan(PFMM_LAPLACE, e1, e2, 1e-6, NULL, &plan) == PFMM_OK && plan);
  CHECK(pfmm_plan_get_info(plan, &info) == PFMM_OK);
  CHECK(info.kernel == PFMM_LAPLACE && info.precision == PFMM_FP64 && info.n_dens == 1);
  CHECK(info.d > 0 && info.eta > 0 && info.n_images == 3 * (2 * info.m0 + 1));
  CHECK(pfmm_workspace_bytes(plan, 1000, 500) > 0);
  CHECK(pfmm_workspace_bytes(plan, -1, 500) == 0);
  CHECK(pfmm_plan_get_tuning(plan, &tune) == PFMM_OK);
  /* argument errors are reported before anything is launched */
  CHECK(pfmm_eval(plan, -1, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL) == PFMM_EINVAL);
  CHECK(pfmm_eval(plan, PFMM_MAX_POINTS + 1, NULL, NULL, 1, NULL, NULL, NULL, NULL, 0, NULL) == PFMM_EINVAL);
  pfmm_destroy(plan);

  /* every kernel and precision with explicit options */
  for (k = 0; k < 3; ++k) {
    memset(&o, 0, sizeof o);
    o.beta = 4.0;
    o.precision = PFMM_MIXED;
    o.far_mode = PFMM_FAR_AUTO;
    o.n_dens = 2;
    o.self_exclude = 1;
    plan = NULL;
    CHECK(pfmm_plan(k, e1, e2, 1e-6, &o, &plan) == PFMM_OK && plan);
    CHECK(pfmm_plan_get_info(plan, &info) == PFMM_OK);
    CHECK(info.kernel == k && info.precision == PFMM_MIXED && info.n_dens == 2 && info.self_exclude == 1);
    CHECK(pfmm_workspace_bytes(plan, 2000, 2000) > 0);
    CHECK(pfmm_workspace_bytes(plan, 0, 0) > 0);
    pfmm_destroy(plan);
  }

  /* planning errors */
  plan = NULL;
  CHECK(pfmm_plan(PFMM_LAPLACE, e1, bad, 1e-6, NULL, &plan) == PFMM_EINVAL_LATTICE && !plan);
  CHECK(pfmm_plan(PFMM_LAPLACE, e1, e2, 0.5, NULL, &plan) == PFMM_EINVAL_TOL && !plan);
  CHECK(pfmm_plan(7, e1, e2, 1e-6, NULL, &plan) == PFMM_EINVAL && !plan);
  CHECK(pfmm_strerror(PFMM_EWORKSPACE) != NULL && strlen(pfmm_strerror(PFMM_EWORKSPACE)) > 0);
  pfmm_destroy(NULL);
  printf("ok\n");
  return 0;
}
