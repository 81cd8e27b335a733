/* Host-only plans through the C ABI (test code, built with the address and
 * undefined-behaviour sanitizers): every channel table the tests use is
 * compiled, every table of the program is read twice (size query, then
 * copy), launch shapes are set and rejected, and the documented argument
 * errors are returned. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nbs.h"

static int fails = 0;
#define CHECK(cond)                                         \
  do {                                                      \
    if (!(cond)) {                                          \
      printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                              \
    }                                                       \
  } while (0)

static const char* INT_TABLES[] = {"op_code", "op_nterm", "op_term_trip", "op_term_perm", "group_op1", "group_op2",
                                   "group_prod", "group_task", "group_ch", "group_channels", "ch_contrib",
                                   "contrib_prod", "prod_desc", "task_lanes", "op_alias", "group_op1_iso",
                                   "group_op2_iso", "op_pair", "seg_task", "group_stask", "prod_ext"};
static const char* DBL_TABLES[] = {"contrib_coef", "op_term_w", "op_alias_coef", "contrib_coef_iso"};

static void exercise(const nbs_channel* ch, int n_ch, nbs_precision prec) {
  nbs_geometry g = {{4, 3, 2}, 8, 0, 2, 3};
  nbs_plan p = NULL;
  CHECK(nbs_plan_create(&p, &g, 1, ch, n_ch, prec, -1) == NBS_OK);
  if (!p) return;
  nbs_plan_info_t info;
  CHECK(nbs_plan_info(p, &info) == NBS_OK);
  CHECK(info.n_channels == n_ch);
  for (size_t k = 0; k < sizeof INT_TABLES / sizeof *INT_TABLES; ++k) {
    int64_t n = -1;
    CHECK(nbs_plan_table(p, INT_TABLES[k], NULL, 0, &n) == NBS_OK);
    CHECK(n >= 0);
    int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t m = -1;
    CHECK(nbs_plan_table(p, INT_TABLES[k], buf, n, &m) == NBS_OK && m == n);
    if (n > 1) CHECK(nbs_plan_table(p, INT_TABLES[k], buf, n - 1, &m) == NBS_OK && m == n);  /* short buffer */
    free(buf);
  }
  for (size_t k = 0; k < sizeof DBL_TABLES / sizeof *DBL_TABLES; ++k) {
    int64_t n = -1;
    CHECK(nbs_plan_table(p, DBL_TABLES[k], NULL, 0, &n) == NBS_OK);
    double* buf = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    int64_t m = -1;
    CHECK(nbs_plan_table(p, DBL_TABLES[k], buf, n, &m) == NBS_OK && m == n);
    free(buf);
  }
  int64_t n = 0;
  CHECK(nbs_plan_table(p, "no_such_table", NULL, 0, &n) == NBS_ERR_INVALID);
  int32_t nd = 0;
  CHECK(nbs_plan_diagrams(p, -1, NULL, 0, &nd) == NBS_OK && nd == info.n_diagrams);
  nbs_diagram_t* d = (nbs_diagram_t*)calloc((size_t)nd + 1, sizeof *d);
  CHECK(nbs_plan_diagrams(p, -1, d, nd, &nd) == NBS_OK);
  CHECK(nbs_plan_diagrams(p, 0, d, nd, &nd) == NBS_OK);
  free(d);
  int32_t params[4], tune[4], bad[4];
  CHECK(nbs_plan_params(p, params) == NBS_OK);
  CHECK(nbs_plan_tuning(p, tune) == NBS_OK);
  /* the other engine and back, other group ranges */
  int32_t t2[4] = {tune[0], tune[1], prec == NBS_FP64 ? 8 : 4, tune[3] & ~16};
  CHECK(nbs_plan_set_tuning(p, t2) == NBS_OK);
  for (int gc = 0; gc < 3; ++gc) {
    t2[3] = (t2[3] & ~12) | (gc << 2);
    CHECK(nbs_plan_set_tuning(p, t2) == NBS_OK);
  }
  CHECK(nbs_plan_set_tuning(p, tune) == NBS_OK);
  memcpy(bad, tune, sizeof bad);
  bad[1] = 300;
  CHECK(nbs_plan_set_tuning(p, bad) == NBS_ERR_INVALID);
  memcpy(bad, tune, sizeof bad);
  bad[3] = 1 << 7;
  CHECK(nbs_plan_set_tuning(p, bad) == NBS_ERR_INVALID);
  size_t ws = 1;
  CHECK(nbs_workspace_bytes(p, &ws) == NBS_OK && ws == 0);
  CHECK(nbs_plan_destroy(p) == NBS_OK);
}

int main(void) {
  /* the worked example, a mixed list, every octet operator at the sink */
  nbs_channel w = {{NBS_P, NBS_LAMBDA}, {NBS_P, NBS_X_U}};
  exercise(&w, 1, NBS_FP64);
  nbs_channel mix[] = {{{NBS_P, NBS_P}, {NBS_P, NBS_P}},
                       {{NBS_LAMBDA, NBS_LAMBDA}, {NBS_SIGMA_P, NBS_SIGMA_M}},
                       {{NBS_XI_0, NBS_SIGMA_0}, {NBS_XI_M, NBS_SIGMA_P}},
                       {{NBS_N, NBS_XI_0}, {NBS_LAMBDA, NBS_LAMBDA}},
                       {{NBS_XI_0, NBS_XI_M}, {NBS_XI_0, NBS_XI_M}},
                       {{NBS_SIGMA_M, NBS_N}, {NBS_SIGMA_M, NBS_N}}};
  exercise(mix, 6, NBS_FP64);
  exercise(mix, 6, NBS_FP32_MFMA);
  /* errors, each before any allocation */
  nbs_geometry g = {{4, 4, 4}, 8, 0, 0, 8};
  nbs_plan q = (nbs_plan)1;
  CHECK(nbs_plan_create(&q, &g, 0, &w, 1, NBS_FP64, -1) == NBS_ERR_INVALID && q == NULL);
  nbs_geometry g7 = {{7, 4, 4}, 8, 0, 0, 8};
  CHECK(nbs_plan_create(&q, &g7, 1, &w, 1, NBS_FP64, -1) == NBS_ERR_INVALID);
  nbs_geometry gt = {{4, 4, 4}, 8, 0, 6, 3};
  CHECK(nbs_plan_create(&q, &gt, 1, &w, 1, NBS_FP64, -1) == NBS_ERR_INVALID);
  nbs_channel badflav = {{NBS_P, NBS_P}, {NBS_N, NBS_N}};
  CHECK(nbs_plan_create(&q, &g, 1, &badflav, 1, NBS_FP64, -1) == NBS_ERR_INVALID);
  nbs_channel badop = {{NBS_P, 42}, {NBS_P, NBS_P}};
  CHECK(nbs_plan_create(&q, &g, 1, &badop, 1, NBS_FP64, -1) == NBS_ERR_INVALID);
  CHECK(nbs_plan_create(&q, &g, 1, &w, 1, (nbs_precision)7, -1) == NBS_ERR_INVALID);
  CHECK(nbs_plan_create(NULL, &g, 1, &w, 1, NBS_FP64, -1) == NBS_ERR_INVALID);
  for (int s = 0; s <= 6; ++s) CHECK(strlen(nbs_status_string((nbs_status)s)) > 0);
  printf(fails ? "plan_host_checks: %d failures\n" : "plan_host_checks: ok\n", fails);
  return fails ? 1 : 0;
}
