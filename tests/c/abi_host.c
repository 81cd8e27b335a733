/* A plain C consumer of libnbs (test code): creates a host-only plan for the
 * worked-example channel and a small R52-like list, reads its counts and
 * checks the documented errors of the compute calls on a host-only plan. */
#include <stdio.h>
#include <string.h>

#include "nbs.h"

static int fails = 0;
#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond);      \
      ++fails;                                                   \
    }                                                            \
  } while (0)

int main(void) {
  nbs_geometry g = {{4, 4, 4}, 8, 0, 0, 8};
  /* <p Lambda | pbar X_u-bar> */
  nbs_channel c = {{NBS_P, NBS_LAMBDA}, {NBS_P, NBS_X_U}};
  nbs_plan p = NULL;
  CHECK(nbs_plan_create(&p, &g, 1, &c, 1, NBS_FP64, -1) == NBS_OK);
  CHECK(p != NULL);
  nbs_plan_info_t info;
  memset(&info, 0, sizeof info);
  CHECK(nbs_plan_info(p, &info) == NBS_OK);
  CHECK(info.n_channels == 1);
  CHECK(info.n_diagrams == 6); /* the six terms of the worked example */
  void* ptr[1] = {(void*)1};
  const void* cptr[1] = {(const void*)1};
  CHECK(nbs_build_blocks(p, cptr, cptr, cptr, NULL) == NBS_ERR_STATE);
  CHECK(nbs_contract_channels(p, NULL) == NBS_ERR_STATE);
  CHECK(nbs_relative_sum(p, ptr, NULL) == NBS_ERR_STATE);
  nbs_baryon_pair bp = {NBS_P, NBS_P};
  CHECK(nbs_two_point(p, &bp, 1, ptr, NULL) == NBS_ERR_STATE);
  CHECK(strlen(nbs_last_error(p)) > 0);
  CHECK(nbs_plan_destroy(p) == NBS_OK);
  CHECK(nbs_plan_destroy(NULL) == NBS_OK);
  /* invalid arguments are rejected before anything is allocated */
  nbs_plan q = (nbs_plan)1;
  CHECK(nbs_plan_create(&q, &g, 0, &c, 1, NBS_FP64, -1) == NBS_ERR_INVALID);
  CHECK(q == NULL);
  CHECK(strcmp(nbs_status_string(NBS_ERR_NOMEM), "out of device memory") == 0);
  printf(fails ? "abi_host: %d failures\n" : "abi_host: ok\n", fails);
  return fails ? 1 : 0;
}
