#include <stdio.h>
#include <string.h>
#include "tflbm.h"
/* Drives the host-side paths of the C ABI that make no HIP call (parameter
 * checks, handle lifetime, sizes, call-order errors), for a build of the
 * library whose host code carries AddressSanitizer (tests/test_abi_asan.py). */
int main(void) {
  int fails = 0;
#define EXPECT(c) do { if (!(c)) { printf("FAIL line %d: %s\n", __LINE__, #c); ++fails; } } while (0)
  tflbm_params p;
  tflbm_default_params(&p);
  p.nx = 100; p.ny = 30;
  EXPECT(tflbm_check_params(&p) == TFLBM_OK);
  EXPECT(tflbm_check_params(NULL) == TFLBM_EINVAL);
  tflbm_params q = p; q.nx = 0; EXPECT(tflbm_check_params(&q) == TFLBM_EINVAL);
  q = p; q.tau = 0.5; EXPECT(tflbm_check_params(&q) == TFLBM_EINVAL);
  q = p; q.prec = 7; EXPECT(tflbm_check_params(&q) == TFLBM_EINVAL);
  for (int prec = 0; prec < 3; ++prec) {
    p.prec = prec;
    tflbm_sim *s = NULL;
    EXPECT(tflbm_create(&p, &s) == TFLBM_OK && s != NULL);
    EXPECT(tflbm_workspace_bytes(s) > 0 && tflbm_state_bytes(s) > 0);
    EXPECT(tflbm_capture_bytes(s) > 0 && tflbm_adj_bytes(s) > 0);
    EXPECT(tflbm_bind(s, NULL, 0) == TFLBM_EINVAL);
    EXPECT(tflbm_step(s, 1, NULL) == TFLBM_ESTATE);
    double m = 0.0, norms[8];
    EXPECT(tflbm_mass(s, &m, NULL) == TFLBM_ESTATE);
    EXPECT(tflbm_term_norms(s, norms, NULL) == TFLBM_ESTATE);
    char fake[256];
    EXPECT(tflbm_adj_step(s, fake, fake, NULL) == TFLBM_ESTATE);
    EXPECT(tflbm_adj_steps(s, fake, fake, 3, NULL) == TFLBM_ESTATE);
    EXPECT(tflbm_adj_steps(s, fake, fake, -1, NULL) == TFLBM_EINVAL);
    EXPECT(tflbm_step_count(s) == 0);
    EXPECT(tflbm_step_graphs(s) == 0);
    EXPECT(strlen(tflbm_strerror(TFLBM_ESTATE)) > 0 && strlen(tflbm_last_error(s)) == 0);
    tflbm_destroy(s);
  }
  EXPECT(tflbm_create(NULL, NULL) == TFLBM_EINVAL);
  EXPECT(tflbm_step_graphs(NULL) == -1);
  tflbm_destroy(NULL);
  printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
  return fails != 0;
}
