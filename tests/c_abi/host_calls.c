/* Plain C caller of libhfqmc's host-only entry points (no GPU needed): the
 * U = 0 Bethe bath, its imaginary-time transform and the chain-split plan.
 * Prints the values on stdout for the test that compiles and runs it. */
#include <stdio.h>
#include <stdlib.h>

#include "hfqmc.h"

int main(void) {
  const double beta = 10.0, t = 1.0;
  const int n_iw = 4096, L = 20;
  double *bath = malloc(sizeof(double) * 2 * n_iw);
  double g[20];
  if (!bath) return 2;
  if (bethe_semicircle_bath(beta, t, n_iw, bath) != HFQMC_OK) return 3;
  if (bath_to_tau(bath, n_iw, t * t, beta, L, g) != HFQMC_OK) return 4;
  for (int k = 0; k < L; ++k) printf("g %d %.17g\n", k, g[k]);
  const int32_t Ls[8] = {250, 286, 333, 400, 500, 667, 1000, 2000};
  int32_t f[8];
  double span[2];
  if (hfqmc_plan_balance(8, Ls, 32, 100, 1000, 1, 256, f, span) != HFQMC_OK) return 5;
  for (int i = 0; i < 8; ++i) printf("f %d %d\n", i, f[i]);
  printf("span %.17g %.17g\n", span[0], span[1]);
  /* an invalid call reports through the error string */
  if (hfqmc_plan_balance(0, Ls, 32, 100, 1000, 1, 256, f, span) != HFQMC_EINVAL) return 6;
  printf("error %s\n", hfqmc_last_error());
  free(bath);
  return 0;
}
