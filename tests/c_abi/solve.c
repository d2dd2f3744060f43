/* Plain C caller of the device entry points: one fixed-dtau solve (FP64
 * rank-1 and the mixed path) and one multigrid step, printed on stdout for
 * the test that compiles and runs it (no Python, no PyTorch in the process). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hfqmc.h"

static int check(int rc, const char *what) {
  if (rc != HFQMC_OK) fprintf(stderr, "%s failed (%d): %s\n", what, rc, hfqmc_last_error());
  return rc;
}

int main(void) {
  const double beta = 10.0, U = 4.0, t = 1.0;
  const int n_iw = 4096, L = 20;
  hfqmc_ctx *ctx = NULL;
  if (check(hfqmc_create(&ctx, 0), "hfqmc_create")) return 2;
  double *bath = malloc(sizeof(double) * 2 * n_iw);
  double g0[20], g[21], ge[21], d[2];
  if (check(bethe_semicircle_bath(beta, t, n_iw, bath), "bath")) return 3;
  if (check(bath_to_tau(bath, n_iw, t * t, beta, L, g0), "bath_to_tau")) return 4;
  for (int mode = 0; mode < 3; mode += 2) {
    hfqmc_opts o;
    memset(&o, 0, sizeof o);
    o.n_chains = 4;
    o.mode = mode;
    o.warmup = 20;
    o.sweeps = 200;
    o.delay_k = mode ? 16 : 0;
    hfqmc_stats st;
    if (check(hfqmc_solve(ctx, g0, L, U, beta, beta / L, 3, &o, g, ge, d, &st), "hfqmc_solve"))
      return 5;
    printf("solve %d D %.17g %.17g acc %.17g\n", mode, d[0], d[1], st.acc_rate);
    for (int k = 0; k <= L; ++k) printf("solve %d g %d %.17g\n", mode, k, g[k]);
  }
  const double dtaus[3] = {0.5, 0.4, 0.25};
  double gf[41], gfe[41], dx[2];
  hfqmc_opts o;
  memset(&o, 0, sizeof o);
  o.n_chains = 4;
  o.mode = HFQMC_MODE_RANK1;
  o.warmup = 20;
  o.sweeps = 200;
  if (check(multigrid_solve(ctx, bath, n_iw, t * t, U, beta, dtaus, 3, 5, &o, 41, gf, gfe, NULL, NULL,
                            NULL, dx), "multigrid_solve"))
    return 6;
  printf("multigrid D %.17g %.17g\n", dx[0], dx[1]);
  for (int k = 0; k < 41; ++k) printf("multigrid g %d %.17g\n", k, gf[k]);
  hfqmc_destroy(ctx);
  free(bath);
  return 0;
}
