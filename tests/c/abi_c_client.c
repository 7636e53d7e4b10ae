/* A plain C99 client of libgw: includes only the public headers, builds a
 * tiny synthetic problem and calls the entry points through the C-ABI.  In
 * launch-audit mode (no GPU needed) every call walks its launches and the
 * result-returning ones answer GW_EAUDIT.  Exit status 0 when every call
 * returned what the headers promise. */
#include <stdio.h>
#include <stdlib.h>

#include "gw.h"
#include "gw_audit.h"

static int expect(const char* what, int rc, int want) {
  if (rc != want) {
    fprintf(stderr, "%s: returned %d, expected %d (%s)\n", what, rc, want, gw_last_error());
    return 1;
  }
  return 0;
}

int main(void) {
  enum { N_MO = 6, N_OCC = 2, N_AUX = 5, N_ROWS = 2, G = 4 };
  const int n_virt = N_MO - N_OCC;
  double eps[N_MO] = {-1.2, -0.6, 0.2, 0.5, 1.1, 2.0};
  double B_ov[N_AUX * N_OCC * (N_MO - N_OCC)];
  double B_rows[N_ROWS * N_MO * N_AUX];
  int rows[N_ROWS] = {1, 2};
  int states[N_ROWS] = {1, 2};
  double xi[G], w[G], E[N_ROWS], S[N_ROWS], Z[N_ROWS];
  int st[N_ROWS], bad = 0;
  unsigned s = 12345u;
  for (int i = 0; i < N_AUX * N_OCC * n_virt; ++i) {
    s = s * 1103515245u + 12345u;
    B_ov[i] = ((double)(s >> 8) / 16777216.0 - 0.5) * 0.2;
  }
  for (int i = 0; i < N_ROWS * N_MO * N_AUX; ++i) {
    s = s * 1103515245u + 12345u;
    B_rows[i] = ((double)(s >> 8) / 16777216.0 - 0.5) * 0.2;
  }
  bad |= expect("gw_audit_enable", gw_audit_enable(), 0);
  bad |= expect("gw_grid_gauss_legendre", gw_grid_gauss_legendre(G, 0.5, xi, w), 0);
  gw_grid grid = {G, xi, w};
  gw_opts opts = {0};
  gw_ctx* ctx = NULL;
  bad |= expect("gw_setup", gw_setup(&ctx, N_MO, N_OCC, N_AUX, eps, B_ov, N_ROWS, rows, B_rows,
                                     &opts), 0);
  if (!ctx) return 1;
  bad |= expect("gw_qp", gw_qp(ctx, N_ROWS, states, &grid, E, S, Z, st), GW_EAUDIT);
  bad |= expect("gw_evgw", gw_evgw(ctx, GW_EVGW0, 2, 0.0, N_ROWS, states, &grid, E, S, Z, st,
                                   NULL, NULL), GW_EAUDIT);
  bad |= expect("gw_qp_sd", gw_qp_sd(ctx, N_ROWS, states, E, S, Z, st), GW_EAUDIT);
  bad |= expect("gw_qp bad state", gw_qp(ctx, 1, (int[]){0}, &grid, E, S, Z, st), GW_EINVAL);
  bad |= expect("gw_set_pi_prec", gw_set_pi_prec(ctx, GW_PI_BF16X3), 0);
  bad |= expect("gw_qp bf16x3", gw_qp(ctx, N_ROWS, states, &grid, E, S, Z, st), GW_EAUDIT);
  gw_free(ctx);
  if (gw_footprint(N_MO, N_OCC, N_AUX, N_ROWS, N_ROWS, G, &opts) == 0) {
    fprintf(stderr, "gw_footprint returned 0\n");
    bad = 1;
  }
  printf("%s (%ld launches checked)\n", bad ? "FAILED" : "c client ok", gw_audit_launch_count());
  return bad;
}
