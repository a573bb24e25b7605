/* Drives the oracle through every boundary type, both time schemes and
 * limiters, force, one-step and multi-step chemistry, and every output
 * routine; built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include "dbm_oracle.h"
static void run(int bcx, int bcy, int scheme, int react, double ay, int nchem, int lim) {
  or_species sp[3]; memset(sp, 0, sizeof sp);
  double ms[3] = {2, 32, 18}, as[3] = {-2, -1, 2};
  for (int k = 0; k < 3; ++k) {
    double s = sqrt(1.0 / ms[k]);
    sp[k].m = ms[k]; sp[k].I = 3; sp[k].tau = 2e-5; sp[k].a = as[k];
    sp[k].v[0] = 1.5 * s; sp[k].v[1] = 0.8 * s; sp[k].v[2] = 2.2 * s; sp[k].v[3] = 2.6 * s; sp[k].eta[0] = 2.5 * s;
  }
  or_reaction_step ch[2]; memset(ch, 0, sizeof ch);
  ch[0].fuel = 0; ch[0].oxid = 1; ch[0].k = 1e3; ch[0].Ea_over_R = 10; ch[0].Q = 5; ch[0].a[0] = -2; ch[0].a[1] = -1; ch[0].a[2] = 2;
  ch[1].fuel = 0; ch[1].oxid = 2; ch[1].k = 5e2; ch[1].Ea_over_R = 8; ch[1].Q = 3; ch[1].a[0] = -1; ch[1].a[2] = -1; ch[1].a[1] = 1;
  or_config c; memset(&c, 0, sizeof c);
  c.nx = 13; c.ny = 7; c.dx = c.dy = 1e-3; c.dt = 1e-5; c.bc_x = bcx; c.bc_y = bcy; c.S = 3; c.sp = sp;
  c.reaction_on = react; c.fuel = 0; c.oxid = 1; c.k_ov = 1e3; c.Ea_over_R = 10; c.Q = 2;
  c.ay = ay; c.scheme = scheme; c.limiter = lim; c.nchem = nchem; c.chem = nchem ? ch : NULL;
  or_model *md = NULL;
  int rc = or_create(&c, &md);
  if (rc) { printf("create rc=%d\n", rc); return; }
  int cells = c.nx * c.ny;
  double *n = malloc(sizeof(double) * 3 * cells), *ux = calloc(cells, 8), *uy = calloc(cells, 8), *T = malloc(8 * cells);
  for (int i = 0; i < cells; ++i) { n[i] = 0.05 + 0.001 * (i % 5); n[cells + i] = 0.03; n[2 * cells + i] = 0.001 * (i % 3); T[i] = 1 + 0.5 * ((i * 7) % 11) / 11.0; ux[i] = 0.1 * ((i % 4) - 1.5); }
  double *f = malloc(sizeof(double) * 3 * 16 * cells);
  or_init_equilibrium(md, n, ux, uy, T, f);
  or_run(md, f, 5);
  double *rho = malloc(sizeof(double) * 3 * cells), *delta = malloc(sizeof(double) * 3 * 12 * cells), tot[6], *en = malloc(sizeof(double) * 3 * 8 * cells), etot[24];
  or_moments(md, f, rho, ux, uy, T);
  or_noneq(md, f, delta, tot);
  or_energy(md, f, en, etot);
  printf("bc %d %d sch %d react %d ay %g nchem %d lim %d: T0 %.6f mass %.6e\n", bcx, bcy, scheme, react, ay, nchem, lim, T[0], tot[0]);
  free(n); free(ux); free(uy); free(T); free(f); free(rho); free(delta); free(en);
  or_destroy(md);
}
int main(void) {
  run(OR_BC_PERIODIC, OR_BC_PERIODIC, OR_EULER, 1, 0, 0, OR_LIM_MINMOD);
  run(OR_BC_OUTFLOW, OR_BC_WALL, OR_RK3, 1, -0.1, 0, OR_LIM_NONE);
  run(OR_BC_WALL, OR_BC_OUTFLOW, OR_EULER, 0, -0.1, 0, OR_LIM_MINMOD);
  run(OR_BC_PERIODIC, OR_BC_WALL, OR_RK3, 1, 0, 2, OR_LIM_MINMOD);
  return 0;
}
