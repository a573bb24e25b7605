/* A plain C99 consumer of include/dbm.h, built and run by
 * tests/test_abi_host.py: the header compiles as C, the library links from
 * C, and the host-only entry points behave as documented (no GPU needed). */
#include <stdio.h>
#include <string.h>

#include "dbm.h"

static int fail(const char *what) {
  printf("FAIL %s\n", what);
  return 1;
}

int main(void) {
  dbm_species sp[2];
  dbm_config c;
  size_t b32, b64, bx, big;
  dbm_handle h = NULL;
  int k, rc;
  memset(sp, 0, sizeof sp);
  for (k = 0; k < 2; ++k) {
    sp[k].m = 1.0 + k;
    sp[k].I = 3.0;
    sp[k].tau = 2e-5;
    sp[k].v[0] = 1.5; sp[k].v[1] = 0.8; sp[k].v[2] = 2.2; sp[k].v[3] = 2.6;
    sp[k].eta[0] = 2.5;
  }
  memset(&c, 0, sizeof c);
  c.nx = 64; c.ny = 48;
  c.dx = c.dy = 1e-3; c.dt = 1e-5;
  c.bc_x = DBM_BC_PERIODIC; c.bc_y = DBM_BC_OUTFLOW;
  c.nspecies = 2; c.species = sp;
  c.time_scheme = DBM_EULER; c.limiter = DBM_LIM_MINMOD;
  c.precision = DBM_FP32_BULK; b32 = dbm_workspace_bytes(&c, 1);
  c.precision = DBM_FP32X;     bx = dbm_workspace_bytes(&c, 1);
  c.precision = DBM_FP64;      b64 = dbm_workspace_bytes(&c, 1);
  if (!(b32 > 0 && b32 < bx && bx < b64)) return fail("workspace ordering FP32 < FP32X < FP64");
  if (b32 < 3u * 2u * 16u * 64u * 48u * 4u) return fail("three FP32 buffers fit");
  c.nx = 128; c.ny = 96; big = dbm_workspace_bytes(&c, 1);
  if (big < 3 * b64 || big > 5 * b64) return fail("workspace scales with the grid");
  c.nx = 0;
  if (dbm_workspace_bytes(&c, 1) != 0) return fail("bad grid gives 0 bytes");
  c.nx = 64; c.ny = 48;
  rc = dbm_create(&c, 1, NULL, NULL, b64, &h);
  if (rc != DBM_ERR_WORKSPACE || h != NULL) return fail("missing workspace rejected");
  if (dbm_last_error() == NULL || dbm_last_error()[0] == 0) return fail("error message kept");
  c.precision = 7;
  if (dbm_workspace_bytes(&c, 1) != 0) return fail("bad precision gives 0 bytes");
  if (dbm_destroy(NULL) != DBM_ERR_ARG) return fail("null handle rejected");
  printf("OK %zu %zu %zu\n", b32, bx, b64);
  return 0;
}
