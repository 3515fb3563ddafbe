/* Host-side exercise of the C ABI for a sanitizer build of the library
 * (AddressSanitizer + UndefinedBehaviorSanitizer on host code).  It runs
 * without a GPU: argument validation, NULL and destroyed handles, the
 * thermal plan's host set-up, batch argument checks, error strings, and the
 * release of a plan whose device set-up fails (no device).  Exit status: the
 * number of failed expectations; a sanitizer report aborts the run. */
#include <stdio.h>
#include <string.h>

#include "shg.h"

static int failures = 0;

#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "%s:%d: expected %s (last error: %s)\n", __FILE__, \
              __LINE__, #cond, shg_last_error());                       \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

static shg_params good(void) {
  shg_params p;
  memset(&p, 0, sizeof p);
  p.nx = 64;
  p.ny = 32;
  p.nz = 10;
  p.lx = 1e-3;
  p.ly = 0.5e-3;
  p.lcr = 1e-2;
  p.lambda_f = 1064e-9;
  p.n_f = 2.14;
  p.n_sh = 2.18;
  p.d_eff = 10e-12;
  p.alpha_f = 0.05;
  p.alpha_sh = 0.2;
  p.t_ref = 330.0;
  return p;
}

static void check_params(void) {
  shg_plan *pl = (shg_plan *)0x1;
  shg_params p = good();
  p.nx = 63;
  EXPECT(shg_plan_create(&pl, &p, SHG_C64) == SHG_EINVAL && pl == NULL);
  EXPECT(strstr(shg_last_error(), "power of two") != NULL);
  p = good();
  p.nz = 0;
  EXPECT(shg_plan_create(&pl, &p, SHG_C64) == SHG_EINVAL);
  p = good();
  p.lcr = -1.0;
  EXPECT(shg_plan_create(&pl, &p, SHG_C64) == SHG_EINVAL);
  p = good();
  p.flags = 1u << 9;
  EXPECT(shg_plan_create(&pl, &p, SHG_C64) == SHG_EINVAL);
  p = good();
  p.grating_period = 8e-6;
  p.grating_a = -1.0;
  EXPECT(shg_plan_create(&pl, &p, SHG_C64) == SHG_EINVAL);
  p = good();
  EXPECT(shg_plan_create(&pl, &p, (shg_dtype)7) == SHG_EINVAL);
  EXPECT(shg_plan_create(NULL, &p, SHG_C64) == SHG_EINVAL);
  EXPECT(shg_plan_create(&pl, NULL, SHG_C64) == SHG_EINVAL);
  /* valid parameters: without a device the set-up fails after validation and
   * must release what it built; with one the plan is created and destroyed */
  int rc = shg_plan_create(&pl, &p, SHG_C64);
  EXPECT(rc == SHG_OK || rc == SHG_EDEVICE || rc == SHG_ENOMEM);
  if (rc == SHG_OK) {
    char buf[8];
    EXPECT(shg_plan_describe(pl, buf, sizeof buf) == SHG_OK && strlen(buf) < sizeof buf);
    EXPECT(shg_workspace_bytes(pl, 0) > 0 && shg_workspace_bytes(pl, 1) > 0);
    EXPECT(shg_plan_set_schedule(pl, 3, 7, 0, 0) == SHG_EUNSUPPORTED);
    EXPECT(shg_plan_destroy(pl) == SHG_OK);
  } else {
    EXPECT(pl == NULL);
  }
}

static void check_handles(void) {
  char buf[64];
  double out[4];
  EXPECT(shg_plan_destroy(NULL) == SHG_OK);
  EXPECT(shg_workspace_bytes(NULL, 0) == 0);
  EXPECT(shg_propagate(NULL, NULL, NULL, NULL, NULL, 0, 1, NULL, NULL, NULL) == SHG_ESTATE);
  EXPECT(shg_propagate_heat(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == SHG_ESTATE);
  EXPECT(shg_propagate_adjoint(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL,
                               NULL, NULL, NULL, NULL, NULL, NULL) == SHG_ESTATE);
  EXPECT(shg_plan_describe(NULL, buf, sizeof buf) == SHG_ESTATE);
  EXPECT(shg_plan_kernel_times(NULL, out) == SHG_ESTATE);
  EXPECT(shg_plan_set_timing(NULL, 1) == SHG_ESTATE);
  EXPECT(shg_plan_set_schedule(NULL, 0, 0, 0, 0) == SHG_ESTATE);
  EXPECT(shg_batch_workspace_bytes(0, NULL) == 0);
  EXPECT(shg_propagate_batch(0, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == SHG_EINVAL);
  shg_plan *none[1] = {NULL};
  void *f[1] = {NULL};
  EXPECT(shg_propagate_batch(1, none, f, f, NULL, NULL, NULL, NULL) != SHG_OK);
  EXPECT(shg_thermal_destroy(NULL) == SHG_OK);
  EXPECT(shg_thermal_workspace_bytes(NULL) == 0);
  EXPECT(shg_last_error() != NULL);
}

static void check_thermal(void) {
  shg_thermal_params tp;
  memset(&tp, 0, sizeof tp);
  tp.nx = 32;
  tp.ny = 32;
  tp.nz = 8;
  tp.lx = 1e-3;
  tp.ly = 1e-3;
  tp.lcr = 2e-3;
  tp.k_th = 5.0;
  tp.h_conv = 20.0;
  tp.t_inf = 295.0;
  tp.t_oven = 330.0;
  tp.faces[2] = SHG_FACE_OVEN;
  shg_thermal *th = NULL;
  shg_thermal_params bad = tp;
  bad.k_th = 0.0;
  EXPECT(shg_thermal_create(&th, &bad, SHG_C64) == SHG_EINVAL && th == NULL);
  bad = tp;
  bad.faces[0] = 9;
  EXPECT(shg_thermal_create(&th, &bad, SHG_C64) == SHG_EINVAL);
  bad = tp;
  bad.faces[2] = SHG_FACE_INSULATED;
  bad.h_conv = 0.0;   /* no oven and no cooled face: T undetermined */
  EXPECT(shg_thermal_create(&th, &bad, SHG_C64) == SHG_EINVAL);
  EXPECT(shg_thermal_create(&th, &tp, SHG_C128) == SHG_OK && th != NULL);
  if (th) {
    EXPECT(shg_thermal_workspace_bytes(th) > 0);
    EXPECT(shg_thermal_solve(th, NULL, NULL, NULL, 1e-6, 10, NULL, NULL, NULL, NULL) == SHG_EINVAL);
    EXPECT(shg_thermal_destroy(th) == SHG_OK);
  }
}

int main(void) {
  check_params();
  check_handles();
  check_thermal();
  printf("abi harness: %d failure(s)\n", failures);
  return failures;
}
