/* Host driver for the sanitizer build of libcgkmc's host code (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host side only, CPU only).  It calls only what runs
 * without a device: arena planning for every kernel family and its refusals, and the
 * argument checks that every entry point makes before any HIP call.  No kernel is launched:
 * cg_create is given no arena, so it returns before touching device memory.  Exit status 0
 * when every call behaved. */
#include <stdio.h>
#include <string.h>

#include "cgkmc.h"

#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #c, cg_last_error()); \
      return 1;                                                        \
    }                                                                  \
  } while (0)

static cg_sample_desc sample(int32_t L, double rc, uint32_t id, int32_t dim) {
  cg_sample_desc s;
  memset(&s, 0, sizeof s);
  s.L = L;
  s.n_electrons = dim == 3 ? L * L * L / 2 : L * L / 2;
  s.W = 1.0;
  s.xi = 1.0;
  s.rc = rc;
  s.T = 0.05;
  s.E = 0.005;
  s.seed = 3;
  s.sample_id = id;
  s.dim = dim;
  return s;
}

static cg_run_opts opts(int32_t precision, int32_t variant) {
  cg_run_opts o;
  memset(&o, 0, sizeof o);
  o.precision = precision;
  o.variant = variant;
  return o;
}

int main(void) {
  size_t bytes = 0;
  cg_sample_desc s[6];
  cg_run_opts o;
  /* every planning path: exact-geometry FP32 / FP64, generic, arena energies, whole-GPU,
     label-parallel, cubic */
  for (int k = 0; k < 4; ++k) s[k] = sample(128, 10.0, (uint32_t)k, 2);
  o = opts(CG_FP32_REFRESH, 0);
  CHECK(cg_arena_bytes(s, 4, &o, &bytes) == CG_OK && bytes > 0);
  o = opts(CG_FP64, 0);
  CHECK(cg_arena_bytes(s, 4, &o, &bytes) == CG_OK && bytes > 0);
  s[1] = sample(33, 8.0, 1, 2);
  s[2] = sample(160, 10.0, 2, 2);
  o = opts(CG_FP32_REFRESH, 1);
  CHECK(cg_arena_bytes(s, 3, &o, &bytes) == CG_OK && bytes > 0);
  o = opts(CG_FP32_REFRESH, 2);
  s[2] = sample(64, 8.0, 2, 2);
  CHECK(cg_arena_bytes(s, 3, &o, &bytes) == CG_OK);
  s[0] = sample(1024, 10.0, 0, 2);
  o = opts(CG_FP64, 0);
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_OK && bytes > 0);
  s[0] = sample(256, 10.0, 0, 2);
  o.spread = 16;
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_OK);
  o.spread = 8;
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL);
  s[0] = sample(64, 10.0, 0, 2);
  o = opts(CG_FP64, 6);
  o.spread = 32;
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_OK);
  s[0] = sample(16, 4.0, 0, 3);
  o = opts(CG_FP64, 0);
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_OK);
  /* refusals */
  s[0] = sample(128, 64.0, 0, 2);
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL && strlen(cg_last_error()) > 0);
  s[0] = sample(2, 0.5, 0, 2);
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL);
  s[0] = sample(300, 10.0, 0, 2);
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL);
  s[0] = sample(64, 8.0, 0, 2);
  s[0].T = 0.0;
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL);
  s[0] = sample(64, 8.0, 0, 4);
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL);
  s[0] = sample(64, 8.0, 0, 2);
  o.precision = 7;
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL);
  o = opts(CG_FP64, 9);
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL);
  o = opts(CG_FP64, 0);
  o.block = 100;
  CHECK(cg_arena_bytes(s, 1, &o, &bytes) == CG_EINVAL);
  o = opts(CG_FP64, 0);
  CHECK(cg_arena_bytes(s, 0, &o, &bytes) == CG_EINVAL);
  CHECK(cg_arena_bytes(NULL, 1, &o, &bytes) == CG_EINVAL);
  CHECK(cg_arena_bytes(s, 1, &o, NULL) == CG_EINVAL);
  /* entry points refuse a null context or output before any device work */
  cg_ctx* ctx = NULL;
  CHECK(cg_create(NULL, s, 1, &o, NULL, 0, NULL) == CG_EINVAL);
  CHECK(cg_create(&ctx, s, 1, &o, NULL, 0, NULL) != CG_OK && ctx == NULL);
  CHECK(cg_destroy(NULL) == CG_OK);
  CHECK(cg_run_hops(NULL, 10) == CG_EINVAL);
  CHECK(cg_run_time(NULL, 1.0) == CG_EINVAL);
  CHECK(cg_refresh(NULL) == CG_EINVAL);
  CHECK(cg_set_TE(NULL, 0, 0.1, 0.0) == CG_EINVAL);
  double t;
  cg_stats st;
  uint8_t occ[4];
  CHECK(cg_get_stats(NULL, 0, &st) == CG_EINVAL);
  CHECK(cg_get_clock(NULL, 0, &t) == CG_EINVAL);
  CHECK(cg_get_occupation(NULL, 0, occ) == CG_EINVAL);
  CHECK(cg_take_kernel_time(NULL, NULL, NULL, NULL, NULL) == CG_EINVAL);
  printf("host driver ok\n");
  return 0;
}
