/* Host driver for the sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, CPU only): exercises every exported function on small
 * lattices, including the refusals.  Exit status 0 when every call behaved. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static int square(int32_t L, int32_t n_e, double rc, double T, double E, int32_t clock, int64_t hops) {
  or_params p = {L, n_e, 1.0, 1.0, rc, T, E, 11, 2, clock};
  or_state* st = NULL;
  CHECK(or_create(&p, &st) == 0 && st);
  int32_t N, no, nv;
  or_dims(st, &N, &no, &nv);
  CHECK(N == L * L && no > 0 && nv > 0);
  uint64_t* thr = malloc(sizeof(uint64_t) * (size_t)no);
  int32_t* size = malloc(sizeof(int32_t) * (size_t)no);
  int32_t* first = malloc(sizeof(int32_t) * (size_t)no);
  int32_t* vx = malloc(sizeof(int32_t) * (size_t)nv);
  int32_t* vy = malloc(sizeof(int32_t) * (size_t)nv);
  double ws, G;
  or_tower(st, thr, size, first, vx, vy, &ws, &G);
  CHECK(thr[no - 1] == ((uint64_t)1 << 32) && G > 0.0);
  for (int32_t v = 0; v < nv; ++v) CHECK(or_vec_prob(st, v) > 0.0);
  uint64_t* lab = malloc(sizeof(uint64_t) * (size_t)hops);
  int32_t* li = malloc(sizeof(int32_t) * (size_t)hops);
  int32_t* lj = malloc(sizeof(int32_t) * (size_t)hops);
  CHECK(or_run(st, hops, -1.0, 0, lab, li, lj, hops, NULL) == hops);
  CHECK(or_run(st, 5, -1.0, 0, NULL, NULL, NULL, 0, NULL) == 5);
  double* e = malloc(sizeof(double) * (size_t)N);
  double* e2 = malloc(sizeof(double) * (size_t)N);
  double* phi = malloc(sizeof(double) * (size_t)N);
  uint8_t* n = malloc((size_t)N);
  or_get_eps(st, e);
  or_recompute_eps(st, e2);
  for (int32_t l = 0; l < N; ++l) CHECK(fabs(e[l] - e2[l]) < 1e-9);
  or_get_phi(st, phi);
  or_get_occ(st, n);
  CHECK(or_set_occ(st, n) == 0);
  CHECK(isfinite(or_energy(st)));
  CHECK(isnan(or_site_eps(st, -1)) && isnan(or_site_eps(st, N)));
  double dH;
  int32_t i, v;
  double u;
  or_draw(st, 12345, &i, &v, &u);
  CHECK(i >= 0 && i < N && v >= 0 && v < nv && u > 0.0 && u < 1.0);
  double pacc = or_move(st, i, v, &dH);
  CHECK(pacc >= 0.0 && pacc <= 1.0);
  if (L <= 8) CHECK(or_acceptance(st) > 0.0);
  (void)or_invr(st, -3, 5);
  or_scalars sc;
  or_get_scalars(st, &sc);
  CHECK(sc.hops == (uint64_t)hops + 5);
  CHECK(or_naive_run(st, sc.t + 1e-3) >= 0);
  or_run(st, 0, sc.t + 1.0, 0, NULL, NULL, NULL, 0, NULL);
  n[0] = (uint8_t)(1 - n[0]);
  CHECK(or_set_occ(st, n) != 0); /* wrong electron count */
  or_destroy(st);
  or_state* lz = NULL;
  CHECK(or_create_lazy(&p, &lz) == 0);
  CHECK(isfinite(or_site_eps(lz, 0)));
  CHECK(or_run(lz, 3, -1.0, 0, NULL, NULL, NULL, 0, NULL) < 0);
  or_destroy(lz);
  free(thr); free(size); free(first); free(vx); free(vy);
  free(lab); free(li); free(lj); free(e); free(e2); free(phi); free(n);
  return 0;
}

static int cubic(void) {
  or_params p = {6, 108, 1.0, 1.0, 2.0, 0.2, 0.01, 5, 1, 0};
  or3_state* st = NULL;
  CHECK(or3_create(&p, &st) == 0 && st);
  int32_t no, nv;
  or3_tower(st, &no, &nv, NULL, NULL, NULL, NULL, NULL, NULL);
  uint64_t* thr = malloc(sizeof(uint64_t) * (size_t)no);
  int32_t *first = malloc(4 * (size_t)no), *size = malloc(4 * (size_t)no);
  int32_t *vx = malloc(4 * (size_t)nv), *vy = malloc(4 * (size_t)nv), *vz = malloc(4 * (size_t)nv);
  or3_tower(st, &no, &nv, thr, first, size, vx, vy, vz);
  uint64_t lab[200];
  int32_t li[200], lj[200];
  CHECK(or3_run(st, 200, lab, li, lj, 200) == 200);
  uint8_t n[216];
  double e[216], phi[216];
  or3_get(st, n, e, phi);
  or3_set_occ(st, n);
  CHECK(isfinite(or3_energy(st)));
  int32_t i, v;
  double u;
  or3_draw(st, 7, &i, &v, &u);
  (void)or3_invr(st, 1, -2, 3);
  or_scalars sc;
  or3_scalars(st, &sc);
  CHECK(sc.hops == 200);
  or3_destroy(st);
  free(thr); free(first); free(size); free(vx); free(vy); free(vz);
  return 0;
}

int main(void) {
  uint32_t c[4] = {1, 2, 3, 4}, k[2] = {5, 6}, w[4];
  or_philox(c, k, w);
  if (square(8, 32, 3.0, 0.2, 0.05, 0, 400)) return 1;
  if (square(15, 100, 4.0, 0.1, 0.01, 1, 300)) return 1;
  if (square(16, 128, 6.0, 0.05, 0.0, 2, 300)) return 1;
  if (square(3, 4, 1.0, 0.5, 0.0, 0, 50)) return 1;
  {
    /* pair hops: draws, moves and a run */
    or_params pp = {8, 32, 1.0, 1.0, 3.0, 0.2, 0.05, 4, 3, 0, 0.4};
    or_state* ps = NULL;
    CHECK(or_create(&pp, &ps) == 0 && ps);
    int32_t np_ = 0;
    for (uint64_t s = 1; s <= 200; ++s) {
      int32_t ip, i, v1, ve, v2;
      double u, dH;
      or_draw_label(ps, s, &ip, &i, &v1, &ve, &v2, &u);
      if (ip) {
        ++np_;
        double a = or_move_pair(ps, i, v1, ve, v2, &dH);
        CHECK(a >= 0.0 && a <= 1.0);
      }
    }
    CHECK(np_ > 40 && np_ < 120);
    uint64_t lab[400];
    int32_t li[400], lj[400];
    int64_t nl = 0;
    CHECK(or_run(ps, 200, -1.0, 0, lab, li, lj, 400, &nl) == 200 && nl >= 200);
    or_destroy(ps);
    pp.pair = 1.0;
    CHECK(or_create(&pp, &ps) != 0 && ps == NULL);
  }
  if (cubic()) return 1;
  CHECK(or_gamma_dt(3, 1, 7, 40, 123.0) > 0.0);
  or_params bad = {16, 128, 1.0, 1.0, 8.0, 0.1, 0.0, 1, 0, 0}; /* rc >= L/2 */
  or_state* st = NULL;
  CHECK(or_create(&bad, &st) != 0 && st == NULL);
  bad.rc = 4.0;
  bad.T = 0.0;
  CHECK(or_create(&bad, &st) != 0 && st == NULL);
  bad.T = 0.1;
  bad.n_e = 0;
  CHECK(or_create(&bad, &st) != 0 && st == NULL);
  or_destroy(NULL);
  printf("oracle driver ok\n");
  return 0;
}
