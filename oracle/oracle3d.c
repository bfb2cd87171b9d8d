/* oracle3d.c -- serial FP64 oracle of the mixed rejection KMC on the simple cubic lattice.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle.c).  The paper develops the
 * method for D dimensions (Eq. 1-2 hold for any lattice; the 2D square lattice is its test
 * case) and notes that the same algorithm carries over to 3D ("Code performance", last
 * paragraphs).  This file is the 3D counterpart of oracle.c: L^3 sites on a torus with the
 * minimum image convention, hop vectors |d| <= rc grouped in orbits of the cube's symmetry
 * group (48 signed permutations), the serial mixed algorithm with labels s = 1, 2, ...
 * and the deterministic clock t = s_last / Gamma.
 *
 * Proposal of label s: Philox4x32-10 of (s, sample id, PROPOSE) under the seed; site
 * i = mulhi(w0, N); orbit: the first o with w1 < thr[o]; member mulhi(w3, size_o) of the
 * orbit's members sorted by (dz, dy, dx); acceptance uniform u = (w2 + 1/2) 2^-32.
 * Accept iff n_i = 1, n_j = 0 and (dH <= 0 or u < exp(-dH / T)),
 * dH = ((eps_j - eps_i) - 1/r_ij) - E dx.  Executing: n_i = 0, n_j = 1, P += dx,
 * H0 += (eps_j - eps_i) - 1/r_ij, eps_l += 1/r_lj - 1/r_li for every l (1/r(0) := 0).
 * Initial state: the n_e sites with the smallest 64-bit keys w0 w1 of Philox(l, sample id,
 * OCC) (ties by index) are occupied, as in 2D; phi_l = W (2 u - 1) from Philox(l, sample id, PHI) (u from
 * words 0, 1 as in the 2D oracle); eps_l = phi_l + sum_{m != l} (n_m - nu) / r_lm in index
 * order. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

enum { T3_PROPOSE = 0, T3_OCC = 1, T3_PHI = 2 };

struct or3_state {
  or_params p;
  int32_t L, N;
  double nu;
  int32_t n_orb, n_vec;
  int32_t *orb_first, *orb_size, *orb_r2;
  uint64_t* thr;
  int32_t *vx, *vy, *vz;
  double wsum, Gamma;
  double* invr; /* by (wrap dz) L^2 + (wrap dy) L + wrap dx */
  uint8_t* n;
  double *phi, *eps;
  uint64_t s_last, s_scan, hops, theta_pass;
  int64_t P;
  double t, H0;
};

static void st3_stream(const or3_state* st, uint64_t idx, uint32_t tag, uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), st->p.sample_id, tag};
  uint32_t key[2] = {(uint32_t)st->p.seed, (uint32_t)(st->p.seed >> 32)};
  or_philox(ctr, key, w);
}

static int32_t w3(int32_t a, int32_t L) {
  int32_t r = a % L;
  return r < 0 ? r + L : r;
}

static int32_t fold3(int32_t a, int32_t L) {
  a = w3(a, L);
  return L - a < a ? L - a : a;
}

double or3_invr(const or3_state* st, int32_t dx, int32_t dy, int32_t dz) {
  const int32_t L = st->L;
  return st->invr[(w3(dz, L) * L + w3(dy, L)) * L + w3(dx, L)];
}

typedef struct { int32_t a, b, c, r2; } rep3;
typedef struct { int32_t dx, dy, dz; } v3;

static int cmp_rep3(const void* x, const void* y) {
  const rep3 *p = (const rep3*)x, *q = (const rep3*)y;
  if (p->r2 != q->r2) return p->r2 < q->r2 ? -1 : 1;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  return 0;
}

static int cmp_v3(const void* x, const void* y) {
  const v3 *p = (const v3*)x, *q = (const v3*)y;
  if (p->dz != q->dz) return p->dz < q->dz ? -1 : 1;
  if (p->dy != q->dy) return p->dy < q->dy ? -1 : 1;
  if (p->dx != q->dx) return p->dx < q->dx ? -1 : 1;
  return 0;
}

/* Orbits: representatives a >= b >= c >= 0, a >= 1, a^2 + b^2 + c^2 <= rc^2, ordered by
 * (r^2, a, b); members: the distinct signed permutations of (a, b, c); orbit weight
 * size * exp(-2 r / xi); thresholds floor(2^32 cum_o / total), the last one 2^32. */
static int tower3(or3_state* st) {
  const double rc = st->p.rc, xi = st->p.xi;
  const int32_t amax = (int32_t)floor(rc) + 1;
  rep3* reps = (rep3*)malloc(sizeof(rep3) * (size_t)(amax + 1) * (amax + 1) * (amax + 1));
  if (!reps) return -2;
  int32_t n = 0;
  for (int32_t a = 1; a <= amax; ++a)
    for (int32_t b = 0; b <= a; ++b)
      for (int32_t c = 0; c <= b; ++c)
        if ((double)(a * a + b * b + c * c) <= rc * rc) {
          reps[n].a = a; reps[n].b = b; reps[n].c = c; reps[n].r2 = a * a + b * b + c * c; ++n;
        }
  if (n == 0) { free(reps); return -1; }
  qsort(reps, (size_t)n, sizeof(rep3), cmp_rep3);
  st->n_orb = n;
  st->orb_first = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  st->orb_size = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  st->orb_r2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  st->thr = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  st->vx = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * 48);
  st->vy = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * 48);
  st->vz = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * 48);
  double* cum = (double*)malloc(sizeof(double) * (size_t)n);
  if (!st->orb_first || !st->orb_size || !st->orb_r2 || !st->thr || !st->vx || !st->vy || !st->vz || !cum) {
    free(reps); free(cum); return -2;
  }
  static const int32_t perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int32_t nv = 0;
  double acc = 0.0;
  for (int32_t o = 0; o < n; ++o) {
    const int32_t abc[3] = {reps[o].a, reps[o].b, reps[o].c};
    v3 u[48];
    int32_t nu = 0;
    for (int32_t p = 0; p < 6; ++p)
      for (int32_t sgn = 0; sgn < 8; ++sgn) {
        v3 c;
        c.dx = abc[perm[p][0]] * ((sgn & 1) ? -1 : 1);
        c.dy = abc[perm[p][1]] * ((sgn & 2) ? -1 : 1);
        c.dz = abc[perm[p][2]] * ((sgn & 4) ? -1 : 1);
        int dup = 0;
        for (int32_t q = 0; q < nu; ++q)
          if (u[q].dx == c.dx && u[q].dy == c.dy && u[q].dz == c.dz) dup = 1;
        if (!dup) u[nu++] = c;
      }
    qsort(u, (size_t)nu, sizeof(v3), cmp_v3);
    st->orb_first[o] = nv;
    st->orb_size[o] = nu;
    st->orb_r2[o] = reps[o].r2;
    for (int32_t q = 0; q < nu; ++q) {
      st->vx[nv] = u[q].dx; st->vy[nv] = u[q].dy; st->vz[nv] = u[q].dz; ++nv;
    }
    acc = acc + (double)nu * exp(-2.0 * sqrt((double)reps[o].r2) / xi);
    cum[o] = acc;
  }
  st->n_vec = nv;
  st->wsum = acc;
  for (int32_t o = 0; o + 1 < n; ++o) st->thr[o] = (uint64_t)floor(ldexp(cum[o] / acc, 32));
  st->thr[n - 1] = (uint64_t)1 << 32;
  st->Gamma = (double)st->N * acc;
  free(reps);
  free(cum);
  return 0;
}

static double eps3_site(const or3_state* st, int32_t l) {
  const int32_t L = st->L, N = st->N;
  const int32_t xl = l % L, yl = (l / L) % L, zl = l / (L * L);
  double acc = st->phi[l];
  for (int32_t m = 0; m < N; ++m) {
    if (m == l) continue;
    const double q = (double)st->n[m] - st->nu;
    acc = acc + q * or3_invr(st, xl - m % L, yl - (m / L) % L, zl - m / (L * L));
  }
  return acc;
}

double or3_energy(const or3_state* st) {
  const int32_t L = st->L, N = st->N;
  double h1 = 0.0, h2 = 0.0;
  for (int32_t i = 0; i < N; ++i) h1 = h1 + st->phi[i] * (double)st->n[i];
  for (int32_t i = 0; i < N; ++i) {
    const double qi = (double)st->n[i] - st->nu;
    for (int32_t j = 0; j < N; ++j) {
      if (j == i) continue;
      const double qj = (double)st->n[j] - st->nu;
      h2 = h2 + qi * qj * or3_invr(st, i % L - j % L, (i / L) % L - (j / L) % L, i / (L * L) - j / (L * L));
    }
  }
  return h1 + 0.5 * h2;
}

typedef struct { uint64_t key; int32_t idx; } key3;
static int cmp_key3(const void* x, const void* y) {
  const key3 *p = (const key3*)x, *q = (const key3*)y;
  if (p->key != q->key) return p->key < q->key ? -1 : 1;
  return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

int or3_create(const or_params* p, or3_state** out) {
  *out = NULL;
  if (p->L < 3 || p->L > 40) return -1;
  const int32_t N = p->L * p->L * p->L;
  if (p->n_e < 1 || p->n_e >= N) return -1;
  if (!(p->T > 0.0) || !(p->xi > 0.0) || !(p->W >= 0.0)) return -1;
  if (!(p->rc >= 1.0) || !(2.0 * p->rc < (double)p->L)) return -1;
  if (p->clock_mode != 0) return -1;
  or3_state* st = (or3_state*)calloc(1, sizeof(or3_state));
  if (!st) return -2;
  st->p = *p;
  st->L = p->L;
  st->N = N;
  st->nu = (double)p->n_e / (double)N;
  int rc = tower3(st);
  st->invr = (double*)malloc(sizeof(double) * (size_t)N);
  st->n = (uint8_t*)calloc((size_t)N, 1);
  st->phi = (double*)malloc(sizeof(double) * (size_t)N);
  st->eps = (double*)malloc(sizeof(double) * (size_t)N);
  key3* keys = (key3*)malloc(sizeof(key3) * (size_t)N);
  if (rc != 0 || !st->invr || !st->n || !st->phi || !st->eps || !keys) {
    free(keys);
    or3_destroy(st);
    return rc != 0 ? rc : -2;
  }
  const int32_t L = st->L;
  for (int32_t z = 0; z < L; ++z)
    for (int32_t y = 0; y < L; ++y)
      for (int32_t x = 0; x < L; ++x) {
        const int32_t a = fold3(x, L), b = fold3(y, L), c = fold3(z, L);
        const int32_t r2 = a * a + b * b + c * c;
        st->invr[(z * L + y) * L + x] = r2 == 0 ? 0.0 : 1.0 / sqrt((double)r2);
      }
  for (int32_t l = 0; l < N; ++l) {
    uint32_t w[4];
    st3_stream(st, (uint64_t)l, T3_OCC, w);
    keys[l].key = ((uint64_t)w[0] << 32) | (uint64_t)w[1];
    keys[l].idx = l;
  }
  qsort(keys, (size_t)N, sizeof(key3), cmp_key3);
  for (int32_t k = 0; k < p->n_e; ++k) st->n[keys[k].idx] = 1;
  free(keys);
  for (int32_t l = 0; l < N; ++l) {
    uint32_t w[4];
    st3_stream(st, (uint64_t)l, T3_PHI, w);
    const uint64_t k = ((uint64_t)w[0] << 20) | (uint64_t)(w[1] >> 12);
    const double u = (double)(2u * k + 1u) * 0x1p-53;
    st->phi[l] = p->W * (2.0 * u - 1.0);
  }
  for (int32_t l = 0; l < N; ++l) st->eps[l] = eps3_site(st, l);
  st->H0 = or3_energy(st);
  *out = st;
  return 0;
}

void or3_destroy(or3_state* st) {
  if (!st) return;
  free(st->orb_first); free(st->orb_size); free(st->orb_r2); free(st->thr);
  free(st->vx); free(st->vy); free(st->vz); free(st->invr); free(st->n); free(st->phi); free(st->eps);
  free(st);
}

void or3_draw(const or3_state* st, uint64_t s, int32_t* i, int32_t* v, double* u) {
  uint32_t w[4];
  st3_stream(st, s, T3_PROPOSE, w);
  *i = (int32_t)(((uint64_t)w[0] * (uint64_t)st->N) >> 32);
  int32_t o = 0;
  while (!((uint64_t)w[1] < st->thr[o])) ++o;
  *v = st->orb_first[o] + (int32_t)(((uint64_t)w[3] * (uint64_t)st->orb_size[o]) >> 32);
  *u = ((double)w[2] + 0.5) * 0x1p-32;
}

static int32_t partner3(const or3_state* st, int32_t i, int32_t v) {
  const int32_t L = st->L;
  const int32_t x = w3(i % L + st->vx[v], L), y = w3((i / L) % L + st->vy[v], L), z = w3(i / (L * L) + st->vz[v], L);
  return (z * L + y) * L + x;
}

int64_t or3_run(or3_state* st, int64_t n_hops, uint64_t* log_label, int32_t* log_i, int32_t* log_j,
                int64_t log_cap) {
  const int32_t L = st->L, N = st->N;
  int64_t done = 0;
  while (done < n_hops) {
    const uint64_t s = ++st->s_scan;
    int32_t i, v;
    double u;
    or3_draw(st, s, &i, &v, &u);
    const int32_t j = partner3(st, i, v);
    if (!(st->n[i] == 1 && st->n[j] == 0)) continue;
    st->theta_pass++;
    const double vij = or3_invr(st, st->vx[v], st->vy[v], st->vz[v]);
    const double dH = ((st->eps[j] - st->eps[i]) - vij) - st->p.E * (double)st->vx[v];
    if (!(dH <= 0.0 || u < exp(-dH / st->p.T))) continue;
    const double dH0 = (st->eps[j] - st->eps[i]) - vij;
    st->n[i] = 0;
    st->n[j] = 1;
    st->P += st->vx[v];
    st->H0 = st->H0 + dH0;
    st->s_last = s;
    st->hops++;
    if (log_label && done < log_cap) {
      log_label[done] = s;
      log_i[done] = i;
      log_j[done] = j;
    }
    const int32_t xi = i % L, yi = (i / L) % L, zi = i / (L * L);
    const int32_t xj = j % L, yj = (j / L) % L, zj = j / (L * L);
    for (int32_t l = 0; l < N; ++l) {
      const int32_t x = l % L, y = (l / L) % L, z = l / (L * L);
      const double a = or3_invr(st, x - xj, y - yj, z - zj), b = or3_invr(st, x - xi, y - yi, z - zi);
      st->eps[l] = st->eps[l] + (a - b);
    }
    st->t = (double)st->s_last / st->Gamma;
    ++done;
  }
  return done;
}

void or3_get(const or3_state* st, uint8_t* n, double* eps, double* phi) {
  if (n) memcpy(n, st->n, (size_t)st->N);
  if (eps) memcpy(eps, st->eps, sizeof(double) * (size_t)st->N);
  if (phi) memcpy(phi, st->phi, sizeof(double) * (size_t)st->N);
}

void or3_scalars(const or3_state* st, or_scalars* out) {
  memset(out, 0, sizeof(*out));
  out->s_last = st->s_last;
  out->s_scan = st->s_scan;
  out->hops = st->hops;
  out->P = st->P;
  out->t = st->t;
  out->H0 = st->H0;
  out->theta_pass = st->theta_pass;
  out->Gamma = st->Gamma;
}

void or3_tower(const or3_state* st, int32_t* n_orb, int32_t* n_vec, uint64_t* thr, int32_t* first,
               int32_t* size, int32_t* vx, int32_t* vy, int32_t* vz) {
  *n_orb = st->n_orb;
  *n_vec = st->n_vec;
  if (thr) memcpy(thr, st->thr, sizeof(uint64_t) * (size_t)st->n_orb);
  if (first) memcpy(first, st->orb_first, sizeof(int32_t) * (size_t)st->n_orb);
  if (size) memcpy(size, st->orb_size, sizeof(int32_t) * (size_t)st->n_orb);
  if (vx) memcpy(vx, st->vx, sizeof(int32_t) * (size_t)st->n_vec);
  if (vy) memcpy(vy, st->vy, sizeof(int32_t) * (size_t)st->n_vec);
  if (vz) memcpy(vz, st->vz, sizeof(int32_t) * (size_t)st->n_vec);
}

void or3_set_occ(or3_state* st, const uint8_t* n) {
  memcpy(st->n, n, (size_t)st->N);
  for (int32_t l = 0; l < st->N; ++l) st->eps[l] = eps3_site(st, l);
  st->H0 = or3_energy(st);
}
