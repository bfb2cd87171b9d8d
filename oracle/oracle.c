/*
 * oracle.c -- serial FP64 mixed rejection KMC for the 2D lattice Coulomb glass.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain loops, no blocking or fusion;
 * every function names the passage of the paper it follows.  Build:
 *   gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared oracle.c -lm
 * (contraction off so that a*b+c is never fused: the order of every rounding is
 * the one written here).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), the counter-based RNG the
 * paper uses for its many parallel streams (section "Hopping conduction",
 * implementation paragraph).  Round: two 32x32->64 products of counter words 0
 * and 2 with the multipliers, outputs permuted and xored with the key; the key
 * is bumped by the Weyl constants between rounds.                              */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { TAG_PROPOSE = 0, TAG_OCC = 1, TAG_PHI = 2, TAG_CLOCK = 3, TAG_GAMMA = 4, TAG_NAIVE = 5, TAG_PAIR = 6 };

static void stream(const or_state* st, uint64_t idx, uint32_t tag, uint32_t w[4]);

/* uniform in (0,1) on the grid (2k+1) 2^-53, k a 52-bit integer from two words */
static double unit52(uint32_t hi, uint32_t lo) {
  uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
  return (double)(2u * k + 1u) * 0x1p-53;
}

/* ------------------------------------------------------------------------- */
struct or_state {
  or_params p;
  int32_t N;
  int32_t lazy; /* created without energies (occupation and disorder only) */
  double nu;
  /* proposal law */
  int32_t n_orb, n_vec;
  int32_t* orb_r2;
  int32_t* orb_size;
  int32_t* orb_first;
  uint64_t* thr;
  int32_t* vec_dx;
  int32_t* vec_dy;
  double wsum, Gamma;
  /* pair hops: orbit thresholds of the uniform law over the hop vectors (partner offset),
   * the threshold of the pair choice, and the label rate Gamma / (1 - pair) */
  uint64_t* thr_u;
  uint64_t thr_pair;
  double Gamma_lab;
  /* 1/r by separation: invr[(ddy mod L) * L + (ddx mod L)] */
  double* invr;
  /* configuration */
  uint8_t* n;
  double* phi;
  double* eps;
  uint64_t s_last, s_scan, hops, theta_pass;
  int64_t P;
  double t, H0;
  uint64_t naive_k; /* proposals made by the naive algorithm */
};

static void stream(const or_state* st, uint64_t idx, uint32_t tag, uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), st->p.sample_id, tag};
  uint32_t key[2] = {(uint32_t)st->p.seed, (uint32_t)(st->p.seed >> 32)};
  or_philox(ctr, key, w);
}

static int32_t wrap(int32_t a, int32_t L) {
  int32_t r = a % L;
  return r < 0 ? r + L : r;
}

/* Minimum-image distance on the torus (section "Results ... two dimensions":
 * toroidal boundaries, minimal image convention for r_ij and dx_ij). */
static double invr_def(int32_t L, int32_t ddx, int32_t ddy) {
  int32_t a = wrap(ddx, L), b = wrap(ddy, L);
  if (L - a < a) a = L - a;
  if (L - b < b) b = L - b;
  int32_t r2 = a * a + b * b;
  if (r2 == 0) return 0.0;
  return 1.0 / sqrt((double)r2);
}

double or_invr(const or_state* st, int32_t ddx, int32_t ddy) {
  int32_t L = st->p.L;
  return st->invr[wrap(ddy, L) * L + wrap(ddx, L)];
}

/* ------------------------------------------------------------------------- */
/* Proposal law of the mixed algorithm: Q ~ Gamma^T_ij = exp(-2 r_ij / xi), which
 * on a lattice depends only on the displacement (section "Hopping conduction",
 * mixed algorithm and lattice paragraph).  Displacements with |d| <= rc are
 * grouped in orbits of the square's symmetry group (all (+-a,+-b), (+-b,+-a));
 * members of an orbit share r and therefore weight.  Tower sampling over the
 * cumulative orbit weights picks the orbit, a uniform member picks d.          */
typedef struct { int32_t a, b, r2; } orbit_rep;

static int cmp_rep(const void* x, const void* y) {
  const orbit_rep* p = (const orbit_rep*)x;
  const orbit_rep* q = (const orbit_rep*)y;
  if (p->r2 != q->r2) return p->r2 < q->r2 ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  return 0;
}

typedef struct { int32_t dx, dy; } vec2;

static int cmp_vec(const void* x, const void* y) {
  const vec2* p = (const vec2*)x;
  const vec2* q = (const vec2*)y;
  if (p->dy != q->dy) return p->dy < q->dy ? -1 : 1;
  if (p->dx != q->dx) return p->dx < q->dx ? -1 : 1;
  return 0;
}

static int build_tower(or_state* st) {
  const double rc = st->p.rc, xi = st->p.xi;
  int32_t amax = (int32_t)floor(rc) + 1;
  int32_t cap = (amax + 1) * (amax + 1);
  orbit_rep* reps = (orbit_rep*)malloc(sizeof(orbit_rep) * (size_t)cap);
  if (!reps) return -2;
  int32_t n = 0;
  for (int32_t a = 1; a <= amax; ++a)
    for (int32_t b = 0; b <= a; ++b)
      if ((double)(a * a + b * b) <= rc * rc) {
        reps[n].a = a; reps[n].b = b; reps[n].r2 = a * a + b * b; ++n;
      }
  if (n == 0) { free(reps); return -1; }
  qsort(reps, (size_t)n, sizeof(orbit_rep), cmp_rep);

  st->n_orb = n;
  st->orb_r2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  st->orb_size = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  st->orb_first = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  st->thr = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  st->thr_u = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  st->vec_dx = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * 8);
  st->vec_dy = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * 8);
  double* cum = (double*)malloc(sizeof(double) * (size_t)n);
  if (!st->orb_r2 || !st->orb_size || !st->orb_first || !st->thr || !st->thr_u || !st->vec_dx ||
      !st->vec_dy || !cum) { free(reps); free(cum); return -2; }

  int32_t nv = 0;
  double acc = 0.0;
  for (int32_t o = 0; o < n; ++o) {
    int32_t a = reps[o].a, b = reps[o].b;
    vec2 cand[8] = {{a, b}, {-a, b}, {a, -b}, {-a, -b}, {b, a}, {-b, a}, {b, -a}, {-b, -a}};
    vec2 uniq[8];
    int32_t nu = 0;
    for (int k = 0; k < 8; ++k) {
      int dup = 0;
      for (int q = 0; q < nu; ++q)
        if (uniq[q].dx == cand[k].dx && uniq[q].dy == cand[k].dy) dup = 1;
      if (!dup) uniq[nu++] = cand[k];
    }
    qsort(uniq, (size_t)nu, sizeof(vec2), cmp_vec);
    st->orb_r2[o] = reps[o].r2;
    st->orb_size[o] = nu;
    st->orb_first[o] = nv;
    for (int32_t q = 0; q < nu; ++q) {
      st->vec_dx[nv] = uniq[q].dx;
      st->vec_dy[nv] = uniq[q].dy;
      ++nv;
    }
    double r = sqrt((double)reps[o].r2);
    double w = (double)nu * exp(-2.0 * r / xi);
    acc = acc + w;
    cum[o] = acc;
  }
  st->n_vec = nv;
  st->wsum = acc;
  for (int32_t o = 0; o + 1 < n; ++o)
    st->thr[o] = (uint64_t)floor(ldexp(cum[o] / acc, 32));
  st->thr[n - 1] = (uint64_t)1 << 32;
  /* uniform law over the nv hop vectors by orbit: cumulative orbit sizes */
  for (int32_t o = 0; o + 1 < n; ++o)
    st->thr_u[o] = ((uint64_t)(st->orb_first[o] + st->orb_size[o]) << 32) / (uint64_t)nv;
  st->thr_u[n - 1] = (uint64_t)1 << 32;
  /* Gamma = sum_i sum_{j != i} Gamma^T_ij = N * sum_d exp(-2|d|/xi) */
  st->Gamma = (double)st->N * acc;
  free(reps);
  free(cum);
  return 0;
}

void or_draw(const or_state* st, uint64_t s, int32_t* i, int32_t* v, double* u) {
  uint32_t w[4];
  stream(st, s, TAG_PROPOSE, w);
  *i = (int32_t)(((uint64_t)w[0] * (uint64_t)st->N) >> 32);
  int32_t o = 0;
  while (!((uint64_t)w[1] < st->thr[o])) ++o;
  uint32_t member = w[3] & (uint32_t)(st->orb_size[o] - 1);
  *v = st->orb_first[o] + (int32_t)member;
  *u = unit52(w[2], w[3]);
}

double or_vec_prob(const or_state* st, int32_t v) {
  int32_t o = 0;
  while (!(v < st->orb_first[o] + st->orb_size[o])) ++o;
  uint64_t lo = (o == 0) ? 0 : st->thr[o - 1];
  double po = (double)(st->thr[o] - lo) * 0x1p-32;
  return po / (double)st->orb_size[o];
}

/* ------------------------------------------------------------------------- */
/* eps_l = phi_l + sum_{m != l} (n_m - nu) / r_lm, summed over m = 0..N-1 in order
 * (definition of the single-particle energies after Eq. 2).                     */
static double site_eps(const or_state* st, int32_t l) {
  const int32_t L = st->p.L;
  int32_t xl = l % L, yl = l / L;
  double acc = st->phi[l];
  /* m = ym L + xm runs over 0..N-1 in index order */
  for (int32_t ym = 0; ym < L; ++ym) {
    const double* row = st->invr + (size_t)wrap(yl - ym, L) * (size_t)L;
    for (int32_t xm = 0; xm < L; ++xm) {
      int32_t m = ym * L + xm;
      if (m == l) continue;
      int32_t ddx = xl - xm;
      if (ddx < 0) ddx += L;
      double q = (double)st->n[m] - st->nu;
      acc = acc + q * row[ddx];
    }
  }
  return acc;
}

static void eps_from_occ(const or_state* st, double* out) {
  for (int32_t l = 0; l < st->N; ++l) out[l] = site_eps(st, l);
}

void or_recompute_eps(const or_state* st, double* out) { eps_from_occ(st, out); }

double or_site_eps(const or_state* st, int32_t l) {
  if (l < 0 || l >= st->N) return 0.0 / 0.0;
  return site_eps(st, l);
}

/* Field-free part of Eq. 1: sum_i phi_i n_i + 1/2 sum_{i != j} (n_i-nu)(n_j-nu)/r_ij. */
double or_energy(const or_state* st) {
  const int32_t L = st->p.L, N = st->N;
  double h1 = 0.0, h2 = 0.0;
  for (int32_t i = 0; i < N; ++i) h1 = h1 + st->phi[i] * (double)st->n[i];
  for (int32_t i = 0; i < N; ++i) {
    double qi = (double)st->n[i] - st->nu;
    int32_t xi = i % L, yi = i / L;
    /* j = yj L + xj runs over 0..N-1 in index order */
    for (int32_t yj = 0; yj < L; ++yj) {
      const double* row = st->invr + (size_t)wrap(yi - yj, L) * (size_t)L;
      for (int32_t xj = 0; xj < L; ++xj) {
        int32_t j = yj * L + xj;
        if (j == i) continue;
        int32_t ddx = xi - xj;
        if (ddx < 0) ddx += L;
        double qj = (double)st->n[j] - st->nu;
        h2 = h2 + qi * qj * row[ddx];
      }
    }
  }
  return h1 + 0.5 * h2;
}

/* ------------------------------------------------------------------------- */
/* Random initial configuration: the n_e sites with the smallest 64-bit Philox
 * keys (ties by index) are occupied, i.e. a uniform n_e-subset; phi_i uniform in
 * [-W, W] (Eq. 1 and the random-start runs of section "Results").              */
typedef struct { uint64_t key; int32_t i; } site_key;

static int cmp_key(const void* x, const void* y) {
  const site_key* p = (const site_key*)x;
  const site_key* q = (const site_key*)y;
  if (p->key != q->key) return p->key < q->key ? -1 : 1;
  return p->i < q->i ? -1 : (p->i > q->i);
}

static int create(const or_params* p, or_state** out, int32_t lazy) {
  *out = NULL;
  if (p->L < 3 || p->L > 4096) return -1;
  int32_t N = p->L * p->L;
  if (p->n_e < 1 || p->n_e >= N) return -1;
  if (!(p->T > 0.0) || !(p->xi > 0.0) || !(p->W >= 0.0)) return -1;
  if (!(p->rc >= 1.0) || !(2.0 * p->rc < (double)p->L)) return -1;
  if (p->clock_mode < 0 || p->clock_mode > 2) return -1;
  if (!(p->pair >= 0.0) || !(p->pair < 1.0)) return -1;

  or_state* st = (or_state*)calloc(1, sizeof(or_state));
  if (!st) return -2;
  st->p = *p;
  st->N = N;
  st->lazy = lazy;
  st->nu = (double)p->n_e / (double)N;
  int rc = build_tower(st);
  if (rc == 0) {
    st->thr_pair = (uint64_t)floor(ldexp(p->pair, 32));
    st->Gamma_lab = st->Gamma / (1.0 - p->pair);
  }
  st->invr = (double*)malloc(sizeof(double) * (size_t)N);
  st->n = (uint8_t*)calloc((size_t)N, 1);
  st->phi = (double*)malloc(sizeof(double) * (size_t)N);
  st->eps = (double*)malloc(sizeof(double) * (size_t)N);
  site_key* keys = (site_key*)malloc(sizeof(site_key) * (size_t)N);
  if (rc != 0 || !st->invr || !st->n || !st->phi || !st->eps || !keys) {
    free(keys);
    or_destroy(st);
    return rc == -1 ? -1 : -2;
  }
  for (int32_t dy = 0; dy < p->L; ++dy)
    for (int32_t dx = 0; dx < p->L; ++dx) st->invr[dy * p->L + dx] = invr_def(p->L, dx, dy);

  for (int32_t i = 0; i < N; ++i) {
    uint32_t w[4];
    stream(st, (uint64_t)i, TAG_OCC, w);
    keys[i].key = ((uint64_t)w[0] << 32) | (uint64_t)w[1];
    keys[i].i = i;
  }
  qsort(keys, (size_t)N, sizeof(site_key), cmp_key);
  for (int32_t k = 0; k < p->n_e; ++k) st->n[keys[k].i] = 1;
  free(keys);

  for (int32_t i = 0; i < N; ++i) {
    uint32_t w[4];
    stream(st, (uint64_t)i, TAG_PHI, w);
    st->phi[i] = p->W * (2.0 * unit52(w[0], w[1]) - 1.0);
  }
  if (lazy) {
    for (int32_t i = 0; i < N; ++i) st->eps[i] = 0.0 / 0.0;
    st->H0 = 0.0 / 0.0;
  } else {
    eps_from_occ(st, st->eps);
    st->H0 = or_energy(st);
  }
  *out = st;
  return 0;
}

int or_create(const or_params* p, or_state** out) { return create(p, out, 0); }
int or_create_lazy(const or_params* p, or_state** out) { return create(p, out, 1); }

void or_destroy(or_state* st) {
  if (!st) return;
  free(st->orb_r2); free(st->orb_size); free(st->orb_first); free(st->thr); free(st->thr_u);
  free(st->vec_dx); free(st->vec_dy); free(st->invr);
  free(st->n); free(st->phi); free(st->eps);
  free(st);
}

void or_dims(const or_state* st, int32_t* N, int32_t* n_orb, int32_t* n_vec) {
  if (N) *N = st->N;
  if (n_orb) *n_orb = st->n_orb;
  if (n_vec) *n_vec = st->n_vec;
}

void or_tower(const or_state* st, uint64_t* thr, int32_t* orb_size, int32_t* orb_first,
              int32_t* vec_dx, int32_t* vec_dy, double* wsum, double* Gamma) {
  if (thr) memcpy(thr, st->thr, sizeof(uint64_t) * (size_t)st->n_orb);
  if (orb_size) memcpy(orb_size, st->orb_size, sizeof(int32_t) * (size_t)st->n_orb);
  if (orb_first) memcpy(orb_first, st->orb_first, sizeof(int32_t) * (size_t)st->n_orb);
  if (vec_dx) memcpy(vec_dx, st->vec_dx, sizeof(int32_t) * (size_t)st->n_vec);
  if (vec_dy) memcpy(vec_dy, st->vec_dy, sizeof(int32_t) * (size_t)st->n_vec);
  if (wsum) *wsum = st->wsum;
  if (Gamma) *Gamma = st->Gamma;
}

void or_get_occ(const or_state* st, uint8_t* out) { memcpy(out, st->n, (size_t)st->N); }
void or_get_phi(const or_state* st, double* out) { memcpy(out, st->phi, sizeof(double) * (size_t)st->N); }
void or_get_eps(const or_state* st, double* out) { memcpy(out, st->eps, sizeof(double) * (size_t)st->N); }

void or_get_scalars(const or_state* st, or_scalars* out) {
  out->s_last = st->s_last;
  out->s_scan = st->s_scan;
  out->hops = st->hops;
  out->P = st->P;
  out->t = st->t;
  out->H0 = st->H0;
  out->theta_pass = st->theta_pass;
  out->Gamma = st->Gamma;
  out->Gamma_lab = st->Gamma_lab;
}

int or_set_occ(or_state* st, const uint8_t* n) {
  int32_t c = 0;
  for (int32_t i = 0; i < st->N; ++i) {
    if (n[i] > 1) return -1;
    c += n[i];
  }
  if (c != st->p.n_e) return -1;
  memcpy(st->n, n, (size_t)st->N);
  if (!st->lazy) {
    eps_from_occ(st, st->eps);
    st->H0 = or_energy(st);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* dH_ij = eps_j - eps_i - 1/r_ij - E dx_ij (text after Eq. 2), evaluated in this
 * order: ((eps_j - eps_i) - 1/r) - E*dx.                                        */
static double delta_h(const or_state* st, int32_t i, int32_t j, int32_t v) {
  double vij = or_invr(st, st->vec_dx[v], st->vec_dy[v]);
  double dx = (double)st->vec_dx[v];
  return ((st->eps[j] - st->eps[i]) - vij) - st->p.E * dx;
}

static int32_t partner(const or_state* st, int32_t i, int32_t v) {
  const int32_t L = st->p.L;
  int32_t xj = wrap(i % L + st->vec_dx[v], L);
  int32_t yj = wrap(i / L + st->vec_dy[v], L);
  return yj * L + xj;
}

/* Acceptance of the mixed algorithm: Gamma^A_ij = theta_ij min(1, exp(-dH/T)),
 * theta_ij = n_i (1 - n_j) (Eq. 2 and the factorisation that follows it).      */
static double metropolis(const or_state* st, double dH) {
  if (dH <= 0.0) return 1.0;
  return exp(-dH / st->p.T);
}

double or_move(const or_state* st, int32_t i, int32_t v, double* dH) {
  int32_t j = partner(st, i, v);
  double d = delta_h(st, i, j, v);
  if (dH) *dH = d;
  if (!(st->n[i] == 1 && st->n[j] == 0)) return 0.0;
  double a = metropolis(st, d);
  return a > 1.0 ? 1.0 : a;
}

double or_acceptance(const or_state* st) {
  /* P(site i) = #{w0 : floor(w0 N / 2^32) = i} / 2^32, exactly */
  const uint64_t two32 = (uint64_t)1 << 32;
  const uint64_t N = (uint64_t)st->N;
  double acc = 0.0;
  for (int32_t i = 0; i < st->N; ++i) {
    uint64_t lo = ((uint64_t)i * two32 + N - 1) / N;
    uint64_t hi = ((uint64_t)(i + 1) * two32 + N - 1) / N;
    double pi = (double)(hi - lo) * 0x1p-32;
    double s = 0.0;
    for (int32_t v = 0; v < st->n_vec; ++v) s = s + or_vec_prob(st, v) * or_move(st, i, v, NULL);
    acc = acc + pi * s;
  }
  return acc;
}

/* ------------------------------------------------------------------------- */
/* Pair hops.  The paper considers single-electron hops only (Eq. 2) and names
 * multi-electron hops as an extension its code can take (sections "Code
 * performance" and "Conclusions") without giving their rates.  The reading
 * implemented here: a pair hop moves two electrons at once, i -> j and k -> l (four
 * distinct sites), with a rate of Eq. 2's form,
 *   Gamma_{ij,kl} = lambda theta_ij theta_kl exp(-2 (r_ij + r_kl) / xi) min(1, exp(-dH/T)),
 * restricted to compact pairs: the two starting sites and the two final sites are each
 * within the hop cutoff of one another (|k - i| <= rc and |l - j| <= rc, minimum image).
 * dH is the change of Eq. 1's H; moving i -> j and then k -> l with the energies updated
 * in between (step 3b) gives
 *   dH = dH_ij + dH_kl + 1/r_ik + 1/r_jl - 1/r_il - 1/r_jk.
 * The mixed algorithm's factorisation carries over: the tunnelling part is configuration
 * independent and is sampled without rejection, the rest is the acceptance.  A label is a
 * pair proposal with probability `pair` (else the single-hop proposal of or_draw):
 * i and d1 (j = i + d1) and u are the single hop's; the partner offset e (k = i + e) is
 * uniform over the hop vectors |e| <= rc, and d2 (l = k + d2) follows the tunnelling tower.
 * A move is proposed with the same probability as its reverse (j -> i, l -> k): e and -e,
 * d and -d share an orbit, and the labelling with k first has the same probability, so
 * Metropolis acceptance of the total dH keeps detailed balance with exp(-H/T).  Stream
 * PAIR at the label gives the words: w0 < pair 2^32 chooses a pair proposal, w1 picks the
 * orbit of e from the uniform thresholds and w3 & (size - 1) its member, w2 the orbit of
 * d2 from the tunnelling tower and (w3 >> 3) & (size - 1) its member.  Each single hop
 * keeps its rate Gamma^T_ij, so labels arrive at the rate Gamma / (1 - pair), and a given
 * pair move (proposed with probability 2 / (N n_vec) q(d1) q(d2) per pair label, q(d) =
 * exp(-2|d|/xi) / S, S = sum_d exp(-2|d|/xi), n_vec hop vectors) has
 * lambda = 2 pair / ((1 - pair) n_vec S).                                        */
void or_draw_label(const or_state* st, uint64_t s, int32_t* is_pair, int32_t* i, int32_t* v1,
                   int32_t* ve, int32_t* v2, double* u) {
  or_draw(st, s, i, v1, u);
  *is_pair = 0;
  *ve = -1;
  *v2 = -1;
  if (st->thr_pair == 0) return;
  uint32_t w[4];
  stream(st, s, TAG_PAIR, w);
  if (!((uint64_t)w[0] < st->thr_pair)) return;
  *is_pair = 1;
  int32_t o = 0;
  while (!((uint64_t)w[1] < st->thr_u[o])) ++o;
  *ve = st->orb_first[o] + (int32_t)(w[3] & (uint32_t)(st->orb_size[o] - 1));
  o = 0;
  while (!((uint64_t)w[2] < st->thr[o])) ++o;
  *v2 = st->orb_first[o] + (int32_t)((w[3] >> 3) & (uint32_t)(st->orb_size[o] - 1));
}

static int32_t shift(const or_state* st, int32_t i, int32_t v) {
  const int32_t L = st->p.L;
  return wrap(i / L + st->vec_dy[v], L) * L + wrap(i % L + st->vec_dx[v], L);
}

static double vsite(const or_state* st, int32_t a, int32_t b) {
  const int32_t L = st->p.L;
  return or_invr(st, a % L - b % L, a / L - b / L);
}

/* Sites of a pair proposal and whether the final sites are within the cutoff. */
static int pair_sites(const or_state* st, int32_t i, int32_t v1, int32_t ve, int32_t v2, int32_t* j,
                      int32_t* k, int32_t* l) {
  const int32_t L = st->p.L;
  *j = shift(st, i, v1);
  *k = shift(st, i, ve);
  *l = shift(st, *k, v2);
  int32_t dx = wrap(*l % L - *j % L, L), dy = wrap(*l / L - *j / L, L);
  if (L - dx < dx) dx = L - dx;
  if (L - dy < dy) dy = L - dy;
  return (double)(dx * dx + dy * dy) <= st->p.rc * st->p.rc;
}

/* Filters of a pair proposal: theta_ij theta_kl (i and k occupied, j and l empty), j != l
 * (the two electrons may not end on one site) and the final sites within the cutoff. */
static int pair_valid(const or_state* st, int32_t i, int32_t j, int32_t k, int32_t l, int near) {
  return st->n[i] == 1 && st->n[k] == 1 && st->n[j] == 0 && st->n[l] == 0 && j != l && near;
}

/* Field-free energy change of the pair move from the energies before it, in this order:
 * ((eps_j - eps_i) - 1/r_ij) + ((eps_l - eps_k) - 1/r_kl), plus
 * ((1/r_ik + 1/r_jl) - 1/r_il) - 1/r_jk.  The field term is -E (dx1 + dx2).     */
static double pair_dh0(const or_state* st, int32_t i, int32_t j, int32_t k, int32_t l, int32_t v1, int32_t v2) {
  const double* e = st->eps;
  double h1 = (e[j] - e[i]) - or_invr(st, st->vec_dx[v1], st->vec_dy[v1]);
  double h2 = (e[l] - e[k]) - or_invr(st, st->vec_dx[v2], st->vec_dy[v2]);
  double hi = ((vsite(st, i, k) + vsite(st, j, l)) - vsite(st, i, l)) - vsite(st, j, k);
  return (h1 + h2) + hi;
}

/* Acceptance probability of a pair proposal in the current configuration (0 when a site
 * coincides or the occupancy or final-separation filter fails); *dH receives the energy
 * change when the sites are valid. */
double or_move_pair(const or_state* st, int32_t i, int32_t v1, int32_t ve, int32_t v2, double* dH) {
  int32_t j, k, l;
  int near = pair_sites(st, i, v1, ve, v2, &j, &k, &l);
  if (dH) *dH = 0.0 / 0.0;
  if (!pair_valid(st, i, j, k, l, near)) return 0.0;
  double d = pair_dh0(st, i, j, k, l, v1, v2) - st->p.E * (double)(st->vec_dx[v1] + st->vec_dx[v2]);
  if (dH) *dH = d;
  double a = metropolis(st, d);
  return a > 1.0 ? 1.0 : a;
}

/* ------------------------------------------------------------------------- */
/* Step 3b: after hop i -> j, eps_l += 1/r_lj - 1/r_li for every l, with
 * 1/r(0) = 0 giving +1/r_ij at i and -1/r_ij at j.                             */
static void update_eps(or_state* st, int32_t i, int32_t j) {
  const int32_t L = st->p.L;
  const int32_t xi = i % L, yi = i / L, xj = j % L, yj = j / L;
  for (int32_t y = 0; y < L; ++y)
    for (int32_t x = 0; x < L; ++x) {
      int32_t l = y * L + x;
      double a = or_invr(st, x - xj, y - yj), b = or_invr(st, x - xi, y - yi);
      st->eps[l] = st->eps[l] + (a - b);
    }
}

/* Exact serial clock: the serial mixed algorithm adds an Exp(Gamma) waiting time
 * after every proposal, so the m proposals up to and including an executed hop add
 * a Gamma(m, Gamma) time (shape m, rate Gamma).  Sampled by Marsaglia and Tsang's
 * method for shape a >= 1 ("A simple method for generating gamma variables",
 * 2000): d = a - 1/3, c = 1/sqrt(9 d); draw a standard normal x and a uniform u;
 * with v = (1 + c x)^3 > 0 accept d v if u < 1 - 0.0331 x^4 or
 * ln u < x^2/2 + d (1 - v + ln v), else try again.  Attempt k of hop h (h counts the
 * executed hops, this one included) reads the
 * stream GAMMA | k << 8 at index h: x by Box-Muller from a 52-bit uniform and a
 * 32-bit angle, u from the fourth word.  After 64 rejected attempts (probability
 * below 1e-80) the mean m / Gamma is used.  Returns the increment.  */
double or_gamma_dt(uint64_t seed, uint32_t sample_id, uint64_t hop, uint64_t m, double Gamma) {
  const double d = (double)m - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
  for (uint32_t k = 0; k < 64; ++k) {
    uint32_t ctr[4] = {(uint32_t)hop, (uint32_t)(hop >> 32), sample_id, (uint32_t)TAG_GAMMA | (k << 8)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    or_philox(ctr, key, w);
    const double u1 = unit52(w[0], w[1]);
    const double u2 = ((double)w[2] + 0.5) * 0x1p-32;
    const double u = ((double)w[3] + 0.5) * 0x1p-32;
    const double x = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    double v = 1.0 + c * x;
    if (v <= 0.0) continue;
    v = v * v * v;
    const double x2 = x * x;
    if (u < 1.0 - 0.0331 * (x2 * x2)) return d * v / Gamma;
    if (log(u) < 0.5 * x2 + d * (1.0 - v + log(v))) return d * v / Gamma;
  }
  return (double)m / Gamma;
}

/* Clock: after each executed hop with m serial proposals since the previous
 * one, t advances by m/Gamma (deterministic increment used for the conductivity
 * figure), by a Gaussian of mean m/Gamma and deviation sqrt(m)/Gamma (step 3c),
 * clamped at zero, or by the exact Gamma(m, Gamma) time of the serial algorithm.
 * The Gaussian uses Box-Muller on stream CLOCK, index = hop.  */
static void advance_clock(or_state* st, uint64_t m) {
  const double G = st->Gamma_lab;
  if (st->p.clock_mode == 0) {
    st->t = (double)st->s_last / G;
    return;
  }
  if (st->p.clock_mode == 2) {
    st->t = st->t + or_gamma_dt(st->p.seed, st->p.sample_id, st->hops, m, G);
    return;
  }
  uint32_t w[4];
  stream(st, st->hops, TAG_CLOCK, w);
  double u1 = unit52(w[0], w[1]), u2 = unit52(w[2], w[3]);
  double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  double mean = (double)m / G;
  double sd = sqrt((double)m) / G;
  double dt = mean + sd * z;
  if (dt < 0.0) dt = 0.0;
  st->t = st->t + dt;
}

/* Naive serial KMC (section "Hopping conduction in the Coulomb glass"): a proposal
 * picks i and j != i uniformly among the N sites and is accepted with probability
 * tau_0 Gamma_ij = Gamma^T_ij Gamma^A_ij, Gamma^T_ij = exp(-2 r_ij / xi) for the hops
 * the mixed algorithm's tower holds (minimum-image r_ij^2 <= rc^2), 0 otherwise, and
 * Gamma^A_ij = theta_ij min(1, exp(-dH/T)); the clock is (proposals made) / (N (N - 1)),
 * i.e. +1 per N (N - 1) proposals.  Proposal k reads stream NAIVE at index k: i from
 * w0, j from w1 (uniform over the N - 1 other sites), the acceptance uniform from
 * w2, w3.  Runs until the clock reaches t_end and returns the hops executed.  */
int64_t or_naive_run(or_state* st, double t_end) {
  if (st->lazy) return -1;
  const int32_t L = st->p.L, N = st->N;
  const double pairs = (double)N * (double)(N - 1);
  int64_t done = 0;
  while ((double)st->naive_k / pairs < t_end) {
    uint32_t w[4];
    stream(st, st->naive_k, TAG_NAIVE, w);
    st->naive_k++;
    const int32_t i = (int32_t)(((uint64_t)w[0] * (uint64_t)N) >> 32);
    int32_t j = (int32_t)(((uint64_t)w[1] * (uint64_t)(N - 1)) >> 32);
    if (j >= i) ++j;
    if (!(st->n[i] == 1 && st->n[j] == 0)) continue;
    int32_t dx = wrap(j % L - i % L, L), dy = wrap(j / L - i / L, L);
    if (dx >= L - dx) dx -= L;
    if (dy >= L - dy) dy -= L;
    if (!((double)(dx * dx + dy * dy) <= st->p.rc * st->p.rc)) continue;
    const double vij = or_invr(st, dx, dy);
    const double dH = ((st->eps[j] - st->eps[i]) - vij) - st->p.E * (double)dx;
    const double gA = dH <= 0.0 ? 1.0 : exp(-dH / st->p.T);
    const double gT = exp(-2.0 * sqrt((double)(dx * dx + dy * dy)) / st->p.xi);
    if (!(unit52(w[2], w[3]) < gT * gA)) continue;
    st->n[i] = 0;
    st->n[j] = 1;
    st->P += dx;
    st->H0 = st->H0 + ((st->eps[j] - st->eps[i]) - vij);
    st->hops++;
    update_eps(st, i, j);
    ++done;
  }
  st->t = (double)st->naive_k / pairs;
  return done;
}

int64_t or_run(or_state* st, int64_t n_hops, double t_end, int64_t max_labels,
               uint64_t* log_label, int32_t* log_i, int32_t* log_j, int64_t log_cap, int64_t* n_logged) {
  int64_t done = 0, scanned = 0, logged = 0;
  if (n_logged) *n_logged = 0;
  if (st->lazy) return -1; /* no energies to run with */
  for (;;) {
    if (n_hops > 0 && done >= n_hops) break;
    if (t_end >= 0.0 && st->t >= t_end) break;
    if (max_labels > 0 && scanned >= max_labels) break;
    /* step 1: propose (i, j) with probability Gamma^T_ij / Gamma */
    uint64_t s = st->s_scan + 1;
    st->s_scan = s;
    ++scanned;
    int32_t i, v, is_pair, ve, v2;
    double u;
    or_draw_label(st, s, &is_pair, &i, &v, &ve, &v2, &u);
    if (is_pair) {
      /* a pair proposal: filters, then Metropolis on the total dH */
      int32_t j, k, l;
      int near = pair_sites(st, i, v, ve, v2, &j, &k, &l);
      if (!pair_valid(st, i, j, k, l, near)) continue;
      st->theta_pass++;
      double dH0 = pair_dh0(st, i, j, k, l, v, v2);
      double dH = dH0 - st->p.E * (double)(st->vec_dx[v] + st->vec_dx[v2]);
      if (!(dH <= 0.0 || u < metropolis(st, dH))) continue;
      st->n[i] = 0;
      st->n[j] = 1;
      st->n[k] = 0;
      st->n[l] = 1;
      st->P += st->vec_dx[v] + st->vec_dx[v2];
      st->H0 = st->H0 + dH0;
      uint64_t m = s - st->s_last;
      st->s_last = s;
      st->hops++;
      for (int e = 0; e < 2; ++e) {
        if (log_label && logged < log_cap) {
          log_label[logged] = s;
          log_i[logged] = e ? k : i;
          log_j[logged] = e ? l : j;
          ++logged;
        }
      }
      update_eps(st, i, j);
      update_eps(st, k, l);
      advance_clock(st, m);
      ++done;
      continue;
    }
    int32_t j = partner(st, i, v);
    /* step 2: accept with theta_ij min(1, exp(-dH/T)) */
    if (!(st->n[i] == 1 && st->n[j] == 0)) continue;
    st->theta_pass++;
    double dH = delta_h(st, i, j, v);
    if (!(dH <= 0.0 || u < metropolis(st, dH))) continue;
    /* step 3: execute the hop, update dipole, energies and clock */
    double dH0 = (st->eps[j] - st->eps[i]) - or_invr(st, st->vec_dx[v], st->vec_dy[v]);
    st->n[i] = 0;
    st->n[j] = 1;
    st->P += st->vec_dx[v];
    st->H0 = st->H0 + dH0;
    uint64_t m = s - st->s_last;
    st->s_last = s;
    st->hops++;
    if (log_label && logged < log_cap) {
      log_label[logged] = s;
      log_i[logged] = i;
      log_j[logged] = j;
      ++logged;
    }
    update_eps(st, i, j);
    advance_clock(st, m);
    ++done;
  }
  if (n_logged) *n_logged = logged;
  return done;
}
