/*
 * oracle.h -- serial FP64 reference for the mixed rejection kinetic Monte Carlo
 * of the two-dimensional lattice Coulomb glass (Ferrero, Kolton, Palassini,
 * "Parallel kinetic Monte Carlo simulation of Coulomb glasses").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain definition that the
 * GPU path is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product library never does.
 * It shares no source, header, table or constant generator with the GPU path.
 *
 * What it computes (section "Hopping conduction in the Coulomb glass"):
 *   H  = sum_i phi_i n_i + 1/2 sum_{i!=j} (n_i-nu)(n_j-nu)/r_ij - E sum_i n_i x_i   (Eq. 1)
 *   eps_i = phi_i + sum_{j!=i} (n_j-nu)/r_ij                        (single-particle energies)
 *   dH_ij = eps_j - eps_i - 1/r_ij - E dx_ij                        (energy change of hop i->j)
 *   rate  ~ theta_ij exp(-2 r_ij/xi) min(1, exp(-dH/T))             (Eq. 2)
 * simulated by the serial "mixed" algorithm: propose (i, j) with probability
 * proportional to exp(-2 r_ij / xi) (rejection-free, tower sampling), accept with
 * theta_ij min(1, exp(-dH/T)), and after an executed hop update every local energy
 * (step 3b of the mixed parallel-rejection algorithm).  The parallel-rejection form
 * is mathematically equivalent to this serial chain; with counter-based random
 * numbers indexed by the serial proposal label the equivalence is path by path,
 * so this serial loop is the exact reference for any number of parallel threads.
 *
 * Conventions (the paper leaves these open; the same readings are documented
 * with the GPU library):
 *   sites l = y*L + x on an L x L torus, minimum-image distances, 1/r(0) := 0;
 *   displacements d with 0 < |d|^2 <= rc^2, rc < L/2, grouped in square-symmetry
 *   orbits; Philox4x32-10 streams keyed by the seed, counter (lo, hi, sample, tag).
 */
#ifndef CG_ORACLE_H
#define CG_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_params {
  int32_t L;          /* lattice side; N = L*L */
  int32_t n_e;        /* electrons; filling nu = n_e / N */
  double W;           /* phi_i uniform in [-W, W] */
  double xi;          /* localization length */
  double rc;          /* hop cutoff (inclusive), must be < L/2 */
  double T;           /* temperature (> 0) */
  double E;           /* field strength along +x */
  uint64_t seed;      /* Philox key (lo, hi) */
  uint32_t sample_id; /* Philox counter word 2 */
  int32_t clock_mode; /* 0: dt = m/Gamma ; 1: Gaussian dt (mean m/Gamma, sd sqrt(m)/Gamma) ;
                         2: exact Gamma(m, Gamma) dt of the serial algorithm */
  double pair;        /* probability that a label proposes a pair hop, in [0, 1); 0 = the
                         paper's single-electron model (see or_draw_label) */
} or_params;

typedef struct or_scalars {
  uint64_t s_last;       /* label of the last executed hop (0 before the first) */
  uint64_t s_scan;       /* highest label examined so far */
  uint64_t hops;         /* executed hops */
  int64_t P;             /* dipole moment change: sum of executed dx */
  double t;              /* simulated clock */
  double H0;             /* field-free energy, updated by the executed dH */
  uint64_t theta_pass;   /* labels that passed the occupancy filter */
  double Gamma;          /* total proposal rate N * sum_d exp(-2|d|/xi) */
  double Gamma_lab;      /* label rate Gamma / (1 - pair): the clock's rate */
} or_scalars;

typedef struct or_state or_state;

/* Philox4x32-10 bijection: ctr[4], key[2] -> out[4]. */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Create and initialise a sample (random occupation, disorder, energies).
 * Returns 0 on success, -1 on invalid parameters, -2 on allocation failure. */
int or_create(const or_params* p, or_state** out);
/* The same without the O(N^2) energies and energy total (for lattices too large for
 * them): occupation, disorder and proposal law only.  or_run refuses such a state;
 * or_site_eps works on it. */
int or_create_lazy(const or_params* p, or_state** out);
/* eps_l of the current occupation in O(N): phi_l + sum_{m != l} (n_m - nu) / r_lm with m
 * summed in index order, the same arithmetic as the full recompute. */
double or_site_eps(const or_state* st, int32_t l);
void or_destroy(or_state* st);

/* Sizes of the proposal law. */
void or_dims(const or_state* st, int32_t* N, int32_t* n_orb, int32_t* n_vec);
/* Proposal law: cumulative orbit thresholds (thr[n_orb], last = 2^32), orbit sizes and
 * first member index, member displacements, sum of weights and Gamma. Any pointer may be NULL. */
void or_tower(const or_state* st, uint64_t* thr, int32_t* orb_size, int32_t* orb_first,
              int32_t* vec_dx, int32_t* vec_dy, double* wsum, double* Gamma);
/* Proposal drawn for serial label s (>= 1): site i, displacement index v, uniform u. */
void or_draw(const or_state* st, uint64_t s, int32_t* i, int32_t* v, double* u);
/* Probability that a proposal uses displacement index v. */
double or_vec_prob(const or_state* st, int32_t v);
/* 1/r for a lattice separation under the minimum image convention (0 for r = 0). */
double or_invr(const or_state* st, int32_t ddx, int32_t ddy);

void or_get_occ(const or_state* st, uint8_t* out);
void or_get_phi(const or_state* st, double* out);
void or_get_eps(const or_state* st, double* out);
void or_get_scalars(const or_state* st, or_scalars* out);

/* Replace the occupation (exactly n_e ones) and recompute eps and H0 from it (a lazy state
 * only takes the occupation).
 * Clock, dipole and labels are left unchanged.  Returns 0 or -1. */
int or_set_occ(or_state* st, const uint8_t* n);

/* Run the serial chain (not on a lazy state: returns -1) until n_hops more hops have executed, or (t_end >= 0)
 * until the first hop that brings the clock to t >= t_end, or until max_labels
 * more labels were examined (max_labels <= 0: no cap).  Executed hops are
 * logged (label, i, j) while log_cap allows (a pair hop logs two entries with its label,
 * i -> j then k -> l); logs may be NULL, n_logged (may be NULL) receives the entries
 * written.  Returns the number of hops (single or pair) executed in this call. */
int64_t or_run(or_state* st, int64_t n_hops, double t_end, int64_t max_labels,
               uint64_t* log_label, int32_t* log_i, int32_t* log_j, int64_t log_cap, int64_t* n_logged);

/* Label s of the model with pair hops: the single-hop draw of or_draw (i, v1, u) and,
 * when stream PAIR makes it a pair proposal (*is_pair = 1), the partner offset vector ve
 * (k = i + vec[ve]) and the second hop vector v2 (l = k + vec[v2]); else ve = v2 = -1. */
void or_draw_label(const or_state* st, uint64_t s, int32_t* is_pair, int32_t* i, int32_t* v1,
                   int32_t* ve, int32_t* v2, double* u);
/* Acceptance probability of the pair proposal (i, v1, ve, v2) in the current configuration:
 * theta_ij theta_kl min(1, exp(-dH/T)), 0 when j == l or the final sites are farther apart
 * than rc; *dH (may be NULL) receives dH when the sites are valid, else NaN. */
double or_move_pair(const or_state* st, int32_t i, int32_t v1, int32_t ve, int32_t v2, double* dH);

/* Naive serial KMC on the current configuration (uniform pair proposals, acceptance
 * exp(-2 r/xi) theta min(1, exp(-dH/T)) within the cutoff, clock +1 per N (N - 1)
 * proposals, its own proposal counter and stream), until the clock reaches t_end.  For the
 * equivalence check against the mixed algorithm; not on a lazy state (-1).  Returns the
 * hops executed. */
int64_t or_naive_run(or_state* st, double t_end);

/* O(N^2) recomputation of the local energies from the current occupation. */
void or_recompute_eps(const or_state* st, double* out);
/* Field-free energy of the current occupation from Eq. 1, O(N^2). */
double or_energy(const or_state* st);
/* dH of hop (i, v) in the current configuration and its acceptance probability
 * theta * min(1, exp(-dH/T)); returns the probability. */
double or_move(const or_state* st, int32_t i, int32_t v, double* dH);
/* Exact acceptance probability of one proposal in the current configuration. */
double or_acceptance(const or_state* st);

/* Exact serial clock increment of hop `hop` after m proposals: a Gamma(m, Gamma) draw
 * (Marsaglia-Tsang) from the GAMMA stream of (seed, sample_id). */
double or_gamma_dt(uint64_t seed, uint32_t sample_id, uint64_t hop, uint64_t m, double Gamma);

/* ---- simple cubic lattice (oracle3d.c): L^3 sites, the same parameters (clock_mode 0
 * only), hop vectors in orbits of the cube's 48 symmetries, member mulhi(w3, size),
 * acceptance uniform (w2 + 1/2) 2^-32. ---- */
typedef struct or3_state or3_state;
int or3_create(const or_params* p, or3_state** out);
void or3_destroy(or3_state* st);
void or3_draw(const or3_state* st, uint64_t s, int32_t* i, int32_t* v, double* u);
double or3_invr(const or3_state* st, int32_t dx, int32_t dy, int32_t dz);
int64_t or3_run(or3_state* st, int64_t n_hops, uint64_t* log_label, int32_t* log_i, int32_t* log_j,
                int64_t log_cap);
double or3_energy(const or3_state* st);
void or3_get(const or3_state* st, uint8_t* n, double* eps, double* phi);
void or3_scalars(const or3_state* st, or_scalars* out);
void or3_tower(const or3_state* st, int32_t* n_orb, int32_t* n_vec, uint64_t* thr, int32_t* first,
               int32_t* size, int32_t* vx, int32_t* vy, int32_t* vz);
void or3_set_occ(or3_state* st, const uint8_t* n);

#ifdef __cplusplus
}
#endif
#endif
