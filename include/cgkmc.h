/*
 * cgkmc.h -- C ABI of the MI355X parallel-rejection kinetic Monte Carlo library for
 * electron hopping in the two-dimensional lattice Coulomb glass.
 *
 * Model (Ferrero, Kolton, Palassini, section "Hopping conduction in the Coulomb
 * glass", Eq. 1 and Eq. 2): N = L*L sites on a torus, occupations n_i in {0,1} with
 * n_electrons = nu*N electrons, random site energies phi_i uniform in [-W, W],
 * Coulomb 1/r under the minimum-image convention, field E along +x.  Hops i -> j are
 * proposed with probability proportional to exp(-2 r_ij / xi) for |d| <= rc (tower
 * sampling), accepted with theta_ij min(1, exp(-dH/T)) where
 * dH = eps_j - eps_i - 1/r_ij - E dx, and the lowest-labelled accepted proposal of a
 * parallel iteration is executed (section "Parallel rejection algorithm", steps 1-3,
 * and the mixed parallel-rejection algorithm, steps 1, 2, 3a-3c).  After a hop every
 * local energy is updated (step 3b).
 *
 * Random numbers: Philox4x32-10 keyed by the sample's seed; proposal label s (1-based,
 * counted from the creation of the sample) uses counter (s_lo, s_hi, sample_id, 0).
 * Labels beyond the executed one in a parallel iteration are re-used against the new
 * configuration, so the executed hop sequence equals that of the serial mixed
 * algorithm for any parallel width M (the paper states the two are mathematically
 * equivalent; with label-indexed numbers the equivalence holds path by path).
 *
 * Memory and streams: every device buffer lives in one caller-owned arena (device
 * memory, size from cg_arena_bytes, alignment 256 bytes) that must outlive the
 * context; the library allocates no device memory.  All work is enqueued on the HIP
 * stream given at creation, in stream order.  Getters copy to caller-owned host
 * memory and synchronise that stream.  A context is not thread-safe.
 *
 * Errors: functions return CG_OK (0) or a negative code; cg_last_error() returns a
 * thread-local message describing the last failure.
 */
#ifndef CGKMC_H
#define CGKMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CG_OK 0
#define CG_EINVAL (-1)   /* invalid argument (rc >= L/2, T <= 0, bad index, ...)        */
#define CG_ENOSPC (-2)   /* arena too small, or a sample does not fit the kernel's LDS */
#define CG_EHIP (-3)     /* HIP runtime error, or a workgroup of the whole-GPU kernel missed a
                            grid barrier (bounded wait); message in cg_last_error()      */
#define CG_ESTALL (-4)   /* label cap reached before the requested hops; state is valid */

#define CG_FP64 0          /* proposals, acceptance and energy update in FP64            */
#define CG_FP32_REFRESH 1  /* FP32 proposals and update with each energy kept as an FP32 pair
                              (exact-geometry kernel: hi + lo renormalised by Fast2Sum every 16
                              hops; other kernels: Kahan-compensated sums), FP64 refresh every
                              K hops */

#define CG_CLOCK_DET 0    /* dt = m / Gamma (deterministic increment)                    */
#define CG_CLOCK_GAUSS 1  /* dt ~ Gaussian(m/Gamma, sqrt(m)/Gamma), clamped at 0 (step 3c) */
#define CG_CLOCK_GAMMA 2  /* dt ~ Gamma(m, Gamma): the serial mixed algorithm's m Exp(Gamma)
                             waiting times (section "Hopping conduction in the Coulomb
                             glass"), drawn by Marsaglia-Tsang from stream GAMMA            */

/* One independent sample (disorder realisation / temperature / size).
 * Requirements: 3 <= L <= 192, or L a power of two in [256, 2048]; 1 <= n_electrons < L*L;
 * W >= 0; xi > 0; 1 <= rc < L/2 (hops longer than L/2 are excluded, section "Results ...
 * two dimensions"); T > 0.  A batch with any L > 192 runs every sample, one after the other,
 * on the whole GPU (one cooperative launch per sample, FP64 form, every L a power of two in
 * [128, 2048], no use_graph). */
typedef struct cg_sample_desc {
  int32_t L;
  int32_t n_electrons;
  double W;
  double xi;
  double rc;
  double T;
  double E;
  uint64_t seed;
  uint32_t sample_id;
  int32_t dim;       /* lattice: 0 or 2 = square (L^2 sites), 3 = simple cubic (L^3 sites;
                        FP64 form, deterministic clock, 3 <= L <= 24, every sample of the
                        batch cubic); CG_EINVAL otherwise */
  double pair;       /* probability in [0, 1) that a label proposes a pair hop, two electrons
                        at once (the multi-electron extension named in sections "Code
                        performance" and "Conclusions"; rates read as Eq. 2's with the
                        Eq. 1 energy change of the joint move): i -> j as a single hop and
                        k -> l with k = i + e, e uniform over the hop vectors, l = k + d2
                        from the tunnelling tower, both pairs within rc.  0 = the paper's
                        single-electron model.  pair > 0 in any sample runs the batch on the
                        pair-hop kernel: square lattices, L <= 128, FP64 form, variant 0 or
                        1; labels arrive at Gamma / (1 - pair), the clock's rate; a pair
                        hop logs two entries (i -> j, k -> l) with its label */
  int32_t M;         /* parallel width of this sample's PR iterations (section "Parallel
                        rejection algorithm": a hop found after m serial proposals takes
                        p = ceil(m / M) iterations, reported in cg_stats.sum_p); a power of two
                        in [1, 2^24], or 0 for cg_run_opts.M.  The executed hops do not depend on
                        it: labels past the executed one are re-used */
} cg_sample_desc;

typedef struct cg_run_opts {
  int32_t precision;   /* CG_FP64 or CG_FP32_REFRESH                                    */
  int32_t M;           /* parallel width of one PR iteration (power of two; 0 = 1024): the
                          iteration count p = ceil(m / M) is reported per hop; the kernel
                          evaluates labels in chunks of 1024 (M <= 1024) or 2048 and the
                          executed hops do not depend on M                               */
  int32_t block;       /* threads per workgroup: 1024 (0 = 1024); 512 selects the
                          exact-geometry kernel's 8-wave form (same hops and energies
                          bit for bit, 13% fewer hops/s at L = 128); CG_EINVAL otherwise */
  int32_t K_refresh;   /* FP32 form: hops between FP64 refreshes (>= 1); 0 = 4096       */
  int32_t clock_mode;  /* CG_CLOCK_DET, CG_CLOCK_GAUSS or CG_CLOCK_GAMMA                 */
  int32_t log_hops;    /* per-sample capacity of the executed-hop log (0 = no log)       */
  int32_t phase_timers;/* 1: accumulate per-phase shader cycles into cg_stats            */
  int32_t use_graph;   /* 1: cg_run_hops captures its launch sequence once per (n_hops,
                          refresh phase) as a hipGraph and replays it; needs a stream
                          other than the legacy default stream                          */
  int32_t variant;     /* hop kernel: 0 = automatic (3 or 5 where they apply, else 1);
                          1 = two workgroup barriers per hop, any L;
                          2 = one barrier per hop (FP32 form, L <= 128: double-buffered
                          energies, the next round corrects for the hop in flight);
                          3 = exact-geometry FP32 kernel (every sample L = 64, or every
                          sample L = 128): table by raw row difference, energies as
                          hi + lo pairs renormalised every 16 hops, precomputed
                          acceptance thresholds;
                          4 = whole-GPU kernel (FP64, L a power of two >= 128): each
                          sample on every CU, automatic for L > 192;
                          5 = exact-geometry FP64 kernel (every sample L = 64, or every
                          sample L = 128; deterministic clock; chunks of 1024 labels for
                          any M): energies in registers, value words in LDS, triangle-
                          ordered FP64 table; the same hops as 1;
                          6 = label-parallel kernel (FP64; square lattices with L a power of
                          two in [16, 128], or cubic lattices, deterministic clock):
                          one sample at a time on `spread` workgroups, each holding a
                          replica of the sample and evaluating its own 1024 U labels of a
                          round of spread x 1024 U labels; the round's lowest accepted label
                          is a global minimum behind one grid barrier (the paper's setting:
                          one sample, a parallel width of the order of 1/A).  The same hops
                          as 1 for any spread                                            */
  int32_t spread;      /* variant 6: workgroups per sample (0 = one per CU; at most the
                          number that can be co-resident, else CG_ENOSPC).  Whole-GPU
                          kernel (variant 4 or L > 192): 0 = the size's grid, or that grid's
                          workgroup count, or 16 at L = 256 (four sites per thread);
                          CG_EINVAL for other counts.  0 for every other kernel         */
  uint64_t max_labels_per_call; /* stall guard per sample and call; 0 = 2^32            */
} cg_run_opts;

/* Per-sample counters and observables. */
typedef struct cg_stats {
  uint64_t hops;        /* executed hops since creation                                 */
  uint64_t s_last;      /* label of the last executed hop (0 before the first)          */
  uint64_t s_scan;      /* every label <= s_scan has been decided                       */
  int64_t P;            /* dipole moment change: sum of executed dx                     */
  double t;             /* simulated clock (units of tau_0)                             */
  double H0;            /* field-free energy of Eq. 1 (FP64 total)                      */
  uint64_t sum_p;       /* sum over hops of the parallel iterations p = ceil(m / M)     */
  uint64_t rounds;      /* barrier-separated evaluation rounds executed by the kernel   */
  uint64_t evaluated;   /* label evaluations, re-evaluations after a hop included       */
  uint64_t theta_pass;  /* evaluations that passed the occupancy filter                 */
  uint64_t refreshes;   /* FP64 refreshes done (FP32 form)                              */
  double max_drift;     /* max over refreshes of max_l |eps32_l - eps64_l|              */
  double last_drift;    /* the same for the most recent refresh                         */
  int32_t status;       /* CG_OK, or CG_ESTALL if the label cap stopped this sample     */
  int32_t since_refresh;/* hops since the last refresh (FP32 form)                      */
  int64_t logged;       /* entries written to the hop log                              */
  uint64_t phase_cycles[4]; /* with phase_timers, shader cycles of workgroup wave 0 in:
                               [0] label drawing, [1] evaluation up to the round barrier,
                               [2] (exact-geometry kernel) the round barrier and hop
                               execution, else evaluation's barrier is in [1] and [2] is
                               hop execution, [3] the energy update and its barrier      */
} cg_stats;

typedef struct cg_ctx cg_ctx;

/* Device bytes needed for n samples under the given options (alignment 256): per sample the
 * state of the chain the paper's algorithm carries (occupations and local energies of Eq. 1
 * and the text after Eq. 2, the dipole, the clock), the proposal tables of the mixed
 * algorithm's tower sampling (section "Hopping conduction in the Coulomb glass") and the
 * refresh tables.  Host-only: validates the samples and options like cg_create (CG_EINVAL,
 * CG_ENOSPC) and writes *bytes. */
int cg_arena_bytes(const cg_sample_desc* samples, int32_t n, const cg_run_opts* opts,
                   size_t* bytes);

/* Set up a batch of independent samples of Eq. 1 (section "Hopping conduction in the Coulomb
 * glass"; the runs of section "Results for the lattice model in two dimensions" start from a
 * random configuration): build the proposal tables (Gamma^T_ij = exp(-2 r_ij / xi) over the
 * hop vectors |d| <= rc, tower thresholds, Gamma = N sum_d exp(-2|d|/xi)), draw the random
 * initial occupation (a uniform n_electrons-subset) and the disorder phi_i uniform in [-W, W],
 * and compute the initial single-particle energies (definition after Eq. 2)
 *   eps_l = phi_l + sum_{m != l} (n_m - nu) / r_lm
 * in FP64 with m summed in index order, all on the GPU.  `samples` (n >= 1 host structs) and
 * `opts` are read during the call only.  `arena` is caller-owned device memory of at least
 * cg_arena_bytes (256-byte aligned) that must outlive the context; `hip_stream` is a
 * hipStream_t (NULL = default stream) on which all later work is enqueued.  Returns CG_OK and
 * *out; or CG_EINVAL (invalid sample or option), CG_ENOSPC (arena too small, or a sample
 * does not fit the chosen kernel), CG_EHIP (HIP error); then no context is created. */
int cg_create(cg_ctx** out, const cg_sample_desc* samples, int32_t n, const cg_run_opts* opts,
              void* arena, size_t arena_bytes, void* hip_stream);
/* Release the context's host objects (graphs, events); the arena stays the caller's.
 * Synchronises the context stream.  NULL is accepted. */
int cg_destroy(cg_ctx* ctx);

/* The mixed parallel-rejection algorithm (section "Hopping conduction in the Coulomb glass",
 * steps 1, 2 and 3a-3c, with the generic scheme of section "Parallel rejection algorithm"):
 * every sample executes exactly n_hops more hops (n_hops >= 1).  Per parallel iteration the
 * labels s_last + 1 ... are proposed (step 1), filtered by theta_ij and accepted with
 * min(1, exp(-dH/T)) (step 2); the lowest accepted label is executed, the dipole and every
 * local energy updated (steps 3a, 3b) and the clock advanced (step 3c).  In the FP32 form an
 * FP64 refresh of the energies ends every K_refresh hops.  Enqueued on the context stream
 * (asynchronous).  Returns CG_OK, CG_EINVAL (n_hops < 1, null context), CG_EHIP, or
 * CG_ESTALL if a sample reached max_labels_per_call first (its state stays consistent; call
 * again to continue). */
int cg_run_hops(cg_ctx* ctx, int64_t n_hops);
/* As cg_run_hops, but every sample runs until the first hop that brings its clock (step 3c;
 * the deterministic, Gaussian or Gamma increment of clock_mode) to t >= t_end; samples
 * already there execute nothing.  Synchronises the context stream (the stopping test reads
 * the samples' state).  Returns CG_OK, CG_EINVAL (t_end not finite), CG_EHIP or CG_ESTALL as
 * above (t_end must be finite and >= 0). */
int cg_run_time(cg_ctx* ctx, double t_end);
/* FP32 form: recompute every sample's energies now from their definition after Eq. 2 in FP64
 * (the refresh that otherwise ends each K_refresh interval) and record the drift
 * max_l |eps32_l - eps64_l|; in the FP64 form the exact recompute replaces the incrementally
 * updated energies.  Synchronises the context stream.  CG_OK, CG_EINVAL (null context) or
 * CG_EHIP. */
int cg_refresh(cg_ctx* ctx);

/* Set the temperature T (> 0) and the field E of one sample: the T of Eq. 2's thermal factor
 * and the E of Eq. 1's field term (-E sum_i n_i x_i, so dH contains -E dx).  Takes effect at
 * the next run call; the configuration and clock are kept.  Synchronises the context stream.
 * CG_EINVAL for a bad index, T <= 0 or non-finite values. */
int cg_set_TE(cg_ctx* ctx, int32_t sample, double T, double E);

/* Host copies of one sample's state, into caller-owned host memory; each synchronises the
 * context stream and returns CG_EINVAL for a bad sample index or a null pointer.
 *   cg_get_occupation: the occupation numbers n_i of Eq. 1 (N bytes, 0 or 1, site
 *     i = y L + x, or (z L + y) L + x on the cubic lattice);
 *   cg_get_local_energies: the single-particle energies eps_i (definition after Eq. 2) as N
 *     doubles; the FP32 form returns its FP32 pair's sum;
 *   cg_get_phi: the random site energies phi_i of Eq. 1 (N doubles);
 *   cg_get_stats: the counters of the parallel-rejection run (section "Parallel rejection
 *     algorithm": iterations p per hop summed, labels evaluated) and the observables (dipole
 *     change P, clock, Eq. 1 field-free energy, refresh drift). */
int cg_get_occupation(cg_ctx* ctx, int32_t sample, uint8_t* host_out);
int cg_get_local_energies(cg_ctx* ctx, int32_t sample, double* host_out);
int cg_get_phi(cg_ctx* ctx, int32_t sample, double* host_out);
int cg_get_stats(cg_ctx* ctx, int32_t sample, cg_stats* out);
/* Simulated clock of one sample (units of the attempt time): the deterministic form
 * t = s_last / Gamma, or the sum of the drawn increments (section "Hopping conduction in the
 * Coulomb glass", step 3c).  Synchronizes the context stream; CG_EINVAL for a bad sample
 * index or a null pointer. */
int cg_get_clock(cg_ctx* ctx, int32_t sample, double* t);
/* Clock and current of one sample: t, the dipole change P = sum of executed dx (step 3b) and
 * the conductivity sigma = P / (N E t), the average of Eq. 3's sigma(t) = (1/(N E)) dP/dt
 * over [0, t] (0 if E t == 0).  Synchronises the context stream; CG_EINVAL for a bad index
 * or a null pointer. */
int cg_get_current(cg_ctx* ctx, int32_t sample, double* t, int64_t* P, double* sigma);
/* Executed-hop log of one sample (step 3a's executed hops i_q -> j_q with their labels q):
 * labels, origin and destination sites into caller-owned host arrays of `cap` entries each;
 * *count receives the number copied (at most the log_hops capacity, first hops first).
 * Synchronises the context stream; CG_EINVAL for a bad index, cap < 0 or null pointers. */
int cg_get_hop_log(cg_ctx* ctx, int32_t sample, uint64_t* labels, int32_t* from, int32_t* to,
                   int64_t cap, int64_t* count);

/* Single-particle density of states (section "Results": the normalized histogram
 * g(eps, T) = sum_k delta_{d eps}(eps - eps_k) of the local energies of Eq. 2) of samples
 * first .. first + count - 1, in their current configurations: every site's energy (FP64,
 * or the FP32 pair's FP64 sum) goes to bin floor((eps - e_lo) * nbins / (e_hi - e_lo))
 * computed in FP64 (nbins / (e_hi - e_lo) evaluated first).  host_occupied[nbins] and
 * host_empty[nbins] receive the counts of occupied and empty sites per bin,
 * host_outside[2] the sites below e_lo and at or above e_hi.  Dividing by the number of
 * sites and the bin width (e_hi - e_lo) / nbins normalizes.  1 <= nbins <= 4096,
 * e_lo < e_hi finite, 1 <= count <= 65535 (CG_EINVAL otherwise).  Synchronises the
 * context stream; the counts use a scratch region of the arena. */
int cg_dos(cg_ctx* ctx, int32_t first, int32_t count, double e_lo, double e_hi, int32_t nbins,
           uint64_t* host_occupied, uint64_t* host_empty, uint64_t* host_outside);
/* cg_dos for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same arguments, checks and counts,
 * but the bin counts live in a file-scope device array of 2 * 4096 + 2 slots (64 KiB + 16
 * bytes, one copy per device for the life of the process) rather than in the arena, and the
 * results are copied straight into the caller's host arrays.  It calls no hipMalloc, hipFree
 * or other allocating routine; the array's device address is resolved by cg_create on the
 * device current there.  nbins above 4096 is CG_EINVAL.  Every call on one device shares that
 * device's array and clears it first: calls that overlap on one device (two contexts or two
 * host threads) race.  Synchronises the context stream. */
int cg_dos_noalloc(cg_ctx* ctx, int32_t first, int32_t count, double e_lo, double e_hi, int32_t nbins,
                   uint64_t* host_occupied, uint64_t* host_empty, uint64_t* host_outside);

/* Checkpoint of one sample (the state the paper's algorithm carries from hop to hop: the
 * occupation of Eq. 1, the local energies of Eq. 2, the clock, the next label and the
 * counters; section "Hopping conduction in the Coulomb glass", steps 1-3).
 * cg_save with host_blob == NULL stores the size in *bytes; otherwise *bytes is the buffer
 * size (CG_ENOSPC if too small) and receives the bytes written.  The blob is a header
 * (magic "CGKMCSV1", version 2, precision, the sample's L, n_e, W, xi, rc, seed, sample id,
 * pair probability and current T and E), the sample state, the occupation words and the energies (8 bytes
 * per site: FP64, or the FP32 pair).  cg_load checks the header against sample `sample`
 * of this context (same version, precision and sample parameters, exact size; CG_EINVAL
 * otherwise), restores the state, occupation, energies and T, E, and empties the sample's
 * hop log; the sample then continues exactly as the saved one would have (the labels are
 * counter-based).  The caller owns the blob; both calls synchronise the context stream. */
int cg_save(cg_ctx* ctx, int32_t sample, void* host_blob, size_t* bytes);
int cg_load(cg_ctx* ctx, int32_t sample, const void* host_blob, size_t bytes);

/* Device time of the hop kernel launches since the last call (ms) and launch count, and
 * the same for refreshes; resets them (the per-hop wall-clock cost the paper splits into
 * W_R and W_U in section "Code performance").  Timing uses HIP events on the context
 * stream; with use_graph, each replay is timed as a whole and added to the hop time.
 * Waits for the recorded events; null outputs are skipped. */
int cg_take_kernel_time(cg_ctx* ctx, double* hop_ms, int64_t* hop_launches, double* refresh_ms,
                        int64_t* refresh_launches);

/* Autotuner (section "Parallel rejection algorithm": the best parallel width is of the order
 * of min(1/A, C), the inverse acceptance or the parallel capacity).  Chooses opts->M, the
 * kernel's label chunk (1024 or 2048), by the hop-kernel time of trial runs of trial_hops
 * hops; in the FP32 form opts->K_refresh as the largest of 8192, 4096, 2048, 1024 whose drift
 * over 2K hops from the initial state stays below drift_target / 2 (else 1024); and, when
 * widths is not NULL, each sample's PR width widths[b] = min(1/A_b, 16384) rounded up to a
 * power of two and at least 512, with A_b = hops / serial proposals of that sample over the
 * second half of a trial run of 2 trial_hops hops from its initial state (copy it into the
 * samples' M).  Each trial creates and destroys a context on `arena` (at least
 * cg_arena_bytes for these samples and options), whose contents are overwritten; no context
 * is left behind.  Runs on hip_stream and synchronises it.  CG_EINVAL for trial_hops < 64 or
 * drift_target <= 0; errors of the trial contexts otherwise. */
int cg_autotune(const cg_sample_desc* samples, int32_t n, cg_run_opts* opts, void* arena,
                size_t arena_bytes, void* hip_stream, int64_t trial_hops, double drift_target,
                int32_t* widths);

/* Thread-local description of the last error (empty string if none). */
const char* cg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
