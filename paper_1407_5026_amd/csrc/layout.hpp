// layout.hpp -- data structures shared by the host side and the kernels of libcgkmc.
//
// The arena holds one SampleState per sample (counters, clock, energy totals, run targets)
// in a contiguous array, and per sample (each block 256-byte aligned):
//   eps   [N]    double | float2         local energies (FP64, or FP32 value + Kahan low part)
//   phi   [N]    double                  disorder (scratch for init keys before that)
//   occ   [NW]   u32                     occupation bits, site l -> word l>>5, bit l&31
//   tab64 [(H+1)^2] double               1/r by folded separation (|dy|, |dx|), H = L/2
//   tabk  [ntab] float | double          the hop kernel's 1/r table (full or triangular)
//   thr   [n_orb] u32                    cumulative orbit thresholds (last one unused)
//   orb   [n_orb] u32                    first member | (orbit size - 1) << 16
//   vec   [n_vec] i32                    member displacement (dx & 0xffff) | dy << 16
//   guide [1024] u8                      orbit at the start of each 2^22-wide bucket of w1
//   thr_u [n_orb] u32                    cumulative orbit sizes over the hop vectors (pair hops)
//   dft_tw [L] double2, dft_T [(H+1) L] double   twiddles and transformed 1/r for the refresh
//   vec8  [n_orb][8] int2, guide16 [1024] u16   proposal tables of the exact-geometry and
//                                        large-sample kernels; tdo64 [n_orb] double (large)
//   mirror [N] double                    large-sample kernel: energies read by the proposals
//   sel   OccSelect                      large-sample initial-occupation selection scratch
//   part  [2 * nblk] double              per-block partial sums (energy, drift)
//   log   [cap] u64 + 2 x [cap] i32      executed-hop log (label, from, to)
#pragma once

#include <stdint.h>

namespace cg {

constexpr int kGuideBits = 10;
constexpr int kGuideSize = 1 << kGuideBits;
// 16-bit guide of the exact-geometry, large-sample and label-parallel kernels: 4096 buckets,
// entry = orbit of the bucket's smallest word | 0x8000 when two or more thresholds lie inside
// Split mode (FP32 pairs, value words in LDS): each thread keeps its sites' low parts in
// its own 16-byte groups of four slots during a launch, group g of thread t at float index
// 4 (1024 g + t); at most 36 slots (9 groups) per thread
constexpr int kSplitGroups = 9;
constexpr size_t kSplitLoBytes = (size_t)kSplitGroups * 1024 * 16;
constexpr int kGuide16Bits = 12;
constexpr int kGuide16Size = 1 << kGuide16Bits;
constexpr int kMaxWaves = 16;       // 1024 threads of 64 lanes
constexpr int kMaxCols = 4;         // columns per lane in the row update: L <= 256
constexpr int kInitBlock = 256;     // threads per block of the init / refresh kernels

// kFull: (H+1)^2 table by (|dy|, |dx|); kTri: its triangle |dx| <= |dy|; kRaw: the exact-geometry
// FP32 kernel's table by raw row difference dy + L and folded column distance (see fx_pitch).
// kBig: the large-sample kernel (one sample on the whole GPU): the FP64 (|dy|, |dx|) table in
// global memory, no kernel table.
enum TableLayout : int32_t { kFull = 0, kTri = 1, kRaw = 2, kBig = 3, kCube = 4, kFx64 = 5 };

struct SampleState {
  uint64_t s_last;        // label of the last executed hop
  uint64_t s_scan;        // all labels <= s_scan decided
  uint64_t hops;          // executed hops
  uint64_t hop_target;    // stop when hops reaches this (per call)
  uint64_t call_scan0;    // s_scan at the start of the current call
  int64_t P;              // sum of executed dx
  double t;               // clock
  double H0;              // field-free energy
  double t_end;           // run-to-time target of the current call (< 0: none)
  uint64_t sum_p;         // sum of ceil(m / M)
  uint64_t rounds;        // evaluation rounds
  uint64_t evaluated;     // label evaluations
  uint64_t theta_pass;    // evaluations passing the occupancy filter
  uint64_t refreshes;     // FP64 refreshes done
  double max_drift;       // max over refreshes of max |eps32 - eps64|
  double last_drift;
  int64_t logged;         // hop-log entries written (capped at the capacity)
  int32_t status;         // 0 ok, CG_ESTALL
  int32_t since_refresh;  // hops since last refresh
  int32_t force_refresh;  // refresh kernel: refresh regardless of since_refresh
  uint32_t grid_bar;      // unused (kept for the checkpoint layout; the barrier words are DevSample::bar)
  uint64_t phase_cycles[4];  // shader cycles: refill, evaluate, execute, update (if timed)
};

struct DevSample {
  int32_t L, N, H, n_e;
  int32_t NW, n_orb, n_vec, ntab;   // ntab: entries of the hop kernel's table
  int32_t nblk, log_cap, layout, dft;  // dft: refresh by Fourier transform along x
  int32_t dft_kc, dft_rows;   // frequencies per LDS chunk, outputs per thread
  int32_t log2M, pad2_;       // the sample's PR width M = 2^log2M (iterations p = ceil(m / M))
  uint32_t seed_lo, seed_hi, sample_id, magic_L;  // magic_L = ceil(2^32 / L)
  double nu, W, T, E, Gamma;
  double mrT;  // -1/T: the FP64 kernels form the thermal factor exp(-dH/T) as exp(dH mrT)
  float T32, E32, invT32, mTln2_32;  // mTln2_32 = -T ln 2 (acceptance thresholds)
  SampleState* st;
  void* eps;
  double* phi;
  uint32_t* occ;
  const double* tab64;
  const void* tabk;
  const uint32_t* thr;
  const uint32_t* orb;
  const int32_t* vec;
  const uint8_t* guide;
  const int32_t* vec8;    // kRaw: [n_orb][8] (dx & 0xffff | dy << 16, bits of FP32 1/|d|)
  const uint16_t* guide16;  // orbit at each bucket start | 0x8000 if two or more thresholds lie inside
  const double* tdo64;    // large-sample kernel: FP64 1/|d| per orbit
  double* mirror;         // large-sample kernel: global copy of the energies for the proposals;
                          // FP32 batches above L = 128: the low parts (float) during a launch,
                          // in each thread's own 16-byte groups (kSplitGroups)
  double* mirror2;        // large-sample kernel: the second copy (odd hops of a launch)
  uint32_t* occ2;         // large-sample kernel: second copy of the occupation words
  uint32_t* bar;          // large-sample kernel: grid-barrier words, one per 128-byte line
  double* part;
  const double* dft_tw;   // [L] (cos, sin)(2 pi j / L)
  const double* dft_T;    // [(H+1) x L] sum_dx T(dx, dy) cos(2 pi k dx / L), row k
  uint64_t* log_label;
  int32_t* log_from;
  int32_t* log_to;
  // pair hops: cumulative orbit sizes (uniform law over the hop vectors, last one unused),
  // the pair-choice threshold floor(pair 2^32) (0: single hops only) and floor(rc^2)
  const uint32_t* thr_u;
  uint32_t thr_pair;
  int32_t pair_r2;
};

// Knobs of one hop-kernel launch (uniform over the batch).
struct RunArgs {
  int32_t K;            // FP32 form: stop a sample when since_refresh reaches K (0: never)
  int32_t time_mode;    // 1: stop after the hop that brings t >= t_end
  int32_t clock_mode;   // 0: t = s_last / Gamma ; 1: Gaussian increments ; 2: Gamma(m) increments
  int32_t timers;       // 1: accumulate per-phase shader cycles
  uint64_t max_labels;  // per-call label cap (stall guard)
};

__host__ __device__ inline int32_t align16(int32_t b) { return (b + 15) & ~15; }

// Dynamic LDS layout of the hop kernel (byte offsets); identical on host and device.
struct HopLds {
  int32_t eps, occ, tab, vec, thr, orb, guide, ctrl, info, total;
};

constexpr int32_t kInfoBytes = 32;

__host__ __device__ inline HopLds hop_lds(int32_t N, int32_t NW, int32_t ntab, int32_t n_vec,
                                          int32_t n_orb, int32_t energy_bytes, int32_t real_bytes) {
  HopLds o;
  int32_t b = 0;
  o.eps = b;   b = align16(b + N * energy_bytes);
  o.occ = b;   b = align16(b + NW * 4);
  o.tab = b;   b = align16(b + ntab * real_bytes);
  o.vec = b;   b = align16(b + n_vec * 4);
  o.thr = b;   b = align16(b + n_orb * 4);
  o.orb = b;   b = align16(b + n_orb * 4);
  o.guide = b; b = align16(b + kGuideSize);
  o.ctrl = b;  b = align16(b + 96);
  o.info = b;  b = align16(b + 2 * kMaxWaves * kInfoBytes);
  o.total = b;
  return o;
}

// LDS of the pair-hop kernel: the generic kernel's FP64 layout and the uniform orbit
// thresholds of the partner offset.
struct PairLds {
  HopLds h;
  int32_t thr_u, total;
};

__host__ __device__ inline PairLds pair_lds(int32_t N, int32_t NW, int32_t ntab, int32_t n_vec, int32_t n_orb) {
  PairLds o;
  o.h = hop_lds(N, NW, ntab, n_vec, n_orb, 8, 8);
  o.thr_u = o.h.total;
  o.total = align16(o.thr_u + n_orb * 4);
  return o;
}

// Exact-geometry FP32 kernel (L = 64 or 128, NW waves of 64 lanes; every thread owns
// L*L/(64 NW) sites).  Its 1/r table holds row b in [0, 2L) for the raw row difference
// dy = b - L and column u for the folded column distance u <= L/2: entry
// 1/sqrt(fold(b - L)^2 + u^2), 0 at the origin and beyond u = L/2.  The row pitch is a
// multiple of 64 / NW floats so that a wave's rows, NW apart, are a multiple of 256 bytes
// apart (one two-row read each).
__host__ __device__ constexpr int32_t fx_pitch(int32_t L, int32_t NW = 16) {
  return ((L / 2 + 1) + 64 / NW - 1) / (64 / NW) * (64 / NW);
}
__host__ __device__ constexpr int32_t fx_tab_entries(int32_t L, int32_t NW = 16) { return 2 * L * fx_pitch(L, NW); }

struct FxLds {
  int32_t ev, occ, tab, thr, guide, ctrl, info, vec8, total;
};

// LDS of the exact-geometry kernel: energy values, occupation, table, thresholds, guide,
// control words, per-wave winner records, displacement table.
__host__ __device__ inline FxLds fx_lds(int32_t L, int32_t n_orb, int32_t NW = 16) {
  FxLds o;
  int32_t b = 0;
  o.ev = b;    b = align16(b + L * L * 4);
  o.occ = b;   b = align16(b + L * L / 8);
  o.tab = b;   b = align16(b + fx_tab_entries(L, NW) * 4);
  o.thr = b;   b = align16(b + n_orb * 4);
  o.guide = b; b = align16(b + kGuide16Size * 2);
  o.ctrl = b;  b = align16(b + 64);
  o.info = b;  b = align16(b + kMaxWaves * 16);
  o.vec8 = b;  b = align16(b + n_orb * 64);
  o.total = b;
  return o;
}

__host__ __device__ inline int32_t tri_entries(int32_t H) { return (H + 1) * (H + 2) / 2; }
__host__ __device__ inline int32_t full_entries(int32_t H) { return (H + 1) * (H + 1); }

}  // namespace cg
