// hop_fx.hpp -- FP32 hop kernel for lattices that fill a workgroup of NW = 16 or 8 waves
// exactly (L = 64 or 128; wave w owns rows w + NW r, lane the columns lane + 64 c).
//
// It runs the same mixed parallel-rejection step as k_hops (section "Hopping conduction in
// the Coulomb glass", steps 1, 2, 3a-3c, with the labels of a chunk drawn once and re-used
// after a hop) and executes the same hops, with three changes in how the work is laid out:
//
//  * The 1/r table is indexed by the raw row difference b = dy + L in [1, 2L) and the folded
//    column distance.  In step 3b a lane's table address for its row y = w + NW r is then a
//    per-hop base plus NW r rows, a compile-time offset, so the row terms need neither
//    scalar nor vector arithmetic.
//  * A site's FP32 energy is a pair hi + lo.  Step 3b adds the FP32 increment
//    1/r_lj - 1/r_li to lo, the proposals read fl(hi + lo) from LDS, and every kRenorm hops
//    the pair is renormalised exactly (Fast2Sum) so that lo stays of the order of the recent
//    increments: its rounding errors stay far below those of a single FP32 running sum, at
//    three vector operations per site and hop.
//  * A site's occupation travels in the lowest bit of its energy value word: hi's lowest
//    mantissa bit is kept equal to n_l (the change is moved into lo, so hi + lo keeps its
//    value) and the value word fl(hi + lo) carries hi's lowest bit.  A proposal reads two
//    words, not four (random LDS reads cost ~16 cycles per wave instruction); the value it
//    compares is within one ulp of fl(hi + lo).
//  * Every label carries its LDS addresses and its acceptance threshold
//    th = 1/r_ij + E dx - T ln u, so the test of Eq. 2, dH <= 0 or u < exp(-dH/T) with
//    dH = eps_j - eps_i - 1/r_ij - E dx, is the single comparison eps_j - eps_i <= th
//    (the two forms agree up to FP32 rounding of th).
#pragma once

#include "kernels.hpp"

namespace cg {

// One cached label: sites, LDS byte addresses of their energy value words, displacement dx,
// acceptance threshold and 1/r_ij.
struct FxLabel {
  int32_t i, j, dx;
  uint32_t ai, aj;
  float th, td;
};

// Sets hi's lowest mantissa bit to the occupation n and moves the change (one ulp of hi, or
// zero) into lo: hi + lo keeps its value up to the rounding of that addition (2^-24 ulp).
__device__ __forceinline__ void set_mark(float& hi, float& lo, uint32_t n) {
  const float h2 = __uint_as_float((__float_as_uint(hi) & ~1u) | n);
  lo = lo + (hi - h2);
  hi = h2;
}

// The value word the proposals read: fl(hi + lo) with hi's lowest bit (the occupation).
__device__ __forceinline__ float marked(float hi, float lo) {
  return __uint_as_float((__float_as_uint(hi + lo) & ~1u) | (__float_as_uint(hi) & 1u));
}

struct FxShared {
  uint32_t theta;
  uint32_t pad_;
  double t;                // Gaussian clock
  unsigned long long nev;  // label evaluations of the launch (summed over lanes at its end)
};

template <int L, int NW>
struct FxGeo {
  static constexpr int LG = L == 64 ? 6 : 7;
  static constexpr int N = L * L;
  static constexpr int NT = 64 * NW;  // threads
  static constexpr int LW = NW == 16 ? 4 : 3;
  static constexpr int NC = L / 64;
  static constexpr int RPW = L / NW;
  static constexpr int P = fx_pitch(L, NW);
  static constexpr int SPL = RPW * NC;  // sites per lane
  static_assert(L == 64 || L == 128, "exact geometry: L = 64 or 128");
  static_assert(NW == 16 || NW == 8, "16 or 8 waves");
  static_assert(SPL % 4 == 0 && SPL <= 32, "whole 16-byte chunks, at most 32 sites per lane");
  // LDS word of site (x, y)'s energy value.  The owner is wave y % NW, lane x & 63, slot
  // s = (y / NW) NC + (x >> 6); each wave's 64 SPL words are laid out as [s / 4][lane][s % 4],
  // so the wave stores its values with SPL / 4 16-byte stores, each covering 1024
  // contiguous bytes (lane-consecutive: no bank conflicts)
  __device__ static int ev_slot(int x, int y) {
    const int s = (y >> LW) * NC + (x >> 6);
    return (y & (NW - 1)) * 64 * SPL + (s >> 2) * 256 + (x & 63) * 4 + (s & 3);
  }
};

// LDS accesses by 32-bit local address.  The dynamic LDS base is added once where an
// address is formed, so a load or store costs no address arithmetic of its own and a
// constant offset lands in the instruction's offset field.
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lds_addr_of(const uint8_t* p) {
  return (uint32_t)(uintptr_t)(lds_ptr<const uint8_t>)p;
}
template <typename T>
__device__ __forceinline__ T lds_ld(uint32_t a) {
  return *(lds_ptr<const T>)a;
}
template <typename T>
__device__ __forceinline__ void lds_st(uint32_t a, T v) {
  *(lds_ptr<T>)a = v;
}

// Orbit of a proposal (step 1's choice of the hop length) from its 32-bit word c1: the first
// orbit o with c1 < thr[o], the last orbit taking the rest.  g is the 16-bit guide entry of
// c1's bucket: the orbit of the bucket's smallest word, with 0x8000 set when two or more
// thresholds lie inside the bucket.  One comparison (no branch) settles every bucket holding
// at most one threshold; only the flagged buckets (the far orbits' thresholds crowd into the
// top buckets) continue the search in a loop.
__device__ __forceinline__ int orbit_guided(uint32_t g, uint32_t c1, uint32_t thr, int last) {
  int o = (int)(g & 0x7fffu);
  const uint32_t t = lds_ld<uint32_t>(thr + 4 * o);  // o <= last: inside the table
  o += (int)((o < last ? 1u : 0u) & (c1 >= t ? 1u : 0u));
  if (g & 0x8000u) {
    while (o < last && c1 >= lds_ld<uint32_t>(thr + 4 * o)) ++o;
  }
  return o;
}

__device__ __forceinline__ uint32_t guide16_at(uint32_t guide, uint32_t c1) {
  return lds_ld<uint16_t>(guide + 2 * (c1 >> (32 - kGuide16Bits)));
}

// Folded column distance min(|x - x0|, L - |x - x0|) for x, x0 in [0, L), L a power of two.
template <int L>
__device__ __forceinline__ int fold_col(int x, int x0) {
  const int d = (x - x0) & (L - 1);
  const int e = L - d;
  return d < e ? d : e;
}

// Step 1 for this lane's labels of the chunk starting after `base`: Philox4x32-10 of
// (label, sample, PROPOSE); site i = mulhi(w0, N) = w0 >> (32 - log2 N); orbit from the
// 16-bit guide (one threshold comparison; a search only in buckets holding two or more); member
// w3 & (size - 1), read as w3 & 7 from the 8-slot table; acceptance uniform
// (2 (w2 >> 9) + 1) 2^-24.
// Per-sample values the hop loop keeps in scalar registers (read once per launch).
struct FxConst {
  uint32_t k0, k1, sid;  // Philox key and sample id
  int32_t last;          // index of the last orbit
  float Ef, mTln2;       // E and -T ln 2 in FP32
};

template <int L, int U, int NW>
__device__ __forceinline__ void draw_fx(uint64_t base, int tid, const FxConst& C, uint32_t lds0,
                                        const FxLds& lo, FxLabel (&lb)[U]) {
  using G = FxGeo<L, NW>;
  const uint32_t guide = lds0 + lo.guide, thr = lds0 + lo.thr, vec8 = lds0 + lo.vec8;
  const uint32_t ev = lds0 + lo.ev;
  const int last = C.last;
  const float Ef = C.Ef, mTln2 = C.mTln2;
  // the Philox words of every label first (pure VALU, no LDS access), then the table lookups
  // of all of them: the lane waits for LDS once per lookup stage, not once per label
  uint32_t w0[U], w1[U], w2[U], w3[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t lab = base + 1 + (uint64_t)(tid * U + k);
    w0[k] = (uint32_t)lab;
    w1[k] = (uint32_t)(lab >> 32);
    w2[k] = C.sid;
    w3[k] = kTagPropose;
    philox10(w0[k], w1[k], w2[k], w3[k], C.k0, C.k1);
  }
  uint32_t g[U];
#pragma unroll
  for (int k = 0; k < U; ++k) g[k] = guide16_at(guide, w1[k]);
  uint64_t v[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const int o = orbit_guided(g[k], w1[k], thr, last);
    v[k] = lds_ld<uint64_t>(vec8 + 8 * (o * 8 + (int)(w3[k] & 7u)));
  }
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const int i = (int)(w0[k] >> (32 - 2 * G::LG));
    const int vx = (int)(uint32_t)v[k];
    const int dx = (int)(int16_t)(vx & 0xffff), dy = vx >> 16;
    const int xi = i & (L - 1), yi = i >> G::LG;
    const int xj = (xi + dx) & (L - 1), yj = (yi + dy) & (L - 1);
    const int j = (yj << G::LG) | xj;
    const float td = __uint_as_float((uint32_t)(v[k] >> 32));
    const float u = (float)(2u * (w2[k] >> 9) + 1u) * 0x1p-24f;
    FxLabel& b = lb[k];
    b.i = i;
    b.j = j;
    b.ai = ev + 4 * G::ev_slot(xi, yi);
    b.aj = ev + 4 * G::ev_slot(xj, yj);
    b.dx = dx;
    b.td = td;
    b.th = (td + Ef * (float)dx) + mTln2 * __log2f(u);
  }
}

// CLOCK = 0: deterministic clock t = s_last / Gamma; 1: Gaussian increments (step 3c), the
// only per-hop call, kept out of the deterministic instance.  TIM: per-phase shader-cycle
// timers, compiled only into the instances that run with them (a runtime test of the flag
// at every phase costs the untimed kernel ~4%).
template <int L, int U, int CLOCK, int NW, bool TIM>
__global__ void __launch_bounds__(64 * NW) k_hops_fx(const DevSample* __restrict__ samples,
                                                  const int32_t* __restrict__ order, RunArgs ra) {
  using G = FxGeo<L, NW>;
  constexpr int NT = G::NT, NC = G::NC, RPW = G::RPW, P = G::P, SPL = G::SPL;
  constexpr uint32_t M = (uint32_t)NT * U;
  constexpr int kRenorm = 16;
  const DevSample& S = samples[order[blockIdx.x]];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = uni((int32_t)(tid >> 6));

  uint64_t hops = uni(gs->hops);
  uint64_t s_last = uni(gs->s_last);
  int32_t since = uni(gs->since_refresh);
  const uint64_t target = uni(gs->hop_target);
  const uint64_t scan0 = uni(gs->call_scan0);
  const double t_end = uni(gs->t_end);
  const double t_start = uni(gs->t);
  {
    const bool idle = uni(gs->status) != 0 || hops >= target || (ra.time_mode && t_start >= t_end) ||
                      (ra.K > 0 && since >= ra.K);
    if (idle) return;
  }
  // hops this launch may still execute: up to the call's target and to the next refresh
  // (launch-local 32-bit counters keep 64-bit scalar arithmetic out of the hop loop)
  const uint64_t hops0 = hops;
  uint32_t hleft;
  {
    const uint64_t lim_t = target - hops0;
    const uint64_t lim_k = ra.K > 0 ? (uint64_t)(ra.K - since) : ~0ull;
    const uint64_t lim = lim_t < lim_k ? lim_t : lim_k;
    hleft = uni((uint32_t)(lim < 0xffffffffull ? lim : 0xffffffffull));
  }
  uint32_t hcnt = (uint32_t)hops0;  // low bits of the hop count (the renormalisation phase)
  uint64_t base = uni(gs->s_scan);  // labels base + 1 .. base + M form the current chunk
  uint32_t dpos = 0;                // labels up to base + dpos are decided
  int64_t P_ = uni(gs->P);
  double H0 = uni(gs->H0);
  uint64_t sum_p = uni(gs->sum_p), rounds = uni(gs->rounds), evaluated = uni(gs->evaluated);
  int64_t logged = uni(gs->logged);
  int32_t status = 0;

  extern __shared__ __align__(16) uint8_t smem[];
  const FxLds lo = fx_lds(L, S.n_orb, NW);
  const uint32_t lds0 = lds_addr_of(smem);
  float* __restrict__ ev = (float*)(smem + lo.ev);
  uint32_t* __restrict__ occ = (uint32_t*)(smem + lo.occ);
  FxShared* __restrict__ sh = (FxShared*)(smem + lo.ctrl);
  uint4* __restrict__ info = (uint4*)(smem + lo.info);

  // owned energies (hi, lo) in registers, fl(hi + lo) in LDS
  float eh[RPW][NC], el[RPW][NC];
  {
    const float2* __restrict__ g = (const float2*)S.eps;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int l = (wid + NW * r) * L + lane + 64 * c;
        const float2 e = g[l];
        eh[r][c] = e.x;
        el[r][c] = e.y;
        set_mark(eh[r][c], el[r][c], (S.occ[l >> 5] >> (l & 31)) & 1u);
        ev[wid * 64 * SPL + ((r * NC + c) >> 2) * 256 + lane * 4 + ((r * NC + c) & 3)] = marked(eh[r][c], el[r][c]);
      }
    }
    const uint4* __restrict__ gt = (const uint4*)S.tabk;
    uint4* __restrict__ st = (uint4*)(smem + lo.tab);
    for (int k = tid; k < fx_tab_entries(L, NW) / 4; k += NT) st[k] = gt[k];
  }
  for (int k = tid; k < G::N / 32; k += NT) occ[k] = S.occ[k];
  for (int k = tid; k < S.n_orb; k += NT) ((uint32_t*)(smem + lo.thr))[k] = S.thr[k];
  for (int k = tid; k < kGuide16Size; k += NT) ((uint16_t*)(smem + lo.guide))[k] = S.guide16[k];
  for (int k = tid; k < S.n_orb * 8; k += NT) ((int2*)(smem + lo.vec8))[k] = ((const int2*)S.vec8)[k];
  if (tid < kMaxWaves) info[tid] = make_uint4(0u, 0u, 0u, ~0u);  // no round has this tag
  if (tid == 0) {
    sh->theta = 0u;
    sh->t = t_start;
    sh->nev = 0ull;
  }
  __syncthreads();

  FxConst C;
  C.k0 = uni(S.seed_lo);
  C.k1 = uni(S.seed_hi);
  C.sid = uni(S.sample_id);
  C.last = uni(S.n_orb - 1);
  C.Ef = __uint_as_float(uni(__float_as_uint(S.E32)));
  C.mTln2 = __uint_as_float(uni(__float_as_uint(S.mTln2_32)));
  const double Gamma = uni(S.Gamma);
  const int32_t l2m = uni(S.log2M);  // the sample's PR width 2^l2m
  const int64_t log_cap = uni((int64_t)S.log_cap);
  uint64_t* __restrict__ log_label = S.log_label;
  int32_t* __restrict__ log_from = S.log_from;
  int32_t* __restrict__ log_to = S.log_to;
  const uint64_t s_end = uni((ra.time_mode && CLOCK == 0) ? label_at_time(t_end, Gamma) : (uint64_t)0);
  // this lane's energy values (row wid + NW r, column lane + 64 c at slot s = r NC + c): chunk
  // s / 4 at ev_lane + 1024 (s / 4)
  const uint32_t ev_lane = opaque(lds0 + lo.ev + 4u * (uint32_t)(wid * 64 * SPL + lane * 4));
  constexpr int kRowTab = NW * P * 4;
  const uint32_t info_lane = opaque(lds0 + lo.info + 16u * (uint32_t)(lane & (kMaxWaves - 1)));
  bool cached = false;
  // owner test: site l = (y << LG) | x belongs to thread (y % NW) 64 + (x & 63), i.e. to the
  // thread whose tid - own_off equals l & own_mask
  constexpr uint32_t own_mask = 63u | ((uint32_t)(NW - 1) << G::LG);
  const uint32_t own_off = uni((uint32_t)(wid * 64) - ((uint32_t)wid << G::LG));
  // table row of origin row 0 for this wave's first row (wid + L)
  const uint32_t tab_w = uni(lds0 + lo.tab + (uint32_t)((wid + L) * P * 4));
  FxLabel lb[U];
  // the chunk after the current one, drawn during a hop's update (the labels do not depend on
  // the configuration): lbn holds chunk base + M when pre is set
  FxLabel lbn[U];
  bool pre = false;
  uint32_t theta_cnt = 0;
  uint32_t nev = 0;    // this lane's label evaluations (labels at or after dpos in a round)
  uint32_t round = 0;  // tag of the current evaluation round = rounds of this launch so far
  uint64_t tc0 = 0, tc1 = 0, tc2 = 0, tc3 = 0, tmark = 0;
  constexpr bool timers = TIM;
#define CG_MARK(acc)                                          \
  if (timers) {                                               \
    const uint64_t now_ = __builtin_amdgcn_s_memtime();       \
    acc += now_ - tmark;                                      \
    tmark = now_;                                             \
  }
  if (timers) tmark = __builtin_amdgcn_s_memtime();

  // one iteration per executed hop; the energies change only in its straight-line part
  for (;;) {
    // rounds until a round accepts a label (or the label cap stops the sample)
    uint32_t mk = 0u, win0 = 0u, win1 = 0u, win2 = 0u;
    for (;;) {
    if (!cached) {
      if (pre) {
#pragma unroll
        for (int k = 0; k < U; ++k) lb[k] = lbn[k];
        pre = false;
      } else {
        draw_fx<L, U, NW>(base, tid, C, lds0, lo, lb);
      }
      cached = true;
      CG_MARK(tc0)
    }

    // step 2 for the undecided labels: occupancy filter and Metropolis; the lane keeps its
    // first accepted label (selects, no divergent blocks: the exec mask stays whole)
    // (0/1 integers in vector registers rather than lane masks: the decision costs vector
    // instructions only, none of the workgroup's shared scalar unit)
    uint32_t found = 0u;
    uint32_t pub0 = 0u, pub1 = 0u;
    float pdh = 0.f;
    // the value words of every undecided label are read at once (an accepted label makes the
    // lane's later labels moot, but waiting for its decision would add an LDS round trip)
    // (a lane with any undecided label reads all of its labels' words: one branch per round;
    // the words of its decided labels are ignored below)
    uint32_t wis[U], wjs[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      wis[k] = 0u;
      wjs[k] = 0u;
    }
    if ((uint32_t)(tid * U + U - 1) >= dpos) {
#pragma unroll
      for (int k = 0; k < U; ++k) {
        wis[k] = lds_ld<uint32_t>(lb[k].ai);
        wjs[k] = lds_ld<uint32_t>(lb[k].aj);
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const FxLabel& b = lb[k];
      const uint32_t key = (uint32_t)(tid * U + k);
      // not yet decided: key >= dpos (both below 2^31) and no earlier label of the lane accepted
      const uint32_t undec = ((key - dpos) >> 31) ^ 1u;
      nev += undec;
      const uint32_t open = undec & (found ^ 1u);
      const uint32_t wi = wis[k], wj = wjs[k];
      const float de = __uint_as_float(wj) - __uint_as_float(wi);
      const uint32_t th = open & wi & ~wj & 1u;  // n_i (1 - n_j) from the value words
      // de <= th exactly when th - de >= 0: the difference of two FP32 values of like size is
      // exact (Sterbenz), so its sign bit decides
      const uint32_t le = (__float_as_uint(b.th - de) >> 31) ^ 1u;
      const uint32_t acc = th & le;
      theta_cnt += th;
      pub0 = acc ? ((uint32_t)b.i | ((uint32_t)b.j << 16)) : pub0;
      pub1 = acc ? (key | ((uint32_t)b.dx << 16)) : pub1;
      pdh = acc ? de - b.td : pdh;
      found |= acc;
    }
    // the wave's lowest accepting lane publishes its label in the wave's record, tagged with
    // the round; after the barrier lanes 0..15 read the 16 records (waves beyond NW never
    // write theirs, whose initial tag no round carries) and the round's winner is
    // the lowest wave whose record carries this round's tag (keys grow with the thread
    // index).  A record is rewritten only by its own wave: in a later round, which only
    // happens before another wave reads it for this round if this round executed no hop
    // from that wave, and then the later tag is simply not this round's.
    const unsigned long long bal = __ballot(found != 0u);
    {
      // the lowest accepting lane: found, and no accepting lane below it (a lane count, so
      // that the test is vector arithmetic and one branch)
      const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      if (((found ^ 1u) | below) == 0u) info[wid] = make_uint4(pub0, pub1, __float_as_uint(pdh), round);
    }
    CG_MARK(tc1)
    __syncthreads();
    // every lane reads a whole record in one 16-byte load (lanes l and l + 16 k share one:
    // broadcast reads), only the first 16 lanes vote; the winner's words are read from its
    // lane unconditionally (lane 63 when no record carries the tag), so that the record costs
    // one LDS round trip
    const u32x4 rec = lds_ld<u32x4>(info_lane);
    const unsigned long long won = __ballot(rec.w == round) & ((1ull << kMaxWaves) - 1ull);
    mk = won != 0ull ? 1u : 0u;
    const int wl = __ffsll(won | (1ull << 63)) - 1;
    win0 = (uint32_t)__builtin_amdgcn_readlane((int)rec.x, wl);
    win1 = (uint32_t)__builtin_amdgcn_readlane((int)rec.y, wl);
    win2 = (uint32_t)__builtin_amdgcn_readlane((int)rec.z, wl);
    ++round;
    CG_MARK(tc2)
    if (mk != 0u) break;
    // every label of the chunk is rejected
    base += M;
    dpos = 0;
    cached = false;
    if (base - scan0 >= ra.max_labels) {
      status = -4;  // CG_ESTALL
      break;
    }
    }
    if (mk == 0u) break;

    // step 3: execute the lowest accepted label
    const uint32_t w0 = win0, w1 = win1;
    const float dh0 = __uint_as_float(win2);
    const int hi = (int)(w0 & 0xffffu), hj = (int)(w0 >> 16);
    const uint32_t key = w1 & 0xffffu;
    const int hdx = (int)w1 >> 16;
    dpos = key + 1;
    ++hcnt;
    --hleft;
    // the state written back at the end (by thread 0): kept by wave 0 only, so that the
    // other waves' scalar work after the barrier is just what their update needs
    if (wid == 0) {
      const uint64_t q = base + 1 + key;
      const uint64_t m = q - s_last;
      s_last = q;
      P_ += hdx;
      H0 = H0 + (double)dh0;
      sum_p += p_iterations(m, l2m);
      if (tid == 0) {
        atomicAnd(&occ[hi >> 5], ~(1u << (hi & 31)));
        atomicOr(&occ[hj >> 5], 1u << (hj & 31));
        if (logged < log_cap) {
          log_label[logged] = q;
          log_from[logged] = hi;
          log_to[logged] = hj;
        }
        if (CLOCK != 0)
          sh->t = sh->t + clock_dt(ra.clock_mode, hops0 + (uint32_t)(hcnt - (uint32_t)hops0), m, C.sid, C.k0, C.k1,
                                   Gamma);
      }
      logged += logged < log_cap ? 1 : 0;
    }
    // the owners of i and j move their occupation marks: site (x, y) is slot (y / NW) NC +
    // (x >> 6) of lane x & 63 in wave y % NW; the slot index is wave-uniform, so a short
    // branch tree picks the register
    {
      const int xi = hi & (L - 1), yi = hi >> G::LG, xj = hj & (L - 1), yj = hj >> G::LG;
#define CG_SLOT(k)                                                                   \
  case k:                                                                            \
    if constexpr (k < SPL) {                                                         \
      set_mark(eh[k / NC][k % NC], el[k / NC][k % NC], n);                           \
    }                                                                                \
    break;
#define CG_SLOTS(sl)                                                                 \
  switch (sl) {                                                                      \
    CG_SLOT(0) CG_SLOT(1) CG_SLOT(2) CG_SLOT(3) CG_SLOT(4) CG_SLOT(5) CG_SLOT(6)     \
    CG_SLOT(7) CG_SLOT(8) CG_SLOT(9) CG_SLOT(10) CG_SLOT(11) CG_SLOT(12) CG_SLOT(13) \
    CG_SLOT(14) CG_SLOT(15) CG_SLOT(16) CG_SLOT(17) CG_SLOT(18) CG_SLOT(19) CG_SLOT(20) \
    CG_SLOT(21) CG_SLOT(22) CG_SLOT(23) CG_SLOT(24) CG_SLOT(25) CG_SLOT(26) CG_SLOT(27) \
    CG_SLOT(28) CG_SLOT(29) CG_SLOT(30) CG_SLOT(31) default: break;                  \
  }
      // the owner thread of a site: one masked vector compare each
      const uint32_t me = (uint32_t)tid - own_off;
      if (me == ((uint32_t)hi & own_mask)) {
        const uint32_t n = 0u;
        CG_SLOTS((yi >> G::LW) * NC + (xi >> 6))
      }
      if (me == ((uint32_t)hj & own_mask)) {
        const uint32_t n = 1u;
        CG_SLOTS((yj >> G::LW) * NC + (xj >> 6))
      }
#undef CG_SLOTS
#undef CG_SLOT
    }
    CG_MARK(tc2)

    // step 3b on the owned sites: lo += 1/r_lj - 1/r_li, LDS value fl(hi + lo).  Row
    // y = wid + NW r of the table for origin row y0 is row wid - y0 + L + NW r.  All table
    // loads are issued before the first store.
    {
      const int xi = hi & (L - 1), yi = hi >> G::LG, xj = hj & (L - 1), yj = hj >> G::LG;
      const uint32_t rj = tab_w - (uint32_t)(yj * P * 4);
      const uint32_t ri = tab_w - (uint32_t)(yi * P * 4);
      uint32_t aj[NC], ai[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int x = lane + 64 * c;
        aj[c] = opaque(rj + 4 * (uint32_t)fold_col<L>(x, xj));
        ai[c] = opaque(ri + 4 * (uint32_t)fold_col<L>(x, xi));
      }
      float d[RPW][NC];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
          d[r][c] = lds_ld<float>(aj[c] + r * kRowTab) - lds_ld<float>(ai[c] + r * kRowTab);
      }
      // while the table loads are in flight: draw the next chunk if it is not drawn yet
      if (!pre) {
        pre = true;
        draw_fx<L, U, NW>(base + M, tid, C, lds0, lo, lbn);
      }
      float v[SPL];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          el[r][c] = el[r][c] + d[r][c];
          v[r * NC + c] = marked(eh[r][c], el[r][c]);
        }
      }
#pragma unroll
      for (int q = 0; q < SPL / 4; ++q) {
        f32x4 w;
        w.x = v[4 * q];
        w.y = v[4 * q + 1];
        w.z = v[4 * q + 2];
        w.w = v[4 * q + 3];
        lds_st<f32x4>(ev_lane + 1024 * q, w);
      }
      if ((hcnt & (uint32_t)(kRenorm - 1)) == 0) {
        // Fast2Sum: z = fl(hi + lo) - hi is exact and hi + z = fl(hi + lo), so the pair
        // keeps its sum while hi absorbs lo (written as updates of hi and lo in place); the
        // occupation bit is then put back into hi
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const uint32_t n = __float_as_uint(eh[r][c]) & 1u;
            const float z = (eh[r][c] + el[r][c]) - eh[r][c];
            el[r][c] = el[r][c] - z;
            eh[r][c] = eh[r][c] + z;
            set_mark(eh[r][c], el[r][c], n);
          }
        }
      }
    }
    __syncthreads();
    CG_MARK(tc3)
    if (dpos == M) {
      base += M;
      dpos = 0;
      cached = false;
    }
    if (hleft == 0u) break;
    if (ra.time_mode) {
      if (CLOCK == 0 ? base + dpos >= s_end : uni(sh->t) >= t_end) break;
    }
  }
  hops = hops0 + (uint32_t)(hcnt - (uint32_t)hops0);
  since += (int32_t)(uint32_t)(hops - hops0);

  atomicAdd(&sh->theta, theta_cnt);
  atomicAdd(&sh->nev, (unsigned long long)nev);
  {
    float2* __restrict__ g = (float2*)S.eps;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
#pragma unroll
      for (int c = 0; c < NC; ++c) g[(wid + NW * r) * L + lane + 64 * c] = make_float2(eh[r][c], el[r][c]);
    }
  }
  __syncthreads();
  for (int k = tid; k < G::N / 32; k += NT) S.occ[k] = occ[k];
  if (tid == 0) {
    gs->hops = hops;
    gs->s_last = s_last;
    gs->s_scan = base + dpos;
    gs->P = P_;
    gs->t = CLOCK == 0 ? (double)s_last / Gamma : sh->t;
    gs->H0 = H0;
    gs->since_refresh = since;
    gs->status = status;
    gs->sum_p = sum_p;
    gs->rounds = rounds + round;
    gs->evaluated = evaluated + sh->nev;
    gs->theta_pass += sh->theta;
    gs->logged = logged;
    if (timers) {
      gs->phase_cycles[0] += tc0;
      gs->phase_cycles[1] += tc1;
      gs->phase_cycles[2] += tc2;
      gs->phase_cycles[3] += tc3;
    }
  }
#undef CG_MARK
}

}  // namespace cg
