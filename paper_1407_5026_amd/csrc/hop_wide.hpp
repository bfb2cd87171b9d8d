// hop_wide.hpp -- one sample, G workgroups, the parallel-rejection width spread over the GPU
// (L = 16 ... 128, a power of two; FP64 form).
//
// The per-sample kernels give a sample one workgroup, so one round evaluates at most 2048
// labels; at low T, where the mean number of proposals per hop 1/A reaches 10^5, a hop then
// takes many rounds on one CU.  The paper's own GPU runs widen the iteration instead: one
// sample, M ~ 1/A labels evaluated at once by the whole GPU ("Parallel rejection",
// "Code performance").  Here every workgroup of a cooperative launch keeps a full replica of
// the sample (FP64 energies and occupation in LDS) and evaluates its own slice of each round:
//   * round r covers labels base + 1 ... base + G Mw (Mw = 1024 U per workgroup); workgroup g
//     evaluates base + g Mw + 1 ... base + (g + 1) Mw, the labels above the last executed one
//     (position dpos) being the undecided ones;
//   * each workgroup finds its lowest accepted label, and one global atomic minimum per
//     workgroup over the round's slot gives the round's lowest accepted label; the last
//     arriver at the round's grid barrier reads the slot and publishes it in the barrier's
//     release word, so every workgroup leaves the barrier with the same winner;
//   * every workgroup then executes that hop on its own replica (draw of the winning label
//     recomputed from its counter, the energy update of step 3b in LDS), so a hop needs no
//     data exchange and no second barrier.
// The labels, streams, decisions and FP64 arithmetic are those of the other kernels, so the
// hops equal the oracle's for every G.  Four round slots rotate; the slot of round r + 2 is
// reset by workgroup 0 during round r: round r - 2's barrier was released (after its last
// arriver read that slot) before workgroup 0 left it, and every minimum of round r + 2
// follows workgroup 0's release at the barrier of round r + 1.
#pragma once

#include "hop_big.hpp"

namespace cg {

constexpr uint32_t kWideSlots = 4;  // round slots (one 128-byte line each) after the barrier words
// after the slots: one line holding the 64-bit release word of the round barrier
constexpr int kWideRel = kBarWords + (int)kWideSlots * kBarLine;
constexpr int kWideSyncWords = kWideRel + kBarLine;

// The grid barrier of a round, which also hands out the round's winner: the two-level
// counter tree of grid_barrier, whose last arriver reads the round's slot (every
// workgroup's minimum is in it, released before its arrival) and stores (n << 32 | slot)
// as the release word that every workgroup polls, so no workgroup reads the slot itself.
__device__ __forceinline__ bool round_barrier(uint32_t* bar, uint32_t& n, uint32_t G, uint32_t* ok_sh,
                                              const uint32_t* slot, uint32_t* win_sh) {
  __syncthreads();
  ++n;
  if (threadIdx.x == 0) {
    const uint32_t g = blockIdx.x;
    const uint32_t gsize = (G + 7u - (g & 7u)) / 8u;
    const uint32_t ngroups = G < 8u ? G : 8u;
    uint64_t* rel = (uint64_t*)(bar + kWideRel);
    const uint32_t old =
        __hip_atomic_fetch_add(bar + (2 + (g & 7u)) * kBarLine, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (old == n * gsize - 1u) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint32_t o2 = __hip_atomic_fetch_add(bar + kBarLine, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 == n * ngroups - 1u) {
        const uint32_t w = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(rel, ((uint64_t)n << 32) | w, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    uint32_t ok = 1u, spins = 0u;
    uint64_t v = __hip_atomic_load(rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while ((uint32_t)(v >> 32) < n) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins >= kBarrierSpins) {
        ok = 0u;
        break;
      }
      v = __hip_atomic_load(rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *win_sh = (uint32_t)v;
    *ok_sh = ok;
  }
  __syncthreads();
  return *ok_sh != 0u;
}

// LDS of the wide kernel: the large-sample kernel's proposal tables and records, then the
// replica's FP64 energies and occupation words, and the FP64 (|dy|, |dx|) table when L <= 64.
struct WideLds {
  BigLds b;
  int32_t eps, occ, tab, total;
};
__host__ __device__ inline WideLds wide_lds(int32_t L, int32_t n_orb) {
  WideLds o;
  o.b = big_lds(n_orb);
  const int32_t N = L * L, H1 = L / 2 + 1;
  int32_t b = o.b.total;
  o.eps = b; b = align16(b + N * 8);
  o.occ = b; b = align16(b + (N / 32) * 4);
  o.tab = b; b = align16(b + (L <= 64 ? H1 * H1 * 8 : 0));
  o.total = b;
  return o;
}

template <int LG, int U, int CLOCK>
__global__ void __launch_bounds__(1024) k_hops_wide(const DevSample* __restrict__ samples, int32_t sample,
                                                    RunArgs ra) {
  constexpr int L = 1 << LG, N = L * L, NWD = N / 32, H1 = L / 2 + 1;
  constexpr int SPT = (N + 1023) / 1024;  // replica sites per thread in the update
  constexpr bool kTabLds = L <= 64;
  constexpr uint32_t Mw = 1024u * U;      // labels per workgroup and round
  const DevSample& S = samples[sample];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = uni((int32_t)(tid >> 6));
  const uint32_t G = gridDim.x;
  const uint32_t MC = G * Mw;             // labels per round
  const uint32_t koff = blockIdx.x * Mw;  // this workgroup's first key of a round
  const bool lead = blockIdx.x == 0;

  uint64_t hops = uni(gs->hops);
  uint64_t s_last = uni(gs->s_last);
  const uint64_t target = uni(gs->hop_target);
  const uint64_t scan0 = uni(gs->call_scan0);
  const double t_end = uni(gs->t_end);
  const double t_start = uni(gs->t);
  {
    const bool idle = uni(gs->status) != 0 || hops >= target || (ra.time_mode && t_start >= t_end);
    if (idle) return;
  }
  uint64_t base = uni(gs->s_scan);
  uint32_t dpos = 0;
  int64_t P_ = uni(gs->P);
  double H0 = uni(gs->H0);
  uint64_t sum_p = uni(gs->sum_p), rounds = uni(gs->rounds), evaluated = uni(gs->evaluated);
  int64_t logged = uni(gs->logged);
  int32_t status = 0;

  extern __shared__ __align__(16) uint8_t smem[];
  const WideLds lo = wide_lds(L, S.n_orb);
  const uint32_t lds0 = lds_addr_of(smem);
  uint4* __restrict__ rec = (uint4*)(smem + lo.b.rec);
  double* __restrict__ tclock = (double*)(smem + lo.b.ctrl);
  uint32_t* __restrict__ bar_ok = (uint32_t*)(smem + lo.b.ctrl + 12);
  uint32_t* __restrict__ win_sh = (uint32_t*)(smem + lo.b.ctrl + 16);
  double* __restrict__ eps = (double*)(smem + lo.eps);
  uint32_t* __restrict__ occ = (uint32_t*)(smem + lo.occ);
  const double* __restrict__ tab = kTabLds ? (const double*)(smem + lo.tab) : S.tab64;
  uint32_t* __restrict__ slot = S.bar + kBarWords;  // kWideSlots round slots, kBarLine apart
  uint32_t bar_n = 0;

  for (int l = tid; l < N; l += 1024) eps[l] = ((const double*)S.eps)[l];
  for (int w = tid; w < NWD; w += 1024) occ[w] = S.occ[w];
  if (kTabLds)
    for (int k = tid; k < H1 * H1; k += 1024) ((double*)(smem + lo.tab))[k] = S.tab64[k];
  for (int k = tid; k < S.n_orb; k += 1024) {
    ((uint32_t*)(smem + lo.b.thr))[k] = S.thr[k];
    ((double*)(smem + lo.b.td))[k] = S.tdo64[k];
  }
  for (int k = tid; k < kGuide16Size; k += 1024) ((uint16_t*)(smem + lo.b.guide))[k] = S.guide16[k];
  for (int k = tid; k < S.n_orb * 8; k += 1024) ((int2*)(smem + lo.b.vec8))[k] = ((const int2*)S.vec8)[k];
  if (tid < kMaxWaves) rec[tid] = make_uint4(0u, 0u, 0u, ~0u);  // no round has this tag
  if (tid == 0) *tclock = t_start;
  __syncthreads();

  FxConst C;
  C.k0 = uni(S.seed_lo);
  C.k1 = uni(S.seed_hi);
  C.sid = uni(S.sample_id);
  C.last = uni(S.n_orb - 1);
  C.Ef = 0.f;
  C.mTln2 = 0.f;
  const double Ef = uni(S.E), mrT = uni(S.mrT), Gamma = uni(S.Gamma);
  const int64_t log_cap = uni((int64_t)S.log_cap);
  const uint64_t s_end = uni((ra.time_mode && CLOCK == 0) ? label_at_time(t_end, Gamma) : (uint64_t)0);
  bool cached = false;
  BigLabel lb[U];
  uint32_t theta_cnt = 0;
  uint32_t round = 0;

  for (;;) {
    uint32_t win = ~0u;
    for (;;) {
      if (!cached) {
        draw_big<LG, U>(base + koff, tid, C, lds0, lo.b, lb);
        cached = true;
      }
      // step 2 on this workgroup's slice against the replica; the lane keeps its first
      // accepted label
      uint32_t mine = ~0u;
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const BigLabel& b = lb[k];
        const uint32_t key = koff + (uint32_t)(tid * U + k);
        const bool open = (mine == ~0u) & (key >= dpos);
        const bool th = open && ((((occ[b.i >> 5] >> (b.i & 31)) & ~(occ[b.j >> 5] >> (b.j & 31))) & 1u) != 0u);
        if (th) {
          const double dH = ((eps[b.j] - eps[b.i]) - b.td) - Ef * (double)b.dx;
          bool a = dH <= 0.0;
          if (!a) a = b.u < exp(dH * mrT);
          if (a) mine = key;
        }
        theta_cnt += th ? 1u : 0u;
      }
      // the workgroup's lowest accepted key: the wave's lowest accepting lane publishes it,
      // tagged with the round; keys grow with the thread index, so the lowest wave holding a
      // record of this round has it
      const unsigned long long bal = __ballot(mine != ~0u);
      if (bal != 0ull && lane == __ffsll(bal) - 1) rec[wid] = make_uint4(mine, 0u, 0u, round);
      if (lead && tid == 0)
        __hip_atomic_store(slot + ((round + 2u) % kWideSlots) * kBarLine, ~0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      if (wid == 0) {
        uint4 r = make_uint4(~0u, 0u, 0u, ~round);
        if (lane < kMaxWaves) r = rec[lane];
        const unsigned long long won = __ballot(r.w == round);
        if (won != 0ull && lane == __ffsll(won) - 1)
          __hip_atomic_fetch_min(slot + (round % kWideSlots) * kBarLine, r.x, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
      if (!round_barrier(S.bar, bar_n, G, bar_ok, slot + (round % kWideSlots) * kBarLine, win_sh)) {
        status = -3;  // CG_EHIP: a workgroup did not arrive
        break;
      }
      win = uni(*win_sh);
      ++round;
      ++rounds;
      evaluated += MC - dpos;
      if (win != ~0u) break;
      // every label of the round is rejected
      base += MC;
      dpos = 0;
      cached = false;
      if (base - scan0 >= ra.max_labels) {
        status = -4;  // CG_ESTALL
        break;
      }
    }
    if (win == ~0u) break;

    // step 3: the winning label's proposal, recomputed from its counter (uniform), executed on
    // every replica; workgroup 0 writes the hop log
    const uint64_t q = base + 1 + win;
    int hi, hj, hdx;
    double td;
    {
      const uint32_t guide = lds0 + lo.b.guide, thr = lds0 + lo.b.thr, vec8 = lds0 + lo.b.vec8;
      uint32_t c0 = (uint32_t)q, c1 = (uint32_t)(q >> 32), c2 = C.sid, c3 = kTagPropose;
      philox10(c0, c1, c2, c3, C.k0, C.k1);
      const int i = (int)(c0 >> (32 - 2 * LG));
      const int o = orbit_guided(guide16_at(guide, c1), c1, thr, C.last);
      const uint64_t v = lds_ld<uint64_t>(vec8 + 8 * (o * 8 + (int)(c3 & 7u)));
      const int vx = (int)(uint32_t)v;
      const int dx = (int)(int16_t)(vx & 0xffff), dy = vx >> 16;
      const int xi = i & (L - 1), yi = i >> LG;
      hi = uni(i);
      hj = uni((((yi + dy) & (L - 1)) << LG) | ((xi + dx) & (L - 1)));
      hdx = uni(dx);
      td = uni(lds_ld<double>(lds0 + lo.b.td + 8 * o));
    }
    const double dh0 = (eps[hj] - eps[hi]) - td;
    const uint64_t m = q - s_last;
    s_last = q;
    dpos = win + 1;
    ++hops;
    P_ += hdx;
    H0 = H0 + dh0;
    sum_p += p_iterations(m, S.log2M);
    const bool log_it = logged < log_cap;
    const int64_t log_at = logged;
    logged += log_it ? 1 : 0;
    // every lane has read eps[i], eps[j] before they change
    __syncthreads();
    if (tid == 0) {
      occ[hi >> 5] &= ~(1u << (hi & 31));
      occ[hj >> 5] |= 1u << (hj & 31);
      if (lead && log_it) {
        S.log_label[log_at] = q;
        S.log_from[log_at] = hi;
        S.log_to[log_at] = hj;
      }
      if (CLOCK != 0) *tclock = *tclock + clock_dt(ra.clock_mode, hops, m, C.sid, C.k0, C.k1, Gamma);
    }
    // step 3b on the replica: eps_l += 1/r_lj - 1/r_li (1/r(0) = 0 from the table)
    {
      const int xi = hi & (L - 1), yi = hi >> LG, xj = hj & (L - 1), yj = hj >> LG;
#pragma unroll
      for (int s = 0; s < SPT; ++s) {
        const int l = tid + 1024 * s;
        if (N % 1024 == 0 || l < N) {
          const int x = l & (L - 1), y = l >> LG;
          const double tj = tab[fold(y - yj, L) * H1 + fold(x - xj, L)];
          const double ti = tab[fold(y - yi, L) * H1 + fold(x - xi, L)];
          eps[l] = eps[l] + (tj - ti);
        }
      }
    }
    __syncthreads();
    if (dpos == MC) {
      base += MC;
      dpos = 0;
      cached = false;
    }
    if (hops >= target) break;
    if (ra.time_mode) {
      if (CLOCK == 0 ? s_last >= s_end : uni(*tclock) >= t_end) break;
    }
  }

  if (theta_cnt != 0u) atomicAdd((unsigned long long*)&gs->theta_pass, (unsigned long long)theta_cnt);
  if (lead) {
    for (int l = tid; l < N; l += 1024) ((double*)S.eps)[l] = eps[l];
    for (int w = tid; w < NWD; w += 1024) S.occ[w] = occ[w];
    if (tid == 0) {
      gs->hops = hops;
      gs->s_last = s_last;
      gs->s_scan = base + dpos;
      gs->P = P_;
      gs->t = CLOCK == 0 ? (double)s_last / Gamma : *tclock;
      gs->H0 = H0;
      gs->status = status;
      gs->sum_p = sum_p;
      gs->rounds = rounds;
      gs->evaluated = evaluated;
      gs->logged = logged;
    }
  }
}

__global__ void k_wide_reset(const DevSample* __restrict__ samples, int32_t sample) {
  const DevSample& S = samples[sample];
  if (threadIdx.x < 10) S.bar[threadIdx.x * kBarLine] = 0u;
  if (threadIdx.x < kWideSlots) S.bar[kBarWords + threadIdx.x * kBarLine] = ~0u;
  if (threadIdx.x == 0) *(uint64_t*)(S.bar + kWideRel) = 0ull;
}

}  // namespace cg
