// hop_big.hpp -- one sample on the whole GPU, for lattices too large for one workgroup's
// LDS (L = 128 ... 2048, a power of two; FP64 form).
//
// The hop kernel is the mixed parallel-rejection step of section "Hopping conduction in the
// Coulomb glass" (steps 1, 2, 3a-3c) with the same labels, streams and arithmetic as the
// per-sample kernels, distributed over G workgroups of one cooperative launch:
//   * workgroup g owns the 1024 SPT consecutive sites g 1024 SPT + t + 1024 s (thread t,
//     s < SPT) and keeps their FP64 energies in registers; a global mirror of all energies
//     serves the proposals;
//   * every workgroup evaluates the same chunk of labels against the global occupation and
//     mirror, so all of them find the same lowest accepted label without exchanging it;
//   * every workgroup executes the hop's bookkeeping, workgroup 0 alone writes the global
//     occupation bits, the hop log and the sample state;
//   * each workgroup applies step 3b to its own sites and writes them to the mirror.
// Two grid-wide barriers per hop keep every workgroup's view identical: one after the
// accepting round (no workgroup writes mirror or occupation while another still reads them
// for that round) and one after the update (the next round reads the new values).  Rounds
// without an accepted label write nothing and need no barrier.  Every workgroup takes the
// same decisions from the same data, so all of them reach every barrier.
// Initialisation for these sizes: the occupation by an exact selection of the n_e smallest
// (key, index) pairs through a histogram of the top 16 key bits (instead of the O(N^2) rank
// count), and the energies by the ordered FP64 sum reading occupation and 1/r table from
// global memory.
#pragma once

#include "hop_fx.hpp"

namespace cg {

constexpr int kSelCap = 4096;  // keys of one 2^48-wide bucket the selection can hold

// Scratch of the initial-occupation selection (one per large sample, in the arena).
struct OccSelect {
  uint32_t bucket;    // top-16-bit bucket holding the n_e-th smallest key
  uint32_t below;     // keys in lower buckets
  uint32_t count;     // keys of that bucket seen by the collection pass
  uint32_t overflow;  // set when the bucket holds more than kSelCap keys (an error)
  uint64_t thr_key;   // the n_e-th smallest (key, index) pair: occupied iff (key, i) <= it
  uint32_t thr_i;
  uint32_t pad_;
  uint32_t hist[65536];
  uint64_t list_key[kSelCap];
  uint32_t list_i[kSelCap];
};

__global__ void __launch_bounds__(kInitBlock) k_occ_clear(OccSelect* __restrict__ sel) {
  const int k = blockIdx.x * kInitBlock + threadIdx.x;
  if (k < 65536) sel->hist[k] = 0u;
  if (k == 0) {
    sel->count = 0u;
    sel->overflow = 0u;
  }
}

// Histogram of the top 16 bits of every site's 64-bit key (keys in the phi buffer).
__global__ void __launch_bounds__(kInitBlock) k_occ_hist(const DevSample* __restrict__ S, OccSelect* __restrict__ sel) {
  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  if (l >= S->N) return;
  const uint64_t key = ((const uint64_t*)S->phi)[l];
  atomicAdd(&sel->hist[(uint32_t)(key >> 48)], 1u);
}

// The bucket b with (keys below b) < n_e <= (keys below b) + hist[b]: one workgroup, a
// sequential prefix over 1024 per-thread partial sums, then over the chosen thread's bins.
__global__ void __launch_bounds__(1024) k_occ_select(const DevSample* __restrict__ S, OccSelect* __restrict__ sel) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  uint32_t s = 0;
  for (int k = 0; k < 64; ++k) s += sel->hist[64 * t + k];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    const uint32_t ne = (uint32_t)S->n_e;
    uint32_t below = 0;
    int tt = 0;
    while (tt < 1023 && below + part[tt] < ne) below += part[tt++];
    int b = 64 * tt;
    while (b < 64 * tt + 63 && below + sel->hist[b] < ne) below += sel->hist[b++];
    sel->bucket = (uint32_t)b;
    sel->below = below;
  }
}

// Keys of the chosen bucket, with their site index.
__global__ void __launch_bounds__(kInitBlock) k_occ_collect(const DevSample* __restrict__ S, OccSelect* __restrict__ sel) {
  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  if (l >= S->N) return;
  const uint64_t key = ((const uint64_t*)S->phi)[l];
  if ((uint32_t)(key >> 48) != sel->bucket) return;
  const uint32_t k = atomicAdd(&sel->count, 1u);
  if (k < (uint32_t)kSelCap) {
    sel->list_key[k] = key;
    sel->list_i[k] = (uint32_t)l;
  } else {
    sel->overflow = 1u;
  }
}

// The (n_e - below)-th smallest (key, index) pair of the bucket by rank counting (pairs are
// distinct, so exactly one has that rank).
__global__ void __launch_bounds__(1024) k_occ_threshold(const DevSample* __restrict__ S, OccSelect* __restrict__ sel) {
  __shared__ uint64_t kk[kSelCap];
  __shared__ uint32_t ki[kSelCap];
  const uint32_t cnt = sel->count < (uint32_t)kSelCap ? sel->count : (uint32_t)kSelCap;
  for (uint32_t k = threadIdx.x; k < cnt; k += 1024) {
    kk[k] = sel->list_key[k];
    ki[k] = sel->list_i[k];
  }
  __syncthreads();
  const uint32_t want = (uint32_t)S->n_e - sel->below - 1u;  // 0-based rank in the bucket
  for (uint32_t e = threadIdx.x; e < cnt; e += 1024) {
    uint32_t rank = 0;
    for (uint32_t f = 0; f < cnt; ++f) rank += (kk[f] < kk[e]) || (kk[f] == kk[e] && ki[f] < ki[e]);
    if (rank == want) {
      sel->thr_key = kk[e];
      sel->thr_i = ki[e];
    }
  }
}

// Occupied iff (key, i) <= the threshold pair; 64 sites of a wave form two occupation words.
__global__ void __launch_bounds__(kInitBlock) k_occ_mark(const DevSample* __restrict__ S, const OccSelect* __restrict__ sel) {
  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  const bool in = l < S->N;
  bool occupied = false;
  if (in) {
    const uint64_t key = ((const uint64_t*)S->phi)[l];
    const uint32_t b = (uint32_t)(key >> 48);
    occupied = b < sel->bucket ||
               (b == sel->bucket && (key < sel->thr_key || (key == sel->thr_key && (uint32_t)l <= sel->thr_i)));
  }
  const unsigned long long bal = __ballot(occupied);
  if ((threadIdx.x & 63) == 0 && in) {
    const int w = l >> 5;  // l is the wave's first site, a multiple of 64
    if (w < S->NW) S->occ[w] = (uint32_t)bal;
    if (w + 1 < S->NW) S->occ[w + 1] = (uint32_t)(bal >> 32);
  }
}

// FP64 energies from scratch for a large sample: eps_l = phi_l + sum_{m != l} (n_m - nu) / r_lm
// with m in index order (the definition's order, as in the per-sample init), the occupation
// and the 1/r table read from global memory; also fills the mirror and the per-block energy
// partial sums.  refresh = 1: a forced recompute (cg_refresh) that also records the largest
// change |eps_old - eps_new| per block.
__global__ void __launch_bounds__(kInitBlock) k_eps_big(const DevSample* __restrict__ samples, int refresh) {
  const DevSample& S = samples[0];
  if (refresh && !S.st->force_refresh) return;
  const int N = S.N, L = S.L, H1 = S.H + 1;
  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  __shared__ double red_sum[kInitBlock];
  __shared__ double red_max[kInitBlock];
  double contrib = 0.0, drift = 0.0;
  if (l < N) {
    const int yl = row_of(l, S.magic_L), xl = l - yl * L;
    const double q1 = 1.0 - S.nu, q0 = 0.0 - S.nu;
    const double* __restrict__ tab = S.tab64;
    const uint32_t* __restrict__ occ = S.occ;
    double acc = S.phi[l];
    for (int ym = 0; ym < L; ++ym) {
      const double* row = tab + fold(yl - ym, L) * H1;
      const int mb = ym * L;
      for (int xm = 0; xm < L; ++xm) {
        const int m = mb + xm;
        if (m == l) continue;
        const double q = ((occ[m >> 5] >> (m & 31)) & 1u) ? q1 : q0;
        acc = acc + q * row[fold(xl - xm, L)];
      }
    }
    if (refresh) drift = fabs(((const double*)S.eps)[l] - acc);
    ((double*)S.eps)[l] = acc;
    S.mirror[l] = acc;
    const bool nl = (occ[l >> 5] >> (l & 31)) & 1u;
    const double ph = S.phi[l];
    contrib = (nl ? ph : 0.0) + 0.5 * ((nl ? q1 : q0) * (acc - ph));
  }
  red_sum[threadIdx.x] = contrib;
  red_max[threadIdx.x] = drift;
  __syncthreads();
  for (int s = kInitBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red_sum[threadIdx.x] = red_sum[threadIdx.x] + red_sum[threadIdx.x + s];
      red_max[threadIdx.x] = fmax(red_max[threadIdx.x], red_max[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    S.part[blockIdx.x] = red_sum[0];
    S.part[S.nblk + blockIdx.x] = red_max[0];
  }
}

// Grid-wide barrier of one cooperative launch, a two-level counter tree: workgroup g counts
// into the counter of group g % 8 (a release add: its writes are made visible first); the
// last arriver of a group counts into the top counter, and the top's last arriver stores the
// barrier's number in the release word, which every workgroup polls with plain coherent
// loads before one acquire fence.  Counters are zeroed before each launch and only grow, so
// the n-th barrier is complete when the release word reaches n.  The wait is bounded: after
// kBarrierSpins polls a workgroup gives up and returns false, so none can wait forever.
// Per-workgroup fences, not the atomics, dominate a grid barrier on this GPU (a full fence
// at every poll costs 16.7 us per barrier at 256 workgroups, this form 5.1 us), hence one
// release at arrival and one acquire after the wait.
constexpr uint32_t kBarrierSpins = 1u << 22;
constexpr int kBarLine = 32;              // words per 128-byte line
constexpr int kBarWords = 10 * kBarLine;  // release word, top counter, 8 group counters

__device__ __forceinline__ bool grid_barrier(uint32_t* bar, uint32_t& n, uint32_t G, uint32_t* ok_sh) {
  __syncthreads();
  ++n;
  if (threadIdx.x == 0) {
    const uint32_t g = blockIdx.x;
    const uint32_t gsize = (G + 7u - (g & 7u)) / 8u;  // workgroups of this group
    const uint32_t ngroups = G < 8u ? G : 8u;
    const uint32_t old =
        __hip_atomic_fetch_add(bar + (2 + (g & 7u)) * kBarLine, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (old == n * gsize - 1u) {
      // the group is complete: take over its releases and pass them on to the top
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint32_t o2 = __hip_atomic_fetch_add(bar + kBarLine, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 == n * ngroups - 1u) __hip_atomic_store(bar, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t ok = 1u, spins = 0u;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins >= kBarrierSpins) {
        ok = 0u;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *ok_sh = ok;
  }
  __syncthreads();
  return *ok_sh != 0u;
}

__global__ void k_bar_reset(const DevSample* __restrict__ samples, int32_t sample) {
  if (threadIdx.x < 10) samples[sample].bar[threadIdx.x * kBarLine] = 0u;
  if (threadIdx.x == 0) samples[sample].st->grid_bar = 0u;
}

// LDS of the large-sample hop kernel: thresholds, 16-bit guide, 8-slot member table, FP64
// 1/r per orbit, winner records (two 16-byte words per wave), control words.
struct BigLds {
  int32_t thr, guide, vec8, td, rec, ctrl, total;
};
__host__ __device__ inline BigLds big_lds(int32_t n_orb) {
  BigLds o;
  int32_t b = 0;
  o.thr = b;   b = align16(b + n_orb * 4);
  o.guide = b; b = align16(b + kGuide16Size * 2);
  o.vec8 = b;  b = align16(b + n_orb * 64);
  o.td = b;    b = align16(b + n_orb * 8);
  o.rec = b;   b = align16(b + kMaxWaves * 32);
  o.ctrl = b;  b = align16(b + 64);
  o.total = b;
  return o;
}

struct BigLabel {
  int32_t i, j, dx;
  double td, u;
};

// Step 1 for labels base + 1 + tid U + k: the same streams and decoding as the per-sample
// kernels; the FP64 acceptance uniform (2k+1) 2^-53 with k = w2:w3 >> 12.
template <int LG, int U>
__device__ __forceinline__ void draw_big(uint64_t base, int tid, const FxConst& C, uint32_t lds0, const BigLds& lo,
                                         BigLabel (&lb)[U]) {
  constexpr int L = 1 << LG;
  const uint32_t guide = lds0 + lo.guide, thr = lds0 + lo.thr, vec8 = lds0 + lo.vec8, tdo = lds0 + lo.td;
  const int last = C.last;
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t lab = base + 1 + (uint64_t)(tid * U + k);
    uint32_t c0 = (uint32_t)lab, c1 = (uint32_t)(lab >> 32), c2 = C.sid, c3 = kTagPropose;
    philox10(c0, c1, c2, c3, C.k0, C.k1);
    const int i = (int)(c0 >> (32 - 2 * LG));
    const int o = orbit_guided(guide16_at(guide, c1), c1, thr, last);
    const uint64_t v = lds_ld<uint64_t>(vec8 + 8 * (o * 8 + (int)(c3 & 7u)));
    const int vx = (int)(uint32_t)v;
    const int dx = (int)(int16_t)(vx & 0xffff), dy = vx >> 16;
    const int xi = i & (L - 1), yi = i >> LG;
    BigLabel& b = lb[k];
    b.i = i;
    b.j = (((yi + dy) & (L - 1)) << LG) | ((xi + dx) & (L - 1));
    b.dx = dx;
    b.td = lds_ld<double>(tdo + 8 * o);
    b.u = unit52(c2, c3);
  }
}

template <int LG, int SPT, int U, int CLOCK>
__global__ void __launch_bounds__(1024) k_hops_big(const DevSample* __restrict__ samples, int32_t sample,
                                                   RunArgs ra) {
  constexpr int L = 1 << LG;
  constexpr uint32_t M = 1024u * U;
  const DevSample& S = samples[sample];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = uni((int32_t)(tid >> 6));
  const bool lead = blockIdx.x == 0;  // writes the shared results of the sample

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
  const BigLds lo = big_lds(S.n_orb);
  const uint32_t lds0 = lds_addr_of(smem);
  uint4* __restrict__ rec = (uint4*)(smem + lo.rec);
  double* __restrict__ tclock = (double*)(smem + lo.ctrl);
  uint32_t* __restrict__ theta_sh = (uint32_t*)(smem + lo.ctrl + 8);
  uint32_t* __restrict__ bar_ok = (uint32_t*)(smem + lo.ctrl + 12);
  uint32_t bar_n = 0;
  const uint32_t G = gridDim.x;

  // owned sites and their energies
  const int first_site = (int)blockIdx.x * 1024 * SPT + tid;
  double e[SPT];
  {
    const double* __restrict__ g = (const double*)S.eps;
#pragma unroll
    for (int s = 0; s < SPT; ++s) e[s] = g[first_site + 1024 * s];
  }
  for (int k = tid; k < S.n_orb; k += 1024) {
    ((uint32_t*)(smem + lo.thr))[k] = S.thr[k];
    ((double*)(smem + lo.td))[k] = S.tdo64[k];
  }
  for (int k = tid; k < kGuide16Size; k += 1024) ((uint16_t*)(smem + lo.guide))[k] = S.guide16[k];
  for (int k = tid; k < S.n_orb * 8; k += 1024) ((int2*)(smem + lo.vec8))[k] = ((const int2*)S.vec8)[k];
  if (tid < kMaxWaves) {
    rec[2 * tid] = make_uint4(0u, 0u, 0u, ~0u);
    rec[2 * tid + 1] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (tid == 0) {
    *tclock = t_start;
    *theta_sh = 0u;
  }
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
  const double* __restrict__ tab = S.tab64;
  constexpr int H1 = L / 2 + 1;
  const uint64_t s_end = uni((ra.time_mode && CLOCK == 0) ? label_at_time(t_end, Gamma) : (uint64_t)0);
  bool cached = false;
  BigLabel lb[U];
  uint32_t theta_cnt = 0;
  uint32_t round = 0;

  // Two copies of the proposals' view (occupation words and energy mirror): hop k of this
  // launch reads copy k % 2 and writes the state after the hop into the other copy, so one
  // grid barrier per hop (after the writes) suffices: the copy a hop writes was last read
  // before the previous hop's barrier.  Copy 0 (S.occ, S.mirror) holds the state at launch
  // start and again at launch end; copy 1 starts as copy 0's occupation.
  {
    const int nw = S.NW;
    for (int w = (int)blockIdx.x * 1024 + tid; w < nw; w += (int)G * 1024) S.occ2[w] = S.occ[w];
  }
  if (!grid_barrier(S.bar, bar_n, G, bar_ok)) status = -3;
  uint32_t kh = 0;           // hops executed by this launch
  int prev_i = 0, prev_j = 0;  // sites of the previous hop of this launch

  for (; status == 0;) {
    const uint32_t* __restrict__ occ = (kh & 1u) ? S.occ2 : S.occ;
    const double* __restrict__ mirror = (kh & 1u) ? S.mirror2 : S.mirror;
    uint32_t* __restrict__ occ_w = (kh & 1u) ? S.occ : S.occ2;
    double* __restrict__ mirror_w = (kh & 1u) ? S.mirror : S.mirror2;
    uint32_t found = 0u, win0 = 0u, win1 = 0u, win2 = 0u;
    uint64_t wdh = 0;
    for (;;) {
      if (!cached) {
        draw_big<LG, U>(base, tid, C, lds0, lo, lb);
        cached = true;
      }
      // step 2 against the global occupation and mirror (published by the last grid barrier)
      int first = U;
      uint32_t pub0 = 0u, pub1 = 0u, pub2 = 0u;
      double pdh = 0.0;
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const BigLabel& b = lb[k];
        const uint32_t key = (uint32_t)(tid * U + k);
        const uint32_t wi = occ[b.i >> 5], wj = occ[b.j >> 5];
        const double ei = mirror[b.i], ej = mirror[b.j];
        const bool th = (first == U) & (key >= dpos) & ((((wi >> (b.i & 31)) & ~(wj >> (b.j & 31))) & 1u) != 0u);
        const double dh0 = (ej - ei) - b.td;
        const double dH = dh0 - Ef * (double)b.dx;
        bool a = dH <= 0.0;
        if (th && !a) a = b.u < exp(dH * mrT);
        theta_cnt += th ? 1u : 0u;
        if (th && a) {
          first = k;
          pub0 = (uint32_t)b.i;
          pub1 = (uint32_t)b.j;
          pub2 = key | ((uint32_t)b.dx << 16);
          pdh = dh0;
        }
      }
      const unsigned long long bal = __ballot(first < U);
      if (bal != 0ull) {
        if (lane == __ffsll(bal) - 1) {
          const uint64_t d = (uint64_t)__double_as_longlong(pdh);
          rec[2 * wid] = make_uint4(pub0, pub1, pub2, round);
          rec[2 * wid + 1] = make_uint4((uint32_t)d, (uint32_t)(d >> 32), 0u, 0u);
        }
      }
      __syncthreads();
      uint4 r0 = make_uint4(0u, 0u, 0u, ~round), r1 = make_uint4(0u, 0u, 0u, 0u);
      if (lane < kMaxWaves) {
        r0 = rec[2 * lane];
        r1 = rec[2 * lane + 1];
      }
      const unsigned long long won = __ballot(r0.w == round);
      if (won != 0ull) {
        const int wl = __ffsll(won) - 1;
        found = 1u;
        win0 = (uint32_t)__builtin_amdgcn_readlane((int)r0.x, wl);
        win1 = (uint32_t)__builtin_amdgcn_readlane((int)r0.y, wl);
        win2 = (uint32_t)__builtin_amdgcn_readlane((int)r0.z, wl);
        wdh = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)r1.x, wl) |
              ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)r1.y, wl) << 32);
      }
      ++round;
      ++rounds;
      evaluated += M - dpos;
      if (found) break;
      base += M;
      dpos = 0;
      cached = false;
      if (base - scan0 >= ra.max_labels) {
        status = -4;  // CG_ESTALL
        break;
      }
    }
    if (!found) break;

    // step 3: every workgroup executes the same hop; workgroup 0 writes the shared state
    const int hi = (int)win0, hj = (int)win1;
    const uint32_t key = win2 & 0xffffu;
    const int hdx = (int)win2 >> 16;
    const double dh0 = __longlong_as_double((long long)wdh);
    const uint64_t q = base + 1 + key;
    const uint64_t m = q - s_last;
    s_last = q;
    dpos = key + 1;
    ++hops;
    P_ += hdx;
    H0 = H0 + dh0;
    sum_p += p_iterations(m, S.log2M);
    if (tid == 0) {
      if (lead) {
        // the written copy missed the previous hop of this launch and now takes both, in
        // order (one thread, plain read-modify-writes of the same words in program order)
        if (kh > 0) {
          occ_w[prev_i >> 5] &= ~(1u << (prev_i & 31));
          occ_w[prev_j >> 5] |= 1u << (prev_j & 31);
        }
        occ_w[hi >> 5] &= ~(1u << (hi & 31));
        occ_w[hj >> 5] |= 1u << (hj & 31);
        if (logged < log_cap) {
          S.log_label[logged] = q;
          S.log_from[logged] = hi;
          S.log_to[logged] = hj;
        }
      }
      if (CLOCK != 0) *tclock = *tclock + clock_dt(ra.clock_mode, hops, m, C.sid, C.k0, C.k1, Gamma);
    }
    logged += logged < log_cap ? 1 : 0;

    // step 3b on the owned sites, into registers and the mirror
    {
      const int xi = hi & (L - 1), yi = hi >> LG, xj = hj & (L - 1), yj = hj >> LG;
      constexpr int CH = SPT < 4 ? SPT : 4;  // sites whose table loads are in flight together
#pragma unroll
      for (int s0 = 0; s0 < SPT; s0 += CH) {
        double tj[CH], ti[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int l = first_site + 1024 * (s0 + c);
          const int x = l & (L - 1), y = l >> LG;
          tj[c] = tab[fold(y - yj, L) * H1 + fold(x - xj, L)];
          ti[c] = tab[fold(y - yi, L) * H1 + fold(x - xi, L)];
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          e[s0 + c] = e[s0 + c] + (tj[c] - ti[c]);
          mirror_w[first_site + 1024 * (s0 + c)] = e[s0 + c];
        }
      }
    }
    prev_i = hi;
    prev_j = hj;
    ++kh;
    // the written copy visible to every workgroup (the barrier also orders the Gaussian clock
    // in LDS)
    if (!grid_barrier(S.bar, bar_n, G, bar_ok)) {
      status = -3;
      break;
    }
    if (dpos == M) {
      base += M;
      dpos = 0;
      cached = false;
    }
    if (hops >= target) break;
    if (ra.time_mode) {
      if (CLOCK == 0 ? s_last >= s_end : uni(*tclock) >= t_end) break;
    }
  }

  {
    double* __restrict__ g = (double*)S.eps;
#pragma unroll
    for (int s = 0; s < SPT; ++s) g[first_site + 1024 * s] = e[s];
  }
  atomicAdd(theta_sh, theta_cnt);
  // every workgroup has read the sample state and the occupation before workgroup 0 rewrites
  // the state and copy 1's occupation (current after an odd number of hops) returns to copy 0
  if (!grid_barrier(S.bar, bar_n, G, bar_ok)) status = -3;
  if (kh & 1u) {
    const int nw = S.NW;
    for (int w = (int)blockIdx.x * 1024 + tid; w < nw; w += (int)G * 1024) S.occ[w] = S.occ2[w];
#pragma unroll
    for (int s = 0; s < SPT; ++s) S.mirror[first_site + 1024 * s] = e[s];
  }
  if (lead && tid == 0) {
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
    gs->theta_pass += *theta_sh;
    gs->logged = logged;
  }
}

}  // namespace cg
