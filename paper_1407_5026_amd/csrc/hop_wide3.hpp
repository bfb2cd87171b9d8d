// hop_wide3.hpp -- one simple cubic sample on G workgroups, the parallel-rejection width spread
// over the GPU (FP64 form, deterministic clock, L <= 24).
//
// The cubic counterpart of the label-parallel kernel: the paper expects the method to pay
// off more in 3D because the acceptance is lower there ("Code performance"), and a round of
// 1024 labels on one workgroup then takes many rounds per hop.  Every workgroup keeps a
// replica of the sample in LDS (the layout of the one-workgroup cubic kernel) and evaluates
// its own 1024 labels of each round of G x 1024: label base + 1 + g 1024 + t.  The round's
// lowest accepted label is a global minimum handed out by the round barrier of the
// label-parallel kernel; every workgroup recomputes that label's proposal and executes the
// hop on its replica.  Labels, streams and FP64 arithmetic are those of the one-workgroup
// cubic kernel, so the hops equal the oracle's for every G.
#pragma once

#include "hop3d.hpp"
#include "hop_wide.hpp"

namespace cg {

template <int SPT>
__global__ void __launch_bounds__(kCubeThreads) k_hops_wide3(const DevSample* __restrict__ samples, int32_t sample,
                                                            RunArgs ra) {
  constexpr uint32_t Mw = kCubeThreads;  // labels per workgroup and round
  const DevSample& S = samples[sample];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int L = S.L, N = S.N, H1 = S.H + 1, n_orb = S.n_orb;
  const uint32_t magic = S.magic_L;
  const uint32_t G = gridDim.x;
  const uint32_t MC = G * Mw;
  const uint32_t koff = blockIdx.x * Mw;
  const bool lead = blockIdx.x == 0;

  uint64_t hops = uni(gs->hops);
  uint64_t s_last = uni(gs->s_last);
  const uint64_t target = uni(gs->hop_target);
  const uint64_t scan0 = uni(gs->call_scan0);
  const double t_end = uni(gs->t_end);
  const double Gamma = uni(S.Gamma);
  if (uni(gs->status) != 0 || hops >= target || (ra.time_mode && (double)s_last / Gamma >= t_end)) return;
  uint64_t base = uni(gs->s_scan);
  uint32_t dpos = 0;
  int64_t P_ = uni(gs->P);
  double H0 = uni(gs->H0);
  uint64_t sum_p = uni(gs->sum_p), rounds = uni(gs->rounds), evaluated = uni(gs->evaluated);
  int64_t logged = uni(gs->logged);
  int32_t status = 0;

  extern __shared__ __align__(16) uint8_t smem[];
  const CubeLds lo = cube_lds(L, n_orb, S.n_vec);
  double* __restrict__ eps = (double*)(smem + lo.eps);
  uint32_t* __restrict__ occ = (uint32_t*)(smem + lo.occ);
  double* __restrict__ tab = (double*)(smem + lo.tab);
  uint32_t* __restrict__ thr = (uint32_t*)(smem + lo.thr);
  uint32_t* __restrict__ orb = (uint32_t*)(smem + lo.orb);
  uint32_t* __restrict__ vec = (uint32_t*)(smem + lo.vec);
  uint32_t* __restrict__ keys = (uint32_t*)(smem + lo.info);
  uint32_t* __restrict__ tag = (uint32_t*)(smem + lo.tag);
  uint32_t* __restrict__ bar_ok = (uint32_t*)(smem + lo.ctrl + 4);
  uint32_t* __restrict__ win_sh = (uint32_t*)(smem + lo.ctrl + 8);
  uint32_t* __restrict__ slot = S.bar + kBarWords;
  uint32_t bar_n = 0;
  for (int k = tid; k < N; k += kCubeThreads) eps[k] = ((const double*)S.eps)[k];
  for (int k = tid; k < S.NW; k += kCubeThreads) occ[k] = S.occ[k];
  for (int k = tid; k < H1 * H1 * H1; k += kCubeThreads) tab[k] = S.tab64[k];
  for (int k = tid; k < n_orb; k += kCubeThreads) {
    thr[k] = S.thr[k];
    orb[k] = S.orb[k];
  }
  for (int k = tid; k < S.n_vec; k += kCubeThreads) vec[k] = (uint32_t)S.vec[k];
  if (tid < 16) tag[tid] = ~0u;  // no round carries this tag
  // replica sites t + 1024 s of this thread: coordinates x | y << 8 | z << 16
  uint32_t pc[SPT];
#pragma unroll
  for (int s = 0; s < SPT; ++s) {
    const int l = tid + kCubeThreads * s;
    pc[s] = 0u;
    if (l < N) {
      int x, y, z;
      coords3(l, L, magic, x, y, z);
      pc[s] = (uint32_t)x | ((uint32_t)y << 8) | ((uint32_t)z << 16);
    }
  }
  int steps = 0;
  while ((1 << steps) < n_orb) ++steps;
  __syncthreads();

  const uint32_t k0 = uni(S.seed_lo), k1 = uni(S.seed_hi), sid = uni(S.sample_id);
  const double mrT = uni(S.mrT), E = uni(S.E);
  const int64_t log_cap = uni((int64_t)S.log_cap);
  const uint64_t s_end = uni(ra.time_mode ? label_at_time(t_end, Gamma) : (uint64_t)0);
  uint32_t theta_cnt = 0, round = 0;
  bool cached = false;
  Cube3Label lb;
  lb.i = lb.j = lb.dx = 0;
  lb.r = lb.u = 0.0;

  for (;;) {
    uint32_t win = ~0u;
    for (;;) {
      if (!cached) {
        lb = draw3(base + 1 + koff + (uint64_t)tid, k0, k1, sid, L, N, H1, n_orb, steps, magic, thr, orb, vec, tab);
        cached = true;
      }
      // step 2 for this workgroup's label of the round
      const uint32_t key = koff + (uint32_t)tid;
      bool acc = false;
      if (key >= dpos) {
        const bool th = ((occ[lb.i >> 5] >> (lb.i & 31)) & 1u) && !((occ[lb.j >> 5] >> (lb.j & 31)) & 1u);
        if (th) {
          ++theta_cnt;
          const double dH = ((eps[lb.j] - eps[lb.i]) - lb.r) - E * (double)lb.dx;
          acc = dH <= 0.0 || lb.u < exp(dH * mrT);
        }
      }
      // the lowest accepted key of the workgroup (keys grow with the thread index), then the
      // round's global minimum
      const unsigned long long bal = __ballot(acc);
      if (bal != 0ull && lane == __ffsll(bal) - 1) {
        keys[4 * wid] = key;
        tag[wid] = round;
      }
      if (lead && tid == 0)
        __hip_atomic_store(slot + ((round + 2u) % kWideSlots) * kBarLine, ~0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      if (wid == 0) {
        uint32_t rt = ~round, rk = ~0u;
        if (lane < 16) {
          rt = tag[lane];
          rk = keys[4 * lane];
        }
        const unsigned long long won = __ballot(rt == round);
        if (won != 0ull && lane == __ffsll(won) - 1)
          __hip_atomic_fetch_min(slot + (round % kWideSlots) * kBarLine, rk, __ATOMIC_RELAXED,
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
      base += MC;
      dpos = 0;
      cached = false;
      if (base - scan0 >= ra.max_labels) {
        status = -4;  // CG_ESTALL
        break;
      }
    }
    if (win == ~0u) break;

    // step 3: the winning label's proposal, recomputed on every replica
    const uint64_t q = base + 1 + win;
    const Cube3Label h = draw3(q, k0, k1, sid, L, N, H1, n_orb, steps, magic, thr, orb, vec, tab);
    const int hi = uni(h.i), hj = uni(h.j);
    const double dh0 = (eps[hj] - eps[hi]) - h.r;
    const uint64_t m = q - s_last;
    s_last = q;
    dpos = win + 1;
    ++hops;
    P_ += uni(h.dx);
    H0 = H0 + dh0;
    sum_p += p_iterations(m, S.log2M);
    const bool log_it = logged < log_cap;
    const int64_t log_at = logged;
    logged += log_it ? 1 : 0;
    // every lane has read eps_i and eps_j before they change
    __syncthreads();
    if (tid == 0) {
      occ[hi >> 5] &= ~(1u << (hi & 31));
      occ[hj >> 5] |= 1u << (hj & 31);
      if (lead && log_it) {
        S.log_label[log_at] = q;
        S.log_from[log_at] = hi;
        S.log_to[log_at] = hj;
      }
    }
    // step 3b on the replica: eps_l += 1/r_lj - 1/r_li (the table's 1/r(0) is 0)
    {
      int xi, yi, zi, xj, yj, zj;
      coords3(hi, L, magic, xi, yi, zi);
      coords3(hj, L, magic, xj, yj, zj);
      const uint32_t h1 = (uint32_t)H1;
#pragma unroll
      for (int s = 0; s < SPT; ++s) {
        const int l = tid + kCubeThreads * s;
        if (l < N) {
          const int x = (int)(pc[s] & 255u), y = (int)((pc[s] >> 8) & 255u), z = (int)(pc[s] >> 16);
          const uint32_t ja =
              __umul24(__umul24((uint32_t)fold_l(z - zj, L), h1) + (uint32_t)fold_l(y - yj, L), h1) +
              (uint32_t)fold_l(x - xj, L);
          const uint32_t ib =
              __umul24(__umul24((uint32_t)fold_l(z - zi, L), h1) + (uint32_t)fold_l(y - yi, L), h1) +
              (uint32_t)fold_l(x - xi, L);
          eps[l] = eps[l] + (tab[ja] - tab[ib]);
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
    if (ra.time_mode && s_last >= s_end) break;
  }

  if (theta_cnt != 0u) atomicAdd((unsigned long long*)&gs->theta_pass, (unsigned long long)theta_cnt);
  if (lead) {
    for (int k = tid; k < N; k += kCubeThreads) ((double*)S.eps)[k] = eps[k];
    for (int k = tid; k < S.NW; k += kCubeThreads) S.occ[k] = occ[k];
    if (tid == 0) {
      gs->hops = hops;
      gs->s_last = s_last;
      gs->s_scan = base + dpos;
      gs->P = P_;
      gs->t = (double)s_last / Gamma;
      gs->H0 = H0;
      gs->status = status;
      gs->sum_p = sum_p;
      gs->rounds = rounds;
      gs->evaluated = evaluated;
      gs->logged = logged;
    }
  }
}

}  // namespace cg
