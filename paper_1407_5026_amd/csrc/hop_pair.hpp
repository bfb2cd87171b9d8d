// hop_pair.hpp -- FP64 hop kernel of the model with pair hops: a label proposes, with
// probability `pair`, that two electrons move at once.
//
// The paper treats single-electron hops (Eq. 2) and names multi-electron hops as the
// natural extension of its parallel-rejection code (sections "Code performance" and
// "Conclusions"), without giving their rates.  The reading built here: a pair move takes
// i -> j and k -> l together, four distinct sites, at a rate of Eq. 2's form,
//   theta_ij theta_kl exp(-2 (r_ij + r_kl) / xi) min(1, exp(-dH/T)),
// restricted to compact pairs (|k - i| <= rc and |l - j| <= rc, minimum image).  dH is the
// change of Eq. 1's H: moving i -> j and then k -> l with step 3b's energy update in
// between gives
//   dH = dH_ij + dH_kl + 1/r_ik + 1/r_jl - 1/r_il - 1/r_jk,
// with dH_ij = (eps_j - eps_i) - 1/r_ij - E dx_ij as for a single hop.  As in the mixed
// algorithm, the configuration-independent tunnelling part is drawn without rejection
// and the rest is the acceptance:
//   * stream PROPOSE of label s gives i, d1 (j = i + d1) and u exactly as for a single hop;
//   * stream PAIR of s: w0 < pair 2^32 makes s a pair proposal; the partner offset e
//     (k = i + e) is uniform over the hop vectors (orbit by w1 against cumulative orbit
//     sizes, member w3 & (size - 1)); d2 (l = k + d2) follows the tunnelling tower (orbit
//     by w2, member (w3 >> 3) & (size - 1)).
// A move and its reverse (j -> i, l -> k) are proposed with equal probability, so the
// Metropolis test of the total dH keeps detailed balance with exp(-H/T).  Labels arrive at
// Gamma / (1 - pair), the rate the clock runs at.  pair = 0 is the paper's chain.
//
// Layout: the generic FP64 kernel's (energies in LDS, updated in place; wave w owns rows
// w + 16 r, lane the columns lane + 64 c), with one label per thread and chunk (1024).
// Step 3b of a pair hop applies the two single-hop updates in order, ij then kl, each
// eps_l += 1/r_lj - 1/r_li -- the order of the serial chain, so the FP64 energies and the
// executed hops equal the oracle's.
#pragma once

#include "kernels.hpp"

namespace cg {

constexpr uint32_t kTagPair = 6;

// Site reached from site `i` (row yi, column xi) by the packed displacement pv.
__device__ __forceinline__ int shift_site(int xi, int yi, int pv, int L, int& xo, int& yo) {
  const int dx = (int)(int16_t)(pv & 0xffff), dy = pv >> 16;
  int x = xi + dx, y = yi + dy;
  x += x < 0 ? L : 0;
  x -= x >= L ? L : 0;
  y += y < 0 ? L : 0;
  y -= y >= L ? L : 0;
  xo = x;
  yo = y;
  return y * L + x;
}

// One cached label: single hop (kind 0), pair hop whose sites pass the geometric filters
// (kind 1: j != l and |l - j| <= rc), or pair hop that never can (kind 2).
struct PairLabel {
  int32_t i, j, k, l;
  int32_t t1, t2, te, tjl, til, tjk;  // 1/r table indices: d1, d2, ik, jl, il, jk
  int32_t dx, kind;
  double u;
  double lam;  // -T ln u, formed when the label is drawn
};

// First orbit o with w < thr[o] (the last orbit takes the rest), from a lower bound o0.
__device__ __forceinline__ int orbit_from(const uint32_t* thr, int o0, int n_orb, uint32_t w) {
  int o = o0;
  while (o < n_orb - 1 && w >= thr[o]) ++o;
  return o;
}

template <bool TRI>
__device__ __forceinline__ int pair_tidx(int xa, int ya, int xb, int yb, int L, int H1) {
  return tidx<TRI>(fold(ya - yb, L), fold(xa - xb, L), H1);
}

// Step 1 of label `lab`: the single-hop draw and, for a pair proposal, the partner and
// second hop.
template <bool TRI>
__device__ __forceinline__ void draw_pair_label(uint64_t lab, const DevSample& S, const uint8_t* guide,
                                                const uint32_t* thr, const uint32_t* thr_u, const uint32_t* orb,
                                                const int32_t* vec, PairLabel& b) {
  const int L = S.L, N = S.N, H1 = S.H + 1, n_orb = S.n_orb;
  uint32_t c0 = (uint32_t)lab, c1 = (uint32_t)(lab >> 32), c2 = S.sample_id, c3 = kTagPropose;
  philox10(c0, c1, c2, c3, S.seed_lo, S.seed_hi);
  const int i = (int)__umulhi(c0, (uint32_t)N);
  const int o1 = orbit_from(thr, guide[c1 >> (32 - kGuideBits)], n_orb, c1);
  const uint32_t ob1 = orb[o1];
  const int pv1 = vec[(int)(ob1 & 0xffffu) + (int)(c3 & (ob1 >> 16))];
  const int yi = row_of(i, S.magic_L), xi = i - yi * L;
  int xj, yj;
  const int j = shift_site(xi, yi, pv1, L, xj, yj);
  const int dx1 = (int)(int16_t)(pv1 & 0xffff), dy1 = pv1 >> 16;
  b.i = i;
  b.j = j;
  b.k = i;
  b.l = j;
  b.t1 = tidx<TRI>(dy1 < 0 ? -dy1 : dy1, dx1 < 0 ? -dx1 : dx1, H1);
  b.t2 = b.te = b.tjl = b.til = b.tjk = 0;
  b.dx = dx1;
  b.kind = 0;
  b.u = accept_uniform<double>(c2, c3);
  b.lam = -S.T * log(b.u);
  if (S.thr_pair == 0u) return;
  uint32_t p0 = (uint32_t)lab, p1 = (uint32_t)(lab >> 32), p2 = S.sample_id, p3 = kTagPair;
  philox10(p0, p1, p2, p3, S.seed_lo, S.seed_hi);
  if (!(p0 < S.thr_pair)) return;
  // partner offset e: uniform over the hop vectors
  int oe = 0;
  while (oe < n_orb - 1 && p1 >= thr_u[oe]) ++oe;
  const uint32_t obe = orb[oe];
  const int pve = vec[(int)(obe & 0xffffu) + (int)(p3 & (obe >> 16))];
  // second hop d2: the tunnelling tower
  const int o2 = orbit_from(thr, guide[p2 >> (32 - kGuideBits)], n_orb, p2);
  const uint32_t ob2 = orb[o2];
  const int pv2 = vec[(int)(ob2 & 0xffffu) + (int)((p3 >> 3) & (ob2 >> 16))];
  int xk, yk, xl, yl;
  const int k = shift_site(xi, yi, pve, L, xk, yk);
  const int l = shift_site(xk, yk, pv2, L, xl, yl);
  const int ex = (int)(int16_t)(pve & 0xffff), ey = pve >> 16;
  const int dx2 = (int)(int16_t)(pv2 & 0xffff), dy2 = pv2 >> 16;
  const int fx = fold(xl - xj, L), fy = fold(yl - yj, L);
  b.k = k;
  b.l = l;
  b.t2 = tidx<TRI>(dy2 < 0 ? -dy2 : dy2, dx2 < 0 ? -dx2 : dx2, H1);
  b.te = tidx<TRI>(ey < 0 ? -ey : ey, ex < 0 ? -ex : ex, H1);
  b.tjl = tidx<TRI>(fy, fx, H1);
  b.til = pair_tidx<TRI>(xi, yi, xl, yl, L, H1);
  b.tjk = pair_tidx<TRI>(xj, yj, xk, yk, L, H1);
  b.dx = dx1 + dx2;
  b.kind = (j != l && fx * fx + fy * fy <= S.pair_r2) ? 1 : 2;
}

// Winner record of a wave: its lowest accepting lane's label.
struct PairInfo {
  uint32_t key;
  int32_t i, j, k, l, dx;
  double dH0;
};

template <bool TRI, int NC, int RPW, bool EXACT>
__global__ void __launch_bounds__(1024) k_hops_pair(const DevSample* __restrict__ samples,
                                                    const int32_t* __restrict__ order, RunArgs ra) {
  constexpr int NW = 16;
  const DevSample& S = samples[order[blockIdx.x]];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);

  uint64_t hops = uni(gs->hops);
  uint64_t s_last = uni(gs->s_last);
  uint64_t done = uni(gs->s_scan);
  const uint64_t target = uni(gs->hop_target);
  const uint64_t scan0 = uni(gs->call_scan0);
  const double t_end = uni(gs->t_end);
  const double t_start = uni(gs->t);
  {
    const bool idle = uni(gs->status) != 0 || hops >= target || (ra.time_mode && t_start >= t_end);
    if (idle) return;
  }
  int64_t P = uni(gs->P);
  double H0 = uni(gs->H0);
  uint64_t sum_p = uni(gs->sum_p), rounds = uni(gs->rounds), evaluated = uni(gs->evaluated);
  int64_t logged = uni(gs->logged);
  int32_t status = 0;

  const int L = S.L, N = S.N, H1 = S.H + 1, n_orb = S.n_orb;
  const uint32_t magic = S.magic_L;
  extern __shared__ __align__(16) uint8_t smem[];
  const PairLds lo = pair_lds(N, S.NW, S.ntab, S.n_vec, n_orb);
  double* __restrict__ es = (double*)(smem + lo.h.eps);
  uint32_t* __restrict__ occ = (uint32_t*)(smem + lo.h.occ);
  double* __restrict__ tab = (double*)(smem + lo.h.tab);
  int32_t* __restrict__ vec = (int32_t*)(smem + lo.h.vec);
  uint32_t* __restrict__ thr = (uint32_t*)(smem + lo.h.thr);
  uint32_t* __restrict__ orb = (uint32_t*)(smem + lo.h.orb);
  uint8_t* __restrict__ guide = smem + lo.h.guide;
  HopShared* __restrict__ sh = (HopShared*)(smem + lo.h.ctrl);
  PairInfo* __restrict__ info = (PairInfo*)(smem + lo.h.info);
  uint32_t* __restrict__ thr_u = (uint32_t*)(smem + lo.thr_u);

  {
    const double* __restrict__ g = (const double*)S.eps;
    for (int k = tid; k < N; k += 1024) es[k] = g[k];
    const double* gt = (const double*)S.tabk;
    for (int k = tid; k < S.ntab; k += 1024) tab[k] = gt[k];
  }
  for (int k = tid; k < S.NW; k += 1024) occ[k] = S.occ[k];
  for (int k = tid; k < S.n_vec; k += 1024) vec[k] = S.vec[k];
  for (int k = tid; k < n_orb; k += 1024) {
    thr[k] = S.thr[k];
    orb[k] = S.orb[k];
    thr_u[k] = S.thr_u[k];
  }
  for (int k = tid; k < kGuideSize; k += 1024) guide[k] = S.guide[k];
  if (tid == 0) {
    sh->best[0] = sh->best[1] = sh->best[2] = ~0ull;
    sh->theta = 0u;
    sh->t = t_start;
  }
  __syncthreads();

  const uint32_t k0 = S.seed_lo, k1 = S.seed_hi, sid = S.sample_id;
  constexpr uint64_t M = 1024;
  const uint64_t s_end = uni((ra.time_mode && ra.clock_mode == 0) ? label_at_time(t_end, S.Gamma) : (uint64_t)0);
  const double Ef = S.E;
  uint64_t base = done;  // current chunk: labels base+1 .. base+M
  bool cached = false;
  PairLabel lb;
  uint32_t theta_cnt = 0;
  uint32_t it = 0;

  for (;;) {
    if (!cached) {
      draw_pair_label<TRI>(base + 1 + (uint64_t)tid, S, guide, thr, thr_u, orb, vec, lb);
      cached = true;
    }

    // step 2 for this lane's label if it is still undecided
    const uint64_t active = base + M - done;
    const uint64_t lab = base + 1 + (uint64_t)tid;
    bool acc = false;
    double dh0 = 0.0;
    if (lab > done && lb.kind != 2) {
      const int i = lb.i, j = lb.j;
      const uint32_t ni = (occ[i >> 5] >> (i & 31)) & 1u, nj = (occ[j >> 5] >> (j & 31)) & 1u;
      const double ei = es[i], ej = es[j], t1 = tab[lb.t1];
      bool th = ni == 1u && nj == 0u;
      dh0 = (ej - ei) - t1;
      if (lb.kind == 1) {
        const int k = lb.k, l = lb.l;
        const uint32_t nk = (occ[k >> 5] >> (k & 31)) & 1u, nl = (occ[l >> 5] >> (l & 31)) & 1u;
        const double ek = es[k], el = es[l];
        th = th && nk == 1u && nl == 0u;
        const double h2 = (el - ek) - tab[lb.t2];
        const double hint = ((tab[lb.te] + tab[lb.tjl]) - tab[lb.til]) - tab[lb.tjk];
        dh0 = (dh0 + h2) + hint;
      }
      const double dH = dh0 - Ef * (double)lb.dx;
      // Metropolis as dH < lam = -T ln u: beyond 1e-12 (T + lam) of the threshold the
      // comparison decides as the exponential test does (the roundings of lam, of dH/T and of
      // the exponential move it by a few units of 1e-16 (T + lam)); nearer to it the lane
      // evaluates the exponential test itself (a branch that practically no wave takes)
      const double gap = dH - lb.lam;
      bool a = gap < 0.0;
      const bool near = fabs(gap) <= 1e-12 * (S.T + lb.lam);
      if (__ballot(near) != 0ull) {
        asm volatile("" ::: "memory");  // a real branch: keeps this path from being speculated
        if (near) a = metropolis_nb(dH, lb.u, true, S);
      }
      acc = th && a;
      theta_cnt += th ? 1u : 0u;
    }
    // the wave's lowest accepting lane publishes its label; the round's minimum key over
    // the workgroup (one 64-bit LDS min) is the lowest accepted label
    const unsigned long long bal = __ballot(acc);
    if (bal != 0ull) {
      const int wl = __ffsll(bal) - 1;
      if (lane == wl) {
        PairInfo h;
        h.key = (uint32_t)tid;
        h.i = lb.i;
        h.j = lb.j;
        h.k = lb.kind == 1 ? lb.k : -1;
        h.l = lb.l;
        h.dx = lb.dx;
        h.dH0 = dh0;
        info[wid] = h;
        atomicMin(&sh->best[it % 3], (uint64_t)h.key << 32);
      }
    }
    if (tid == 0) sh->best[(it + 1) % 3] = ~0ull;
    __syncthreads();
    const uint64_t best = uni(sh->best[it % 3]);
    ++it;
    ++rounds;
    evaluated += active;

    if (best == ~0ull) {
      done = base + M;
      base = done;
      cached = false;
      if (done - scan0 >= ra.max_labels) {
        status = -4;  // CG_ESTALL
        break;
      }
      continue;
    }

    // step 3: execute the lowest accepted label (both moves of a pair)
    const uint32_t key = (uint32_t)(best >> 32);
    const PairInfo& w = info[key >> 6];  // written by the winning wave
    const int hi = uni(w.i), hj = uni(w.j), hk = uni(w.k), hl = uni(w.l), hdx = uni(w.dx);
    const double hdh0 = uni(w.dH0);
    const bool two = hk >= 0;
    const uint64_t q = base + 1 + (uint64_t)key;
    const uint64_t m = q - s_last;
    s_last = q;
    done = q;
    ++hops;
    P += hdx;
    H0 = H0 + hdh0;
    sum_p += p_iterations(m, S.log2M);
    if (tid == 0) {
      atomicAnd(&occ[hi >> 5], ~(1u << (hi & 31)));
      atomicOr(&occ[hj >> 5], 1u << (hj & 31));
      if (two) {
        atomicAnd(&occ[hk >> 5], ~(1u << (hk & 31)));
        atomicOr(&occ[hl >> 5], 1u << (hl & 31));
      }
      int64_t e = logged;
      if (e < S.log_cap) {
        S.log_label[e] = q;
        S.log_from[e] = hi;
        S.log_to[e] = hj;
        ++e;
      }
      if (two && e < S.log_cap) {
        S.log_label[e] = q;
        S.log_from[e] = hk;
        S.log_to[e] = hl;
      }
      if (ra.clock_mode != 0) sh->t = sh->t + clock_dt(ra.clock_mode, hops, m, sid, k0, k1, S.Gamma);
    }
    if (logged < S.log_cap) ++logged;
    if (two && logged < S.log_cap) ++logged;

    // step 3b on the owned sites: eps += 1/r_lj - 1/r_li, then (pair) += 1/r_ll' - 1/r_lk
    {
      const int yi = row_of(hi, magic), xi = hi - yi * L;
      const int yj = row_of(hj, magic), xj = hj - yj * L;
      const int kk = two ? hk : hi, ll = two ? hl : hj;
      const int yk = row_of(kk, magic), xk = kk - yk * L;
      const int yl = row_of(ll, magic), xl = ll - yl * L;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int y = wid + NW * r;
        if (!EXACT && y >= L) continue;
        const int ayj = fold(y - yj, L), ayi = fold(y - yi, L), ayl = fold(y - yl, L), ayk = fold(y - yk, L);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int x = lane + 64 * c;
          if (!EXACT && x >= L) continue;
          const int s = y * L + x;
          double e = es[s];
          e = e + (tab[tidx<TRI>(ayj, fold(x - xj, L), H1)] - tab[tidx<TRI>(ayi, fold(x - xi, L), H1)]);
          if (two) e = e + (tab[tidx<TRI>(ayl, fold(x - xl, L), H1)] - tab[tidx<TRI>(ayk, fold(x - xk, L), H1)]);
          es[s] = e;
        }
      }
    }
    __syncthreads();
    if (done == base + M) {
      base = done;
      cached = false;
    }
    if (hops >= target) break;
    if (ra.time_mode) {
      if (ra.clock_mode == 0 ? s_last >= s_end : uni(sh->t) >= t_end) break;
    }
  }

  atomicAdd(&sh->theta, theta_cnt);
  __syncthreads();
  {
    double* __restrict__ g = (double*)S.eps;
    for (int k = tid; k < N; k += 1024) g[k] = es[k];
  }
  for (int k = tid; k < S.NW; k += 1024) S.occ[k] = occ[k];
  if (tid == 0) {
    gs->hops = hops;
    gs->s_last = s_last;
    gs->s_scan = done;
    gs->P = P;
    gs->t = ra.clock_mode == 0 ? (double)s_last / S.Gamma : sh->t;
    gs->H0 = H0;
    gs->status = status;
    gs->sum_p = sum_p;
    gs->rounds = rounds;
    gs->evaluated = evaluated;
    gs->theta_pass += sh->theta;
    gs->logged = logged;
  }
}

}  // namespace cg
