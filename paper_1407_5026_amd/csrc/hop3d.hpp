// hop3d.hpp -- the mixed parallel-rejection step on the simple cubic lattice (FP64 form).
//
// The paper states the method for a lattice of any dimension (Eq. 1-2, section "Hopping
// conduction in the Coulomb glass") and expects it to pay off more in 3D, where N grows
// faster with L and the acceptance is lower ("Code performance").  This is that step for
// L^3 sites on a torus (minimum image), one workgroup of 1024 threads per sample:
//   * the FP64 energies, occupation bits, the 1/r table by folded (|dz|, |dy|, |dx|) and the
//     proposal tables live in LDS; thread t owns sites t + 1024 k;
//   * step 1: label s = base + 1 + t: Philox4x32-10 of (s, sample, PROPOSE); site
//     i = mulhi(w0, N), orbit: the first o with w1 < thr[o], member mulhi(w3, size_o) of the
//     orbit's displacements, acceptance uniform (w2 + 1/2) 2^-32;
//   * step 2: theta_ij, dH = ((eps_j - eps_i) - 1/r_ij) - E dx, accept when dH <= 0 or
//     u < exp(-dH / T); the wave's lowest accepting lane publishes its label, the barrier
//     makes the lowest accepting wave the round's winner (keys grow with the thread index);
//   * step 3: the executed hop's occupation, dipole, energy, clock (t = s_last / Gamma) and
//     eps_l += 1/r_lj - 1/r_li on every owned site.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "layout.hpp"

namespace cg {

constexpr int kCubeMaxL = 24;  // N = 13824: FP64 energies and the table fit the LDS
constexpr int kCubeThreads = 1024;
constexpr int kCubeSPT = (kCubeMaxL * kCubeMaxL * kCubeMaxL + kCubeThreads - 1) / kCubeThreads;

// Displacement packing: dx, dy, dz as 10-bit two's complement fields.
__host__ __device__ inline uint32_t pack3(int32_t dx, int32_t dy, int32_t dz) {
  return ((uint32_t)dx & 0x3ffu) | (((uint32_t)dy & 0x3ffu) << 10) | (((uint32_t)dz & 0x3ffu) << 20);
}
__device__ inline int32_t unpack10(uint32_t w, int shift) { return ((int32_t)(w << (22 - shift))) >> 22; }

struct CubeLds {
  int32_t eps, occ, tab, thr, orb, vec, info, tag, ctrl, total;
};

// LDS of the cubic hop kernel: energies (N doubles), occupation words, table ((H+1)^3
// doubles), thresholds, orbits (first | size << 16), packed displacements, winner records
// (16 uint4 + 16 tags), control word.
__host__ __device__ inline CubeLds cube_lds(int32_t L, int32_t n_orb, int32_t n_vec) {
  const int32_t N = L * L * L, H1 = L / 2 + 1;
  CubeLds o;
  int32_t b = 0;
  o.eps = b;  b = align16(b + N * 8);
  o.occ = b;  b = align16(b + ((N + 31) / 32) * 4);
  o.tab = b;  b = align16(b + H1 * H1 * H1 * 8);
  o.thr = b;  b = align16(b + n_orb * 4);
  o.orb = b;  b = align16(b + n_orb * 4);
  o.vec = b;  b = align16(b + n_vec * 4);
  o.info = b; b = align16(b + 16 * 16);
  o.tag = b;  b = align16(b + 16 * 4);
  o.ctrl = b; b = align16(b + 16);
  o.total = b;
  return o;
}

__device__ __forceinline__ int fold_l(int a, int L) {
  a = a < 0 ? a + L : a;
  a = a >= L ? a - L : a;
  return L - a < a ? L - a : a;
}

// Site coordinates: l = (z L + y) L + x.
__device__ __forceinline__ void coords3(int l, int L, uint32_t magic, int& x, int& y, int& z) {
  const int q = row_of(l, magic);
  x = l - q * L;
  z = row_of(q, magic);
  y = q - z * L;
}

// Step 1 for one label: site, displacement, target, 1/|d| and acceptance uniform.  The orbit
// is the smallest o < n_orb - 1 with w1 < thr[o] (else the last), found by `steps` bisection
// steps over the nondecreasing thresholds; the member is mulhi(w3, size of the orbit).
struct Cube3Label {
  int i, j, dx;
  double r, u;
};
__device__ __forceinline__ Cube3Label draw3(uint64_t lab, uint32_t k0, uint32_t k1, uint32_t sid, int L, int N,
                                            int H1, int n_orb, int steps, uint32_t magic,
                                            const uint32_t* __restrict__ thr, const uint32_t* __restrict__ orb,
                                            const uint32_t* __restrict__ vec, const double* __restrict__ tab) {
  uint32_t c0 = (uint32_t)lab, c1 = (uint32_t)(lab >> 32), c2 = sid, c3 = kTagPropose;
  philox10(c0, c1, c2, c3, k0, k1);
  Cube3Label b;
  b.i = (int)(((uint64_t)c0 * (uint64_t)N) >> 32);
  int o = 0, hi_o = n_orb - 1;  // the answer lies in [o, hi_o]
  for (int k = 0; k < steps; ++k) {
    if (o < hi_o) {
      const int mid = (o + hi_o) >> 1;
      if (c1 >= thr[mid]) o = mid + 1;
      else hi_o = mid;
    }
  }
  const uint32_t ob = orb[o];
  const uint32_t member = (uint32_t)(((uint64_t)c3 * (uint64_t)(ob >> 16)) >> 32);
  const uint32_t pv = vec[(ob & 0xffffu) + member];
  const int dx = unpack10(pv, 0), dy = unpack10(pv, 10), dz = unpack10(pv, 20);
  int x, y, z;
  coords3(b.i, L, magic, x, y, z);
  x += dx;
  y += dy;
  z += dz;
  x = x < 0 ? x + L : (x >= L ? x - L : x);
  y = y < 0 ? y + L : (y >= L ? y - L : y);
  z = z < 0 ? z + L : (z >= L ? z - L : z);
  b.j = (z * L + y) * L + x;
  b.dx = dx;
  b.r = tab[(fold_l(dz, L) * H1 + fold_l(dy, L)) * H1 + fold_l(dx, L)];
  b.u = ((double)c2 + 0.5) * 0x1p-32;
  return b;
}

// FP64 energies of L^3 sites from the definition, m in index order (grid: x over blocks
// of kInitBlock sites, y over samples); per-block partial sums of the energy (Eq. 1 field-free
// part: n_l phi_l + 1/2 (n_l - nu)(eps_l - phi_l)) and, for a forced recompute (refresh = 1),
// the largest change of an energy, for k_finalize.
__global__ void __launch_bounds__(kInitBlock) k_eps3(const DevSample* __restrict__ samples, int refresh) {
  const DevSample& S = samples[blockIdx.y];
  const int N = S.N, L = S.L, H1 = S.H + 1;
  if ((int)(blockIdx.x * kInitBlock) >= N) return;
  if (refresh && !S.st->force_refresh) return;
  extern __shared__ __align__(16) uint8_t smem[];
  uint32_t* occ = (uint32_t*)smem;
  double* tab = (double*)(smem + align16(S.NW * 4));
  for (int k = threadIdx.x; k < S.NW; k += kInitBlock) occ[k] = S.occ[k];
  for (int k = threadIdx.x; k < H1 * H1 * H1; k += kInitBlock) tab[k] = S.tab64[k];
  __shared__ double red_sum[kInitBlock];
  __shared__ double red_max[kInitBlock];
  __syncthreads();
  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  double contrib = 0.0, drift = 0.0;
  if (l < N) {
    int xl, yl, zl;
    coords3(l, L, S.magic_L, xl, yl, zl);
    const double q1 = 1.0 - S.nu, q0 = 0.0 - S.nu;
    double acc = S.phi[l];
    int m = 0;
    for (int zm = 0; zm < L; ++zm) {
      const int fz = fold_l(zl - zm, L);
      for (int ym = 0; ym < L; ++ym) {
        const double* row = tab + (fz * H1 + fold_l(yl - ym, L)) * H1;
        for (int xm = 0; xm < L; ++xm, ++m) {
          if (m == l) continue;
          const double q = ((occ[m >> 5] >> (m & 31)) & 1u) ? q1 : q0;
          acc = acc + q * row[fold_l(xl - xm, L)];
        }
      }
    }
    if (refresh) drift = fabs(((const double*)S.eps)[l] - acc);
    ((double*)S.eps)[l] = acc;
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

// SPT: sites per thread (a power of two >= ceil(N / 1024) for the batch's largest lattice);
// thread t owns sites t + 1024 s and keeps their packed coordinates in registers, and for
// SPT <= 8 also their FP64 energies (each updated energy is written to LDS for the
// proposals); at SPT = 16 the energies are updated in LDS, which keeps the kernel within its
// register budget.
template <int SPT>
__global__ void __launch_bounds__(kCubeThreads) k_hops3(const DevSample* __restrict__ samples,
                                                       const int32_t* __restrict__ order, RunArgs ra) {
  constexpr uint32_t M = kCubeThreads;
  const DevSample& S = samples[order[blockIdx.x]];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int L = S.L, N = S.N, H1 = S.H + 1, n_orb = S.n_orb;
  const uint32_t magic = S.magic_L;

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
  uint4* __restrict__ info = (uint4*)(smem + lo.info);
  uint32_t* __restrict__ tag = (uint32_t*)(smem + lo.tag);
  uint32_t* __restrict__ theta_sh = (uint32_t*)(smem + lo.ctrl);
  for (int k = tid; k < N; k += kCubeThreads) eps[k] = ((const double*)S.eps)[k];
  for (int k = tid; k < S.NW; k += kCubeThreads) occ[k] = S.occ[k];
  for (int k = tid; k < H1 * H1 * H1; k += kCubeThreads) tab[k] = S.tab64[k];
  for (int k = tid; k < n_orb; k += kCubeThreads) {
    thr[k] = S.thr[k];
    orb[k] = S.orb[k];
  }
  for (int k = tid; k < S.n_vec; k += kCubeThreads) vec[k] = (uint32_t)S.vec[k];
  if (tid < 16) tag[tid] = ~0u;  // no round carries this tag
  if (tid == 0) *theta_sh = 0u;
  // owned sites: coordinates x | y << 8 | z << 16 (L <= 24 < 256) and energies
  constexpr bool kRegE = SPT <= 8;
  double e[kRegE ? SPT : 1];
  uint32_t pc[SPT];
#pragma unroll
  for (int s = 0; s < SPT; ++s) {
    const int l = tid + kCubeThreads * s;
    if (kRegE) e[kRegE ? s : 0] = 0.0;
    pc[s] = 0u;
    if (l < N) {
      int x, y, z;
      coords3(l, L, magic, x, y, z);
      if (kRegE) e[kRegE ? s : 0] = ((const double*)S.eps)[l];
      pc[s] = (uint32_t)x | ((uint32_t)y << 8) | ((uint32_t)z << 16);
    }
  }
  // orbit search: smallest o < n_orb - 1 with w1 < thr[o], else the last orbit, by a
  // fixed number of bisection steps over the nondecreasing thresholds
  int steps = 0;
  while ((1 << steps) < n_orb) ++steps;
  __syncthreads();

  const uint32_t k0 = uni(S.seed_lo), k1 = uni(S.seed_hi), sid = uni(S.sample_id);
  const double mrT = uni(S.mrT), E = uni(S.E);
  const int64_t log_cap = uni((int64_t)S.log_cap);
  const uint64_t s_end = uni(ra.time_mode ? label_at_time(t_end, Gamma) : (uint64_t)0);
  uint32_t theta_cnt = 0, round = 0;
  bool cached = false;
  int li = 0, lj = 0, ldx = 0;
  double lu = 0.0, lr = 0.0;

  for (;;) {
    uint32_t mk = 0u, win0 = 0u, win1 = 0u, win2 = 0u, win3 = 0u;
    for (;;) {
      if (!cached) {
        // step 1 for label base + 1 + tid
        const Cube3Label d = draw3(base + 1 + (uint64_t)tid, k0, k1, sid, L, N, H1, n_orb, steps, magic, thr, orb,
                                   vec, tab);
        li = d.i;
        lj = d.j;
        ldx = d.dx;
        lr = d.r;
        lu = d.u;
        cached = true;
      }
      // step 2
      const uint32_t key = (uint32_t)tid;
      bool acc = false;
      double dH0 = 0.0;
      if (key >= dpos) {
        const bool th = ((occ[li >> 5] >> (li & 31)) & 1u) && !((occ[lj >> 5] >> (lj & 31)) & 1u);
        if (th) {
          ++theta_cnt;
          dH0 = (eps[lj] - eps[li]) - lr;
          const double dH = dH0 - E * (double)ldx;
          acc = dH <= 0.0 || lu < exp(dH * mrT);
        }
      }
      const unsigned long long bal = __ballot(acc);
      if (bal != 0ull && lane == __ffsll(bal) - 1) {
        const uint64_t bits = (uint64_t)__double_as_longlong(dH0);
        info[wid] = make_uint4((uint32_t)li | ((uint32_t)lj << 16), key | ((uint32_t)ldx << 16), (uint32_t)bits,
                               (uint32_t)(bits >> 32));
        tag[wid] = round;
      }
      __syncthreads();
      uint4 rec = make_uint4(0u, 0u, 0u, 0u);
      uint32_t rt = ~round;
      if (lane < 16) {
        rec = info[lane];
        rt = tag[lane];
      }
      const unsigned long long won = __ballot(rt == round);
      mk = won != 0ull ? 1u : 0u;
      if (won != 0ull) {
        const int wl = __ffsll(won) - 1;
        win0 = (uint32_t)__builtin_amdgcn_readlane((int)rec.x, wl);
        win1 = (uint32_t)__builtin_amdgcn_readlane((int)rec.y, wl);
        win2 = (uint32_t)__builtin_amdgcn_readlane((int)rec.z, wl);
        win3 = (uint32_t)__builtin_amdgcn_readlane((int)rec.w, wl);
      }
      ++round;
      ++rounds;
      evaluated += M - dpos;
      if (mk != 0u) break;
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
    const int hi = (int)(win0 & 0xffffu), hj = (int)(win0 >> 16);
    const uint32_t key = win1 & 0xffffu;
    const int hdx = (int)win1 >> 16;
    const double dh0 = __hiloint2double((int)win3, (int)win2);
    const uint64_t q = base + 1 + key;
    const uint64_t m = q - s_last;
    s_last = q;
    dpos = key + 1;
    ++hops;
    P_ += hdx;
    H0 = H0 + dh0;
    sum_p += p_iterations(m, S.log2M);
    if (tid == 0) {
      atomicAnd(&occ[hi >> 5], ~(1u << (hi & 31)));
      atomicOr(&occ[hj >> 5], 1u << (hj & 31));
      if (logged < log_cap) {
        S.log_label[logged] = q;
        S.log_from[logged] = hi;
        S.log_to[logged] = hj;
      }
    }
    logged += logged < log_cap ? 1 : 0;
    // step 3b on the owned sites: eps_l += 1/r_lj - 1/r_li (the table's 1/r(0) is 0); every
    // lane has read eps_i and eps_j of this round before the barrier that ended it
    {
      int xi, yi, zi, xj, yj, zj;
      coords3(hi, L, magic, xi, yi, zi);
      coords3(hj, L, magic, xj, yj, zj);
      const uint32_t h1 = (uint32_t)H1;
      // groups of 4 sites, kept apart by scheduling barriers so that the loads of one group
      // are in flight together without the whole update's loads held in registers
#pragma unroll
      for (int s0 = 0; s0 < SPT; s0 += 4) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int s = s0 + c;
          const int l = tid + kCubeThreads * s;
          if (s < SPT && l < N) {
            const int x = (int)(pc[s] & 255u), y = (int)((pc[s] >> 8) & 255u), z = (int)(pc[s] >> 16);
            const uint32_t ja =
                __umul24(__umul24((uint32_t)fold_l(z - zj, L), h1) + (uint32_t)fold_l(y - yj, L), h1) +
                (uint32_t)fold_l(x - xj, L);
            const uint32_t ib =
                __umul24(__umul24((uint32_t)fold_l(z - zi, L), h1) + (uint32_t)fold_l(y - yi, L), h1) +
                (uint32_t)fold_l(x - xi, L);
            if (kRegE) {
              double& es = e[kRegE ? s : 0];
              es = es + (tab[ja] - tab[ib]);
              eps[l] = es;
            } else {
              eps[l] = eps[l] + (tab[ja] - tab[ib]);
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
    if (dpos == M) {
      base += M;
      dpos = 0;
      cached = false;
    }
    if (hops >= target) break;
    if (ra.time_mode && s_last >= s_end) break;
  }

  atomicAdd(theta_sh, theta_cnt);
#pragma unroll
  for (int s = 0; s < SPT; ++s) {
    const int l = tid + kCubeThreads * s;
    if (l < N) ((double*)S.eps)[l] = kRegE ? e[kRegE ? s : 0] : eps[l];
  }
  __syncthreads();
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
    gs->theta_pass += *theta_sh;
    gs->logged = logged;
  }
}

}  // namespace cg
