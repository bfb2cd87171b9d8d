// kernels.hpp -- gfx950 kernels of the parallel-rejection KMC (one workgroup per sample).
//
// k_hops runs the mixed parallel-rejection algorithm (section "Hopping conduction in the
// Coulomb glass", steps 1, 2, 3a-3c) entirely inside one persistent workgroup per sample,
// with the local energies, occupation bits, the 1/r table and the proposal tower resident
// in LDS:
//   P  each lane owns U consecutive labels of the current chunk of M = blockDim*U labels;
//      Philox4x32-10 of (label, sample) gives the site, the displacement orbit/member and
//      the acceptance uniform, computed once per label and kept in registers;
//   R  lanes test theta and Metropolis for their labels above the last decided one; a
//      64-bit wave ballot gives each wave's lowest accepting lane, an LDS bitmask of waves
//      (one ds_or per wave, one barrier) gives the workgroup's lowest accepted label;
//   X  the winning hop is executed (bits, dipole, energy total, clock, log);
//   U  every site's energy gets 1/r_lj - 1/r_li from the LDS table, one lattice row per
//      wave so that the row terms are wave-uniform; then a barrier.
// Labels after the executed one stay in registers and are re-evaluated against the new
// configuration in the next round, so every label is drawn once and the executed hop
// sequence is that of the serial chain for any M.
#pragma once

#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace cg {

// ---------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64-bit
// products of counter words 0 and 2, outputs permuted and xored with the key, key
// bumped by the Weyl increments between rounds.
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
}

enum : uint32_t { kTagPropose = 0, kTagOcc = 1, kTagPhi = 2, kTagClock = 3 };

// (2k+1) 2^-53 with k the 52 bits hi:lo>>12 -- uniform in (0,1), exact in FP64.
__device__ __forceinline__ double unit52(uint32_t hi, uint32_t lo) {
  const uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
  return (double)(2u * k + 1u) * 0x1p-53;
}

template <typename R> __device__ __forceinline__ R accept_uniform(uint32_t w2, uint32_t w3);
template <> __device__ __forceinline__ double accept_uniform<double>(uint32_t w2, uint32_t w3) {
  return unit52(w2, w3);
}
// FP32 form: the top 23 bits of w2, (2k+1) 2^-24, exact in FP32.
template <> __device__ __forceinline__ float accept_uniform<float>(uint32_t w2, uint32_t) {
  return (float)(2u * (w2 >> 9) + 1u) * 0x1p-24f;
}

// Metropolis factor of Eq. 2: accept iff dH <= 0 or u < exp(-dH/T).
__device__ __forceinline__ bool metropolis(double dH, double u, const DevSample& S) {
  return dH <= 0.0 || u < exp(-dH / S.T);
}
__device__ __forceinline__ bool metropolis(float dH, float u, const DevSample& S) {
  return dH <= 0.0f || u < __expf(-dH * S.invT32);
}
__device__ __forceinline__ double field(const DevSample& S, double) { return S.E; }
__device__ __forceinline__ float field(const DevSample& S, float) { return S.E32; }

// Minimum-image |d| for d in (-L, L).
__device__ __forceinline__ int fold(int d, int L) {
  const int a = d < 0 ? -d : d;
  const int b = L - a;
  return a < b ? a : b;
}

template <bool TRI>
__device__ __forceinline__ int tidx(int ady, int adx, int H1) {
  if (TRI) {
    const int a = ady > adx ? ady : adx;
    const int b = ady > adx ? adx : ady;
    return ((a * (a + 1)) >> 1) + b;
  }
  return ady * H1 + adx;
}

__device__ __forceinline__ int row_of(int i, uint32_t magic) { return (int)__umulhi((uint32_t)i, magic); }

struct HopInfo {
  uint32_t key;  // position of the label in the chunk: tid * U + k
  int32_t i, j, v;
  double dH0;    // (eps_j - eps_i) - 1/r_ij of the executed hop
  int32_t pad[2];
};
static_assert(sizeof(HopInfo) == kInfoBytes, "HopInfo size");

// Step 3b on the LDS-resident energies: eps_l += 1/r_lj - 1/r_li for every l.  Lane
// handles columns lane + 64 c (outer loop), wave w rows w, w + nw, ... (inner loop), so the
// folded column separations are per-lane constants of the inner loop and the folded row
// separations are wave-uniform.
template <typename R, bool TRI>
__device__ __forceinline__ void update_energies(R* __restrict__ eps, const R* __restrict__ tab,
                                                int i, int j, int L, int H1, uint32_t magic,
                                                int lane, int wid, int nw) {
  const int yi = row_of(i, magic), xi = i - yi * L;
  const int yj = row_of(j, magic), xj = j - yj * L;
  for (int x0 = 0; x0 < L; x0 += 64) {
    const int x = x0 + lane;
    if (x < L) {
      const int axi = fold(x - xi, L), axj = fold(x - xj, L);
      for (int y = wid; y < L; y += nw) {
        const int ayi = fold(y - yi, L), ayj = fold(y - yj, L);
        const R tj = tab[tidx<TRI>(ayj, axj, H1)];
        const R ti = tab[tidx<TRI>(ayi, axi, H1)];
        R* __restrict__ e = eps + y * L + x;
        *e = *e + (tj - ti);
      }
    }
  }
}

// Per-sample scalars in LDS: written by thread 0 only, read by all after a barrier.
struct HopShared {
  uint32_t wmask[3];   // per-round bitmask of waves holding an accepted label
  uint32_t theta;      // theta-pass count (summed at exit)
  double t;            // clock after the last executed hop
  int64_t P;
  double H0;
  uint64_t sum_p, rounds, evaluated;
  int64_t logged;
};

template <typename R, int U, bool TRI>
__global__ void __launch_bounds__(1024) k_hops(const DevSample* __restrict__ samples,
                                               const int32_t* __restrict__ order, RunArgs ra) {
  const DevSample& S = samples[order[blockIdx.x]];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wid = tid >> 6, nw = nthr >> 6;

  {
    const bool idle = gs->status != 0 || gs->hops >= gs->hop_target ||
                      (ra.time_mode && gs->t >= gs->t_end) || (ra.K > 0 && gs->since_refresh >= ra.K);
    if (idle) return;
  }
  uint64_t hops = gs->hops;
  uint64_t s_last = gs->s_last;
  uint64_t done = gs->s_scan;
  int32_t since = gs->since_refresh;
  int32_t status = 0;

  const int L = S.L, N = S.N, H1 = S.H + 1, n_orb = S.n_orb;
  const uint32_t magic = S.magic_L;
  extern __shared__ __align__(16) uint8_t smem[];
  const HopLds lo = hop_lds(N, S.NW, S.ntab, S.n_vec, n_orb, (int32_t)sizeof(R));
  R* __restrict__ eps = (R*)(smem + lo.eps);
  uint32_t* __restrict__ occ = (uint32_t*)(smem + lo.occ);
  R* __restrict__ tab = (R*)(smem + lo.tab);
  int32_t* __restrict__ vec = (int32_t*)(smem + lo.vec);
  uint32_t* __restrict__ thr = (uint32_t*)(smem + lo.thr);
  uint32_t* __restrict__ orb = (uint32_t*)(smem + lo.orb);
  uint8_t* __restrict__ guide = smem + lo.guide;
  HopShared* __restrict__ sh = (HopShared*)(smem + lo.ctrl);
  HopInfo* __restrict__ info = (HopInfo*)(smem + lo.info);

  {
    const R* g = (const R*)S.eps;
    for (int k = tid; k < N; k += nthr) eps[k] = g[k];
    const R* gt = (const R*)S.tabk;
    for (int k = tid; k < S.ntab; k += nthr) tab[k] = gt[k];
  }
  for (int k = tid; k < S.NW; k += nthr) occ[k] = S.occ[k];
  for (int k = tid; k < S.n_vec; k += nthr) vec[k] = S.vec[k];
  for (int k = tid; k < n_orb; k += nthr) {
    thr[k] = S.thr[k];
    orb[k] = S.orb[k];
  }
  for (int k = tid; k < kGuideSize; k += nthr) guide[k] = S.guide[k];
  if (tid == 0) {
    sh->wmask[0] = sh->wmask[1] = sh->wmask[2] = 0u;
    sh->theta = 0u;
    sh->t = gs->t;
    sh->P = gs->P;
    sh->H0 = gs->H0;
    sh->sum_p = gs->sum_p;
    sh->rounds = gs->rounds;
    sh->evaluated = gs->evaluated;
    sh->logged = gs->logged;
  }
  __syncthreads();

  const uint32_t k0 = S.seed_lo, k1 = S.seed_hi, sid = S.sample_id;
  const uint64_t M = (uint64_t)ra.M;
  const R Ef = field(S, R(0));
  uint64_t base = done;  // current chunk: labels base+1 .. base+M
  bool cached = false;
  int ci[U], cj[U], cv[U];
  R cu[U];
  uint32_t theta_cnt = 0;
  uint32_t it = 0;

  for (;;) {
    if (!cached) {
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const uint64_t lab = base + 1 + (uint64_t)(tid * U + k);
        uint32_t c0 = (uint32_t)lab, c1 = (uint32_t)(lab >> 32), c2 = sid, c3 = kTagPropose;
        philox10(c0, c1, c2, c3, k0, k1);
        const int i = (int)__umulhi(c0, (uint32_t)N);
        int o = guide[c1 >> (32 - kGuideBits)];
        while (o < n_orb - 1 && c1 >= thr[o]) ++o;
        const uint32_t ob = orb[o];
        const int v = (int)(ob & 0xffffu) + (int)(c3 & (ob >> 16));
        const int pv = vec[v];
        const int dx = (int)(int16_t)(pv & 0xffff), dy = pv >> 16;
        const int yi = row_of(i, magic), xi = i - yi * L;
        int xj = xi + dx, yj = yi + dy;
        xj += xj < 0 ? L : 0;
        xj -= xj >= L ? L : 0;
        yj += yj < 0 ? L : 0;
        yj -= yj >= L ? L : 0;
        ci[k] = i;
        cj[k] = yj * L + xj;
        cv[k] = v;
        cu[k] = accept_uniform<R>(c2, c3);
      }
      cached = true;
    }

    // R: evaluate the undecided labels of this lane, keep the first accepted one
    const uint64_t active = base + M - done;
    int first = U, fi = 0, fj = 0, fv = 0;
    double fdh0 = 0.0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t lab = base + 1 + (uint64_t)(tid * U + k);
      if (first == U && lab > done) {
        const int i = ci[k], j = cj[k];
        const bool th = ((occ[i >> 5] >> (i & 31)) & 1u) && !((occ[j >> 5] >> (j & 31)) & 1u);
        if (th) {
          ++theta_cnt;
          const int pv = vec[cv[k]];
          const int dx = (int)(int16_t)(pv & 0xffff), dy = pv >> 16;
          const R td = tab[tidx<TRI>(dy < 0 ? -dy : dy, dx < 0 ? -dx : dx, H1)];
          const R dh0 = (eps[j] - eps[i]) - td;
          const R dH = dh0 - Ef * (R)dx;
          if (metropolis(dH, cu[k], S)) {
            first = k;
            fi = i;
            fj = j;
            fv = cv[k];
            fdh0 = (double)dh0;
          }
        }
      }
    }
    const unsigned long long bal = __ballot(first < U);
    if (bal != 0ull) {
      const int wl = __ffsll(bal) - 1;
      if (lane == wl) {
        HopInfo h;
        h.key = (uint32_t)(tid * U + first);
        h.i = fi;
        h.j = fj;
        h.v = fv;
        h.dH0 = fdh0;
        info[wid] = h;
        atomicOr(&sh->wmask[it % 3], 1u << wid);
      }
    }
    if (tid == 0) {
      sh->wmask[(it + 1) % 3] = 0u;
      sh->rounds += 1;
      sh->evaluated += active;
    }
    __syncthreads();
    const uint32_t wmask = __builtin_amdgcn_readfirstlane(sh->wmask[it % 3]);
    ++it;

    if (wmask == 0u) {
      // no accepted label in this chunk: every label in it is decided (rejected)
      done = base + M;
      base = done;
      cached = false;
      if (done - gs->call_scan0 >= ra.max_labels) {
        status = -4;  // CG_ESTALL
        break;
      }
      continue;
    }

    // X: execute the lowest accepted label of the chunk
    const HopInfo h = info[__ffs(wmask) - 1];
    const uint64_t q = base + 1 + (uint64_t)h.key;
    const uint64_t m = q - s_last;
    s_last = q;
    done = q;
    ++hops;
    ++since;
    if (tid == 0) {
      occ[h.i >> 5] &= ~(1u << (h.i & 31));
      occ[h.j >> 5] |= 1u << (h.j & 31);
      const int hv = vec[h.v];
      sh->P += (int64_t)(int16_t)(hv & 0xffff);
      sh->H0 = sh->H0 + h.dH0;
      sh->sum_p += (m + M - 1) / M;
      const int64_t lg = sh->logged;
      if (lg < S.log_cap) {
        S.log_label[lg] = q;
        S.log_from[lg] = h.i;
        S.log_to[lg] = h.j;
        sh->logged = lg + 1;
      }
      if (ra.clock_mode == 0) {
        sh->t = (double)s_last / S.Gamma;
      } else {
        uint32_t c0 = (uint32_t)hops, c1 = (uint32_t)(hops >> 32), c2 = sid, c3 = kTagClock;
        philox10(c0, c1, c2, c3, k0, k1);
        const double u1 = unit52(c0, c1), u2 = unit52(c2, c3);
        const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        const double mean = (double)m / S.Gamma;
        const double sd = sqrt((double)m) / S.Gamma;
        double dt = mean + sd * z;
        if (dt < 0.0) dt = 0.0;
        sh->t = sh->t + dt;
      }
    }
    update_energies<R, TRI>(eps, tab, h.i, h.j, L, H1, magic, lane, wid, nw);
    __syncthreads();
    if (done == base + M) {
      base = done;
      cached = false;
    }
    if (hops >= gs->hop_target) break;
    if (ra.time_mode && sh->t >= gs->t_end) break;
    if (ra.K > 0 && since >= ra.K) break;
  }

  atomicAdd(&sh->theta, theta_cnt);
  __syncthreads();
  {
    R* g = (R*)S.eps;
    for (int k = tid; k < N; k += nthr) g[k] = eps[k];
  }
  for (int k = tid; k < S.NW; k += nthr) S.occ[k] = occ[k];
  if (tid == 0) {
    gs->hops = hops;
    gs->s_last = s_last;
    gs->s_scan = done;
    gs->P = sh->P;
    gs->t = sh->t;
    gs->H0 = sh->H0;
    gs->since_refresh = since;
    gs->status = status;
    gs->sum_p = sh->sum_p;
    gs->rounds = sh->rounds;
    gs->evaluated = sh->evaluated;
    gs->theta_pass += sh->theta;
    gs->logged = sh->logged;
  }
}

// ---------------------------------------------------------------------------------
// Initial occupation: a uniform n_e-subset, the sites with the smallest 64-bit keys
// (w0:w1 of the OCC stream), ties by index.  Keys go to the phi buffer as scratch.
__global__ void __launch_bounds__(kInitBlock) k_init_keys(const DevSample* __restrict__ samples) {
  const DevSample& S = samples[blockIdx.y];
  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  if (l >= S.N) return;
  uint32_t c0 = (uint32_t)l, c1 = 0, c2 = S.sample_id, c3 = kTagOcc;
  philox10(c0, c1, c2, c3, S.seed_lo, S.seed_hi);
  ((uint64_t*)S.phi)[l] = ((uint64_t)c0 << 32) | (uint64_t)c1;
}

__global__ void __launch_bounds__(kInitBlock) k_init_rank(const DevSample* __restrict__ samples) {
  const DevSample& S = samples[blockIdx.y];
  const int N = S.N;
  if ((int)(blockIdx.x * kInitBlock) >= N) return;
  constexpr int kTile = 2048;
  __shared__ uint64_t tile[kTile];
  const uint64_t* keys = (const uint64_t*)S.phi;
  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  const uint64_t mine = l < N ? keys[l] : ~0ull;
  uint32_t rank = 0;
  for (int b = 0; b < N; b += kTile) {
    const int cnt = N - b < kTile ? N - b : kTile;
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += kInitBlock) tile[k] = keys[b + k];
    __syncthreads();
    for (int k = 0; k < cnt; ++k) {
      const uint64_t o = tile[k];
      rank += (o < mine) || (o == mine && b + k < l);
    }
  }
  const bool occupied = l < N && rank < (uint32_t)S.n_e;
  const unsigned long long bal = __ballot(occupied);
  if ((threadIdx.x & 63) == 0) {
    const int w = l >> 5;  // l is the wave's first site, a multiple of 64
    if (w < S.NW) S.occ[w] = (uint32_t)bal;
    if (w + 1 < S.NW) S.occ[w + 1] = (uint32_t)(bal >> 32);
  }
}

// phi_i = W (2u - 1), u from the PHI stream (Eq. 1's random potentials).
__global__ void __launch_bounds__(kInitBlock) k_init_phi(const DevSample* __restrict__ samples) {
  const DevSample& S = samples[blockIdx.y];
  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  if (l >= S.N) return;
  uint32_t c0 = (uint32_t)l, c1 = 0, c2 = S.sample_id, c3 = kTagPhi;
  philox10(c0, c1, c2, c3, S.seed_lo, S.seed_hi);
  S.phi[l] = S.W * (2.0 * unit52(c0, c1) - 1.0);
}

// ---------------------------------------------------------------------------------
// FP64 local energies from scratch: eps_l = phi_l + sum_{m != l} (n_m - nu) / r_lm, m in
// index order, one site per thread (the same rounding sequence as the definition).
// refresh = 0: initialisation.  refresh = 1: FP32 form, for samples due a refresh
// (since_refresh >= K or forced): records max |eps32 - eps64| and writes fl32(eps64).
// Per-block partial sums of the energy and maxima of the drift go to S.part.
template <typename R>
__global__ void __launch_bounds__(kInitBlock) k_eps_exact(const DevSample* __restrict__ samples,
                                                          int refresh, int K) {
  const DevSample& S = samples[blockIdx.y];
  const int N = S.N, L = S.L, H1 = S.H + 1;
  if ((int)(blockIdx.x * kInitBlock) >= N) return;
  if (refresh) {
    const SampleState* st = S.st;
    if (!(st->force_refresh || (K > 0 && st->since_refresh >= K))) return;
  }
  extern __shared__ __align__(16) uint8_t smem[];
  uint32_t* occ = (uint32_t*)smem;
  double* tab = (double*)(smem + align16(S.NW * 4));
  for (int k = threadIdx.x; k < S.NW; k += kInitBlock) occ[k] = S.occ[k];
  for (int k = threadIdx.x; k < H1 * H1; k += kInitBlock) tab[k] = S.tab64[k];
  __shared__ double red_sum[kInitBlock];
  __shared__ double red_max[kInitBlock];
  __syncthreads();

  const int l = blockIdx.x * kInitBlock + threadIdx.x;
  double contrib = 0.0, drift = 0.0;
  if (l < N) {
    const int yl = row_of(l, S.magic_L), xl = l - yl * L;
    const double q1 = 1.0 - S.nu, q0 = 0.0 - S.nu;
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
    R* e = (R*)S.eps;
    if (refresh) drift = fabs((double)e[l] - acc);
    e[l] = (R)acc;
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

// Folds the per-block partials of k_eps_exact into the sample state (one block per sample).
__global__ void __launch_bounds__(64) k_finalize(const DevSample* __restrict__ samples, int refresh, int K) {
  const DevSample& S = samples[blockIdx.x];
  SampleState* st = S.st;
  if (threadIdx.x != 0) return;
  if (refresh && !(st->force_refresh || (K > 0 && st->since_refresh >= K))) return;
  double h = 0.0, d = 0.0;
  for (int b = 0; b < S.nblk; ++b) {
    h = h + S.part[b];
    d = fmax(d, S.part[S.nblk + b]);
  }
  st->H0 = h;
  if (refresh) {
    st->refreshes += 1;
    st->last_drift = d;
    st->max_drift = fmax(st->max_drift, d);
    st->since_refresh = 0;
    st->force_refresh = 0;
  }
}

// Per-call targets: run n_hops more hops, or run until t >= t_end.
__global__ void k_begin_call(const DevSample* __restrict__ samples, int n, int64_t n_hops,
                             double t_end, int time_mode) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  SampleState* st = samples[b].st;
  st->hop_target = time_mode ? ~0ull : st->hops + (uint64_t)n_hops;
  st->t_end = time_mode ? t_end : -1.0;
  st->call_scan0 = st->s_scan;
  st->status = 0;
}

__global__ void k_force_refresh(const DevSample* __restrict__ samples, int n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) samples[b].st->force_refresh = 1;
}

// Counts samples that still have work in the current call.
__global__ void k_pending(const DevSample* __restrict__ samples, int n, int32_t* out) {
  __shared__ int32_t cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int b = threadIdx.x; b < n; b += blockDim.x) {
    const SampleState* st = samples[b].st;
    const bool more = st->status == 0 && st->hops < st->hop_target &&
                      !(st->t_end >= 0.0 && st->t >= st->t_end);
    if (more) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *out = cnt;
}

}  // namespace cg
