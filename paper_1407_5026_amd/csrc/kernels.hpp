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
    // three-input xor in one gfx950 v_bitop3_b32 (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
}

enum : uint32_t { kTagPropose = 0, kTagOcc = 1, kTagPhi = 2, kTagClock = 3, kTagGamma = 4 };

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
  return dH <= 0.0 || u < exp(dH * S.mrT);
}
__device__ __forceinline__ bool metropolis(float dH, float u, const DevSample& S) {
  return dH <= 0.0f || u < __expf(-dH * S.invT32);
}
// Branch-free forms for the evaluation round.  FP32: the exponential is evaluated on every
// lane (v_exp_f32); FP64: only lanes that passed the occupancy filter with dH > 0 call exp.
__device__ __forceinline__ bool metropolis_nb(float dH, float u, bool, const DevSample& S) {
  return (dH <= 0.0f) | (u < __expf(-dH * S.invT32));
}
__device__ __forceinline__ bool metropolis_nb(double dH, double u, bool th, const DevSample& S) {
  bool a = dH <= 0.0;
  if (th && !a) a = u < exp(dH * S.mrT);
  return a;
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

// Values equal on every lane, moved to scalar registers so that the compiler treats
// branches on them as uniform.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v); }
__device__ __forceinline__ uint64_t uni(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | (uint64_t)uni((uint32_t)v);
}
__device__ __forceinline__ int64_t uni(int64_t v) { return (int64_t)uni((uint64_t)v); }
__device__ __forceinline__ double uni(double v) { return __longlong_as_double((long long)uni((uint64_t)__double_as_longlong(v))); }

// Parallel iterations p = ceil(m / M) of a hop found after m serial proposals, M = 2^l2m the
// sample's width (section "Parallel rejection algorithm"; the hop itself does not depend on M).
__device__ __forceinline__ uint64_t p_iterations(uint64_t m, int32_t l2m) {
  const uint32_t l = (uint32_t)uni(l2m);
  return (m + ((1ull << l) - 1ull)) >> l;
}

struct HopInfo {
  uint32_t key;  // position of the label in the chunk: tid * U + k
  int32_t i, j, v;
  double dH0;    // (eps_j - eps_i) - 1/r_ij of the executed hop
  int32_t pad[2];
};
static_assert(sizeof(HopInfo) == kInfoBytes, "HopInfo size");

// Storage of one local energy.  FP64 form: the FP64 value, updated as e + (t_j - t_i)
// exactly like the definition.  FP32 form: an FP32 pair (value, low part) updated by
// Kahan's compensated summation, so that the pair tracks the exact running sum of the FP32
// increments and the value word -- the FP32 energy every proposal reads -- stays within
// about one rounding of it between refreshes.
// Keeps a per-lane value opaque to the optimizer: constant offsets added to an address are
// not merged into a wave-uniform part of its computation, and the value is formed where it
// is written (not hoisted out of a loop).
__device__ __forceinline__ uint32_t opaque(uint32_t a) {
  asm volatile("" : "+v"(a));
  return a;
}

// Energies in the arena addressed through the global address space: the compiler then
// knows an access cannot alias the LDS words written beside it and keeps several in flight
// (a generic pointer makes it wait for every access before the next LDS store).
// Addresses are a uniform base plus a 32-bit byte offset per lane (the load's scalar-base
// form: no 64-bit vector address per site).
template <typename T>
using gbl_ptr = __attribute__((address_space(1))) T*;
template <typename ET, typename R>
__device__ __forceinline__ ET gload(gbl_ptr<R> p, uint32_t byte_off) {
  const gbl_ptr<R> q = (gbl_ptr<R>)((__attribute__((address_space(1))) char*)p + byte_off);
  if constexpr (sizeof(ET) == 2 * sizeof(R)) {
    ET e;
    e.x = q[0];
    e.y = q[1];
    return e;
  } else {
    return q[0];
  }
}
template <typename ET, typename R>
__device__ __forceinline__ void gstore(gbl_ptr<R> p, uint32_t byte_off, ET e) {
  const gbl_ptr<R> q = (gbl_ptr<R>)((__attribute__((address_space(1))) char*)p + byte_off);
  if constexpr (sizeof(ET) == 2 * sizeof(R)) {
    q[0] = e.x;
    q[1] = e.y;
  } else {
    q[0] = e;
  }
}

template <typename R> struct Energy;
template <> struct Energy<double> {
  using T = double;
  __device__ static double value(T e) { return e; }
  __device__ static double total(T e) { return e; }
  __device__ static T add(T e, double d) { return e + d; }
  __device__ static T from64(double v) { return v; }
};
template <> struct Energy<float> {
  using T = float2;
  __device__ static float value(T e) { return e.x; }
  // the energy the pair represents (value + low part, exact in FP64)
  __device__ static double total(T e) { return (double)e.x + (double)e.y; }
  __device__ static T add(T e, float d) {
    const float y = d + e.y;
    const float t = e.x + y;
    return make_float2(t, y - (t - e.x));
  }
  __device__ static T from64(double v) {
    const float h = (float)v;
    return make_float2(h, (float)(v - (double)h));
  }
};

template <bool TRI>
__device__ __forceinline__ int tri_of(int a) { return (a * (a + 1)) >> 1; }

// Table index of the folded distances (ay, ax) in step 3b with tay = tri(ay), tax = tri(ax)
// already formed (TRI): the triangle entry tri(max) + min is max(tay, tax) + min(ay, ax),
// since tri(a) = a (a + 1) / 2 grows with a; otherwise the row-major ay H1 + ax.
template <bool TRI>
__device__ __forceinline__ int tidx_pre(int ay, int tay, int ax, int tax, int H1) {
  if (TRI) return (tay > tax ? tay : tax) + (ay < ax ? ay : ax);
  return ay * H1 + ax;
}

// Gaussian clock increment of step 3c for hop number h with m serial proposals:
// Box-Muller on the CLOCK stream, mean m/Gamma, deviation sqrt(m)/Gamma, clamped at 0.
__device__ __noinline__ double gauss_dt(uint64_t h, uint64_t m, uint32_t sid, uint32_t k0, uint32_t k1,
                                        double Gamma) {
  uint32_t c0 = (uint32_t)h, c1 = (uint32_t)(h >> 32), c2 = sid, c3 = kTagClock;
  philox10(c0, c1, c2, c3, k0, k1);
  const double u1 = unit52(c0, c1), u2 = unit52(c2, c3);
  const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  const double mean = (double)m / Gamma;
  const double sd = sqrt((double)m) / Gamma;
  const double dt = mean + sd * z;
  return dt < 0.0 ? 0.0 : dt;
}

// Exact serial clock (clock mode 2): the m proposals up to an executed hop each add an
// Exp(Gamma) waiting time in the serial mixed algorithm, so the hop adds a Gamma(m, Gamma)
// time.  Marsaglia and Tsang's method for shape m >= 1 (2000): d = m - 1/3,
// c = 1/sqrt(9 d); from a standard normal x (Box-Muller: 52-bit uniform, 32-bit angle) and a
// 32-bit uniform u, with v = (1 + c x)^3 > 0, accept d v when u < 1 - 0.0331 x^4 or
// ln u < x^2/2 + d (1 - v + ln v).  Attempt k of hop h draws Philox4x32-10 of
// (h, sample, GAMMA | k << 8); after 64 rejections (probability < 1e-80) the mean m / Gamma.
__device__ __noinline__ double gamma_dt(uint64_t h, uint64_t m, uint32_t sid, uint32_t k0, uint32_t k1,
                                        double Gamma) {
  const double d = (double)m - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
  for (uint32_t k = 0; k < 64; ++k) {
    uint32_t c0 = (uint32_t)h, c1 = (uint32_t)(h >> 32), c2 = sid, c3 = kTagGamma | (k << 8);
    philox10(c0, c1, c2, c3, k0, k1);
    const double u1 = unit52(c0, c1);
    const double u2 = ((double)c2 + 0.5) * 0x1p-32;
    const double u = ((double)c3 + 0.5) * 0x1p-32;
    const double x = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    double v = 1.0 + c * x;
    if (v <= 0.0) continue;
    v = v * v * v;
    const double x2 = x * x;
    if (u < 1.0 - 0.0331 * (x2 * x2)) return d * v / Gamma;
    if (log(u) < 0.5 * x2 + d * (1.0 - v + log(v))) return d * v / Gamma;
  }
  return (double)m / Gamma;
}

// Clock increment of a stochastic clock mode: 1 Gaussian (step 3c), 2 exact Gamma(m).
__device__ __forceinline__ double clock_dt(int mode, uint64_t h, uint64_t m, uint32_t sid, uint32_t k0,
                                           uint32_t k1, double Gamma) {
  return mode == 2 ? gamma_dt(h, m, sid, k0, k1, Gamma) : gauss_dt(h, m, sid, k0, k1, Gamma);
}

// Smallest label s with s / Gamma >= t_end (the deterministic clock is s_last / Gamma).
__device__ __noinline__ uint64_t label_at_time(double t_end, double Gamma) {
  double g = ceil(t_end * Gamma);
  uint64_t s = g > 0.0 ? (uint64_t)g : 0;
  while (s > 0 && (double)(s - 1) / Gamma >= t_end) --s;
  while ((double)s / Gamma < t_end) ++s;
  return s;
}

// Step 1 for this lane's labels base + 1 + tid U + k, k < U: Philox4x32-10 of (label,
// sample, PROPOSE) gives the site i = mulhi(w0, N), the displacement orbit (first o with
// w1 < thr[o], started from the guide bucket of w1) and member (w3 & (size - 1)), and the
// acceptance uniform; cached as (i, j, 1/r table index, dx, u).
template <typename R, int U, bool TRI>
__device__ __forceinline__ void draw_labels(uint64_t base, int tid, const DevSample& S, const uint8_t* guide,
                                            const uint32_t* thr, const uint32_t* orb, const int32_t* vec,
                                            int (&ci)[U], int (&cj)[U], int (&ct)[U], int (&cdx)[U],
                                            R (&cu)[U]) {
  const int L = S.L, N = S.N, H1 = S.H + 1, n_orb = S.n_orb;
  const uint32_t magic = S.magic_L;
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t lab = base + 1 + (uint64_t)(tid * U + k);
    uint32_t c0 = (uint32_t)lab, c1 = (uint32_t)(lab >> 32), c2 = S.sample_id, c3 = kTagPropose;
    philox10(c0, c1, c2, c3, S.seed_lo, S.seed_hi);
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
    ct[k] = tidx<TRI>(dy < 0 ? -dy : dy, dx < 0 ? -dx : dx, H1);
    cdx[k] = dx;
    cu[k] = accept_uniform<R>(c2, c3);
  }
}

// Workgroup-shared control words: per-round bitmask of waves holding an accepted label
// (triple-buffered, see the round loop), the clock of the Gaussian mode, theta count.
struct HopShared {
  uint64_t best[3];  // per-round minimum of (label key << 32 | i << 16 | j), triple-buffered
  uint32_t theta;
  uint32_t pad_;
  double t;
  double dummy;  // sink for the stores of lanes beyond the lattice
};

// The persistent hop kernel.  Threads own sites: wave w (16 waves) owns rows w + 16 r,
// r < RPW, and lane the columns lane + 64 c, c < NC; the owned energies live in registers
// (FP64, or the compensated FP32 pair) and their value words are mirrored in LDS for the
// proposals.  Step 3b then costs, per site and hop, two LDS reads of the 1/r table, one
// register update and one LDS write; the row separations of a wave are scalar.
// Where the energies live during a launch.
enum EnergyMode : int {
  kModeReg = 0,     // owned energies in registers, value words mirrored in LDS
  kModeLds = 1,     // energies in LDS, updated in place (FP64: value = storage)
  kModeGlobal = 2,  // energies in the arena (HBM/L2), updated in place; for lattices whose
                    // energies do not fit LDS
  kModeSplit = 3,   // FP32: value words in LDS, updated in place, and the pairs' low parts in
                    // each thread's own 16-byte groups in the arena (4 bytes per site each
                    // way per hop, four sites per access); the pairs are rebuilt at the end
                    // of a launch
};

template <typename R, int U, bool TRI, int NC, int RPW, bool EXACT, int MODE>
__global__ void __launch_bounds__(1024) k_hops(const DevSample* __restrict__ samples,
                                               const int32_t* __restrict__ order, RunArgs ra) {
  constexpr int NW = 16;
  using ET = typename Energy<R>::T;
  const DevSample& S = samples[order[blockIdx.x]];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);

  uint64_t hops = uni(gs->hops);
  uint64_t s_last = uni(gs->s_last);
  uint64_t done = uni(gs->s_scan);
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
  int64_t P = uni(gs->P);
  double H0 = uni(gs->H0);
  uint64_t sum_p = uni(gs->sum_p), rounds = uni(gs->rounds), evaluated = uni(gs->evaluated);
  int64_t logged = uni(gs->logged);
  int32_t status = 0;

  const int L = S.L, N = S.N, H1 = S.H + 1, n_orb = S.n_orb;
  const uint32_t magic = S.magic_L;
  extern __shared__ __align__(16) uint8_t smem[];
  const int32_t eb = (MODE == kModeReg || MODE == kModeSplit) ? (int32_t)sizeof(R)
                                                                : (MODE == kModeLds ? (int32_t)sizeof(ET) : 0);
  const HopLds lo = hop_lds(N, S.NW, S.ntab, S.n_vec, n_orb, eb, (int32_t)sizeof(R));
  R* __restrict__ ev = (R*)(smem + lo.eps);  // kModeReg, kModeSplit: value words of all energies
  ET* __restrict__ es = MODE == kModeLds ? (ET*)(smem + lo.eps) : (ET*)S.eps;  // in-place storage
  const gbl_ptr<R> eg = (gbl_ptr<R>)S.eps;  // the same storage in the arena modes
  uint32_t* __restrict__ occ = (uint32_t*)(smem + lo.occ);
  R* __restrict__ tab = (R*)(smem + lo.tab);
  int32_t* __restrict__ vec = (int32_t*)(smem + lo.vec);
  uint32_t* __restrict__ thr = (uint32_t*)(smem + lo.thr);
  uint32_t* __restrict__ orb = (uint32_t*)(smem + lo.orb);
  uint8_t* __restrict__ guide = smem + lo.guide;
  HopShared* __restrict__ sh = (HopShared*)(smem + lo.ctrl);
  HopInfo* __restrict__ info = (HopInfo*)(smem + lo.info);

  // owned energies: registers mirrored in LDS, or in-place LDS storage, or the arena
  ET E[MODE == kModeReg ? RPW : 1][MODE == kModeReg ? NC : 1];
  {
    const ET* __restrict__ g = (const ET*)S.eps;
    if constexpr (MODE == kModeReg) {
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int y = wid + NW * r;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int x = lane + 64 * c;
          if (y < L && x < L) {
            E[r][c] = g[y * L + x];
            ev[y * L + x] = Energy<R>::value(E[r][c]);
          } else {
            E[r][c] = ET();
          }
        }
      }
    } else if constexpr (MODE == kModeLds) {
      for (int k = tid; k < N; k += 1024) es[k] = g[k];
    } else if constexpr (MODE == kModeSplit) {
      // value words of every site; the low parts of the lane's own sites (the only ones it
      // reads and writes until the end of the launch)
      for (int k = tid; k < N; k += 1024) ev[k] = Energy<R>::value(g[k]);
      R* __restrict__ lw = (R*)S.mirror;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int y = wid + NW * r;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int x = lane + 64 * c, s = r * NC + c;
          if (y < L && x < L) lw[4 * (1024 * (s >> 2) + tid) + (s & 3)] = ((const R*)&g[y * L + x])[1];
        }
      }
    }
    const R* gt = (const R*)S.tabk;
    for (int k = tid; k < S.ntab; k += 1024) tab[k] = gt[k];
  }
  for (int k = tid; k < S.NW; k += 1024) occ[k] = S.occ[k];
  for (int k = tid; k < S.n_vec; k += 1024) vec[k] = S.vec[k];
  for (int k = tid; k < n_orb; k += 1024) {
    thr[k] = S.thr[k];
    orb[k] = S.orb[k];
  }
  for (int k = tid; k < kGuideSize; k += 1024) guide[k] = S.guide[k];
  if (tid == 0) {
    sh->best[0] = sh->best[1] = sh->best[2] = ~0ull;
    sh->theta = 0u;
    sh->t = t_start;
  }
  __syncthreads();

  const uint32_t k0 = S.seed_lo, k1 = S.seed_hi, sid = S.sample_id;
  const uint64_t M = (uint64_t)(1024 * U);
  // deterministic clock in run-to-time mode: stop at the first hop with label >= s_end
  const uint64_t s_end = uni((ra.time_mode && ra.clock_mode == 0) ? label_at_time(t_end, S.Gamma) : (uint64_t)0);
  const R Ef = field(S, R(0));
  uint64_t base = done;  // current chunk: labels base+1 .. base+M
  bool cached = false;
  int ci[U], cj[U], ct[U], cdx[U];
  R cu[U];
  uint32_t theta_cnt = 0;
  uint32_t it = 0;
  // optional phase timers (shader clock): refill, evaluate + round barrier, execute, update + barrier
  uint64_t tc0 = 0, tc1 = 0, tc2 = 0, tc3 = 0, tmark = 0;
  const bool timers = ra.timers != 0;
#define CG_MARK(acc)                                          \
  if (timers) {                                               \
    const uint64_t now_ = __builtin_amdgcn_s_memtime();       \
    acc += now_ - tmark;                                      \
    tmark = now_;                                             \
  }
  if (timers) tmark = __builtin_amdgcn_s_memtime();

  for (;;) {
    // P: draw this lane's labels of the chunk once; they are re-used after a hop
    if (!cached) {
      draw_labels<R, U, TRI>(base, tid, S, guide, thr, orb, vec, ci, cj, ct, cdx, cu);
      cached = true;
      CG_MARK(tc0)
    }

    // R: evaluate the undecided labels of this lane, keep the first accepted one.  The two
    // occupation words, both energies and 1/r are loaded unconditionally and combined
    // without branches, so a round costs one LDS round trip.
    const uint64_t active = base + M - done;
    int first = U, fi = 0, fj = 0, fdx = 0;
    double fdh0 = 0.0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t lab = base + 1 + (uint64_t)(tid * U + k);
      const int i = ci[k], j = cj[k];
      const uint32_t wi = occ[i >> 5], wj = occ[j >> 5];
      R ei, ej;
      if constexpr (MODE == kModeReg || MODE == kModeSplit) {
        ei = ev[i];
        ej = ev[j];
      } else if constexpr (MODE == kModeGlobal) {
        ei = Energy<R>::value(gload<ET, R>(eg, (uint32_t)i * (uint32_t)sizeof(ET)));
        ej = Energy<R>::value(gload<ET, R>(eg, (uint32_t)j * (uint32_t)sizeof(ET)));
      } else {
        ei = Energy<R>::value(es[i]);
        ej = Energy<R>::value(es[j]);
      }
      const R td = tab[ct[k]];
      const bool th = (first == U) & (lab > done) & ((((wi >> (i & 31)) & ~(wj >> (j & 31))) & 1u) != 0u);
      const R dh0 = (ej - ei) - td;
      const R dH = dh0 - Ef * (R)cdx[k];
      const bool acc = th & metropolis_nb(dH, cu[k], th, S);
      theta_cnt += th ? 1u : 0u;
      if (acc) {
        first = k;
        fi = i;
        fj = j;
        fdx = cdx[k];
        fdh0 = (double)dh0;
      }
    }
    // the wave's lowest accepting lane publishes (key, i, j) with one 64-bit LDS min; the
    // round's minimum is the workgroup's lowest accepted label (i, j < 2^16 since N <= 36864)
    const unsigned long long bal = __ballot(first < U);
    if (bal != 0ull) {
      const int wl = __ffsll(bal) - 1;
      if (lane == wl) {
        HopInfo h;
        h.key = (uint32_t)(tid * U + first);
        h.i = fi;
        h.j = fj;
        h.v = 0;
        h.dH0 = fdh0;
        h.pad[0] = fdx;
        info[wid] = h;
        atomicMin(&sh->best[it % 3], ((uint64_t)h.key << 32) | ((uint64_t)fi << 16) | (uint64_t)fj);
      }
    }
    if (tid == 0) sh->best[(it + 1) % 3] = ~0ull;
    __syncthreads();
    const uint64_t best = uni(sh->best[it % 3]);
    ++it;
    ++rounds;
    evaluated += active;
    CG_MARK(tc1)

    if (best == ~0ull) {
      // no accepted label in this chunk: every label in it is decided (rejected)
      done = base + M;
      base = done;
      cached = false;
      if (done - scan0 >= ra.max_labels) {
        status = -4;  // CG_ESTALL
        break;
      }
      continue;
    }

    // X: execute the lowest accepted label of the chunk
    HopInfo h;
    h.key = (uint32_t)(best >> 32);
    h.i = (int)((best >> 16) & 0xffffu);
    h.j = (int)(best & 0xffffu);
    {
      const HopInfo& w = info[(h.key / U) >> 6];  // written by the winning wave
      h.dH0 = uni(w.dH0);
      h.pad[0] = uni(w.pad[0]);
    }
    const int hdx = h.pad[0];
    const uint64_t q = base + 1 + (uint64_t)h.key;
    const uint64_t m = q - s_last;
    s_last = q;
    done = q;
    ++hops;
    ++since;
    P += hdx;
    H0 = H0 + h.dH0;
    sum_p += p_iterations(m, S.log2M);
    if (tid == 0) {
      atomicAnd(&occ[h.i >> 5], ~(1u << (h.i & 31)));
      atomicOr(&occ[h.j >> 5], 1u << (h.j & 31));
      if (logged < S.log_cap) {
        S.log_label[logged] = q;
        S.log_from[logged] = h.i;
        S.log_to[logged] = h.j;
      }
      if (ra.clock_mode != 0) sh->t = sh->t + clock_dt(ra.clock_mode, hops, m, sid, k0, k1, S.Gamma);
    }
    if (logged < S.log_cap) ++logged;
    CG_MARK(tc2)

    // U: step 3b on the owned sites.  All table loads are issued before the first use;
    // in an inexact geometry, rows/columns beyond L read a valid table entry and store to a
    // dummy LDS word, so no lane branches.
    {
      const int yi = row_of(h.i, magic), xi = h.i - yi * L;
      const int yj = row_of(h.j, magic), xj = h.j - yj * L;
      int cjx[NC], cix[NC], tjx[NC], tix[NC], sto[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int x = lane + 64 * c;
        const bool xv = EXACT || x < L;
        cjx[c] = xv ? fold(x - xj, L) : 0;
        cix[c] = xv ? fold(x - xi, L) : 0;
        tjx[c] = TRI ? tri_of<TRI>(cjx[c]) : 0;
        tix[c] = TRI ? tri_of<TRI>(cix[c]) : 0;
        sto[c] = xv ? x : -1;
      }
      // arena modes: byte offset of the lane's site in column block c and its first row, and
      // the stride to its next row; a lane beyond the lattice's edge reads and writes the
      // sample's sink word (after the N energies) instead, so no access needs a lane branch.
      // Formed here, not hoisted out of the hop loop (one address per site would occupy
      // registers for the whole launch).
      // (kModeSplit: offsets into the low-part array, 4 bytes per site, sink after N)
      constexpr int kEs = MODE == kModeSplit ? (int)sizeof(R) : (int)sizeof(ET);
      uint32_t gco[NC], grs[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const bool xv = sto[c] >= 0;
        gco[c] = opaque(xv ? (uint32_t)((wid * L + lane + 64 * c) * kEs) : (uint32_t)(N * kEs));
        grs[c] = xv ? (uint32_t)(NW * L * kEs) : 0u;
      }
      // kModeSplit: LDS byte address of the lane's value word in column block c and its first
      // row, and the stride to its next row (the sink word past the lattice's edge)
      using lds_r = __attribute__((address_space(3))) R*;
      uint32_t lco[NC], lrs[NC];
      if constexpr (MODE == kModeSplit) {
        const uint32_t ev0 = (uint32_t)(uintptr_t)(lds_r)ev;
        const uint32_t lsink = (uint32_t)(uintptr_t)(lds_r)(R*)&sh->dummy;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const bool xv = sto[c] >= 0;
          lco[c] = opaque(xv ? ev0 + (uint32_t)((wid * L + lane + 64 * c) * (int)sizeof(R)) : lsink);
          lrs[c] = xv ? (uint32_t)(NW * L * (int)sizeof(R)) : 0u;
        }
      }
      // rows in groups of RG: every load of a group is issued before its first use (the split
      // mode takes one row at a time, which measured fastest)
      constexpr int RG = (MODE == kModeReg && EXACT) ? RPW : MODE == kModeGlobal ? 2 : MODE == kModeSplit ? 1 : 4;
      // kModeSplit: the lane's low parts, slot s = r NC + c in component s % 4 of its group
      // s / 4 (16 bytes, 1024 g + tid in float4 units).  Four groups are in flight: group
      // g + 4 is loaded once group g is stored, about four rows' work before its first use.
      // A slot of a site past the lattice's edge is the lane's own, so no access needs a sink.
      constexpr int SPL = RPW * NC, NG = (SPL + 3) / 4, NB = 4;
      using lgrp_t = __attribute__((ext_vector_type(4))) float;
      const gbl_ptr<lgrp_t> lw4 = (gbl_ptr<lgrp_t>)S.mirror;
      lgrp_t lgrp[NB], lout = {0.f, 0.f, 0.f, 0.f};
      if constexpr (MODE == kModeSplit) {
#pragma unroll
        for (int g = 0; g < NB && g < NG; ++g) lgrp[g] = lw4[1024 * g + tid];
      }
#pragma unroll
      for (int r0 = 0; r0 < RPW; r0 += RG) {
        R d[RG][NC];
        ET e[MODE == kModeReg ? 1 : RG][NC];  // kModeSplit: (value from LDS, low part)
#pragma unroll
        for (int rr = 0; rr < RG; ++rr) {
          const int y = wid + NW * (r0 + rr);
          const bool yv = EXACT || y < L;
          const int ayj = yv ? fold(y - yj, L) : 0, ayi = yv ? fold(y - yi, L) : 0;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const int kj = tidx_pre<TRI>(ayj, TRI ? tri_of<TRI>(ayj) : 0, cjx[c], tjx[c], H1);
            const int ki = tidx_pre<TRI>(ayi, TRI ? tri_of<TRI>(ayi) : 0, cix[c], tix[c], H1);
            d[rr][c] = tab[kj] - tab[ki];
            if constexpr (MODE == kModeLds) {
              if (EXACT || (yv && sto[c] >= 0)) e[rr][c] = es[y * L + lane + 64 * c];
            } else if constexpr (MODE == kModeSplit) {
              const int s = (r0 + rr) * NC + c;
              // a row past the lattice's edge updates an arbitrary (but defined) value into
              // the lane's unused slot; no code is spent on it
              R v = __builtin_nondeterministic_value(R(0));
              if (EXACT || yv) v = *(lds_r)(lco[c] + (uint32_t)(r0 + rr) * lrs[c]);
              ((R*)&e[rr][c])[0] = v;
              ((R*)&e[rr][c])[1] = lgrp[(s >> 2) % NB][s & 3];
            } else if constexpr (MODE != kModeReg) {
              if (EXACT || yv) e[rr][c] = gload<ET, R>(eg, gco[c] + (uint32_t)(r0 + rr) * grs[c]);
            }
          }
        }
#pragma unroll
        for (int rr = 0; rr < RG; ++rr) {
          const int r = r0 + rr;
          const int y = wid + NW * r;
          const bool yv = EXACT || y < L;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            if constexpr (MODE == kModeReg) {
              E[r][c] = Energy<R>::add(E[r][c], d[rr][c]);
              R* dst = (EXACT || (yv && sto[c] >= 0)) ? ev + (y * L + lane + 64 * c) : (R*)&sh->dummy;
              *dst = Energy<R>::value(E[r][c]);
            } else if constexpr (MODE == kModeSplit) {
              const int s = r * NC + c, gi = s >> 2;
              const ET a = Energy<R>::add(e[rr][c], d[rr][c]);
              lout[s & 3] = ((const R*)&a)[1];
              if (EXACT || yv) *(lds_r)(lco[c] + (uint32_t)r * lrs[c]) = Energy<R>::value(a);
              if ((s & 3) == 3 || s == SPL - 1) {
                lw4[1024 * gi + tid] = lout;
                if (gi + NB < NG) lgrp[gi % NB] = lw4[1024 * (gi + NB) + tid];
              }
            } else if constexpr (MODE == kModeGlobal) {
              if (EXACT || yv) gstore<ET, R>(eg, gco[c] + (uint32_t)r * grs[c], Energy<R>::add(e[rr][c], d[rr][c]));
            } else {
              if (EXACT || (yv && sto[c] >= 0)) es[y * L + lane + 64 * c] = Energy<R>::add(e[rr][c], d[rr][c]);
            }
          }
        }
      }
    }
    __syncthreads();
    CG_MARK(tc3)
    if (done == base + M) {
      base = done;
      cached = false;
    }
    if (hops >= target) break;
    if (ra.time_mode) {
      if (ra.clock_mode == 0 ? s_last >= s_end : uni(sh->t) >= t_end) break;
    }
    if (ra.K > 0 && since >= ra.K) break;
  }

  atomicAdd(&sh->theta, theta_cnt);
  {
    ET* __restrict__ g = (ET*)S.eps;
    if constexpr (MODE == kModeReg) {
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int y = wid + NW * r;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int x = lane + 64 * c;
          if (y < L && x < L) g[y * L + x] = E[r][c];
        }
      }
    } else if constexpr (MODE == kModeSplit) {
      // the pairs of the lane's own sites: value words and low parts both last written by it
      const R* __restrict__ lw = (const R*)S.mirror;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int y = wid + NW * r;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int x = lane + 64 * c, s = r * NC + c;
          if (y < L && x < L) {
            ET a;
            ((R*)&a)[0] = ev[y * L + x];
            ((R*)&a)[1] = lw[4 * (1024 * (s >> 2) + tid) + (s & 3)];
            g[y * L + x] = a;
          }
        }
      }
    }
    __syncthreads();
    if constexpr (MODE == kModeLds)
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
    gs->since_refresh = since;
    gs->status = status;
    gs->sum_p = sum_p;
    gs->rounds = rounds;
    gs->evaluated = evaluated;
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

// ---------------------------------------------------------------------------------
// FP32 hop kernel with one workgroup barrier per hop.  The value words of the energies are
// double-buffered in LDS.  When the round ending at barrier B_r selects hop h, each wave
// runs step 3b for h on its owned sites (registers, Kahan) and writes the new values into
// the buffer not being read, while the next round evaluates its labels against the other
// buffer (energies before h) plus hop h's own contribution, 1/r_xj - 1/r_xi, computed by
// each lane for its two sites, and with the occupation of h's two sites overridden.  The
// update is complete at the next barrier, where the buffers swap.  The executed hops are
// those of the two-barrier kernel (same labels, same decisions up to FP32 rounding).
template <int U, int NC, int RPW, bool EXACT>
__global__ void __launch_bounds__(1024) k_hops_db(const DevSample* __restrict__ samples,
                                                  const int32_t* __restrict__ order, RunArgs ra) {
  using R = float;
  using ET = float2;
  constexpr int NW = 16;
  const DevSample& S = samples[order[blockIdx.x]];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);

  uint64_t hops = uni(gs->hops);
  uint64_t s_last = uni(gs->s_last);
  uint64_t done = uni(gs->s_scan);
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
  int64_t P = uni(gs->P);
  double H0 = uni(gs->H0);
  uint64_t sum_p = uni(gs->sum_p), rounds = uni(gs->rounds), evaluated = uni(gs->evaluated);
  int64_t logged = uni(gs->logged);
  int32_t status = 0;

  const int L = S.L, N = S.N, H1 = S.H + 1, n_orb = S.n_orb;
  const uint32_t magic = S.magic_L;
  extern __shared__ __align__(16) uint8_t smem[];
  const HopLds lo = hop_lds(N, S.NW, S.ntab, S.n_vec, n_orb, 2 * (int32_t)sizeof(R), (int32_t)sizeof(R));
  R* __restrict__ buf = (R*)(smem + lo.eps);  // two value buffers of N words
  uint32_t* __restrict__ occ = (uint32_t*)(smem + lo.occ);
  R* __restrict__ tab = (R*)(smem + lo.tab);
  int32_t* __restrict__ vec = (int32_t*)(smem + lo.vec);
  uint32_t* __restrict__ thr = (uint32_t*)(smem + lo.thr);
  uint32_t* __restrict__ orb = (uint32_t*)(smem + lo.orb);
  uint8_t* __restrict__ guide = smem + lo.guide;
  HopShared* __restrict__ sh = (HopShared*)(smem + lo.ctrl);
  HopInfo* __restrict__ info = (HopInfo*)(smem + lo.info);  // [2][16], by round parity

  ET E[RPW][NC];
  {
    const ET* __restrict__ g = (const ET*)S.eps;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int y = wid + NW * r;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int x = lane + 64 * c;
        if (y < L && x < L) {
          E[r][c] = g[y * L + x];
          buf[y * L + x] = E[r][c].x;
        } else {
          E[r][c] = ET();
        }
      }
    }
    const R* gt = (const R*)S.tabk;
    for (int k = tid; k < S.ntab; k += 1024) tab[k] = gt[k];
  }
  for (int k = tid; k < S.NW; k += 1024) occ[k] = S.occ[k];
  for (int k = tid; k < S.n_vec; k += 1024) vec[k] = S.vec[k];
  for (int k = tid; k < n_orb; k += 1024) {
    thr[k] = S.thr[k];
    orb[k] = S.orb[k];
  }
  for (int k = tid; k < kGuideSize; k += 1024) guide[k] = S.guide[k];
  if (tid == 0) {
    sh->best[0] = sh->best[1] = sh->best[2] = ~0ull;
    sh->theta = 0u;
    sh->t = t_start;
  }
  __syncthreads();

  const uint32_t sid = S.sample_id, k0 = S.seed_lo, k1 = S.seed_hi;
  const uint64_t M = (uint64_t)(1024 * U);
  const uint64_t s_end = uni((ra.time_mode && ra.clock_mode == 0) ? label_at_time(t_end, S.Gamma) : (uint64_t)0);
  const R Ef = S.E32;
  uint64_t base = done;
  bool cached = false;
  int ci[U], cj[U], ct[U], cdx[U];
  R cu[U];
  uint32_t theta_cnt = 0;
  uint32_t it = 0;
  int cur = 0;          // buffer holding the energies after every completed update
  bool pend = false;    // a hop's update runs in this round (writes buffer cur ^ 1)
  int pi = 0, pj = 0;   // the pending hop
  uint64_t tc0 = 0, tc1 = 0, tc2 = 0, tc3 = 0, tmark = 0;
  const bool timers = ra.timers != 0;
#define CG_MARK(acc)                                          \
  if (timers) {                                               \
    const uint64_t now_ = __builtin_amdgcn_s_memtime();       \
    acc += now_ - tmark;                                      \
    tmark = now_;                                             \
  }
  if (timers) tmark = __builtin_amdgcn_s_memtime();

  // per-hop constants of the pending hop for the lanes' own-site corrections
  int pxi = 0, pyi = 0, pxj = 0, pyj = 0;

  for (;;) {
    if (!cached) {
      draw_labels<R, U, false>(base, tid, S, guide, thr, orb, vec, ci, cj, ct, cdx, cu);
      cached = true;
      CG_MARK(tc0)
    }
    R* __restrict__ rd = buf + (cur ? N : 0);
    // U: step 3b of the pending hop on the owned sites, into the other buffer
    if (pend) {
      R* __restrict__ wr = buf + (cur ? 0 : N);
      int cjx[NC], cix[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int x = lane + 64 * c;
        const bool xv = EXACT || x < L;
        cjx[c] = xv ? fold(x - pxj, L) : 0;
        cix[c] = xv ? fold(x - pxi, L) : 0;
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int y = wid + NW * r;
        const bool yv = EXACT || y < L;
        const int ayj = yv ? fold(y - pyj, L) : 0, ayi = yv ? fold(y - pyi, L) : 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const R d = tab[ayj * H1 + cjx[c]] - tab[ayi * H1 + cix[c]];
          E[r][c] = Energy<R>::add(E[r][c], d);
          const bool ok = EXACT || (yv && lane + 64 * c < L);
          R* dst = ok ? wr + (y * L + lane + 64 * c) : (R*)&sh->dummy;
          *dst = E[r][c].x;
        }
      }
      CG_MARK(tc3)
    }

    // R: evaluate against rd plus the pending hop's contribution to the lane's two sites
    const uint64_t active = base + M - done;
    int first = U, fi = 0, fj = 0, fdx = 0;
    double fdh0 = 0.0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t lab = base + 1 + (uint64_t)(tid * U + k);
      const int i = ci[k], j = cj[k];
      const uint32_t wi = occ[i >> 5], wj = occ[j >> 5];
      R ei = rd[i], ej = rd[j];
      const R td = tab[ct[k]];
      uint32_t ni = (wi >> (i & 31)) & 1u, nj = (wj >> (j & 31)) & 1u;
      if (pend) {
        const int yi = row_of(i, magic), xi = i - yi * L;
        const int yj = row_of(j, magic), xj = j - yj * L;
        const R ci_ = tab[fold(yi - pyj, L) * H1 + fold(xi - pxj, L)] - tab[fold(yi - pyi, L) * H1 + fold(xi - pxi, L)];
        const R cj_ = tab[fold(yj - pyj, L) * H1 + fold(xj - pxj, L)] - tab[fold(yj - pyi, L) * H1 + fold(xj - pxi, L)];
        ei = ei + ci_;
        ej = ej + cj_;
        ni = i == pi ? 0u : (i == pj ? 1u : ni);
        nj = j == pi ? 0u : (j == pj ? 1u : nj);
      }
      const bool th = (first == U) & (lab > done) & ((ni & (nj ^ 1u)) != 0u);
      const R dh0 = (ej - ei) - td;
      const R dH = dh0 - Ef * (R)cdx[k];
      const bool acc = th & metropolis_nb(dH, cu[k], th, S);
      theta_cnt += th ? 1u : 0u;
      if (acc) {
        first = k;
        fi = i;
        fj = j;
        fdx = cdx[k];
        fdh0 = (double)dh0;
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
        h.v = 0;
        h.dH0 = fdh0;
        h.pad[0] = fdx;
        info[(it & 1) * kMaxWaves + wid] = h;
        atomicMin(&sh->best[it % 3], ((uint64_t)h.key << 32) | ((uint64_t)fi << 16) | (uint64_t)fj);
      }
    }
    if (tid == 0) sh->best[(it + 1) % 3] = ~0ull;
    __syncthreads();
    const uint64_t best = uni(sh->best[it % 3]);
    const HopInfo* infr = info + (it & 1) * kMaxWaves;
    ++it;
    ++rounds;
    evaluated += active;
    if (pend) {
      cur ^= 1;
      pend = false;
    }
    CG_MARK(tc1)

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

    // X: the round's lowest accepted label becomes the pending hop
    const uint32_t key = (uint32_t)(best >> 32);
    const int hi = (int)((best >> 16) & 0xffffu), hj = (int)(best & 0xffffu);
    double hdH0;
    int hdx;
    {
      const HopInfo& w = infr[(key / U) >> 6];
      hdH0 = uni(w.dH0);
      hdx = uni(w.pad[0]);
    }
    const uint64_t q = base + 1 + (uint64_t)key;
    const uint64_t m = q - s_last;
    s_last = q;
    done = q;
    ++hops;
    ++since;
    P += hdx;
    H0 = H0 + hdH0;
    sum_p += p_iterations(m, S.log2M);
    if (tid == 0) {
      atomicAnd(&occ[hi >> 5], ~(1u << (hi & 31)));
      atomicOr(&occ[hj >> 5], 1u << (hj & 31));
      if (logged < S.log_cap) {
        S.log_label[logged] = q;
        S.log_from[logged] = hi;
        S.log_to[logged] = hj;
      }
      if (ra.clock_mode != 0) sh->t = sh->t + clock_dt(ra.clock_mode, hops, m, sid, k0, k1, S.Gamma);
    }
    if (logged < S.log_cap) ++logged;
    pend = true;
    pi = hi;
    pj = hj;
    pyi = row_of(hi, magic);
    pxi = hi - pyi * L;
    pyj = row_of(hj, magic);
    pxj = hj - pyj * L;
    CG_MARK(tc2)
    if (done == base + M) {
      base = done;
      cached = false;
    }
    if (hops >= target) break;
    if (ra.K > 0 && since >= ra.K) break;
    if (ra.time_mode) {
      if (ra.clock_mode == 0) {
        if (s_last >= s_end) break;
      } else {
        __syncthreads();  // the Gaussian clock is advanced by thread 0
        if (uni(sh->t) >= t_end) break;
      }
    }
  }

  // the last hop's update (registers only: the values are not read again)
  if (pend) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int x = lane + 64 * c;
      const bool xv = EXACT || x < L;
      const int cjx = xv ? fold(x - pxj, L) : 0, cix = xv ? fold(x - pxi, L) : 0;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int y = wid + NW * r;
        const bool yv = EXACT || y < L;
        const int ayj = yv ? fold(y - pyj, L) : 0, ayi = yv ? fold(y - pyi, L) : 0;
        E[r][c] = Energy<R>::add(E[r][c], tab[ayj * H1 + cjx] - tab[ayi * H1 + cix]);
      }
    }
  }
  atomicAdd(&sh->theta, theta_cnt);
  {
    ET* __restrict__ g = (ET*)S.eps;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int y = wid + NW * r;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int x = lane + 64 * c;
        if (y < L && x < L) g[y * L + x] = E[r][c];
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < S.NW; k += 1024) S.occ[k] = occ[k];
  if (tid == 0) {
    gs->hops = hops;
    gs->s_last = s_last;
    gs->s_scan = done;
    gs->P = P;
    gs->t = ra.clock_mode == 0 ? (double)s_last / S.Gamma : sh->t;
    gs->H0 = H0;
    gs->since_refresh = since;
    gs->status = status;
    gs->sum_p = sum_p;
    gs->rounds = rounds;
    gs->evaluated = evaluated;
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
    if (S.dft || !(st->force_refresh || (K > 0 && st->since_refresh >= K))) return;
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
    typename Energy<R>::T* e = (typename Energy<R>::T*)S.eps;
    if (refresh) drift = fabs(Energy<R>::total(e[l]) - acc);
    e[l] = Energy<R>::from64(acc);
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

// ---------------------------------------------------------------------------------
// FP64 refresh by Fourier transform along x.  The energies of step 3b's definition are
// a circular convolution on the torus, eps = phi + (n - nu) (*) T with T(0) = 0, so with
// Q(k, y) = sum_x (n - nu)(x, y) e^{-2 pi i k x / L} and That(k, dy) = sum_dx T(dx, dy)
// cos(2 pi k dx / L) (real: T is even in dx):
//   C(k, y)   = sum_y' That(k, y - y') Q(k, y')                   (per-frequency convolution)
//   eps(x, y) = phi(x, y) + (1/L) sum_k w_k Re[C(k, y) e^{2 pi i k x / L}],
// k = 0..L/2 with w_k = 2 except w_0 = 1 and, for even L, w_{L/2} = 1.  Frequencies are
// processed in chunks of KC that fit LDS; every thread owns the outputs (x, g + G r) and
// accumulates them in registers over the chunks.  One workgroup per sample; samples not
// due a refresh return at once.  Records max |eps32 - eps64|, writes fl(eps64), recomputes
// the energy total in FP64.
constexpr int kDftRowsMax = 32;  // outputs per thread: ceil(L / floor(1024 / L)) <= 32
constexpr int kDftItems = 4;     // convolution items per thread: KC * L <= 4 * 1024

template <typename R, int kDftRows>
__global__ void __launch_bounds__(1024) k_refresh_dft(const DevSample* __restrict__ samples, int K) {
  const DevSample& S = samples[blockIdx.x];
  SampleState* __restrict__ st = S.st;
  if (!S.dft || ((S.dft_rows > 16) != (kDftRows > 16))) return;
  if (!(st->force_refresh || (K > 0 && st->since_refresh >= K))) return;
  const int L = S.L, NK = S.H + 1, KC = S.dft_kc;
  const int tid = threadIdx.x, nthr = blockDim.x;
  extern __shared__ __align__(16) uint8_t smem[];
  uint32_t* __restrict__ occ = (uint32_t*)smem;
  double2* __restrict__ tw = (double2*)(smem + align16(S.NW * 4));
  double2* __restrict__ Q = tw + L;
  double* __restrict__ Th = (double*)(Q + KC * L);
  __shared__ double red_h[kMaxWaves], red_d[kMaxWaves];
  for (int k = tid; k < S.NW; k += nthr) occ[k] = S.occ[k];
  for (int k = tid; k < L; k += nthr) tw[k] = ((const double2*)S.dft_tw)[k];

  const double q1 = 1.0 - S.nu, q0 = 0.0 - S.nu;
  const int G = nthr / L;
  const int x = tid % L, g = tid / L;
  const bool owner = g < G;
  double acc[kDftRows];
#pragma unroll
  for (int r = 0; r < kDftRows; ++r) acc[r] = 0.0;

  for (int k0 = 0; k0 < NK; k0 += KC) {
    const int kc = NK - k0 < KC ? NK - k0 : KC;
    const int items = kc * L;
    __syncthreads();
    for (int w = tid; w < items; w += nthr) Th[w] = S.dft_T[(size_t)k0 * L + w];
    // forward transform along x: item w = (frequency k0 + w / L, row w % L)
    for (int w = tid; w < items; w += nthr) {
      const int kk = w / L, y = w - kk * L, k = k0 + kk;
      double re = 0.0, im = 0.0;
      int idx = 0;
      const uint32_t* orow = occ;
      for (int xx = 0; xx < L; ++xx) {
        const int m = y * L + xx;
        const double qv = ((orow[m >> 5] >> (m & 31)) & 1u) ? q1 : q0;
        const double2 t = tw[idx];
        re = re + qv * t.x;
        im = im - qv * t.y;
        idx += k;
        idx -= idx >= L ? L : 0;
      }
      Q[w] = make_double2(re, im);
    }
    __syncthreads();
    // convolution along y, into registers, then back into Q
    double2 res[kDftItems];
#pragma unroll
    for (int r = 0; r < kDftItems; ++r) {
      const int w = tid + r * nthr;
      res[r] = make_double2(0.0, 0.0);
      if (w < items) {
        const int kk = w / L, y = w - kk * L;
        const double* th = Th + kk * L;
        const double2* qk = Q + kk * L;
        double re = 0.0, im = 0.0;
        int d = y;
        for (int yp = 0; yp < L; ++yp) {
          const double t = th[d];
          const double2 qv = qk[yp];
          re = re + t * qv.x;
          im = im + t * qv.y;
          d = d == 0 ? L - 1 : d - 1;
        }
        res[r] = make_double2(re, im);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kDftItems; ++r) {
      const int w = tid + r * nthr;
      if (w < items) Q[w] = res[r];
    }
    __syncthreads();
    // inverse transform along x, accumulated per owned output
    if (owner) {
      int idx = (int)(((int64_t)k0 * x) % L);
      for (int kk = 0; kk < kc; ++kk) {
        const int k = k0 + kk;
        const double wk = (k == 0 || 2 * k == L) ? 1.0 : 2.0;
        const double2 t = tw[idx];
        const double c = wk * t.x, sn = wk * t.y;
        const double2* ck = Q + kk * L;
#pragma unroll
        for (int r = 0; r < kDftRows; ++r) {
          const int y = g + G * r;
          if (y < L) {
            const double2 cv = ck[y];
            acc[r] = acc[r] + (cv.x * c - cv.y * sn);
          }
        }
        idx += x;
        idx -= idx >= L ? L : 0;
      }
    }
  }

  double hsum = 0.0, dmax = 0.0;
  if (owner) {
    const double invL = 1.0 / (double)L;
    typename Energy<R>::T* e = (typename Energy<R>::T*)S.eps;
#pragma unroll
    for (int r = 0; r < kDftRows; ++r) {
      const int y = g + G * r;
      if (y < L) {
        const int l = y * L + x;
        const double ph = S.phi[l];
        const double e64 = ph + acc[r] * invL;
        dmax = fmax(dmax, fabs(Energy<R>::total(e[l]) - e64));
        e[l] = Energy<R>::from64(e64);
        const bool nl = (occ[l >> 5] >> (l & 31)) & 1u;
        hsum = hsum + ((nl ? ph : 0.0) + 0.5 * ((nl ? q1 : q0) * (e64 - ph)));
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    hsum += __shfl_xor(hsum, off);
    dmax = fmax(dmax, __shfl_xor(dmax, off));
  }
  const int lane = tid & 63, wv = tid >> 6;
  if (lane == 0) {
    red_h[wv] = hsum;
    red_d[wv] = dmax;
  }
  __syncthreads();
  if (tid == 0) {
    double h = 0.0, d = 0.0;
    for (int k = 0; k < (nthr >> 6); ++k) {
      h = h + red_h[k];
      d = fmax(d, red_d[k]);
    }
    st->H0 = h;
    st->refreshes += 1;
    st->last_drift = d;
    st->max_drift = fmax(st->max_drift, d);
    st->since_refresh = 0;
    st->force_refresh = 0;
  }
}

// Folds the per-block partials of k_eps_exact into the sample state (one block per sample).
__global__ void __launch_bounds__(64) k_finalize(const DevSample* __restrict__ samples, int refresh, int K) {
  const DevSample& S = samples[blockIdx.x];
  SampleState* st = S.st;
  if (threadIdx.x != 0) return;
  if (refresh && (S.dft || !(st->force_refresh || (K > 0 && st->since_refresh >= K)))) return;
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
