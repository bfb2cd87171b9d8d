// hop_fx64.hpp -- FP64 hop kernel for lattices that fill the 1024-thread geometry exactly
// (L = 64 or 128; wave w owns rows w + 16 r, lane the columns lane + 64 c).
//
// The plain FP64 form of the mixed parallel-rejection step (section "Hopping conduction in
// the Coulomb glass", steps 1, 2, 3a-3c): the same labels, decisions and arithmetic as the
// generic kernel k_hops and the serial FP64 chain (hop for hop), laid out as k_hops_fx:
//  * owned FP64 energies in registers, their value words in LDS for the proposals, stored
//    per wave as [slot / 2][lane][slot % 2] so that a lane writes two sites per 16-byte
//    store and a store covers 1024 contiguous bytes;
//  * the FP64 1/r table in triangle order (index a(a+1)/2 + b of the folded separation
//    a >= b), the only FP64 table that fits beside the energies; in step 3b a row's folded
//    distance is the same for the whole wave, so it costs scalar work only;
//  * the proposal tables of the FP32 kernel (16-bit guide, 8-slot members) and the labels
//    of a chunk cached, the next chunk drawn during a hop's update, winner records tagged
//    with the round.
#pragma once

#include "hop_fx.hpp"
#include "kernels.hpp"

namespace cg {

struct Fx64Lds {
  int32_t ev, occ, tab, thr, guide, vec8, info, tag, ctrl, total;
};

// LDS of the FP64 exact-geometry kernel (byte offsets).
__host__ __device__ inline Fx64Lds fx64_lds(int32_t L, int32_t n_orb) {
  const int32_t H = L / 2;
  Fx64Lds o;
  int32_t b = 0;
  o.ev = b;    b = align16(b + L * L * 8);
  o.occ = b;   b = align16(b + L * L / 8);
  o.tab = b;   b = align16(b + ((H + 1) * (H + 2) / 2) * 8);
  o.thr = b;   b = align16(b + n_orb * 4);
  o.guide = b; b = align16(b + kGuide16Size * 2);
  o.vec8 = b;  b = align16(b + n_orb * 64);
  o.info = b;  b = align16(b + 16 * 16);
  o.tag = b;   b = align16(b + 16 * 4);
  o.ctrl = b;  b = align16(b + (int32_t)sizeof(FxShared));
  o.total = b;
  return o;
}

template <int L>
struct Fx64Geo {
  static constexpr int LG = L == 64 ? 6 : 7;
  static constexpr int N = L * L;
  static constexpr int NC = L / 64;
  static constexpr int RPW = L / 16;
  static constexpr int SPL = RPW * NC;
  static constexpr int H1 = L / 2 + 1;
  static_assert(L == 64 || L == 128, "exact geometry: L = 64 or 128");
  // LDS double index of site (x, y)'s value word: owner wave y & 15, lane x & 63, slot
  // s = (y >> 4) NC + (x >> 6)
  __device__ static int ev_slot(int x, int y) {
    const int s = (y >> 4) * NC + (x >> 6);
    return (y & 15) * 64 * SPL + (s >> 1) * 128 + (x & 63) * 2 + (s & 1);
  }
};

typedef double f64x2 __attribute__((ext_vector_type(2)));

// Folded row distances of step 3b.  For a wave w and an origin row y0, the wave's row
// y = w + 16 r lies at folded distance a = min(v, L - v) from y0, v = (d + 16 r) mod L with
// d = (w - y0) mod L; row d of the table holds 8 a for r < L / 16 and, beside it,
// 8 a (a + 1) / 2, the byte offset of row a of the triangle-ordered 1/r table.  Read with
// scalar loads, it takes the per-row distance arithmetic off the CU's shared scalar unit.
template <int L>
struct RowFold {
  uint32_t a8[L][L / 16];
  uint32_t t8[L][L / 16];
};
template <int L>
constexpr RowFold<L> make_row_fold() {
  RowFold<L> f{};
  for (int d = 0; d < L; ++d)
    for (int r = 0; r < L / 16; ++r) {
      const int v = (d + 16 * r) & (L - 1);
      const int a = v < L - v ? v : L - v;
      f.a8[d][r] = (uint32_t)(8 * a);
      f.t8[d][r] = (uint32_t)(8 * ((a * (a + 1)) >> 1));
    }
  return f;
}
__constant__ const RowFold<64> kRowFold64 = make_row_fold<64>();
__constant__ const RowFold<128> kRowFold128 = make_row_fold<128>();
template <int L>
__device__ __forceinline__ const RowFold<L>& row_fold() {
  if constexpr (L == 64)
    return kRowFold64;
  else
    return kRowFold128;
}

// a (a + 1) / 2: start of row a of the triangle-ordered table
__device__ __forceinline__ int tri_start(int a) { return (a * (a + 1)) >> 1; }

struct Fx64Label {
  uint32_t ij;      // i | j << 16
  uint32_t aidx;    // LDS byte address of eps_i's value word | (dx & 0xff) << 24
  uint32_t aj;      // LDS byte address of eps_j's value word
  double td, u;     // 1/r_ij, acceptance uniform
};

// Step 1 for this lane's labels of the chunk after `base` (the proposal law of the FP32
// kernel; the acceptance uniform is the 52-bit (2k + 1) 2^-53 of words 2, 3 and 1/r_ij the
// FP64 table entry).
template <int L, int U>
__device__ __forceinline__ void draw_fx64(uint64_t base, int tid, const FxConst& C, uint32_t lds0,
                                          const Fx64Lds& lo, Fx64Label (&lb)[U]) {
  using G = Fx64Geo<L>;
  const uint32_t guide = lds0 + lo.guide, thr = lds0 + lo.thr, vec8 = lds0 + lo.vec8, tab = lds0 + lo.tab;
  const uint32_t ev = lds0 + lo.ev;
  const int last = C.last;
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t lab = base + 1 + (uint64_t)(tid * U + k);
    uint32_t c0 = (uint32_t)lab, c1 = (uint32_t)(lab >> 32), c2 = C.sid, c3 = kTagPropose;
    philox10(c0, c1, c2, c3, C.k0, C.k1);
    const int i = (int)(c0 >> (32 - 2 * G::LG));
    const int o = orbit_guided(guide16_at(guide, c1), c1, thr, last);
    const int vx = (int)lds_ld<uint32_t>(vec8 + 8 * (o * 8 + (int)(c3 & 7u)));
    const int dx = (int)(int16_t)(vx & 0xffff), dy = vx >> 16;
    const int xi = i & (L - 1), yi = i >> G::LG;
    const int xj = (xi + dx) & (L - 1), yj = (yi + dy) & (L - 1);
    const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
    const int a = ax > ay ? ax : ay, bb = ax > ay ? ay : ax;
    Fx64Label& b = lb[k];
    b.ij = (uint32_t)i | ((uint32_t)((yj << G::LG) | xj) << 16);
    b.aidx = (ev + 8 * G::ev_slot(xi, yi)) | ((uint32_t)dx << 24);
    b.aj = ev + 8 * G::ev_slot(xj, yj);
    b.td = lds_ld<double>(tab + 8 * (tri_start(a) + bb));
    b.u = unit52(c2, c3);
  }
}

template <int L, int U, int CLOCK>
__global__ void __launch_bounds__(1024) k_hops_fx64(const DevSample* __restrict__ samples,
                                                    const int32_t* __restrict__ order, RunArgs ra) {
  using G = Fx64Geo<L>;
  constexpr int NW = 16, NC = G::NC, RPW = G::RPW, SPL = G::SPL, H1 = G::H1;
  constexpr uint32_t M = 1024u * U;
  constexpr int RG = RPW < 4 ? RPW : 4;  // rows per group of table loads in step 3b
  const DevSample& S = samples[order[blockIdx.x]];
  SampleState* __restrict__ gs = S.st;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = uni((int32_t)(tid >> 6));

  uint64_t hops = uni(gs->hops);
  uint64_t s_last = uni(gs->s_last);
  const uint64_t target = uni(gs->hop_target);
  const uint64_t scan0 = uni(gs->call_scan0);
  const double t_end = uni(gs->t_end);
  const double t_start = uni(gs->t);
  if (uni(gs->status) != 0 || hops >= target || (ra.time_mode && t_start >= t_end)) return;
  uint64_t base = uni(gs->s_scan);
  uint32_t dpos = 0;
  int64_t P_ = uni(gs->P);
  double H0 = uni(gs->H0);
  uint64_t sum_p = uni(gs->sum_p), rounds = uni(gs->rounds), evaluated = uni(gs->evaluated);
  int64_t logged = uni(gs->logged);
  int32_t status = 0;

  extern __shared__ __align__(16) uint8_t smem[];
  const Fx64Lds lo = fx64_lds(L, S.n_orb);
  const uint32_t lds0 = lds_addr_of(smem);
  double* __restrict__ ev = (double*)(smem + lo.ev);
  uint32_t* __restrict__ occ = (uint32_t*)(smem + lo.occ);
  double* __restrict__ tab = (double*)(smem + lo.tab);
  uint4* __restrict__ info = (uint4*)(smem + lo.info);
  uint32_t* __restrict__ tag = (uint32_t*)(smem + lo.tag);
  FxShared* __restrict__ sh = (FxShared*)(smem + lo.ctrl);

  // owned FP64 energies in registers, their value words in LDS
  double E[RPW][NC];
  {
    const double* __restrict__ g = (const double*)S.eps;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        E[r][c] = g[(wid + NW * r) * L + lane + 64 * c];
        ev[G::ev_slot(lane + 64 * c, wid + NW * r)] = E[r][c];
      }
    }
  }
  for (int k = tid; k < G::N / 32; k += 1024) occ[k] = S.occ[k];
  for (int k = tid; k < H1 * (H1 + 1) / 2; k += 1024) tab[k] = ((const double*)S.tabk)[k];
  for (int k = tid; k < S.n_orb; k += 1024) ((uint32_t*)(smem + lo.thr))[k] = S.thr[k];
  for (int k = tid; k < kGuide16Size; k += 1024) ((uint16_t*)(smem + lo.guide))[k] = S.guide16[k];
  for (int k = tid; k < S.n_orb * 8; k += 1024) ((int2*)(smem + lo.vec8))[k] = ((const int2*)S.vec8)[k];
  if (tid < 16) tag[tid] = ~0u;  // no round carries this tag
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
  C.Ef = 0.f;
  C.mTln2 = 0.f;
  const double Ed = uni(S.E), mrT = uni(S.mrT), Gamma = uni(S.Gamma);
  const int64_t log_cap = uni((int64_t)S.log_cap);
  const uint64_t s_end = uni((ra.time_mode && CLOCK == 0) ? label_at_time(t_end, Gamma) : (uint64_t)0);
  // this lane's value words: slot pair q = (s0, s0 + 1) at ev_lane + 1024 q
  const uint32_t ev_lane = opaque(lds0 + lo.ev + 8u * (uint32_t)(wid * 64 * SPL + lane * 2));
  bool cached = false;
  Fx64Label lb[U];
  Fx64Label lbn[U];  // the next chunk, drawn during a hop's update; valid when next_base == base + M
  uint64_t next_base = ~0ull;
  uint32_t theta_cnt = 0;
  uint32_t nev = 0;    // this lane's label evaluations (labels at or after dpos in a round)
  uint32_t round = 0;  // rounds of this launch so far

  for (;;) {
    uint32_t mk = 0u, win0 = 0u, win1 = 0u, win2 = 0u, win3 = 0u;
    for (;;) {
      if (!cached) {
        if (next_base == base) {
#pragma unroll
          for (int k = 0; k < U; ++k) lb[k] = lbn[k];
        } else {
          draw_fx64<L, U>(base, tid, C, lds0, lo, lb);
        }
        cached = true;
      }
      // step 2: occupancy filter, dH, Metropolis; the lane keeps its first accepted label.
      // The flags are 0/1 integers in vector registers and the thermal factor is evaluated
      // for every lane (nearly every wave needs it anyway), so the decision uses none of
      // the workgroup's shared scalar unit for lane masks or divergent branches.
      uint32_t found = 0u;
      uint32_t pub0 = 0u, pub1 = 0u;
      double pdh = 0.0;
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const Fx64Label& b = lb[k];
        const uint32_t key = (uint32_t)(tid * U + k);
        const uint32_t undec = ((key - dpos) >> 31) ^ 1u;
        nev += undec;
        const uint32_t open = undec & (found ^ 1u);
        const int bi = (int)(b.ij & 0xffffu), bj = (int)(b.ij >> 16), bdx = (int)b.aidx >> 24;
        const uint32_t wi = occ[bi >> 5], wj = occ[bj >> 5];
        const double ei = lds_ld<double>(b.aidx & 0xffffffu), ej = lds_ld<double>(b.aj);
        const uint32_t th = open & (wi >> (bi & 31)) & ~(wj >> (bj & 31)) & 1u;
        const double dh0 = (ej - ei) - b.td;
        const double dH = dh0 - Ed * (double)bdx;
        const double pth = exp(dH * mrT);
        const uint32_t acc = th & ((dH <= 0.0) | (b.u < pth) ? 1u : 0u);
        theta_cnt += th;
        pub0 = acc ? b.ij : pub0;
        pub1 = acc ? (key | ((uint32_t)bdx << 16)) : pub1;
        pdh = acc ? dh0 : pdh;
        found |= acc;
      }
      // the wave's lowest accepting lane publishes its label in the wave's record, tagged
      // with the round; after the barrier lanes 0..15 read the records and the winner is
      // the lowest wave whose tag is this round's (keys grow with the thread index); a
      // record is rewritten only by its own wave in a later round
      const unsigned long long bal = __ballot(found != 0u);
      const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      if (((found ^ 1u) | below) == 0u) {  // found, and no accepting lane below this one
        const uint64_t bits = (uint64_t)__double_as_longlong(pdh);
        info[wid] = make_uint4(pub0, pub1, (uint32_t)bits, (uint32_t)(bits >> 32));
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
    // the state written back at the end (by thread 0): kept by wave 0 only, so that the
    // other waves' scalar work after the barrier is just what their update needs
    if (wid == 0) {
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
        if (CLOCK != 0) sh->t = sh->t + clock_dt(ra.clock_mode, hops, m, C.sid, C.k0, C.k1, Gamma);
      }
      logged += logged < log_cap ? 1 : 0;
    }

    // step 3b on the owned sites: eps += 1/r_lj - 1/r_li from the triangle table.  The
    // column distances are per lane, a row's distance is the same for the whole wave.  The
    // entry of distances (a, b) sits at tri(max) + min, and since tri(a) = a (a + 1) / 2
    // grows with a, tri(max(a, b)) = max(tri(a), tri(b)): three vector operations per
    // entry, all in byte units.
    {
      const int xi = hi & (L - 1), yi = hi >> G::LG, xj = hj & (L - 1), yj = hj >> G::LG;
      uint32_t cj[NC], ci[NC], tj[NC], tiv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int x = lane + 64 * c;
        const int fj = fold(x - xj, L), fi = fold(x - xi, L);
        cj[c] = 8u * (uint32_t)fj;
        ci[c] = 8u * (uint32_t)fi;
        tj[c] = 8u * (uint32_t)tri_start(fj);
        tiv[c] = 8u * (uint32_t)tri_start(fi);
      }
      const uint32_t tb = lds0 + lo.tab;
      const RowFold<L>& F = row_fold<L>();
      const int dj = (wid - yj) & (L - 1), di = (wid - yi) & (L - 1);
#pragma unroll
      for (int r0 = 0; r0 < RPW; r0 += RG) {
        double a[RG][NC], bv[RG][NC];
#pragma unroll
        for (int rr = 0; rr < RG; ++rr) {
          const uint32_t ayj = F.a8[dj][r0 + rr], ayi = F.a8[di][r0 + rr];
          const uint32_t tyj = F.t8[dj][r0 + rr], tyi = F.t8[di][r0 + rr];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const uint32_t kj = (tj[c] > tyj ? tj[c] : tyj) + (cj[c] < ayj ? cj[c] : ayj);
            const uint32_t ki = (tiv[c] > tyi ? tiv[c] : tyi) + (ci[c] < ayi ? ci[c] : ayi);
            a[rr][c] = lds_ld<double>(tb + kj);
            bv[rr][c] = lds_ld<double>(tb + ki);
          }
        }
        // while the first group's loads are in flight: draw the next chunk if needed
        if (r0 == 0 && next_base != base + M) {
          next_base = base + M;
          draw_fx64<L, U>(next_base, tid, C, lds0, lo, lbn);
        }
#pragma unroll
        for (int rr = 0; rr < RG; ++rr) {
#pragma unroll
          for (int c = 0; c < NC; ++c) E[r0 + rr][c] = E[r0 + rr][c] + (a[rr][c] - bv[rr][c]);
        }
        // value words of slots s = r NC + c, two per 16-byte store
#pragma unroll
        for (int s = (r0 * NC) & ~1; s < (r0 + RG) * NC; s += 2) {
          f64x2 w;
          w.x = E[s / NC][s % NC];
          w.y = E[(s + 1) / NC][(s + 1) % NC];
          lds_st<f64x2>(ev_lane + 1024u * (uint32_t)(s >> 1), w);
        }
      }
    }
    __syncthreads();
    if (dpos == M) {
      base += M;
      dpos = 0;
      cached = false;
    }
    if (hops >= target) break;
    if (ra.time_mode) {
      if (CLOCK == 0 ? s_last >= s_end : uni(sh->t) >= t_end) break;
    }
  }

  atomicAdd(&sh->theta, theta_cnt);
  atomicAdd(&sh->nev, (unsigned long long)nev);
  {
    double* __restrict__ g = (double*)S.eps;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
#pragma unroll
      for (int c = 0; c < NC; ++c) g[(wid + NW * r) * L + lane + 64 * c] = E[r][c];
    }
  }
  __syncthreads();
  for (int k = tid; k < G::N / 32; k += 1024) S.occ[k] = occ[k];
  if (tid == 0) {
    gs->hops = hops;
    gs->s_last = s_last;
    gs->s_scan = base + dpos;
    gs->P = P_;
    gs->t = CLOCK == 0 ? (double)s_last / Gamma : sh->t;
    gs->H0 = H0;
    gs->status = status;
    gs->sum_p = sum_p;
    gs->rounds = rounds + round;
    gs->evaluated = evaluated + sh->nev;
    gs->theta_pass += sh->theta;
    gs->logged = logged;
  }
}

}  // namespace cg
