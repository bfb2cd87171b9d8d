// cgkmc.hip -- host side of libcgkmc: validation, proposal tables, arena plan, launches.
//
// The C ABI is declared in include/cgkmc.h.  All device memory comes from the caller's
// arena; all work goes to the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "cgkmc.h"
#include "hop3d.hpp"
#include "hop_big.hpp"
#include "hop_fx.hpp"
#include "hop_fx64.hpp"
#include "hop_pair.hpp"
#include "hop_wide.hpp"
#include "hop_wide3.hpp"
#include "kernels.hpp"
#include "layout.hpp"
#include "observables.hpp"

using namespace cg;

namespace {

thread_local char g_err[512] = "";

int set_err(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return set_err(CG_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,   \
                     __LINE__);                                                           \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// Scratch of the allocation-free density-of-states call: the bin counts of one call
// (2 kDosMaxBins + 2 slots of 8 bytes, 64 KiB) in a file-scope device array instead of the
// arena's histogram region.  Every device the library runs on holds its own copy for the
// life of the process.  In host code the array's name is not a device address: the address
// comes from hipGetSymbolAddress, resolved once per device with that device current and kept
// in g_scratch_dev.
constexpr int kScratchSlots = 2 * kDosMaxBins + 2;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_dev[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned long long scratch[kScratchSlots];

namespace {

// Address of the scratch array on the current device (resolved on the first call per device).
int scratch_address(unsigned long long** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_err(CG_EINVAL, "device %d beyond %d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_err(CG_EHIP, "no device address for the scratch array on device %d", dev);
    g_scratch_dev[dev] = (unsigned long long*)p;
  }
  *out = g_scratch_dev[dev];
  return CG_OK;
}

// ---------------------------------------------------------------------------------
// Proposal law of the mixed algorithm on the lattice: displacements d with
// 0 < |d|^2 <= rc^2, weight exp(-2|d|/xi) (section "Hopping conduction", mixed algorithm
// and lattice implementation paragraph).  They are grouped in orbits of the square's
// symmetry group -- all (+-a,+-b), (+-b,+-a) -- ordered by (|d|^2, smaller coordinate);
// members within an orbit in ascending (dy, dx).  Tower sampling: the orbit is the
// first o with w1 < thr[o], thr[o] = floor(2^32 * cumulative weight / total); the
// member is w3 & (size - 1) (sizes are 4 or 8).
struct HostTables {
  int32_t n_orb = 0, n_vec = 0, H = 0;
  std::vector<uint32_t> thr, orb;
  std::vector<uint32_t> thr_u;    // pair hops: floor(2^32 * cumulative orbit size / n_vec)
  std::vector<int32_t> vec;
  std::vector<uint8_t> guide;
  std::vector<uint16_t> guide16;  // orbit | 0x8000 when two or more thresholds lie inside the bucket
  std::vector<int32_t> vec8;      // kRaw: [n_orb][8][2] member (dx, dy) packed, FP32 1/|d| bits
  std::vector<double> tdo64;      // kBig: FP64 1/|d| per orbit
  std::vector<double> tab64;  // full folded table
  std::vector<double> tabk64;
  std::vector<float> tabk32;
  std::vector<double> dft_tw;  // [L][2]
  std::vector<double> dft_T;   // [H+1][L]
  double wsum = 0.0, Gamma = 0.0;
};

struct Rep {
  int32_t a, b, r2;
};

int build_tables(const cg_sample_desc& d, int32_t layout, int32_t precision, int32_t fx_waves, HostTables& t) {
  const double rc = d.rc, xi = d.xi;
  const int32_t L = d.L, N = L * L;
  std::vector<Rep> reps;
  const int32_t amax = (int32_t)std::floor(rc) + 1;
  for (int32_t a = 1; a <= amax; ++a)
    for (int32_t b = 0; b <= a; ++b)
      if ((double)(a * a + b * b) <= rc * rc) reps.push_back({a, b, a * a + b * b});
  std::sort(reps.begin(), reps.end(), [](const Rep& p, const Rep& q) {
    return p.r2 != q.r2 ? p.r2 < q.r2 : p.b < q.b;
  });
  const int32_t n_orb = (int32_t)reps.size();
  if (n_orb < 1 || n_orb > 255)
    return set_err(CG_EINVAL, "hop cutoff rc=%g gives %d displacement orbits (1..255 supported)",
                   rc, n_orb);
  t.n_orb = n_orb;
  t.thr.assign(n_orb, 0u);
  t.orb.assign(n_orb, 0u);
  t.vec.clear();
  std::vector<double> cum(n_orb);
  double acc = 0.0;
  for (int32_t o = 0; o < n_orb; ++o) {
    const int32_t a = reps[o].a, b = reps[o].b;
    std::vector<std::pair<int32_t, int32_t>> m;  // (dy, dx)
    const int32_t cand[8][2] = {{a, b}, {-a, b}, {a, -b}, {-a, -b}, {b, a}, {-b, a}, {b, -a}, {-b, -a}};
    for (auto& c : cand) {
      std::pair<int32_t, int32_t> p(c[1], c[0]);
      if (std::find(m.begin(), m.end(), p) == m.end()) m.push_back(p);
    }
    std::sort(m.begin(), m.end());
    const int32_t size = (int32_t)m.size();
    t.orb[o] = (uint32_t)t.vec.size() | ((uint32_t)(size - 1) << 16);
    for (auto& p : m) t.vec.push_back((int32_t)((uint32_t)(p.second & 0xffff) | ((uint32_t)p.first << 16)));
    const double r = std::sqrt((double)reps[o].r2);
    const double w = (double)size * std::exp(-2.0 * r / xi);
    acc = acc + w;
    cum[o] = acc;
  }
  t.n_vec = (int32_t)t.vec.size();
  for (int32_t o = 0; o + 1 < n_orb; ++o) {
    const double c = std::floor(std::ldexp(cum[o] / acc, 32));
    if (!(c < 4294967296.0))
      return set_err(CG_EINVAL, "rc=%g: orbit weights beyond %d are below the 2^-32 resolution", rc, o);
    t.thr[o] = (uint32_t)(uint64_t)c;
  }
  t.thr[n_orb - 1] = 0xffffffffu;  // never compared: the last orbit takes the rest
  // uniform law over the n_vec hop vectors by orbit (the partner offset of a pair hop)
  t.thr_u.assign(n_orb, 0xffffffffu);
  for (int32_t o = 0; o + 1 < n_orb; ++o) {
    const uint64_t upto = (uint64_t)(t.orb[o] & 0xffffu) + (uint64_t)(t.orb[o] >> 16) + 1u;
    t.thr_u[o] = (uint32_t)((upto << 32) / (uint64_t)t.vec.size());
  }
  t.wsum = acc;
  t.Gamma = (double)N * acc;
  // guide: orbit of the smallest w1 in each bucket of width 2^(32 - kGuideBits)
  t.guide.assign(kGuideSize, 0);
  for (int32_t k = 0; k < kGuideSize; ++k) {
    const uint64_t w = (uint64_t)k << (32 - kGuideBits);
    int32_t o = 0;
    while (o < n_orb - 1 && w >= (uint64_t)t.thr[o]) ++o;
    t.guide[k] = (uint8_t)o;
  }
  if (layout == kRaw || layout == kBig || layout == kFx64) {
    // 16-bit guide over buckets [w, w + 2^20): the orbit of the bucket's smallest word, and
    // 0x8000 when the thresholds of two or more orbits before the last lie inside the bucket
    // (a word of the bucket is then more than one comparison away from its orbit)
    t.guide16.assign(kGuide16Size, 0);
    for (int32_t k = 0; k < kGuide16Size; ++k) {
      const uint64_t w = (uint64_t)k << (32 - kGuide16Bits), w_end = w + ((uint64_t)1 << (32 - kGuide16Bits));
      int32_t o = 0;
      while (o < n_orb - 1 && w >= (uint64_t)t.thr[o]) ++o;
      int32_t inside = 0;
      for (int32_t q = o; q < n_orb - 1 && (uint64_t)t.thr[q] < w_end; ++q) ++inside;
      t.guide16[k] = (uint16_t)(o | (inside >= 2 ? 0x8000 : 0));
    }
    // 8 slots per orbit: member m & (size - 1) in slot m, so that slot w3 & 7 is member
    // w3 & (size - 1) for sizes 4 and 8
    t.vec8.assign((size_t)n_orb * 16, 0);
    for (int32_t o = 0; o < n_orb; ++o) {
      const int32_t first = (int32_t)(t.orb[o] & 0xffffu), msk = (int32_t)(t.orb[o] >> 16);
      const double r = std::sqrt((double)reps[o].r2);
      const float td = (float)(1.0 / r);
      int32_t bits;
      std::memcpy(&bits, &td, 4);
      for (int32_t m = 0; m < 8; ++m) {
        t.vec8[(size_t)(o * 8 + m) * 2] = t.vec[first + (m & msk)];
        t.vec8[(size_t)(o * 8 + m) * 2 + 1] = bits;
      }
    }
    t.tdo64.resize(n_orb);
    for (int32_t o = 0; o < n_orb; ++o) t.tdo64[o] = 1.0 / std::sqrt((double)reps[o].r2);
  }
  // 1/r by folded separation (|dy|, |dx|), minimum image, 1/r(0) := 0
  const int32_t H = L / 2, H1 = H + 1;
  t.H = H;
  t.tab64.assign((size_t)H1 * H1, 0.0);
  for (int32_t ay = 0; ay < H1; ++ay)
    for (int32_t ax = 0; ax < H1; ++ax) {
      const int32_t r2 = ax * ax + ay * ay;
      t.tab64[(size_t)ay * H1 + ax] = r2 == 0 ? 0.0 : 1.0 / std::sqrt((double)r2);
    }
  const size_t nk = (layout == kTri || layout == kFx64) ? (size_t)tri_entries(H)
                    : layout == kRaw ? (size_t)fx_tab_entries(L, fx_waves) : layout == kBig ? 0 : (size_t)full_entries(H);
  std::vector<double> k64(nk, 0.0);
  if (layout == kRaw) {
    // row b = dy + L, column u = folded |dx| (zero beyond L/2)
    const int32_t Pp = fx_pitch(L, fx_waves);
    for (int32_t b = 0; b < 2 * L; ++b) {
      const int32_t a = std::abs(b - L), ay = std::min(a, L - a);
      for (int32_t u = 0; u < H1; ++u) k64[(size_t)b * Pp + u] = t.tab64[(size_t)ay * H1 + u];
    }
  } else if (layout != kBig) {
    for (int32_t ay = 0; ay < H1; ++ay)
      for (int32_t ax = 0; ax < H1; ++ax) {
        size_t idx;
        if (layout == kTri || layout == kFx64) {
          const int32_t a = std::max(ay, ax), b = std::min(ay, ax);
          idx = (size_t)(a * (a + 1) / 2 + b);
        } else {
          idx = (size_t)ay * H1 + ax;
        }
        k64[idx] = t.tab64[(size_t)ay * H1 + ax];
      }
  }
  if (precision == CG_FP64) {
    t.tabk64 = std::move(k64);
  } else {
    t.tabk32.resize(nk);
    for (size_t k = 0; k < nk; ++k) t.tabk32[k] = (float)k64[k];
  }
  if (layout == kBig) return CG_OK;  // FP64 form only: no transform-based refresh
  // refresh tables: twiddles (cos, sin)(2 pi j / L) and the x-transform of 1/r,
  // That(k, dy) = sum_dx T(fold dx, fold dy) cos(2 pi k dx / L) -- real because T is even in dx
  const double two_pi = 6.283185307179586;
  t.dft_tw.resize((size_t)2 * L);
  for (int32_t jj = 0; jj < L; ++jj) {
    t.dft_tw[2 * jj] = std::cos(two_pi * (double)jj / (double)L);
    t.dft_tw[2 * jj + 1] = std::sin(two_pi * (double)jj / (double)L);
  }
  t.dft_T.assign((size_t)H1 * L, 0.0);
  for (int32_t k = 0; k < H1; ++k)
    for (int32_t dy = 0; dy < L; ++dy) {
      const int32_t ay = std::min(dy, L - dy);
      double acc2 = 0.0;
      for (int32_t dx = 0; dx < L; ++dx) {
        const int32_t ax = std::min(dx, L - dx);
        acc2 += t.tab64[(size_t)ay * H1 + ax] * t.dft_tw[2 * (size_t)(((int64_t)k * dx) % L)];
      }
      t.dft_T[(size_t)k * L + dy] = acc2;
    }
  return CG_OK;
}

int32_t count_orbits(double rc) {
  int32_t n = 0;
  const int32_t amax = (int32_t)std::floor(rc) + 1;
  for (int32_t a = 1; a <= amax; ++a)
    for (int32_t b = 0; b <= a; ++b)
      if ((double)(a * a + b * b) <= rc * rc) ++n;
  return n;
}

int32_t count_vectors(double rc) {
  int32_t n = 0;
  const int32_t k = (int32_t)std::floor(rc) + 1;
  for (int32_t dx = -k; dx <= k; ++dx)
    for (int32_t dy = -k; dy <= k; ++dy)
      if ((dx || dy) && (double)(dx * dx + dy * dy) <= rc * rc) ++n;
  return n;
}

// ---------------------------------------------------------------------------------
struct SampleLayout {
  size_t tab64, tabk, thr, orb, vec, guide, vec8, guide16, tdo64, dft_tw, dft_T, thr_u, static_end;  // uploaded in one copy
  size_t eps, phi, occ, part, log_label, log_from, log_to, mirror, sel, mirror2, occ2, bar, end;
  int32_t dft, dft_kc, dft_rows;
};

struct Plan {
  int32_t precision = CG_FP64, block = 1024, U = 1, M = 1024, K = 4096, clock = 0, log_cap = 0, timers = 0;
  int32_t use_graph = 0, variant = 0;
  bool use_db = false, use_fx = false, use_fx64 = false;
  bool pair = false;  // some sample proposes pair hops: the pair-hop kernel runs the batch
  bool split = false;  // FP32, largest L above 128: pairs in the arena, value words in LDS
  int32_t max_L = 0;   // the batch's largest lattice
  bool big = false;  // one sample at a time on the whole GPU (large-sample kernel)
  bool wide = false; // one sample at a time on G workgroups, each with a replica (variant 6)
  bool coop = false; // hop kernels run as one cooperative launch per sample (big or wide)
  int32_t spread = 0;  // wide: workgroups per sample (0 = one per CU)
  int32_t layout = kFull, real_bytes = 8, lds_hop = 0, lds_exact = 0, lds_dft = 0, max_N = 0, NC = 1;
  bool any_exact_refresh = false, dft16 = false, dft32 = false, exact = false;
  uint64_t max_labels = 1ull << 32;
  size_t states_off = 0, samples_off = 0, order_off = 0, scratch_off = 0, hist_off = 0, total = 0;
  std::vector<SampleLayout> sl;
  std::vector<int32_t> order;
};

int max_lds_bytes(int32_t* out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int v = 0, w = 0;
  HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (hipDeviceGetAttribute(&w, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) w = 0;
  *out = std::max(v, w);
  return CG_OK;
}

bool big_eligible(int32_t L) { return L >= 128 && L <= 2048 && (L & (L - 1)) == 0; }
bool wide_eligible(int32_t L) { return L >= 16 && L <= 128 && (L & (L - 1)) == 0; }

bool is_cube(const cg_sample_desc& d) { return d.dim == 3; }
int32_t sites_of(const cg_sample_desc& d) { return is_cube(d) ? d.L * d.L * d.L : d.L * d.L; }

// Proposal law on the simple cubic lattice: displacements 0 < |d|^2 <= rc^2, weight
// exp(-2|d|/xi), in orbits of the cube's 48 signed permutations ordered by (|d|^2, largest
// coordinate, middle coordinate); members in ascending (dz, dy, dx); orbit o is the first
// with w1 < thr[o], thr[o] = floor(2^32 * cumulative weight / total); member
// mulhi(w3, size).  orb[o] = first | size << 16, vec = packed (dx, dy, dz).  Table: 1/r by
// folded (|dz|, |dy|, |dx|), 0 at the origin.
struct Rep3 {
  int32_t a, b, c, r2;
};

void cube_reps(double rc, std::vector<Rep3>& reps) {
  reps.clear();
  const int32_t amax = (int32_t)std::floor(rc) + 1;
  for (int32_t a = 1; a <= amax; ++a)
    for (int32_t b = 0; b <= a; ++b)
      for (int32_t c = 0; c <= b; ++c)
        if ((double)(a * a + b * b + c * c) <= rc * rc) reps.push_back({a, b, c, a * a + b * b + c * c});
  std::sort(reps.begin(), reps.end(), [](const Rep3& p, const Rep3& q) {
    if (p.r2 != q.r2) return p.r2 < q.r2;
    if (p.a != q.a) return p.a < q.a;
    return p.b < q.b;
  });
}

int32_t count_vectors3(double rc) {
  int32_t n = 0;
  const int32_t k = (int32_t)std::floor(rc) + 1;
  for (int32_t dz = -k; dz <= k; ++dz)
    for (int32_t dy = -k; dy <= k; ++dy)
      for (int32_t dx = -k; dx <= k; ++dx)
        if ((dx || dy || dz) && (double)(dx * dx + dy * dy + dz * dz) <= rc * rc) ++n;
  return n;
}

int build_tables3(const cg_sample_desc& d, HostTables& t) {
  const int32_t L = d.L, N = L * L * L, H = L / 2, H1 = H + 1;
  std::vector<Rep3> reps;
  cube_reps(d.rc, reps);
  const int32_t n_orb = (int32_t)reps.size();
  if (n_orb < 1) return set_err(CG_EINVAL, "rc=%g gives no hop vector", d.rc);
  t.n_orb = n_orb;
  t.thr.assign(n_orb, 0u);
  t.orb.assign(n_orb, 0u);
  t.vec.clear();
  std::vector<double> cum(n_orb);
  double acc = 0.0;
  for (int32_t o = 0; o < n_orb; ++o) {
    const int32_t abc[3] = {reps[o].a, reps[o].b, reps[o].c};
    std::vector<std::array<int32_t, 3>> m;  // (dz, dy, dx)
    const int32_t perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (auto& pm : perm)
      for (int32_t sg = 0; sg < 8; ++sg) {
        const int32_t dx = abc[pm[0]] * ((sg & 1) ? -1 : 1), dy = abc[pm[1]] * ((sg & 2) ? -1 : 1),
                      dz = abc[pm[2]] * ((sg & 4) ? -1 : 1);
        const std::array<int32_t, 3> v = {dz, dy, dx};
        if (std::find(m.begin(), m.end(), v) == m.end()) m.push_back(v);
      }
    std::sort(m.begin(), m.end());
    t.orb[o] = (uint32_t)t.vec.size() | ((uint32_t)m.size() << 16);
    for (auto& v : m) t.vec.push_back((int32_t)pack3(v[2], v[1], v[0]));
    acc = acc + (double)m.size() * std::exp(-2.0 * std::sqrt((double)reps[o].r2) / d.xi);
    cum[o] = acc;
  }
  t.n_vec = (int32_t)t.vec.size();
  for (int32_t o = 0; o + 1 < n_orb; ++o) {
    const double c = std::floor(std::ldexp(cum[o] / acc, 32));
    if (!(c < 4294967296.0))
      return set_err(CG_EINVAL, "rc=%g: orbit weights beyond %d are below the 2^-32 resolution", d.rc, o);
    t.thr[o] = (uint32_t)(uint64_t)c;
  }
  t.thr[n_orb - 1] = 0xffffffffu;  // never compared: the last orbit takes the rest
  t.wsum = acc;
  t.Gamma = (double)N * acc;
  t.H = H;
  t.tab64.assign((size_t)H1 * H1 * H1, 0.0);
  for (int32_t c = 0; c < H1; ++c)
    for (int32_t b = 0; b < H1; ++b)
      for (int32_t a = 0; a < H1; ++a) {
        const int32_t r2 = a * a + b * b + c * c;
        t.tab64[((size_t)c * H1 + b) * H1 + a] = r2 == 0 ? 0.0 : 1.0 / std::sqrt((double)r2);
      }
  return CG_OK;
}

int validate(const cg_sample_desc& d, int32_t b) {
  const int32_t L = d.L;
  if (d.M < 0 || d.M > (1 << 24) || (d.M & (d.M - 1)) != 0)
    return set_err(CG_EINVAL, "sample %d: M=%d must be 0 or a power of two in [1, 2^24]", b, d.M);
  if (d.dim != 0 && d.dim != 2 && d.dim != 3) return set_err(CG_EINVAL, "sample %d: dim=%d", b, d.dim);
  if (is_cube(d)) {
    if (L < 3 || L > kCubeMaxL) return set_err(CG_EINVAL, "sample %d: cubic L=%d outside [3, %d]", b, L, kCubeMaxL);
    const int32_t N = L * L * L;
    if (d.n_electrons < 1 || d.n_electrons >= N)
      return set_err(CG_EINVAL, "sample %d: n_electrons=%d outside [1, N-1]", b, d.n_electrons);
    if (!(d.W >= 0.0) || !std::isfinite(d.W)) return set_err(CG_EINVAL, "sample %d: W=%g", b, d.W);
    if (!(d.xi > 0.0) || !std::isfinite(d.xi)) return set_err(CG_EINVAL, "sample %d: xi=%g", b, d.xi);
    if (!(d.rc >= 1.0) || !(2.0 * d.rc < (double)L))
      return set_err(CG_EINVAL, "sample %d: rc=%g must satisfy 1 <= rc < L/2 = %g", b, d.rc, 0.5 * L);
    if (!(d.T > 0.0) || !std::isfinite(d.T)) return set_err(CG_EINVAL, "sample %d: T=%g must be > 0", b, d.T);
    if (!std::isfinite(d.E)) return set_err(CG_EINVAL, "sample %d: E=%g", b, d.E);
    if (d.pair != 0.0) return set_err(CG_EINVAL, "sample %d: pair hops run on the square lattice only", b);
    return CG_OK;
  }
  if (!(d.pair >= 0.0) || !(d.pair < 1.0)) return set_err(CG_EINVAL, "sample %d: pair=%g outside [0, 1)", b, d.pair);
  if (L < 3 || (L > 192 && !big_eligible(L)))
    return set_err(CG_EINVAL, "sample %d: L=%d outside [3, 192] and not a power of two in [256, 2048]", b, L);
  const int32_t N = L * L;
  if (d.n_electrons < 1 || d.n_electrons >= N)
    return set_err(CG_EINVAL, "sample %d: n_electrons=%d outside [1, N-1]", b, d.n_electrons);
  if (!(d.W >= 0.0) || !std::isfinite(d.W)) return set_err(CG_EINVAL, "sample %d: W=%g", b, d.W);
  if (!(d.xi > 0.0) || !std::isfinite(d.xi)) return set_err(CG_EINVAL, "sample %d: xi=%g", b, d.xi);
  if (!(d.rc >= 1.0) || !(2.0 * d.rc < (double)L))
    return set_err(CG_EINVAL, "sample %d: rc=%g must satisfy 1 <= rc < L/2 = %g", b, d.rc, 0.5 * L);
  if (!(d.T > 0.0) || !std::isfinite(d.T)) return set_err(CG_EINVAL, "sample %d: T=%g must be > 0", b, d.T);
  if (!std::isfinite(d.E)) return set_err(CG_EINVAL, "sample %d: E=%g", b, d.E);
  return CG_OK;
}

// Offsets of the batch-wide blocks after the samples' regions, and the launch order.
void plan_tail(const cg_sample_desc* s, int32_t n, Plan& p, size_t off) {
  p.samples_off = off; off = align_up(off + sizeof(DevSample) * (size_t)n);
  p.order_off = off;   off = align_up(off + sizeof(int32_t) * (size_t)n);
  p.scratch_off = off; off = align_up(off + 64);
  p.hist_off = off;    off = align_up(off + (size_t)(2 * kDosMaxBins + 2) * 8);
  p.total = off;
  // launch order: largest lattices first (a one-workgroup-per-sample batch finishes
  // with its slowest sample)
  p.order.resize(n);
  for (int32_t b = 0; b < n; ++b) p.order[b] = b;
  std::stable_sort(p.order.begin(), p.order.end(), [&](int32_t a, int32_t c) { return s[a].L > s[c].L; });
}

// Batch of simple cubic samples: FP64 energies and tables in LDS (k_hops3), initial energies
// by k_eps3, no refresh.
int plan_cube(const cg_sample_desc* s, int32_t n, Plan& p, int32_t lds_cap) {
  for (int32_t b = 0; b < n; ++b) {
    if (!is_cube(s[b])) return set_err(CG_EINVAL, "sample %d: a batch is either all square or all cubic", b);
    int rc = validate(s[b], b);
    if (rc != CG_OK) return rc;
  }
  if (p.precision != CG_FP64) return set_err(CG_EINVAL, "cubic lattices run the FP64 form");
  if (p.clock != CG_CLOCK_DET) return set_err(CG_EINVAL, "cubic lattices use the deterministic clock");
  if ((p.variant != 0 && p.variant != 6) || p.block != 1024)
    return set_err(CG_EINVAL, "cubic lattices: variant 0 or 6, block 1024");
  p.layout = kCube;
  p.big = false;
  p.wide = p.coop = p.variant == 6;
  if (p.wide && p.use_graph) return set_err(CG_EINVAL, "use_graph is not available with the label-parallel kernel");
  p.U = 1;
  int32_t need = 0, need_exact = 0, max_N = 0;
  for (int32_t b = 0; b < n; ++b) {
    std::vector<Rep3> reps;
    cube_reps(s[b].rc, reps);
    const int32_t L = s[b].L, N = L * L * L, H1 = L / 2 + 1;
    need = std::max(need, cube_lds(L, (int32_t)reps.size(), count_vectors3(s[b].rc)).total);
    need_exact = std::max(need_exact, align16(((N + 31) / 32) * 4) + H1 * H1 * H1 * 8);
    max_N = std::max(max_N, N);
  }
  if (need > lds_cap) return set_err(CG_ENOSPC, "cubic samples need %d bytes of LDS (%d available)", need, lds_cap);
  if (need_exact + 2 * kInitBlock * 8 > lds_cap)
    return set_err(CG_ENOSPC, "cubic energy kernel needs %d bytes of LDS", need_exact);
  p.lds_hop = need;
  p.lds_exact = need_exact;
  p.max_N = max_N;
  // sites per thread of the hop kernel: the power of two covering the largest lattice
  p.NC = 1;
  while (p.NC * kCubeThreads < max_N) p.NC *= 2;
  size_t off = 0;
  p.sl.resize(n);
  p.states_off = off;
  off = align_up(off + sizeof(SampleState) * (size_t)n);
  for (int32_t b = 0; b < n; ++b) {
    std::vector<Rep3> reps;
    cube_reps(s[b].rc, reps);
    const int32_t L = s[b].L, N = L * L * L, NW = (N + 31) / 32, H1 = L / 2 + 1;
    const int32_t n_orb = (int32_t)reps.size(), n_vec = count_vectors3(s[b].rc);
    const int32_t nblk = (N + kInitBlock - 1) / kInitBlock;
    SampleLayout& q = p.sl[b];
    q.dft = 0;
    q.tab64 = off;     off = align_up(off + (size_t)H1 * H1 * H1 * 8);
    q.tabk = off;
    q.thr = off;       off = align_up(off + (size_t)n_orb * 4);
    q.orb = off;       off = align_up(off + (size_t)n_orb * 4);
    q.vec = off;       off = align_up(off + (size_t)n_vec * 4);
    q.guide = q.vec8 = q.guide16 = q.tdo64 = q.dft_tw = q.dft_T = off;
    q.static_end = off;
    q.eps = off;       off = align_up(off + (size_t)N * 8);
    q.phi = off;       off = align_up(off + (size_t)N * 8);
    q.occ = off;       off = align_up(off + (size_t)NW * 4);
    q.part = off;      off = align_up(off + (size_t)2 * nblk * 8);
    q.log_label = off; off = align_up(off + (size_t)p.log_cap * 8);
    q.log_from = off;  off = align_up(off + (size_t)p.log_cap * 4);
    q.log_to = off;    off = align_up(off + (size_t)p.log_cap * 4);
    q.mirror = q.sel = q.mirror2 = q.occ2 = off;
    q.bar = off;       off = align_up(off + (p.wide ? (size_t)kWideSyncWords * 4 : 0));
    q.end = off;
  }
  plan_tail(s, n, p, off);
  return CG_OK;
}

using BigFn = void (*)(const DevSample*, int32_t, RunArgs);
BigFn pick_big(int32_t L, int32_t U, int32_t clock, int32_t spread, int32_t* grid);

int make_plan(const cg_sample_desc* s, int32_t n, const cg_run_opts* o, Plan& p, bool query_lds) {
  if (!s || n < 1 || n > 65535) return set_err(CG_EINVAL, "need 1..65535 samples (got %d)", n);
  cg_run_opts def{};
  if (!o) o = &def;
  p.precision = o->precision;
  if (p.precision != CG_FP64 && p.precision != CG_FP32_REFRESH)
    return set_err(CG_EINVAL, "precision=%d", o->precision);
  p.block = o->block ? o->block : 1024;
  if (p.block != 1024 && p.block != 512)
    return set_err(CG_EINVAL, "block=%d (the hop kernels run 1024 threads per sample, the exact-geometry "
                   "kernel also 512)", o->block);
  // M: the paper's parallel width, used for the iteration count p = ceil(m / M); the kernel
  // evaluates labels in chunks of 1024 U (the executed hops do not depend on either)
  p.M = o->M ? o->M : 1024;
  if (p.M < 1 || (p.M & (p.M - 1)) != 0 || p.M > (1 << 20))
    return set_err(CG_EINVAL, "M=%d must be a power of two in [1, 2^20]", o->M);
  p.U = p.M > 1024 ? 2 : 1;
  if (o->phase_timers != 0 && o->phase_timers != 1) return set_err(CG_EINVAL, "phase_timers=%d", o->phase_timers);
  p.timers = o->phase_timers;
  if (o->use_graph != 0 && o->use_graph != 1) return set_err(CG_EINVAL, "use_graph=%d", o->use_graph);
  p.use_graph = o->use_graph;
  if (o->variant < 0 || o->variant > 6) return set_err(CG_EINVAL, "variant=%d", o->variant);
  p.variant = o->variant;
  if (o->spread < 0 || (o->spread != 0 && p.variant != 0 && p.variant != 4 && p.variant != 6))
    return set_err(CG_EINVAL, "spread=%d (workgroups per sample of the label-parallel or whole-GPU kernel, or 0)",
                   o->spread);
  p.spread = o->spread;
  p.K = o->K_refresh ? o->K_refresh : 4096;
  if (p.K < 1) return set_err(CG_EINVAL, "K_refresh=%d", o->K_refresh);
  if (p.precision == CG_FP64) p.K = 0;
  p.clock = o->clock_mode;
  if (p.clock != CG_CLOCK_DET && p.clock != CG_CLOCK_GAUSS && p.clock != CG_CLOCK_GAMMA)
    return set_err(CG_EINVAL, "clock_mode=%d", p.clock);
  if (o->log_hops < 0) return set_err(CG_EINVAL, "log_hops=%d", o->log_hops);
  p.log_cap = o->log_hops;
  p.max_labels = o->max_labels_per_call ? o->max_labels_per_call : (1ull << 32);
  p.real_bytes = p.precision == CG_FP64 ? 8 : 4;

  int32_t lds_cap = 163840;
  if (query_lds) {
    int rc = max_lds_bytes(&lds_cap);
    if (rc != CG_OK) return rc;
  }
  if (is_cube(s[0])) return plan_cube(s, n, p, lds_cap);
  // table layout: full (|dy|,|dx|) table if every sample fits, else the triangle
  bool full_fits = true, tri_fits = true, db_fits = true;
  int32_t need_db = 0;
  int32_t max_L_all = 0;
  for (int32_t b = 0; b < n; ++b) max_L_all = std::max(max_L_all, s[b].L);
  for (int32_t b = 0; b < n; ++b) p.pair = p.pair || s[b].pair != 0.0;
  if (p.pair) {
    // the pair-hop kernel: the generic FP64 layout (energies in LDS), one label per thread
    if (p.precision != CG_FP64) return set_err(CG_EINVAL, "pair hops run in the FP64 form");
    if (p.variant != 0 && p.variant != 1)
      return set_err(CG_EINVAL, "variant=%d: pair hops run on their own kernel (variant 0 or 1)", p.variant);
    if (max_L_all > 128) return set_err(CG_EINVAL, "pair hops need every L <= 128 (got %d)", max_L_all);
    if (p.block != 1024) return set_err(CG_EINVAL, "block=%d: the pair-hop kernel runs 1024 threads", p.block);
    p.U = 1;
  }
  p.wide = p.variant == 6;
  if (p.wide) {
    for (int32_t b = 0; b < n; ++b) {
      int rc = validate(s[b], b);
      if (rc != CG_OK) return rc;
      if (!wide_eligible(s[b].L))
        return set_err(CG_EINVAL, "sample %d: L=%d; the label-parallel kernel (variant 6) needs every L a power of two "
                       "in [16, 128]", b, s[b].L);
    }
    if (p.precision != CG_FP64) return set_err(CG_EINVAL, "the label-parallel kernel (variant 6) runs the FP64 form");
    if (p.use_graph) return set_err(CG_EINVAL, "use_graph is not available with the label-parallel kernel");
  }
  p.big = max_L_all > 192 || p.variant == 4 || p.wide;
  p.coop = p.big;
  if (p.big && !p.wide) {
    for (int32_t b = 0; b < n; ++b) {
      int rc = validate(s[b], b);
      if (rc != CG_OK) return rc;
      if (!big_eligible(s[b].L))
        return set_err(CG_EINVAL, "sample %d: L=%d; the whole-GPU kernel (L > 192 or variant 4) needs every L a "
                       "power of two in [128, 2048]", b, s[b].L);
    }
    if (p.precision != CG_FP64) return set_err(CG_EINVAL, "the whole-GPU kernel (L > 192 or variant 4) runs the FP64 form");
    if (p.use_graph) return set_err(CG_EINVAL, "use_graph is not available with the whole-GPU kernel");
    for (int32_t b = 0; b < n && p.spread != 0; ++b) {
      int32_t g = 0;
      if (!pick_big(s[b].L, 1, CG_CLOCK_DET, p.spread, &g))
        return set_err(CG_EINVAL, "sample %d: L=%d has no whole-GPU kernel on %d workgroups", b, s[b].L, p.spread);
    }
  } else if (p.spread != 0 && !p.wide) {
    return set_err(CG_EINVAL, "spread=%d: only the label-parallel and whole-GPU kernels take a workgroup count",
                   p.spread);
  }
  int32_t need_full = 0, need_tri = 0, need_exact = 0, max_N = 0;
  // FP32 form, largest lattice above 128: the pairs stay in the arena and only their value
  // words live in LDS (the proposals' random reads), when every sample's fit
  p.max_L = max_L_all;
  p.split = p.precision == CG_FP32_REFRESH && max_L_all > 128 && !p.pair && !p.big;
  for (int32_t b = 0; b < n && p.split; ++b) {
    const int32_t L = s[b].L, N = L * L, NW = (N + 31) / 32, H = L / 2;
    p.split = hop_lds(N, NW, full_entries(H), count_vectors(s[b].rc), count_orbits(s[b].rc), 4, 4).total <= lds_cap;
  }
  for (int32_t b = 0; b < n && !p.big; ++b) {
    int rc = validate(s[b], b);
    if (rc != CG_OK) return rc;
    const int32_t L = s[b].L, N = L * L, NW = (N + 31) / 32, H = L / 2;
    const int32_t n_orb = count_orbits(s[b].rc), n_vec = count_vectors(s[b].rc);
    // energy bytes in LDS: FP32 value words (registers hold the pairs), FP64 values in place,
    // none when the batch's largest lattice exceeds 128 (energies stay in the arena)
    const int32_t eb = max_L_all > 128 && !p.split ? 0 : p.real_bytes;
    const int32_t f = p.pair ? pair_lds(N, NW, full_entries(H), n_vec, n_orb).total
                             : hop_lds(N, NW, full_entries(H), n_vec, n_orb, eb, p.real_bytes).total;
    const int32_t t = p.pair ? pair_lds(N, NW, tri_entries(H), n_vec, n_orb).total
                             : hop_lds(N, NW, tri_entries(H), n_vec, n_orb, eb, p.real_bytes).total;
    need_full = std::max(need_full, f);
    need_tri = std::max(need_tri, t);
    full_fits = full_fits && f <= lds_cap;
    tri_fits = tri_fits && t <= lds_cap;
    // one-barrier FP32 kernel: two buffers of FP32 value words
    const int32_t dbb = hop_lds(N, NW, full_entries(H), n_vec, n_orb, 8, 4).total;
    need_db = std::max(need_db, dbb);
    db_fits = db_fits && dbb <= lds_cap;
    need_exact = std::max(need_exact, align16(NW * 4) + full_entries(H) * 8);
    max_N = std::max(max_N, N);
  }
  // exact-geometry FP32 kernel: every sample has the same L, 64 or 128
  bool same_L = true;
  int32_t max_orb = 0;
  for (int32_t b = 0; b < n; ++b) {
    same_L = same_L && s[b].L == s[0].L;
    max_orb = std::max(max_orb, count_orbits(s[b].rc));
  }
  const int32_t need_fx = fx_lds(s[0].L, max_orb, p.block / 64).total;
  const bool fx_ok = !p.big && !p.pair && p.precision == CG_FP32_REFRESH && same_L && (s[0].L == 64 || s[0].L == 128) &&
                     need_fx <= lds_cap;
  p.use_fx = fx_ok && (p.variant == 0 || p.variant == 3);
  // exact-geometry FP64 kernel: the same lattices in the FP64 form
  const int32_t need_fx64 = fx64_lds(s[0].L, max_orb).total;
  // (deterministic clock: the stochastic clocks' calls need more registers than the kernel
  // keeps free, and run on the generic kernel; it evaluates chunks of 1024 labels for any M)
  const bool fx64_ok = !p.big && !p.pair && p.precision == CG_FP64 && same_L && (s[0].L == 64 || s[0].L == 128) &&
                       need_fx64 <= lds_cap && p.block == 1024 && p.clock == CG_CLOCK_DET;
  p.use_fx64 = fx64_ok && (p.variant == 0 || p.variant == 5);
  if (p.variant == 5 && !p.use_fx64)
    return set_err(CG_EINVAL, "variant 5 (exact-geometry FP64 kernel) needs the FP64 form, one L in {64, 128} "
                   "for all samples, the deterministic clock and %d bytes of LDS", need_fx64);
  if (p.use_fx64) p.U = 1;
  if (p.variant == 3 && !p.use_fx)
    return set_err(CG_EINVAL, "variant 3 (exact-geometry kernel) needs the FP32 form, one L in {64, 128} "
                   "for all samples and %d bytes of LDS", need_fx);
  if (p.block != 1024 && !p.use_fx)
    return set_err(CG_EINVAL, "block=%d needs the exact-geometry kernel (FP32 form, one L in {64, 128})", p.block);
  // automatic choice otherwise: two barriers (measured faster at L = 128: 81e6 vs 75e6 hops/s)
  p.use_db = p.precision == CG_FP32_REFRESH && max_L_all <= 128 && db_fits && p.variant == 2;
  if (p.variant == 2 && !p.use_db)
    return set_err(CG_EINVAL, "variant 2 (one barrier per hop) needs the FP32 form, L <= 128 and %d bytes of LDS",
                   need_db);
  if (p.big) {
    p.layout = kBig;
    p.lds_hop = big_lds(max_orb).total;
    if (p.wide) {
      for (int32_t b = 0; b < n; ++b) p.lds_hop = std::max(p.lds_hop, wide_lds(s[b].L, max_orb).total);
      if (p.lds_hop > lds_cap)
        return set_err(CG_ENOSPC, "the label-parallel kernel needs %d bytes of LDS (%d available)", p.lds_hop, lds_cap);
    }
  } else if (p.use_fx64) {
    p.layout = kFx64;
    p.lds_hop = need_fx64;
  } else if (p.use_fx) {
    p.layout = kRaw;
    p.lds_hop = need_fx;
  } else if (p.use_db) {
    p.layout = kFull;
    p.lds_hop = need_db;
  } else if (full_fits) {
    p.layout = kFull;
    p.lds_hop = need_full;
  } else if (tri_fits && p.precision == CG_FP64) {
    p.layout = kTri;
    p.lds_hop = need_tri;
  } else {
    return set_err(CG_ENOSPC, "a sample needs %d bytes of LDS for its energies and tables (%d available)",
                   p.precision == CG_FP64 ? need_tri : need_full, lds_cap);
  }
  if (!p.big && need_exact + 2 * kInitBlock * 8 > lds_cap)
    return set_err(CG_ENOSPC, "refresh kernel needs %d bytes of LDS", need_exact);
  p.lds_exact = need_exact;
  if (p.big)
    for (int32_t b = 0; b < n; ++b) max_N = std::max(max_N, s[b].L * s[b].L);
  p.max_N = max_N;

  size_t off = 0;
  p.sl.resize(n);
  p.states_off = off;
  off = align_up(off + sizeof(SampleState) * (size_t)n);
  int32_t max_L = 0;
  for (int32_t b = 0; b < n; ++b) {
    const int32_t L = s[b].L, N = L * L, NW = (N + 31) / 32, H = L / 2;
    const int32_t n_orb = count_orbits(s[b].rc), n_vec = count_vectors(s[b].rc);
    const int32_t ntab = (p.layout == kTri || p.layout == kFx64) ? tri_entries(H)
                         : p.layout == kRaw ? fx_tab_entries(L, p.block / 64) : p.layout == kBig ? 0 : full_entries(H);
    const int32_t nblk = (N + kInitBlock - 1) / kInitBlock;
    const bool bigl = p.layout == kBig, sel16 = p.layout == kRaw || p.layout == kFx64 || bigl;
    max_L = std::max(max_L, L);
    SampleLayout& q = p.sl[b];
    // refresh by Fourier transform when every thread's outputs fit its registers and a
    // frequency chunk fits LDS; otherwise the O(N^2) exact-order kernel refreshes it
    const int32_t G = 1024 / L;
    const int32_t fixed = align16(NW * 4) + L * 16 + 512;
    int32_t kc = std::min<int32_t>(H + 1, (lds_cap - fixed) / (24 * L));
    kc = std::min<int32_t>(kc, kDftItems * 1024 / L);
    q.dft = (!bigl && G >= 1 && (L + G - 1) / G <= kDftRowsMax && kc >= 1) ? 1 : 0;
    q.dft_rows = G >= 1 ? (L + G - 1) / G : 0;
    if (q.dft) (q.dft_rows > 16 ? p.dft32 : p.dft16) = true;
    q.dft_kc = q.dft ? kc : 0;
    if (q.dft) p.lds_dft = std::max(p.lds_dft, fixed + kc * L * 24);
    else p.any_exact_refresh = true;
    q.tab64 = off;     off = align_up(off + (size_t)full_entries(H) * 8);
    q.tabk = off;      off = align_up(off + (size_t)ntab * p.real_bytes);
    q.thr = off;       off = align_up(off + (size_t)n_orb * 4);
    q.orb = off;       off = align_up(off + (size_t)n_orb * 4);
    q.vec = off;       off = align_up(off + (size_t)n_vec * 4);
    q.guide = off;     off = align_up(off + kGuideSize);
    q.vec8 = off;      off = align_up(off + (sel16 ? (size_t)n_orb * 64 : 0));
    q.guide16 = off;   off = align_up(off + (sel16 ? (size_t)kGuide16Size * 2 : 0));
    q.tdo64 = off;     off = align_up(off + (bigl ? (size_t)n_orb * 8 : 0));
    q.dft_tw = off;    off = align_up(off + (bigl ? 0 : (size_t)L * 16));
    q.dft_T = off;     off = align_up(off + (bigl ? 0 : (size_t)(H + 1) * L * 8));
    q.thr_u = off;     off = align_up(off + (size_t)n_orb * 4);
    q.static_end = off;
    // double, or FP32 value + low part; then one 8-byte sink word that the arena-energy hop
    // kernels write in place of the sites beyond L of lanes past the lattice's edge
    q.eps = off;       off = align_up(off + (size_t)N * 8 + 8);
    q.phi = off;       off = align_up(off + (size_t)N * 8);
    q.occ = off;       off = align_up(off + (size_t)NW * 4);
    q.part = off;      off = align_up(off + (size_t)2 * nblk * 8);
    q.log_label = off; off = align_up(off + (size_t)p.log_cap * 8);
    q.log_from = off;  off = align_up(off + (size_t)p.log_cap * 4);
    q.log_to = off;    off = align_up(off + (size_t)p.log_cap * 4);
    // the large-sample kernel's energy mirror; FP32 batches above L = 128 with their value
    // words in LDS: the pairs' low parts during a launch (N + 1 floats, the last a sink)
    q.mirror = off;    off = align_up(off + (bigl ? (size_t)N * 8 : (p.split ? kSplitLoBytes : 0)));
    q.sel = off;       off = align_up(off + (bigl ? sizeof(OccSelect) : 0));
    q.mirror2 = off;   off = align_up(off + (bigl ? (size_t)N * 8 : 0));
    q.occ2 = off;      off = align_up(off + (bigl ? (size_t)NW * 4 : 0));
    q.bar = off;       off = align_up(off + (bigl ? (size_t)kWideSyncWords * 4 : 0));
    q.end = off;
  }
  p.NC = max_L <= 64 ? 1 : (max_L <= 128 ? 2 : 3);
  p.exact = true;
  for (int32_t b = 0; b < n; ++b) p.exact = p.exact && s[b].L == 64 * p.NC;
  plan_tail(s, n, p, off);
  return CG_OK;
}

using HopFn = void (*)(const DevSample*, const int32_t*, RunArgs);

// Kernel geometry from the largest lattice: NC column blocks of 64 and RPW rows per wave;
// "exact" when every sample fills it (L = 64 NC = 16 RPW), which removes all bounds checks.
// Energy storage: FP32 registers + LDS values, FP64 in LDS, both in the arena beyond L = 128.
template <typename R, int U, bool TRI, int MODE>
HopFn pick_geo(int32_t NC, bool exact) {
  if (NC == 1) return exact ? k_hops<R, U, TRI, 1, 4, true, MODE> : k_hops<R, U, TRI, 1, 4, false, MODE>;
  return exact ? k_hops<R, U, TRI, 2, 8, true, MODE> : k_hops<R, U, TRI, 2, 8, false, MODE>;
}

HopFn pick_db(int32_t U, int32_t NC, bool exact) {
  if (NC == 1) {
    if (U == 1) return exact ? k_hops_db<1, 1, 4, true> : k_hops_db<1, 1, 4, false>;
    return exact ? k_hops_db<2, 1, 4, true> : k_hops_db<2, 1, 4, false>;
  }
  if (U == 1) return exact ? k_hops_db<1, 2, 8, true> : k_hops_db<1, 2, 8, false>;
  return exact ? k_hops_db<2, 2, 8, true> : k_hops_db<2, 2, 8, false>;
}

// Whole-GPU kernel for one sample of side L: workgroups of 1024 threads owning SPT sites per
// thread, G = L^2 / (1024 SPT) workgroups.  A grid barrier costs more with more workgroups
// (2.3 us at 64, 3.2 at 128, 5.1 at 256), the update less: measured per hop, L = 512 takes
// 12.1 / 9.2 / 8.4 us on 256 / 128 / 64 workgroups, L = 1024 16.6 / 12.9 / 13.8 us, and
// L = 2048 22.0 us on 256 (128 needs more registers than a thread has).
// `spread` (0 = the size's default) may also select L = 256 on 16 workgroups (four sites per
// thread), the same kernel with several sites per thread at a size the full oracle can check.
template <int U, int CLOCK>
BigFn pick_big_uc(int32_t L, int32_t spread, int32_t* grid) {
  *grid = 0;
  BigFn fn = nullptr;
  int32_t g = 0;
  switch (L) {
    case 128: g = 16; fn = k_hops_big<7, 1, U, CLOCK>; break;
    case 256:
      if (spread == 16) {
        g = 16;
        fn = k_hops_big<8, 4, U, CLOCK>;
      } else {
        g = 64;
        fn = k_hops_big<8, 1, U, CLOCK>;
      }
      break;
    case 512: g = 64; fn = k_hops_big<9, 4, U, CLOCK>; break;
    case 1024: g = 128; fn = k_hops_big<10, 8, U, CLOCK>; break;
    case 2048: g = 256; fn = k_hops_big<11, 16, U, CLOCK>; break;
    default: return nullptr;
  }
  if (spread != 0 && spread != g) return nullptr;
  *grid = g;
  return fn;
}

BigFn pick_big(int32_t L, int32_t U, int32_t clock, int32_t spread, int32_t* grid) {
  if (clock != CG_CLOCK_DET) return U == 1 ? pick_big_uc<1, 1>(L, spread, grid) : pick_big_uc<2, 1>(L, spread, grid);
  return U == 1 ? pick_big_uc<1, 0>(L, spread, grid) : pick_big_uc<2, 0>(L, spread, grid);
}

// Label-parallel kernel for one sample of side L (a replica per workgroup).
template <int U, int CLOCK>
BigFn pick_wide_uc(int32_t L) {
  switch (L) {
    case 16: return k_hops_wide<4, U, CLOCK>;
    case 32: return k_hops_wide<5, U, CLOCK>;
    case 64: return k_hops_wide<6, U, CLOCK>;
    case 128: return k_hops_wide<7, U, CLOCK>;
    default: return nullptr;
  }
}

// Label-parallel kernel for cubic samples: SPT sites per thread of the replica update.
BigFn pick_wide3(int32_t spt) {
  switch (spt) {
    case 1: return k_hops_wide3<1>;
    case 2: return k_hops_wide3<2>;
    case 4: return k_hops_wide3<4>;
    case 8: return k_hops_wide3<8>;
    default: return k_hops_wide3<16>;
  }
}

BigFn pick_wide(int32_t L, int32_t U, int32_t clock) {
  if (clock != CG_CLOCK_DET) return U == 1 ? pick_wide_uc<1, 1>(L) : pick_wide_uc<2, 1>(L);
  return U == 1 ? pick_wide_uc<1, 0>(L) : pick_wide_uc<2, 0>(L);
}

// chunks of 1024 U labels: U labels per thread with 16 waves, 2 U with 8
template <int CLOCK, bool TIM>
HopFn pick_fx_t(int32_t U, int32_t NC, int32_t NW) {
  if (NW == 8) {
    if (NC == 1) return U == 1 ? k_hops_fx<64, 2, CLOCK, 8, TIM> : k_hops_fx<64, 4, CLOCK, 8, TIM>;
    return U == 1 ? k_hops_fx<128, 2, CLOCK, 8, TIM> : k_hops_fx<128, 4, CLOCK, 8, TIM>;
  }
  if (NC == 1) return U == 1 ? k_hops_fx<64, 1, CLOCK, 16, TIM> : k_hops_fx<64, 2, CLOCK, 16, TIM>;
  return U == 1 ? k_hops_fx<128, 1, CLOCK, 16, TIM> : k_hops_fx<128, 2, CLOCK, 16, TIM>;
}

template <int CLOCK>
HopFn pick_fx(int32_t U, int32_t NC, int32_t NW, bool timers) {
  return timers ? pick_fx_t<CLOCK, true>(U, NC, NW) : pick_fx_t<CLOCK, false>(U, NC, NW);
}

// Pair-hop kernel (FP64, L <= 128): geometry from the largest lattice as pick_geo.
HopFn pick_pair(int32_t layout, int32_t NC, bool exact) {
  if (layout == kTri) {
    if (NC == 1) return exact ? k_hops_pair<true, 1, 4, true> : k_hops_pair<true, 1, 4, false>;
    return exact ? k_hops_pair<true, 2, 8, true> : k_hops_pair<true, 2, 8, false>;
  }
  if (NC == 1) return exact ? k_hops_pair<false, 1, 4, true> : k_hops_pair<false, 1, 4, false>;
  return exact ? k_hops_pair<false, 2, 8, true> : k_hops_pair<false, 2, 8, false>;
}

HopFn pick_hop(int32_t precision, int32_t U, int32_t layout, int32_t NC, bool exact, bool db, int32_t clock,
              int32_t block, bool timers, bool split, bool rows10) {
  if (layout == kCube) {
    switch (NC) {
      case 1: return k_hops3<1>;
      case 2: return k_hops3<2>;
      case 4: return k_hops3<4>;
      case 8: return k_hops3<8>;
      default: return k_hops3<16>;
    }
  }
  if (layout == kFx64) return NC == 1 ? k_hops_fx64<64, 1, 0> : k_hops_fx64<128, 1, 0>;
  if (layout == kRaw)
    return clock != CG_CLOCK_DET ? pick_fx<1>(U, NC, block / 64, timers) : pick_fx<0>(U, NC, block / 64, timers);
  if (db) return pick_db(U, NC, exact);
  // FP32, L > 128: pairs in the arena, value words in LDS; up to L = 160 the instance with 10
  // rows per wave (16 x 10 rows: no wave runs an idle row group)
  if (NC >= 3 && split)
    return rows10 ? (U == 1 ? k_hops<float, 1, false, 3, 10, false, kModeSplit> : k_hops<float, 2, false, 3, 10, false, kModeSplit>)
                  : (U == 1 ? k_hops<float, 1, false, 3, 12, false, kModeSplit> : k_hops<float, 2, false, 3, 12, false, kModeSplit>);
  if (NC >= 3) {  // L > 128: energies in the arena
    if (precision == CG_FP64) return k_hops<double, 1, false, 3, 12, false, kModeGlobal>;
    return k_hops<float, 1, false, 3, 12, false, kModeGlobal>;
  }
  if (precision == CG_FP64) {
    if (layout == kTri)
      return U == 1 ? pick_geo<double, 1, true, kModeLds>(NC, exact) : pick_geo<double, 2, true, kModeLds>(NC, exact);
    return U == 1 ? pick_geo<double, 1, false, kModeLds>(NC, exact) : pick_geo<double, 2, false, kModeLds>(NC, exact);
  }
  return U == 1 ? pick_geo<float, 1, false, kModeReg>(NC, exact) : pick_geo<float, 2, false, kModeReg>(NC, exact);
}

}  // namespace

// ---------------------------------------------------------------------------------
struct cg_ctx {
  Plan plan;
  std::vector<cg_sample_desc> desc;
  std::vector<DevSample> dev;
  uint8_t* arena = nullptr;
  hipStream_t stream = nullptr;
  DevSample* d_samples = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_pending = nullptr;
  HopFn hop = nullptr;
  std::vector<std::pair<BigFn, int32_t>> big;  // whole-GPU kernel and grid per sample
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_hop, ev_ref;
  double acc_hop_ms = 0.0, acc_ref_ms = 0.0;
  int64_t n_hop = 0, n_ref = 0;
  // hops since the last refresh when every sample is known to have the same count
  // (true from creation until a run-to-time call or a stall); -1 when unknown
  int64_t lockstep_since = 0;
  // captured launch sequences of cg_run_hops, keyed by (n_hops, lockstep_since)
  struct Graph {
    int64_t n_hops, since0, since1;
    int32_t hop_launches, ref_launches;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  bool capturing = false;
  double acc_graph_ms = 0.0;
  int64_t n_graph = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_graph;
  // device address of the file-scope scratch array on the device current at creation
  unsigned long long* scratch_dev = nullptr;
};

namespace {

int fold_events(std::vector<std::pair<hipEvent_t, hipEvent_t>>& ev, double& acc) {
  for (auto& e : ev) {
    HIPCHK(hipEventSynchronize(e.second));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
    acc += ms;
    HIPCHK(hipEventDestroy(e.first));
    HIPCHK(hipEventDestroy(e.second));
  }
  ev.clear();
  return CG_OK;
}

int ev_begin(cg_ctx* c, std::vector<std::pair<hipEvent_t, hipEvent_t>>& ev, double& acc,
             hipEvent_t* start) {
  if (ev.size() >= 1024) {
    int rc = fold_events(ev, acc);
    if (rc != CG_OK) return rc;
  }
  HIPCHK(hipEventCreate(start));
  HIPCHK(hipEventRecord(*start, c->stream));
  return CG_OK;
}

int ev_end(cg_ctx* c, std::vector<std::pair<hipEvent_t, hipEvent_t>>& ev, hipEvent_t start) {
  hipEvent_t stop;
  HIPCHK(hipEventCreate(&stop));
  HIPCHK(hipEventRecord(stop, c->stream));
  ev.emplace_back(start, stop);
  return CG_OK;
}

int launch_hops(cg_ctx* c, int time_mode) {
  if (c->capturing) {
    const Plan& p = c->plan;
    RunArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.K = p.K;
    ra.time_mode = time_mode;
    ra.clock_mode = p.clock;
    ra.timers = p.timers;
    ra.max_labels = p.max_labels;
    hipLaunchKernelGGL(c->hop, dim3((int32_t)c->desc.size()), dim3(p.block), p.lds_hop, c->stream, c->d_samples,
                       c->d_order, ra);
    HIPCHK(hipGetLastError());
    ++c->n_hop;
    return CG_OK;
  }
  const Plan& p = c->plan;
  RunArgs ra;
  std::memset(&ra, 0, sizeof(ra));
  ra.K = p.K;
  ra.time_mode = time_mode;
  ra.clock_mode = p.clock;
  ra.timers = p.timers;
  ra.max_labels = p.max_labels;
  hipEvent_t start;
  int rc = ev_begin(c, c->ev_hop, c->acc_hop_ms, &start);
  if (rc != CG_OK) return rc;
  const int32_t n = (int32_t)c->desc.size();
  if (p.coop) {
    // one cooperative launch per sample, each on the whole GPU
    for (int32_t b = 0; b < n; ++b) {
      const DevSample* ds = c->d_samples;
      int32_t sb = b;
      if (p.wide) hipLaunchKernelGGL(k_wide_reset, dim3(1), dim3(64), 0, c->stream, c->d_samples, b);
      else hipLaunchKernelGGL(k_bar_reset, dim3(1), dim3(64), 0, c->stream, c->d_samples, b);
      HIPCHK(hipGetLastError());
      void* args[] = {(void*)&ds, (void*)&sb, (void*)&ra};
      HIPCHK(hipLaunchCooperativeKernel((const void*)c->big[b].first, dim3(c->big[b].second), dim3(1024), args,
                                        (unsigned)p.lds_hop, c->stream));
    }
  } else {
    hipLaunchKernelGGL(c->hop, dim3(n), dim3(p.block), p.lds_hop, c->stream, c->d_samples, c->d_order, ra);
    HIPCHK(hipGetLastError());
  }
  ++c->n_hop;
  return ev_end(c, c->ev_hop, start);
}

int launch_exact(cg_ctx* c, int refresh) {
  const Plan& p = c->plan;
  const int32_t n = (int32_t)c->desc.size();
  const dim3 grid((p.max_N + kInitBlock - 1) / kInitBlock, n);
  hipEvent_t start = nullptr;
  const bool timed = refresh && !c->capturing;
  if (refresh) {
    if (timed) {
      int rc = ev_begin(c, c->ev_ref, c->acc_ref_ms, &start);
      if (rc != CG_OK) return rc;
    }
    if (p.precision != CG_FP64 && p.dft16) {
      hipLaunchKernelGGL((k_refresh_dft<float, 16>), dim3(n), dim3(1024), p.lds_dft, c->stream, c->d_samples, p.K);
      HIPCHK(hipGetLastError());
    }
    if (p.precision != CG_FP64 && p.dft32) {
      hipLaunchKernelGGL((k_refresh_dft<float, 32>), dim3(n), dim3(1024), p.lds_dft, c->stream, c->d_samples, p.K);
      HIPCHK(hipGetLastError());
    }
  }
  if (p.layout == kCube) {
    // FP64 form: the initial energies, or a forced recompute (cg_refresh)
    hipLaunchKernelGGL(k_eps3, grid, dim3(kInitBlock), p.lds_exact, c->stream, c->d_samples, refresh);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_finalize, dim3(n), dim3(64), 0, c->stream, c->d_samples, refresh, p.K);
    HIPCHK(hipGetLastError());
  } else if (p.big) {
    for (int32_t b = 0; b < n; ++b) {
      const int32_t nb = (c->desc[b].L * c->desc[b].L + kInitBlock - 1) / kInitBlock;
      hipLaunchKernelGGL(k_eps_big, dim3(nb), dim3(kInitBlock), 0, c->stream, c->d_samples + b, refresh);
    }
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_finalize, dim3(n), dim3(64), 0, c->stream, c->d_samples, refresh, p.K);
    HIPCHK(hipGetLastError());
  } else if (!refresh || p.any_exact_refresh || p.precision == CG_FP64) {
    if (p.precision == CG_FP64)
      hipLaunchKernelGGL(k_eps_exact<double>, grid, dim3(kInitBlock), p.lds_exact, c->stream, c->d_samples,
                         refresh, p.K);
    else
      hipLaunchKernelGGL(k_eps_exact<float>, grid, dim3(kInitBlock), p.lds_exact, c->stream, c->d_samples,
                         refresh, p.K);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_finalize, dim3(n), dim3(64), 0, c->stream, c->d_samples, refresh, p.K);
    HIPCHK(hipGetLastError());
  }
  if (refresh) ++c->n_ref;
  if (timed) return ev_end(c, c->ev_ref, start);
  return CG_OK;
}

int read_states(cg_ctx* c, std::vector<SampleState>& out) {
  const int32_t n = (int32_t)c->desc.size();
  out.resize(n);
  HIPCHK(hipMemcpyAsync(out.data(), c->arena + c->plan.states_off, sizeof(SampleState) * n, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CG_OK;
}

int check_stall(cg_ctx* c) {
  std::vector<SampleState> st;
  int rc = read_states(c, st);
  if (rc != CG_OK) return rc;
  for (size_t b = 0; b < st.size(); ++b)
    if (st[b].status == -3)
      return set_err(CG_EHIP, "sample %zu: a workgroup of the whole-GPU kernel missed a grid barrier", b);
  for (size_t b = 0; b < st.size(); ++b)
    if (st[b].status != 0)
      return set_err(CG_ESTALL, "sample %zu reached the label cap (%llu labels) before its target", b,
                     (unsigned long long)c->plan.max_labels);
  return CG_OK;
}

int sample_ok(cg_ctx* c, int32_t b) {
  if (!c) return set_err(CG_EINVAL, "null context");
  if (b < 0 || b >= (int32_t)c->desc.size()) return set_err(CG_EINVAL, "sample index %d out of range", b);
  return CG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------
extern "C" {

const char* cg_last_error(void) { return g_err; }

int cg_arena_bytes(const cg_sample_desc* samples, int32_t n, const cg_run_opts* opts, size_t* bytes) {
  if (!bytes) return set_err(CG_EINVAL, "null output");
  Plan p;
  int rc = make_plan(samples, n, opts, p, false);
  if (rc != CG_OK) return rc;
  *bytes = p.total;
  return CG_OK;
}

int cg_create(cg_ctx** out, const cg_sample_desc* samples, int32_t n, const cg_run_opts* opts, void* arena,
              size_t arena_bytes, void* hip_stream) {
  if (!out) return set_err(CG_EINVAL, "null output");
  *out = nullptr;
  g_err[0] = 0;
  Plan p;
  int rc = make_plan(samples, n, opts, p, true);
  if (rc != CG_OK) return rc;
  if (!arena) return set_err(CG_EINVAL, "null arena");
  if ((uintptr_t)arena % kAlign != 0) return set_err(CG_EINVAL, "arena must be %zu-byte aligned", kAlign);
  if (arena_bytes < p.total) return set_err(CG_ENOSPC, "arena has %zu bytes, needs %zu", arena_bytes, p.total);

  cg_ctx* c = new cg_ctx();
  c->plan = p;
  c->desc.assign(samples, samples + n);
  c->arena = (uint8_t*)arena;
  c->stream = (hipStream_t)hip_stream;
  {
    const int r = scratch_address(&c->scratch_dev);
    if (r != CG_OK) {
      delete c;
      return r;
    }
  }
  c->d_samples = (DevSample*)(c->arena + p.samples_off);
  c->d_order = (int32_t*)(c->arena + p.order_off);
  c->d_pending = (int32_t*)(c->arena + p.scratch_off);
  if (p.coop) {
    int ncu = 0, dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    c->big.resize(n);
    for (int32_t b = 0; b < n && e == hipSuccess; ++b) {
      int32_t g = 0;
      BigFn fn = nullptr;
      if (p.wide) {
        fn = p.layout == kCube ? pick_wide3(p.NC) : pick_wide(samples[b].L, p.U, p.clock);
        g = p.spread ? p.spread : ncu;
        if (fn) e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_hop);
      } else {
        fn = pick_big(samples[b].L, p.U, p.clock, p.spread, &g);
      }
      int per_cu = 0;
      if (fn) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, 1024, p.lds_hop);
      if (e == hipSuccess && (!fn || (int64_t)per_cu * ncu < g)) {
        delete c;
        return set_err(CG_ENOSPC, "sample %d: the whole-GPU kernel needs %d co-resident workgroups (%d x %d available)",
                       b, g, per_cu, ncu);
      }
      c->big[b] = {fn, g};
    }
    if (e != hipSuccess) {
      delete c;
      return set_err(CG_EHIP, "whole-GPU kernel set-up: %s", hipGetErrorString(e));
    }
  } else {
    c->hop = p.pair ? pick_pair(p.layout, p.NC, p.exact)
                    : pick_hop(p.precision, p.U, p.layout, p.NC, p.exact, p.use_db, p.clock, p.block, p.timers != 0,
                               p.split, p.max_L <= 160);
  }

  auto fail = [&](int code) {
    delete c;
    return code;
  };
  // host staging of every sample's static blocks (state, tables), then one copy each
  std::vector<std::vector<uint8_t>> staging(n);
  c->dev.resize(n);
  for (int32_t b = 0; b < n; ++b) {
    const cg_sample_desc& d = samples[b];
    const SampleLayout& q = p.sl[b];
    HostTables t;
    rc = p.layout == kCube ? build_tables3(d, t) : build_tables(d, p.layout, p.precision, p.block / 64, t);
    if (rc != CG_OK) return fail(rc);
    const int32_t L = d.L, N = sites_of(d);
    const uint32_t magic = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)L - 1) / (uint64_t)L);
    for (int32_t i = 0; i < N; ++i)
      if ((int32_t)(((uint64_t)i * magic) >> 32) != i / L)
        return fail(set_err(CG_EINVAL, "internal: row division check failed for L=%d", L));
    std::vector<uint8_t>& sb = staging[b];
    sb.assign(q.static_end - q.tab64, 0);
    uint8_t* base = sb.data() - q.tab64;
    std::memcpy(base + q.tab64, t.tab64.data(), t.tab64.size() * 8);
    if (p.layout == kCube)
      ;  // no kernel table beyond the FP64 one
    else if (p.precision == CG_FP64)
      std::memcpy(base + q.tabk, t.tabk64.data(), t.tabk64.size() * 8);
    else
      std::memcpy(base + q.tabk, t.tabk32.data(), t.tabk32.size() * 4);
    std::memcpy(base + q.thr, t.thr.data(), t.thr.size() * 4);
    if (!t.thr_u.empty()) std::memcpy(base + q.thr_u, t.thr_u.data(), t.thr_u.size() * 4);
    std::memcpy(base + q.orb, t.orb.data(), t.orb.size() * 4);
    std::memcpy(base + q.vec, t.vec.data(), t.vec.size() * 4);
    std::memcpy(base + q.guide, t.guide.data(), t.guide.size());
    if (p.layout == kRaw || p.layout == kBig || p.layout == kFx64) {
      std::memcpy(base + q.vec8, t.vec8.data(), t.vec8.size() * 4);
      std::memcpy(base + q.guide16, t.guide16.data(), t.guide16.size() * 2);
    }
    if (p.layout == kBig) std::memcpy(base + q.tdo64, t.tdo64.data(), t.tdo64.size() * 8);
    std::memcpy(base + q.dft_tw, t.dft_tw.data(), t.dft_tw.size() * 8);
    std::memcpy(base + q.dft_T, t.dft_T.data(), t.dft_T.size() * 8);

    DevSample& s = c->dev[b];
    std::memset(&s, 0, sizeof(s));
    s.L = L;
    s.N = N;
    s.H = t.H;
    s.n_e = d.n_electrons;
    s.NW = (N + 31) / 32;
    s.n_orb = t.n_orb;
    s.n_vec = t.n_vec;
    s.ntab = (p.layout == kTri || p.layout == kFx64) ? tri_entries(t.H)
             : p.layout == kRaw  ? fx_tab_entries(L, p.block / 64)
             : p.layout == kCube ? (t.H + 1) * (t.H + 1) * (t.H + 1)
                                 : full_entries(t.H);
    s.nblk = (N + kInitBlock - 1) / kInitBlock;
    s.log_cap = p.log_cap;
    s.layout = p.layout;
    s.dft = q.dft;
    s.dft_kc = q.dft_kc;
    s.dft_rows = q.dft_rows;
    {
      const int32_t Mw = d.M ? d.M : p.M;  // the sample's PR width
      s.log2M = 0;
      while ((1 << s.log2M) < Mw) ++s.log2M;
    }
    s.seed_lo = (uint32_t)d.seed;
    s.seed_hi = (uint32_t)(d.seed >> 32);
    s.sample_id = d.sample_id;
    s.magic_L = magic;
    s.nu = (double)d.n_electrons / (double)N;
    s.W = d.W;
    s.T = d.T;
    s.mrT = -1.0 / d.T;
    s.E = d.E;
    // labels arrive at Gamma / (1 - pair): the clock's rate (Gamma itself without pair hops)
    s.Gamma = t.Gamma / (1.0 - d.pair);
    s.thr_pair = (uint32_t)(uint64_t)std::floor(std::ldexp(d.pair, 32));
    s.pair_r2 = (int32_t)std::floor(d.rc * d.rc);
    s.T32 = (float)d.T;
    s.E32 = (float)d.E;
    s.invT32 = (float)(1.0 / d.T);
    s.mTln2_32 = (float)(-d.T * 0.6931471805599453);
    uint8_t* a = c->arena;
    s.st = (SampleState*)(a + p.states_off) + b;
    s.eps = a + q.eps;
    s.phi = (double*)(a + q.phi);
    s.occ = (uint32_t*)(a + q.occ);
    s.tab64 = (const double*)(a + q.tab64);
    s.tabk = a + q.tabk;
    s.thr = (const uint32_t*)(a + q.thr);
    s.orb = (const uint32_t*)(a + q.orb);
    s.vec = (const int32_t*)(a + q.vec);
    s.guide = a + q.guide;
    s.vec8 = (const int32_t*)(a + q.vec8);
    s.guide16 = (const uint16_t*)(a + q.guide16);
    s.tdo64 = (const double*)(a + q.tdo64);
    s.mirror = (double*)(a + q.mirror);
    s.mirror2 = (double*)(a + q.mirror2);
    s.occ2 = (uint32_t*)(a + q.occ2);
    s.bar = (uint32_t*)(a + q.bar);
    s.part = (double*)(a + q.part);
    s.dft_tw = (const double*)(a + q.dft_tw);
    s.dft_T = (const double*)(a + q.dft_T);
    s.log_label = (uint64_t*)(a + q.log_label);
    s.log_from = (int32_t*)(a + q.log_from);
    s.log_to = (int32_t*)(a + q.log_to);
    s.thr_u = (const uint32_t*)(a + q.thr_u);
  }
#define HIPCHK_C(expr)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(set_err(CG_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                          __LINE__));                                                      \
  } while (0)
  for (int32_t b = 0; b < n; ++b)
    HIPCHK_C(hipMemcpyAsync(c->arena + p.sl[b].tab64, staging[b].data(), staging[b].size(), hipMemcpyHostToDevice,
                            c->stream));
  {
    std::vector<SampleState> zero(n);
    std::memset(zero.data(), 0, sizeof(SampleState) * n);
    HIPCHK_C(hipMemcpyAsync(c->arena + p.states_off, zero.data(), sizeof(SampleState) * n, hipMemcpyHostToDevice,
                            c->stream));
    HIPCHK_C(hipStreamSynchronize(c->stream));
  }
  HIPCHK_C(hipMemcpyAsync(c->d_samples, c->dev.data(), sizeof(DevSample) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK_C(hipMemcpyAsync(c->d_order, p.order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));

  if (!p.coop)
    HIPCHK_C(hipFuncSetAttribute((const void*)c->hop, hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_hop));
  if (p.layout == kCube) {
    HIPCHK_C(hipFuncSetAttribute((const void*)k_eps3, hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_exact));
  } else if (p.precision == CG_FP64) {
    HIPCHK_C(hipFuncSetAttribute((const void*)k_eps_exact<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 p.lds_exact));
  } else {
    HIPCHK_C(hipFuncSetAttribute((const void*)k_eps_exact<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 p.lds_exact));
    if (p.lds_dft > 0) {
      HIPCHK_C(hipFuncSetAttribute((const void*)k_refresh_dft<float, 16>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_dft));
      HIPCHK_C(hipFuncSetAttribute((const void*)k_refresh_dft<float, 32>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_dft));
    }
  }

  // random initial state and FP64 energies, all on the device
  const dim3 grid((p.max_N + kInitBlock - 1) / kInitBlock, n);
  hipLaunchKernelGGL(k_init_keys, grid, dim3(kInitBlock), 0, c->stream, c->d_samples);
  HIPCHK_C(hipGetLastError());
  if (p.big) {
    // exact selection of the n_e smallest keys, one sample at a time
    for (int32_t b = 0; b < n; ++b) {
      const DevSample* ds = c->d_samples + b;
      OccSelect* sel = (OccSelect*)(c->arena + p.sl[b].sel);
      const int32_t nb = (samples[b].L * samples[b].L + kInitBlock - 1) / kInitBlock;
      hipLaunchKernelGGL(k_occ_clear, dim3(65536 / kInitBlock), dim3(kInitBlock), 0, c->stream, sel);
      hipLaunchKernelGGL(k_occ_hist, dim3(nb), dim3(kInitBlock), 0, c->stream, ds, sel);
      hipLaunchKernelGGL(k_occ_select, dim3(1), dim3(1024), 0, c->stream, ds, sel);
      hipLaunchKernelGGL(k_occ_collect, dim3(nb), dim3(kInitBlock), 0, c->stream, ds, sel);
      hipLaunchKernelGGL(k_occ_threshold, dim3(1), dim3(1024), 0, c->stream, ds, sel);
      hipLaunchKernelGGL(k_occ_mark, dim3(nb), dim3(kInitBlock), 0, c->stream, ds, sel);
      HIPCHK_C(hipGetLastError());
    }
  } else {
    hipLaunchKernelGGL(k_init_rank, grid, dim3(kInitBlock), 0, c->stream, c->d_samples);
    HIPCHK_C(hipGetLastError());
  }
  hipLaunchKernelGGL(k_init_phi, grid, dim3(kInitBlock), 0, c->stream, c->d_samples);
  HIPCHK_C(hipGetLastError());
  rc = launch_exact(c, 0);
  if (rc != CG_OK) return fail(rc);
  HIPCHK_C(hipStreamSynchronize(c->stream));
  if (p.big) {
    for (int32_t b = 0; b < n; ++b) {
      uint32_t ovf = 0;
      HIPCHK_C(hipMemcpy(&ovf, c->arena + p.sl[b].sel + offsetof(OccSelect, overflow), 4, hipMemcpyDeviceToHost));
      if (ovf) return fail(set_err(CG_EHIP, "sample %d: initial-occupation selection overflow", b));
    }
  }
#undef HIPCHK_C
  *out = c;
  return CG_OK;
}

int cg_destroy(cg_ctx* c) {
  if (!c) return CG_OK;
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev_hop) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& e : c->ev_ref) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& e : c->ev_graph) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  delete c;
  return CG_OK;
}

namespace {

// Enqueue the launch sequence of run_hops(n_hops) (no synchronisation, no host reads).
int enqueue_run_hops(cg_ctx* c, int64_t n_hops) {
  const int32_t n = (int32_t)c->desc.size();
  hipLaunchKernelGGL(k_begin_call, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->d_samples, n, n_hops, -1.0, 0);
  HIPCHK(hipGetLastError());
  int rc;
  if (c->plan.precision == CG_FP64) {
    rc = launch_hops(c, 0);
    if (rc != CG_OK) return rc;
  } else if (c->lockstep_since >= 0) {
    // every sample has the same hops-since-refresh: launch exactly one hop kernel per
    // refresh interval and a refresh where an interval completes
    const int64_t K = c->plan.K;
    int64_t left = n_hops, since = c->lockstep_since;
    while (left > 0) {
      const int64_t k = std::min(left, K - since);
      rc = launch_hops(c, 0);
      if (rc != CG_OK) return rc;
      left -= k;
      since += k;
      if (since == K) {
        rc = launch_exact(c, 1);
        if (rc != CG_OK) return rc;
        since = 0;
      }
    }
    c->lockstep_since = since;
  } else {
    // unknown per-sample counts: at most ceil(n/K) + 1 launches; finished samples exit at once
    const int64_t K = c->plan.K;
    const int64_t rounds = (n_hops + K - 1) / K + 1;
    for (int64_t r = 0; r < rounds; ++r) {
      rc = launch_hops(c, 0);
      if (rc != CG_OK) return rc;
      rc = launch_exact(c, 1);
      if (rc != CG_OK) return rc;
    }
  }
  return CG_OK;
}

}  // namespace

int cg_run_hops(cg_ctx* c, int64_t n_hops) {
  if (!c) return set_err(CG_EINVAL, "null context");
  if (n_hops < 1) return set_err(CG_EINVAL, "n_hops=%lld must be >= 1", (long long)n_hops);
  int rc;
  const bool graph = c->plan.use_graph && (c->plan.precision == CG_FP64 || c->lockstep_since >= 0);
  if (!graph) {
    rc = enqueue_run_hops(c, n_hops);
    if (rc != CG_OK) return rc;
  } else {
    // replay the captured launch sequence of this (n_hops, refresh phase); capture on first use
    const int64_t since0 = c->lockstep_since;
    cg_ctx::Graph* g = nullptr;
    for (auto& e : c->graphs)
      if (e.n_hops == n_hops && e.since0 == since0) g = &e;
    if (!g) {
      cg_ctx::Graph e;
      e.n_hops = n_hops;
      e.since0 = since0;
      const int64_t h0 = c->n_hop, r0 = c->n_ref;
      HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      c->capturing = true;
      rc = enqueue_run_hops(c, n_hops);
      c->capturing = false;
      hipGraph_t graph_ = nullptr;
      const hipError_t ec = hipStreamEndCapture(c->stream, &graph_);
      if (rc != CG_OK) {
        if (graph_) (void)hipGraphDestroy(graph_);
        return rc;
      }
      if (ec != hipSuccess)
        return set_err(CG_EHIP, "stream capture failed (%s); graph replay needs a non-default stream",
                       hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&e.exec, graph_, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph_);
      HIPCHK(ei);
      e.since1 = c->lockstep_since;
      e.hop_launches = (int32_t)(c->n_hop - h0);
      e.ref_launches = (int32_t)(c->n_ref - r0);
      c->n_hop = h0;
      c->n_ref = r0;
      c->lockstep_since = since0;
      c->graphs.push_back(e);
      g = &c->graphs.back();
    }
    hipEvent_t start;
    rc = ev_begin(c, c->ev_graph, c->acc_graph_ms, &start);
    if (rc != CG_OK) return rc;
    HIPCHK(hipGraphLaunch(g->exec, c->stream));
    rc = ev_end(c, c->ev_graph, start);
    if (rc != CG_OK) return rc;
    ++c->n_graph;
    c->n_hop += g->hop_launches;
    c->n_ref += g->ref_launches;
    c->lockstep_since = g->since1;
  }
  rc = check_stall(c);
  if (rc == CG_ESTALL) c->lockstep_since = -1;
  return rc;
}

int cg_run_time(cg_ctx* c, double t_end) {
  if (!c) return set_err(CG_EINVAL, "null context");
  if (!(t_end >= 0.0) || !std::isfinite(t_end)) return set_err(CG_EINVAL, "t_end=%g", t_end);
  const int32_t n = (int32_t)c->desc.size();
  hipLaunchKernelGGL(k_begin_call, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->d_samples, n, (int64_t)0,
                     t_end, 1);
  HIPCHK(hipGetLastError());
  c->lockstep_since = -1;
  for (;;) {
    int rc = launch_hops(c, 1);
    if (rc != CG_OK) return rc;
    if (c->plan.precision != CG_FP64) {
      rc = launch_exact(c, 1);
      if (rc != CG_OK) return rc;
    }
    hipLaunchKernelGGL(k_pending, dim3(1), dim3(256), 0, c->stream, c->d_samples, n, c->d_pending);
    HIPCHK(hipGetLastError());
    int32_t pending = 0;
    HIPCHK(hipMemcpyAsync(&pending, c->d_pending, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (pending == 0) break;
  }
  return check_stall(c);
}

int cg_refresh(cg_ctx* c) {
  if (!c) return set_err(CG_EINVAL, "null context");
  const int32_t n = (int32_t)c->desc.size();
  hipLaunchKernelGGL(k_force_refresh, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->d_samples, n);
  HIPCHK(hipGetLastError());
  int rc = launch_exact(c, 1);
  if (rc != CG_OK) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->lockstep_since >= 0) c->lockstep_since = 0;
  return CG_OK;
}

int cg_set_TE(cg_ctx* c, int32_t b, double T, double E) {
  int rc = sample_ok(c, b);
  if (rc != CG_OK) return rc;
  if (!(T > 0.0) || !std::isfinite(T) || !std::isfinite(E)) return set_err(CG_EINVAL, "T=%g E=%g", T, E);
  c->desc[b].T = T;
  c->desc[b].E = E;
  DevSample& s = c->dev[b];
  s.T = T;
  s.mrT = -1.0 / T;
  s.E = E;
  s.T32 = (float)T;
  s.E32 = (float)E;
  s.invT32 = (float)(1.0 / T);
  s.mTln2_32 = (float)(-T * 0.6931471805599453);
  HIPCHK(hipMemcpyAsync(c->d_samples + b, &s, sizeof(DevSample), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CG_OK;
}

int cg_get_occupation(cg_ctx* c, int32_t b, uint8_t* host_out) {
  int rc = sample_ok(c, b);
  if (rc != CG_OK) return rc;
  if (!host_out) return set_err(CG_EINVAL, "null output");
  const DevSample& s = c->dev[b];
  std::vector<uint32_t> w(s.NW);
  HIPCHK(hipMemcpyAsync(w.data(), s.occ, 4 * (size_t)s.NW, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int32_t l = 0; l < s.N; ++l) host_out[l] = (uint8_t)((w[l >> 5] >> (l & 31)) & 1u);
  return CG_OK;
}

int cg_get_local_energies(cg_ctx* c, int32_t b, double* host_out) {
  int rc = sample_ok(c, b);
  if (rc != CG_OK) return rc;
  if (!host_out) return set_err(CG_EINVAL, "null output");
  const DevSample& s = c->dev[b];
  if (c->plan.precision == CG_FP64) {
    HIPCHK(hipMemcpyAsync(host_out, s.eps, 8 * (size_t)s.N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  } else {
    // FP32 form: value word plus its compensated low part
    std::vector<float> f(2 * (size_t)s.N);
    HIPCHK(hipMemcpyAsync(f.data(), s.eps, 8 * (size_t)s.N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int32_t l = 0; l < s.N; ++l) host_out[l] = (double)f[2 * l] + (double)f[2 * l + 1];
  }
  return CG_OK;
}

int cg_get_phi(cg_ctx* c, int32_t b, double* host_out) {
  int rc = sample_ok(c, b);
  if (rc != CG_OK) return rc;
  if (!host_out) return set_err(CG_EINVAL, "null output");
  const DevSample& s = c->dev[b];
  HIPCHK(hipMemcpyAsync(host_out, s.phi, 8 * (size_t)s.N, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CG_OK;
}

int cg_get_stats(cg_ctx* c, int32_t b, cg_stats* out) {
  int rc = sample_ok(c, b);
  if (rc != CG_OK) return rc;
  if (!out) return set_err(CG_EINVAL, "null output");
  SampleState st;
  HIPCHK(hipMemcpyAsync(&st, c->dev[b].st, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  out->hops = st.hops;
  out->s_last = st.s_last;
  out->s_scan = st.s_scan;
  out->P = st.P;
  out->t = st.t;
  out->H0 = st.H0;
  out->sum_p = st.sum_p;
  out->rounds = st.rounds;
  out->evaluated = st.evaluated;
  out->theta_pass = st.theta_pass;
  out->refreshes = st.refreshes;
  out->max_drift = st.max_drift;
  out->last_drift = st.last_drift;
  out->status = st.status;
  out->since_refresh = st.since_refresh;
  out->logged = st.logged;
  for (int k = 0; k < 4; ++k) out->phase_cycles[k] = st.phase_cycles[k];
  return CG_OK;
}

int cg_get_clock(cg_ctx* c, int32_t b, double* t) {
  if (!t) return set_err(CG_EINVAL, "null output");
  cg_stats s;
  int rc = cg_get_stats(c, b, &s);
  if (rc != CG_OK) return rc;
  *t = s.t;
  return CG_OK;
}

int cg_get_current(cg_ctx* c, int32_t b, double* t, int64_t* P, double* sigma) {
  cg_stats s;
  int rc = cg_get_stats(c, b, &s);
  if (rc != CG_OK) return rc;
  const double N = (double)c->dev[b].N, E = c->desc[b].E;
  if (t) *t = s.t;
  if (P) *P = s.P;
  if (sigma) *sigma = (E * s.t != 0.0) ? (double)s.P / (N * E * s.t) : 0.0;
  return CG_OK;
}

int cg_get_hop_log(cg_ctx* c, int32_t b, uint64_t* labels, int32_t* from, int32_t* to, int64_t cap,
                   int64_t* count) {
  cg_stats s;
  int rc = cg_get_stats(c, b, &s);
  if (rc != CG_OK) return rc;
  if (cap < 0 || !count) return set_err(CG_EINVAL, "bad log arguments");
  const int64_t k = std::min<int64_t>(cap, s.logged);
  const DevSample& d = c->dev[b];
  if (k > 0) {
    if (!labels || !from || !to) return set_err(CG_EINVAL, "null log output");
    HIPCHK(hipMemcpyAsync(labels, d.log_label, 8 * (size_t)k, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(from, d.log_from, 4 * (size_t)k, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(to, d.log_to, 4 * (size_t)k, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  *count = k;
  return CG_OK;
}

namespace {

// Arguments of the density-of-states calls: CG_OK or CG_EINVAL with a message.
int dos_args(const cg_ctx* c, int32_t first, int32_t count, double e_lo, double e_hi, int32_t nbins,
             const uint64_t* host_occupied, const uint64_t* host_empty, const uint64_t* host_outside) {
  if (!c) return set_err(CG_EINVAL, "null context");
  const int32_t n = (int32_t)c->desc.size();
  if (first < 0 || count < 1 || first + count > n)
    return set_err(CG_EINVAL, "samples %d .. %d outside 0 .. %d", first, first + count - 1, n - 1);
  if (nbins < 1 || nbins > kDosMaxBins) return set_err(CG_EINVAL, "nbins=%d must be in 1 .. %d", nbins, kDosMaxBins);
  if (!(e_hi > e_lo) || !std::isfinite(e_lo) || !std::isfinite(e_hi))
    return set_err(CG_EINVAL, "energy range [%g, %g)", e_lo, e_hi);
  if (!host_occupied || !host_empty || !host_outside) return set_err(CG_EINVAL, "null output");
  if (count > 65535) return set_err(CG_EINVAL, "count=%d exceeds 65535", count);
  return CG_OK;
}

// Clears the 2 nbins + 2 count slots at d_hist and counts samples first .. first + count - 1
// into them, on the context stream.
int dos_launch(const cg_ctx* c, int32_t first, int32_t count, double e_lo, double e_hi, int32_t nbins,
               unsigned long long* d_hist) {
  int32_t max_N = 0;
  for (int32_t b = first; b < first + count; ++b) max_N = std::max(max_N, c->dev[b].N);
  const int slots = 2 * nbins + 2;
  // a fill kernel, not hipMemsetAsync: the calls may sit inside a captured graph
  hipLaunchKernelGGL(k_fill_u64, dim3((slots + 255) / 256), dim3(256), 0, c->stream, d_hist, slots);
  const double scale = (double)nbins / (e_hi - e_lo);
  const int chunks = (max_N + kDosBlock * kDosSitesPerThread - 1) / (kDosBlock * kDosSitesPerThread);
  hipLaunchKernelGGL(k_dos, dim3(chunks, count), dim3(kDosBlock), 0, c->stream, c->d_samples, first,
                     c->plan.precision == CG_FP64 ? 0 : 1, e_lo, scale, nbins, d_hist);
  HIPCHK(hipGetLastError());
  return CG_OK;
}

}  // namespace

int cg_dos(cg_ctx* c, int32_t first, int32_t count, double e_lo, double e_hi, int32_t nbins,
           uint64_t* host_occupied, uint64_t* host_empty, uint64_t* host_outside) {
  int rc = dos_args(c, first, count, e_lo, e_hi, nbins, host_occupied, host_empty, host_outside);
  if (rc != CG_OK) return rc;
  unsigned long long* d_hist = (unsigned long long*)(c->arena + c->plan.hist_off);
  rc = dos_launch(c, first, count, e_lo, e_hi, nbins, d_hist);
  if (rc != CG_OK) return rc;
  const int slots = 2 * nbins + 2;
  std::vector<uint64_t> h((size_t)slots);
  HIPCHK(hipMemcpyAsync(h.data(), d_hist, 8 * (size_t)slots, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::memcpy(host_occupied, h.data(), 8 * (size_t)nbins);
  std::memcpy(host_empty, h.data() + nbins, 8 * (size_t)nbins);
  host_outside[0] = h[2 * (size_t)nbins];
  host_outside[1] = h[2 * (size_t)nbins + 1];
  return CG_OK;
}

int cg_dos_noalloc(cg_ctx* c, int32_t first, int32_t count, double e_lo, double e_hi, int32_t nbins,
                   uint64_t* host_occupied, uint64_t* host_empty, uint64_t* host_outside) {
  int rc = dos_args(c, first, count, e_lo, e_hi, nbins, host_occupied, host_empty, host_outside);
  if (rc != CG_OK) return rc;
  if (2 * nbins + 2 > kScratchSlots) return set_err(CG_EINVAL, "nbins=%d exceeds the scratch of %d bins", nbins, kDosMaxBins);
  unsigned long long* d = c->scratch_dev;
  if (!d) return set_err(CG_EHIP, "scratch array not resolved for this context");
  rc = dos_launch(c, first, count, e_lo, e_hi, nbins, d);
  if (rc != CG_OK) return rc;
  HIPCHK(hipMemcpyAsync(host_occupied, d, 8 * (size_t)nbins, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(host_empty, d + nbins, 8 * (size_t)nbins, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(host_outside, d + 2 * (size_t)nbins, 16, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CG_OK;
}

// Checkpoint blob of one sample: header, the sample state, occupation words, energies.
struct SaveHeader {
  char magic[8];  // "CGKMCSV1"
  uint32_t version, state_bytes;
  int32_t precision, L, n_e, dim;
  double W, xi, rc, T, E;
  uint64_t seed;
  uint32_t sample_id, occ_words;
  uint64_t eps_bytes;
  double pair;
};
constexpr char kSaveMagic[8] = {'C', 'G', 'K', 'M', 'C', 'S', 'V', '1'};
constexpr uint32_t kSaveVersion = 2;  // 2: the header carries the pair-hop probability

size_t save_bytes(const DevSample& s) { return sizeof(SaveHeader) + sizeof(SampleState) + 4 * (size_t)s.NW + 8 * (size_t)s.N; }

int cg_save(cg_ctx* c, int32_t b, void* host_blob, size_t* bytes) {
  int rc = sample_ok(c, b);
  if (rc != CG_OK) return rc;
  if (!bytes) return set_err(CG_EINVAL, "null size");
  const DevSample& s = c->dev[b];
  const size_t need = save_bytes(s);
  if (!host_blob) {
    *bytes = need;
    return CG_OK;
  }
  if (*bytes < need) return set_err(CG_ENOSPC, "checkpoint needs %zu bytes (%zu given)", need, *bytes);
  const cg_sample_desc& d = c->desc[b];
  SaveHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kSaveMagic, 8);
  h.version = kSaveVersion;
  h.state_bytes = (uint32_t)sizeof(SampleState);
  h.precision = c->plan.precision;
  h.L = d.L;
  h.dim = d.dim;
  h.n_e = d.n_electrons;
  h.W = d.W;
  h.xi = d.xi;
  h.rc = d.rc;
  h.T = d.T;
  h.E = d.E;
  h.seed = d.seed;
  h.sample_id = d.sample_id;
  h.pair = d.pair;
  h.occ_words = (uint32_t)s.NW;
  h.eps_bytes = 8 * (size_t)s.N;
  uint8_t* out = (uint8_t*)host_blob;
  std::memcpy(out, &h, sizeof(h));
  out += sizeof(h);
  HIPCHK(hipMemcpyAsync(out, s.st, sizeof(SampleState), hipMemcpyDeviceToHost, c->stream));
  out += sizeof(SampleState);
  HIPCHK(hipMemcpyAsync(out, s.occ, 4 * (size_t)s.NW, hipMemcpyDeviceToHost, c->stream));
  out += 4 * (size_t)s.NW;
  HIPCHK(hipMemcpyAsync(out, s.eps, h.eps_bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *bytes = need;
  return CG_OK;
}

int cg_load(cg_ctx* c, int32_t b, const void* host_blob, size_t bytes) {
  int rc = sample_ok(c, b);
  if (rc != CG_OK) return rc;
  if (!host_blob) return set_err(CG_EINVAL, "null checkpoint");
  const DevSample& s = c->dev[b];
  const size_t need = save_bytes(s);
  if (bytes < sizeof(SaveHeader)) return set_err(CG_EINVAL, "checkpoint of %zu bytes has no header", bytes);
  SaveHeader h;
  std::memcpy(&h, host_blob, sizeof(h));
  const cg_sample_desc& d = c->desc[b];
  if (std::memcmp(h.magic, kSaveMagic, 8) != 0 || h.version != kSaveVersion || h.state_bytes != sizeof(SampleState))
    return set_err(CG_EINVAL, "not a checkpoint of this library version");
  if (bytes != need || h.occ_words != (uint32_t)s.NW || h.eps_bytes != 8 * (size_t)s.N)
    return set_err(CG_EINVAL, "checkpoint of %zu bytes does not match sample %d (%zu bytes)", bytes, b, need);
  if (h.precision != c->plan.precision)
    return set_err(CG_EINVAL, "checkpoint precision %d, context precision %d", h.precision, c->plan.precision);
  if (h.L != d.L || h.dim != d.dim || h.n_e != d.n_electrons || h.W != d.W || h.xi != d.xi || h.rc != d.rc || h.seed != d.seed ||
      h.sample_id != d.sample_id || h.pair != d.pair)
    return set_err(CG_EINVAL, "checkpoint is of another sample (L, n_e, W, xi, rc, seed, sample id or pair differ)");
  SampleState st;
  const uint8_t* in = (const uint8_t*)host_blob + sizeof(h);
  std::memcpy(&st, in, sizeof(st));
  in += sizeof(st);
  st.logged = 0;  // the hop log is not part of a checkpoint
  st.grid_bar = 0;
  st.force_refresh = 0;
  // the blob's T and E were current when it was written
  rc = cg_set_TE(c, b, h.T, h.E);
  if (rc != CG_OK) return rc;
  HIPCHK(hipMemcpyAsync(s.st, &st, sizeof(st), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(s.occ, in, 4 * (size_t)s.NW, hipMemcpyHostToDevice, c->stream));
  in += 4 * (size_t)s.NW;
  HIPCHK(hipMemcpyAsync(s.eps, in, h.eps_bytes, hipMemcpyHostToDevice, c->stream));
  // the large-sample kernel's proposals read a mirror of the energies (empty otherwise)
  if (c->plan.layout == kBig) HIPCHK(hipMemcpyAsync(s.mirror, in, h.eps_bytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->lockstep_since = -1;  // this sample's refresh phase may now differ from the others'
  return CG_OK;
}

int cg_autotune(const cg_sample_desc* samples, int32_t n, cg_run_opts* opts, void* arena, size_t arena_bytes,
                void* hip_stream, int64_t trial_hops, double drift_target, int32_t* widths) {
  if (!opts) return set_err(CG_EINVAL, "null options");
  if (trial_hops < 64) return set_err(CG_EINVAL, "trial_hops=%lld must be >= 64", (long long)trial_hops);
  if (!(drift_target > 0.0)) return set_err(CG_EINVAL, "drift_target=%g", drift_target);
  // 1) chunk width: the candidate with the least hop-kernel time over trial_hops hops
  const int32_t Ms[2] = {1024, 2048};
  double best_ms = 0.0;
  int32_t best_M = Ms[0];
  for (int32_t M : Ms) {
    cg_run_opts o = *opts;
    o.M = M;
    o.log_hops = 0;
    o.phase_timers = 0;
    o.use_graph = 0;
    if (o.precision != CG_FP64) o.K_refresh = 1 << 20;  // no refresh inside the timing trial
    cg_ctx* c = nullptr;
    int rc = cg_create(&c, samples, n, &o, arena, arena_bytes, hip_stream);
    if (rc != CG_OK) return rc;
    rc = cg_run_hops(c, trial_hops / 2);
    double ms = 0.0;
    if (rc == CG_OK) rc = cg_take_kernel_time(c, nullptr, nullptr, nullptr, nullptr);
    if (rc == CG_OK) rc = cg_run_hops(c, trial_hops);
    if (rc == CG_OK) rc = cg_take_kernel_time(c, &ms, nullptr, nullptr, nullptr);
    cg_destroy(c);
    if (rc != CG_OK) return rc;
    if (M == Ms[0] || ms < best_ms) {
      best_ms = ms;
      best_M = M;
    }
  }
  opts->M = best_M;
  // 2) refresh period: the largest K whose drift over 2K hops from the initial state, where
  //    the energies are widest, stays below half the target
  const int32_t Ks[4] = {8192, 4096, 2048, 1024};
  for (int32_t K : Ks) {
    if (opts->precision == CG_FP64) break;
    cg_run_opts o = *opts;
    o.K_refresh = K;
    o.log_hops = 0;
    o.phase_timers = 0;
    o.use_graph = 0;
    cg_ctx* c = nullptr;
    int rc = cg_create(&c, samples, n, &o, arena, arena_bytes, hip_stream);
    if (rc != CG_OK) return rc;
    rc = cg_run_hops(c, 2 * (int64_t)K);
    double worst = 0.0;
    for (int32_t b = 0; b < n && rc == CG_OK; ++b) {
      cg_stats st;
      rc = cg_get_stats(c, b, &st);
      worst = std::max(worst, st.max_drift);
    }
    cg_destroy(c);
    if (rc != CG_OK) return rc;
    opts->K_refresh = K;
    if (worst <= 0.5 * drift_target) break;
  }
  if (!widths) return CG_OK;
  // 3) per-sample PR width M* = min(1/A, C): A = hops per serial proposal over the second
  //    half of a 2 trial_hops run from the initial state, C = 16384; a power of two >= 512
  cg_run_opts o = *opts;
  o.log_hops = 0;
  o.phase_timers = 0;
  o.use_graph = 0;
  cg_ctx* c = nullptr;
  int rc = cg_create(&c, samples, n, &o, arena, arena_bytes, hip_stream);
  if (rc != CG_OK) return rc;
  std::vector<cg_stats> st0((size_t)n), st1((size_t)n);
  rc = cg_run_hops(c, trial_hops);
  for (int32_t b = 0; b < n && rc == CG_OK; ++b) rc = cg_get_stats(c, b, &st0[b]);
  if (rc == CG_OK) rc = cg_run_hops(c, trial_hops);
  for (int32_t b = 0; b < n && rc == CG_OK; ++b) rc = cg_get_stats(c, b, &st1[b]);
  cg_destroy(c);
  if (rc != CG_OK) return rc;
  for (int32_t b = 0; b < n; ++b) {
    const double props = (double)(st1[b].s_last - st0[b].s_last), hops = (double)(st1[b].hops - st0[b].hops);
    const double inv_a = hops > 0.0 ? props / hops : 16384.0;
    int32_t w = 512;
    while (w < 16384 && (double)w < inv_a) w *= 2;
    widths[b] = w;
  }
  return CG_OK;
}

int cg_take_kernel_time(cg_ctx* c, double* hop_ms, int64_t* hop_launches, double* refresh_ms,
                        int64_t* refresh_launches) {
  if (!c) return set_err(CG_EINVAL, "null context");
  int rc = fold_events(c->ev_hop, c->acc_hop_ms);
  if (rc != CG_OK) return rc;
  rc = fold_events(c->ev_ref, c->acc_ref_ms);
  if (rc != CG_OK) return rc;
  rc = fold_events(c->ev_graph, c->acc_graph_ms);
  if (rc != CG_OK) return rc;
  // graph replays are timed as a whole and counted with the hop launches they contain
  c->acc_hop_ms += c->acc_graph_ms;
  c->acc_graph_ms = 0.0;
  c->n_graph = 0;
  if (hop_ms) *hop_ms = c->acc_hop_ms;
  if (hop_launches) *hop_launches = c->n_hop;
  if (refresh_ms) *refresh_ms = c->acc_ref_ms;
  if (refresh_launches) *refresh_launches = c->n_ref;
  c->acc_hop_ms = c->acc_ref_ms = 0.0;
  c->n_hop = c->n_ref = 0;
  return CG_OK;
}

}  // extern "C"
