// lds_probe.hip -- throughput of the gfx950 units the hop kernels use, for the roofline
// denominators: LDS reads and writes of 4/8/16 bytes per lane, the hop
// kernel's update pattern (per lane 32 table reads in pairs and 16 value stores, and two
// table layouts with 16-byte value stores), FP32
// multiplies, 32x32->64-bit integer multiplies and log2.  One workgroup of 1024 threads per
// CU; every address stays inside the workgroup's LDS array; loop-carried offsets are opaque
// to the compiler so that no load is hoisted out of the timed loop.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#define CHK(x)                                                                          \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);       \
      return 1;                                                                         \
    }                                                                                   \
  } while (0)

constexpr int kWords = 16384;  // 64 KB of LDS per workgroup for the read/write tests

__device__ __forceinline__ int opaque_int(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <int W>  // dwords per lane and load: 1, 2, 4
__global__ void __launch_bounds__(1024) k_read(uint32_t* out, int iters) {
  __shared__ __align__(16) uint32_t buf[kWords];
  for (int k = threadIdx.x; k < kWords; k += 1024) buf[k] = k * 2654435761u;
  __syncthreads();
  uint32_t acc = 0;
  const int base = threadIdx.x * W;
  for (int it = 0; it < iters; ++it) {
    const int off = opaque_int((it & 1) * 64);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int a = (base + u * 1024 * W + off) & (kWords - 1);  // lane-consecutive, in range
      if constexpr (W == 1) {
        acc ^= buf[a];
      } else if constexpr (W == 2) {
        const uint2 v = *(const uint2*)&buf[a & ~1];
        acc ^= v.x ^ v.y;
      } else {
        const uint4 v = *(const uint4*)&buf[a & ~3];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
      }
    }
  }
  if (acc == 0x12345678u) out[blockIdx.x * 1024 + threadIdx.x] = acc;
}

// Random-address 4-byte reads (the proposals' energy and occupation reads): each lane's next
// address comes from a multiplicative hash of the value just read, so every read is random
// and depends on the previous one (four independent chains per lane).
__global__ void __launch_bounds__(1024) k_read_random(uint32_t* out, int iters) {
  __shared__ __align__(16) uint32_t buf[kWords];
  for (int k = threadIdx.x; k < kWords; k += 1024) buf[k] = (uint32_t)k * 2654435761u;
  __syncthreads();
  uint32_t a0 = threadIdx.x * 7u, a1 = threadIdx.x * 13u + 1u, a2 = threadIdx.x * 29u + 2u, a3 = threadIdx.x * 31u + 3u;
  for (int it = 0; it < iters; ++it) {
    a0 = (buf[a0 & (kWords - 1)] ^ a0) * 2246822519u;  // index always masked into the array
    a1 = (buf[a1 & (kWords - 1)] ^ a1) * 2246822519u;
    a2 = (buf[a2 & (kWords - 1)] ^ a2) * 2246822519u;
    a3 = (buf[a3 & (kWords - 1)] ^ a3) * 2246822519u;
    a0 >>= 3; a1 >>= 3; a2 >>= 3; a3 >>= 3;
  }
  if ((a0 ^ a1 ^ a2 ^ a3) == 0x12345678u) out[blockIdx.x * 1024 + threadIdx.x] = 1;
}

// Workgroup barriers only (the cost of one round trip through s_barrier with 16 waves).
__global__ void __launch_bounds__(1024) k_barrier(uint32_t* out, int iters) {
  uint32_t v = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    v = v * 1664525u + 1013904223u;
    __syncthreads();
  }
  if (v == 0x12345678u) out[blockIdx.x * 1024 + threadIdx.x] = 1;
}

template <int W>  // dwords per lane and store: 1, 2, 4
__global__ void __launch_bounds__(1024) k_write(uint32_t* out, int iters) {
  __shared__ __align__(16) uint32_t buf[kWords];
  uint32_t v = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    const int off = opaque_int((it & 1) * 64);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int a = (threadIdx.x * W + u * 1024 * W + off) & (kWords - 1);  // lane-consecutive
      if constexpr (W == 1) {
        buf[a] = v;
      } else if constexpr (W == 2) {
        *(uint2*)&buf[a & ~1] = make_uint2(v, v + 1);
      } else {
        *(uint4*)&buf[a & ~3] = make_uint4(v, v + 1, v + 2, v + 3);
      }
      v += 1;
    }
  }
  __syncthreads();
  if (buf[threadIdx.x] == 0x12345678u) out[blockIdx.x * 1024 + threadIdx.x] = 1;
}

// The hop kernel's update at L = 128: per lane two table bases (rows 1088 floats apart, two
// columns 17 floats apart) and 16 stores (rows 2048 floats apart, columns 64 apart).
constexpr int kUpdWords = 34816;  // 136 KB: 16384 value words + table rows
__global__ void __launch_bounds__(1024) k_update(uint32_t* out, int iters) {
  extern __shared__ __align__(16) float sm[];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < kUpdWords; k += 1024) sm[k] = k * 1e-3f;
  __syncthreads();
  float acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.f;
  for (int it = 0; it < iters; ++it) {
    // largest index: 16384 + 52 * 68 + 63 + 7 * 1088 + 17 = 27616 < kUpdWords
    const int bj = opaque_int(16384 + wid * 68 + ((lane * 3 + it) & 63));
    const int bi = opaque_int(16384 + (wid + 37) * 68 + ((lane * 5 + it) & 63));
    float d[16];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int c = 0; c < 2; ++c) d[2 * r + c] = sm[bj + r * 1088 + c * 17] - sm[bi + r * 1088 + c * 17];
    }
    const int ev = opaque_int(wid * 128 + lane);  // largest store index 1983 + 14336 + 64 < 16384
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        acc[2 * r + c] += d[2 * r + c];
        sm[ev + r * 2048 + c * 64] = acc[2 * r + c];
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += acc[k];
  if (s == 1.2345f) out[blockIdx.x * 1024 + threadIdx.x] = 1;
}

typedef float probe_f4 __attribute__((ext_vector_type(4)));

// The update with 16-byte value stores (four per lane, chunk-major) and two table layouts at
// L = 128.  rows: table rows 68 floats wide by raw row difference, two folded columns per
// lane, rows 16 apart read in pairs (16 two-address reads per lane).  pairs: per column pair
// (c, 64 - c) and row, two floats side by side; a lane's 8 rows (one residue class mod 16)
// are 8 consecutive pairs, read as 4 double-pair reads per base (8 per lane).
// cols: the table column-major (260 floats per folded column, raw row difference inside), a
// wave owning 8 consecutive rows: a lane's 8 rows per column are 8 consecutive floats, read
// as three aligned 16-byte loads (12 per lane).
template <int LAYOUT, bool STORES = true>  // 0 rows, 1 pairs, 2 cols; STORES off: reads only
__global__ void __launch_bounds__(1024) k_update_layout(uint32_t* out, int iters) {
  extern __shared__ __align__(16) float sm[];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < kUpdWords; k += 1024) sm[k] = k * 1e-3f;
  __syncthreads();
  float acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.f;
  for (int it = 0; it < iters; ++it) {
    const int yj = it & 127, yi = (it * 5 + 3) & 127, xj = (it * 7) & 127, xi = (it * 11 + 1) & 127;
    const int dj = (lane - xj) & 127, di = (lane - xi) & 127;
    const int cj = dj < 128 - dj ? dj : 128 - dj, ci = di < 128 - di ? di : 128 - di;  // 0..64
    float d[16];
    if constexpr (LAYOUT == 2) {
      const int dj1 = (lane + 64 - xj) & 127, di1 = (lane + 64 - xi) & 127;
      const int cj1 = dj1 < 128 - dj1 ? dj1 : 128 - dj1, ci1 = di1 < 128 - di1 ? di1 : 128 - di1;
      const int sj = 8 * wid - yj + 128, si = 8 * wid - yi + 128;  // 1..248
      // largest index 16384 + 64 * 260 + 248 + 11 = 33283 < kUpdWords
      const int aj0 = opaque_int((16384 + cj * 260 + sj) >> 2) * 4, aj1 = opaque_int((16384 + cj1 * 260 + sj) >> 2) * 4;
      const int ai0 = opaque_int((16384 + ci * 260 + si) >> 2) * 4, ai1 = opaque_int((16384 + ci1 * 260 + si) >> 2) * 4;
      float fj0[12], fj1[12], fi0[12], fi1[12];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const probe_f4 a = *(const probe_f4*)&sm[aj0 + 4 * k], b = *(const probe_f4*)&sm[aj1 + 4 * k];
        const probe_f4 c = *(const probe_f4*)&sm[ai0 + 4 * k], e = *(const probe_f4*)&sm[ai1 + 4 * k];
        fj0[4 * k] = a.x; fj0[4 * k + 1] = a.y; fj0[4 * k + 2] = a.z; fj0[4 * k + 3] = a.w;
        fj1[4 * k] = b.x; fj1[4 * k + 1] = b.y; fj1[4 * k + 2] = b.z; fj1[4 * k + 3] = b.w;
        fi0[4 * k] = c.x; fi0[4 * k + 1] = c.y; fi0[4 * k + 2] = c.z; fi0[4 * k + 3] = c.w;
        fi1[4 * k] = e.x; fi1[4 * k + 1] = e.y; fi1[4 * k + 2] = e.z; fi1[4 * k + 3] = e.w;
      }
      // the kernel picks 8 of the 12 floats by a uniform shift; here every float is used
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        d[k] = (fj0[k] - fi0[k]) + (fj0[k + 4] - fi0[k + 4]);
        d[8 + k] = (fj1[k] - fi1[k]) + (fj1[k + 4] - fi1[k + 4]);
      }
    } else if constexpr (LAYOUT == 1) {
      // pair column min(c, 64 - c) in 0..32, 516 floats each; start pair in 0..248
      const int pj = cj < 64 - cj ? cj : 64 - cj, pi = ci < 64 - ci ? ci : 64 - ci;
      const int bj = wid - yj + 128, bi = wid - yi + 128;  // 1..143
      const int aj = opaque_int(16384 + pj * 516 + 2 * ((bj & 15) * 16 + (bj >> 4)));
      const int ai = opaque_int(16384 + pi * 516 + 2 * ((bi & 15) * 16 + (bi >> 4)));
      // largest index 16384 + 32 * 516 + 2 * 248 + 15 = 33407 < kUpdWords
      const float2* qj = (const float2*)&sm[aj];
      const float2* qi = (const float2*)&sm[ai];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float2 vj = qj[k], vi = qi[k];
        d[2 * k] = vj.x - vi.x;
        d[2 * k + 1] = vj.y - vi.y;
      }
    } else {
      const int dj1 = (lane + 64 - xj) & 127, di1 = (lane + 64 - xi) & 127;
      const int cj1 = dj1 < 128 - dj1 ? dj1 : 128 - dj1, ci1 = di1 < 128 - di1 ? di1 : 128 - di1;
      const int rj = 16384 + (wid - yj + 128) * 68, ri = 16384 + (wid - yi + 128) * 68;
      const int aj0 = opaque_int(rj + cj), aj1 = opaque_int(rj + cj1);
      const int ai0 = opaque_int(ri + ci), ai1 = opaque_int(ri + ci1);
      // largest index 16384 + 143 * 68 + 64 + 7 * 1088 = 33788 < kUpdWords
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        d[2 * r] = sm[aj0 + r * 1088] - sm[ai0 + r * 1088];
        d[2 * r + 1] = sm[aj1 + r * 1088] - sm[ai1 + r * 1088];
      }
    }
    const int ev = opaque_int(wid * 256 + lane) * 4;  // largest 15360 + 252 + 768 + 3 < 16384
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      probe_f4 w;
      acc[4 * q] += d[4 * q];
      acc[4 * q + 1] += d[4 * q + 1];
      acc[4 * q + 2] += d[4 * q + 2];
      acc[4 * q + 3] += d[4 * q + 3];
      w.x = acc[4 * q];
      w.y = acc[4 * q + 1];
      w.z = acc[4 * q + 2];
      w.w = acc[4 * q + 3];
      if constexpr (STORES) *(probe_f4*)&sm[ev + 256 * q] = w;
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += acc[k];
  if (s == 1.2345f) out[blockIdx.x * 1024 + threadIdx.x] = 1;
}

__global__ void __launch_bounds__(1024) k_fmul(float* out, int iters) {
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = threadIdx.x + k;
  const float d = 1.0001f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = a[k] * d;
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  if (s == 1.2345f) out[blockIdx.x * 1024 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(1024) k_imul(uint32_t* out, int iters) {
  uint32_t a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = threadIdx.x * 7 + k;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint64_t p = (uint64_t)a[k] * 0xD2511F53u;
        a[k] = (uint32_t)(p >> 32) + (uint32_t)p;
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s ^= a[k];
  if (s == 0x12345678u) out[blockIdx.x * 1024 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(1024) k_log2(float* out, int iters) {
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 1.5f + threadIdx.x * 1e-4f + k;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = __log2f(a[k]) + 1.5f;
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  if (s == 1.2345f) out[blockIdx.x * 1024 + threadIdx.x] = s;
}

// Grid-wide barriers over G workgroups of one cooperative launch (the whole-GPU hop kernel's
// synchronisation), iters barriers per launch.  Every wait is bounded (kGbarSpins polls); a
// workgroup that gives up counts a failure and leaves, and the others then give up in turn.
constexpr uint32_t kGbarSpins = 1u << 20;
constexpr int kLine = 32;  // words per 128-byte line: one flag or counter per line

__device__ __forceinline__ uint32_t ld_acq(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool spin_until(const uint32_t* p, uint32_t target) {
  uint32_t spins = 0;
  while (ld_acq(p) < target) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins >= kGbarSpins) return false;
  }
  return true;
}
// relaxed polls (no cache maintenance per poll)
__device__ __forceinline__ bool spin_rlx(const uint32_t* p, uint32_t target) {
  uint32_t spins = 0;
  while (ld_rlx(p) < target) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins >= kGbarSpins) return false;
  }
  return true;
}

// MODE 0: one counter, every workgroup adds 1 and polls it.
// MODE 1: per-workgroup arrival flags (own line each) polled by workgroup 0's threads, which
//         then store the release generation that everyone polls.
// MODE 2: 8 group counters (workgroup g in group g % 8) whose last arriver adds 1 to a top
//         counter; the top's last arriver stores the release generation.
// MODE 3: one counter, release add, relaxed polls, one acquire fence after the wait.
// MODE 4: one counter, relaxed add and polls, no fence (the cost of the atomics alone).
// MODE 5: MODE 2's tree with a release add, relaxed polls and one acquire fence.
template <int MODE>
__global__ void __launch_bounds__(1024) k_gbar(uint32_t* sync, uint32_t* fail, int iters) {
  __shared__ uint32_t ok;
  const uint32_t G = gridDim.x, g = blockIdx.x;
  uint32_t* rel = sync;                       // release generation
  uint32_t* top = sync + kLine;               // MODE 0 counter / MODE 2 top counter
  uint32_t* grp = sync + 2 * kLine;           // MODE 2: 8 group counters
  uint32_t* flag = sync + 10 * kLine;         // MODE 1: G arrival flags
  const uint32_t gsize = (G + 7 - (g & 7)) / 8;  // workgroups in this one's group
  for (uint32_t it = 1; it <= (uint32_t)iters; ++it) {
    __syncthreads();
    bool good = true;
    if (MODE == 0) {
      if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(top, 1u);
        good = spin_until(top, it * G);
        __threadfence();
      }
    } else if (MODE == 1) {
      if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_store(flag + g * kLine, it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (g == 0) {
        if (threadIdx.x < G) good = spin_until(flag + threadIdx.x * kLine, it);
        good = __syncthreads_and(good);
        if (threadIdx.x == 0 && good) {
          __threadfence();
          __hip_atomic_store(rel, it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (threadIdx.x == 0 && good) {
        good = spin_until(rel, it);
        __threadfence();
      }
    } else if (MODE == 3) {
      if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        good = spin_rlx(top, it * G);
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
      }
    } else if (MODE == 4) {
      if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = spin_rlx(top, it * G);
      }
    } else if (MODE == 5) {
      if (threadIdx.x == 0) {
        const uint32_t old = __hip_atomic_fetch_add(grp + (g & 7) * kLine, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (old == it * gsize - 1) {
          const uint32_t ngroups = G < 8 ? G : 8;
          const uint32_t o2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (o2 == it * ngroups - 1) __hip_atomic_store(rel, it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        good = spin_rlx(rel, it);
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
      }
    } else {
      if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t old = atomicAdd(grp + (g & 7) * kLine, 1u);
        if (old == it * gsize - 1) {
          const uint32_t ngroups = G < 8 ? G : 8;
          const uint32_t o2 = atomicAdd(top, 1u);
          if (o2 == it * ngroups - 1) {
            __threadfence();
            __hip_atomic_store(rel, it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        good = spin_until(rel, it);
        __threadfence();
      }
    }
    if (threadIdx.x == 0) ok = good ? 1u : 0u;
    __syncthreads();
    if (ok == 0u) {
      if (threadIdx.x == 0) atomicAdd(fail, 1u);
      return;
    }
  }
}

// Grid-barrier costs for G = 64, 128, 256 workgroups: microseconds per barrier.
static int run_grid_barriers(int ncu) {
  const int n_sync = (10 + 1024) * kLine;
  uint32_t *sync = nullptr, *fail = nullptr;
  CHK(hipMalloc(&sync, n_sync * 4));
  CHK(hipMalloc(&fail, 4));
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0));
  CHK(hipEventCreate(&e1));
  const int iters = 2000;
  for (int G : {64, 128, 256}) {
    if (G > ncu) break;
    for (int mode = 0; mode < 6; ++mode) {
      void* const fns[6] = {(void*)k_gbar<0>, (void*)k_gbar<1>, (void*)k_gbar<2>,
                            (void*)k_gbar<3>, (void*)k_gbar<4>, (void*)k_gbar<5>};
      void* fn = fns[mode];
      int it = iters;
      void* args[] = {&sync, &fail, &it};
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        CHK(hipMemset(sync, 0, n_sync * 4));
        CHK(hipMemset(fail, 0, 4));
        CHK(hipDeviceSynchronize());
        CHK(hipEventRecord(e0));
        CHK(hipLaunchCooperativeKernel(fn, dim3(G), dim3(1024), args, 0, 0));
        CHK(hipEventRecord(e1));
        CHK(hipEventSynchronize(e1));
        CHK(hipEventElapsedTime(&ms, e0, e1));
      }
      uint32_t nf = 0;
      CHK(hipMemcpy(&nf, fail, 4, hipMemcpyDeviceToHost));
      const char* const names[6] = {"one counter", "flags + master", "8 group counters",
                                    "counter, release add, relaxed polls, one acquire",
                                    "counter, relaxed, no fence", "8 groups, release add, relaxed polls, one acquire"};
      std::printf("grid barrier mode %d (%s), %3d workgroups  %7.2f us per barrier%s\n", mode, names[mode], G,
                  ms * 1e3 / iters, nf ? "  (a wait gave up)" : "");
    }
  }
  CHK(hipFree(sync));
  CHK(hipFree(fail));
  return 0;
}

int main(int argc, char** argv) {
  int ncu = 0;
  CHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0));
  if (argc > 1 && std::string(argv[1]) == "barrier") return run_grid_barriers(ncu);
  const double clk = 2.4e9;  // MI355X peak engine clock
  std::printf("CUs %d; rates below per CU at %.1f GHz\n", ncu, clk * 1e-9);
  uint32_t* out = nullptr;
  CHK(hipMalloc(&out, (size_t)ncu * 1024 * 4));
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0));
  CHK(hipEventCreate(&e1));
  CHK(hipFuncSetAttribute((const void*)k_update, hipFuncAttributeMaxDynamicSharedMemorySize, kUpdWords * 4));
  CHK(hipFuncSetAttribute((const void*)k_update_layout<0>, hipFuncAttributeMaxDynamicSharedMemorySize, kUpdWords * 4));
  CHK(hipFuncSetAttribute((const void*)k_update_layout<1>, hipFuncAttributeMaxDynamicSharedMemorySize, kUpdWords * 4));
  CHK(hipFuncSetAttribute((const void*)k_update_layout<2>, hipFuncAttributeMaxDynamicSharedMemorySize, kUpdWords * 4));
  CHK(hipFuncSetAttribute((const void*)k_update_layout<0, false>, hipFuncAttributeMaxDynamicSharedMemorySize, kUpdWords * 4));
  CHK(hipFuncSetAttribute((const void*)k_update_layout<2, false>, hipFuncAttributeMaxDynamicSharedMemorySize, kUpdWords * 4));
  const int iters = 20000;
  float ms = 0.f;
  auto timed = [&](auto launch) -> int {
    launch();
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    CHK(hipEventRecord(e0));
    launch();
    CHK(hipEventRecord(e1));
    CHK(hipEventSynchronize(e1));
    CHK(hipEventElapsedTime(&ms, e0, e1));
    return 0;
  };
  const dim3 g(ncu), b(1024);
  const double lane_ops = (double)ncu * 1024 * iters * 8;  // per lane: 8 accesses per iteration
  auto per_cu = [&](double bytes) { return bytes / (ms * 1e-3) / ncu / clk; };
  if (timed([&] { hipLaunchKernelGGL(k_read<1>, g, b, 0, 0, out, iters); })) return 1;
  std::printf("ds_read_b32   %8.3f ms  %7.1f B/clk\n", ms, per_cu(lane_ops * 4));
  if (timed([&] { hipLaunchKernelGGL(k_read<2>, g, b, 0, 0, out, iters); })) return 1;
  std::printf("ds_read_b64   %8.3f ms  %7.1f B/clk\n", ms, per_cu(lane_ops * 8));
  if (timed([&] { hipLaunchKernelGGL(k_read<4>, g, b, 0, 0, out, iters); })) return 1;
  std::printf("ds_read_b128  %8.3f ms  %7.1f B/clk\n", ms, per_cu(lane_ops * 16));
  if (timed([&] { hipLaunchKernelGGL(k_read_random, g, b, 0, 0, out, iters); })) return 1;
  std::printf("ds_read_b32 random addresses  %8.3f ms  %7.2f clk per wave instruction per CU\n", ms,
              ms * 1e-3 * clk / ((double)iters * 4 * 16));
  if (timed([&] { hipLaunchKernelGGL(k_barrier, g, b, 0, 0, out, iters); })) return 1;
  std::printf("s_barrier, 16 waves           %8.3f ms  %7.1f clk per barrier\n", ms, ms * 1e-3 * clk / iters);
  if (timed([&] { hipLaunchKernelGGL(k_write<1>, g, b, 0, 0, out, iters); })) return 1;
  std::printf("ds_write_b32  %8.3f ms  %7.1f B/clk\n", ms, per_cu(lane_ops * 4));
  if (timed([&] { hipLaunchKernelGGL(k_write<2>, g, b, 0, 0, out, iters); })) return 1;
  std::printf("ds_write_b64  %8.3f ms  %7.1f B/clk\n", ms, per_cu(lane_ops * 8));
  if (timed([&] { hipLaunchKernelGGL(k_write<4>, g, b, 0, 0, out, iters); })) return 1;
  std::printf("ds_write_b128 %8.3f ms  %7.1f B/clk\n", ms, per_cu(lane_ops * 16));
  const int upd_iters = iters / 8;
  if (timed([&] { hipLaunchKernelGGL(k_update, g, b, kUpdWords * 4, 0, out, upd_iters); })) return 1;
  std::printf("update        %8.3f ms  %7.1f B/clk  %6.0f clk per pass (32 reads + 16 stores per lane)\n", ms,
              per_cu((double)ncu * 1024 * upd_iters * 48 * 4), ms * 1e-3 * clk / upd_iters);
  if (timed([&] { hipLaunchKernelGGL(k_update_layout<0>, g, b, kUpdWords * 4, 0, out, upd_iters); })) return 1;
  std::printf("update, row table    %8.3f ms  %6.0f clk per pass (16 paired 4-byte reads, 4 16-byte stores per lane)\n",
              ms, ms * 1e-3 * clk / upd_iters);
  if (timed([&] { hipLaunchKernelGGL(k_update_layout<1>, g, b, kUpdWords * 4, 0, out, upd_iters); })) return 1;
  std::printf("update, pair table   %8.3f ms  %6.0f clk per pass (8 paired 8-byte reads, 4 16-byte stores per lane)\n",
              ms, ms * 1e-3 * clk / upd_iters);
  if (timed([&] { hipLaunchKernelGGL(k_update_layout<2>, g, b, kUpdWords * 4, 0, out, upd_iters); })) return 1;
  std::printf("update, column table %8.3f ms  %6.0f clk per pass (12 16-byte reads, 4 16-byte stores per lane)\n",
              ms, ms * 1e-3 * clk / upd_iters);
  if (timed([&] { hipLaunchKernelGGL((k_update_layout<0, false>), g, b, kUpdWords * 4, 0, out, upd_iters); })) return 1;
  std::printf("update reads only, row table    %8.3f ms  %6.0f clk per pass\n", ms, ms * 1e-3 * clk / upd_iters);
  if (timed([&] { hipLaunchKernelGGL((k_update_layout<2, false>), g, b, kUpdWords * 4, 0, out, upd_iters); })) return 1;
  std::printf("update reads only, column table %8.3f ms  %6.0f clk per pass\n", ms, ms * 1e-3 * clk / upd_iters);
  const double wave_ops = (double)ncu * 16 * iters * 64;  // wave instructions per kernel
  if (timed([&] { hipLaunchKernelGGL(k_fmul, g, b, 0, 0, (float*)out, iters); })) return 1;
  std::printf("v_mul_f32     %8.3f ms  %7.2f wave instr/clk\n", ms, wave_ops / (ms * 1e-3) / ncu / clk);
  if (timed([&] { hipLaunchKernelGGL(k_imul, g, b, 0, 0, out, iters); })) return 1;
  std::printf("v_mad_u64_u32 + v_add_u32  %8.3f ms  %7.2f pairs/clk\n", ms, wave_ops / (ms * 1e-3) / ncu / clk);
  if (timed([&] { hipLaunchKernelGGL(k_log2, g, b, 0, 0, (float*)out, iters); })) return 1;
  std::printf("v_log_f32 + v_add_f32      %8.3f ms  %7.2f pairs/clk\n", ms, wave_ops / (ms * 1e-3) / ncu / clk);
  CHK(hipFree(out));
  return 0;
}
