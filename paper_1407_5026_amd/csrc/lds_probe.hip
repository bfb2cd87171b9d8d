// lds_probe.hip -- throughput of the gfx950 units the hop kernels use, for the roofline
// denominators: LDS reads and writes of 4/8/16 bytes per lane, random 4-byte reads, the
// 16-wave workgroup barrier, FP32 multiplies, 32x32->64-bit integer multiplies and log2
// (one workgroup of 1024 threads per CU; every address stays inside the workgroup's LDS
// array; loop-carried offsets are opaque to the compiler so that no load is hoisted out of
// the timed loop), and with the argument `barrier` the whole-GPU hop kernel's grid barrier
// on 64, 128 and 256 workgroups.  Build: python paper_1407_5026_amd/build.py probe.
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

__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// The whole-GPU hop kernel's grid barrier: 8 group counters (workgroup g in group g % 8)
// whose last arriver adds 1 to a top counter, the top's last arriver storing the release
// generation; release adds, relaxed polls and one acquire fence after the wait.
__global__ void __launch_bounds__(1024) k_gbar(uint32_t* sync, uint32_t* fail, int iters) {
  __shared__ uint32_t ok;
  const uint32_t G = gridDim.x, g = blockIdx.x;
  uint32_t* rel = sync;                       // release generation
  uint32_t* top = sync + kLine;               // top counter
  uint32_t* grp = sync + 2 * kLine;           // 8 group counters
  const uint32_t gsize = (G + 7 - (g & 7)) / 8;  // workgroups in this one's group
  for (uint32_t it = 1; it <= (uint32_t)iters; ++it) {
    __syncthreads();
    bool good = true;
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
    {
      void* fn = (void*)k_gbar;
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
      std::printf("grid barrier (8 group counters + top), %3d workgroups  %7.2f us per barrier%s\n", G,
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
