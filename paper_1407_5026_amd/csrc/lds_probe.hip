// lds_probe.hip -- throughput of the gfx950 units the hop kernels use, for the roofline
// denominators: LDS reads of 4/8/16 bytes per lane, LDS writes of 4 bytes, the hop
// kernel's update pattern (per lane 32 table reads in pairs and 16 value stores), FP32
// multiplies, 32x32->64-bit integer multiplies and log2.  One workgroup of 1024 threads per
// CU; every address stays inside the workgroup's LDS array; loop-carried offsets are opaque
// to the compiler so that no load is hoisted out of the timed loop.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

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

__global__ void __launch_bounds__(1024) k_write(uint32_t* out, int iters) {
  __shared__ __align__(16) uint32_t buf[kWords];
  uint32_t v = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    const int off = opaque_int((it & 1) * 64);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      buf[(threadIdx.x + u * 1024 + off) & (kWords - 1)] = v;
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

int main() {
  int ncu = 0;
  CHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0));
  const double clk = 2.4e9;  // MI355X peak engine clock
  std::printf("CUs %d; rates below per CU at %.1f GHz\n", ncu, clk * 1e-9);
  uint32_t* out = nullptr;
  CHK(hipMalloc(&out, (size_t)ncu * 1024 * 4));
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0));
  CHK(hipEventCreate(&e1));
  CHK(hipFuncSetAttribute((const void*)k_update, hipFuncAttributeMaxDynamicSharedMemorySize, kUpdWords * 4));
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
  if (timed([&] { hipLaunchKernelGGL(k_write, g, b, 0, 0, out, iters); })) return 1;
  std::printf("ds_write_b32  %8.3f ms  %7.1f B/clk\n", ms, per_cu(lane_ops * 4));
  const int upd_iters = iters / 8;
  if (timed([&] { hipLaunchKernelGGL(k_update, g, b, kUpdWords * 4, 0, out, upd_iters); })) return 1;
  std::printf("update        %8.3f ms  %7.1f B/clk  %6.0f clk per pass (32 reads + 16 stores per lane)\n", ms,
              per_cu((double)ncu * 1024 * upd_iters * 48 * 4), ms * 1e-3 * clk / upd_iters);
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
