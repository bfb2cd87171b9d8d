// observables.hpp -- single-particle density of states of the current configurations.
//
// The paper validates its dynamics with the normalized histogram g(eps, T) of the local
// energies eps_k (section "Results", density of states; Eq. 2 defines eps_k).  k_dos counts,
// for a range of samples, every site's energy into nbins equal bins of [e_lo, e_hi):
// bin k = floor((eps - e_lo) * nbins / (e_hi - e_lo)) in FP64, split by the site's
// occupation, plus the sites below and above the range.  Normalization (dividing by the
// number of sites and the bin width) is left to the caller, who holds the integer counts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.hpp"

namespace cg {

constexpr int kDosMaxBins = 4096;
constexpr int kDosBlock = 1024;
constexpr int kDosSitesPerThread = 16;  // one block per L = 128 sample: few global atomics per bin

// Histogram layout in the arena: [0, nbins) occupied, [nbins, 2 nbins) empty, then the counts
// below and above the range.
__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* __restrict__ p, int n) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) p[k] = 0ull;
}

// grid: x over chunks of kDosBlock * kDosSitesPerThread sites, y over the samples first ..
// first + gridDim.y - 1.  pair = 1: energies stored as FP32 (value, low part), whose FP64
// sum is the energy; else FP64.
__global__ void __launch_bounds__(kDosBlock) k_dos(const DevSample* __restrict__ samples, int first, int pair,
                                                  double e_lo, double scale, int nbins,
                                                  unsigned long long* __restrict__ hist) {
  __shared__ uint32_t h[2 * kDosMaxBins + 2];
  const DevSample& S = samples[first + blockIdx.y];
  const int n_slots = 2 * nbins + 2;
  for (int k = threadIdx.x; k < n_slots; k += kDosBlock) h[k] = 0u;
  __syncthreads();
  const int N = S.N;
  const int l0 = blockIdx.x * (kDosBlock * kDosSitesPerThread) + threadIdx.x;
  // all loads first, then the counting
  double ev[kDosSitesPerThread];
  uint32_t nv[kDosSitesPerThread];
#pragma unroll
  for (int s = 0; s < kDosSitesPerThread; ++s) {
    const int l = l0 + s * kDosBlock;
    ev[s] = 0.0;
    nv[s] = 0u;
    if (l < N) {
      if (pair) {
        const float2 v = ((const float2*)S.eps)[l];
        ev[s] = (double)v.x + (double)v.y;
      } else {
        ev[s] = ((const double*)S.eps)[l];
      }
      nv[s] = (S.occ[l >> 5] >> (l & 31)) & 1u;
    }
  }
#pragma unroll
  for (int s = 0; s < kDosSitesPerThread; ++s) {
    if (l0 + s * kDosBlock >= N) break;
    const double e = ev[s];
    const uint32_t n = nv[s];
    const double x = floor((e - e_lo) * scale);
    int slot;
    if (x < 0.0) {
      slot = 2 * nbins;
    } else if (x >= (double)nbins) {
      slot = 2 * nbins + 1;
    } else {
      slot = (int)x + (n ? 0 : nbins);
    }
    atomicAdd(&h[slot], 1u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_slots; k += kDosBlock) {
    if (h[k] != 0u) atomicAdd(&hist[k], (unsigned long long)h[k]);
  }
}

}  // namespace cg
