// Device helpers shared by the kernels: Philox4x32-10, deterministic block
// reductions and tree arithmetic.
#pragma once

#include "qram_internal.h"

namespace qr {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the Philox S-box, the
// key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32 x 32 -> 64-bit product in one multiply (both halves)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// u = (u64 >> 11) 2^-53 with u64 = w0 | w1 << 32 of the Philox block.
__device__ __forceinline__ double uniform53(uint64_t seed, uint32_t c0,
                                            uint32_t c1, uint32_t traj,
                                            uint32_t tag) {
  const uint4 w = philox10(make_uint4(c0, c1, traj, tag), (uint32_t)seed,
                           (uint32_t)(seed >> 32));
  const uint64_t u = (uint64_t)w.x | ((uint64_t)w.y << 32);
  return (double)(u >> 11) * 0x1.0p-53;
}

// Layer of tree node v (the root is layer 0).
__device__ __forceinline__ int layer_of(uint32_t v) { return 31 - __clz(v + 1); }

// Sum of N doubles over the block: xor butterfly inside each wave, then the
// wave partials added in wave order by every thread (bitwise identical in
// every thread, independent of scheduling).
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[i] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) buf[wave * N + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += buf[w * N + i];
    v[i] = t;
  }
}

// Exclusive prefix sum of one double over the block, in thread order.
__device__ __forceinline__ double block_excl_scan(double x, double *buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) buf[wave] = incl;
  __syncthreads();
  double base = 0.0;
  for (int w = 0; w < wave; ++w) base += buf[w];
  return base + incl - x;
}

__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t x,
                                                        uint32_t *buf,
                                                        uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) buf[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wave) base += buf[w];
    tot += buf[w];
  }
  *total = tot;
  return base + incl - x;
}

}  // namespace qr
