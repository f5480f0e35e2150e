// cx_device.h -- device helpers shared by the library's kernels: the
// counter-based generator and global-address-space loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cx_internal.h"

namespace cx {
namespace {

struct U4 {
  uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon et al., SC'11).  The key is wave-uniform, so its
// schedule stays in scalar registers.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1) {
  // keep the round keys from being precomputed (and held in 20 scalar
  // registers) outside the step loop: bumping them costs two scalar adds
  asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 multiply per product gives both halves (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    c1 = (uint32_t)p1;
    c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// Exploring starts: the price day of the episode that began at global step g0,
// (word 0 of Philox (env, g0, 0, DAY) * n_days) >> 32.
__device__ __forceinline__ int episode_day(uint32_t env, uint32_t g0, uint32_t k0, uint32_t k1, int n_days) {
  return (int)__umulhi(philox(env, g0, 0u, kDomDay, k0, k1).x, (uint32_t)n_days);
}

// Loads through the global address space (the tables live in device memory;
// plain pointers from a struct would be generic and compile to flat loads).
template <class T>
__device__ __forceinline__ T gld(const T *p, int64_t i) {
  return ((const __attribute__((address_space(1))) T *)p)[i];
}

// Load through the constant address space: with a wave-uniform address this
// is a scalar load (counted apart from the vector stores in flight, so using it
// does not wait for them).
template <class T>
__device__ __forceinline__ T sld(const T *p, int64_t i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

}  // namespace
}  // namespace cx
