// Raw buffer access (gfx9 buffer resources) and wave-uniform values.
//
// A load whose byte offset lies outside [0, num_records) returns zero without
// touching memory, and such a store is dropped.  Absent arrays get
// num_records = 0, absent positions an offset of kNoOffset, so loads can be
// issued unconditionally.  The base address sits in scalar registers and the
// per-lane part is a 32-bit byte offset, so an array is limited to 4 GiB.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kiops {

constexpr uint32_t kNoOffset = 0xFFFFFFF0u;

// Every array a resource is made for is the same for the whole wave; the base
// and extent are read from the first active lane so that the resource sits in
// scalar registers even where the compiler cannot prove the pointer uniform
// (a parameter block read from memory), which would otherwise wrap each
// access in a loop over the distinct values of the lanes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint64_t bytes) {
  const uint64_t b = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  const int n = __builtin_amdgcn_readfirstlane((p && bytes < 0xFFFFFFFFull) ? (int)(uint32_t)bytes : 0);
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0, n,
                                           0x00020000);
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
typedef unsigned int kiops_u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));
typedef unsigned int kiops_u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned int))));
// Stores of pass outputs carry device scope (the sc1 cache-policy bit): they
// are written through the XCD's L2 instead of staying there dirty, so the
// agent-scope release fence of the grid barrier that follows every pass has
// little left to write back (the arrival fence had taken 3-5 us per
// workgroup at 2048^2; with these stores the sweep is 1.7% faster).  The
// fences are unchanged: the policy is a placement hint, not the ordering.
constexpr int kStoreDeviceScope = 16;
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(kiops_u32x2, v), r, off, 0, kStoreDeviceScope);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, kStoreDeviceScope);
}
// two consecutive doubles (16-byte aligned offset)
__device__ __forceinline__ void buf_ld2(__amdgpu_buffer_rsrc_t r, uint32_t off, double& x, double& y) {
  const kiops_u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  x = __builtin_bit_cast(double, kiops_u32x2{v[0], v[1]});
  y = __builtin_bit_cast(double, kiops_u32x2{v[2], v[3]});
}

// The value of the first active lane, for values the program knows to be the
// same across the wave (lets the compiler keep them in scalar registers).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uniform(T* p) {
  const uint64_t b = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Copy of a small trivially-copyable struct that is the same for the whole
// wave, read word by word from memory and converted to wave-uniform values:
// its fields can then live in scalar registers even though the memory it
// came from may change later in the launch (so scalar loads are not allowed).
template <class S>
__device__ __forceinline__ S load_uniform(const S* src) {
  static_assert(sizeof(S) % 4 == 0, "word-sized struct");
  S out;
  const uint32_t* from = reinterpret_cast<const uint32_t*>(src);
  uint32_t words[sizeof(S) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) words[i] = __builtin_amdgcn_readfirstlane(from[i]);
  __builtin_memcpy(&out, words, sizeof(S));
  return out;
}

}  // namespace kiops
