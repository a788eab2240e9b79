// Device helpers shared by the sweep kernels: address-space casts and raw
// buffer access with per-lane masking by offset.
#pragma once

#include <hip/hip_runtime.h>

namespace bte {

#define GAS __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ GAS T* gp(T* p) {
  return (GAS T*)p;
}
template <typename T>
__device__ __forceinline__ const GAS T* gp(const T* p) {
  return (const GAS T*)p;
}

// Read-only tables (job list, instance records, group constants, flags, the
// status written by the previous kernel) read at uniform addresses through the
// constant address space: scalar loads into SGPRs, so everything derived from
// them, the loop bounds and the choice of step body included, stays uniform.
#ifdef __HIP_DEVICE_COMPILE__
#define CAS __attribute__((address_space(4)))
#else
#define CAS  // the host pass only parses the kernels
#endif
template <typename T>
__device__ __forceinline__ const CAS T* cp(const T* p) {
  return (const CAS T*)p;
}

// Raw buffer access with per-lane masking by offset: a byte offset at or past
// the buffer's size reads 0 and drops a store (the hardware range check), so
// a masked access needs no branch. The sweeps' chunk loops access global
// memory this way: with no branch around them the memory counters seen by
// each wait are exact, and a wait for prefetched data never also waits for
// the loads issued after it.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kBufWord3 = 0x00020000;  // raw 32-bit elements, no swizzle
constexpr int kOOB = (int)0x80000000;  // past every buffer
template <typename Ptr>
__device__ __forceinline__ rsrc_t mkrsrc(Ptr p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, kBufWord3);
}
__device__ __forceinline__ void bst(float v, rsrc_t r, int off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void bst(double v, rsrc_t r, int off) {
  typedef unsigned u2_t __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_t, v), r, off, 0, 0);
}
template <typename T>
__device__ __forceinline__ T bld(rsrc_t r, int off);
template <>
__device__ __forceinline__ float bld<float>(rsrc_t r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double bld<double>(rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ int bld<int>(rsrc_t r, int off) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// a record {cell, flags} and a vector of V at byte offsets voff (per lane) +
// soff (uniform)
__device__ __forceinline__ int2 ldrec_b(rsrc_t r, int voff, int soff) {
  typedef unsigned u2_t __attribute__((ext_vector_type(2)));
  const u2_t v = __builtin_bit_cast(u2_t, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  return make_int2((int)v.x, (int)v.y);
}
template <typename V>
__device__ __forceinline__ V ldv(rsrc_t r, int voff, int soff) {
  constexpr int B = (int)sizeof(V);
  static_assert(B == 4 || B == 8 || B % 16 == 0, "vector loads of 4 or 8 bytes or whole 16-byte parts");
  if constexpr (B == 4) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else if constexpr (B == 8) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    typedef unsigned u4_t __attribute__((ext_vector_type(4)));
    struct Parts {
      u4_t q[B / 16];
    } t;
#pragma unroll
    for (int i = 0; i < B / 16; ++i) t.q[i] = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16 * i, soff, 0);
    return __builtin_bit_cast(V, t);
  }
}

// store of a vector of V at byte offsets voff (per lane) + soff (uniform); an
// offset past the buffer drops the store
template <typename V>
__device__ __forceinline__ void stv(const V& v, rsrc_t r, int voff, int soff) {
  constexpr int B = (int)sizeof(V);
  static_assert(B == 4 || B == 8 || B % 16 == 0, "vector stores of 4 or 8 bytes or whole 16-byte parts");
  if constexpr (B == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
  } else if constexpr (B == 8) {
    typedef unsigned u2_t __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_t, v), r, voff, soff, 0);
  } else {
    typedef unsigned u4_t __attribute__((ext_vector_type(4)));
    struct Parts {
      u4_t q[B / 16];
    };
    const Parts t = __builtin_bit_cast(Parts, v);
#pragma unroll
    for (int i = 0; i < B / 16; ++i) __builtin_amdgcn_raw_buffer_store_b128(t.q[i], r, voff + 16 * i, soff, 0);
  }
}

// as ldv, at device scope (cache policy sc1: the load misses the CU's vector
// cache and reads L2), for data the same wave stored earlier
template <typename V>
__device__ __forceinline__ V ldv_glc(rsrc_t r, int voff, int soff) {
  constexpr int B = (int)sizeof(V);
  constexpr int kSc1 = 0x10;
  static_assert(B == 4 || B == 8 || B == 16, "vector loads of 4, 8 or 16 bytes");
  if constexpr (B == 4) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kSc1));
  } else if constexpr (B == 8) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kSc1));
  } else {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kSc1));
  }
}

}  // namespace bte
