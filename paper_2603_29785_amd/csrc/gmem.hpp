// Buffer-resource access to global memory for gfx950.
//
// A buffer resource (V#) holds a wave-uniform base address and a size in
// bytes. Loads and stores take a per-lane 32-bit byte offset plus a
// wave-uniform offset held in a scalar register, so a constant part of an
// address costs no vector instruction. Loads at or beyond the size return
// zero and stores there are dropped (range check on the per-lane offset), which
// lets a workgroup past the end of the work run the same code path as the
// others without touching memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtam {

// Third descriptor word for raw (untyped, unswizzled) buffers on gfx9-family
// parts, gfx950 included.
constexpr int kRawBufferWord3 = 0x00020000;

using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0),
                                           static_cast<int>(bytes), kRawBufferWord3);
}

// Cache policy of one access (the instruction's cache-policy bits): kCacheNT
// marks a stream that is not read again soon, so it does not displace lines
// that are (gfx940-family encoding: bit 1 = NT).
constexpr int kCacheDefault = 0;
constexpr int kCacheNT = 2;

template <typename V> struct BufIO;

template <> struct BufIO<float2> {
  template <int AUX>
  __device__ static __forceinline__ float2 load(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
  }
  template <int AUX>
  __device__ static __forceinline__ void store(rsrc_t r, float2 v, uint32_t voff, uint32_t soff) {
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, voff, soff, AUX);
  }
};

template <> struct BufIO<double2> {
  template <int AUX>
  __device__ static __forceinline__ double2 load(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
  }
  template <int AUX>
  __device__ static __forceinline__ void store(rsrc_t r, double2 v, uint32_t voff, uint32_t soff) {
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, v), r, voff, soff, AUX);
  }
};

template <> struct BufIO<float> {
  template <int AUX>
  __device__ static __forceinline__ float load(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
  }
};

template <> struct BufIO<double> {
  template <int AUX>
  __device__ static __forceinline__ double load(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
  }
};

template <typename V, int AUX = kCacheDefault>
__device__ __forceinline__ V bload(rsrc_t r, uint32_t voff, uint32_t soff = 0) {
  return BufIO<V>::template load<AUX>(r, voff, soff);
}

template <typename V, int AUX = kCacheDefault>
__device__ __forceinline__ void bstore(rsrc_t r, V v, uint32_t voff, uint32_t soff = 0) {
  BufIO<V>::template store<AUX>(r, v, voff, soff);
}

}  // namespace qtam
