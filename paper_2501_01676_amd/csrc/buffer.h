// Raw buffer access (CDNA buffer descriptors: record count 2^31 - 1 bytes,
// no stride, word 3 = 0x00020000, i.e. data format 32 bits, which untyped
// buffer loads and stores need on this architecture family).  A load whose
// offset is at or past the record count returns zero and such a store is
// dropped, so elements outside a matrix are selected to BUF_OUT instead of
// branched around.  Offsets are 32-bit byte offsets from the descriptor's
// base: every matrix read or written this way spans less than BUF_LIMIT
// bytes (checked on the host where the launch descriptors are built).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace abddc {

constexpr int BUF_OUT = int(0x80000000u);
constexpr int64_t BUF_LIMIT = int64_t(1) << 31;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7fffffff, 0x00020000);
}
template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <class T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

}  // namespace abddc
