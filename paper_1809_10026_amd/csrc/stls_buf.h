// Range-checked buffer access for gfx950 kernels.
//
// A lane whose byte offset lies past the buffer's size is dropped by the
// hardware (store) or reads 0 (load), with no memory access.  Every lane
// issues the instruction, so a wave issues a fixed number of memory
// operations per work item whatever the padding, no select has to wait for a
// loaded value, and the compiler can wait for exactly the prefetched loads
// (on gfx9 one counter covers loads and stores).  Word 3 of the resource:
// 32-bit data format, no swizzle.  Buffers addressed this way are below
// 2 GiB.
#pragma once

#include <hip/hip_runtime.h>

namespace stls {

constexpr int kBufWord3 = 0x00020000;
constexpr int kOutOfRange = 0x7fffffff;  // beyond every buffer addressed this way
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3);
}
__device__ inline void buf_store(float v, __amdgpu_buffer_rsrc_t r, int off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}
__device__ inline void buf_store(double v, __amdgpu_buffer_rsrc_t r, int off) {
  typedef unsigned int u2_t __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_t, v), r, off, 0, 0);
}
__device__ inline float buf_load_f32(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline double buf_load_f64(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

}  // namespace stls
