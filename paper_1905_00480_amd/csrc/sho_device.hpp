// sho_device.hpp -- device helpers shared by the FP64 and FP32 kernel units
// of libsho.so (included by HIP translation units only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sho {

// Read-only data that every lane of a wave reads at the same address goes
// through the constant address space, i.e. scalar loads.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ inline cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}

// Copies a record that all lanes read at the same address (scalar loads).
template <typename T>
__device__ inline T load_uniform(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "record size");
  T out;
  const cptr<uint32_t> src = (cptr<uint32_t>)p;
  uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
  return out;
}

// Wave index within the workgroup (uniform: a scalar register).
__device__ inline int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

}  // namespace sho
