// ring_common.h -- device helpers shared by the ring-window kernels (the
// forward ring march and the ring adjoint): uniform-value helpers, wave
// reductions, the direct global->LDS load and its wait, and the window record.
#pragma once

#include "vr_internal.h"

namespace vr {
namespace ring {

typedef const float __attribute__((address_space(1))) gfloat;

__device__ __forceinline__ float wmin4(float v) {
  v = fminf(v, __shfl_xor(v, 1));
  return fminf(v, __shfl_xor(v, 2));
}
__device__ __forceinline__ float wmax4(float v) {
  v = fmaxf(v, __shfl_xor(v, 1));
  return fmaxf(v, __shfl_xor(v, 2));
}
__device__ __forceinline__ int wave_imin(int v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ int wave_imax(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// a pointer the compiler must treat as uniform (it lives in scalar registers)
__device__ __forceinline__ gfloat* unip(gfloat* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gfloat*)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float unif(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
// wave vote known to the compiler as uniform
__device__ __forceinline__ bool wany(bool p) { return uni(__any(p) ? 1 : 0) != 0; }
// value of v in lane l (uniform)
__device__ __forceinline__ float lanef(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Wait until every global->LDS load this wavefront issued has landed (the
// memory clobber keeps LDS reads from moving above the wait).
__device__ __forceinline__ void wait_loads() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// 16 bytes per lane from global memory (base + voff bytes; base uniform, voff
// per lane) straight into LDS at lds_base + 16 lane (a byte address, uniform
// over the wavefront).  Written as inline assembly so that the compiler does
// not guard later LDS reads with waits for these loads: the code waits for
// them explicitly with wait_loads().  The kernel keeps no value of its own in
// M0 (it uses no instruction that reads M0 besides this one).
__device__ __forceinline__ void lds_dma16(gfloat* base, unsigned voff, unsigned lds_base) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
               :
               : "v"(voff), "s"(base), "s"(lds_base)
               : "memory", "m0");
}

__device__ __forceinline__ unsigned lds_addr(const float* p) {
  return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) float*)p;
}

// Window of one voxel layer: rows along axis 1 (f), `pitch` floats each, NG rows
// along the in-plane axis g; origin (f0, g0) in brick-local voxel indices.
struct Window {
  int f0, g0;
};

}  // namespace ring
}  // namespace vr
