// Device helpers shared by the gfx950 kernels: wave64 reductions, wave-local
// memory ordering, and error plumbing for the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define NRTO_WAVE 64

namespace nrto {

// Sum over the 64 lanes of a wavefront (butterfly; every lane gets the total).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, NRTO_WAVE);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, NRTO_WAVE);
    v = v > w ? v : w;
  }
  return v;
}

// Order this wave's LDS/global accesses before the following ones, as seen by
// the other lanes of the same wave (lanes exchange data through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (NRTO_WAVE - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / NRTO_WAVE; }

}  // namespace nrto
