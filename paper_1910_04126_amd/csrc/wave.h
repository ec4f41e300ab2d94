// Wavefront (64-lane) primitives for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ft {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// Inclusive prefix sum over lanes.
template <class T>
__device__ __forceinline__ T wave_incl_sum(T v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (l >= o) v += u;
  }
  return v;
}

// Inclusive prefix max over lanes.
template <class T>
__device__ __forceinline__ T wave_incl_max(T v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (l >= o && u > v) v = u;
  }
  return v;
}

// Inclusive suffix min over lanes (lane l gets min over lanes l..63).
template <class T>
__device__ __forceinline__ T wave_suffix_min(T v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_down(v, o, 64);
    if (l + o < 64 && u < v) v = u;
  }
  return v;
}

// Inclusive segmented sum of two values at once; `start` marks lanes that
// begin a new segment (the segment's own value is kept, earlier ones are not
// added).  Returns the flag "some lane at or before me started a segment".
__device__ __forceinline__ bool wave_seg_incl_sum2(uint32_t& a, uint32_t& b, bool start) {
  const int l = lane_id();
  uint32_t f = start ? 1u : 0u;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t ua = __shfl_up(a, o, 64);
    uint32_t ub = __shfl_up(b, o, 64);
    uint32_t uf = __shfl_up(f, o, 64);
    if (l >= o) {
      if (!f) {
        a += ua;
        b += ub;
      }
      f |= uf;
    }
  }
  return f != 0;
}

}  // namespace ft
