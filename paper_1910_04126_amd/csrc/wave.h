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

// DPP moves (GFX9 controls): the value of the lane that CTRL selects, or
// `old` where that lane lies outside the row or the row is off in ROWS (with
// bound_ctrl off, such a lane's write is disabled and it keeps `old`).
// row_shr:n is 0x110 + n, row_shl:n 0x100 + n, wave_shr:1 0x138, wave_shl:1
// 0x130, row_bcast:15 0x142 (lane 15 of a row to the whole next row),
// row_bcast:31 0x143 (lane 31 to rows 2 and 3).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}

template <class T>
__device__ __forceinline__ uint32_t bits32(T v) {
  static_assert(sizeof(T) == 4, "32-bit lanes only");
  return __builtin_bit_cast(uint32_t, v);
}

template <class T>
__device__ __forceinline__ T from32(uint32_t v) {
  return __builtin_bit_cast(T, v);
}

// Value of lane l - 1 (lane 0 gets `old`) and of lane l + 1 (lane 63 gets
// `old`).
template <class T>
__device__ __forceinline__ T wave_shr1(T v, T old) {
  return from32<T>(dpp_u32<0x138>(bits32(old), bits32(v)));
}
template <class T>
__device__ __forceinline__ T wave_shl1(T v, T old) {
  return from32<T>(dpp_u32<0x130>(bits32(old), bits32(v)));
}

// Lane `l`'s value in every lane (a scalar read).
template <class T>
__device__ __forceinline__ T lane_value(T v, int l) {
  return from32<T>((uint32_t)__builtin_amdgcn_readlane((int)bits32(v), l));
}

// Inclusive scan over lanes of a 32-bit value under an associative op with
// identity `id`: rows of 16 by row shifts of 1, 2, 4, 8 (a lane with no
// source that far back in its row takes `id`), then rows 1 and 3 take lane
// 15 of the row before, then rows 2 and 3 take lane 31.  All of it runs on
// DPP moves in the vector ALU.
template <class T, class Op>
__device__ __forceinline__ T wave_scan32(T v, const T id, Op op) {
  v = op(v, from32<T>(dpp_u32<0x111>(bits32(id), bits32(v))));
  v = op(v, from32<T>(dpp_u32<0x112>(bits32(id), bits32(v))));
  v = op(v, from32<T>(dpp_u32<0x114>(bits32(id), bits32(v))));
  v = op(v, from32<T>(dpp_u32<0x118>(bits32(id), bits32(v))));
  v = op(v, from32<T>(dpp_u32<0x142, 0xA>(bits32(id), bits32(v))));
  v = op(v, from32<T>(dpp_u32<0x143, 0xC>(bits32(id), bits32(v))));
  return v;
}

// Inclusive prefix sum over lanes.
template <class T>
__device__ __forceinline__ T wave_incl_sum(T v) {
  if constexpr (sizeof(T) == 4) {
    return wave_scan32(v, T(0), [](T x, T y) { return x + y; });
  } else {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      T u = __shfl_up(v, o, 64);
      if (l >= o) v += u;
    }
    return v;
  }
}

// Inclusive prefix max over lanes (32-bit signed).
__device__ __forceinline__ int wave_incl_max(int v) {
  return wave_scan32(v, (int)0x80000000, [](int x, int y) { return x > y ? x : y; });
}

// Inclusive suffix min over lanes (lane l gets the min over lanes l..63;
// 32-bit signed): row shifts towards lane 0 inside rows of 16, then each row
// takes the minima of the rows after it, read from their first lanes.
__device__ __forceinline__ int wave_suffix_min(int v) {
  const int l = lane_id();
  const uint32_t id = 0x7FFFFFFFu;
  v = min(v, (int)dpp_u32<0x101>(id, (uint32_t)v));
  v = min(v, (int)dpp_u32<0x102>(id, (uint32_t)v));
  v = min(v, (int)dpp_u32<0x104>(id, (uint32_t)v));
  v = min(v, (int)dpp_u32<0x108>(id, (uint32_t)v));
  const int m3 = lane_value(v, 48);
  const int m2 = min(lane_value(v, 32), m3);
  const int m1 = min(lane_value(v, 16), m2);
  const int row = l >> 4;
  const int after = row == 0 ? m1 : row == 1 ? m2 : row == 2 ? m3 : 0x7FFFFFFF;
  return v < after ? v : after;
}

// Inclusive segmented sum of two values at once; `start` marks lanes that
// begin a new segment (the segment's own value is kept, earlier ones are not
// added).  Returns the flag "some lane at or before me started a segment".
// Same DPP steps as wave_scan32 on the (a, b, flag) triple.
__device__ __forceinline__ bool wave_seg_incl_sum2(uint32_t& a, uint32_t& b, bool start) {
  uint32_t f = start ? 1u : 0u;
  // a lane with no source takes (0, 0, 0), which changes nothing
#define FT_SEG_STEP(CTRL, ROWS)                        \
  {                                                    \
    const uint32_t ua = dpp_u32<CTRL, ROWS>(0u, a);    \
    const uint32_t ub = dpp_u32<CTRL, ROWS>(0u, b);    \
    const uint32_t uf = dpp_u32<CTRL, ROWS>(0u, f);    \
    const uint32_t keep = f ? 0u : 0xFFFFFFFFu;        \
    a += ua & keep;                                    \
    b += ub & keep;                                    \
    f |= uf;                                           \
  }
  FT_SEG_STEP(0x111, 0xF)
  FT_SEG_STEP(0x112, 0xF)
  FT_SEG_STEP(0x114, 0xF)
  FT_SEG_STEP(0x118, 0xF)
  FT_SEG_STEP(0x142, 0xA)
  FT_SEG_STEP(0x143, 0xC)
#undef FT_SEG_STEP
  return f != 0;
}

}  // namespace ft
