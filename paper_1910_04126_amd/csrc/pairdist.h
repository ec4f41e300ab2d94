// Squared Euclidean distances of all (doc item, query item) pairs of one
// (query, dataset distribution) pair, 32 x 32 at a time, for the
// quadratic-time estimates (R-WMD / ACT, Sinkhorn).
//
// D^2 = |x|^2 + |y|^2 - 2 <x, y> with the fp32 coordinates widened exactly
// and every product and sum in fp64, the inner products on the fp64 matrix
// cores (v_mfma_f64_16x16x4_f64): a 32 x 32 block is four 16 x 16 tiles fed
// straight from L2.  In fp64 the cancellation of that form leaves an
// absolute error near 1e-16 (|x|^2 + |y|^2) on D^2, so the result is
// rounded to fp32, except for the rare entries within 2^-40 (|x|^2 + |y|^2)
// of zero, which are recomputed in the difference form; points of the same
// id are at distance exactly 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "flow.h"

namespace ft {

typedef double pd_f64x4 __attribute__((ext_vector_type(4)));

// The coordinate table of the index.
struct PairRows {
  const float* X;    // Morton-ordered rows, stride dp, padded with zeros
  const double* Xn;  // their squared norms (fp64)
  int dp;
  int NS;            // float4 steps of 16 coordinates: ceil(dp / 16)
};

inline PairRows pair_rows(const ft_index* ix) {
  PairRows r;
  r.X = ix->Xm.as<float>();
  r.Xn = ix->Xn.as<double>();
  r.dp = ix->dp;
  r.NS = (int)ceil_div(ix->dp, 16);
  return r;
}

// One wavefront's block buffers.
struct BlockLds {
  float tile[32][33];     // D^2 of the current block: [doc item][query item]
  double nr[32], nc[32];  // squared norms of the block's rows and columns
  uint32_t rr[32], rc[32];
};

// Inner products of the 16-row halves a0 / a1 (doc rows) with b0 / b1 (query
// rows) over the full coordinate axis; TA / TB: the second halves exist.
// Step s: lane group g (lanes 16 g .. 16 g + 15, one row each) takes
// coordinates 16 s + 4 g .. 16 s + 4 g + 3 of its rows, so each load reads 64
// contiguous bytes of every row it touches; all steps but the last lie inside
// the rows, the last is cut at dp.  Rows past the block's items point at a
// valid row; their results are never read.
template <bool TA, bool TB>
__device__ __forceinline__ void block_dots(const float* __restrict__ pa0, const float* __restrict__ pa1,
                                           const float* __restrict__ pb0, const float* __restrict__ pb1, int NS,
                                           bool tail_in, pd_f64x4& c00, pd_f64x4& c01, pd_f64x4& c10,
                                           pd_f64x4& c11) {
  constexpr int PF = 2;
  float4 x0[PF], x1[PF], y0[PF], y1[PF];
  const int full = NS - 1;  // steps entirely inside the rows
  auto issue = [&](int t, int s) {
    x0[t] = *(const float4*)(pa0 + 16 * s);
    y0[t] = *(const float4*)(pb0 + 16 * s);
    if (TA) x1[t] = *(const float4*)(pa1 + 16 * s);
    if (TB) y1[t] = *(const float4*)(pb1 + 16 * s);
  };
  auto step = [&](const float4& xa4, const float4& xb4, const float4& ya4, const float4& yb4) {
    const float ea[4] = {xa4.x, xa4.y, xa4.z, xa4.w}, eb[4] = {xb4.x, xb4.y, xb4.z, xb4.w};
    const float fa[4] = {ya4.x, ya4.y, ya4.z, ya4.w}, fb[4] = {yb4.x, yb4.y, yb4.z, yb4.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double p = ea[c], q = fa[c];
      c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(p, q, c00, 0, 0, 0);
      if (TB) c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(p, (double)fb[c], c01, 0, 0, 0);
      if (TA) c10 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)eb[c], q, c10, 0, 0, 0);
      if (TA && TB) c11 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)eb[c], (double)fb[c], c11, 0, 0, 0);
    }
  };
  // a ring of PF steps in flight: the steady loop has no conditions, the
  // ragged end is unrolled with wave-uniform ones
  int s0 = 0;
  if (full >= PF) {
#pragma unroll
    for (int t = 0; t < PF; ++t) issue(t, t);
    for (; s0 + 2 * PF <= full; s0 += PF) {
#pragma unroll
      for (int t = 0; t < PF; ++t) {
        step(x0[t], x1[t], y0[t], y1[t]);
        issue(t, s0 + PF + t);
      }
    }
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      step(x0[t], x1[t], y0[t], y1[t]);
      if (s0 + PF + t < full) issue(t, s0 + PF + t);
    }
#pragma unroll
    for (int t = 0; t < PF; ++t)
      if (s0 + PF + t < full) step(x0[t], x1[t], y0[t], y1[t]);
  } else {
    for (int t = 0; t < full; ++t) {
      issue(0, t);
      step(x0[0], x1[0], y0[0], y1[0]);
    }
  }
  // the last step, cut at dp (lanes whose coordinates lie past it add zeros)
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  const int o = tail_in ? 16 * full : 0;
  float4 xa = *(const float4*)(pa0 + o), ya = *(const float4*)(pb0 + o);
  float4 xb = TA ? *(const float4*)(pa1 + o) : z, yb = TB ? *(const float4*)(pb1 + o) : z;
  if (!tail_in) xa = xb = ya = yb = z;
  step(xa, xb, ya, yb);
}

// D^2 of doc items ib.. x query items jb.. (Morton ranks dr, qr) into
// L.tile (32 x 32; entries past ni / nj are not written).  Called by a whole
// wavefront; ends with the tile visible to all its lanes.
__device__ __forceinline__ void block_d2(BlockLds& L, const PairRows& a, const uint32_t* __restrict__ dr,
                                         const uint32_t* __restrict__ qr, int ib, int ni, int jb, int nj) {
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  const bool two_a = ni > 16, two_b = nj > 16;  // wave-uniform: skip empty 16-row halves
  const uint32_t ra0 = dr[ib + min(r16, ni - 1)], ra1 = dr[ib + min(16 + r16, ni - 1)];
  const uint32_t rb0 = qr[jb + min(r16, nj - 1)], rb1 = qr[jb + min(16 + r16, nj - 1)];
  const float* pa0 = a.X + (size_t)ra0 * a.dp + 4 * g;
  const float* pa1 = a.X + (size_t)ra1 * a.dp + 4 * g;
  const float* pb0 = a.X + (size_t)rb0 * a.dp + 4 * g;
  const float* pb1 = a.X + (size_t)rb1 * a.dp + 4 * g;
  const bool tail_in = 16 * (a.NS - 1) + 4 * g < a.dp;
  pd_f64x4 c00, c01, c10, c11;
#pragma unroll
  for (int r = 0; r < 4; ++r) c00[r] = c01[r] = c10[r] = c11[r] = 0.0;
  if (two_a) {
    if (two_b) block_dots<true, true>(pa0, pa1, pb0, pb1, a.NS, tail_in, c00, c01, c10, c11);
    else block_dots<true, false>(pa0, pa1, pb0, pb1, a.NS, tail_in, c00, c01, c10, c11);
  } else {
    if (two_b) block_dots<false, true>(pa0, pa1, pb0, pb1, a.NS, tail_in, c00, c01, c10, c11);
    else block_dots<false, false>(pa0, pa1, pb0, pb1, a.NS, tail_in, c00, c01, c10, c11);
  }
  double* nr = L.nr;
  double* nc = L.nc;
  uint32_t* rr = L.rr;
  uint32_t* rc = L.rc;
  if (lane < 32) {
    const bool va = lane < ni, vb = lane < nj;
    const uint32_t ka = va ? dr[ib + lane] : 0u, kb = vb ? qr[jb + lane] : 0u;
    nr[lane] = va ? a.Xn[ka] : 0.0;
    nc[lane] = vb ? a.Xn[kb] : 0.0;
    rr[lane] = va ? ka : 0xFFFFFFFFu;
    rc[lane] = vb ? kb : 0xFFFFFFFEu;
  }
  __syncthreads();
  float(&tile)[32][33] = L.tile;
  // 16x16 fp64 result layout: lane l holds column l % 16, rows l / 16 + 4 r
  auto put = [&](const pd_f64x4& c, int i0, int j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + g + 4 * r;
      if (i < ni && j < nj) {
        const double sn = nr[i] + nc[j];
        const double d2 = sn - 2.0 * c[r];
        float v = (float)d2;
        if (rr[i] == rc[j]) {
          v = 0.0f;
        } else if (d2 <= 0x1p-40 * sn) {
          // within the rounding of the inner-product form: the difference
          // form of the two rows (exact differences, fp64 squares and sum)
          const float* x = a.X + (size_t)rr[i] * a.dp;
          const float* y = a.X + (size_t)rc[j] * a.dp;
          double e = 0.0;
          for (int k = 0; k < a.dp; ++k) {
            const double t = (double)x[k] - (double)y[k];
            e = fma(t, t, e);
          }
          v = (float)e;
        }
        tile[i][j] = v;
      }
    }
  };
  put(c00, 0, r16);
  if (two_b) put(c01, 0, 16 + r16);
  if (two_a) put(c10, 16, r16);
  if (two_a && two_b) put(c11, 16, 16 + r16);
  __syncthreads();
}

// Sum over the wavefront in a fixed order (rows of 16 by DPP, then the four
// rows), valid in every lane.
__device__ __forceinline__ double pair_wave_sum(double v) {
  v = row_sum_f64(v);
  return (__shfl(v, 0, 64) + __shfl(v, 16, 64)) + (__shfl(v, 32, 64) + __shfl(v, 48, 64));
}

}  // namespace ft
