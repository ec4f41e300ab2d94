// Relaxed WMD (paper Section 1.1) and ACT-i (Section 4.1: R-WMD with
// capacity constraints added over i iterations; i = 0 is R-WMD) for
// (query, candidate) pairs -- the quadratic-time stage that follows Flowtree
// in the paper's pipelines.
//
// Per pair, every support point of one side needs its i + 1 nearest points
// of the other side, in both directions.  All squared distances of a pair
// come from inner products of its two sets of rows, a dense contraction, on
// the fp64 matrix cores: D^2 = |x|^2 + |y|^2 - 2 <x, y>, with the fp32
// coordinates widened exactly and every product and sum in fp64.  That form
// cancels where x is close to y; in fp64 the cancellation leaves an absolute
// error near 1e-16 (|x|^2 + |y|^2) on D^2, so the result is rounded to fp32
// and selected on directly, except for the rare entries within 2^-40
// (|x|^2 + |y|^2) of zero, which are recomputed in the difference form.
// Points of the same id are at distance exactly 0.  The capacity walk then
// runs with integer masses, D = sqrt(D^2) and fp64 products and sums.
//
// A 32 x 32 block of the (doc item x query item)
// matrix is four 16 x 16 tiles of v_mfma_f64_16x16x4_f64, fed straight from
// L2: per step the four lane groups of 16 take four consecutive float4s of
// their rows (the contraction order is immaterial), so each load reads 64
// contiguous bytes of every row it touches.  The block's
// D^2 goes through LDS; lanes 0..31 then walk its rows (doc items, whose i+1
// nearest stay in registers across the row of blocks), lanes 32..63 its
// columns (query items, whose i+1 nearest stay in LDS).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "flow.h"
#include "select.h"
#include "wave.h"

namespace ft {

typedef double act_f64x4 __attribute__((ext_vector_type(4)));

struct ActArgs {
  const int64_t* q_off;
  const uint32_t* q_rank;
  const uint32_t* q_mass;
  const int64_t* d_off;
  const uint32_t* d_rank;
  const uint32_t* d_mass;
  const int64_t* cand;    // knn form: [n_q * n_cols] doc per (query, column), or NULL (column = doc)
  int64_t n_cols;
  const int64_t* qlist;   // knn form: the queries of this launch (workgroup b: query qlist[b / n_cols])
  const int64_t* pair_q;  // pairs form: explicit (query, doc) pairs
  const int64_t* pair_d;
  const float* X;         // Morton-ordered rows, stride dp, padded with zeros
  const double* Xn;       // their squared norms (fp64)
  int dp;
  int NS;                 // float4 steps of 16 coordinates: ceil(dp / 16)
  int Q;
  int iters;
  uint32_t* status;
  float* cost;            // knn form: [query * n_cols + column]; pairs form: [pair]
};

// K1: how many nearest points an item keeps (a power of two >= iters + 1).
template <int K1, int QMAX>
struct ActLds {
  float tile[32][33];    // D^2 of the current block: [doc item][query item]
  double nr[32], nc[32]; // squared norms of the block's rows and columns
  uint32_t rr[32], rc[32];
  float cd[K1][QMAX];    // per query item: its K1 smallest D^2 so far, ascending
  uint16_t ci[K1][QMAX]; // and the doc items they belong to
};


// Keeps the K1 smallest values, ascending; an equal value does not displace
// an earlier one (indices arrive in ascending order, so ties keep the lower
// index first).
template <int K1>
__device__ __forceinline__ void keep_nearest(float (&v)[K1], int (&ix)[K1], float u, int j) {
  if (u < v[K1 - 1]) {
    v[K1 - 1] = u;
    ix[K1 - 1] = j;
#pragma unroll
    for (int t = K1 - 1; t > 0; --t) {
      if (v[t] < v[t - 1]) {
        const float w = v[t];
        v[t] = v[t - 1];
        v[t - 1] = w;
        const int wi = ix[t];
        ix[t] = ix[t - 1];
        ix[t - 1] = wi;
      }
    }
  }
}

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
                                           bool tail_in, act_f64x4& c00, act_f64x4& c01, act_f64x4& c10,
                                           act_f64x4& c11) {
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

// D^2 of doc items ib.. x query items jb.. into L.tile (32 x 32; entries
// past ni / nj are not written).
template <int K1, int QMAX>
__device__ __forceinline__ void block_d2(ActLds<K1, QMAX>& L, const ActArgs& a, const uint32_t* __restrict__ dr,
                                         const uint32_t* __restrict__ qr, int ib, int ni, int jb, int nj) {
  const int lane = threadIdx.x;
  const int r16 = lane & 15, g = lane >> 4;
  const bool two_a = ni > 16, two_b = nj > 16;  // wave-uniform: skip empty 16-row halves
  const uint32_t ra0 = dr[ib + min(r16, ni - 1)], ra1 = dr[ib + min(16 + r16, ni - 1)];
  const uint32_t rb0 = qr[jb + min(r16, nj - 1)], rb1 = qr[jb + min(16 + r16, nj - 1)];
  const float* pa0 = a.X + (size_t)ra0 * a.dp + 4 * g;
  const float* pa1 = a.X + (size_t)ra1 * a.dp + 4 * g;
  const float* pb0 = a.X + (size_t)rb0 * a.dp + 4 * g;
  const float* pb1 = a.X + (size_t)rb1 * a.dp + 4 * g;
  const bool tail_in = 16 * (a.NS - 1) + 4 * g < a.dp;
  act_f64x4 c00, c01, c10, c11;
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
  auto put = [&](const act_f64x4& c, int i0, int j) {
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
}

// The capacity walk of one item over its K1 nearest points of the other
// side (ascending D^2): the first `iters` take at most their own mass, the
// next one takes the rest.  Returns sum mass x distance.
template <int K1>
__device__ __forceinline__ double capacity_walk(const float (&d2)[K1], const int (&ix)[K1], uint32_t r,
                                                const uint32_t* __restrict__ cap_mass, int iters, int n_other) {
  double contrib = 0.0;
  const int capped = min(iters, n_other);
#pragma unroll
  for (int t = 0; t < K1; ++t) {
    const double D = sqrt((double)d2[t]);
    if (t < capped) {
      const uint32_t f = min(r, cap_mass[ix[t]]);
      contrib += (double)f * D;
      r -= f;
    } else if (t == iters && iters < n_other) {
      contrib += (double)r * D;
      r = 0;
    }
  }
  return contrib;
}

// Sum over the wavefront in a fixed order (rows of 16 by DPP, then the four
// rows), valid in every lane.
__device__ __forceinline__ double act_wave_sum(double v) {
  v = row_sum_f64(v);
  return (__shfl(v, 0, 64) + __shfl(v, 16, 64)) + (__shfl(v, 32, 64) + __shfl(v, 48, 64));
}

// One wavefront per pair, held to 128 registers (no accumulators in AGPRs)
// so that four fit on a SIMD: while one walks its block, others keep the
// matrix core busy.
template <int K1, int QMAX>
__global__ __launch_bounds__(64, 4) void k_act(ActArgs a) {
  __shared__ ActLds<K1, QMAX> L;
  const int lane = threadIdx.x;
  const int me = lane & 31;
  // workgroups are dealt to the 8 XCDs in turn; give each XCD a contiguous
  // range of pairs, so the candidates of one query share that XCD's L2
  const int64_t nb = gridDim.x, x = blockIdx.x & 7, per = nb >> 3, rem = nb & 7;
  const int64_t b = x * per + (x < rem ? x : rem) + (blockIdx.x >> 3);
  int64_t q, doc, out;
  if (a.pair_q) {
    out = b;
    q = a.pair_q[out];
    doc = a.pair_d[out];
  } else {
    const int64_t qi = b / a.n_cols, c = b - qi * a.n_cols;
    q = a.qlist[qi];
    out = q * a.n_cols + c;
    doc = a.cand ? a.cand[out] : c;
  }
  const int64_t qa = a.q_off[q], da = a.d_off[doc];
  // the same in every lane; held in scalar registers
  const int nq = __builtin_amdgcn_readfirstlane((int)(a.q_off[q + 1] - qa));
  const int nd = __builtin_amdgcn_readfirstlane((int)(a.d_off[doc + 1] - da));
  if (nq > QMAX || nd > FT_MAX_SUPPORT) {  // the host picks the class; never taken
    if (lane == 0) atomicOr(a.status, ERR_SIZE);
    return;
  }
  const uint32_t* dr = a.d_rank + da;
  const uint32_t* dm = a.d_mass + da;
  const uint32_t* qr = a.q_rank + qa;
  const uint32_t* qm = a.q_mass + qa;
  for (int j = lane; j < nq; j += 64) {
#pragma unroll
    for (int t = 0; t < K1; ++t) L.cd[t][j] = INFINITY;
  }
  double tot_d = 0.0;
  for (int ib = 0; ib < nd; ib += 32) {
    const int ni = min(32, nd - ib);
    float rv[K1];
    int rix[K1];
#pragma unroll
    for (int t = 0; t < K1; ++t) {
      rv[t] = INFINITY;
      rix[t] = 0;
    }
    for (int jb = 0; jb < nq; jb += 32) {
      const int nj = min(32, nq - jb);
      block_d2(L, a, dr, qr, ib, ni, jb, nj);
      __syncthreads();
      if (lane < 32) {
        if (me < ni)
          for (int x = 0; x < nj; ++x) keep_nearest<K1>(rv, rix, L.tile[me][x], jb + x);
      } else if (me < nj) {
        const int j = jb + me;
        float cv[K1];
        int cix[K1];
#pragma unroll
        for (int t = 0; t < K1; ++t) {
          cv[t] = L.cd[t][j];
          cix[t] = L.ci[t][j];
        }
        for (int x = 0; x < ni; ++x) keep_nearest<K1>(cv, cix, L.tile[x][me], ib + x);
#pragma unroll
        for (int t = 0; t < K1; ++t) {
          L.cd[t][j] = cv[t];
          L.ci[t][j] = (uint16_t)cix[t];
        }
      }
      __syncthreads();
    }
    const double c = lane < ni ? capacity_walk<K1>(rv, rix, dm[ib + lane], qm, a.iters, nq) : 0.0;
    tot_d += act_wave_sum(c);
  }
  double tot_q = 0.0;
  for (int c0 = 0; c0 < nq; c0 += 64) {
    const int j = c0 + lane;
    double c = 0.0;
    if (j < nq) {
      float cv[K1];
      int cix[K1];
#pragma unroll
      for (int t = 0; t < K1; ++t) {
        cv[t] = L.cd[t][j];
        cix[t] = L.ci[t][j];
      }
      c = capacity_walk<K1>(cv, cix, qm[j], dm, a.iters, nd);
    }
    tot_q += act_wave_sum(c);
  }
  if (lane == 0) a.cost[out] = (float)ldexp(tot_d > tot_q ? tot_d : tot_q, -a.Q);
}

// ------------------------------------------------------------- dispatch --

constexpr int ACT_QMAX[3] = {128, 512, FT_MAX_SUPPORT};

static int act_class(int nq) {
  for (int c = 0; c < 3; ++c)
    if (nq <= ACT_QMAX[c]) return c;
  return -1;
}

template <int K1>
static void launch_k1(int cls, int64_t grid, const ActArgs& a, hipStream_t s) {
  if (cls == 0) k_act<K1, 128><<<dim3((unsigned)grid), 64, 0, s>>>(a);
  else if (cls == 1) k_act<K1, 512><<<dim3((unsigned)grid), 64, 0, s>>>(a);
  else k_act<K1, FT_MAX_SUPPORT><<<dim3((unsigned)grid), 64, 0, s>>>(a);
}

static void launch_act(int cls, int64_t grid, const ActArgs& a, hipStream_t s) {
  if (grid <= 0) return;
  FT_REQUIRE(grid < (int64_t(1) << 31), FT_ERANGE, "too many pairs in one launch");
  if (a.iters == 0) launch_k1<1>(cls, grid, a, s);
  else if (a.iters == 1) launch_k1<2>(cls, grid, a, s);
  else if (a.iters <= 3) launch_k1<4>(cls, grid, a, s);
  else launch_k1<8>(cls, grid, a, s);
  FT_HIP(hipGetLastError());
}

static ActArgs act_args(ft_index* ix, int32_t iters) {
  ActArgs a{};
  a.q_rank = ix->qry.rank.as<uint32_t>();
  a.q_mass = ix->qry.mass.as<uint32_t>();
  a.d_off = ix->docs.off.as<int64_t>();
  a.d_rank = ix->docs.rank.as<uint32_t>();
  a.d_mass = ix->docs.mass.as<uint32_t>();
  a.X = ix->Xm.as<float>();
  a.Xn = ix->Xn.as<double>();
  a.dp = ix->dp;
  a.NS = (int)ceil_div(ix->dp, 16);
  a.Q = ix->Q;
  a.iters = iters;
  a.status = ix->status.as<uint32_t>();
  return a;
}

}  // namespace ft

using namespace ft;

extern "C" ft_status ft_act_knn(ft_index* ix, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                                int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t iters, int32_t k,
                                float* out_cost, int64_t* out_doc, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && out_cost && out_doc, FT_EINVAL, "NULL argument");
    FT_REQUIRE(iters >= 0 && iters <= 7, FT_EINVAL, "iters must lie in [0, 7]");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_cols = cand ? (int64_t)n_cand : ix->docs.n;
    FT_REQUIRE(!cand || (n_cand >= 1 && n_cand <= 4096), FT_ERANGE, "n_cand must lie in [1, 4096]");
    FT_REQUIRE(k >= 1 && k <= n_cols, FT_EINVAL, "k must lie in [1, number of candidates]");
    FT_REQUIRE(n_cols <= 4096 || k <= 1024, FT_ERANGE, "k > 1024 needs at most 4096 candidates");
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    if (cand) check_indices(ix, cand, n_q * n_cand, ix->docs.n, s, "cand");
    FT_REQUIRE(act_class(ix->qry.max_size) >= 0, FT_ERANGE, "query larger than FT_MAX_SUPPORT points");
    // queries grouped by size class (host copy of the offsets)
    std::vector<int64_t> qoff(n_q + 1);
    FT_HIP(hipMemcpyAsync(qoff.data(), ix->qry.off.as<int64_t>(), (n_q + 1) * 8, hipMemcpyDeviceToHost, s));
    FT_HIP(hipStreamSynchronize(s));
    const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(n_q, (int64_t(1) << 28) / n_cols));
    float* cost = (float*)ix->ws_cost.ensure(rows * n_cols * 4);
    int64_t* qlist = (int64_t*)ix->ws_misc.ensure(rows * 8);
    std::vector<int64_t> hl(rows);
    for (int64_t r0 = 0; r0 < n_q; r0 += rows) {
      const int64_t r1 = std::min(n_q, r0 + rows);
      // per class, the chunk's queries (relative to r0), in order
      int64_t pos = 0, start[4] = {0, 0, 0, 0};
      for (int c = 0; c < 3; ++c) {
        start[c] = pos;
        for (int64_t q = r0; q < r1; ++q)
          if (act_class((int)(qoff[q + 1] - qoff[q])) == c) hl[pos++] = q - r0;
      }
      start[3] = pos;
      FT_HIP(hipMemcpyAsync(qlist, hl.data(), pos * 8, hipMemcpyHostToDevice, s));
      ActArgs a = act_args(ix, iters);
      a.q_off = ix->qry.off.as<int64_t>() + r0;
      a.cand = cand ? cand + r0 * n_cols : nullptr;
      a.n_cols = n_cols;
      a.cost = cost;
      if (r0 == 0) FT_HIP(hipEventRecord(ix->ev_t0, s));
      for (int c = 0; c < 3; ++c) {
        a.qlist = qlist + start[c];
        launch_act(c, (start[c + 1] - start[c]) * n_cols, a, s);
      }
      if (r1 == n_q) FT_HIP(hipEventRecord(ix->ev_t1, s));
      topk_rows(cost, r1 - r0, n_cols, a.cand, k, out_cost + r0 * k, out_doc + r0 * k, s);
      FT_HIP(hipStreamSynchronize(s));  // hl is reused by the next chunk
    }
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "act kernel reported:" + describe_flags(flags));
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ix->ev_t0, ix->ev_t1) == hipSuccess) ix->last_act_ms = ms;
  });
}

extern "C" ft_status ft_last_act_stats(const ft_index* ix, double* ms) {
  return guarded([&] {
    FT_REQUIRE(ix && ms, FT_EINVAL, "NULL argument");
    *ms = ix->last_act_ms;
  });
}

extern "C" ft_status ft_act_pairs(ft_index* ix, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                                  int64_t n_q, const int64_t* pair_q, const int64_t* pair_d, int64_t n_pairs,
                                  int32_t iters, float* out_cost, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && pair_q && pair_d && out_cost, FT_EINVAL, "NULL argument");
    FT_REQUIRE(iters >= 0 && iters <= 7, FT_EINVAL, "iters must lie in [0, 7]");
    FT_REQUIRE(n_pairs >= 0, FT_EINVAL, "n_pairs must be >= 0");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    if (n_pairs == 0) return;
    check_indices(ix, pair_q, n_pairs, n_q, s, "pair_q");
    check_indices(ix, pair_d, n_pairs, ix->docs.n, s, "pair_d");
    const int cls = act_class(ix->qry.max_size);
    FT_REQUIRE(cls >= 0, FT_ERANGE, "query larger than FT_MAX_SUPPORT points");
    ActArgs a = act_args(ix, iters);
    a.q_off = ix->qry.off.as<int64_t>();
    a.pair_q = pair_q;
    a.pair_d = pair_d;
    a.cost = out_cost;
    launch_act(cls, n_pairs, a, s);
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "act kernel reported:" + describe_flags(flags));
  });
}
