// Sinkhorn with a fixed small number of iterations (paper Section 4.1
// baseline; the regularisation is set per pair from its largest cost, as the
// appendix on the Sinkhorn regularisation parameter does, eta = 30 there)
// for (query, candidate) pairs -- one of the quadratic-time stages that
// follow Flowtree in the paper's pipelines.
//
// Per pair: the full distance matrix D (fp32, from the fp64 matrix-core
// blocks of pairdist.h) is written once to the workgroup's slot of a scratch
// area, with its largest entry M.  The Gibbs kernel K = exp(-eta D / M) is
// recomputed from D on every pass (one exp2 per entry), never stored.  Each
// iteration scales rows, u = a / (K v), then columns, v = b / (K^T u),
// starting from v = 1; the estimate is sum_ij u_i K_ij v_j D_ij.  Row sums
// are taken with the lanes across the row and a fixed-order wavefront sum,
// column sums with one lane per column; all sums are fp64, so the result
// does not depend on the schedule.  Workgroups are persistent: each takes
// pairs blockIdx.x, blockIdx.x + gridDim.x, ... and reuses its slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "pairdist.h"
#include "select.h"
#include "wave.h"

namespace ft {

struct SinkArgs {
  const int64_t* q_off;
  const uint32_t* q_rank;
  const uint32_t* q_mass;
  const int64_t* d_off;
  const uint32_t* d_rank;
  const uint32_t* d_mass;
  const int64_t* cand;    // knn form: [n_q * n_cols] doc per (query, column), or NULL (column = doc)
  int64_t n_cols;
  const int64_t* pair_q;  // pairs form: explicit (query, doc) pairs
  const int64_t* pair_d;
  int64_t n_pairs;
  PairRows rows;
  int Q;
  int iters;
  float eta;
  float* scratch;         // gridDim.x slots of `slot` floats
  int64_t slot;
  uint32_t* status;
  float* cost;            // knn form: [query * n_cols + column]; pairs form: [pair]
};

struct SinkLds {
  BlockLds blk;
  float u[FT_MAX_SUPPORT];  // row scalings (doc items)
  float v[FT_MAX_SUPPORT];  // column scalings (query items)
};

constexpr int SR = 4;  // rows summed together

// Sums over j of K_ij v_j (WITH_D: times D_ij) for rows i0 .. i0 + SR - 1
// (rows past nd give 0): lanes across the row, then a fixed-order wavefront
// sum per row; the result is valid in every lane.
template <bool WITH_D>
__device__ __forceinline__ void row_sums(const float* __restrict__ S, int nq, int nd, int i0, float cexp,
                                         const float* __restrict__ v, double (&acc)[SR]) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int r = 0; r < SR; ++r) acc[r] = 0.0;
  for (int j = lane; j < nq; j += 64) {
    float d[SR];
#pragma unroll
    for (int r = 0; r < SR; ++r) d[r] = i0 + r < nd ? S[(int64_t)(i0 + r) * nq + j] : 0.0f;
    const float vj = v[j];
#pragma unroll
    for (int r = 0; r < SR; ++r) {
      const double t = (double)(exp2f(cexp * d[r]) * vj);
      acc[r] += WITH_D ? t * (double)d[r] : t;
    }
  }
#pragma unroll
  for (int r = 0; r < SR; ++r) acc[r] = i0 + r < nd ? pair_wave_sum(acc[r]) : 0.0;
}

__global__ __launch_bounds__(64) void k_sinkhorn(SinkArgs a) {
  __shared__ SinkLds L;
  const int lane = threadIdx.x;
  float* S = a.scratch + (int64_t)blockIdx.x * a.slot;
  for (int64_t p = blockIdx.x; p < a.n_pairs; p += gridDim.x) {
    int64_t q, doc;
    if (a.pair_q) {
      q = a.pair_q[p];
      doc = a.pair_d[p];
    } else {
      q = p / a.n_cols;
      const int64_t c = p - q * a.n_cols;
      doc = a.cand ? a.cand[p] : c;
    }
    const int64_t qa = a.q_off[q], da = a.d_off[doc];
    const int nq = __builtin_amdgcn_readfirstlane((int)(a.q_off[q + 1] - qa));
    const int nd = __builtin_amdgcn_readfirstlane((int)(a.d_off[doc + 1] - da));
    if ((int64_t)nq * nd > a.slot) {  // the host sizes the slots; never taken
      if (lane == 0) atomicOr(a.status, ERR_SIZE);
      continue;
    }
    const uint32_t* dr = a.d_rank + da;
    const uint32_t* dm = a.d_mass + da;
    const uint32_t* qr = a.q_rank + qa;
    const uint32_t* qm = a.q_mass + qa;
    // the distance matrix [nd][nq] and its largest entry
    float mx = 0.0f;
    for (int ib = 0; ib < nd; ib += 32) {
      const int ni = min(32, nd - ib);
      for (int jb = 0; jb < nq; jb += 32) {
        const int nj = min(32, nq - jb);
        block_d2(L.blk, a.rows, dr, qr, ib, ni, jb, nj);
        const int col = lane & 31;
        for (int r = lane >> 5; r < ni; r += 2) {
          if (col < nj) {
            const float d = sqrtf(L.blk.tile[r][col]);
            S[(int64_t)(ib + r) * nq + jb + col] = d;
            mx = fmaxf(mx, d);
          }
        }
        __syncthreads();
      }
    }
    const float M = wave_max(mx);
    double est = 0.0;
    if (M > 0.0f) {
      // K = exp(-eta D / M) = exp2(c D)
      const float cexp = (float)(-(double)a.eta * 1.4426950408889634 / (double)M);
      const double scale = ldexp(1.0, -a.Q);
      for (int j = lane; j < nq; j += 64) L.v[j] = 1.0f;
      __syncthreads();
      for (int it = 0; it < a.iters; ++it) {
        // rows, SR at a time (their loads and sums interleave): u = a / (K v)
        for (int i0 = 0; i0 < nd; i0 += SR) {
          double acc[SR];
          row_sums<false>(S, nq, nd, i0, cexp, L.v, acc);
          if (lane < SR && i0 + lane < nd) {
            double mine = acc[0];
#pragma unroll
            for (int r = 1; r < SR; ++r)
              if (lane == r) mine = acc[r];
            L.u[i0 + lane] = (float)((double)dm[i0 + lane] * scale / mine);
          }
        }
        __syncthreads();
        // columns, one lane each: v = b / (K^T u)
        for (int j = lane; j < nq; j += 64) {
          double acc = 0.0;
          int i = 0;
          for (; i + 8 <= nd; i += 8) {
            float d[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) d[r] = S[(int64_t)(i + r) * nq + j];
#pragma unroll
            for (int r = 0; r < 8; ++r) acc += (double)(exp2f(cexp * d[r]) * L.u[i + r]);
          }
          for (; i < nd; ++i) acc += (double)(exp2f(cexp * S[(int64_t)i * nq + j]) * L.u[i]);
          L.v[j] = (float)((double)qm[j] * scale / acc);
        }
        __syncthreads();
      }
      // the estimate: sum_i u_i sum_j K_ij v_j D_ij, rows in order
      for (int i0 = 0; i0 < nd; i0 += SR) {
        double acc[SR];
        row_sums<true>(S, nq, nd, i0, cexp, L.v, acc);
#pragma unroll
        for (int r = 0; r < SR; ++r)
          if (i0 + r < nd) est += (double)L.u[i0 + r] * acc[r];
      }
    }
    if (lane == 0) a.cost[p] = (float)est;
    __syncthreads();
  }
}

static SinkArgs sink_args(ft_index* ix, int32_t iters, float eta) {
  SinkArgs a{};
  a.q_rank = ix->qry.rank.as<uint32_t>();
  a.q_mass = ix->qry.mass.as<uint32_t>();
  a.d_off = ix->docs.off.as<int64_t>();
  a.d_rank = ix->docs.rank.as<uint32_t>();
  a.d_mass = ix->docs.mass.as<uint32_t>();
  a.rows = pair_rows(ix);
  a.Q = ix->Q;
  a.iters = iters;
  a.eta = eta;
  a.status = ix->status.as<uint32_t>();
  return a;
}

// Persistent grid: as many workgroups as are resident at once (pairs are
// dealt to them by stride, so none may wait for a slot), fewer when the
// slots would pass 4 GiB.
static void launch_sinkhorn(ft_index* ix, SinkArgs a, hipStream_t s) {
  if (a.n_pairs <= 0) return;
  a.slot = std::max<int64_t>(1, (int64_t)ix->docs.max_size * ix->qry.max_size);
  const int64_t budget = int64_t(1) << 30;  // floats
  int per_cu = 0;
  FT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sinkhorn, 64, 0));
  int64_t grid = std::min<int64_t>((int64_t)ix->n_cu * std::max(1, per_cu), a.n_pairs);
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, budget / a.slot));
  a.scratch = (float*)ix->ws_rerank.ensure((size_t)(grid * a.slot) * sizeof(float));
  k_sinkhorn<<<dim3((unsigned)grid), 64, 0, s>>>(a);
  FT_HIP(hipGetLastError());
}

}  // namespace ft

using namespace ft;

extern "C" ft_status ft_sinkhorn_knn(ft_index* ix, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                                     int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t iters, float eta,
                                     int32_t k, float* out_cost, int64_t* out_doc, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && out_cost && out_doc, FT_EINVAL, "NULL argument");
    FT_REQUIRE(iters >= 1 && iters <= 64, FT_EINVAL, "iters must lie in [1, 64]");
    FT_REQUIRE(eta > 0.0f && std::isfinite(eta), FT_EINVAL, "eta must be positive");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_cols = cand ? (int64_t)n_cand : ix->docs.n;
    FT_REQUIRE(!cand || (n_cand >= 1 && n_cand <= 4096), FT_ERANGE, "n_cand must lie in [1, 4096]");
    FT_REQUIRE(k >= 1 && k <= n_cols, FT_EINVAL, "k must lie in [1, number of candidates]");
    FT_REQUIRE(n_cols <= 4096 || k <= 1024, FT_ERANGE, "k > 1024 needs at most 4096 candidates");
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    if (cand) check_indices(ix, cand, n_q * n_cand, ix->docs.n, s, "cand");
    const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(n_q, (int64_t(1) << 28) / n_cols));
    float* cost = (float*)ix->ws_cost.ensure(rows * n_cols * 4);
    for (int64_t r0 = 0; r0 < n_q; r0 += rows) {
      const int64_t r1 = std::min(n_q, r0 + rows);
      SinkArgs a = sink_args(ix, iters, eta);
      a.q_off = ix->qry.off.as<int64_t>() + r0;
      a.cand = cand ? cand + r0 * n_cols : nullptr;
      a.n_cols = n_cols;
      a.n_pairs = (r1 - r0) * n_cols;
      a.cost = cost;
      if (r0 == 0) FT_HIP(hipEventRecord(ix->ev_t0, s));
      launch_sinkhorn(ix, a, s);
      if (r1 == n_q) FT_HIP(hipEventRecord(ix->ev_t1, s));
      topk_rows(cost, r1 - r0, n_cols, a.cand, k, out_cost + r0 * k, out_doc + r0 * k, s);
    }
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "sinkhorn kernel reported:" + describe_flags(flags));
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ix->ev_t0, ix->ev_t1) == hipSuccess) ix->last_rerank_ms = ms;
  });
}

extern "C" ft_status ft_sinkhorn_pairs(ft_index* ix, const int64_t* q_off, const uint32_t* q_id,
                                       const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                                       const int64_t* pair_d, int64_t n_pairs, int32_t iters, float eta,
                                       float* out_cost, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && pair_q && pair_d && out_cost, FT_EINVAL, "NULL argument");
    FT_REQUIRE(iters >= 1 && iters <= 64, FT_EINVAL, "iters must lie in [1, 64]");
    FT_REQUIRE(eta > 0.0f && std::isfinite(eta), FT_EINVAL, "eta must be positive");
    FT_REQUIRE(n_pairs >= 0, FT_EINVAL, "n_pairs must be >= 0");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    if (n_pairs == 0) return;
    check_indices(ix, pair_q, n_pairs, n_q, s, "pair_q");
    check_indices(ix, pair_d, n_pairs, ix->docs.n, s, "pair_d");
    SinkArgs a = sink_args(ix, iters, eta);
    a.q_off = ix->qry.off.as<int64_t>();
    a.pair_q = pair_q;
    a.pair_d = pair_d;
    a.n_pairs = n_pairs;
    a.cost = out_cost;
    launch_sinkhorn(ix, a, s);
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "sinkhorn kernel reported:" + describe_flags(flags));
  });
}
