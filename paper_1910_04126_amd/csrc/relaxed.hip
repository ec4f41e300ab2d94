// Relaxed WMD (paper Section 1.1) and ACT-i (Section 4.1: R-WMD with
// capacity constraints added over i iterations; i = 0 is R-WMD) for
// (query, candidate) pairs -- the quadratic-time stage that follows Flowtree
// in the paper's pipelines.
//
// Per pair, every support point of one side needs its i + 1 nearest points
// of the other side, in both directions.  The squared distances come 32 x 32
// at a time from the fp64 matrix cores (pairdist.h).  The block's D^2 goes
// through LDS; lanes 0..31 then walk its rows (doc items, whose i+1 nearest
// stay in registers across the row of blocks), lanes 32..63 its columns
// (query items, whose i+1 nearest stay in LDS).  The capacity walk runs with
// integer masses, D = sqrt(D^2) and fp64 products and sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "flow.h"
#include "pairdist.h"
#include "select.h"
#include "wave.h"

namespace ft {

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
  PairRows rows;
  int Q;
  int iters;
  uint32_t* status;
  float* cost;            // knn form: [query * n_cols + column]; pairs form: [pair]
};

// K1: how many nearest points an item keeps (a power of two >= iters + 1).
template <int K1, int QMAX>
struct ActLds {
  BlockLds blk;
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
      block_d2(L.blk, a.rows, dr, qr, ib, ni, jb, nj);
      if (lane < 32) {
        if (me < ni)
          for (int x = 0; x < nj; ++x) keep_nearest<K1>(rv, rix, L.blk.tile[me][x], jb + x);
      } else if (me < nj) {
        const int j = jb + me;
        float cv[K1];
        int cix[K1];
#pragma unroll
        for (int t = 0; t < K1; ++t) {
          cv[t] = L.cd[t][j];
          cix[t] = L.ci[t][j];
        }
        for (int x = 0; x < ni; ++x) keep_nearest<K1>(cv, cix, L.blk.tile[x][me], ib + x);
#pragma unroll
        for (int t = 0; t < K1; ++t) {
          L.cd[t][j] = cv[t];
          L.ci[t][j] = (uint16_t)cix[t];
        }
      }
      __syncthreads();
    }
    const double c = lane < ni ? capacity_walk<K1>(rv, rix, dm[ib + lane], qm, a.iters, nq) : 0.0;
    tot_d += pair_wave_sum(c);
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
    tot_q += pair_wave_sum(c);
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
  a.rows = pair_rows(ix);
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
    if (hipEventElapsedTime(&ms, ix->ev_t0, ix->ev_t1) == hipSuccess) ix->last_rerank_ms = ms;
  });
}

extern "C" ft_status ft_last_rerank_stats(const ft_index* ix, double* ms) {
  return guarded([&] {
    FT_REQUIRE(ix && ms, FT_EINVAL, "NULL argument");
    *ms = ix->last_rerank_ms;
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
