// Exact W1 (paper Section 1, eq. (1): the optimal transport cost under the
// Euclidean metric) for (query, candidate) pairs -- the last stage of the
// paper's pipelines, run on the few candidates the estimates leave.
//
// Per pair, a transportation problem between the doc items (supplies, the
// integer masses) and the query items (demands), solved exactly by
// successive shortest paths with node potentials (the primal-dual method):
// each round runs Dijkstra from every item that still has supply over the
// residual graph (forward edges doc -> query always, backward edges where a
// flow is positive), with costs reduced by the potentials so that every
// residual edge costs >= 0, stops at the first query item with unmet
// demand, pushes the largest amount the path allows, and moves the
// potentials by the distances.  Masses and flows are integers, so every
// round ends at least one supply, demand or backward flow, and the flow at
// the end is optimal for the fp32 distance matrix; the value is summed in
// fp64.
//
// One wavefront per pair, persistent over the pairs with a scratch slot per
// workgroup: the distance matrix (fp32, row per doc item, from the fp64
// matrix-core blocks of pairdist.h) and the flow (u32, row per query item,
// so that the backward edges into a query item are contiguous).  Dijkstra
// keeps its arrays in LDS and runs level by level: each step finds the
// smallest distance among unsettled nodes (a wavefront min), ends if a
// query item with unmet demand is at it (the lowest such index), else
// settles every node at that distance at once and relaxes their edges with
// the lanes across the other side (ties between predecessors: the first in
// the level's order).  After the potentials move, many nodes share a
// distance, so a round takes few steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "pairdist.h"
#include "select.h"
#include "wave.h"

namespace ft {

struct ExactArgs {
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
  float* scratch;         // gridDim.x slots of 2 * `slot` words: distances, then flows
  int64_t slot;
  uint32_t* status;
  float* cost;            // knn form: [query * n_cols + column]; pairs form: [pair]
  const int64_t* order;   // pairs in the order they are taken: largest estimated work first
  unsigned long long* next;  // work counter, zero at launch
};

// The (query, doc) of pair p, in either form.
__device__ __forceinline__ void exact_pair(const ExactArgs& a, int64_t p, int64_t& q, int64_t& doc) {
  if (a.pair_q) {
    q = a.pair_q[p];
    doc = a.pair_d[p];
  } else {
    q = p / a.n_cols;
    const int64_t c = p - q * a.n_cols;
    doc = a.cand ? a.cand[p] : c;
  }
}

// Largest-first order of the pairs, by a bucket of their estimated work
// s_q * s_d * (s_q + s_d) (a round per item at most, each over the s_q * s_d
// edges): 64 buckets by the estimate's highest bit, taken from the highest.
constexpr int EX_BUCKETS = 64;

__global__ void k_exact_zero(unsigned long long* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

__global__ void k_exact_bucket(ExactArgs a, unsigned long long* __restrict__ cnt, uint8_t* __restrict__ bkt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_pairs) return;
  int64_t q, doc;
  exact_pair(a, p, q, doc);
  const uint64_t nq = (uint64_t)(a.q_off[q + 1] - a.q_off[q]), nd = (uint64_t)(a.d_off[doc + 1] - a.d_off[doc]);
  const uint64_t est = nq * nd * (nq + nd) | 1ull;
  const int b = 63 - __clzll((long long)est);
  bkt[p] = (uint8_t)b;
  atomicAdd(&cnt[b], 1ull);
}

// One thread: bucket starts, highest bucket first (cnt becomes the cursor).
__global__ void k_exact_scan(unsigned long long* __restrict__ cnt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long at = 0;
  for (int b = EX_BUCKETS - 1; b >= 0; --b) {
    const unsigned long long c = cnt[b];
    cnt[b] = at;
    at += c;
  }
}

__global__ void k_exact_scatter(int64_t n_pairs, const uint8_t* __restrict__ bkt, unsigned long long* __restrict__ cur,
                                int64_t* __restrict__ order) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  order[atomicAdd(&cur[bkt[p]], 1ull)] = p;
}

constexpr uint16_t EX_NONE = 0xFFFF;

// Per-item arrays for supports of at most NMAX items: 25 KB at 512 (six
// workgroups per CU), 50 KB at FT_MAX_SUPPORT = 1024 (three).
template <int NMAX>
struct ExactLds {
  // the distance blocks are needed only while a pair's distance matrix is
  // built, the Dijkstra distances only after: they share their space
  union {
    BlockLds blk;
    struct {
      double ds[NMAX], dt[NMAX];  // Dijkstra distances (reduced costs)
    } dj;
  } u;
  uint16_t bs[NMAX], bt[NMAX];  // the nodes of one distance level
  double ps[NMAX], pt[NMAX];  // potentials: doc items, query items
  uint32_t es[NMAX], et[NMAX];  // supply / demand not yet moved
  uint16_t prs[NMAX], prt[NMAX];  // predecessor on the other side
  uint8_t vs[NMAX], vt[NMAX];  // settled
  uint32_t delta;  // the round's push, for every lane
};

// Wavefront minima on DPP moves (row shifts of 1, 2, 4, 8, then lane 15 of
// each row to the next and lane 31 to rows 2 and 3): lane 63 ends with the
// minimum, read back as a scalar.  A lane with no source takes the identity.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_min_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t id = __builtin_bit_cast(uint64_t, (double)INFINITY);
  const uint32_t lo = dpp_u32<CTRL, ROWS>((uint32_t)id, (uint32_t)b);
  const uint32_t hi = dpp_u32<CTRL, ROWS>((uint32_t)(id >> 32), (uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double wave_min_f64(double v) {
  v = fmin(v, dpp_min_f64<0x111>(v));
  v = fmin(v, dpp_min_f64<0x112>(v));
  v = fmin(v, dpp_min_f64<0x114>(v));
  v = fmin(v, dpp_min_f64<0x118>(v));
  v = fmin(v, dpp_min_f64<0x142, 0xA>(v));
  v = fmin(v, dpp_min_f64<0x143, 0xC>(v));
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, dpp_u32<0x111>(0xFFFFFFFFu, v));
  v = min(v, dpp_u32<0x112>(0xFFFFFFFFu, v));
  v = min(v, dpp_u32<0x114>(0xFFFFFFFFu, v));
  v = min(v, dpp_u32<0x118>(0xFFFFFFFFu, v));
  v = min(v, dpp_u32<0x142, 0xA>(0xFFFFFFFFu, v));
  v = min(v, dpp_u32<0x143, 0xC>(0xFFFFFFFFu, v));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

template <int NMAX>
__global__ __launch_bounds__(64) void k_exact(ExactArgs a) {
  __shared__ ExactLds<NMAX> L;
  const int lane = threadIdx.x;
  float* S = a.scratch + (int64_t)blockIdx.x * 2 * a.slot;
  uint32_t* F = (uint32_t*)(S + a.slot);
  // pairs are taken from a counter in the largest-first order, so the
  // longest solves start first and the last ones to finish are short
  for (;;) {
    unsigned long long t = 0ull;
    if (lane == 0) t = atomicAdd(a.next, 1ull);
    const int64_t i = (int64_t)(((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(t >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)t));
    if (i >= a.n_pairs) break;
    const int64_t p = a.order[i];
    int64_t q, doc;
    exact_pair(a, p, q, doc);
    const int64_t qa = a.q_off[q], da = a.d_off[doc];
    const int nq = __builtin_amdgcn_readfirstlane((int)(a.q_off[q + 1] - qa));
    const int nd = __builtin_amdgcn_readfirstlane((int)(a.d_off[doc + 1] - da));
    if ((int64_t)nq * nd > a.slot || nq > NMAX || nd > NMAX) {  // the host sizes both; never taken
      if (lane == 0) atomicOr(a.status, ERR_SIZE);
      continue;
    }
    const uint32_t* dr = a.d_rank + da;
    const uint32_t* dm = a.d_mass + da;
    const uint32_t* qr = a.q_rank + qa;
    const uint32_t* qm = a.q_mass + qa;
    // distances D[i][j] (row per doc item), zero flows F[j][i] (row per query item)
    for (int ib = 0; ib < nd; ib += 32) {
      const int ni = min(32, nd - ib);
      for (int jb = 0; jb < nq; jb += 32) {
        const int nj = min(32, nq - jb);
        block_d2(L.u.blk, a.rows, dr, qr, ib, ni, jb, nj);
        const int col = lane & 31;
        for (int r = lane >> 5; r < ni; r += 2)
          if (col < nj) S[(int64_t)(ib + r) * nq + jb + col] = sqrtf(L.u.blk.tile[r][col]);
        __syncthreads();
      }
    }
    for (int64_t e = lane; e < (int64_t)nq * nd; e += 64) F[e] = 0u;
    for (int i = lane; i < nd; i += 64) {
      L.ps[i] = 0.0;
      L.es[i] = dm[i];
    }
    for (int j = lane; j < nq; j += 64) {
      L.pt[j] = 0.0;
      L.et[j] = qm[j];
    }
    __syncthreads();
    uint32_t left = 1u << a.Q;  // mass still to move
    const int64_t max_rounds = 16 * (int64_t)(nd + nq) + 4096;
    bool failed = false;
    for (int64_t round = 0; left > 0; ++round) {
      if (round >= max_rounds) {  // cannot happen for valid masses; flagged, not looped on
        failed = true;
        break;
      }
      // Dijkstra from every doc item with supply left; lmin is this lane's
      // smallest distance among its unsettled nodes
      double lmin = INFINITY;
      for (int i = lane; i < nd; i += 64) {
        L.u.dj.ds[i] = L.es[i] > 0 ? 0.0 : INFINITY;
        L.prs[i] = EX_NONE;
        L.vs[i] = 0;
        lmin = fmin(lmin, L.u.dj.ds[i]);
      }
      for (int j = lane; j < nq; j += 64) {
        L.u.dj.dt[j] = INFINITY;
        L.prt[j] = EX_NONE;
        L.vt[j] = 0;
      }
      __syncthreads();
      int target = -1;
      double dist_t = 0.0;
      // the nodes settled at one distance level (ids, in index order)
      uint16_t* bs = L.bs;
      uint16_t* bt = L.bt;
      const unsigned long long below = (1ull << lane) - 1ull;
      while (true) {
        // the level: the smallest distance of a node not yet settled
        const double bd = wave_min_f64(lmin);
        if (bd == INFINITY) {  // no path to unmet demand: cannot happen for valid masses
          failed = true;
          break;
        }
        // the level's query items, in index order; one with unmet demand
        // ends the search (the lowest index)
        uint32_t tj = 0xFFFFFFFFu;
        int nt = 0;
        for (int j0 = 0; j0 < nq; j0 += 64) {
          const int j = j0 + lane;
          const bool eq = j < nq && !L.vt[j] && L.u.dj.dt[j] == bd;
          if (eq && L.et[j] > 0 && (uint32_t)j < tj) tj = (uint32_t)j;
          const unsigned long long m = __ballot(eq);
          if (eq) bt[nt + __popcll(m & below)] = (uint16_t)j;
          nt += __popcll(m);
        }
        tj = wave_min_u32(tj);
        if (tj != 0xFFFFFFFFu) {
          target = (int)tj;
          dist_t = bd;
          break;
        }
        // the level's doc items, in index order; then settle both sides
        int ns = 0;
        for (int i0 = 0; i0 < nd; i0 += 64) {
          const int i = i0 + lane;
          const bool eq = i < nd && !L.vs[i] && L.u.dj.ds[i] == bd;
          const unsigned long long m = __ballot(eq);
          if (eq) {
            bs[ns + __popcll(m & below)] = (uint16_t)i;
            L.vs[i] = 1;
          }
          ns += __popcll(m);
        }
        __syncthreads();
        for (int b = lane; b < nt; b += 64) L.vt[bt[b]] = 1;
        __syncthreads();
        lmin = INFINITY;
        // forward edges from the level's doc items
        for (int j = lane; j < nq; j += 64) {
          if (L.vt[j]) continue;
          double best = L.u.dj.dt[j];
          int pred = L.prt[j];
          const double pj = L.pt[j];
#pragma unroll 4
          for (int b = 0; b < ns; ++b) {
            const int i = bs[b];
            const double rc = (double)S[(int64_t)i * nq + j] + L.ps[i] - pj;
            const double nd2 = bd + (rc > 0.0 ? rc : 0.0);
            if (nd2 < best) {
              best = nd2;
              pred = i;
            }
          }
          L.u.dj.dt[j] = best;
          L.prt[j] = (uint16_t)pred;
          lmin = fmin(lmin, best);
        }
        // backward edges from the level's query items, where a flow is positive
        for (int i = lane; i < nd; i += 64) {
          if (L.vs[i]) continue;
          double best = L.u.dj.ds[i];
          int pred = L.prs[i];
          const double pi = L.ps[i];
          for (int b = 0; b < nt; ++b) {
            const int j = bt[b];
            if (F[(int64_t)j * nd + i] > 0u) {
              const double rc = -((double)S[(int64_t)i * nq + j] + pi - L.pt[j]);
              const double nd2 = bd + (rc > 0.0 ? rc : 0.0);
              if (nd2 < best) {
                best = nd2;
                pred = j;
              }
            }
          }
          L.u.dj.ds[i] = best;
          L.prs[i] = (uint16_t)pred;
          lmin = fmin(lmin, best);
        }
        __syncthreads();
      }
      if (failed) break;
      // the amount the path allows, then the push (one lane walks the path)
      if (lane == 0) {
        uint32_t delta = min(L.et[target], left);
        int j = target;
        while (true) {
          const int i = L.prt[j];
          const int jb = L.prs[i];
          if (jb == EX_NONE) {
            delta = min(delta, L.es[i]);
            break;
          }
          delta = min(delta, F[(int64_t)jb * nd + i]);
          j = jb;
        }
        j = target;
        while (true) {
          const int i = L.prt[j];
          F[(int64_t)j * nd + i] += delta;
          const int jb = L.prs[i];
          if (jb == EX_NONE) {
            L.es[i] -= delta;
            break;
          }
          F[(int64_t)jb * nd + i] -= delta;
          j = jb;
        }
        L.et[target] -= delta;
        L.delta = delta;
      }
      __syncthreads();
      left -= L.delta;
      // potentials move by the distances, capped at the target's (nodes not
      // settled are at least that far)
      for (int i = lane; i < nd; i += 64) L.ps[i] += fmin(L.u.dj.ds[i], dist_t);
      for (int j = lane; j < nq; j += 64) L.pt[j] += fmin(L.u.dj.dt[j], dist_t);
      __syncthreads();
    }
    // the flow's cost, rows of query items in order
    double acc = 0.0;
    if (!failed) {
      for (int j = 0; j < nq; ++j) {
        double t = 0.0;
        for (int i = lane; i < nd; i += 64) {
          const uint32_t f = F[(int64_t)j * nd + i];
          if (f) t += (double)f * (double)S[(int64_t)i * nq + j];
        }
        acc += pair_wave_sum(t);
      }
    } else if (lane == 0) {
      atomicOr(a.status, ERR_FLOW);
    }
    if (lane == 0) a.cost[p] = failed ? NAN : (float)ldexp(acc, -a.Q);
    __syncthreads();
  }
}

static ExactArgs exact_args(ft_index* ix) {
  ExactArgs a{};
  a.q_rank = ix->qry.rank.as<uint32_t>();
  a.q_mass = ix->qry.mass.as<uint32_t>();
  a.d_off = ix->docs.off.as<int64_t>();
  a.d_rank = ix->docs.rank.as<uint32_t>();
  a.d_mass = ix->docs.mass.as<uint32_t>();
  a.rows = pair_rows(ix);
  a.Q = ix->Q;
  a.status = ix->status.as<uint32_t>();
  return a;
}

// Persistent grid: as many workgroups as are resident at once, fewer when
// the slots (distances and flows) would pass 4 GiB.  Supports of at most 512
// items take the 512-item LDS layout.
static void launch_exact(ft_index* ix, ExactArgs a, hipStream_t s) {
  if (a.n_pairs <= 0) return;
  a.slot = std::max<int64_t>(1, (int64_t)ix->docs.max_size * ix->qry.max_size);
  const int64_t budget = int64_t(1) << 30;  // words
  // the smaller LDS layout when every support fits it
  const bool small = std::max(ix->docs.max_size, ix->qry.max_size) <= 512;
  const void* kern = small ? (const void*)k_exact<512> : (const void*)k_exact<FT_MAX_SUPPORT>;
  int per_cu = 0;
  FT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, 0));
  int64_t grid = std::min<int64_t>((int64_t)ix->n_cu * std::max(1, per_cu), a.n_pairs);
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, budget / (2 * a.slot)));
  a.scratch = (float*)ix->ws_rerank.ensure((size_t)(grid * 2 * a.slot) * sizeof(float));
  // work counter and bucket cursors, then the bucket of each pair and the order
  const int64_t n = a.n_pairs;
  char* w = (char*)ix->ws_misc.ensure(8 * (1 + EX_BUCKETS) + ((n + 15) & ~int64_t(15)) + 8 * n);
  unsigned long long* next = (unsigned long long*)w;
  unsigned long long* cnt = next + 1;
  uint8_t* bkt = (uint8_t*)(cnt + EX_BUCKETS);
  int64_t* order = (int64_t*)(bkt + ((n + 15) & ~int64_t(15)));
  k_exact_zero<<<1, 64, 0, s>>>(next, 1 + EX_BUCKETS);
  k_exact_bucket<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(a, cnt, bkt);
  k_exact_scan<<<1, 1, 0, s>>>(cnt);
  k_exact_scatter<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, bkt, cnt, order);
  a.order = order;
  a.next = next;
  if (small)
    k_exact<512><<<dim3((unsigned)grid), 64, 0, s>>>(a);
  else
    k_exact<FT_MAX_SUPPORT><<<dim3((unsigned)grid), 64, 0, s>>>(a);
  FT_HIP(hipGetLastError());
}

}  // namespace ft

using namespace ft;

extern "C" ft_status ft_exact_knn(ft_index* ix, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                                  int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t k, float* out_cost,
                                  int64_t* out_doc, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && out_cost && out_doc, FT_EINVAL, "NULL argument");
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
      ExactArgs a = exact_args(ix);
      a.q_off = ix->qry.off.as<int64_t>() + r0;
      a.cand = cand ? cand + r0 * n_cols : nullptr;
      a.n_cols = n_cols;
      a.n_pairs = (r1 - r0) * n_cols;
      a.cost = cost;
      if (r0 == 0) FT_HIP(hipEventRecord(ix->ev_t0, s));
      launch_exact(ix, a, s);
      if (r1 == n_q) FT_HIP(hipEventRecord(ix->ev_t1, s));
      topk_rows(cost, r1 - r0, n_cols, a.cand, k, out_cost + r0 * k, out_doc + r0 * k, s);
    }
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "exact kernel reported:" + describe_flags(flags));
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ix->ev_t0, ix->ev_t1) == hipSuccess) ix->last_rerank_ms = ms;
  });
}

extern "C" ft_status ft_exact_pairs(ft_index* ix, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                                    int64_t n_q, const int64_t* pair_q, const int64_t* pair_d, int64_t n_pairs,
                                    float* out_cost, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && pair_q && pair_d && out_cost, FT_EINVAL, "NULL argument");
    FT_REQUIRE(n_pairs >= 0, FT_EINVAL, "n_pairs must be >= 0");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    if (n_pairs == 0) return;
    check_indices(ix, pair_q, n_pairs, n_q, s, "pair_q");
    check_indices(ix, pair_d, n_pairs, ix->docs.n, s, "pair_d");
    ExactArgs a = exact_args(ix);
    a.q_off = ix->qry.off.as<int64_t>();
    a.pair_q = pair_q;
    a.pair_d = pair_d;
    a.n_pairs = n_pairs;
    a.cost = out_cost;
    launch_exact(ix, a, s);
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "exact kernel reported:" + describe_flags(flags));
  });
}
