// Flowtree k-NN (paper Section 3; greedy of Appendix A.1): plain launches
// (one per query) and the batched persistent schedule (all pairs, one launch
// per pair-size class, replayed as HIP graphs, schedule picked by timing).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <mutex>
#include <sstream>
#include <type_traits>
#include <vector>

#include "common.h"
#include "flow.h"
#include "select.h"
#include "wave.h"

namespace ft {

struct PairArgs {
  const int64_t* q_off;
  const uint32_t* q_rank;
  const uint32_t* q_mass;
  const int64_t* d_off;
  const uint32_t* d_rank;
  const uint32_t* d_mass;
  const int64_t* cand;  // [n_q * n_cols] or NULL (column = doc)
  int64_t n_cols;
  const uint8_t* st;
  int64_t V;
  int B, Q;
  const float* X;  // Morton-ordered, padded rows
  int stride;
  uint32_t* status;
  float* cost;  // [n_q * n_cols]
};

template <int C, int W, int G>
__device__ __forceinline__ void flow_one(FlowLds<C, W>& L, const PairArgs& a, const int64_t p) {
  const int64_t q = p / a.n_cols;
  const int64_t c = p - q * a.n_cols;
  const int64_t doc = a.cand ? a.cand[p] : c;
  const int64_t qa = a.q_off[q], da = a.d_off[doc];
  const int nq = (int)(a.q_off[q + 1] - qa), nd = (int)(a.d_off[doc + 1] - da);
  if (nq + nd > FlowLds<C, W>::N) {  // the host sizes the class; never taken
    if (threadIdx.x == 0) atomicOr(a.status, ERR_FLOW);
    return;
  }
  flow_stage(L, a.q_rank + qa, a.q_mass + qa, nq, a.d_rank + da, a.d_mass + da, nd);
  const int E = flow_match<C, W, false>(L, nq, nd, a.st, a.V, a.B, FlowSave{}, a.status);
  const double cost = flow_price_tiled<C, W, G>(L, E, nq, nd, a.X, a.stride, a.status);
  if (threadIdx.x == 0) a.cost[p] = (float)ldexp(cost, -a.Q);
  __syncthreads();
}

// Persistent workgroups with 4 items per lane are latency-bound on their row
// reads and LDS round trips: they are held to 96 VGPRs, five wavefronts per
// SIMD (for W >= 2 the most their LDS allows).  The few values that spill
// cost less than the extra wavefront gains (at 128 VGPRs and four wavefronts
// per SIMD the batched kernels took 4 % longer and the image-grid ones 13 %;
// the one-wavefront (4,1) class gained 2 % on the batched workload when held
// to five).  With one lane per match (rows of at most 4 floats) the pricing
// needs few registers, and six wavefronts at 80 VGPRs ran the image grid 2 %
// faster (the batched workload, 16 and 8 lanes per match, 30 % slower).
template <int C, int W, int G>
constexpr int flow_min_waves() { return C == 4 ? (G == 1 ? 6 : 5) : 1; }

// Plain: workgroup b handles column b of query q.
template <int C, int W, int G>
__global__ __launch_bounds__(64 * W) void k_flow_plain(PairArgs a, int64_t q) {
  __shared__ FlowLds<C, W> L;
  flow_one<C, W, G>(L, a, q * a.n_cols + blockIdx.x);
}

// Persistent: workgroups grab chunks of the class's pair list until it is
// used up.
template <int C, int W, int G>
__device__ __forceinline__ void persistent_body(FlowLds<C, W>& L, const PairArgs& a, const int64_t* __restrict__ list,
                                                const int64_t* __restrict__ offsets, int64_t n_q, int cls,
                                                uint32_t* __restrict__ counters, int chunk) {
  const int64_t begin = offsets[(int64_t)cls * n_q], end = offsets[(int64_t)(cls + 1) * n_q];
  while (true) {
    if (threadIdx.x == 0) L.work = (int64_t)atomicAdd(&counters[cls], 1u);
    __syncthreads();
    const int64_t i0 = begin + L.work * chunk;
    __syncthreads();  // everyone has read the grab before thread 0 makes the next
    if (i0 >= end) break;
    const int64_t i1 = min(end, i0 + chunk);
    for (int64_t i = i0; i < i1; ++i) flow_one<C, W, G>(L, a, list[i]);
  }
}

template <int C, int W, int G>
__global__ __launch_bounds__(64 * W, (flow_min_waves<C, W, G>())) void k_flow_persistent(PairArgs a, const int64_t* __restrict__ list,
                                                            const int64_t* __restrict__ offsets, int64_t n_q, int cls,
                                                            uint32_t* __restrict__ counters, int chunk) {
  __shared__ FlowLds<C, W> L;
  persistent_body<C, W, G>(L, a, list, offsets, n_q, cls, counters, chunk);
}

// The smallest class (one wavefront, 2 items per lane) fits seven
// wavefronts per SIMD by its vector registers; its scalar registers are held
// to 72 so that they do not cap it lower.
template <int G>
__global__ __launch_bounds__(64) __attribute__((amdgpu_num_sgpr(72))) void k_flow_persistent_small(
    PairArgs a, const int64_t* __restrict__ list, const int64_t* __restrict__ offsets, int64_t n_q, int cls,
    uint32_t* __restrict__ counters, int chunk) {
  __shared__ FlowLds<2, 1> L;
  persistent_body<2, 1, G>(L, a, list, offsets, n_q, cls, counters, chunk);
}

// All pairs of one size class out of a flat list of n_pairs (query p /
// n_cols, doc cand[p]): workgroups stride over the list and skip the pairs
// of other classes (the no-allocation path has no room for class lists).
template <int C, int W, int G>
__global__ __launch_bounds__(64 * W, (flow_min_waves<C, W, G>())) void k_flow_class_stride(PairArgs a, int64_t n_pairs,
                                                                                    int cls) {
  __shared__ FlowLds<C, W> L;
  for (int64_t p = blockIdx.x; p < n_pairs; p += gridDim.x) {
    const int64_t q = p / a.n_cols;
    const int64_t doc = a.cand[p];
    const int n = (int)(a.q_off[q + 1] - a.q_off[q]) + (int)(a.d_off[doc + 1] - a.d_off[doc]);
    if (class_for_dev(n) == cls) flow_one<C, W, G>(L, a, p);
  }
}

// status[0] |= ERR_ID_RANGE unless every v[i] lies in [0, bound).
__global__ void k_check_range(const int64_t* __restrict__ v, int64_t n, int64_t bound, uint32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (v[i] < 0 || v[i] >= bound)) atomicOr(status, ERR_ID_RANGE);
}

__global__ void k_fill_u32(uint32_t* p, int n, uint32_t v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per query: the largest support among its candidates (the plain
// schedule's workgroup shape).
__global__ __launch_bounds__(256) void k_cand_max_size(PairArgs a, int32_t* __restrict__ out) {
  __shared__ int32_t wmax[4];
  const int64_t q = blockIdx.x;
  int m = 0;
  for (int64_t c = threadIdx.x; c < a.n_cols; c += blockDim.x) {
    const int64_t doc = a.cand ? a.cand[q * a.n_cols + c] : c;
    m = max(m, (int)(a.d_off[doc + 1] - a.d_off[doc]));
  }
  m = wave_max(m);
  if (lane_id() == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[q] = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
}

// Per query: count candidate pairs of each size class.
__global__ __launch_bounds__(256) void k_bucket_count(PairArgs a, int64_t n_q, int64_t* __restrict__ counts) {
  __shared__ int64_t cnt[N_CLASSES];
  const int64_t q = blockIdx.x;
  if (threadIdx.x < N_CLASSES) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int nq = (int)(a.q_off[q + 1] - a.q_off[q]);
  for (int64_t c = threadIdx.x; c < a.n_cols; c += blockDim.x) {
    const int64_t doc = a.cand ? a.cand[q * a.n_cols + c] : c;
    const int n = nq + (int)(a.d_off[doc + 1] - a.d_off[doc]);
    atomicAdd((unsigned long long*)&cnt[class_for_dev(n)], 1ull);
  }
  __syncthreads();
  if (threadIdx.x < N_CLASSES) counts[(int64_t)threadIdx.x * n_q + q] = cnt[threadIdx.x];
}

// Per query (one wavefront): place its pairs into the class lists, in
// column order.
__global__ __launch_bounds__(64) void k_bucket_scatter(PairArgs a, int64_t n_q, const int64_t* __restrict__ offsets,
                                                       int64_t* __restrict__ list) {
  const int64_t q = blockIdx.x;
  const int lane = lane_id();
  const int nq = (int)(a.q_off[q + 1] - a.q_off[q]);
  const int64_t per = (a.n_cols + 63) / 64;
  const int64_t c0 = min(a.n_cols, lane * per), c1 = min(a.n_cols, c0 + per);
  int64_t local[N_CLASSES] = {0, 0, 0, 0, 0};
  for (int64_t c = c0; c < c1; ++c) {
    const int64_t doc = a.cand ? a.cand[q * a.n_cols + c] : c;
    ++local[class_for_dev(nq + (int)(a.d_off[doc + 1] - a.d_off[doc]))];
  }
  int64_t pos[N_CLASSES];
#pragma unroll
  for (int k = 0; k < N_CLASSES; ++k) pos[k] = offsets[(int64_t)k * n_q + q] + wave_incl_sum(local[k]) - local[k];
  for (int64_t c = c0; c < c1; ++c) {
    const int64_t doc = a.cand ? a.cand[q * a.n_cols + c] : c;
    const int k = class_for_dev(nq + (int)(a.d_off[doc + 1] - a.d_off[doc]));
    list[pos[k]++] = q * a.n_cols + c;
  }
}

// ------------------------------------------------------------ dispatch --

// Calls f(integral_constant C, integral_constant W) for a size class.
template <class F>
static void with_class(int cls, F&& f) {
  switch (cls) {
    case 0: f(std::integral_constant<int, CLASS_C[0]>{}, std::integral_constant<int, CLASS_W[0]>{}); break;
    case 1: f(std::integral_constant<int, CLASS_C[1]>{}, std::integral_constant<int, CLASS_W[1]>{}); break;
    case 2: f(std::integral_constant<int, CLASS_C[2]>{}, std::integral_constant<int, CLASS_W[2]>{}); break;
    case 3: f(std::integral_constant<int, CLASS_C[3]>{}, std::integral_constant<int, CLASS_W[3]>{}); break;
    default: f(std::integral_constant<int, CLASS_C[4]>{}, std::integral_constant<int, CLASS_W[4]>{}); break;
  }
}

// Calls f(integral_constant G) for the lanes per match.
template <class F>
static void with_lanes(int G, F&& f) {
  switch (G) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: f(std::integral_constant<int, 16>{}); break;
  }
}

static void launch_plain(int cls, int G, const PairArgs& a, int64_t q, hipStream_t s) {
  with_class(cls, [&](auto cc, auto ww) {
    with_lanes(G, [&](auto gg) {
      constexpr int C = decltype(cc)::value, W = decltype(ww)::value, GG = decltype(gg)::value;
      k_flow_plain<C, W, GG><<<(unsigned)a.n_cols, 64 * W, 0, s>>>(a, q);
    });
  });
}

static const void* persistent_kernel(int cls, int G) {
  const void* fn = nullptr;
  with_class(cls, [&](auto cc, auto ww) {
    with_lanes(G, [&](auto gg) {
      constexpr int C = decltype(cc)::value, W = decltype(ww)::value, GG = decltype(gg)::value;
      if constexpr (C == 2 && W == 1) fn = reinterpret_cast<const void*>(&k_flow_persistent_small<GG>);
      else fn = reinterpret_cast<const void*>(&k_flow_persistent<C, W, GG>);
    });
  });
  return fn;
}

static void launch_persistent(int cls, int G, unsigned blocks, const PairArgs& a, const int64_t* list,
                              const int64_t* offsets, int64_t n_q, uint32_t* counters, int chunk, hipStream_t s) {
  with_class(cls, [&](auto cc, auto ww) {
    with_lanes(G, [&](auto gg) {
      constexpr int C = decltype(cc)::value, W = decltype(ww)::value, GG = decltype(gg)::value;
      if constexpr (C == 2 && W == 1)
        k_flow_persistent_small<GG><<<blocks, 64, 0, s>>>(a, list, offsets, n_q, cls, counters, chunk);
      else
        k_flow_persistent<C, W, GG><<<blocks, 64 * W, 0, s>>>(a, list, offsets, n_q, cls, counters, chunk);
    });
  });
}

// ------------------------------------------------------------- batched --

struct BatchedPlan {
  int G = 16;
  int64_t n_q = 0, n_cols = 0;
  int64_t* counts = nullptr;   // [N_CLASSES * n_q]
  int64_t* offsets = nullptr;  // [N_CLASSES * n_q + 1]
  int64_t* scan_tmp = nullptr;
  int64_t* list = nullptr;     // [n_q * n_cols]
  uint32_t* counters = nullptr;
  unsigned blocks[N_CLASSES] = {0, 0, 0, 0, 0};
  int chunk = 4;
};

static void enqueue_bucketing(const PairArgs& a, const BatchedPlan& P, hipStream_t s) {
  k_fill_u32<<<1, 64, 0, s>>>(P.counters, N_CLASSES, 0u);
  k_bucket_count<<<(unsigned)P.n_q, 256, 0, s>>>(a, P.n_q, P.counts);
  exclusive_scan_i64(P.counts, P.offsets, (int64_t)N_CLASSES * P.n_q, P.scan_tmp, s);
  k_bucket_scatter<<<(unsigned)P.n_q, 64, 0, s>>>(a, P.n_q, P.offsets, P.list);
  FT_HIP(hipGetLastError());
}

static void enqueue_persistent(const PairArgs& a, const BatchedPlan& P, hipStream_t s) {
  for (int cls = 0; cls < N_CLASSES; ++cls)
    if (P.blocks[cls]) launch_persistent(cls, P.G, P.blocks[cls], a, P.list, P.offsets, P.n_q, P.counters, P.chunk, s);
  FT_HIP(hipGetLastError());
}

static unsigned occupancy_blocks(ft_index* ix, int cls, int G) {
  int per_cu = 0;
  FT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel(cls, G), 64 * CLASS_W[cls], 0));
  per_cu = std::max(1, per_cu);
  return (unsigned)(per_cu * ix->n_cu);
}

static hipGraphExec_t capture(ft_index* ix, const std::function<void(hipStream_t)>& body) {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  FT_HIP(hipStreamBeginCapture(ix->work, hipStreamCaptureModeThreadLocal));
  try {
    body(ix->work);
  } catch (...) {
    (void)hipStreamEndCapture(ix->work, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  FT_HIP(hipStreamEndCapture(ix->work, &g));
  hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  FT_HIP(err);
  return e;
}

static std::string tune_signature(const ft_index* ix, int64_t n_q, int64_t n_cols, bool all_docs) {
  std::ostringstream o;
  o << "gfx950/V" << ix->V << "/d" << ix->d << "/docs" << ix->docs.n << "/maxd" << ix->docs.max_size << "/nq" << n_q
    << "/cols" << n_cols << (all_docs ? "/all" : "/cand");
  return o.str();
}

static void load_tune_cache(ft_index* ix) {
  const char* path = getenv("FT_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    // one entry per line: "signature chunk occupancy_percent"
    std::istringstream ls(line);
    std::string sig;
    TuneChoice c;
    if (ls >> sig >> c.chunk >> c.blocks_per_cu) ix->tuned[sig] = c;
  }
}

static void save_tune_cache(const ft_index* ix) {
  const char* path = getenv("FT_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path);
  for (auto& kv : ix->tuned) f << kv.first << " " << kv.second.chunk << " " << kv.second.blocks_per_cu << "\n";
}

static void set_blocks(ft_index* ix, BatchedPlan& P, int occupancy_percent) {
  for (int cls = 0; cls < N_CLASSES; ++cls) {
    unsigned full = occupancy_blocks(ix, cls, P.G);
    P.blocks[cls] = std::max(1u, (unsigned)((uint64_t)full * occupancy_percent / 100));
  }
}

}  // namespace ft

using namespace ft;

// Plain schedule: one launch per query, its workgroup shape sized by the
// query's largest pair (the query's support plus its largest candidate,
// found on the device first).
static void flowtree_plain(ft_index* ix, const PairArgs& a, int64_t n_q, hipStream_t s) {
  std::vector<int64_t> qoff(n_q + 1);
  std::vector<int32_t> dmax(n_q);
  int32_t* dev_max = (int32_t*)ix->ws_misc.ensure(n_q * sizeof(int32_t));
  k_cand_max_size<<<(unsigned)n_q, 256, 0, s>>>(a, dev_max);
  FT_HIP(hipGetLastError());
  FT_HIP(hipMemcpyAsync(qoff.data(), a.q_off, (n_q + 1) * 8, hipMemcpyDeviceToHost, s));
  FT_HIP(hipMemcpyAsync(dmax.data(), dev_max, n_q * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
  const int G = knn_lanes(ix->dp);
  for (int64_t q = 0; q < n_q; ++q) {
    const int cls = class_for((int)(qoff[q + 1] - qoff[q]) + dmax[q]);
    FT_REQUIRE(cls >= 0, FT_ERANGE, "pair larger than 2048 items");
    launch_plain(cls, G, a, q, s);
  }
  FT_HIP(hipGetLastError());
}

static void flowtree_batched(ft_index* ix, const PairArgs& a, int64_t n_q, hipStream_t s) {
  const int64_t n_cols = a.n_cols;
  const int64_t npairs = n_q * n_cols;
  BatchedPlan P;
  P.G = knn_lanes(ix->dp);
  P.n_q = n_q;
  P.n_cols = n_cols;
  const int64_t nc = (int64_t)N_CLASSES * n_q;
  int64_t* misc = (int64_t*)ix->ws_counts.ensure((nc + nc + 1 + scan_tmp_elems(nc) + 8) * 8);
  P.counts = misc;
  P.offsets = misc + nc;
  P.scan_tmp = misc + 2 * nc + 1;
  P.counters = (uint32_t*)(misc + 2 * nc + 1 + scan_tmp_elems(nc));
  P.list = (int64_t*)ix->ws_lists.ensure(npairs * 8);

  // schedule: tuned on first use of a shape
  if (ix->tuned.empty()) load_tune_cache(ix);
  const std::string sig = tune_signature(ix, n_q, n_cols, a.cand == nullptr);
  auto it = ix->tuned.find(sig);
  TuneChoice choice;
  if (it != ix->tuned.end()) {
    choice = it->second;
  } else if (ix->autotune > 0) {
    // time the persistent launches for each candidate schedule
    enqueue_bucketing(a, P, s);
    float best = 1e30f;
    for (int occ : {100, 50}) {
      for (int chunk : {1, 2, 4, 8, 16}) {
        P.chunk = chunk;
        set_blocks(ix, P, occ);
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {
          k_fill_u32<<<1, 64, 0, s>>>(P.counters, N_CLASSES, 0u);
          FT_HIP(hipEventRecord(ix->ev_t0, s));
          enqueue_persistent(a, P, s);
          FT_HIP(hipEventRecord(ix->ev_t1, s));
          FT_HIP(hipEventSynchronize(ix->ev_t1));
          FT_HIP(hipEventElapsedTime(&ms, ix->ev_t0, ix->ev_t1));
        }
        if (ms < best) {
          best = ms;
          choice.chunk = chunk;
          choice.blocks_per_cu = occ;
        }
      }
    }
    ix->tuned[sig] = choice;
    save_tune_cache(ix);
  } else {
    choice.chunk = 4;
    choice.blocks_per_cu = 100;
  }
  P.chunk = choice.chunk;
  set_blocks(ix, P, choice.blocks_per_cu > 0 ? choice.blocks_per_cu : 100);
  {
    std::ostringstream o;
    o << "chunk=" << P.chunk << " occupancy=" << (choice.blocks_per_cu > 0 ? choice.blocks_per_cu : 100)
      << "% blocks=";
    for (int cls = 0; cls < N_CLASSES; ++cls) o << (cls ? "," : "") << P.blocks[cls];
    o << " lanes_per_match=" << P.G;
    ix->last_schedule = o.str();
  }

  // two graphs, bucketing and the persistent Flowtree launches; events
  // between them time the persistent launches
  BatchedGraphs& BG = ix->graphs;
  std::vector<uint64_t> key = {(uint64_t)a.q_off,   (uint64_t)a.q_rank,  (uint64_t)a.q_mass, (uint64_t)a.cand,
                               (uint64_t)n_cols,    (uint64_t)n_q,       (uint64_t)a.cost,   (uint64_t)P.list,
                               (uint64_t)P.counts,  (uint64_t)P.chunk,   (uint64_t)P.blocks[0], (uint64_t)P.blocks[4],
                               (uint64_t)a.status};
  if (BG.key != key) {
    BG.reset();
    BG.pre = capture(ix, [&](hipStream_t w) { enqueue_bucketing(a, P, w); });
    BG.main = capture(ix, [&](hipStream_t w) { enqueue_persistent(a, P, w); });
    BG.key = key;
  }
  FT_HIP(hipEventRecord(ix->ev_a, s));
  FT_HIP(hipStreamWaitEvent(ix->work, ix->ev_a, 0));
  FT_HIP(hipGraphLaunch(BG.pre, ix->work));
  FT_HIP(hipEventRecord(ix->ev_t0, ix->work));
  FT_HIP(hipGraphLaunch(BG.main, ix->work));
  FT_HIP(hipEventRecord(ix->ev_t1, ix->work));
  FT_HIP(hipEventRecord(ix->ev_b, ix->work));
  FT_HIP(hipStreamWaitEvent(s, ix->ev_b, 0));
}

// ft_flowtree_knn after its argument checks, on the prepared queries
// (ix->qry) and checked candidate lists; the caller reads the status.
void ft::flowtree_knn_prepared(ft_index* ix, int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t k, int32_t mode,
                           float* out_cost, int64_t* out_doc, hipStream_t s) {
  const int64_t n_cols = cand ? (int64_t)n_cand : ix->docs.n;
  FT_REQUIRE(class_for(ix->qry.max_size + ix->docs.max_size) >= 0, FT_ERANGE, "pair larger than 2048 items");
  // queries in chunks so the cost buffer stays near 1 GiB
  const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(n_q, (int64_t(1) << 28) / n_cols));
  float* cost = (float*)ix->ws_cost.ensure(rows * n_cols * 4);
  for (int64_t r0 = 0; r0 < n_q; r0 += rows) {
    const int64_t r1 = std::min(n_q, r0 + rows);
    PairArgs a;
    a.q_off = ix->qry.off.as<int64_t>() + r0;
    a.q_rank = ix->qry.rank.as<uint32_t>();
    a.q_mass = ix->qry.mass.as<uint32_t>();
    a.d_off = ix->docs.off.as<int64_t>();
    a.d_rank = ix->docs.rank.as<uint32_t>();
    a.d_mass = ix->docs.mass.as<uint32_t>();
    a.cand = cand ? cand + r0 * n_cols : nullptr;
    a.n_cols = n_cols;
    a.st = ix->st.as<uint8_t>();
    a.V = ix->V;
    a.B = ix->B;
    a.Q = ix->Q;
    a.X = ix->Xm.as<float>();
    a.stride = ix->dp;
    a.status = ix->status.as<uint32_t>();
    a.cost = cost;
    if (mode == FT_PLAIN) flowtree_plain(ix, a, r1 - r0, s);
    else flowtree_batched(ix, a, r1 - r0, s);
    topk_rows(cost, r1 - r0, n_cols, a.cand, k, out_cost + r0 * k, out_doc + r0 * k, s);
  }
}

extern "C" ft_status ft_flowtree_knn(ft_index* ix, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                                     int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t k, int32_t mode,
                                     float* out_cost, int64_t* out_doc, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && out_cost && out_doc, FT_EINVAL, "NULL argument");
    FT_REQUIRE(mode == FT_PLAIN || mode == FT_BATCHED, FT_EINVAL, "mode must be FT_PLAIN or FT_BATCHED");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_cols = cand ? (int64_t)n_cand : ix->docs.n;
    FT_REQUIRE(!cand || (n_cand >= 1 && n_cand <= 4096), FT_ERANGE, "n_cand must lie in [1, 4096]");
    FT_REQUIRE(k >= 1 && k <= n_cols, FT_EINVAL, "k must lie in [1, number of candidates]");
    FT_REQUIRE(cand || n_cols <= 4096 || k <= 1024, FT_ERANGE, "k > 1024 needs at most 4096 candidates");
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    if (cand) check_indices(ix, cand, n_q * n_cand, ix->docs.n, s, "cand");
    flowtree_knn_prepared(ix, n_q, cand, n_cand, k, mode, out_cost, out_doc, s);
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "flowtree kernel reported:" + describe_flags(flags));
    if (mode == FT_BATCHED) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ix->ev_t0, ix->ev_t1) == hipSuccess) ix->last_batched_ms = ms;
    }
  });
}

extern "C" ft_status ft_knn_pipeline(ft_index* ix, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                                     int64_t n_q, int32_t prune_k, int32_t k, float* out_cost, int64_t* out_doc,
                                     void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && out_cost && out_doc, FT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_docs = ix->docs.n;
    FT_REQUIRE(prune_k >= 1 && prune_k <= n_docs, FT_EINVAL, "prune_k must lie in [1, number of docs]");
    FT_REQUIRE(prune_k <= 4096, FT_ERANGE, "prune_k must be at most 4096");
    FT_REQUIRE(n_docs <= 4096 || prune_k <= 1024, FT_ERANGE, "prune_k > 1024 needs at most 4096 docs");
    FT_REQUIRE(k >= 1 && k <= prune_k, FT_EINVAL, "k must lie in [1, prune_k]");
    // the queries are prepared once (validated, sorted, embedded) for both stages
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, true, s, "queries");
    uint64_t* keys = (uint64_t*)ix->ws_pipe.ensure(n_q * prune_k * 16);
    int64_t* cand = reinterpret_cast<int64_t*>(keys + n_q * prune_k);
    FT_HIP(hipEventRecord(ix->ev_p[0], s));
    quadtree_knn_prepared(ix, n_q, nullptr, 0, prune_k, keys, cand, s);
    FT_HIP(hipEventRecord(ix->ev_p[1], s));
    // the candidate docs come from the select over the docs' own range: no check
    flowtree_knn_prepared(ix, n_q, cand, prune_k, k, FT_BATCHED, out_cost, out_doc, s);
    FT_HIP(hipEventRecord(ix->ev_p[2], s));
    // the one read of the validation and kernel flags of the whole pipeline
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "pipeline kernel reported:" + describe_flags(flags));
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ix->ev_p[0], ix->ev_p[1]) == hipSuccess) ix->last_pipe_ms[0] = ms;
    if (hipEventElapsedTime(&ms, ix->ev_p[1], ix->ev_p[2]) == hipSuccess) ix->last_pipe_ms[1] = ms;
    if (hipEventElapsedTime(&ms, ix->ev_t0, ix->ev_t1) == hipSuccess) ix->last_batched_ms = ms;
  });
}

extern "C" ft_status ft_last_pipeline_stats(const ft_index* ix, double* prune_ms, double* rerank_ms) {
  return guarded([&] {
    FT_REQUIRE(ix, FT_EINVAL, "NULL index");
    if (prune_ms) *prune_ms = ix->last_pipe_ms[0];
    if (rerank_ms) *rerank_ms = ix->last_pipe_ms[1];
  });
}

extern "C" ft_status ft_set_autotune(ft_index* ix, int32_t level) {
  return guarded([&] {
    FT_REQUIRE(ix, FT_EINVAL, "NULL index");
    FT_REQUIRE(level == 0 || level == 1, FT_EINVAL, "level must be 0 or 1");
    ix->autotune = level;
  });
}

extern "C" ft_status ft_last_batched_stats(const ft_index* ix, double* ms, char* schedule, int32_t len) {
  return guarded([&] {
    FT_REQUIRE(ix, FT_EINVAL, "NULL index");
    if (ms) *ms = ix->last_batched_ms;
    if (schedule && len > 0) {
      std::snprintf(schedule, (size_t)len, "%s", ix->last_schedule.c_str());
    }
  });
}


// ---------------------------------------------------- no allocation --
//
// ft_flowtree_knn_noalloc keeps everything beyond its inputs and outputs in
// `scratch`, one array per GPU (each device holds its own copy at its own
// address).  In host code `scratch` only names the symbol: its device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is handed to kernels and copies.

namespace {

constexpr int64_t na_align(int64_t x) { return (x + 255) & ~int64_t(255); }

constexpr int64_t NA_STATUS = 0;                                                      // u32 [64]
constexpr int64_t NA_OFF = na_align(NA_STATUS + 64 * 4);                              // int64 [MAX_Q + 1]
constexpr int64_t NA_RANK = na_align(NA_OFF + (FT_NOALLOC_MAX_QUERIES + 1) * 8);      // u32 [MAX_ITEMS]
constexpr int64_t NA_MASS = na_align(NA_RANK + (int64_t)FT_NOALLOC_MAX_ITEMS * 4);    // u32 [MAX_ITEMS]
constexpr int64_t NA_POS = na_align(NA_MASS + (int64_t)FT_NOALLOC_MAX_ITEMS * 4);     // u16 [MAX_ITEMS]
constexpr int64_t NA_LCP = na_align(NA_POS + (int64_t)FT_NOALLOC_MAX_ITEMS * 2);      // u8  [MAX_ITEMS]
constexpr int64_t NA_CNT = na_align(NA_LCP + (int64_t)FT_NOALLOC_MAX_ITEMS);          // int64 [MAX_Q]
constexpr int64_t NA_COST = na_align(NA_CNT + (int64_t)FT_NOALLOC_MAX_QUERIES * 8);   // f32 [MAX_PAIRS]
constexpr int64_t NA_BYTES = na_align(NA_COST + (int64_t)FT_NOALLOC_MAX_PAIRS * 4);

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_na_mu;
void* g_na_ptr[NA_MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

void* ft::noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_na_mu);
  FT_REQUIRE(device >= 0 && device < NA_MAX_DEVICES, FT_EINVAL, "device ordinal out of range");
  if (!g_na_ptr[device]) {
    int cur = -1;
    FT_HIP(hipGetDevice(&cur));
    FT_REQUIRE(cur == device, FT_EINVAL, "the index's device must be current");
    void* p = nullptr;
    FT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    FT_REQUIRE(p != nullptr, FT_EHIP, "no device address for the scratch array");
    g_na_ptr[device] = p;
  }
  return g_na_ptr[device];
}

// Copies the status words of the scratch array to the host (synchronises s).
static void na_read_status(const uint32_t* status, uint32_t* h, hipStream_t s) {
  FT_HIP(hipMemcpyAsync(h, status, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
}

extern "C" ft_status ft_flowtree_knn_noalloc(ft_index* ix, const int64_t* q_off, const uint32_t* q_id,
                                             const uint32_t* q_mass, int64_t n_q, const int64_t* cand, int32_t n_cand,
                                             int32_t k, float* out_cost, int64_t* out_doc, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && q_off && q_id && q_mass && cand && out_cost && out_doc, FT_EINVAL, "NULL argument");
    FT_REQUIRE(n_q >= 1, FT_EINVAL, "queries: need at least one distribution");
    FT_REQUIRE(n_cand >= 1 && n_cand <= 4096, FT_ERANGE, "n_cand must lie in [1, 4096]");
    FT_REQUIRE(k >= 1 && k <= n_cand, FT_EINVAL, "k must lie in [1, number of candidates]");
    FT_REQUIRE(n_q <= FT_NOALLOC_MAX_QUERIES, FT_ERANGE, "n_q exceeds FT_NOALLOC_MAX_QUERIES");
    FT_REQUIRE(n_q * (int64_t)n_cand <= FT_NOALLOC_MAX_PAIRS, FT_ERANGE,
               "n_q * n_cand exceeds FT_NOALLOC_MAX_PAIRS");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    char* base = static_cast<char*>(noalloc_scratch(ix->device));
    uint32_t* status = reinterpret_cast<uint32_t*>(base + NA_STATUS);
    int64_t* off = reinterpret_cast<int64_t*>(base + NA_OFF);
    uint32_t* rank = reinterpret_cast<uint32_t*>(base + NA_RANK);
    uint32_t* mass = reinterpret_cast<uint32_t*>(base + NA_MASS);
    uint16_t* pos = reinterpret_cast<uint16_t*>(base + NA_POS);
    uint8_t* lcp = reinterpret_cast<uint8_t*>(base + NA_LCP);
    int64_t* cnt = reinterpret_cast<int64_t*>(base + NA_CNT);
    float* cost = reinterpret_cast<float*>(base + NA_COST);
    uint32_t h[8];

    // the previous call left its status words behind: clear them
    k_fill_u32<<<1, 64, 0, s>>>(status, 64, 0u);
    FT_HIP(hipGetLastError());
    // query offsets: validated, and the total support bounded before any
    // item is written
    FT_HIP(hipMemcpyAsync(off, q_off, (n_q + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    launch_check_offsets(off, n_q, status, s);
    int64_t nnz = 0;
    FT_HIP(hipMemcpyAsync(&nnz, off + n_q, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    na_read_status(status, h, s);
    if (h[0] & ERR_SIZE) throw Error(FT_ERANGE, "queries: support larger than FT_MAX_SUPPORT");
    if (h[0]) throw Error(FT_EINVAL, "queries:" + describe_flags(h[0]));
    FT_REQUIRE(nnz <= FT_NOALLOC_MAX_ITEMS, FT_ERANGE, "total query support exceeds FT_NOALLOC_MAX_ITEMS");
    const int max_q = (int)h[1];
    const int top_cls = class_for(max_q + ix->docs.max_size);
    FT_REQUIRE(top_cls >= 0, FT_ERANGE, "pair larger than 2048 items");
    // queries sorted into Morton ranks; candidates in range
    launch_prep_sort(ix, off, q_id, q_mass, n_q, rank, mass, pos, lcp, cnt, status, s);
    const int64_t n_pairs = n_q * (int64_t)n_cand;
    k_check_range<<<(unsigned)ceil_div(n_pairs, 256), 256, 0, s>>>(cand, n_pairs, ix->docs.n, status);
    FT_HIP(hipGetLastError());
    na_read_status(status, h, s);
    if (h[0]) throw Error(FT_EINVAL, "queries or cand:" + describe_flags(h[0]));

    PairArgs a;
    a.q_off = off;
    a.q_rank = rank;
    a.q_mass = mass;
    a.d_off = ix->docs.off.as<int64_t>();
    a.d_rank = ix->docs.rank.as<uint32_t>();
    a.d_mass = ix->docs.mass.as<uint32_t>();
    a.cand = cand;
    a.n_cols = n_cand;
    a.st = ix->st.as<uint8_t>();
    a.V = ix->V;
    a.B = ix->B;
    a.Q = ix->Q;
    a.X = ix->Xm.as<float>();
    a.stride = ix->dp;
    a.status = status;
    a.cost = cost;
    const int G = knn_lanes(ix->dp);
    for (int cls = 0; cls <= top_cls; ++cls) {
      with_class(cls, [&](auto cc, auto ww) {
        with_lanes(G, [&](auto gg) {
          constexpr int C = decltype(cc)::value, W = decltype(ww)::value, GG = decltype(gg)::value;
          int per_cu = 0;
          FT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &per_cu, reinterpret_cast<const void*>(&k_flow_class_stride<C, W, GG>), 64 * W, 0));
          const unsigned blocks = (unsigned)std::min<int64_t>(n_pairs, (int64_t)std::max(1, per_cu) * ix->n_cu);
          k_flow_class_stride<C, W, GG><<<blocks, 64 * W, 0, s>>>(a, n_pairs, cls);
        });
      });
      FT_HIP(hipGetLastError());
    }
    topk_rows(cost, n_q, n_cand, cand, k, out_cost, out_doc, s);
    na_read_status(status, h, s);
    FT_REQUIRE(h[0] == 0, FT_EHIP, "flowtree kernel reported:" + describe_flags(h[0]));
  });
}
