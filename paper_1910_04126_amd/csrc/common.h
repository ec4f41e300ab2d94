// Internal declarations shared by the ftree HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ftree.h"

namespace ft {

// ---------------------------------------------------------------- errors --

struct Error : std::runtime_error {
  ft_status status;
  Error(ft_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void set_last_error(const std::string& msg);

#define FT_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::ft::Error(FT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define FT_REQUIRE(cond, status, msg)                          \
  do {                                                         \
    if (!(cond)) throw ::ft::Error((status), (msg));           \
  } while (0)

// Runs f, turning exceptions into an ft_status and the thread's last error.
template <class F>
ft_status guarded(F&& f) {
  try {
    f();
    return FT_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return FT_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return FT_EHIP;
  }
}

// ------------------------------------------------------- device buffers --

// A growable device allocation owned by the index.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void* ensure(size_t n);
  void release();
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Validation flags written by kernels (device u32 each).
enum : uint32_t {
  ERR_ID_RANGE = 1u,
  ERR_ZERO_MASS = 2u,
  ERR_MASS_SUM = 4u,
  ERR_DUPLICATE = 8u,
  ERR_SIZE = 16u,
  ERR_EMPTY = 32u,
  ERR_FLOW = 64u,  // internal consistency of the greedy (must never fire)
  ERR_NONFINITE = 128u,  // a non-finite input value
};
std::string describe_flags(uint32_t f);

// Sorted, validated distributions in Morton-rank order (docs or queries).
struct Dists {
  int64_t n = 0, nnz = 0;
  int32_t max_size = 0;
  int64_t emb_nnz = 0;
  DevBuf off;      // int64 [n+1] (copy of the caller's offsets)
  DevBuf rank;     // u32 [nnz]  Morton ranks, ascending within a distribution
  DevBuf mass;     // u32 [nnz]
  DevBuf pos;      // u16 [nnz]  position of the item in the caller's CSR row
  DevBuf lcp;      // u8  [nnz]  depth of the deepest cell shared with the next item
  DevBuf ecnt;     // int64 [n+1] embedding offsets
  DevBuf ekey;     // u32 [emb_nnz] node key: depth << 27 | index within depth
  DevBuf emass;    // u32 [emb_nnz]
  DevBuf S;        // u64 [n]  sum of 2^(B-depth) * mass over embedding entries
  DevBuf tmp;      // scratch for the preparation
  void release();
};

struct TuneChoice {
  int32_t chunk = 4;        // pairs per work grab of the persistent kernel
  int32_t blocks_per_cu = 0; // 0: from occupancy
  int32_t classes = 0;       // bitmask of pair-size classes used (0: all)
};

// Captured graphs of the batched Flowtree path: the bucketing of pairs into
// size classes, and the persistent launches.  Rebuilt when any baked
// argument changes.
struct BatchedGraphs {
  hipGraphExec_t pre = nullptr, main = nullptr;
  std::vector<uint64_t> key;
  void reset();
};

}  // namespace ft

struct ft_index {
  int64_t V = 0;
  int32_t d = 0, dp = 0, B = 0, Q = 0, height = 0, st_levels = 0;
  int64_t n_nodes = 0;
  int device = 0;
  int n_cu = 0;
  hipStream_t work = nullptr;  // internal stream for graph capture
  hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  hipEvent_t ev_rank[2] = {nullptr, nullptr}, ev_sel[2] = {nullptr, nullptr};  // Quadtree chunk pipeline
  hipEvent_t ev_p[3] = {nullptr, nullptr, nullptr};  // ft_knn_pipeline: prune / rerank boundaries
  ft::DevBuf Xm;        // float [V * dp], Morton order, rows zero-padded to dp = padded_row(d)
  ft::DevBuf Xn;        // double [V] squared norms of the Xm rows
  ft::DevBuf perm;      // u32 [V] rank -> original id
  ft::DevBuf inv;       // u32 [V] original id -> rank
  ft::DevBuf st;        // u8  [st_levels * V] range-minimum table over adjacent LCA depths
  ft::DevBuf leafd;     // u8  [V]
  ft::DevBuf anc;       // u32 [height * V] index of the depth-(k+1) node of each rank
  ft::DevBuf status;    // u32 [8] validation flags and counters
  ft::Dists docs;
  std::vector<int64_t> depth_nodes;  // [height + 1] nodes at each depth
  // inverted doc lists for ranking all docs (built on first use)
  ft::DevBuf post;         // u16 [docs.emb_nnz] doc within slice, then (16-byte aligned) u32 [docs.emb_nnz]
                           // cell mass; by slice, then cell, then doc
  ft::DevBuf post_dir;     // u32 [post_nsl * post_cells] end offset of each cell's list in its slice
  ft::DevBuf post_cbase;   // u32 [32] first cell number of each depth
  ft::DevBuf post_head;     // u32 [post_nsl][post_nhead][post_slice] dense cell masses of the head cells, by doc
  ft::DevBuf post_s32;      // u32 [docs] S_d in compact key units (when the keys are compact)
  ft::DevBuf post_hcell;    // u8 [post_cells] head index of each cell (0xFF: a listed cell)
  int64_t post_slice = 0, post_cells = 0, post_nsl = 0;
  int32_t post_nhead = 0;
  // per-call workspaces
  ft::Dists qry;
  ft::DevBuf ws_keys, ws_cost, ws_tiles, ws_lists, ws_counts, ws_misc, ws_sel, ws_rerank;
  ft::DevBuf ws_gx64, ws_adj, ws_glist;  // backward: fixed-point dX, per-pair weight adjoints, pair lists
  ft::DevBuf ws_pipe;    // ft_knn_pipeline: prune keys, then candidate docs
  ft::DevBuf sel_exact;  // u32: rows of the last all-docs Quadtree select that took the exact path
  ft::DevBuf fwd_id, fwd_eta, fwd_key, fwd_bind, fwd_cnt, fwd_base;  // saved flows (FT_FWD)
  int64_t fwd_pairs = 0, fwd_cap = 0;
  ft::DevBuf fwd_sig;          // copies of the FT_FWD query CSR and pairs
  int64_t fwd_sig_bytes = 0;
  bool fwd_valid = false;
  int32_t autotune = 1;
  std::map<std::string, ft::TuneChoice> tuned;
  ft::BatchedGraphs graphs;
  double last_batched_ms = 0.0;
  double last_rerank_ms = 0.0;  // device time of the last ACT / Sinkhorn knn kernels
  double last_pipe_ms[2] = {0.0, 0.0};  // last ft_knn_pipeline: prune stage, rerank stage
  std::string last_schedule;
  std::mutex mu;
};

namespace ft {

// -------------------------------------------------------- shared device --

constexpr uint32_t KEY_DEPTH_SHIFT = 27;
constexpr uint32_t KEY_INDEX_MASK = (1u << KEY_DEPTH_SHIFT) - 1u;

// Depth of the deepest cell shared by Morton ranks a <= b: the minimum of
// the adjacent LCA depths over [a, b), from the range-minimum table.
__device__ __forceinline__ int lca_depth(const uint8_t* __restrict__ st, int64_t V, int B,
                                         uint32_t a, uint32_t b) {
  if (a == b) return B;
  uint32_t len = b - a;
  int j = 31 - __clz(len);
  uint8_t x = st[(int64_t)j * V + a];
  uint8_t y = st[(int64_t)j * V + (b - (1u << j))];
  return x < y ? x : y;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Row length in floats of the index's Morton-ordered coordinate copy: d
// rounded up so that the G lanes that share a row in the Flowtree pricing
// (the power of two up to 16 that covers the row in float4s) read the same
// number of float4s each; the padding is zero.
inline int padded_row(int d) {
  const int nv = (d + 3) / 4;
  int g = 1;
  while (g < 16 && g < nv) g <<= 1;
  return (int)ceil_div(nv, g) * g * 4;
}

// Host helpers implemented in build.hip.
void prepare_dists(ft_index* ix, Dists& D, const int64_t* off, const uint32_t* id,
                   const uint32_t* mass, int64_t n, bool with_embedding, hipStream_t s,
                   const char* what);
// Launch-only pieces of prepare_dists over caller-provided memory: offsets
// validation (status[0] flags, status[1] largest support) and the
// per-distribution sort into Morton ranks (status[0] flags).
void launch_check_offsets(const int64_t* off, int64_t n, uint32_t* status, hipStream_t s);
void launch_prep_sort(const ft_index* ix, const int64_t* off, const uint32_t* id, const uint32_t* mass, int64_t n,
                      uint32_t* rank, uint32_t* mass_out, uint16_t* pos, uint8_t* lcp, int64_t* cnt,
                      uint32_t* status, hipStream_t s);
// Device address of the no-allocation entry point's scratch array on a
// device (looked up once per device; that device must be current).
void* noalloc_scratch(int device);

// The bodies of ft_quadtree_knn and ft_flowtree_knn after their argument
// checks, on queries already prepared in ix->qry (with the embedding for the
// Quadtree) and candidate lists already checked; neither reads the status.
void quadtree_knn_prepared(ft_index* ix, int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t k,
                           uint64_t* out_key, int64_t* out_doc, hipStream_t s);
void flowtree_knn_prepared(ft_index* ix, int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t k, int32_t mode,
                           float* out_cost, int64_t* out_doc, hipStream_t s);
int64_t scan_tmp_elems(int64_t n);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
uint32_t read_and_clear_status(ft_index* ix, hipStream_t s);
// FT_EINVAL unless every v[i] lies in [0, bound) (synchronises s).
void check_indices(ft_index* ix, const int64_t* v, int64_t n, int64_t bound, hipStream_t s, const char* what);

}  // namespace ft
