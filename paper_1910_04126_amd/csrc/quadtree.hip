// Quadtree estimate (paper Section 2, "Wasserstein-1 on Quadtree"): the tree
// W1 between mu and nu is sum over cells v of side(v) * |mu(v) - nu(v)|.
// With each distribution stored as its l1 embedding (one entry per cell it
// touches: node key, cell mass) and S = sum side * mass, the estimate is
//     U = S_q + S_d - 2 * sum_{v in q and d} side(v) * min(m_q(v), m_d(v)),
// so a pair costs one LDS hash lookup per doc entry.  Queries are tiled: a
// workgroup holds the hash tables of T queries and streams doc embeddings;
// each thread owns one (doc, query) pair and accumulates an exact u64 key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "select.h"
#include "wave.h"

namespace ft {

constexpr uint32_t EMPTY_KEY = 0xFFFFFFFFu;
constexpr int QT_THREADS = 256;

struct QtTile {
  int32_t q0;     // first query of the tile
  int32_t T;      // queries in the tile (power of two, <= 16)
  int32_t lgcap;  // log2 of each query's hash capacity
  int32_t pad;
};

__device__ __forceinline__ uint32_t slot_hash(uint32_t key, int lgcap) {
  return (key * 0x9E3779B1u) >> (32 - lgcap);
}

template <int SLOTS>
__device__ __forceinline__ void qt_build_tables(uint32_t* tk, uint32_t* tm, const QtTile& tile,
                                                const int64_t* __restrict__ q_eoff,
                                                const uint32_t* __restrict__ q_ekey,
                                                const uint32_t* __restrict__ q_emass) {
  const int cap = 1 << tile.lgcap;
  for (int i = threadIdx.x; i < tile.T * cap; i += blockDim.x) tk[i] = EMPTY_KEY;
  __syncthreads();
  for (int t = 0; t < tile.T; ++t) {
    const int64_t e0 = q_eoff[tile.q0 + t], e1 = q_eoff[tile.q0 + t + 1];
    uint32_t* k = tk + t * cap;
    uint32_t* m = tm + t * cap;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const uint32_t key = q_ekey[e];
      uint32_t h = slot_hash(key, tile.lgcap);
      while (true) {
        uint32_t prev = atomicCAS(&k[h], EMPTY_KEY, key);
        if (prev == EMPTY_KEY || prev == key) {
          m[h] = q_emass[e];
          break;
        }
        h = (h + 1) & (cap - 1);
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ uint32_t qt_lookup(const uint32_t* tk, const uint32_t* tm, int lgcap, uint32_t key) {
  const uint32_t mask = (1u << lgcap) - 1;
  uint32_t h = slot_hash(key, lgcap);
  while (true) {
    const uint32_t k = tk[h];
    if (k == key) return tm[h];
    if (k == EMPTY_KEY) return 0u;
    h = (h + 1) & mask;
  }
}

// Keys for a tile of queries against columns [blockIdx.y * per_block, ...):
// column c is doc c, or cand[q * n_cols + c] when a candidate list is given.
template <int SLOTS>
__global__ __launch_bounds__(QT_THREADS) void k_qt_tile(
    const QtTile* __restrict__ tiles, const int64_t* __restrict__ q_eoff, const uint32_t* __restrict__ q_ekey,
    const uint32_t* __restrict__ q_emass, const uint64_t* __restrict__ q_S, const int64_t* __restrict__ d_eoff,
    const uint32_t* __restrict__ d_ekey, const uint32_t* __restrict__ d_emass, const uint64_t* __restrict__ d_S,
    const int64_t* __restrict__ cand, int64_t n_cols, int64_t per_block, int B, int64_t row0,
    uint64_t* __restrict__ keys) {
  __shared__ uint32_t tk[SLOTS];
  __shared__ uint32_t tm[SLOTS];
  const QtTile tile = tiles[blockIdx.x];
  qt_build_tables<SLOTS>(tk, tm, tile, q_eoff, q_ekey, q_emass);
  const int T = tile.T;
  const int t = threadIdx.x & (T - 1);
  const int slot = threadIdx.x / T;
  const int per = QT_THREADS / T;
  const int cap = 1 << tile.lgcap;
  const uint32_t* mk = tk + t * cap;
  const uint32_t* mm = tm + t * cap;
  const int64_t q = tile.q0 + t;
  const uint64_t Sq = q_S[q];
  const int64_t c_begin = (int64_t)blockIdx.y * per_block;
  const int64_t c_end = min(n_cols, c_begin + per_block);
  for (int64_t c = c_begin + slot; c < c_end; c += per) {
    const int64_t doc = cand ? cand[q * n_cols + c] : c;
    const int64_t e0 = d_eoff[doc], e1 = d_eoff[doc + 1];
    uint64_t acc = 0;
    for (int64_t e = e0; e < e1; ++e) {
      const uint32_t key = d_ekey[e];
      const uint32_t b = qt_lookup(mk, mm, tile.lgcap, key);
      if (b) {
        const uint32_t a = d_emass[e];
        acc += (uint64_t)(a < b ? a : b) << (B - (int)(key >> KEY_DEPTH_SHIFT));
      }
    }
    keys[(q - row0) * n_cols + c] = Sq + d_S[doc] - 2 * acc;
  }
}

// Explicit (query, doc) pairs: one wavefront per pair, the query table in LDS.
__global__ __launch_bounds__(64) void k_qt_pairs(const int64_t* __restrict__ pair_q, const int64_t* __restrict__ pair_d,
                                                 int64_t n_pairs, const int64_t* __restrict__ q_eoff,
                                                 const uint32_t* __restrict__ q_ekey,
                                                 const uint32_t* __restrict__ q_emass,
                                                 const uint64_t* __restrict__ q_S, const int64_t* __restrict__ d_eoff,
                                                 const uint32_t* __restrict__ d_ekey,
                                                 const uint32_t* __restrict__ d_emass,
                                                 const uint64_t* __restrict__ d_S, int B, uint64_t* __restrict__ out) {
  __shared__ uint32_t tk[8192];
  __shared__ uint32_t tm[8192];
  const int64_t p = blockIdx.x;
  if (p >= n_pairs) return;
  const int64_t q = pair_q[p], doc = pair_d[p];
  const int64_t nq = q_eoff[q + 1] - q_eoff[q];
  int lg = 1;
  while ((1ll << lg) < 2 * nq) ++lg;
  QtTile tile{(int32_t)q, 1, lg, 0};
  qt_build_tables<8192>(tk, tm, tile, q_eoff, q_ekey, q_emass);
  uint64_t acc = 0;
  for (int64_t e = d_eoff[doc] + threadIdx.x; e < d_eoff[doc + 1]; e += 64) {
    const uint32_t key = d_ekey[e];
    const uint32_t b = qt_lookup(tk, tm, lg, key);
    if (b) {
      const uint32_t a = d_emass[e];
      acc += (uint64_t)(a < b ? a : b) << (B - (int)(key >> KEY_DEPTH_SHIFT));
    }
  }
  acc = wave_sum(acc);
  if (threadIdx.x == 0) out[p] = q_S[q] + d_S[doc] - 2 * acc;
}

__global__ void k_check_index(const int64_t* __restrict__ v, int64_t n, int64_t bound, uint32_t* __restrict__ status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (v[i] < 0 || v[i] >= bound)) atomicOr(status, ERR_ID_RANGE);
}

void check_indices(ft_index* ix, const int64_t* v, int64_t n, int64_t bound, hipStream_t s, const char* what) {
  if (n <= 0) return;
  k_check_index<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(v, n, bound, ix->status.as<uint32_t>());
  FT_HIP(hipGetLastError());
  if (read_and_clear_status(ix, s)) throw Error(FT_EINVAL, std::string(what) + ": index out of range");
}

// Greedy tiling of queries: consecutive queries share a tile while T * cap
// fits the slot budget; cap = next power of two >= 2 * embedding size.
static std::vector<QtTile> plan_tiles(const std::vector<int64_t>& eoff, int64_t q_begin, int64_t q_end, int slots,
                                      int max_T) {
  std::vector<QtTile> tiles;
  int64_t q = q_begin;
  while (q < q_end) {
    int T = 1;
    int lg = 1;
    auto need_lg = [&](int64_t qq) {
      int64_t ne = eoff[qq + 1] - eoff[qq];
      int l = 1;
      while ((1ll << l) < 2 * ne) ++l;
      return l;
    };
    lg = need_lg(q);
    while (T * 2 <= max_T && q + 2 * T <= q_end) {
      int lg2 = lg;
      for (int64_t qq = q + T; qq < q + 2 * T; ++qq) lg2 = std::max(lg2, need_lg(qq));
      if ((int64_t)(2 * T) << lg2 > slots) break;
      T *= 2;
      lg = lg2;
    }
    tiles.push_back(QtTile{(int32_t)q, T, lg, 0});
    q += T;
  }
  return tiles;
}

constexpr int SLOTS_SMALL = 4096, SLOTS_LARGE = 8192;

}  // namespace ft

using namespace ft;

extern "C" ft_status ft_quadtree_knn(ft_index* ix, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                                     int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t k, uint64_t* out_key,
                                     int64_t* out_doc, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && out_key && out_doc, FT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_cols = cand ? (int64_t)n_cand : ix->docs.n;
    FT_REQUIRE(!cand || (n_cand >= 1 && n_cand <= 4096), FT_ERANGE, "n_cand must lie in [1, 4096]");
    FT_REQUIRE(k >= 1 && k <= n_cols, FT_EINVAL, "k must lie in [1, number of candidates]");
    FT_REQUIRE(cand || n_cols <= 4096 || k <= 1024, FT_ERANGE, "k > 1024 needs at most 4096 candidates");
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, true, s, "queries");
    if (cand) check_indices(ix, cand, n_q * n_cand, ix->docs.n, s, "cand");
    std::vector<int64_t> eoff(n_q + 1);
    FT_HIP(hipMemcpyAsync(eoff.data(), ix->qry.ecnt.p, (n_q + 1) * 8, hipMemcpyDeviceToHost, s));
    FT_HIP(hipStreamSynchronize(s));
    for (int64_t q = 0; q < n_q; ++q)
      FT_REQUIRE(eoff[q + 1] - eoff[q] <= SLOTS_LARGE / 2, FT_ERANGE,
                 "a query touches more than 4096 tree cells");
    // query chunks bound the key buffer to about 2 GiB
    const int64_t rows_per_chunk = std::max<int64_t>(1, std::min<int64_t>(n_q, (int64_t(1) << 28) / n_cols));
    uint64_t* keys = (uint64_t*)ix->ws_keys.ensure(rows_per_chunk * n_cols * 8);
    const int64_t per_block = cand ? n_cols : 2048;
    for (int64_t r0 = 0; r0 < n_q; r0 += rows_per_chunk) {
      const int64_t r1 = std::min(n_q, r0 + rows_per_chunk);
      for (int pass = 0; pass < 2; ++pass) {
        // pass 0: tiles whose tables fit SLOTS_SMALL; pass 1: the rest
        std::vector<QtTile> tiles;
        int64_t q = r0;
        while (q < r1) {
          int64_t ne = eoff[q + 1] - eoff[q];
          bool small = 2 * ne <= SLOTS_SMALL;
          int64_t q2 = q;
          while (q2 < r1 && ((2 * (eoff[q2 + 1] - eoff[q2]) <= SLOTS_SMALL) == small)) ++q2;
          if (small == (pass == 0)) {
            auto t = plan_tiles(eoff, q, q2, small ? SLOTS_SMALL : SLOTS_LARGE, cand ? 1 : 16);
            tiles.insert(tiles.end(), t.begin(), t.end());
          }
          q = q2;
        }
        if (tiles.empty()) continue;
        QtTile* dt = (QtTile*)ix->ws_tiles.ensure(tiles.size() * sizeof(QtTile));
        FT_HIP(hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(QtTile), hipMemcpyHostToDevice, s));
        dim3 grid((unsigned)tiles.size(), (unsigned)ceil_div(n_cols, per_block));
        auto args = std::make_tuple(dt, ix->qry.ecnt.as<int64_t>(), ix->qry.ekey.as<uint32_t>(),
                                    ix->qry.emass.as<uint32_t>(), ix->qry.S.as<uint64_t>(),
                                    ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(),
                                    ix->docs.emass.as<uint32_t>(), ix->docs.S.as<uint64_t>());
        if (pass == 0)
          k_qt_tile<SLOTS_SMALL><<<grid, QT_THREADS, 0, s>>>(
              std::get<0>(args), std::get<1>(args), std::get<2>(args), std::get<3>(args), std::get<4>(args),
              std::get<5>(args), std::get<6>(args), std::get<7>(args), std::get<8>(args), cand, n_cols, per_block,
              ix->B, r0, keys);
        else
          k_qt_tile<SLOTS_LARGE><<<grid, QT_THREADS, 0, s>>>(
              std::get<0>(args), std::get<1>(args), std::get<2>(args), std::get<3>(args), std::get<4>(args),
              std::get<5>(args), std::get<6>(args), std::get<7>(args), std::get<8>(args), cand, n_cols, per_block,
              ix->B, r0, keys);
        FT_HIP(hipGetLastError());
        // the tile table is reused by the next pass: wait before overwriting it
        FT_HIP(hipStreamSynchronize(s));
      }
      topk_rows(keys, r1 - r0, n_cols, cand ? cand + r0 * n_cols : nullptr, k, out_key + r0 * k, out_doc + r0 * k,
                s);
    }
  });
}

extern "C" ft_status ft_quadtree_pairs(ft_index* ix, const int64_t* q_off, const uint32_t* q_id,
                                       const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                                       const int64_t* pair_d, int64_t n_pairs, uint64_t* out_key, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && pair_q && pair_d && out_key, FT_EINVAL, "NULL argument");
    FT_REQUIRE(n_pairs >= 0, FT_EINVAL, "n_pairs < 0");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, true, s, "queries");
    check_indices(ix, pair_q, n_pairs, n_q, s, "pair_q");
    check_indices(ix, pair_d, n_pairs, ix->docs.n, s, "pair_d");
    if (n_pairs == 0) return;
    k_qt_pairs<<<(unsigned)n_pairs, 64, 0, s>>>(pair_q, pair_d, n_pairs, ix->qry.ecnt.as<int64_t>(),
                                               ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(),
                                               ix->qry.S.as<uint64_t>(), ix->docs.ecnt.as<int64_t>(),
                                               ix->docs.ekey.as<uint32_t>(), ix->docs.emass.as<uint32_t>(),
                                               ix->docs.S.as<uint64_t>(), ix->B, out_key);
    FT_HIP(hipGetLastError());
  });
}
