// Quadtree estimate (paper Section 2, "Wasserstein-1 on Quadtree"): the tree
// W1 between mu and nu is sum over cells v of side(v) * |mu(v) - nu(v)|.
// With each distribution stored as its l1 embedding (one entry per cell it
// touches: node key, cell mass) and S = sum side * mass, the estimate is
//     U = S_q + S_d - 2 * sum_{v in q and d} side(v) * min(m_q(v), m_d(v)),
// so a pair costs one LDS hash lookup per entry of one side, accumulated as an
// exact u64 key.  Ranking all docs holds doc tables in LDS and streams the
// (cache-resident) queries; candidate lists hold one query table per
// workgroup and stream its candidates.
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

// ------------------------------------------------------- doc-tile kernel --
//
// Ranking all docs: a workgroup holds the hash tables of T consecutive docs
// (packed key | mass << 32 slots) and streams queries, whose embeddings are
// small enough to stay in cache.  In a wavefront, lane l works for doc
// t = l % T on the query entries l / T, l / T + 64 / T, ...; the 64 / T lanes
// of a doc are then summed by xor-shuffles.  Every lane does the same number
// of lookups, whatever the sizes.

constexpr uint64_t EMPTY_SLOT = 0x00000000FFFFFFFFull;
constexpr int QT_STAGE = 256;  // query entries staged per wavefront at a time

struct DocTile {
  int64_t d0;     // first doc
  int32_t T;      // docs (power of two, <= 64)
  int32_t lgcap;  // log2 slots per doc
};

__device__ __forceinline__ uint32_t probe(const uint64_t* __restrict__ tab, int lgcap, uint32_t key) {
  const uint32_t mask = (1u << lgcap) - 1;
  uint32_t h = slot_hash(key, lgcap);
  while (true) {
    const uint64_t v = tab[h];
    const uint32_t k = (uint32_t)v;
    if (k == key) return (uint32_t)(v >> 32);
    if (k == EMPTY_KEY) return 0u;
    h = (h + 1) & mask;
  }
}

template <int SLOTS>
__global__ __launch_bounds__(QT_THREADS) void k_qt_doctile(
    const DocTile* __restrict__ tiles, const int64_t* __restrict__ d_eoff, const uint32_t* __restrict__ d_ekey,
    const uint32_t* __restrict__ d_emass, const uint64_t* __restrict__ d_S, const int64_t* __restrict__ q_eoff,
    const uint32_t* __restrict__ q_ekey, const uint32_t* __restrict__ q_emass, const uint64_t* __restrict__ q_S,
    int64_t q_begin, int64_t q_end, int64_t q_per_block, int64_t n_docs, int B, uint64_t* __restrict__ keys) {
  __shared__ uint64_t tab[SLOTS];
  __shared__ uint64_t stage[QT_THREADS / 64][QT_STAGE];
  const DocTile tile = tiles[blockIdx.x];
  const int cap = 1 << tile.lgcap;
  for (int i = threadIdx.x; i < tile.T * cap; i += blockDim.x) tab[i] = EMPTY_SLOT;
  __syncthreads();
  for (int t = 0; t < tile.T; ++t) {
    const int64_t doc = tile.d0 + t;
    uint64_t* base = tab + t * cap;
    for (int64_t e = d_eoff[doc] + threadIdx.x; e < d_eoff[doc + 1]; e += blockDim.x) {
      const uint32_t key = d_ekey[e];
      const uint64_t v = ((uint64_t)d_emass[e] << 32) | key;
      uint32_t h = slot_hash(key, tile.lgcap);
      while (atomicCAS((unsigned long long*)&base[h], EMPTY_SLOT, v) != EMPTY_SLOT) h = (h + 1) & (cap - 1);
    }
  }
  __syncthreads();
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int T = tile.T, J = 64 / T;
  const int t = lane & (T - 1), j0 = lane / T;
  const uint64_t* mytab = tab + t * cap;
  const int64_t doc = tile.d0 + t;
  const uint64_t Sd = d_S[doc];
  uint64_t* st = stage[w];
  const int64_t qa = q_begin + (int64_t)blockIdx.y * q_per_block;
  const int64_t qb = min(q_end, qa + q_per_block);
  for (int64_t q = qa + w; q < qb; q += QT_THREADS / 64) {
    const int64_t e0 = q_eoff[q];
    const int ne = (int)(q_eoff[q + 1] - e0);
    uint64_t acc = 0;
    for (int c0 = 0; c0 < ne; c0 += QT_STAGE) {
      const int cn = min(QT_STAGE, ne - c0);
      __builtin_amdgcn_wave_barrier();
      for (int i = lane; i < cn; i += 64) st[i] = ((uint64_t)q_emass[e0 + c0 + i] << 32) | q_ekey[e0 + c0 + i];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int i = j0; i < cn; i += J) {
        const uint64_t ent = st[i];
        const uint32_t key = (uint32_t)ent;
        const uint32_t b = probe(mytab, tile.lgcap, key);
        const uint32_t a = (uint32_t)(ent >> 32);
        acc += (uint64_t)(a < b ? a : b) << (B - (int)(key >> KEY_DEPTH_SHIFT));
      }
    }
    for (int o = T; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (j0 == 0) keys[(q - q_begin) * n_docs + doc] = q_S[q] + Sd - 2 * acc;
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

constexpr int SLOTS_SMALL = 4096, SLOTS_LARGE = 8192;

// Doc tiles for ranking all docs, planned once per index: consecutive docs
// share a tile while T * cap fits SLOTS_SMALL (docs needing more go alone
// into SLOTS_LARGE tiles).  Returns the number of small tiles; large ones
// follow in the same array.
static void plan_doc_tiles(ft_index* ix, hipStream_t s) {
  if (ix->doc_tiles_small + ix->doc_tiles_large > 0) return;
  const int64_t n = ix->docs.n;
  std::vector<int64_t> eoff(n + 1);
  FT_HIP(hipMemcpyAsync(eoff.data(), ix->docs.ecnt.p, (n + 1) * 8, hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
  auto need_lg = [&](int64_t d) {
    int64_t ne = eoff[d + 1] - eoff[d];
    int l = 1;
    while ((1ll << l) < 2 * ne) ++l;
    return l;
  };
  std::vector<DocTile> small, large;
  int64_t d = 0;
  while (d < n) {
    int lg = need_lg(d);
    if ((1ll << lg) > SLOTS_SMALL) {
      FT_REQUIRE((1ll << lg) <= SLOTS_LARGE, FT_ERANGE, "a dataset distribution touches more than 4096 tree cells");
      large.push_back(DocTile{d, 1, lg});
      ++d;
      continue;
    }
    int T = 1;
    while (T * 2 <= 64 && d + 2 * T <= n) {
      int lg2 = lg;
      for (int64_t x = d + T; x < d + 2 * T; ++x) lg2 = std::max(lg2, need_lg(x));
      if (((int64_t)(2 * T) << lg2) > SLOTS_SMALL) break;
      T *= 2;
      lg = lg2;
    }
    small.push_back(DocTile{d, T, lg});
    d += T;
  }
  ix->doc_tiles_small = (int64_t)small.size();
  ix->doc_tiles_large = (int64_t)large.size();
  small.insert(small.end(), large.begin(), large.end());
  DocTile* dt = (DocTile*)ix->doc_tiles.ensure(small.size() * sizeof(DocTile));
  FT_HIP(hipMemcpyAsync(dt, small.data(), small.size() * sizeof(DocTile), hipMemcpyHostToDevice, s));
  FT_HIP(hipStreamSynchronize(s));
}

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
    // query chunks bound the key buffer to about 4 GiB
    const int64_t rows_per_chunk = std::max<int64_t>(1, std::min<int64_t>(n_q, (int64_t(1) << 29) / n_cols));
    uint64_t* keys = (uint64_t*)ix->ws_keys.ensure(rows_per_chunk * n_cols * 8);
    if (!cand) plan_doc_tiles(ix, s);
    for (int64_t r0 = 0; r0 < n_q; r0 += rows_per_chunk) {
      const int64_t r1 = std::min(n_q, r0 + rows_per_chunk);
      if (!cand) {
        // all docs: doc tiles in LDS, queries streamed
        const int64_t qpb = 128;
        const DocTile* dt = ix->doc_tiles.as<DocTile>();
        const unsigned gy = (unsigned)ceil_div(r1 - r0, qpb);
        if (ix->doc_tiles_small)
          k_qt_doctile<SLOTS_SMALL><<<dim3((unsigned)ix->doc_tiles_small, gy), QT_THREADS, 0, s>>>(
              dt, ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(), ix->docs.emass.as<uint32_t>(),
              ix->docs.S.as<uint64_t>(), ix->qry.ecnt.as<int64_t>(), ix->qry.ekey.as<uint32_t>(),
              ix->qry.emass.as<uint32_t>(), ix->qry.S.as<uint64_t>(), r0, r1, qpb, n_cols, ix->B, keys);
        if (ix->doc_tiles_large)
          k_qt_doctile<SLOTS_LARGE><<<dim3((unsigned)ix->doc_tiles_large, gy), QT_THREADS, 0, s>>>(
              dt + ix->doc_tiles_small, ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(),
              ix->docs.emass.as<uint32_t>(), ix->docs.S.as<uint64_t>(), ix->qry.ecnt.as<int64_t>(),
              ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(), ix->qry.S.as<uint64_t>(), r0, r1, qpb,
              n_cols, ix->B, keys);
        FT_HIP(hipGetLastError());
      } else {
        // candidate lists: one query per workgroup, its table in LDS
        std::vector<QtTile> tiles;
        int64_t big = 0;
        for (int64_t q = r0; q < r1; ++q) {
          int64_t ne = eoff[q + 1] - eoff[q];
          int l = 1;
          while ((1ll << l) < 2 * ne) ++l;
          tiles.push_back(QtTile{(int32_t)q, 1, l, 0});
          big = std::max<int64_t>(big, 1ll << l);
        }
        QtTile* dt = (QtTile*)ix->ws_tiles.ensure(tiles.size() * sizeof(QtTile));
        FT_HIP(hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(QtTile), hipMemcpyHostToDevice, s));
        dim3 grid((unsigned)tiles.size(), 1);
        if (big <= SLOTS_SMALL)
          k_qt_tile<SLOTS_SMALL><<<grid, QT_THREADS, 0, s>>>(
              dt, ix->qry.ecnt.as<int64_t>(), ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(),
              ix->qry.S.as<uint64_t>(), ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(),
              ix->docs.emass.as<uint32_t>(), ix->docs.S.as<uint64_t>(), cand, n_cols, n_cols, ix->B, r0, keys);
        else
          k_qt_tile<SLOTS_LARGE><<<grid, QT_THREADS, 0, s>>>(
              dt, ix->qry.ecnt.as<int64_t>(), ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(),
              ix->qry.S.as<uint64_t>(), ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(),
              ix->docs.emass.as<uint32_t>(), ix->docs.S.as<uint64_t>(), cand, n_cols, n_cols, ix->B, r0, keys);
        FT_HIP(hipGetLastError());
        FT_HIP(hipStreamSynchronize(s));  // the tile table is reused by the next chunk
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
