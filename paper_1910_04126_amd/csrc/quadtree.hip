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
// Ranking all docs.  Every doc owns a hash table of its embedding, built once
// per index in HBM: nb = max(2, nnz) buckets of two (key, mass) slots (load
// at most 1/2), bucket = high half of (key * golden) * nb, linear probing
// with wrap-around.  A workgroup copies the tables of T consecutive docs into
// LDS and streams the (cache-resident) query embeddings; lane l works for doc
// l % T on the query entries l / T, l / T + 64 / T, ..., four lookups in
// flight, and the 64 / T lanes of a doc are summed by xor-shuffles.  One
// 16-byte LDS read answers a lookup unless the bucket is full without the
// key.  A bucket's second slot is only used once its first is taken, so an
// empty second slot ends a miss.

constexpr uint32_t NO_KEY = 0xFFFFFFFEu;  // padding entry: never a node key
constexpr uint32_t HASH_MUL = 0x9E3779B1u;
constexpr int QT_BUCKETS = 4096;           // LDS buckets per workgroup (64 KiB)
constexpr int QT_TILE_THREADS = 512;

struct DocTile {
  int64_t d0;     // first doc
  int32_t T;      // docs (power of two, <= 32)
  int32_t pad;
};

// One wavefront per doc: insert its embedding into its table.
__global__ __launch_bounds__(64) void k_build_doc_tables(const int64_t* __restrict__ d_eoff,
                                                         const uint32_t* __restrict__ d_ekey,
                                                         const uint32_t* __restrict__ d_emass,
                                                         const int64_t* __restrict__ tb_off, int64_t n,
                                                         uint4* __restrict__ tables) {
  const int64_t d = blockIdx.x;
  if (d >= n) return;
  uint4* tb = tables + tb_off[d];
  const uint32_t nb = (uint32_t)(tb_off[d + 1] - tb_off[d]);
  for (uint32_t i = threadIdx.x; i < nb; i += 64) tb[i] = make_uint4(EMPTY_KEY, 0u, EMPTY_KEY, 0u);
  __syncthreads();
  for (int64_t e = d_eoff[d] + threadIdx.x; e < d_eoff[d + 1]; e += 64) {
    const uint32_t key = d_ekey[e];
    uint32_t h = __umulhi(key * HASH_MUL, nb);
    while (true) {
      uint32_t* w = reinterpret_cast<uint32_t*>(&tb[h]);
      if (atomicCAS(&w[0], EMPTY_KEY, key) == EMPTY_KEY) {
        w[1] = d_emass[e];
        break;
      }
      if (atomicCAS(&w[2], EMPTY_KEY, key) == EMPTY_KEY) {
        w[3] = d_emass[e];
        break;
      }
      h = h + 1 == nb ? 0 : h + 1;
    }
  }
}

// Query entries with their hash product and weight shift precomputed.
__global__ void k_stage_query_entries(const uint32_t* __restrict__ ekey, const uint32_t* __restrict__ emass,
                                      int64_t nnz, int B, uint4* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t key = ekey[e];
  out[e] = make_uint4(key, emass[e], key * HASH_MUL, (uint32_t)(B - (int)(key >> KEY_DEPTH_SHIFT)));
}

__global__ __launch_bounds__(QT_TILE_THREADS) void k_qt_doctile(
    const DocTile* __restrict__ tiles, const uint4* __restrict__ tables, const int64_t* __restrict__ tb_off,
    const uint64_t* __restrict__ d_S, const int64_t* __restrict__ q_eoff, const uint4* __restrict__ q_ent,
    const uint64_t* __restrict__ q_S, int64_t q_begin, int64_t q_end, int64_t q_per_block, int64_t n_docs,
    uint64_t* __restrict__ keys) {
  __shared__ uint4 tab[QT_BUCKETS];
  const DocTile tile = tiles[blockIdx.x];
  const int64_t base = tb_off[tile.d0];
  const int nbt = (int)(tb_off[tile.d0 + tile.T] - base);
  for (int i = threadIdx.x; i < nbt; i += blockDim.x) tab[i] = tables[base + i];
  __syncthreads();
  const int lane = lane_id(), w = threadIdx.x >> 6;
  constexpr int NW = QT_TILE_THREADS / 64;
  const int T = tile.T, J = 64 / T;
  const int t = lane & (T - 1), j0 = lane / T;
  const int64_t doc = tile.d0 + t;
  const uint4* tb = tab + (tb_off[doc] - base);
  const uint32_t nb = (uint32_t)(tb_off[doc + 1] - tb_off[doc]);
  const uint64_t Sd = d_S[doc];
  const int64_t qa = q_begin + (int64_t)blockIdx.y * q_per_block;
  const int64_t qb = min(q_end, qa + q_per_block);
  constexpr int U = 4;  // lookups in flight per lane
  for (int64_t q = qa + w; q < qb; q += NW) {
    const int64_t e0 = q_eoff[q];
    const int ne = (int)(q_eoff[q + 1] - e0);
    const uint4* qe = q_ent + e0;
    uint64_t acc = 0;
    for (int i0 = j0; i0 < ne; i0 += U * J) {
      uint4 en[U];
      uint4 v[U];
      uint32_t bk[U];
      // the entry array is padded, so these loads never leave it; entries past
      // the query's end are turned into padding keys
#pragma unroll
      for (int u = 0; u < U; ++u) en[u] = qe[i0 + u * J];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        en[u].x = i0 + u * J < ne ? en[u].x : NO_KEY;
        bk[u] = __umulhi(en[u].z, nb);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = tb[bk[u]];
      uint32_t m[U];
      uint32_t pend = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t key = en[u].x;
        const bool hx = v[u].x == key, hz = v[u].z == key;
        m[u] = hx ? v[u].y : (hz ? v[u].w : 0u);
        const bool more = !hx & !hz & (v[u].z != EMPTY_KEY) & (key != NO_KEY);
        pend |= (uint32_t)more << u;
      }
      // a full bucket without the key: continue in the next buckets
      while (pend) {
        const int u = __builtin_ctz(pend);
        const uint32_t key = en[0].x * (u == 0) + en[1].x * (u == 1) + en[2].x * (u == 2) + en[3].x * (u == 3);
        uint32_t b = bk[0] * (u == 0) + bk[1] * (u == 1) + bk[2] * (u == 2) + bk[3] * (u == 3);
        uint32_t got = 0;
        while (true) {
          b = b + 1 == nb ? 0 : b + 1;
          const uint4 x = tb[b];
          if (x.x == key) {
            got = x.y;
            break;
          }
          if (x.z == key) {
            got = x.w;
            break;
          }
          if (x.z == EMPTY_KEY) break;
        }
#pragma unroll
        for (int uu = 0; uu < U; ++uu)
          if (uu == u) m[uu] = got;
        pend &= pend - 1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += (uint64_t)(en[u].y < m[u] ? en[u].y : m[u]) << en[u].w;
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

// Doc tables and tiles for ranking all docs, made once per index: table
// sizes from the embedding sizes, tables built on the device, tiles of up to
// 32 consecutive docs whose tables fit QT_BUCKETS.
static void prepare_doc_tables(ft_index* ix, hipStream_t s) {
  if (ix->doc_tiles_small > 0) return;
  const int64_t n = ix->docs.n;
  std::vector<int64_t> eoff(n + 1), tb(n + 1);
  FT_HIP(hipMemcpyAsync(eoff.data(), ix->docs.ecnt.p, (n + 1) * 8, hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
  tb[0] = 0;
  for (int64_t d = 0; d < n; ++d) {
    const int64_t nb = std::max<int64_t>(2, eoff[d + 1] - eoff[d]);
    FT_REQUIRE(nb <= QT_BUCKETS, FT_ERANGE, "a dataset distribution touches more than 4096 tree cells");
    tb[d + 1] = tb[d] + nb;
  }
  std::vector<DocTile> tiles;
  int64_t d = 0;
  while (d < n) {
    int T = 1;
    while (T * 2 <= 32 && d + 2 * T <= n && tb[d + 2 * T] - tb[d] <= QT_BUCKETS) T *= 2;
    tiles.push_back(DocTile{d, T, 0});
    d += T;
  }
  int64_t* dtb = (int64_t*)ix->doc_tb_off.ensure((n + 1) * 8);
  FT_HIP(hipMemcpyAsync(dtb, tb.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
  uint4* tables = (uint4*)ix->doc_tables.ensure(tb[n] * sizeof(uint4));
  k_build_doc_tables<<<(unsigned)n, 64, 0, s>>>(ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(),
                                                ix->docs.emass.as<uint32_t>(), dtb, n, tables);
  FT_HIP(hipGetLastError());
  DocTile* dt = (DocTile*)ix->doc_tiles.ensure(tiles.size() * sizeof(DocTile));
  FT_HIP(hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(DocTile), hipMemcpyHostToDevice, s));
  FT_HIP(hipStreamSynchronize(s));
  ix->doc_tiles_small = (int64_t)tiles.size();
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
    uint4* q_ent = nullptr;
    if (!cand) {
      prepare_doc_tables(ix, s);
      // padded by the furthest a lookup group can reach past a query's end
      q_ent = (uint4*)ix->ws_misc.ensure((ix->qry.emb_nnz + 4 * 64) * sizeof(uint4));
      FT_HIP(hipMemsetAsync(q_ent + ix->qry.emb_nnz, 0, 4 * 64 * sizeof(uint4), s));
      if (ix->qry.emb_nnz > 0)
        k_stage_query_entries<<<(unsigned)ceil_div(ix->qry.emb_nnz, 256), 256, 0, s>>>(
            ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(), ix->qry.emb_nnz, ix->B, q_ent);
      FT_HIP(hipGetLastError());
    }
    for (int64_t r0 = 0; r0 < n_q; r0 += rows_per_chunk) {
      const int64_t r1 = std::min(n_q, r0 + rows_per_chunk);
      if (!cand) {
        // all docs: doc tables in LDS, queries streamed
        const int64_t qpb = 256;
        const unsigned gy = (unsigned)ceil_div(r1 - r0, qpb);
        k_qt_doctile<<<dim3((unsigned)ix->doc_tiles_small, gy), QT_TILE_THREADS, 0, s>>>(
            ix->doc_tiles.as<DocTile>(), ix->doc_tables.as<uint4>(), ix->doc_tb_off.as<int64_t>(),
            ix->docs.S.as<uint64_t>(), ix->qry.ecnt.as<int64_t>(), q_ent, ix->qry.S.as<uint64_t>(), r0, r1, qpb,
            n_cols, keys);
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
