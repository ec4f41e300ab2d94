// Quadtree estimate (paper Section 2, "Wasserstein-1 on Quadtree"): the tree
// W1 between mu and nu is sum over cells v of side(v) * |mu(v) - nu(v)|.
// With each distribution stored as its l1 embedding (one entry per cell it
// touches: node key, cell mass) and S = sum side * mass, the estimate is
//     U = S_q + S_d - 2 * sum_{v in q and d} side(v) * min(m_q(v), m_d(v)),
// accumulated as an exact u64 key.  Ranking all docs walks inverted doc lists
// of the query's cells, so a pair costs only its shared cells; candidate
// lists hold one query hash table per workgroup and stream the candidates'
// entries through it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
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

// ------------------------------------------------- posting-list kernels --
//
// Ranking all docs.  A pair only gains from the cells it shares, and a
// (query, doc) pair of word-embedding-shaped data shares about a tenth of the
// query's cells, so the docs are stored inverted: cut into slices of S
// consecutive docs, and inside a slice, for every tree cell, the list of
// (doc within the slice, cell mass) of the docs that touch it.  Cells are
// numbered densely (all depth-1 nodes, then depth 2, ...), so a slice's list
// directory is a plain array of end offsets indexed by cell number.
//
// A workgroup takes one (query, slice): it looks up up to QP_ENTRIES of the
// query's cells at a time in the slice directory, cuts the non-empty lists
// into pieces of QP_PIECE entries (a table in LDS maps each piece to its
// list), and its wavefronts, QP_U pieces at a time, add
// side(depth) * min(query mass, doc mass) into one LDS counter per doc; the
// keys S_q + S_d - 2 * counter follow.  Counters are u32 in units of the
// deepest side when every sum fits (Q + height <= 32: a depth's cells
// partition the mass, so the sum is below 2^(Q + height)), else u64 in grid
// units; either way they fill 32 KB, so a slice is 8192 or 4096 docs.  With
// 128 cells per round and two pieces in flight a workgroup needs under 40 KB
// of LDS and 52 VGPRs, so a CU holds four of them (8 wavefronts per SIMD):
// the kernel spends most of its time waiting on list reads and LDS atomics.

constexpr int QP_THREADS = 512;
constexpr int QP_WAVES = QP_THREADS / 64;
constexpr int QP_ACC_BYTES = 32 * 1024;
constexpr int QP_ENTRIES = 128;  // query cells per round (an item index fits a byte)
constexpr int QP_PIECE = 256;    // list entries per piece
constexpr int QP_U = 2;          // pieces in flight per wavefront
// a list in a slice has at most one entry per doc
constexpr int QP_MAX_PIECES = QP_ENTRIES * (QP_ACC_BYTES / 4) / QP_PIECE;
// Head cells: a few cells are touched by a large share of all docs and carry
// most of the list entries (on word-embedding-shaped data the 64 longest
// lists hold about 70 % of the (query, doc, shared cell) work).  For the
// cells touched by at least half of the docs (up to QP_HEAD_MAX) a slice
// keeps a dense row of cell masses, one u32 per doc, and each thread adds
// its own 16 docs' terms in registers: no atomics for those cells.  Half is
// where a dense row stops costing more than the list it replaces (measured:
// a quarter and three quarters were both slower).  Only with narrow counters
// over full 8192-doc slices.
constexpr int QP_HEAD_MAX = 64;
constexpr int QP_HEAD_SLICE = 8192;  // QP_THREADS threads x 16 docs

inline bool post_narrow(int Q, int height) { return Q + height <= 32; }
// With Q + height <= 31 every key U < 2^(Q + height + 1) once expressed in
// units of the deepest side 2^(B - height) (S_q, S_d and the counters are
// multiples of it): the ranking then writes u32 keys.
inline bool post_compact(int Q, int height) { return Q + height <= 31; }

// Slice size for n docs: at least 8 slices when the docs allow, at most
// smax docs each.
inline int64_t post_slice_size(int64_t n, int64_t smax) {
  int64_t S = 64;
  while (S * 2 <= smax && S * 2 * 8 <= n) S *= 2;
  return S;
}

__device__ __forceinline__ uint32_t cell_number(const uint32_t* __restrict__ cbase, uint32_t key) {
  return cbase[key >> KEY_DEPTH_SHIFT] + (key & KEY_INDEX_MASK);
}

// Wavefront per doc: count the doc's cells into its slice's directory.
__global__ __launch_bounds__(64) void k_post_count(const int64_t* __restrict__ eoff, const uint32_t* __restrict__ ekey,
                                                   int64_t n_docs, int64_t S, int64_t n_cells,
                                                   const uint32_t* __restrict__ cbase, uint32_t* __restrict__ dir) {
  for (int64_t d = blockIdx.x; d < n_docs; d += gridDim.x) {
    uint32_t* D = dir + (d / S) * n_cells;
    for (int64_t e = eoff[d] + lane_id(); e < eoff[d + 1]; e += 64) atomicAdd(&D[cell_number(cbase, ekey[e])], 1u);
  }
}

// Workgroup per slice: exclusive scan of its directory counts, in place.
__global__ __launch_bounds__(1024) void k_post_scan(uint32_t* __restrict__ dir, int64_t n_cells) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry;
  uint32_t* D = dir + (int64_t)blockIdx.x * n_cells;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < n_cells; c0 += 4 * 1024) {
    uint32_t v[4], t = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t c = c0 + 4 * threadIdx.x + u;
      v[u] = c < n_cells ? D[c] : 0u;
      t += v[u];
    }
    const uint32_t incl = wave_incl_sum(t);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = carry;
    for (int j = 0; j < w; ++j) before += wsum[j];
    before += incl - t;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t c = c0 + 4 * threadIdx.x + u;
      if (c < n_cells) D[c] = before;
      before += v[u];
    }
    __syncthreads();
    if (threadIdx.x == 1023) carry = before;
    __syncthreads();
  }
}

// Wavefront per slice: place the slice's (doc in slice, mass) entries doc by
// doc, so every cell's list comes out in doc order (consecutive lanes of the
// ranking kernel then add into nearby, mostly distinct LDS banks).  A doc
// touches each cell once, so its lanes never share a counter; the barrier
// after each doc orders its counter updates before the next doc's.  The
// directory counters run from each list's start to its end, which is what
// the ranking kernel reads.  The doc is stored as the byte offset of its
// counter in the ranking kernel's LDS array (acc_bytes per counter).
__global__ __launch_bounds__(64) void k_post_fill(const int64_t* __restrict__ eoff, const uint32_t* __restrict__ ekey,
                                                  const uint32_t* __restrict__ emass, int64_t n_docs, int64_t S,
                                                  int64_t n_cells, const uint32_t* __restrict__ cbase,
                                                  uint32_t* __restrict__ dir, uint16_t* __restrict__ post_doc,
                                                  uint32_t* __restrict__ post_mass, uint32_t acc_bytes) {
  const int64_t sl = blockIdx.x;
  const int64_t d0 = sl * S, d1 = d0 + S < n_docs ? d0 + S : n_docs;
  uint32_t* D = dir + sl * n_cells;
  uint16_t* Pd = post_doc + eoff[d0];
  uint32_t* Pm = post_mass + eoff[d0];
  for (int64_t d = d0; d < d1; ++d) {
    const uint32_t local = (uint32_t)(d - d0);
    for (int64_t e = eoff[d] + lane_id(); e < eoff[d + 1]; e += 64) {
      const uint32_t pos = atomicAdd(&D[cell_number(cbase, ekey[e])], 1u);
      Pd[pos] = (uint16_t)(local * acc_bytes);
      Pm[pos] = emass[e];
    }
    __threadfence();
    __syncthreads();
  }
}

// S_d in units of 2^up (a multiple of it when keys are compact), as u32.
__global__ void k_s32(const uint64_t* __restrict__ S, int64_t n, int up, uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint32_t)(S[i] >> up);
}

// Wavefront per doc: its masses in the head cells, into the dense rows of
// its slice (rows start zeroed).
__global__ __launch_bounds__(64) void k_head_fill(const int64_t* __restrict__ eoff, const uint32_t* __restrict__ ekey,
                                                  const uint32_t* __restrict__ emass, int64_t n_docs,
                                                  const uint32_t* __restrict__ cbase, const uint8_t* __restrict__ hcell,
                                                  int nhead, uint32_t* __restrict__ rows) {
  for (int64_t d = blockIdx.x; d < n_docs; d += gridDim.x) {
    const int64_t sl = d / QP_HEAD_SLICE, local = d - sl * QP_HEAD_SLICE;
    for (int64_t e = eoff[d] + lane_id(); e < eoff[d + 1]; e += 64) {
      const uint8_t h = hcell[cell_number(cbase, ekey[e])];
      if (h != 0xFFu) rows[((size_t)sl * nhead + h) * QP_HEAD_SLICE + local] = emass[e];
    }
  }
}

// Workgroup per query, once per call: the query's cells split into its head
// cells (head row, mass, shift; at most QP_HEAD_MAX) and the others (cell
// number, mass, shift), so that the ranking kernel's workgroups, one per
// (query, slice), read them ready instead of looking each cell up again.
// The order within each list is arbitrary (the sums are exact integers).
__global__ __launch_bounds__(256) void k_qt_prep(const int64_t* __restrict__ q_eoff, const uint32_t* __restrict__ q_ekey,
                                                 const uint32_t* __restrict__ q_emass,
                                                 const uint32_t* __restrict__ cbase,
                                                 const uint8_t* __restrict__ hcell, int top, int64_t q0,
                                                 uint2* __restrict__ counts, uint2* __restrict__ head,
                                                 uint4* __restrict__ listed) {
  __shared__ uint32_t nh, nl;
  const int64_t q = q0 + blockIdx.x;
  if (threadIdx.x == 0) nh = nl = 0u;
  __syncthreads();
  const int64_t e0 = q_eoff[q], ne = q_eoff[q + 1] - e0;
  for (int64_t e = threadIdx.x; e < ne; e += blockDim.x) {
    const uint32_t key = q_ekey[e0 + e];
    const uint32_t c = cell_number(cbase, key);
    const uint32_t m = q_emass[e0 + e];
    const uint32_t sh = (uint32_t)(top - (int)(key >> KEY_DEPTH_SHIFT));
    const uint8_t h = hcell ? hcell[c] : (uint8_t)0xFFu;
    if (h != 0xFFu) {
      const uint32_t i = atomicAdd(&nh, 1u);
      head[blockIdx.x * QP_HEAD_MAX + i] = make_uint2(m, (uint32_t)h | (sh << 8));
    } else {
      const uint32_t i = atomicAdd(&nl, 1u);
      listed[e0 + i] = make_uint4(c, m, sh, 0u);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = make_uint2(nh, nl);
}

// Workgroup per (query, slice).  Workgroups are dealt to the 8 XCDs in turn,
// so block b runs on XCD b % 8; slices are given out so that each XCD walks
// one slice at a time through all the queries of the launch, keeping that
// slice's lists in its L2.  H: the tree height (narrow counters).
// Held to 72 scalar registers: at 82 the kernel allocated 96 and ran
// 15 % slower (fewer workgroups per CU), although its vector registers and
// LDS allow four.
template <bool NARROW, bool COMPACT, bool HEAD>
__global__ __launch_bounds__(QP_THREADS) __attribute__((amdgpu_num_sgpr(72))) void k_qt_post(
    const uint16_t* __restrict__ post_doc, const uint32_t* __restrict__ post_mass, const uint32_t* __restrict__ dir,
    const uint32_t* __restrict__ cbase, const uint32_t* __restrict__ head_rows, const uint8_t* __restrict__ hcell,
    int nhead,
    int64_t n_cells, int64_t S, int64_t n_sl, const int64_t* __restrict__ d_eoff, const uint64_t* __restrict__ d_S,
    const uint32_t* __restrict__ d_S32, int64_t n_docs, const int64_t* __restrict__ q_eoff, const uint32_t* __restrict__ q_ekey,
    const uint32_t* __restrict__ q_emass, const uint64_t* __restrict__ q_S, int64_t r0, int64_t n_rows, int B, int H,
    void* __restrict__ keys_out, unsigned long long* __restrict__ minmax, const uint2* __restrict__ q_counts,
    const uint2* __restrict__ q_head, const uint4* __restrict__ q_listed) {
  static_assert(NARROW || !COMPACT, "compact keys need narrow counters");
  static_assert(NARROW || !HEAD, "dense head rows need narrow counters");
  using Acc = typename std::conditional<NARROW, uint32_t, unsigned long long>::type;
  using Key = typename std::conditional<COMPACT, uint32_t, uint64_t>::type;
  constexpr int SMAX = QP_ACC_BYTES / sizeof(Acc);
  __shared__ Acc acc[SMAX];
  __shared__ uint4 items[QP_ENTRIES];          // list start, length, query mass, shift
  __shared__ uint32_t pstart[QP_ENTRIES];      // first piece of each list
  __shared__ uint8_t pitem[QP_MAX_PIECES];     // list of each piece
  __shared__ unsigned long long red[2][QP_WAVES];
  __shared__ unsigned long long ctr[2];  // (items << 32 | pieces) of a round, two rounds in turn
  const int64_t blk = blockIdx.x;
  const int64_t local = blk >> 3;
  const int64_t grp = local / n_rows, row = local - grp * n_rows;
  const int64_t sl = grp * 8 + (blk & 7);
  if (sl >= n_sl) return;
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const int64_t q = r0 + row, d0 = sl * S;
  const int nd = (int)(n_docs - d0 < S ? n_docs - d0 : S);
  const uint32_t* D = dir + sl * n_cells;
  const uint16_t* Pd = post_doc + d_eoff[d0];
  const uint32_t* Pm = post_mass + d_eoff[d0];
  const int64_t e0 = q_eoff[q];
  if constexpr (HEAD) {
    // the query's head cells, prepared once per call (row, mass, shift)
    const uint2* hq = q_head + row * QP_HEAD_MAX;
    // thread t owns docs j * 2048 + 4t + k (j, k < 4): its row reads are
    // 16 bytes at consecutive addresses across the wavefront
    // (the cell's row, mass and shift are the same for every lane: scalars;
    // the rows are read at 32-bit byte offsets from the slice's base)
    const int nh = (int)__builtin_amdgcn_readfirstlane(q_counts[row].x);
    const char* rbase = reinterpret_cast<const char*>(head_rows + (size_t)sl * nhead * QP_HEAD_SLICE);
    const uint32_t lane_off = 16u * (uint32_t)tid;
    Acc a16[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a16[k] = 0;
    for (int i = 0; i < nh; i += 2) {
      uint4 v[2][4];
      uint32_t am[2], sh[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool live = i + u < nh;
        const uint2 hd = live ? hq[i + u] : make_uint2(0u, 0u);
        const uint32_t id = __builtin_amdgcn_readfirstlane(hd.y & 0xFFu);
        am[u] = __builtin_amdgcn_readfirstlane(hd.x);
        sh[u] = __builtin_amdgcn_readfirstlane(hd.y >> 8);
        const uint32_t o = id * (uint32_t)(QP_HEAD_SLICE * 4) + lane_off;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          v[u][j] = live ? *reinterpret_cast<const uint4*>(rbase + (o + (uint32_t)j * 8192u)) : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a16[4 * j + 0] += (Acc)min(am[u], v[u][j].x) << sh[u];
          a16[4 * j + 1] += (Acc)min(am[u], v[u][j].y) << sh[u];
          a16[4 * j + 2] += (Acc)min(am[u], v[u][j].z) << sh[u];
          a16[4 * j + 3] += (Acc)min(am[u], v[u][j].w) << sh[u];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int doc = j * 2048 + 4 * tid + k;
        if (doc < nd) acc[doc] = a16[4 * j + k];
      }
  } else {
    for (int i = tid; i < nd; i += QP_THREADS) acc[i] = 0;
  }
  // the query's other cells, prepared once per call (cell number, mass, shift)
  const int nl = (int)__builtin_amdgcn_readfirstlane(q_counts[row].y);
  const uint4* ql = q_listed + e0;
  // Rounds of up to QP_ENTRIES cells: the thread that finds a non-empty list
  // claims its item and its pieces and writes their piece table entries
  // itself; the round's counter was cleared during the previous round (the
  // two counters alternate), so a round takes two barriers.
  if (tid == 0) ctr[0] = ctr[1] = 0ull;
  __syncthreads();
  for (int c0 = 0, rnd = 0; c0 < nl; c0 += QP_ENTRIES, rnd ^= 1) {
    if (tid < QP_ENTRIES && c0 + tid < nl) {
      const uint4 ent = ql[c0 + tid];
      const uint32_t c = ent.x;
      const uint32_t o1 = D[c], o0 = c ? D[c - 1] : 0u;
      if (o1 > o0) {
        const uint32_t len = o1 - o0, np = (len + QP_PIECE - 1) / QP_PIECE;
        const unsigned long long old = atomicAdd(&ctr[rnd], (1ull << 32) | np);
        const uint32_t idx = (uint32_t)(old >> 32), p0 = (uint32_t)old;
        items[idx] = make_uint4(o0, len, ent.y, ent.z);
        pstart[idx] = p0;
        for (uint32_t j = 0; j < np; ++j) pitem[p0 + j] = (uint8_t)idx;
      }
    }
    __syncthreads();
    const unsigned long long cc = ctr[rnd];
    if (tid == 0) ctr[rnd ^ 1] = 0ull;
    const uint32_t n_pieces = (uint32_t)cc;
    // a piece belongs to one wavefront, so its list offset, length, query
    // mass and shift are scalars; the entries are read at 32-bit byte offsets
    // from the slice's list base, and a full piece (every piece of a list but
    // its last) needs no per-lane bound
    const char* pd_base = reinterpret_cast<const char*>(Pd);
    const char* pm_base = reinterpret_cast<const char*>(Pm);
    // piece p's entry count, query mass, shift and first entry (zero count
    // past the last piece)
    auto piece = [&](uint32_t p, uint32_t& c, uint32_t& a, uint32_t& s, uint32_t& at) {
      c = a = s = at = 0;
      if (p < n_pieces) {
        const uint32_t it = pitem[p];
        const uint4 item = items[it];
        const uint32_t off = (p - pstart[it]) * QP_PIECE;
        c = min((uint32_t)QP_PIECE, item.y - off);
        a = item.z;
        s = item.w;
        at = item.x + off;
      }
      c = __builtin_amdgcn_readfirstlane(c);
      a = __builtin_amdgcn_readfirstlane(a);
      s = __builtin_amdgcn_readfirstlane(s);
      at = __builtin_amdgcn_readfirstlane(at);
    };
    // The next pieces' descriptors are read from LDS after this round's list
    // loads are issued and before its atomics: LDS operations complete in
    // order, so waiting for them does not wait for the atomics, and the next
    // loads go out while the atomics drain.
    uint32_t cnt[QP_U], am[QP_U], sh[QP_U], at[QP_U];
#pragma unroll
    for (int u = 0; u < QP_U; ++u) piece(w * QP_U + u, cnt[u], am[u], sh[u], at[u]);
    for (uint32_t p0 = w * QP_U; p0 < n_pieces; p0 += QP_WAVES * QP_U) {
      uint32_t ed[QP_U][QP_PIECE / 64], em[QP_U][QP_PIECE / 64];
#pragma unroll
      for (int u = 0; u < QP_U; ++u) {
        if (cnt[u] == (uint32_t)QP_PIECE) {
          const char* pd_lane = pd_base + 2u * (at[u] + lane);
          const char* pm_lane = pm_base + 4u * (at[u] + lane);
#pragma unroll
          for (int j = 0; j < QP_PIECE / 64; ++j) {
            ed[u][j] = *reinterpret_cast<const uint16_t*>(pd_lane + 128 * j);
            em[u][j] = *reinterpret_cast<const uint32_t*>(pm_lane + 256 * j);
          }
        } else {
#pragma unroll
          for (int j = 0; j < QP_PIECE / 64; ++j) {
            const uint32_t x = j * 64 + lane;
            ed[u][j] = x < cnt[u] ? (uint32_t)*reinterpret_cast<const uint16_t*>(pd_base + 2u * (at[u] + x)) : 0u;
            em[u][j] = x < cnt[u] ? *reinterpret_cast<const uint32_t*>(pm_base + 4u * (at[u] + x)) : 0u;
          }
        }
      }
      uint32_t ncnt[QP_U], nam[QP_U], nsh[QP_U], nat[QP_U];
#pragma unroll
      for (int u = 0; u < QP_U; ++u) piece(p0 + QP_WAVES * QP_U + u, ncnt[u], nam[u], nsh[u], nat[u]);
#pragma unroll
      for (int u = 0; u < QP_U; ++u) {
        if (cnt[u] == (uint32_t)QP_PIECE) {
#pragma unroll
          for (int j = 0; j < QP_PIECE / 64; ++j)
            atomicAdd(reinterpret_cast<Acc*>(reinterpret_cast<char*>(acc) + ed[u][j]), (Acc)min(am[u], em[u][j]) << sh[u]);
        } else {
#pragma unroll
          for (int j = 0; j < QP_PIECE / 64; ++j)
            if ((uint32_t)(j * 64 + lane) < cnt[u])
              atomicAdd(reinterpret_cast<Acc*>(reinterpret_cast<char*>(acc) + ed[u][j]), (Acc)min(am[u], em[u][j]) << sh[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < QP_U; ++u) {
        cnt[u] = ncnt[u];
        am[u] = nam[u];
        sh[u] = nsh[u];
        at[u] = nat[u];
      }
    }
    __syncthreads();
  }
  const uint64_t Sq = q_S[q];
  Key* out = reinterpret_cast<Key*>(keys_out) + row * n_docs + d0;
  const uint64_t* Sd = d_S + d0;
  const int up = NARROW ? B - H : 0;
  unsigned long long mn = ~0ull, mx = 0ull;
  if constexpr (COMPACT) {
    // in units of 2^(B - H): S_q and S_d are multiples of it, and the key
    // fits 32 bits
    const uint32_t sq = (uint32_t)(Sq >> up);
    const uint32_t* Sd32 = d_S32 + d0;
    uint32_t mn32 = 0xFFFFFFFFu, mx32 = 0u;
    for (int i = tid; i < nd; i += QP_THREADS) {
      const uint32_t key = sq + Sd32[i] - ((uint32_t)acc[i] << 1);
      out[i] = (Key)key;
      mn32 = key < mn32 ? key : mn32;
      mx32 = key > mx32 ? key : mx32;
    }
    mn = mn32 == 0xFFFFFFFFu ? ~0ull : (unsigned long long)mn32;
    mx = mx32;
  } else {
    for (int i = tid; i < nd; i += QP_THREADS) {
      const uint64_t key = Sq + Sd[i] - (((uint64_t)acc[i] << up) << 1);
      out[i] = (Key)key;
      mn = key < mn ? key : mn;
      mx = key > mx ? key : mx;
    }
  }
  // the row's smallest and largest key, for the selection that follows
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if (lane == 0) {
    red[0][w] = mn;
    red[1][w] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 1; j < QP_WAVES; ++j) {
      mn = red[0][j] < mn ? red[0][j] : mn;
      mx = red[1][j] > mx ? red[1][j] : mx;
    }
    atomicMin(&minmax[2 * row], mn);
    atomicMax(&minmax[2 * row + 1], mx);
  }
}

__global__ void k_zero_u32(uint32_t* __restrict__ p) { *p = 0u; }

__global__ void k_minmax_init(unsigned long long* __restrict__ minmax, int64_t rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) {
    minmax[2 * i] = ~0ull;
    minmax[2 * i + 1] = 0ull;
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

// The eps-weighted Quadtree (the tree of the proof of the uniform-distribution
// Flowtree upper bound: the edge above a depth-k cell weighs w[k] =
// (2^(B-k))^(1-eps)) of (query, doc) pairs, as
// sum_v w (a_v + b_v - 2 min(a_v, b_v)) over the cells of either side, in
// fp64 with integer masses; one wavefront per pair, the query table in LDS.
// Pairs: explicit (pair_q, pair_d), or query p / n_cols against
// cand[p].  Output: out_d (fp64) or out_f (fp32), in units of mass fraction
// x grid unit^(1-eps).
__global__ __launch_bounds__(64) void k_qt_eps(const int64_t* __restrict__ pair_q, const int64_t* __restrict__ pair_d,
                                               const int64_t* __restrict__ cand, int64_t n_cols, int64_t n_pairs,
                                               const int64_t* __restrict__ q_eoff, const uint32_t* __restrict__ q_ekey,
                                               const uint32_t* __restrict__ q_emass,
                                               const int64_t* __restrict__ d_eoff, const uint32_t* __restrict__ d_ekey,
                                               const uint32_t* __restrict__ d_emass, const double* __restrict__ w,
                                               int Q, double* __restrict__ out_d, float* __restrict__ out_f) {
  __shared__ uint32_t tk[8192];
  __shared__ uint32_t tm[8192];
  const int64_t p = blockIdx.x;
  if (p >= n_pairs) return;
  int64_t q, doc;
  if (pair_q) {
    q = pair_q[p];
    doc = pair_d[p];
  } else {
    q = p / n_cols;
    doc = cand[p];
  }
  const int64_t nq = q_eoff[q + 1] - q_eoff[q];
  int lg = 1;
  while ((1ll << lg) < 2 * nq) ++lg;
  QtTile tile{(int32_t)q, 1, lg, 0};
  qt_build_tables<8192>(tk, tm, tile, q_eoff, q_ekey, q_emass);
  double acc = 0.0;
  for (int64_t e = d_eoff[doc] + threadIdx.x; e < d_eoff[doc + 1]; e += 64) {
    const uint32_t key = d_ekey[e];
    const uint32_t a = d_emass[e], b = qt_lookup(tk, tm, lg, key);
    acc += w[key >> KEY_DEPTH_SHIFT] * ((double)a - 2.0 * (double)(a < b ? a : b));
  }
  for (int64_t e = q_eoff[q] + threadIdx.x; e < q_eoff[q + 1]; e += 64)
    acc += w[q_ekey[e] >> KEY_DEPTH_SHIFT] * (double)q_emass[e];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) {
    const double v = ldexp(acc, -Q);
    if (out_d) out_d[p] = v;
    else out_f[p] = (float)v;
  }
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

// The query hash tables in LDS hold at most SLOTS_LARGE / 2 cells of one
// query (load factor 1/2): FT_ERANGE for a query that touches more.
static void require_query_cells(ft_index* ix, int64_t n_q, hipStream_t s) {
  std::vector<int64_t> eoff(n_q + 1);
  FT_HIP(hipMemcpyAsync(eoff.data(), ix->qry.ecnt.p, (n_q + 1) * 8, hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
  for (int64_t q = 0; q < n_q; ++q)
    FT_REQUIRE(eoff[q + 1] - eoff[q] <= SLOTS_LARGE / 2, FT_ERANGE,
               "a query may touch at most 4096 tree cells here");
}

// Inverted doc lists for ranking all docs, made once per index.
static void prepare_postings(ft_index* ix, hipStream_t s) {
  if (ix->post_nsl > 0) return;
  const int64_t n = ix->docs.n;
  const bool narrow = post_narrow(ix->Q, ix->height);
  const int64_t S = post_slice_size(n, narrow ? QP_ACC_BYTES / 4 : QP_ACC_BYTES / 8), n_sl = ceil_div(n, S);
  const int64_t n_cells = std::max<int64_t>(1, ix->n_nodes - 1);
  FT_REQUIRE(n_sl * n_cells <= (int64_t(1) << 32), FT_ERANGE,
             "the inverted Quadtree lists would need more than 16 GiB of directory");
  uint32_t cb[32] = {0};
  for (int k = 2; k <= ix->height; ++k) cb[k] = cb[k - 1] + (uint32_t)ix->depth_nodes[k - 1];
  uint32_t* cbase = (uint32_t*)ix->post_cbase.ensure(sizeof(cb));
  FT_HIP(hipMemcpyAsync(cbase, cb, sizeof(cb), hipMemcpyHostToDevice, s));
  uint32_t* dir = (uint32_t*)ix->post_dir.ensure(n_sl * n_cells * 4);
  FT_HIP(hipMemsetAsync(dir, 0, n_sl * n_cells * 4, s));
  // list entries as two arrays: doc within the slice as the byte offset of
  // its counter (u16: 8192 docs x 4 bytes or 4096 x 8 at most) and cell mass
  // (u32), 6 bytes an entry
  const int64_t ne = std::max<int64_t>(1, ix->docs.emb_nnz);
  uint16_t* post_doc = (uint16_t*)ix->post.ensure(ne * 6 + 16);
  uint32_t* post_mass = (uint32_t*)((char*)ix->post.p + ((ne * 2 + 15) & ~int64_t(15)));
  const unsigned g = (unsigned)std::min<int64_t>(n, 1 << 20);
  k_post_count<<<g, 64, 0, s>>>(ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(), n, S, n_cells, cbase, dir);
  k_post_scan<<<(unsigned)n_sl, 1024, 0, s>>>(dir, n_cells);
  k_post_fill<<<(unsigned)n_sl, 64, 0, s>>>(ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(),
                                            ix->docs.emass.as<uint32_t>(), n, S, n_cells, cbase, dir, post_doc,
                                            post_mass, narrow ? 4u : 8u);
  FT_HIP(hipGetLastError());
  FT_HIP(hipStreamSynchronize(s));
  ix->post_slice = S;
  ix->post_cells = n_cells;
  ix->post_nsl = n_sl;
  // head cells: touched by at least half of the docs, the longest
  // first (ties by cell number), at most QP_HEAD_MAX; dense rows only with
  // narrow counters over full 8192-doc slices
  if (narrow && post_compact(ix->Q, ix->height)) {
    // compact keys: the docs' S in key units, 4 bytes per doc for the
    // ranking kernel's last pass instead of 8
    uint32_t* s32 = (uint32_t*)ix->post_s32.ensure(n * 4);
    k_s32<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(ix->docs.S.as<uint64_t>(), n, ix->B - ix->height, s32);
    FT_HIP(hipGetLastError());
  }
  ix->post_nhead = 0;
  if (!narrow || S != QP_HEAD_SLICE) return;
  std::vector<uint32_t> hdir(n_sl * n_cells);
  FT_HIP(hipMemcpy(hdir.data(), dir, hdir.size() * 4, hipMemcpyDeviceToHost));
  std::vector<int64_t> total(n_cells, 0);
  for (int64_t sl = 0; sl < n_sl; ++sl)
    for (int64_t c = 0; c < n_cells; ++c)
      total[c] += hdir[sl * n_cells + c] - (c ? hdir[sl * n_cells + c - 1] : 0u);
  std::vector<int64_t> cand;
  for (int64_t c = 0; c < n_cells; ++c)
    if (2 * total[c] >= n) cand.push_back(c);
  std::sort(cand.begin(), cand.end(), [&](int64_t a, int64_t b) {
    return total[a] != total[b] ? total[a] > total[b] : a < b;
  });
  if (cand.size() > (size_t)QP_HEAD_MAX) cand.resize(QP_HEAD_MAX);
  if (cand.empty()) return;
  const int nh = (int)cand.size();
  std::vector<uint8_t> hc(n_cells, 0xFFu);
  for (int h = 0; h < nh; ++h) hc[cand[h]] = (uint8_t)h;
  uint8_t* hcell = (uint8_t*)ix->post_hcell.ensure(n_cells);
  FT_HIP(hipMemcpy(hcell, hc.data(), n_cells, hipMemcpyHostToDevice));
  const size_t rows_bytes = (size_t)n_sl * nh * QP_HEAD_SLICE * 4;
  uint32_t* rows = (uint32_t*)ix->post_head.ensure(rows_bytes);
  FT_HIP(hipMemsetAsync(rows, 0, rows_bytes, s));
  k_head_fill<<<g, 64, 0, s>>>(ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(),
                              ix->docs.emass.as<uint32_t>(), n, cbase, hcell, nh, rows);
  FT_HIP(hipGetLastError());
  FT_HIP(hipStreamSynchronize(s));
  ix->post_nhead = nh;
}

}  // namespace ft

using namespace ft;

namespace ft {

// ft_quadtree_knn after its argument checks, on the prepared queries
// (ix->qry, with embedding) and checked candidate lists.
void quadtree_knn_prepared(ft_index* ix, int64_t n_q, const int64_t* cand, int32_t n_cand, int32_t k,
                           uint64_t* out_key, int64_t* out_doc, hipStream_t s) {
  const int64_t n_cols = cand ? (int64_t)n_cand : ix->docs.n;
  // the per-query cell counts size the candidate-list tables (all docs: not
  // needed, and not read back)
  std::vector<int64_t> eoff(n_q + 1);
  if (cand) {
    FT_HIP(hipMemcpyAsync(eoff.data(), ix->qry.ecnt.p, (n_q + 1) * 8, hipMemcpyDeviceToHost, s));
    FT_HIP(hipStreamSynchronize(s));
    for (int64_t q = 0; q < n_q; ++q)
      FT_REQUIRE(eoff[q + 1] - eoff[q] <= SLOTS_LARGE / 2, FT_ERANGE,
                 "with candidate lists, a query may touch at most 4096 tree cells");
  }
  // query chunks bound the key buffer to about 8 GiB (two of them: 16 GiB
  // of the 288 GB of HBM); two chunks of 2048 queries over 1M docs beat
  // four of 1024 and eight of 512 (fewer launches, one select tail)
  const bool compact = !cand && post_narrow(ix->Q, ix->height) && post_compact(ix->Q, ix->height);
  const int64_t key_bytes = compact ? 4 : 8;
  const int64_t rows_per_chunk =
      std::max<int64_t>(1, std::min<int64_t>(n_q, (int64_t(1) << 33) / key_bytes / n_cols));
  // Ranking all docs in several chunks runs each chunk's select on the
  // internal stream while the next chunk is ranked (they are bound by
  // different units), with two key buffers in turn.
  const bool pipe = !cand && rows_per_chunk < n_q;
  const int64_t chunk_bytes = (rows_per_chunk * n_cols * key_bytes + 255) & ~int64_t(255);
  char* key_base = (char*)ix->ws_keys.ensure(chunk_bytes * (pipe ? 2 : 1));
  uint64_t* keys = (uint64_t*)key_base;
  uint32_t* ckey_tmp = compact ? (uint32_t*)ix->ws_tiles.ensure(rows_per_chunk * k * 4) : nullptr;
  if (!cand) prepare_postings(ix, s);
  // per-chunk query preparation for ranking all docs: counts and head cells
  // per row, the other cells at the queries' own cell offsets
  uint2* qp_counts = nullptr;
  uint2* qp_head = nullptr;
  uint4* qp_listed = nullptr;
  if (!cand) {
    const int64_t hb = (rows_per_chunk * 8 + 255) & ~int64_t(255), hh = rows_per_chunk * QP_HEAD_MAX * 8;
    char* qp = (char*)ix->ws_misc.ensure(hb + hh + std::max<int64_t>(1, ix->qry.emb_nnz) * 16 + 16);
    qp_counts = (uint2*)qp;
    qp_head = (uint2*)(qp + hb);
    qp_listed = (uint4*)(qp + hb + hh);
  }
  hipStream_t s_sel = pipe ? ix->work : s;
  if (pipe) {
    FT_HIP(hipEventRecord(ix->ev_a, s));
    FT_HIP(hipStreamWaitEvent(s_sel, ix->ev_a, 0));
  }
  unsigned long long* minmax_base =
      cand ? nullptr : (unsigned long long*)ix->ws_sel.ensure(rows_per_chunk * 16 * (pipe ? 2 : 1));
  // the per-row key ranges start empty; with several chunks, the select
  // stream empties a buffer again right after its select has read it, so
  // no clearing kernel waits for a CU between two ranking launches
  if (minmax_base) {
    const int64_t mm_rows = rows_per_chunk * (pipe ? 2 : 1);
    k_minmax_init<<<(unsigned)ceil_div(mm_rows, 256), 256, 0, s>>>(minmax_base, mm_rows);
    FT_HIP(hipGetLastError());
  }
  // rows whose sampled select falls back to the exact path, counted
  uint32_t* sel_exact = (uint32_t*)ix->sel_exact.ensure(4);
  k_zero_u32<<<1, 1, 0, s>>>(sel_exact);
  FT_HIP(hipGetLastError());
  const int64_t n_chunks = ceil_div(n_q, rows_per_chunk);
  int64_t chunk = 0;
  for (int64_t r0 = 0; r0 < n_q; r0 += rows_per_chunk, ++chunk) {
    const int64_t r1 = std::min(n_q, r0 + rows_per_chunk);
    const int b = pipe ? (int)(chunk & 1) : 0;
    keys = (uint64_t*)(key_base + b * chunk_bytes);
    unsigned long long* minmax = nullptr;  // per-row key range, when the ranking kernel gives it
    if (!cand) {
      // all docs: the inverted lists, one workgroup per (query, slice)
      const int64_t rows = r1 - r0, groups = ceil_div(ix->post_nsl, 8);
      FT_REQUIRE(groups * 8 * rows < (int64_t(1) << 31), FT_ERANGE, "too many (query, slice) workgroups");
      minmax = minmax_base + b * rows_per_chunk * 2;
      // the buffers of chunk - 2 must have been read by its select (and
      // the key ranges emptied again)
      if (pipe && chunk >= 2) FT_HIP(hipStreamWaitEvent(s, ix->ev_sel[b], 0));
      // the chunk's queries split into head and listed cells, once
      k_qt_prep<<<(unsigned)rows, 256, 0, s>>>(
          ix->qry.ecnt.as<int64_t>(), ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(),
          ix->post_cbase.as<uint32_t>(), ix->post_nhead > 0 ? ix->post_hcell.as<uint8_t>() : nullptr,
          post_narrow(ix->Q, ix->height) ? ix->height : ix->B, r0, qp_counts, qp_head, qp_listed);
      auto go = [&](auto narrow, auto packed, auto head) {
        k_qt_post<decltype(narrow)::value, decltype(packed)::value, decltype(head)::value>
            <<<(unsigned)(groups * 8 * rows), QP_THREADS, 0, s>>>(
            ix->post.as<uint16_t>(),
            (const uint32_t*)((const char*)ix->post.p + ((std::max<int64_t>(1, ix->docs.emb_nnz) * 2 + 15) & ~int64_t(15))),
            ix->post_dir.as<uint32_t>(), ix->post_cbase.as<uint32_t>(), ix->post_head.as<uint32_t>(),
            ix->post_hcell.as<uint8_t>(), ix->post_nhead, ix->post_cells,
            ix->post_slice, ix->post_nsl, ix->docs.ecnt.as<int64_t>(), ix->docs.S.as<uint64_t>(),
            ix->post_s32.as<uint32_t>(), n_cols,
            ix->qry.ecnt.as<int64_t>(), ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(),
            ix->qry.S.as<uint64_t>(), r0, rows, ix->B, ix->height, keys, minmax, qp_counts, qp_head, qp_listed);
      };
      const bool head = ix->post_nhead > 0;
      if (compact && head) go(std::true_type{}, std::true_type{}, std::true_type{});
      else if (compact) go(std::true_type{}, std::true_type{}, std::false_type{});
      else if (post_narrow(ix->Q, ix->height) && head) go(std::true_type{}, std::false_type{}, std::true_type{});
      else if (post_narrow(ix->Q, ix->height)) go(std::true_type{}, std::false_type{}, std::false_type{});
      else go(std::false_type{}, std::false_type{}, std::false_type{});
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
    if (pipe) {
      FT_HIP(hipEventRecord(ix->ev_rank[b], s));
      FT_HIP(hipStreamWaitEvent(s_sel, ix->ev_rank[b], 0));
    }
    if (compact)
      topk_rows(reinterpret_cast<const uint32_t*>(keys), r1 - r0, n_cols, nullptr, k, out_key + r0 * k,
                ix->B - ix->height, out_doc + r0 * k, ckey_tmp, s_sel, reinterpret_cast<const uint64_t*>(minmax),
                sel_exact);
    else
      topk_rows(keys, r1 - r0, n_cols, cand ? cand + r0 * n_cols : nullptr, k, out_key + r0 * k, out_doc + r0 * k,
                s_sel, reinterpret_cast<const uint64_t*>(minmax), sel_exact);
    if (minmax && pipe && chunk + 2 < n_chunks) {
      k_minmax_init<<<(unsigned)ceil_div(rows_per_chunk, 256), 256, 0, s_sel>>>(minmax, rows_per_chunk);
      FT_HIP(hipGetLastError());
    }
    if (pipe) FT_HIP(hipEventRecord(ix->ev_sel[b], s_sel));
  }
  if (pipe) {
    FT_HIP(hipEventRecord(ix->ev_b, s_sel));
    FT_HIP(hipStreamWaitEvent(s, ix->ev_b, 0));
  }
}

}  // namespace ft

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
    quadtree_knn_prepared(ix, n_q, cand, n_cand, k, out_key, out_doc, s);
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
    require_query_cells(ix, n_q, s);
    k_qt_pairs<<<(unsigned)n_pairs, 64, 0, s>>>(pair_q, pair_d, n_pairs, ix->qry.ecnt.as<int64_t>(),
                                               ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(),
                                               ix->qry.S.as<uint64_t>(), ix->docs.ecnt.as<int64_t>(),
                                               ix->docs.ekey.as<uint32_t>(), ix->docs.emass.as<uint32_t>(),
                                               ix->docs.S.as<uint64_t>(), ix->B, out_key);
    FT_HIP(hipGetLastError());
  });
}

// Edge weights (2^(B-k))^(1-eps) for depths k = 0..B, on the device.
static const double* eps_weights(ft_index* ix, double eps, hipStream_t s) {
  std::vector<double> w(ix->B + 1);
  for (int k = 0; k <= ix->B; ++k) w[k] = std::pow(2.0, (double)(ix->B - k) * (1.0 - eps));
  double* d = (double*)ix->ws_misc.ensure(w.size() * sizeof(double));
  FT_HIP(hipMemcpyAsync(d, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s));
  FT_HIP(hipStreamSynchronize(s));
  return d;
}

extern "C" ft_status ft_quadtree_eps_pairs(ft_index* ix, const int64_t* q_off, const uint32_t* q_id,
                                           const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                                           const int64_t* pair_d, int64_t n_pairs, double eps, double* out,
                                           void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && pair_q && pair_d && out, FT_EINVAL, "NULL argument");
    FT_REQUIRE(n_pairs >= 0, FT_EINVAL, "n_pairs < 0");
    FT_REQUIRE(eps >= 0.0 && eps <= 1.0, FT_EINVAL, "eps must lie in [0, 1]");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, true, s, "queries");
    check_indices(ix, pair_q, n_pairs, n_q, s, "pair_q");
    check_indices(ix, pair_d, n_pairs, ix->docs.n, s, "pair_d");
    if (n_pairs == 0) return;
    require_query_cells(ix, n_q, s);
    const double* w = eps_weights(ix, eps, s);
    k_qt_eps<<<(unsigned)n_pairs, 64, 0, s>>>(pair_q, pair_d, nullptr, 1, n_pairs, ix->qry.ecnt.as<int64_t>(),
                                             ix->qry.ekey.as<uint32_t>(), ix->qry.emass.as<uint32_t>(),
                                             ix->docs.ecnt.as<int64_t>(), ix->docs.ekey.as<uint32_t>(),
                                             ix->docs.emass.as<uint32_t>(), w, ix->Q, out, nullptr);
    FT_HIP(hipGetLastError());
    FT_HIP(hipStreamSynchronize(s));
  });
}

extern "C" ft_status ft_quadtree_eps_knn(ft_index* ix, const int64_t* q_off, const uint32_t* q_id,
                                         const uint32_t* q_mass, int64_t n_q, const int64_t* cand, int32_t n_cand,
                                         double eps, int32_t k, float* out_cost, int64_t* out_doc, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && cand && out_cost && out_doc, FT_EINVAL, "NULL argument");
    FT_REQUIRE(eps >= 0.0 && eps <= 1.0, FT_EINVAL, "eps must lie in [0, 1]");
    FT_REQUIRE(n_cand >= 1 && n_cand <= 4096, FT_ERANGE, "n_cand must lie in [1, 4096]");
    FT_REQUIRE(k >= 1 && k <= n_cand, FT_EINVAL, "k must lie in [1, n_cand]");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, true, s, "queries");
    check_indices(ix, cand, n_q * n_cand, ix->docs.n, s, "cand");
    require_query_cells(ix, n_q, s);
    const double* w = eps_weights(ix, eps, s);
    const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(n_q, (int64_t(1) << 28) / n_cand));
    float* cost = (float*)ix->ws_cost.ensure(rows * n_cand * 4);
    for (int64_t r0 = 0; r0 < n_q; r0 += rows) {
      const int64_t r1 = std::min(n_q, r0 + rows);
      const int64_t np = (r1 - r0) * n_cand;
      k_qt_eps<<<(unsigned)np, 64, 0, s>>>(nullptr, nullptr, cand + r0 * n_cand, n_cand, np,
                                          ix->qry.ecnt.as<int64_t>() + r0, ix->qry.ekey.as<uint32_t>(),
                                          ix->qry.emass.as<uint32_t>(), ix->docs.ecnt.as<int64_t>(),
                                          ix->docs.ekey.as<uint32_t>(), ix->docs.emass.as<uint32_t>(), w, ix->Q,
                                          nullptr, cost);
      FT_HIP(hipGetLastError());
      topk_rows(cost, r1 - r0, n_cand, cand + r0 * n_cand, k, out_cost + r0 * k, out_doc + r0 * k, s);
    }
    FT_HIP(hipStreamSynchronize(s));
  });
}

extern "C" ft_status ft_last_quadtree_stats(const ft_index* ix, int64_t* select_exact_rows) {
  return guarded([&] {
    FT_REQUIRE(ix && select_exact_rows, FT_EINVAL, "NULL argument");
    uint32_t v = 0;
    if (ix->sel_exact.p) FT_HIP(hipMemcpy(&v, ix->sel_exact.p, 4, hipMemcpyDeviceToHost));
    *select_exact_rows = v;
  });
}
