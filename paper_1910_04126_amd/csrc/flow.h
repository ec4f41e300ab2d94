// Flowtree for one (query, doc) pair on one wavefront (paper Section 3 and
// Appendix A.1).
//
// The greedy processes cells bottom-up; a cell matches the unmatched doc
// (mu) and query (nu) mass collected from its children and passes the rest
// up.  Listing both supports in Morton order makes every cell a contiguous
// run of the merged item list, and the cells of one depth k are the maximal
// runs whose adjacent LCA depths are >= k.  Cells of equal depth are
// disjoint, so a whole depth is processed at once:
//   * inclusive segmented prefix sums P+ (doc mass) and P- (query mass);
//   * with M = min(total P+, total P-) of the run, the front-to-front
//     matching of the run's doc items against its query items (both in
//     Morton order) pairs the overlaps of the intervals [P - r, P) inside
//     [0, M): every such overlap starts at some item's interval start, so
//     each item finds the match starting at its own interval start by one
//     binary search on the other side's prefix sums (a doc item wins a tie);
//   * an item keeps the part of its interval beyond M.
// Only depths that occur among the adjacent LCA depths (plus the root) can
// change anything; the others are skipped.
//
// Layout: a workgroup of W wavefronts owns NMAX = 64 * W * C merged items,
// thread t the items [t*C, t*C + C); per-item state lives in LDS.  Scans run
// per wavefront with DPP/shuffles, and their carries cross wavefronts through
// one LDS slot per wavefront, so large pairs spread over several wavefronts
// instead of crowding one.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "common.h"
#include "wave.h"

namespace ft {

template <int C, int W = 1>
struct FlowLds {
  static constexpr int N = 64 * C * W;
  int64_t work;        // persistent kernels: the grabbed chunk, broadcast
  uint32_t rank[N];    // merged Morton ranks
  uint32_t pp[N];      // doc-side inclusive prefix (before the merge: input ranks)
  uint32_t pn[N];      // query-side inclusive prefix (before the merge: input masses)
  uint32_t em_pos[N];  // match: merged position of the doc item | query item << 16
  uint32_t em_eta[N];  // match: integer mass moved
  uint16_t slot[N];    // merged position -> input slot (query [0, nq), doc [nq, nq + nd))
  int8_t lcn[N];       // LCA depth of (t, t + 1); -1 after the last item
  // one slot per wavefront for cross-wavefront scan carries
  uint32_t x_p[W], x_n[W], x_f[W], x_c[W], x_m[W];
  int32_t x_s[W], x_e[W];
};

// Where a saved flow goes (gradient and inspection paths).
struct FlowSave {
  uint32_t* id;     // doc slot << 16 | query slot (slots inside each sorted support)
  uint32_t* eta;
  uint64_t* key;    // (31 - depth) << 48 | segment start << 32 | interval start
  uint8_t* bind;    // 0: doc item used up, 1: query item, 2: both
  int64_t base;
};

// Stage a pair: query items into slots [0, nq), doc items into [nq, nq + nd).
template <int C, int W>
__device__ __forceinline__ void flow_stage(FlowLds<C, W>& L, const uint32_t* __restrict__ qr,
                                           const uint32_t* __restrict__ qm, int nq,
                                           const uint32_t* __restrict__ dr,
                                           const uint32_t* __restrict__ dm, int nd) {
  const int tid = threadIdx.x;
  for (int i = tid; i < nq; i += 64 * W) {
    L.pp[i] = qr[i];
    L.pn[i] = qm[i];
  }
  for (int i = tid; i < nd; i += 64 * W) {
    L.pp[nq + i] = dr[i];
    L.pn[nq + i] = dm[i];
  }
  __syncthreads();
}

// The greedy flow of a staged pair; returns the number of matches in
// L.em_pos / L.em_eta (uniform across the workgroup).  Without SAVE the list
// leaves out the matches between equal ranks, whose distance is 0.
template <int C, int W, bool SAVE>
__device__ int flow_match(FlowLds<C, W>& L, const int nq, const int nd, const uint8_t* __restrict__ st,
                          const int64_t V, const int B, FlowSave sv, uint32_t* __restrict__ status) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n = nq + nd;
  const int t0 = tid * C;
  // A thread's own items t0 + c keep their state in registers across the
  // depths: unmatched mass, side, and the LCA depth with the next item.
  uint32_t res[C];
  bool isq[C];
  int lcn[C];
  // ---- merge both supports by rank (doc first on equal ranks)
  {
    const uint32_t* qr = L.pp;
    const uint32_t* dr = L.pp + nq;
    const int k0 = min(t0, n);
    int lo = max(0, k0 - nq), hi = min(k0, nd);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (dr[mid] <= qr[k0 - mid - 1]) lo = mid + 1;
      else hi = mid;
    }
    int j = lo, i = k0 - lo;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = t0 + c;
      res[c] = 0u;
      isq[c] = false;
      if (t < n) {
        const bool take_d = j < nd && (i >= nq || dr[j] <= qr[i]);
        const int s = take_d ? nq + j : i;
        if (take_d) ++j;
        else ++i;
        L.rank[t] = L.pp[s];
        res[c] = L.pn[s];
        isq[c] = !take_d;
        L.slot[t] = (uint16_t)s;
      }
    }
  }
  __syncthreads();
  // ---- adjacent LCA depths and the depths present: all range-minimum reads
  // of a lane are issued before any is used
  uint32_t mask = 1u;
  {
    int64_t ia[C], ib[C];
    uint8_t va[C], vb[C];
    bool same[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = t0 + c;
      const bool valid = t + 1 < n;
      const uint32_t ra = valid ? L.rank[t] : 0u, rb = valid ? L.rank[t + 1] : 0u;
      const uint32_t len = rb - ra;  // Morton order: ra <= rb
      same[c] = len == 0u;
      const int j = same[c] ? 0 : 31 - __clz(len);
      ia[c] = (int64_t)j * V + ra;
      ib[c] = (int64_t)j * V + (rb - (same[c] ? 0u : (1u << j)));
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      va[c] = st[ia[c]];
      vb[c] = st[ib[c]];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = t0 + c;
      int l = -1;
      if (t + 1 < n) {
        l = same[c] ? B : (va[c] < vb[c] ? va[c] : vb[c]);
        mask |= 1u << l;
      }
      lcn[c] = l;
      if (t < n) L.lcn[t] = (int8_t)l;
    }
  }
  mask = wave_or(mask);
  if (W > 1) {
    if (lane == 0) L.x_m[w] = mask;
  }
  __syncthreads();
  if (W > 1)
    for (int j = 0; j < W; ++j) mask |= L.x_m[j];
  // LCA depth of the item before this thread's first (-1 for item 0: every
  // depth starts a segment there)
  const int lcn_prev = (t0 > 0 && t0 <= n) ? (int)L.lcn[t0 - 1] : -1;
  int E = 0;
  while (mask) {
    const int k = 31 - __clz(mask);
    mask &= ~(1u << k);
    // local segmented sums of this lane's items
    // (items past n are neutral: no mass, and each starts and ends its own
    // segment after every real one, so no test of t < n is needed)
    uint32_t run_p = 0, run_n = 0;
    int last_start = -1, first_end = 0x7FFFFFFF;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = t0 + c;
      if ((c ? lcn[c - 1] : lcn_prev) < k) {
        run_p = run_n = 0;
        last_start = t;
      }
      if (isq[c]) run_n += res[c];
      else run_p += res[c];
      if (lcn[c] < k && first_end == 0x7FFFFFFF) first_end = t;
    }
    uint32_t tp = run_p, tn = run_n;
    const bool has = wave_seg_incl_sum2(tp, tn, last_start >= 0);
    const int ls_incl = wave_incl_max(last_start);
    const int fe_suf = wave_suffix_min(first_end);
    // carries from the other wavefronts: the segmented sums reaching this
    // wavefront's first lane, the latest segment start before it, and the
    // earliest segment end after it
    uint32_t kp = 0, kn = 0;
    int ks = 0, ke = 0x7FFFFFFF;
    if (W > 1) {
      if (lane == 63) {
        L.x_p[w] = tp;
        L.x_n[w] = tn;
        L.x_f[w] = has ? 1u : 0u;
        L.x_s[w] = ls_incl;
      }
      if (lane == 0) L.x_e[w] = fe_suf;
      __syncthreads();
      for (int j = w - 1; j >= 0; --j) {
        kp += L.x_p[j];
        kn += L.x_n[j];
        if (L.x_f[j]) break;
      }
      for (int j = 0; j < w; ++j) ks = max(ks, L.x_s[j]);
      for (int j = w + 1; j < W; ++j) ke = min(ke, L.x_e[j]);
      if (!has) {
        tp += kp;
        tn += kn;
      }
    }
    // exclusive carries: lane 0 takes the other wavefronts', lane 63's next
    // end comes from them
    uint32_t cp = wave_shr1(tp, kp), cn = wave_shr1(tn, kn);
    int prev_start = max(ks, wave_shr1(ls_incl, ks));
    int next_end = min(ke, wave_shl1(fe_suf, ke));
    if (lane == 0) {
      cp = kp;
      cn = kn;
      prev_start = ks;
    }
    if (lane == 63) next_end = ke;
    // inclusive prefixes with the carry from earlier lanes, into LDS for the
    // searches of other items and into registers for this lane's own
    uint32_t hi[C];
    int a0[C], e0[C];
    run_p = cp;
    run_n = cn;
    int s0 = prev_start;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = t0 + c;
      if ((c ? lcn[c - 1] : lcn_prev) < k) {
        run_p = run_n = 0;
        s0 = t;
      }
      if (isq[c]) run_n += res[c];
      else run_p += res[c];
      L.pp[t] = run_p;  // t < N always; past n the values are never read
      L.pn[t] = run_n;
      hi[c] = isq[c] ? run_n : run_p;
      a0[c] = s0;
    }
    {
      int e = next_end;
#pragma unroll
      for (int c = C - 1; c >= 0; --c) {
        if (lcn[c] < k) e = t0 + c;
        e0[c] = e;
      }
    }
    __syncthreads();
    // each item with mass left finds the match that starts at its own
    // interval start: the first item of the other side in its segment whose
    // inclusive prefix exceeds that start.  The searches of a lane's items run
    // side by side, a fixed number of halvings each (branch-free lower bound
    // over [a0, e0], whose last prefix, the side's total, exceeds the start).
    uint32_t lo[C], M[C];
    int base[C], len[C];
    bool want[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const uint32_t Tp = L.pp[e0[c]], Tn = L.pn[e0[c]];
      M[c] = Tp < Tn ? Tp : Tn;
      lo[c] = hi[c] - res[c];
      want[c] = res[c] > 0u && lo[c] < M[c];
      base[c] = a0[c];
      len[c] = want[c] ? e0[c] - a0[c] + 1 : 1;
    }
    int span = 1;
#pragma unroll
    for (int c = 0; c < C; ++c) span = max(span, len[c]);
    span = lane_value(wave_incl_max(span), 63);
    while (span > 1) {
      uint32_t v[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int half = len[c] >> 1;
        const uint32_t* opp = isq[c] ? L.pp : L.pn;
        v[c] = opp[base[c] + (half > 0 ? half - 1 : 0)];
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int half = len[c] >> 1;
        if (half > 0 && v[c] <= lo[c]) base[c] += half;
        len[c] -= half;
      }
      span -= span >> 1;
    }
    // the match found: a query item yields to a doc item that starts at the
    // same point (that doc item owns the match)
    uint32_t m_pos[C], m_eta[C];
    uint8_t m_bind[C];
    int cnt = 0;
    {
      uint32_t ho[C], lp[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int p = base[c];
        const uint32_t* opp = isq[c] ? L.pp : L.pn;
        ho[c] = opp[p];
        lp[c] = L.pp[p > a0[c] ? p - 1 : p];
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int t = t0 + c, p = base[c];
        m_eta[c] = 0;
        m_pos[c] = 0;
        m_bind[c] = 0;
        bool own = want[c];
        if (isq[c]) own = own && (p == a0[c] ? 0u : lp[c]) != lo[c];
        // pricing-only runs drop a match between equal ranks (distance 0);
        // only a segment of depth B can hold one
        if (!SAVE && k == B && own) own = L.rank[t] != L.rank[p];
        if (own) {
          uint32_t end = hi[c] < ho[c] ? hi[c] : ho[c];
          end = end < M[c] ? end : M[c];
          m_eta[c] = end - lo[c];
          m_pos[c] = isq[c] ? ((uint32_t)p | ((uint32_t)t << 16)) : ((uint32_t)t | ((uint32_t)p << 16));
          if (SAVE) {
            const uint32_t hd = isq[c] ? ho[c] : hi[c], hq = isq[c] ? hi[c] : ho[c];
            m_bind[c] = (end == hd && end == hq) ? 2 : (end == hd ? 0 : 1);
          }
          ++cnt;
        }
        if (res[c] > 0u) res[c] = hi[c] > M[c] ? hi[c] - (lo[c] > M[c] ? lo[c] : M[c]) : 0u;
      }
    }
    const int incl = wave_incl_sum(cnt);
    int before = 0, total;
    if (W > 1) {
      if (lane == 63) L.x_c[w] = (uint32_t)incl;
      __syncthreads();
      total = 0;
      for (int j = 0; j < W; ++j) {
        if (j < w) before += (int)L.x_c[j];
        total += (int)L.x_c[j];
      }
    } else {
      total = lane_value(incl, 63);
    }
    int off = E + before + incl - cnt;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (m_eta[c]) {
        L.em_pos[off] = m_pos[c];
        L.em_eta[off] = m_eta[c];
        if (SAVE) {
          const int64_t g = sv.base + off;
          const uint32_t pd = m_pos[c] & 0xFFFFu, pq = m_pos[c] >> 16;
          sv.id[g] = ((uint32_t)(L.slot[pd] - nq) << 16) | (uint32_t)L.slot[pq];
          sv.eta[g] = m_eta[c];
          sv.key[g] = ((uint64_t)(31 - k) << 48) | ((uint64_t)a0[c] << 32) | lo[c];
          sv.bind[g] = m_bind[c];
        }
        ++off;
      }
    }
    E += total;
    // no barrier here: the next depth's first one (W > 1) precedes its
    // prefix writes, and one wavefront reads its own LDS writes in order
  }
  __syncthreads();  // the match list is complete
  // every unit of mass must have been matched by the root
  bool left = false;
#pragma unroll
  for (int c = 0; c < C; ++c)
    if (res[c] != 0u) left = true;
  if (__ballot(left) && lane == 0) atomicOr(status, ERR_FLOW);
  return E;
}

// Sum over aligned groups of G lanes (G <= 16, inside one DPP row of 16),
// left in every lane of the group: neighbours, then pairs of neighbours by
// quad permutes, then halves and whole rows by mirrors.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

template <int G>
__device__ __forceinline__ float group_sum(float v) {
  static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "G must be a power of two <= 16");
  if (G >= 2) v += dpp_f32<0xB1>(v);   // quad_perm [1,0,3,2]
  if (G >= 4) v += dpp_f32<0x4E>(v);   // quad_perm [2,3,0,1]
  if (G >= 8) v += dpp_f32<0x141>(v);  // row_half_mirror
  if (G >= 16) v += dpp_f32<0x140>(v); // row_mirror
  return v;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over each row of 16 lanes, left in every lane of the row.
__device__ __forceinline__ double row_sum_f64(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return v;
}

// Pairs of matches that share the item of the smaller side (by_doc: the doc
// item): a counting sort in LDS (pp and slot are free once the matching is
// done) groups the matches by that item, each item's run padded to even
// length, and unit u is the two entries ord[2u], ord[2u + 1] of L.slot (the
// second 0xFFFF when the run was odd).  The padded order needs up to
// (n - 1) + n / 2 entries (at most n - 1 matches, at most n / 2 odd runs):
// slot and the byte array after it (both dead by now) hold 1.5 N.  Returns
// the number of units, uniform across the workgroup.
template <int C, int W>
__device__ int pair_units(FlowLds<C, W>& L, const int E, const int n, const bool by_doc,
                          uint32_t* __restrict__ status) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  using Lds = FlowLds<C, W>;
  static_assert(offsetof(Lds, lcn) == offsetof(Lds, slot) + 2 * Lds::N, "slot and lcn must be adjacent");
  uint32_t* cnt = L.pp;  // the prefix sums are dead, the products not yet written
  uint16_t* ord = L.slot;
  constexpr uint16_t NONE = 0xFFFFu;
  for (int i = tid; i < n; i += 64 * W) cnt[i] = 0u;
  __syncthreads();
  for (int e = tid; e < E; e += 64 * W) {
    const uint32_t pos = L.em_pos[e];
    atomicAdd(&cnt[by_doc ? (pos & 0xFFFFu) : (pos >> 16)], 1u);
  }
  __syncthreads();
  int units;
  {
    // exclusive scan of the even-rounded counts: thread t holds [t*C, t*C + C)
    const int t0 = tid * C;
    uint32_t v[C], tot = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      v[c] = t0 + c < n ? (cnt[t0 + c] + 1u) & ~1u : 0u;
      tot += v[c];
    }
    const uint32_t incl = wave_incl_sum(tot);
    uint32_t base = incl - tot;
    uint32_t all = __shfl(incl, 63, 64);
    if (W > 1) {
      if (lane == 63) L.x_c[w] = incl;
      __syncthreads();
      all = 0;
      for (int j = 0; j < W; ++j) {
        if (j < w) base += L.x_c[j];
        all += L.x_c[j];
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (t0 + c < n) cnt[t0 + c] = base;
      base += v[c];
    }
    units = (int)(all >> 1);
  }
  if (2 * units > 3 * FlowLds<C, W>::N / 2) {
    // cannot happen (the bound above); never overrun, report it instead
    if (tid == 0) atomicOr(status, ERR_FLOW);
    units = 0;
  }
  for (int i = tid; i < 2 * units; i += 64 * W) ord[i] = NONE;
  __syncthreads();
  for (int e = tid; e < E; e += 64 * W) {
    const uint32_t pos = L.em_pos[e];
    ord[atomicAdd(&cnt[by_doc ? (pos & 0xFFFFu) : (pos >> 16)], 1u)] = (uint16_t)e;
  }
  __syncthreads();
  return units;
}

// The sum of the E per-match products in an order that depends on E only:
// lane j of wavefront 0 adds the products j, j + 64, ... in turn, then the 64
// lane sums are combined by a fixed tree (rows of 16 by DPP, then the four
// rows).  Valid in wavefront 0.
__device__ __forceinline__ double sum_products(const double* prod, const int E) {
  double cost = 0.0;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    for (int e0 = lane; e0 < E; e0 += 4 * 64) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = e0 + 64 * u < E ? prod[e0 + 64 * u] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) cost += v[u];
    }
    cost = row_sum_f64(cost);
    cost = (__shfl(cost, 0, 64) + __shfl(cost, 16, 64)) + (__shfl(cost, 32, 64) + __shfl(cost, 48, 64));
  }
  return cost;
}

// Euclidean price of the matches: sum eta * ||x_doc - x_query||_2 (float32
// distances, float64 accumulation).  G lanes share one match, and a lane
// reads up to PV float4 (or floats when VEC == 1) of each row per pass, all
// issued before any is used.  Each match's product lands in LDS (over the
// prefix arrays, free by now) and wavefront 0 adds them up in an order fixed
// by the number of matches alone, so a cost does not depend on W, G or the
// schedule.  The result is valid in wavefront 0.
template <int C, int W, int G, int VEC>
__device__ double flow_price(FlowLds<C, W>& L, const int E, const int nq, const int nd, const float* __restrict__ X,
                             const uint32_t* __restrict__ row_of_rank, const int stride, const int d,
                             uint32_t* __restrict__ status) {
  constexpr int PER = 64 * W / G;
  constexpr int PV = C * W >= 8 ? 5 : 2;
  using V4 = typename std::conditional<VEC == 4, float4, float>::type;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = tid / G, sub = tid % G;
  const int nv = VEC == 4 ? stride >> 2 : d;
  const int n = nq + nd;
  double* prod = reinterpret_cast<double*>(L.pp);  // pp and pn are contiguous: 8 * N bytes
  if constexpr (C * W < 4) {
    // short pairs: one match per lane group, in match order
    for (int e0 = 0; e0 < E; e0 += PER) {
      const int e = e0 + g;
      const V4* pa = nullptr;
      const V4* pb = nullptr;
      uint32_t eta = 0;
      bool live = false;
      if (e < E) {
        const uint32_t pos = L.em_pos[e];
        const uint32_t rd = L.rank[pos & 0xFFFFu], rq = L.rank[pos >> 16];
        eta = L.em_eta[e];
        live = rd != rq;
        const int64_t rowd = row_of_rank ? row_of_rank[rd] : rd;
        const int64_t rowq = row_of_rank ? row_of_rank[rq] : rq;
        pa = reinterpret_cast<const V4*>(X + rowd * stride);
        pb = reinterpret_cast<const V4*>(X + rowq * stride);
      }
      float acc = 0.0f;
      for (int v0 = 0; v0 < nv; v0 += G * PV) {
        V4 xa[PV], xb[PV];
#pragma unroll
        for (int t = 0; t < PV; ++t) {
          const int v = v0 + t * G + sub;
          const bool in = live && v < nv;
          xa[t] = in ? pa[v] : V4{};
          xb[t] = in ? pb[v] : V4{};
        }
#pragma unroll
        for (int t = 0; t < PV; ++t) {
          if constexpr (VEC == 4) {
            const float dx = xa[t].x - xb[t].x, dy = xa[t].y - xb[t].y;
            const float dz = xa[t].z - xb[t].z, dw = xa[t].w - xb[t].w;
            acc += dx * dx + dy * dy + dz * dz + dw * dw;
          } else {
            const float dx = xa[t] - xb[t];
            acc += dx * dx;
          }
        }
      }
      acc = group_sum<G>(acc);
      if (sub == 0 && e < E) prod[e] = live ? (double)eta * (double)sqrtf(acc) : 0.0;
    }
  } else {
    // Matches are priced two at a time that share the item of the smaller
    // side (pair_units), and a lane group reads the shared row once for both
    // (three rows for two matches).  Products stay indexed by match.
    const bool by_doc = nd <= nq;
    const int units = pair_units(L, E, n, by_doc, status);
    const uint16_t* ord = L.slot;
    constexpr uint16_t NONE = 0xFFFFu;
    for (int u0 = 0; u0 < units; u0 += PER) {
      const int u = u0 + g;
      int e1 = E, e2 = E;
      if (u < units) {
        e1 = ord[2 * u];  // a run starts at an even slot, so the first is a match
        const uint16_t o2 = ord[2 * u + 1];
        e2 = o2 == NONE ? E : (int)o2;
      }
      const V4* ps = nullptr;
      const V4* p1 = nullptr;
      const V4* p2 = nullptr;
      uint32_t eta1 = 0, eta2 = 0;
      bool live1 = false, live2 = false;
      if (e1 < E) {
        const uint32_t pos = L.em_pos[e1];
        const uint32_t rd = L.rank[pos & 0xFFFFu], rq = L.rank[pos >> 16];
        eta1 = L.em_eta[e1];
        live1 = rd != rq;
        const uint32_t rs = by_doc ? rd : rq, ro = by_doc ? rq : rd;
        const int64_t rows = row_of_rank ? row_of_rank[rs] : rs;
        const int64_t rowo = row_of_rank ? row_of_rank[ro] : ro;
        ps = reinterpret_cast<const V4*>(X + rows * stride);
        p1 = reinterpret_cast<const V4*>(X + rowo * stride);
      }
      if (e2 < E) {
        const uint32_t pos = L.em_pos[e2];
        const uint32_t rd = L.rank[pos & 0xFFFFu], rq = L.rank[pos >> 16];
        eta2 = L.em_eta[e2];
        live2 = rd != rq;
        const uint32_t ro = by_doc ? rq : rd;
        const int64_t rowo = row_of_rank ? row_of_rank[ro] : ro;
        p2 = reinterpret_cast<const V4*>(X + rowo * stride);
      }
      const bool lives = live1 || live2;
      float acc1 = 0.0f, acc2 = 0.0f;
      for (int v0 = 0; v0 < nv; v0 += G * PV) {
        V4 xs[PV], x1[PV], x2[PV];
#pragma unroll
        for (int t = 0; t < PV; ++t) {
          const int v = v0 + t * G + sub;
          const bool in = v < nv;
          xs[t] = lives && in ? ps[v] : V4{};
          x1[t] = live1 && in ? p1[v] : V4{};
          x2[t] = live2 && in ? p2[v] : V4{};
        }
#pragma unroll
        for (int t = 0; t < PV; ++t) {
          if constexpr (VEC == 4) {
            float dx = xs[t].x - x1[t].x, dy = xs[t].y - x1[t].y, dz = xs[t].z - x1[t].z, dw = xs[t].w - x1[t].w;
            acc1 += dx * dx + dy * dy + dz * dz + dw * dw;
            dx = xs[t].x - x2[t].x, dy = xs[t].y - x2[t].y, dz = xs[t].z - x2[t].z, dw = xs[t].w - x2[t].w;
            acc2 += dx * dx + dy * dy + dz * dz + dw * dw;
          } else {
            const float d1 = xs[t] - x1[t], d2 = xs[t] - x2[t];
            acc1 += d1 * d1;
            acc2 += d2 * d2;
          }
        }
      }
      acc1 = group_sum<G>(acc1);
      acc2 = group_sum<G>(acc2);
      if (sub == 0) {
        if (e1 < E) prod[e1] = live1 ? (double)eta1 * (double)sqrtf(acc1) : 0.0;
        if (e2 < E) prod[e2] = live2 ? (double)eta2 * (double)sqrtf(acc2) : 0.0;
      }
    }
  }
  __syncthreads();
  return sum_products(prod, E);
}

// squared distance of two float4 slices added to acc, one fma per component
__device__ __forceinline__ float dist2_acc(float acc, const float4 a, const float4 b) {
  const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, dw = a.w - b.w;
  acc = fmaf(dx, dx, acc);
  acc = fmaf(dy, dy, acc);
  acc = fmaf(dz, dz, acc);
  return fmaf(dw, dw, acc);
}

// flow_price over the index's own coordinate copy: row r of X (Morton rank r)
// holds `stride` floats, zero past d, with stride a multiple of 4 G, so each
// lane of a group reads exactly stride / (4 G) float4 of a row and no load
// needs a bound check; and the match list (flow_match without SAVE) holds no
// zero-distance match, so no match is skipped.  A lane group that has no
// match in a pass branches around its loads.  The square root is the
// hardware one (at most 1 ulp from the rounded root, 22 fewer instructions
// per match).  Products and their sum as in flow_price.
template <int C, int W, int G>
__device__ double flow_price_tiled(FlowLds<C, W>& L, const int E, const int nq, const int nd,
                                   const float* __restrict__ X, const int stride, uint32_t* __restrict__ status) {
  constexpr int PER = 64 * W / G;
  constexpr int PV = C * W >= 8 ? 5 : 2;
  const int tid = threadIdx.x;
  const int g = tid / G, sub = tid % G;
  const int per = stride / (4 * G);  // float4 per lane per row
  const int n = nq + nd;
  double* prod = reinterpret_cast<double*>(L.pp);
  if constexpr (C * W < 4) {
    // short pairs: one match per lane group, in match order
    for (int e0 = 0; e0 < E; e0 += PER) {
      const int e = e0 + g;
      float acc = 0.0f;
      if (e < E) {
        const uint32_t pos = L.em_pos[e];
        const float4* pa = reinterpret_cast<const float4*>(X + (int64_t)L.rank[pos & 0xFFFFu] * stride) + sub;
        const float4* pb = reinterpret_cast<const float4*>(X + (int64_t)L.rank[pos >> 16] * stride) + sub;
        for (int b = 0; b < per; b += PV) {
          float4 xa[PV], xb[PV];
#pragma unroll
          for (int t = 0; t < PV; ++t)
            if (b + t < per) {
              xa[t] = pa[(b + t) * G];
              xb[t] = pb[(b + t) * G];
            }
#pragma unroll
          for (int t = 0; t < PV; ++t)
            if (b + t < per) acc = dist2_acc(acc, xa[t], xb[t]);
        }
      }
      acc = group_sum<G>(acc);
      if (sub == 0 && e < E) prod[e] = (double)L.em_eta[e] * (double)__builtin_amdgcn_sqrtf(acc);
    }
  } else {
    // two matches that share the item of the smaller side per lane group
    // (pair_units); a unit that holds one match (the end of an odd run) reads
    // the shared row in place of a second row, so every lane loads the same
    // three rows (a masked third load measured slower) and the second sum, 0,
    // is not stored
    const bool by_doc = nd <= nq;
    const int units = pair_units(L, E, n, by_doc, status);
    const uint16_t* ord = L.slot;
    for (int u0 = 0; u0 < units; u0 += PER) {
      const int u = u0 + g;
      int e1 = E, e2 = E;
      float acc1 = 0.0f, acc2 = 0.0f;
      if (u < units) {
        e1 = ord[2 * u];
        const uint16_t o2 = ord[2 * u + 1];
        e2 = o2 == 0xFFFFu ? E : (int)o2;
        const uint32_t pos1 = L.em_pos[e1];
        const uint32_t rs = L.rank[by_doc ? (pos1 & 0xFFFFu) : (pos1 >> 16)];
        const uint32_t r1 = L.rank[by_doc ? (pos1 >> 16) : (pos1 & 0xFFFFu)];
        uint32_t r2 = rs;
        if (e2 < E) {
          const uint32_t pos2 = L.em_pos[e2];
          r2 = L.rank[by_doc ? (pos2 >> 16) : (pos2 & 0xFFFFu)];
        }
        const float4* ps = reinterpret_cast<const float4*>(X + (int64_t)rs * stride) + sub;
        const float4* p1 = reinterpret_cast<const float4*>(X + (int64_t)r1 * stride) + sub;
        const float4* p2 = reinterpret_cast<const float4*>(X + (int64_t)r2 * stride) + sub;
        for (int b = 0; b < per; b += PV) {
          float4 xs[PV], x1[PV], x2[PV];
#pragma unroll
          for (int t = 0; t < PV; ++t)
            if (b + t < per) {
              xs[t] = ps[(b + t) * G];
              x1[t] = p1[(b + t) * G];
              x2[t] = p2[(b + t) * G];
            }
#pragma unroll
          for (int t = 0; t < PV; ++t)
            if (b + t < per) {
              acc1 = dist2_acc(acc1, xs[t], x1[t]);
              acc2 = dist2_acc(acc2, xs[t], x2[t]);
            }
        }
      }
      acc1 = group_sum<G>(acc1);
      acc2 = group_sum<G>(acc2);
      if (sub == 0) {
        if (e1 < E) prod[e1] = (double)L.em_eta[e1] * (double)__builtin_amdgcn_sqrtf(acc1);
        if (e2 < E) prod[e2] = (double)L.em_eta[e2] * (double)__builtin_amdgcn_sqrtf(acc2);
      }
    }
  }
  __syncthreads();
  return sum_products(prod, E);
}

// Lanes per match from the row length in float4 units.
inline int lanes_for(int nvec) {
  int g = 1;
  while (g < 16 && g < nvec) g <<= 1;
  return g;
}

// Lanes per match of the k-NN pricing over the index's rows (dp floats, a
// multiple of 4 * lanes_for(dp / 4)): at most 8, so a wavefront prices 8
// units at once and each lane takes two passes of 5 float4 over a 300-float
// row (16 lanes with one pass took 3 % longer on the batched workload, 4
// lanes 17 % longer).
inline int knn_lanes(int dp) {
  const int g = lanes_for(dp / 4);
  return g < 8 ? g : 8;
}

// Merged-item capacity classes: NMAX = 64 * W * C items on W wavefronts of C
// items per lane (128, 256, 512, 1024, 2048).
constexpr int N_CLASSES = 5;
constexpr int CLASS_C[N_CLASSES] = {2, 4, 4, 4, 8};
constexpr int CLASS_W[N_CLASSES] = {1, 1, 2, 4, 4};

inline int class_for(int n) {
  for (int i = 0; i < N_CLASSES; ++i)
    if (n <= 64 * CLASS_W[i] * CLASS_C[i]) return i;
  return -1;
}

__device__ __forceinline__ int class_for_dev(int n) {
  return n <= 128 ? 0 : n <= 256 ? 1 : n <= 512 ? 2 : n <= 1024 ? 3 : 4;
}

}  // namespace ft
