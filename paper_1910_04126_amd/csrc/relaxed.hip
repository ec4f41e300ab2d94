// Relaxed WMD (paper Section 1.1) and ACT-i (Section 4.1: R-WMD with
// capacity constraints added over i iterations; i = 0 is R-WMD) for
// (query, candidate) pairs -- the quadratic-time stage that follows Flowtree
// in the paper's pipelines.
//
// Per pair, every support point of one side needs its i + 1 nearest points
// of the other side, in both directions.  The distances come from the inner
// products of the two sets of rows, a dense contraction, on the fp32 matrix
// cores: D^2 = |x|^2 + |y|^2 - 2 <x, y>.  That form cancels when x is close to
// y, so it only screens: with a rigorous bound e on its error, a point whose
// lower bound D^2 - e exceeds the (i+1)-th smallest upper bound D^2 + e cannot
// be among the i + 1 nearest.  The survivors (usually i + 1 of them) are then
// priced in the difference form sqrt(sum (x - y)^2) in fp32, the same
// arithmetic as the Flowtree price, and the capacity walk runs on those exact
// values with integer masses, products and sums in fp64.
//
// One wavefront per pair.  32 x 32 tiles of the (doc item x query item)
// product matrix are computed with v_mfma_f32_32x32x2_f32 straight from L2
// (lanes 0..31 and 32..63 take the two halves of the coordinate axis, so
// every lane streams contiguous float4s of one row), written to LDS, and
// screened: lanes 0..31 walk the tile's rows (doc items), lanes 32..63 its
// columns (query items).  Each item keeps its i + 1 smallest upper bounds and
// a short list of candidates whose lower bound is under the threshold; a
// list that fills up with live entries marks the item for a full exact scan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "flow.h"
#include "select.h"
#include "wave.h"

namespace ft {

typedef float act_f32x16 __attribute__((ext_vector_type(16)));

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
  const float* X;         // Morton-ordered rows, stride dp, padded with zeros
  int dp;
  int KH;                 // half of the padded contraction length (multiple of 4)
  int Q;
  int iters;
  float tau;              // relative error bound of the screened D^2 (times |x|^2 + |y|^2)
  uint32_t* status;
  float* cost;            // knn form: [query * n_cols + column]; pairs form: [pair]
};

constexpr int ACT_JOBS = 256;       // exact distances per round
constexpr uint8_t ACT_OVF = 0xFF;   // list overflowed: scan every point of the other side
constexpr float ACT_EPS = 1e-30f;   // absolute slack of the bound (flushed subnormal products)

// K1: how many nearest points an item keeps (a power of two >= iters + 1).
// Entries 0..31 are the doc items of the current row block, 32.. the query
// items.
template <int K1, int QMAX>
struct ActLds {
  static constexpr int CAP = K1 + 5;
  static constexpr int NE = 32 + QMAX;
  float tile[32][33];
  float nr[32], nc[32];
  float thr[NE];                       // K1-th smallest upper bound so far
  float top[K1 > 1 ? K1 - 1 : 1][NE];  // the K1 - 1 smaller ones, ascending
  float candL[CAP][NE];
  uint16_t cand[CAP][NE];
  uint8_t cnt[NE];
  uint32_t job[ACT_JOBS];              // doc item << 16 | query item
  float jres[ACT_JOBS];
};

template <int K1>
__device__ __forceinline__ void keep_smallest(float (&v)[K1], float u) {
  if (u < v[K1 - 1]) {
    v[K1 - 1] = u;
#pragma unroll
    for (int t = K1 - 1; t > 0; --t) {
      if (v[t] < v[t - 1]) {
        const float w = v[t];
        v[t] = v[t - 1];
        v[t - 1] = w;
      }
    }
  }
}

template <int K1, int QMAX>
__device__ __forceinline__ void init_entry(ActLds<K1, QMAX>& L, int e) {
  L.thr[e] = INFINITY;
#pragma unroll
  for (int t = 0; t < K1 - 1; ++t) L.top[t][e] = INFINITY;
  L.cnt[e] = 0;
}

// Inner products of doc rows ib.. and query rows jb.. into L.tile[i][j]
// (32 x 32, zeros past the items), squared norms into L.nr / L.nc.
template <int K1, int QMAX>
__device__ __forceinline__ void tile_dots(ActLds<K1, QMAX>& L, const ActArgs& a, const uint32_t* __restrict__ dr,
                                          const uint32_t* __restrict__ qr, int ib, int ni, int jb, int nj) {
  const int lane = threadIdx.x;
  const int me = lane & 31, h = lane >> 5;
  const bool va = me < ni, vb = me < nj;
  const float* ap = a.X + (size_t)(va ? dr[ib + me] : 0u) * a.dp + h * a.KH;
  const float* bp = a.X + (size_t)(vb ? qr[jb + me] : 0u) * a.dp + h * a.KH;
  const int lim = a.dp - h * a.KH;  // coordinates of this half: [0, lim)
  const int NS = a.KH / 4;
  constexpr int PF = 4;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 ra[PF], rb[PF];
#pragma unroll
  for (int t = 0; t < PF; ++t) {
    ra[t] = (va && 4 * t < lim && t < NS) ? *(const float4*)(ap + 4 * t) : z;
    rb[t] = (vb && 4 * t < lim && t < NS) ? *(const float4*)(bp + 4 * t) : z;
  }
  act_f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  float na = 0.f, nb = 0.f;
  for (int s0 = 0; s0 < NS; s0 += PF) {
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const float4 x = ra[t], y = rb[t];
      const int sn = s0 + t + PF;
      ra[t] = (va && 4 * sn < lim && sn < NS) ? *(const float4*)(ap + 4 * sn) : z;
      rb[t] = (vb && 4 * sn < lim && sn < NS) ? *(const float4*)(bp + 4 * sn) : z;
      na += x.x * x.x + x.y * x.y + x.z * x.z + x.w * x.w;
      nb += y.x * y.x + y.y * y.y + y.z * y.z + y.w * y.w;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x.x, y.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x.y, y.y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x.z, y.z, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x.w, y.w, acc, 0, 0, 0);
    }
  }
  na += __shfl_xor(na, 32, 64);
  nb += __shfl_xor(nb, 32, 64);
  if (lane < 32) {
    L.nr[me] = na;
    L.nc[me] = nb;
  }
  // 32x32 result layout: lane l holds column l % 32, rows 8 (r / 4) + 4 (l / 32) + r % 4
#pragma unroll
  for (int r = 0; r < 16; ++r) L.tile[8 * (r >> 2) + 4 * h + (r & 3)][me] = acc[r];
}

// Screens one tile for one entry (a row when ROW, else a column).
template <int K1, int QMAX>
__device__ __forceinline__ void screen(ActLds<K1, QMAX>& L, const ActArgs& a, bool row, int e, int me, int nx,
                                       int other0) {
  constexpr int CAP = ActLds<K1, QMAX>::CAP;
  const float nme = row ? L.nr[me] : L.nc[me];
  float v[K1];
#pragma unroll
  for (int t = 0; t < K1 - 1; ++t) v[t] = L.top[t][e];
  v[K1 - 1] = L.thr[e];
  for (int x = 0; x < nx; ++x) {
    const float c = row ? L.tile[me][x] : L.tile[x][me];
    const float sn = nme + (row ? L.nc[x] : L.nr[x]);
    const float d2 = sn - 2.0f * c;
    keep_smallest<K1>(v, d2 + (a.tau * sn + ACT_EPS));
  }
  const float thr = v[K1 - 1];
  uint32_t cnt = L.cnt[e];
  if (cnt != ACT_OVF) {
    for (int x = 0; x < nx; ++x) {
      const float c = row ? L.tile[me][x] : L.tile[x][me];
      const float sn = nme + (row ? L.nc[x] : L.nr[x]);
      const float d2 = sn - 2.0f * c;
      const float lo = d2 - (a.tau * sn + ACT_EPS);
      if (lo <= thr) {
        if (cnt == CAP) {  // drop entries the threshold has passed
          uint32_t w = 0;
          for (int t = 0; t < CAP; ++t) {
            const float lt = L.candL[t][e];
            if (lt <= thr) {
              L.candL[w][e] = lt;
              L.cand[w][e] = L.cand[t][e];
              ++w;
            }
          }
          cnt = w;
        }
        if (cnt < CAP) {
          L.candL[cnt][e] = lo;
          L.cand[cnt][e] = (uint16_t)(other0 + x);
          ++cnt;
        } else {
          cnt = ACT_OVF;
          break;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < K1 - 1; ++t) L.top[t][e] = v[t];
  L.thr[e] = thr;
  L.cnt[e] = (uint8_t)cnt;
}

// Exact phase for up to 64 entries (one per lane; `active` lanes only):
// prices the survivors in the difference form, keeps each entry's K1 nearest
// by (distance, index), runs the capacity walk and returns the sum of the
// entries' mass x distance in fixed lane order (valid in every lane).
template <int K1, int QMAX, bool ROW>
__device__ double exact_phase(ActLds<K1, QMAX>& L, const ActArgs& a, const uint32_t* __restrict__ dr,
                              const uint32_t* __restrict__ dm, const uint32_t* __restrict__ qr,
                              const uint32_t* __restrict__ qm, bool active, int e, int self, int n_other) {
  const int lane = threadIdx.x;
  float eD[K1];
  int eO[K1];
#pragma unroll
  for (int t = 0; t < K1; ++t) {
    eD[t] = INFINITY;
    eO[t] = 0xFFFF;
  }
  int mine = 0;
  bool ovf = false;
  float thr = 0.f;
  if (active) {
    const uint32_t cnt = L.cnt[e];
    thr = L.thr[e];
    ovf = cnt == ACT_OVF;
    if (ovf) {
      mine = n_other;
    } else {
      for (uint32_t t = 0; t < cnt; ++t) mine += L.candL[t][e] <= thr ? 1 : 0;
    }
  }
  int done = 0, cursor = 0;
  while (true) {
    const int want = mine - done;
    if (wave_or(want > 0 ? 1u : 0u) == 0u) break;
    const int incl = wave_incl_sum(want);
    const int off = incl - want;
    const int total = __shfl(incl, 63, 64);
    const int take = max(0, min(want, ACT_JOBS - off));
    for (int t = 0; t < take; ++t) {
      int o;
      if (ovf) {
        o = done + t;
      } else {
        while (L.candL[cursor][e] > thr) ++cursor;
        o = L.cand[cursor][e];
        ++cursor;
      }
      const uint32_t di = ROW ? (uint32_t)self : (uint32_t)o, qj = ROW ? (uint32_t)o : (uint32_t)self;
      L.job[off + t] = di << 16 | qj;
    }
    __syncthreads();
    const int nj = min(total, ACT_JOBS);
    for (int b = lane >> 4; b < nj; b += 4) {
      const uint32_t jv = L.job[b];
      const float* xr = a.X + (size_t)dr[jv >> 16] * a.dp;
      const float* yr = a.X + (size_t)qr[jv & 0xFFFFu] * a.dp;
      float acc = 0.f;
      for (int k = 4 * (lane & 15); k < a.dp; k += 64) {
        const float4 x = *(const float4*)(xr + k), y = *(const float4*)(yr + k);
        const float d0 = x.x - y.x, d1 = x.y - y.y, d2 = x.z - y.z, d3 = x.w - y.w;
        acc += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
      }
      acc = group_sum<16>(acc);
      if ((lane & 15) == 0) L.jres[b] = sqrtf(acc);
    }
    __syncthreads();
    for (int t = 0; t < take; ++t) {
      const float D = L.jres[off + t];
      const uint32_t jv = L.job[off + t];
      const int o = ROW ? (int)(jv & 0xFFFFu) : (int)(jv >> 16);
      if (D < eD[K1 - 1] || (D == eD[K1 - 1] && o < eO[K1 - 1])) {
        eD[K1 - 1] = D;
        eO[K1 - 1] = o;
#pragma unroll
        for (int u = K1 - 1; u > 0; --u) {
          if (eD[u] < eD[u - 1] || (eD[u] == eD[u - 1] && eO[u] < eO[u - 1])) {
            const float wd = eD[u];
            eD[u] = eD[u - 1];
            eD[u - 1] = wd;
            const int wo = eO[u];
            eO[u] = eO[u - 1];
            eO[u - 1] = wo;
          }
        }
      }
    }
    done += take;
    __syncthreads();
  }
  // the capacity walk: the first `iters` nearest take at most their own mass,
  // the next nearest takes the rest
  double contrib = 0.0;
  if (active) {
    uint32_t r = ROW ? dm[self] : qm[self];
    const int capped = min(a.iters, n_other);
#pragma unroll
    for (int t = 0; t < K1; ++t) {
      if (t < capped) {
        const uint32_t cap = ROW ? qm[eO[t]] : dm[eO[t]];
        const uint32_t f = min(r, cap);
        contrib += (double)f * (double)eD[t];
        r -= f;
      } else if (t == a.iters && a.iters < n_other) {
        contrib += (double)r * (double)eD[t];
        r = 0;
      }
    }
  }
  contrib = row_sum_f64(contrib);
  return (__shfl(contrib, 0, 64) + __shfl(contrib, 16, 64)) + (__shfl(contrib, 32, 64) + __shfl(contrib, 48, 64));
}

template <int K1, int QMAX>
__global__ __launch_bounds__(64) void k_act(ActArgs a) {
  __shared__ ActLds<K1, QMAX> L;
  const int lane = threadIdx.x;
  const int me = lane & 31;
  int64_t q, doc, out;
  if (a.pair_q) {
    out = blockIdx.x;
    q = a.pair_q[out];
    doc = a.pair_d[out];
  } else {
    const int64_t b = blockIdx.x;
    const int64_t qi = b / a.n_cols, c = b - qi * a.n_cols;
    q = a.qlist[qi];
    out = q * a.n_cols + c;
    doc = a.cand ? a.cand[out] : c;
  }
  const int64_t qa = a.q_off[q], da = a.d_off[doc];
  const int nq = (int)(a.q_off[q + 1] - qa), nd = (int)(a.d_off[doc + 1] - da);
  if (nq > QMAX || nd > 65535) {  // the host picks the class; never taken
    if (lane == 0) atomicOr(a.status, ERR_SIZE);
    return;
  }
  const uint32_t* dr = a.d_rank + da;
  const uint32_t* dm = a.d_mass + da;
  const uint32_t* qr = a.q_rank + qa;
  const uint32_t* qm = a.q_mass + qa;
  for (int e = 32 + lane; e < 32 + nq; e += 64) init_entry(L, e);
  double tot_d = 0.0;
  for (int ib = 0; ib < nd; ib += 32) {
    const int ni = min(32, nd - ib);
    if (lane < 32) init_entry(L, lane);
    for (int jb = 0; jb < nq; jb += 32) {
      const int nj = min(32, nq - jb);
      tile_dots(L, a, dr, qr, ib, ni, jb, nj);
      __syncthreads();
      if (lane < 32) {
        if (me < ni) screen(L, a, true, me, me, nj, jb);
      } else {
        if (me < nj) screen(L, a, false, 32 + jb + me, me, ni, ib);
      }
      __syncthreads();
    }
    tot_d += exact_phase<K1, QMAX, true>(L, a, dr, dm, qr, qm, lane < ni, lane, ib + lane, nq);
  }
  double tot_q = 0.0;
  for (int c0 = 0; c0 < nq; c0 += 64)
    tot_q += exact_phase<K1, QMAX, false>(L, a, dr, dm, qr, qm, c0 + lane < nq, 32 + c0 + lane, c0 + lane, nd);
  if (lane == 0) a.cost[out] = (float)ldexp(tot_d > tot_q ? tot_d : tot_q, -a.Q);
}

// ------------------------------------------------------------- dispatch --

constexpr int ACT_QMAX[3] = {128, 512, 2048};

static int act_class(int nq) {
  for (int c = 0; c < 3; ++c)
    if (nq <= ACT_QMAX[c]) return c;
  return -1;
}

// The 2048-point query class keeps its per-item state in LDS for K1 <= 2
// only (ACT with at most one iteration).
template <int K1>
static void launch_k1(int cls, int64_t grid, const ActArgs& a, hipStream_t s) {
  if (cls == 0) {
    k_act<K1, 128><<<dim3((unsigned)grid), 64, 0, s>>>(a);
  } else if (cls == 1) {
    k_act<K1, 512><<<dim3((unsigned)grid), 64, 0, s>>>(a);
  } else {
    if constexpr (K1 <= 2) k_act<K1, 2048><<<dim3((unsigned)grid), 64, 0, s>>>(a);
    else throw Error(FT_ERANGE, "ACT with more than one iteration needs queries of at most 512 points");
  }
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
  a.X = ix->Xm.as<float>();
  a.dp = ix->dp;
  a.KH = (int)(ceil_div(ix->dp, 8) * 4);
  a.Q = ix->Q;
  a.iters = iters;
  // |D^2_screened - D^2| <= (2 gamma_K + 3u)(|x|^2 + |y|^2) for K = 2 KH terms
  // with unit roundoff u = 2^-24; four times that, which also covers
  // truncating accumulation
  a.tau = (float)(4.0 * (2.0 * (2 * a.KH) + 4.0) * std::ldexp(1.0, -24));
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
    FT_REQUIRE(ix->docs.max_size <= 65535, FT_ERANGE, "dataset distributions larger than 65535 points");
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    if (cand) check_indices(ix, cand, n_q * n_cand, ix->docs.n, s, "cand");
    FT_REQUIRE(act_class(ix->qry.max_size) >= 0, FT_ERANGE, "query larger than 2048 points");
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
      for (int c = 0; c < 3; ++c) {
        a.qlist = qlist + start[c];
        launch_act(c, (start[c + 1] - start[c]) * n_cols, a, s);
      }
      topk_rows(cost, r1 - r0, n_cols, a.cand, k, out_cost + r0 * k, out_doc + r0 * k, s);
      FT_HIP(hipStreamSynchronize(s));  // hl is reused by the next chunk
    }
    uint32_t flags = read_and_clear_status(ix, s);
    FT_REQUIRE(flags == 0, FT_EHIP, "act kernel reported:" + describe_flags(flags));
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
    FT_REQUIRE(ix->docs.max_size <= 65535, FT_ERANGE, "dataset distributions larger than 65535 points");
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    if (n_pairs == 0) return;
    check_indices(ix, pair_q, n_pairs, n_q, s, "pair_q");
    check_indices(ix, pair_d, n_pairs, ix->docs.n, s, "pair_d");
    const int cls = act_class(ix->qry.max_size);
    FT_REQUIRE(cls >= 0, FT_ERANGE, "query larger than 2048 points");
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
