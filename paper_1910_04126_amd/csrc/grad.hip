// Flowtree of explicit pairs with the flow kept: inspection of the flow, and
// the cost's gradient with the tree and the flow pattern frozen.
//
// The paper defines no gradient.  With the pattern frozen, each match moves
// the unmatched mass of the item it used up (the doc item when both were used
// up), so every moved mass is a linear function of the weights w = mass/2^Q:
//   eta_e = r(bind_e);  r(doc_e) -= eta_e;  r(query_e) -= eta_e,
// and C = sum_e eta_e * D_e with D_e = ||x_doc - x_query||_2.  Then
//   dC/dx = eta_e (x_doc - x_query) / D_e on the doc point (minus on the query
//           point), 0 when D_e = 0;
//   dC/dw by reverse accumulation in the greedy's own order:
//           lambda_e = D_e - acc[doc_e] - acc[query_e];  acc[bind_e] += lambda_e
//           for e from the last match to the first; dC/dw_i = acc[i].
// The greedy's order is deepest cells first, and inside a cell increasing
// position of the match along the cumulative-mass axis; every saved match
// carries that order as a sort key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "common.h"
#include "flow.h"
#include "wave.h"

namespace ft {

struct SaveArgs {
  const int64_t* pair_q;
  const int64_t* pair_d;
  const int64_t* base;  // first saved entry of each pair
  const int64_t* q_off;
  const uint32_t* q_rank;
  const uint32_t* q_mass;
  const int64_t* d_off;
  const uint32_t* d_rank;
  const uint32_t* d_mass;
  const uint8_t* st;
  int64_t V;
  int B, Q;
  const float* X;  // caller's coordinates, original order
  const uint32_t* perm;
  int d;
  uint32_t* status;
  FlowSave sv;
  int32_t* count;
  float* cost;  // NULL: do not price
};

template <int C, int W, int G, int VEC>
__global__ __launch_bounds__(64 * W) void k_flow_save(SaveArgs a) {
  __shared__ FlowLds<C, W> L;
  const int64_t p = blockIdx.x;
  const int64_t q = a.pair_q[p], doc = a.pair_d[p];
  const int64_t qa = a.q_off[q], da = a.d_off[doc];
  const int nq = (int)(a.q_off[q + 1] - qa), nd = (int)(a.d_off[doc + 1] - da);
  if (nq + nd > FlowLds<C, W>::N) {
    if (threadIdx.x == 0) atomicOr(a.status, ERR_FLOW);
    return;
  }
  flow_stage(L, a.q_rank + qa, a.q_mass + qa, nq, a.d_rank + da, a.d_mass + da, nd);
  FlowSave sv = a.sv;
  sv.base = a.base[p];
  const int E = flow_match<C, W, true>(L, nq, nd, a.st, a.V, a.B, sv, a.status);
  if (threadIdx.x == 0) a.count[p] = E;
  if (a.cost) {
    const double c = flow_price<C, W, G, VEC>(L, E, nq, nd, a.X, a.perm, a.d, a.d, a.status);
    if (threadIdx.x == 0) a.cost[p] = (float)ldexp(c, -a.Q);
  }
}

__global__ void k_pair_sizes(const int64_t* __restrict__ pair_q, const int64_t* __restrict__ pair_d, int64_t n,
                             const int64_t* __restrict__ q_off, const int64_t* __restrict__ d_off,
                             int64_t* __restrict__ out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  out[p] = (q_off[pair_q[p] + 1] - q_off[pair_q[p]]) + (d_off[pair_d[p] + 1] - d_off[pair_d[p]]);
}

// Saved flow -> caller arrays of original point ids.
__global__ void k_flows_out(const int64_t* __restrict__ pair_q, const int64_t* __restrict__ pair_d, int64_t n,
                            const int64_t* __restrict__ base, const int32_t* __restrict__ cnt,
                            const int64_t* __restrict__ cap_off, const uint32_t* __restrict__ id,
                            const uint32_t* __restrict__ eta, const uint8_t* __restrict__ bind,
                            const int64_t* __restrict__ q_off, const uint32_t* __restrict__ q_rank,
                            const int64_t* __restrict__ d_off, const uint32_t* __restrict__ d_rank,
                            const uint32_t* __restrict__ perm, int32_t* __restrict__ count,
                            uint32_t* __restrict__ fd, uint32_t* __restrict__ fq, uint32_t* __restrict__ fe,
                            uint8_t* __restrict__ fb, uint32_t* __restrict__ status) {
  const int64_t p = blockIdx.x;
  if (p >= n) return;
  const int E = cnt[p];
  const int64_t o = cap_off[p];
  if (cap_off[p + 1] - o < E) {
    if (threadIdx.x == 0) atomicOr(status, ERR_SIZE);
    return;
  }
  const int64_t qa = q_off[pair_q[p]], da = d_off[pair_d[p]];
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const uint32_t v = id[base[p] + e];
    fd[o + e] = perm[d_rank[da + (v >> 16)]];
    fq[o + e] = perm[q_rank[qa + (v & 0xFFFFu)]];
    fe[o + e] = eta[base[p] + e];
    fb[o + e] = bind[base[p] + e];
  }
  if (threadIdx.x == 0) count[p] = E;
}

// Backward of one pair on one workgroup of BWD_THREADS threads: the saved
// matches are sorted into the greedy's order, every match's distance and
// coordinate gradient is computed by a group of G lanes (BWD_THREADS / G
// matches in flight), and one lane runs the reverse sweep for the weights.
constexpr int BWD_THREADS = 1024;

template <int C, int G, int VEC>
__global__ __launch_bounds__(BWD_THREADS) void k_flow_bwd(
    const int64_t* __restrict__ pair_q, const int64_t* __restrict__ pair_d, const int64_t* __restrict__ base,
    const int32_t* __restrict__ cnt, const uint32_t* __restrict__ fid, const uint32_t* __restrict__ feta,
    const uint64_t* __restrict__ fkey, const uint8_t* __restrict__ fbind, const int64_t* __restrict__ q_off,
    const uint32_t* __restrict__ q_rank, const uint16_t* __restrict__ q_pos, const int64_t* __restrict__ d_off,
    const uint32_t* __restrict__ d_rank, const uint16_t* __restrict__ d_pos, const uint32_t* __restrict__ perm,
    const float* __restrict__ X, int d, int Q, const float* __restrict__ grad_out,
    const double* __restrict__ unit, unsigned long long* __restrict__ gx64, double* __restrict__ adj) {
  constexpr int N = 64 * C;
  __shared__ uint64_t skey[N];
  __shared__ uint16_t sidx[N];
  __shared__ float sD[N];
  __shared__ double acc[N];
  __shared__ uint32_t srow[N];  // row of X of every item: query items, then doc items
  const int64_t p = blockIdx.x;
  const int tid = threadIdx.x;
  const float g = grad_out[p];
  const int E = cnt[p];
  const int64_t b0 = base[p];
  const int64_t qa = q_off[pair_q[p]], da = d_off[pair_d[p]];
  const int nq = (int)(q_off[pair_q[p] + 1] - qa), nd = (int)(d_off[pair_d[p] + 1] - da);
  int P = 1;
  while (P < E) P <<= 1;
  for (int e = tid; e < P; e += BWD_THREADS) {
    skey[e] = e < E ? fkey[b0 + e] : ~0ull;
    sidx[e] = (uint16_t)e;
  }
  for (int i = tid; i < nq + nd; i += BWD_THREADS) {
    acc[i] = 0.0;
    srow[i] = perm[i < nq ? q_rank[qa + i] : d_rank[da + (i - nq)]];
  }
  __syncthreads();
  // the greedy's order
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = tid; t < P; t += BWD_THREADS) {
        const int l = t ^ j;
        if (l > t) {
          const uint64_t x = skey[t], y = skey[l];
          const bool up = (t & k) == 0;
          if (up ? (y < x) : (x < y)) {
            skey[t] = y;
            skey[l] = x;
            const uint16_t u = sidx[t];
            sidx[t] = sidx[l];
            sidx[l] = u;
          }
        }
      }
      __syncthreads();
    }
  // distances and coordinate gradients: G lanes per match
  const int grp = tid / G, sub = tid % G;
  constexpr int PER = BWD_THREADS / G;
  const double wscale = ldexp(1.0, -Q);
  for (int r0 = 0; r0 < E; r0 += PER) {
    const int r = r0 + grp;
    float dd = 0.0f;
    const float* xd = nullptr;
    const float* xq = nullptr;
    unsigned long long* gxd = nullptr;
    unsigned long long* gxq = nullptr;
    uint32_t eta = 0;
    if (r < E) {
      const int e = sidx[r];
      const uint32_t v = fid[b0 + e];
      eta = feta[b0 + e];
      const int64_t rowd = srow[nq + (int)(v >> 16)], rowq = srow[v & 0xFFFFu];
      if (rowd != rowq) {
        xd = X + rowd * d;
        xq = X + rowq * d;
        gxd = gx64 ? gx64 + rowd * d : nullptr;
        gxq = gx64 ? gx64 + rowq * d : nullptr;
        if (VEC == 4) {
          for (int i = sub; i < d / 4; i += G) {
            const float4 a4 = reinterpret_cast<const float4*>(xd)[i], b4 = reinterpret_cast<const float4*>(xq)[i];
            const float dx = a4.x - b4.x, dy = a4.y - b4.y, dz = a4.z - b4.z, dw = a4.w - b4.w;
            dd += dx * dx + dy * dy + dz * dz + dw * dw;
          }
        } else {
          for (int i = sub; i < d; i += G) {
            const float dx = xd[i] - xq[i];
            dd += dx * dx;
          }
        }
      }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) dd += __shfl_xor(dd, o, 64);
    const float D = sqrtf(dd);
    if (r < E && sub == 0) {
      sD[r] = D;
      // the sort keys are dead now: keep the match's items and bind pattern
      // in its sorted slot so the sweep below reads LDS only
      const int e = sidx[r];
      skey[r] = ((uint64_t)fbind[b0 + e] << 32) | fid[b0 + e];
    }
    if (r < E && xd && D > 0.0f && gxd) {
      // fixed point in units of unit[0] (a power of two): integer sums do not
      // depend on the order of the additions, so dX is reproducible
      const float coef = (float)((double)g * (double)eta * wscale / (double)D);
      const double inv = unit[1];
      for (int i = sub; i < d; i += G) {
        const long long v = __double2ll_rn((double)((xd[i] - xq[i]) * coef) * inv);
        atomicAdd(gxd + i, (unsigned long long)v);
        atomicAdd(gxq + i, (unsigned long long)(-v));
      }
    }
  }
  __syncthreads();
  // weight adjoints: reverse sweep in the greedy's order (one lane)
  if (tid == 0) {
    for (int r = E - 1; r >= 0; --r) {
      const uint64_t kv = skey[r];
      const uint32_t v = (uint32_t)kv;
      const int sd = nq + (int)(v >> 16), sq = (int)(v & 0xFFFFu);
      const double lam = (double)sD[r] - acc[sd] - acc[sq];
      if ((kv >> 32) == 1) acc[sq] += lam;
      else acc[sd] += lam;
    }
  }
  __syncthreads();
  // the pair's weight adjoints, query items then doc items; summed over the
  // pairs of each query and each doc in pair order afterwards
  if (adj)
    for (int i = tid; i < nq + nd; i += BWD_THREADS) adj[b0 + i] = (double)g * acc[i];
}

// The fixed-point unit of dX: with G = max |grad_out| < 2^e and F fraction
// bits, unit = 2^(e - F).  A match adds at most G * eta / 2^Q to an entry in
// magnitude, and a pair's eta sum to 2^Q, so an entry's sum stays below
// n_pairs * 2^F units (the host picks F accordingly).  Non-finite grad_out
// is reported.
__global__ __launch_bounds__(256) void k_grad_unit(const float* __restrict__ g, int64_t n, int frac_bits,
                                                   double* __restrict__ unit, uint32_t* __restrict__ status) {
  __shared__ float wmax[4];
  float m = 0.0f;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float v = fabsf(g[i]);
    if (!(v <= 3.4e38f)) bad = true;
    else m = fmaxf(m, v);
  }
  m = wave_max(m);
  if (__ballot(bad) && lane_id() == 0) atomicOr(status, ERR_NONFINITE);
  if (lane_id() == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    const int e = m > 0.0f ? ilogbf(m) + 1 : 0;
    unit[0] = ldexp(1.0, e - frac_bits);
    unit[1] = ldexp(1.0, frac_bits - e);
  }
}

// gX += fixed-point sums (entries no match touched are left alone).
__global__ void k_grad_x_finish(const unsigned long long* __restrict__ gx64, int64_t n, const double* __restrict__ unit,
                                float* __restrict__ gX) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && gx64[i]) gX[i] += (float)((double)(long long)gx64[i] * unit[0]);
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Query weight gradients: one wavefront per query, its pairs in increasing
// pair order (list[lo[q]..lo[q+1])), each item's adjoints summed in that
// order.
__global__ __launch_bounds__(64) void k_grad_w_query(const int64_t* __restrict__ lo, const int64_t* __restrict__ list,
                                                     const int64_t* __restrict__ base, const double* __restrict__ adj,
                                                     const int64_t* __restrict__ q_off,
                                                     const uint16_t* __restrict__ q_pos, float* __restrict__ gq) {
  const int64_t q = blockIdx.x;
  const int64_t qa = q_off[q];
  const int nq = (int)(q_off[q + 1] - qa);
  for (int i = threadIdx.x; i < nq; i += 64) {
    double s = 0.0;
    for (int64_t k = lo[q]; k < lo[q + 1]; ++k) s += adj[base[list[k]] + i];
    if (lo[q + 1] > lo[q]) gq[qa + q_pos[qa + i]] += (float)s;
  }
}

// Doc weight gradients: one wavefront per distinct doc of the pairs
// (docs[j], its pairs list[lo[j]..lo[j+1]) in increasing pair order); a doc
// item's slot in its pair follows the query's items.
__global__ __launch_bounds__(64) void k_grad_w_doc(const int64_t* __restrict__ docs, const int64_t* __restrict__ lo,
                                                   const int64_t* __restrict__ list, const int64_t* __restrict__ base,
                                                   const double* __restrict__ adj, const int64_t* __restrict__ pair_q,
                                                   const int64_t* __restrict__ q_off, const int64_t* __restrict__ d_off,
                                                   const uint16_t* __restrict__ d_pos, float* __restrict__ gd) {
  const int64_t j = blockIdx.x;
  const int64_t doc = docs[j];
  const int64_t da = d_off[doc];
  const int nd = (int)(d_off[doc + 1] - da);
  for (int i = threadIdx.x; i < nd; i += 64) {
    double s = 0.0;
    for (int64_t k = lo[j]; k < lo[j + 1]; ++k) {
      const int64_t p = list[k];
      const int64_t nq = q_off[pair_q[p] + 1] - q_off[pair_q[p]];
      s += adj[base[p] + nq + i];
    }
    gd[da + d_pos[da + i]] += (float)s;
  }
}

// Copies of the FT_FWD arguments, compared element by element in FT_BWD.
__global__ void k_copy_or_compare(const uint8_t* __restrict__ a, uint8_t* __restrict__ keep, int64_t n, int compare,
                                  uint32_t* __restrict__ status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (compare) {
    if (a[i] != keep[i]) atomicOr(status, ERR_EMPTY);
  } else {
    keep[i] = a[i];
  }
}

// ------------------------------------------------------------- dispatch --

#define FT_DISPATCH_CG(KERNEL, cls, G, VEC, grid, block, s, ...)                             \
  do {                                                                                       \
    auto go = [&](auto cc, auto gg, auto vv) {                                              \
      KERNEL<decltype(cc)::value, decltype(gg)::value, decltype(vv)::value><<<grid, block, 0, s>>>(__VA_ARGS__); \
    };                                                                                       \
    auto gsel = [&](auto cc, auto vv) {                                                      \
      switch (G) {                                                                           \
        case 1: go(cc, std::integral_constant<int, 1>{}, vv); break;                         \
        case 2: go(cc, std::integral_constant<int, 2>{}, vv); break;                         \
        case 4: go(cc, std::integral_constant<int, 4>{}, vv); break;                         \
        case 8: go(cc, std::integral_constant<int, 8>{}, vv); break;                         \
        default: go(cc, std::integral_constant<int, 16>{}, vv); break;                       \
      }                                                                                      \
    };                                                                                       \
    auto vsel = [&](auto cc) {                                                               \
      if (VEC == 4) gsel(cc, std::integral_constant<int, 4>{});                              \
      else gsel(cc, std::integral_constant<int, 1>{});                                       \
    };                                                                                       \
    switch (cls) {                                                                           \
      case 0: vsel(std::integral_constant<int, 2>{}); break;                                 \
      case 1: vsel(std::integral_constant<int, 4>{}); break;                                 \
      case 2: vsel(std::integral_constant<int, 8>{}); break;                                 \
      case 3: vsel(std::integral_constant<int, 16>{}); break;                                \
      default: vsel(std::integral_constant<int, 32>{}); break;                               \
    }                                                                                        \
  } while (0)

// The saving kernel in the size class's shape (C items per lane, W wavefronts).
#define FT_DISPATCH_SAVE(cls, G, VEC, grid, s, ...)                                          \
  do {                                                                                       \
    auto go = [&](auto cc, auto ww, auto gg, auto vv) {                                     \
      k_flow_save<decltype(cc)::value, decltype(ww)::value, decltype(gg)::value, decltype(vv)::value> \
          <<<grid, 64 * decltype(ww)::value, 0, s>>>(__VA_ARGS__);                           \
    };                                                                                       \
    auto gsel = [&](auto cc, auto ww, auto vv) {                                             \
      switch (G) {                                                                           \
        case 1: go(cc, ww, std::integral_constant<int, 1>{}, vv); break;                     \
        case 2: go(cc, ww, std::integral_constant<int, 2>{}, vv); break;                     \
        case 4: go(cc, ww, std::integral_constant<int, 4>{}, vv); break;                     \
        case 8: go(cc, ww, std::integral_constant<int, 8>{}, vv); break;                     \
        default: go(cc, ww, std::integral_constant<int, 16>{}, vv); break;                   \
      }                                                                                      \
    };                                                                                       \
    auto vsel = [&](auto cc, auto ww) {                                                      \
      if (VEC == 4) gsel(cc, ww, std::integral_constant<int, 4>{});                          \
      else gsel(cc, ww, std::integral_constant<int, 1>{});                                   \
    };                                                                                       \
    using I = std::integral_constant<int, 1>;                                                \
    using I2 = std::integral_constant<int, 2>;                                               \
    using I4 = std::integral_constant<int, 4>;                                               \
    using I8 = std::integral_constant<int, 8>;                                               \
    switch (cls) {                                                                           \
      case 0: vsel(I2{}, I{}); break;                                                        \
      case 1: vsel(I4{}, I{}); break;                                                        \
      case 2: vsel(I4{}, I2{}); break;                                                       \
      case 3: vsel(I4{}, I4{}); break;                                                       \
      default: vsel(I8{}, I4{}); break;                                                      \
    }                                                                                        \
  } while (0)

// Prepare queries, validate pairs, compute per-pair saved-entry offsets and run
// the saving kernel.  Returns the class used.
static int run_save(ft_index* ix, const float* X, const int64_t* q_off, const uint32_t* q_id, const uint32_t* q_mass,
                    int64_t n_q, const int64_t* pair_q, const int64_t* pair_d, int64_t n_pairs, float* cost,
                    hipStream_t s) {
  prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
  check_indices(ix, pair_q, n_pairs, n_q, s, "pair_q");
  check_indices(ix, pair_d, n_pairs, ix->docs.n, s, "pair_d");
  const int cls = class_for(ix->qry.max_size + ix->docs.max_size);
  FT_REQUIRE(cls >= 0, FT_ERANGE, "pair larger than 2048 items");
  int64_t* sizes = (int64_t*)ix->ws_misc.ensure((n_pairs + scan_tmp_elems(n_pairs)) * 8);
  int64_t* base = (int64_t*)ix->fwd_base.ensure((n_pairs + 1) * 8);
  k_pair_sizes<<<(unsigned)ceil_div(n_pairs, 256), 256, 0, s>>>(pair_q, pair_d, n_pairs, ix->qry.off.as<int64_t>(),
                                                                ix->docs.off.as<int64_t>(), sizes);
  exclusive_scan_i64(sizes, base, n_pairs, sizes + n_pairs, s);
  int64_t total = 0;
  FT_HIP(hipMemcpyAsync(&total, base + n_pairs, 8, hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
  SaveArgs a;
  a.pair_q = pair_q;
  a.pair_d = pair_d;
  a.base = base;
  a.q_off = ix->qry.off.as<int64_t>();
  a.q_rank = ix->qry.rank.as<uint32_t>();
  a.q_mass = ix->qry.mass.as<uint32_t>();
  a.d_off = ix->docs.off.as<int64_t>();
  a.d_rank = ix->docs.rank.as<uint32_t>();
  a.d_mass = ix->docs.mass.as<uint32_t>();
  a.st = ix->st.as<uint8_t>();
  a.V = ix->V;
  a.B = ix->B;
  a.Q = ix->Q;
  a.X = X;
  a.perm = ix->perm.as<uint32_t>();
  a.d = ix->d;
  a.status = ix->status.as<uint32_t>();
  a.sv.id = (uint32_t*)ix->fwd_id.ensure(std::max<int64_t>(total, 1) * 4);
  a.sv.eta = (uint32_t*)ix->fwd_eta.ensure(std::max<int64_t>(total, 1) * 4);
  a.sv.key = (uint64_t*)ix->fwd_key.ensure(std::max<int64_t>(total, 1) * 8);
  a.sv.bind = (uint8_t*)ix->fwd_bind.ensure(std::max<int64_t>(total, 1));
  a.sv.base = 0;
  a.count = (int32_t*)ix->fwd_cnt.ensure(n_pairs * 4);
  a.cost = cost;
  const int G = lanes_for((ix->d + 3) / 4);
  const int VEC = (X && ix->d % 4 == 0 && ((uintptr_t)X & 15) == 0) ? 4 : 1;
  FT_DISPATCH_SAVE(cls, G, VEC, dim3((unsigned)n_pairs), s, a);
  FT_HIP(hipGetLastError());
  ix->fwd_pairs = n_pairs;
  ix->fwd_cap = total;
  return cls;
}

}  // namespace ft

using namespace ft;

extern "C" ft_status ft_flowtree_flows(ft_index* ix, const int64_t* q_off, const uint32_t* q_id,
                                       const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                                       const int64_t* pair_d, int64_t n_pairs, const int64_t* cap_off, int32_t* count,
                                       uint32_t* flow_d, uint32_t* flow_q, uint32_t* flow_eta, uint8_t* flow_bind,
                                       void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && pair_q && pair_d && cap_off && count && flow_d && flow_q && flow_eta && flow_bind, FT_EINVAL,
               "NULL argument");
    FT_REQUIRE(n_pairs >= 1, FT_EINVAL, "need at least one pair");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    run_save(ix, nullptr, q_off, q_id, q_mass, n_q, pair_q, pair_d, n_pairs, nullptr, s);
    ix->fwd_valid = false;  // the saved flow no longer matches any FT_FWD call
    k_flows_out<<<(unsigned)n_pairs, 64, 0, s>>>(
        pair_q, pair_d, n_pairs, ix->fwd_base.as<int64_t>(), ix->fwd_cnt.as<int32_t>(), cap_off,
        ix->fwd_id.as<uint32_t>(), ix->fwd_eta.as<uint32_t>(), ix->fwd_bind.as<uint8_t>(), ix->qry.off.as<int64_t>(),
        ix->qry.rank.as<uint32_t>(), ix->docs.off.as<int64_t>(), ix->docs.rank.as<uint32_t>(),
        ix->perm.as<uint32_t>(), count, flow_d, flow_q, flow_eta, flow_bind, ix->status.as<uint32_t>());
    FT_HIP(hipGetLastError());
    uint32_t flags = read_and_clear_status(ix, s);
    if (flags & ERR_SIZE) throw Error(FT_EINVAL, "cap_off leaves a pair too few slots");
    FT_REQUIRE(flags == 0, FT_EHIP, "flowtree kernel reported:" + describe_flags(flags));
  });
}

extern "C" ft_status ft_flowtree_cost_grad(ft_index* ix, const float* X, const int64_t* q_off, const uint32_t* q_id,
                                           const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                                           const int64_t* pair_d, int64_t n_pairs, int32_t mode,
                                           const float* grad_out, float* cost, float* grad_X, float* grad_qmass,
                                           float* grad_dmass, void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix && X && pair_q && pair_d, FT_EINVAL, "NULL argument");
    FT_REQUIRE(n_pairs >= 1, FT_EINVAL, "need at least one pair");
    FT_REQUIRE(mode == FT_FWD || mode == FT_BWD, FT_EINVAL, "mode must be FT_FWD or FT_BWD");
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    // byte images of the arguments that define the saved flows
    auto keep_args = [&](int compare) {
      int64_t nnz = 0;
      FT_HIP(hipMemcpyAsync(&nnz, q_off + n_q, 8, hipMemcpyDeviceToHost, s));
      FT_HIP(hipStreamSynchronize(s));
      const int64_t sizes[5] = {(n_q + 1) * 8, nnz * 4, nnz * 4, n_pairs * 8, n_pairs * 8};
      const void* src[5] = {q_off, q_id, q_mass, pair_q, pair_d};
      int64_t total = sizes[0] + sizes[1] + sizes[2] + sizes[3] + sizes[4];
      if (compare && (int64_t)ix->fwd_sig.bytes < total) return false;
      uint8_t* keep = (uint8_t*)(compare ? ix->fwd_sig.p : ix->fwd_sig.ensure(total));
      if (compare && ix->fwd_sig_bytes != total) return false;
      for (int i = 0; i < 5; ++i) {
        if (sizes[i] > 0)
          k_copy_or_compare<<<(unsigned)ceil_div(sizes[i], 256), 256, 0, s>>>((const uint8_t*)src[i], keep,
                                                                            sizes[i], compare,
                                                                            ix->status.as<uint32_t>());
        keep += sizes[i];
      }
      FT_HIP(hipGetLastError());
      ix->fwd_sig_bytes = total;
      return compare ? read_and_clear_status(ix, s) == 0 : true;
    };
    if (mode == FT_FWD) {
      FT_REQUIRE(cost, FT_EINVAL, "cost is NULL");
      run_save(ix, X, q_off, q_id, q_mass, n_q, pair_q, pair_d, n_pairs, cost, s);
      uint32_t flags = read_and_clear_status(ix, s);
      FT_REQUIRE(flags == 0, FT_EHIP, "flowtree kernel reported:" + describe_flags(flags));
      ix->fwd_valid = false;
      keep_args(0);
      ix->fwd_valid = true;
      return;
    }
    FT_REQUIRE(grad_out, FT_EINVAL, "grad_out is NULL");
    FT_REQUIRE(ix->fwd_valid && keep_args(1), FT_EINVAL,
               "FT_BWD needs the pairs and queries of the preceding FT_FWD call");
    // the query preparation is deterministic: redo it in case another call
    // reused the workspace
    prepare_dists(ix, ix->qry, q_off, q_id, q_mass, n_q, false, s, "queries");
    const int cls = class_for(ix->qry.max_size + ix->docs.max_size);
    const int G = lanes_for((ix->d + 3) / 4);
    const int VEC = (ix->d % 4 == 0 && ((uintptr_t)X & 15) == 0) ? 4 : 1;
    // each query's and each doc's pairs in increasing pair order, for the
    // weight gradients (made before any buffer below is sized)
    const bool want_w = grad_qmass || grad_dmass;
    std::vector<int64_t> qlo, qlist, ddocs, dlo, dlist;
    if (want_w) {
      std::vector<int64_t> hq(n_pairs), hd(n_pairs);
      FT_HIP(hipMemcpyAsync(hq.data(), pair_q, n_pairs * 8, hipMemcpyDeviceToHost, s));
      FT_HIP(hipMemcpyAsync(hd.data(), pair_d, n_pairs * 8, hipMemcpyDeviceToHost, s));
      FT_HIP(hipStreamSynchronize(s));
      qlo.assign(n_q + 1, 0);
      qlist.resize(n_pairs);
      for (int64_t p = 0; p < n_pairs; ++p) ++qlo[hq[p] + 1];
      for (int64_t q = 0; q < n_q; ++q) qlo[q + 1] += qlo[q];
      std::vector<int64_t> at(qlo.begin(), qlo.end() - 1);
      for (int64_t p = 0; p < n_pairs; ++p) qlist[at[hq[p]]++] = p;
      std::vector<std::pair<int64_t, int64_t>> dp(n_pairs);
      for (int64_t p = 0; p < n_pairs; ++p) dp[p] = {hd[p], p};
      std::sort(dp.begin(), dp.end());
      dlist.resize(n_pairs);
      for (int64_t k = 0; k < n_pairs; ++k) {
        if (k == 0 || dp[k].first != dp[k - 1].first) {
          ddocs.push_back(dp[k].first);
          dlo.push_back(k);
        }
        dlist[k] = dp[k].second;
      }
      dlo.push_back(n_pairs);
    }
    const int64_t nu = (int64_t)ddocs.size();
    // one buffer: the fixed-point unit (and its inverse), then the lists
    int64_t* g = (int64_t*)ix->ws_glist.ensure((8 + (want_w ? (n_q + 1) + 2 * n_pairs + 2 * nu + 1 : 0)) * 8);
    double* unit = reinterpret_cast<double*>(g);
    unsigned long long* gx64 = nullptr;
    const int64_t nx = ix->V * (int64_t)ix->d;
    if (grad_X) gx64 = (unsigned long long*)ix->ws_gx64.ensure(nx * 8);
    double* adj = want_w ? (double*)ix->ws_adj.ensure(std::max<int64_t>(ix->fwd_cap, 1) * 8) : nullptr;
    // dX in fixed point: F fraction bits keep n_pairs * 2^F below 2^62
    int frac = 40;
    while (frac > 8 && (double)n_pairs * std::ldexp(1.0, frac) >= std::ldexp(1.0, 62)) --frac;
    k_grad_unit<<<1, 256, 0, s>>>(grad_out, n_pairs, frac, unit, ix->status.as<uint32_t>());
    FT_HIP(hipGetLastError());
    if (read_and_clear_status(ix, s)) throw Error(FT_EINVAL, "grad_out must be finite");
    if (gx64) {
      k_zero_u64<<<(unsigned)ceil_div(nx, 256), 256, 0, s>>>(gx64, nx);
      FT_HIP(hipGetLastError());
    }
    FT_DISPATCH_CG(k_flow_bwd, cls, G, VEC, dim3((unsigned)n_pairs), BWD_THREADS, s, pair_q, pair_d, ix->fwd_base.as<int64_t>(),
                   ix->fwd_cnt.as<int32_t>(), ix->fwd_id.as<uint32_t>(), ix->fwd_eta.as<uint32_t>(),
                   ix->fwd_key.as<uint64_t>(), ix->fwd_bind.as<uint8_t>(), ix->qry.off.as<int64_t>(),
                   ix->qry.rank.as<uint32_t>(), ix->qry.pos.as<uint16_t>(), ix->docs.off.as<int64_t>(),
                   ix->docs.rank.as<uint32_t>(), ix->docs.pos.as<uint16_t>(), ix->perm.as<uint32_t>(), X, ix->d,
                   ix->Q, grad_out, unit, gx64, adj);
    FT_HIP(hipGetLastError());
    if (gx64) {
      k_grad_x_finish<<<(unsigned)ceil_div(nx, 256), 256, 0, s>>>(gx64, nx, unit, grad_X);
      FT_HIP(hipGetLastError());
    }
    if (!want_w) return;
    int64_t* d_qlo = g + 8;
    int64_t* d_qlist = d_qlo + (n_q + 1);
    int64_t* d_docs = d_qlist + n_pairs;
    int64_t* d_dlo = d_docs + nu;
    int64_t* d_dlist = d_dlo + (nu + 1);
    FT_HIP(hipMemcpyAsync(d_qlo, qlo.data(), (n_q + 1) * 8, hipMemcpyHostToDevice, s));
    FT_HIP(hipMemcpyAsync(d_qlist, qlist.data(), n_pairs * 8, hipMemcpyHostToDevice, s));
    FT_HIP(hipMemcpyAsync(d_docs, ddocs.data(), nu * 8, hipMemcpyHostToDevice, s));
    FT_HIP(hipMemcpyAsync(d_dlo, dlo.data(), (nu + 1) * 8, hipMemcpyHostToDevice, s));
    FT_HIP(hipMemcpyAsync(d_dlist, dlist.data(), n_pairs * 8, hipMemcpyHostToDevice, s));
    if (grad_qmass)
      k_grad_w_query<<<(unsigned)n_q, 64, 0, s>>>(d_qlo, d_qlist, ix->fwd_base.as<int64_t>(), adj,
                                                  ix->qry.off.as<int64_t>(), ix->qry.pos.as<uint16_t>(), grad_qmass);
    if (grad_dmass)
      k_grad_w_doc<<<(unsigned)nu, 64, 0, s>>>(d_docs, d_dlo, d_dlist, ix->fwd_base.as<int64_t>(), adj, pair_q,
                                               ix->qry.off.as<int64_t>(), ix->docs.off.as<int64_t>(),
                                               ix->docs.pos.as<uint16_t>(), grad_dmass);
    FT_HIP(hipGetLastError());
    // the host lists must outlive the copies
    FT_HIP(hipStreamSynchronize(s));
  });
}
