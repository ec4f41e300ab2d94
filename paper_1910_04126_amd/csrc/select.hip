// Top-k selection per query row: the k smallest (key, doc index) pairs in
// ascending order (the k-NNS output of the Section 1 problem statement).
#include <hip/hip_runtime.h>

#include "common.h"
#include "select.h"
#include "wave.h"

namespace ft {

// Sort keys: 64-bit integer keys, or float32 costs mapped to their bit
// pattern (non-negative floats order like their bits; -0 is folded to 0).
__device__ __forceinline__ uint64_t sort_bits(uint64_t k) { return k; }
__device__ __forceinline__ uint64_t sort_bits(float c) {
  uint32_t b = __float_as_uint(c);
  return b == 0x80000000u ? 0ull : (uint64_t)b;
}
__device__ __forceinline__ void store_key(uint64_t* out, uint64_t b) { *out = b; }
__device__ __forceinline__ void store_key(float* out, uint64_t b) { *out = __uint_as_float((uint32_t)b); }

constexpr int SMALL_MAX = 4096;

// Per-row fallback flags of the window select (grown on demand, kept for the
// life of the process).
static uint32_t* topk_flags(int64_t rows) {
  static std::mutex mu;
  static DevBuf buf;
  std::lock_guard<std::mutex> lock(mu);
  return (uint32_t*)buf.ensure(rows * 4);
}

// Bitonic sort of P (power of two) (key, doc) pairs in LDS by the whole block.
__device__ void block_bitonic(uint64_t* key, uint32_t* doc, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < P; t += blockDim.x) {
        int l = t ^ j;
        if (l > t) {
          uint64_t a = key[t], b = key[l];
          uint32_t da = doc[t], db = doc[l];
          bool gt = a > b || (a == b && da > db);
          bool up = (t & k) == 0;
          if (up ? gt : !gt) {
            key[t] = b;
            key[l] = a;
            doc[t] = db;
            doc[l] = da;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Rows of at most SMALL_MAX entries: sort the whole row in LDS.
template <class K>
__global__ __launch_bounds__(256) void k_topk_small(const K* __restrict__ keys, int64_t n, const int64_t* __restrict__ docs,
                                                    int k, K* __restrict__ out_key, int64_t* __restrict__ out_doc) {
  __shared__ uint64_t sk[SMALL_MAX];
  __shared__ uint32_t sd[SMALL_MAX];
  const int64_t row = blockIdx.x;
  int P = 1;
  while (P < n) P <<= 1;
  for (int t = threadIdx.x; t < P; t += blockDim.x) {
    if (t < n) {
      sk[t] = sort_bits(keys[row * n + t]);
      sd[t] = docs ? (uint32_t)docs[row * n + t] : (uint32_t)t;
    } else {
      sk[t] = ~0ull;
      sd[t] = 0xFFFFFFFFu;
    }
  }
  __syncthreads();
  block_bitonic(sk, sd, P);
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    store_key(out_key + row * k + t, sk[t]);
    out_doc[row * k + t] = sd[t];
  }
}

// Rows of any length with the column index as doc index: radix selection of
// the k-th smallest key (11-bit digits from the top), then an ordered
// compaction of the keys below it and of the first needed keys equal to it.
template <class K, int KEYBITS>
__device__ void k_topk_radix_body(const K* __restrict__ keys, int64_t n, int k, K* __restrict__ out_key,
                                  int64_t* __restrict__ out_doc) {
  constexpr int W = 11;
  __shared__ uint32_t hist[1 << W];
  __shared__ uint64_t sk[1024];
  __shared__ uint32_t sd[1024];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_need;
  const int64_t row = blockIdx.x;
  const K* rk = keys + row * n;
  uint64_t prefix = 0, mask = 0;
  uint32_t need = (uint32_t)k;  // rank (1-based) of the wanted key among those matching the prefix
  for (int hi = KEYBITS; hi > 0; hi -= W) {
    const int w = hi >= W ? W : hi;
    const int shift = hi - w;
    const uint64_t dm = (1ull << w) - 1;
    for (int b = threadIdx.x; b < (1 << W); b += blockDim.x) hist[b] = 0;
    __syncthreads();
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
      uint64_t x = sort_bits(rk[c]);
      if ((x & mask) == prefix) atomicAdd(&hist[(x >> shift) & dm], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      // the first wavefront scans the histogram
      const int per = (1 << W) / 64;
      uint32_t loc = 0;
      for (int i = 0; i < per; ++i) loc += hist[threadIdx.x * per + i];
      uint32_t incl = wave_incl_sum(loc);
      uint32_t excl = incl - loc;
      if (excl < need && need <= incl) {
        uint32_t run = excl;
        for (int i = 0; i < per; ++i) {
          uint32_t h = hist[threadIdx.x * per + i];
          if (run + h >= need) {
            s_prefix = prefix | ((uint64_t)(threadIdx.x * per + i) << shift);
            s_need = need - run;
            break;
          }
          run += h;
        }
      }
    }
    __syncthreads();
    prefix = s_prefix;
    need = s_need;
    mask |= dm << shift;
    __syncthreads();
  }
  // prefix = the k-th smallest key T; need = how many keys equal to T to take
  const uint64_t T = prefix;
  const uint32_t take_less = (uint32_t)k - need;
  // ordered compaction: thread t owns a contiguous column range
  const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
  const int64_t c0 = min(n, (int64_t)threadIdx.x * chunk), c1 = min(n, c0 + chunk);
  uint32_t nl = 0, ne = 0;
  for (int64_t c = c0; c < c1; ++c) {
    uint64_t x = sort_bits(rk[c]);
    nl += x < T;
    ne += x == T;
  }
  // block exclusive scans of nl and ne (wave scans + per-wave totals)
  __shared__ uint32_t wl[16], we[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t il = wave_incl_sum(nl), ie = wave_incl_sum(ne);
  if (lane == 63) {
    wl[wv] = il;
    we[wv] = ie;
  }
  __syncthreads();
  uint32_t bl = 0, be = 0;
  for (int i = 0; i < wv; ++i) {
    bl += wl[i];
    be += we[i];
  }
  uint32_t pl = bl + il - nl, pe = be + ie - ne;
  for (int64_t c = c0; c < c1; ++c) {
    uint64_t x = sort_bits(rk[c]);
    if (x < T) {
      sk[pl] = x;
      sd[pl] = (uint32_t)c;
      ++pl;
    } else if (x == T) {
      if (pe < need) {
        sk[take_less + pe] = x;
        sd[take_less + pe] = (uint32_t)c;
      }
      ++pe;
    }
  }
  __syncthreads();
  int P = 1;
  while (P < k) P <<= 1;
  for (int t = k + threadIdx.x; t < P; t += blockDim.x) {
    sk[t] = ~0ull;
    sd[t] = 0xFFFFFFFFu;
  }
  __syncthreads();
  block_bitonic(sk, sd, P);
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    store_key(out_key + row * k + t, sk[t]);
    out_doc[row * k + t] = sd[t];
  }
}

// Long rows, fast path: (1) min and max of the row; all keys share the bits
// above the highest bit where min and max differ, so (2) an 11-bit histogram
// just below it splits the row finely, and (3) one more pass keeps the keys of
// lower buckets and gathers the bucket holding the k-th key into LDS, where it
// is sorted.  A bucket too large for LDS falls back to k_topk_radix.
constexpr int TIE_CAP = 2048;  // a power of two: the bitonic sort pads to one

template <class K>
__global__ __launch_bounds__(1024) void k_topk_window(const K* __restrict__ keys, int64_t n, int k,
                                                      K* __restrict__ out_key, int64_t* __restrict__ out_doc,
                                                      uint32_t* __restrict__ fallback) {
  constexpr int W = 11;
  __shared__ uint32_t hist[1 << W];
  __shared__ uint64_t sk[1024];
  __shared__ uint32_t sd[1024];
  __shared__ uint64_t tk[TIE_CAP];
  __shared__ uint32_t td[TIE_CAP];
  __shared__ uint64_t red_min[16], red_max[16];
  __shared__ uint32_t s_b, s_below, s_nl, s_nt;
  const int64_t row = blockIdx.x;
  const K* rk = keys + row * n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t mn = ~0ull, mx = 0;
  for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
    const uint64_t x = sort_bits(rk[c]);
    mn = x < mn ? x : mn;
    mx = x > mx ? x : mx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if (lane == 0) {
    red_min[wv] = mn;
    red_max[wv] = mx;
  }
  for (int b = threadIdx.x; b < (1 << W); b += blockDim.x) hist[b] = 0;
  __syncthreads();
  mn = red_min[0];
  mx = red_max[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
    mn = red_min[i] < mn ? red_min[i] : mn;
    mx = red_max[i] > mx ? red_max[i] : mx;
  }
  const uint64_t diff = mn ^ mx;
  const int D = diff ? 63 - __clzll((long long)diff) : 0;
  const int lo = D >= W - 1 ? D - (W - 1) : 0;
  for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
    const uint64_t x = sort_bits(rk[c]);
    atomicAdd(&hist[(x >> lo) & ((1u << W) - 1)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int per = (1 << W) / 64;
    uint32_t loc = 0;
    for (int i = 0; i < per; ++i) loc += hist[threadIdx.x * per + i];
    const uint32_t incl = wave_incl_sum(loc), excl = incl - loc;
    if (excl < (uint32_t)k && (uint32_t)k <= incl) {
      uint32_t run = excl;
      for (int i = 0; i < per; ++i) {
        const uint32_t h = hist[threadIdx.x * per + i];
        if (run + h >= (uint32_t)k) {
          s_b = threadIdx.x * per + i;
          s_below = run;
          break;
        }
        run += h;
      }
    }
    if (threadIdx.x == 0) s_nl = s_nt = 0;
  }
  __syncthreads();
  const uint32_t bstar = s_b, below = s_below, nties = hist[bstar];
  if (threadIdx.x == 0) fallback[row] = nties > TIE_CAP ? 1u : 0u;
  if (nties > TIE_CAP) return;
  for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
    const uint64_t x = sort_bits(rk[c]);
    const uint32_t dg = (uint32_t)((x >> lo) & ((1u << W) - 1));
    if (dg < bstar) {
      const uint32_t p = atomicAdd(&s_nl, 1u);
      sk[p] = x;
      sd[p] = (uint32_t)c;
    } else if (dg == bstar) {
      const uint32_t p = atomicAdd(&s_nt, 1u);
      tk[p] = x;
      td[p] = (uint32_t)c;
    }
  }
  __syncthreads();
  int P = 1;
  while (P < (int)nties) P <<= 1;
  for (int t = nties + threadIdx.x; t < P; t += blockDim.x) {
    tk[t] = ~0ull;
    td[t] = 0xFFFFFFFFu;
  }
  __syncthreads();
  block_bitonic(tk, td, P);
  const int need = k - (int)below;
  for (int t = threadIdx.x; t < need; t += blockDim.x) {
    sk[below + t] = tk[t];
    sd[below + t] = td[t];
  }
  int Pk = 1;
  while (Pk < k) Pk <<= 1;
  for (int t = k + threadIdx.x; t < Pk; t += blockDim.x) {
    sk[t] = ~0ull;
    sd[t] = 0xFFFFFFFFu;
  }
  __syncthreads();
  block_bitonic(sk, sd, Pk);
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    store_key(out_key + row * k + t, sk[t]);
    out_doc[row * k + t] = sd[t];
  }
}

// Rows the fast path gave up on (flag set) are redone by the radix path.
template <class K, int KEYBITS>
__global__ __launch_bounds__(1024) void k_topk_radix_if(const K* __restrict__ keys, int64_t n, int k,
                                                        K* __restrict__ out_key, int64_t* __restrict__ out_doc,
                                                        const uint32_t* __restrict__ fallback) {
  if (fallback[blockIdx.x] == 0) return;
  k_topk_radix_body<K, KEYBITS>(keys, n, k, out_key, out_doc);
}

template <class K, int KEYBITS>
static void topk_rows_impl(const K* keys, int64_t rows, int64_t n, const int64_t* docs, int k, K* out_key,
                           int64_t* out_doc, hipStream_t s) {
  FT_REQUIRE(k >= 1 && k <= n, FT_EINVAL, "k must lie in [1, number of candidates]");
  if (rows <= 0) return;
  if (n <= SMALL_MAX) {
    k_topk_small<K><<<(unsigned)rows, 256, 0, s>>>(keys, n, docs, k, out_key, out_doc);
  } else {
    FT_REQUIRE(docs == nullptr, FT_ERANGE, "candidate lists longer than 4096 are not supported");
    FT_REQUIRE(k <= 1024, FT_ERANGE, "k > 1024 needs at most 4096 candidates");
    // the fast path flags rows it could not finish; those are redone
    uint32_t* flag = topk_flags(rows);
    k_topk_window<K><<<(unsigned)rows, 1024, 0, s>>>(keys, n, k, out_key, out_doc, flag);
    k_topk_radix_if<K, KEYBITS><<<(unsigned)rows, 1024, 0, s>>>(keys, n, k, out_key, out_doc, flag);
  }
  FT_HIP(hipGetLastError());
}

void topk_rows(const uint64_t* keys, int64_t rows, int64_t n, const int64_t* docs, int k, uint64_t* out_key,
               int64_t* out_doc, hipStream_t s) {
  topk_rows_impl<uint64_t, 64>(keys, rows, n, docs, k, out_key, out_doc, s);
}

void topk_rows(const float* keys, int64_t rows, int64_t n, const int64_t* docs, int k, float* out_key,
               int64_t* out_doc, hipStream_t s) {
  topk_rows_impl<float, 32>(keys, rows, n, docs, k, out_key, out_doc, s);
}

}  // namespace ft
