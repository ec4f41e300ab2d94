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
__device__ __forceinline__ uint64_t sort_bits(uint32_t k) { return (uint64_t)k; }
__device__ __forceinline__ uint64_t sort_bits(float c) {
  uint32_t b = __float_as_uint(c);
  return b == 0x80000000u ? 0ull : (uint64_t)b;
}
// sort_bits of a 4-byte key given by its bit pattern
template <class K>
__device__ __forceinline__ uint64_t sort_bits_of(uint32_t b);
template <>
__device__ __forceinline__ uint64_t sort_bits_of<uint32_t>(uint32_t b) { return (uint64_t)b; }
template <>
__device__ __forceinline__ uint64_t sort_bits_of<float>(uint32_t b) { return sort_bits(__uint_as_float(b)); }
__device__ __forceinline__ void store_key(uint64_t* out, uint64_t b) { *out = b; }
__device__ __forceinline__ void store_key(uint32_t* out, uint64_t b) { *out = (uint32_t)b; }
__device__ __forceinline__ void store_key(float* out, uint64_t b) { *out = __uint_as_float((uint32_t)b); }

constexpr int SMALL_MAX = 4096;

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

constexpr int TIE_CAP = 2048;  // a power of two: the bitonic sort pads to one

__device__ __forceinline__ uint64_t shr64(uint64_t x, int s) { return s >= 64 ? 0ull : x >> s; }

constexpr int COLLECT_CAP = 4096;  // keys gathered by the one-pass path (a power of two)

// Block-wide digit histograms over the keys of columns [0, n_cols): starting
// with the bits >= hs fixed to sel, find the 11-bit bucket (then the next 11
// bits inside it, ...) holding the target-th smallest key, until that bucket
// holds at most stop keys or the last bit is reached.  On return, keys with
// shr64(x, hs) < sel number `below`, and those equal to sel number `nties`.
// Columns: [0, n_cols) when bstride == 16, else the n_cols / 16 blocks of 16
// consecutive columns starting every bstride columns (a sample spread over
// the whole row; bstride a multiple of 16).
template <class K>
__device__ void digit_levels(const K* __restrict__ rk, int64_t n_cols, int64_t bstride, uint32_t target,
                             uint32_t stop, int& hs, uint64_t& sel, uint32_t& below, uint32_t& nties,
                             uint32_t* hist, uint32_t* s_b, uint32_t* s_below) {
  constexpr int W = 11;
  int lo = hs - W;
  below = 0;
  while (true) {
    const uint32_t dmask = (1u << (hs - lo)) - 1u;
    for (int b = threadIdx.x; b < (1 << W); b += blockDim.x) hist[b] = 0;
    __syncthreads();
    auto count = [&](uint64_t x) {
      if (shr64(x, hs) == sel) atomicAdd(&hist[(uint32_t)(x >> lo) & dmask], 1u);
    };
    bool done = false;
    if constexpr (sizeof(K) == 4) {
      // 4-byte keys of a 16-byte aligned prefix: four per load
      if ((n_cols & 3) == 0 && (reinterpret_cast<uintptr_t>(rk) & 15) == 0) {
        const uint4* r4 = reinterpret_cast<const uint4*>(rk);
        for (int64_t c = threadIdx.x; c < (n_cols >> 2); c += blockDim.x) {
          const uint4 v = r4[(c >> 2) * (bstride >> 2) + (c & 3)];
          count(sort_bits_of<K>(v.x));
          count(sort_bits_of<K>(v.y));
          count(sort_bits_of<K>(v.z));
          count(sort_bits_of<K>(v.w));
        }
        done = true;
      }
    }
    if (!done)
      for (int64_t c = threadIdx.x; c < n_cols; c += blockDim.x) count(sort_bits(rk[(c >> 4) * bstride + (c & 15)]));
    __syncthreads();
    if (threadIdx.x < 64) {
      const int per = (1 << W) / 64;
      uint32_t loc = 0;
      for (int i = 0; i < per; ++i) loc += hist[threadIdx.x * per + i];
      const uint32_t incl = wave_incl_sum(loc) + below, excl = incl - loc;
      if (excl < target && target <= incl) {
        uint32_t run = excl;
        for (int i = 0; i < per; ++i) {
          const uint32_t h = hist[threadIdx.x * per + i];
          if (run + h >= target) {
            *s_b = threadIdx.x * per + i;
            *s_below = run;
            break;
          }
          run += h;
        }
      }
    }
    __syncthreads();
    const uint32_t b = *s_b;
    below = *s_below;
    nties = hist[b];
    sel = (sel << (hs - lo)) | b;
    hs = lo;
    __syncthreads();  // hist and s_b are rewritten by the next level
    if (nties <= stop || lo == 0) break;
    lo = lo >= W ? lo - W : 0;
  }
}

// Rows longer than SMALL_MAX.  All keys share the bits above the highest bit
// where the row's min and max differ (given, or found in a first pass).
//  * One-pass path: digit histograms over a sample of the row (blocks of 16
//    consecutive columns spread evenly over the whole row, a sixteenth of it
//    and at least 16384 columns; the whole row when short) find a threshold
//    below which a little more than k * sample / n of the sample keys lie;
//    one pass over the row gathers every key at or below it into
//    LDS.  When that gathers between k and COLLECT_CAP keys, the k smallest
//    are among them (every key left out is larger than every key taken), and
//    a sort of the gathered keys finishes the row.
//  * Otherwise (a threshold too tight or too loose, or a long run of equal
//    keys) the exact path: digit histograms over the whole row, refined
//    inside the bucket of the k-th key while it holds more than TIE_CAP keys;
//    one pass collects the keys below that bucket and the bucket itself,
//    which are sorted in LDS.  A final bucket of more than TIE_CAP keys is a
//    run of equal keys, of which the lowest columns are taken in order.
template <class K>
__global__ __launch_bounds__(1024) void k_topk_window(const K* __restrict__ keys, int64_t n, int k,
                                                      const uint64_t* __restrict__ minmax,
                                                      K* __restrict__ out_key, int64_t* __restrict__ out_doc,
                                                      uint32_t* __restrict__ exact_rows) {
  constexpr int W = 11;
  __shared__ uint32_t hist[1 << W];
  __shared__ uint64_t bufk[COLLECT_CAP];
  __shared__ uint32_t bufd[COLLECT_CAP];
  __shared__ uint64_t red_min[16], red_max[16];
  __shared__ uint32_t s_b, s_below, s_nl, s_nt;
  // the exact path's arrays live in the same buffers
  uint64_t* sk = bufk;          // [1024] keys below the final bucket, then the answer
  uint32_t* sd = bufd;
  uint64_t* tk = bufk + 1024;   // [TIE_CAP] the final bucket
  uint32_t* td = bufd + 1024;
  const int64_t row = blockIdx.x;
  const K* rk = keys + row * n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t mn, mx;
  if (minmax) {
    mn = minmax[2 * row];
    mx = minmax[2 * row + 1];
  } else {
    mn = ~0ull;
    mx = 0;
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
    __syncthreads();
    mn = red_min[0];
    mx = red_max[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      mn = red_min[i] < mn ? red_min[i] : mn;
      mx = red_max[i] > mx ? red_max[i] : mx;
    }
  }
  const uint64_t diff = mn ^ mx;
  const int D = diff ? 63 - __clzll((long long)diff) : 0;
  const int hs0 = D >= W - 1 ? D + 1 : W;  // bits >= hs0 are the same in every key
  int hs;
  uint64_t sel;
  uint32_t below, nties;

  // ---- one-pass path
  {
    // sample: nb blocks of 16 columns, one every bstride columns
    const int64_t want = n <= 65536 ? n : (n / 16 > 16384 ? n / 16 : 16384);
    const int64_t nb = want == n ? 0 : want / 16;
    const int64_t bstride = nb ? (n / nb) & ~int64_t(15) : 16;
    const int64_t ns = nb ? nb * 16 : n;
    const uint32_t target =
        ns == n ? (uint32_t)k : (uint32_t)min((int64_t)ns, (int64_t)k * ns / n * 115 / 100 + 16);
    hs = hs0;
    sel = shr64(mn, hs0);
    digit_levels(rk, ns, bstride, target, 16u, hs, sel, below, nties, hist, &s_b, &s_below);
    if (threadIdx.x == 0) s_nl = 0;
    __syncthreads();
    auto collect = [&](uint64_t x, int64_t c) {
      if (shr64(x, hs) <= sel) {
        const uint32_t p = atomicAdd(&s_nl, 1u);
        if (p < (uint32_t)COLLECT_CAP) {
          bufk[p] = x;
          bufd[p] = (uint32_t)c;
        }
      }
    };
    bool done = false;
    if constexpr (sizeof(K) == 4) {
      // 4-byte keys of a 16-byte aligned row: four per load
      if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(rk) & 15) == 0) {
        const uint4* r4 = reinterpret_cast<const uint4*>(rk);
        for (int64_t c = threadIdx.x; c < (n >> 2); c += blockDim.x) {
          const uint4 v = r4[c];
          collect(sort_bits_of<K>(v.x), 4 * c);
          collect(sort_bits_of<K>(v.y), 4 * c + 1);
          collect(sort_bits_of<K>(v.z), 4 * c + 2);
          collect(sort_bits_of<K>(v.w), 4 * c + 3);
        }
        done = true;
      }
    }
    if (!done)
      for (int64_t c = threadIdx.x; c < n; c += blockDim.x) collect(sort_bits(rk[c]), c);
    __syncthreads();
    const uint32_t got = s_nl;
    if (got >= (uint32_t)k && got <= (uint32_t)COLLECT_CAP) {
      int P = 1;
      while (P < (int)got) P <<= 1;
      for (int t = got + threadIdx.x; t < P; t += blockDim.x) {
        bufk[t] = ~0ull;
        bufd[t] = 0xFFFFFFFFu;
      }
      __syncthreads();
      block_bitonic(bufk, bufd, P);
      for (int t = threadIdx.x; t < k; t += blockDim.x) {
        store_key(out_key + row * k + t, bufk[t]);
        out_doc[row * k + t] = bufd[t];
      }
      return;
    }
    __syncthreads();  // the buffers are reused below
  }

  // ---- exact path
  if (exact_rows && threadIdx.x == 0) atomicAdd(exact_rows, 1u);
  hs = hs0;
  sel = shr64(mn, hs0);
  digit_levels(rk, n, 16, (uint32_t)k, (uint32_t)TIE_CAP, hs, sel, below, nties, hist, &s_b, &s_below);
  if (threadIdx.x == 0) s_nl = s_nt = 0;
  __syncthreads();
  const bool many = nties > TIE_CAP;  // then every tie key is the same value
  for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
    const uint64_t x = sort_bits(rk[c]);
    const uint64_t h = shr64(x, hs);
    // (below < k <= 1024 keys lie under the bucket and nties <= TIE_CAP in
    // it when every key lies in [min, max]; the bounds keep the writes in
    // their arrays even for a row that breaks that)
    if (h < sel) {
      const uint32_t p = atomicAdd(&s_nl, 1u);
      if (p < 1024u) {
        sk[p] = x;
        sd[p] = (uint32_t)c;
      }
    } else if (h == sel && !many) {
      const uint32_t p = atomicAdd(&s_nt, 1u);
      if (p < (uint32_t)TIE_CAP) {
        tk[p] = x;
        td[p] = (uint32_t)c;
      }
    }
  }
  if (many) {
    // equal keys go to the lowest columns: collect the first k - below of
    // them in column order, a block-wide ordered compaction per stretch
    const uint32_t need = (uint32_t)k - below;
    uint32_t have = 0;
    for (int64_t c0 = 0; c0 < n && have < need; c0 += blockDim.x) {
      const int64_t c = c0 + threadIdx.x;
      const bool hit = c < n && shr64(sort_bits(rk[c]), hs) == sel;
      const uint64_t m = __ballot(hit);
      const uint32_t before_lane = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) hist[wv] = (uint32_t)__popcll(m);
      __syncthreads();
      uint32_t pos = have + before_lane;
      uint32_t tot = 0;
      for (int j = 0; j < (int)(blockDim.x >> 6); ++j) {
        if (j < wv) pos += hist[j];
        tot += hist[j];
      }
      if (hit && pos < need) {
        tk[pos] = sort_bits(rk[c]);
        td[pos] = (uint32_t)c;
      }
      have += tot;
      __syncthreads();  // hist is rewritten by the next stretch
    }
    nties = need;
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

template <class K>
static void topk_rows_impl(const K* keys, int64_t rows, int64_t n, const int64_t* docs, int k, K* out_key,
                           int64_t* out_doc, const uint64_t* minmax, hipStream_t s, uint32_t* exact_rows) {
  FT_REQUIRE(k >= 1 && k <= n, FT_EINVAL, "k must lie in [1, number of candidates]");
  if (rows <= 0) return;
  if (n <= SMALL_MAX) {
    k_topk_small<K><<<(unsigned)rows, 256, 0, s>>>(keys, n, docs, k, out_key, out_doc);
  } else {
    FT_REQUIRE(docs == nullptr, FT_ERANGE, "candidate lists longer than 4096 are not supported");
    FT_REQUIRE(k <= 1024, FT_ERANGE, "k > 1024 needs at most 4096 candidates");
    k_topk_window<K><<<(unsigned)rows, 1024, 0, s>>>(keys, n, k, minmax, out_key, out_doc, exact_rows);
  }
  FT_HIP(hipGetLastError());
}

void topk_rows(const uint64_t* keys, int64_t rows, int64_t n, const int64_t* docs, int k, uint64_t* out_key,
               int64_t* out_doc, hipStream_t s, const uint64_t* minmax, uint32_t* exact_rows) {
  topk_rows_impl<uint64_t>(keys, rows, n, docs, k, out_key, out_doc, minmax, s, exact_rows);
}

__global__ void k_widen_keys(const uint32_t* __restrict__ in, int64_t n, int shift, uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint64_t)in[i] << shift;
}

void topk_rows(const uint32_t* keys, int64_t rows, int64_t n, const int64_t* docs, int k, uint64_t* out_key, int shift,
               int64_t* out_doc, uint32_t* tmp_key, hipStream_t s, const uint64_t* minmax, uint32_t* exact_rows) {
  topk_rows_impl<uint32_t>(keys, rows, n, docs, k, tmp_key, out_doc, minmax, s, exact_rows);
  if (rows > 0) {
    k_widen_keys<<<(unsigned)ceil_div(rows * k, 256), 256, 0, s>>>(tmp_key, rows * k, shift, out_key);
    FT_HIP(hipGetLastError());
  }
}

void topk_rows(const float* keys, int64_t rows, int64_t n, const int64_t* docs, int k, float* out_key,
               int64_t* out_doc, hipStream_t s) {
  topk_rows_impl<float>(keys, rows, n, docs, k, out_key, out_doc, nullptr, s, nullptr);
}

}  // namespace ft
