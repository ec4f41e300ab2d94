// Preprocessing: the randomly shifted quadtree over the ground points and the
// packed, Morton-sorted dataset (paper Section 2, "Generic Quadtree"; the
// dataset preprocessing of the Section 1 problem statement).
//
// Everything runs on the device.  The tree is never materialised as nodes:
// points are renumbered in Morton (depth-first) order, so every cell is a
// contiguous rank range and the depth of the deepest cell shared by two
// ranks a < b is the minimum of the adjacent-pair LCA depths over [a, b),
// answered by a range-minimum table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "wave.h"

namespace ft {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

void* DevBuf::ensure(size_t n) {
  if (n <= bytes && p) return p;
  release();
  size_t want = std::max<size_t>(n, 256);
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    throw Error(FT_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  bytes = want;
  return p;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void Dists::release() {
  for (DevBuf* b : {&off, &rank, &mass, &pos, &lcp, &ecnt, &ekey, &emass, &S, &tmp}) b->release();
  n = nnz = emb_nnz = 0;
  max_size = 0;
}

void BatchedGraphs::reset() {
  for (hipGraphExec_t* e : {&pre, &main})
    if (*e) (void)hipGraphExecDestroy(*e);
  pre = main = nullptr;
  key.clear();
}

std::string describe_flags(uint32_t f) {
  std::string s;
  if (f & ERR_ID_RANGE) s += " point id >= V;";
  if (f & ERR_ZERO_MASS) s += " zero mass;";
  if (f & ERR_MASS_SUM) s += " masses do not sum to 2^Q;";
  if (f & ERR_DUPLICATE) s += " duplicate point id in a distribution;";
  if (f & ERR_SIZE) s += " support larger than FT_MAX_SUPPORT;";
  if (f & ERR_EMPTY) s += " empty distribution or bad offsets;";
  if (f & ERR_FLOW) s += " internal flow inconsistency;";
  if (f & ERR_NONFINITE) s += " non-finite value;";
  return s;
}

uint32_t read_and_clear_status(ft_index* ix, hipStream_t s) {
  uint32_t h[8];
  FT_HIP(hipMemcpyAsync(h, ix->status.p, sizeof(h), hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
  FT_HIP(hipMemsetAsync(ix->status.p, 0, sizeof(h), s));
  return h[0];
}

// ------------------------------------------------------------- scan (i64) --

constexpr int SCAN_TB = 1024;  // elements per block (256 threads x 4)

__global__ void k_scan_blocksum(const int64_t* __restrict__ in, int64_t n, int64_t* __restrict__ bsum) {
  __shared__ int64_t red[256];
  int64_t base = (int64_t)blockIdx.x * SCAN_TB;
  int64_t s = 0;
  for (int i = threadIdx.x; i < SCAN_TB; i += 256)
    if (base + i < n) s += in[base + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// Block-local exclusive scan of SCAN_TB values held 4 per thread.
__device__ void block_excl_scan_1024(int64_t v[4], int64_t* sh, int64_t carry_in, int64_t* total) {
  int t = threadIdx.x;
  int64_t loc = v[0] + v[1] + v[2] + v[3];
  sh[t] = loc;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int64_t u = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += u;
    __syncthreads();
  }
  int64_t excl = sh[t] - loc + carry_in;
  if (total) *total = sh[255];
  __syncthreads();
  int64_t run = excl;
  for (int i = 0; i < 4; ++i) {
    int64_t x = v[i];
    v[i] = run;
    run += x;
  }
}

__global__ void k_scan_serial_blocks(int64_t* __restrict__ bsum, int64_t nb) {
  // exclusive scan of nb block sums by one block, 1024 at a time
  __shared__ int64_t sh[256];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += SCAN_TB) {
    int64_t v[4];
    for (int i = 0; i < 4; ++i) {
      int64_t idx = base + threadIdx.x * 4 + i;
      v[i] = idx < nb ? bsum[idx] : 0;
    }
    int64_t tot;
    block_excl_scan_1024(v, sh, carry, &tot);
    for (int i = 0; i < 4; ++i) {
      int64_t idx = base + threadIdx.x * 4 + i;
      if (idx < nb) bsum[idx] = v[i];
    }
    carry += tot;
    __syncthreads();
  }
}

__global__ void k_scan_apply(const int64_t* __restrict__ in, int64_t n, const int64_t* __restrict__ boff,
                             int64_t* __restrict__ out) {
  __shared__ int64_t sh[256];
  int64_t base = (int64_t)blockIdx.x * SCAN_TB;
  int64_t v[4];
  for (int i = 0; i < 4; ++i) {
    int64_t idx = base + threadIdx.x * 4 + i;
    v[i] = idx < n ? in[idx] : 0;
  }
  block_excl_scan_1024(v, sh, boff[blockIdx.x], nullptr);
  for (int i = 0; i < 4; ++i) {
    int64_t idx = base + threadIdx.x * 4 + i;
    if (idx < n) out[idx] = v[i];
    if (idx == n - 1) out[n] = v[i] + in[n - 1];  // total
  }
}

int64_t scan_tmp_elems(int64_t n) { return ceil_div(std::max<int64_t>(n, 1), SCAN_TB); }

// out[0..n] = exclusive prefix sums of in[0..n) (out has n + 1 entries);
// tmp holds scan_tmp_elems(n) int64.  Launches only (capturable).
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
  int64_t nb = scan_tmp_elems(n);
  k_scan_blocksum<<<(unsigned)nb, 256, 0, s>>>(in, n, tmp);
  k_scan_serial_blocks<<<1, 256, 0, s>>>(tmp, nb);
  k_scan_apply<<<(unsigned)nb, 256, 0, s>>>(in, n, tmp, out);
  FT_HIP(hipGetLastError());
}

// ------------------------------------------------------------ grid codes --

constexpr int MM_ROWS = 512;

__global__ void k_minmax_part(const float* __restrict__ X, int64_t V, int d, float* __restrict__ pmin,
                              float* __restrict__ pmax) {
  int64_t r0 = (int64_t)blockIdx.x * MM_ROWS;
  int64_t r1 = min(V, r0 + MM_ROWS);
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    float mn = INFINITY, mx = -INFINITY;
    bool bad = false;
    for (int64_t r = r0; r < r1; ++r) {
      float x = X[r * d + i];
      if (!(x == x) || isinf(x)) bad = true;
      mn = fminf(mn, x);
      mx = fmaxf(mx, x);
    }
    pmin[(int64_t)blockIdx.x * d + i] = bad ? NAN : mn;
    pmax[(int64_t)blockIdx.x * d + i] = mx;
  }
}

__global__ void k_minmax_final(const float* __restrict__ pmin, const float* __restrict__ pmax, int nb, int d,
                               float* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d) return;
  float mn = INFINITY, mx = -INFINITY;
  bool bad = false;
  for (int b = 0; b < nb; ++b) {
    float a = pmin[(int64_t)b * d + i];
    if (!(a == a)) bad = true;
    mn = fminf(mn, a);
    mx = fmaxf(mx, pmax[(int64_t)b * d + i]);
  }
  out[i] = bad ? NAN : mn;
  out[d + i] = mx;
}

// code = floor((x - lo_i) * scale) clamped to [0, 2^(B-1)], + 2^(B-1) - shift_i,
// in IEEE float64 without contraction.
__global__ void k_codes(const float* __restrict__ X, int64_t V, int d, const double* __restrict__ lo,
                        const int64_t* __restrict__ shift, double scale, int B, uint32_t* __restrict__ code) {
#pragma clang fp contract(off)
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= V * d) return;
  int i = (int)(idx % d);
  const double half = (double)(1ll << (B - 1));
  double diff = (double)X[idx] - lo[i];
  double y = diff * scale;
  double g = floor(y);
  if (g < 0.0) g = 0.0;
  if (g > half) g = half;
  code[idx] = (uint32_t)((int64_t)g + (1ll << (B - 1)) - shift[i]);
}

// Morton order of two points by their grid codes: the first level at which
// their cells differ is the highest differing bit over all dimensions; at
// that level the lowest such dimension decides, 0 before 1.  Equal codes fall
// back to the point id.
__device__ __forceinline__ bool morton_less(const uint32_t* __restrict__ code, int d, int B, uint32_t a,
                                            uint32_t b) {
  if (b == 0xFFFFFFFFu) return a != b;
  if (a == 0xFFFFFFFFu) return false;
  const uint32_t* qa = code + (int64_t)a * d;
  const uint32_t* qb = code + (int64_t)b * d;
  int best = -1, dim = 0;
  for (int i = 0; i < d; ++i) {
    uint32_t x = qa[i] ^ qb[i];
    if (x) {
      int hb = 31 - __clz(x);
      if (hb > best) {
        best = hb;
        dim = i;
        if (hb == B - 1) break;  // nothing can be higher; lowest dim wins
      }
    }
  }
  if (best < 0) return a < b;
  return ((qa[dim] >> best) & 1u) == 0u;
}

__global__ void k_iota_pad(uint32_t* __restrict__ idx, int64_t V, int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) idx[i] = i < V ? (uint32_t)i : 0xFFFFFFFFu;
}

__global__ void k_bitonic_step(uint32_t* __restrict__ idx, int64_t N, int64_t k, int64_t j,
                               const uint32_t* __restrict__ code, int d, int B) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t l = i ^ j;
  if (l <= i) return;
  uint32_t a = idx[i], b = idx[l];
  bool up = (i & k) == 0;
  bool swap = up ? morton_less(code, d, B, b, a) : morton_less(code, d, B, a, b);
  if (swap) {
    idx[i] = b;
    idx[l] = a;
  }
}

// Depth of the deepest cell shared by Morton neighbours r and r+1.
__global__ void k_adjacent_lcp(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ code, int64_t V,
                               int d, int B, uint8_t* __restrict__ glcp) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= V) return;
  if (r == V - 1) {
    glcp[r] = 0;
    return;
  }
  const uint32_t* qa = code + (int64_t)perm[r] * d;
  const uint32_t* qb = code + (int64_t)perm[r + 1] * d;
  uint32_t orx = 0;
  for (int i = 0; i < d; ++i) orx |= qa[i] ^ qb[i];
  glcp[r] = orx ? (uint8_t)(B - 1 - (31 - __clz(orx))) : (uint8_t)B;
}

// A point is alone from the depth after the deepest cell it shares with a
// Morton neighbour; depth B ends every path.
__global__ void k_leaf_depth(const uint8_t* __restrict__ glcp, int64_t V, int B, uint8_t* __restrict__ leafd,
                             uint32_t* __restrict__ status) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= V) return;
  int left = r > 0 ? glcp[r - 1] : -1;
  int right = r < V - 1 ? glcp[r] : -1;
  int l = max(left, right) + 1;
  if (l > B) l = B;
  leafd[r] = (uint8_t)l;
  atomicMax(status + 2, (uint32_t)l);
}

__global__ void k_node_start(const uint8_t* __restrict__ glcp, const uint8_t* __restrict__ leafd, int64_t V, int k,
                             int64_t* __restrict__ flag) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= V) return;
  flag[r] = (leafd[r] >= k && (r == 0 || glcp[r - 1] < k)) ? 1 : 0;
}

__global__ void k_node_index(const int64_t* __restrict__ flag, const int64_t* __restrict__ excl,
                             const uint8_t* __restrict__ leafd, int64_t V, int k, uint32_t* __restrict__ anc) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= V) return;
  anc[r] = leafd[r] >= k ? (uint32_t)(excl[r] + flag[r] - 1) : 0xFFFFFFFFu;
}

__global__ void k_st_level(uint8_t* __restrict__ st, int64_t V, int j) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= V) return;
  const uint8_t* prev = st + (int64_t)(j - 1) * V;
  int64_t h = 1ll << (j - 1);
  uint8_t v = 0;
  if (r + 2 * h <= V - 1) v = min(prev[r], prev[r + h]);
  st[(int64_t)j * V + r] = v;
}

// One wavefront per row: the row in Morton order, padded with zeros, and its
// squared norm in fp64.
__global__ __launch_bounds__(64) void k_permute_rows(const float* __restrict__ X, const uint32_t* __restrict__ perm,
                                                     int64_t V, int d, int dp, float* __restrict__ Xm,
                                                     double* __restrict__ Xn, uint32_t* __restrict__ inv) {
  int64_t r = blockIdx.x;
  if (r >= V) return;
  uint32_t p = perm[r];
  double n2 = 0.0;
  for (int c = threadIdx.x; c < dp; c += 64) {
    const float v = c < d ? X[(int64_t)p * d + c] : 0.0f;
    Xm[r * dp + c] = v;
    n2 = fma((double)v, (double)v, n2);
  }
  n2 = wave_sum(n2);
  if (threadIdx.x == 0) {
    inv[p] = (uint32_t)r;
    Xn[r] = n2;
  }
}

// ---------------------------------------------------------- distributions --

__global__ void k_check_offsets(const int64_t* __restrict__ off, int64_t n, uint32_t* __restrict__ status) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0 && off[0] != 0) atomicOr(status, ERR_EMPTY);
  if (j >= n) return;
  int64_t s = off[j + 1] - off[j];
  if (s < 1) atomicOr(status, ERR_EMPTY);
  else if (s > FT_MAX_SUPPORT) atomicOr(status, ERR_SIZE);
  else atomicMax(status + 1, (uint32_t)s);
}

// One wavefront per distribution: validate, map ids to Morton ranks, sort by
// rank, record adjacent LCA depths and count l1-embedding entries.
__global__ __launch_bounds__(64) void k_prep_sort(
    const int64_t* __restrict__ off, const uint32_t* __restrict__ id, const uint32_t* __restrict__ mass_in,
    int64_t n, const uint32_t* __restrict__ inv, const uint8_t* __restrict__ st, const uint8_t* __restrict__ leafd,
    int64_t V, int B, int Q, uint32_t* __restrict__ rank_out, uint32_t* __restrict__ mass_out,
    uint16_t* __restrict__ pos_out, uint8_t* __restrict__ lcp_out, int64_t* __restrict__ ecnt,
    uint32_t* __restrict__ status) {
  __shared__ uint64_t key[FT_MAX_SUPPORT];
  const int64_t j = blockIdx.x;
  if (j >= n) return;
  const int lane = lane_id();
  const int64_t a = off[j];
  const int s = (int)(off[j + 1] - a);
  if (s < 1 || s > FT_MAX_SUPPORT) return;  // reported by k_check_offsets
  int P = 1;
  while (P < s) P <<= 1;
  uint64_t msum = 0;
  uint32_t bad = 0;
  for (int t = lane; t < P; t += 64) {
    if (t < s) {
      uint32_t p = id[a + t];
      uint32_t m = mass_in[a + t];
      msum += m;
      if (m == 0) bad |= ERR_ZERO_MASS;
      uint32_t r = 0xFFFFFFFFu;
      if (p >= (uint64_t)V) bad |= ERR_ID_RANGE;
      else r = inv[p];
      key[t] = ((uint64_t)r << 16) | (uint32_t)t;
    } else {
      key[t] = ~0ull;
    }
  }
  msum = wave_sum(msum);
  if (lane == 0 && msum != (1ull << Q)) bad |= ERR_MASS_SUM;
  __syncthreads();
  // bitonic sort of P keys by one wavefront
  for (int k = 2; k <= P; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int t = lane; t < P; t += 64) {
        int l = t ^ jj;
        if (l > t) {
          uint64_t x = key[t], y = key[l];
          bool up = (t & k) == 0;
          if (up ? (y < x) : (x < y)) {
            key[t] = y;
            key[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  int64_t cnt = 0;
  for (int t = lane; t < s; t += 64) {
    uint32_t r = (uint32_t)(key[t] >> 16);
    uint32_t p = (uint32_t)(key[t] & 0xFFFFu);
    rank_out[a + t] = r;
    mass_out[a + t] = mass_in[a + p];
    pos_out[a + t] = (uint16_t)p;
    int lc = 0;
    if (t + 1 < s) {
      uint32_t r2 = (uint32_t)(key[t + 1] >> 16);
      if (r2 == r) bad |= ERR_DUPLICATE;
      if (!(bad & ERR_ID_RANGE) && r2 != 0xFFFFFFFFu && r != 0xFFFFFFFFu) lc = lca_depth(st, V, B, r, r2);
    }
    lcp_out[a + t] = (uint8_t)lc;
    int prev = 0;
    if (t > 0) {
      uint32_t r0 = (uint32_t)(key[t - 1] >> 16);
      if (r0 != 0xFFFFFFFFu && r != 0xFFFFFFFFu && r0 != r) prev = lca_depth(st, V, B, r0, r);
    }
    int ld = r != 0xFFFFFFFFu ? (int)leafd[r] : 0;
    cnt += ld > prev ? ld - prev : 0;
  }
  cnt = wave_sum(cnt);
  bad = wave_or(bad);
  if (lane == 0) {
    ecnt[j] = cnt;
    if (bad) atomicOr(status, bad);
  }
}

// One wavefront per distribution: write the l1-embedding entries (node key,
// node mass) depth by depth (all depth-1 cells first), and the weighted total
// S = sum 2^(B-depth) * mass.  Item t opens the cells of depths
// (lcp(t-1, t), leaf depth of t]; a cell's mass runs over the following items
// while their adjacent LCA depth stays >= its depth.
__global__ __launch_bounds__(64) void k_emb_fill(
    const int64_t* __restrict__ off, const uint32_t* __restrict__ rank, const uint32_t* __restrict__ mass,
    const uint8_t* __restrict__ lcp, int64_t n, const int64_t* __restrict__ eoff,
    const uint8_t* __restrict__ leafd, const uint32_t* __restrict__ anc, int64_t V, int B,
    uint32_t* __restrict__ ekey, uint32_t* __restrict__ emass, uint64_t* __restrict__ S) {
  const int64_t j = blockIdx.x;
  if (j >= n) return;
  const int lane = lane_id();
  const int64_t a = off[j];
  const int s = (int)(off[j + 1] - a);
  const int C = (s + 63) / 64;
  const int t0 = min(s, lane * C), t1 = min(s, t0 + C);
  int maxd = 0;
  for (int t = t0; t < t1; ++t) maxd = max(maxd, (int)leafd[rank[a + t]]);
  maxd = wave_max(maxd);
  int64_t base = eoff[j];
  uint64_t Ssum = 0;
  for (int k = 1; k <= maxd; ++k) {
    int mine = 0;
    for (int t = t0; t < t1; ++t) {
      const int prev = t > 0 ? lcp[a + t - 1] : 0;
      mine += (prev < k && k <= (int)leafd[rank[a + t]]) ? 1 : 0;
    }
    const int incl = wave_incl_sum(mine);
    int64_t pos = base + incl - mine;
    for (int t = t0; t < t1; ++t) {
      const uint32_t r = rank[a + t];
      const int prev = t > 0 ? lcp[a + t - 1] : 0;
      if (prev < k && k <= (int)leafd[r]) {
        uint64_t m = mass[a + t];
        for (int u = t; u + 1 < s && lcp[a + u] >= k; ++u) m += mass[a + u + 1];
        ekey[pos] = ((uint32_t)k << KEY_DEPTH_SHIFT) | anc[(int64_t)(k - 1) * V + r];
        emass[pos] = (uint32_t)m;
        Ssum += m << (B - k);
        ++pos;
      }
    }
    base += __shfl(incl, 63, 64);
  }
  Ssum = wave_sum(Ssum);
  if (lane == 0) S[j] = Ssum;
}

void launch_check_offsets(const int64_t* off, int64_t n, uint32_t* status, hipStream_t s) {
  k_check_offsets<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(off, n, status);
  FT_HIP(hipGetLastError());
}

void launch_prep_sort(const ft_index* ix, const int64_t* off, const uint32_t* id, const uint32_t* mass, int64_t n,
                      uint32_t* rank, uint32_t* mass_out, uint16_t* pos, uint8_t* lcp, int64_t* cnt,
                      uint32_t* status, hipStream_t s) {
  k_prep_sort<<<(unsigned)n, 64, 0, s>>>(off, id, mass, n, ix->inv.as<uint32_t>(), ix->st.as<uint8_t>(),
                                        ix->leafd.as<uint8_t>(), ix->V, ix->B, ix->Q, rank, mass_out, pos, lcp, cnt,
                                        status);
  FT_HIP(hipGetLastError());
}

void prepare_dists(ft_index* ix, Dists& D, const int64_t* off, const uint32_t* id, const uint32_t* mass,
                   int64_t n, bool with_embedding, hipStream_t s, const char* what) {
  FT_REQUIRE(n >= 1, FT_EINVAL, std::string(what) + ": need at least one distribution");
  FT_REQUIRE(off && id && mass, FT_EINVAL, std::string(what) + ": null array");
  D.n = n;
  int64_t* doff = (int64_t*)D.off.ensure((n + 1) * sizeof(int64_t));
  FT_HIP(hipMemcpyAsync(doff, off, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  k_check_offsets<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(doff, n, ix->status.as<uint32_t>());
  FT_HIP(hipGetLastError());
  uint32_t h[8];
  int64_t nnz = 0;
  FT_HIP(hipMemcpyAsync(h, ix->status.p, sizeof(h), hipMemcpyDeviceToHost, s));
  FT_HIP(hipMemcpyAsync(&nnz, doff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
  FT_HIP(hipMemsetAsync(ix->status.p, 0, sizeof(h), s));
  if (h[0] & ERR_SIZE) throw Error(FT_ERANGE, std::string(what) + ": support larger than FT_MAX_SUPPORT");
  if (h[0]) throw Error(FT_EINVAL, std::string(what) + ":" + describe_flags(h[0]));
  D.nnz = nnz;
  D.max_size = (int32_t)h[1];
  D.rank.ensure(nnz * 4);
  D.mass.ensure(nnz * 4);
  D.pos.ensure(nnz * 2);
  D.lcp.ensure(nnz);
  int64_t* cnt = (int64_t*)D.ecnt.ensure((n + 1) * sizeof(int64_t));
  // per-distribution counts, then the scan's block sums
  int64_t* tmp = (int64_t*)D.tmp.ensure((n + scan_tmp_elems(n)) * sizeof(int64_t));
  k_prep_sort<<<(unsigned)n, 64, 0, s>>>(doff, id, mass, n, ix->inv.as<uint32_t>(), ix->st.as<uint8_t>(),
                                        ix->leafd.as<uint8_t>(), ix->V, ix->B, ix->Q, D.rank.as<uint32_t>(),
                                        D.mass.as<uint32_t>(), D.pos.as<uint16_t>(), D.lcp.as<uint8_t>(), tmp,
                                        ix->status.as<uint32_t>());
  FT_HIP(hipGetLastError());
  uint32_t flags = read_and_clear_status(ix, s);
  if (flags) throw Error(FT_EINVAL, std::string(what) + ":" + describe_flags(flags));
  if (!with_embedding) {
    D.emb_nnz = 0;
    return;
  }
  exclusive_scan_i64(tmp, cnt, n, tmp + n, s);
  int64_t tot = 0;
  FT_HIP(hipMemcpyAsync(&tot, cnt + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FT_HIP(hipStreamSynchronize(s));
  D.emb_nnz = tot;
  D.ekey.ensure(std::max<int64_t>(tot, 1) * 4);
  D.emass.ensure(std::max<int64_t>(tot, 1) * 4);
  D.S.ensure(n * 8);
  k_emb_fill<<<(unsigned)n, 64, 0, s>>>(doff, D.rank.as<uint32_t>(), D.mass.as<uint32_t>(), D.lcp.as<uint8_t>(), n,
                                       cnt, ix->leafd.as<uint8_t>(), ix->anc.as<uint32_t>(), ix->V, ix->B,
                                       D.ekey.as<uint32_t>(), D.emass.as<uint32_t>(), D.S.as<uint64_t>());
  FT_HIP(hipGetLastError());
}

}  // namespace ft

using namespace ft;

extern "C" const char* ft_last_error(void) { return ft::g_last_error.c_str(); }

extern "C" void ft_free(ft_index* ix) {
  if (!ix) return;
  ix->graphs.reset();
  for (DevBuf* b : {&ix->post, &ix->post_dir, &ix->post_cbase, &ix->post_head, &ix->post_hcell, &ix->post_s32, &ix->ws_pipe, &ix->Xm, &ix->Xn, &ix->perm, &ix->inv, &ix->st, &ix->leafd, &ix->anc, &ix->status, &ix->ws_keys,
                    &ix->ws_cost, &ix->ws_tiles, &ix->ws_lists, &ix->ws_counts, &ix->ws_misc, &ix->ws_sel, &ix->ws_rerank,
                    &ix->ws_gx64, &ix->ws_adj, &ix->ws_glist, &ix->sel_exact,
                    &ix->fwd_id, &ix->fwd_eta, &ix->fwd_key, &ix->fwd_bind, &ix->fwd_cnt, &ix->fwd_base, &ix->fwd_sig})
    b->release();
  ix->docs.release();
  ix->qry.release();
  if (ix->ev_a) (void)hipEventDestroy(ix->ev_a);
  if (ix->ev_b) (void)hipEventDestroy(ix->ev_b);
  if (ix->ev_t0) (void)hipEventDestroy(ix->ev_t0);
  if (ix->ev_t1) (void)hipEventDestroy(ix->ev_t1);
  for (hipEvent_t e : ix->ev_p)
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < 2; ++i) {
    if (ix->ev_rank[i]) (void)hipEventDestroy(ix->ev_rank[i]);
    if (ix->ev_sel[i]) (void)hipEventDestroy(ix->ev_sel[i]);
  }
  if (ix->work) (void)hipStreamDestroy(ix->work);
  delete ix;
}

extern "C" ft_status ft_build_tree(const float* X, int64_t V, int32_t d, const int64_t* shift, int32_t B,
                                   const int64_t* doc_off, const uint32_t* doc_id, const uint32_t* doc_mass,
                                   int64_t n_docs, int32_t Q, void* stream, ft_index** out) {
  return guarded([&] {
    FT_REQUIRE(out, FT_EINVAL, "out is NULL");
    *out = nullptr;
    FT_REQUIRE(X && shift, FT_EINVAL, "X or shift is NULL");
    FT_REQUIRE(V >= 1 && d >= 1, FT_EINVAL, "need V >= 1 and d >= 1");
    FT_REQUIRE(V < (1ll << KEY_DEPTH_SHIFT), FT_ERANGE, "V must be below 2^27");
    FT_REQUIRE(B >= 1 && B <= FT_MAX_B, FT_EINVAL, "B must lie in [1, 30]");
    FT_REQUIRE(Q >= 1 && Q <= FT_MAX_Q, FT_EINVAL, "Q must lie in [1, 31]");
    FT_REQUIRE(n_docs >= 1, FT_EINVAL, "need at least one dataset distribution");
    for (int i = 0; i < d; ++i)
      FT_REQUIRE(shift[i] >= 1 && shift[i] <= (1ll << (B - 1)), FT_EINVAL, "shift out of [1, 2^(B-1)]");
    hipStream_t s = (hipStream_t)stream;
    ft_index* ix = new ft_index();
    try {
      ix->V = V;
      ix->d = d;
      ix->dp = padded_row(d);
      ix->B = B;
      ix->Q = Q;
      FT_HIP(hipGetDevice(&ix->device));
      FT_HIP(hipDeviceGetAttribute(&ix->n_cu, hipDeviceAttributeMultiprocessorCount, ix->device));
      (void)noalloc_scratch(ix->device);  // set-up of the no-allocation entry point on this device
      FT_HIP(hipStreamCreateWithFlags(&ix->work, hipStreamNonBlocking));
      FT_HIP(hipEventCreateWithFlags(&ix->ev_a, hipEventDisableTiming));
      FT_HIP(hipEventCreateWithFlags(&ix->ev_b, hipEventDisableTiming));
      FT_HIP(hipEventCreate(&ix->ev_t0));
      FT_HIP(hipEventCreate(&ix->ev_t1));
      for (hipEvent_t& e : ix->ev_p) FT_HIP(hipEventCreate(&e));
      for (int i = 0; i < 2; ++i) {
        FT_HIP(hipEventCreateWithFlags(&ix->ev_rank[i], hipEventDisableTiming));
        FT_HIP(hipEventCreateWithFlags(&ix->ev_sel[i], hipEventDisableTiming));
      }
      ix->status.ensure(64);
      FT_HIP(hipMemsetAsync(ix->status.p, 0, 64, s));
      if (const char* e = getenv("FT_AUTOTUNE")) ix->autotune = atoi(e);

      // grid: per-dimension range, Phi, scale (host float64), codes (device)
      int nb = (int)ceil_div(V, MM_ROWS);
      float* part = nullptr;
      FT_HIP(hipMalloc((void**)&part, ((int64_t)2 * nb * d + 2 * d) * sizeof(float)));
      k_minmax_part<<<nb, 256, 0, s>>>(X, V, d, part, part + (int64_t)nb * d);
      k_minmax_final<<<(unsigned)ceil_div(d, 256), 256, 0, s>>>(part, part + (int64_t)nb * d, nb, d,
                                                                 part + (int64_t)2 * nb * d);
      FT_HIP(hipGetLastError());
      std::vector<float> mm(2 * d);
      FT_HIP(hipMemcpyAsync(mm.data(), part + (int64_t)2 * nb * d, 2 * d * sizeof(float), hipMemcpyDeviceToHost, s));
      FT_HIP(hipStreamSynchronize(s));
      FT_HIP(hipFree(part));
      std::vector<double> lo(d);
      double phi = 0.0;
      for (int i = 0; i < d; ++i) {
        FT_REQUIRE(std::isfinite(mm[i]) && std::isfinite(mm[d + i]), FT_EINVAL, "X holds NaN or Inf");
        lo[i] = (double)mm[i];
        double r = (double)mm[d + i] - lo[i];
        if (r > phi) phi = r;
      }
      const double half = (double)(1ll << (B - 1));
      const double scale = phi > 0.0 ? half / phi : 0.0;

      double* dlo = nullptr;
      int64_t* dshift = nullptr;
      uint32_t* code = nullptr;
      FT_HIP(hipMalloc((void**)&dlo, d * sizeof(double)));
      FT_HIP(hipMalloc((void**)&dshift, d * sizeof(int64_t)));
      FT_HIP(hipMalloc((void**)&code, V * d * sizeof(uint32_t)));
      FT_HIP(hipMemcpyAsync(dlo, lo.data(), d * sizeof(double), hipMemcpyHostToDevice, s));
      FT_HIP(hipMemcpyAsync(dshift, shift, d * sizeof(int64_t), hipMemcpyHostToDevice, s));
      k_codes<<<(unsigned)ceil_div(V * d, 256), 256, 0, s>>>(X, V, d, dlo, dshift, scale, B, code);
      FT_HIP(hipGetLastError());

      // Morton order by a bitonic network over point ids
      int64_t N = 1;
      while (N < V) N <<= 1;
      uint32_t* idx = nullptr;
      FT_HIP(hipMalloc((void**)&idx, N * sizeof(uint32_t)));
      k_iota_pad<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(idx, V, N);
      for (int64_t k = 2; k <= N; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
          k_bitonic_step<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(idx, N, k, j, code, d, B);
      FT_HIP(hipGetLastError());
      uint32_t* perm = (uint32_t*)ix->perm.ensure(V * 4);
      FT_HIP(hipMemcpyAsync(perm, idx, V * 4, hipMemcpyDeviceToDevice, s));
      FT_HIP(hipStreamSynchronize(s));
      FT_HIP(hipFree(idx));

      // adjacent LCA depths, leaf depths, height
      int levels = 1;
      while ((1ll << levels) <= V - 1) ++levels;
      ix->st_levels = levels;
      uint8_t* st = (uint8_t*)ix->st.ensure((int64_t)levels * V);
      unsigned gV = (unsigned)ceil_div(V, 256);
      k_adjacent_lcp<<<gV, 256, 0, s>>>(perm, code, V, d, B, st);
      uint8_t* leafd = (uint8_t*)ix->leafd.ensure(V);
      k_leaf_depth<<<gV, 256, 0, s>>>(st, V, B, leafd, ix->status.as<uint32_t>());
      for (int j = 1; j < levels; ++j) k_st_level<<<gV, 256, 0, s>>>(st, V, j);
      FT_HIP(hipGetLastError());
      uint32_t h[8];
      FT_HIP(hipMemcpyAsync(h, ix->status.p, sizeof(h), hipMemcpyDeviceToHost, s));
      FT_HIP(hipStreamSynchronize(s));
      FT_HIP(hipMemsetAsync(ix->status.p, 0, sizeof(h), s));
      ix->height = (int)h[2];

      // node index of every rank at every depth (cells are rank ranges)
      uint32_t* anc = (uint32_t*)ix->anc.ensure(std::max<int64_t>(1, (int64_t)ix->height * V) * 4);
      int64_t* flag = nullptr;
      int64_t* excl = nullptr;
      int64_t* stmp = nullptr;
      FT_HIP(hipMalloc((void**)&flag, V * sizeof(int64_t)));
      FT_HIP(hipMalloc((void**)&excl, (V + 1) * sizeof(int64_t)));
      FT_HIP(hipMalloc((void**)&stmp, scan_tmp_elems(V) * sizeof(int64_t)));
      std::vector<int64_t> counts(ix->height + 1, 0);
      for (int k = 1; k <= ix->height; ++k) {
        k_node_start<<<gV, 256, 0, s>>>(st, leafd, V, k, flag);
        exclusive_scan_i64(flag, excl, V, stmp, s);
        k_node_index<<<gV, 256, 0, s>>>(flag, excl, leafd, V, k, anc + (int64_t)(k - 1) * V);
        FT_HIP(hipMemcpyAsync(&counts[k], excl + V, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      }
      FT_HIP(hipGetLastError());
      FT_HIP(hipStreamSynchronize(s));
      FT_HIP(hipFree(flag));
      FT_HIP(hipFree(excl));
      FT_HIP(hipFree(stmp));
      ix->n_nodes = 1;
      for (int k = 1; k <= ix->height; ++k) ix->n_nodes += counts[k];
      ix->depth_nodes = counts;

      // Morton-ordered, padded coordinates and the inverse permutation
      float* Xm = (float*)ix->Xm.ensure(V * ix->dp * sizeof(float));
      uint32_t* inv = (uint32_t*)ix->inv.ensure(V * 4);
      double* Xn = (double*)ix->Xn.ensure(V * sizeof(double));
      k_permute_rows<<<(unsigned)V, 64, 0, s>>>(X, perm, V, d, ix->dp, Xm, Xn, inv);
      FT_HIP(hipGetLastError());
      FT_HIP(hipStreamSynchronize(s));
      FT_HIP(hipFree(code));
      FT_HIP(hipFree(dlo));
      FT_HIP(hipFree(dshift));

      prepare_dists(ix, ix->docs, doc_off, doc_id, doc_mass, n_docs, true, s, "dataset");
      FT_HIP(hipStreamSynchronize(s));
      *out = ix;
    } catch (...) {
      ft_free(ix);
      throw;
    }
  });
}

extern "C" ft_status ft_index_info(const ft_index* ix, int64_t* info) {
  return guarded([&] {
    FT_REQUIRE(ix && info, FT_EINVAL, "NULL argument");
    info[0] = ix->V;
    info[1] = ix->d;
    info[2] = ix->B;
    info[3] = ix->Q;
    info[4] = ix->docs.n;
    info[5] = ix->height;
    info[6] = ix->n_nodes;
    info[7] = ix->docs.max_size;
  });
}

extern "C" ft_status ft_export_tree(const ft_index* ix, uint32_t* perm, uint8_t* adj_lcp, uint8_t* leaf_depth,
                                    void* stream) {
  return guarded([&] {
    FT_REQUIRE(ix, FT_EINVAL, "NULL index");
    hipStream_t s = (hipStream_t)stream;
    if (perm) FT_HIP(hipMemcpyAsync(perm, ix->perm.p, ix->V * 4, hipMemcpyDeviceToDevice, s));
    if (adj_lcp) FT_HIP(hipMemcpyAsync(adj_lcp, ix->st.p, ix->V, hipMemcpyDeviceToDevice, s));
    if (leaf_depth) FT_HIP(hipMemcpyAsync(leaf_depth, ix->leafd.p, ix->V, hipMemcpyDeviceToDevice, s));
  });
}
