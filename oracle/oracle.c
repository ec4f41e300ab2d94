/* CPU oracle for the Quadtree and Flowtree estimates of W1.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header or table with the GPU library; both start from the same seeded
 * inputs (points, supports, integer masses, integer shift) and nothing else.
 *
 * Everything here is a plain transcription of the definitions in the paper
 * (arXiv 1910.04126), written for obviousness rather than speed:
 *
 *   - Section 2 ("Generic Quadtree"): a randomly shifted hypercube of side
 *     2*Phi encloses X; it is halved along every dimension recursively, empty
 *     cells are dropped and a cell holding exactly one point is a leaf.  The
 *     edge above a cell weighs its side length.
 *   - Section 2 ("Wasserstein-1 on Quadtree"): the tree W1 has the closed form
 *     sum over nodes v of w(v) * |mu(v) - nu(v)|.
 *   - Section 3 and Appendix A.1: Flowtree computes the tree-optimal flow by
 *     the bottom-up greedy (each node matches the unmatched mu- and
 *     nu-demands collected from its children and passes the rest up), then
 *     prices it with Euclidean distances between the original points.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   (1) grid: lo_i = min_p X[p,i]; Phi = max_i (max_p X[p,i] - lo_i), in
 *       float64; scale = 2^(B-1) / Phi; g = floor((X - lo) * scale) clamped to
 *       [0, 2^(B-1)]; code = g + 2^(B-1) - s_i with the integer shift s_i in
 *       [1, 2^(B-1)] (the paper's sigma_i = s_i / scale).  Cells are
 *       half-open; the depth-k cell of a point is (code >> (B - k)) per
 *       dimension.  No fused multiply-add (built with -ffp-contract=off).
 *   (2) a cell with one point is a leaf; a depth-B cell is a leaf whatever
 *       it holds (coincident or grid-identical points).
 *   (3) weight of the edge above a depth-k node: 2^(B-k) grid units (its
 *       side); grid unit = 2*Phi / 2^B.
 *   (4) "matched arbitrarily": children are ordered by their cell code
 *       compared bit by bit, dimension 0 first (0 before 1); the points of a
 *       multi-point leaf by id.  Leaves in that depth-first order define the
 *       Morton rank.  At every node the unmatched mu-items and nu-items are
 *       each listed in ascending Morton rank and matched by two pointers
 *       (north-west corner rule); a leaf holding both mu- and nu-mass of one
 *       point matches it to itself there.
 *   (5) masses are integers summing to 2^Q; costs are returned in float64 as
 *       2^-Q * sum(eta * ||x - y||_2) with the difference form of the norm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

typedef struct {
  int64_t V;
  int32_t d, B, words; /* words: 64-bit words per packed child code */
  double phi, scale;
  uint32_t* code; /* V*d grid codes */
  /* nodes, numbered in creation (depth-first, Morton) order; node 0 = root */
  int64_t n_nodes, cap_nodes;
  int32_t* depth;
  int64_t* parent;
  int64_t* first_rank; /* Morton rank range [first_rank, last_rank] */
  int64_t* last_rank;
  /* points */
  int64_t* leaf_of; /* point -> leaf node */
  int64_t* rank_of; /* point -> Morton rank */
  int64_t* point_at; /* rank -> point */
  int64_t next_rank;
  /* per-pair scratch */
  int64_t* acc;     /* n_nodes, signed mass per node */
  int64_t* inbox_head; /* n_nodes, head of a linked list of items */
  int64_t* stamp;   /* n_nodes */
  int64_t stamp_id;
  int64_t* pstamp;  /* V, duplicate detection */
  int64_t pstamp_id;
} otree;

/* ---------------------------------------------------------------- tree -- */

static int grow_nodes(otree* t) {
  if (t->n_nodes < t->cap_nodes) return OR_OK;
  int64_t cap = t->cap_nodes ? 2 * t->cap_nodes : 1024;
  void* a = realloc(t->depth, cap * sizeof(int32_t));
  if (!a) return OR_ENOMEM;
  t->depth = (int32_t*)a;
  a = realloc(t->parent, cap * sizeof(int64_t));
  if (!a) return OR_ENOMEM;
  t->parent = (int64_t*)a;
  a = realloc(t->first_rank, cap * sizeof(int64_t));
  if (!a) return OR_ENOMEM;
  t->first_rank = (int64_t*)a;
  a = realloc(t->last_rank, cap * sizeof(int64_t));
  if (!a) return OR_ENOMEM;
  t->last_rank = (int64_t*)a;
  t->cap_nodes = cap;
  return OR_OK;
}

static int64_t new_node(otree* t, int32_t depth, int64_t parent) {
  if (grow_nodes(t) != OR_OK) return -1;
  int64_t v = t->n_nodes++;
  t->depth[v] = depth;
  t->parent[v] = parent;
  t->first_rank[v] = t->last_rank[v] = -1;
  return v;
}

/* child code of point p below a depth-k cell: bit (B-k-1) of every
 * coordinate code, packed so that dimension 0 is the most significant bit of
 * word 0; comparing the words as unsigned integers then compares the bits in
 * dimension order. */
static void child_code(const otree* t, int64_t p, int32_t k, uint64_t* out) {
  int sh = t->B - k - 1;
  for (int w = 0; w < t->words; ++w) out[w] = 0;
  for (int i = 0; i < t->d; ++i) {
    uint64_t bit = (t->code[p * t->d + i] >> sh) & 1u;
    out[i / 64] |= bit << (63 - (i % 64));
  }
}

static int cmp_words(const uint64_t* a, const uint64_t* b, int words) {
  for (int w = 0; w < words; ++w) {
    if (a[w] < b[w]) return -1;
    if (a[w] > b[w]) return 1;
  }
  return 0;
}

/* stable merge sort of pts[0..n) by their packed codes (keys row-major) */
static void msort(int64_t* pts, uint64_t* keys, int64_t n, int words,
                  int64_t* tp, uint64_t* tk) {
  if (n < 2) return;
  int64_t h = n / 2;
  msort(pts, keys, h, words, tp, tk);
  msort(pts + h, keys + h * words, n - h, words, tp, tk);
  int64_t i = 0, j = h, o = 0;
  while (i < h || j < n) {
    int take_left;
    if (i >= h) take_left = 0;
    else if (j >= n) take_left = 1;
    else take_left = cmp_words(keys + i * words, keys + j * words, words) <= 0;
    int64_t s = take_left ? i++ : j++;
    tp[o] = pts[s];
    memcpy(tk + o * words, keys + s * words, words * sizeof(uint64_t));
    ++o;
  }
  memcpy(pts, tp, n * sizeof(int64_t));
  memcpy(keys, tk, n * words * sizeof(uint64_t));
}

/* Build the subtree of cell `node` (depth k) over the points pts[0..n),
 * which arrive in ascending id order within every group of equal codes. */
static int build_rec(otree* t, int64_t node, int32_t k, int64_t* pts, int64_t n,
                     uint64_t* keys, int64_t* tp, uint64_t* tk) {
  if (n == 1 || k == t->B) {
    /* leaf: one point, or the depth-B cell with all its points in id order */
    for (int64_t a = 0; a < n; ++a) {
      int64_t best = a;
      for (int64_t b = a + 1; b < n; ++b)
        if (pts[b] < pts[best]) best = b;
      int64_t x = pts[a]; pts[a] = pts[best]; pts[best] = x;
    }
    t->first_rank[node] = t->next_rank;
    for (int64_t a = 0; a < n; ++a) {
      t->leaf_of[pts[a]] = node;
      t->rank_of[pts[a]] = t->next_rank;
      t->point_at[t->next_rank] = pts[a];
      t->next_rank++;
    }
    t->last_rank[node] = t->next_rank - 1;
    return OR_OK;
  }
  int W = t->words;
  for (int64_t a = 0; a < n; ++a) child_code(t, pts[a], k, keys + a * W);
  msort(pts, keys, n, W, tp, tk);
  t->first_rank[node] = t->next_rank;
  int64_t a = 0;
  while (a < n) {
    int64_t b = a + 1;
    while (b < n && cmp_words(keys + a * W, keys + b * W, W) == 0) ++b;
    int64_t child = new_node(t, k + 1, node);
    if (child < 0) return OR_ENOMEM;
    /* the child's recursion overwrites keys[a..b); it uses its own slice */
    int rc = build_rec(t, child, k + 1, pts + a, b - a, keys + a * W, tp, tk);
    if (rc != OR_OK) return rc;
    a = b;
  }
  t->last_rank[node] = t->next_rank - 1;
  return OR_OK;
}

void oracle_tree_free(otree* t) {
  if (!t) return;
  free(t->code);
  free(t->depth);
  free(t->parent);
  free(t->first_rank);
  free(t->last_rank);
  free(t->leaf_of);
  free(t->rank_of);
  free(t->point_at);
  free(t->acc);
  free(t->inbox_head);
  free(t->stamp);
  free(t->pstamp);
  free(t);
}

/* Quadtree over X (V x d float32, row-major) with integer shift s[d]. */
int oracle_tree_build(const float* X, int64_t V, int32_t d, const int64_t* shift,
                      int32_t B, otree** out) {
  *out = NULL;
  if (V < 1 || d < 1 || B < 1 || B > 31) return OR_EINVAL;
  for (int i = 0; i < d; ++i)
    if (shift[i] < 1 || shift[i] > ((int64_t)1 << (B - 1))) return OR_EINVAL;
  otree* t = (otree*)calloc(1, sizeof(otree));
  if (!t) return OR_ENOMEM;
  t->V = V;
  t->d = d;
  t->B = B;
  t->words = (d + 63) / 64;
  t->code = (uint32_t*)malloc((size_t)V * d * sizeof(uint32_t));
  t->leaf_of = (int64_t*)malloc(V * sizeof(int64_t));
  t->rank_of = (int64_t*)malloc(V * sizeof(int64_t));
  t->point_at = (int64_t*)malloc(V * sizeof(int64_t));
  if (!t->code || !t->leaf_of || !t->rank_of || !t->point_at) {
    oracle_tree_free(t);
    return OR_ENOMEM;
  }
  /* (1) grid: per-dimension minimum, Phi = largest per-dimension range */
  double* lo = (double*)malloc(d * sizeof(double));
  double phi = 0.0;
  for (int i = 0; i < d; ++i) {
    double mn = (double)X[i], mx = (double)X[i];
    for (int64_t p = 1; p < V; ++p) {
      double x = (double)X[p * d + i];
      if (x < mn) mn = x;
      if (x > mx) mx = x;
    }
    lo[i] = mn;
    if (mx - mn > phi) phi = mx - mn;
  }
  t->phi = phi;
  const double half = (double)((int64_t)1 << (B - 1));
  t->scale = phi > 0.0 ? half / phi : 0.0;
  for (int64_t p = 0; p < V; ++p)
    for (int i = 0; i < d; ++i) {
      double diff = (double)X[p * d + i] - lo[i];
      double y = diff * t->scale;
      double g = floor(y);
      if (g < 0.0) g = 0.0;
      if (g > half) g = half;
      t->code[p * d + i] = (uint32_t)((int64_t)g + ((int64_t)1 << (B - 1)) - shift[i]);
    }
  free(lo);
  /* (2) recursive halving from the root cell */
  int64_t* pts = (int64_t*)malloc(V * sizeof(int64_t));
  int64_t* tp = (int64_t*)malloc(V * sizeof(int64_t));
  uint64_t* keys = (uint64_t*)malloc((size_t)V * t->words * sizeof(uint64_t));
  uint64_t* tk = (uint64_t*)malloc((size_t)V * t->words * sizeof(uint64_t));
  int rc = (pts && tp && keys && tk) ? OR_OK : OR_ENOMEM;
  if (rc == OR_OK) {
    for (int64_t p = 0; p < V; ++p) pts[p] = p;
    int64_t root = new_node(t, 0, -1);
    rc = root == 0 ? build_rec(t, root, 0, pts, V, keys, tp, tk) : OR_ENOMEM;
  }
  free(pts);
  free(tp);
  free(keys);
  free(tk);
  if (rc == OR_OK) {
    t->acc = (int64_t*)calloc(t->n_nodes, sizeof(int64_t));
    t->inbox_head = (int64_t*)malloc(t->n_nodes * sizeof(int64_t));
    t->stamp = (int64_t*)calloc(t->n_nodes, sizeof(int64_t));
    t->pstamp = (int64_t*)calloc(t->V, sizeof(int64_t));
    if (!t->acc || !t->inbox_head || !t->stamp || !t->pstamp) rc = OR_ENOMEM;
  }
  if (rc != OR_OK) {
    oracle_tree_free(t);
    return rc;
  }
  *out = t;
  return OR_OK;
}

int64_t oracle_tree_nodes(const otree* t) { return t->n_nodes; }
double oracle_tree_phi(const otree* t) { return t->phi; }

/* Export: grid codes (V*d), rank_of (V), leaf depth per point (V), and per
 * node depth / parent / rank range (n_nodes each).  Any pointer may be NULL. */
void oracle_tree_export(const otree* t, uint32_t* code, int64_t* rank_of,
                        int32_t* leaf_depth, int32_t* node_depth,
                        int64_t* node_parent, int64_t* node_first,
                        int64_t* node_last) {
  if (code) memcpy(code, t->code, (size_t)t->V * t->d * sizeof(uint32_t));
  for (int64_t p = 0; p < t->V; ++p) {
    if (rank_of) rank_of[p] = t->rank_of[p];
    if (leaf_depth) leaf_depth[p] = t->depth[t->leaf_of[p]];
  }
  for (int64_t v = 0; v < t->n_nodes; ++v) {
    if (node_depth) node_depth[v] = t->depth[v];
    if (node_parent) node_parent[v] = t->parent[v];
    if (node_first) node_first[v] = t->first_rank[v];
    if (node_last) node_last[v] = t->last_rank[v];
  }
}

/* Tree distance t(x, y) in grid units: edge weights on the leaf-to-leaf path
 * (Section 2); the edge above a depth-k node weighs 2^(B-k). */
uint64_t oracle_tree_dist(const otree* t, int64_t x, int64_t y) {
  int64_t a = t->leaf_of[x], b = t->leaf_of[y];
  uint64_t s = 0;
  while (a != b) {
    if (t->depth[a] >= t->depth[b]) {
      s += (uint64_t)1 << (t->B - t->depth[a]);
      a = t->parent[a];
    } else {
      s += (uint64_t)1 << (t->B - t->depth[b]);
      b = t->parent[b];
    }
  }
  return s;
}

/* Depth of the deepest common cell of points x and y. */
int32_t oracle_lca_depth(const otree* t, int64_t x, int64_t y) {
  int64_t a = t->leaf_of[x], b = t->leaf_of[y];
  while (a != b) {
    if (t->depth[a] >= t->depth[b]) a = t->parent[a];
    else b = t->parent[b];
  }
  return t->depth[a];
}

/* ------------------------------------------------------------ validation -- */

/* A distribution is valid when it has at least one point, its ids are
 * distinct and below V, its masses are positive and they sum to 2^Q (W1 needs
 * equal total mass on both sides, Section 1). */
static int check_dist(otree* t, const uint32_t* id, const uint32_t* m,
                      int64_t n, int32_t Q) {
  if (n < 1 || Q < 1 || Q > 31) return OR_EINVAL;
  uint64_t s = 0;
  t->pstamp_id++;
  for (int64_t a = 0; a < n; ++a) {
    if (id[a] >= (uint64_t)t->V || m[a] == 0) return OR_EINVAL;
    if (t->pstamp[id[a]] == t->pstamp_id) return OR_EINVAL;
    t->pstamp[id[a]] = t->pstamp_id;
    s += m[a];
  }
  return s == ((uint64_t)1 << Q) ? OR_OK : OR_EINVAL;
}

/* -------------------------------------------------------------- quadtree -- */

/* mu(v) - nu(v) for every non-root cell v that either distribution touches,
 * left in t->acc[v]; returns the list of those cells (caller frees) and its
 * length in *nt, or NULL when out of memory. */
static int64_t* cell_mass_differences(otree* t, const uint32_t* mu_id, const uint32_t* mu_m, int64_t n_mu,
                                      const uint32_t* nu_id, const uint32_t* nu_m, int64_t n_nu,
                                      int64_t* nt_out) {
  t->stamp_id++;
  int64_t cap = (n_mu + n_nu) * (t->B + 1) + 1, nt = 0;
  int64_t* touched = (int64_t*)malloc(cap * sizeof(int64_t));
  if (!touched) return NULL;
  for (int side = 0; side < 2; ++side) {
    const uint32_t* id = side ? nu_id : mu_id;
    const uint32_t* m = side ? nu_m : mu_m;
    int64_t n = side ? n_nu : n_mu;
    for (int64_t a = 0; a < n; ++a) {
      for (int64_t v = t->leaf_of[id[a]]; v != 0; v = t->parent[v]) {
        if (t->stamp[v] != t->stamp_id) {
          t->stamp[v] = t->stamp_id;
          t->acc[v] = 0;
          touched[nt++] = v;
        }
        t->acc[v] += side ? -(int64_t)m[a] : (int64_t)m[a];
      }
    }
  }
  *nt_out = nt;
  return touched;
}

/* Quadtree estimate in integer units of 2^-Q mass x grid unit:
 * U = sum over non-root nodes v of 2^(B - depth v) * |mu(v) - nu(v)|,
 * with mu(v) the mass of mu's points inside v (Section 2, closed form).
 * Returns 0 and writes *out, or a negative status. */
int oracle_quadtree(otree* t, const uint32_t* mu_id, const uint32_t* mu_m, int64_t n_mu,
                    const uint32_t* nu_id, const uint32_t* nu_m, int64_t n_nu,
                    int32_t Q, uint64_t* out) {
  if (check_dist(t, mu_id, mu_m, n_mu, Q) || check_dist(t, nu_id, nu_m, n_nu, Q))
    return OR_EINVAL;
  int64_t nt = 0;
  int64_t* touched = cell_mass_differences(t, mu_id, mu_m, n_mu, nu_id, nu_m, n_nu, &nt);
  if (!touched) return OR_ENOMEM;
  unsigned __int128 s = 0;
  for (int64_t i = 0; i < nt; ++i) {
    int64_t v = touched[i];
    int64_t a = t->acc[v] < 0 ? -t->acc[v] : t->acc[v];
    s += (unsigned __int128)a << (t->B - t->depth[v]);
  }
  free(touched);
  if (s >> 64) return OR_EINVAL;
  *out = (uint64_t)s;
  return OR_OK;
}

/* -------------------------------------------------------------- flowtree -- */

typedef struct {
  int64_t point, rank; /* ground point and its Morton rank */
  int64_t resid;       /* unmatched mass */
  int32_t side;        /* 0 = mu (dataset distribution), 1 = nu (query) */
  int32_t index;       /* position in the caller's support array */
  int64_t next;        /* inbox linked list */
} item_t;

/* Quadtree with the edge above a depth-k cell weighted (2^(B-k))^(1-eps)
 * (the eps-weighted tree of the proof of the uniform-distribution upper
 * bound for Flowtree): sum over non-root cells of the weight times
 * |mu(v) - nu(v)|, masses as fractions of 2^Q, float64. */
int oracle_quadtree_eps(otree* t, const uint32_t* mu_id, const uint32_t* mu_m, int64_t n_mu,
                        const uint32_t* nu_id, const uint32_t* nu_m, int64_t n_nu,
                        int32_t Q, double eps, double* out) {
  if (check_dist(t, mu_id, mu_m, n_mu, Q) || check_dist(t, nu_id, nu_m, n_nu, Q))
    return OR_EINVAL;
  int64_t nt = 0;
  int64_t* touched = cell_mass_differences(t, mu_id, mu_m, n_mu, nu_id, nu_m, n_nu, &nt);
  if (!touched) return OR_ENOMEM;
  double s = 0.0;
  for (int64_t i = 0; i < nt; ++i) {
    int64_t v = touched[i];
    int64_t a = t->acc[v] < 0 ? -t->acc[v] : t->acc[v];
    s += (double)a * pow(2.0, (double)(t->B - t->depth[v]) * (1.0 - eps));
  }
  free(touched);
  *out = ldexp(s, -Q);
  return OR_OK;
}

static int cmp_rank(const void* a, const void* b) {
  const item_t* x = *(item_t* const*)a;
  const item_t* y = *(item_t* const*)b;
  return (x->rank > y->rank) - (x->rank < y->rank);
}

static _Thread_local const otree* g_sort_tree; /* qsort has no context argument; one per thread */
static int cmp_node_depth(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  int32_t dx = g_sort_tree->depth[x], dy = g_sort_tree->depth[y];
  if (dx != dy) return dx > dy ? -1 : 1; /* deeper first */
  return (x > y) - (x < y);
}

/* Flowtree (Appendix A.1).  mu = dataset distribution, nu = query.
 * Emissions are written in the order the greedy makes them:
 * em_mu[e] / em_nu[e] = index into the mu / nu support arrays, em_eta[e] =
 * transported integer mass, em_bind[e] = which side the match exhausted
 * (0 = mu only, 1 = nu only, 2 = both).  Capacity must be >= n_mu + n_nu.
 * *n_em receives the count; *cost = 2^-Q * sum(eta * ||x_mu - x_nu||_2) over
 * the float32 points X (V x d), computed in float64.  Pass X = NULL to skip
 * the cost. */
int oracle_flowtree(otree* t, const float* X, const uint32_t* mu_id,
                    const uint32_t* mu_m, int64_t n_mu, const uint32_t* nu_id,
                    const uint32_t* nu_m, int64_t n_nu, int32_t Q, int32_t* em_mu,
                    int32_t* em_nu, uint32_t* em_eta, int8_t* em_bind,
                    int64_t* n_em, double* cost) {
  if (check_dist(t, mu_id, mu_m, n_mu, Q) || check_dist(t, nu_id, nu_m, n_nu, Q))
    return OR_EINVAL;
  int64_t n = n_mu + n_nu;
  item_t* it = (item_t*)malloc(n * sizeof(item_t));
  item_t** lm = (item_t**)malloc(n * sizeof(item_t*));
  item_t** ln = (item_t**)malloc(n * sizeof(item_t*));
  int64_t cap = n * (t->B + 1) + 1, nt = 0;
  int64_t* nodes = (int64_t*)malloc(cap * sizeof(int64_t));
  if (!it || !lm || !ln || !nodes) {
    free(it); free(lm); free(ln); free(nodes);
    return OR_ENOMEM;
  }
  t->stamp_id++;
  /* every node on a path from an item's leaf to the root takes part */
  for (int64_t a = 0; a < n; ++a) {
    int side = a >= n_mu;
    int64_t i = side ? a - n_mu : a;
    it[a].point = side ? nu_id[i] : mu_id[i];
    it[a].rank = t->rank_of[it[a].point];
    it[a].resid = side ? nu_m[i] : mu_m[i];
    it[a].side = side;
    it[a].index = (int32_t)i;
    for (int64_t v = t->leaf_of[it[a].point]; v >= 0; v = t->parent[v]) {
      if (t->stamp[v] == t->stamp_id) break;
      t->stamp[v] = t->stamp_id;
      t->inbox_head[v] = -1;
      nodes[nt++] = v;
    }
  }
  /* a leaf starts with the items of its own point(s) */
  for (int64_t a = n - 1; a >= 0; --a) {
    int64_t v = t->leaf_of[it[a].point];
    it[a].next = t->inbox_head[v];
    t->inbox_head[v] = a;
  }
  /* bottom-up: children are processed before parents */
  g_sort_tree = t;
  qsort(nodes, nt, sizeof(int64_t), cmp_node_depth);
  int64_t ne = 0;
  int rc = OR_OK;
  for (int64_t q = 0; q < nt && rc == OR_OK; ++q) {
    int64_t v = nodes[q];
    int64_t cm = 0, cn = 0;
    for (int64_t a = t->inbox_head[v]; a >= 0; a = it[a].next) {
      if (it[a].resid == 0) continue;
      if (it[a].side == 0) lm[cm++] = &it[a];
      else ln[cn++] = &it[a];
    }
    qsort(lm, cm, sizeof(item_t*), cmp_rank);
    qsort(ln, cn, sizeof(item_t*), cmp_rank);
    /* match the two lists front to front until one runs out */
    int64_t i = 0, j = 0;
    while (i < cm && j < cn) {
      int64_t eta = lm[i]->resid < ln[j]->resid ? lm[i]->resid : ln[j]->resid;
      lm[i]->resid -= eta;
      ln[j]->resid -= eta;
      em_mu[ne] = lm[i]->index;
      em_nu[ne] = ln[j]->index;
      em_eta[ne] = (uint32_t)eta;
      em_bind[ne] = (lm[i]->resid == 0 && ln[j]->resid == 0) ? 2 : (lm[i]->resid == 0 ? 0 : 1);
      ++ne;
      if (lm[i]->resid == 0) ++i;
      if (ln[j]->resid == 0) ++j;
    }
    /* whatever is left (one side only) goes up to the parent */
    int64_t p = t->parent[v];
    item_t** rest = i < cm ? lm + i : ln + j;
    int64_t nr = i < cm ? cm - i : cn - j;
    if (p < 0) {
      if (nr != 0) rc = OR_EINVAL; /* marginals did not balance */
      break;
    }
    for (int64_t r = nr - 1; r >= 0; --r) {
      int64_t a = rest[r] - it;
      it[a].next = t->inbox_head[p];
      t->inbox_head[p] = a;
    }
  }
  *n_em = ne;
  if (rc == OR_OK && X && cost) {
    double s = 0.0;
    for (int64_t e = 0; e < ne; ++e) {
      const float* x = X + (int64_t)mu_id[em_mu[e]] * t->d;
      const float* y = X + (int64_t)nu_id[em_nu[e]] * t->d;
      double acc = 0.0;
      for (int i = 0; i < t->d; ++i) {
        double df = (double)x[i] - (double)y[i];
        acc += df * df;
      }
      s += (double)em_eta[e] * sqrt(acc);
    }
    *cost = ldexp(s, -Q);
  }
  free(it); free(lm); free(ln); free(nodes);
  return rc;
}

/* ------------------------------------------------------- exact W1 (tiny) -- */

/* Exact W1 by successive shortest paths on the transportation network
 * source -> mu_i (capacity m_i) -> nu_j (uncapacitated, cost ||x_i - y_j||)
 * -> sink (capacity n_j), Bellman-Ford on the residual graph.  Integer
 * masses, float64 costs.  Returns 2^-Q * optimal cost.  Tiny inputs only. */
int oracle_exact_w1_ssp(const float* X, int32_t d, const uint32_t* mu_id,
                        const uint32_t* mu_m, int64_t n_mu, const uint32_t* nu_id,
                        const uint32_t* nu_m, int64_t n_nu, int32_t Q, double* out) {
  int64_t N = n_mu + n_nu + 2, S = n_mu + n_nu, T = S + 1;
  int64_t E = 2 * (n_mu + n_nu + n_mu * n_nu);
  int64_t* to = (int64_t*)malloc(E * sizeof(int64_t));
  int64_t* capa = (int64_t*)malloc(E * sizeof(int64_t));
  double* cst = (double*)malloc(E * sizeof(double));
  int64_t* from = (int64_t*)malloc(E * sizeof(int64_t));
  double* dist = (double*)malloc(N * sizeof(double));
  int64_t* pe = (int64_t*)malloc(N * sizeof(int64_t));
  if (!to || !capa || !cst || !from || !dist || !pe) {
    free(to); free(capa); free(cst); free(from); free(dist); free(pe);
    return OR_ENOMEM;
  }
  int64_t ne = 0;
#define ADD_EDGE(u, v, c, w)                                     \
  do {                                                          \
    from[ne] = (u); to[ne] = (v); capa[ne] = (c); cst[ne] = (w); ++ne; \
    from[ne] = (v); to[ne] = (u); capa[ne] = 0; cst[ne] = -(w); ++ne;  \
  } while (0)
  const int64_t INF = (int64_t)1 << 62;
  for (int64_t i = 0; i < n_mu; ++i) ADD_EDGE(S, i, (int64_t)mu_m[i], 0.0);
  for (int64_t j = 0; j < n_nu; ++j) ADD_EDGE(n_mu + j, T, (int64_t)nu_m[j], 0.0);
  for (int64_t i = 0; i < n_mu; ++i)
    for (int64_t j = 0; j < n_nu; ++j) {
      const float* x = X + (int64_t)mu_id[i] * d;
      const float* y = X + (int64_t)nu_id[j] * d;
      double acc = 0.0;
      for (int k = 0; k < d; ++k) {
        double df = (double)x[k] - (double)y[k];
        acc += df * df;
      }
      ADD_EDGE(i, n_mu + j, INF, sqrt(acc));
    }
#undef ADD_EDGE
  int64_t need = (int64_t)1 << Q;
  double total = 0.0;
  int rc = OR_OK;
  while (need > 0) {
    for (int64_t v = 0; v < N; ++v) { dist[v] = INFINITY; pe[v] = -1; }
    dist[S] = 0.0;
    for (int64_t round = 0; round < N; ++round) {
      int changed = 0;
      for (int64_t e = 0; e < ne; ++e)
        if (capa[e] > 0 && dist[from[e]] < INFINITY &&
            (dist[to[e]] == INFINITY ||
             dist[from[e]] + cst[e] < dist[to[e]] - 1e-15 * (1.0 + fabs(dist[to[e]])))) {
          dist[to[e]] = dist[from[e]] + cst[e];
          pe[to[e]] = e;
          changed = 1;
        }
      if (!changed) break;
    }
    if (pe[T] < 0) { rc = OR_EINVAL; break; }
    int64_t f = need;
    for (int64_t v = T; v != S; v = from[pe[v]])
      if (capa[pe[v]] < f) f = capa[pe[v]];
    for (int64_t v = T; v != S; v = from[pe[v]]) {
      capa[pe[v]] -= f;
      capa[pe[v] ^ 1] += f;
    }
    total += (double)f * dist[T];
    need -= f;
  }
  *out = ldexp(total, -Q);
  free(to); free(capa); free(cst); free(from); free(dist); free(pe);
  return rc;
}

/* -------------------------------------------------------- batch helpers -- */

/* Quadtree keys for pairs (query qi, doc di) of CSR distributions. */
int oracle_quadtree_pairs(otree* t, const int64_t* q_off, const uint32_t* q_id,
                          const uint32_t* q_m, const int64_t* d_off,
                          const uint32_t* d_id, const uint32_t* d_m,
                          const int64_t* pair_q, const int64_t* pair_d,
                          int64_t n_pairs, int32_t Q, uint64_t* out) {
  for (int64_t p = 0; p < n_pairs; ++p) {
    int64_t qa = q_off[pair_q[p]], qb = q_off[pair_q[p] + 1];
    int64_t da = d_off[pair_d[p]], db = d_off[pair_d[p] + 1];
    int rc = oracle_quadtree(t, d_id + da, d_m + da, db - da, q_id + qa, q_m + qa,
                             qb - qa, Q, out + p);
    if (rc != OR_OK) return rc;
  }
  return OR_OK;
}

/* Flowtree costs for pairs (query qi, doc di). */
int oracle_flowtree_pairs(otree* t, const float* X, const int64_t* q_off,
                          const uint32_t* q_id, const uint32_t* q_m,
                          const int64_t* d_off, const uint32_t* d_id,
                          const uint32_t* d_m, const int64_t* pair_q,
                          const int64_t* pair_d, int64_t n_pairs, int32_t Q,
                          double* out) {
  int64_t cap = 0;
  for (int64_t p = 0; p < n_pairs; ++p) {
    int64_t n = (q_off[pair_q[p] + 1] - q_off[pair_q[p]]) +
                (d_off[pair_d[p] + 1] - d_off[pair_d[p]]);
    if (n > cap) cap = n;
  }
  int32_t* a = (int32_t*)malloc((cap + 1) * sizeof(int32_t));
  int32_t* b = (int32_t*)malloc((cap + 1) * sizeof(int32_t));
  uint32_t* eta = (uint32_t*)malloc((cap + 1) * sizeof(uint32_t));
  int8_t* bind = (int8_t*)malloc(cap + 1);
  int rc = (a && b && eta && bind) ? OR_OK : OR_ENOMEM;
  for (int64_t p = 0; p < n_pairs && rc == OR_OK; ++p) {
    int64_t qa = q_off[pair_q[p]], qb = q_off[pair_q[p] + 1];
    int64_t da = d_off[pair_d[p]], db = d_off[pair_d[p] + 1];
    int64_t ne = 0;
    rc = oracle_flowtree(t, X, d_id + da, d_m + da, db - da, q_id + qa, q_m + qa,
                         qb - qa, Q, a, b, eta, bind, &ne, out + p);
  }
  free(a); free(b); free(eta); free(bind);
  return rc;
}
