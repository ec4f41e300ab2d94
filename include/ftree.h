/* ftree: Quadtree and Flowtree nearest-neighbour search for Wasserstein-1 on
 * AMD Instinct MI355X (gfx950).
 *
 * The calls follow the problem statement of Backurs, Dong, Indyk,
 * Razenshteyn and Wagner, "Scalable Nearest Neighbor Search for Optimal
 * Transport" (arXiv 1910.04126), Section 1: preprocess a dataset of n
 * distributions supported on a ground set X in R^d; given a query
 * distribution, return the k dataset distributions nearest to it under an
 * estimate of W1.  Two estimates are provided, both on one randomly shifted
 * quadtree over X (Section 2):
 *   - Quadtree: the tree W1, sum over cells v of side(v) * |mu(v) - nu(v)|
 *     (Section 2, closed form);
 *   - Flowtree: the tree-optimal flow computed by the bottom-up greedy of
 *     Appendix A.1, priced with Euclidean distances between the original
 *     points (Section 3).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All array arguments are DEVICE pointers on the current HIP device,
 *   except where a comment says "host".  The library never frees caller
 *   memory; outputs are caller-allocated and are written completely, or not
 *   at all when the call returns an error.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *   enqueue their work on it and return after validating inputs; outputs are
 *   ready when the stream reaches the call's end.  A call may synchronise the
 *   stream to read small validation results.
 * - Distributions are CSR: off[n+1] (int64, off[0] = 0, increasing), ids
 *   (uint32 original point ids, distinct within a distribution, < V) and
 *   masses (uint32, positive, summing to exactly 2^Q).  Support sizes are at
 *   most FT_MAX_SUPPORT.  Ids are always the caller's point ids.
 * - The mass unit is 2^-Q; the length unit of Quadtree keys is one grid unit
 *   2*Phi / 2^B (Phi = largest per-dimension range of X).
 * - Nothing throws across this interface.  Every call returns an ft_status;
 *   ft_last_error() gives a message for the last failing call of the
 *   calling thread.
 * - Calls on one index from several host threads must be serialised by the
 *   caller (the index owns reusable workspaces).
 */
#ifndef FTREE_H
#define FTREE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ft_index ft_index;

typedef enum {
  FT_OK = 0,
  FT_EINVAL = -1, /* invalid argument or input data (ids, masses, sizes) */
  FT_ENOMEM = -2, /* device or host allocation failed */
  FT_EHIP = -3,   /* a HIP runtime call or kernel failed */
  FT_ERANGE = -4  /* a size exceeds a documented limit */
} ft_status;

enum { FT_PLAIN = 0, FT_BATCHED = 1 };
enum { FT_FWD = 0, FT_BWD = 1 };

#define FT_MAX_SUPPORT 1024 /* largest support of one distribution */
#define FT_MAX_B 30         /* largest number of grid bits */
#define FT_MAX_Q 31         /* largest number of mass bits */

/* Message of the last failing call on this thread ("" if none). */
const char* ft_last_error(void);

/* ------------------------------------------------------------------------
 * ft_build_tree -- preprocessing (Section 1 problem statement; Section 2
 * quadtree construction).
 *
 * X[V*d]      float32 row-major ground points (device).
 * shift[d]    HOST int64 random shift per dimension, each in [1, 2^(B-1)];
 *             the paper's sigma_i in (0, Phi] expressed in grid units.
 * B           grid bits, 1..FT_MAX_B.  The grid maps X into [0, 2^B)^d:
 *             code = floor((x - min_i) * 2^(B-1) / Phi) + 2^(B-1) - shift_i;
 *             cells of depth k are code >> (B - k); a cell holding one point
 *             is a leaf; depth B ends every path.
 * doc_off[n_docs+1], doc_id, doc_mass: the dataset distributions (device).
 * Q           mass bits, 1..FT_MAX_Q.
 * *out        receives a new index owning device copies of everything it
 *             needs (the caller may free X and the doc arrays afterwards).
 * Errors: FT_EINVAL (sizes, shift out of range, invalid distribution),
 * FT_ERANGE (support > FT_MAX_SUPPORT, V >= 2^27), FT_ENOMEM, FT_EHIP.
 * ---------------------------------------------------------------------- */
ft_status ft_build_tree(const float* X, int64_t V, int32_t d, const int64_t* shift,
                        int32_t B, const int64_t* doc_off, const uint32_t* doc_id,
                        const uint32_t* doc_mass, int64_t n_docs, int32_t Q, void* stream,
                        ft_index** out);

/* Release an index and all its device memory.  NULL is ignored. */
void ft_free(ft_index* index);

/* Host int64 info[8]: V, d, B, Q, n_docs, tree height (deepest leaf),
 * number of tree nodes (root included), largest doc support. */
ft_status ft_index_info(const ft_index* index, int64_t* info);

/* Export of the tree for inspection (device outputs, each V entries):
 * perm[r]      original id of the point with Morton rank r;
 * adj_lcp[r]   depth of the deepest cell shared by ranks r and r+1
 *              (adj_lcp[V-1] = 0);
 * leaf_depth[r] depth of the leaf of rank r.
 * Morton rank: leaves in depth-first order, children ordered by their cell
 * code compared bit by bit with dimension 0 first; points of one depth-B
 * cell by id. */
ft_status ft_export_tree(const ft_index* index, uint32_t* perm, uint8_t* adj_lcp,
                         uint8_t* leaf_depth, void* stream);

/* ------------------------------------------------------------------------
 * ft_quadtree_knn -- k nearest dataset distributions by the Quadtree
 * estimate (Section 2 closed form; its l1-embedding view).
 *
 * Queries: q_off[n_q+1], q_id, q_mass (device CSR as above).
 * cand        NULL: rank all dataset distributions; else int64
 *             [n_q * n_cand] doc indices per query (n_cand <= 4096).
 * k           1 <= k <= number ranked per query.
 * out_key[n_q*k]  exact uint64 keys U = sum_{v != root} 2^(B - depth v) *
 *             |m_q(v) - m_d(v)| in units of 2^-Q mass x grid unit.
 * out_doc[n_q*k]  doc indices, ordered by (key, doc index) ascending.
 * ---------------------------------------------------------------------- */
ft_status ft_quadtree_knn(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                          const uint32_t* q_mass, int64_t n_q, const int64_t* cand,
                          int32_t n_cand, int32_t k, uint64_t* out_key, int64_t* out_doc,
                          void* stream);

/* ------------------------------------------------------------------------
 * ft_flowtree_knn -- k nearest dataset distributions by the Flowtree
 * estimate (Section 3; greedy flow of Appendix A.1).
 *
 * Arguments as ft_quadtree_knn, plus
 * mode        FT_PLAIN: one kernel launch per query over its candidates;
 *             FT_BATCHED: all (query, candidate) pairs in one persistent
 *             launch per pair-size class, replayed as two HIP graphs
 *             (bucketing, then the class launches), schedule picked by the
 *             built-in autotuner.
 * out_cost[n_q*k] float32 Flowtree values 2^-Q * sum eta * ||x - y||_2 in
 *             the units of X, ordered with out_doc by (cost, doc index).
 * The greedy matches, at every cell, the unmatched dataset-side and
 * query-side items each in ascending Morton rank, front to front.
 * ---------------------------------------------------------------------- */
ft_status ft_flowtree_knn(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                          const uint32_t* q_mass, int64_t n_q, const int64_t* cand,
                          int32_t n_cand, int32_t k, int32_t mode, float* out_cost,
                          int64_t* out_doc, void* stream);


/* ------------------------------------------------------------------------
 * ft_knn_pipeline -- the two-stage search of Section 4.3: the Quadtree
 * estimate (Section 2) ranks every dataset distribution and keeps the
 * prune_k best per query, then the Flowtree estimate (Section 3, greedy of
 * Appendix A.1) reranks those and returns the k best.
 *
 * Queries as ft_quadtree_knn.  1 <= k <= prune_k <= min(number of docs,
 * 4096); prune_k <= 1024 when there are more than 4096 docs.
 * out_cost[n_q*k], out_doc[n_q*k] as ft_flowtree_knn (FT_BATCHED); they
 * equal ft_flowtree_knn(cand = the doc lists of ft_quadtree_knn(k =
 * prune_k)) bit for bit.  The queries are prepared once for both stages and
 * the validation and kernel flags are read once, at the end; the candidate
 * lists, which the call makes itself, are not checked again.  Device
 * scratch of n_q * prune_k * 16 bytes is kept with the index.
 * Errors: as ft_quadtree_knn and ft_flowtree_knn.
 * ---------------------------------------------------------------------- */
ft_status ft_knn_pipeline(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                          const uint32_t* q_mass, int64_t n_q, int32_t prune_k, int32_t k,
                          float* out_cost, int64_t* out_doc, void* stream);

/* Host timing of the last ft_knn_pipeline call (milliseconds, HIP events on
 * its stream): the Quadtree stage (ranking and select) and the Flowtree
 * stage (batched rerank and select).  Either pointer may be NULL. */
ft_status ft_last_pipeline_stats(const ft_index* index, double* prune_ms, double* rerank_ms);
/* ------------------------------------------------------------------------
 * ft_flowtree_knn_noalloc -- ft_flowtree_knn over candidate lists for callers
 * that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc).
 *
 * Arguments and results as ft_flowtree_knn with a candidate list (cand must
 * not be NULL); the output equals ft_flowtree_knn's bit for bit.  The call
 * allocates nothing: the prepared queries, the candidate costs and the
 * status words live in one static device array of about 7.8 MB per GPU,
 * held until the process ends and found at index build time.  Limits:
 * n_q <= FT_NOALLOC_MAX_QUERIES, total query support <= FT_NOALLOC_MAX_ITEMS,
 * n_q * n_cand <= FT_NOALLOC_MAX_PAIRS, n_cand <= 4096; larger inputs return
 * FT_ERANGE before any device work.  The index's device must be current.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (from several host threads, or on several streams without ordering)
 * race and must be serialised by the caller.  The call synchronises the
 * stream to read validation results, so it cannot be captured in a graph.
 * ---------------------------------------------------------------------- */
#define FT_NOALLOC_MAX_QUERIES 65536
#define FT_NOALLOC_MAX_ITEMS 262144
#define FT_NOALLOC_MAX_PAIRS 1048576
ft_status ft_flowtree_knn_noalloc(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                                  const uint32_t* q_mass, int64_t n_q, const int64_t* cand,
                                  int32_t n_cand, int32_t k, float* out_cost, int64_t* out_doc,
                                  void* stream);

/* ------------------------------------------------------------------------
 * ft_flowtree_cost_grad -- Flowtree cost of explicit (query, doc) pairs and
 * its gradient with the tree and the flow pattern held fixed.
 *
 * X[V*d]      float32 coordinates used to price the flow (device); same
 *             shape as the build's X, may differ in value (the tree and the
 *             flow come from the build and the integer masses).
 * pair_q[n], pair_d[n]  query index and doc index of each pair (device).
 * mode FT_FWD: cost[n] (float32) is written; the flow pattern of every pair
 *             is saved in the index for a following FT_BWD call with the
 *             same pairs and queries.
 * mode FT_BWD: grad_out[n] (float32 dL/dcost) is read; the call ADDS
 *             dL/dX to grad_X[V*d], dL/dw_q to grad_qmass[nnz_q] and dL/dw_d
 *             to grad_dmass[nnz_docs] (aligned with the caller's query CSR
 *             and the build's doc CSR), where w = mass / 2^Q.  Any of the
 *             three may be NULL.  With the pattern frozen, each match
 *             carries the unmatched mass of the item it used up (the dataset
 *             item when both were used up), which makes the cost linear in
 *             w; the gradient in X is eta * (x - y) / ||x - y|| per match
 *             (0 for coincident points).  The gradients are reproducible to
 *             the bit: dX is summed in 64-bit fixed point (unit 2^-40 of the
 *             largest |grad_out|, fewer fraction bits past 2^21 pairs), the
 *             weight gradients over each query's and each doc's pairs in pair
 *             order.  A non-finite grad_out gives FT_EINVAL.
 * ---------------------------------------------------------------------- */
ft_status ft_flowtree_cost_grad(ft_index* index, const float* X, const int64_t* q_off,
                                const uint32_t* q_id, const uint32_t* q_mass, int64_t n_q,
                                const int64_t* pair_q, const int64_t* pair_d, int64_t n_pairs,
                                int32_t mode, const float* grad_out, float* cost,
                                float* grad_X, float* grad_qmass, float* grad_dmass,
                                void* stream);

/* ------------------------------------------------------------------------
 * ft_flowtree_flows -- the Flowtree flow of explicit pairs, for inspection.
 *
 * cap_off[n_pairs+1] (device int64): pair p may write entries
 *             [cap_off[p], cap_off[p+1]); the slot count must be at least
 *             |supp q| + |supp d| (a flow has at most that many pairs minus
 *             one, Appendix A.1).
 * count[n_pairs] (int32) entries written per pair;
 * flow_d, flow_q (uint32): original point ids on the doc / query side;
 * flow_eta (uint32): integer mass moved; flow_bind (uint8): 0 = the match
 *             used up the doc item, 1 = the query item, 2 = both.
 * Entries appear level by level from the deepest cell up (not sorted).
 * ---------------------------------------------------------------------- */
ft_status ft_flowtree_flows(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                            const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                            const int64_t* pair_d, int64_t n_pairs, const int64_t* cap_off,
                            int32_t* count, uint32_t* flow_d, uint32_t* flow_q,
                            uint32_t* flow_eta, uint8_t* flow_bind, void* stream);

/* ------------------------------------------------------------------------
 * ft_quadtree_eps_pairs / ft_quadtree_eps_knn -- the Quadtree estimate on
 * the tree with eps-weighted edges used in the proof of the
 * uniform-distribution Flowtree upper bound: the edge above a cell of side
 * 2^l grid units weighs 2^(l (1 - eps)); eps = 0 is ft_quadtree_knn's key /
 * 2^Q.  Values sum_v w(v) |mu(v) - nu(v)| in units of mass fraction x grid
 * unit^(1 - eps), fp64 with integer masses.
 * eps         in [0, 1].
 * _pairs: out[n_pairs] device float64 for pairs (pair_q[p], pair_d[p]).
 * _knn:   candidate lists only (cand[n_q * n_cand], n_cand <= 4096);
 *         out_cost[n_q*k] float32 and out_doc ordered by (value, doc index).
 * A query may touch at most 4096 tree cells (FT_ERANGE).
 * (The Flowtree flow does not depend on the edge weights: the greedy is
 * optimal for any positive weights, so Flowtree has no eps variant.)
 * ---------------------------------------------------------------------- */
ft_status ft_quadtree_eps_pairs(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                                const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                                const int64_t* pair_d, int64_t n_pairs, double eps, double* out,
                                void* stream);
ft_status ft_quadtree_eps_knn(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                              const uint32_t* q_mass, int64_t n_q, const int64_t* cand,
                              int32_t n_cand, double eps, int32_t k, float* out_cost,
                              int64_t* out_doc, void* stream);

/* Quadtree keys (as ft_quadtree_knn) of explicit pairs: out_key[n_pairs].
 * A query may touch at most 4096 tree cells (FT_ERANGE). */
ft_status ft_quadtree_pairs(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                            const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                            const int64_t* pair_d, int64_t n_pairs, uint64_t* out_key,
                            void* stream);

/* ------------------------------------------------------------------------
 * ft_act_knn -- k nearest dataset distributions by ACT-iters, the capacity
 * constrained relaxation of W1 (Section 4.1 baseline; iters = 0 is Relaxed
 * WMD of Section 1.1): for every support point of one distribution, its
 * iters nearest points of the other each take at most their own mass and
 * the next nearest takes the rest; the larger of the two directions.
 * This is the quadratic-time stage the paper's pipelines place after
 * Flowtree.
 *
 * Arguments as ft_flowtree_knn, plus
 * iters       0..7.
 * out_cost[n_q*k] float32 2^-Q * sum mass x ||x - y||_2 in the units of X,
 *             ordered with out_doc by (cost, doc index).
 * Squared distances are |x|^2 + |y|^2 - 2<x,y> with every product and sum in
 * fp64 (exact widening of the fp32 coordinates), then rounded to fp32;
 * points of the same id are at distance 0, and values within 2^-40
 * (|x|^2 + |y|^2) of zero are recomputed in the difference form.  Nearest points at equal
 * distance are taken by ascending Morton rank (the value does not depend on
 * that order).
 * ---------------------------------------------------------------------- */
ft_status ft_act_knn(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                     const uint32_t* q_mass, int64_t n_q, const int64_t* cand, int32_t n_cand,
                     int32_t iters, int32_t k, float* out_cost, int64_t* out_doc, void* stream);

/* ACT-iters values (as ft_act_knn) of explicit pairs: out_cost[n_pairs]
 * (device float32), pair p = (query pair_q[p], doc pair_d[p]). */
ft_status ft_act_pairs(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                       const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                       const int64_t* pair_d, int64_t n_pairs, int32_t iters, float* out_cost,
                       void* stream);

/* ------------------------------------------------------------------------
 * ft_sinkhorn_knn -- k nearest dataset distributions by Sinkhorn with a
 * fixed number of iterations (Section 4.1 baseline; the regularisation is
 * set per pair from its largest cost, as in the appendix): with C the
 * pair's Euclidean cost matrix and M its largest entry, K = exp(-eta C / M);
 * from v = 1, each iteration sets u = a / (K v) then v = b / (K^T u); the
 * estimate is sum_ij u_i K_ij v_j C_ij (0 when M = 0).
 *
 * Arguments as ft_flowtree_knn, plus
 * iters       1..64 (the paper uses 1 and 3);
 * eta         > 0 (the paper uses 30).
 * out_cost[n_q*k] float32 estimates in the units of X, ordered with
 *             out_doc by (cost, doc index).
 * Costs come from the same fp64 inner-product blocks as ft_act_knn, rounded
 * to fp32; K is evaluated in fp32, sums in fp64.  Device scratch of up to
 * 4 GiB (largest doc support x largest query support floats per resident
 * workgroup) is kept with the index.
 * ---------------------------------------------------------------------- */
ft_status ft_sinkhorn_knn(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                          const uint32_t* q_mass, int64_t n_q, const int64_t* cand, int32_t n_cand,
                          int32_t iters, float eta, int32_t k, float* out_cost, int64_t* out_doc,
                          void* stream);

/* Sinkhorn values (as ft_sinkhorn_knn) of explicit pairs: out_cost[n_pairs]
 * (device float32), pair p = (query pair_q[p], doc pair_d[p]). */
ft_status ft_sinkhorn_pairs(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                            const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                            const int64_t* pair_d, int64_t n_pairs, int32_t iters, float eta,
                            float* out_cost, void* stream);

/* ------------------------------------------------------------------------
 * ft_exact_knn -- k nearest dataset distributions by the exact W1 distance
 * (Section 1, eq. (1): the cheapest transport of one distribution onto the
 * other at Euclidean cost), the last stage of the paper's pipelines.
 *
 * Arguments as ft_flowtree_knn.
 * out_cost[n_q*k] float32 W1 in the units of X, ordered with out_doc by
 *             (cost, doc index).
 * Each pair is solved exactly by successive shortest paths with node
 * potentials on the fp32 distance matrix (from the fp64 inner-product
 * blocks of ft_act_knn) with the integer masses; the value is summed in
 * fp64.  Cost grows with the pair sizes (quadratic per shortest path):
 * meant for a few candidates per query.  Device scratch of up to 4 GiB is
 * kept with the index.
 * ---------------------------------------------------------------------- */
ft_status ft_exact_knn(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                       const uint32_t* q_mass, int64_t n_q, const int64_t* cand, int32_t n_cand,
                       int32_t k, float* out_cost, int64_t* out_doc, void* stream);

/* Exact W1 (as ft_exact_knn) of explicit pairs: out_cost[n_pairs] (device
 * float32), pair p = (query pair_q[p], doc pair_d[p]). */
ft_status ft_exact_pairs(ft_index* index, const int64_t* q_off, const uint32_t* q_id,
                         const uint32_t* q_mass, int64_t n_q, const int64_t* pair_q,
                         const int64_t* pair_d, int64_t n_pairs, float* out_cost, void* stream);

/* Batched-schedule autotuner control.  level 0: fixed default schedule;
 * 1: tune on the first FT_BATCHED call of each workload shape and reuse the
 * winner (the default).  A JSON cache file is read and written at the path
 * in the environment variable FT_TUNE_CACHE when it is set. */
ft_status ft_set_autotune(ft_index* index, int32_t level);

/* Host timing of the last FT_BATCHED ft_flowtree_knn call (milliseconds,
 * measured with HIP events around the persistent Flowtree launches only),
 * and the schedule it used as text. */
ft_status ft_last_batched_stats(const ft_index* index, double* ms_flowtree, char* schedule,
                                int32_t schedule_len);

/* Rows of the last ft_quadtree_knn call (more than 4096 candidates per row)
 * whose one-pass select, which takes its threshold from a sample spread over
 * the row, found too few or too many keys under it and ran the exact
 * multi-pass select instead (the result is the same; the time is longer).
 * Waits for the device. */
ft_status ft_last_quadtree_stats(const ft_index* index, int64_t* select_exact_rows);

/* Device time of the kernels of the last ft_act_knn, ft_sinkhorn_knn or
 * ft_exact_knn call (milliseconds, HIP events recorded on the caller's
 * stream around the kernel launches; the query preparation and the top-k
 * select are outside). */
ft_status ft_last_rerank_stats(const ft_index* index, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* FTREE_H */
