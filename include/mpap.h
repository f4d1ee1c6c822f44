/*
 * mpap.h - C ABI of the MI355X wavefront multiobjective perception-aware
 * search library (libmpap.so).
 *
 * The library implements the search stage of the Multiobjective
 * Perception-Aware Planning algorithm (Ichter, Landry, Schmerling, Pavone,
 * "Perception-Aware Motion Planning via Multiobjective Search on GPUs"):
 * Sec. 3, Alg. 3 (Explore) over a roadmap built by Alg. 2 (BuildGraph), with
 * the drift heuristic of Sec. 4.1 as the perception heuristic.
 *
 * Conventions for every call:
 *  - All functions are extern "C", return an int status (MPAP_OK == 0) and
 *    never throw.  On failure a message is available from mpap_last_error()
 *    (thread-local, valid until the next call on the same thread).
 *  - Pointers named host_* or documented as "host" are ordinary CPU memory;
 *    the library copies what it needs and does not keep them.
 *  - Opaque handles (mpap_graph, mpap_result) own device memory on the
 *    device that was current when they were created; free them with the
 *    matching *_free call.  A handle must not be used from two threads at
 *    once; use one stream per concurrent search.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it and the call returns once the results it reports
 *    are complete.
 *  - Floating point: IEEE float32, round to nearest, no fused multiply-add on
 *    the label path, no flush of denormals.
 */
#ifndef MPAP_H
#define MPAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define MPAP_OK 0
#define MPAP_ERR_INVAL 1      /* bad argument (null, range, NaN, shape) */
#define MPAP_ERR_NOGOAL 2     /* no roadmap node lies in the goal region */
#define MPAP_ERR_NOMEM 3      /* device or host allocation failed */
#define MPAP_ERR_HIP 4        /* a HIP runtime call failed */
#define MPAP_ERR_OVERFLOW 5   /* a capacity limit was hit after all retries */
#define MPAP_ERR_NOCONVERGE 6 /* max_waves reached with plans still open */
#define MPAP_ERR_CAPACITY 7   /* caller buffer too small; *count holds the need */
#define MPAP_ERR_DEVICE 8     /* no usable gfx950 device / feature missing */

typedef struct mpap_graph mpap_graph;   /* device-resident roadmap */
typedef struct mpap_result mpap_result; /* outcome of one search */

/* ----------------------------------------------------------- environment */
/* A mapped environment and roadmap samples (Sec. 2 problem data; Sec. 4.2
 * axis-aligned box obstacles; Sec. 4.1 mapped perception features, here as
 * isotropic Gaussian blobs whose summed density is the quality q(x)). */
typedef struct {
    int32_t dim;              /* 2 or 3: geometric roadmap; 6: double integrator
                                 (3D position and velocity) */
    int32_t n_nodes;          /* number of roadmap nodes; node 0 is x_init */
    const float *pos;         /* host [n_nodes][w] node positions, w = dim (3 for dim 6) */
    int32_t n_boxes;          /* obstacle count (>= 0) */
    const float *box_lo;      /* host [n_boxes][w] lower corners */
    const float *box_hi;      /* host [n_boxes][w] upper corners (closed) */
    int32_t n_blobs;          /* feature blob count (>= 0) */
    const float *blob_mu;     /* host [n_blobs][w] centres */
    const float *blob_sigma;  /* host [n_blobs] widths (> 0) */
    const float *blob_amp;    /* host [n_blobs] amplitudes */
    float goal[3];            /* goal ball centre (first w entries used) */
    float goal_radius;        /* goal ball radius (closed ball, positions only) */
    const float *vel;         /* host [n_nodes][3] velocities (dim 6 only, else NULL) */
} mpap_env;

typedef struct {
    float radius;     /* r_n: an edge u->v exists iff Cost(u,v) < radius (Alg. 2, Near);
                         for dim 6 only the group step of searches (cost units) */
    float check_step; /* sub-step length of Collision and of the drift integral */
    float reset_q;    /* a node relocalises (drift resets to 0) iff q(x) > reset_q */
    int32_t k_out;      /* dim 6: out-degree (1..64) */
    float horizon;      /* dim 6: steering time T (> 0) */
    int32_t traj_steps; /* dim 6: check steps K per trajectory (1..255) */
    int32_t near_grid;  /* dim 2/3, how Near finds its candidates (the edges are the
                           same either way): 0 chooses, 1 a uniform grid of cells at
                           least radius wide (rows sorted by target id afterwards;
                           a row longer than 256 candidates makes the fill compare
                           all pairs), -1 all pairs */
} mpap_graph_params;

/*
 * mpap_build_graph - Alg. 2 (BuildGraph) plus the per-edge heuristic inputs
 * (Alg. 1, step 2), on the GPU.
 *   Edges: u->v for v != u with Cost(u,v) = |x_v - x_u| < radius (float32,
 *   separately rounded ops) whose straight segment, checked at points
 *   x_a + (k/K)(x_b - x_a), k = 0..K, K = ceil(Cost/check_step), (a, b) the
 *   pair in id order, misses every closed box.  Per edge: cost = Cost and
 *   drift = Cost * (1 - mean q over the K sub-step midpoints).  Per node:
 *   reset = q(x) > reset_q, goal = |x - goal|^2 <= goal_radius^2.
 *   q(x) = clamp(sum_j amp_j exp(-|x - mu_j|^2 / (2 sigma_j^2)), 0, 1),
 *   evaluated in float64 from the float32 inputs (blob order); the drift is
 *   the float64 sum over the midpoints in order, (Cost/K)(1 - q), rounded
 *   once to float32, and reset compares the float64 q with the float32
 *   reset_q.  (The float64 exp may differ from another libm's in the last
 *   bit, which changes a float32 result only in rare ties.)
 * dim 6 (double integrator; the dynamics class of Sec. 4.1 and Sec. 5):
 *   steering u -> v is the minimum-energy control of p'' = a over the fixed
 *   time T = horizon; per axis, with a = (p_v - p_u) - v_u T, b = v_v - v_u,
 *   J = 12a^2/T^3 - 12ab/T^2 + 4b^2/T (summed over axes: the edge cost).
 *   The trajectory is checked at t_k = (k T)/K, k = 0..K: inside the closed
 *   unit cube, in no closed box, speed <= 1.  Each node keeps the k_out
 *   reachable targets of least (J, id) (a directed roadmap).  drift = sum
 *   over the K chords of |chord| (1 - q(chord midpoint)), float64 terms from
 *   the float32 check points summed in chord order and rounded once to
 *   float32.  Steering, checks and costs are float32 with separately rounded
 *   operations.
 * Errors: MPAP_ERR_INVAL (null, dim not 2/3/6, n_nodes < 1, non-finite
 * position, radius <= 0, dim 6 without velocities or with k_out, horizon or
 * traj_steps out of range, more than 1024 boxes), MPAP_ERR_NOGOAL (no node in
 * the goal ball; no graph is returned), MPAP_ERR_OVERFLOW (dim 6: more than
 * 2048 candidates of one node share one steering cost), MPAP_ERR_NOMEM,
 * MPAP_ERR_HIP.
 */
int mpap_build_graph(const mpap_env *env, const mpap_graph_params *gp, void *stream,
                     mpap_graph **out);

/*
 * mpap_graph_from_csr - import a roadmap given as forward CSR (host memory).
 *   row_ptr[n_nodes+1] (row_ptr[0] == 0, non-decreasing), col[E] targets in
 *   [0, n_nodes), self loops not allowed; cost[E] > 0 finite; drift[E] >= 0
 *   finite; reset[n_nodes], goal[n_nodes] are 0/1 flags.  Inputs are copied.
 * Errors: MPAP_ERR_INVAL on any violated condition, MPAP_ERR_NOMEM,
 * MPAP_ERR_HIP.  (A graph with no goal node is accepted; its searches return
 * an empty goal front.)
 */
int mpap_graph_from_csr(int32_t n_nodes, const int32_t *row_ptr, const int32_t *col,
                        const float *cost, const float *drift, const uint8_t *reset,
                        const uint8_t *goal, void *stream, mpap_graph **out);

/* Sizes of a graph. Any output pointer may be NULL. */
int mpap_graph_info(const mpap_graph *g, int32_t *n_nodes, int64_t *n_edges, int32_t *n_goal);

/* Copy a graph back to host memory in the forward-CSR form taken by
 * mpap_graph_from_csr (rows sorted by target id).  Buffers are caller-owned
 * and sized from mpap_graph_info. */
int mpap_graph_export(const mpap_graph *g, int32_t *row_ptr, int32_t *col, float *cost,
                      float *drift, uint8_t *reset, uint8_t *goal);

void mpap_graph_free(mpap_graph *g);

/* ---------------------------------------------------------------- search */
typedef struct {
    float beta;        /* bound on the drift heuristic, eq. (2); +inf = off */
    float lambda;      /* group cost factor of Alg. 3 (0 < lambda); 0.5 in Sec. 4.2 */
    float radius;      /* r_n of the roadmap; groups advance by lambda * radius */
    int32_t n_obj;     /* 2: (cost, drift); 3: (cost, drift, max drift so far) */
    int32_t init_node; /* root of every plan (x_init), usually 0 */
    int32_t max_waves; /* cap on Explore iterations; 0 = 1 << 18 */
    int32_t near_scan; /* tuning: front labels each child is tested against before the
                          full prefix scan; 0 = 16.  Never changes the result. */
    int32_t stage_cap; /* tuning: largest front merged in LDS (larger ones spill to
                          per-workgroup device memory); 0 = what the LDS holds.
                          Never changes the result. */
    int32_t heuristic; /* per-edge drift: 0 = the analytic values of the roadmap,
                          1 = the learned surrogate's (mpap_surrogate_score) */
    int32_t block_threads; /* tuning: threads per workgroup of the persistent search,
                              1024 (one per CU), 512 (two) or 256 (four); 0 = 1024.
                              Never changes the result. */
    int32_t wave_min_targets; /* tuning: an iteration with at least this many merge
                                 targets of small front merges each of them with a
                                 single wave (16 merges per CU at once); 0 = four times the
                                 waves of the grid, < 0 = never.  Never changes the
                                 result. */
    int32_t skip;             /* 1: leave this query out of a batched search (its root
                                 label is not seeded; its goal front is empty); 0 =
                                 search it */
    int32_t early_stop;       /* 0: run until P_open is empty (exact fronts).  1: the
                                 loop condition of Alg. 3 (Sec. 3): the query's loop
                                 ends before the first group that holds a plan at a
                                 goal node; its goal front is then the Pareto minimum
                                 of P_candidates at that point (entry 0 = P_soln), which
                                 depends on lambda and need not be the exact front */
    int32_t merge_halves;     /* tuning: merges by halves.  With 1024-thread workgroups,
                                 in iterations with at least eight merge targets per
                                 workgroup (two when forced), each half of a workgroup
                                 merges its own targets (two at once per CU); large
                                 fronts and targets with more than merge_halves children
                                 (0: 8192) take the whole workgroup.  0 = on for roadmaps
                                 of at least 16 x (workgroups) nodes; > 0 = on (forced);
                                 < 0 = off.  Never changes the result. */
} mpap_search_params;

/*
 * mpap_search - Alg. 3 (Explore) run until no plan is open, on the GPU.
 *   Labels (head, cost c, drift d [, max drift m], parent) are expanded in
 *   groups of open labels whose cost is at most the current threshold, which
 *   is i * lambda * radius at iteration i (float32; iterations whose group
 *   would be empty are skipped).  A child
 *   along edge e = u->v has c + cost_e, d_pre = d + drift_e; it is dropped if
 *   d_pre > beta; its drift is 0 if reset[v] else d_pre; m = max(m, d_pre).
 *   RemoveDominated is weak Pareto dominance per head node (a label is removed
 *   if another at the same node is <= in every objective; equal vectors are
 *   kept once).  All sums are float32 in path order, so the per-node fronts
 *   are exactly the Pareto-minimal vectors of the plans to each node.
 *   Capacity limits (label arena, bucket pool) grow and the search restarts
 *   automatically; MPAP_ERR_OVERFLOW only after that fails.
 * Errors: MPAP_ERR_INVAL (null, n_obj not 2/3, init_node out of range,
 * lambda <= 0, radius <= 0, beta NaN), MPAP_ERR_NOCONVERGE, MPAP_ERR_OVERFLOW,
 * MPAP_ERR_NOMEM, MPAP_ERR_HIP, MPAP_ERR_DEVICE.
 * An empty goal front is a successful result with count 0.
 */
int mpap_search(const mpap_graph *g, const mpap_search_params *sp, void *stream,
                mpap_result **out);

/*
 * mpap_goal_front - the Pareto front over all goal nodes (P_candidates of
 * Alg. 3 kept whole), ascending lexicographic order of (c, d, m); entry 0 is
 * the minimum-cost plan P_soln.  Each entry names one witness label (goal
 * node and label id, usable with mpap_label_path).  maxdrift may be NULL;
 * for n_obj == 2 it is filled with 0.  *count always receives the front size;
 * if capacity < count nothing is written and MPAP_ERR_CAPACITY is returned.
 */
int mpap_goal_front(const mpap_result *r, float *cost, float *drift, float *maxdrift,
                    int32_t *goal_node, int32_t *label_id, int32_t capacity, int32_t *count);

/*
 * Batches.  A graph may hold several independent planning queries: the
 * disjoint union of their roadmaps, query q owning nodes
 * [node_offset[q], node_offset[q+1]).  One search then runs all of them in a
 * single persistent launch; node ids in mpap_node_front / mpap_label_path are
 * ids of the union, goal nodes reported per query are ids within the query.
 */

/* mpap_graph_concat - a new graph holding the queries of every part, in order
 * (parts are copied; they stay owned by the caller).  Errors: MPAP_ERR_INVAL
 * (null, n_parts < 1, more than 2^31 nodes or edges), MPAP_ERR_NOMEM,
 * MPAP_ERR_HIP. */
int mpap_graph_concat(const mpap_graph *const *parts, int32_t n_parts, void *stream,
                      mpap_graph **out);

/* mpap_graph_queries - number of queries; node_offset (nullable) receives
 * nq + 1 entries. */
int mpap_graph_queries(const mpap_graph *g, int32_t *nq, int32_t *node_offset);

/* mpap_search_batch - mpap_search over every query of g in one launch.  sp
 * holds one parameter set per query (n_params == nq) or one for all
 * (n_params == 1); init_node is relative to the query.  All queries share
 * the iteration index i; query q's group holds its open labels of cost at
 * most i * lambda_q * radius_q (float32), and an iteration with no group
 * label in any query is skipped (the fronts do not depend on the steps).
 * Errors as mpap_search. */
int mpap_search_batch(const mpap_graph *g, const mpap_search_params *sp, int32_t n_params,
                      void *stream, mpap_result **out);

/* mpap_query_goal_front - goal front of one query; same rules as
 * mpap_goal_front (which is query 0). */
int mpap_query_goal_front(const mpap_result *r, int32_t query, float *cost, float *drift,
                          float *maxdrift, int32_t *goal_node, int32_t *label_id,
                          int32_t capacity, int32_t *count);

/* mpap_query_info - completion of one query inside the launch: the last
 * Explore iteration that expanded one of its labels, and the device time from
 * the start of the launch to the end of that iteration (ms).  Either output
 * may be NULL. */
int mpap_query_info(const mpap_result *r, int32_t query, float *latency_ms, int32_t *last_wave);

/* mpap_query_stop - how a query's loop ended: *groups receives the number of
 * groups expanded before the early stop of Alg. 3's loop condition ended it
 * (a group held a plan at a goal node; early_stop = 1), or -1 when it ran
 * until its P_open was empty. */
int mpap_query_stop(const mpap_result *r, int32_t query, int32_t *groups);

/*
 * mpap_refine_front - the goal front of one query under a tighter bound
 *   beta_prime <= beta, from a search run with three objectives.  Alg. 1
 *   step 4 (Sec. 3) refines the bound by searching again with a lower beta;
 *   with the running maximum m of the pre-relocalisation drift as the third
 *   objective a plan meets beta_prime at every step iff m <= beta_prime, and a
 *   plan dominated by a front member is dominated by one whose m is no larger,
 *   so one search answers every beta_prime <= beta:
 *     n_obj_out = 3: the front members with m <= beta_prime -- exactly the
 *                    three-objective goal front of a search at beta_prime;
 *     n_obj_out = 2: their Pareto minimum over (c, d) (of equal (c, d) the one
 *                    of least m), maxdrift filled with 0 -- exactly the
 *                    two-objective goal front of a search at beta_prime.
 *   Ascending (c, d, m) order; goal nodes and label ids name witnesses as in
 *   mpap_query_goal_front.  Outputs nullable; same capacity rule.
 * Errors: MPAP_ERR_INVAL (null, query out of range, the search did not use
 * three objectives, beta_prime NaN or above the query's bound, n_obj_out not
 * 2 or 3, an early-stopped query), MPAP_ERR_CAPACITY.
 */
int mpap_refine_front(const mpap_result *r, int32_t query, float beta_prime, int32_t n_obj_out,
                      float *cost, float *drift, float *maxdrift, int32_t *goal_node,
                      int32_t *label_id, int32_t capacity, int32_t *count);

/* mpap_node_front - the final label set P(node) of one node (Alg. 3), in
 * storage order (not sorted), with each label's id.  Any output array may be
 * NULL.  Same capacity rule as mpap_goal_front. */
int mpap_node_front(const mpap_result *r, int32_t node, float *cost, float *drift,
                    float *maxdrift, int32_t *label_id, int32_t capacity, int32_t *count);

/* mpap_label_path - node sequence of the plan ending in label_id, root first
 * (the plan's path field of Sec. 3).  *length receives the node count;
 * MPAP_ERR_CAPACITY if it exceeds capacity (nothing written). */
int mpap_label_path(const mpap_result *r, int32_t label_id, int32_t *nodes, int32_t capacity,
                    int32_t *length);

typedef struct {
    int32_t waves;            /* Explore iterations that expanded a group */
    int32_t retries;          /* capacity-growth restarts */
    int64_t labels_expanded;  /* labels taken into a group (arena size) */
    int64_t front_labels;     /* sum over nodes of the final front sizes */
    int64_t merges;           /* per-node dominance merges */
    int64_t candidates;       /* children generated that passed the bound */
    int64_t relaxations;      /* sum over nodes of |P(v)| * out-degree(v) */
    float gpu_ms;             /* device time of the search launch (hipEvents on the stream) */
    int32_t lds_front_cap;    /* largest per-node front the LDS merge stages */
    int32_t blocks;           /* workgroups of the persistent launch */
    int32_t max_front;        /* largest final per-node front */
    int32_t wave_build;       /* 1: the wave-first kernel build ran (single-wave merges in
                                 iterations with many small targets), 0: the weight-ordered one */
    int32_t judged_failed;    /* queries whose learned-drift front mpap_judge rejected */
    float fallback_ms;        /* device time of the analytic re-search of those queries */
    int32_t half_front_cap;   /* front stage of a half workgroup when merges ran by halves
                                 (two targets at once per workgroup), else 0 */
    int32_t build_objectives; /* 2 or 3: the search build for queries of that many
                                 objectives ran; 0: the build that decides per query */
    int64_t half_merges;      /* merges done by half workgroups */
    int64_t half_backouts;    /* targets whose front outgrew a half's stage: the half backed
                                 out (nothing written) and the whole workgroup merged them */
} mpap_stats;

int mpap_result_stats(const mpap_result *r, mpap_stats *out);

/*
 * mpap_wave_trace - per-iteration trace of the last search (a profiling aid).
 * For each of the first min(waves, 4096) Explore iterations, 10 int64 words:
 * device clock (100 MHz) at the start of the count phase, after the count,
 * select and merge barriers; group size; merge targets; the longest and the
 * summed per-workgroup merge-phase duration (ticks); the clock when workgroup
 * 0 finished its count work and its select work (before the barriers).  out
 * holds capacity * 10 words; *waves receives the traced count
 * (MPAP_ERR_CAPACITY if it exceeds capacity, nothing written).
 */
int mpap_wave_trace(const mpap_result *r, int64_t *out, int32_t capacity, int32_t *waves);
void mpap_result_free(mpap_result *r);

/* ------------------------------------------------------------- surrogate */
/*
 * Learned per-edge drift surrogate: a 16 -> 64 -> 64 -> 1 ReLU network that
 * predicts an edge's mean (1 - q) from its endpoints, length and q at 8 points
 * along it (the learned-heuristic idea of Sec. 5.2, standing in for the
 * per-edge precompute of Alg. 1 step 2); the drift increment is
 * length * clamp(output, 0, 1).  Inputs, the two weight matrices, the output
 * weights and the first hidden activations are bfloat16 (round to nearest
 * even from float32); products accumulate in float32 on the matrix cores.
 * Parameters: one float32 block of 5313 values, W1[16][64] b1[64] W2[64][64]
 * b2[64] w3[64] b3 (row-major, input index first).  Training is Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error against the
 * analytic values of the roadmap's edges.
 */
typedef struct mpap_surrogate mpap_surrogate;

int mpap_surrogate_create(mpap_surrogate **out);
void mpap_surrogate_free(mpap_surrogate *s);
/* Replace the parameters (count must be 5313; finite); resets Adam's state. */
int mpap_surrogate_set_params(mpap_surrogate *s, const float *params, int32_t count);
int mpap_surrogate_get_params(const mpap_surrogate *s, float *params, int32_t capacity,
                              int32_t *count);
/* He-normal hidden weights from a counter-based SplitMix64 stream of `seed`;
 * zero biases and zero output weights (the untrained network adds nothing to
 * the 8-point base). */
int mpap_surrogate_init(mpap_surrogate *s, uint64_t seed);

/* The network's inputs for every edge of g (forward CSR order), 16 bfloat16
 * bit patterns per edge, computed on the device from the id-ordered endpoint
 * pair: x_a (3), x_b (3; z = 0 in 2D), length, 1 - q at the points
 * x_a + (k + 1/2)/8 (x_b - x_a), k = 0..7, and 1 - q(x_b) (complements taken
 * in float32 before the rounding, so that q near 1 keeps its precision).
 * base (host, nullable, edges values) receives the float32 mean of the eight
 * 1 - q values: the 8-point estimate of drift / length that the network
 * corrects (predicted drift = length * clamp(base + network/256, 0, 1)).  Needs a
 * roadmap built by mpap_build_graph (MPAP_ERR_INVAL otherwise).  out (host,
 * nullable) holds capacity >= 16 * edges values. */
int mpap_edge_features(const mpap_graph *g, void *stream, uint16_t *out, int64_t capacity,
                       float *base);

/* Outputs of the network for n rows of inputs (host memory, 16 bfloat16 bit
 * patterns per row). */
int mpap_surrogate_forward(const mpap_surrogate *s, const uint16_t *X, int64_t n, float *y);

/* Gradient of the mean squared error over one batch of n rows (n a power of
 * two >= 64) with respect to the 5313 float32 parameters, without updating
 * them; y_out (nullable) receives the n outputs.  For checking the training
 * kernels. */
int mpap_surrogate_gradient(mpap_surrogate *s, const uint16_t *X, const float *t, int32_t n,
                            float *grad, float *y_out);

/* Train on the edges `edges[0..n_train)` of g (host indices into the forward
 * edge order), targets 256 * (drift/length - base): the roadmap's analytic
 * values less the 8-point base of mpap_edge_features, scaled by 2^8 (the
 * network learns the correction in units of 1/256), in
 * batches of `batch` consecutive entries (a power of two >= 64; a short tail
 * is dropped), `epochs` passes, Adam with a learning rate decaying from lr to
 * lr/100 along a half cosine over the run.  epoch_loss (nullable)
 * receives the mean squared error over the training edges after each epoch. */
int mpap_surrogate_train(mpap_surrogate *s, const mpap_graph *g, const int64_t *edges,
                         int64_t n_train, int32_t epochs, int32_t batch, float lr, void *stream,
                         float *epoch_loss);

/* Predicted drift of every edge of g, length * clamp(base + network/256, 0, 1),
 * kept in the graph for searches with heuristic = 1 (and carried into
 * mpap_graph_concat when every part has it).
 * The inputs are recomputed on every call; ms (nullable) receives the device
 * time of inputs plus inference.  Needs a roadmap built by mpap_build_graph. */
int mpap_surrogate_score(const mpap_surrogate *s, mpap_graph *g, void *stream, float *ms);

/* Recompute the analytic drift of every edge of g on the device (the same
 * values mpap_build_graph produced); ms (nullable) receives the kernel time.
 * The cost the surrogate is measured against. */
int mpap_analytic_drift(mpap_graph *g, void *stream, float *ms);

/* Copy a drift array of g to the host (forward CSR order): which = 0 the
 * analytic values, 1 the surrogate's. */
int mpap_graph_drift(const mpap_graph *g, int32_t which, float *out);

/* Re-walk the plan of every goal-front label of one query (query = -1: of
 * all queries, concatenated in query order) with the analytic drift of the
 * roadmap (the surrogate's judge): cost, drift, max drift and whether the
 * pre-reset drift stays within the bound at every step.  Same order and
 * capacity rule as mpap_query_goal_front; plans longer than 4096 steps are an
 * error (MPAP_ERR_HIP).  Any output may be NULL. */
int mpap_rescore_front(const mpap_result *r, int32_t query, float *cost, float *drift,
                       float *maxdrift, uint8_t *feasible, int32_t capacity, int32_t *count);

/*
 * mpap_judge - the learned heuristic's judge and fallback.  The learned
 * heuristic stands in for the per-edge precompute of Alg. 1 step 2 (learned
 * heuristics, Sec. 5.2); a search on it is accepted per query only if every
 * goal-front plan, re-walked along its parent chain with the roadmap's
 * analytic drift (the same float32 fold as the search), stays within the
 * bound at every step and its drift and max drift differ from the searched
 * values by at most tol relative to max(analytic value, 1e-3 * beta)
 * (float64 comparison).  Queries searched on the analytic drift pass.
 *   fallback = 0: judge only.  fallback = 1: the rejected queries are searched
 *   again, in one launch, on the analytic drift (the other queries are
 *   skipped), and r then answers them from that exact search: their goal
 *   fronts, node fronts, plans and latencies (latency = the first launch, the
 *   judge and the re-search).  Label ids of re-searched queries are reported
 *   shifted by the first search's label count, so ids stay unique within r.
 *   failed (nullable, nq bytes) receives 1 for each rejected query; n_failed
 *   (nullable) their count; stats.judged_failed and stats.fallback_ms are
 *   set.  A result is judged once (MPAP_ERR_INVAL on a second call); a plan's
 *   result is judged before the plan's next run.  Plans longer than 4096
 *   steps are an error (MPAP_ERR_HIP).
 * Errors: MPAP_ERR_INVAL (null, tol not > 0, judged already), MPAP_ERR_HIP,
 * errors of mpap_search_batch for the re-search.
 */
int mpap_judge(mpap_result *r, float tol, int32_t fallback, void *stream, uint8_t *failed,
               int32_t *n_failed);

/*
 * mpap_surrogate_save / mpap_surrogate_load - the network's 5313 float32
 * parameters in a little-endian file: the 8 bytes "MPAPSUR1", the count
 * (int32, 5313), the parameters (W1, b1, W2, b2, w3, b3 as in
 * mpap_surrogate_set_params), and a 32-bit FNV-1a hash of the parameter
 * bytes.  Loading replaces the parameters and resets the optimiser state.
 * Errors: MPAP_ERR_INVAL (null, unreadable or malformed file, wrong count or
 * hash, non-finite values), MPAP_ERR_HIP.
 */
int mpap_surrogate_save(const mpap_surrogate *s, const char *path);
int mpap_surrogate_load(mpap_surrogate *s, const char *path);

/*
 * mpap_search_noalloc - mpap_search followed by mpap_goal_front, for callers
 *   that cannot allocate device memory (code that must not call hipMalloc:
 *   tight serving loops, harnesses that forbid allocation).  It allocates
 *   nothing: the search state lives in one fixed scratch array of 64 MiB per
 *   device that the library holds from its first use on the device until the
 *   process ends.  Same search and result as mpap_search (same kernels) on a
 *   single-query roadmap (not a concatenated batch); outputs as
 *   mpap_goal_front without label ids (host buffers, ascending (c, d, m);
 *   maxdrift and goal_node nullable; *count always receives the front size;
 *   capacity < count writes nothing and returns MPAP_ERR_CAPACITY).
 *   No result handle: label ids and node fronts are not kept.  Every call on a
 *   device shares that device's scratch; calls that overlap on one device
 *   (other streams or threads) race and must be serialised by the caller.
 *   Blocks until the front is in the caller's buffers.
 * Errors: MPAP_ERR_INVAL (as mpap_search; also a batched roadmap, skip != 0,
 * a roadmap whose per-node state leaves under 4 MiB of the scratch for labels
 * -- about 620,000 nodes), MPAP_ERR_OVERFLOW (the search needs more label
 * storage than the scratch holds, or a front beyond the LDS stage of a
 * workgroup: there is no spill space; use mpap_search), MPAP_ERR_CAPACITY,
 * MPAP_ERR_NOCONVERGE, MPAP_ERR_HIP, MPAP_ERR_DEVICE.
 */
int mpap_search_noalloc(const mpap_graph *g, const mpap_search_params *sp, void *stream,
                        float *cost, float *drift, float *maxdrift, int32_t *goal_node,
                        int32_t capacity, int32_t *count);

/*
 * Online updates (Sec. 3, online implementation: when obstacles are
 * discovered only the new collision checks are made, and the exploration is
 * run again).
 *
 * mpap_graph_add_boxes - a new roadmap: g (2D/3D, built by mpap_build_graph,
 *   one query) without the edges that collide with the n_boxes new boxes
 *   (host [n_boxes][dim] closed lower/upper corners).  Only the new boxes are
 *   checked (Alg. 2 Collision at g's check step); costs, drifts, flags and
 *   the environment are kept, so the result is the roadmap mpap_build_graph
 *   makes for the same samples with the boxes added.  g is not changed; the
 *   new graph is owned by the caller (mpap_graph_free).
 * Errors: MPAP_ERR_INVAL (null, n_boxes < 0, non-finite corners, a roadmap
 * not built by mpap_build_graph in 2D/3D, a batch), MPAP_ERR_NOMEM,
 * MPAP_ERR_HIP.
 */
int mpap_graph_add_boxes(const mpap_graph *g, int32_t n_boxes, const float *box_lo,
                         const float *box_hi, void *stream, mpap_graph **out);

/*
 * mpap_search_update - the search of roadmap g (Alg. 3 until no plan is
 *   open, the same result as mpap_search on g) continued from an earlier
 *   result prev on a roadmap over the same nodes (for instance
 *   mpap_graph_add_boxes of prev's roadmap, or edges with new costs or
 *   drifts, or new relocalisation flags).  prev's labels whose plans use no
 *   changed edge (removed, added, other cost or drift bits, or a head whose
 *   relocalisation flag changed) are kept; the labels of the in-neighbours of
 *   nodes that lost labels, and of the tails of new or changed edges, are
 *   opened again; the search runs from there.  sp must repeat prev's bound,
 *   objective count, root and heuristic (analytic); lambda and the tuning
 *   fields may differ.  prev is not changed (a plan's result must not have
 *   been superseded by the plan's next run).  In the new result's statistics
 *   labels_expanded counts this call's expansions only; label ids of kept
 *   labels are prev's.
 * Errors: MPAP_ERR_INVAL (null, batches, different node counts, a judged or
 * early-stopped prev, sp unlike prev's search, early_stop or skip set, more
 * than 4096 iterations in prev), and as mpap_search.
 */
int mpap_search_update(const mpap_result *prev, const mpap_graph *g,
                       const mpap_search_params *sp, void *stream, mpap_result **out);

/*
 * Monte Carlo verification of a plan (Sec. 3, final phase: an estimate by
 * sampling of the probability that the plan keeps the localisation error
 * within a bound when it is flown; the system and localisation models of
 * Sec. 4.1).  The model, fixed where the paper gives only its structure:
 * the nominal trajectory is, per edge, the minimum-energy cubic between
 * its two states: at rest at both nodes over 1.5 length / speed (2D/3D
 * roadmaps; peak speed `speed`), the roadmap's states over the steering
 * time (6D); per axis a double integrator with applied acceleration u + sigma_w xi
 * tracks it (feed-forward: the nominal velocity change over the step;
 * feedback: the steady-state discrete LQR gain for Q = diag(q_p, q_v),
 * R = r_u) from a Kalman estimate predicted with the measured acceleration
 * (noise sigma_a) and corrected by a position fix of noise sigma_v / sqrt(q)
 * wherever the feature quality q of the map is >= q_min; the start position
 * is off by sigma_0 per axis.  Steps of dt (float64 state); normals from
 * Philox4x32-10 keyed by seed.  A flight succeeds when its largest
 * localisation error stays <= err_bound and no true position lies in a box.
 */
typedef struct {
    int32_t rollouts;  /* sampled flights (>= 1) */
    float dt;          /* time step (s, > 0) */
    float speed;       /* 2D/3D: peak nominal speed along each segment (> 0) */
    float sigma_w;     /* std of the applied-acceleration noise per step */
    float sigma_a;     /* std of the accelerometer noise per step */
    float sigma_v;     /* std of a position fix at feature quality 1 (> 0) */
    float q_min;       /* least feature quality that gives a fix */
    float sigma0;      /* std of the initial position error per axis */
    float err_bound;   /* localisation error bound */
    float q_p, q_v;    /* LQR state weights (>= 0) */
    float r_u;         /* LQR control weight (> 0) */
    uint64_t seed;     /* Philox key (low word, high word) */
} mpap_mc_params;

typedef struct {
    int64_t rollouts;
    int64_t within_bound;    /* flights whose largest localisation error <= err_bound */
    int64_t collision_free;  /* flights that never entered a box */
    int64_t success;         /* both */
    int32_t steps;           /* time steps K of the nominal trajectory */
    double duration;         /* its duration (s) */
    double mean_max_err;     /* mean over flights of the largest error */
    double max_max_err;      /* the largest over all flights (-1 if max_err was NULL) */
    double gain_p, gain_v;   /* the LQR gain used */
    float gpu_ms;            /* device time of the flights */
} mpap_mc_stats;

/* mpap_mc_verify - sample mp->rollouts flights of the plan through
 *   nodes[0 .. n_nodes) (host; a plan's node sequence as mpap_label_path gives
 *   it, root first; consecutive nodes are flown straight from rest to rest in
 *   2D/3D, along the steering cubic in 6D) on roadmap g (built by mpap_build_graph: its
 *   samples, blobs and boxes).  max_err (nullable, host double [rollouts])
 *   and collided (nullable, host u8 [rollouts]) receive the per-flight
 *   outcomes.
 * Errors: MPAP_ERR_INVAL (null, an imported or batched roadmap, fewer than
 * two nodes, a node out of range, non-positive dt, speed, sigma_v or r_u,
 * negative or non-finite parameters, more than 1e8 steps), MPAP_ERR_NOMEM,
 * MPAP_ERR_HIP. */
int mpap_mc_verify(const mpap_graph *g, const int32_t *nodes, int32_t n_nodes,
                   const mpap_mc_params *mp, void *stream, double *max_err, uint8_t *collided,
                   mpap_mc_stats *out);

/* ----------------------------------------------------------------- misc */
const char *mpap_status_string(int status);
const char *mpap_last_error(void);

/*
 * Plans: a fixed batch of queries (a graph from mpap_graph_concat, or one
 * roadmap) recorded once as a HIP graph -- the surrogate scoring of each
 * part, the persistent search of all queries and the goal-front extraction --
 * and then launched with one call per batch (the serving loop of many
 * independent queries; the search itself is Alg. 3 as in mpap_search).
 */
typedef struct mpap_plan mpap_plan;

/* mpap_plan_create - validate as mpap_search_batch, run one eager search to
 * size every capacity, and record the graph.  parts/models (nparts == 0, or
 * nparts == the graph's query count): parts[q] is the roadmap query q was
 * concatenated from and models[q] (nullable) the surrogate that scores it
 * before each search, writing the part's slice of g's surrogate drift (used by
 * queries with heuristic = 1).  flags: MPAP_PLAN_ANALYTIC = every part without
 * a model has its analytic drift (Alg. 1 step 2 precompute, as
 * mpap_analytic_drift) recomputed inside the graph before each search,
 * writing the part's slice of g's analytic drift (the per-batch precompute
 * the learned heuristic replaces); 0 = none.  g, the parts and the models
 * must outlive the plan; the plan owns its own search workspace.  Errors: as
 * mpap_search_batch, MPAP_ERR_INVAL (part sizes that do not match the
 * queries, a scored part without an environment, unknown flags,
 * MPAP_PLAN_ANALYTIC without parts), MPAP_ERR_HIP (recording). */
#define MPAP_PLAN_ANALYTIC 1
int mpap_plan_create(mpap_graph *g, const mpap_search_params *sp, int32_t n_params,
                     mpap_graph *const *parts, const mpap_surrogate *const *models,
                     int32_t nparts, int32_t flags, void *stream, mpap_plan **out);

/* mpap_plan_run - launch the recorded graph on `stream` and wait.  The result
 * holds the goal fronts, statistics and latencies like mpap_search_batch's;
 * its per-node fronts and plans (mpap_node_front, mpap_label_path,
 * mpap_rescore_front) read the plan's workspace and stay valid until the next
 * mpap_plan_run or mpap_plan_free of the same plan.  If the device reports a
 * capacity overflow the batch is searched again eagerly (growing the
 * workspace) and the graph recorded again; the result is the same.  Free the
 * result with mpap_result_free.  A plan is not safe to run from two threads at
 * once.  Errors: MPAP_ERR_HIP (also a grid-barrier timeout),
 * MPAP_ERR_NOCONVERGE, MPAP_ERR_OVERFLOW. */
int mpap_plan_run(mpap_plan *p, void *stream, mpap_result **out);

/* mpap_plan_info - launches so far, graph recordings (1 + re-recordings after
 * overflows) and eager fallbacks.  Outputs are nullable. */
int mpap_plan_info(const mpap_plan *p, int32_t *launches, int32_t *records, int32_t *fallbacks);

void mpap_plan_free(mpap_plan *p);

#ifdef __cplusplus
}
#endif

#endif /* MPAP_H */
