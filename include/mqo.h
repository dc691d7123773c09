/*
 * mqo.h -- C-ABI of libmqo, the MI355X (gfx950) implementation of the
 * data-parallel hot path of mutation-guided quadratic optimisation for
 * Maximum Independent Set and MaxCut (arXiv 2605.06921).
 *
 * Conventions (every entry point):
 *   - Array arguments are DEVICE pointers unless marked (host).  The caller
 *     allocates and owns every buffer; the library keeps no device memory
 *     between calls except its launch-plan and hipGraph caches, released by
 *     mqo_clear_caches().  Scratch memory is the caller's workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Every function returns an mqo_status; no C++ exception crosses the
 *     ABI.  On failure nothing was enqueued unless the status is
 *     MQO_ERR_HIP, and mqo_last_error() (thread-local) holds the detail.
 *   - Iterates are float32, vertex-major: X[v * B + b] is vertex v of
 *     trajectory b.  Binary solutions are int8 in the same layout: MIS z in
 *     {0,1}, MaxCut s in {-1,+1}.
 *   - Trajectory b of graph g has the id t = g * B + b; random draws are
 *     keyed by (seed, purpose, t, round, local vertex index), so results do
 *     not depend on the launch plan or on the graph's position in a batch.
 *   - Float32 steps follow one fixed operation order (per row, neighbours
 *     summed in ascending CSR order with one rounding per add, no fused
 *     multiply-add except -lambda - 2 * acc, whose product is exact so that
 *     one rounding gives the same result), so every launch plan gives
 *     bit-identical iterates.
 *   - The blocking entry points (the solves, mqo_local_search,
 *     mqo_pair_search, mqo_validate_graph) share the library's pinned read-back buffer and
 *     internal stream and run one at a time per process (an internal lock);
 *     the asynchronous ones may be called concurrently on different
 *     streams with different workspaces.
 */
#ifndef MQO_H
#define MQO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MQO_VERSION 110

typedef enum {
  MQO_OK = 0,
  MQO_ERR_INVALID_ARG = -1,   /* a parameter or pointer is out of range      */
  MQO_ERR_INVALID_GRAPH = -2, /* the CSR is not canonical (see mqo_graph)    */
  MQO_ERR_WORKSPACE = -3,     /* workspace NULL or smaller than required     */
  MQO_ERR_HIP = -4,           /* a HIP runtime call failed                   */
  MQO_ERR_UNSUPPORTED = -5,   /* valid request not offered for these arguments */
  MQO_ERR_INTERNAL = -6       /* an internal invariant failed                */
} mqo_status;

/* The relaxed objective that is ascended.
 * MQO_OBJ_MIS_H:     h(x) = 1^T x - (gamma/2) x^T A x on [0,1]^n, gamma > 1
 *                    (Sec. 3, Eq. (3)); grad = 1 - gamma A x.
 * MQO_OBJ_MAXCUT_FB: f_B(x) = -lambda 1^T x - x^T A x on [-1,1]^n,
 *                    0 < lambda < 2 (Sec. 3, Eq. (7), Thm. 3.6);
 *                    grad = -2 A x - lambda.  A_uv = w_uv when weighted. */
/* Relaxed objectives (Sec. 3): MIS h (Eq. (3), parameter gamma > 1);
 * MaxCut perturbed bias f_B (Eq. (7), lambda in (0,2), the formulation the
 * algorithms use), Laplacian f_L (Eq. (4), no parameter), perturbed
 * Laplacian f_P (Eq. (5), lambda > 0) and adjacency f_A (Eq. (6), no
 * parameter), all on the box [-1,1]^n.  The MaxCut formulations share
 * rounding, cut evaluation and local search; f_L, f_P and f_A run on the
 * batched and plain plans (not the persistent one) and without
 * check_every. */
typedef enum {
  MQO_OBJ_MIS_H = 0,
  MQO_OBJ_MAXCUT_FB = 1,
  MQO_OBJ_MAXCUT_FL = 2,
  MQO_OBJ_MAXCUT_FP = 3,
  MQO_OBJ_MAXCUT_FA = 4
} mqo_objective;

enum { MQO_INIT_UNIFORM = 0, MQO_INIT_DEGREE = 1 };
enum { MQO_RESET_ZERO = 0, MQO_RESET_FLIP = 1 };
enum { MQO_LS_NONE = 0, MQO_LS_ONE_FLIP = 1 };
/* search on the incumbents after the last round (mqo_params.final_search) */
enum { MQO_FINAL_NONE = 0, MQO_FINAL_PAIR = 1 };
enum { MQO_PLAN_AUTO = 0, MQO_PLAN_PLAIN = 1, MQO_PLAN_BATCHED = 2, MQO_PLAN_PERSISTENT = 3 };

/* Graph (notation of Sec. 2): one undirected graph, or G graphs as one
 * block-diagonal CSR with global column indices.  Canonical form: row_ptr
 * monotone with row_ptr[0] = 0 and row_ptr[n_total] = nnz_total; columns
 * strictly ascending inside a row; symmetric; no self loops; every column
 * inside its own graph's vertex range; weight (MaxCut only) symmetric. */
typedef struct {
  int32_t num_graphs;         /* G >= 1                                       */
  const int64_t *vtx_offset;  /* (host) [G+1], vtx_offset[0] = 0, increasing  */
  int64_t n_total;            /* = vtx_offset[G]                              */
  int64_t nnz_total;          /* stored entries = 2 |E|, < 2^31               */
  const int32_t *row_ptr;     /* [n_total + 1]                                */
  const int32_t *col_idx;     /* [nnz_total]                                  */
  const int32_t *weight;      /* [nnz_total] or NULL (unit weights)           */
  /* Optional list of high-degree rows ("hubs"); hub_offset = NULL for none.
   * The sparse-product kernels (PGA step, objective gradient, adjoint) give
   * every listed row column slices of their own workgroups instead of one
   * lane group, so that a row of very high degree (preferential-attachment
   * graphs) does not hold up a whole step.  Results are bit-identical with
   * and without the list.  hub_rows holds, graph after graph, the global
   * ids of EXACTLY the rows of degree > hub_min_degree, ascending;
   * hub_offset[i] .. hub_offset[i+1] delimits graph i's part.  The solves
   * check the list on the device (MQO_ERR_INVALID_GRAPH); the asynchronous
   * entry points trust it. */
  int32_t hub_min_degree;     /* >= 0                                         */
  const int64_t *hub_offset;  /* (host) [G+1], hub_offset[0] = 0, or NULL     */
  const int32_t *hub_rows;    /* [hub_offset[G]]                              */
  /* Optional hint: the largest row degree, or 0 if unknown.  It only picks
   * kernel shapes (near-regular graphs take rows in pairs); results do not
   * depend on it, and the solves measure the degree themselves. */
  int32_t max_degree;
  /* Optional hint: 1 when the neighbours of a row are mostly close to it in
   * the vertex order (grids, tori, banded orders: mean |u - v| over the
   * stored entries well below n_g / 8), 0 if not or unknown.  With 1 the
   * sparse-product kernels hand each XCD one contiguous range of rows, so
   * that rows sharing neighbours share an L2; with 0 rows are spread over
   * the XCDs, which balances graphs whose heavy rows are clustered in the
   * vertex order (preferential attachment).  Results do not depend on it. */
  int32_t local_rows;
} mqo_graph;

/* Search parameters.  Fill with mqo_params_default() first. */
typedef struct {
  uint32_t struct_size;    /* sizeof(mqo_params)                                */
  int32_t batch;           /* B >= 1 trajectories per graph                     */
  int32_t steps_per_round; /* PGA steps per round, >= 0                         */
  int32_t rounds;          /* >= 1; round 0 starts from x0, later rounds from
                              the incumbent after the reset of Sec. 4         */
  int32_t check_every;     /* 0 = off; c > 0: after every c PGA steps of a
                              round (before its end) a trajectory whose rounded
                              point is a fixed point of the projected step
                              (the checker of Eq. (8) for MIS, s_v t_v < 0 or
                              s_v t_v = 0 with s_v = -1 for f_B) stops
                              stepping for the rest of the round; edge_updates
                              then counts the steps actually executed       */
  float alpha;             /* step size, > 0                                    */
  float momentum;          /* heavy-ball coefficient in [0, 1); 0 = plain PGA   */
  float gamma;             /* MIS edge penalty, > 1                             */
  float lambda;            /* MaxCut bias, in (0, 2)                            */
  double rho;              /* reset fraction in [0, 1); |R| = floor(rho * n_g)  */
  float init_sigma;        /* noise of the degree-based initialisation, >= 0    */
  int32_t init_mode;       /* MQO_INIT_*                                        */
  int32_t reset_mode;      /* MQO_RESET_*                                       */
  int32_t local_search;    /* MQO_LS_*                                          */
  int32_t plan;            /* MQO_PLAN_*                                        */
  int32_t tile_cols;       /* persistent plan: trajectories per workgroup, a
                              power of two <= 64, or 0 = autotune             */
  int32_t tile_threads;    /* persistent plan: 256, 512 or 1024, 0 = autotune   */
  int32_t tile_vec;        /* persistent plan: trajectories per lane in the
                              step loop, 1, 2 or 4, 0 = autotune             */
  int32_t tile_csr;        /* persistent plan: 1 = column indices from global
                              memory, 2 = staged in LDS, 0 = autotune        */
  int32_t tile_reg;        /* persistent plan, unweighted graphs of degree
                              <= 16: 2 = neighbour offsets in registers,
                              1 = never, 0 = autotune                        */
  uint64_t seed;
  double time_budget_s;    /* 0 = none; otherwise no round r > 0 starts after
                              it (round 0 of every trajectory always runs, so
                              every incumbent is written); the pass it cuts
                              short still ends with the final_search.  The
                              clock starts at the first round, after any
                              autotuning or plan trial (MQO_PLAN_AUTO)       */
  int32_t maxcut_objective; /* mqo_solve_maxcut: MQO_OBJ_MAXCUT_FB (default),
                              _FL, _FP or _FA                                  */
  int32_t final_search;    /* MQO_FINAL_NONE (default) or MQO_FINAL_PAIR: the
                              paper's own search closes every pass of the
                              outer loop (Alg. 1 / Alg. 2; a pass ends after
                              every restart_every-th round and after the last
                              round): every incumbent goes through
                              mqo_pair_search (round index = rounds + the
                              pass number) and is replaced when strictly
                              better, so the next pass resets from the
                              searched sets.  With pool_k see there        */
  int32_t pool_k;          /* 0 = independent trajectories (default); K in
                              [1, min(64, batch)]: the pmQO pool of Alg. 3 /
                              Alg. 4 -- after every round the K best distinct
                              solutions of the pool and the round's
                              candidates (MIS: independent sets only) form the
                              pool, ranked by value, ties to the earlier
                              (pool slots, then trajectories); duplicates are
                              recognised by value and a 64-bit SplitMix64 sum
                              hash of the set; round r > 0 restarts
                              trajectory t from slot (u K') >> 32 of the pool
                              (K' filled slots, u the Philox draw (seed, 8)
                              for counter (0, t, r, 0)).  Each graph keeps
                              its best set (I_sol / S_sol), replaced by the
                              pool's best member after every round when that
                              is strictly better; it is the answer.  With
                              final_search the pool is left alone and each
                              pass ends with the search of I_sol alone (MIS,
                              Alg. 3, trajectory id g K) or of every pool
                              member (MaxCut, Alg. 4, trajectory ids g K +
                              slot, offered to S_sol in slot order and each
                              taken when strictly better).
                              Batched and persistent plans (the persistent
                              plan launches each round on its own, the pool
                              updated between launches); the plain plan
                              returns MQO_ERR_UNSUPPORTED                   */
  int32_t restart_every;   /* 0 = off (default); R > 0: the outer loop of
                              Alg. 1-4 -- every round r > 0 with r % R == 0
                              starts from a fresh point of the initialisation
                              rule (Philox round field = r / R) instead of a
                              reset; incumbents and the pool carry over     */
  int32_t traj_count;      /* plain plan: 0 = every trajectory (default);
                              c > 0: only the c trajectories traj_ids[0..c)
                              run (ids t = g B + b, strictly ascending, each
                              < G B), each exactly as in a full solve (the
                              trajectories are independent chains); the
                              others keep traj_best_value INT64_MIN and
                              traj_best_x zeros.  Other plans:
                              MQO_ERR_UNSUPPORTED                          */
  const int64_t *traj_ids; /* (host) [traj_count], read during the call     */
  int32_t step_vec;        /* streaming step kernel (batched plan): columns per
                              lane, 1, 2 or 4, 0 = autotune                 */
  int32_t step_lanes;      /* streaming step kernel: lanes per row, a power of
                              two <= 64, 0 = autotune (every shape computes
                              the same sums in the same order)              */
  int32_t tile_sb;         /* persistent plan: 1 = two iterate buffers in LDS
                              (a step reads one, writes the other), 2 = one
                              buffer (a step gathers into registers, then
                              writes in place: twice the trajectories per
                              workgroup fit), 0 = autotune                  */
} mqo_params;

/* Outputs of a solve.  Device arrays are written; host fields are set. */
typedef struct {
  int8_t *best_x;              /* [n_total]: answer of each graph             */
  int64_t *best_value;         /* [G]: MIS size / cut weight (-1 = none)       */
  int64_t *traj_best_value;    /* [G*B] incumbent values, or NULL             */
  int8_t *traj_best_x;         /* [n_total*B] incumbents, or NULL             */
  int64_t edge_updates;        /* (host) sum over trajectories of the steps
                                  each executed x nnz of its graph            */
  int64_t steps_executed;      /* (host) PGA steps per trajectory              */
  int32_t rounds_executed;     /* (host)                                       */
  int32_t plan_used;           /* (host) MQO_PLAN_PLAIN/BATCHED/PERSISTENT     */
  int32_t tile_cols_used;      /* (host) persistent plan choice, else 0        */
  int32_t tile_threads_used;   /* (host)                                       */
  int32_t tile_vec_used;       /* (host) trajectories per lane in the steps    */
  int32_t tile_csr_lds_used;   /* (host) 1 = column indices staged in LDS      */
  int32_t tile_reg_degree_used;/* (host) padded degree of the register
                                  adjacency, 0 = not used                    */
  int64_t ls_iterations;       /* (host) local-search iterations summed over
                                  rounds (per round: the largest count of any
                                  graph / trajectory tile)                   */
  double step_kernel_ms;       /* (host) HIP-event time of the launches that
                                  run the PGA steps (persistent plan: the
                                  whole-round tile kernel), on the stream
                                  they run on                               */
  int64_t step_kernel_launches;/* (host) number of such launches            */
  int64_t final_search_alternations; /* (host) final_search: pair iterations
                                  that applied a move, summed over the
                                  searches that closed the passes           */
  int8_t *pool_x;              /* [n_total*K] pool solutions (pool_k > 0), or
                                  NULL; empty slots are zeros               */
  int64_t *pool_value;         /* [G*K] pool values, INT64_MIN = empty slot,
                                  or NULL                                   */
  int32_t step_vec_used;       /* (host) streaming plans: columns per lane of
                                  the step kernel (0 on the persistent plan) */
  int32_t step_lanes_used;     /* (host) streaming plans: lanes per row       */
  int32_t tile_single_buffer_used; /* (host) persistent plan: 1 = one iterate
                                  buffer in LDS                              */
} mqo_result;

void mqo_params_default(mqo_params *p);

/* Bytes of workspace a solve needs (0 on invalid input).  The same size
 * covers every plan. */
size_t mqo_workspace_size(const mqo_graph *g, const mqo_params *p, mqo_objective obj);

/* Batched mutation-guided search (Alg. 1 for MIS, Alg. 2 for MaxCut, run as
 * B independent trajectories per graph, the batch form of Alg. 3 / 4).
 * Round r of trajectory t: r = 0 starts from x0 (or the init rule), r > 0
 * from the incumbent with floor(rho n) uniformly chosen coordinates set to 0
 * (Sec. 4); then steps_per_round PGA steps x <- Pi(x + alpha grad);
 * threshold rounding (x > 0.5 / x > 0, Sec. 3); optional 1-flip local
 * search; exact int64 evaluation (MIS size if independent else -1; cut
 * weight); the incumbent is replaced only on strict improvement (Sec. 4).
 * x0: [n_total*B] start iterate or NULL.  Blocks until done; validates the
 * graph on the device first.  ws must hold mqo_workspace_size() bytes. */
int mqo_solve_mis(const mqo_graph *g, const mqo_params *p, const float *x0,
                  mqo_result *r, void *ws, size_t ws_bytes, void *stream);
int mqo_solve_maxcut(const mqo_graph *g, const mqo_params *p, const float *x0,
                     mqo_result *r, void *ws, size_t ws_bytes, void *stream);

/* Objective and gradient (Eq. (3) / Eq. (7)) of B iterates per graph:
 * f_out[g*B+b] = c^T x + (1/2) x^T H x accumulated in float64 (H = -gamma A,
 * c = 1 for MIS; H = -2A, c = -lambda for MaxCut), and
 * grad_out = scale_b * (c + H x) in float32 (the SpMM gradient).  Either
 * output may be NULL.  scale: [G*B] or NULL (= 1).  Asynchronous on
 * `stream`; the graph is assumed canonical (see mqo_validate_graph).
 * ws: mqo_objective_workspace_size() bytes (may be NULL when f_out is). */
size_t mqo_objective_workspace_size(const mqo_graph *g, int32_t B);
int mqo_objective_grad(const mqo_graph *g, mqo_objective obj, float param,
                       const float *X, int32_t B, const float *scale,
                       double *f_out, float *grad_out,
                       void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as mqo_objective_grad, with the float64 partial sums of f_out in the
 * library's own device scratch of MQO_STATIC_SCRATCH_BYTES bytes instead of
 * a caller workspace.  Allocates nothing, neither on the device nor pinned.
 * When f_out is requested and mqo_objective_workspace_size(g, B) exceeds
 * MQO_STATIC_SCRATCH_BYTES it returns MQO_ERR_WORKSPACE before anything is
 * enqueued.  Each GPU holds one copy of the scratch until the process ends
 * and every call on that GPU uses it: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be
 * serialised by the caller; calls in one stream order are safe.  The
 * partial sums are written whole by every call, nothing is carried over. */
#define MQO_STATIC_SCRATCH_BYTES (16u << 20)
int mqo_objective_grad_static(const mqo_graph *g, mqo_objective obj, float param,
                              const float *X, int32_t B, const float *scale,
                              double *f_out, float *grad_out, void *stream);

/* K unrolled PGA steps x_{k+1} = Pi(x_k + alpha grad(x_k)) (momentum 0).
 * Forward stores x_{j*ckpt_every} in ckpt[j] ([K/ckpt_every][n_total*B])
 * and x_K in XK.  K must be a multiple of ckpt_every.  Backward takes
 * dL/dx_K and returns dL/dx_0 and dL/dalpha per trajectory ([G*B], float64),
 * recomputing each segment from its checkpoint.  Clip derivative: 1 iff
 * lo <= x + alpha grad <= hi.  Asynchronous on `stream`; ws holds
 * mqo_unrolled_workspace_size() bytes. */
size_t mqo_unrolled_workspace_size(const mqo_graph *g, int32_t B, int32_t ckpt_every);
int mqo_pga_unrolled_forward(const mqo_graph *g, mqo_objective obj, float param, float alpha,
                             int32_t K, int32_t ckpt_every, const float *X0, float *ckpt,
                             float *XK, int32_t B, void *ws, size_t ws_bytes, void *stream);
/* dL_dalpha_sum (device, or NULL): the sum of dL_dalpha over all G*B
 * trajectories (one float64, summed in a fixed order), the derivative of
 * the loss with respect to a step size shared by every trajectory. */
int mqo_pga_unrolled_backward(const mqo_graph *g, mqo_objective obj, float param, float alpha,
                              int32_t K, int32_t ckpt_every, const float *ckpt,
                              const float *dL_dXK, float *dL_dX0, double *dL_dalpha,
                              double *dL_dalpha_sum, int32_t B, void *ws, size_t ws_bytes,
                              void *stream);

/* ---- building blocks of one round (asynchronous, stream-ordered) ---- */

/* x0 by the initialisation rule: MQO_INIT_UNIFORM draws u ~ U[0,1) with 24
 * random bits (MIS x = u; MaxCut x = 2u - 1); MQO_INIT_DEGREE is
 * Pi(d_base + N(0, sigma^2)) of Alg. 1 / Alg. 2.  Uses p->batch, seed,
 * init_mode, init_sigma.  ws: caller-owned device scratch of at least
 * MQO_INIT_WORKSPACE_BYTES bytes for MQO_INIT_DEGREE (the graphs' largest
 * degrees are measured into it), NULL allowed for MQO_INIT_UNIFORM; calls on
 * different streams need different ws. */
#define MQO_INIT_WORKSPACE_BYTES 256
int mqo_init_iterate(const mqo_graph *g, mqo_objective obj, const mqo_params *p,
                     float *X, void *ws, size_t ws_bytes, void *stream);

/* `nsteps` PGA steps in place on X (and V, the momentum, when
 * p->momentum != 0; V may be NULL otherwise).  Uses p->batch, alpha,
 * momentum, gamma / lambda.  tmp: [n_total*B] float scratch. */
int mqo_pga_steps(const mqo_graph *g, mqo_objective obj, const mqo_params *p,
                  float *X, float *V, float *tmp, int32_t nsteps, void *stream);

/* The building blocks below take the workspace of a solve with the same
 * graph and batch (mqo_workspace_size). */

/* Threshold rounding and exact evaluation of X ([n_total*B]):
 * Z = rounding (int8), value[G*B] as in mqo_solve_*, and for MIS
 * conflicts[G*B] (edges inside I, or NULL) and fixed[G*B] (int8, the
 * checker of Eq. (8): 1 iff I is a maximal independent set; or NULL). */
int mqo_round_evaluate(const mqo_graph *g, mqo_objective obj, const float *X, int32_t B,
                       int8_t *Z, int64_t *value, int64_t *conflicts, int8_t *fixed,
                       void *ws, size_t ws_bytes, void *stream);

/* 1-flip local search in place on Z (parallel independent-set rule: every
 * iteration flips the positive-gain vertices whose key (gain, Philox
 * priority, -v) beats all positive-gain neighbours; stops when no gain is
 * positive).  `round` keys the priorities.  iterations: (host) out or NULL.
 * Blocks (the stopping test reads a device flag). */
int mqo_local_search(const mqo_graph *g, mqo_objective obj, int32_t B, uint64_t seed,
                     int32_t round, int8_t *Z, int64_t *iterations,
                     void *ws, size_t ws_bytes, void *stream);

/* The paper's own local search in place on Z: OneTwoSwap for MIS (the
 * (1,2)-swap of Def. 2.3) and OneTwoFlip for MaxCut (the 2-flip of
 * Def. 2.5 with the 1-flip of Def. 2.4), as described in Sec. 4, in a
 * parallel form: the 1-flip search of mqo_local_search (same seed and
 * round), then pair iterations, each followed by the 1-flip search again,
 * until an iteration applies no move.  A pair iteration applies a set of
 * moves whose gains add: MIS -- every v in I proposes the first pair (u, w)
 * of its neighbours in CSR order whose only neighbour in I is v and that
 * are not adjacent; a proposal is applied when its key (Philox priority of
 * purpose SWAP for (t, round, v), -v) beats every proposal that inserts a
 * neighbour of u or w.  MaxCut -- every v picks the cut edge (v, u) of
 * largest pair key (gain g_v + g_u + 2 w_vu > 0 with g = s (A s), then
 * (prio_v + prio_u) mod 2^32, then the smaller vertex pair); a mutual pair
 * is applied when no other vertex adjacent to it holds a larger key.
 * Z ([n_total*B]) may be any binary point (MIS: the 1-flip stage repairs
 * conflicts first).  Every graph of the batch is searched at once.  MIS
 * graphs carry no weights; MaxCut weights enter the gains.
 * alternations: (host) out or NULL, the pair iterations that applied a move
 * (the search runs one more, which finds none).  candidate_kernel_ms: (host)
 * out or NULL, HIP-event time on `stream` of the candidate launches of every
 * pair iteration (MIS: owner clear + proposals; MaxCut: best pair per
 * vertex), summed.  Blocks (the stopping tests read device flags).
 * ws: mqo_workspace_size() bytes for this graph and B. */
int mqo_pair_search(const mqo_graph *g, mqo_objective obj, int32_t B, uint64_t seed,
                    int32_t round, int8_t *Z, int64_t *alternations,
                    double *candidate_kernel_ms, void *ws, size_t ws_bytes, void *stream);

/* Mutation reset (Sec. 4): X = Zbest as float, then in every trajectory the
 * k = floor(rho n_g) vertices with the smallest (key, v) are set to 0
 * (MQO_RESET_ZERO) or to the complement (MQO_RESET_FLIP).  key = Philox
 * draw (seed, round) or, when keys != NULL, keys[v*B+b] (uint32). */
int mqo_reset(const mqo_graph *g, mqo_objective obj, int32_t B, uint64_t seed, int32_t round,
              double rho, int32_t mode, const int8_t *Zbest, const uint32_t *keys,
              float *X, void *ws, size_t ws_bytes, void *stream);

/* ---- Prop. 4.1's separable toy ---- */

enum { MQO_TOY_GLOBAL_RESET = 0, MQO_TOY_FULL_RESTART = 1 };

/* Independent trials of the analysis of Prop. 4.1 (Sec. 4): minimise
 * F(x) = sum_i phi(x_i) on [-1,1]^n, phi(x) = -x^2/2 - beta x^3/3, whose
 * projected descent x <- Pi(x + alpha (x + beta x^2)) (`steps` float32 steps,
 * no fused operations) sends (0,1] to 1 and [-1,0) to -1; x* = (1,...,1).
 * Value draws: Philox4x64-10, y = (2 (w >> 8) + 1 - 2^24) / 2^24.
 * MQO_TOY_GLOBAL_RESET: the start is restart 0 descended; then `attempts`
 * times one coordinate i = (w0 n) >> 32 is reset to a drawn y, descended,
 * and kept iff phi (float64) strictly decreases; first_hit[t] = the number
 * of attempts after which the point first equals x* (0 = at the start), else
 * -1; x_out ([trials][n], or NULL) = the final points.
 * MQO_TOY_FULL_RESTART: restarts j = 0 .. attempts draw and descend a whole
 * point; first_hit[t] = the first j that gives x*, else -1 (x_out unused).
 * Keys: (seed, 6) for resets with counter (0, t, attempt, 0) lanes 0-1, and
 * (seed, 7) for restart j with counter (v >> 3, t, j, 0) lane v & 7.
 * 1 <= n <= 64, 0 < beta < 1, alpha > 0, steps, attempts >= 0, trials >= 0.
 * Asynchronous on `stream`. */
int mqo_toy_reset(uint64_t seed, int32_t n, float alpha, float beta, int32_t steps,
                  int32_t attempts, int32_t trials, int32_t mode, int32_t *first_hit,
                  float *x_out, void *stream);

/* ---- validation and misc ---- */

/* Canonical-form check of a host CSR (no GPU needed). */
int mqo_validate_graph_host(int64_t n, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col_idx, const int32_t *weight);
/* The same check on the device arrays of g; blocks. */
int mqo_validate_graph(const mqo_graph *g, void *stream);

const char *mqo_status_string(int status);
const char *mqo_last_error(void);
int mqo_version(void);
/* Forgets every autotuner choice held in memory (the file is not touched). */
void mqo_clear_caches(void);

/* The autotuner (the batch form of the step-size / batch choice of Alg. 3:
 * the persistent plan's tile shape, the streaming step kernel's columns per
 * lane and lanes per row, and the plan chosen for MQO_PLAN_AUTO) times the
 * candidate launch shapes of a shape key once and keeps the fastest.  Keys
 * hold the kind of choice, the GPU (architecture and compute units), the
 * problem and objective, the graph size range, its mean degree and the
 * batch.  Choices never change results, only speed.  The cache lives in
 * memory; with MQO_TUNE_CACHE=<path> in the environment the file's entries
 * are read at the first use and every new choice is appended to it.  The
 * file is text, one "key<TAB>value" per line ('#' lines are comments).
 * Host only: no GPU is needed for these three calls.
 * load: merges the file's entries (MQO_ERR_INVALID_ARG and nothing merged on
 * a malformed line or an unreadable file); save: writes every entry;
 * size: the number of entries held. */
int mqo_tune_cache_load(const char *path);
int mqo_tune_cache_save(const char *path);
int64_t mqo_tune_cache_size(void);

#ifdef __cplusplus
}
#endif
#endif /* MQO_H */
