/*
 * lge.h — C ABI of the MI355X edge-centric graphlet estimator.
 *
 * The library computes, for an undirected simple graph G=(V,E), a sampling
 * probability p and a seed, the localized graphlet estimates of "Estimation
 * of Graphlet Statistics" (Rossi, Zhou, Ahmed): every edge is sampled
 * independently with probability p (Alg. 1 with a Bernoulli design, Sec. 2.4),
 * each sampled edge is counted locally (Alg. 2: triangles and 2-stars by
 * neighbourhood intersection; Alg. 3/5: 4-cliques; Alg. 4/6: 4-cycles), the
 * unrestricted counts (eqs. non-induced-conn-n1..n4, non-induced-disconn-n1..n4)
 * are summed exactly, and the estimates of all 2-, 3- and 4-vertex graphlets
 * G1..G17 (Table 1) follow from the X equations (eq. graphlet-X-start ..
 * graphlet-X-end) with sigma = 1/p, together with an unbiased variance
 * estimate and 95% bounds (eq. bounds-95).
 *
 * Conventions
 *  - Graphs are int32 CSR: row_ptr[n+1] (row_ptr[0] = 0, non-decreasing),
 *    col[row_ptr[n]]; each undirected edge is stored in both rows; rows are
 *    strictly increasing (sorted, no duplicates); no self-loops.
 *  - Canonical edge id: rank of (u, v), u < v, in row-major order of the
 *    sorted CSR (0-based).  Edge e is sampled iff the Philox4x32-10 block of
 *    key (seed lo32, seed hi32) and counter (e lo32, e hi32, 0, 0), reduced to
 *    u = ((x1 << 32 | x0) >> 11) * 2^-53, satisfies u < p.
 *  - All counts are exact integers.  Sums that can exceed 64 bits are
 *    returned as 128-bit two's complement values split into (lo, hi) limbs.
 *    Floating point (double) is used only for the sampling compare and the
 *    final scaling, variance and bounds.
 *  - Arrays indexed by graphlet number have 18 slots; slot i holds G_i
 *    (slot 0 unused).
 *  - Every call returns LGE_OK (0) or a negative LGE_E* code; no exception
 *    crosses the ABI.  lge_strerror() names a code.
 *  - One lge_ctx drives one GPU through one HIP stream.  Calls on one ctx must
 *    not overlap (use one ctx per host thread); the server API below is the
 *    thread-safe way to share a GPU.
 */
#ifndef LGE_H
#define LGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define LGE_API __attribute__((visibility("default")))
#else
#define LGE_API
#endif

#define LGE_OK 0
#define LGE_EINVAL (-1)     /* bad argument (p outside (0,1], null pointer, bad size) */
#define LGE_ENOMEM (-2)     /* device or host allocation failed */
#define LGE_EGRAPH (-3)     /* CSR is not a sorted, symmetric, loop-free simple graph */
#define LGE_EDEVICE (-4)    /* HIP runtime error or no usable GPU */
#define LGE_ERANGE (-5)     /* sizes beyond the exact 128-bit range (see lge_graph_create_*) */
#define LGE_EBUSY (-6)      /* server admission queue full */
#define LGE_ETIMEDOUT (-7)  /* lge_wait timed out (the ticket stays valid) */
#define LGE_ECANCELED (-8)  /* request cancelled or server shut down */
#define LGE_ENOTFOUND (-9)  /* unknown ticket or graph id */
#define LGE_EINTERNAL (-10) /* a device-side consistency check failed (a library bug) */

/* lge_graph_create_* flag: skip validation of the CSR (caller guarantees it) */
#define LGE_FLAG_TRUSTED 1u
/* lge_graph_create_* flag: keep the per-graph co-degree rows of the hubs
 * and the co-degree table small (at most 4 GB and 1 GiB, and smaller
 * build-work budgets) instead of up to 32 GB and 32 GiB; for callers holding
 * many large graphs at once.  Results do not change, only the speed on
 * graphs with many vertices of high degree. */
#define LGE_FLAG_COMPACT 2u
/* lge_graph_create_* flag: build no co-degree table, bit rows or co-degree
 * rows (hub tables only): the smallest state and the shortest build, every
 * neighbour walked or looked up.  Results do not change, only the speed. */
#define LGE_FLAG_NO_TABLES 4u

typedef struct lge_ctx lge_ctx;
typedef struct lge_graph lge_graph;
typedef struct lge_event lge_event;
typedef struct lge_server lge_server;

typedef struct {
  uint64_t lo, hi;
} lge_u128;

/*
 * Result of one estimate (caller-owned).  Indices follow G1..G17.
 *  csum[i]   C_i = sum over sampled edges of the unrestricted count of G_i,
 *            for i in {3,4,5,7,...,16} (others 0).  Per edge, with
 *            t = |T_e|, s_u, s_v the 2-star sets, r = n - |Gamma(u) u Gamma(v)|,
 *            f = m - d_u - d_v + 1:
 *              C3 += t, C4 += s_u+s_v, C5 += r, C7 += edges inside T_e,
 *              C8 += t(t-1)/2, C9 += t(s_u+s_v), C10 += edges between S_u and S_v,
 *              C11 += C(s_u,2)+C(s_v,2), C12 += s_u s_v, C13 += t r,
 *              C14 += (s_u+s_v) r, C15 += f, C16 += r(r-1)/2.
 *  z[i]      Z_i = sum over sampled edges of 12*Y_i(e), where Y_i(e) is edge e's
 *            term of the X equations with sigma = 1 (signed), i = 3..17.
 *  q[i]      Q_i = sum over sampled edges of (12*Y_i(e))^2, i = 3..17.
 *  exact[i]  exact count of G_i; valid when every edge is sampled (p == 1),
 *            exact[1] = m and exact[2] = C(n,2) - m always.
 *  estimate  X_i = K_i + (Z_i * (1/p)) / 12 with K_6 = C(n,3), K_17 = C(n,4),
 *            else 0; X_1 = m, X_2 = C(n,2) - m; at p == 1, X_i = exact[i].
 *  variance  V_i = Q_i * ((1-p)/p^2) / 144 (0 for i = 1, 2 and at p == 1).
 *  lower95/upper95  X_i -/+ 1.96 sqrt(V_i).
 */
typedef struct {
  int64_t n, m;
  double p;
  uint64_t seed;
  uint64_t sampled_edges;
  lge_u128 csum[18];
  lge_u128 z[18];
  lge_u128 q[18];
  lge_u128 exact[18];
  double estimate[18];
  double variance[18];
  double lower95[18];
  double upper95[18];
} lge_result;

/*
 * Tunables.  Results never depend on them (exact integer sums are
 * order-independent); only the speed does.  Zero-initialise and call
 * lge_opts_default(), or pass NULL for defaults.
 *  wave_max_deg   edges whose endpoints both have degree <= this are counted
 *                 by one wavefront with LDS tables (1..512, default 256)
 *  block_max_deg  edges outside the wavefront class whose endpoints both
 *                 have degree <= this (1..1024, default 1024) are counted by
 *                 one 256-thread workgroup with LDS tables;
 *                 others are split across workgroups and use the per-vertex
 *                 global hash tables kept for every vertex of degree > 32
 *  probe_ratio    per neighbour w, look the target set up inside Gamma(w)
 *                 (binary search or w's table) instead of scanning Gamma(w)
 *                 when |target| * lookup_cost(d_w) * probe_ratio < d_w
 *                 (0 disables lookups; default 4)
 *  grid_per_cu    persistent workgroups per compute unit for each counting
 *                 kernel (0 = library default)
 *  global_chunk   Gamma(a) positions per work item of the split class
 *                 (1..1024, default 1024)
 *  flags          LGE_OPT_SORT_HUB: order split-class edges by their
 *                 table-side endpoint so consecutive work items share its
 *                 hub table; LGE_OPT_XCD_LOCAL: each XCD (workgroups
 *                 blockIdx % 8) takes work items from its own contiguous
 *                 segment first, so each L2 sees a fraction of the tables
 *                 (default: both)
 *  max_list_mib   bound, in MiB, on the split-class work lists (work items
 *                 and T_e entries) one launch sequence may hold (0 = a
 *                 quarter of the device's memory).  A sequence whose lists
 *                 would need more runs its edge-id range in consecutive
 *                 pieces, each within the bound (a single edge may exceed
 *                 it); the exact sums, so the results, are the same.
 *  grid_share     percent (1..100, 0 = 100) of the default persistent grid
 *                 of each counting kernel: a sequence that runs beside
 *                 others (the serving lanes) leaves workgroup slots free.
 */
#define LGE_OPT_SORT_HUB 1u
#define LGE_OPT_XCD_LOCAL 2u
typedef struct {
  int32_t wave_max_deg;
  int32_t block_max_deg;
  int32_t probe_ratio;
  int32_t grid_per_cu;
  int32_t global_chunk;
  uint32_t flags;
  int32_t max_list_mib;
  int32_t grid_share;
} lge_opts;

/* Device-time breakdown of the last estimate/batch call on a ctx. */
typedef struct {
  float total_ms;          /* first kernel start to last kernel end */
  float sample_ms;         /* sampling + binning kernel */
  float count_ms[3];       /* counting kernels: wavefront, workgroup and split global classes
                              (count_ms[2] is k_count_global alone; the fold of
                              edges counted by several work items that follows
                              it is in total_ms only) */
  float global_prep_ms;    /* global class set-up: work items, T_e lists */
  uint64_t class_edges[3]; /* sampled edges per class */
  uint64_t words_read[3];  /* 4-byte words each class's counting kernels read (algorithmic) */
  uint64_t launches;       /* kernel launches issued */
  float micro_ms;          /* lge_micro only: the row kernel (after the counting pass) */
  uint32_t host_waits;     /* host waits on the device: 1, or 2 when the split-class work lists outgrew
                              the context's buffers (which then grow for later calls) */
  uint64_t alg_bytes[3];   /* per class: bytes the neighbour iteration of Alg. 2-4 would read for the
                              sampled edges, 16 + 4(d_u + d_v) + sum over w in Gamma(a)\{b} of (8 + 4 d_w) */
} lge_timing;

LGE_API const char *lge_strerror(int code);

/* Fills *o with the library defaults. */
LGE_API int lge_opts_default(lge_opts *o);

/* Opens device `device` (HIP ordinal); *out owns a stream and workspaces.
 * LGE_EDEVICE when no such GPU; LGE_ENOMEM on allocation failure. */
LGE_API int lge_open(int device, lge_ctx **out);
LGE_API int lge_close(lge_ctx *ctx);

/*
 * Host-side CSR check (no GPU needed): sizes, sorted strictly increasing
 * rows, ids in [0,n), no self-loops, symmetry.  LGE_OK or LGE_EGRAPH
 * (LGE_EINVAL for null pointers or negative n).
 */
LGE_API int lge_validate_csr_host(int64_t n, const int32_t *row_ptr, const int32_t *col);

/*
 * Graph from host arrays (copied into HBM; the caller keeps its arrays).
 * Validates on the GPU unless LGE_FLAG_TRUSTED.  Preprocesses once: the
 * canonical edge list and per-vertex 2-hop volumes used for scheduling, hash
 * tables of the vertices of degree > 32, the co-degree table and adjacency
 * bit rows of the vertices of degree > 96 (the highest-degree 131,008 of
 * them at most, in 2-byte entries: at most 32 GiB of table and 64 times the
 * graph's CSR bytes; 1 GiB with LGE_FLAG_COMPACT; lge_set_table_budget caps
 * both), and co-degree rows (one byte per entry, two when an unranked
 * degree exceeds 254) |Gamma(y) n Gamma(w)| over the unranked w above a
 * small degree floor for the highest-degree ranked vertices y, within a
 * build-work budget and up to 32 GB of HBM and 256 times the CSR bytes (4 GB
 * with LGE_FLAG_COMPACT).  The budgets depend on the graph and the caller,
 * never on what else is resident.
 * LGE_ERANGE if n >= 2^29 or a per-edge numerator could leave int64 or a sum
 * of squares 128 bits (bound: 16 * max(C(n,2), 2 dmax n, 4 dmax^2, m)).
 */
LGE_API int lge_graph_create_host(lge_ctx *ctx, int64_t n, const int32_t *row_ptr, const int32_t *col,
                          uint32_t flags, lge_graph **out);

/*
 * Graph adopting device buffers (zero copy, e.g. PyTorch tensors on the
 * ctx's device).  The caller keeps them alive and unchanged until
 * lge_graph_destroy.  hip_stream (may be NULL) is waited on before the
 * buffers are read.  Same validation and errors as the host variant.
 */
LGE_API int lge_graph_create_device(lge_ctx *ctx, int64_t n, const int32_t *d_row_ptr, const int32_t *d_col,
                            void *hip_stream, uint32_t flags, lge_graph **out);
LGE_API int lge_graph_destroy(lge_graph *g);

/* Number of vertices / undirected edges of a graph (host-side, no GPU call). */
LGE_API int64_t lge_graph_n(const lge_graph *g);
LGE_API int64_t lge_graph_m(const lge_graph *g);

/*
 * What a resident graph holds (host-side, no GPU call): sizes, the ranked
 * vertices of the co-degree table, the co-degree rows, their column floor
 * (unranked vertices above this degree have a column) and entry width, the
 * device bytes the library holds for the graph (including state built on
 * first use by lge_micro / lge_estimate_weighted, excluding adopted device
 * buffers), and the preprocessing wall time at creation.
 */
typedef struct {
  int64_t n, m;
  int32_t max_deg;
  int32_t ranked;
  int32_t rows;
  int32_t rows_floor;
  int32_t rows_width;
  int32_t pad;
  uint64_t state_bytes;
  double build_ms;
} lge_graph_info;
LGE_API int lge_graph_query(const lge_graph *g, lge_graph_info *out);

/* Estimate (synchronous on the ctx stream).  p in (0,1] else LGE_EINVAL;
 * opts may be NULL; out caller-owned. */
LGE_API int lge_estimate(lge_ctx *ctx, const lge_graph *g, double p, uint64_t seed, const lge_opts *opts,
                 lge_result *out);

/*
 * lge_estimate without any allocation, for callers that cannot allocate
 * device or pinned memory during the call: code under HIP graph capture,
 * tight serving loops, hosts that forbid hipMalloc.  Same arguments and
 * result as lge_estimate with default options (bit-identical integers and
 * FP64 values); the call itself makes no hipMalloc, hipHostMalloc or hipFree.
 * Its workspace is a fixed array of 128 MiB in device memory that every GPU
 * the library runs on holds from lge_open until the process ends, laid out
 * for graphs of at most 262,144 edges (2^18), 16,384 split-class work items
 * and 2,097,152 split-class T_e entries; calls on one GPU share it and are
 * serialised inside the process (each keeps the array until it returns; the
 * array keeps the last call's contents, and the call clears what it needs).
 * Errors: LGE_EINVAL as lge_estimate; LGE_ERANGE when m exceeds 2^18, or when
 * the sampled split-class work (edges with an endpoint of degree > 1024)
 * needs more work items or T_e entries than the layout holds (lge_estimate
 * then serves); LGE_EDEVICE.
 */
LGE_API int lge_estimate_noalloc(lge_ctx *ctx, const lge_graph *g, double p, uint64_t seed, lge_result *out);

/*
 * Estimate restricted to the canonical edge ids [e0, e1): edges outside the
 * range are never sampled; scaling still uses 1/p.  Sums over a partition of
 * [0, m) into ranges add up to the full estimate's integers, which is how
 * the work shards (Sec. 5: edge neighbourhoods are independent tasks).
 * 0 <= e0 <= e1 <= m else LGE_EINVAL.
 */
LGE_API int lge_estimate_range(lge_ctx *ctx, const lge_graph *g, double p, uint64_t seed, int64_t e0, int64_t e1,
                               const lge_opts *opts, lge_result *out);

/*
 * Asynchronous estimate: returns at once; the launch sequence runs after the
 * work already queued on hip_stream (NULL = none), driven by a worker thread
 * of the library, and `out` is filled before lge_event_wait returns.  `out`
 * must stay valid and the ctx must not be used for another call until then.
 * lge_event_wait returns the estimate's status and frees ev.
 */
LGE_API int lge_estimate_async(lge_ctx *ctx, const lge_graph *g, double p, uint64_t seed, void *hip_stream,
                       lge_result *out, lge_event **ev);
LGE_API int lge_event_wait(lge_event *ev);

/*
 * Batched estimate of many independent graphs in one launch sequence.
 * Concatenated CSR: graph k has n_k = vtx_off[k+1]-vtx_off[k] vertices, its
 * local row_ptr (n_k+1 entries, starting at 0) at row_ptr[vtx_off[k] + k],
 * and its local column ids at col[nnz_off[k] .. nnz_off[k+1]).
 * p[k], seed[k] per graph.  Host arrays; outs[count] caller-owned.
 */
typedef struct {
  int32_t count;
  const int64_t *vtx_off; /* count+1 */
  const int64_t *nnz_off; /* count+1 */
  const int32_t *row_ptr; /* vtx_off[count] + count entries */
  const int32_t *col;     /* nnz_off[count] entries */
  const double *p;        /* count */
  const uint64_t *seed;   /* count */
  uint32_t flags;         /* LGE_FLAG_TRUSTED skips validation */
} lge_batch;

LGE_API int lge_count_batch(lge_ctx *ctx, const lge_batch *b, const lge_opts *opts, lge_result *outs);

/*
 * Many resident graphs (created on this ctx) estimated in one launch
 * sequence: graph k with p[k], seed[k]; outs[count] caller-owned.  Results
 * equal `count` separate lge_estimate calls.
 */
LGE_API int lge_estimate_many(lge_ctx *ctx, const lge_graph *const *graphs, const double *p, const uint64_t *seed,
                              int32_t count, const lge_opts *opts, lge_result *outs);

/*
 * Adaptive estimation (Sec. 4, Alg. 8).  Starting from an empty sample,
 * round t grows it by a fraction phi of the edges not yet sampled,
 * p_t = p_{t-1} + phi (1 - p_{t-1}), and halves phi (phi0 = 0 picks
 * 1/sqrt(m)); the loop stops when the largest relative change of the
 * 4-vertex estimates G7..G17 between consecutive rounds is <= beta (a zero
 * previous estimate with a non-zero new one counts as change 1), or after
 * t_max rounds.  The samples are nested (one Philox uniform per edge against
 * growing thresholds), so each round counts only its new edges and *out is
 * exactly lge_estimate(g, p_T, seed) for the final p_T.  trace (may be NULL)
 * records p_t, the change (-1 in the first round) and |J| per round.
 */
#define LGE_ADAPTIVE_MAX_ROUNDS 64
typedef struct {
  double beta;   /* tolerance on the max relative change (default 0.01) */
  int32_t t_max; /* maximum rounds, 1..64 (default 20) */
  int32_t pad;
  double phi0;   /* initial growth fraction in (0, 1]; 0 = 1/sqrt(m) */
} lge_adaptive_cfg;

typedef struct {
  int32_t rounds;
  int32_t pad;
  double p[LGE_ADAPTIVE_MAX_ROUNDS];
  double delta[LGE_ADAPTIVE_MAX_ROUNDS];
  uint64_t sampled[LGE_ADAPTIVE_MAX_ROUNDS];
} lge_adaptive_trace;

LGE_API int lge_adaptive_cfg_default(lge_adaptive_cfg *cfg);
LGE_API int lge_estimate_adaptive(lge_ctx *ctx, const lge_graph *g, uint64_t seed, const lge_adaptive_cfg *cfg,
                                  lge_result *out, lge_adaptive_trace *trace);

/*
 * Weighted edge sampling (Sec. 2.2: the edge neighbourhoods may be drawn by
 * an arbitrary weighted distribution F, e.g. k-core numbers or degrees; Sec. 5
 * biases the sample towards large k-cores).  Edge e has weight
 *   LGE_WEIGHT_DEGREE : w_e = d_u + d_v - 2 (the edges sharing an end with e)
 *   LGE_WEIGHT_KCORE  : w_e = min(core(u), core(v))
 * quantised to 16 classes, class(e) = min(15, floor(log2 max(1, w_e))), and is
 * kept iff its Philox uniform (as in lge_estimate) is below
 * p_class = min(1, c 2^class), with c chosen so that the expected sample size
 * is p_mean * m.  The estimate is the Horvitz-Thompson sum
 * X_i = K_i + sum_{e in J} Y_i(e) / p_e, the variance estimate
 * V_i = sum_{e in J} (1 - p_e) / p_e^2 Y_i(e)^2 (the Sec. 2.4 argument with a
 * per-edge probability), both exact integers per class combined in FP64 in
 * class order.  out->csum, z, q and sampled_edges are totals over the
 * classes, out->p = p_mean.  info (may be NULL) receives the class
 * probabilities, class sizes and sampled edges per class, and the graph's
 * largest core number (k-core mode; -1 before it is computed).  The first
 * call per mode builds and caches the classes (m bytes; k-core mode also the
 * core numbers, 4n bytes).  Errors: LGE_EINVAL (mode, p_mean outside (0,1],
 * null pointers), LGE_ENOMEM, LGE_EDEVICE, LGE_EINTERNAL.
 */
#define LGE_WEIGHT_DEGREE 1
#define LGE_WEIGHT_KCORE 2
#define LGE_WEIGHT_CLASSES 16
typedef struct {
  double p_level[LGE_WEIGHT_CLASSES];
  uint64_t edges[LGE_WEIGHT_CLASSES];
  uint64_t sampled[LGE_WEIGHT_CLASSES];
  int32_t max_core;
  int32_t pad;
} lge_weight_info;

LGE_API int lge_estimate_weighted(lge_ctx *ctx, const lge_graph *g, int32_t mode, double p_mean, uint64_t seed,
                                  const lge_opts *opts, lge_result *out, lge_weight_info *info);

/*
 * k-core numbers (the weights of the Sec. 5 extremal estimation): core(v) is
 * the largest k such that v survives the repeated deletion of vertices of
 * degree < k.  core_out: DEVICE pointer to n int32 (may be NULL); max_core:
 * host pointer (may be NULL).  Computed once per graph by level-synchronous
 * peeling on the device and cached.  Errors: LGE_EINVAL, LGE_ENOMEM,
 * LGE_EDEVICE, LGE_EINTERNAL.
 */
LGE_API int lge_core_numbers(lge_ctx *ctx, const lge_graph *g, int32_t *core_out, int32_t *max_core);

/*
 * Fixed-size sample (Alg. 1 with a sample size K) and the ratio estimator
 * sigma = m / K (the printed p_i = |J| / |E| of Sec. 2.3): the K edges with
 * the smallest 64-bit Philox keys (x1:x0 of the draw lge_estimate uses; ties
 * broken by edge id) form a uniformly random K-subset;
 * X_i = K_i + (m / K) sum_{e in J} Y_i(e) and the unbiased variance estimate
 * of sampling without replacement V_i = m (m - K) s_i^2 / K, s_i^2 the sample
 * variance of Y_i(e) (NaN for K = 1; 0 for K = m, where X is exact).  The
 * numerator K Q_i - Z_i^2 is formed exactly in 256 bits.  out->p = K / m.
 * Errors: LGE_EINVAL (K = 0 or K > m, null pointers), LGE_ENOMEM, LGE_EDEVICE,
 * LGE_EINTERNAL.
 */
LGE_API int lge_estimate_fixed_k(lge_ctx *ctx, const lge_graph *g, uint64_t k, uint64_t seed, const lge_opts *opts,
                                 lge_result *out);

/*
 * Micro-level graphlet statistics (Sec. 3, the micro problem and Alg. 7 with
 * p_e = 1, every neighbour examined once): for every edge e = (u, v) with
 * canonical id in [e0, e1), row e - e0 of `out` holds 17 int64, column i-1 =
 * the number of induced k-vertex subgraphs of type G_i (k = 2, 3, 4, numbered
 * as in Table 1) whose vertex set contains both u and v.  Column 0 (G1) is 1;
 * G2, G6 and G17 (no edges) are 0.  Alg. 7 counts some graphlets with e in one
 * role only (G8 with e as the chord, G9 with e as the tail, G12 with e in the
 * middle) and leaves G13, G14, G16 unrestricted; these rows count every
 * role, induced, so column i summed over all edges is (edges of G_i) x (number
 * of G_i) for i >= 3.
 *   out    : DEVICE pointer, (e1 - e0) x 17 int64, row-major, caller-owned;
 *            may be NULL only when e1 == e0.  Overwritten; on error its
 *            contents are unspecified.
 *   colmax : HOST pointer to 18 int64 or NULL: colmax[i] = largest value of
 *            column i-1 over the rows (the max graphlet statistic
 *            Z_i = max_e X_i(e) of Sec. 5 over the range; 0 for an empty
 *            range), colmax[0] = 0.
 * Blocks until the rows are written.  The first call on a graph builds and
 * caches per-arc triangle counts (8m + 8n bytes of device memory, freed with
 * the graph).  Errors: LGE_EINVAL (null ctx/graph, foreign graph, bad range),
 * LGE_ENOMEM, LGE_EDEVICE, LGE_EINTERNAL.
 */
#define LGE_MICRO_COLS 17
LGE_API int lge_micro(lge_ctx *ctx, const lge_graph *g, int64_t e0, int64_t e1, int64_t *out, int64_t *colmax);

/* Timing of the last lge_estimate / lge_count_batch on ctx. */
LGE_API int lge_last_timing(const lge_ctx *ctx, lge_timing *out);

/*
 * Autotuner (the order of work by hardness, Sec. 5): times candidate
 * settings on (g, p) by coordinate descent over wave_max_deg, block_max_deg,
 * probe_ratio, global_chunk, flags and grid_per_cu, and writes the fastest
 * to *out.  The choice is cached on ctx per graph class (bit lengths of m
 * and of the maximum degree, and p rounded to a quarter octave): a later
 * call for a graph of the same class returns the cached options without
 * timing.  Costs tens of estimates on a cache miss.  The choice never
 * changes results.  Errors: LGE_EINVAL, any lge_estimate error.
 */
LGE_API int lge_autotune(lge_ctx *ctx, const lge_graph *g, double p, lge_opts *out);

/* Empties ctx's autotuner cache.  Errors: LGE_EINVAL (null ctx). */
LGE_API int lge_autotune_reset(lge_ctx *ctx);

/*
 * Caps, in bytes, on the co-degree table and on the co-degree rows of the
 * graphs created on ctx from now on (0 = the library's own budgets, which
 * depend on the graph alone).  A resident set of many graphs shares HBM
 * this way; smaller tables mean more neighbour walks (slower estimates),
 * never different results.  Errors: LGE_EINVAL (null ctx).
 */
LGE_API int lge_set_table_budget(lge_ctx *ctx, uint64_t codeg_bytes, uint64_t rows_bytes);

/*
 * Cap, in bytes, on the temporary device memory a graph creation on ctx
 * takes for the ends of every vertex's neighbour segments at the co-degree
 * row tiles (Sec. 2.6 tables; 1 GiB by default, 0 restores it; freed before
 * the creation returns).  At least 8 bytes per vertex are taken whatever the
 * cap: a smaller cap means more passes over the tiles, never different
 * tables.  Errors: LGE_EINVAL (null ctx).
 */
LGE_API int lge_set_build_scratch(lge_ctx *ctx, uint64_t bytes);

/*
 * Serving.  A server owns `ctx` (no other call may use that ctx while the
 * server exists) and runs `workers` step threads: the first steps on ctx,
 * the others on contexts the server opens on the same device (own stream and
 * workspace), so one step's host round trips and tail overlap another step's
 * kernels.  Graphs are added once and stay resident.  Requests (graph, p,
 * seed) queue FIFO; up to max_inflight of them run at once.  Every step a
 * worker gives running requests the next chunks of their canonical edge-id
 * ranges: chunks share the step's work budget (measured work rate x
 * target_step_us) equally, each sized by its graph's work profile along the
 * edge ids (hub rows cost more), and together fit the step's device work
 * lists into hbm_budget_bytes (the admission bound by HBM footprint); with
 * three or more workers the last one is a short lane: it steps only requests
 * whose remaining expected time is below short_us, in steps of at most
 * short_us, and the other workers leave those to it, so short requests do
 * not queue behind long steps.  A worker runs all chunks
 * in one launch sequence and finalises the requests whose range is done and
 * whose chunks have all returned.  Requests arriving meanwhile join at the
 * next step (continuous batching).  A request's result equals lge_estimate on
 * the same (graph, p, seed): exact sums do not depend on chunking, order or
 * neighbours.  lge_submit / lge_wait / lge_cancel / lge_server_get_stats are
 * thread-safe; one thread may wait on a given ticket.
 */
typedef struct {
  int32_t max_inflight;     /* requests running at once (default 64) */
  int32_t queue_capacity;   /* queued + running requests before LGE_EBUSY (default 4096) */
  int64_t hbm_budget_bytes; /* device workspace budget of one step and worker (default 8 GiB): half for the
                               per-edge-id arrays of the step's ids (class lists, per-edge records), half
                               for its split-class work lists (a step needing more runs in pieces) */
  int64_t min_chunk_edges;  /* smallest edge-id chunk per request and step (default 4096) */
  int64_t target_step_us;   /* aimed duration of one step (default 20000); chunks are sized by each
                               graph's per-edge work estimate and the measured work rate */
  int32_t workers;          /* step threads, 1..4 (default 3; 0 = default) */
  int32_t short_us;         /* short-lane bound on a request's remaining expected time, microseconds
                               (default 20000; negative: no short lane) */
} lge_server_cfg;

typedef struct {
  uint64_t submitted, completed, canceled, rejected;
  uint64_t steps;   /* launch sequences run */
  uint64_t queued;  /* waiting for a running slot, now */
  uint64_t running; /* admitted and not finished, now */
  double busy_s;    /* wall time spent inside steps */
  uint64_t workspace_bytes; /* largest device workspace a worker has held after a step */
} lge_server_stats;

LGE_API int lge_server_cfg_default(lge_server_cfg *cfg);
/* cfg may be NULL (defaults); zero fields take defaults; negative -> LGE_EINVAL. */
LGE_API int lge_server_create(lge_ctx *ctx, const lge_server_cfg *cfg, lge_server **out);
/* g must belong to the server's ctx and outlive the server; *gid names it. */
LGE_API int lge_server_add_graph(lge_server *srv, const lge_graph *g, int32_t *gid);
/* p in (0,1] else LGE_EINVAL; unknown gid LGE_ENOTFOUND; full LGE_EBUSY;
 * after shutdown LGE_ECANCELED. */
LGE_API int lge_submit(lge_server *srv, int32_t gid, double p, uint64_t seed, uint64_t *ticket);
/* Waits up to timeout_us (< 0: forever).  LGE_OK fills *out and retires the
 * ticket; LGE_ETIMEDOUT keeps it; LGE_ECANCELED (cancelled or shut down) and
 * device errors retire it; unknown ticket LGE_ENOTFOUND. */
LGE_API int lge_wait(lge_server *srv, uint64_t ticket, int64_t timeout_us, lge_result *out);
/* Cancels a queued or running request (its wait returns LGE_ECANCELED). */
LGE_API int lge_cancel(lge_server *srv, uint64_t ticket);
LGE_API int lge_server_get_stats(lge_server *srv, lge_server_stats *out);
/* Stops the scheduler after the step in flight, resolves every pending
 * ticket with LGE_ECANCELED (threads blocked in lge_wait return), frees. */
LGE_API int lge_server_destroy(lge_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* LGE_H */
