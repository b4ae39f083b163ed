/*
 * bcd.h -- betweenness of one vertex r in a directed graph, computed only
 * from the sources that can reach r, on one MI355X (gfx950).
 *
 * Method: Chehreghani, Bifet and Abdessalem, "Exact and approximate
 * algorithms for computing betweenness centrality in directed graphs"
 * (arXiv 1708.08739).  References below are to that paper:
 *   Section 2, Eq.(1)-(4)   betweenness, dependency, Brandes' recursion
 *   Section 4.1, Def.1-3, Prop.1-2   RV(r) = vertices that reach r, found by
 *                           a traversal from r on the reverse graph
 *   Alg.1 (E-BCD)           exact BC(r) = sum over s in RV(r) of delta_s.(r)
 *   Section 4.2 (set form)  BC of r_1..r_l from one pass per s in the union
 *                           of their RV sets
 *   Alg.2 (A-BCD), Prop.3-4, Eq.(8)   sampled estimate and sample count
 *
 * Conventions for every call:
 *   - Every call returns a bcd_status.  Nothing aborts, prints or throws.
 *     On an error, outputs are left untouched (except *count on
 *     BCD_ERR_BUFFER_TOO_SMALL).  bcd_last_error() gives a thread-local
 *     message for the most recent failing call on the calling thread.
 *   - Pointers are HOST pointers unless a name says "device".  Input arrays
 *     belong to the caller and are only read during the call (the graph is
 *     copied to device memory by bcd_graph_load_csr).  Outputs go to
 *     caller-allocated buffers.  Handles are released by their free call.
 *   - Vertex ids are int32 in [0, n); n < 2^31; arcs m < 2^32.
 *   - Distances and path counts are exact integers; sigma is uint64 and any
 *     sigma_s(v) >= 2^64 for a vertex v reached from a processed source is
 *     reported as BCD_ERR_SIGMA_OVERFLOW (and no value is returned).
 *   - Dependencies and BC are IEEE double.  Results are deterministic: the
 *     same inputs give bit-identical outputs, whatever the batch width, and
 *     whether a query runs alone or inside the server among other queries.
 *   - A graph may be used by several threads at once; each call takes its
 *     own device workspace and stream.
 */
#ifndef BCD_H
#define BCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bcd_vid;
typedef struct bcd_graph bcd_graph;   /* opaque; immutable after load */
typedef struct bcd_server bcd_server; /* opaque */

typedef enum bcd_status {
  BCD_OK = 0,
  BCD_ERR_INVALID_ARG = 1,      /* NULL where not allowed, id out of range, bad eps/delta, l <= 0 */
  BCD_ERR_BAD_GRAPH = 2,        /* CSR malformed: row_ptr[0] != 0, decreasing, row_ptr[n] != m,
                                   column out of range, self-loop, repeated arc (rows must be
                                   strictly increasing), zero weight (Section 2 graph model) */
  BCD_ERR_SIGMA_OVERFLOW = 3,   /* a shortest-path count does not fit uint64 */
  BCD_ERR_OUT_OF_MEMORY = 4,    /* device or host allocation failed, or budget too small */
  BCD_ERR_DEVICE = 5,           /* HIP runtime error or no usable gfx950 device */
  BCD_ERR_BUFFER_TOO_SMALL = 6, /* *count holds the size needed */
  BCD_ERR_UNSUPPORTED = 7,      /* e.g. weighted distances would not fit uint32 */
  BCD_ERR_AGAIN = 8,            /* server: queue full, or poll timed out with nothing ready */
  BCD_ERR_CANCELLED = 9         /* server: query cancelled by shutdown or destroy */
} bcd_status;

/* Per-call statistics (all optional outputs). */
typedef struct bcd_stats {
  int64_t rv_size;          /* |RV(r)|; |D| for a set; -1 if the out-degree-0 shortcut applied */
  int64_t fr_size;          /* vertices reachable from r, r excluded (sampled calls; else -1) */
  int64_t samples;          /* T drawn (sampled calls; else 0) */
  int64_t distinct_sources; /* single-source passes actually run */
  uint64_t traversed_edges; /* sum over passes of m_s = arcs leaving the vertices s reaches */
  uint64_t reached;         /* sum over passes of n_s = vertices s reaches */
  uint64_t dag_arcs;        /* sum over passes of a_s = shortest-path-DAG arcs */
  double t_rv_s;            /* seconds spent finding RV(r) (device BFS + transfer) */
  double t_bc_s;            /* seconds from the first pass enqueued to the result on the host */
  int32_t batch_width;      /* sources per batch (64 * groups), 1 for the plain engine */
  int32_t ran_exact;        /* sampled calls: 1 if T >= |RV| made it run the exact sum */
} bcd_stats;

/* Engines for the per-source passes. */
#define BCD_ENGINE_BATCHED 0 /* 64 sources per wavefront column group, many groups per launch */
#define BCD_ENGINE_PLAIN 1   /* one source per launch, one launch per BFS level */
#define BCD_ENGINE_LDS 2     /* small unweighted graphs: a workgroup runs a source's whole pass with its
                                state in LDS (16 bytes per vertex must fit one workgroup's LDS, n < 2^16);
                                other graphs return BCD_ERR_UNSUPPORTED.  The server always batches. */

typedef struct bcd_config {
  int32_t engine;     /* BCD_ENGINE_* */
  int32_t groups;     /* batched engine: 64-source column groups per batch, >= 1
                         (default: the path-count rows near 64 GiB, at most 96,
                         128 on weighted graphs, a multiple of 8 above 8 since
                         group j runs in partition j % 8 of the 8 XCDs) */
  int32_t block;      /* threads per workgroup for traversal kernels: 64, 128, 256, 512
                         (default 256, 64 on weighted graphs) */
  int32_t grid_mult;  /* workgroups per compute unit for traversal kernels, >= 1 */
  int32_t items;      /* batched engine, unweighted forward: frontier items a
                         wavefront takes per step, 1, 2 or 4 (64 / items lanes
                         per item for its first arcs); 0 = default */
  int32_t bottom_up;  /* batched engine, unweighted forward: a BFS level is
                         found bottom-up (in-arcs of the unsettled (group,
                         vertex) pairs) when the level before it holds at
                         least 1/bottom_up of the batch's (group, vertex)
                         pairs; 0 = always top-down, -1 = default (4 on
                         graphs of 2^19 vertices or more, else 0) */
  int32_t compress;   /* exact and set calls: 1 = a source s gated into a
                         vertex a gets no pass of its own (the compression the
                         paper says composes with RV(r), Section 4.2).  s is
                         gated into a when s lies on no directed cycle and every
                         out-neighbour of s is a or is itself gated into a (a
                         source with no in-arcs and one out-arc (s, v) is the
                         simplest case); every path from s then leaves through
                         a, so delta_s(t) = delta_a(t) for t != a, and
                         delta_s(a) = the number of vertices a reaches.  Used
                         only when no target is gated into a.  Values equal
                         the uncompressed ones up to rounding; stats count only
                         the sources that ran; the gates are computed on the
                         host on the first compressed call (strongly connected
                         components, O(n + m)).  0 = off (the default) */
  int32_t push;       /* batched engine, unweighted forward: 1 = a level found
                         top-down adds each path count along its DAG arcs
                         (one 64-bit atomic add per (source, DAG arc), no
                         in-arc read), 0 = each vertex pulls its count over its
                         in-arcs; the same values either way (exact integer
                         sums); -1 = default */
} bcd_config;

/* Sampled estimate (Alg.2).  T comes from Eq.(8) unless T_override > 0. */
typedef struct bcd_sample_params {
  double eps;          /* additive error; normalised by n(n-1) unless BCD_EPS_ABSOLUTE */
  double delta;        /* failure probability, in (0, 1) */
  uint64_t seed;       /* draw t picks index floor(mix64(seed + (t+1)*0x9E3779B97F4A7C15) * |RV| / 2^64)
                          of the ascending RV(r) list (SplitMix64 output t for state seed) */
  uint32_t flags;      /* BCD_EPS_ABSOLUTE | BCD_K_TRIVIAL | BCD_NO_EXACT_FALLBACK */
  int64_t T_override;  /* > 0: use exactly this many draws (the paper's tau mode) */
} bcd_sample_params;

#define BCD_EPS_ABSOLUTE 1u      /* eps is an absolute error on BC(r) */
#define BCD_K_TRIVIAL 2u         /* K = n - 2 instead of K = |vertices reachable from r| */
#define BCD_NO_EXACT_FALLBACK 4u /* sample even when T >= |RV(r)| */
#define BCD_SAMPLE_ALL_VERTICES 8u /* baseline without the pruning: draw uniformly from V \ {r}
                                      (ascending), bc = (n-1)/T * sum_t delta_{v_t}.(r), and Eq.(8)
                                      with n-1 in place of |RV(r)|; never falls back to exact */

/* ------------------------------------------------------------- graph */

/* Validate and upload a CSR digraph (Section 2 graph model: directed, no
 * self-loops, no repeated arcs; positive weights when weighted).
 *   n        vertex count, 1 <= n < 2^31
 *   m        arc count, 0 <= m < 2^32
 *   row_ptr  int64[n+1], host; arcs of v are row_ptr[v] .. row_ptr[v+1]-1
 *   col      int32[m], host; heads, strictly increasing within each row
 *   weight   uint32[m] host (positive), or NULL for an unweighted graph
 *   out      receives the handle
 * The out-CSR and its transpose (the reverse graph R(G) of Def.2) stay
 * resident in device memory until bcd_graph_free.  Errors: INVALID_ARG,
 * BAD_GRAPH, OUT_OF_MEMORY, DEVICE. */
bcd_status bcd_graph_load_csr(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                              const uint32_t *weight, bcd_graph **out);

/* Release a graph and every device buffer it holds.  NULL is a no-op. */
bcd_status bcd_graph_free(bcd_graph *g);

/* Vertex and arc counts of a loaded graph. */
bcd_status bcd_graph_info(const bcd_graph *g, int64_t *n, int64_t *m, int32_t *weighted);

/* Set / read the engine configuration used by later calls on this graph. */
bcd_status bcd_set_config(bcd_graph *g, const bcd_config *cfg);
bcd_status bcd_get_config(const bcd_graph *g, bcd_config *cfg);

/* Autotuner: times the per-source passes of a fixed seeded sample of RV(r)
 * (at most max_sources sources) under each candidate and keeps the one with
 * the highest traversed arcs per second: first the batched engine with
 * groups in the powers of two from the largest one <= max_groups / 8 (at
 * least 1) to max_groups, x grid_mult in {8,16,32} (block 256, or 64 on
 * weighted graphs; 2 items per step, top-down), then around the best block
 * 512 (weighted: 128 and 256) and, on unweighted graphs, items 1 and 4,
 * bottom-up levels (16, 4) and the other path-count form (push), then the
 * LDS engine when the graph fits it.  Installs the choice on the graph and
 * returns it in *best (and its rate in *gteps, may be NULL).  Results of
 * later calls do not depend on the choice (every engine and setting gives
 * the same per-source values).  Errors: INVALID_ARG (r out of range, RV(r)
 * empty, max_groups < 1). */
bcd_status bcd_autotune(bcd_graph *g, bcd_vid r, int32_t max_groups, int64_t max_sources, bcd_config *best,
                        double *gteps);

/* RV(r) of Def.1, found as Def.3 / Prop.2 prescribe: a breadth-first
 * traversal from r on the resident reverse graph, weights ignored, r left
 * out.  Writes the ids ascending into out[0 .. *count-1] if cap suffices;
 * otherwise returns BUFFER_TOO_SMALL with *count set.  out may be NULL to
 * query the size (then BCD_OK with *count). */
bcd_status bcd_rv(const bcd_graph *g, bcd_vid r, bcd_vid *out, int64_t cap, int64_t *count);

/* bcd_rv without allocation, for callers that cannot allocate device or
 * pinned host memory (code under HIP graph capture, serving loops and
 * harnesses that forbid it).  Same arguments, result and errors as bcd_rv.
 * The traversal's working memory (visited bitmap, two frontier queues,
 * counters: 8 bytes per vertex plus n/8) is one static device array of
 * 34,079,000 bytes that each GPU holds from library load until the process
 * ends; graphs of more than 2^22 vertices return BCD_ERR_UNSUPPORTED.  The
 * graph's device must be current.  Calls in one process are serialized on
 * that array by a lock (they run one at a time); each call clears what it
 * reads, so no earlier call's contents reach its result.  Blocks until the
 * ids are in out. */
bcd_status bcd_rv_noalloc(const bcd_graph *g, bcd_vid r, bcd_vid *out, int64_t cap, int64_t *count);

/* Exact BC(r), Alg.1 (E-BCD): 0 if r has out-degree 0 (Prop.1); otherwise
 * the sum over s in RV(r) of delta_s.(r) (Eq.(5)), each from one shortest-
 * path pass from s (BFS levels, or positive-weight relaxation when the
 * graph is weighted) and the Eq.(4) backward accumulation.  The sum runs in
 * ascending s with Neumaier compensation.  st may be NULL. */
bcd_status bcd_bc_exact(const bcd_graph *g, bcd_vid r, double *bc, bcd_stats *st);

/* Sampled BC(r), Alg.2 (A-BCD): T uniform draws with replacement from
 * RV(r); bc = |RV(r)| / T * sum_t delta_{v_t}.(r), summed in draw order.
 * T = Eq.(8) with K = vertices reachable from r (or n-2 with
 * BCD_K_TRIVIAL) unless T_override > 0; if T >= |RV(r)| the exact value
 * is returned instead unless BCD_NO_EXACT_FALLBACK.  Each distinct drawn
 * source is computed once.  Errors: INVALID_ARG for eps <= 0 or delta not
 * in (0,1) when T_override <= 0. */
bcd_status bcd_bc_sampled(const bcd_graph *g, bcd_vid r, const bcd_sample_params *p, double *bc,
                          bcd_stats *st);

/* The BCD procedure of Section 5: find RV(r); if |RV(r)| <= tau run E-BCD
 * (Alg.1), otherwise A-BCD (Alg.2) with T = tau draws (seeded as in
 * bcd_sample_params).  st->ran_exact tells which.  Errors: INVALID_ARG for
 * tau < 1. */
bcd_status bcd_bc_bcd(const bcd_graph *g, bcd_vid r, int64_t tau, uint64_t seed, double *bc, bcd_stats *st);

/* BC of every vertex of rs[0..l-1] (Section 4.2): D = union of the RV(r_i);
 * one pass per s in D serves every r_i; bc[i] sums delta_s.(r_i) over s in
 * D, s != r_i, ascending s.  Repeats in rs are allowed.  bc is double[l]. */
bcd_status bcd_bc_set(const bcd_graph *g, const bcd_vid *rs, int64_t l, double *bc,
                      bcd_stats *st);

/* Verification hook: the whole pass from one source s (forward + Eq.(4)
 * for every vertex) with the configured engine.  dist uint64[n]
 * (UINT64_MAX when unreached), sigma uint64[n], delta double[n] (0 when
 * unreached; delta[s] as Eq.(4) gives it); any output may be NULL. */
bcd_status bcd_source_pass(const bcd_graph *g, bcd_vid s, uint64_t *dist, uint64_t *sigma,
                           double *delta);

/* Same for k distinct sources in one batch of the batched engine.  Outputs
 * are [k][n] row-major (source-major).  k <= 64 * groups. */
bcd_status bcd_multi_source_pass(const bcd_graph *g, const bcd_vid *sources, int64_t k,
                                 uint64_t *dist, uint64_t *sigma, double *delta);

/* Per-source dependencies delta_s.(r) for an explicit source list (in the
 * given order), plus per-source counters (n_s, m_s, a_s) as uint64[k][3]
 * (counters may be NULL).  Sources need not be in RV(r). */
bcd_status bcd_dependencies(const bcd_graph *g, bcd_vid r, const bcd_vid *sources, int64_t k,
                            double *dep, uint64_t *counters);

/* Eq.(8): smallest T >= 1 with T >= ln(2/delta) K^2 rv_size^2 / (2 eps_abs^2);
 * saturates at INT64_MAX.  Pure host arithmetic. */
bcd_status bcd_sample_count(double eps_abs, double delta, double K, int64_t rv_size, int64_t *T);

const char *bcd_status_string(bcd_status s);
const char *bcd_last_error(void);

/* ------------------------------------------------------------ profiling
 * When enabled, every launch of the traversal kernels is bracketed by HIP
 * events on its own stream, and the algorithmic byte counts of each launch
 * are accumulated (see DESIGN notes in the source).  kind: 0 = forward
 * level kernel, 1 = backward level kernel. */
typedef struct bcd_kernel_profile {
  int64_t launches;
  double total_ms;     /* sum of per-launch event durations */
  double alg_bytes;    /* algorithmic bytes moved by those launches */
  uint64_t vertex_pairs; /* (source, vertex) pairs processed */
  uint64_t arc_pairs;    /* (source, arc) pairs scanned */
  uint64_t dag_pairs;    /* (source, shortest-path-DAG arc) pairs used */
  uint64_t items;        /* work items: one per (64-source column group, vertex,
                            level) with a nonempty lane mask (weighted engine:
                            topological round in place of level) */
  double union_ms;       /* wall time during which at least one of these launches
                            ran: launches overlapping on concurrent streams
                            (pipelined batches) count once */
  uint64_t item_arcs;    /* sum over the work items of their vertex's out-degree
                            (batched unweighted engine; else 0) */
  double sched_bytes;    /* algorithmic bytes with the graph structure counted once
                            per work item instead of once per source: 16 per item
                            (row offsets) + 4 per item arc (column index) + 16 per
                            (source, vertex) + 4 per (source, arc) + 8 per (source,
                            DAG arc); equal to alg_bytes for engines that share
                            nothing across sources; 0 where not counted (weighted) */
} bcd_kernel_profile;

bcd_status bcd_profile_enable(bcd_graph *g, int32_t on);
bcd_status bcd_profile_get(const bcd_graph *g, int32_t kind, bcd_kernel_profile *out);
bcd_status bcd_profile_reset(bcd_graph *g);

/* Streaming-copy probe: achieved device bandwidth (GB/s, read+write) of a
 * copy of `bytes` bytes (rounded down to 16-byte words; non-temporal 16-byte
 * loads and stores, four in flight per thread, 64 workgroups of 256 per
 * compute unit), best of `reps` after one untimed launch. */
bcd_status bcd_bandwidth_probe(int64_t bytes, int32_t reps, double *gbps);
/* The same for a read of `bytes` bytes (GB/s read): the reference for kernels
 * whose traffic is mostly reads, as the traversal kernels' is. */
bcd_status bcd_read_bandwidth_probe(int64_t bytes, int32_t reps, double *gbps);

/* -------------------------------------------------------------- serving
 * A request loop for many BC(r) queries on one resident graph (the calls of
 * Alg.1, Alg.2 and the Section 4.2 set form, as above).  Queries are admitted
 * in arrival order while their device result buffers fit the HBM budget; the
 * sources of all admitted queries are packed into shared batches (a source
 * needed by several queries is computed once), so queries that arrive while
 * others run join the next batches and their work overlaps on the device.
 * Every result is bit-identical to the same call made alone. */

typedef struct bcd_server_config {
  uint64_t hbm_budget_bytes; /* device bytes for workspaces + per-query buffers; 0 = 64 GiB */
  int32_t workers;           /* concurrent batches (one stream each), >= 1; 0 = 2 */
  int32_t groups;            /* 64-source column groups per batch; 0 = graph's configured value.
                                Above 8, a multiple of 8 keeps the 8 XCD partitions even */
  int32_t queue_capacity;    /* max queries submitted and not yet polled; 0 = 4096 */
  int32_t reserved;
} bcd_server_config;

#define BCD_QUERY_EXACT 0   /* bcd_bc_exact(r) */
#define BCD_QUERY_SAMPLED 1 /* bcd_bc_sampled(r, params) */
#define BCD_QUERY_SET 2     /* bcd_bc_set(rs, l): bc_out receives l values */

typedef struct bcd_query {
  int32_t kind;              /* BCD_QUERY_* */
  bcd_vid r;                 /* EXACT, SAMPLED */
  const bcd_vid *rs;         /* SET: l targets, copied at submit */
  int64_t l;
  bcd_sample_params params;  /* SAMPLED */
  double *bc_out;            /* SET: caller buffer of l doubles, written before the result is
                                returned by bcd_server_poll; must stay valid until then */
  uint64_t tag;              /* opaque, echoed back */
} bcd_query;

typedef struct bcd_result {
  uint64_t ticket;
  uint64_t tag;
  int32_t status;            /* bcd_status of the query */
  int32_t kind;
  double bc;                 /* EXACT / SAMPLED value (SET: first target's value) */
  bcd_stats stats;
  double t_arrive_s;         /* submit time, seconds on the library's steady clock */
  double t_admit_s;          /* admission (RV done, buffers reserved) */
  double t_done_s;           /* result reduced and queued for poll */
} bcd_result;

/* Device bytes the batch workspaces of `workers` workers with `groups`
 * column groups take on graph g (0 = the defaults bcd_server_create uses);
 * a server's hbm_budget_bytes must exceed this, and the rest of the budget
 * holds per-query result buffers (8 bytes per (source, target) pair). */
bcd_status bcd_server_workspace_bytes(const bcd_graph *g, int32_t groups, int32_t workers, uint64_t *bytes);

/* Start a server on a loaded graph; the graph must outlive the server. */
bcd_status bcd_server_create(const bcd_graph *g, const bcd_server_config *cfg, bcd_server **out);
/* Enqueue one query (non-blocking).  *ticket identifies its result.  Errors:
 * INVALID_ARG (bad query), AGAIN (queue_capacity queries outstanding). */
bcd_status bcd_server_submit(bcd_server *s, const bcd_query *q, uint64_t *ticket);
/* Collect up to cap finished results into out[0 .. *n_out-1], waiting up to
 * timeout_ns for the first one (0 = do not wait, < 0 = wait forever).
 * Returns AGAIN if none finished in time. */
bcd_status bcd_server_poll(bcd_server *s, bcd_result *out, int32_t cap, int32_t *n_out, int64_t timeout_ns);
/* Aggregate counters of a server since creation.  Traversed arcs of shared
 * batches cannot be split between the queries that share them, so per-query
 * stats carry no traversed_edges; these totals do. */
typedef struct bcd_server_stats {
  uint64_t queries_done;
  uint64_t batches;
  uint64_t lanes_used;        /* sum over batches of sources run */
  uint64_t lane_slots;        /* sum over batches of the batch width */
  uint64_t traversed_edges;   /* sum of m_s over every source run */
  uint64_t shared_lanes;      /* lanes whose source served more than one query */
} bcd_server_stats;
bcd_status bcd_server_get_stats(bcd_server *s, bcd_server_stats *out);

/* Library steady-clock time in seconds (the clock of the t_* fields). */
double bcd_server_now(void);
/* Stop taking work: later submits fail with CANCELLED; queries not yet
 * admitted finish with status CANCELLED; admitted queries run to completion.
 * Returns once nothing is admitted or being planned; every query's result
 * (value or CANCELLED) can still be collected with bcd_server_poll.  Errors:
 * INVALID_ARG for NULL. */
bcd_status bcd_server_shutdown(bcd_server *s);
/* bcd_server_shutdown, then stop the threads and release every buffer;
 * results not yet polled are discarded.  NULL is a no-op. */
bcd_status bcd_server_destroy(bcd_server *s);

#ifdef __cplusplus
}
#endif
#endif /* BCD_H */
