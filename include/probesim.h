/*
 * probesim.h -- C ABI of the MI355X ProbeSim library.
 *
 * The library answers approximate single-source and top-k SimRank queries
 * with ProbeSim (Liu et al., "ProbeSim: Scalable Single-Source and Top-k
 * SimRank Computations on Dynamic Graphs", PVLDB 11(1), 2017) on one AMD
 * Instinct MI355X (gfx950).  Every step of a query -- sqrt(c)-walk sampling,
 * the reverse reachability tree, PROBE level expansion with both pruning
 * rules, accumulation of the estimate and top-k selection -- runs in the
 * library's own HIP kernels.
 *
 * Conventions for every entry point:
 *  - Nothing throws across the ABI; every call returns a ps_status.
 *  - Graph input arrays are borrowed for the duration of the call only; the
 *    library copies what it keeps.
 *  - Output buffers are owned by the caller.  A pointer is accepted either as
 *    host memory or as device memory of the context's GPU (for instance a
 *    torch tensor's data_ptr()); the library tells the two apart with
 *    hipPointerGetAttributes.  Synchronous calls have finished writing their
 *    outputs when they return.
 *  - Node ids are int32 in [0, n).  An edge x -> y means x is an in-neighbour
 *    of y (x in I(y)); walks follow in-edges, PROBE follows out-edges.
 *  - Calls on one context are not thread-safe unless stated otherwise; the
 *    server (ps_server_*) is the thread-safe entry.
 *
 * Precision.  Probe scores (Alg. 2) are FP32 numbers: a contribution is
 * fl32(fl32(Score(x) * fl32(sqrt c)) * fl32(1/|I(v)|)) (fl32: nearest FP32
 * number), the contributions to a node are summed exactly as 64-bit integers
 * on the grid 2^-62, an inner level's score is that sum rounded to FP32 and
 * Pruning Rule 2 compares it with fl32(eps_p / sqrt(c)^(i-j-1)).  Estimates
 * are accumulated in FP64.  So a query's result does not depend on the
 * order of the device's atomic adds, on the batch or server mix it runs in,
 * on the number of probe slots or on pushing versus pulling: only the order
 * of the FP64 additions varies.  Against the plain FP64 evaluation of the
 * method a result differs by FP32 rounding (about 1e-7 relative) and by the
 * Rule-2 tests that rounding decides, which ps_result.flip_allowance bounds.
 */
#ifndef PROBESIM_H
#define PROBESIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ps_status {
  PS_OK = 0,
  PS_ERR_INVALID_ARG = 1, /* c, eps or delta outside (0,1); bad k; bad options */
  PS_ERR_NODE_RANGE = 2,  /* a node id outside [0, n) */
  PS_ERR_SELF_LOOP = 3,   /* edge x -> x in a simple digraph (Section 2.1) */
  PS_ERR_DUP_EDGE = 4,    /* edge already present */
  PS_ERR_NO_EDGE = 5,     /* deleting an edge that is absent */
  PS_ERR_OOM = 6,         /* device or host allocation failed */
  PS_ERR_BUSY = 7,        /* server request ring is full */
  PS_ERR_DEVICE = 8,      /* a HIP runtime call failed */
  PS_ERR_TIMEOUT = 9,     /* ps_wait ran out of time */
  PS_ERR_STATE = 10       /* call not valid in the object's current state */
} ps_status;

typedef struct ps_ctx ps_ctx;
typedef struct ps_graph ps_graph;
typedef struct ps_server ps_server;

/* Human-readable name of a status code (static storage). */
const char* ps_status_string(ps_status s);

/* ------------------------------------------------------------ context -- */

/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * to launch on (for example torch.cuda.current_stream().cuda_stream); NULL
 * makes the library create its own stream.  The context owns its device
 * workspace, which grows on demand and is freed by ps_ctx_destroy. */
ps_status ps_ctx_create(int device, void* hip_stream, ps_ctx** out);
void ps_ctx_destroy(ps_ctx* ctx);

/* With enable != 0 every PROBE expansion launch is bracketed by HIP events on
 * the context's stream; ps_get_stats then reports their summed duration. */
ps_status ps_ctx_set_timing(ps_ctx* ctx, int enable);

/* -------------------------------------------------------------- graph -- */

#define PS_LOAD_DEDUP 1u           /* drop duplicate edges instead of failing */
#define PS_LOAD_DROP_SELF_LOOPS 2u /* drop self-loops instead of failing */

/* Loads the directed simple graph G = (V, E), |V| = n, with m edges
 * src[i] -> dst[i] (arrays of m int32, host memory or device memory of the
 * context's GPU, borrowed for the call only).  Builds, on the device, the
 * in-adjacency (each row in ascending source id: the canonical order walks
 * index into) and the out-adjacency, plus 1/|I(v)|.  Errors:
 * PS_ERR_NODE_RANGE for an id outside [0, n); PS_ERR_SELF_LOOP /
 * PS_ERR_DUP_EDGE unless the matching PS_LOAD_* flag is set;
 * PS_ERR_INVALID_ARG for n <= 0, m < 0 or m >= 2^31. */
ps_status ps_graph_load(ps_ctx* ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        uint32_t flags, ps_graph** out);
void ps_graph_free(ps_graph* g);

/* n, live edge count and version (starts at 0, +1 per applied update batch). */
ps_status ps_graph_info(const ps_graph* g, int32_t* n, int64_t* m, uint64_t* version);

/* Applies k edge updates in order: op[i] = 0 inserts src[i] -> dst[i], 1
 * deletes it.  The paper's method is index-free (abstract; Section 1), so an
 * update only rewrites the affected adjacency rows (copy-on-write into a
 * device delta region) and 1/|I(v)|; queries issued afterwards see the new
 * version.  Invalid single updates (self-loop, inserting an existing edge,
 * deleting an absent one) are skipped; their status goes to per_edge[i]
 * (nullable: without it the first such error is returned after all valid
 * updates are applied).  An id outside [0, n) fails the whole call before
 * anything changes.  *version (nullable) receives the new version. */
ps_status ps_graph_update(ps_graph* g, int64_t k, const int32_t* src, const int32_t* dst,
                          const uint8_t* op, int32_t* per_edge, uint64_t* version);

/* Copies the current edge list (ascending by (src, dst)) into host arrays of
 * capacity `cap`; *m receives the edge count.  PS_ERR_INVALID_ARG if cap is
 * too small (with *m set). */
ps_status ps_graph_edges(const ps_graph* g, int64_t cap, int32_t* src, int32_t* dst, int64_t* m);

/* --------------------------------------------------------- parameters -- */

typedef struct ps_options {
  double eps_s;       /* sampling error; < 0: eps/2 */
  double eps_t;       /* Rule 1 truncation parameter; < 0: eps/4 */
  double eps_p;       /* Rule 2 pruning parameter; < 0: (eps/4)(1-sqrt c)/(1+eps_s); 0: no pruning */
  int32_t max_len;    /* > 0: walk length cap L overriding Rule 1 (at most PS_MAX_WALK_LEN) */
  int32_t bias_shift; /* nonzero: add eps_t/2 to every estimate but u's (Section 4.1) */
  int64_t walk_begin; /* first walk index (default 0) */
  int64_t walk_end;   /* one past the last walk index; < 0: n_r.  A sub-range
                         returns that range's share of the sum over walks
                         (still divided by the full n_r), so shards add up;
                         under PS_PROBE_HYBRID a shard's tree weights, and so
                         its switches, are the shard's own, so its shards
                         give another valid estimate, not the whole's. */
  int32_t slots;      /* concurrent probes on the device; 0: the graph's autotuned
                         setting, else 1024; at most 2000.  A slot holds a few
                         hundred bytes; its frontier lives in lists shared by
                         all slots and sized from the graph's edge count. */
  int32_t probe_mode; /* PS_PROBE_DETERMINISTIC (Alg. 2 with Rule 2, the
                         default), PS_PROBE_RANDOMIZED (Alg. 4, Section 4.3:
                         one randomized probe per walk and prefix, no Rule 2;
                         candidate v of iteration j of the probe of prefix
                         (u_1..u_i) of walk k draws Philox4x32-10 with key
                         (seed_lo, seed_hi ^ 0x9E3779B9) and counter
                         (k, i * 2^16 + j, v, 1): words 1:0 pick its
                         in-neighbour as walks do, word 2 < floor(sqrt(c) *
                         2^32) is the sqrt(c) coin) or PS_PROBE_HYBRID (the
                         switch of Section 4.4: each tree node of weight w
                         runs Alg. 2 with Rule 2; when a level about to be
                         expanded, H_0 included, keeps entries with more than
                         hybrid_c0 * w * n out-edges in total, that probe is
                         dropped and each of the w walks through the node runs
                         Alg. 4 on the prefix, drawing what it draws in
                         randomized mode) or PS_PROBE_MERGED (Alg. 3 with
                         Rule 2 off, eps_p taken as 0: PROBE is linear in
                         H_0 (Lemma 2), so the weighted probes of each
                         subtree are summed at its root and pushed once
                         through the level maps they share; FP64 sums, the
                         plain definition's values up to the order of the
                         additions; not for ps_server) */
  int64_t pull_edges; /* a probe level whose kept entries have at least this many
                         out-edges is computed by pulling along in-edges over
                         all nodes instead of pushing along its out-edges (same
                         sums, other order); 0: automatic, < 0: never */
  double hybrid_c0;   /* the constant c0 of PS_PROBE_HYBRID (>= 0, infinity
                         allowed; the paper gives no value): default 0.003,
                         the fastest of 0.001..1 on power-law graphs */
  int32_t rule2_bound; /* which per-probe error of Pruning Rule 2 the default
                         eps_p (and ps_tune_split's candidates) are derived
                         from in Theorem 2's inequality.  PS_RULE2_AS_STATED
                         (default): the paper's lemma, eps_p per probe, so the
                         pruning term is (1 + eps_s) / (1 - sqrt c) * eps_p
                         (E[l] = 1/(1 - sqrt c) probes per walk).
                         PS_RULE2_PROVEN: the bound the lemma's induction
                         gives when the pruned node's own score is kept,
                         (i - 1) * eps_p for a probe of depth i, so a walk of
                         l nodes loses at most l(l-1)/2 * eps_p and the term
                         is (1 + eps_s) * sqrt(c) / (1 - sqrt c)^2 * eps_p
                         (E[l(l-1)/2] = sqrt(c) / (1 - sqrt c)^2 for
                         geometric lengths; truncation and dead ends only
                         shorten walks): about 3.4x smaller eps_p at c = 0.6,
                         more work, a proven guarantee. */
  int32_t pad;
} ps_options;

#define PS_RULE2_AS_STATED 0
#define PS_RULE2_PROVEN 1

#define PS_MAX_WALK_LEN 64
#define PS_PROBE_DETERMINISTIC 0
#define PS_PROBE_RANDOMIZED 1
#define PS_PROBE_HYBRID 2
#define PS_PROBE_MERGED 3

/* Fills the defaults above. */
void ps_options_default(ps_options* opt);

typedef struct ps_params {
  double c, eps_a, delta;
  double eps_s, eps_t, eps_p;
  int64_t n_r;     /* number of sqrt(c)-walks: ceil(3c ln(n/delta) / eps_s^2) (Alg. 1) */
  int32_t L;       /* walks keep nodes u_1..u_L, L = floor(ln eps_t / ln sqrt c) (Rule 1) */
  uint32_t t_stop; /* a walk stops at a node when its Philox word 0 < t_stop = floor((1-sqrt c) 2^32) */
} ps_params;

/* Derives the query parameters for a graph of n nodes.  Default split of the
 * absolute error eps (Definition 1) into sampling, truncation and pruning
 * error satisfies Theorem 2 with the optional shift off:
 *   eps_s = eps/2, eps_t = eps/4, eps_p = (eps/4)(1 - sqrt c)/(1 + eps_s)
 * (with opt->rule2_bound = PS_RULE2_PROVEN instead
 *   eps_p = (eps/4)(1 - sqrt c)^2 / ((1 + eps_s) sqrt c)).
 * PS_ERR_INVALID_ARG for c, eps, delta outside (0,1), for L < 2 or
 * L > PS_MAX_WALK_LEN. */
ps_status ps_derive_params(int32_t n, double c, double eps, double delta, const ps_options* opt,
                           ps_params* out);

/* -------------------------------------------------------------- query -- */

/* The sqrt(c)-walks of a query (Definition of the sqrt(c)-walk, Section 2.2),
 * as the query itself samples them: walk k stops at a node v when v has no
 * in-neighbour or word 0 of Philox4x32-10(key = seed, counter = (k, t, u, 0))
 * is below t_stop (t = index of v in the walk, from 0); otherwise it moves to
 * the in-neighbour with index floor(r64 * |I(v)| / 2^64), r64 = word2 << 32 |
 * word1, of v's ascending in-row; it keeps at most L nodes (Rule 1).  Writes
 * walks k_begin .. k_begin+count-1 as rows of L int32 (unused entries -1) to
 * `nodes` and their lengths to `lens` (host or device). */
ps_status ps_walks(ps_graph* g, int32_t u, double c, double eps, double delta, uint64_t seed,
                   const ps_options* opt, int64_t k_begin, int64_t count, int32_t* nodes, int32_t* lens);

/* Approximate single-source query (Definition 1): writes n doubles,
 * out[v] = estimate of s(u, v), out[u] = 1.  Samples n_r sqrt(c)-walks
 * from u, merges them into the reverse reachability tree (Alg. 3), runs
 * deterministic PROBE (Alg. 2) once per tree node with Rule 2 pruning and
 * adds weight/n_r * Score to the estimate.  Probe scores are FP32 with exact
 * sums, the estimate is accumulated in FP64 (see Precision above).
 * Deterministic for fixed (graph version, u, c, eps, delta, seed, walk
 * range) up to the order of the FP64 additions. */
ps_status ps_single_source(ps_graph* g, int32_t u, double c, double eps, double delta, uint64_t seed,
                           const ps_options* opt, double* out);

/* The same query as ps_single_source, returned sparsely: the nodes with a
 * nonzero estimate (u included, with 1) in ascending id order, with their
 * estimates.  Writes min(total, cap) pairs to nodes/scores (host or device)
 * and the total to *count (host).  Returns PS_ERR_INVALID_ARG when total >
 * cap (the first cap pairs are still written), so a caller can retry with
 * cap = *count.  With bias_shift every node is nonzero. */
ps_status ps_single_source_sparse(ps_graph* g, int32_t u, double c, double eps, double delta, uint64_t seed,
                                  const ps_options* opt, int64_t cap, int32_t* nodes, double* scores,
                                  int64_t* count);

/* Approximate top-k query (Definition 2): the k nodes v != u with the largest
 * estimates, ties broken by ascending node id, written to nodes[k] and their
 * estimates to scores[k].  k must lie in [1, n-1]. */
ps_status ps_topk(ps_graph* g, int32_t u, int32_t k, double c, double eps, double delta, uint64_t seed,
                  const ps_options* opt, int32_t* nodes, double* scores);

/* The selection step of Definition 2 on its own: given estimates s[n] of
 * s(u, .) (host or device; for instance the sum of walk-range shards
 * computed on several devices), writes the k nodes v != u with the largest
 * s[v], ties broken by ascending node id, to nodes[k] and their values to
 * out_scores[k] (host or device), in that order.  ps_topk ends with the same
 * selection.  PS_ERR_NODE_RANGE for u outside [0, n); PS_ERR_INVALID_ARG for
 * n < 2 or k outside [1, n-1].  Runs on the context's stream and returns
 * when the outputs are written. */
ps_status ps_select_topk(ps_ctx* c, const double* s, int32_t n, int32_t u, int32_t k, int32_t* nodes,
                         double* out_scores);

/* ps_select_topk for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same selection and results, with no hipMalloc, hipFree or
 * other allocating call.  Its scratch is a fixed array in the library's
 * device memory (about 0.8 MB per device, kept until the process ends).
 * s[n], nodes[k] and out_scores[k] must be device memory of the context's
 * device; k must lie in [1, min(n-1, PS_NOALLOC_MAX_K)] (PS_ERR_INVALID_ARG
 * otherwise, also for host pointers).  Asynchronous: the work is queued on
 * the context's stream and the outputs are ready when the stream reaches it.
 * Every call on one device shares that device's scratch, so calls that
 * overlap on one device (other streams, other contexts) race; calls queued
 * on one stream do not. */
#define PS_NOALLOC_MAX_K 65536
ps_status ps_select_topk_noalloc(ps_ctx* c, const double* s, int32_t n, int32_t u, int32_t k, int32_t* nodes,
                                 double* out_scores);

typedef struct ps_query {
  int32_t u;
  int32_t k; /* 0: single-source (n scores); > 0: top-k */
  double c, eps, delta;
  uint64_t seed;
  int32_t probe_mode; /* as ps_options.probe_mode */
  int32_t pad;
  double hybrid_c0;   /* c0 when this query's own probe_mode is PS_PROBE_HYBRID */
} ps_query;

typedef struct ps_result {
  double* scores; /* n doubles for single-source, k for top-k (caller-owned) */
  int32_t* nodes; /* k node ids for top-k; unused for single-source */
  int32_t status; /* ps_status of this query */
  int32_t count;  /* entries written */
  double flip_allowance; /* how far the FP32 scores may move an estimate away
                            from the plain FP64 evaluation through Rule 2: the
                            sum, over pruning tests whose score fell within
                            1e-5 relative of the threshold, of eps_p * (walks
                            sharing the probe) / n_r.  The stated error
                            against the FP64 evaluation is 1e-5 plus this. */
} ps_result;

/* Runs nq queries together: all their walks, trees and probes share the
 * device's probe slots and one level-synchronous launch sequence.  Each
 * result equals the same query run alone (up to FP64 summation order).  opt
 * applies to every query (its walk range must be the default); a query's
 * nonzero probe_mode overrides opt's.  Per-query
 * argument errors are reported in r[i].status and do not stop the others. */
ps_status ps_batch(ps_graph* g, int32_t nq, const ps_query* q, const ps_options* opt, ps_result* r);

/* ------------------------------------------------------------ tuning -- */

typedef struct ps_tune {
  int32_t slots;       /* probe slots chosen */
  int32_t from_cache;  /* 1 when read from the cache file */
  int64_t dense_edges; /* dense-level threshold chosen (< 0: never) */
  double ms_per_query; /* measured time of the chosen setting */
} ps_tune;

/* Autotuner of the launch settings that do not change results (beyond
 * the order of FP64 additions): the number of probe slots and the
 * out-edge threshold above which a probe level moves to the dense pass.  It
 * times the nsample query nodes `nodes` (host array) as plain single-source
 * queries under each candidate setting (one untimed run first) and keeps the
 * fastest as this graph's automatic setting (ps_options fields left at 0,
 * and servers started on it afterwards).
 * With cache_path non-NULL the choice is looked up in / appended to that text
 * file, keyed by the graph's n and m and the query's eps.  The context must
 * not have a running server. */
ps_status ps_autotune(ps_graph* g, int32_t nsample, const int32_t* nodes, double c, double eps, double delta,
                      const char* cache_path, ps_tune* out);

/* Split of the error eps_a among sampling, truncation and pruning chosen by
 * measurement (Theorem 2).  Candidates: eps_s = a_s * eps and eps_t = a_t *
 * eps for a_s in {0.5, 0.6, 0.7, 0.75, 0.8, 0.85} and a_t in {1/4, 1/16,
 * 1/256} (those whose parameters are valid: L within PS_MAX_WALK_LEN), with
 * eps_p taking the rest of the inequality of Theorem 2:
 *   eps_s + (1 + eps_s) / (1 - sqrt c) * eps_p + eps_t' = eps
 * (eps_t' = eps_t / 2 when opt->bias_shift is set, Section 4.1; else eps_t;
 * with opt->rule2_bound = PS_RULE2_PROVEN the pruning term is
 * (1 + eps_s) sqrt(c) / (1 - sqrt c)^2 * eps_p).  Every candidate meets
 * Theorem 2 under the chosen bound.  The nsample query
 * nodes `nodes` (host array) are timed under each (one untimed run first)
 * with the rest of *opt as given (probe mode, slots, ...), and the fastest
 * split is written into opt->eps_s, eps_t and eps_p.  The estimates change
 * with the split (another estimate with the same guarantee), so unlike
 * ps_autotune the choice is applied only through the options it returns.
 * PS_ERR_INVALID_ARG when opt's walk range or split fields are not the
 * defaults.  The context must not have a running server. */
typedef struct ps_split {
  double eps_s, eps_t, eps_p;  /* the split chosen (also written into opt) */
  double ms_per_query;         /* measured time of the chosen split */
  double default_ms_per_query; /* measured time of the first candidate (a_s 0.5, a_t 1/4:
                                  the default split when the shift is off) */
} ps_split;

ps_status ps_tune_split(ps_graph* g, int32_t nsample, const int32_t* nodes, double c, double eps, double delta,
                        ps_options* opt, ps_split* out);

/* Work counters and timings of the last query call on this context. */
typedef struct ps_stats {
  int64_t queries;
  int64_t walks;            /* walks sampled */
  int64_t walk_nodes;       /* sum of walk lengths */
  int64_t tree_nodes;       /* probes: reverse reachability tree nodes below the roots */
  int64_t probe_levels;     /* sum over probes of (depth - 1), switched probes' walks included */
  int64_t steps;            /* level steps launched */
  int64_t entries_expanded; /* frontier entries kept by Rule 2 and expanded */
  int64_t entries_pruned;   /* frontier entries removed by Rule 2 */
  int64_t edges_scanned;    /* out-edges of expanded entries */
  int64_t next_entries;     /* distinct (probe, node) entries created in inner levels */
  int64_t final_adds;       /* contributions added into estimates */
  int64_t expand_launches;  /* PROBE expansion (push) kernel launches */
  int64_t pull_levels;      /* probe levels computed by pulling */
  int64_t pull_edges;       /* in-edges read by those pulls */
  int64_t near_threshold;   /* Rule 2 tests within 1e-5 relative of the threshold */
  double flip_allowance;    /* largest per-query allowance of the call (ps_result) */
  double expand_ms;         /* summed duration of the push launches (timing enabled) */
  double pull_ms;           /* summed duration of the pull launches (timing enabled) */
  double total_ms;          /* wall time of the call */
  /* probe levels by the out-edge count E of their kept entries: bin b holds
     levels with 2^b <= E < 2^(b+1) (count, and the sum of E) */
  int64_t level_hist_count[32];
  int64_t level_hist_edges[32];
  int64_t switched_probes;  /* PS_PROBE_HYBRID: tree-node probes that switched */
  int64_t pushed_edges;     /* edges_scanned less those of levels pulled or switched instead
                               of pushed: the out-edges the push kernel visits */
  int64_t pushed_final_adds; /* final_adds made by the push kernel (the rest by pulls) */
  int64_t reduce_bins;      /* bins of pushed records summed (per level step: node ranges) */
  int64_t reduce_slices;    /* passes over those bins (more than one when a bin's keys
                               overflow the workgroup's table) */
  int64_t reduce_max_records; /* most records in one bin */
} ps_stats;

ps_status ps_get_stats(ps_ctx* ctx, ps_stats* out);

/* ------------------------------------------------------------- server -- */

typedef struct ps_server_cfg {
  int32_t ring;           /* request ring capacity (0: 1024) */
  int32_t max_inflight;   /* queries admitted on the device at once (0: 64) */
  int32_t slots;          /* probe slots (0: the graph's autotuned setting, else automatic) */
  int32_t reserved;
  int64_t frontier_bytes; /* device memory budget for the queries admitted at once
                             (0: none beyond max_inflight): a query holds 8 * n bytes of
                             FP64 accumulators plus its tree region, about 40 bytes per
                             entry of the power of two covering twice its measured walk
                             nodes; a query's tree is built only while the admitted
                             queries fit (one always runs), the others wait */
  const ps_options* defaults; /* nullable: options every served query runs with (the
                                 error split, probe mode and its c0, bias shift), copied
                                 at start; a query's own nonzero probe_mode (and then its
                                 hybrid_c0) overrides them.  Walk ranges must be the
                                 defaults (PS_ERR_INVALID_ARG) */
} ps_server_cfg;

typedef struct ps_server_stats {
  int64_t queries_done;          /* results handed back */
  int64_t update_batches;        /* ps_server_update batches applied */
  int64_t updates;               /* edge updates in them */
  double update_latency_ms_mean; /* ps_server_update call to the batch applied */
  double update_latency_ms_max;
  double update_apply_ms_mean;   /* host time to apply one batch (new graph version queued) */
  double update_apply_ms_max;
} ps_server_stats;

/* Starts a serving loop on the graph's context: a host thread that drains
 * the request ring, admits queries onto the device while slots and the
 * memory budget allow, runs level steps of all admitted queries together
 * (continuous batching: a query that arrives while others are running joins
 * at the next level step) and applies edge updates between level steps.  The
 * context must not be used directly while the server runs. */
ps_status ps_server_start(ps_graph* g, const ps_server_cfg* cfg, ps_server** out);

/* Counters of the serving loop so far (thread-safe). */
ps_status ps_server_get_stats(ps_server* s, ps_server_stats* out);

/* Queues one query.  r->scores / r->nodes must be host buffers that stay
 * valid until ps_wait returns for the ticket.  PS_ERR_BUSY when the ring is
 * full.  Thread-safe. */
ps_status ps_submit(ps_server* s, const ps_query* q, ps_result* r, uint64_t* ticket);

/* Waits up to timeout_us microseconds (< 0: forever) for a ticket; returns
 * the query's status, or PS_ERR_TIMEOUT.  Thread-safe. */
ps_status ps_wait(ps_server* s, uint64_t ticket, int64_t timeout_us);

/* Queues edge updates (as ps_graph_update); they are applied between level
 * steps.  A query reads exactly the edge set left by the updates submitted
 * before it (submission order is the order in which ps_submit and
 * ps_server_update calls take the server's lock); queries already running
 * keep their version.  Thread-safe; the arrays are copied. */
ps_status ps_server_update(ps_server* s, int64_t k, const int32_t* src, const int32_t* dst,
                           const uint8_t* op);

/* Stops accepting requests, finishes the queued and running ones, joins the
 * loop and frees the server. */
ps_status ps_server_stop(ps_server* s);

#ifdef __cplusplus
}
#endif

#endif /* PROBESIM_H */
