// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "probesim.h"

// A named range on a profiler's host timeline (rocprofv3 --marker-trace):
// the query phases, each batch of level steps, graph updates and top-k
// selections.  Without a profiler attached it costs one library call.
struct TraceRange {
  explicit TraceRange(const char* what) { roctxRangePushA(what); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

#define PS_HIP(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) {                        \
      ps_note_hip_error(e_, #x, __FILE__, __LINE__); \
      return PS_ERR_DEVICE;                        \
    }                                              \
  } while (0)

#define PS_TRY(x)                \
  do {                           \
    ps_status s_ = (x);          \
    if (s_ != PS_OK) return s_;  \
  } while (0)

void ps_note_hip_error(hipError_t e, const char* what, const char* file, int line);

// Grow-only device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};
ps_status devbuf_reserve(DevBuf& b, size_t bytes);
void devbuf_free(DevBuf& b);

// Whether `p` is device memory of the current device.
bool ps_is_device_ptr(const void* p);

// ------------------------------------------------------------------ graph --

// Column storage of one adjacency direction: rows live anywhere inside `col`
// (the base CSR first, then rows rewritten by updates in the delta region).
struct ColStore {
  int32_t* col = nullptr;
  uint64_t cap = 0;   // entries
  uint64_t used = 0;  // entries in use (base + delta)
  int refs = 0;       // graph versions pointing into it
};

// One immutable snapshot of the graph as queries read it.
struct GraphVersion {
  uint64_t version = 0;
  uint2* in_rows = nullptr;   // (start, len) of each node's in-row in in_store->col
  uint2* out_rows = nullptr;  // (start, len) of each node's out-row in out_store->col
  float* inv_indeg = nullptr; // 1/|I(v)| (0 when I(v) is empty)
  // Nodes whose in-row is longer than a lane should sum alone, and their
  // in-rows cut into fixed chunks, for levels computed by pulling.  Counts
  // (nodes, chunks) live on the device.
  int32_t* heavy_nodes = nullptr;
  int2* heavy_chunks = nullptr;          // (node, first in-row offset)
  unsigned long long* heavy_cnt = nullptr;
  uint64_t heavy_chunk_cap = 0;          // entries of heavy_chunks
  std::shared_ptr<ColStore> in_store, out_store;
  int refs = 0;               // queries reading this version + 1 while current
};

struct ps_graph {
  ps_ctx* ctx = nullptr;
  int32_t n = 0;
  int64_t m = 0;
  // Host mirror: the base CSR plus rows rewritten since the last compaction.
  std::vector<int64_t> h_in_ptr, h_out_ptr;
  std::vector<int32_t> h_in_col, h_out_col;
  std::unordered_map<int32_t, std::vector<int32_t>> mod_in, mod_out;
  GraphVersion* cur = nullptr;
  std::vector<GraphVersion*> retired;  // superseded versions still read by queries
  std::vector<GraphVersion*> spare;    // freed versions whose row arrays are reused
  // staging of update batches: rewritten rows and (node, row) patches go
  // through pinned host memory into a device buffer.  A ring of kStages
  // buffers: a batch refills the one used kStages batches earlier after its
  // event shows those uploads done, so a batch rarely waits for the level
  // steps queued ahead of it.
  static constexpr int kStages = 4;
  void* h_stage[kStages] = {};
  size_t h_stage_bytes[kStages] = {};
  DevBuf d_stage[kStages];
  hipEvent_t stage_ev[kStages] = {};
  bool stage_live[kStages] = {};
  int stage_next = 0;
  int tuned_slots = 0;                 // autotuned probe slots (0: none)
  int64_t tuned_dense = 0;             // autotuned dense threshold (0: none)
  std::mutex mu;
};

// Takes a reference on the current version (released with graph_release).
GraphVersion* graph_acquire(ps_graph* g);
void graph_release(ps_graph* g, GraphVersion* v);
// In-degree of v in the current host mirror.
int64_t graph_host_indeg(const ps_graph* g, int32_t v);
// In-degree cut-offs of the pull path: in-rows up to kPullLane edges are
// summed by one lane, longer ones in chunks of kPullChunk edges.
constexpr uint32_t kPullLane = 64;
constexpr uint32_t kPullChunk = 256;
// Applies a batch of updates (shared by ps_graph_update and the server).
ps_status graph_apply_updates(ps_graph* g, int64_t k, const int32_t* src, const int32_t* dst,
                              const uint8_t* op, int32_t* per_edge, uint64_t* version);

// ----------------------------------------------------------------- engine --

// Device record of one query admitted to a session.
struct QueryDev {
  int32_t u;
  int32_t L;
  uint32_t t_stop;
  int32_t topk;
  uint64_t seed;
  int64_t walk_begin;  // first walk index k
  int64_t walk_count;  // walks of this query
  int64_t walk_base;   // offset of its walks in the current walk launch
  float sc;            // sqrt(c) in FP32 (multiplies probe scores)
  int32_t pad;
  double inv_nr;       // 1 / n_r
  double shift;        // eps_t/2 when the bias shift is on, else 0
  uint64_t tree_base;  // first entry of the query's region in the tree pool
  uint64_t tree_mask;  // region capacity - 1 (a power of two)
  const uint2* in_rows;  // graph version the query reads
  const int32_t* in_col;
  const uint2* out_rows;
  const int32_t* out_col;
  const float* inv_indeg;
  double* acc;         // n FP64 accumulators, then the estimate
  const int32_t* heavy_nodes;
  const int2* heavy_chunks;
  const unsigned long long* heavy_cnt;
  double* flip;        // Rule-2 near-threshold allowance of the query
  double flip_unit;    // eps_p / n_r (times a walk count when charged)
  int32_t randomized;  // probes run Alg. 4, one per walk and prefix
  uint32_t t_sc;       // floor(sqrt(c) * 2^32): the sqrt(c) coin of Alg. 4
  uint2 key2;          // Philox key of Alg. 4's draws
  double c0;           // Section 4.4: switch constant (hybrid queries)
  int32_t hybrid;      // deterministic probes switch to Alg. 4 past c0 * w * n out-edges
  int32_t merged;      // tree only: its probes are merged per depth, not queued
};

// Host view of a query.
struct QueryRun {
  int32_t u = 0, k = 0;
  ps_params prm{};
  uint64_t seed = 0;
  int64_t walk_begin = 0, walk_end = 0;
  int bias_shift = 0;
  int randomized = 0;  // Alg. 4 instead of Alg. 2
  int hybrid = 0;      // Alg. 2 per tree node, switching to Alg. 4 (Section 4.4)
  double c0 = 0.0;     // the switch constant of a hybrid query
  int merged = 0;      // merged probing over the tree, Rule 2 off (merged.hip)
};

// A frontier list is kSubLists sub-lists, each with its own counter, so that
// appends from many wavefronts spread their atomics over several addresses.
constexpr int kSubLists = 16;

// State of one probe slot on the device.  The fields the expansion and the
// reduction read per edge or per entry come first (one cache line).
struct Slot {
  const int32_t* out_col;
  const float* inv_indeg;
  const uint2* out_rows;
  double* acc;
  double w;          // number of walks sharing the probed prefix (1 for a randomized probe)
  int32_t excl;      // graph node u_{i-j-1}, skipped by this level's expansion
  float sc;          // sqrt(c)
  float thr_next;    // Rule 2 threshold of the next level (score <= thr_next is removed)
  int32_t last;      // this level's expansion produces the returned score set
  int32_t mode;      // 1: randomized PROBE (Alg. 4) of walk wk's prefix
  uint32_t wk;       // walk index of a randomized probe
  int32_t probe;     // tree node of the probe being run, -1 when idle
  int32_t level;     // PROBE iteration j of the entries currently listed
  int32_t depth;     // i: the probe runs on (u_1..u_i)
  int32_t cursor;    // tree node whose graph node is excluded at this level
  int32_t query;     // query record
  int32_t lane;      // column of the dense frontier matrix, -1 for a sparse frontier
  float thr;         // Rule 2 threshold of the level being expanded
  uint32_t t_sc;     // floor(sqrt(c) * 2^32)
  uint2 key2;        // Philox key of Alg. 4's draws
  const uint2* in_rows;  // for levels computed by pulling and Alg. 4's draws
  const int32_t* in_col;
  const int32_t* heavy_nodes;
  const int2* heavy_chunks;
  const unsigned long long* heavy_cnt;
  double* flip;      // the query's near-threshold allowance
  double flip_unit;  // eps_p * w / n_r: what one Rule-2 flip can move an estimate by
  double hyb_thr;    // Section 4.4: switch when a level to expand has more out-edges (< 0: never)
};

enum CounterIdx {
  C_TAIL = 0,    // probes appended to the ring
  C_HEAD,        // probes handed to slots
  C_DONE,        // queries completed (entries in the done ring)
  C_LEVELS,      // sum over inserted probes of (depth - 1)
  C_WALK_NODES,
  C_KEPT,
  C_PRUNED,
  C_EDGES,
  C_NEXT,
  C_FINAL,
  C_LEVEL0,
  C_OVERFLOW,
  C_GHI,         // dense lanes in use this step: 1 + highest active lane
  C_GW,          // dense columns written this step (covers lanes freed last step)
  C_GPREV,       // C_GHI of the previous step
  C_PULLS,       // probe levels computed by the dense pass
  C_PULL_EDGES,  // in-edges read by dense passes
  C_PULL_T,      // dense threshold in out-edges (set by the host)
  C_NEAR,        // Rule 2 tests within 1e-5 relative of the threshold
  C_NZROWS0,     // rows of dense matrix 0 that may hold a nonzero score
  C_NZROWS1,     // the same for matrix 1
  C_SWITCH,      // deterministic probes switched to randomized ones (Section 4.4)
  C_HYBMASK,     // dense columns whose next level k_hyb_count measures (bit per column)
  C_EDGES_UNPUSHED,  // listed out-edges of levels k_expand does not push (pulled or switched)
  C_FINAL_PULL,  // final contributions added by the dense pass
  C_REC,         // records reserved by this step's expansion
  C_BIN,         // bins taken by this step's reduction
  C_TAIL_SNAP,   // C_TAIL when the last step's reduction started: what k_sched may claim
  C_TOT_E,       // out-edges of the levels to push this step (deterministic)
  C_TOT_N,       // bound on the next list's entries from this step's levels
  C_TOT_F,       // listed entries of this step's levels
  C_SWLANES,     // dense columns freed by switches this step (bit per column)
  C_PAUSED,      // slot levels held back a step by the per-step budget
  C_SH,          // bin shift of this step's records
  C_NB,          // bins of this step's records
  C_RBINS,       // bins summed by k_reduce (with records)
  C_RSLICES,     // slices summed (a bin whose keys overflow the table is summed in several)
  C_RMAX,        // most records in one bin
  C_HIST_N,      // 32 bins: probe levels by floor(log2 of their out-edge count)
  C_HIST_E = C_HIST_N + 32,  // 32 bins: out-edges of those levels
  // entries and chunks of the frontier lists: kSubLists counters per parity
  C_LIST = C_HIST_E + 32,
  C_CHUNK = C_LIST + 2 * kSubLists,
  C_COUNT = C_CHUNK + 2 * kSubLists
};

struct QueryOut {
  double* scores = nullptr;  // n (single-source) or k (top-k); host or device
  int32_t* nodes = nullptr;  // k (top-k)
  double* flip = nullptr;    // the query's near-threshold allowance (host or device)
  // sparse single-source output (cap >= 0): ascending nonzero entries
  int64_t cap = -1;
  int64_t* count = nullptr;  // host
};

// Output selection (select.hip).  Buffers grow on demand and are reused.
struct SelectBufs {
  DevBuf state, keys, ids;
  unsigned long long h_total = 0;
};

// A persistent set of device buffers that runs the level steps of every
// admitted query: P probe slots, a ring of pending probes, a pool of tree
// regions and per-query records with FP64 accumulators.
struct Session {
  int32_t n = 0;
  int P = 0;
  int qmax = 0;
  int sh = 0;               // smallest bin shift of the records (at most kMaxBins bins)
  uint64_t list_cap = 0, chunk_cap = 0, rec_cap = 0, list_soft = 0;  // lists: all sub-lists together
  uint64_t tree_pool = 0;   // entries
  uint64_t ring_cap = 0;    // power of two
  DevBuf slots, has_next, pull_flag, was_paused, slot_edges, slot_cnt, cost, counters;
  DevBuf l_sn[2], l_val[2], l_row[2], l_chunk[2];  // frontier lists by step parity
  DevBuf rec, seg, part;                           // records, bin segments, per-slot partial sums
  bool dense_on = false;                           // dense lanes allocated
  bool pull = false;                               // levels may be pulled: steps run the dense pass
  DevBuf mat[2], rowmap[2], npart, lane_slot, dense_ver;  // dense frontier lanes
  DevBuf qrec, thr, remaining, done_ring, qbound, acc, lq, flip;
  DevBuf keys, t_parent, t_node, t_depth, t_query, t_weight, ring, ring_k;
  // Section 4.4: out-edges of dense-lane frontiers (per slot), and per tree
  // node the walks through it (t_walks[t_woff[t] - weight .. t_woff[t]))
  DevBuf hyb_edges, t_woff, t_walks, wcount;
  DevBuf out_ids, out_scores;
  DevBuf m_keys[2], m_vals[2], m_list, m_ctr;  // merged probing
  SelectBufs sel;
  uint64_t* h_ctr = nullptr;  // pinned mirror of the counters
  uint64_t steps = 0;         // level steps launched (parity of the lists)
  hipGraphExec_t step_pair = nullptr;  // captured even + odd level step
  bool pair_dense = false;             // whether the captured steps include the dense pass
  // host bookkeeping
  std::vector<int> free_recs;
  std::vector<QueryDev> h_rec;
  // walk-bound read-back of session_begin (pinned, qmax entries) and the
  // event that marks it complete
  unsigned long long* h_qbound = nullptr;
  int h_qbound_n = 0;
  hipEvent_t begin_ev = nullptr;
  bool begin_pending = false;
  std::vector<GraphVersion*> rec_version;
  std::vector<std::pair<uint64_t, uint64_t>> tree_free;  // [start, len) free regions
  std::vector<std::pair<uint64_t, uint64_t>> rec_tree;   // region of each record
  uint64_t ring_outstanding = 0;  // probe bound of admitted, unfinished queries
  std::vector<uint64_t> rec_ring;
};

struct ps_ctx {
  int refs = 1;          // the caller's handle + one per live graph
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool timing = false;
  Session* sess = nullptr;
  SelectBufs sel;                          // ps_select_topk
  DevBuf sel_in, sel_ids, sel_scores;
  ps_stats last{};
  std::vector<hipEvent_t> ev_pool;
  std::mutex mu;
};

// Drops one reference; the context is freed with the last one.
void ctx_release(ps_ctx* c);

// Session lifecycle (engine.hip).  session_ensure (re)allocates when the
// requested shape exceeds the current one; only while no query is admitted.
ps_status session_ensure(ps_ctx* ctx, int32_t n, uint64_t m_cap, int P, int qmax, uint64_t tree_pool,
                         uint64_t ring_cap);
// Prints which frontier capacity guard tripped (counters as read back).
void report_overflow(const Session* s, const uint64_t* h);
// Clears the capacity-guard flag (stream-ordered).
void session_clear_guard(Session* s, hipStream_t st);
void session_free(Session* s);
int session_slots_for(int32_t n, int opt);
// Admission, phase 1: takes records for the queries (all reading graph
// version gv) and queues a pass over their walks that sizes each tree; it
// does not wait for it.  One such pass may be outstanding at a time.
ps_status session_begin(ps_ctx* ctx, ps_graph* g, GraphVersion* gv, const std::vector<QueryRun>& qs,
                        std::vector<int>* recs);
// The tree-size bounds of the records of the last session_begin, once its
// walk pass has finished: waits for it (wait) or reports *ready = false.
ps_status session_bounds(ps_ctx* ctx, const std::vector<int>& recs, std::vector<uint64_t>* bounds, bool wait,
                         bool* ready);
// Grows the tree pool and the ring to hold the trees of records recs; only
// while no other query is admitted.
ps_status session_fit_trees(ps_ctx* ctx, const std::vector<int>& recs, const std::vector<uint64_t>& bounds);
// Admission, phase 2: tree regions, tree construction, probes queued.
// PS_ERR_BUSY when tree or ring space is short.
ps_status session_build(ps_ctx* ctx, const std::vector<int>& recs, const std::vector<uint64_t>& bounds);
// Releases a record whose tree was never built.
void session_abandon(ps_ctx* ctx, ps_graph* g, int r);
// Launches `count` level steps (timings added when the pointers are given
// and the context times launches).
ps_status session_steps(ps_ctx* ctx, uint64_t count, double* expand_ms, double* pull_ms);
// Finalises record r (divide by n_r, s(u,u) = 1, top-k), copies its result
// to `out` on the context stream and frees the record.
ps_status session_finish(ps_ctx* ctx, ps_graph* g, int r, const QueryRun& q, const QueryOut& out);

// Copies device bytes to a host or device destination (stream-ordered).
ps_status copy_out(void* dst, const void* src, size_t bytes, hipStream_t st);

// Output selection (select.hip).
// The k nodes v != u of largest s[v] (ties to the smaller id), in that order,
// with their values; 1 <= k <= n - 1.  Asynchronous on `st`.
ps_status select_topk(SelectBufs& b, const double* s, int32_t n, int32_t u, int32_t k, int32_t* out_ids,
                      double* out_s, hipStream_t st);
// Looks up, once per device and with that device current, the device
// address of the scratch array of ps_select_topk_noalloc.
ps_status select_scratch_init(int device);
// The first `cap` nodes with s[v] != 0 in ascending id order, with their
// values; `*total` receives the count of all of them (synchronises `st`).
ps_status select_nonzero(SelectBufs& b, const double* s, int32_t n, int64_t cap, int32_t* out_ids, double* out_s,
                         int64_t* total, hipStream_t st);
ps_status make_query_run(const ps_graph* g, int32_t u, int32_t k, double c, double eps, double delta,
                         uint64_t seed, const ps_options* opt, QueryRun* q);

// Runs a set of queries to completion on one graph version and writes every
// result (ps_single_source, ps_topk, ps_batch).
ps_status engine_run(ps_ctx* ctx, ps_graph* g, GraphVersion* gv, const std::vector<QueryRun>& qs,
                     const std::vector<QueryOut>& outs, int slots_opt, int64_t pull_opt);
uint64_t pull_threshold(int64_t m, int64_t opt);
// One query by merged probing (merged.hip): walks, tree, then one expansion
// per tree node; adds its work to *st and writes the result.
ps_status engine_merged(ps_ctx* ctx, ps_graph* g, GraphVersion* gv, const QueryRun& q, const QueryOut& out,
                        ps_stats* st);
ps_status session_set_pull(ps_ctx* ctx, uint64_t threshold);

ps_status engine_walks(ps_ctx* ctx, GraphVersion* gv, int32_t n, const QueryRun& q, int64_t k_begin,
                       int64_t count, int32_t* nodes, int32_t* lens);


ps_status derive_params(int32_t n, double c, double eps, double delta, const ps_options* opt,
                        ps_params* out);
