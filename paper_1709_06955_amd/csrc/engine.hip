// ProbeSim query engine: sqrt(c)-walks, reverse reachability tree, PROBE
// level expansion with both pruning rules, FP64 accumulation, top-k.
//
// A session holds the device state that level steps run on; queries are
// admitted into it at any time (continuous batching) and leave it when their
// last probe finishes.
//
//   admission    k_walk_bound samples every walk of the admitted queries once
//                to size their trees (sum of len-1); k_walk_tree samples the
//                same walks again (Philox is counter-based) and inserts every
//                prefix (u_1..u_i), i >= 2, into the query's hash-addressed
//                tree region (Alg. 3).  The hash slot of a prefix is its tree
//                node id, its weight counts the walks sharing it, and each new
//                tree node is appended to the ring of pending probes.
//   level step   every tree node is one PROBE (Alg. 2).  Probes run in P
//                slots; k_sched (one workgroup) advances every slot by one
//                iteration, retires finished probes (a query is complete when
//                its last probe retires) and hands free slots the next
//                pending probes; k_prep reads and clears the scores of the
//                listed frontier entries, applies Rule 2 and records the
//                surviving rows; k_expand pushes scores along out-edges,
//                load-balanced per edge over tiles of entries (long rows in
//                fixed-size chunks).  Each slot owns a dense vector of exact
//                score sums (64-bit integers on the grid 2^-62) per level
//                parity; the atomic add that turns an entry nonzero appends
//                (slot, node) to the next frontier list, so frontiers stay
//                sparse lists while the sums stay exact and independent of
//                the order of the adds.  A probe's last level adds weight *
//                score straight into the query's FP64 estimate.
//   switch       for a hybrid query (Section 4.4) k_pick stops a
//                deterministic probe whose level about to be expanded keeps
//                more than c0 * w * n out-edges and queues one randomized
//                probe (Alg. 4) per walk through its tree node; the walks of
//                each tree node are listed at admission (k_walk_offsets,
//                k_walk_lists), and k_hyb_count measures the levels of
//                probes held in dense columns.
//   finish       k_finalize divides by n_r and sets s(u,u) = 1; top-k sorts.

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "ps_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kSchedThreads = 1024;
constexpr int kSlotsPerSchedThread = 4;  // P <= 4096
constexpr uint32_t kBigDeg = 1024;       // longer rows: one wavefront per kChunk edges
constexpr uint32_t kChunk = 512;
constexpr uint32_t kBigFlag = 0x80000000u;
constexpr int kTile = 1024;              // listed entries per workgroup tile in k_expand
constexpr int kWaveBuf = 512;            // staged new frontier entries per wavefront
constexpr int kLanes = 64;               // dense frontier columns (one wavefront lane each)
constexpr unsigned long long kEmpty = ~0ull;
constexpr int kStepGrid = 2048;          // 8 workgroups per CU for the step kernels

// ------------------------------------------------------------- Philox ----

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the Weyl key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint32_t alo = 0xD2511F53u * x.x, ahi = __umulhi(0xD2511F53u, x.x);
    const uint32_t blo = 0xCD9E8D57u * x.z, bhi = __umulhi(0xCD9E8D57u, x.z);
    x = make_uint4(bhi ^ x.y ^ k.x, blo, ahi ^ x.w ^ k.y, alo);
  }
  return x;
}

// One move of a sqrt(c)-walk: at node v (index t of walk k) the walk stops
// when v has no in-neighbour or Philox word 0 < t_stop; otherwise it goes to
// in-neighbour floor(r64 * |I(v)| / 2^64) of v's ascending in-row.
__device__ __forceinline__ int32_t walk_move(int32_t v, uint32_t k, uint32_t t, const QueryDev& q) {
  const uint4 w = philox4x32_10(make_uint4(k, t, (uint32_t)q.u, 0u),
                                make_uint2((uint32_t)q.seed, (uint32_t)(q.seed >> 32)));
  const uint2 row = q.in_rows[v];
  if (row.y == 0u || w.x < q.t_stop) return -1;
  const uint64_t r = ((uint64_t)w.z << 32) | w.y;
  const uint32_t idx = (uint32_t)__umul64hi(r, (uint64_t)row.y);
  return q.in_col[row.x + idx];
}

// Record of global walk g in a walk launch over records lq[0..nl).
__device__ __forceinline__ int find_record(const QueryDev* __restrict__ qr, const int32_t* __restrict__ lq, int nl,
                                           int64_t g) {
  int lo = 0, hi = nl - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (qr[lq[mid]].walk_base <= g) lo = mid; else hi = mid - 1;
  }
  return lq[lo];
}

// ------------------------------------------------------ wave utilities ----

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Reserves one output position per lane with `flag` set; one atomic per wave.
// Every lane active at the call takes part.
__device__ __forceinline__ unsigned long long wave_reserve(bool flag, unsigned long long* counter,
                                                           unsigned long long* leader_total) {
  const unsigned long long mask = __ballot(flag);
  if (!mask) return 0;
  const int lane = lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  const unsigned long long rank = __popcll(mask & ((1ull << lane) - 1ull));
  unsigned long long base = 0;
  if (lane == leader) {
    base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    if (leader_total) *leader_total += __popcll(mask);
  }
  base = __shfl(base, leader, 64);
  return base + rank;
}

// Inclusive prefix sum over all 64 lanes (every lane must be active).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 33;
  z *= 0xff51afd7ed558ccdull;
  z ^= z >> 33;
  z *= 0xc4ceb9fe1a85ec53ull;
  z ^= z >> 33;
  return z;
}

// ------------------------------------------------------------- walks ----

__global__ void k_walk_bound(const QueryDev* __restrict__ qr, const int32_t* __restrict__ lq, int nl, int64_t total,
                             unsigned long long* __restrict__ qbound, unsigned long long* __restrict__ ctr) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int r = -1;
  unsigned long long extra = 0, nodes = 0;
  if (g < total) {
    r = find_record(qr, lq, nl, g);
    const QueryDev q = qr[r];
    const uint32_t k = (uint32_t)(q.walk_begin + (g - q.walk_base));
    int32_t v = q.u;
    int len = 1;
    for (uint32_t t = 0; len < q.L; ++t) {
      const int32_t nx = walk_move(v, k, t, q);
      if (nx < 0) break;
      v = nx;
      ++len;
    }
    extra = (unsigned long long)(len - 1);
    nodes = (unsigned long long)len;
  }
  // one atomic per wavefront when all its walks belong to one query
  const int r0 = __shfl(r, 0, 64);
  const bool uniform = __ballot(r != r0 && r >= 0) == 0ull;
  const unsigned long long wn = wave_sum(nodes);
  if (uniform) {
    const unsigned long long we = wave_sum(extra);
    if (lane_id() == 0 && r0 >= 0 && we) atomicAdd(&qbound[r0], we);
  } else if (r >= 0 && extra) {
    atomicAdd(&qbound[r], extra);
  }
  if (lane_id() == 0 && wn) atomicAdd(&ctr[C_WALK_NODES], wn);
}

__global__ void k_walk_export(QueryDev q, int64_t k_begin, int64_t count, int32_t* __restrict__ nodes,
                              int32_t* __restrict__ lens) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const uint32_t k = (uint32_t)(k_begin + g);
  int32_t* row = nodes + g * q.L;
  int32_t v = q.u;
  int len = 1;
  row[0] = v;
  for (uint32_t t = 0; len < q.L; ++t) {
    const int32_t nx = walk_move(v, k, t, q);
    if (nx < 0) break;
    v = nx;
    row[len++] = v;
  }
  lens[g] = len;
  for (int i = len; i < q.L; ++i) row[i] = -1;
}

// Inserts key = (parent tree node << 32 | graph node) by linear probing in the
// region [base, base + mask + 1).  The slot is the tree node id.  A region
// holds at least twice as many slots as the query has keys, so the probe
// sequence always ends.
__device__ __forceinline__ uint32_t tree_insert(unsigned long long* __restrict__ keys, uint64_t base, uint64_t mask,
                                                unsigned long long key, bool& inserted) {
  uint64_t s = mix64(key) & mask;
  inserted = false;
  while (true) {
    unsigned long long* slot = keys + base + s;
    const unsigned long long cur = *slot;
    if (cur == key) return (uint32_t)(base + s);
    if (cur == kEmpty) {
      const unsigned long long prev = atomicCAS(slot, kEmpty, key);
      if (prev == kEmpty) {
        inserted = true;
        return (uint32_t)(base + s);
      }
      if (prev == key) return (uint32_t)(base + s);
    }
    s = (s + 1) & mask;
  }
}

struct TreeArgs {
  const QueryDev* qr;
  const int32_t* lq;
  int nl;
  int64_t total;
  uint64_t root_base;  // tree id of the root of record r is root_base + r
  unsigned long long* keys;
  int32_t* t_parent;
  int32_t* t_node;
  int32_t* t_depth;
  int32_t* t_query;
  int32_t* t_weight;
  int32_t* ring;
  int32_t* ring_k;  // walk index of each pending probe (randomized queries)
  uint64_t ring_mask;
  unsigned long long* remaining;
  unsigned long long* ctr;
};

// Alg. 3, tree construction: walk k of query q descends from q's root through
// one tree node per prefix, creating it on first visit (and queueing its
// probe) and adding one to its weight.
__global__ void k_walk_tree(TreeArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.total) return;
  const int r = find_record(a.qr, a.lq, a.nl, g);
  const QueryDev q = a.qr[r];
  const uint32_t k = (uint32_t)(q.walk_begin + (g - q.walk_base));
  uint32_t parent = (uint32_t)(a.root_base + r);
  int32_t v = q.u;
  int len = 1;
  for (uint32_t t = 0; len < q.L; ++t) {
    const int32_t nx = walk_move(v, k, t, q);
    if (nx < 0) break;
    v = nx;
    ++len;
    const unsigned long long key = ((unsigned long long)parent << 32) | (uint32_t)v;
    bool inserted;
    const uint32_t id = tree_insert(a.keys, q.tree_base, q.tree_mask, key, inserted);
    if (inserted) {
      a.t_parent[id] = (int32_t)parent;
      a.t_node[id] = v;
      a.t_depth[id] = len;
      a.t_query[id] = r;
    }
    // a deterministic probe per tree node; a randomized one per walk and
    // prefix (their draws differ per walk, so sharing saves nothing).  The
    // ring's walk index marks a randomized probe; -1 a deterministic one.
    if (inserted || q.randomized) {
      atomicAdd(&a.remaining[r], 1ull);
      atomicAdd(&a.ctr[C_LEVELS], (unsigned long long)(len - 1));
      const unsigned long long pos = atomicAdd(&a.ctr[C_TAIL], 1ull);
      a.ring[pos & a.ring_mask] = (int32_t)id;
      a.ring_k[pos & a.ring_mask] = q.randomized ? (int32_t)k : -1;
    }
    atomicAdd(&a.t_weight[id], 1);
    parent = id;
  }
}

// Section 4.4, one hybrid query: gives every tree node of its region a range
// of t_walks as long as its weight (ranges in hash order, which only decides
// where a node's walks are kept); t_woff[t] is left at the range's start.
// The weights sum to at most half the region, so the ranges stay inside it.
__global__ void k_walk_offsets(const unsigned long long* __restrict__ keys, const int32_t* __restrict__ t_weight,
                               uint32_t* __restrict__ t_woff, uint64_t base, uint64_t cap,
                               unsigned long long* __restrict__ count) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap || keys[base + i] == kEmpty) return;
  t_woff[base + i] = (uint32_t)(base + atomicAdd(count, (unsigned long long)t_weight[base + i]));
}

// Section 4.4: samples the walks of the hybrid queries again (Philox is
// counter-based) and files walk k under every tree node it passes.  Every
// key is present, so the tree lookup inserts nothing.  Afterwards t_woff[t]
// is one past t's range, which starts at t_woff[t] - weight.
__global__ void k_walk_lists(TreeArgs a, uint32_t* __restrict__ t_woff, int32_t* __restrict__ t_walks) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.total) return;
  const int r = find_record(a.qr, a.lq, a.nl, g);
  const QueryDev q = a.qr[r];
  if (!q.hybrid) return;
  const uint32_t k = (uint32_t)(q.walk_begin + (g - q.walk_base));
  uint32_t parent = (uint32_t)(a.root_base + r);
  int32_t v = q.u;
  int len = 1;
  for (uint32_t t = 0; len < q.L; ++t) {
    const int32_t nx = walk_move(v, k, t, q);
    if (nx < 0) break;
    v = nx;
    ++len;
    bool inserted;
    const uint32_t id = tree_insert(a.keys, q.tree_base, q.tree_mask, ((unsigned long long)parent << 32) | (uint32_t)v,
                                    inserted);
    t_walks[atomicAdd(&t_woff[id], 1u)] = (int32_t)k;
    parent = id;
  }
}

__global__ void k_init_roots(const QueryDev* __restrict__ qr, const int32_t* __restrict__ lq, int nl,
                             uint64_t root_base, int32_t* t_parent, int32_t* t_node, int32_t* t_depth,
                             int32_t* t_query) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  const int r = lq[i];
  t_parent[root_base + r] = -1;
  t_node[root_base + r] = qr[r].u;
  t_depth[root_base + r] = 1;
  t_query[root_base + r] = r;
}

template <typename T>
__global__ void k_fill(T* p, T v, uint64_t cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

__global__ void k_reset_slots(Slot* slots, int32_t* has_next, int P) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= P) return;
  Slot st{};
  st.probe = -1;
  st.lane = -1;
  slots[s] = st;
  has_next[s] = 0;
}

// Graph version whose in-rows the dense pass reads (all dense lanes share it).
struct DenseVer {
  const uint2* out_rows;  // out-degrees of the targets (Section 4.4 counts)
  const uint2* in_rows;
  const int32_t* in_col;
  const float* inv_indeg;
  const int32_t* heavy_nodes;
  const int2* heavy_chunks;
  const unsigned long long* heavy_cnt;
};

__global__ void k_reset_lanes(int32_t* lane_slot) {
  if (threadIdx.x < kLanes) lane_slot[threadIdx.x] = -1;
}

// ------------------------------------------------------- level steps ----

// Probe scores.  The scores of inner levels are FP32 numbers.  The
// contributions that make up a level are summed exactly, as 64-bit integers
// on the grid 2^-62 (a level's scores never exceed 1), so no order of atomic
// adds changes a bit; a level's FP32 score is its sum rounded to nearest.
// Rule 2 then compares FP32 numbers only, and the same query gives the same
// result alone, in a batch, pushed or pulled.
__device__ __forceinline__ long long to_grid(float c) { return __float2ll_rn(c * 0x1p62f); }
__device__ __forceinline__ float grid_f32(long long q) { return __ll2float_rn(q) * 0x1p-62f; }
__device__ __forceinline__ double grid_f64(long long q) { return (double)q * 0x1p-62; }
constexpr long long kGridOne = 1ll << 62;

struct SchedArgs {
  int P;
  int32_t n;
  int qmax;
  Slot* slots;
  int32_t* has_next;
  const int32_t* ring;
  const int32_t* ring_k;
  uint64_t ring_mask;
  const int32_t* t_parent;
  const int32_t* t_node;
  const int32_t* t_depth;
  const int32_t* t_query;
  const int32_t* t_weight;
  const QueryDev* qr;
  const float* thr_tab;
  unsigned long long* remaining;
  int32_t* done_ring;
  long long* dense_cur;
  int2* list_cur;
  uint64_t list_cap;
  unsigned long long* slot_edges;
  int32_t* lane_slot;
  unsigned long long* ctr;
  int cur;
};

// One workgroup: advances every slot by one PROBE iteration, retires probes
// whose last level (i-2) ran or whose frontier Rule 2 emptied, and hands free
// slots the next pending probes in ring order.  A new probe on (u_1..u_i)
// starts with H_0 = {u_i: 1}.
__global__ void __launch_bounds__(kSchedThreads) k_sched(SchedArgs a) {
  __shared__ uint32_t wave_tot[kSchedThreads / 64];
  __shared__ unsigned long long s_head, s_avail;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid >> 6;
  if (tid == 0) {
    a.ctr[C_SMALL] = 0;
    a.ctr[C_CHUNK] = 0;
    a.ctr[C_LIST0 + (a.cur ^ 1)] = 0;
    a.ctr[C_NZROWS0 + (a.cur ^ 1)] = 0;  // k_dense rewrites that matrix this step
    s_head = a.ctr[C_HEAD];
    s_avail = a.ctr[C_TAIL] - s_head;
  }
  __syncthreads();
  // Slots are updated field by field in place (a whole Slot per register set
  // would spill).
  bool need[kSlotsPerSchedThread];
  uint32_t cnt = 0;
#pragma unroll
  for (int r = 0; r < kSlotsPerSchedThread; ++r) {
    const int s = tid * kSlotsPerSchedThread + r;
    need[r] = false;
    if (s >= a.P) continue;
    Slot& S = a.slots[s];
    if (S.probe >= 0) {
      if (S.last || !a.has_next[s]) {
        const int q = S.query;
        if (atomicAdd(&a.remaining[q], ~0ull) == 1ull) {  // last probe of the query
          const unsigned long long pos = atomicAdd(&a.ctr[C_DONE], 1ull);
          a.done_ring[pos % (unsigned long long)a.qmax] = q;
        }
        if (S.lane >= 0) a.lane_slot[S.lane] = -1;  // dense column free again
        S.probe = -1;
        S.lane = -1;
        need[r] = true;
      } else {
        S.level = S.level + 1;
        S.cursor = a.t_parent[S.cursor];
      }
    } else {
      need[r] = true;
    }
    a.has_next[s] = 0;
    a.slot_edges[s] = 0;
    cnt += need[r] ? 1u : 0u;
  }
  // Exclusive scan of the per-thread counts of free slots.
  const uint32_t incl = wave_incl_scan(cnt);
  if (lane == 63) wave_tot[wv] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int w = 0; w < kSchedThreads / 64; ++w) {
    if (w < wv) before += wave_tot[w];
    total += wave_tot[w];
  }
  unsigned long long rank = before + incl - cnt;
  const unsigned long long head = s_head, avail = s_avail;
#pragma unroll
  for (int r = 0; r < kSlotsPerSchedThread; ++r) {
    const int s = tid * kSlotsPerSchedThread + r;
    if (s >= a.P) continue;
    Slot& S = a.slots[s];
    if (need[r]) {
      if (rank < avail) {
        const uint64_t rp = (head + rank) & a.ring_mask;
        const int32_t t = a.ring[rp];
        const int q = a.t_query[t];
        const QueryDev& Q = a.qr[q];
        const int32_t wk = a.ring_k[rp];
        const int mode = wk >= 0;  // a randomized probe of walk wk's prefix
        const double w = mode ? 1.0 : (double)a.t_weight[t];
        S.probe = t;
        S.lane = -1;
        S.level = 0;
        S.depth = a.t_depth[t];
        S.cursor = a.t_parent[t];
        S.query = q;
        S.mode = mode;
        S.wk = mode ? (uint32_t)wk : 0u;
        S.t_sc = Q.t_sc;
        S.key2 = Q.key2;
        S.w = w;
        S.sc = Q.sc;
        S.out_rows = Q.out_rows;
        S.out_col = Q.out_col;
        S.inv_indeg = Q.inv_indeg;
        S.acc = Q.acc;
        S.in_rows = Q.in_rows;
        S.in_col = Q.in_col;
        S.heavy_nodes = Q.heavy_nodes;
        S.heavy_chunks = Q.heavy_chunks;
        S.heavy_cnt = Q.heavy_cnt;
        S.flip = Q.flip;
        S.flip_unit = mode ? 0.0 : Q.flip_unit * w;
        // Section 4.4: a hybrid query's deterministic probe of weight w
        // switches past c0 * w * n out-edges
        S.hyb_thr = !mode && Q.hybrid ? (Q.c0 * w) * (double)a.n : -1.0;
        const int32_t x = a.t_node[t];
        const unsigned long long pos = atomicAdd(&a.ctr[C_LIST0 + a.cur], 1ull);
        if (pos < a.list_cap) {
          // H_0 = {u_i: 1} (a randomized probe's sets are its lists alone)
          if (!mode) a.dense_cur[(size_t)s * a.n + x] = kGridOne;
          a.list_cur[pos] = make_int2(s, x);
        } else {
          atomicOr(&a.ctr[C_OVERFLOW], 1ull);
        }
        atomicAdd(&a.ctr[C_LEVEL0], 1ull);
      }
      ++rank;
    }
    const int32_t probe = S.probe;
    if (probe >= 0) {
      const int level = S.level, depth = S.depth, q = S.query;
      const int e = depth - level - 1;  // iterations left, i-j-1 >= 1
      S.thr = a.thr_tab[q * PS_MAX_WALK_LEN + e];
      S.thr_next = e > 1 ? a.thr_tab[q * PS_MAX_WALK_LEN + e - 1] : 0.0f;
      S.excl = a.t_node[S.cursor];
      S.last = level == depth - 2;
    }
  }
  if (tid == 0) a.ctr[C_HEAD] = head + (total < avail ? total : avail);
}

// Reads the scores of the listed entries and applies Rule 2 (remove x when
// Score(x) * sqrt(c)^(i-j-1) <= eps_p, i.e. Score(x) <= thr).  Removed
// entries and entries without out-edges are cleared at once; the others keep
// their score in the dense vector (a pulled slot reads it there) and get
// their out-row and sqrt(c) * Score(x) recorded.  Rows longer than kBigDeg are
// also cut into kChunk-edge chunks for the wavefront-per-chunk part of
// k_expand (marked with the top bit of the length so that the tile part skips
// them).  Per slot, the out-degrees of its kept entries are summed: that
// decides between pushing and pulling the slot's level.  A randomized probe
// (Alg. 4) lists exactly the members of its set: they are kept as listed.
__global__ void __launch_bounds__(kBlock) k_prep(int32_t n, const Slot* __restrict__ slots,
                                                 const int2* __restrict__ list_cur, long long* __restrict__ dense_cur,
                                                 float* __restrict__ item_val, uint2* __restrict__ item_row,
                                                 int2* __restrict__ chunk_list, uint64_t list_cap, uint64_t chunk_cap,
                                                 unsigned long long* __restrict__ slot_edges,
                                                 unsigned long long* __restrict__ ctr, int cur) {
  // after an overflow the counter runs past the list; never read beyond it
  const unsigned long long cnt = min(ctr[C_LIST0 + cur], (unsigned long long)list_cap);
  const int lane = lane_id();
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long kept = 0, pruned = 0, edges = 0, near = 0;
  for (uint64_t i0 = gtid - lane; i0 < cnt; i0 += stride) {
    const uint64_t i = i0 + lane;
    uint32_t nch = 0;
    int32_t myslot = -1;
    unsigned long long mydeg = 0;
    if (i < cnt) {
      const int2 it = list_cur[i];
      long long* d = dense_cur + (size_t)it.x * n + it.y;
      const Slot& sl = slots[it.x];
      uint2 row = make_uint2(0u, 0u);
      bool keep = true;  // Alg. 4: a randomized probe lists exactly its members
      float val = 0.0f;
      if (!sl.mode) {
        val = grid_f32(*d);
        if (fabsf(val - sl.thr) <= 1e-5f * sl.thr) {  // FP32 rounding may decide this test
          ++near;
          unsafeAtomicAdd(sl.flip, sl.flip_unit);
        }
        keep = val > sl.thr;
      }
      if (keep) {
        ++kept;
        row = sl.out_rows[it.y];
        edges += row.y;
        item_val[i] = val * sl.sc;
        myslot = it.x;
        mydeg = row.y;
        if (row.y > kBigDeg) {
          nch = (row.y + kChunk - 1) / kChunk;
          row.y |= kBigFlag;
        }
      } else {
        ++pruned;
      }
      if (!sl.mode && !row.y) *d = 0;
      item_row[i] = row;
    }
    // segmented sum of out-degrees per slot over the wavefront
    for (;;) {
      const unsigned long long live = __ballot(myslot >= 0 && mydeg > 0);
      if (!live) break;
      const int leader = __ffsll((long long)live) - 1;
      const int32_t s0 = __shfl(myslot, leader, 64);
      const bool mine = myslot == s0;
      const unsigned long long sum = wave_sum(mine ? mydeg : 0ull);
      if (lane == leader) atomicAdd(&slot_edges[s0], sum);
      if (mine) myslot = -1;
    }
    const uint32_t incl = wave_incl_scan(nch);
    const uint32_t total = __shfl(incl, 63, 64);
    if (total) {
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(&ctr[C_CHUNK], (unsigned long long)total);
      base = __shfl(base, 0, 64);
      const uint64_t first = base + incl - nch;
      if (first + nch <= chunk_cap) {
        for (uint32_t c = 0; c < nch; ++c) chunk_list[first + c] = make_int2((int32_t)i, (int32_t)c);
      } else if (nch) {
        atomicOr(&ctr[C_OVERFLOW], 2ull);
      }
    }
  }
  kept = wave_sum(kept);
  pruned = wave_sum(pruned);
  edges = wave_sum(edges);
  near = wave_sum(near);
  if (lane == 0) {
    if (near) atomicAdd(&ctr[C_NEAR], near);
    if (kept) atomicAdd(&ctr[C_KEPT], kept);
    if (pruned) atomicAdd(&ctr[C_PRUNED], pruned);
    if (edges) atomicAdd(&ctr[C_EDGES], edges);
  }
}

struct PickArgs {
  int P;
  unsigned long long* slot_edges;
  unsigned long long* hyb_edges;
  Slot* slots;
  int32_t* pull_flag;
  int32_t* lane_slot;
  DenseVer* dv;
  // Section 4.4 switches
  const int32_t* t_weight;
  const uint32_t* t_woff;
  const int32_t* t_walks;
  int32_t* ring;
  int32_t* ring_k;
  uint64_t ring_mask;
  unsigned long long* remaining;
  unsigned long long* ctr;
};

// Section 4.4: the deterministic probe in slot S stops (k_expand drops its
// level, so it retires at the next step) and each walk through its tree node
// is queued for a randomized probe of the same prefix.  A dense column it
// held is free again; this step's pass writes that column as zeros.
__device__ void switch_probe(const PickArgs& a, Slot& S) {
  if (S.lane >= 0) {
    a.lane_slot[S.lane] = -1;
    S.lane = -1;
  }
  const int32_t t = S.probe;
  const uint32_t w = (uint32_t)a.t_weight[t];
  const uint32_t first = a.t_woff[t] - w;
  atomicAdd(&a.remaining[S.query], (unsigned long long)w);  // before the switched probe retires
  atomicAdd(&a.ctr[C_LEVELS], (unsigned long long)w * (unsigned long long)(S.depth - 1));
  atomicAdd(&a.ctr[C_SWITCH], 1ull);
  const unsigned long long pos = atomicAdd(&a.ctr[C_TAIL], (unsigned long long)w);
  // admission reserves ring room for every walk of a hybrid query; a guard
  if (pos + w - a.ctr[C_HEAD] > a.ring_mask + 1) atomicOr(&a.ctr[C_OVERFLOW], 16ull);
  for (uint32_t m = 0; m < w; ++m) {
    a.ring[(pos + m) & a.ring_mask] = t;
    a.ring_k[(pos + m) & a.ring_mask] = a.t_walks[first + m];
  }
}

// One workgroup.  First the switch of Section 4.4 for hybrid queries: a
// deterministic probe switches when the level it is about to expand has more
// kept out-edges than c0 * w * n (k_prep's sum for a sparse frontier, the
// count of the last dense pass for a dense column).  Then it moves sparse
// slots whose kept entries have at least ctr[C_PULL_T] out-edges into free
// dense columns, as long as they read the graph version the dense pass uses
// (fixed by the columns active at the start, or by the first slot moved).
// Their entries are scattered into the dense matrix by k_expand this step.
// A column freed by a switch is handed out at the next step only.  Also sets
// the column range of this step's dense pass and records the version's
// arrays for it.
__global__ void __launch_bounds__(kSchedThreads) k_pick(PickArgs a) {
  __shared__ int32_t s_free[kLanes];
  __shared__ uint32_t s_nfree, s_ncand, s_fhi;
  __shared__ unsigned long long s_ver;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_nfree = 0;
    s_ncand = 0;
    s_fhi = 0;
    s_ver = 0ull;
  }
  __syncthreads();
  if (tid < kLanes) {  // one wavefront: free columns listed lowest first
    const int32_t ls = a.lane_slot[tid];
    const unsigned long long freem = __ballot(ls < 0);
    if (ls < 0) s_free[__popcll(freem & ((1ull << tid) - 1ull))] = tid;
    else s_ver = (unsigned long long)a.slots[ls].in_rows;  // all active columns share it
    if (tid == 0) s_nfree = (uint32_t)__popcll(freem);
  }
  __syncthreads();
  unsigned long long* ctr = a.ctr;
  const unsigned long long T = ctr[C_PULL_T];
  for (int s = tid; s < a.P; s += blockDim.x) {
    Slot& S = a.slots[s];
    unsigned long long e = a.slot_edges[s];
    const unsigned long long he = a.hyb_edges[s];
    if (he) a.hyb_edges[s] = 0;
    int32_t flag = 0;
    if (S.probe >= 0 && S.hyb_thr >= 0.0 && (double)(S.lane >= 0 ? he : e) > S.hyb_thr) {
      if (S.lane >= 0) atomicMax(&s_fhi, (uint32_t)S.lane + 1u);
      switch_probe(a, S);
      flag = 2;
      if (e) atomicAdd(&ctr[C_EDGES_UNPUSHED], e);  // k_prep counted them
      e = 0;
    }
    if (e) {
      const int b = 63 - __clzll((long long)e);
      atomicAdd(&ctr[C_HIST_N + b], 1ull);
      atomicAdd(&ctr[C_HIST_E + b], e);
      if (e >= T && S.lane < 0 && !S.mode) {
        const unsigned long long ver = (unsigned long long)S.in_rows;
        const unsigned long long old = atomicCAS(&s_ver, 0ull, ver);
        if ((old == 0ull ? ver : old) == ver) {
          const uint32_t k = atomicAdd(&s_ncand, 1u);
          if (k < s_nfree) {
            const int32_t lane = s_free[k];
            S.lane = lane;
            a.lane_slot[lane] = s;
            flag = 1;
            atomicAdd(&ctr[C_EDGES_UNPUSHED], e);  // pulled, not pushed
          }
        }
      }
    }
    a.pull_flag[s] = flag;
  }
  __syncthreads();
  if (tid < kLanes) {  // the first wavefront: one lane per column
    const int32_t ls = a.lane_slot[tid];
    // columns of hybrid queries' deterministic probes with a level after
    // this one: k_hyb_count measures their next level
    const bool hyb = ls >= 0 && a.slots[ls].hyb_thr >= 0.0 && !a.slots[ls].last;
    const unsigned long long act = __ballot(ls >= 0);
    const unsigned long long hmask = __ballot(hyb);
    if (tid == 0) {
      const unsigned long long hi = act ? (unsigned long long)(64 - __clzll((long long)act)) : 0ull;
      const unsigned long long prev = ctr[C_GPREV];
      ctr[C_GHI] = hi;
      ctr[C_GW] = hi > prev ? hi : prev;
      // a column freed by a switch still holds its level in this step's
      // input matrix, which the next step writes: it counts as in use until then
      ctr[C_GPREV] = hi > s_fhi ? hi : s_fhi;
      if (act) atomicAdd(&ctr[C_PULLS], (unsigned long long)__popcll(act));
      ctr[C_HYBMASK] = hmask;
    }
    if (act && tid == __ffsll((long long)act) - 1) {  // the version's arrays, from the lowest active column
      const Slot& sl = a.slots[ls];
      a.dv->out_rows = sl.out_rows;
      a.dv->in_rows = sl.in_rows;
      a.dv->in_col = sl.in_col;
      a.dv->inv_indeg = sl.inv_indeg;
      a.dv->heavy_nodes = sl.heavy_nodes;
      a.dv->heavy_chunks = sl.heavy_chunks;
      a.dv->heavy_cnt = sl.heavy_cnt;
    }
  }
}

struct ExpandArgs {
  int32_t n;
  long long* dense_cur;
  float* mat_cur;  // dense frontier matrix (n x kLanes) of this step
  uint8_t* map_cur;  // its row map (rows given a score here are flagged)
  const int32_t* pull_flag;
  const int2* list_cur;
  const float* item_val;
  const uint2* item_row;
  const int2* chunk_list;
  const Slot* slots;
  long long* dense_next;
  int2* list_next;
  uint64_t list_cap;
  uint64_t chunk_cap;
  int32_t* has_next;
  unsigned long long* ctr;
  int cur;
  int nxt;
};

// Per-wavefront staging of new frontier entries in LDS: one global atomic per
// flush instead of one per append.  Every lane of the wavefront must call
// these together (the callers' loops are wavefront-uniform).
struct WaveBuf {
  int2* buf;   // kWaveBuf entries of this wavefront
  uint32_t n;  // entries staged (same value in every lane)
};

__device__ __forceinline__ void wave_flush(WaveBuf& wb, const ExpandArgs& a, unsigned long long& nnext) {
  if (wb.n == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int lane = lane_id();
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(&a.ctr[C_LIST0 + a.nxt], (unsigned long long)wb.n);
  base = __shfl(base, 0, 64);
  for (uint32_t k = (uint32_t)lane; k < wb.n; k += 64) {
    const unsigned long long pos = base + k;
    if (pos < a.list_cap) a.list_next[pos] = wb.buf[k];
    else atomicOr(&a.ctr[C_OVERFLOW], 4ull);
  }
  if (lane == 0) nnext += wb.n;
  wb.n = 0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void wave_append(WaveBuf& wb, bool flag, int32_t s, int32_t v, const ExpandArgs& a,
                                            unsigned long long& nnext) {
  const unsigned long long mask = __ballot(flag);
  if (!mask) return;
  const uint32_t cnt = (uint32_t)__popcll(mask);
  if (wb.n + cnt > (uint32_t)kWaveBuf) wave_flush(wb, a, nnext);
  const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane_id()) - 1ull));
  if (flag) wb.buf[wb.n + rank] = make_int2(s, v);
  wb.n += cnt;
}

// One out-edge x -> v of a listed entry of slot s: add sqrt(c)/|I(v)| *
// Score(x) to H_{j+1}[v] unless v is the excluded walk node u_{i-j-1}
// (Alg. 2); sv = fl32(Score(x) * sqrt(c)).  Returns whether (s, v) became a
// new frontier entry.
__device__ __forceinline__ bool visit_edge(const ExpandArgs& a, int32_t s, int32_t v, float sv, const Slot& sl,
                                           unsigned long long& nfinal) {
  if (v == sl.excl) return false;
  const float c = sv * sl.inv_indeg[v];
  const long long q = to_grid(c);
  if (q == 0) return false;  // below the grid
  if (sl.last) {
    unsafeAtomicAdd(&sl.acc[v], (double)c * sl.w);
    ++nfinal;
    return false;
  }
  const unsigned long long old =
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.dense_next[(size_t)s * a.n + v]), (unsigned long long)q);
  return old == 0ull;
}

// One out-edge x -> v of a member x of randomized probe slot s (Alg. 4).
// Candidate v (any out-neighbour of a member but the excluded walk node)
// draws its in-neighbour and sqrt(c) coin from Philox with counter (walk,
// i * 2^16 + j, v, 1), the same numbers whichever member reaches it; v joins
// the next set when the drawn in-neighbour is a member and the coin falls
// below sqrt(c).  The draw depends on v alone, so it is tested on the visit
// from the drawn in-neighbour itself: that visit happens exactly when the
// drawn node is a member.  Each selected v is so found once, with no marks
// and no lookups of membership.  On the probe's last level a selected v adds
// 1 to the estimate.  Returns whether v is listed for the next level.
__device__ __forceinline__ bool visit_random(const ExpandArgs& a, int32_t v, int32_t x, const Slot& sl,
                                             unsigned long long& nfinal) {
  if (v == sl.excl) return false;
  const uint4 w = philox4x32_10(make_uint4(sl.wk, ((uint32_t)sl.depth << 16) | (uint32_t)sl.level, (uint32_t)v, 1u),
                                sl.key2);
  if (w.z >= sl.t_sc) return false;  // the coin
  const uint2 row = sl.in_rows[v];   // |I(v)| >= 1: x is an in-neighbour
  const uint64_t r = ((uint64_t)w.y << 32) | w.x;
  if (sl.in_col[row.x + (uint32_t)__umul64hi(r, (uint64_t)row.y)] != x) return false;
  if (sl.last) {
    unsafeAtomicAdd(&sl.acc[v], sl.w);
    ++nfinal;
    return false;
  }
  return true;
}

// PROBE expansion.  Part 1: workgroups take tiles of kTile listed entries,
// scan their out-degrees in LDS and walk the tile's edges 256 at a time, each
// lane finding its entry by binary search, so the work per lane is one edge
// whatever the degree mix.  Part 2: one wavefront per kChunk-edge chunk of the
// long rows.
__global__ void __launch_bounds__(kBlock) k_expand(ExpandArgs a) {
  __shared__ uint32_t s_pref[kTile + 1];
  __shared__ int32_t s_slot[kTile];
  __shared__ uint32_t s_start[kTile];
  __shared__ float s_val[kTile];
  __shared__ int32_t s_flag[kTile];
  __shared__ uint32_t s_wtot[kBlock / 64];
  __shared__ int2 s_buf[kBlock / 64][kWaveBuf];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid >> 6;
  WaveBuf wb{s_buf[wv], 0u};
  unsigned long long nfinal = 0, nnext = 0, nconv = 0;

  const unsigned long long cnt = min(a.ctr[C_LIST0 + a.cur], (unsigned long long)a.list_cap);
  for (uint64_t tile0 = (uint64_t)blockIdx.x * kTile; tile0 < cnt; tile0 += (uint64_t)gridDim.x * kTile) {
    constexpr int kPer = kTile / kBlock;
    uint32_t deg[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int j = tid * kPer + r;
      const uint64_t i = tile0 + j;
      deg[r] = 0;
      if (i < cnt) {
        const uint2 row = a.item_row[i];
        if (row.y) {
          const int2 it = a.list_cur[i];
          long long* dc = a.dense_cur + (size_t)it.x * a.n + it.y;
          const int32_t pf = a.pull_flag[it.x];
          if (pf == 1) {  // slot moved to a dense column: scatter
            a.mat_cur[(size_t)it.y * kLanes + a.slots[it.x].lane] = grid_f32(*dc);
            a.map_cur[it.y] = 1;
            ++nconv;
            *dc = 0;
          } else if (pf == 2) {  // switched probe (Section 4.4): the level is dropped
            *dc = 0;
          } else {  // pushed: its score is consumed here (a randomized
                    // probe's entries never hold one)
            if (!a.slots[it.x].mode) *dc = 0;
            if (!(row.y & kBigFlag)) {
              deg[r] = row.y;
              s_start[j] = row.x;
              s_val[j] = a.item_val[i];
              s_slot[j] = it.x;
            }
          }
        }
      }
      s_flag[j] = 0;
      sum += deg[r];
    }
    const uint32_t incl = wave_incl_scan(sum);
    if (lane == 63) s_wtot[wv] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      if (w < wv) before += s_wtot[w];
      total += s_wtot[w];
    }
    uint32_t run = before + incl - sum;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      s_pref[tid * kPer + r] = run;
      run += deg[r];
    }
    if (tid == 0) s_pref[kTile] = total;
    __syncthreads();
    for (uint32_t e0 = 0; e0 < total; e0 += kBlock) {
      const uint32_t e = e0 + (uint32_t)tid;
      bool app = false;
      int32_t s = 0, v = 0;
      if (e < total) {
        int lo = 0, hi = kTile - 1;  // last entry j with s_pref[j] <= e
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pref[mid] <= e) lo = mid; else hi = mid - 1;
        }
        s = s_slot[lo];
        const Slot& sl = a.slots[s];
        v = sl.out_col[s_start[lo] + (e - s_pref[lo])];
        app = sl.mode ? visit_random(a, v, a.list_cur[tile0 + lo].y, sl, nfinal)
                      : visit_edge(a, s, v, s_val[lo], sl, nfinal);
        if (app) s_flag[lo] = 1;
      }
      wave_append(wb, app, s, v, a, nnext);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int j = tid * kPer + r;
      if (s_flag[j]) a.has_next[s_slot[j]] = 1;
    }
    __syncthreads();
  }

  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + tid) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const unsigned long long nchunk = min(a.ctr[C_CHUNK], (unsigned long long)a.chunk_cap);
  for (uint64_t c = wave; c < nchunk; c += nwaves) {
    const int2 ch = a.chunk_list[c];
    const int2 it = a.list_cur[ch.x];
    const int32_t s = it.x;
    if (a.pull_flag[s]) continue;  // pulled or switched
    const Slot sl = a.slots[s];
    const float sv = a.item_val[ch.x];
    const uint2 row = a.item_row[ch.x];
    const uint32_t len = row.y & ~kBigFlag;
    const uint32_t b = (uint32_t)ch.y * kChunk;
    const uint32_t e = min(len, b + kChunk);
    bool any = false;
    for (uint32_t t0 = b; t0 < e; t0 += 64) {
      const uint32_t t = t0 + lane;
      bool app = false;
      int32_t v = 0;
      if (t < e) {
        v = sl.out_col[row.x + t];
        app = sl.mode ? visit_random(a, v, it.y, sl, nfinal) : visit_edge(a, s, v, sv, sl, nfinal);
      }
      any |= app;
      wave_append(wb, app, s, v, a, nnext);
    }
    if (__ballot(any) && lane == 0) a.has_next[s] = 1;
  }
  wave_flush(wb, a, nnext);

  nfinal = wave_sum(nfinal);
  nnext = wave_sum(nnext);
  nconv = wave_sum(nconv);
  if (lane == 0) {
    if (nfinal) atomicAdd(&a.ctr[C_FINAL], nfinal);
    if (nnext) atomicAdd(&a.ctr[C_NEXT], nnext);
    if (nconv) atomicAdd(&a.ctr[C_NZROWS0 + a.cur], nconv);  // rows given scores in the dense matrix
  }
}

// Dense levels.  Up to kLanes slots keep their frontier as a column of a
// node-major matrix M (n x kLanes FP32 scores, one 256-byte row per node).
// One pass per step advances all of them together, by pulling: for every
// target v, H_{j+1}[v] is the grid sum over in-neighbours x of v of the same
// per-edge contributions the push path adds, with Rule 2 applied to H_j[x]
// as it is read and the excluded walk node skipped (Alg. 2 accumulated per
// target; exact sums make it equal to pushing).  A wavefront handles one
// target and its 64 lanes the 64 columns, so each in-neighbour costs one
// contiguous row read; the row of v in the next matrix is written whole.
// In-rows longer than kPullLane edges are summed in kPullChunk-edge chunks
// into partial grid sums, finished by k_dense_fin.  On a probe's last level
// the value goes into the FP64 estimate instead (one add per target).

struct DenseArgs {
  int32_t n;
  const Slot* slots;
  const int32_t* lane_slot;
  const DenseVer* dv;
  const float* mat_cur;
  float* mat_next;
  const uint8_t* map_cur;  // per node: its row of mat_cur may hold a nonzero score
  uint8_t* map_next;       // the same for mat_next, written with it
  long long* npart;  // n x kLanes partial grid sums of long in-rows
  unsigned long long* hyb_edges;  // Section 4.4: kept out-edges of each column's next level
  int32_t* has_next;
  unsigned long long* ctr;
  int cur;
};

struct LaneInfo {
  bool active;
  bool last;
  float thr, sc;
  int32_t excl;
  double w;
  double* acc;
  double* flip;
  double flip_unit;
};

__device__ __forceinline__ LaneInfo lane_info(const DenseArgs& a, int g, unsigned long long ghi) {
  LaneInfo li{};
  li.active = false;
  if ((unsigned long long)g < ghi) {
    const int32_t s = a.lane_slot[g];
    if (s >= 0) {
      const Slot& sl = a.slots[s];
      li.active = true;
      li.last = sl.last != 0;
      li.thr = sl.thr;
      li.sc = sl.sc;
      li.excl = sl.excl;
      li.w = sl.w;
      li.acc = sl.acc;
      li.flip = sl.flip;
      li.flip_unit = sl.flip_unit;
    }
  }
  return li;
}

// Target v of column g with grid sum q of its contributions: the FP64
// estimate on a probe's last level, else the next level's FP32 score.  Only
// writer lanes (one per column) act; every lane of the wavefront calls it.
__device__ __forceinline__ bool dense_finish(const DenseArgs& a, const LaneInfo& li, int g, bool writer, int32_t v,
                                             long long q, unsigned long long gw, unsigned long long& nfinal,
                                             unsigned long long& nzrows) {
  float out = 0.0f;
  bool nz = false;
  if (writer && li.active && v != li.excl && q > 0) {
    if (li.last) {
      unsafeAtomicAdd(&li.acc[v], grid_f64(q) * li.w);
      ++nfinal;
    } else {
      out = grid_f32(q);
      nz = true;
      // the next level tests this value against thr * sqrt(c)
      const float t = li.thr * li.sc;
      if (fabsf(out - t) <= 1e-5f * t) unsafeAtomicAdd(li.flip, li.flip_unit);
    }
  }
  if (writer && (unsigned long long)g < gw) a.mat_next[(size_t)v * kLanes + g] = out;
  const bool any = __ballot(nz) != 0ull;  // the whole row is rewritten: its flag too
  if (lane_id() == 0) a.map_next[v] = any ? 1 : 0;
  nzrows += any ? 1ull : 0ull;
  return nz;
}

// Grid value of the contribution of in-neighbour score h to target v (the
// push path's fl32(fl32(h * sqrt c) * 1/|I(v)|)); 0 when Rule 2 removes h.
__device__ __forceinline__ long long pull_term(float h, float thr, float sc, float inv) {
  return h > thr ? to_grid((h * sc) * inv) : 0ll;
}

// Score of in-neighbour x in this lane's column.  With kMap the row is read
// only when the row map says it may be nonzero (all lanes of a wavefront
// share x); that saves the gathers of a sparse matrix and costs a dependent
// load on a dense one.
template <bool kMap>
__device__ __forceinline__ float lane_score(const DenseArgs& a, const float* m, int32_t x) {
  if (kMap && !a.map_cur[x]) return 0.0f;
  return m[(size_t)x * kLanes];
}

// The pulls of one pass.  A wavefront works on one target at a time; its 64
// lanes form 64/L groups of L lanes (L = the power of two covering the
// columns in use), lane g handling column g % L of every L-th in-edge, so few
// columns still keep the whole wavefront busy.  Group sums are combined by
// shuffles.  Short in-rows are finished per target, long in-rows summed in
// kPullChunk-edge chunks into partial sums.
template <bool kMap>
__device__ __forceinline__ void dense_rows(const DenseArgs& a, const LaneInfo& li, const DenseVer& dv, int col,
                                           int grp, int L, uint64_t wave, uint64_t nwaves, unsigned long long gw,
                                           unsigned long long& nz_mask, unsigned long long& nfinal,
                                           unsigned long long& inedges, unsigned long long& nzrows) {
  const float* m = a.mat_cur + col;
  const uint32_t T = 64u / (uint32_t)L;
  const bool writer = grp == 0;
  for (uint64_t v = wave; v < (uint64_t)a.n; v += nwaves) {
    const uint2 row = dv.in_rows[v];
    if (row.y > kPullLane) continue;  // long in-row: chunks + k_dense_fin
    long long s0 = 0, s1 = 0;
    if (li.active) {
      const float inv = dv.inv_indeg[v];
      uint32_t k = (uint32_t)grp;
      for (; k + T < row.y; k += 2 * T) {
        const int32_t x0 = dv.in_col[row.x + k], x1 = dv.in_col[row.x + k + T];
        s0 += pull_term(lane_score<kMap>(a, m, x0), li.thr, li.sc, inv);
        s1 += pull_term(lane_score<kMap>(a, m, x1), li.thr, li.sc, inv);
      }
      if (k < row.y) s0 += pull_term(lane_score<kMap>(a, m, dv.in_col[row.x + k]), li.thr, li.sc, inv);
    }
    long long q = s0 + s1;
    for (int off = L; off < 64; off <<= 1) q += __shfl_xor(q, off, 64);
    inedges += row.y;
    const bool nz = dense_finish(a, li, col, writer, (int32_t)v, q, gw, nfinal, nzrows);
    nz_mask |= __ballot(nz);
  }
  const unsigned long long nch = dv.heavy_cnt[1];
  for (uint64_t c = wave; c < nch; c += nwaves) {
    const int2 ch = dv.heavy_chunks[c];
    const uint2 row = dv.in_rows[ch.x];
    const uint32_t e = min(row.y, (uint32_t)ch.y + kPullChunk);
    inedges += e - (uint32_t)ch.y;
    long long s0 = 0, s1 = 0;
    if (li.active) {
      const float inv = dv.inv_indeg[ch.x];
      uint32_t k = (uint32_t)ch.y + (uint32_t)grp;
      for (; k + T < e; k += 2 * T) {
        s0 += pull_term(lane_score<kMap>(a, m, dv.in_col[row.x + k]), li.thr, li.sc, inv);
        s1 += pull_term(lane_score<kMap>(a, m, dv.in_col[row.x + k + T]), li.thr, li.sc, inv);
      }
      if (k < e) s0 += pull_term(lane_score<kMap>(a, m, dv.in_col[row.x + k]), li.thr, li.sc, inv);
    }
    long long part = s0 + s1;
    for (int off = L; off < 64; off <<= 1) part += __shfl_xor(part, off, 64);
    if (writer && li.active && part > 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.npart[(size_t)ch.x * kLanes + col]),
                (unsigned long long)part);
  }
}

__global__ void __launch_bounds__(kBlock) k_dense(DenseArgs a) {
  __shared__ unsigned long long s_nz;
  const unsigned long long ghi = a.ctr[C_GHI], gw = a.ctr[C_GW];
  if (gw == 0) return;
  const int tid = threadIdx.x;
  const int g = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + tid) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  if (ghi == 0) {  // no column in use: clear the columns used last step
    for (uint64_t v = wave; v < (uint64_t)a.n; v += nwaves) {
      if ((unsigned long long)g < gw) a.mat_next[v * kLanes + g] = 0.0f;
      if (g == 0) a.map_next[v] = 0;
    }
    return;
  }
  if (tid == 0) s_nz = 0ull;
  __syncthreads();
  int L = 1;  // lanes per group: the power of two covering the columns to write
  while ((unsigned long long)L < gw) L <<= 1;
  const int col = g & (L - 1), grp = g / L;
  const LaneInfo li = lane_info(a, col, ghi);
  const DenseVer dv = *a.dv;
  unsigned long long nz_mask = 0, nfinal = 0, inedges = 0, nzrows = 0;
  // the row map pays off when fewer than half of the rows may be nonzero
  if (2ull * a.ctr[C_NZROWS0 + a.cur] < (unsigned long long)a.n)
    dense_rows<true>(a, li, dv, col, grp, L, wave, nwaves, gw, nz_mask, nfinal, inedges, nzrows);
  else
    dense_rows<false>(a, li, dv, col, grp, L, wave, nwaves, gw, nz_mask, nfinal, inedges, nzrows);
  if (g == 0 && nzrows) atomicAdd(&a.ctr[C_NZROWS0 + (a.cur ^ 1)], nzrows);
  if (g == 0 && nz_mask) atomicOr(&s_nz, nz_mask);
  nfinal = wave_sum(nfinal);
  if (g == 0) {
    if (nfinal) atomicAdd(&a.ctr[C_FINAL_PULL], nfinal);
    if (inedges) atomicAdd(&a.ctr[C_PULL_EDGES], inedges);
  }
  __syncthreads();
  if (tid < kLanes && ((s_nz >> tid) & 1ull)) a.has_next[a.lane_slot[tid]] = 1;
}

// Finishes the targets with long in-rows from their raw partial sums.
__global__ void __launch_bounds__(kBlock) k_dense_fin(DenseArgs a) {
  __shared__ unsigned long long s_nz;
  const unsigned long long ghi = a.ctr[C_GHI], gw = a.ctr[C_GW];
  if (ghi == 0) return;
  const int tid = threadIdx.x;
  const int g = lane_id();
  if (tid == 0) s_nz = 0ull;
  __syncthreads();
  const LaneInfo li = lane_info(a, g, ghi);
  const DenseVer dv = *a.dv;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + tid) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long nz_mask = 0, nfinal = 0, nzrows = 0;
  const unsigned long long nh = dv.heavy_cnt[0];
  for (uint64_t i = wave; i < nh; i += nwaves) {
    const int32_t v = dv.heavy_nodes[i];
    long long sum = 0;
    if (li.active) {
      long long* p = a.npart + (size_t)v * kLanes + g;
      sum = *p;
      *p = 0;
    }
    const bool nz = dense_finish(a, li, g, true, v, sum, gw, nfinal, nzrows);
    nz_mask |= __ballot(nz);
  }
  if (g == 0 && nz_mask) atomicOr(&s_nz, nz_mask);
  if (g == 0 && nzrows) atomicAdd(&a.ctr[C_NZROWS0 + (a.cur ^ 1)], nzrows);
  nfinal = wave_sum(nfinal);
  if (g == 0 && nfinal) atomicAdd(&a.ctr[C_FINAL_PULL], nfinal);
  __syncthreads();
  if (tid < kLanes && ((s_nz >> tid) & 1ull)) a.has_next[a.lane_slot[tid]] = 1;
}

// Section 4.4 for probes in dense columns: the out-edges of the entries of
// the level just written to the next matrix that Rule 2 will keep there
// (score above the next level's threshold), per hybrid column, into
// hyb_edges for k_pick's test at the next step.  One wavefront per row, one
// lane per column; rows the row map marks zero are skipped.  A pass of its
// own: counting inside k_dense slows every dense pass, hybrid or not.
__global__ void __launch_bounds__(kBlock) k_hyb_count(DenseArgs a) {
  __shared__ unsigned long long s_cnt[kLanes];
  const unsigned long long mask = a.ctr[C_HYBMASK];
  if (mask == 0ull) return;
  const int tid = threadIdx.x;
  const int g = lane_id();
  if (tid < kLanes) s_cnt[tid] = 0ull;
  __syncthreads();
  const bool mine = (mask >> g) & 1ull;
  float thr = 0.0f;
  int32_t slot = -1;
  if (mine) {
    slot = a.lane_slot[g];
    thr = a.slots[slot].thr_next;
  }
  const uint2* out_rows = a.dv->out_rows;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + tid) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long cnt = 0;
  for (uint64_t v = wave; v < (uint64_t)a.n; v += nwaves) {
    if (!a.map_next[v]) continue;
    if (mine && a.mat_next[v * kLanes + g] > thr) cnt += out_rows[v].y;
  }
  if (cnt) atomicAdd(&s_cnt[g], cnt);
  __syncthreads();
  if (tid < kLanes && s_cnt[tid]) atomicAdd(&a.hyb_edges[a.lane_slot[tid]], s_cnt[tid]);
}

// s^(u, v) = acc / n_r (+ shift for v != u), s^(u, u) = 1.
__global__ void k_finalize(int32_t n, const QueryDev* __restrict__ qr, int r) {
  const QueryDev Q = qr[r];
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    Q.acc[v] = v == Q.u ? 1.0 : Q.acc[v] * Q.inv_nr + Q.shift;
}

// Sort keys for top-k: the estimate, with u itself pushed below every node.
__global__ void k_topk_keys(int32_t n, int32_t u, const double* __restrict__ s, double* __restrict__ keys,
                            int32_t* __restrict__ ids) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    keys[v] = v == u ? -1.0 : s[v];
    ids[v] = (int32_t)v;
  }
}

struct NonZero {
  const double* acc;
  __device__ bool operator()(int32_t v) const { return acc[v] != 0.0; }
};

__global__ void k_gather_scores(const double* __restrict__ acc, const int32_t* __restrict__ ids, int64_t cnt,
                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) out[i] = acc[ids[i]];
}

// ------------------------------------------------------------- host side ----

uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

int grid_for(uint64_t work, int block) {
  const uint64_t g = (work + block - 1) / block;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(g, 1u << 30));
}

ps_status copy_out(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!bytes) return PS_OK;
  const hipMemcpyKind kind = ps_is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  PS_HIP(hipMemcpyAsync(dst, src, bytes, kind, st));
  return PS_OK;
}

bool tree_alloc(Session* s, uint64_t len, uint64_t* start) {
  for (size_t i = 0; i < s->tree_free.size(); ++i) {
    auto& f = s->tree_free[i];
    if (f.second >= len) {
      *start = f.first;
      f.first += len;
      f.second -= len;
      if (!f.second) s->tree_free.erase(s->tree_free.begin() + (long)i);
      return true;
    }
  }
  return false;
}

void tree_release(Session* s, uint64_t start, uint64_t len) {
  if (!len) return;
  auto& fl = s->tree_free;
  auto it = std::lower_bound(fl.begin(), fl.end(), std::make_pair(start, (uint64_t)0));
  it = fl.insert(it, {start, len});
  // coalesce with the neighbours
  if (it + 1 != fl.end() && it->first + it->second == (it + 1)->first) {
    it->second += (it + 1)->second;
    fl.erase(it + 1);
  }
  if (it != fl.begin() && (it - 1)->first + (it - 1)->second == it->first) {
    (it - 1)->second += it->second;
    fl.erase(it);
  }
}

}  // namespace

void report_overflow(const Session* s, const uint64_t* h) {
  std::fprintf(stderr,
               "probesim: capacity guard tripped (sites 0x%llx: 1 roots, 2 chunks, 4 next level, 16 ring); "
               "P %d n %d list cap %llu (lists %llu, %llu) chunk cap %llu (chunks %llu)\n",
               (unsigned long long)h[C_OVERFLOW], s->P, s->n, (unsigned long long)s->list_cap,
               (unsigned long long)h[C_LIST0], (unsigned long long)h[C_LIST1], (unsigned long long)s->chunk_cap,
               (unsigned long long)h[C_CHUNK]);
}

void session_clear_guard(Session* s, hipStream_t st) {
  k_set_u64<<<1, 1, 0, st>>>(s->counters.as<unsigned long long>() + C_OVERFLOW, 0ull);
}

ps_status devbuf_reserve(DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes && b.p) return PS_OK;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  const size_t want = std::max<size_t>(bytes, 256);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    std::fprintf(stderr, "probesim: device allocation of %zu bytes failed\n", want);
    b.p = nullptr;
    return PS_ERR_OOM;
  }
  b.bytes = want;
  return PS_OK;
}

void devbuf_free(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

void session_free(Session* s) {
  if (!s) return;
  DevBuf* bufs[] = {&s->mat[0], &s->mat[1], &s->rowmap[0], &s->rowmap[1], &s->npart, &s->lane_slot, &s->dense_ver, &s->slot_edges, &s->pull_flag, &s->slots,    &s->has_next,  &s->dense[0],   &s->dense[1],    &s->list[0],      &s->list[1],
                    &s->item_val, &s->item_row, &s->chunk_list, &s->counters,   &s->qrec,         &s->thr,
                    &s->remaining, &s->done_ring, &s->qbound,     &s->acc,         &s->lq,           &s->flip,
                    &s->keys,
                    &s->t_parent, &s->t_node,    &s->t_depth,     &s->t_query,     &s->t_weight,     &s->ring, &s->ring_k,
                    &s->hyb_edges, &s->t_woff, &s->t_walks, &s->wcount,
                    &s->sort_keys[0], &s->sort_keys[1], &s->sort_vals[0], &s->sort_vals[1], &s->sort_tmp,
                    &s->sel_count};
  for (DevBuf* b : bufs) devbuf_free(*b);
  if (s->h_ctr) (void)hipHostFree(s->h_ctr);
  if (s->step_pair) (void)hipGraphExecDestroy(s->step_pair);
  delete s;
}

// Probe slots: enough concurrent probes to fill the GPU (more slots also
// mean fewer level steps), at most 1024 by default, and never more than the
// per-slot buffers (grid sums 16 B, frontier lists 16 B, scaled scores 4 B,
// rows 8 B, chunks 8 B per node) fit in a fixed share of HBM, with slot * n
// within 31 bits.  An explicit request is clamped the same way.
int session_slots_for(int32_t n, int opt) {
  const uint64_t budget = 56ull << 30;
  uint64_t p = budget / (52ull * (uint64_t)n);
  p = std::min<uint64_t>(p, ((1ull << 31) - 1) / (uint64_t)n);
  p = std::min<uint64_t>(p, opt > 0 ? (uint64_t)std::min(opt, kSchedThreads * kSlotsPerSchedThread) : 1024ull);
  return (int)std::max<uint64_t>(p, 1);
}

ps_status session_ensure(ps_ctx* ctx, int32_t n, uint64_t m_cap, int P, int qmax, uint64_t tree_pool,
                         uint64_t ring_cap) {
  Session*& s = ctx->sess;
  hipStream_t st = ctx->stream;
  ring_cap = next_pow2(std::max<uint64_t>(ring_cap, 1024));
  tree_pool = std::max<uint64_t>(tree_pool, 1024);
  if (s && s->n == n && s->P == P && s->qmax >= qmax && s->tree_pool >= tree_pool && s->ring_cap >= ring_cap &&
      s->chunk_cap >= s->list_cap + ((uint64_t)P * m_cap) / kChunk + 1)
    return PS_OK;
  if (s && (int)s->free_recs.size() != s->qmax) return PS_ERR_STATE;  // queries admitted
  if (!s) s = new Session();
  if (s->step_pair) {  // captured with the old buffers
    (void)hipGraphExecDestroy(s->step_pair);
    s->step_pair = nullptr;
  }
  const bool shape = s->n != n || s->P != P;
  s->n = n;
  s->P = P;
  s->qmax = std::max(qmax, s->qmax);
  s->tree_pool = std::max(tree_pool, s->tree_pool);
  s->ring_cap = std::max(ring_cap, s->ring_cap);
  // Every (slot, node) pair enters a frontier list at most once per step, so
  // P * n entries never overflow; chunks add at most m / 512 per slot.
  s->list_cap = (uint64_t)P * (uint64_t)n;
  s->chunk_cap = s->list_cap + ((uint64_t)P * m_cap) / kChunk + 1;
  PS_TRY(devbuf_reserve(s->slots, sizeof(Slot) * (size_t)P));
  PS_TRY(devbuf_reserve(s->has_next, sizeof(int32_t) * (size_t)P));
  PS_TRY(devbuf_reserve(s->slot_edges, sizeof(unsigned long long) * (size_t)P));
  PS_TRY(devbuf_reserve(s->hyb_edges, sizeof(unsigned long long) * (size_t)P));
  PS_TRY(devbuf_reserve(s->pull_flag, sizeof(int32_t) * (size_t)P));
  PS_TRY(devbuf_reserve(s->mat[0], sizeof(float) * (size_t)n * kLanes));
  PS_TRY(devbuf_reserve(s->mat[1], sizeof(float) * (size_t)n * kLanes));
  PS_TRY(devbuf_reserve(s->npart, sizeof(long long) * (size_t)n * kLanes));
  PS_TRY(devbuf_reserve(s->rowmap[0], (size_t)n));
  PS_TRY(devbuf_reserve(s->rowmap[1], (size_t)n));
  PS_TRY(devbuf_reserve(s->lane_slot, sizeof(int32_t) * kLanes));
  PS_TRY(devbuf_reserve(s->dense_ver, sizeof(DenseVer)));
  const bool fresh = !s->dense[0].p || shape;
  PS_TRY(devbuf_reserve(s->dense[0], sizeof(long long) * s->list_cap));
  PS_TRY(devbuf_reserve(s->dense[1], sizeof(long long) * s->list_cap));
  PS_TRY(devbuf_reserve(s->list[0], sizeof(int2) * s->list_cap));
  PS_TRY(devbuf_reserve(s->list[1], sizeof(int2) * s->list_cap));
  PS_TRY(devbuf_reserve(s->item_val, sizeof(float) * s->list_cap));
  PS_TRY(devbuf_reserve(s->item_row, sizeof(uint2) * s->list_cap));
  PS_TRY(devbuf_reserve(s->chunk_list, sizeof(int2) * s->chunk_cap));
  PS_TRY(devbuf_reserve(s->counters, sizeof(unsigned long long) * C_COUNT));
  PS_TRY(devbuf_reserve(s->qrec, sizeof(QueryDev) * (size_t)s->qmax));
  PS_TRY(devbuf_reserve(s->thr, sizeof(float) * (size_t)s->qmax * PS_MAX_WALK_LEN));
  PS_TRY(devbuf_reserve(s->remaining, sizeof(unsigned long long) * (size_t)s->qmax));
  PS_TRY(devbuf_reserve(s->done_ring, sizeof(int32_t) * (size_t)s->qmax));
  PS_TRY(devbuf_reserve(s->qbound, sizeof(unsigned long long) * (size_t)s->qmax));
  PS_TRY(devbuf_reserve(s->acc, sizeof(double) * (size_t)s->qmax * (size_t)n));
  PS_TRY(devbuf_reserve(s->lq, sizeof(int32_t) * (size_t)s->qmax));
  PS_TRY(devbuf_reserve(s->flip, sizeof(double) * (size_t)s->qmax));
  PS_TRY(devbuf_reserve(s->keys, sizeof(unsigned long long) * s->tree_pool));
  PS_TRY(devbuf_reserve(s->t_parent, sizeof(int32_t) * (s->tree_pool + s->qmax)));
  PS_TRY(devbuf_reserve(s->t_node, sizeof(int32_t) * (s->tree_pool + s->qmax)));
  PS_TRY(devbuf_reserve(s->t_depth, sizeof(int32_t) * (s->tree_pool + s->qmax)));
  PS_TRY(devbuf_reserve(s->t_query, sizeof(int32_t) * (s->tree_pool + s->qmax)));
  PS_TRY(devbuf_reserve(s->t_weight, sizeof(int32_t) * (s->tree_pool + s->qmax)));
  PS_TRY(devbuf_reserve(s->t_woff, sizeof(uint32_t) * s->tree_pool));
  PS_TRY(devbuf_reserve(s->t_walks, sizeof(int32_t) * s->tree_pool));
  PS_TRY(devbuf_reserve(s->wcount, sizeof(unsigned long long) * (size_t)s->qmax));
  PS_TRY(devbuf_reserve(s->ring, sizeof(int32_t) * s->ring_cap));
  PS_TRY(devbuf_reserve(s->ring_k, sizeof(int32_t) * s->ring_cap));
  if (!s->h_ctr) PS_HIP(hipHostMalloc((void**)&s->h_ctr, sizeof(uint64_t) * C_COUNT, 0));
  if (fresh) {
    PS_HIP(hipMemsetAsync(s->dense[0].p, 0, sizeof(long long) * s->list_cap, st));
    PS_HIP(hipMemsetAsync(s->dense[1].p, 0, sizeof(long long) * s->list_cap, st));
  }
  for (DevBuf* b : {&s->mat[0], &s->mat[1]}) PS_HIP(hipMemsetAsync(b->p, 0, sizeof(float) * (size_t)n * kLanes, st));
  PS_HIP(hipMemsetAsync(s->npart.p, 0, sizeof(long long) * (size_t)n * kLanes, st));
  for (DevBuf* b : {&s->rowmap[0], &s->rowmap[1]}) PS_HIP(hipMemsetAsync(b->p, 0, (size_t)n, st));
  k_reset_lanes<<<1, kLanes, 0, st>>>(s->lane_slot.as<int32_t>());
  PS_HIP(hipMemsetAsync(s->counters.p, 0, sizeof(unsigned long long) * C_COUNT, st));
  PS_HIP(hipMemsetAsync(s->hyb_edges.p, 0, sizeof(unsigned long long) * (size_t)P, st));
  k_reset_slots<<<grid_for((uint64_t)P, kBlock), kBlock, 0, st>>>(s->slots.as<Slot>(), s->has_next.as<int32_t>(), P);
  PS_HIP(hipGetLastError());
  s->steps = 0;
  s->free_recs.clear();
  for (int r = s->qmax - 1; r >= 0; --r) s->free_recs.push_back(r);
  s->h_rec.assign((size_t)s->qmax, QueryDev{});
  s->rec_version.assign((size_t)s->qmax, nullptr);
  s->rec_tree.assign((size_t)s->qmax, {0, 0});
  s->rec_ring.assign((size_t)s->qmax, 0);
  s->tree_free.assign(1, {0, s->tree_pool});
  s->ring_outstanding = 0;
  PS_HIP(hipStreamSynchronize(st));
  return PS_OK;
}

// Phase 1 of admission: records, walk sampling, tree sizes (one sync).
ps_status session_begin(ps_ctx* ctx, ps_graph* g, GraphVersion* gv, const std::vector<QueryRun>& qs,
                        std::vector<int>* recs, std::vector<uint64_t>* bounds) {
  Session* s = ctx->sess;
  hipStream_t st = ctx->stream;
  if ((size_t)s->free_recs.size() < qs.size()) return PS_ERR_BUSY;
  recs->clear();
  bounds->assign(qs.size(), 0);
  if (qs.empty()) return PS_OK;
  // one threshold row per query, alive until the synchronisation below
  std::vector<float> thr_all(qs.size() * PS_MAX_WALK_LEN, 0.0f);
  int64_t total = 0;
  for (const QueryRun& q : qs) {
    float* thr = thr_all.data() + recs->size() * PS_MAX_WALK_LEN;
    const int r = s->free_recs.back();
    s->free_recs.pop_back();
    recs->push_back(r);
    QueryDev d{};
    d.u = q.u;
    d.L = q.prm.L;
    d.t_stop = q.prm.t_stop;
    d.topk = q.k;
    d.seed = q.seed;
    d.walk_begin = q.walk_begin;
    d.walk_count = q.walk_end - q.walk_begin;
    d.walk_base = total;
    const double sc = std::sqrt(q.prm.c);
    d.sc = (float)sc;
    d.inv_nr = 1.0 / (double)q.prm.n_r;
    d.shift = q.bias_shift ? q.prm.eps_t / 2.0 : 0.0;
    d.in_rows = gv->in_rows;
    d.in_col = gv->in_store->col;
    d.out_rows = gv->out_rows;
    d.out_col = gv->out_store->col;
    d.inv_indeg = gv->inv_indeg;
    d.heavy_nodes = gv->heavy_nodes;
    d.heavy_chunks = gv->heavy_chunks;
    d.heavy_cnt = gv->heavy_cnt;
    d.acc = s->acc.as<double>() + (size_t)r * (size_t)s->n;
    d.flip = s->flip.as<double>() + r;
    // one flip moves an estimate by at most Score * sqrt(c)^e ~ eps_p per
    // walk sharing the probe (the near band is 1e-5 relative wide)
    d.flip_unit = q.randomized ? 0.0 : q.prm.eps_p * (1.0 + 1e-4) / (double)q.prm.n_r;
    d.randomized = q.randomized;
    d.hybrid = q.hybrid;
    d.c0 = q.c0;
    d.t_sc = (uint32_t)std::floor(sc * 4294967296.0);
    d.key2 = make_uint2((uint32_t)q.seed, (uint32_t)(q.seed >> 32) ^ 0x9E3779B9u);
    total += d.walk_count;
    s->h_rec[(size_t)r] = d;
    {
      std::lock_guard<std::mutex> lk(g->mu);
      gv->refs++;
    }
    s->rec_version[(size_t)r] = gv;
    // Rule 2 thresholds thr[e] = eps_p / sqrt(c)^e (0 = no pruning)
    for (int x = 1; x < PS_MAX_WALK_LEN; ++x)
      thr[x] = q.prm.eps_p > 0.0 ? (float)(q.prm.eps_p / std::pow(sc, (double)x)) : 0.0f;
    PS_HIP(hipMemcpyAsync(s->thr.as<float>() + (size_t)r * PS_MAX_WALK_LEN, thr, sizeof(float) * PS_MAX_WALK_LEN,
                          hipMemcpyHostToDevice, st));
    PS_HIP(hipMemcpyAsync(s->qrec.as<QueryDev>() + r, &s->h_rec[(size_t)r], sizeof(QueryDev), hipMemcpyHostToDevice,
                          st));
    PS_HIP(hipMemsetAsync(d.acc, 0, sizeof(double) * (size_t)s->n, st));
    PS_HIP(hipMemsetAsync(s->qbound.as<unsigned long long>() + r, 0, sizeof(unsigned long long), st));
    PS_HIP(hipMemsetAsync(s->remaining.as<unsigned long long>() + r, 0, sizeof(unsigned long long), st));
    PS_HIP(hipMemsetAsync(d.flip, 0, sizeof(double), st));
  }
  PS_HIP(hipMemcpyAsync(s->lq.p, recs->data(), sizeof(int32_t) * recs->size(), hipMemcpyHostToDevice, st));
  if (total > 0) {
    k_walk_bound<<<grid_for((uint64_t)total, kBlock), kBlock, 0, st>>>(
        s->qrec.as<QueryDev>(), s->lq.as<int32_t>(), (int)recs->size(), total, s->qbound.as<unsigned long long>(),
        s->counters.as<unsigned long long>());
    PS_HIP(hipGetLastError());
  }
  std::vector<unsigned long long> hb((size_t)s->qmax);
  PS_HIP(hipMemcpyAsync(hb.data(), s->qbound.p, sizeof(unsigned long long) * (size_t)s->qmax, hipMemcpyDeviceToHost,
                        st));
  PS_HIP(hipStreamSynchronize(st));
  for (size_t i = 0; i < recs->size(); ++i) (*bounds)[i] = hb[(size_t)(*recs)[i]];
  return PS_OK;
}

// Ring entries record r may need: one per tree node, plus one per walk and
// prefix for the probes a hybrid query switches (Section 4.4).
static uint64_t ring_share(const Session* s, int r, uint64_t bound) {
  return s->h_rec[(size_t)r].hybrid ? 2 * bound : bound;
}

// Phase 2 of admission: tree regions, tree construction, probes queued.
// Records with bound 0 have no probe and need no tree.
ps_status session_build(ps_ctx* ctx, const std::vector<int>& recs, const std::vector<uint64_t>& bounds) {
  Session* s = ctx->sess;
  hipStream_t st = ctx->stream;
  std::vector<int32_t> launch;
  int64_t total = 0;
  uint64_t ring_need = 0;
  for (size_t i = 0; i < recs.size(); ++i) ring_need += ring_share(s, recs[i], bounds[i]);
  if (s->ring_outstanding + ring_need > s->ring_cap) return PS_ERR_BUSY;
  std::vector<std::pair<int, uint64_t>> got;
  for (size_t i = 0; i < recs.size(); ++i) {
    if (!bounds[i]) continue;
    const int r = recs[i];
    const uint64_t cap = next_pow2(std::max<uint64_t>(2 * bounds[i], 64));
    uint64_t start;
    if (!tree_alloc(s, cap, &start)) {
      for (auto& gr : got) tree_release(s, s->rec_tree[(size_t)gr.first].first, gr.second);
      return PS_ERR_BUSY;
    }
    got.push_back({r, cap});
    s->rec_tree[(size_t)r] = {start, cap};
  }
  for (size_t i = 0; i < recs.size(); ++i) {
    if (!bounds[i]) continue;
    const int r = recs[i];
    QueryDev& d = s->h_rec[(size_t)r];
    d.tree_base = s->rec_tree[(size_t)r].first;
    d.tree_mask = s->rec_tree[(size_t)r].second - 1;
    d.walk_base = total;
    total += d.walk_count;
    s->rec_ring[(size_t)r] = ring_share(s, r, bounds[i]);
    s->ring_outstanding += s->rec_ring[(size_t)r];
    launch.push_back(r);
    PS_HIP(hipMemcpyAsync(s->qrec.as<QueryDev>() + r, &d, sizeof(QueryDev), hipMemcpyHostToDevice, st));
    PS_HIP(hipMemsetAsync(s->keys.as<unsigned long long>() + d.tree_base, 0xFF,
                          sizeof(unsigned long long) * (d.tree_mask + 1), st));
    PS_HIP(hipMemsetAsync(s->t_weight.as<int32_t>() + d.tree_base, 0, sizeof(int32_t) * (d.tree_mask + 1), st));
  }
  if (launch.empty()) return PS_OK;
  PS_HIP(hipMemcpyAsync(s->lq.p, launch.data(), sizeof(int32_t) * launch.size(), hipMemcpyHostToDevice, st));
  k_init_roots<<<grid_for(launch.size(), kBlock), kBlock, 0, st>>>(
      s->qrec.as<QueryDev>(), s->lq.as<int32_t>(), (int)launch.size(), s->tree_pool, s->t_parent.as<int32_t>(),
      s->t_node.as<int32_t>(), s->t_depth.as<int32_t>(), s->t_query.as<int32_t>());
  PS_HIP(hipGetLastError());
  TreeArgs a{};
  a.qr = s->qrec.as<QueryDev>();
  a.lq = s->lq.as<int32_t>();
  a.nl = (int)launch.size();
  a.total = total;
  a.root_base = s->tree_pool;
  a.keys = s->keys.as<unsigned long long>();
  a.t_parent = s->t_parent.as<int32_t>();
  a.t_node = s->t_node.as<int32_t>();
  a.t_depth = s->t_depth.as<int32_t>();
  a.t_query = s->t_query.as<int32_t>();
  a.t_weight = s->t_weight.as<int32_t>();
  a.ring = s->ring.as<int32_t>();
  a.ring_k = s->ring_k.as<int32_t>();
  a.ring_mask = s->ring_cap - 1;
  a.remaining = s->remaining.as<unsigned long long>();
  a.ctr = s->counters.as<unsigned long long>();
  if (total > 0) {
    k_walk_tree<<<grid_for((uint64_t)total, kBlock), kBlock, 0, st>>>(a);
    PS_HIP(hipGetLastError());
  }
  // Section 4.4: the walks through each tree node of the hybrid queries
  bool hybrid = false;
  for (int r : launch) {
    const QueryDev& d = s->h_rec[(size_t)r];
    if (!d.hybrid) continue;
    hybrid = true;
    unsigned long long* cnt = s->wcount.as<unsigned long long>() + r;
    PS_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st));
    k_walk_offsets<<<grid_for(d.tree_mask + 1, kBlock), kBlock, 0, st>>>(
        s->keys.as<unsigned long long>(), s->t_weight.as<int32_t>(), s->t_woff.as<uint32_t>(), d.tree_base,
        d.tree_mask + 1, cnt);
    PS_HIP(hipGetLastError());
  }
  if (hybrid && total > 0) {
    k_walk_lists<<<grid_for((uint64_t)total, kBlock), kBlock, 0, st>>>(a, s->t_woff.as<uint32_t>(),
                                                                      s->t_walks.as<int32_t>());
    PS_HIP(hipGetLastError());
  }
  return PS_OK;
}

namespace {

struct StepKernels {
  SchedArgs sa;
  ExpandArgs ea;
};

StepKernels step_args(Session* s) {
  StepKernels k{};
  unsigned long long* ctr = s->counters.as<unsigned long long>();
  SchedArgs& sa = k.sa;
  sa.P = s->P;
  sa.n = s->n;
  sa.qmax = s->qmax;
  sa.slots = s->slots.as<Slot>();
  sa.has_next = s->has_next.as<int32_t>();
  sa.ring = s->ring.as<int32_t>();
  sa.ring_k = s->ring_k.as<int32_t>();
  sa.ring_mask = s->ring_cap - 1;
  sa.t_parent = s->t_parent.as<int32_t>();
  sa.t_node = s->t_node.as<int32_t>();
  sa.t_depth = s->t_depth.as<int32_t>();
  sa.t_query = s->t_query.as<int32_t>();
  sa.t_weight = s->t_weight.as<int32_t>();
  sa.qr = s->qrec.as<QueryDev>();
  sa.thr_tab = s->thr.as<float>();
  sa.remaining = s->remaining.as<unsigned long long>();
  sa.done_ring = s->done_ring.as<int32_t>();
  sa.list_cap = s->list_cap;
  sa.slot_edges = s->slot_edges.as<unsigned long long>();
  sa.lane_slot = s->lane_slot.as<int32_t>();
  sa.ctr = ctr;
  ExpandArgs& ea = k.ea;
  ea.pull_flag = s->pull_flag.as<int32_t>();
  ea.n = s->n;
  ea.item_val = s->item_val.as<float>();
  ea.item_row = s->item_row.as<uint2>();
  ea.chunk_list = s->chunk_list.as<int2>();
  ea.slots = s->slots.as<Slot>();
  ea.list_cap = s->list_cap;
  ea.chunk_cap = s->chunk_cap;
  ea.has_next = s->has_next.as<int32_t>();
  ea.ctr = ctr;
  return k;
}

// One level step with the frontier lists of parity `cur`.
void launch_step(Session* s, StepKernels& k, int cur, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                 hipEvent_t ev2) {
  const int nxt = cur ^ 1;
  unsigned long long* ctr = s->counters.as<unsigned long long>();
  k.sa.dense_cur = s->dense[cur].as<long long>();
  k.sa.list_cur = s->list[cur].as<int2>();
  k.sa.cur = cur;
  k_sched<<<1, kSchedThreads, 0, st>>>(k.sa);
  k_prep<<<kStepGrid, kBlock, 0, st>>>(s->n, s->slots.as<Slot>(), s->list[cur].as<int2>(), s->dense[cur].as<long long>(),
                                       s->item_val.as<float>(), s->item_row.as<uint2>(), s->chunk_list.as<int2>(),
                                       s->list_cap, s->chunk_cap, s->slot_edges.as<unsigned long long>(), ctr, cur);
  PickArgs pa{};
  pa.P = s->P;
  pa.slot_edges = s->slot_edges.as<unsigned long long>();
  pa.hyb_edges = s->hyb_edges.as<unsigned long long>();
  pa.slots = s->slots.as<Slot>();
  pa.pull_flag = s->pull_flag.as<int32_t>();
  pa.lane_slot = s->lane_slot.as<int32_t>();
  pa.dv = s->dense_ver.as<DenseVer>();
  pa.t_weight = s->t_weight.as<int32_t>();
  pa.t_woff = s->t_woff.as<uint32_t>();
  pa.t_walks = s->t_walks.as<int32_t>();
  pa.ring = s->ring.as<int32_t>();
  pa.ring_k = s->ring_k.as<int32_t>();
  pa.ring_mask = s->ring_cap - 1;
  pa.remaining = s->remaining.as<unsigned long long>();
  pa.ctr = ctr;
  k_pick<<<1, kSchedThreads, 0, st>>>(pa);
  k.ea.list_cur = s->list[cur].as<int2>();
  k.ea.cur = cur;
  k.ea.dense_cur = s->dense[cur].as<long long>();
  k.ea.mat_cur = s->mat[cur].as<float>();
  k.ea.map_cur = s->rowmap[cur].as<uint8_t>();
  k.ea.dense_next = s->dense[nxt].as<long long>();
  k.ea.list_next = s->list[nxt].as<int2>();
  k.ea.nxt = nxt;
  if (ev0) (void)hipEventRecord(ev0, st);
  k_expand<<<kStepGrid, kBlock, 0, st>>>(k.ea);
  if (ev1) (void)hipEventRecord(ev1, st);
  DenseArgs da{};
  da.n = s->n;
  da.slots = s->slots.as<Slot>();
  da.lane_slot = s->lane_slot.as<int32_t>();
  da.dv = s->dense_ver.as<DenseVer>();
  da.mat_cur = s->mat[cur].as<float>();
  da.mat_next = s->mat[nxt].as<float>();
  da.map_cur = s->rowmap[cur].as<uint8_t>();
  da.map_next = s->rowmap[nxt].as<uint8_t>();
  da.npart = s->npart.as<long long>();
  da.hyb_edges = s->hyb_edges.as<unsigned long long>();
  da.has_next = s->has_next.as<int32_t>();
  da.ctr = ctr;
  da.cur = cur;
  k_dense<<<kStepGrid, kBlock, 0, st>>>(da);
  k_dense_fin<<<kStepGrid / 4, kBlock, 0, st>>>(da);
  k_hyb_count<<<kStepGrid / 4, kBlock, 0, st>>>(da);
  if (ev2) (void)hipEventRecord(ev2, st);
}

}  // namespace

// Launches `count` level steps.  Without timing they run as replays of a
// captured pair of steps (even then odd list parity), one graph launch per
// pair; with timing every expansion is bracketed by events.
ps_status session_steps(ps_ctx* ctx, uint64_t count, double* expand_ms, double* pull_ms) {
  Session* s = ctx->sess;
  hipStream_t st = ctx->stream;
  StepKernels k = step_args(s);
  const bool timing = ctx->timing && expand_ms;
  if (timing) {
    while (ctx->ev_pool.size() < 3 * count) {
      hipEvent_t ev;
      PS_HIP(hipEventCreate(&ev));
      ctx->ev_pool.push_back(ev);
    }
    for (uint64_t t = 0; t < count; ++t) {
      launch_step(s, k, (int)(s->steps & 1), st, ctx->ev_pool[3 * t], ctx->ev_pool[3 * t + 1],
                  ctx->ev_pool[3 * t + 2]);
      s->steps++;
    }
    PS_HIP(hipGetLastError());
    PS_HIP(hipStreamSynchronize(st));
    double ms = 0.0, pms = 0.0;
    for (uint64_t t = 0; t < count; ++t) {
      float x = 0.0f, y = 0.0f;
      PS_HIP(hipEventElapsedTime(&x, ctx->ev_pool[3 * t], ctx->ev_pool[3 * t + 1]));
      PS_HIP(hipEventElapsedTime(&y, ctx->ev_pool[3 * t + 1], ctx->ev_pool[3 * t + 2]));
      ms += x;
      pms += y;
    }
    *expand_ms += ms;
    if (pull_ms) *pull_ms += pms;
    return PS_OK;
  }
  if (count >= 4) {
    if (s->steps & 1) {
      launch_step(s, k, 1, st, nullptr, nullptr, nullptr);
      s->steps++;
      count--;
    }
    if (!s->step_pair) {
      hipGraph_t graph = nullptr;
      PS_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      launch_step(s, k, 0, st, nullptr, nullptr, nullptr);
      launch_step(s, k, 1, st, nullptr, nullptr, nullptr);
      PS_HIP(hipStreamEndCapture(st, &graph));
      const hipError_t e = hipGraphInstantiate(&s->step_pair, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      PS_HIP(e);
    }
    for (; count >= 2; count -= 2) {
      PS_HIP(hipGraphLaunch(s->step_pair, st));
      s->steps += 2;
    }
  }
  for (; count > 0; --count) {
    launch_step(s, k, (int)(s->steps & 1), st, nullptr, nullptr, nullptr);
    s->steps++;
  }
  PS_HIP(hipGetLastError());
  return PS_OK;
}

// Finalises record r and writes its result; frees the record.
ps_status session_finish(ps_ctx* ctx, ps_graph* g, int r, const QueryRun& q, const QueryOut& out) {
  Session* s = ctx->sess;
  hipStream_t st = ctx->stream;
  const int32_t n = s->n;
  double* acc = s->h_rec[(size_t)r].acc;
  k_finalize<<<grid_for((uint64_t)n, kBlock) > 4096 ? 4096 : grid_for((uint64_t)n, kBlock), kBlock, 0, st>>>(
      n, s->qrec.as<QueryDev>(), r);
  PS_HIP(hipGetLastError());
  if (out.cap >= 0) {
    // nonzero estimates in ascending node order (stable selection)
    PS_TRY(devbuf_reserve(s->sort_vals[0], sizeof(int32_t) * (size_t)n));
    PS_TRY(devbuf_reserve(s->sort_keys[0], sizeof(double) * (size_t)n));
    PS_TRY(devbuf_reserve(s->sel_count, sizeof(int64_t)));
    const NonZero pred{acc};
    const hipcub::CountingInputIterator<int32_t> ids(0);
    size_t tmp = 0;
    PS_HIP(hipcub::DeviceSelect::If(nullptr, tmp, ids, s->sort_vals[0].as<int32_t>(), s->sel_count.as<int64_t>(), n,
                                    pred, st));
    PS_TRY(devbuf_reserve(s->sort_tmp, tmp));
    PS_HIP(hipcub::DeviceSelect::If(s->sort_tmp.p, tmp, ids, s->sort_vals[0].as<int32_t>(), s->sel_count.as<int64_t>(),
                                    n, pred, st));
    int64_t total = 0;
    PS_HIP(hipMemcpyAsync(&total, s->sel_count.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    const int64_t w = std::min(total, out.cap);
    if (w > 0) {
      k_gather_scores<<<grid_for((uint64_t)w, kBlock), kBlock, 0, st>>>(acc, s->sort_vals[0].as<int32_t>(), w,
                                                                         s->sort_keys[0].as<double>());
      PS_HIP(hipGetLastError());
      PS_TRY(copy_out(out.nodes, s->sort_vals[0].p, sizeof(int32_t) * (size_t)w, st));
      PS_TRY(copy_out(out.scores, s->sort_keys[0].p, sizeof(double) * (size_t)w, st));
    }
    *out.count = total;
  } else if (q.k <= 0) {
    PS_TRY(copy_out(out.scores, acc, sizeof(double) * (size_t)n, st));
  } else {
    PS_TRY(devbuf_reserve(s->sort_keys[0], sizeof(double) * (size_t)n));
    PS_TRY(devbuf_reserve(s->sort_keys[1], sizeof(double) * (size_t)n));
    PS_TRY(devbuf_reserve(s->sort_vals[0], sizeof(int32_t) * (size_t)n));
    PS_TRY(devbuf_reserve(s->sort_vals[1], sizeof(int32_t) * (size_t)n));
    k_topk_keys<<<kStepGrid, kBlock, 0, st>>>(n, q.u, acc, s->sort_keys[0].as<double>(), s->sort_vals[0].as<int32_t>());
    PS_HIP(hipGetLastError());
    size_t tmp = 0;
    PS_HIP(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tmp, s->sort_keys[0].as<double>(),
                                                         s->sort_keys[1].as<double>(), s->sort_vals[0].as<int32_t>(),
                                                         s->sort_vals[1].as<int32_t>(), n, 0, 64, st));
    PS_TRY(devbuf_reserve(s->sort_tmp, tmp));
    PS_HIP(hipcub::DeviceRadixSort::SortPairsDescending(s->sort_tmp.p, tmp, s->sort_keys[0].as<double>(),
                                                         s->sort_keys[1].as<double>(), s->sort_vals[0].as<int32_t>(),
                                                         s->sort_vals[1].as<int32_t>(), n, 0, 64, st));
    PS_TRY(copy_out(out.scores, s->sort_keys[1].p, sizeof(double) * (size_t)q.k, st));
    PS_TRY(copy_out(out.nodes, s->sort_vals[1].p, sizeof(int32_t) * (size_t)q.k, st));
  }
  if (out.flip) PS_TRY(copy_out(out.flip, s->flip.as<double>() + r, sizeof(double), st));
  // release the record (later users are ordered after these copies on the stream)
  auto tr = s->rec_tree[(size_t)r];
  tree_release(s, tr.first, tr.second);
  s->rec_tree[(size_t)r] = {0, 0};
  s->ring_outstanding -= s->rec_ring[(size_t)r];
  s->rec_ring[(size_t)r] = 0;
  if (s->rec_version[(size_t)r]) graph_release(g, s->rec_version[(size_t)r]);
  s->rec_version[(size_t)r] = nullptr;
  s->free_recs.push_back(r);
  return PS_OK;
}

// Releases a record whose tree was never built (admission failed).
void session_abandon(ps_ctx* ctx, ps_graph* g, int r) {
  Session* s = ctx->sess;
  if (s->rec_version[(size_t)r]) graph_release(g, s->rec_version[(size_t)r]);
  s->rec_version[(size_t)r] = nullptr;
  s->free_recs.push_back(r);
}

ps_status engine_walks(ps_ctx* ctx, GraphVersion* gv, int32_t n, const QueryRun& q, int64_t k_begin, int64_t count,
                       int32_t* nodes, int32_t* lens) {
  (void)n;
  hipStream_t st = ctx->stream;
  QueryDev d{};
  d.u = q.u;
  d.L = q.prm.L;
  d.t_stop = q.prm.t_stop;
  d.seed = q.seed;
  d.in_rows = gv->in_rows;
  d.in_col = gv->in_store->col;
  const size_t nb = sizeof(int32_t) * (size_t)count * (size_t)d.L;
  int32_t* dn = nullptr;
  if (count > 0) {
    PS_HIP(hipMalloc(&dn, nb + sizeof(int32_t) * (size_t)count));
    int32_t* dl = dn + (size_t)count * d.L;
    k_walk_export<<<grid_for((uint64_t)count, kBlock), kBlock, 0, st>>>(d, k_begin, count, dn, dl);
    PS_HIP(hipGetLastError());
    PS_TRY(copy_out(nodes, dn, nb, st));
    PS_TRY(copy_out(lens, dl, sizeof(int32_t) * (size_t)count, st));
  }
  PS_HIP(hipStreamSynchronize(st));
  if (dn) (void)hipFree(dn);
  return PS_OK;
}

// Pull threshold in out-edges of a slot's kept entries: a pull reads every
// in-edge of the graph once, so it pays off when the level would push along
// a sizable share of them.
uint64_t pull_threshold(int64_t m, int64_t opt) {
  if (opt < 0) return ~0ull;
  if (opt > 0) return (uint64_t)opt;
  return std::max<uint64_t>((uint64_t)m / 20, 4096);
}

ps_status session_set_pull(ps_ctx* ctx, uint64_t threshold) {
  Session* s = ctx->sess;
  k_set_u64<<<1, 1, 0, ctx->stream>>>(s->counters.as<unsigned long long>() + C_PULL_T,
                                      (unsigned long long)threshold);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

ps_status engine_run(ps_ctx* ctx, ps_graph* g, GraphVersion* gv, const std::vector<QueryRun>& qs,
                     const std::vector<QueryOut>& outs, int slots_opt, int64_t pull_opt) {
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t st = ctx->stream;
  const int32_t n = g->n;
  const int nq = (int)qs.size();
  ps_stats stats{};
  stats.queries = nq;
  if (nq == 0) {
    ctx->last = stats;
    return PS_OK;
  }
  const int P = session_slots_for(n, slots_opt);
  const uint64_t m_cap = std::max<uint64_t>(gv->out_store->cap, 1);
  Session* s = ctx->sess;
  PS_TRY(session_ensure(ctx, n, m_cap, P, std::max(nq, s ? s->qmax : 0), s ? s->tree_pool : 0,
                        s ? s->ring_cap : 0));
  s = ctx->sess;
  session_clear_guard(s, st);
  PS_HIP(hipMemcpyAsync(s->h_ctr, s->counters.p, sizeof(uint64_t) * C_COUNT, hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  std::vector<uint64_t> before(s->h_ctr, s->h_ctr + C_COUNT);

  std::vector<int> recs;
  std::vector<uint64_t> bounds;
  PS_TRY(session_begin(ctx, g, gv, qs, &recs, &bounds));
  uint64_t pool_need = 0, ring_need = 0;
  for (size_t i = 0; i < bounds.size(); ++i) {
    const uint64_t b = bounds[i];
    if (b) pool_need += next_pow2(std::max<uint64_t>(2 * b, 64));
    ring_need += ring_share(s, recs[i], b);
  }
  if (pool_need > s->tree_pool || ring_need > s->ring_cap) {
    // Grow the tree pool / ring: only this call's records are admitted and
    // their trees are not built yet, so the buffers can be replaced.  The
    // captured level steps point at the old buffers and are dropped.
    if (s->step_pair) {
      PS_HIP(hipStreamSynchronize(st));
      (void)hipGraphExecDestroy(s->step_pair);
      s->step_pair = nullptr;
    }
    s->tree_pool = std::max(pool_need, s->tree_pool);
    s->ring_cap = next_pow2(std::max(ring_need, s->ring_cap));
    PS_TRY(devbuf_reserve(s->keys, sizeof(unsigned long long) * s->tree_pool));
    for (DevBuf* b : {&s->t_parent, &s->t_node, &s->t_depth, &s->t_query, &s->t_weight})
      PS_TRY(devbuf_reserve(*b, sizeof(int32_t) * (s->tree_pool + s->qmax)));
    PS_TRY(devbuf_reserve(s->t_woff, sizeof(uint32_t) * s->tree_pool));
    PS_TRY(devbuf_reserve(s->t_walks, sizeof(int32_t) * s->tree_pool));
    PS_TRY(devbuf_reserve(s->ring, sizeof(int32_t) * s->ring_cap));
    PS_TRY(devbuf_reserve(s->ring_k, sizeof(int32_t) * s->ring_cap));
    s->tree_free.assign(1, {0, s->tree_pool});
  }
  PS_TRY(session_build(ctx, recs, bounds));
  PS_HIP(hipMemcpyAsync(s->h_ctr, s->counters.p, sizeof(uint64_t) * C_COUNT, hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  uint64_t levels = s->h_ctr[C_LEVELS] - before[C_LEVELS];
  const uint64_t probes = s->h_ctr[C_TAIL] - before[C_TAIL];
  int maxL = 2;
  for (auto& q : qs) maxL = std::max(maxL, q.prm.L);
  // Greedy list scheduling: every slot is busy while probes are pending, and a
  // probe holds its slot for depth-1 steps, so this many steps finish them all.
  uint64_t steps = probes ? (levels + P - 1) / P + (uint64_t)maxL + 2 : 0;
  double expand_ms = 0.0, pull_ms = 0.0;
  PS_TRY(session_set_pull(ctx, pull_threshold(g->m, pull_opt)));
  PS_TRY(session_steps(ctx, steps, &expand_ms, &pull_ms));
  bool hybrid = false;
  uint64_t with_probes = 0;
  for (size_t i = 0; i < qs.size(); ++i) {
    hybrid |= qs[i].hybrid != 0;
    with_probes += bounds[i] ? 1 : 0;
  }
  uint64_t total_steps = steps;
  // Probes switched under Section 4.4 queue randomized probes while the
  // steps run: those run in further batches of steps, sized the same way,
  // until every query is complete (a few batches at most; the cap is a guard).
  for (int round = 0; hybrid && round < 16; ++round) {
    PS_HIP(hipMemcpyAsync(s->h_ctr, s->counters.p, sizeof(uint64_t) * C_COUNT, hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    if (s->h_ctr[C_OVERFLOW] || s->h_ctr[C_DONE] - before[C_DONE] >= with_probes) break;
    const uint64_t lv = s->h_ctr[C_LEVELS] - before[C_LEVELS];
    steps = (lv - levels + P - 1) / P + (uint64_t)maxL + 2;
    levels = lv;
    PS_TRY(session_steps(ctx, steps, &expand_ms, &pull_ms));
    total_steps += steps;
  }
  std::vector<double> flips((size_t)nq, 0.0);
  for (int i = 0; i < nq; ++i) {
    QueryOut o = outs[(size_t)i];
    if (!o.flip) o.flip = &flips[(size_t)i];
    PS_TRY(session_finish(ctx, g, recs[(size_t)i], qs[(size_t)i], o));
  }
  PS_HIP(hipMemcpyAsync(s->h_ctr, s->counters.p, sizeof(uint64_t) * C_COUNT, hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nq; ++i) {
    const double f = outs[(size_t)i].flip && !ps_is_device_ptr(outs[(size_t)i].flip) ? *outs[(size_t)i].flip
                                                                                       : flips[(size_t)i];
    stats.flip_allowance = std::max(stats.flip_allowance, f);
  }
  const uint64_t* h = s->h_ctr;
  if (h[C_OVERFLOW]) {  // impossible with worst-case capacities; a guard
    report_overflow(s, h);
    return PS_ERR_OOM;
  }
  if (h[C_HEAD] != h[C_TAIL]) return PS_ERR_STATE;
  stats.walks = 0;
  for (auto& q : qs) stats.walks += q.walk_end - q.walk_begin;
  stats.walk_nodes = (int64_t)(h[C_WALK_NODES] - before[C_WALK_NODES]);
  stats.tree_nodes = (int64_t)probes;
  stats.probe_levels = (int64_t)(h[C_LEVELS] - before[C_LEVELS]);
  stats.steps = (int64_t)total_steps;
  stats.switched_probes = (int64_t)(h[C_SWITCH] - before[C_SWITCH]);
  stats.entries_expanded = (int64_t)(h[C_KEPT] - before[C_KEPT]);
  stats.entries_pruned = (int64_t)(h[C_PRUNED] - before[C_PRUNED]);
  stats.edges_scanned = (int64_t)(h[C_EDGES] - before[C_EDGES]);
  stats.next_entries = (int64_t)(h[C_NEXT] - before[C_NEXT]);
  stats.final_adds = (int64_t)(h[C_FINAL] - before[C_FINAL] + h[C_FINAL_PULL] - before[C_FINAL_PULL]);
  stats.pushed_final_adds = (int64_t)(h[C_FINAL] - before[C_FINAL]);
  stats.pushed_edges = stats.edges_scanned - (int64_t)(h[C_EDGES_UNPUSHED] - before[C_EDGES_UNPUSHED]);
  stats.expand_launches = (int64_t)total_steps;
  stats.pull_levels = (int64_t)(h[C_PULLS] - before[C_PULLS]);
  stats.pull_edges = (int64_t)(h[C_PULL_EDGES] - before[C_PULL_EDGES]);
  stats.near_threshold = (int64_t)(h[C_NEAR] - before[C_NEAR]);
  stats.expand_ms = expand_ms;
  stats.pull_ms = pull_ms;
  for (int b = 0; b < 32; ++b) {
    stats.level_hist_count[b] = (int64_t)(h[C_HIST_N + b] - before[C_HIST_N + b]);
    stats.level_hist_edges[b] = (int64_t)(h[C_HIST_E + b] - before[C_HIST_E + b]);
  }
  stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  ctx->last = stats;
  return PS_OK;
}
