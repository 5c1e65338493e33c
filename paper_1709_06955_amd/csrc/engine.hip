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


#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "ps_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kSchedBlock = 256;         // k_sched: one thread per slot
constexpr int kPickThreads = 1024;       // k_pick: one workgroup
constexpr int kThreads = 1024;           // k_expand and k_reduce workgroups
constexpr int kExpGrid = 256;            // k_expand workgroups (one per CU); segments per bin
constexpr int kRedGrid = 256;            // k_reduce workgroups
constexpr int kTile = kThreads;          // listed entries per tile in k_expand (one per thread)
constexpr uint32_t kBigDeg = 256;        // longer out-rows: one wavefront per kChunk edges
constexpr uint32_t kChunk = 512;
constexpr uint32_t kBigFlag = 0x80000000u;
constexpr int kMaxBins = 16384;          // record bins of a step: node ranges of 2^sh nodes
constexpr uint32_t kBinRecords = 8192;   // records per bin a step's bin width aims at
constexpr int kPartRows = 16;            // rows of per-slot partial sums (workgroups add into row wg % 16)
constexpr uint64_t kStepRecords = (uint64_t)kMaxBins * kBinRecords;  // records a step may write
constexpr int kMaxSh = 20;               // bin width limit: slot ids keep 12 bits of a key
constexpr int kTblBits = 13;             // LDS hash table of k_reduce: 2^13 (key, sum) pairs
constexpr uint32_t kTbl = 1u << kTblBits;
constexpr int kMaxProbe = 64;            // linear-probe steps before a slice splits
constexpr uint32_t kNoKey = 0xFFFFFFFFu;
constexpr int kMaxSlots = 2048;          // LDS arrays are sized for this many slots
constexpr int kSlotCap = 2000;           // slot ids stay below it, so no key equals kNoKey
constexpr int kWaveStage = 128;          // listed entries a wavefront of k_reduce stages in LDS
constexpr int kLanes = 64;               // dense frontier columns (one wavefront lane each)
constexpr unsigned long long kEmpty = ~0ull;
constexpr int kStepGrid = 2048;          // 8 workgroups per CU for the dense kernels

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
    if ((inserted || q.randomized) && !q.merged) {
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

// Publishes the probes queued so far to the next k_sched.
__global__ void k_snap_tail(unsigned long long* ctr) { ctr[C_TAIL_SNAP] = ctr[C_TAIL]; }

__global__ void k_reset_slots(Slot* slots, int32_t* has_next, int P) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= P) return;
  Slot st{};
  st.probe = -1;
  st.lane = -1;
  slots[s] = st;
  has_next[s] = 0;
}

__global__ void k_reset_lanes(int32_t* lane_slot) {
  if (threadIdx.x < kLanes) lane_slot[threadIdx.x] = -1;
}

// ------------------------------------------------------- level steps ----
//
// Probe scores.  The scores of inner levels are FP32 numbers.  The
// contributions that make up a level are summed exactly, as 64-bit integers
// on the grid 2^-62 (a level's scores never exceed 1), so no order of adds
// changes a bit; a level's FP32 score is its sum rounded to nearest.  Rule 2
// then compares FP32 numbers only, and the same query gives the same result
// alone, in a batch, pushed or pulled.
//
// Frontier lists.  The entries of every probe level about to be expanded
// (Rule 2 already applied) form one list of (slot, node) pairs with the
// node's FP32 score and out-row; lists alternate between two buffers by step
// parity.  An out-row longer than kBigDeg edges also gets chunks of kChunk
// edges in a chunk list, so that one wavefront takes each chunk (best effort:
// when the chunk list is full the row is expanded whole).
//
// A step.  k_sched advances, retires and assigns slots, lists the H_0 of new
// probes and takes the switch of Section 4.4; k_pick (only when levels may be
// pulled) moves large levels to dense columns.  k_expand pushes every listed
// entry along its out-edges: the contribution to (slot s, node v) becomes an
// 8-byte record in the bin of v's node range; each workgroup first counts
// its records per bin, so it writes them to exact, contiguous places.
// k_reduce sums each bin's records per (s, v) exactly in an LDS hash table,
// then applies Rule 2 to the next level and lists its survivors, or, on a
// probe's last level, adds weight * sum to the FP64 estimate.  No per-slot
// vector of n scores exists and no device-scope atomic is made per edge.
__device__ __forceinline__ long long to_grid(float c) { return __float2ll_rn(c * 0x1p62f); }
__device__ __forceinline__ float grid_f32(long long q) { return __ll2float_rn(q) * 0x1p-62f; }
__device__ __forceinline__ double grid_f64(long long q) { return (double)q * 0x1p-62; }

// Bijective mix of a 32-bit key (the MurmurHash3 finaliser): its low bits
// split a bin into slices, its high bits place a key in the LDS table.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

struct FList {
  int2* sn;     // (slot, node)
  float* val;   // the node's FP32 score (unused by randomized probes)
  uint2* row;   // its out-row: start, length | kBigFlag when chunked
  int2* chunk;  // (entry position, chunk index) of chunked rows; entry -1: empty
  unsigned long long* n_ent;    // kSubLists counters
  unsigned long long* n_chunk;  // kSubLists counters
  uint64_t sub_cap, sub_chunk_cap;  // places of one sub-list; sub-list k starts at k * sub_cap
};

__device__ __forceinline__ int wave_sublist() {
  return (int)(((blockIdx.x * blockDim.x + threadIdx.x) >> 6) & (kSubLists - 1));
}

// Writes n entries (at most 128, two per lane) to the wavefront's sub-list:
// entry i is (sn[i], h[i]) with out-row rowp[i]; rows longer than kBigDeg get
// chunks when the chunk sub-list has room.  One atomic for the entries and
// one for the chunks.  Every lane of the wavefront takes part.
__device__ void wave_write(int n, const int2* sn, const float* h, const uint2* rowp, const FList& L,
                           unsigned long long* ctr) {
  const int lane = lane_id();
  const int k = wave_sublist();
  uint2 row[2];
  uint32_t nch[2], mine = 0;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i = lane + 64 * j;
    row[j] = make_uint2(0u, 0u);
    nch[j] = 0;
    if (i < n) {
      row[j] = rowp[i];
      nch[j] = row[j].y > kBigDeg ? (row[j].y + kChunk - 1) / kChunk : 0u;
      mine += nch[j];
    }
  }
  const uint32_t incl = wave_incl_scan(mine);
  const uint32_t tot = __shfl(incl, 63, 64);
  unsigned long long eb = 0, cb = 0;
  if (lane == 0) {
    eb = atomicAdd(&L.n_ent[k], (unsigned long long)n);
    if (tot) cb = atomicAdd(&L.n_chunk[k], (unsigned long long)tot);
  }
  eb = __shfl(eb, 0, 64);
  cb = __shfl(cb, 0, 64);
  const bool room = cb + tot <= L.sub_chunk_cap;
  uint32_t c = incl - mine;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i = lane + 64 * j;
    if (i >= n) break;
    const unsigned long long off = eb + (unsigned long long)i;
    const bool fits = off < L.sub_cap;
    const unsigned long long pos = (unsigned long long)k * L.sub_cap + off;
    for (uint32_t q = 0; q < nch[j]; ++q, ++c) {
      const unsigned long long cq = cb + c;
      if (room && fits) L.chunk[(unsigned long long)k * L.sub_chunk_cap + cq] = make_int2((int32_t)pos, (int32_t)q);
      else if (cq < L.sub_chunk_cap) L.chunk[(unsigned long long)k * L.sub_chunk_cap + cq] = make_int2(-1, 0);
    }
    if (fits) {
      L.sn[pos] = sn[i];
      L.val[pos] = h[i];
      L.row[pos] = make_uint2(row[j].x, room && nch[j] ? (row[j].y | kBigFlag) : row[j].y);
    } else {
      atomicOr(&ctr[C_OVERFLOW], 4ull);
    }
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wavefront staging of listed entries in LDS: lanes put entries with no
// global atomic; a flush writes up to kWaveStage of them with one (and one
// for their chunks) to the wavefront's sub-list.  The wavefront's lanes all
// take part in every call (loops around the calls are wavefront-uniform).
struct WaveStage {
  int2* sn;
  float* h;
  uint2* row;
  int cap;  // at most kWaveStage
  int n;    // the same value in every lane
};

__device__ __forceinline__ void stage_flush(WaveStage& ws, const FList& L, unsigned long long* ctr) {
  if (ws.n == 0) return;
  wave_sync_lds();
  wave_write(ws.n, ws.sn, ws.h, ws.row, L, ctr);
  wave_sync_lds();
  ws.n = 0;
}

__device__ __forceinline__ void stage_put(bool want, int32_t s, int32_t v, float h, uint2 row, WaveStage& ws,
                                          const FList& L, unsigned long long* ctr) {
  const unsigned long long mask = __ballot(want);
  if (!mask) return;
  const int cnt = __popcll(mask);
  if (ws.n + cnt > ws.cap) stage_flush(ws, L, ctr);
  if (want) {
    const int pos = ws.n + __popcll(mask & ((1ull << lane_id()) - 1ull));
    ws.sn[pos] = make_int2(s, v);
    ws.h[pos] = h;
    ws.row[pos] = row;
  }
  ws.n += cnt;
}

// Exclusive scan of one value per thread over the workgroup; returns the
// prefix and writes the total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_wtot, uint32_t* total) {
  const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
  const uint32_t incl = wave_incl_scan(x);
  if (lane == 63) s_wtot[wv] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wv) before += s_wtot[w];
    tot += s_wtot[w];
  }
  *total = tot;
  __syncthreads();
  return before + incl - x;
}

struct SchedArgs {
  int P;
  int32_t n;
  int qmax;
  Slot* slots;
  int32_t* has_next;
  int32_t* pull_flag;  // in: last step's decision (3: paused); out: 0 push, 2 switched
  uint8_t* was_paused;
  int32_t* ring;
  int32_t* ring_k;
  uint64_t ring_mask;
  const int32_t* t_parent;
  const int32_t* t_node;
  const int32_t* t_depth;
  const int32_t* t_query;
  const int32_t* t_weight;
  const uint32_t* t_woff;
  const int32_t* t_walks;
  const QueryDev* qr;
  const float* thr_tab;
  unsigned long long* remaining;
  int32_t* done_ring;
  unsigned long long* hyb_edges;
  int32_t* lane_slot;
  uint32_t* part;  // kPartRows rows of partial (edges, entries) per slot of this step's list
  uint32_t* slot_edges;  // out: out-edges of each slot's listed entries
  uint32_t* slot_cnt;    // out: its listed entries
  uint4* cost;           // out: (records, next-list bound, entries, flags) of a pushed level
  FList list;            // this step's list (new probes' H_0 appended)
  FList next;            // next step's list (its counters cleared here)
  unsigned long long* ctr;
  int cur;
};

// Section 4.4: the deterministic probe in slot S stops (its listed level is
// dropped, so it retires at the next step) and each walk through its tree
// node is queued for a randomized probe of the same prefix.  A dense column it
// held still holds its level, which this step's pass overwrites with zeros,
// so it is free again only at the next step.
__device__ void switch_probe(const SchedArgs& a, Slot& S) {
  if (S.lane >= 0) {
    a.lane_slot[S.lane] = -2;
    atomicOr(&a.ctr[C_SWLANES], 1ull << S.lane);
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

// One thread per slot.  Advances every slot by one PROBE iteration (a slot
// paused last step stays at its level), retires probes whose last level
// (i-2) ran or whose frontier Rule 2 emptied, and hands free slots the next
// pending probes in ring order (each workgroup claims a range of the ring).
// A new probe on (u_1..u_i) starts with H_0 = {u_i: 1}, listed here after
// Rule 2.  Sums each slot's listed out-edges and entries from the partial
// sums of the last step's kernels, then takes the switch of Section 4.4 for
// hybrid queries: a deterministic probe switches when the level it is about
// to expand keeps more than c0 * w * n out-edges.
__global__ void __launch_bounds__(kSchedBlock) k_sched(SchedArgs a) {
  __shared__ uint32_t s_wtot[kSchedBlock / 64];
  __shared__ unsigned long long s_base, s_take;

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid >> 6;
  const int s = blockIdx.x * kSchedBlock + tid;
  unsigned long long* ctr = a.ctr;
  __shared__ int2 w_sn[kSchedBlock];
  __shared__ float w_h[kSchedBlock];
  __shared__ uint2 w_row[kSchedBlock];
  if (blockIdx.x == 0 && tid < kSubLists) {
    a.next.n_ent[tid] = 0;
    a.next.n_chunk[tid] = 0;
  }
  if (blockIdx.x == 0 && tid == 0) {
    ctr[C_REC] = 0;
    ctr[C_BIN] = kRedGrid;  // k_reduce's workgroups start on bins 0..kRedGrid-1
    ctr[C_NZROWS0 + (a.cur ^ 1)] = 0;  // the dense pass rewrites that matrix this step
  }
  const bool valid = s < a.P;
  bool need = false, paused = false;
  uint32_t E = 0, F = 0;
  if (valid) {
    Slot& S = a.slots[s];
    paused = a.pull_flag[s] == 3;
    a.was_paused[s] = paused ? 1 : 0;
    if (S.probe >= 0) {
      if (paused) {
        // its entries were carried into this step's list unchanged
      } else if (S.last || !a.has_next[s]) {
        const int q = S.query;
        if (atomicAdd(&a.remaining[q], ~0ull) == 1ull) {  // last probe of the query
          const unsigned long long pos = atomicAdd(&ctr[C_DONE], 1ull);
          a.done_ring[pos % (unsigned long long)a.qmax] = q;
        }
        // a column after a last or empty level holds zeros: free at once
        if (S.lane >= 0) a.lane_slot[S.lane] = -1;
        S.probe = -1;
        S.lane = -1;
        need = true;
      } else {
        S.level = S.level + 1;
        S.cursor = a.t_parent[S.cursor];
      }
    } else {
      need = true;
    }
    a.has_next[s] = 0;
    // the sums the last step's kernels added for this slot; the rows are
    // cleared for this step's kernels
    uint32_t pe[kPartRows], pf[kPartRows];
#pragma unroll
    for (int r = 0; r < kPartRows; ++r) {
      pe[r] = a.part[(size_t)r * 2 * a.P + s];
      pf[r] = a.part[(size_t)r * 2 * a.P + a.P + s];
    }
#pragma unroll
    for (int r = 0; r < kPartRows; ++r) {
      a.part[(size_t)r * 2 * a.P + s] = 0u;
      a.part[(size_t)r * 2 * a.P + a.P + s] = 0u;
      if (!need && S.lane < 0) {
        E += pe[r];
        F += pf[r];
      }
    }
  }
  // free slots of this workgroup claim a range of pending probes
  const uint32_t incl = wave_incl_scan(need ? 1u : 0u);
  if (lane == 63) s_wtot[wv] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kSchedBlock / 64; ++w) {
    if (w < wv) before += s_wtot[w];
    total += s_wtot[w];
  }
  if (tid == 0) {
    unsigned long long h = 0, take = 0;
    if (total) {
      const unsigned long long lim = __hip_atomic_load(&ctr[C_TAIL_SNAP], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      h = __hip_atomic_load(&ctr[C_HEAD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (;;) {
        take = h < lim ? min((unsigned long long)total, lim - h) : 0ull;
        if (!take) break;
        const unsigned long long prev = atomicCAS(&ctr[C_HEAD], h, h + take);
        if (prev == h) break;
        h = prev;
      }
    }
    s_base = h;
    s_take = take;
  }
  __syncthreads();
  const unsigned long long rank = before + incl - (need ? 1u : 0u);
  bool want = false;
  int32_t x = 0;
  uint2 row = make_uint2(0u, 0u);
  unsigned long long n0 = 0, kept = 0, pruned = 0, near = 0;
  if (valid && need && rank < s_take) {
    Slot& S = a.slots[s];
    const uint64_t rp = (s_base + rank) & a.ring_mask;
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
    x = a.t_node[t];
    row = Q.out_rows[x];
    n0 = 1;
    bool keep = true;  // Alg. 4 has no Rule 2
    if (!mode) {       // Rule 2 on H_0 = {u_i: 1}
      const float thr = a.thr_tab[q * PS_MAX_WALK_LEN + S.depth - 1];
      if (fabsf(1.0f - thr) <= 1e-5f * thr) {
        ++near;
        unsafeAtomicAdd(S.flip, S.flip_unit);
      }
      keep = 1.0f > thr;
      kept = keep ? 1 : 0;
      pruned = keep ? 0 : 1;
    }
    want = keep && row.y > 0;
  }
  {
    WaveStage ws{w_sn + (tid & ~63), w_h + (tid & ~63), w_row + (tid & ~63), 64, 0};
    stage_put(want, s, x, 1.0f, row, ws, a.list, ctr);
    stage_flush(ws, a.list, ctr);
  }
  if (want) {
    E = row.y;
    F = 1;
  }
  int32_t pf = 0;
  unsigned long long te = 0, tn = 0, tf = 0;
  if (valid) {
    Slot& S = a.slots[s];
    if (S.probe >= 0) {
      const int level = S.level, depth = S.depth, q = S.query;
      const int e = depth - level - 1;  // iterations left, i-j-1 >= 1
      S.thr = a.thr_tab[q * PS_MAX_WALK_LEN + e];
      S.thr_next = e > 1 ? a.thr_tab[q * PS_MAX_WALK_LEN + e - 1] : 0.0f;
      S.excl = a.t_node[S.cursor];
      S.last = level == depth - 2;
      if (S.hyb_thr >= 0.0) {
        unsigned long long he = E;
        if (S.lane >= 0) {  // dense column: the count of the last pass
          he = a.hyb_edges[s];
          a.hyb_edges[s] = 0;
        }
        if ((double)he > S.hyb_thr) {
          switch_probe(a, S);
          pf = 2;
        }
      }
      if (E && !paused) {  // probe levels by the out-edge count of their kept entries
        const int b = 31 - __clz((int)E);
        atomicAdd(&ctr[C_HIST_N + b], 1ull);
        atomicAdd(&ctr[C_HIST_E + b], (unsigned long long)E);
      }
      if (pf == 0 && S.lane < 0) {
        te = S.mode ? 0 : E;
        tn = S.last ? 0 : min(E, (uint32_t)a.n);
        tf = F;
      }
    }
    a.pull_flag[s] = pf;
    a.slot_edges[s] = E;
    a.slot_cnt[s] = F;
    // what pushing this level costs the step budget (k_expand); flag bit 0:
    // a candidate, bit 1: not paused last step (lower priority)
    const bool cand = S.probe >= 0 && S.lane < 0 && pf == 0 && F > 0;
    a.cost[s] = make_uint4((uint32_t)te, (uint32_t)tn, F, (cand ? 1u : 0u) | (paused ? 0u : 2u));
  }
  n0 = wave_sum(n0);
  kept = wave_sum(kept);
  pruned = wave_sum(pruned);
  near = wave_sum(near);
  te = wave_sum(te);
  tn = wave_sum(tn);
  tf = wave_sum(tf);
  if (lane == 0) {
    if (n0) atomicAdd(&ctr[C_LEVEL0], n0);
    if (kept) atomicAdd(&ctr[C_KEPT], kept);
    if (pruned) atomicAdd(&ctr[C_PRUNED], pruned);
    if (near) atomicAdd(&ctr[C_NEAR], near);
    if (te) atomicAdd(&ctr[C_TOT_E], te);
    if (tn) atomicAdd(&ctr[C_TOT_N], tn);
    if (tf) atomicAdd(&ctr[C_TOT_F], tf);
  }
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

struct PickArgs {
  int P;
  int32_t n;
  uint4* cost;
  Slot* slots;
  int32_t* pull_flag;
  int32_t* lane_slot;
  DenseVer* dv;
  const uint32_t* slot_edges;
  const uint32_t* slot_cnt;
  unsigned long long* ctr;
};

// One workgroup, run only when levels may be pulled.  Moves pushed sparse
// slots whose listed entries have at least ctr[C_PULL_T] out-edges into free
// dense columns, as long as they read the graph version the dense pass uses
// (fixed by the columns active at the start, or by the first slot moved).
// Their entries are scattered into the dense matrix by k_expand this step.
// A column freed by a switch becomes free one step later.  Also sets the
// column range of this step's dense pass and records the version's arrays.
__global__ void __launch_bounds__(kPickThreads) k_pick(PickArgs a) {
  __shared__ int32_t s_free[kLanes];
  __shared__ uint32_t s_nfree, s_ncand;
  __shared__ unsigned long long s_ver;
  const int tid = threadIdx.x;
  unsigned long long* ctr = a.ctr;
  const unsigned long long sw = ctr[C_SWLANES];
  if (tid == 0) {
    s_nfree = 0;
    s_ncand = 0;
    s_ver = 0ull;
  }
  __syncthreads();
  if (tid < kLanes) {  // one wavefront: free columns listed lowest first
    int32_t ls = a.lane_slot[tid];
    if (ls == -2 && !((sw >> tid) & 1ull)) {  // switched at an earlier step: zero by now
      a.lane_slot[tid] = -1;
      ls = -1;
    }
    const unsigned long long freem = __ballot(ls == -1);
    if (ls == -1) s_free[__popcll(freem & ((1ull << tid) - 1ull))] = tid;
    else if (ls >= 0) s_ver = (unsigned long long)a.slots[ls].in_rows;  // all active columns share it
    if (tid == 0) s_nfree = (uint32_t)__popcll(freem);
  }
  __syncthreads();
  const unsigned long long T = ctr[C_PULL_T];
  unsigned long long de = 0, dn = 0, df = 0;
  for (int s = tid; s < a.P; s += blockDim.x) {
    Slot& S = a.slots[s];
    const uint32_t e = a.slot_edges[s];
    if (S.probe < 0 || S.lane >= 0 || S.mode || a.pull_flag[s] != 0 || e == 0 || e < T) continue;
    const unsigned long long ver = (unsigned long long)S.in_rows;
    const unsigned long long old = atomicCAS(&s_ver, 0ull, ver);
    if ((old == 0ull ? ver : old) != ver) continue;
    const uint32_t k = atomicAdd(&s_ncand, 1u);
    if (k >= s_nfree) continue;
    const int32_t lane = s_free[k];
    S.lane = lane;
    a.lane_slot[lane] = s;
    a.pull_flag[s] = 1;
    a.cost[s].w &= ~1u;  // pulled: not pushed
    de += e;
    dn += S.last ? 0 : min(e, (uint32_t)a.n);
    df += a.slot_cnt[s];
  }
  if (de) atomicAdd(&ctr[C_TOT_E], 0ull - de);
  if (dn) atomicAdd(&ctr[C_TOT_N], 0ull - dn);
  if (df) atomicAdd(&ctr[C_TOT_F], 0ull - df);
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
      const unsigned long long fhi = sw ? (unsigned long long)(64 - __clzll((long long)sw)) : 0ull;
      const unsigned long long prev = ctr[C_GPREV];
      ctr[C_GHI] = hi;
      ctr[C_GW] = max(max(hi, prev), fhi);
      // a column freed by a switch still holds its level in this step's
      // input matrix, which the next step writes: it counts as in use until then
      ctr[C_GPREV] = max(hi, fhi);
      if (act) atomicAdd(&ctr[C_PULLS], (unsigned long long)__popcll(act));
      ctr[C_HYBMASK] = hmask;
      ctr[C_SWLANES] = 0ull;
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
  int P;
  int sh_min;  // smallest bin shift that keeps the bins within kMaxBins
  const Slot* slots;
  int32_t* pull_flag;
  const uint4* cost;
  FList cur, nxt;
  uint2* rec;  // records: (slot << sh | v & mask, FP32 contribution bits)
  uint64_t rec_cap;
  uint2* seg;  // seg[bin * kExpGrid + workgroup] = (first record, count)
  float* mat_cur;
  uint8_t* map_cur;
  int32_t* has_next;
  uint32_t* part;
  uint64_t list_soft;  // entries the next list may take before slots pause
  unsigned long long* ctr;
  int cur_par;
};

__device__ __forceinline__ long long wave_incl_scan64(long long x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Pauses (slow path of the per-step budget).  The records of the pushed
// levels must fit rec_cap, and the next list list_soft: a pushed inner
// level lists at most min(out-edges, n) entries, a paused level keeps its
// entries, a pushed last level lists none.  Every workgroup decides the same
// way: slots in priority order (those paused last step first, then by
// index) are pushed as long as the running sums fit; the others keep their
// listed level for a later step.  The first slot in that order is always
// pushed (the capacity guards report it if even that does not fit).
// Returns the records of the pushed levels.
__device__ unsigned long long decide_pauses(const ExpandArgs& a, uint32_t* s_pause, long long* s_w0,
                                            long long* s_w1) {
  __shared__ unsigned long long s_base, s_adm;
  __shared__ int s_first;
  const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
  const int per = (a.P + (int)blockDim.x - 1) / (int)blockDim.x;
  for (int i = tid; i < (a.P + 31) / 32; i += blockDim.x) s_pause[i] = 0u;
  if (tid == 0) {
    s_base = 0;
    s_adm = 0;
    s_first = 0x7fffffff;
  }
  __syncthreads();
  unsigned long long base = 0;  // entries of every candidate, as if all were carried
  long long rec[2] = {0, 0}, grow[2] = {0, 0};
  for (int k = 0; k < per; ++k) {
    const int s = tid * per + k;
    if (s >= a.P) break;
    const uint4 c = a.cost[s];
    if (!(c.w & 1u)) continue;
    const int g = (c.w >> 1) & 1u;
    base += c.z;
    rec[g] += (long long)c.x;
    grow[g] += (long long)c.y - (long long)c.z;
    atomicMin(&s_first, g * a.P + s);
  }
  base = wave_sum(base);
  if (lane == 0 && base) atomicAdd(&s_base, base);
  // prefix sums in priority order: group 0 (paused last step), then group 1
  long long pre_rec[2], pre_grow[2];
  for (int g = 0; g < 2; ++g) {
    const long long ir = wave_incl_scan64(rec[g]);
    const long long ig = wave_incl_scan64(grow[g]);
    if (lane == 63) {
      s_w0[g * 32 + wv] = ir;
      s_w1[g * 32 + wv] = ig;
    }
    pre_rec[g] = ir - rec[g];
    pre_grow[g] = ig - grow[g];
  }
  __syncthreads();
  long long tot_rec0 = 0, tot_grow0 = 0;
  for (int g = 0; g < 2; ++g) {
    long long br = 0, bg = 0, tr = 0, tg = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      if (w < wv) {
        br += s_w0[g * 32 + w];
        bg += s_w1[g * 32 + w];
      }
      tr += s_w0[g * 32 + w];
      tg += s_w1[g * 32 + w];
    }
    pre_rec[g] += br;
    pre_grow[g] += bg;
    if (g == 0) {
      tot_rec0 = tr;
      tot_grow0 = tg;
    }
  }
  const long long lim_rec = (long long)min(a.rec_cap, (unsigned long long)kStepRecords);
  const long long lim_list = (long long)a.list_soft - (long long)s_base;
  unsigned long long paused = 0, adm = 0;
  for (int g = 0; g < 2; ++g) {
    long long cr = pre_rec[g] + (g ? tot_rec0 : 0), cg = pre_grow[g] + (g ? tot_grow0 : 0);
    for (int k = 0; k < per; ++k) {
      const int s = tid * per + k;
      if (s >= a.P) break;
      const uint4 c = a.cost[s];
      if (!(c.w & 1u) || (int)((c.w >> 1) & 1u) != g) continue;
      cr += (long long)c.x;
      cg += (long long)c.y - (long long)c.z;
      if ((cr <= lim_rec && cg <= lim_list) || g * a.P + s == s_first) {
        adm += c.x;
      } else {
        atomicOr(&s_pause[s >> 5], 1u << (s & 31));
        ++paused;
      }
    }
  }
  adm = wave_sum(adm);
  if (lane == 0 && adm) atomicAdd(&s_adm, adm);
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int s = tid; s < a.P; s += blockDim.x)
      if ((s_pause[s >> 5] >> (s & 31)) & 1u) a.pull_flag[s] = 3;
    paused = wave_sum(paused);
    if (lane == 0 && paused) atomicAdd(&a.ctr[C_PAUSED], paused);
  }
  return s_adm;
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
__device__ __forceinline__ bool visit_random(int32_t v, int32_t x, const Slot& sl, unsigned long long& nfinal) {
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

// What happens to a listed entry of slot s this step.
enum EntryFate { kPush = 0, kPull = 1, kDrop = 2, kCarry = 3 };

__device__ __forceinline__ int entry_fate(const ExpandArgs& a, int32_t s, bool slow, const uint32_t* s_pause) {
  const int32_t pf = a.pull_flag[s];
  if (pf == 1) return kPull;
  if (pf == 2) return kDrop;
  // 0 or 3 (the pause flag other workgroups may be writing)
  if (slow && ((s_pause[s >> 5] >> (s & 31)) & 1u)) return kCarry;
  return kPush;
}

// PROBE expansion (Alg. 2 per listed entry, Alg. 4 for randomized probes).
// Workgroups take tiles of kTile listed entries, scan their out-degrees in
// LDS and walk the tile's edges kThreads at a time, each thread finding its
// entry by binary search, so the work per thread is one edge whatever the
// degree mix; chunked long rows go one wavefront per chunk.  Pass 1 counts
// the records of each bin, pass 2 writes them (and lists randomized probes'
// next sets, carries paused slots' entries and scatters pulled slots'
// entries into the dense matrix).
constexpr int kEdgeBatch = 4;  // edges a thread has in flight

// Entry j of a tile whose edge e (tile-relative) a thread takes: the last j
// with s_pref[j] <= e.
__device__ __forceinline__ int tile_entry(const uint32_t* s_pref, uint32_t e) {
  int lo = 0, hi = kTile - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_pref[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(kThreads) k_expand(ExpandArgs a) {
  __shared__ uint32_t s_hist[kMaxBins];
  __shared__ uint32_t s_pref[kTile + 1];
  __shared__ int32_t s_slot[kTile];  // slot, with kBigFlag set for a randomized probe
  __shared__ const int32_t* s_col[kTile];  // the entry's out-row
  __shared__ int32_t s_excl[kTile];
  __shared__ float s_sv[kTile];
  __shared__ int32_t s_x[kTile];
  __shared__ uint32_t s_part[2 * kMaxSlots];
  __shared__ uint32_t s_pause[kMaxSlots / 32];
  __shared__ uint32_t s_wtot[kThreads / 64];
  __shared__ long long s_w0[64], s_w1[64];
  __shared__ unsigned long long s_rbase;
  __shared__ int s_dirty, s_skip;
  __shared__ uint32_t s_cnt[kSubLists], s_tpre[kSubLists + 1], s_cpre[kSubLists + 1];
  __shared__ int2 w_sn[kThreads];  // one 64-entry stage per wavefront
  __shared__ float w_h[kThreads];
  __shared__ uint2 w_row[kThreads];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  unsigned long long* ctr = a.ctr;
  const unsigned long long tot_e = ctr[C_TOT_E], tot_n = ctr[C_TOT_N];
  const bool slow = tot_e > min(a.rec_cap, (unsigned long long)kStepRecords) || tot_n > a.list_soft;
  const unsigned long long recs = slow ? decide_pauses(a, s_pause, s_w0, s_w1) : tot_e;
  // bin width of this step: about kBinRecords records per bin (v >> sh)
  uint32_t sh = (uint32_t)a.sh_min;
  while (sh < (uint32_t)kMaxSh && ((unsigned long long)a.n >> (sh + 1)) * kBinRecords >= recs) ++sh;
  const int nbins = (int)(((uint32_t)a.n - 1u) >> sh) + 1;
  if (blockIdx.x == 0 && tid == 0) {
    ctr[C_SH] = sh;
    ctr[C_NB] = (unsigned long long)nbins;
  }
  for (int b = tid; b < nbins; b += kThreads) s_hist[b] = 0u;
  if (tid == 0) {
    s_dirty = 0;
    s_skip = 0;
    // tiles of kTile entries and chunks in each sub-list of this step's list
    uint32_t tp = 0, cp = 0;
    for (int k = 0; k < kSubLists; ++k) {
      const uint32_t c = (uint32_t)min(a.cur.n_ent[k], (unsigned long long)a.cur.sub_cap);
      s_cnt[k] = c;
      s_tpre[k] = tp;
      s_cpre[k] = cp;
      tp += (c + kTile - 1) / kTile;
      cp += (uint32_t)min(a.cur.n_chunk[k], (unsigned long long)a.cur.sub_chunk_cap);
    }
    s_tpre[kSubLists] = tp;
    s_cpre[kSubLists] = cp;
  }
  __syncthreads();
  const uint32_t ntiles = s_tpre[kSubLists];
  const uint32_t nchunk = s_cpre[kSubLists];
  const uint32_t vmask = (1u << sh) - 1u;
  const uint64_t wave = ((uint64_t)blockIdx.x * kThreads + tid) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * kThreads) >> 6;

  // ---- pass 1: records per bin
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int k = 0;
    while (k + 1 < kSubLists && s_tpre[k + 1] <= t) ++k;
    const uint32_t lt = t - s_tpre[k];
    const bool in = lt * kTile + (uint32_t)tid < s_cnt[k];  // this thread's entry exists
    const uint64_t i = (uint64_t)k * a.cur.sub_cap + (uint64_t)lt * kTile + tid;
    uint32_t deg = 0;
    if (in) {
      const uint2 row = a.cur.row[i];
      if (!(row.y & kBigFlag)) {
        const int32_t s = a.cur.sn[i].x;
        const Slot& sl = a.slots[s];
        if (entry_fate(a, s, slow, s_pause) == kPush && !sl.mode) {
          deg = row.y;
          s_col[tid] = sl.out_col + row.x;
          s_excl[tid] = sl.excl;
        }
      }
    }
    uint32_t total;
    s_pref[tid] = block_excl_scan(deg, s_wtot, &total);
    if (tid == 0) s_pref[kTile] = total;
    __syncthreads();
    for (uint32_t e0 = 0; e0 < total; e0 += kThreads * kEdgeBatch) {
      int32_t v[kEdgeBatch], ex[kEdgeBatch];
#pragma unroll
      for (int k = 0; k < kEdgeBatch; ++k) {
        const uint32_t e = e0 + (uint32_t)(k * kThreads + tid);
        v[k] = -1;
        ex[k] = -1;
        if (e < total) {
          const int lo = tile_entry(s_pref, e);
          v[k] = s_col[lo][e - s_pref[lo]];
          ex[k] = s_excl[lo];
        }
      }
#pragma unroll
      for (int k = 0; k < kEdgeBatch; ++k)
        if (v[k] >= 0 && v[k] != ex[k]) atomicAdd(&s_hist[(uint32_t)v[k] >> sh], 1u);
    }
    __syncthreads();
  }
  for (uint64_t c = wave; c < nchunk; c += nwaves) {
    int k = 0;
    while (k + 1 < kSubLists && s_cpre[k + 1] <= c) ++k;
    const int2 ch = a.cur.chunk[(uint64_t)k * a.cur.sub_chunk_cap + (c - s_cpre[k])];
    if (ch.x < 0) continue;
    const uint64_t ek = (uint64_t)ch.x / a.cur.sub_cap;  // the entry's sub-list
    if (ek >= kSubLists || (uint64_t)ch.x - ek * a.cur.sub_cap >= s_cnt[ek]) continue;
    const int32_t s = a.cur.sn[ch.x].x;
    if (entry_fate(a, s, slow, s_pause) != kPush) continue;
    const Slot& sl = a.slots[s];
    if (sl.mode) continue;
    const uint2 row = a.cur.row[ch.x];
    const uint32_t len = row.y & ~kBigFlag;
    const uint32_t b = (uint32_t)ch.y * kChunk, e = min(len, b + kChunk);
    const int32_t* col = sl.out_col + row.x;
    const int32_t ex = sl.excl;
    for (uint32_t t0 = b; t0 < e; t0 += 64 * kEdgeBatch) {
      int32_t v[kEdgeBatch];
#pragma unroll
      for (int k = 0; k < kEdgeBatch; ++k) {
        const uint32_t t = t0 + (uint32_t)(k * 64 + lane);
        v[k] = t < e ? col[t] : -1;
      }
#pragma unroll
      for (int k = 0; k < kEdgeBatch; ++k)
        if (v[k] >= 0 && v[k] != ex) atomicAdd(&s_hist[(uint32_t)v[k] >> sh], 1u);
    }
  }
  __syncthreads();
  // this workgroup's records: one contiguous range, cut by bin
  {
    uint32_t mine = 0;
    const int per = (nbins + kThreads - 1) / kThreads;
    for (int k = 0; k < per; ++k) {
      const int b = tid * per + k;
      if (b < nbins) mine += s_hist[b];
    }
    uint32_t total;
    const uint32_t pre = block_excl_scan(mine, s_wtot, &total);
    if (tid == 0) {
      const unsigned long long base = total ? atomicAdd(&ctr[C_REC], (unsigned long long)total) : 0ull;
      s_rbase = base;
      if (base + total > a.rec_cap) {
        s_skip = 1;  // a guard: the budget keeps records within capacity
        atomicOr(&ctr[C_OVERFLOW], 8ull);
      }
    }
    __syncthreads();
    uint32_t run = (uint32_t)s_rbase + pre;
    for (int k = 0; k < per; ++k) {
      const int b = tid * per + k;
      if (b >= nbins) break;
      const uint32_t c = s_hist[b];
      a.seg[(size_t)b * kExpGrid + blockIdx.x] = make_uint2(run, s_skip ? 0u : c);
      s_hist[b] = run;  // write cursor of pass 2
      run += c;
    }
  }
  for (int i = tid; i < 2 * a.P; i += kThreads) s_part[i] = 0u;
  __syncthreads();

  // ---- pass 2
  const bool skip = s_skip != 0;
  WaveStage ws{w_sn + (tid & ~63), w_h + (tid & ~63), w_row + (tid & ~63), 64, 0};
  unsigned long long nfinal = 0, nnext = 0, nconv = 0, edges = 0, unpushed = 0;
  bool dirty = false;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int k = 0;
    while (k + 1 < kSubLists && s_tpre[k + 1] <= t) ++k;
    const uint32_t lt = t - s_tpre[k];
    const bool in = lt * kTile + (uint32_t)tid < s_cnt[k];  // this thread's entry exists
    const uint64_t i = (uint64_t)k * a.cur.sub_cap + (uint64_t)lt * kTile + tid;
    uint32_t deg = 0;
    bool carry = false;
    int32_t cs = 0, cx = 0;
    float cval = 0.0f;
    uint2 crow = make_uint2(0u, 0u);
    if (in) {
      const int2 it = a.cur.sn[i];
      const uint2 row = a.cur.row[i];
      const uint32_t len = row.y & ~kBigFlag;
      const int fate = entry_fate(a, it.x, slow, s_pause);
      if (fate == kPull) {  // scattered into the slot's dense column
        a.mat_cur[(size_t)it.y * kLanes + a.slots[it.x].lane] = a.cur.val[i];
        a.map_cur[it.y] = 1;
        ++nconv;
        edges += len;
        unpushed += len;
      } else if (fate == kDrop) {  // switched probe (Section 4.4): the level is dropped
        edges += len;
        unpushed += len;
      } else if (fate == kCarry) {
        carry = true;
        cs = it.x;
        cx = it.y;
        cval = a.cur.val[i];
        crow = make_uint2(row.x, len);
      } else {
        edges += len;
        if (!(row.y & kBigFlag)) {
          const Slot& sl = a.slots[it.x];
          deg = row.y;
          s_slot[tid] = sl.mode ? (int32_t)((uint32_t)it.x | kBigFlag) : it.x;
          s_col[tid] = sl.out_col + row.x;
          s_excl[tid] = sl.excl;
          s_x[tid] = it.y;
          s_sv[tid] = a.cur.val[i] * sl.sc;  // fl32(Score(x) * sqrt c)
        }
      }
    }
    stage_put(carry, cs, cx, cval, crow, ws, a.nxt, ctr);
    if (carry) {
      a.has_next[cs] = 1;
      atomicAdd(&s_part[cs], crow.y);
      atomicAdd(&s_part[a.P + cs], 1u);
      dirty = true;
    }
    uint32_t total;
    s_pref[tid] = block_excl_scan(deg, s_wtot, &total);
    if (tid == 0) s_pref[kTile] = total;
    __syncthreads();
    for (uint32_t e0 = 0; e0 < total; e0 += kThreads * kEdgeBatch) {
      int32_t v[kEdgeBatch], lo[kEdgeBatch];
#pragma unroll
      for (int k = 0; k < kEdgeBatch; ++k) {
        const uint32_t e = e0 + (uint32_t)(k * kThreads + tid);
        v[k] = -1;
        lo[k] = 0;
        if (e < total) {
          lo[k] = tile_entry(s_pref, e);
          v[k] = s_col[lo[k]][e - s_pref[lo[k]]];
        }
      }
#pragma unroll
      for (int k = 0; k < kEdgeBatch; ++k) {  // Alg. 2: the deterministic entries' records
        const int32_t s = s_slot[lo[k]];
        if (v[k] >= 0 && s >= 0 && v[k] != s_excl[lo[k]] && !skip) {
          const uint32_t pos = atomicAdd(&s_hist[(uint32_t)v[k] >> sh], 1u);
          a.rec[pos] = make_uint2(((uint32_t)s << sh) | ((uint32_t)v[k] & vmask), __float_as_uint(s_sv[lo[k]]));
        }
      }
#pragma unroll
      for (int k = 0; k < kEdgeBatch; ++k) {  // Alg. 4: the randomized entries
        bool app = false;
        int32_t s = 0;
        uint2 vrow = make_uint2(0u, 0u);
        if (v[k] >= 0 && s_slot[lo[k]] < 0) {
          s = (int32_t)((uint32_t)s_slot[lo[k]] & ~kBigFlag);
          const Slot& sl = a.slots[s];
          if (visit_random(v[k], s_x[lo[k]], sl, nfinal)) {
            ++nnext;
            vrow = sl.out_rows[v[k]];
            app = vrow.y > 0;
          }
        }
        stage_put(app, s, v[k], 0.0f, vrow, ws, a.nxt, ctr);
        if (app) {
          a.has_next[s] = 1;
          atomicAdd(&s_part[s], vrow.y);
          atomicAdd(&s_part[a.P + s], 1u);
          dirty = true;
        }
      }
    }
    __syncthreads();
  }
  for (uint64_t c = wave; c < nchunk; c += nwaves) {
    int k = 0;
    while (k + 1 < kSubLists && s_cpre[k + 1] <= c) ++k;
    const int2 ch = a.cur.chunk[(uint64_t)k * a.cur.sub_chunk_cap + (c - s_cpre[k])];
    if (ch.x < 0) continue;
    const uint64_t ek = (uint64_t)ch.x / a.cur.sub_cap;  // the entry's sub-list
    if (ek >= kSubLists || (uint64_t)ch.x - ek * a.cur.sub_cap >= s_cnt[ek]) continue;
    const int2 it = a.cur.sn[ch.x];
    const int32_t s = it.x;
    if (entry_fate(a, s, slow, s_pause) != kPush) continue;
    const Slot& sl = a.slots[s];
    const uint2 row = a.cur.row[ch.x];
    const float sv = a.cur.val[ch.x] * sl.sc;
    const uint32_t len = row.y & ~kBigFlag;
    const uint32_t b = (uint32_t)ch.y * kChunk, e = min(len, b + kChunk);
    const int32_t* col = sl.out_col + row.x;
    if (!sl.mode) {  // Alg. 2
      for (uint32_t t0 = b; t0 < e; t0 += 64 * kEdgeBatch) {
        int32_t v[kEdgeBatch];
#pragma unroll
        for (int k = 0; k < kEdgeBatch; ++k) {
          const uint32_t t = t0 + (uint32_t)(k * 64 + lane);
          v[k] = t < e ? col[t] : -1;
        }
#pragma unroll
        for (int k = 0; k < kEdgeBatch; ++k) {
          if (v[k] >= 0 && v[k] != sl.excl && !skip) {
            const uint32_t pos = atomicAdd(&s_hist[(uint32_t)v[k] >> sh], 1u);
            a.rec[pos] = make_uint2(((uint32_t)s << sh) | ((uint32_t)v[k] & vmask), __float_as_uint(sv));
          }
        }
      }
      continue;
    }
    for (uint32_t t0 = b; t0 < e; t0 += 64) {  // Alg. 4
      const uint32_t t = t0 + lane;
      bool app = false;
      int32_t v = 0;
      uint2 vrow = make_uint2(0u, 0u);
      if (t < e) {
        v = col[t];
        if (visit_random(v, it.y, sl, nfinal)) {
          ++nnext;
          vrow = sl.out_rows[v];
          app = vrow.y > 0;
        }
      }
      stage_put(app, s, v, 0.0f, vrow, ws, a.nxt, ctr);
      if (app) {
        a.has_next[s] = 1;
        atomicAdd(&s_part[s], vrow.y);
        atomicAdd(&s_part[a.P + s], 1u);
        dirty = true;
      }
    }
  }
  stage_flush(ws, a.nxt, ctr);
  if (dirty) s_dirty = 1;
  __syncthreads();
  // partial per-slot sums of what this workgroup listed (k_sched adds them up)
  if (s_dirty) {
    uint32_t* prow = a.part + (size_t)(blockIdx.x % kPartRows) * 2 * a.P;
    for (int i = tid; i < 2 * a.P; i += kThreads)
      if (s_part[i]) atomicAdd(&prow[i], s_part[i]);
  }
  nfinal = wave_sum(nfinal);
  nnext = wave_sum(nnext);
  nconv = wave_sum(nconv);
  edges = wave_sum(edges);
  unpushed = wave_sum(unpushed);
  if (lane == 0) {
    if (nfinal) atomicAdd(&ctr[C_FINAL], nfinal);
    if (nnext) atomicAdd(&ctr[C_NEXT], nnext);
    if (nconv) atomicAdd(&ctr[C_NZROWS0 + a.cur_par], nconv);  // rows given scores in the dense matrix
    if (edges) atomicAdd(&ctr[C_EDGES], edges);
    if (unpushed) atomicAdd(&ctr[C_EDGES_UNPUSHED], unpushed);
  }
}

struct ReduceArgs {
  int32_t n;
  int P;
  const Slot* slots;
  const uint2* rec;
  const uint2* seg;
  FList nxt;
  int32_t* has_next;
  uint32_t* part;
  unsigned long long* ctr;
};

constexpr int kRecBatch = 4;  // records a thread loads before it inserts them
constexpr int kEmit = 3;      // table places a thread emits at a time

// Sums the records of each bin per (slot, node) exactly: 64-bit integer
// adds on the grid 2^-62 in an LDS hash table (linear probing) of at least
// twice as many places as the bin has records.  A bin whose keys still
// overflow the table is split by the low bits of the key's mix into slices,
// each summed on its own (the mix is a bijection, so slices end up small
// enough).  Then each sum is the next level's score: on a probe's last
// level weight * sum goes into the FP64 estimate; otherwise Rule 2 keeps the
// node when its FP32 score exceeds the next level's threshold, and a kept
// node with out-edges is listed.  Workgroup w takes bins w, w + kRedGrid, ...
__global__ void __launch_bounds__(kThreads) k_reduce(ReduceArgs a) {
  __shared__ uint32_t s_key[kTbl];
  __shared__ unsigned long long s_val[kTbl];
  __shared__ uint32_t s_part[2 * kMaxSlots];
  __shared__ uint32_t s_pre[kExpGrid + 1];
  __shared__ uint32_t s_st[kExpGrid];
  __shared__ uint32_t s_wtot[kThreads / 64];
  __shared__ int s_ovf, s_dirty;
  __shared__ uint32_t s_next;
  __shared__ int2 w_sn[kThreads / 64 * kWaveStage];  // one stage per wavefront
  __shared__ float w_h[kThreads / 64 * kWaveStage];
  __shared__ uint2 w_row[kThreads / 64 * kWaveStage];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  unsigned long long* ctr = a.ctr;
  const uint32_t sh = (uint32_t)ctr[C_SH], nbins = (uint32_t)ctr[C_NB];
  const int wv = tid >> 6;
  WaveStage ws{w_sn + wv * kWaveStage, w_h + wv * kWaveStage, w_row + wv * kWaveStage, kWaveStage, 0};
  __syncthreads();  // every thread has read the bin layout before block 0 moves on
  if (blockIdx.x == 0 && tid == 0) {
    // pending probes the next k_sched may claim (switches made this step included)
    ctr[C_TAIL_SNAP] = ctr[C_TAIL];
    ctr[C_TOT_E] = 0;
    ctr[C_TOT_N] = 0;
    ctr[C_TOT_F] = 0;
  }
  for (uint32_t t = tid; t < kTbl; t += kThreads) {
    s_key[t] = kNoKey;
    s_val[t] = 0ull;
  }
  for (int i = tid; i < 2 * a.P; i += kThreads) s_part[i] = 0u;
  if (tid == 0) s_dirty = 0;
  const uint32_t vmask = (1u << sh) - 1u;
  unsigned long long nfin = 0, nnext = 0, kept = 0, pruned = 0, near = 0;
  bool dirty = false;
  // Bins are taken from a counter (workgroup w starts on bin w): the next
  // bin is claimed while this one is summed, and its segments are loaded
  // ahead.
  uint2 nseg = make_uint2(0u, 0u);
  if (blockIdx.x < nbins && tid < kExpGrid) nseg = a.seg[(size_t)blockIdx.x * kExpGrid + tid];
  uint32_t b = blockIdx.x;
  while (b < nbins) {
    const uint2 sg = nseg;
    __syncthreads();  // the last bin's table and segments are no longer read
    if (tid == 0) s_next = (uint32_t)atomicAdd(&ctr[C_BIN], 1ull);
    if (tid < kExpGrid) s_st[tid] = sg.x;
    uint32_t R;
    const uint32_t pre = block_excl_scan(tid < kExpGrid ? sg.y : 0u, s_wtot, &R);
    if (tid < kExpGrid) s_pre[tid] = pre;
    if (tid == 0) {
      s_pre[kExpGrid] = R;
      s_ovf = 0;
    }
    __syncthreads();
    if (R == 0) {
      const uint32_t bn = s_next;
      if (bn < nbins && tid < kExpGrid) nseg = a.seg[(size_t)bn * kExpGrid + tid];
      b = bn;
      continue;
    }
    if (tid == 0) {
      atomicAdd(&ctr[C_RBINS], 1ull);
      atomicMax(&ctr[C_RMAX], (unsigned long long)R);
    }
    uint32_t tb = 9;  // table of 2^tb places, at least 2R
    while (tb < (uint32_t)kTblBits && (1u << tb) < 2u * R) ++tb;
    const uint32_t T = 1u << tb;
    // Slices, depth first: slice (M, r) holds the keys whose mix is r mod M;
    // one that overflows is replaced by its halves (2M, r) and (2M, r + M).
    // Every thread keeps the same (M, r).
    uint32_t M = 1u, r = 0u;
    for (;;) {
      for (uint32_t i0 = 0; i0 < R; i0 += kThreads * kRecBatch) {
        uint2 rc[kRecBatch];
#pragma unroll
        for (int k = 0; k < kRecBatch; ++k) {
          const uint32_t i = i0 + (uint32_t)k * kThreads + tid;
          rc[k] = make_uint2(kNoKey, 0u);
          if (i < R) {
            int lo = 0, hi = kExpGrid - 1;  // last segment g with s_pre[g] <= i
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (s_pre[mid] <= i) lo = mid; else hi = mid - 1;
            }
            rc[k] = a.rec[s_st[lo] + (i - s_pre[lo])];
          }
        }
        // the contribution fl32(Score(x) sqrt(c)) * fl32(1/|I(v)|): the record
        // carries the first factor, the target's 1/|I(v)| (its slot's graph
        // version) is read here, where a bin's targets are a narrow node range
        float inv[kRecBatch];
#pragma unroll
        for (int k = 0; k < kRecBatch; ++k) {
          inv[k] = 0.0f;
          if (rc[k].x != kNoKey && (fmix32(rc[k].x) & (M - 1u)) == r) {
            const Slot& S = a.slots[rc[k].x >> sh];
            inv[k] = S.inv_indeg[(b << sh) | (rc[k].x & vmask)];
          }
        }
#pragma unroll
        for (int k = 0; k < kRecBatch; ++k) {
          if (rc[k].x == kNoKey) continue;
          const uint32_t h = fmix32(rc[k].x);
          if ((h & (M - 1u)) != r) continue;
          const long long q = to_grid(__uint_as_float(rc[k].y) * inv[k]);
          if (q == 0) continue;  // below the grid
          uint32_t p = h >> (32 - tb);
          for (int probe = 0;; ++probe) {
            if (probe == kMaxProbe || s_ovf) {
              s_ovf = 1;
              break;
            }
            const uint32_t k0 = __hip_atomic_load(&s_key[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k0 == rc[k].x) {
              atomicAdd(&s_val[p], (unsigned long long)q);
              break;
            }
            if (k0 == kNoKey) {
              const uint32_t prev = atomicCAS(&s_key[p], kNoKey, rc[k].x);
              if (prev == kNoKey || prev == rc[k].x) {
                atomicAdd(&s_val[p], (unsigned long long)q);
                break;
              }
            }
            p = (p + 1u) & (T - 1u);
          }
        }
      }
      __syncthreads();
      if (tid == 0) atomicAdd(&ctr[C_RSLICES], 1ull);
      if (s_ovf) {  // split this slice in two and clear the table
        for (uint32_t t = tid; t < T; t += kThreads) {
          s_key[t] = kNoKey;
          s_val[t] = 0ull;
        }
        __syncthreads();
        if (tid == 0) s_ovf = 0;
        __syncthreads();
        M *= 2u;
        continue;
      }
      // Emit the sums, kEmit table places per thread at a time: the table
      // reads, then the slot fields, then the out-rows of kept nodes, each a
      // round of independent loads.
      for (uint32_t t0 = 0; t0 < T; t0 += kThreads * kEmit) {
        uint32_t key[kEmit];
        long long q[kEmit];
        int32_t s[kEmit], v[kEmit], last[kEmit];
        float thr[kEmit], h[kEmit];
        const uint2* orow[kEmit];
        uint2 row[kEmit];
        bool want[kEmit];
#pragma unroll
        for (int j = 0; j < kEmit; ++j) {
          const uint32_t t = t0 + (uint32_t)j * kThreads + tid;
          key[j] = t < T ? s_key[t] : kNoKey;
          q[j] = 0;
          s[j] = 0;
          v[j] = 0;
          if (key[j] != kNoKey) {
            q[j] = (long long)s_val[t];
            s_key[t] = kNoKey;
            s_val[t] = 0ull;
            s[j] = (int32_t)(key[j] >> sh);
            v[j] = (int32_t)((b << sh) | (key[j] & vmask));
          }
        }
#pragma unroll
        for (int j = 0; j < kEmit; ++j) {
          last[j] = 0;
          thr[j] = 0.0f;
          orow[j] = nullptr;
          if (key[j] != kNoKey) {
            const Slot& S = a.slots[s[j]];
            last[j] = S.last;
            thr[j] = S.thr_next;
            orow[j] = S.out_rows;
          }
        }
#pragma unroll
        for (int j = 0; j < kEmit; ++j) {
          want[j] = false;
          h[j] = 0.0f;
          row[j] = make_uint2(0u, 0u);
          if (key[j] != kNoKey && !last[j]) {
            h[j] = grid_f32(q[j]);
            // Rule 2 on the next level: keep v when Score(v) > eps_p / sqrt(c)^(i-j-2)
            if (h[j] > thr[j]) {
              row[j] = orow[j][v[j]];
              want[j] = row[j].y > 0;
            }
          }
        }
#pragma unroll
        for (int j = 0; j < kEmit; ++j) {
          if (key[j] != kNoKey) {
            const Slot& S = a.slots[s[j]];
            if (last[j]) {  // the returned level: weight * exact sum into the estimate
              unsafeAtomicAdd(&S.acc[v[j]], grid_f64(q[j]) * S.w);
              ++nfin;
            } else {
              ++nnext;
              if (fabsf(h[j] - thr[j]) <= 1e-5f * thr[j]) {  // FP32 rounding may decide this test
                ++near;
                unsafeAtomicAdd(S.flip, S.flip_unit);
              }
              if (h[j] > thr[j]) ++kept;
              else ++pruned;
            }
          }
          if (want[j]) {
            a.has_next[s[j]] = 1;
            atomicAdd(&s_part[s[j]], row[j].y);
            atomicAdd(&s_part[a.P + s[j]], 1u);
            dirty = true;
          }
          stage_put(want[j], s[j], v[j], h[j], row[j], ws, a.nxt, ctr);
        }
      }
      // next slice: the sibling of the nearest first-half ancestor
      while (M > 1u && r >= (M >> 1)) {
        r -= M >> 1;
        M >>= 1;
      }
      if (M == 1u) break;
      r += M >> 1;
      __syncthreads();  // this slice's table is emptied before the next fills it
    }
    const uint32_t bn = s_next;
    if (bn < nbins && tid < kExpGrid) nseg = a.seg[(size_t)bn * kExpGrid + tid];
    b = bn;
  }
  stage_flush(ws, a.nxt, ctr);
  if (dirty) s_dirty = 1;
  __syncthreads();
  if (s_dirty) {  // partial per-slot sums of what this workgroup listed (k_sched adds them up)
    uint32_t* prow = a.part + (size_t)(blockIdx.x % kPartRows) * 2 * a.P;
    for (int i = tid; i < 2 * a.P; i += kThreads)
      if (s_part[i]) atomicAdd(&prow[i], s_part[i]);
  }
  nfin = wave_sum(nfin);
  nnext = wave_sum(nnext);
  kept = wave_sum(kept);
  pruned = wave_sum(pruned);
  near = wave_sum(near);
  if (lane == 0) {
    if (nfin) atomicAdd(&ctr[C_FINAL], nfin);
    if (nnext) atomicAdd(&ctr[C_NEXT], nnext);
    if (kept) atomicAdd(&ctr[C_KEPT], kept);
    if (pruned) atomicAdd(&ctr[C_PRUNED], pruned);
    if (near) atomicAdd(&ctr[C_NEAR], near);
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

constexpr uint32_t kPullBatch = 4;  // rows each lane group gathers per round

// Grid sum of this lane's column over in-edges cols[0, cnt) of one target,
// for lane group grp of T groups.  Per 64 edges: each lane loads one in-edge
// source (and, with kMap, that row's map byte: the row is read only when it
// may hold a nonzero score), the sources kept are packed into the low lanes
// by a forward lane permute, and then each group gathers its share of the
// kept rows kPullBatch at a time, so a target's edges cost a few rounds of
// independent loads rather than a chain of dependent ones.  Every lane of the
// wavefront must call this (the lanes act as edge slots first); only the
// loads of inactive columns are skipped.  The sum is exact on the grid, so
// the order of the edges does not matter.
template <bool kMap>
__device__ __forceinline__ long long pull_edges(const DenseArgs& a, const LaneInfo& li, const float* m,
                                                const int32_t* __restrict__ cols, uint32_t cnt, float inv, int grp,
                                                uint32_t T) {
  const int lane = lane_id();
  const unsigned long long lt = (1ull << lane) - 1ull;
  long long sum = 0;
  for (uint32_t b = 0; b < cnt; b += 64) {
    const uint32_t k = b + (uint32_t)lane;
    const int32_t x = k < cnt ? cols[k] : -1;
    bool keep = x >= 0;
    if (kMap && keep) keep = a.map_cur[x] != 0;
    const unsigned long long mk = __ballot(keep);
    const uint32_t nk = (uint32_t)__popcll(mk);
    // kept sources to lanes 0..nk-1 in edge order, the others after them
    const uint32_t pos = keep ? (uint32_t)__popcll(mk & lt) : nk + (uint32_t)__popcll(~mk & lt);
    const int32_t xc = __builtin_amdgcn_ds_permute((int)(pos << 2), x);
    for (uint32_t j = 0; j < nk; j += T * kPullBatch) {
      float h[kPullBatch];
#pragma unroll
      for (uint32_t t = 0; t < kPullBatch; ++t) {
        const uint32_t q = j + t * T + (uint32_t)grp;
        const int32_t xs = __shfl(xc, (int)(q & 63u), 64);
        h[t] = 0.0f;
        if (li.active && q < nk) h[t] = m[(size_t)xs * kLanes];
      }
#pragma unroll
      for (uint32_t t = 0; t < kPullBatch; ++t) sum += pull_term(h[t], li.thr, li.sc, inv);
    }
  }
  return sum;
}

// The pulls of one pass.  A wavefront works on one target at a time; its 64
// lanes form 64/L groups of L lanes (L = the power of two covering the
// columns in use), lane g handling column g % L of every (64/L)-th kept
// in-edge, so few columns still keep the whole wavefront busy.  Group sums
// are combined by shuffles.  Short in-rows are finished per target, long
// in-rows summed in kPullChunk-edge chunks into partial sums.
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
    long long q = pull_edges<kMap>(a, li, m, dv.in_col + row.x, row.y, dv.inv_indeg[v], grp, T);
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
    long long part =
        pull_edges<kMap>(a, li, m, dv.in_col + row.x + ch.y, e - (uint32_t)ch.y, dv.inv_indeg[ch.x], grp, T);
    for (int off = L; off < 64; off <<= 1) part += __shfl_xor(part, off, 64);
    if (writer && li.active && part > 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.npart[(size_t)ch.x * kLanes + col]),
                (unsigned long long)part);
  }
}

__global__ void __launch_bounds__(kBlock, 8) k_dense(DenseArgs a) {
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

// Host-to-device uploads of small records travel as kernel arguments, so no
// host buffer has to outlive the call that queues them.
constexpr int kListArg = 256;
struct IdList {
  int32_t n, off;
  int32_t id[kListArg];
};
__global__ void k_put_list(IdList l, int32_t* __restrict__ dst) {
  for (int i = threadIdx.x; i < l.n; i += blockDim.x) dst[l.off + i] = l.id[i];
}

struct ThrRow {
  float t[PS_MAX_WALK_LEN];
};
// Writes record r; a fresh record also gets its Rule 2 thresholds and clears
// its walk bound, pending-probe count and allowance.
__global__ void k_put_record(QueryDev d, ThrRow thr, int r, bool fresh, QueryDev* __restrict__ qrec,
                             float* __restrict__ thr_all, unsigned long long* __restrict__ qbound,
                             unsigned long long* __restrict__ remaining) {
  if (threadIdx.x == 0) {
    qrec[r] = d;
    if (fresh) {
      qbound[r] = 0;
      remaining[r] = 0;
      *d.flip = 0.0;
    }
  }
  if (fresh)
    for (int i = threadIdx.x; i < PS_MAX_WALK_LEN; i += blockDim.x) thr_all[(size_t)r * PS_MAX_WALK_LEN + i] = thr.t[i];
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

ps_status put_list(const std::vector<int32_t>& ids, int32_t* dst, hipStream_t st) {
  for (size_t off = 0; off < ids.size(); off += kListArg) {
    IdList l;
    l.n = (int32_t)std::min<size_t>(kListArg, ids.size() - off);
    l.off = (int32_t)off;
    for (int i = 0; i < l.n; ++i) l.id[i] = ids[off + (size_t)i];
    k_put_list<<<1, kListArg, 0, st>>>(l, dst);
  }
  PS_HIP(hipGetLastError());
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

static uint64_t list_total(const uint64_t* h, int par) {
  uint64_t t = 0;
  for (int k = 0; k < kSubLists; ++k) t += h[C_LIST + par * kSubLists + k];
  return t;
}

void report_overflow(const Session* s, const uint64_t* h) {
  std::fprintf(stderr,
               "probesim: capacity guard tripped (sites 0x%llx: 4 frontier list, 8 records, 16 ring); "
               "P %d n %d list cap %llu (lists %llu, %llu) record cap %llu\n",
               (unsigned long long)h[C_OVERFLOW], s->P, s->n, (unsigned long long)s->list_cap,
               (unsigned long long)list_total(h, 0), (unsigned long long)list_total(h, 1), (unsigned long long)s->rec_cap);
}

void session_clear_guard(Session* s, hipStream_t st) {
  k_set_u64<<<1, 1, 0, st>>>(s->counters.as<unsigned long long>() + C_OVERFLOW, 0ull);
  k_set_u64<<<1, 1, 0, st>>>(s->counters.as<unsigned long long>() + C_RMAX, 0ull);
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
  DevBuf* bufs[] = {&s->mat[0],    &s->mat[1],       &s->rowmap[0],  &s->rowmap[1],  &s->npart,     &s->lane_slot,
                    &s->dense_ver, &s->slots,        &s->has_next,   &s->pull_flag,  &s->was_paused, &s->slot_edges,
                    &s->slot_cnt,  &s->cost, &s->counters,     &s->l_sn[0],    &s->l_sn[1],    &s->l_val[0],  &s->l_val[1],
                    &s->l_row[0],  &s->l_row[1],     &s->l_chunk[0], &s->l_chunk[1], &s->rec,       &s->seg,
                    &s->part,      &s->qrec,       &s->thr,        &s->remaining, &s->done_ring,
                    &s->qbound,    &s->acc,          &s->lq,         &s->flip,       &s->keys,      &s->t_parent,
                    &s->t_node,    &s->t_depth,      &s->t_query,    &s->t_weight,   &s->ring,      &s->ring_k,
                    &s->hyb_edges, &s->t_woff,       &s->t_walks,    &s->wcount,     &s->out_ids,
                    &s->out_scores, &s->sel.state, &s->sel.keys, &s->sel.ids, &s->m_keys[0], &s->m_keys[1],
                    &s->m_vals[0], &s->m_vals[1], &s->m_list, &s->m_ctr};
  for (DevBuf* b : bufs) devbuf_free(*b);
  if (s->h_ctr) (void)hipHostFree(s->h_ctr);
  if (s->h_qbound) (void)hipHostFree(s->h_qbound);
  if (s->begin_ev) (void)hipEventDestroy(s->begin_ev);
  if (s->step_pair) (void)hipGraphExecDestroy(s->step_pair);
  delete s;
}

// Probe slots: enough concurrent probes to fill the GPU (more slots also
// mean fewer level steps).  A slot costs a few hundred bytes; its frontier
// lives in the shared lists, so the count is bounded by the scheduler's LDS
// arrays only.  1024 by default.
int session_slots_for(int32_t n, int opt) {
  (void)n;
  const int p = opt > 0 ? std::min(opt, kSlotCap) : 1024;
  return std::max(p, 1);
}

// Dense lanes (levels computed by pulling): two node-major n x kLanes FP32
// matrices, their row maps and the partial sums of long in-rows; allocated
// the first time levels may be pulled.
static ps_status session_dense(Session* s, hipStream_t st) {
  const size_t n = (size_t)s->n;
  PS_TRY(devbuf_reserve(s->mat[0], sizeof(float) * n * kLanes));
  PS_TRY(devbuf_reserve(s->mat[1], sizeof(float) * n * kLanes));
  PS_TRY(devbuf_reserve(s->npart, sizeof(long long) * n * kLanes));
  PS_TRY(devbuf_reserve(s->rowmap[0], n));
  PS_TRY(devbuf_reserve(s->rowmap[1], n));
  for (DevBuf* b : {&s->mat[0], &s->mat[1]}) PS_HIP(hipMemsetAsync(b->p, 0, sizeof(float) * n * kLanes, st));
  PS_HIP(hipMemsetAsync(s->npart.p, 0, sizeof(long long) * n * kLanes, st));
  for (DevBuf* b : {&s->rowmap[0], &s->rowmap[1]}) PS_HIP(hipMemsetAsync(b->p, 0, n, st));
  s->dense_on = true;
  return PS_OK;
}

ps_status session_ensure(ps_ctx* ctx, int32_t n, uint64_t m_cap, int P, int qmax, uint64_t tree_pool,
                         uint64_t ring_cap) {
  Session*& s = ctx->sess;
  hipStream_t st = ctx->stream;
  ring_cap = next_pow2(std::max<uint64_t>(ring_cap, 1024));
  tree_pool = std::max<uint64_t>(tree_pool, 1024);
  // Capacities of one step, sized by the graph: 8 m records (2^24..2^30)
  // and as many list entries (up to 2^29).  A level step whose levels would
  // write more than kStepRecords records, or list more than the list holds
  // (at most one entry per record for the next levels), pauses slots
  // (k_expand); a single level may still use the whole record store.
  const uint64_t cap8 = 8ull * m_cap;
  const uint64_t rec_cap = std::min<uint64_t>(std::max<uint64_t>(cap8, 1ull << 24), 1ull << 30);
  const uint64_t list_cap = std::min<uint64_t>(std::max<uint64_t>(cap8, 1ull << 24), 1ull << 29);
  const uint64_t chunk_cap = std::max<uint64_t>(list_cap / 8, 1ull << 22);
  if (s && s->n == n && s->P == P && s->qmax >= qmax && s->tree_pool >= tree_pool && s->ring_cap >= ring_cap &&
      s->rec_cap >= rec_cap)
    return PS_OK;
  if (s && (int)s->free_recs.size() != s->qmax) return PS_ERR_STATE;  // queries admitted
  if (!s) s = new Session();
  if (s->step_pair) {  // captured with the old buffers
    (void)hipGraphExecDestroy(s->step_pair);
    s->step_pair = nullptr;
  }
  s->n = n;
  s->P = P;
  s->qmax = std::max(qmax, s->qmax);
  s->tree_pool = std::max(tree_pool, s->tree_pool);
  s->ring_cap = std::max(ring_cap, s->ring_cap);
  s->sh = 0;
  while ((((uint64_t)n - 1) >> s->sh) >= (uint64_t)kMaxBins) ++s->sh;
  s->rec_cap = std::max(rec_cap, s->rec_cap);
  s->list_cap = std::max(list_cap, s->list_cap);
  s->chunk_cap = std::max(chunk_cap, s->chunk_cap);
  s->list_soft = s->list_cap - (uint64_t)P;  // room for every slot's H_0 at the next step
  PS_TRY(devbuf_reserve(s->slots, sizeof(Slot) * (size_t)P));
  PS_TRY(devbuf_reserve(s->has_next, sizeof(int32_t) * (size_t)P));
  PS_TRY(devbuf_reserve(s->pull_flag, sizeof(int32_t) * (size_t)P));
  PS_TRY(devbuf_reserve(s->was_paused, (size_t)P));
  PS_TRY(devbuf_reserve(s->slot_edges, sizeof(uint32_t) * (size_t)P));
  PS_TRY(devbuf_reserve(s->slot_cnt, sizeof(uint32_t) * (size_t)P));
  PS_TRY(devbuf_reserve(s->cost, sizeof(uint4) * (size_t)P));
  PS_TRY(devbuf_reserve(s->hyb_edges, sizeof(unsigned long long) * (size_t)P));
  PS_TRY(devbuf_reserve(s->lane_slot, sizeof(int32_t) * kLanes));
  PS_TRY(devbuf_reserve(s->dense_ver, sizeof(DenseVer)));
  for (int p = 0; p < 2; ++p) {
    PS_TRY(devbuf_reserve(s->l_sn[p], sizeof(int2) * s->list_cap));
    PS_TRY(devbuf_reserve(s->l_val[p], sizeof(float) * s->list_cap));
    PS_TRY(devbuf_reserve(s->l_row[p], sizeof(uint2) * s->list_cap));
    PS_TRY(devbuf_reserve(s->l_chunk[p], sizeof(int2) * s->chunk_cap));
  }
  PS_TRY(devbuf_reserve(s->rec, sizeof(uint2) * s->rec_cap));
  PS_TRY(devbuf_reserve(s->seg, sizeof(uint2) * (size_t)kMaxBins * kExpGrid));
  PS_TRY(devbuf_reserve(s->part, sizeof(uint32_t) * 2 * (size_t)P * kPartRows));

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
  if (s->h_qbound_n < s->qmax) {
    if (s->h_qbound) PS_HIP(hipHostFree(s->h_qbound));
    s->h_qbound = nullptr;
    PS_HIP(hipHostMalloc((void**)&s->h_qbound, sizeof(unsigned long long) * (size_t)s->qmax, 0));
    s->h_qbound_n = s->qmax;
  }
  if (!s->begin_ev) PS_HIP(hipEventCreateWithFlags(&s->begin_ev, hipEventDisableTiming));
  s->begin_pending = false;
  if (s->dense_on) PS_TRY(session_dense(s, st));
  k_reset_lanes<<<1, kLanes, 0, st>>>(s->lane_slot.as<int32_t>());
  PS_HIP(hipMemsetAsync(s->counters.p, 0, sizeof(unsigned long long) * C_COUNT, st));
  PS_HIP(hipMemsetAsync(s->hyb_edges.p, 0, sizeof(unsigned long long) * (size_t)P, st));
  PS_HIP(hipMemsetAsync(s->pull_flag.p, 0, sizeof(int32_t) * (size_t)P, st));
  PS_HIP(hipMemsetAsync(s->part.p, 0, sizeof(uint32_t) * 2 * (size_t)P * kPartRows, st));
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
                        std::vector<int>* recs) {
  Session* s = ctx->sess;
  hipStream_t st = ctx->stream;
  if ((size_t)s->free_recs.size() < qs.size() || s->begin_pending) return PS_ERR_BUSY;
  recs->clear();
  if (qs.empty()) return PS_OK;
  int64_t total = 0;
  for (const QueryRun& q : qs) {
    ThrRow thr{};
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
    d.merged = q.merged;
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
      thr.t[x] = q.prm.eps_p > 0.0 ? (float)(q.prm.eps_p / std::pow(sc, (double)x)) : 0.0f;
    k_put_record<<<1, PS_MAX_WALK_LEN, 0, st>>>(d, thr, r, true, s->qrec.as<QueryDev>(), s->thr.as<float>(),
                                                s->qbound.as<unsigned long long>(),
                                                s->remaining.as<unsigned long long>());
    PS_HIP(hipMemsetAsync(d.acc, 0, sizeof(double) * (size_t)s->n, st));
  }
  PS_TRY(put_list(*recs, s->lq.as<int32_t>(), st));
  if (total > 0) {
    k_walk_bound<<<grid_for((uint64_t)total, kBlock), kBlock, 0, st>>>(
        s->qrec.as<QueryDev>(), s->lq.as<int32_t>(), (int)recs->size(), total, s->qbound.as<unsigned long long>(),
        s->counters.as<unsigned long long>());
    PS_HIP(hipGetLastError());
  }
  // the bounds come back through pinned memory; session_bounds reads them
  PS_HIP(hipMemcpyAsync(s->h_qbound, s->qbound.p, sizeof(unsigned long long) * (size_t)s->qmax, hipMemcpyDeviceToHost,
                        st));
  PS_HIP(hipEventRecord(s->begin_ev, st));
  s->begin_pending = true;
  return PS_OK;
}

ps_status session_bounds(ps_ctx* ctx, const std::vector<int>& recs, std::vector<uint64_t>* bounds, bool wait,
                         bool* ready) {
  Session* s = ctx->sess;
  *ready = false;
  bounds->assign(recs.size(), 0);
  if (recs.empty()) {
    *ready = true;
    return PS_OK;
  }
  if (!s->begin_pending) return PS_ERR_STATE;
  if (wait) {
    PS_HIP(hipEventSynchronize(s->begin_ev));
  } else {
    const hipError_t e = hipEventQuery(s->begin_ev);
    if (e == hipErrorNotReady) return PS_OK;
    PS_HIP(e);
  }
  for (size_t i = 0; i < recs.size(); ++i) (*bounds)[i] = s->h_qbound[(size_t)recs[i]];
  s->begin_pending = false;
  *ready = true;
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
    k_put_record<<<1, 1, 0, st>>>(d, ThrRow{}, r, false, s->qrec.as<QueryDev>(), nullptr, nullptr, nullptr);
    PS_HIP(hipMemsetAsync(s->keys.as<unsigned long long>() + d.tree_base, 0xFF,
                          sizeof(unsigned long long) * (d.tree_mask + 1), st));
    PS_HIP(hipMemsetAsync(s->t_weight.as<int32_t>() + d.tree_base, 0, sizeof(int32_t) * (d.tree_mask + 1), st));
  }
  if (launch.empty()) return PS_OK;
  PS_TRY(put_list(launch, s->lq.as<int32_t>(), st));
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
  k_snap_tail<<<1, 1, 0, st>>>(s->counters.as<unsigned long long>());
  PS_HIP(hipGetLastError());
  return PS_OK;
}

namespace {

FList flist(Session* s, int par) {
  FList L;
  L.sn = s->l_sn[par].as<int2>();
  L.val = s->l_val[par].as<float>();
  L.row = s->l_row[par].as<uint2>();
  L.chunk = s->l_chunk[par].as<int2>();
  L.n_ent = s->counters.as<unsigned long long>() + C_LIST + par * kSubLists;
  L.n_chunk = s->counters.as<unsigned long long>() + C_CHUNK + par * kSubLists;
  L.sub_cap = s->list_cap / kSubLists;
  L.sub_chunk_cap = s->chunk_cap / kSubLists;
  return L;
}

// One level step with the frontier lists of parity `cur`: k_sched, k_pick and
// the dense pass only when levels may be pulled, k_expand, k_reduce.
void launch_step(Session* s, int cur, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2) {
  const int nxt = cur ^ 1;
  unsigned long long* ctr = s->counters.as<unsigned long long>();
  SchedArgs sa{};
  sa.P = s->P;
  sa.n = s->n;
  sa.qmax = s->qmax;
  sa.slots = s->slots.as<Slot>();
  sa.has_next = s->has_next.as<int32_t>();
  sa.pull_flag = s->pull_flag.as<int32_t>();
  sa.was_paused = s->was_paused.as<uint8_t>();
  sa.ring = s->ring.as<int32_t>();
  sa.ring_k = s->ring_k.as<int32_t>();
  sa.ring_mask = s->ring_cap - 1;
  sa.t_parent = s->t_parent.as<int32_t>();
  sa.t_node = s->t_node.as<int32_t>();
  sa.t_depth = s->t_depth.as<int32_t>();
  sa.t_query = s->t_query.as<int32_t>();
  sa.t_weight = s->t_weight.as<int32_t>();
  sa.t_woff = s->t_woff.as<uint32_t>();
  sa.t_walks = s->t_walks.as<int32_t>();
  sa.qr = s->qrec.as<QueryDev>();
  sa.thr_tab = s->thr.as<float>();
  sa.remaining = s->remaining.as<unsigned long long>();
  sa.done_ring = s->done_ring.as<int32_t>();
  sa.hyb_edges = s->hyb_edges.as<unsigned long long>();
  sa.lane_slot = s->lane_slot.as<int32_t>();
  sa.part = s->part.as<uint32_t>();
  sa.slot_edges = s->slot_edges.as<uint32_t>();
  sa.slot_cnt = s->slot_cnt.as<uint32_t>();
  sa.cost = s->cost.as<uint4>();
  sa.list = flist(s, cur);
  sa.next = flist(s, nxt);
  sa.ctr = ctr;
  sa.cur = cur;
  k_sched<<<(s->P + kSchedBlock - 1) / kSchedBlock, kSchedBlock, 0, st>>>(sa);
  if (s->pull) {
    PickArgs pa{};
    pa.P = s->P;
    pa.n = s->n;
    pa.slots = s->slots.as<Slot>();
    pa.pull_flag = s->pull_flag.as<int32_t>();
    pa.lane_slot = s->lane_slot.as<int32_t>();
    pa.dv = s->dense_ver.as<DenseVer>();
    pa.slot_edges = s->slot_edges.as<uint32_t>();
    pa.slot_cnt = s->slot_cnt.as<uint32_t>();
    pa.cost = s->cost.as<uint4>();
    pa.ctr = ctr;
    k_pick<<<1, kPickThreads, 0, st>>>(pa);
  }
  ExpandArgs ea{};
  ea.n = s->n;
  ea.P = s->P;
  ea.sh_min = s->sh;
  ea.cost = s->cost.as<uint4>();
  ea.slots = s->slots.as<Slot>();
  ea.pull_flag = s->pull_flag.as<int32_t>();
  ea.cur = flist(s, cur);
  ea.nxt = flist(s, nxt);
  ea.rec = s->rec.as<uint2>();
  ea.rec_cap = s->rec_cap;
  ea.seg = s->seg.as<uint2>();
  ea.mat_cur = s->dense_on ? s->mat[cur].as<float>() : nullptr;
  ea.map_cur = s->dense_on ? s->rowmap[cur].as<uint8_t>() : nullptr;
  ea.has_next = s->has_next.as<int32_t>();
  ea.part = s->part.as<uint32_t>();
  ea.list_soft = s->list_soft;
  ea.ctr = ctr;
  ea.cur_par = cur;
  if (ev0) (void)hipEventRecord(ev0, st);
  k_expand<<<kExpGrid, kThreads, 0, st>>>(ea);
  ReduceArgs ra{};
  ra.n = s->n;
  ra.P = s->P;
  ra.slots = s->slots.as<Slot>();
  ra.rec = s->rec.as<uint2>();
  ra.seg = s->seg.as<uint2>();
  ra.nxt = flist(s, nxt);
  ra.has_next = s->has_next.as<int32_t>();
  ra.part = s->part.as<uint32_t>();
  ra.ctr = ctr;
  k_reduce<<<kRedGrid, kThreads, 0, st>>>(ra);
  if (ev1) (void)hipEventRecord(ev1, st);
  if (s->pull) {
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
  }
  if (ev2) (void)hipEventRecord(ev2, st);
}

}  // namespace

// Launches `count` level steps.  Without timing they run as replays of a
// captured pair of steps (even then odd list parity), one graph launch per
// pair; with timing every expansion is bracketed by events.
ps_status session_steps(ps_ctx* ctx, uint64_t count, double* expand_ms, double* pull_ms) {
  Session* s = ctx->sess;
  hipStream_t st = ctx->stream;
  const bool timing = ctx->timing && expand_ms;
  if (timing) {
    while (ctx->ev_pool.size() < 3 * count) {
      hipEvent_t ev;
      PS_HIP(hipEventCreate(&ev));
      ctx->ev_pool.push_back(ev);
    }
    for (uint64_t t = 0; t < count; ++t) {
      TraceRange tr("probesim level step");
      launch_step(s, (int)(s->steps & 1), st, ctx->ev_pool[3 * t], ctx->ev_pool[3 * t + 1],
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
      launch_step(s, 1, st, nullptr, nullptr, nullptr);
      s->steps++;
      count--;
    }
    if (!s->step_pair) {
      hipGraph_t graph = nullptr;
      PS_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      launch_step(s, 0, st, nullptr, nullptr, nullptr);
      launch_step(s, 1, st, nullptr, nullptr, nullptr);
      PS_HIP(hipStreamEndCapture(st, &graph));
      const hipError_t e = hipGraphInstantiate(&s->step_pair, graph, nullptr, nullptr, 0);
      s->pair_dense = s->pull;
      (void)hipGraphDestroy(graph);
      PS_HIP(e);
    }
    for (; count >= 2; count -= 2) {
      TraceRange tr("probesim level steps (2, graph)");
      PS_HIP(hipGraphLaunch(s->step_pair, st));
      s->steps += 2;
    }
  }
  for (; count > 0; --count) {
    TraceRange tr("probesim level step");
    launch_step(s, (int)(s->steps & 1), st, nullptr, nullptr, nullptr);
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
  if (out.cap >= 0 || q.k > 0) {
    PS_TRY(devbuf_reserve(s->out_ids, sizeof(int32_t) * (size_t)n));
    PS_TRY(devbuf_reserve(s->out_scores, sizeof(double) * (size_t)n));
  }
  if (out.cap >= 0) {
    int64_t total = 0;
    PS_TRY(select_nonzero(s->sel, acc, n, out.cap, s->out_ids.as<int32_t>(), s->out_scores.as<double>(), &total, st));
    const int64_t w = std::min(total, out.cap);
    if (w > 0) {
      PS_TRY(copy_out(out.nodes, s->out_ids.p, sizeof(int32_t) * (size_t)w, st));
      PS_TRY(copy_out(out.scores, s->out_scores.p, sizeof(double) * (size_t)w, st));
    }
    *out.count = total;
  } else if (q.k <= 0) {
    PS_TRY(copy_out(out.scores, acc, sizeof(double) * (size_t)n, st));
  } else {
    PS_TRY(select_topk(s->sel, acc, n, q.u, q.k, s->out_ids.as<int32_t>(), s->out_scores.as<double>(), st));
    PS_TRY(copy_out(out.scores, s->out_scores.p, sizeof(double) * (size_t)q.k, st));
    PS_TRY(copy_out(out.nodes, s->out_ids.p, sizeof(int32_t) * (size_t)q.k, st));
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
// Pull threshold in out-edges of a slot's listed entries.  Pushing costs
// records per out-edge, pulling reads every in-edge of the graph once for up
// to kLanes levels, so pulling pays off for levels with a sizable share of m
// out-edges: m/20 by default (the fastest of m/80..m/10 and never on the
// 1M-node workload), opt > 0 sets it, opt < 0 never pulls.
uint64_t pull_threshold(int64_t m, int64_t opt) {
  if (opt < 0) return ~0ull;
  if (opt > 0) return (uint64_t)opt;
  return std::max<uint64_t>((uint64_t)m / 20, 4096);
}

ps_status session_set_pull(ps_ctx* ctx, uint64_t threshold) {
  Session* s = ctx->sess;
  const bool dense = threshold != ~0ull;
  if (dense && !s->dense_on) PS_TRY(session_dense(s, ctx->stream));
  if (s->step_pair && s->pair_dense != dense) {  // captured with the other kernel sequence
    PS_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipGraphExecDestroy(s->step_pair);
    s->step_pair = nullptr;
  }
  s->pull = dense;
  k_set_u64<<<1, 1, 0, ctx->stream>>>(s->counters.as<unsigned long long>() + C_PULL_T,
                                      (unsigned long long)threshold);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

// Grows the tree pool and the ring to hold the trees of records recs
// (bounds from session_bounds).  Only valid while no other query is
// admitted: the buffers are replaced, and the captured level steps, which
// point at the old ones, are dropped.
ps_status session_fit_trees(ps_ctx* ctx, const std::vector<int>& recs, const std::vector<uint64_t>& bounds) {
  Session* s = ctx->sess;
  hipStream_t st = ctx->stream;
  uint64_t pool_need = 0, ring_need = 0;
  for (size_t i = 0; i < bounds.size(); ++i) {
    const uint64_t b = bounds[i];
    if (b) pool_need += next_pow2(std::max<uint64_t>(2 * b, 64));
    ring_need += ring_share(s, recs[i], b);
  }
  if (pool_need > s->tree_pool || ring_need > s->ring_cap) {
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
  return PS_OK;
}

static ps_status engine_run_core(ps_ctx* ctx, ps_graph* g, GraphVersion* gv, const std::vector<QueryRun>& qs,
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
  {
    TraceRange tr("probesim walks and trees");
    PS_TRY(session_begin(ctx, g, gv, qs, &recs));
    bool ready = false;
    PS_TRY(session_bounds(ctx, recs, &bounds, true, &ready));
    PS_TRY(session_fit_trees(ctx, recs, bounds));
    PS_TRY(session_build(ctx, recs, bounds));
  }
  PS_HIP(hipMemcpyAsync(s->h_ctr, s->counters.p, sizeof(uint64_t) * C_COUNT, hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  uint64_t levels = s->h_ctr[C_LEVELS] - before[C_LEVELS];
  const uint64_t probes = s->h_ctr[C_TAIL] - before[C_TAIL];
  int maxL = 2;
  for (auto& q : qs) maxL = std::max(maxL, q.prm.L);
  uint64_t with_probes = 0;
  for (size_t i = 0; i < qs.size(); ++i) with_probes += bounds[i] ? 1 : 0;
  // List scheduling: every slot is busy while probes are pending, and a
  // probe holds its slot for depth-1 steps, so this many steps finish them
  // all unless the per-step budget pauses slots or Section 4.4 switches
  // queue more probes; then further batches of steps, sized the same way,
  // run until every query is complete.
  uint64_t steps = probes ? (levels + P - 1) / P + (uint64_t)maxL + 2 : 0;
  double expand_ms = 0.0, pull_ms = 0.0;
  PS_TRY(session_set_pull(ctx, pull_threshold(g->m, pull_opt)));
  const bool progress = std::getenv("PS_PROGRESS") != nullptr;
  uint64_t total_steps = 0;
  // runs `cnt` level steps (in batches of 256 when progress is printed)
  auto run_steps = [&](uint64_t cnt) -> ps_status {
    TraceRange tr("probesim level steps");
    while (cnt) {
      const uint64_t b = progress ? std::min<uint64_t>(cnt, 256) : cnt;
      PS_TRY(session_steps(ctx, b, &expand_ms, &pull_ms));
      total_steps += b;
      cnt -= b;
      if (progress && cnt) {
        PS_HIP(hipMemcpyAsync(s->h_ctr, s->counters.p, sizeof(uint64_t) * C_COUNT, hipMemcpyDeviceToHost, st));
        PS_HIP(hipStreamSynchronize(st));
        std::fprintf(stderr, "probesim: %llu steps, %llu probes handed out, %llu paused\n",
                     (unsigned long long)total_steps, (unsigned long long)(s->h_ctr[C_HEAD] - before[C_HEAD]),
                     (unsigned long long)(s->h_ctr[C_PAUSED] - before[C_PAUSED]));
      }
    }
    return PS_OK;
  };
  PS_TRY(run_steps(steps));
  uint64_t stuck = 0, last_work = ~0ull;
  for (;;) {
    PS_HIP(hipMemcpyAsync(s->h_ctr, s->counters.p, sizeof(uint64_t) * C_COUNT, hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    const uint64_t* h = s->h_ctr;
    if (h[C_OVERFLOW] || h[C_DONE] - before[C_DONE] >= with_probes) break;
    // a guard: no probe handed out, expanded, pulled or finished over whole batches
    const uint64_t work = h[C_HEAD] + h[C_DONE] + h[C_EDGES] + h[C_PULLS] + h[C_FINAL] + h[C_LEVEL0];
    stuck = work == last_work ? stuck + 1 : 0;
    if (stuck > 2) break;
    last_work = work;
    if (progress)
      std::fprintf(stderr, "probesim: %llu steps, %llu of %llu queries done, %llu of %llu probes handed out, %llu paused\n",
                   (unsigned long long)total_steps, (unsigned long long)(h[C_DONE] - before[C_DONE]),
                   (unsigned long long)with_probes, (unsigned long long)(h[C_HEAD] - before[C_HEAD]),
                   (unsigned long long)(h[C_TAIL] - before[C_TAIL]), (unsigned long long)(h[C_PAUSED] - before[C_PAUSED]));
    const uint64_t lv = s->h_ctr[C_LEVELS] - before[C_LEVELS];
    steps = (lv > levels ? (lv - levels + P - 1) / P : 0) + (uint64_t)maxL + 2;
    levels = std::max(levels, lv);
    PS_TRY(run_steps(steps));
  }
  {
    const uint64_t* h = s->h_ctr;
    const bool over = h[C_OVERFLOW] != 0;
    if (over || h[C_DONE] - before[C_DONE] != with_probes) {
      if (over) report_overflow(s, h);
      else
        std::fprintf(stderr, "probesim: level steps ended with %llu of %llu queries complete\n",
                     (unsigned long long)(h[C_DONE] - before[C_DONE]), (unsigned long long)with_probes);
      // the session's device state is not usable any more: drop it
      for (int r : recs)
        if (s->rec_version[(size_t)r]) graph_release(g, s->rec_version[(size_t)r]);
      (void)hipStreamSynchronize(st);
      session_free(s);
      ctx->sess = nullptr;
      return over ? PS_ERR_OOM : PS_ERR_STATE;
    }
  }
  std::vector<double> flips((size_t)nq, 0.0);
  {
    TraceRange tr("probesim finish");
    for (int i = 0; i < nq; ++i) {
      QueryOut o = outs[(size_t)i];
      if (!o.flip) o.flip = &flips[(size_t)i];
      PS_TRY(session_finish(ctx, g, recs[(size_t)i], qs[(size_t)i], o));
    }
  }
  PS_HIP(hipMemcpyAsync(s->h_ctr, s->counters.p, sizeof(uint64_t) * C_COUNT, hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nq; ++i) {
    const double f = outs[(size_t)i].flip && !ps_is_device_ptr(outs[(size_t)i].flip) ? *outs[(size_t)i].flip
                                                                                       : flips[(size_t)i];
    stats.flip_allowance = std::max(stats.flip_allowance, f);
  }
  const uint64_t* h = s->h_ctr;
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
  stats.reduce_bins = (int64_t)(h[C_RBINS] - before[C_RBINS]);
  stats.reduce_slices = (int64_t)(h[C_RSLICES] - before[C_RSLICES]);
  stats.reduce_max_records = (int64_t)h[C_RMAX];
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

// Copies device bytes to a host or device destination (stream-ordered).
ps_status copy_out(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!bytes) return PS_OK;
  const hipMemcpyKind kind = ps_is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  PS_HIP(hipMemcpyAsync(dst, src, bytes, kind, st));
  return PS_OK;
}

// Queries by merged probing run one at a time on their own path; the others
// go through the level-step engine together.
ps_status engine_run(ps_ctx* ctx, ps_graph* g, GraphVersion* gv, const std::vector<QueryRun>& qs,
                     const std::vector<QueryOut>& outs, int slots_opt, int64_t pull_opt) {
  TraceRange tr("probesim queries");
  std::vector<QueryRun> rest;
  std::vector<QueryOut> rest_out;
  std::vector<size_t> merged;
  for (size_t i = 0; i < qs.size(); ++i) {
    if (qs[i].merged) {
      merged.push_back(i);
    } else {
      rest.push_back(qs[i]);
      rest_out.push_back(outs[i]);
    }
  }
  if (merged.empty()) return engine_run_core(ctx, g, gv, qs, outs, slots_opt, pull_opt);
  const auto t0 = std::chrono::steady_clock::now();
  ps_stats ms{};
  const int P = session_slots_for(g->n, slots_opt);
  const uint64_t m_cap = std::max<uint64_t>(gv->out_store->cap, 1);
  Session* s = ctx->sess;
  PS_TRY(session_ensure(ctx, g->n, m_cap, P, std::max<int>((int)qs.size(), s ? s->qmax : 0), s ? s->tree_pool : 0,
                        s ? s->ring_cap : 0));
  for (size_t i : merged) {
    ps_status e = engine_merged(ctx, g, gv, qs[i], outs[i], &ms);
    if (e != PS_OK) return e;
  }
  ms.queries = (int64_t)merged.size();
  if (!rest.empty()) {
    PS_TRY(engine_run_core(ctx, g, gv, rest, rest_out, slots_opt, pull_opt));
    ps_stats& L = ctx->last;
    L.queries += ms.queries;
    L.walks += ms.walks;
    L.tree_nodes += ms.tree_nodes;
    L.probe_levels += ms.probe_levels;
    L.steps += ms.steps;
    L.entries_expanded += ms.entries_expanded;
    L.edges_scanned += ms.edges_scanned;
    L.next_entries += ms.next_entries;
    L.final_adds += ms.final_adds;
    L.expand_launches += ms.expand_launches;
    L.expand_ms += ms.expand_ms;
    L.pushed_edges += ms.pushed_edges;
    L.pushed_final_adds += ms.pushed_final_adds;
  } else {
    ctx->last = ms;
  }
  ctx->last.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return PS_OK;
}
