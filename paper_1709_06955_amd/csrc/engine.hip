// ProbeSim query engine: sqrt(c)-walks, reverse reachability tree, PROBE
// level expansion with both pruning rules, FP64 accumulation, top-k.
//
// Work of one launch (one or many queries, Alg. 3 of the paper):
//   1. k_walk_bound   sample every walk once to size the tree (sum of len-1)
//   2. k_walk_tree    sample the walks again (Philox is counter-based, so the
//                     walks are identical) and insert every prefix
//                     (u_1..u_i), i >= 2, into one hash-addressed tree; the
//                     hash slot of a prefix is its tree node id and its
//                     weight counts the walks sharing it
//   3. level steps    every tree node is one PROBE (Alg. 2).  Probes run in
//                     P device slots; a slot that finishes takes the next
//                     probe, so short and long probes of all queries keep the
//                     slots busy.  One step = k_sched (advance / refill slots)
//                     -> k_prep (read and clear the level's scores, Rule 2,
//                     bin rows by out-degree) -> k_expand (push along
//                     out-edges).  Each slot has a dense FP32 score vector per
//                     level parity; the first atomic add that turns an entry
//                     nonzero appends (slot, node) to the next frontier list,
//                     so frontiers stay sparse lists while sums stay exact.
//                     The last level of a probe adds weight * score straight
//                     into the query's FP64 estimate.
//   4. k_finalize     divide by n_r, set s(u,u) = 1; top-k by sorting.

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "ps_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kSmallDeg = 32;  // rows up to this length: one lane per row
constexpr uint32_t kChunk = 512;    // longer rows: one wavefront per 512 edges
constexpr unsigned long long kEmpty = ~0ull;
constexpr int kOverflowIdx = C_COUNT;  // counters[C_COUNT] = overflow flag

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
__device__ __forceinline__ int32_t walk_move(int32_t v, uint32_t k, uint32_t t, const QueryDev& q,
                                             const uint2* __restrict__ in_rows, const int32_t* __restrict__ in_col) {
  const uint4 w = philox4x32_10(make_uint4(k, t, (uint32_t)q.u, 0u),
                                make_uint2((uint32_t)q.seed, (uint32_t)(q.seed >> 32)));
  const uint2 row = in_rows[v];
  if (row.y == 0u || w.x < q.t_stop) return -1;
  const uint64_t r = ((uint64_t)w.z << 32) | w.y;
  const uint32_t idx = (uint32_t)__umul64hi(r, (uint64_t)row.y);
  return in_col[row.x + idx];
}

__device__ __forceinline__ int find_query(const QueryDev* __restrict__ qs, int nq, int64_t g) {
  int lo = 0, hi = nq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (qs[mid].walk_base <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------ wave utilities ----

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Reserves one output position per lane with `flag` set; one atomic per wave.
// Call with every active lane (inactive lanes do not take part).
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

__global__ void k_walk_bound(const QueryDev* __restrict__ qs, int nq, int64_t total,
                             const uint2* __restrict__ in_rows, const int32_t* __restrict__ in_col,
                             unsigned long long* __restrict__ ctr) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long extra = 0, nodes = 0;
  if (g < total) {
    const QueryDev q = qs[find_query(qs, nq, g)];
    const uint32_t k = (uint32_t)(q.walk_begin + (g - q.walk_base));
    int32_t v = q.u;
    int len = 1;
    for (uint32_t t = 0; len < q.L; ++t) {
      const int32_t nx = walk_move(v, k, t, q, in_rows, in_col);
      if (nx < 0) break;
      v = nx;
      ++len;
    }
    extra = (unsigned long long)(len - 1);
    nodes = (unsigned long long)len;
  }
  extra = wave_sum(extra);
  nodes = wave_sum(nodes);
  if (lane_id() == 0) {
    if (extra) atomicAdd(&ctr[C_TREE_BOUND], extra);
    atomicAdd(&ctr[C_WALK_NODES], nodes);
  }
}

__global__ void k_walk_export(QueryDev q, int64_t k_begin, int64_t count, const uint2* __restrict__ in_rows,
                              const int32_t* __restrict__ in_col, int32_t* __restrict__ nodes,
                              int32_t* __restrict__ lens) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const uint32_t k = (uint32_t)(k_begin + g);
  int32_t* row = nodes + g * q.L;
  int32_t v = q.u;
  int len = 1;
  row[0] = v;
  for (uint32_t t = 0; len < q.L; ++t) {
    const int32_t nx = walk_move(v, k, t, q, in_rows, in_col);
    if (nx < 0) break;
    v = nx;
    row[len++] = v;
  }
  lens[g] = len;
  for (int i = len; i < q.L; ++i) row[i] = -1;
}

// Inserts key = (parent tree node << 32 | graph node) with linear probing.
// The slot index is the tree node id.  The table always has free slots
// (capacity >= 2 * number of keys), so the probe sequence ends.
__device__ __forceinline__ uint32_t tree_insert(unsigned long long* __restrict__ keys, uint64_t mask,
                                                unsigned long long key, bool& inserted) {
  uint64_t s = mix64(key) & mask;
  inserted = false;
  while (true) {
    const unsigned long long cur = keys[s];
    if (cur == key) return (uint32_t)s;
    if (cur == kEmpty) {
      const unsigned long long prev = atomicCAS(&keys[s], kEmpty, key);
      if (prev == kEmpty) {
        inserted = true;
        return (uint32_t)s;
      }
      if (prev == key) return (uint32_t)s;
    }
    s = (s + 1) & mask;
  }
}

// Alg. 3, tree construction: walk k of query q descends from the root of q
// (tree id cap + q) through one tree node per prefix, creating it on first
// visit and adding one to its weight.
__global__ void k_walk_tree(const QueryDev* __restrict__ qs, int nq, int64_t total,
                            const uint2* __restrict__ in_rows, const int32_t* __restrict__ in_col,
                            unsigned long long* __restrict__ keys, uint64_t cap,
                            int32_t* __restrict__ t_parent, int32_t* __restrict__ t_node,
                            int32_t* __restrict__ t_depth, int32_t* __restrict__ t_query,
                            int32_t* __restrict__ t_weight, int32_t* __restrict__ probe_list,
                            unsigned long long* __restrict__ ctr) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int qi = find_query(qs, nq, g);
  const QueryDev q = qs[qi];
  const uint32_t k = (uint32_t)(q.walk_begin + (g - q.walk_base));
  uint32_t parent = (uint32_t)(cap + qi);
  int32_t v = q.u;
  int len = 1;
  for (uint32_t t = 0; len < q.L; ++t) {
    const int32_t nx = walk_move(v, k, t, q, in_rows, in_col);
    if (nx < 0) break;
    v = nx;
    ++len;
    const unsigned long long key = ((unsigned long long)parent << 32) | (uint32_t)v;
    bool inserted;
    const uint32_t id = tree_insert(keys, cap - 1, key, inserted);
    if (inserted) {
      t_parent[id] = (int32_t)parent;
      t_node[id] = v;
      t_depth[id] = len;
      t_query[id] = qi;
      const unsigned long long pos = atomicAdd(&ctr[C_PROBES], 1ull);
      probe_list[pos] = (int32_t)id;
      atomicAdd(&ctr[C_LEVELS], (unsigned long long)(len - 1));
    }
    atomicAdd(&t_weight[id], 1);
    parent = id;
  }
}

__global__ void k_init_roots(const QueryDev* __restrict__ qs, int nq, uint64_t cap, int32_t* t_parent,
                             int32_t* t_node, int32_t* t_depth, int32_t* t_query) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  t_parent[cap + q] = -1;
  t_node[cap + q] = qs[q].u;
  t_depth[cap + q] = 1;
  t_query[cap + q] = q;
}

template <typename T>
__global__ void k_fill(T* p, T v, uint64_t cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_reset_slots(Slot* slots, int32_t* has_next, int P) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= P) return;
  Slot st{};
  st.probe = -1;
  slots[s] = st;
  has_next[s] = 0;
}

// ------------------------------------------------------- level steps ----

// Advances every slot by one PROBE iteration, or hands it the next probe.
// A probe ends after its last level (i-2) or when Rule 2 emptied its
// frontier.  A new probe on (u_1..u_i) starts with H_0 = {u_i: 1}.
__global__ void k_sched(int P, int32_t n, Slot* __restrict__ slots, int32_t* __restrict__ has_next,
                        const int32_t* __restrict__ probe_list, const int32_t* __restrict__ t_parent,
                        const int32_t* __restrict__ t_node, const int32_t* __restrict__ t_depth,
                        const int32_t* __restrict__ t_query, const int32_t* __restrict__ t_weight,
                        const QueryDev* __restrict__ qs, const float* __restrict__ thr_tab,
                        float* __restrict__ dense_cur, int2* __restrict__ list_cur, uint64_t list_cap,
                        unsigned long long* __restrict__ ctr, int cur) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) {
    ctr[C_SMALL] = 0;
    ctr[C_CHUNK] = 0;
    ctr[C_LIST0 + (cur ^ 1)] = 0;
  }
  if (s >= P) return;
  Slot st = slots[s];
  bool fetch = false;
  if (st.probe >= 0) {
    if (st.last || !has_next[s]) {
      st.probe = -1;
      fetch = true;
    } else {
      st.level++;
      st.cursor = t_parent[st.cursor];
    }
  } else {
    fetch = true;
  }
  has_next[s] = 0;
  if (fetch) {
    const unsigned long long p = atomicAdd(&ctr[C_CURSOR], 1ull);
    if (p < ctr[C_PROBES]) {
      const int32_t t = probe_list[p];
      st.probe = t;
      st.level = 0;
      st.depth = t_depth[t];
      st.cursor = t_parent[t];
      st.query = t_query[t];
      st.w = (double)t_weight[t];
      const int32_t x = t_node[t];
      const unsigned long long pos = atomicAdd(&ctr[C_LIST0 + cur], 1ull);
      if (pos < list_cap) {
        dense_cur[(size_t)s * n + x] = 1.0f;
        list_cur[pos] = make_int2(s, x);
      } else {
        ctr[kOverflowIdx] = 1;
      }
      atomicAdd(&ctr[C_LEVEL0], 1ull);
    } else {
      st.probe = -1;
    }
  }
  if (st.probe >= 0) {
    const int e = st.depth - st.level - 1;  // iterations left, i-j-1 >= 1
    st.thr = thr_tab[st.query * PS_MAX_WALK_LEN + e];
    st.sc = qs[st.query].sc;
    st.excl = t_node[st.cursor];
    st.last = st.level == st.depth - 2;
  }
  slots[s] = st;
}

// Reads and clears the scores of the listed entries, applies Rule 2 (remove x
// when Score(x) * sqrt(c)^(i-j-1) <= eps_p, i.e. Score(x) <= thr) and bins
// the surviving rows: short rows go to the lane-per-row list, long rows are
// cut into 512-edge chunks for the wavefront-per-chunk list.
__global__ void __launch_bounds__(kBlock) k_prep(int32_t n, const Slot* __restrict__ slots,
                                                 const int2* __restrict__ list_cur, float* __restrict__ dense_cur,
                                                 float* __restrict__ item_val, const uint2* __restrict__ out_rows,
                                                 int32_t* __restrict__ small_list, int2* __restrict__ chunk_list,
                                                 uint64_t list_cap, uint64_t chunk_cap,
                                                 unsigned long long* __restrict__ ctr, int cur) {
  // after an overflow the counter runs past the list; never read beyond it
  const unsigned long long cnt = min(ctr[C_LIST0 + cur], (unsigned long long)list_cap);
  const int lane = lane_id();
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long kept = 0, pruned = 0, edges = 0;
  for (uint64_t i0 = gtid - lane; i0 < cnt; i0 += stride) {
    const uint64_t i = i0 + lane;
    bool small = false;
    uint32_t nch = 0;
    if (i < cnt) {
      const int2 it = list_cur[i];
      float* d = dense_cur + (size_t)it.x * n + it.y;
      const float val = *d;
      *d = 0.0f;
      const Slot& sl = slots[it.x];
      if (val > sl.thr) {
        ++kept;
        const uint2 row = out_rows[it.y];
        if (row.y) {
          item_val[i] = val * sl.sc;
          edges += row.y;
          if (row.y <= kSmallDeg) small = true;
          else nch = (row.y + kChunk - 1) / kChunk;
        }
      } else {
        ++pruned;
      }
    }
    const unsigned long long sp = wave_reserve(small, &ctr[C_SMALL], nullptr);
    if (small) small_list[sp] = (int32_t)i;
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
        ctr[kOverflowIdx] = 1;
      }
    }
  }
  kept = wave_sum(kept);
  pruned = wave_sum(pruned);
  edges = wave_sum(edges);
  if (lane == 0) {
    if (kept) atomicAdd(&ctr[C_KEPT], kept);
    if (pruned) atomicAdd(&ctr[C_PRUNED], pruned);
    if (edges) atomicAdd(&ctr[C_EDGES], edges);
  }
}

struct ExpandArgs {
  int32_t n;
  const int2* list_cur;
  const float* item_val;
  const int32_t* small_list;
  const int2* chunk_list;
  const Slot* slots;
  const uint2* out_rows;
  const int32_t* out_col;
  const float* inv_indeg;
  float* dense_next;
  double* acc;
  int2* list_next;
  uint64_t list_cap;
  uint64_t chunk_cap;
  int32_t* has_next;
  unsigned long long* ctr;
  int nxt;
};

// One out-edge x -> v of a listed entry: add sqrt(c)/|I(v)| * Score(x) to
// H_{j+1}[v] unless v is the excluded walk node u_{i-j-1} (Alg. 2).
__device__ __forceinline__ void visit_edge(const ExpandArgs& a, bool active, int32_t s, int32_t v, float sv,
                                           const Slot& sl, unsigned long long& nfinal, unsigned long long& nnext) {
  bool append = false;
  if (active && v != sl.excl) {
    const float c = sv * a.inv_indeg[v];
    if (c >= 1.17549435e-38f) {  // contributions below FLT_MIN are dropped
      if (sl.last) {
        unsafeAtomicAdd(&a.acc[(size_t)sl.query * a.n + v], (double)c * sl.w);
        ++nfinal;
      } else {
        const float old = unsafeAtomicAdd(&a.dense_next[(size_t)s * a.n + v], c);
        append = old == 0.0f;
      }
    }
  }
  if (__ballot(append)) {
    const unsigned long long pos = wave_reserve(append, &a.ctr[C_LIST0 + a.nxt], &nnext);
    if (append) {
      if (pos < a.list_cap) {
        a.list_next[pos] = make_int2(s, v);
        a.has_next[s] = 1;
      } else {
        a.ctr[kOverflowIdx] = 1;
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_expand(ExpandArgs a) {
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long nfinal = 0, nnext = 0;
  // Short rows: one lane per listed entry.
  const unsigned long long nsmall = min(a.ctr[C_SMALL], (unsigned long long)a.list_cap);
  for (uint64_t j0 = wave * 64; j0 < nsmall; j0 += nwaves * 64) {
    const uint64_t j = j0 + lane;
    uint32_t deg = 0, start = 0;
    int32_t s = 0;
    float sv = 0.0f;
    Slot sl{};
    if (j < nsmall) {
      const int32_t i = a.small_list[j];
      const int2 it = a.list_cur[i];
      s = it.x;
      sl = a.slots[s];
      sv = a.item_val[i];
      const uint2 row = a.out_rows[it.y];
      start = row.x;
      deg = row.y;
    }
    for (uint32_t t = 0; t < deg; ++t) visit_edge(a, true, s, a.out_col[start + t], sv, sl, nfinal, nnext);
  }
  // Long rows: one wavefront per chunk of 512 consecutive out-edges.
  const unsigned long long nchunk = min(a.ctr[C_CHUNK], (unsigned long long)a.chunk_cap);
  for (uint64_t c = wave; c < nchunk; c += nwaves) {
    const int2 ch = a.chunk_list[c];
    const int2 it = a.list_cur[ch.x];
    const int32_t s = it.x;
    const Slot sl = a.slots[s];
    const float sv = a.item_val[ch.x];
    const uint2 row = a.out_rows[it.y];
    const uint32_t b = (uint32_t)ch.y * kChunk;
    const uint32_t e = min(row.y, b + kChunk);
    for (uint32_t t0 = b; t0 < e; t0 += 64) {
      const uint32_t t = t0 + lane;
      const bool act = t < e;
      const int32_t v = act ? a.out_col[row.x + t] : -1;
      visit_edge(a, act, s, v, sv, sl, nfinal, nnext);
    }
  }
  nfinal = wave_sum(nfinal);
  nnext = wave_sum(nnext);
  if (lane == 0) {
    if (nfinal) atomicAdd(&a.ctr[C_FINAL], nfinal);
    if (nnext) atomicAdd(&a.ctr[C_NEXT], nnext);
  }
}

// s^(u, v) = acc / n_r (+ shift for v != u), s^(u, u) = 1.
__global__ void k_finalize(int32_t n, const QueryDev* __restrict__ qs, int nq, double* __restrict__ acc) {
  const uint64_t total = (uint64_t)n * nq;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const int q = (int)(i / (uint64_t)n);
    const int32_t v = (int32_t)(i - (uint64_t)q * n);
    const QueryDev Q = qs[q];
    acc[i] = v == Q.u ? 1.0 : acc[i] * Q.inv_nr + Q.shift;
  }
}

// Sort keys for top-k: the estimate, with u itself pushed below every node.
__global__ void k_topk_keys(int32_t n, int32_t u, const double* __restrict__ s, double* __restrict__ keys,
                            int32_t* __restrict__ ids) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    keys[v] = v == u ? -1.0 : s[v];
    ids[v] = (int32_t)v;
  }
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

constexpr int kStepGrid = 2048;  // 8 workgroups per CU for the level-step kernels

ps_status copy_out(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!bytes) return PS_OK;
  const hipMemcpyKind kind = ps_is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  PS_HIP(hipMemcpyAsync(dst, src, bytes, kind, st));
  return PS_OK;
}

}  // namespace

ps_status devbuf_reserve(DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes && b.p) return PS_OK;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  const size_t want = std::max<size_t>(bytes, 256);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
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

ps_status engine_walks(ps_ctx* ctx, GraphVersion* gv, int32_t n, const QueryRun& q, int64_t k_begin, int64_t count,
                       int32_t* nodes, int32_t* lens) {
  (void)n;
  hipStream_t st = ctx->stream;
  QueryDev d{};
  d.u = q.u;
  d.L = q.prm.L;
  d.t_stop = q.prm.t_stop;
  d.seed = q.seed;
  Engine& e = ctx->eng;
  const size_t nb = sizeof(int32_t) * (size_t)count * (size_t)d.L;
  PS_TRY(devbuf_reserve(e.stage, nb + sizeof(int32_t) * (size_t)count + 256));
  int32_t* dn = e.stage.as<int32_t>();
  int32_t* dl = dn + (size_t)count * d.L;
  if (count > 0) {
    k_walk_export<<<grid_for((uint64_t)count, kBlock), kBlock, 0, st>>>(d, k_begin, count, gv->in_rows,
                                                                       gv->in_store->col, dn, dl);
    PS_HIP(hipGetLastError());
    PS_TRY(copy_out(nodes, dn, nb, st));
    PS_TRY(copy_out(lens, dl, sizeof(int32_t) * (size_t)count, st));
  }
  PS_HIP(hipStreamSynchronize(st));
  return PS_OK;
}

namespace {

// Chooses the number of probe slots: enough concurrent probes to fill the
// GPU, bounded so that the dense per-slot score vectors (2 x 4 B x n each)
// stay within a fixed share of HBM and slot * n fits in 31 bits.
int choose_slots(int32_t n, uint64_t levels, int opt) {
  if (opt > 0) return opt;
  const uint64_t budget = 16ull << 30;  // bytes for the dense score vectors
  uint64_t p = budget / (8ull * (uint64_t)n);
  p = std::min<uint64_t>(p, ((1ull << 31) - 1) / (uint64_t)n);
  p = std::min<uint64_t>(p, 1024);
  const uint64_t want = std::max<uint64_t>(64, levels / 8);
  p = std::min(p, want);
  return (int)std::max<uint64_t>(p, 1);
}

}  // namespace

ps_status engine_run(ps_ctx* ctx, GraphVersion* gv, int32_t n, const std::vector<QueryRun>& qs,
                     const std::vector<QueryOut>& outs, int slots_opt) {
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t st = ctx->stream;
  Engine& e = ctx->eng;
  const int nq = (int)qs.size();
  ps_stats stats{};
  stats.queries = nq;
  if (nq == 0) {
    ctx->last = stats;
    return PS_OK;
  }
  // Query descriptors and Rule 2 thresholds thr[q][e] = eps_p / sqrt(c)^e.
  std::vector<QueryDev> qd((size_t)nq);
  std::vector<float> thr((size_t)nq * PS_MAX_WALK_LEN, 0.0f);
  int64_t total_walks = 0;
  int maxL = 2;
  for (int i = 0; i < nq; ++i) {
    const QueryRun& q = qs[(size_t)i];
    QueryDev& d = qd[(size_t)i];
    d.u = q.u;
    d.L = q.prm.L;
    d.t_stop = q.prm.t_stop;
    d.topk = q.k;
    d.seed = q.seed;
    d.walk_begin = q.walk_begin;
    d.walk_count = q.walk_end - q.walk_begin;
    d.walk_base = total_walks;
    const double sc = std::sqrt(q.prm.c);
    d.sc = (float)sc;
    d.inv_nr = 1.0 / (double)q.prm.n_r;
    d.shift = q.bias_shift ? q.prm.eps_t / 2.0 : 0.0;
    total_walks += d.walk_count;
    maxL = std::max(maxL, q.prm.L);
    for (int x = 1; x < PS_MAX_WALK_LEN; ++x)
      thr[(size_t)i * PS_MAX_WALK_LEN + x] = q.prm.eps_p > 0.0 ? (float)(q.prm.eps_p / std::pow(sc, (double)x)) : 0.0f;
  }
  stats.walks = total_walks;
  PS_TRY(devbuf_reserve(e.qdesc, sizeof(QueryDev) * (size_t)nq));
  PS_TRY(devbuf_reserve(e.thr, sizeof(float) * thr.size()));
  PS_TRY(devbuf_reserve(e.counters, sizeof(unsigned long long) * (C_COUNT + 1)));
  PS_TRY(devbuf_reserve(e.acc, sizeof(double) * (size_t)nq * (size_t)n));
  if (!e.h_counters) PS_HIP(hipHostMalloc((void**)&e.h_counters, sizeof(uint64_t) * (C_COUNT + 1), 0));
  PS_HIP(hipMemcpyAsync(e.qdesc.p, qd.data(), sizeof(QueryDev) * (size_t)nq, hipMemcpyHostToDevice, st));
  PS_HIP(hipMemcpyAsync(e.thr.p, thr.data(), sizeof(float) * thr.size(), hipMemcpyHostToDevice, st));
  unsigned long long* ctr = e.counters.as<unsigned long long>();
  const QueryDev* dq = e.qdesc.as<QueryDev>();

  // 1. Size the tree.
  PS_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned long long) * (C_COUNT + 1), st));
  if (total_walks > 0) {
    k_walk_bound<<<grid_for((uint64_t)total_walks, kBlock), kBlock, 0, st>>>(dq, nq, total_walks, gv->in_rows,
                                                                            gv->in_store->col, ctr);
    PS_HIP(hipGetLastError());
  }
  PS_HIP(hipMemcpyAsync(e.h_counters, ctr, sizeof(uint64_t) * (C_COUNT + 1), hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  const uint64_t bound = e.h_counters[C_TREE_BOUND];
  stats.walk_nodes = (int64_t)e.h_counters[C_WALK_NODES];

  // 2. Build the reverse reachability tree.
  const uint64_t cap = next_pow2(std::max<uint64_t>(2 * bound, 1024));
  if (cap + (uint64_t)nq >= (1ull << 31)) return PS_ERR_OOM;
  PS_TRY(devbuf_reserve(e.keys, sizeof(unsigned long long) * cap));
  PS_TRY(devbuf_reserve(e.t_parent, sizeof(int32_t) * (cap + nq)));
  PS_TRY(devbuf_reserve(e.t_node, sizeof(int32_t) * (cap + nq)));
  PS_TRY(devbuf_reserve(e.t_depth, sizeof(int32_t) * (cap + nq)));
  PS_TRY(devbuf_reserve(e.t_query, sizeof(int32_t) * (cap + nq)));
  PS_TRY(devbuf_reserve(e.t_weight, sizeof(int32_t) * (cap + nq)));
  PS_TRY(devbuf_reserve(e.probe_list, sizeof(int32_t) * std::max<uint64_t>(bound, 1)));
  PS_HIP(hipMemsetAsync(e.keys.p, 0xFF, sizeof(unsigned long long) * cap, st));
  PS_HIP(hipMemsetAsync(e.t_weight.p, 0, sizeof(int32_t) * (cap + nq), st));
  k_init_roots<<<grid_for((uint64_t)nq, kBlock), kBlock, 0, st>>>(dq, nq, cap, e.t_parent.as<int32_t>(),
                                                                  e.t_node.as<int32_t>(), e.t_depth.as<int32_t>(),
                                                                  e.t_query.as<int32_t>());
  PS_HIP(hipGetLastError());
  if (total_walks > 0) {
    k_walk_tree<<<grid_for((uint64_t)total_walks, kBlock), kBlock, 0, st>>>(
        dq, nq, total_walks, gv->in_rows, gv->in_store->col, e.keys.as<unsigned long long>(), cap,
        e.t_parent.as<int32_t>(), e.t_node.as<int32_t>(), e.t_depth.as<int32_t>(), e.t_query.as<int32_t>(),
        e.t_weight.as<int32_t>(), e.probe_list.as<int32_t>(), ctr);
    PS_HIP(hipGetLastError());
  }
  PS_HIP(hipMemcpyAsync(e.h_counters, ctr, sizeof(uint64_t) * (C_COUNT + 1), hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  const uint64_t n_probes = e.h_counters[C_PROBES];
  const uint64_t levels = e.h_counters[C_LEVELS];
  stats.tree_nodes = (int64_t)n_probes;
  stats.probe_levels = (int64_t)levels;

  // 3. Level steps.
  const int P = choose_slots(n, levels, slots_opt);
  uint64_t list_cap = std::min<uint64_t>((uint64_t)P * (uint64_t)n, std::max<uint64_t>(1ull << 24, 8 * levels + (1ull << 22)));
  list_cap = std::max<uint64_t>(list_cap, e.list_cap);
  list_cap = std::min<uint64_t>(list_cap, (uint64_t)P * (uint64_t)n);
  ps_status rs = PS_OK;
  for (int attempt = 0; attempt < 8; ++attempt) {
    const uint64_t chunk_cap = list_cap / 2 + (1ull << 20);
    const bool fresh_dense = e.P != P || e.n != n || !e.dense[0].p;
    PS_TRY(devbuf_reserve(e.dense[0], sizeof(float) * (size_t)P * n));
    PS_TRY(devbuf_reserve(e.dense[1], sizeof(float) * (size_t)P * n));
    PS_TRY(devbuf_reserve(e.list[0], sizeof(int2) * list_cap));
    PS_TRY(devbuf_reserve(e.list[1], sizeof(int2) * list_cap));
    PS_TRY(devbuf_reserve(e.item_val, sizeof(float) * list_cap));
    PS_TRY(devbuf_reserve(e.small_list, sizeof(int32_t) * list_cap));
    PS_TRY(devbuf_reserve(e.chunk_list, sizeof(int2) * chunk_cap));
    PS_TRY(devbuf_reserve(e.slots, sizeof(Slot) * (size_t)P));
    PS_TRY(devbuf_reserve(e.has_next, sizeof(int32_t) * (size_t)P));
    if (fresh_dense || attempt > 0) {
      PS_HIP(hipMemsetAsync(e.dense[0].p, 0, sizeof(float) * (size_t)P * n, st));
      PS_HIP(hipMemsetAsync(e.dense[1].p, 0, sizeof(float) * (size_t)P * n, st));
    }
    e.P = P;
    e.n = n;
    e.list_cap = list_cap;
    e.chunk_cap = chunk_cap;
    PS_HIP(hipMemsetAsync(e.acc.p, 0, sizeof(double) * (size_t)nq * n, st));
    // keep C_TREE_BOUND .. C_LEVELS; clear the rest
    PS_HIP(hipMemsetAsync(ctr + C_CURSOR, 0, sizeof(unsigned long long) * (C_COUNT + 1 - C_CURSOR), st));
    k_reset_slots<<<grid_for((uint64_t)P, kBlock), kBlock, 0, st>>>(e.slots.as<Slot>(), e.has_next.as<int32_t>(), P);
    PS_HIP(hipGetLastError());

    const uint64_t steps = (levels + P - 1) / P + (uint64_t)maxL + 2;
    stats.steps = (int64_t)steps;
    ExpandArgs a{};
    a.n = n;
    a.item_val = e.item_val.as<float>();
    a.small_list = e.small_list.as<int32_t>();
    a.chunk_list = e.chunk_list.as<int2>();
    a.slots = e.slots.as<Slot>();
    a.out_rows = gv->out_rows;
    a.out_col = gv->out_store->col;
    a.inv_indeg = gv->inv_indeg;
    a.acc = e.acc.as<double>();
    a.list_cap = list_cap;
    a.chunk_cap = chunk_cap;
    a.has_next = e.has_next.as<int32_t>();
    a.ctr = ctr;
    std::vector<hipEvent_t> evs;
    if (ctx->timing) {
      while (ctx->ev_pool.size() < 2 * steps) {
        hipEvent_t ev;
        PS_HIP(hipEventCreate(&ev));
        ctx->ev_pool.push_back(ev);
      }
    }
    for (uint64_t t = 0; t < steps; ++t) {
      const int cur = (int)(t & 1), nxt = cur ^ 1;
      k_sched<<<grid_for((uint64_t)P, kBlock), kBlock, 0, st>>>(
          P, n, e.slots.as<Slot>(), e.has_next.as<int32_t>(), e.probe_list.as<int32_t>(), e.t_parent.as<int32_t>(),
          e.t_node.as<int32_t>(), e.t_depth.as<int32_t>(), e.t_query.as<int32_t>(), e.t_weight.as<int32_t>(), dq,
          e.thr.as<float>(), e.dense[cur].as<float>(), e.list[cur].as<int2>(), list_cap, ctr, cur);
      k_prep<<<kStepGrid, kBlock, 0, st>>>(n, e.slots.as<Slot>(), e.list[cur].as<int2>(), e.dense[cur].as<float>(),
                                           e.item_val.as<float>(), gv->out_rows, e.small_list.as<int32_t>(),
                                           e.chunk_list.as<int2>(), list_cap, chunk_cap, ctr, cur);
      a.list_cur = e.list[cur].as<int2>();
      a.dense_next = e.dense[nxt].as<float>();
      a.list_next = e.list[nxt].as<int2>();
      a.nxt = nxt;
      if (ctx->timing) PS_HIP(hipEventRecord(ctx->ev_pool[2 * t], st));
      k_expand<<<kStepGrid, kBlock, 0, st>>>(a);
      if (ctx->timing) PS_HIP(hipEventRecord(ctx->ev_pool[2 * t + 1], st));
    }
    PS_HIP(hipGetLastError());
    PS_HIP(hipMemcpyAsync(e.h_counters, ctr, sizeof(uint64_t) * (C_COUNT + 1), hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    stats.expand_launches = (int64_t)steps;
    if (ctx->timing) {
      double ms = 0.0;
      for (uint64_t t = 0; t < steps; ++t) {
        float x = 0.0f;
        PS_HIP(hipEventElapsedTime(&x, ctx->ev_pool[2 * t], ctx->ev_pool[2 * t + 1]));
        ms += x;
      }
      stats.expand_ms = ms;
    }
    if (!e.h_counters[kOverflowIdx] && e.h_counters[C_CURSOR] >= n_probes) {
      rs = PS_OK;
      break;
    }
    // A frontier list overflowed (or, impossible by the step bound, probes
    // were left): grow the lists and run the steps again from clean state.
    rs = PS_ERR_OOM;
    if (list_cap >= (uint64_t)P * (uint64_t)n && e.h_counters[kOverflowIdx]) break;
    list_cap = std::min<uint64_t>(list_cap * 4, (uint64_t)P * (uint64_t)n);
  }
  if (rs != PS_OK) return rs;
  stats.entries_expanded = (int64_t)e.h_counters[C_KEPT];
  stats.entries_pruned = (int64_t)e.h_counters[C_PRUNED];
  stats.edges_scanned = (int64_t)e.h_counters[C_EDGES];
  stats.next_entries = (int64_t)e.h_counters[C_NEXT];
  stats.final_adds = (int64_t)e.h_counters[C_FINAL];

  // 4. Finalise and write the results.
  double* acc = e.acc.as<double>();
  k_finalize<<<kStepGrid, kBlock, 0, st>>>(n, dq, nq, acc);
  PS_HIP(hipGetLastError());
  for (int i = 0; i < nq; ++i) {
    const QueryRun& q = qs[(size_t)i];
    const double* row = acc + (size_t)i * n;
    if (q.k <= 0) {
      PS_TRY(copy_out(outs[(size_t)i].scores, row, sizeof(double) * (size_t)n, st));
      continue;
    }
    PS_TRY(devbuf_reserve(e.sort_keys[0], sizeof(double) * (size_t)n));
    PS_TRY(devbuf_reserve(e.sort_keys[1], sizeof(double) * (size_t)n));
    PS_TRY(devbuf_reserve(e.sort_vals[0], sizeof(int32_t) * (size_t)n));
    PS_TRY(devbuf_reserve(e.sort_vals[1], sizeof(int32_t) * (size_t)n));
    k_topk_keys<<<kStepGrid, kBlock, 0, st>>>(n, q.u, row, e.sort_keys[0].as<double>(), e.sort_vals[0].as<int32_t>());
    PS_HIP(hipGetLastError());
    size_t tmp = 0;
    PS_HIP(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tmp, e.sort_keys[0].as<double>(),
                                                         e.sort_keys[1].as<double>(), e.sort_vals[0].as<int32_t>(),
                                                         e.sort_vals[1].as<int32_t>(), n, 0, 64, st));
    PS_TRY(devbuf_reserve(e.sort_tmp, tmp));
    PS_HIP(hipcub::DeviceRadixSort::SortPairsDescending(e.sort_tmp.p, tmp, e.sort_keys[0].as<double>(),
                                                         e.sort_keys[1].as<double>(), e.sort_vals[0].as<int32_t>(),
                                                         e.sort_vals[1].as<int32_t>(), n, 0, 64, st));
    PS_TRY(copy_out(outs[(size_t)i].scores, e.sort_keys[1].p, sizeof(double) * (size_t)q.k, st));
    PS_TRY(copy_out(outs[(size_t)i].nodes, e.sort_vals[1].p, sizeof(int32_t) * (size_t)q.k, st));
  }
  PS_HIP(hipStreamSynchronize(st));
  stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  ctx->last = stats;
  return PS_OK;
}
