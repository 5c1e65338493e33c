// Merged probing over the reverse reachability tree, Rule 2 off (FP64).
//
// PROBE is linear in its start set H_0 (Lemma 2 / the Score equation of
// Section 3.3), and the probe of the tree node (u_1..u_i) applies the level
// maps T_{i-1}, ..., T_1 to e_{u_i}, where T_p moves a score set from walk
// position p+1 to position p and drops u_p:
//   T_p(H)[v] = sum over x in H with v in O(x), v != u_p, of sqrt(c)/|I(v)| H[x].
// T_p depends on the walk only through u_p, the node of the tree ancestor at
// depth p, so the weighted probes of a subtree can be added before the maps
// they share:  X(t) = w(t) e_{node(t)} + sum over the children c of t of
// T_{depth(t)}(X(c)), and the estimate is X(root) / n_r.  The tree is
// processed one depth at a time, deepest first: the sets X(t) of all tree
// nodes of depth d live in one open-addressed table keyed by (t, x); one
// launch expands every entry along its tree edge into the table of depth d-1
// (or, from depth 2, straight into the FP64 estimate).  A tree node's set is
// expanded once, instead of once per probe below it.
//
// Rule 2 prunes each probe by its own scores and has no merged form, so the
// mode runs with eps_p = 0; every sum is FP64, each contribution is
// (sqrt(c) / |I(v)|) * X[x] as in the plain FP64 definition, and results
// differ from it only by the order of the additions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>

#include "ps_internal.h"

namespace {

constexpr int kMBlock = 256;
constexpr int kMaxDepth = PS_MAX_WALK_LEN + 1;
constexpr unsigned long long kNone = ~0ull;
constexpr uint32_t kWaveRow = 16;  // rows longer than this are swept by the whole wavefront
constexpr uint64_t kMaxTable = 1ull << 30;  // places of one level's table (16 GB of keys and sums)
constexpr int kMaxProbeM = 4096;             // linear-probe steps before an add is refused

enum MCounter { M_OVERFLOW = 0, M_ENTRIES, M_EDGES, M_FINAL, M_COUNT };

__device__ __forceinline__ unsigned long long mmix(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Adds x to the entry of key, inserting it (linear probing).  A table holds
// at least twice the entries it can receive unless capped at kMaxTable; a
// probe sequence longer than kMaxProbeM (a table near full) drops the add
// and sets the overflow counter, and the call fails with PS_ERR_OOM.
__device__ __forceinline__ void table_add(unsigned long long* __restrict__ keys, double* __restrict__ vals,
                                          uint64_t mask, unsigned long long key, double x,
                                          unsigned long long* __restrict__ ctr) {
  uint64_t h = mmix(key) & mask;
  for (int probe = 0; probe < kMaxProbeM; ++probe) {
    const unsigned long long cur = keys[h];
    if (cur == key) {
      unsafeAtomicAdd(&vals[h], x);
      return;
    }
    if (cur == kNone) {
      const unsigned long long prev = atomicCAS(&keys[h], kNone, key);
      if (prev == kNone || prev == key) {
        unsafeAtomicAdd(&vals[h], x);
        return;
      }
    }
    h = (h + 1) & mask;
    if ((probe & 255) == 255 && __hip_atomic_load(&ctr[M_OVERFLOW], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;  // the call already failed
  }
  atomicAdd(&ctr[M_OVERFLOW], 1ull);
}

__global__ void k_m_clear(unsigned long long* __restrict__ keys, double* __restrict__ vals, uint64_t cap) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
    keys[i] = kNone;
    vals[i] = 0.0;
  }
}

// Tree nodes of one query's region per depth (counts, then lists).
__global__ void k_m_count(const unsigned long long* __restrict__ tkeys, const int32_t* __restrict__ t_depth,
                          uint64_t base, uint64_t cap, unsigned long long* __restrict__ cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x)
    if (tkeys[base + i] != kNone) atomicAdd(&cnt[t_depth[base + i]], 1ull);
}

__global__ void k_m_fill(const unsigned long long* __restrict__ tkeys, const int32_t* __restrict__ t_depth,
                         uint64_t base, uint64_t cap, const unsigned long long* __restrict__ off,
                         unsigned long long* __restrict__ cursor, int32_t* __restrict__ list) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
    if (tkeys[base + i] == kNone) continue;
    const int d = t_depth[base + i];
    list[off[d] + atomicAdd(&cursor[d], 1ull)] = (int32_t)(base + i);
  }
}

// Each tree node's own probe start: w(t) at its graph node.
__global__ void k_m_starts(const int32_t* __restrict__ list, uint64_t count, const int32_t* __restrict__ t_node,
                           const int32_t* __restrict__ t_weight, unsigned long long* __restrict__ keys,
                           double* __restrict__ vals, uint64_t mask, unsigned long long* __restrict__ ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x) {
    const int32_t t = list[i];
    table_add(keys, vals, mask, ((unsigned long long)(uint32_t)t << 32) | (uint32_t)t_node[t], (double)t_weight[t],
              ctr);
  }
}

// Entries of a table and the out-edges they will push (sizes the next table).
__global__ void k_m_size(const unsigned long long* __restrict__ keys, uint64_t cap, const uint2* __restrict__ out_rows,
                         unsigned long long* __restrict__ ctr) {
  unsigned long long ent = 0, edges = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[i];
    if (k == kNone) continue;
    ++ent;
    edges += out_rows[(uint32_t)k].y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    ent += __shfl_down(ent, off, 64);
    edges += __shfl_down(edges, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (ent) atomicAdd(&ctr[M_ENTRIES], ent);
    if (edges) atomicAdd(&ctr[M_EDGES], edges);
  }
}

struct ExpandArgs {
  const unsigned long long* keys;
  const double* vals;
  uint64_t cap;
  unsigned long long* nkeys;  // next table, or null: add into acc
  double* nvals;
  uint64_t nmask;
  double* acc;
  const int32_t* t_parent;
  const int32_t* t_node;
  const uint2* out_rows;
  const int32_t* out_col;
  const uint2* in_rows;
  double sc;
  unsigned long long* ctr;
};

__device__ __forceinline__ void push_edge(const ExpandArgs& a, int32_t parent, int32_t excl, int32_t v, double x,
                                          unsigned long long& nfinal) {
  if (v == excl) return;
  const double y = a.sc / (double)a.in_rows[v].y * x;
  if (a.nkeys) {
    table_add(a.nkeys, a.nvals, a.nmask, ((unsigned long long)(uint32_t)parent << 32) | (uint32_t)v, y, a.ctr);
  } else {
    unsafeAtomicAdd(&a.acc[v], y);
    ++nfinal;
  }
}

// One wavefront per 64 table slots: short rows are pushed by their own lane,
// long rows by the whole wavefront in turn (lanes stride the row).
__global__ void __launch_bounds__(kMBlock) k_m_expand(ExpandArgs a) {
  const int lane = threadIdx.x & 63;
  const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long nfinal = 0;
  for (uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w * 64 < a.cap; w += waves) {
    // once a table has refused an add the call fails: stop pushing
    const unsigned long long ovf = __hip_atomic_load(&a.ctr[M_OVERFLOW], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__builtin_amdgcn_readfirstlane((uint32_t)(ovf != 0))) break;  // wavefront-uniform
    const uint64_t slot = w * 64 + (uint64_t)lane;
    const unsigned long long k = slot < a.cap ? a.keys[slot] : kNone;
    const bool occ = k != kNone;
    int32_t parent = 0, excl = -1;
    uint2 row = make_uint2(0, 0);
    double x = 0.0;
    if (occ) {
      const int32_t t = (int32_t)(k >> 32);
      parent = a.t_parent[t];
      excl = a.t_node[parent];
      row = a.out_rows[(uint32_t)k];
      x = a.vals[slot];
    }
    if (occ && row.y <= kWaveRow)
      for (uint32_t e = 0; e < row.y; ++e) push_edge(a, parent, excl, a.out_col[row.x + e], x, nfinal);
    unsigned long long big = __ballot(occ && row.y > kWaveRow);
    while (big) {
      const int src = __ffsll(big) - 1;
      big &= big - 1;
      const int32_t p = __shfl(parent, src, 64), ex = __shfl(excl, src, 64);
      const uint32_t rs = __shfl(row.x, src, 64), rl = __shfl(row.y, src, 64);
      const double xs = __shfl(x, src, 64);
      for (uint32_t e = (uint32_t)lane; e < rl; e += 64) push_edge(a, p, ex, a.out_col[rs + e], xs, nfinal);
    }
  }
  for (int off = 32; off > 0; off >>= 1) nfinal += __shfl_down(nfinal, off, 64);
  if (lane == 0 && nfinal) atomicAdd(&a.ctr[M_FINAL], nfinal);
}

int m_grid(uint64_t work) {
  const uint64_t g = (work + kMBlock - 1) / kMBlock;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(g, 8192));
}

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace

ps_status engine_merged(ps_ctx* ctx, ps_graph* g, GraphVersion* gv, const QueryRun& q, const QueryOut& out,
                        ps_stats* st) {
  TraceRange tr("probesim merged probing");
  Session* s = ctx->sess;
  hipStream_t stm = ctx->stream;
  std::vector<int> recs;
  std::vector<uint64_t> bounds;
  PS_TRY(session_begin(ctx, g, gv, {q}, &recs));
  bool ready = false;
  PS_TRY(session_bounds(ctx, recs, &bounds, true, &ready));
  PS_TRY(session_fit_trees(ctx, recs, bounds));
  PS_TRY(session_build(ctx, recs, bounds));
  const int r = recs[0];
  const QueryDev d = s->h_rec[(size_t)r];
  st->walks += d.walk_count;
  if (bounds[0] > 0) {
    const uint64_t base = d.tree_base, cap = d.tree_mask + 1;
    PS_TRY(devbuf_reserve(s->m_ctr, sizeof(unsigned long long) * (M_COUNT + 3 * kMaxDepth)));
    auto* ctr = s->m_ctr.as<unsigned long long>();
    auto* cnt = ctr + M_COUNT;
    auto* off = cnt + kMaxDepth;
    auto* cursor = off + kMaxDepth;
    PS_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned long long) * (M_COUNT + 3 * kMaxDepth), stm));
    auto* tkeys = s->keys.as<unsigned long long>();
    auto* t_depth = s->t_depth.as<int32_t>();
    k_m_count<<<m_grid(cap), kMBlock, 0, stm>>>(tkeys, t_depth, base, cap, cnt);
    PS_HIP(hipGetLastError());
    unsigned long long hc[kMaxDepth];
    PS_HIP(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, stm));
    PS_HIP(hipStreamSynchronize(stm));
    unsigned long long ho[kMaxDepth];
    unsigned long long total = 0;
    int dmax = 1;
    for (int dd = 0; dd < kMaxDepth; ++dd) {
      ho[dd] = total;
      total += hc[dd];
      if (hc[dd]) dmax = std::max(dmax, dd);
    }
    st->tree_nodes += (int64_t)total;
    PS_TRY(devbuf_reserve(s->m_list, sizeof(int32_t) * std::max<uint64_t>(total, 1)));
    PS_HIP(hipMemcpyAsync(off, ho, sizeof(ho), hipMemcpyHostToDevice, stm));
    k_m_fill<<<m_grid(cap), kMBlock, 0, stm>>>(tkeys, t_depth, base, cap, off, cursor, s->m_list.as<int32_t>());
    PS_HIP(hipGetLastError());
    const int32_t* list = s->m_list.as<int32_t>();
    const int32_t* t_node = s->t_node.as<int32_t>();
    const int32_t* t_weight = s->t_weight.as<int32_t>();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
      PS_HIP(hipEventCreate(&e0));
      PS_HIP(hipEventCreate(&e1));
    }
    double expand_ms = 0.0;
    // the table of the deepest level: its nodes' own starts
    int cur = 0;
    uint64_t ccap = pow2_at_least(std::max<uint64_t>(2 * hc[dmax], 1024));
    PS_TRY(devbuf_reserve(s->m_keys[cur], sizeof(unsigned long long) * ccap));
    PS_TRY(devbuf_reserve(s->m_vals[cur], sizeof(double) * ccap));
    k_m_clear<<<m_grid(ccap), kMBlock, 0, stm>>>(s->m_keys[cur].as<unsigned long long>(), s->m_vals[cur].as<double>(),
                                                  ccap);
    k_m_starts<<<m_grid(hc[dmax]), kMBlock, 0, stm>>>(list + ho[dmax], hc[dmax], t_node, t_weight,
                                                       s->m_keys[cur].as<unsigned long long>(),
                                                       s->m_vals[cur].as<double>(), ccap - 1, ctr);
    PS_HIP(hipGetLastError());
    for (int dd = dmax; dd >= 2; --dd) {
      // size the next table from this one's entries and out-edges
      PS_HIP(hipMemsetAsync(ctr + M_ENTRIES, 0, 2 * sizeof(unsigned long long), stm));
      k_m_size<<<m_grid(ccap), kMBlock, 0, stm>>>(s->m_keys[cur].as<unsigned long long>(), ccap, gv->out_rows, ctr);
      PS_HIP(hipGetLastError());
      unsigned long long sz[2];
      PS_HIP(hipMemcpyAsync(sz, ctr + M_ENTRIES, sizeof(sz), hipMemcpyDeviceToHost, stm));
      PS_HIP(hipStreamSynchronize(stm));
      st->entries_expanded += (int64_t)sz[0];
      st->edges_scanned += (int64_t)sz[1];
      if (dd < dmax) st->next_entries += (int64_t)sz[0];
      ExpandArgs a{};
      a.keys = s->m_keys[cur].as<unsigned long long>();
      a.vals = s->m_vals[cur].as<double>();
      a.cap = ccap;
      a.acc = d.acc;
      a.t_parent = s->t_parent.as<int32_t>();
      a.t_node = t_node;
      a.out_rows = gv->out_rows;
      a.out_col = gv->out_store->col;
      a.in_rows = gv->in_rows;
      a.sc = std::sqrt(q.prm.c);
      a.ctr = ctr;
      const int nxt = cur ^ 1;
      uint64_t ncap = 0;
      if (dd > 2) {
        // distinct (parent, v) pairs: at most the pushed edges plus the
        // starts of depth dd-1, and at most (tree nodes of depth dd-1) * n
        const uint64_t bound = std::min<uint64_t>(sz[1] + hc[dd - 1], (uint64_t)hc[dd - 1] * (uint64_t)g->n);
        // (at most kMaxTable places: a level with more distinct pairs than
        // that holds fails the call with PS_ERR_OOM through the overflow flag)
        ncap = std::min<uint64_t>(pow2_at_least(std::max<uint64_t>(2 * bound, 1024)), kMaxTable);
        PS_TRY(devbuf_reserve(s->m_keys[nxt], sizeof(unsigned long long) * ncap));
        PS_TRY(devbuf_reserve(s->m_vals[nxt], sizeof(double) * ncap));
        k_m_clear<<<m_grid(ncap), kMBlock, 0, stm>>>(s->m_keys[nxt].as<unsigned long long>(),
                                                      s->m_vals[nxt].as<double>(), ncap);
        k_m_starts<<<m_grid(hc[dd - 1]), kMBlock, 0, stm>>>(list + ho[dd - 1], hc[dd - 1], t_node, t_weight,
                                                             s->m_keys[nxt].as<unsigned long long>(),
                                                             s->m_vals[nxt].as<double>(), ncap - 1, ctr);
        a.nkeys = s->m_keys[nxt].as<unsigned long long>();
        a.nvals = s->m_vals[nxt].as<double>();
        a.nmask = ncap - 1;
      }
      if (e0) PS_HIP(hipEventRecord(e0, stm));
      k_m_expand<<<m_grid(ccap), kMBlock, 0, stm>>>(a);
      PS_HIP(hipGetLastError());
      if (e1) {
        PS_HIP(hipEventRecord(e1, stm));
        PS_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        PS_HIP(hipEventElapsedTime(&ms, e0, e1));
        expand_ms += ms;
      }
      st->expand_launches++;
      st->steps++;
      cur = nxt;
      ccap = ncap;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    unsigned long long tail[2];
    PS_HIP(hipMemcpyAsync(tail, ctr, sizeof(tail), hipMemcpyDeviceToHost, stm));
    unsigned long long fin = 0;
    PS_HIP(hipMemcpyAsync(&fin, ctr + M_FINAL, sizeof(fin), hipMemcpyDeviceToHost, stm));
    PS_HIP(hipStreamSynchronize(stm));
    st->final_adds += (int64_t)fin;
    st->pushed_final_adds += (int64_t)fin;
    st->probe_levels += (int64_t)dmax - 1;
    st->expand_ms += expand_ms;
    if (tail[M_OVERFLOW]) {  // a table filled up: release the record, fail the call
      PS_TRY(session_finish(ctx, g, r, q, out));
      return PS_ERR_OOM;
    }
  }
  st->pushed_edges = st->edges_scanned;
  return session_finish(ctx, g, r, q, out);
}
