// Device graph store: in- and out-adjacency, 1/|I(v)|, versioned updates.
//
// Layout in HBM (per adjacency direction):
//   col[cap]      int32 neighbour ids.  The base CSR fills col[0, m); rows
//                 rewritten by updates are appended after it (delta region).
//   rows[n]       uint2 (start, len): row of node v is col[start, start+len).
//   inv_indeg[n]  float 1/|I(v)|, read by every PROBE expansion.
// In-rows are kept in ascending source-id order at every version, which is
// the order walks index into, so walks are identical on a graph built by
// updates and on the same edge set loaded from scratch.
//
// A graph version is immutable: an update batch copies the row index arrays,
// appends the rewritten rows to the delta region and publishes the copy as
// the new version.  Queries hold a reference to the version they started on.

#include <algorithm>
#include <cstring>

#include "ps_internal.h"

namespace {

constexpr uint64_t kMinSlack = 1ull << 20;

// 1/d rounded to the nearest FP32 number, in integer arithmetic so that it
// does not depend on how the compiler divides: with 2^k <= d < 2^(k+1) and d
// not a power of two, 1/d lies in (2^-(k+1), 2^-k), its 24-bit mantissa is
// round(2^(24+k) / d) (never a tie) and the value is that times 2^-(24+k).
__host__ __device__ float recip_rn(uint32_t d) {
  const int k = 31 - __builtin_clz(d);
  if ((d & (d - 1)) == 0) return ldexpf(1.0f, -k);
  const uint64_t mant = ((1ull << (24 + k)) + (d >> 1)) / d;
  return ldexpf((float)mant, -(24 + k));
}

__global__ void k_patch_rows(const int32_t* __restrict__ node, const uint2* __restrict__ row, int32_t cnt,
                             uint2* __restrict__ rows, float* __restrict__ inv_indeg) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int32_t v = node[i];
  rows[v] = row[i];
  if (inv_indeg) inv_indeg[v] = row[i].y ? recip_rn(row[i].y) : 0.0f;
}

// Lists the nodes with more than kPullLane in-neighbours and cuts their
// in-rows into kPullChunk-edge chunks (order of the lists is irrelevant).
__global__ void k_heavy(int32_t n, const uint2* __restrict__ in_rows, int32_t* __restrict__ nodes,
                        int2* __restrict__ chunks, unsigned long long* __restrict__ cnt) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t d = in_rows[v].y;
  if (d <= kPullLane) return;
  nodes[atomicAdd(&cnt[0], 1ull)] = (int32_t)v;
  const uint32_t nch = (d + kPullChunk - 1) / kPullChunk;
  const unsigned long long base = atomicAdd(&cnt[1], (unsigned long long)nch);
  for (uint32_t c = 0; c < nch; ++c) chunks[base + c] = make_int2((int32_t)v, (int32_t)(c * kPullChunk));
}

ps_status alloc_version_arrays(GraphVersion* v, int32_t n) {
  PS_HIP(hipMalloc(&v->in_rows, sizeof(uint2) * (size_t)n));
  PS_HIP(hipMalloc(&v->out_rows, sizeof(uint2) * (size_t)n));
  PS_HIP(hipMalloc(&v->inv_indeg, sizeof(float) * (size_t)n));
  return PS_OK;
}

// (Re)builds the heavy in-row lists of a version from its in_rows.  Chunks
// are bounded by m / kPullChunk + (nodes with long rows) <= m_cap / kPullChunk + n.
ps_status build_heavy(GraphVersion* v, int32_t n, uint64_t m_cap, hipStream_t st) {
  const uint64_t chunk_cap = m_cap / kPullChunk + (uint64_t)n + 1;
  if (v->heavy_chunks && v->heavy_chunk_cap < chunk_cap) {  // a compaction grew the column store
    (void)hipFree(v->heavy_chunks);
    v->heavy_chunks = nullptr;
  }
  if (!v->heavy_nodes) {
    PS_HIP(hipMalloc(&v->heavy_nodes, sizeof(int32_t) * (size_t)n));
    PS_HIP(hipMalloc(&v->heavy_cnt, sizeof(unsigned long long) * 2));
  }
  if (!v->heavy_chunks) {
    PS_HIP(hipMalloc(&v->heavy_chunks, sizeof(int2) * chunk_cap));
    v->heavy_chunk_cap = chunk_cap;
  }
  PS_HIP(hipMemsetAsync(v->heavy_cnt, 0, sizeof(unsigned long long) * 2, st));
  k_heavy<<<(n + 255) / 256, 256, 0, st>>>(n, v->in_rows, v->heavy_nodes, v->heavy_chunks, v->heavy_cnt);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

void drop_stores(GraphVersion* v) {
  if (v->in_store && --v->in_store->refs == 0) (void)hipFree(v->in_store->col);
  if (v->out_store && --v->out_store->refs == 0) (void)hipFree(v->out_store->col);
  v->in_store.reset();
  v->out_store.reset();
}

void free_heavy(GraphVersion* v) {
  (void)hipFree(v->heavy_nodes);
  (void)hipFree(v->heavy_chunks);
  (void)hipFree(v->heavy_cnt);
  v->heavy_nodes = nullptr;
  v->heavy_chunks = nullptr;
  v->heavy_cnt = nullptr;
}

void free_version(GraphVersion* v) {
  if (!v) return;
  (void)hipFree(v->in_rows);
  (void)hipFree(v->out_rows);
  (void)hipFree(v->inv_indeg);
  free_heavy(v);
  drop_stores(v);
  delete v;
}

// A superseded version's row arrays are kept for the next update batch
// (a few at most), which saves an allocation per batch.
void retire_version(ps_graph* g, GraphVersion* v) {
  drop_stores(v);
  if (g->spare.size() < 4) {
    g->spare.push_back(v);
  } else {
    free_version(v);
  }
}

GraphVersion* new_version(ps_graph* g) {
  if (!g->spare.empty()) {
    GraphVersion* v = g->spare.back();
    g->spare.pop_back();
    GraphVersion* fresh = new GraphVersion();
    fresh->in_rows = v->in_rows;
    fresh->out_rows = v->out_rows;
    fresh->inv_indeg = v->inv_indeg;
    fresh->heavy_nodes = v->heavy_nodes;
    fresh->heavy_chunks = v->heavy_chunks;
    fresh->heavy_cnt = v->heavy_cnt;
    fresh->heavy_chunk_cap = v->heavy_chunk_cap;
    delete v;
    return fresh;
  }
  return new GraphVersion();
}

// Row of v in the host mirror (rewritten row if any, else the base CSR row).
const int32_t* host_row(const std::vector<int64_t>& ptr, const std::vector<int32_t>& col,
                        const std::unordered_map<int32_t, std::vector<int32_t>>& mod, int32_t v, int64_t* len) {
  auto it = mod.find(v);
  if (it != mod.end()) {
    *len = (int64_t)it->second.size();
    return it->second.data();
  }
  *len = ptr[v + 1] - ptr[v];
  return col.data() + ptr[v];
}

std::vector<int32_t>& mutable_row(const std::vector<int64_t>& ptr, const std::vector<int32_t>& col,
                                  std::unordered_map<int32_t, std::vector<int32_t>>& mod, int32_t v) {
  auto it = mod.find(v);
  if (it != mod.end()) return it->second;
  auto& r = mod[v];
  r.assign(col.begin() + ptr[v], col.begin() + ptr[v + 1]);
  return r;
}

// Uploads the whole host mirror as a fresh column store pair + version.
ps_status upload_full(ps_graph* g, GraphVersion* v) {
  const int32_t n = g->n;
  const uint64_t m = (uint64_t)g->m;
  const uint64_t slack = std::max<uint64_t>(kMinSlack, m / 8);
  auto in_store = std::make_shared<ColStore>();
  auto out_store = std::make_shared<ColStore>();
  in_store->cap = out_store->cap = m + slack;
  if (in_store->cap >= (1ull << 32)) return PS_ERR_INVALID_ARG;
  PS_HIP(hipMalloc(&in_store->col, sizeof(int32_t) * in_store->cap));
  PS_HIP(hipMalloc(&out_store->col, sizeof(int32_t) * out_store->cap));
  std::vector<int32_t> in_col, out_col;
  std::vector<uint2> in_rows((size_t)n), out_rows((size_t)n);
  std::vector<float> inv((size_t)n);
  in_col.reserve(m);
  out_col.reserve(m);
  for (int32_t x = 0; x < n; ++x) {
    int64_t li, lo;
    const int32_t* ri = host_row(g->h_in_ptr, g->h_in_col, g->mod_in, x, &li);
    const int32_t* ro = host_row(g->h_out_ptr, g->h_out_col, g->mod_out, x, &lo);
    in_rows[x] = make_uint2((uint32_t)in_col.size(), (uint32_t)li);
    out_rows[x] = make_uint2((uint32_t)out_col.size(), (uint32_t)lo);
    in_col.insert(in_col.end(), ri, ri + li);
    out_col.insert(out_col.end(), ro, ro + lo);
    inv[x] = li ? recip_rn((uint32_t)li) : 0.0f;
  }
  in_store->used = in_col.size();
  out_store->used = out_col.size();
  hipStream_t st = g->ctx->stream;
  if (!in_col.empty()) {
    PS_HIP(hipMemcpyAsync(in_store->col, in_col.data(), sizeof(int32_t) * in_col.size(), hipMemcpyHostToDevice, st));
    PS_HIP(hipMemcpyAsync(out_store->col, out_col.data(), sizeof(int32_t) * out_col.size(), hipMemcpyHostToDevice, st));
  }
  PS_TRY(alloc_version_arrays(v, n));
  PS_HIP(hipMemcpyAsync(v->in_rows, in_rows.data(), sizeof(uint2) * (size_t)n, hipMemcpyHostToDevice, st));
  PS_HIP(hipMemcpyAsync(v->out_rows, out_rows.data(), sizeof(uint2) * (size_t)n, hipMemcpyHostToDevice, st));
  PS_HIP(hipMemcpyAsync(v->inv_indeg, inv.data(), sizeof(float) * (size_t)n, hipMemcpyHostToDevice, st));
  PS_TRY(build_heavy(v, n, in_store->cap, st));
  PS_HIP(hipStreamSynchronize(st));
  in_store->refs = out_store->refs = 1;
  v->in_store = in_store;
  v->out_store = out_store;
  // Fold the rewritten rows into the base CSR of the mirror.
  g->h_in_col.swap(in_col);
  g->h_out_col.swap(out_col);
  for (int32_t x = 0; x < n; ++x) {
    g->h_in_ptr[x] = in_rows[x].x;
    g->h_out_ptr[x] = out_rows[x].x;
  }
  g->h_in_ptr[n] = (int64_t)g->h_in_col.size();
  g->h_out_ptr[n] = (int64_t)g->h_out_col.size();
  g->mod_in.clear();
  g->mod_out.clear();
  return PS_OK;
}

}  // namespace

GraphVersion* graph_acquire(ps_graph* g) {
  std::lock_guard<std::mutex> lk(g->mu);
  g->cur->refs++;
  return g->cur;
}

void graph_release(ps_graph* g, GraphVersion* v) {
  std::lock_guard<std::mutex> lk(g->mu);
  if (--v->refs == 0) {
    g->retired.erase(std::remove(g->retired.begin(), g->retired.end(), v), g->retired.end());
    retire_version(g, v);
  }
}

int64_t graph_host_indeg(const ps_graph* g, int32_t v) {
  int64_t len;
  host_row(g->h_in_ptr, g->h_in_col, g->mod_in, v, &len);
  return len;
}

extern "C" ps_status ps_graph_load(ps_ctx* ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                                   uint32_t flags, ps_graph** out) {
  if (!out) return PS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!ctx || n <= 0 || m < 0 || m >= (1ll << 31) || (m > 0 && (!src || !dst))) return PS_ERR_INVALID_ARG;
  // Edge lists in device memory (a torch tensor's pointer) are copied to the
  // host first: the host mirror is built from them.
  std::vector<int32_t> hsrc, hdst;
  if (m > 0 && (ps_is_device_ptr(src) || ps_is_device_ptr(dst))) {
    PS_HIP(hipSetDevice(ctx->device));
    hsrc.resize((size_t)m);
    hdst.resize((size_t)m);
    PS_HIP(hipMemcpy(hsrc.data(), src, sizeof(int32_t) * (size_t)m, hipMemcpyDefault));
    PS_HIP(hipMemcpy(hdst.data(), dst, sizeof(int32_t) * (size_t)m, hipMemcpyDefault));
    src = hsrc.data();
    dst = hdst.data();
  }
  for (int64_t i = 0; i < m; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return PS_ERR_NODE_RANGE;
  // Counting sort by source, then sort each out-row by target.
  std::vector<int64_t> optr((size_t)n + 1, 0);
  for (int64_t i = 0; i < m; ++i) optr[src[i] + 1]++;
  for (int32_t v = 0; v < n; ++v) optr[v + 1] += optr[v];
  std::vector<int32_t> ocol((size_t)m);
  {
    std::vector<int64_t> fill(optr.begin(), optr.end() - 1);
    for (int64_t i = 0; i < m; ++i) ocol[fill[src[i]]++] = dst[i];
  }
  // Validate (self-loops, duplicates) and compact per row.
  std::vector<int64_t> nptr((size_t)n + 1, 0);
  int64_t w = 0;
  for (int32_t x = 0; x < n; ++x) {
    const int64_t b = optr[x], e = optr[x + 1];
    std::sort(ocol.begin() + b, ocol.begin() + e);
    nptr[x] = w;
    for (int64_t i = b; i < e; ++i) {
      const int32_t y = ocol[i];
      if (y == x) {
        if (flags & PS_LOAD_DROP_SELF_LOOPS) continue;
        return PS_ERR_SELF_LOOP;
      }
      if (i > b && ocol[i - 1] == y) {
        if (flags & PS_LOAD_DEDUP) continue;
        return PS_ERR_DUP_EDGE;
      }
      ocol[w++] = y;
    }
  }
  nptr[n] = w;
  ocol.resize((size_t)w);
  // In-rows: visiting sources in ascending order leaves each in-row sorted.
  std::vector<int64_t> iptr((size_t)n + 1, 0);
  for (int64_t i = 0; i < w; ++i) iptr[ocol[i] + 1]++;
  for (int32_t v = 0; v < n; ++v) iptr[v + 1] += iptr[v];
  std::vector<int32_t> icol((size_t)w);
  {
    std::vector<int64_t> fill(iptr.begin(), iptr.end() - 1);
    for (int32_t x = 0; x < n; ++x)
      for (int64_t i = nptr[x]; i < nptr[x + 1]; ++i) icol[fill[ocol[i]]++] = x;
  }
  auto* g = new ps_graph();
  g->ctx = ctx;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->refs++;
  }
  g->n = n;
  g->m = w;
  g->h_in_ptr.swap(iptr);
  g->h_in_col.swap(icol);
  g->h_out_ptr.swap(nptr);
  g->h_out_col.swap(ocol);
  PS_HIP(hipSetDevice(ctx->device));
  auto* v = new GraphVersion();
  v->refs = 1;
  ps_status s = upload_full(g, v);
  if (s != PS_OK) {
    free_version(v);
    ctx_release(ctx);
    delete g;
    return s;
  }
  g->cur = v;
  *out = g;
  return PS_OK;
}

extern "C" void ps_graph_free(ps_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->ctx->device);
  (void)hipStreamSynchronize(g->ctx->stream);
  for (auto* v : g->retired) free_version(v);
  for (auto* v : g->spare) free_version(v);
  free_version(g->cur);
  for (int i = 0; i < ps_graph::kStages; ++i) {
    if (g->h_stage[i]) (void)hipHostFree(g->h_stage[i]);
    devbuf_free(g->d_stage[i]);
    if (g->stage_ev[i]) (void)hipEventDestroy(g->stage_ev[i]);
  }
  ps_ctx* ctx = g->ctx;
  delete g;
  ctx_release(ctx);
}

extern "C" ps_status ps_graph_info(const ps_graph* g, int32_t* n, int64_t* m, uint64_t* version) {
  if (!g) return PS_ERR_INVALID_ARG;
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (version) *version = g->cur->version;
  return PS_OK;
}

extern "C" ps_status ps_graph_edges(const ps_graph* g, int64_t cap, int32_t* src, int32_t* dst, int64_t* m) {
  if (!g || !m) return PS_ERR_INVALID_ARG;
  *m = g->m;
  if (cap < g->m || (g->m > 0 && (!src || !dst))) return PS_ERR_INVALID_ARG;
  int64_t w = 0;
  for (int32_t x = 0; x < g->n; ++x) {
    int64_t len;
    const int32_t* r = host_row(g->h_out_ptr, g->h_out_col, g->mod_out, x, &len);
    for (int64_t i = 0; i < len; ++i) {
      src[w] = x;
      dst[w] = r[i];
      ++w;
    }
  }
  return PS_OK;
}

ps_status graph_apply_updates(ps_graph* g, int64_t k, const int32_t* src, const int32_t* dst, const uint8_t* op,
                              int32_t* per_edge, uint64_t* version) {
  TraceRange tr("probesim graph update");
  if (!g || k < 0 || (k > 0 && (!src || !dst || !op))) return PS_ERR_INVALID_ARG;
  for (int64_t i = 0; i < k; ++i) {
    if (src[i] < 0 || src[i] >= g->n || dst[i] < 0 || dst[i] >= g->n) return PS_ERR_NODE_RANGE;
    if (op[i] > 1) return PS_ERR_INVALID_ARG;
  }
  ps_status first_err = PS_OK;
  std::vector<int32_t> touched_in, touched_out;
  for (int64_t i = 0; i < k; ++i) {
    const int32_t x = src[i], y = dst[i];
    ps_status st = PS_OK;
    if (x == y) {
      st = PS_ERR_SELF_LOOP;
    } else {
      auto& orow = mutable_row(g->h_out_ptr, g->h_out_col, g->mod_out, x);
      auto pos = std::lower_bound(orow.begin(), orow.end(), y);
      const bool present = pos != orow.end() && *pos == y;
      if (op[i] == 0 && present) {
        st = PS_ERR_DUP_EDGE;
      } else if (op[i] == 1 && !present) {
        st = PS_ERR_NO_EDGE;
      } else {
        auto& irow = mutable_row(g->h_in_ptr, g->h_in_col, g->mod_in, y);
        auto ipos = std::lower_bound(irow.begin(), irow.end(), x);
        if (op[i] == 0) {
          orow.insert(pos, y);
          irow.insert(ipos, x);
          g->m++;
        } else {
          orow.erase(pos);
          irow.erase(ipos);
          g->m--;
        }
        touched_out.push_back(x);
        touched_in.push_back(y);
      }
    }
    if (per_edge) per_edge[i] = st;
    if (st != PS_OK && first_err == PS_OK) first_err = st;
  }
  std::sort(touched_in.begin(), touched_in.end());
  touched_in.erase(std::unique(touched_in.begin(), touched_in.end()), touched_in.end());
  std::sort(touched_out.begin(), touched_out.end());
  touched_out.erase(std::unique(touched_out.begin(), touched_out.end()), touched_out.end());

  if (!touched_in.empty()) {
    ps_ctx* ctx = g->ctx;
    hipStream_t st = ctx->stream;
    PS_HIP(hipSetDevice(ctx->device));
    GraphVersion* old = g->cur;
    GraphVersion* v;
    {
      std::lock_guard<std::mutex> lk(g->mu);
      v = new_version(g);
    }
    v->version = old->version + 1;
    v->refs = 1;
    uint64_t need_in = 0, need_out = 0;
    for (int32_t y : touched_in) need_in += g->mod_in[y].size();
    for (int32_t x : touched_out) need_out += g->mod_out[x].size();
    const bool fits = old->in_store->used + need_in <= old->in_store->cap &&
                      old->out_store->used + need_out <= old->out_store->cap;
    if (!fits) {
      // Delta region exhausted: compact everything into fresh column stores.
      if (v->in_rows) {
        (void)hipFree(v->in_rows);
        (void)hipFree(v->out_rows);
        (void)hipFree(v->inv_indeg);
        v->in_rows = nullptr;
        v->out_rows = nullptr;
        v->inv_indeg = nullptr;
      }
      ps_status s = upload_full(g, v);
      if (s != PS_OK) {
        free_version(v);
        return s;
      }
    } else {
      if (!v->in_rows) PS_TRY(alloc_version_arrays(v, g->n));
      PS_HIP(hipMemcpyAsync(v->in_rows, old->in_rows, sizeof(uint2) * (size_t)g->n, hipMemcpyDeviceToDevice, st));
      PS_HIP(hipMemcpyAsync(v->out_rows, old->out_rows, sizeof(uint2) * (size_t)g->n, hipMemcpyDeviceToDevice, st));
      PS_HIP(hipMemcpyAsync(v->inv_indeg, old->inv_indeg, sizeof(float) * (size_t)g->n, hipMemcpyDeviceToDevice, st));
      v->in_store = old->in_store;
      v->out_store = old->out_store;
      v->in_store->refs++;
      v->out_store->refs++;
      // Rewritten rows go to the end of the column stores' delta regions;
      // (node, start, len) patches fix the version's row arrays.  Both
      // directions share one pinned staging fill and one device buffer.
      struct Part {
        std::vector<int32_t> cols, nodes;
        std::vector<uint2> rows;
        uint64_t base = 0;
      } parts[2];
      auto gather = [&](const std::vector<int32_t>& nodes, std::unordered_map<int32_t, std::vector<int32_t>>& mod,
                        ColStore* store, Part& P) {
        P.base = store->used;
        for (int32_t a : nodes) {
          auto& r = mod[a];
          P.nodes.push_back(a);
          P.rows.push_back(make_uint2((uint32_t)(P.base + P.cols.size()), (uint32_t)r.size()));
          P.cols.insert(P.cols.end(), r.begin(), r.end());
        }
        store->used = P.base + P.cols.size();
      };
      gather(touched_in, g->mod_in, v->in_store.get(), parts[0]);
      gather(touched_out, g->mod_out, v->out_store.get(), parts[1]);
      auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
      size_t off[2][3], total = 0;
      for (int d = 0; d < 2; ++d) {
        off[d][0] = total;
        total += up(sizeof(int32_t) * parts[d].cols.size());
        off[d][1] = total;
        total += up(sizeof(int32_t) * parts[d].nodes.size());
        off[d][2] = total;
        total += up(sizeof(uint2) * parts[d].rows.size());
      }
      const int sg = g->stage_next;
      g->stage_next = (sg + 1) % ps_graph::kStages;
      if (g->stage_live[sg]) PS_HIP(hipEventSynchronize(g->stage_ev[sg]));  // its last uploads are done
      if (g->h_stage_bytes[sg] < total) {
        if (g->h_stage[sg]) PS_HIP(hipHostFree(g->h_stage[sg]));
        g->h_stage[sg] = nullptr;
        g->h_stage_bytes[sg] = 0;
        PS_HIP(hipHostMalloc(&g->h_stage[sg], total, 0));
        g->h_stage_bytes[sg] = total;
      }
      if (!g->stage_ev[sg]) PS_HIP(hipEventCreateWithFlags(&g->stage_ev[sg], hipEventDisableTiming));
      PS_TRY(devbuf_reserve(g->d_stage[sg], total));
      char* hs = static_cast<char*>(g->h_stage[sg]);
      char* ds = static_cast<char*>(g->d_stage[sg].p);
      for (int d = 0; d < 2; ++d) {
        Part& P = parts[d];
        ColStore* store = d == 0 ? v->in_store.get() : v->out_store.get();
        std::memcpy(hs + off[d][0], P.cols.data(), sizeof(int32_t) * P.cols.size());
        std::memcpy(hs + off[d][1], P.nodes.data(), sizeof(int32_t) * P.nodes.size());
        std::memcpy(hs + off[d][2], P.rows.data(), sizeof(uint2) * P.rows.size());
        if (!P.cols.empty())
          PS_HIP(hipMemcpyAsync(store->col + P.base, hs + off[d][0], sizeof(int32_t) * P.cols.size(),
                                hipMemcpyHostToDevice, st));
        if (P.nodes.empty()) continue;
        PS_HIP(hipMemcpyAsync(ds + off[d][1], hs + off[d][1], off[d][2] - off[d][1] + sizeof(uint2) * P.rows.size(),
                              hipMemcpyHostToDevice, st));
        const int32_t cnt = (int32_t)P.nodes.size();
        k_patch_rows<<<(cnt + 255) / 256, 256, 0, st>>>(reinterpret_cast<const int32_t*>(ds + off[d][1]),
                                                        reinterpret_cast<const uint2*>(ds + off[d][2]), cnt,
                                                        d == 0 ? v->in_rows : v->out_rows,
                                                        d == 0 ? v->inv_indeg : nullptr);
        PS_HIP(hipGetLastError());
      }
      PS_HIP(hipEventRecord(g->stage_ev[sg], st));
      g->stage_live[sg] = true;
      PS_TRY(build_heavy(v, g->n, v->in_store->cap, st));
    }
    {
      std::lock_guard<std::mutex> lk(g->mu);
      g->cur = v;
      if (--old->refs == 0)
        retire_version(g, old);
      else
        g->retired.push_back(old);
    }
  }
  if (version) *version = g->cur->version;
  if (per_edge) return PS_OK;
  return first_err;
}

extern "C" ps_status ps_graph_update(ps_graph* g, int64_t k, const int32_t* src, const int32_t* dst,
                                     const uint8_t* op, int32_t* per_edge, uint64_t* version) {
  return graph_apply_updates(g, k, src, dst, op, per_edge, version);
}
