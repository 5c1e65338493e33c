// C ABI entry points: contexts, parameters, queries, statistics.

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "ps_internal.h"

void ps_note_hip_error(hipError_t e, const char* what, const char* file, int line) {
  fprintf(stderr, "probesim: %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
}

bool ps_is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

extern "C" const char* ps_status_string(ps_status s) {
  switch (s) {
    case PS_OK: return "ok";
    case PS_ERR_INVALID_ARG: return "invalid argument";
    case PS_ERR_NODE_RANGE: return "node id out of range";
    case PS_ERR_SELF_LOOP: return "self-loop";
    case PS_ERR_DUP_EDGE: return "duplicate edge";
    case PS_ERR_NO_EDGE: return "edge not present";
    case PS_ERR_OOM: return "out of memory";
    case PS_ERR_BUSY: return "busy";
    case PS_ERR_DEVICE: return "device error";
    case PS_ERR_TIMEOUT: return "timeout";
    case PS_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

extern "C" ps_status ps_ctx_create(int device, void* hip_stream, ps_ctx** out) {
  if (!out) return PS_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  PS_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return PS_ERR_INVALID_ARG;
  PS_HIP(hipSetDevice(device));
  PS_TRY(select_scratch_init(device));
  auto* c = new ps_ctx();
  c->device = device;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return PS_ERR_DEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return PS_OK;
}

extern "C" void ps_ctx_destroy(ps_ctx* c) { ctx_release(c); }

// Graphs keep their context alive, so destroying a context while graphs
// still use it only drops the caller's reference.
void ctx_release(ps_ctx* c) {
  if (!c) return;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (--c->refs > 0) return;
  }
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  session_free(c->sess);
  c->sess = nullptr;
  for (DevBuf* b : {&c->sel.state, &c->sel.keys, &c->sel.ids, &c->sel_in, &c->sel_ids, &c->sel_scores}) devbuf_free(*b);
  for (hipEvent_t ev : c->ev_pool) (void)hipEventDestroy(ev);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" ps_status ps_ctx_set_timing(ps_ctx* c, int enable) {
  if (!c) return PS_ERR_INVALID_ARG;
  c->timing = enable != 0;
  return PS_OK;
}

extern "C" void ps_options_default(ps_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->eps_s = -1.0;
  o->eps_t = -1.0;
  o->eps_p = -1.0;
  o->walk_begin = 0;
  o->walk_end = -1;
  o->hybrid_c0 = 0.003;  // fastest measured on power-law graphs; the paper leaves c0 open
}

// Theorem 2's pruning term is (1 + eps_s) * eps_p / factor: the expected
// number of probes per walk, 1 / (1 - sqrt c), times eps_p per probe as the
// paper's Rule 2 lemma states; or E[l(l-1)/2] = sqrt(c) / (1 - sqrt c)^2
// times eps_p under the per-probe bound (i - 1) * eps_p that the lemma's
// induction gives with the pruned node's own score kept.
static double rule2_factor(double sc, int32_t bound) {
  return bound == PS_RULE2_PROVEN ? (1.0 - sc) * (1.0 - sc) / sc : 1.0 - sc;
}

// Alg. 1 (number of walks), Rule 1 (truncation), Theorem 2 (error split).
ps_status derive_params(int32_t n, double c, double eps, double delta, const ps_options* opt, ps_params* p) {
  if (!p || n <= 0) return PS_ERR_INVALID_ARG;
  if (!(c > 0.0 && c < 1.0) || !(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0)) return PS_ERR_INVALID_ARG;
  ps_options d;
  ps_options_default(&d);
  if (!opt) opt = &d;
  const double sc = std::sqrt(c);
  p->c = c;
  p->eps_a = eps;
  p->delta = delta;
  p->eps_s = opt->eps_s >= 0.0 ? opt->eps_s : eps / 2.0;
  p->eps_t = opt->eps_t >= 0.0 ? opt->eps_t : eps / 4.0;
  if (opt->rule2_bound != PS_RULE2_AS_STATED && opt->rule2_bound != PS_RULE2_PROVEN) return PS_ERR_INVALID_ARG;
  p->eps_p = opt->eps_p >= 0.0 ? opt->eps_p : (eps / 4.0) * rule2_factor(sc, opt->rule2_bound) / (1.0 + p->eps_s);
  if (!(p->eps_s > 0.0) || !(p->eps_t > 0.0 && p->eps_t < 1.0)) return PS_ERR_INVALID_ARG;
  const double nr = std::ceil(3.0 * c * std::log((double)n / delta) / (p->eps_s * p->eps_s));
  if (!(nr >= 1.0) || nr > 2147483647.0) return PS_ERR_INVALID_ARG;
  p->n_r = (int64_t)nr;
  p->L = opt->max_len > 0 ? opt->max_len : (int32_t)std::floor(std::log(p->eps_t) / std::log(sc));
  if (p->L < 2 || p->L > PS_MAX_WALK_LEN) return PS_ERR_INVALID_ARG;
  p->t_stop = (uint32_t)std::floor((1.0 - sc) * 4294967296.0);
  return PS_OK;
}

extern "C" ps_status ps_derive_params(int32_t n, double c, double eps, double delta, const ps_options* opt,
                                      ps_params* out) {
  return derive_params(n, c, eps, delta, opt, out);
}

ps_status make_query_run(const ps_graph* g, int32_t u, int32_t k, double c, double eps, double delta, uint64_t seed,
                   const ps_options* opt, QueryRun* q) {
  if (u < 0 || u >= g->n) return PS_ERR_NODE_RANGE;
  if (k < 0 || (k > 0 && k > g->n - 1)) return PS_ERR_INVALID_ARG;
  PS_TRY(derive_params(g->n, c, eps, delta, opt, &q->prm));
  q->u = u;
  q->k = k;
  q->seed = seed;
  q->walk_begin = opt ? opt->walk_begin : 0;
  q->walk_end = (opt && opt->walk_end >= 0) ? opt->walk_end : q->prm.n_r;
  q->bias_shift = opt ? opt->bias_shift : 0;
  const int mode = opt ? opt->probe_mode : PS_PROBE_DETERMINISTIC;
  if (mode != PS_PROBE_DETERMINISTIC && mode != PS_PROBE_RANDOMIZED && mode != PS_PROBE_HYBRID &&
      mode != PS_PROBE_MERGED)
    return PS_ERR_INVALID_ARG;
  q->merged = mode == PS_PROBE_MERGED;
  if (q->merged) q->prm.eps_p = 0.0;  // Rule 2 has no merged form
  q->randomized = mode == PS_PROBE_RANDOMIZED;
  q->hybrid = mode == PS_PROBE_HYBRID;
  q->c0 = q->hybrid ? opt->hybrid_c0 : 0.0;
  if (q->hybrid && !(q->c0 >= 0.0)) return PS_ERR_INVALID_ARG;  // NaN too
  if (q->walk_begin < 0 || q->walk_end > q->prm.n_r || q->walk_begin > q->walk_end) return PS_ERR_INVALID_ARG;
  return PS_OK;
}

namespace {

ps_status run_locked(ps_graph* g, const std::vector<QueryRun>& qs, const std::vector<QueryOut>& outs,
                     const ps_options* opt) {
  ps_ctx* ctx = g->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  PS_HIP(hipSetDevice(ctx->device));
  GraphVersion* gv = graph_acquire(g);
  int slots = opt ? opt->slots : 0;
  int64_t dense = opt ? opt->pull_edges : 0;
  if (slots == 0) slots = g->tuned_slots;
  if (dense == 0) dense = g->tuned_dense;
  ps_status s = engine_run(ctx, g, gv, qs, outs, slots, dense);
  graph_release(g, gv);
  return s;
}

}  // namespace

extern "C" ps_status ps_walks(ps_graph* g, int32_t u, double c, double eps, double delta, uint64_t seed,
                              const ps_options* opt, int64_t k_begin, int64_t count, int32_t* nodes, int32_t* lens) {
  if (!g || count < 0 || k_begin < 0 || (count > 0 && (!nodes || !lens))) return PS_ERR_INVALID_ARG;
  QueryRun q;
  PS_TRY(make_query_run(g, u, 0, c, eps, delta, seed, opt, &q));
  if (k_begin + count > (int64_t)1 << 32) return PS_ERR_INVALID_ARG;
  ps_ctx* ctx = g->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  PS_HIP(hipSetDevice(ctx->device));
  GraphVersion* gv = graph_acquire(g);
  ps_status s = engine_walks(ctx, gv, g->n, q, k_begin, count, nodes, lens);
  graph_release(g, gv);
  return s;
}

extern "C" ps_status ps_single_source(ps_graph* g, int32_t u, double c, double eps, double delta, uint64_t seed,
                                      const ps_options* opt, double* out) {
  if (!g || !out) return PS_ERR_INVALID_ARG;
  QueryRun q;
  PS_TRY(make_query_run(g, u, 0, c, eps, delta, seed, opt, &q));
  QueryOut o;
  o.scores = out;
  return run_locked(g, {q}, {o}, opt);
}

extern "C" ps_status ps_single_source_sparse(ps_graph* g, int32_t u, double c, double eps, double delta,
                                             uint64_t seed, const ps_options* opt, int64_t cap, int32_t* nodes,
                                             double* scores, int64_t* count) {
  if (!g || cap < 0 || !count || (cap > 0 && (!nodes || !scores))) return PS_ERR_INVALID_ARG;
  QueryRun q;
  PS_TRY(make_query_run(g, u, 0, c, eps, delta, seed, opt, &q));
  QueryOut o;
  o.scores = scores;
  o.nodes = nodes;
  o.cap = cap;
  o.count = count;
  *count = 0;
  PS_TRY(run_locked(g, {q}, {o}, opt));
  return *count > cap ? PS_ERR_INVALID_ARG : PS_OK;
}

extern "C" ps_status ps_topk(ps_graph* g, int32_t u, int32_t k, double c, double eps, double delta, uint64_t seed,
                             const ps_options* opt, int32_t* nodes, double* scores) {
  if (!g || !nodes || !scores || k < 1) return PS_ERR_INVALID_ARG;
  QueryRun q;
  PS_TRY(make_query_run(g, u, k, c, eps, delta, seed, opt, &q));
  QueryOut o;
  o.scores = scores;
  o.nodes = nodes;
  return run_locked(g, {q}, {o}, opt);
}

extern "C" ps_status ps_select_topk(ps_ctx* c, const double* scores, int32_t n, int32_t u, int32_t k,
                                    int32_t* nodes, double* out_scores) {
  if (!c || !scores || !nodes || !out_scores || n < 2) return PS_ERR_INVALID_ARG;
  if (u < 0 || u >= n) return PS_ERR_NODE_RANGE;
  if (k < 1 || k > n - 1) return PS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  PS_HIP(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const double* s = scores;
  if (!ps_is_device_ptr(scores)) {
    PS_TRY(devbuf_reserve(c->sel_in, sizeof(double) * (size_t)n));
    PS_HIP(hipMemcpyAsync(c->sel_in.p, scores, sizeof(double) * (size_t)n, hipMemcpyHostToDevice, st));
    s = c->sel_in.as<double>();
  }
  PS_TRY(devbuf_reserve(c->sel_ids, sizeof(int32_t) * (size_t)k));
  PS_TRY(devbuf_reserve(c->sel_scores, sizeof(double) * (size_t)k));
  PS_TRY(select_topk(c->sel, s, n, u, k, c->sel_ids.as<int32_t>(), c->sel_scores.as<double>(), st));
  PS_TRY(copy_out(nodes, c->sel_ids.p, sizeof(int32_t) * (size_t)k, st));
  PS_TRY(copy_out(out_scores, c->sel_scores.p, sizeof(double) * (size_t)k, st));
  PS_HIP(hipStreamSynchronize(st));
  return PS_OK;
}

extern "C" ps_status ps_batch(ps_graph* g, int32_t nq, const ps_query* qv, const ps_options* opt, ps_result* r) {
  if (!g || nq < 0 || (nq > 0 && (!qv || !r))) return PS_ERR_INVALID_ARG;
  if (opt && (opt->walk_begin != 0 || opt->walk_end >= 0)) return PS_ERR_INVALID_ARG;
  std::vector<QueryRun> qs;
  std::vector<QueryOut> outs;
  std::vector<int32_t> which;
  for (int32_t i = 0; i < nq; ++i) {
    QueryRun q;
    ps_options qo;
    if (opt) qo = *opt;
    else ps_options_default(&qo);
    if (qv[i].probe_mode) {
      qo.probe_mode = qv[i].probe_mode;
      if (qv[i].probe_mode == PS_PROBE_HYBRID) qo.hybrid_c0 = qv[i].hybrid_c0;
    }
    ps_status s = make_query_run(g, qv[i].u, qv[i].k, qv[i].c, qv[i].eps, qv[i].delta, qv[i].seed, &qo, &q);
    if (s == PS_OK && (!r[i].scores || (qv[i].k > 0 && !r[i].nodes))) s = PS_ERR_INVALID_ARG;
    r[i].status = s;
    r[i].count = 0;
    r[i].flip_allowance = 0.0;
    if (s != PS_OK) continue;
    QueryOut o;
    o.scores = r[i].scores;
    o.nodes = r[i].nodes;
    o.flip = &r[i].flip_allowance;
    qs.push_back(q);
    outs.push_back(o);
    which.push_back(i);
  }
  ps_status s = run_locked(g, qs, outs, opt);
  for (size_t j = 0; j < which.size(); ++j) {
    ps_result& rr = r[which[j]];
    rr.status = s;
    rr.count = s == PS_OK ? (qs[j].k > 0 ? qs[j].k : g->n) : 0;
  }
  return s;
}

extern "C" ps_status ps_get_stats(ps_ctx* c, ps_stats* out) {
  if (!c || !out) return PS_ERR_INVALID_ARG;
  *out = c->last;
  return PS_OK;
}

// ------------------------------------------------------------ autotuner --

namespace {

bool cache_lookup(const char* path, int32_t n, int64_t m, double eps, ps_tune* out) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  long long cn, cm, cd;
  int cs;
  double ce, cms;
  bool hit = false;
  while (fscanf(f, "%lld %lld %lf %d %lld %lf", &cn, &cm, &ce, &cs, &cd, &cms) == 6) {
    if (cn == n && cm == m && std::fabs(ce - eps) < 1e-12) {
      out->slots = cs;
      out->dense_edges = cd;
      out->ms_per_query = cms;
      hit = true;
    }
  }
  fclose(f);
  return hit;
}

}  // namespace

// Theorem 2: the split candidates of ps_tune_split, each meeting the
// inequality with equality (the pruning share takes what sampling and
// truncation leave).
extern "C" ps_status ps_tune_split(ps_graph* g, int32_t nsample, const int32_t* nodes, double c, double eps,
                                   double delta, ps_options* opt, ps_split* out) {
  if (!g || nsample <= 0 || !nodes || !opt || !out) return PS_ERR_INVALID_ARG;
  if (opt->walk_begin != 0 || opt->walk_end >= 0 || opt->eps_s >= 0.0 || opt->eps_t >= 0.0 || opt->eps_p >= 0.0)
    return PS_ERR_INVALID_ARG;
  if (!(c > 0.0 && c < 1.0) || !(eps > 0.0 && eps < 1.0)) return PS_ERR_INVALID_ARG;
  memset(out, 0, sizeof(*out));
  ps_ctx* ctx = g->ctx;
  const double sc = std::sqrt(c);
  const double shift = opt->bias_shift ? 0.5 : 1.0;
  struct Cand {
    double s, t, p;
  };
  std::vector<Cand> cands;
  for (double at : {0.25, 0.0625, 1.0 / 256.0}) {
    for (double as : {0.5, 0.6, 0.7, 0.75, 0.8, 0.85}) {
      const double es = as * eps, et = at * eps;
      const double rest = eps - es - shift * et;
      if (!(rest > 0.0)) continue;
      ps_options o = *opt;
      o.eps_s = es;
      o.eps_t = et;
      o.eps_p = rest * rule2_factor(sc, opt->rule2_bound) / (1.0 + es);
      ps_params prm;
      if (derive_params(g->n, c, eps, delta, &o, &prm) != PS_OK) continue;  // e.g. L beyond the cap
      cands.push_back({es, et, o.eps_p});
    }
  }
  if (cands.empty()) return PS_ERR_INVALID_ARG;
  double* dout = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    PS_HIP(hipSetDevice(ctx->device));
    PS_HIP(hipMalloc(&dout, sizeof(double) * (size_t)g->n));
  }
  double best = 1e300;
  ps_status st = PS_OK;
  for (size_t ci = 0; ci < cands.size() && st == PS_OK; ++ci) {
    ps_options o = *opt;
    o.eps_s = cands[ci].s;
    o.eps_t = cands[ci].t;
    o.eps_p = cands[ci].p;
    std::vector<QueryRun> qs;
    for (int32_t i = 0; i < nsample && st == PS_OK; ++i) {
      QueryRun q;
      st = make_query_run(g, nodes[i], 0, c, eps, delta, (uint64_t)(7 + i), &o, &q);
      qs.push_back(q);
    }
    double ms = 0.0;
    for (int rep = 0; rep < 2 && st == PS_OK; ++rep) {
      const auto t0 = std::chrono::steady_clock::now();
      for (auto& q : qs) {
        QueryOut qo;
        qo.scores = dout;
        std::lock_guard<std::mutex> lk(ctx->mu);
        GraphVersion* gv = graph_acquire(g);
        st = engine_run(ctx, g, gv, {q}, {qo}, o.slots, o.pull_edges);
        graph_release(g, gv);
        if (st != PS_OK) break;
      }
      if (rep == 1)
        ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / nsample;
    }
    if (st != PS_OK) break;
    if (ci == 0) out->default_ms_per_query = ms;
    if (ms < best) {
      best = ms;
      out->eps_s = cands[ci].s;
      out->eps_t = cands[ci].t;
      out->eps_p = cands[ci].p;
      out->ms_per_query = ms;
    }
  }
  (void)hipFree(dout);
  if (st != PS_OK) return st;
  opt->eps_s = out->eps_s;
  opt->eps_t = out->eps_t;
  opt->eps_p = out->eps_p;
  return PS_OK;
}

extern "C" ps_status ps_autotune(ps_graph* g, int32_t nsample, const int32_t* nodes, double c, double eps,
                                 double delta, const char* cache_path, ps_tune* out) {
  if (!g || nsample <= 0 || !nodes || !out) return PS_ERR_INVALID_ARG;
  ps_ctx* ctx = g->ctx;
  memset(out, 0, sizeof(*out));
  if (cache_path && cache_lookup(cache_path, g->n, g->m, eps, out)) {
    g->tuned_slots = out->slots;
    g->tuned_dense = out->dense_edges;
    out->from_cache = 1;
    return PS_OK;
  }
  std::vector<QueryRun> qs;
  for (int32_t i = 0; i < nsample; ++i) {
    QueryRun q;
    PS_TRY(make_query_run(g, nodes[i], 0, c, eps, delta, (uint64_t)(7 + i), nullptr, &q));
    qs.push_back(q);
  }
  double* dout = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    PS_HIP(hipSetDevice(ctx->device));
    PS_HIP(hipMalloc(&dout, sizeof(double) * (size_t)g->n));
  }
  const int max_slots = session_slots_for(g->n, 0);
  std::vector<int> slot_c = {max_slots};
  if (max_slots >= 1024) slot_c.push_back(512);
  const int64_t m = std::max<int64_t>(g->m, 1);
  const std::vector<int64_t> dense_c = {m / 40, m / 20, m / 10, -1};
  double best = 1e300;
  ps_status st = PS_OK;
  for (int sl : slot_c) {
    for (int64_t de : dense_c) {
      if (de == 0) continue;
      double ms = 0.0;
      for (int rep = 0; rep < 2 && st == PS_OK; ++rep) {
        const auto t0 = std::chrono::steady_clock::now();
        for (auto& q : qs) {
          QueryOut o;
          o.scores = dout;
          std::lock_guard<std::mutex> lk(ctx->mu);
          GraphVersion* gv = graph_acquire(g);
          st = engine_run(ctx, g, gv, {q}, {o}, sl, de);
          graph_release(g, gv);
          if (st != PS_OK) break;
        }
        if (rep == 1)
          ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / nsample;
      }
      if (st != PS_OK) break;
      if (ms < best) {
        best = ms;
        out->slots = sl;
        out->dense_edges = de;
        out->ms_per_query = ms;
      }
    }
  }
  (void)hipFree(dout);
  if (st != PS_OK) return st;
  g->tuned_slots = out->slots;
  g->tuned_dense = out->dense_edges;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%d %lld %.17g %d %lld %.6f\n", g->n, (long long)g->m, eps, out->slots, (long long)out->dense_edges,
              out->ms_per_query);
      fclose(f);
    }
  }
  return PS_OK;
}
