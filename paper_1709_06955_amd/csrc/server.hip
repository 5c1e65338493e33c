// Serving loop with continuous batching.
//
// A host thread owns the context's session while the server runs.  Each
// iteration it (1) applies queued edge updates (a new graph version; queries
// already admitted keep reading theirs), (2) admits waiting queries while
// query records, tree space and ring space allow -- their walks and trees are
// built and their probes join the ring behind the probes already pending, so
// they share the next level steps with the queries already running, (3)
// launches a few level steps, and (4) collects the queries whose last probe
// retired (read from the device's done ring one iteration late, so the GPU is
// never left without queued steps), finalises them and hands their results
// through pinned staging buffers to a completer thread that copies them to
// the caller's buffers and wakes ps_wait.

#include <algorithm>
#include <chrono>
#include <cstring>

#include "ps_internal.h"

namespace {

constexpr int kStepsPerIteration = 4;
constexpr double kUpdateIntervalMs = 10.0;

struct Request {
  ps_query q;
  ps_result* r;
  uint64_t ticket;
  uint64_t seq;  // submission order among requests and update batches
};

struct UpdateBatch {
  std::vector<int32_t> src, dst;
  std::vector<uint8_t> op;
  uint64_t seq;
  std::chrono::steady_clock::time_point t_sub;  // when ps_server_update queued it
};

struct Staging {
  void* host = nullptr;  // pinned
  size_t bytes = 0;
};

struct Completion {
  hipEvent_t ev;
  int staging;
  ps_result* r;
  int32_t k;      // 0: n scores
  int32_t count;
  uint64_t ticket;
  ps_status status;
};

}  // namespace

struct ps_server {
  ps_graph* g = nullptr;
  ps_server_cfg cfg{};
  ps_options defaults{};  // options of every served query (cfg.defaults copied)
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_comp;
  std::deque<Request> ring;
  std::deque<UpdateBatch> updates;
  std::unordered_map<uint64_t, ps_status> finished;
  uint64_t next_ticket = 1;
  uint64_t next_seq = 1;
  bool stopping = false;
  bool comp_stop = false;
  std::thread th, comp_th;
  // completer hand-off
  std::deque<Completion> comp_q;
  std::vector<Staging> staging;
  std::vector<int> staging_free;
  std::vector<hipEvent_t> ev_free;
  ps_status fatal = PS_OK;
  ps_server_stats stats{};  // under mu
  double upd_lat_sum = 0.0, upd_apply_sum = 0.0;
};

namespace {

struct Admitted {
  Request req;
  QueryRun run;
  uint64_t bound = 0;  // sum over its walks of (len - 1)
  bool built = false;  // tree built, probes queued
  uint64_t bytes = 0;  // device memory it holds once built
};

// Device memory of an admitted query: its FP64 accumulators and its tree
// region (a power of two of entries of about 40 bytes: key, five node
// fields, walk offset and walk list entry, ring entry).
uint64_t query_bytes(int32_t n, uint64_t bound) {
  uint64_t cap = 64;
  while (cap < 2 * bound) cap <<= 1;
  return 8ull * (uint64_t)n + 40ull * cap;
}

// Queries whose walk pass is queued and whose tree sizes are not back yet.
struct Pending {
  std::vector<int> recs;
  std::vector<QueryRun> runs;
  std::vector<Request> reqs;
  bool live = false;
};

void finish_ticket(ps_server* s, uint64_t ticket, ps_status st) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->finished[ticket] = st;
  s->cv_done.notify_all();
}

void completer(ps_server* s) {
  for (;;) {
    Completion c;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_comp.wait(lk, [&] { return s->comp_stop || !s->comp_q.empty(); });
      if (s->comp_q.empty()) return;
      c = s->comp_q.front();
      s->comp_q.pop_front();
    }
    ps_status st = c.status;
    if (hipEventSynchronize(c.ev) != hipSuccess) st = PS_ERR_DEVICE;
    if (st == PS_OK && c.staging >= 0) {
      const Staging& sg = s->staging[(size_t)c.staging];
      const char* host = (const char*)sg.host;
      std::memcpy(&c.r->flip_allowance, host, sizeof(double));
      if (c.k > 0) {
        std::memcpy(c.r->scores, host + sizeof(double), sizeof(double) * (size_t)c.k);
        std::memcpy(c.r->nodes, host + sizeof(double) * (1 + (size_t)c.k), sizeof(int32_t) * (size_t)c.k);
      } else {
        std::memcpy(c.r->scores, host + sizeof(double), sizeof(double) * (size_t)c.count);
      }
    }
    c.r->status = st;
    c.r->count = st == PS_OK ? c.count : 0;
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats.queries_done++;
    if (c.staging >= 0) s->staging_free.push_back(c.staging);
    s->ev_free.push_back(c.ev);
    s->finished[c.ticket] = st;
    s->cv_done.notify_all();
  }
}

// Takes a free pinned staging buffer (allocating up to a small pool, else
// waiting for the completer to return one).
int take_staging(ps_server* s, size_t bytes) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    for (size_t i = 0; i < s->staging_free.size(); ++i) {
      const int id = s->staging_free[i];
      if (s->staging[(size_t)id].bytes >= bytes) {
        s->staging_free.erase(s->staging_free.begin() + (long)i);
        return id;
      }
    }
    if (s->staging.size() < 16) {
      Staging sg;
      if (hipHostMalloc(&sg.host, bytes, 0) != hipSuccess) return -1;
      sg.bytes = bytes;
      s->staging.push_back(sg);
      return (int)s->staging.size() - 1;
    }
    if (!s->staging_free.empty()) {
      // grow the smallest free buffer
      const int id = s->staging_free.back();
      s->staging_free.pop_back();
      Staging& sg = s->staging[(size_t)id];
      (void)hipHostFree(sg.host);
      sg.host = nullptr;
      sg.bytes = 0;
      if (hipHostMalloc(&sg.host, bytes, 0) != hipSuccess) return -1;
      sg.bytes = bytes;
      return id;
    }
    s->cv_done.wait(lk);
  }
}

hipEvent_t take_event(ps_server* s) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->ev_free.empty()) {
    hipEvent_t e = s->ev_free.back();
    s->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
  return e;
}

// Finalises record r on the device and queues its copy-out.
ps_status complete_record(ps_server* s, int r, Admitted& a) {
  ps_ctx* ctx = s->g->ctx;
  Session* ss = ctx->sess;
  const int32_t n = ss->n;
  const int32_t k = a.run.k;
  // staging layout: allowance, scores, node ids
  const size_t bytes =
      sizeof(double) + (k > 0 ? (sizeof(double) + sizeof(int32_t)) * (size_t)k : sizeof(double) * (size_t)n);
  const int sid = take_staging(s, bytes);
  if (sid < 0) return PS_ERR_OOM;
  QueryOut out;
  char* host = (char*)s->staging[(size_t)sid].host;
  out.flip = (double*)host;
  out.scores = (double*)(host + sizeof(double));
  out.nodes = k > 0 ? (int32_t*)(host + sizeof(double) * (1 + (size_t)k)) : nullptr;
  PS_TRY(session_finish(ctx, s->g, r, a.run, out));
  Completion c;
  c.ev = take_event(s);
  PS_HIP(hipEventRecord(c.ev, ctx->stream));
  c.staging = sid;
  c.r = a.req.r;
  c.k = k;
  c.count = k > 0 ? k : n;
  c.ticket = a.req.ticket;
  c.status = PS_OK;
  std::lock_guard<std::mutex> lk(s->mu);
  s->comp_q.push_back(c);
  s->cv_comp.notify_one();
  return PS_OK;
}

ps_status serve_loop(ps_server* s) {
  ps_graph* g = s->g;
  ps_ctx* ctx = g->ctx;
  PS_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  std::unordered_map<int, Admitted> admitted;  // record -> query
  std::deque<int> waiting_build;               // records begun, trees not yet built
  Pending pend;                                // walk pass queued, tree sizes not back yet
  uint64_t committed = 0;                      // device bytes of the built queries
  Session* ss = ctx->sess;
  // done-ring snapshots, two in flight
  unsigned long long done_seen = 0;
  unsigned long long* snap[2] = {nullptr, nullptr};
  int32_t* snap_ring[2] = {nullptr, nullptr};
  hipEvent_t snap_ev[2];
  bool snap_live[2] = {false, false};
  for (int i = 0; i < 2; ++i) {
    PS_HIP(hipHostMalloc((void**)&snap[i], sizeof(unsigned long long) * C_COUNT, 0));
    PS_HIP(hipHostMalloc((void**)&snap_ring[i], sizeof(int32_t) * (size_t)ss->qmax, 0));
    PS_HIP(hipEventCreateWithFlags(&snap_ev[i], hipEventDisableTiming));
  }
  int snap_i = 0;
  // completions of earlier direct calls on this session are not ours
  session_clear_guard(ss, st);
  PS_HIP(hipMemcpyAsync(snap[0], ss->counters.p, sizeof(unsigned long long) * C_COUNT, hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  done_seen = snap[0][C_DONE];
  auto last_update = std::chrono::steady_clock::now();
  ps_status fatal = PS_OK;
  for (;;) {
    std::vector<Request> fresh;
    std::vector<UpdateBatch> ups;
    bool stopping;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto idle = [&] { return admitted.empty() && waiting_build.empty() && !pend.live; };
      if (idle() && s->ring.empty() && s->updates.empty())
        s->cv_work.wait(lk, [&] { return s->stopping || !s->ring.empty() || !s->updates.empty(); });
      stopping = s->stopping;
      // A query reads exactly the edge set left by the updates submitted
      // before it.  Updates older than the oldest waiting query may be
      // applied at any time (they are coalesced for kUpdateIntervalMs);
      // before that query is admitted they must be.  Admission stops at the
      // next update in submission order, which a later iteration applies.
      const int room = std::min(s->cfg.max_inflight - (int)admitted.size() - (int)waiting_build.size(),
                                (int)ss->free_recs.size());
      const bool admit = !s->ring.empty() && room > 0 && !pend.live;
      const uint64_t oldest = s->ring.empty() ? ~0ull : s->ring.front().seq;
      const double since = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - last_update).count();
      if (admit || since >= kUpdateIntervalMs || idle()) {
        while (!s->updates.empty() && s->updates.front().seq < oldest) {
          ups.push_back(std::move(s->updates.front()));
          s->updates.pop_front();
        }
      }
      while (admit && !s->ring.empty() && (int)fresh.size() < room &&
             (s->updates.empty() || s->ring.front().seq < s->updates.front().seq)) {
        fresh.push_back(s->ring.front());
        s->ring.pop_front();
      }
      if (stopping && s->ring.empty() && s->updates.empty() && idle() && fresh.empty()) break;
    }
    // (1) edge updates between level steps
    if (!ups.empty()) {
      for (auto& u : ups) {
        const auto t0 = std::chrono::steady_clock::now();
        (void)graph_apply_updates(g, (int64_t)u.src.size(), u.src.data(), u.dst.data(), u.op.data(), nullptr, nullptr);
        const auto t1 = std::chrono::steady_clock::now();
        const double apply = std::chrono::duration<double, std::milli>(t1 - t0).count();
        const double lat = std::chrono::duration<double, std::milli>(t1 - u.t_sub).count();
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.update_batches++;
        s->stats.updates += (int64_t)u.src.size();
        s->upd_lat_sum += lat;
        s->upd_apply_sum += apply;
        s->stats.update_latency_ms_max = std::max(s->stats.update_latency_ms_max, lat);
        s->stats.update_apply_ms_max = std::max(s->stats.update_apply_ms_max, apply);
      }
      last_update = std::chrono::steady_clock::now();
    }
    // (2) admission
    if (!fresh.empty()) {
      std::vector<QueryRun> runs;
      std::vector<Request> ok;
      for (auto& rq : fresh) {
        QueryRun qr;
        ps_options opt = s->defaults;
        if (rq.q.probe_mode) {
          opt.probe_mode = rq.q.probe_mode;
          if (rq.q.probe_mode == PS_PROBE_HYBRID) opt.hybrid_c0 = rq.q.hybrid_c0;
        }
        ps_status vs = make_query_run(g, rq.q.u, rq.q.k, rq.q.c, rq.q.eps, rq.q.delta, rq.q.seed, &opt, &qr);
        if (vs == PS_OK && (!rq.r->scores || (rq.q.k > 0 && !rq.r->nodes))) vs = PS_ERR_INVALID_ARG;
        if (vs == PS_OK && qr.merged) vs = PS_ERR_INVALID_ARG;  // merged probing runs through ps_single_source
        if (vs != PS_OK) {
          rq.r->status = vs;
          rq.r->count = 0;
          finish_ticket(s, rq.ticket, vs);
          continue;
        }
        runs.push_back(qr);
        ok.push_back(rq);
      }
      if (!runs.empty()) {
        // the walk pass is queued behind the steps already queued; its tree
        // sizes are picked up by a later iteration without waiting here
        GraphVersion* gv = graph_acquire(g);
        std::vector<int> recs;
        ps_status bs = session_begin(ctx, g, gv, runs, &recs);
        graph_release(g, gv);
        if (bs != PS_OK) {
          for (auto& rq : ok) {
            rq.r->status = bs;
            finish_ticket(s, rq.ticket, bs);
          }
        } else {
          pend.recs = std::move(recs);
          pend.runs = std::move(runs);
          pend.reqs = std::move(ok);
          pend.live = true;
        }
      }
    }
    // tree sizes of the queued walk pass: wait only when nothing else runs
    if (pend.live) {
      bool any_built = false;
      for (auto& kv : admitted) any_built |= kv.second.built;
      std::vector<uint64_t> bounds;
      bool ready = false;
      ps_status bs = session_bounds(ctx, pend.recs, &bounds, !any_built && waiting_build.empty(), &ready);
      if (bs != PS_OK) {
        fatal = bs;
        break;
      }
      if (ready) {
        for (size_t i = 0; i < pend.recs.size(); ++i) {
          Admitted a;
          a.req = pend.reqs[i];
          a.run = pend.runs[i];
          a.bound = bounds[i];
          admitted[pend.recs[i]] = a;
          waiting_build.push_back(pend.recs[i]);
        }
        pend = Pending();
      }
    }
    // build trees in arrival order while tree/ring space allows
    while (!waiting_build.empty()) {
      const int r = waiting_build.front();
      Admitted& a = admitted[r];
      a.bytes = query_bytes(g->n, a.bound);
      if (s->cfg.frontier_bytes > 0 && committed + a.bytes > (uint64_t)s->cfg.frontier_bytes) {
        bool any_built = false;
        for (auto& kv : admitted) any_built |= kv.second.built;
        if (any_built) break;  // the memory budget frees up as running queries finish
      }
      ps_status bs = session_build(ctx, {r}, {a.bound});
      if (bs == PS_ERR_BUSY) {
        bool any_built = false;
        for (auto& kv : admitted) any_built |= kv.second.built;
        if (any_built) break;  // space frees up as running queries finish
        bs = PS_ERR_OOM;       // the tree does not fit even in an empty session
        waiting_build.pop_front();
        session_abandon(ctx, g, r);
        a.req.r->status = bs;
        a.req.r->count = 0;
        finish_ticket(s, a.req.ticket, bs);
        admitted.erase(r);
        continue;
      }
      waiting_build.pop_front();
      if (bs != PS_OK) {
        fatal = bs;
        break;
      }
      a.built = true;
      committed += a.bytes;
      if (a.bound == 0) {  // no probe: the estimate is e_u
        committed -= a.bytes;
        ps_status cs = complete_record(s, r, a);
        if (cs != PS_OK) fatal = cs;
        admitted.erase(r);
      }
    }
    if (fatal != PS_OK) break;
    // (3) level steps for everything admitted
    bool have_probes = false;
    for (auto& kv : admitted)
      if (kv.second.built) have_probes = true;
    if (have_probes) {
      ps_status ss_ = session_steps(ctx, kStepsPerIteration, nullptr, nullptr);
      if (ss_ != PS_OK) {
        fatal = ss_;
        break;
      }
      PS_HIP(hipMemcpyAsync(snap[snap_i], ss->counters.p, sizeof(unsigned long long) * C_COUNT, hipMemcpyDeviceToHost,
                            st));
      PS_HIP(hipMemcpyAsync(snap_ring[snap_i], ss->done_ring.p, sizeof(int32_t) * (size_t)ss->qmax,
                            hipMemcpyDeviceToHost, st));
      PS_HIP(hipEventRecord(snap_ev[snap_i], st));
      snap_live[snap_i] = true;
    }
    // (4) completions seen by the previous iteration's snapshot (or this one
    // when nothing else is queued)
    const int prev = snap_i ^ 1;
    int look = prev;
    if (!snap_live[prev] && snap_live[snap_i]) look = snap_i;
    if (snap_live[look]) {
      PS_HIP(hipEventSynchronize(snap_ev[look]));
      snap_live[look] = false;
      if (snap[look][C_OVERFLOW]) {  // a capacity guard dropped frontier entries
        report_overflow(ss, reinterpret_cast<const uint64_t*>(snap[look]));
        fatal = PS_ERR_OOM;
        break;
      }
      const unsigned long long done = snap[look][C_DONE];
      for (; done_seen < done; ++done_seen) {
        const int r = snap_ring[look][done_seen % (unsigned long long)ss->qmax];
        auto it = admitted.find(r);
        if (it == admitted.end()) continue;
        committed -= it->second.bytes;
        ps_status cs = complete_record(s, r, it->second);
        if (cs != PS_OK) fatal = cs;
        admitted.erase(it);
      }
    }
    if (fatal != PS_OK) break;
    snap_i ^= 1;
  }
  (void)hipStreamSynchronize(st);
  for (int i = 0; i < 2; ++i) {
    (void)hipHostFree(snap[i]);
    (void)hipHostFree(snap_ring[i]);
    (void)hipEventDestroy(snap_ev[i]);
  }
  if (fatal != PS_OK) {
    // fail everything still queued or running
    for (auto& kv : admitted) {
      kv.second.req.r->status = fatal;
      finish_ticket(s, kv.second.req.ticket, fatal);
    }
    for (auto& rq : pend.reqs) {
      rq.r->status = fatal;
      finish_ticket(s, rq.ticket, fatal);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& rq : s->ring) {
      rq.r->status = fatal;
      s->finished[rq.ticket] = fatal;
    }
    s->ring.clear();
    s->cv_done.notify_all();
  }
  return fatal;
}

void serve(ps_server* s) {
  ps_ctx* ctx = s->g->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  s->fatal = serve_loop(s);
  {
    std::lock_guard<std::mutex> lk2(s->mu);
    s->comp_stop = true;
    s->cv_comp.notify_all();
  }
}

}  // namespace

extern "C" ps_status ps_server_start(ps_graph* g, const ps_server_cfg* cfg, ps_server** out) {
  if (!g || !out) return PS_ERR_INVALID_ARG;
  *out = nullptr;
  ps_ctx* ctx = g->ctx;
  auto* s = new ps_server();
  s->g = g;
  if (cfg) s->cfg = *cfg;
  ps_options_default(&s->defaults);
  if (s->cfg.defaults) {
    if (s->cfg.defaults->walk_begin != 0 || s->cfg.defaults->walk_end >= 0 ||
        s->cfg.defaults->probe_mode == PS_PROBE_MERGED) {
      delete s;
      return PS_ERR_INVALID_ARG;
    }
    s->defaults = *s->cfg.defaults;
  }
  s->cfg.defaults = nullptr;  // the caller's struct is not kept
  if (s->cfg.ring <= 0) s->cfg.ring = 1024;
  if (s->cfg.max_inflight <= 0) s->cfg.max_inflight = 64;
  // tree pool / ring sized for max_inflight queries of up to ~1M tree nodes
  const uint64_t per_q = 1ull << 21;
  if (s->cfg.frontier_bytes > 0) {
    // device memory of one admitted query: its FP64 accumulators and its
    // share of the tree pool (key, five int32 node fields, walk offset and
    // walk list per entry) and of the ring; the budget caps how many are
    // admitted at once (at least one), the others wait in the request ring
    const uint64_t each = query_bytes(g->n, 0);
    const uint64_t fit = std::max<uint64_t>((uint64_t)s->cfg.frontier_bytes / each, 1);
    s->cfg.max_inflight = (int32_t)std::min<uint64_t>((uint64_t)s->cfg.max_inflight, fit);
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ps_status st = PS_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) st = PS_ERR_DEVICE;
    const int P = session_slots_for(g->n, s->cfg.slots ? s->cfg.slots : g->tuned_slots);
    const uint64_t pool = std::max<uint64_t>((uint64_t)s->cfg.max_inflight * per_q, 1ull << 22);
    if (st == PS_OK)
      st = session_ensure(ctx, g->n, std::max<uint64_t>(g->cur->out_store->cap, 1), P, s->cfg.max_inflight, pool,
                          pool / 2);
    if (st == PS_OK) st = session_set_pull(ctx, pull_threshold(g->m, g->tuned_dense));
    if (st != PS_OK) {
      delete s;
      return st;
    }
  }
  s->comp_th = std::thread(completer, s);
  s->th = std::thread(serve, s);
  *out = s;
  return PS_OK;
}

extern "C" ps_status ps_submit(ps_server* s, const ps_query* q, ps_result* r, uint64_t* ticket) {
  if (!s || !q || !r || !ticket) return PS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return PS_ERR_STATE;
  if ((int)s->ring.size() >= s->cfg.ring) return PS_ERR_BUSY;
  *ticket = s->next_ticket++;
  s->ring.push_back(Request{*q, r, *ticket, s->next_seq++});
  s->cv_work.notify_one();
  return PS_OK;
}

extern "C" ps_status ps_wait(ps_server* s, uint64_t ticket, int64_t timeout_us) {
  if (!s) return PS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] { return s->finished.count(ticket) != 0; };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return PS_ERR_TIMEOUT;
  }
  ps_status st = s->finished[ticket];
  s->finished.erase(ticket);
  return st;
}

extern "C" ps_status ps_server_update(ps_server* s, int64_t k, const int32_t* src, const int32_t* dst,
                                      const uint8_t* op) {
  if (!s || k < 0 || (k > 0 && (!src || !dst || !op))) return PS_ERR_INVALID_ARG;
  UpdateBatch b;
  b.src.assign(src, src + k);
  b.dst.assign(dst, dst + k);
  b.op.assign(op, op + k);
  b.t_sub = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return PS_ERR_STATE;
  b.seq = s->next_seq++;
  s->updates.push_back(std::move(b));
  s->cv_work.notify_one();
  return PS_OK;
}

extern "C" ps_status ps_server_stop(ps_server* s) {
  if (!s) return PS_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  if (s->comp_th.joinable()) s->comp_th.join();
  for (auto& sg : s->staging)
    if (sg.host) (void)hipHostFree(sg.host);
  for (hipEvent_t e : s->ev_free) (void)hipEventDestroy(e);
  const ps_status st = s->fatal;
  delete s;
  return st;
}

extern "C" ps_status ps_server_get_stats(ps_server* s, ps_server_stats* out) {
  if (!s || !out) return PS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  if (s->stats.update_batches) {
    out->update_latency_ms_mean = s->upd_lat_sum / (double)s->stats.update_batches;
    out->update_apply_ms_mean = s->upd_apply_sum / (double)s->stats.update_batches;
  }
  return PS_OK;
}
