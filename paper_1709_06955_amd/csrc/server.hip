// Serving loop: a host thread that drains a request ring, applies queued edge
// updates between launches and runs the admitted queries together on the
// device.

#include <chrono>

#include "ps_internal.h"

namespace {

struct Request {
  ps_query q;
  ps_result* r;
  uint64_t ticket;
};

struct UpdateBatch {
  std::vector<int32_t> src, dst;
  std::vector<uint8_t> op;
};

}  // namespace

struct ps_server {
  ps_graph* g = nullptr;
  ps_server_cfg cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> ring;
  std::deque<UpdateBatch> updates;
  std::unordered_map<uint64_t, ps_status> finished;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread th;
};

namespace {

void serve(ps_server* s) {
  ps_ctx* ctx = s->g->ctx;
  (void)hipSetDevice(ctx->device);
  for (;;) {
    std::vector<Request> batch;
    std::vector<UpdateBatch> ups;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stopping || !s->ring.empty() || !s->updates.empty(); });
      if (s->ring.empty() && s->updates.empty() && s->stopping) return;
      while (!s->updates.empty()) {
        ups.push_back(std::move(s->updates.front()));
        s->updates.pop_front();
      }
      while (!s->ring.empty() && (int)batch.size() < s->cfg.max_inflight) {
        batch.push_back(s->ring.front());
        s->ring.pop_front();
      }
    }
    for (auto& u : ups) {
      std::lock_guard<std::mutex> lk(ctx->mu);
      (void)graph_apply_updates(s->g, (int64_t)u.src.size(), u.src.data(), u.dst.data(), u.op.data(), nullptr, nullptr);
    }
    if (batch.empty()) continue;
    ps_options opt;
    ps_options_default(&opt);
    opt.slots = s->cfg.slots;
    std::vector<ps_query> qv;
    std::vector<ps_result> rv;
    for (auto& rq : batch) {
      qv.push_back(rq.q);
      rv.push_back(*rq.r);
    }
    (void)ps_batch(s->g, (int32_t)qv.size(), qv.data(), &opt, rv.data());
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t i = 0; i < batch.size(); ++i) {
      *batch[i].r = rv[i];
      s->finished[batch[i].ticket] = (ps_status)rv[i].status;
    }
    s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" ps_status ps_server_start(ps_graph* g, const ps_server_cfg* cfg, ps_server** out) {
  if (!g || !out) return PS_ERR_INVALID_ARG;
  auto* s = new ps_server();
  s->g = g;
  if (cfg) s->cfg = *cfg;
  if (s->cfg.ring <= 0) s->cfg.ring = 1024;
  if (s->cfg.max_inflight <= 0) s->cfg.max_inflight = 64;
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
  s->ring.push_back(Request{*q, r, *ticket});
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
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return PS_ERR_STATE;
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
  delete s;
  return PS_OK;
}
