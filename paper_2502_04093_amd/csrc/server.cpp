// Serving loop: compressed streams and partial reconstructions stay resident
// on the device; retrieval and refinement requests (Alg. 1, Alg. 2) arrive
// from any host thread, are admitted by a device-memory budget as memory
// frees up, and run in continuous batches on one worker thread, every batch
// one ipc_serve_batch call (requests on 3-D streams share the level
// launches).  Written against the public C ABI only.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/ipcomp.h"

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Pending {
  uint64_t ticket;
  const ipc_stream *stream;
  ipc_state *state;
  ipc_target target;
  int refine;
  uint64_t need;    // budget charged while in flight
  uint64_t field;   // field bytes of the stream (kept by a new state)
  double t_submit;
};

struct Done {
  ipc_state *state = nullptr;
  bool fresh = false;  // a new state made by this request
  ipc_info info{};
  int status = IPC_OK;
  double latency_ms = 0;
};

// transient device memory of a request besides its output field: the two
// coarse-grid buffers (1/8 and 1/64 of the field) and small tables
uint64_t transient_bytes(uint64_t field) { return field / 8 + field / 64 + (uint64_t(1) << 20); }

}  // namespace

struct ipc_server {
  ipc_ctx *ctx = nullptr;
  uint64_t budget = 0, used = 0, peak = 0;
  uint32_t max_batch = 64;
  std::mutex mu;                     // queue, results, accounting
  std::mutex ctx_mu;                 // the context: held by the worker around each batch
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, Done> done;
  std::deque<ipc_state *> to_free;
  std::unordered_map<const ipc_state *, uint64_t> charged;  // live states' field bytes
  std::unordered_set<const ipc_state *> busy;               // states being refined
  uint64_t next_ticket = 1;
  uint64_t submitted = 0;            // submissions so far (wakes a worker waiting for room)
  uint64_t batches = 0, served = 0;
  bool stop = false;
  std::thread worker;

  void run();
};

void ipc_server::run() {
  for (;;) {
    std::vector<Pending> batch;
    std::vector<ipc_state *> frees;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || !to_free.empty(); });
      frees.assign(to_free.begin(), to_free.end());
      to_free.clear();
    }
    if (!frees.empty()) {
      {
        std::lock_guard<std::mutex> c(ctx_mu);
        for (ipc_state *st : frees) ipc_state_free(st);
      }
      std::lock_guard<std::mutex> lk(mu);
      for (ipc_state *st : frees) {
        auto it = charged.find(st);
        if (it != charged.end()) {
          used -= it->second;
          charged.erase(it);
        }
      }
    }
    {
      // admission: requests in arrival order, each one that fits the budget
      // (a large request does not hold back smaller ones behind it); a state
      // takes part in at most one request per batch
      std::lock_guard<std::mutex> lk(mu);
      std::unordered_set<const ipc_state *> in_batch;
      for (auto it = queue.begin(); it != queue.end() && batch.size() < max_batch;) {
        const bool blocked = it->refine && (busy.count(it->state) || in_batch.count(it->state));
        if (!blocked && used + it->need <= budget) {
          used += it->need;
          peak = used > peak ? used : peak;
          if (it->refine) {
            busy.insert(it->state);
            in_batch.insert(it->state);
          }
          batch.push_back(*it);
          it = queue.erase(it);
        } else {
          ++it;
        }
      }
      if (batch.empty()) {
        if (stop && queue.empty() && to_free.empty()) return;
        if (!to_free.empty()) continue;
      }
    }
    if (batch.empty()) {
      // nothing fits: wait for a release; once stopping, the requests that
      // cannot be admitted fail with IPC_ENOMEM
      std::unique_lock<std::mutex> lk(mu);
      const uint64_t seen = submitted;
      cv_work.wait(lk, [&] { return !to_free.empty() || stop || submitted != seen; });
      if (submitted != seen && !stop) continue;
      if (to_free.empty() && stop) {
        for (const Pending &p : queue) {
          Done d;
          d.status = IPC_ENOMEM;
          d.state = p.refine ? p.state : nullptr;
          done[p.ticket] = d;
        }
        queue.clear();
        lk.unlock();
        cv_done.notify_all();
        return;
      }
      continue;
    }
    std::vector<ipc_request> req(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
      req[i].stream = batch[i].stream;
      req[i].state = batch[i].refine ? batch[i].state : nullptr;
      req[i].target = batch[i].target;
      req[i].refine = batch[i].refine;
      req[i].status = IPC_OK;
    }
    ipc_status st;
    {
      std::lock_guard<std::mutex> c(ctx_mu);
      st = ipc_serve_batch(ctx, uint32_t(req.size()), req.data());
    }
    const double t_end = now_ms();
    {
      std::lock_guard<std::mutex> lk(mu);
      for (size_t i = 0; i < batch.size(); ++i) {
        const Pending &p = batch[i];
        Done d;
        d.status = st != IPC_OK ? int(st) : req[i].status;
        d.info = req[i].info;
        d.latency_ms = t_end - p.t_submit;
        if (p.refine) {
          busy.erase(p.state);
          used -= p.need;
          d.state = p.state;
        } else {
          used -= p.need;
          if (d.status == IPC_OK && req[i].state) {
            d.state = req[i].state;
            d.fresh = true;
            charged[d.state] = p.field;
            used += p.field;
          }
        }
        done[p.ticket] = d;
      }
      ++batches;
      served += batch.size();
    }
    cv_done.notify_all();
  }
}

extern "C" {

ipc_status ipc_server_create(ipc_ctx *ctx, uint64_t budget_bytes, uint32_t max_batch,
                             ipc_server **out) {
  if (!out) return IPC_EINVAL;
  *out = nullptr;
  if (!ctx || budget_bytes == 0) return IPC_EINVAL;
  ipc_server *s = new (std::nothrow) ipc_server();
  if (!s) return IPC_ENOMEM;
  s->ctx = ctx;
  s->budget = budget_bytes;
  s->max_batch = max_batch ? max_batch : 64;
  try {
    s->worker = std::thread([s] { s->run(); });
  } catch (...) {
    delete s;
    return IPC_ENOMEM;
  }
  *out = s;
  return IPC_OK;
}

ipc_status ipc_server_submit(ipc_server *srv, const ipc_stream *stream, ipc_state *refine_state,
                             ipc_target target, uint64_t *ticket) {
  if (!srv || !ticket || (!stream && !refine_state)) return IPC_EINVAL;
  const int base = target.kind & ~IPC_TARGET_LEVEL_GROUPS;
  if (!(base == IPC_TARGET_EB || base == IPC_TARGET_BITRATE) || !(target.value > 0))
    return IPC_EINVAL;
  Pending p{};
  p.refine = refine_state != nullptr;
  p.state = refine_state;
  p.stream = stream;
  p.target = target;
  uint64_t field = 0;
  const ipc_status q = p.refine ? ipc_state_field_bytes(refine_state, &field)
                                : ipc_stream_field_bytes(stream, &field);
  if (q != IPC_OK) return q;
  p.field = field;
  p.need = (p.refine ? 0 : field) + transient_bytes(field);
  if (p.need > srv->budget) return IPC_ENOMEM;
  p.t_submit = now_ms();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return IPC_ESTATE;
    p.ticket = srv->next_ticket++;
    srv->queue.push_back(p);
    ++srv->submitted;
    *ticket = p.ticket;
  }
  srv->cv_work.notify_one();
  return IPC_OK;
}

ipc_status ipc_server_wait(ipc_server *srv, uint64_t ticket, int64_t timeout_ms, ipc_state **state,
                           ipc_info *info, double *latency_ms) {
  if (!srv) return IPC_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto ready = [&] { return srv->done.count(ticket) != 0; };
  if (timeout_ms < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return IPC_ESTATE;  // not finished yet
  }
  Done d = srv->done[ticket];
  srv->done.erase(ticket);
  if (state) *state = d.state;
  if (info) *info = d.info;
  if (latency_ms) *latency_ms = d.latency_ms;
  return ipc_status(d.status);
}

ipc_status ipc_server_release(ipc_server *srv, ipc_state *st) {
  if (!srv || !st) return IPC_EINVAL;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->to_free.push_back(st);
  }
  srv->cv_work.notify_one();
  return IPC_OK;
}

ipc_status ipc_server_lock(ipc_server *srv) {
  if (!srv) return IPC_EINVAL;
  srv->ctx_mu.lock();
  return IPC_OK;
}

ipc_status ipc_server_unlock(ipc_server *srv) {
  if (!srv) return IPC_EINVAL;
  srv->ctx_mu.unlock();
  return IPC_OK;
}

ipc_status ipc_server_stats(ipc_server *srv, uint64_t *used, uint64_t *peak, uint64_t *batches,
                            uint64_t *served) {
  if (!srv) return IPC_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (used) *used = srv->used;
  if (peak) *peak = srv->peak;
  if (batches) *batches = srv->batches;
  if (served) *served = srv->served;
  return IPC_OK;
}

void ipc_server_destroy(ipc_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  // results never collected: their new states are freed with the server
  for (auto &kv : srv->done)
    if (kv.second.fresh && kv.second.state) ipc_state_free(kv.second.state);
  delete srv;
}

}  // extern "C"
