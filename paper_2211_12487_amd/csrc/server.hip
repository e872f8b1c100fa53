// Serving layer of the TT-ICE library: many independent streams, each a
// resident TT-ICE state, updated by a pool of worker threads that each own a
// HIP stream (default priority).  Host code only; the device work is the
// library's own ttice_update.  See include/ttice.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ttice.h"

namespace {

struct Request {
  int64_t ticket;
  const void* batch;
  int64_t n;
  int32_t dtype;
};

struct Stream {
  ttice_state* st = nullptr;
  int64_t reserved = 0;
  int64_t max_batch = 0;
  bool busy = false;
  bool queued = false;  // in the ready list
  std::deque<Request> q;
};

struct Ticket {
  bool done = false;
  int32_t status = TTICE_OK;
  ttice_update_info info;
};

// Projected device footprint of a stream for increments of up to N tensors
// (an upper estimate of what ttice_update allocates): two level buffers, the
// residual and the column partials (each at most N * prod(dims) doubles), the
// Gram matrix and its partial products and eigen workspace (m <= 4096), the
// cores at their rank bounds with capacity doubling, and the fixed split-K
// workspace.
int64_t projected_bytes(int32_t d, const int64_t* dims, int64_t N) {
  int64_t P = 1;
  for (int i = 0; i < d; ++i) P *= dims[i];
  double left = 1.0, bytes = 4.0 * 8.0 * (double)N * (double)P;
  double rprev = 1.0, mmax = 1.0, cores = 0.0;
  for (int i = 0; i < d; ++i) {
    left *= (double)dims[i];
    const double right = (double)P / left;
    const double rows = rprev * (double)dims[i];
    const double r = std::min(left, std::max(right, 1.0));
    cores += rows * r;
    mmax = std::max(mmax, std::min(rows, (double)N * right));
    rprev = r;
  }
  mmax = std::min(mmax, 4096.0);
  bytes += 16.0 * 8.0 * mmax * mmax + 2.0 * 8.0 * cores + 8.0 * (1 << 20);
  return (int64_t)std::min(bytes, 9.0e18);
}

}  // namespace

struct ttice_server {
  int64_t budget = 0;
  int64_t reserved = 0;
  int64_t next_ticket = 1;
  int32_t next_stream = 0;
  int64_t pending = 0;
  bool stop = false;
  std::mutex mu;
  std::condition_variable work_cv;  // workers: a stream became ready, or stop
  std::condition_variable done_cv;  // waiters: a ticket completed
  std::unordered_map<int32_t, std::unique_ptr<Stream>> streams;
  std::unordered_map<int64_t, Ticket> tickets;
  std::deque<int32_t> ready;  // streams with queued increments, oldest first
  std::vector<std::thread> workers;
  std::vector<hipStream_t> hip_streams;

  void worker(int w) {
    hipStream_t hs = hip_streams[w];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      work_cv.wait(lk, [&] { return stop || !ready.empty(); });
      if (stop) return;
      const int32_t sid = ready.front();
      ready.pop_front();
      Stream& s = *streams.at(sid);
      s.queued = false;
      s.busy = true;
      const Request rq = s.q.front();
      s.q.pop_front();
      lk.unlock();
      ttice_update_info info;
      std::memset(&info, 0, sizeof(info));
      int status = ttice_set_option(s.st, TTICE_OPT_STREAM, &hs);
      if (status == TTICE_OK) status = ttice_update(s.st, rq.batch, rq.n, rq.dtype, &info);
      lk.lock();
      Ticket& t = tickets[rq.ticket];
      t.done = true;
      t.status = status;
      t.info = info;
      --pending;
      s.busy = false;
      if (!s.q.empty()) {
        s.queued = true;
        ready.push_back(sid);
        work_cv.notify_one();
      }
      done_cv.notify_all();
    }
  }
};

#pragma GCC visibility push(default)
extern "C" {

int ttice_server_create(int32_t workers, int64_t budget_bytes, ttice_server** out) {
  if (!out) return TTICE_EINVAL;
  *out = nullptr;
  if (workers < 1 || workers > 64 || budget_bytes <= 0) return TTICE_EINVAL;
  ttice_server* srv = new (std::nothrow) ttice_server();
  if (!srv) return TTICE_ENOMEM;
  srv->budget = budget_bytes;
  for (int w = 0; w < workers; ++w) {
    hipStream_t s = nullptr;
    // non-blocking: a worker's stream never waits for work on the null stream
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      for (hipStream_t x : srv->hip_streams) (void)hipStreamDestroy(x);
      delete srv;
      return TTICE_EDEVICE;
    }
    srv->hip_streams.push_back(s);
  }
  try {
    for (int w = 0; w < workers; ++w) srv->workers.emplace_back(&ttice_server::worker, srv, w);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->stop = true;
    }
    srv->work_cv.notify_all();
    for (auto& t : srv->workers) t.join();
    for (hipStream_t x : srv->hip_streams) (void)hipStreamDestroy(x);
    delete srv;
    return TTICE_ENOMEM;
  }
  *out = srv;
  return TTICE_OK;
}

int ttice_server_add_stream(ttice_server* srv, int32_t d, const int64_t* dims, double eps, int32_t prec,
                            int32_t algo, int64_t max_batch, int32_t* stream_id) {
  if (!srv) return TTICE_ESTATE;
  if (!stream_id || max_batch < 1 || !dims || d < 1 || d > TTICE_MAX_D) return TTICE_EINVAL;
  *stream_id = -1;
  const int64_t need = projected_bytes(d, dims, max_batch);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return TTICE_ESTATE;
    if (need > srv->budget - srv->reserved) return TTICE_ENOMEM;
    srv->reserved += need;  // held while the state is built
  }
  auto release = [&] {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->reserved -= need;
  };
  ttice_state* st = nullptr;
  int rc = ttice_create(d, dims, eps, &st);
  if (rc == TTICE_OK) rc = ttice_set_option(st, TTICE_OPT_PREC, &prec);
  if (rc == TTICE_OK) rc = ttice_set_option(st, TTICE_OPT_ALGO, &algo);
  if (rc == TTICE_OK) rc = ttice_reserve(st, max_batch);  // resident workspace: no allocation per update
  if (rc != TTICE_OK) {
    ttice_destroy(st);
    release();
    return rc;
  }
  std::unique_ptr<Stream> s(new (std::nothrow) Stream());
  if (!s) {
    ttice_destroy(st);
    release();
    return TTICE_ENOMEM;
  }
  s->st = st;
  s->reserved = need;
  s->max_batch = max_batch;
  std::lock_guard<std::mutex> lk(srv->mu);
  const int32_t id = srv->next_stream++;
  srv->streams[id] = std::move(s);
  *stream_id = id;
  return TTICE_OK;
}

int ttice_server_submit(ttice_server* srv, int32_t stream_id, const void* batch, int64_t n, int32_t dtype,
                        int64_t* ticket) {
  if (!srv) return TTICE_ESTATE;
  if (!ticket || n < 0 || (n > 0 && !batch) || (dtype != TTICE_F32 && dtype != TTICE_F64)) return TTICE_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return TTICE_ESTATE;
  auto it = srv->streams.find(stream_id);
  if (it == srv->streams.end() || n > it->second->max_batch) return TTICE_EINVAL;
  Stream& s = *it->second;
  const int64_t id = srv->next_ticket++;
  srv->tickets[id] = Ticket();
  s.q.push_back(Request{id, batch, n, dtype});
  ++srv->pending;
  if (!s.busy && !s.queued) {
    s.queued = true;
    srv->ready.push_back(stream_id);
    srv->work_cv.notify_one();
  }
  *ticket = id;
  return TTICE_OK;
}

int ttice_server_poll(ttice_server* srv, int64_t ticket, int32_t* done, int32_t* status,
                      ttice_update_info* info) {
  if (!srv) return TTICE_ESTATE;
  if (!done) return TTICE_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return TTICE_EINVAL;
  *done = it->second.done ? 1 : 0;
  if (!it->second.done) return TTICE_OK;
  if (status) *status = it->second.status;
  if (info) *info = it->second.info;
  srv->tickets.erase(it);
  return TTICE_OK;
}

int ttice_server_wait(ttice_server* srv, int64_t ticket, int32_t* status, ttice_update_info* info) {
  if (!srv) return TTICE_ESTATE;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return TTICE_EINVAL;
  srv->done_cv.wait(lk, [&] {
    auto t = srv->tickets.find(ticket);
    return t == srv->tickets.end() || t->second.done;
  });
  it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return TTICE_EINVAL;  // reported to another caller meanwhile
  if (status) *status = it->second.status;
  if (info) *info = it->second.info;
  srv->tickets.erase(it);
  return TTICE_OK;
}

int ttice_server_stream_state(ttice_server* srv, int32_t stream_id, ttice_state** st) {
  if (!srv) return TTICE_ESTATE;
  if (!st) return TTICE_EINVAL;
  *st = nullptr;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->streams.find(stream_id);
  if (it == srv->streams.end()) return TTICE_EINVAL;
  if (it->second->busy || !it->second->q.empty()) return TTICE_ESTATE;
  *st = it->second->st;
  return TTICE_OK;
}

int ttice_server_remove_stream(ttice_server* srv, int32_t stream_id) {
  if (!srv) return TTICE_ESTATE;
  std::unique_ptr<Stream> s;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->streams.find(stream_id);
    if (it == srv->streams.end()) return TTICE_EINVAL;
    if (it->second->busy || !it->second->q.empty()) return TTICE_ESTATE;
    s = std::move(it->second);
    srv->streams.erase(it);
    srv->reserved -= s->reserved;
  }
  ttice_destroy(s->st);
  return TTICE_OK;
}

int ttice_server_stats(ttice_server* srv, int64_t* reserved_bytes, int64_t* budget_bytes, int64_t* pending) {
  if (!srv) return TTICE_ESTATE;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (reserved_bytes) *reserved_bytes = srv->reserved;
  if (budget_bytes) *budget_bytes = srv->budget;
  if (pending) *pending = srv->pending;
  return TTICE_OK;
}

void ttice_server_destroy(ttice_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->work_cv.notify_all();
  for (auto& t : srv->workers) t.join();  // running updates finish first
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    for (auto& kv : srv->streams)
      for (const Request& rq : kv.second->q) {
        Ticket& t = srv->tickets[rq.ticket];
        t.done = true;
        t.status = TTICE_ESTATE;
      }
  }
  srv->done_cv.notify_all();
  for (auto& kv : srv->streams) ttice_destroy(kv.second->st);
  for (hipStream_t x : srv->hip_streams) (void)hipStreamDestroy(x);
  delete srv;
}

}  // extern "C"
#pragma GCC visibility pop
