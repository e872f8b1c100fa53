// Serving layer of the TT-ICE library: many independent streams, each a
// resident TT-ICE state, updated by a pool of worker threads that each own a
// HIP stream (default priority).  See include/ttice.h for the contract.
//
// Scheduling.  A free worker first takes an update that is ready to
// continue (below); otherwise it takes the stream that has waited longest
// and, when that stream runs Algorithm 1, up to kGroupMax - 1 more waiting
// Algorithm 1 streams.  It prepares each of their updates up to the level-1
// projection (eq:first_resid: C = U_1^T Z, ||z||^2 and the residual
// energies, the one pass over every tensor of the increment) and makes one
// launch per group of equal launch shape over all of them (ProjGroup), on
// its own HIP stream after each batch's producer event.  An event recorded
// after that launch orders the rest of every member's update, which any
// worker then continues on its own stream.  The grouped kernel computes for
// each stream exactly what that stream's own launch computes (the same
// blocks, the same fixed-order sums), so a stream's cores are bit-identical
// whether it was served alone or in a mix.
//
// Admission.  Each stream reserves a projected device footprint (level
// buffers, residual, Gram and eigen workspace, every core at its rank bound
// with capacity doubling, the last core included at the stream's tensor
// limit).  A stream that does not fit the remaining budget waits, in order
// of arrival, and is admitted when removed streams free enough of it;
// increments submitted meanwhile queue and run once it is admitted.
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

#include "serve.h"

using ttice::kGroupMax;
using ttice::ProjDesc;
using ttice::ProjGroup;

namespace {

struct Request {
  int64_t ticket = 0;
  const void* batch = nullptr;
  int64_t n = 0;
  int32_t dtype = TTICE_F32;
  hipEvent_t ready = nullptr;  // recorded on the producer's stream at submission (n > 0)
};

struct Stream {
  ttice_state* st = nullptr;  // null until admitted
  int32_t d = 0;
  int64_t dims[TTICE_MAX_D] = {};
  double eps = 0.0;
  int32_t prec = 0, algo = 0;
  int64_t need = 0;  // projected footprint, held in the budget once admitted
  int64_t max_batch = 0, max_tensors = 0;
  int64_t accepted = 0;       // tensors submitted so far
  int admit_rc = TTICE_OK;    // a failed admission's status
  bool busy = false;          // an update of this stream is being prepared or run
  bool queued = false;        // in the ready list
  std::deque<Request> q;
};

struct Ticket {
  bool done = false;
  int32_t status = TTICE_OK;
  ttice_update_info info;
};

// An event recorded after a grouped launch; the last member that waited on
// it releases it.
struct GroupEvent {
  hipEvent_t e = nullptr;
  ~GroupEvent() {
    if (e) (void)hipEventDestroy(e);
  }
};

// One stream's update: plain, or continuing after its grouped level-1 launch
struct Job {
  int32_t sid = -1;
  Stream* s = nullptr;
  Request rq;
  std::shared_ptr<GroupEvent> ev;
};

// Projected device footprint of a stream (an upper estimate of what
// ttice_update allocates) for increments of up to N tensors and at most T
// tensors in all: two level buffers, the residual and the column partials
// (each at most N * prod(dims) doubles), the Gram matrix and its partial
// products and eigen workspace (m <= 4096), every core at its rank bounds
// (its capacity never grows past them, serve_limit) plus the projection's
// row over-read, the last core (T x r_d) and the fixed split-K workspace.
int64_t projected_bytes(int32_t d, const int64_t* dims, int64_t N, int64_t T) {
  int64_t rb[TTICE_MAX_D + 1];
  ttice::serve_rank_bounds(d, dims, T, rb);
  double P = 1.0;
  for (int i = 0; i < d; ++i) P *= (double)dims[i];
  double right = P, mmax = 1.0, cores = 0.0;
  for (int i = 0; i < d; ++i) {
    right /= (double)dims[i];  // n_{i+1} ... n_d
    const double rows = (double)rb[i] * (double)dims[i];
    cores += rows * (double)rb[i + 1] + ttice::kProjTail;
    mmax = std::max(mmax, std::min(rows, (double)N * right));
  }
  cores += (double)T * (double)rb[d] + ttice::kProjTail;  // last core: stored tensors x r_d
  mmax = std::min(mmax, 4096.0);
  const double bytes = 4.0 * 8.0 * (double)N * P + 16.0 * 8.0 * mmax * mmax + 8.0 * cores + 8.0 * (double)ttice::kSplitKDoubles;
  return (int64_t)std::min(bytes, 9.0e18);
}

// A new state with the stream's options and its workspace for max_batch
int build_state(const Stream& s, ttice_state** out) {
  *out = nullptr;
  ttice_state* st = nullptr;
  int rc = ttice_create(s.d, s.dims, s.eps, &st);
  if (rc == TTICE_OK) rc = ttice_set_option(st, TTICE_OPT_PREC, &s.prec);
  if (rc == TTICE_OK) rc = ttice_set_option(st, TTICE_OPT_ALGO, &s.algo);
  if (rc == TTICE_OK) {
    ttice::serve_mark(st);
    ttice::serve_limit(st, s.max_tensors);
    rc = ttice_reserve(st, s.max_batch);  // resident workspace: no allocation per update
  }
  if (rc != TTICE_OK) {
    ttice_destroy(st);
    return rc;
  }
  *out = st;
  return TTICE_OK;
}

}  // namespace

struct ttice_server {
  int64_t budget = 0;
  int64_t reserved = 0;
  int64_t next_ticket = 1;
  int32_t next_stream = 0;
  int64_t pending = 0;
  int64_t groups = 0, grouped = 0;
  int device = 0;
  bool stop = false;
  std::mutex mu;
  std::condition_variable work_cv;  // workers: a job or a stream became ready, or stop
  std::condition_variable done_cv;  // waiters: a ticket completed
  std::unordered_map<int32_t, std::unique_ptr<Stream>> streams;
  std::unordered_map<int64_t, Ticket> tickets;
  std::deque<int32_t> ready;    // admitted streams with queued increments, oldest first
  std::deque<int32_t> waiting;  // streams waiting for admission, in order of arrival
  std::deque<Job> jobs;         // prepared updates, taken before new streams
  std::vector<std::thread> workers;
  std::vector<hipStream_t> hip_streams;

  // Algorithm 1 streams whose first core is narrow enough for the fused
  // level-1 projection (read while the stream is idle: no update changes it)
  static bool groupable(const Stream& s) {
    if (s.algo != TTICE_ALG_PLAIN || s.d < 2 || !s.st) return false;
    int64_t rk[TTICE_MAX_D + 2];
    return ttice_ranks(s.st, rk, nullptr) == TTICE_OK && rk[1] <= 64;
  }

  // Takes the stream's next request (lock held)
  Job take(int32_t sid) {
    Stream& s = *streams.at(sid);
    s.queued = false;
    s.busy = true;
    Job j;
    j.sid = sid;
    j.s = &s;
    j.rq = s.q.front();
    s.q.pop_front();
    return j;
  }

  // Runs a job's update on the worker's stream (no lock held)
  static int run(Job& j, hipStream_t hs, ttice_update_info* info) {
    std::memset(info, 0, sizeof(*info));
    int status = ttice_set_option(j.s->st, TTICE_OPT_STREAM, &hs);
    if (status == TTICE_OK) {
      hipEvent_t wait = j.ev ? j.ev->e : j.rq.ready;
      if (wait && hipStreamWaitEvent(hs, wait, 0) != hipSuccess) status = TTICE_EDEVICE;
    }
    if (status == TTICE_OK)
      status = j.ev ? ttice::serve_update_after(j.s->st, j.rq.batch, j.rq.n, j.rq.dtype, info)
                    : ttice_update(j.s->st, j.rq.batch, j.rq.n, j.rq.dtype, info);
    if (j.rq.ready) (void)hipEventDestroy(j.rq.ready);
    j.rq.ready = nullptr;
    j.ev.reset();
    return status;
  }

  // Reports a finished job (lock held)
  void complete(const Job& j, int status, const ttice_update_info& info) {
    Ticket& t = tickets[j.rq.ticket];
    t.done = true;
    t.status = status;
    t.info = info;
    --pending;
    Stream& s = *j.s;
    s.busy = false;
    if (!s.q.empty()) {
      s.queued = true;
      ready.push_back(j.sid);
      work_cv.notify_one();
    }
    done_cv.notify_all();
  }

  // The level-1 launches of a set of taken jobs (no lock held): captured
  // members get their group's event, the others stay plain.
  void launch_groups(std::vector<Job>& grp, hipStream_t hs, int64_t* n_groups, int64_t* n_grouped) {
    const size_t M = grp.size();
    std::vector<ProjDesc> desc(M);
    std::vector<int32_t> key(M, -1);
    std::vector<char> cap(M, 0);
    for (size_t m = 0; m < M; ++m) {
      Job& j = grp[m];
      if (ttice_set_option(j.s->st, TTICE_OPT_STREAM, &hs) != TTICE_OK) continue;
      if (j.rq.ready && hipStreamWaitEvent(hs, j.rq.ready, 0) != hipSuccess) continue;
      cap[m] = ttice::serve_capture(j.s->st, j.rq.batch, j.rq.n, j.rq.dtype, &desc[m], &key[m]) == 1;
    }
    // members that stay plain run on another worker's stream: the work their
    // preparation queued here (padding of the last core) completes first
    if (std::find(cap.begin(), cap.end(), 0) != cap.end()) (void)hipStreamSynchronize(hs);
    std::vector<char> done(M, 0);
    for (size_t a = 0; a < M; ++a) {
      if (!cap[a] || done[a]) continue;
      ProjGroup g;
      std::vector<size_t> mem;
      for (size_t b = a; b < M && g.n < kGroupMax; ++b) {
        if (!cap[b] || done[b] || key[b] != key[a]) continue;
        g.d[g.n] = desc[b];
        g.start[g.n + 1] = g.start[g.n] + (desc[b].Ncol + 15) / 16;
        ++g.n;
        done[b] = 1;
        mem.push_back(b);
      }
      auto ev = std::make_shared<GroupEvent>();
      bool ok = ttice::serve_group_launch(hs, key[a], g) == hipSuccess &&
                hipEventCreateWithFlags(&ev->e, hipEventDisableTiming) == hipSuccess &&
                hipEventRecord(ev->e, hs) == hipSuccess;
      if (!ok) {
        (void)hipGetLastError();
        // the members run as plain updates (their own level-1 launch)
        (void)hipStreamSynchronize(hs);
        continue;
      }
      ++*n_groups;
      *n_grouped += g.n;
      for (size_t b : mem) grp[b].ev = ev;
    }
  }

  void worker(int w) {
    hipStream_t hs = hip_streams[w];
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      work_cv.wait(lk, [&] { return stop || !jobs.empty() || !ready.empty(); });
      if (stop) return;
      Job mine;
      if (!jobs.empty()) {
        mine = std::move(jobs.front());
        jobs.pop_front();
      } else {
        std::vector<Job> grp;
        grp.push_back(take(ready.front()));
        ready.pop_front();
        if (groupable(*grp[0].s)) {
          for (auto it = ready.begin(); it != ready.end() && grp.size() < (size_t)kGroupMax;) {
            if (groupable(*streams.at(*it))) {
              grp.push_back(take(*it));
              it = ready.erase(it);
            } else {
              ++it;
            }
          }
        }
        if (grp.size() > 1) {
          lk.unlock();
          int64_t ng = 0, ni = 0;
          launch_groups(grp, hs, &ng, &ni);
          lk.lock();
          groups += ng;
          grouped += ni;
          for (size_t m = 1; m < grp.size(); ++m) jobs.push_back(std::move(grp[m]));
          work_cv.notify_all();
        }
        mine = std::move(grp[0]);
      }
      lk.unlock();
      ttice_update_info info;
      const int status = run(mine, hs, &info);
      lk.lock();
      complete(mine, status, info);
    }
  }

  // Admits waiting streams, oldest first, while they fit the budget
  void admit_waiting() {
    for (;;) {
      Stream* s = nullptr;
      int32_t sid = -1;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (stop || waiting.empty()) return;
        sid = waiting.front();
        s = streams.at(sid).get();
        if (s->need > budget - reserved) return;
        reserved += s->need;
        waiting.pop_front();
      }
      ttice_state* st = nullptr;
      const int rc = build_state(*s, &st);
      std::lock_guard<std::mutex> lk(mu);
      if (rc != TTICE_OK) {
        reserved -= s->need;
        s->admit_rc = rc;
        // its queued increments fail with the admission's status
        while (!s->q.empty()) {
          Ticket& t = tickets[s->q.front().ticket];
          t.done = true;
          t.status = rc;
          if (s->q.front().ready) (void)hipEventDestroy(s->q.front().ready);
          s->q.pop_front();
          --pending;
        }
        done_cv.notify_all();
        continue;
      }
      s->st = st;
      if (!s->q.empty() && !s->busy && !s->queued) {
        s->queued = true;
        ready.push_back(sid);
        work_cv.notify_one();
      }
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
  if (hipGetDevice(&srv->device) != hipSuccess) {
    delete srv;
    return TTICE_EDEVICE;
  }
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
                            int32_t algo, int64_t max_batch, int64_t max_tensors, int32_t* stream_id) {
  if (!srv) return TTICE_ESTATE;
  if (!stream_id || max_batch < 1 || max_tensors < max_batch || !dims || d < 1 || d > TTICE_MAX_D)
    return TTICE_EINVAL;
  *stream_id = -1;
  for (int i = 0; i < d; ++i)
    if (dims[i] < 1) return TTICE_EINVAL;
  std::unique_ptr<Stream> sp(new (std::nothrow) Stream());
  if (!sp) return TTICE_ENOMEM;
  Stream* s = sp.get();
  s->d = d;
  for (int i = 0; i < d; ++i) s->dims[i] = dims[i];
  s->eps = eps;
  s->prec = prec;
  s->algo = algo;
  s->max_batch = max_batch;
  s->max_tensors = max_tensors;
  s->need = projected_bytes(d, dims, max_batch, max_tensors);
  if (s->need > srv->budget) return TTICE_ENOMEM;  // never admissible
  // options are checked once, on a state that is not kept
  {
    ttice_state* probe = nullptr;
    int rc = ttice_create(d, dims, eps, &probe);
    if (rc == TTICE_OK) rc = ttice_set_option(probe, TTICE_OPT_PREC, &prec);
    if (rc == TTICE_OK) rc = ttice_set_option(probe, TTICE_OPT_ALGO, &algo);
    ttice_destroy(probe);
    if (rc != TTICE_OK) return rc;
  }
  int32_t id;
  bool now;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return TTICE_ESTATE;
    id = srv->next_stream++;
    now = srv->waiting.empty() && s->need <= srv->budget - srv->reserved;
    if (now)
      srv->reserved += s->need;  // held while the state is built
    else
      srv->waiting.push_back(id);
    srv->streams[id] = std::move(sp);
  }
  if (now) {
    ttice_state* st = nullptr;
    const int rc = build_state(*s, &st);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (rc != TTICE_OK) {
      srv->reserved -= s->need;
      srv->streams.erase(id);
      return rc;
    }
    s->st = st;
  }
  *stream_id = id;
  return TTICE_OK;
}

int ttice_server_submit(ttice_server* srv, int32_t stream_id, const void* batch, int64_t n, int32_t dtype,
                        void* producer, int64_t* ticket) {
  if (!srv) return TTICE_ESTATE;
  if (!ticket || n < 0 || (n > 0 && !batch) || (dtype != TTICE_F32 && dtype != TTICE_F64)) return TTICE_EINVAL;
  hipEvent_t ev = nullptr;
  if (n > 0) {
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return TTICE_EDEVICE;
    }
    if (hipEventRecord(ev, (hipStream_t)producer) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipEventDestroy(ev);
      return TTICE_EINVAL;
    }
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  auto fail = [&](int rc) {
    if (ev) (void)hipEventDestroy(ev);
    return rc;
  };
  if (srv->stop) return fail(TTICE_ESTATE);
  auto it = srv->streams.find(stream_id);
  if (it == srv->streams.end()) return fail(TTICE_EINVAL);
  Stream& s = *it->second;
  if (s.admit_rc != TTICE_OK) return fail(s.admit_rc);
  if (n > s.max_batch || s.accepted + n > s.max_tensors) return fail(TTICE_EINVAL);
  const int64_t id = srv->next_ticket++;
  srv->tickets[id] = Ticket();
  Request rq;
  rq.ticket = id;
  rq.batch = batch;
  rq.n = n;
  rq.dtype = dtype;
  rq.ready = ev;
  s.q.push_back(rq);
  s.accepted += n;
  ++srv->pending;
  if (s.st && !s.busy && !s.queued) {
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
  if (!it->second->st || it->second->busy || !it->second->q.empty()) return TTICE_ESTATE;
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
    auto w = std::find(srv->waiting.begin(), srv->waiting.end(), stream_id);
    if (w != srv->waiting.end()) {
      srv->waiting.erase(w);  // never admitted: holds no budget
    } else if (!it->second->st) {
      if (it->second->admit_rc == TTICE_OK) return TTICE_ESTATE;  // being admitted
    } else {
      srv->reserved -= it->second->need;
    }
    s = std::move(it->second);
    srv->streams.erase(it);
  }
  if (s->st) ttice_destroy(s->st);
  srv->admit_waiting();
  return TTICE_OK;
}

int ttice_server_stats(ttice_server* srv, struct ttice_server_counters* out) {
  if (!srv) return TTICE_ESTATE;
  if (!out) return TTICE_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  out->reserved_bytes = srv->reserved;
  out->budget_bytes = srv->budget;
  out->pending = srv->pending;
  out->waiting_streams = (int64_t)srv->waiting.size();
  out->groups = srv->groups;
  out->grouped_increments = srv->grouped;
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
    auto abandon = [&](const Request& rq) {
      Ticket& t = srv->tickets[rq.ticket];
      t.done = true;
      t.status = TTICE_ESTATE;
      if (rq.ready) (void)hipEventDestroy(rq.ready);
    };
    for (const Job& j : srv->jobs) abandon(j.rq);  // prepared but not run
    srv->jobs.clear();
    for (auto& kv : srv->streams)
      for (const Request& rq : kv.second->q) abandon(rq);
  }
  srv->done_cv.notify_all();
  for (hipStream_t x : srv->hip_streams) (void)hipStreamSynchronize(x);
  for (auto& kv : srv->streams)
    if (kv.second->st) ttice_destroy(kv.second->st);
  for (hipStream_t x : srv->hip_streams) (void)hipStreamDestroy(x);
  delete srv;
}

}  // extern "C"
#pragma GCC visibility pop
