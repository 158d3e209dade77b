// Serving loop of the AA-PDHG library: continuous batching of LP requests.
//
// Two threads share the device, each with its own stream:
//   * the admission thread takes queued requests, oldest first, while a slot
//     is free and the estimated device footprint fits in the HBM budget, and
//     creates each one (host tables, uploads, scaling and the power
//     iteration, then the reset and the init step) on the copy stream; a
//     request is ready once an event recorded after its init step is;
//   * the epoch thread, at every epoch boundary, takes the ready requests
//     in (the compute stream waits for their events), rebuilds the launch
//     tables if the resident set changed, advances every resident LP by one
//     epoch of loop passes in shared launches on the compute stream, and
//     retires the LPs that have stopped (evaluation pass, results copied to
//     host memory, device memory released).
// So admitting a request overlaps the epochs of the requests already on the
// device, and a request joins the running set at the first epoch boundary
// after it is ready.  Each LP keeps its own work tables and reduction order,
// so its iterates are the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace aapdhg;

namespace {

enum ReqState { RQ_QUEUED = 0, RQ_ADMITTING = 1, RQ_RESIDENT = 2, RQ_DONE = 3, RQ_FAILED = 4 };

struct Request {
  uint64_t id = 0;
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> colidx;
  std::vector<double> val, c, q, l, u;
  std::vector<uint8_t> rowtype;
  size_t est_bytes = 0;
  double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
  int state = RQ_QUEUED;
  aapdhg_status err = AAPDHG_OK;
  std::string errmsg;
  std::unique_ptr<Problem> prob;
  hipEvent_t ready_ev = nullptr;  // recorded on the copy stream after the init step
  std::vector<double> x, y;
  aapdhg_info info{};
};

// Device bytes of one LP, estimated from its shape before it is created.
size_t estimate_bytes(const aapdhg_options& o, int32_t m, int32_t n, int64_t nnz) {
  const size_t ts = o.precision == 1 ? 8 : 4;
  const size_t N = (size_t)m + n;
  size_t b = 2 * ((size_t)nnz * (4 + ts)) + 8 * ((size_t)m + n + 1);  // CSR + CSC, row orders
  b += ts * ((size_t)3 * n + m + N) + m;                                // c, l, u, q, D-hat, row types
  b += ts * (4 * N + 2 * (size_t)n + 2 * (size_t)o.memory * N);         // iterates, residuals, x_bar, lambda, history
  b += 8 * N + sizeof(Scalars) + 64 * 1024;                             // transfer buffer, scalars, tables
  if (o.pw_period > 0) b += ts * N;                                     // primal-weight anchor
  if (o.variant == AAPDHG_VARIANT_RPDHG) b += 8 * N;                     // restart epoch sum
  b += (size_t)NDOT * 8 * (2 + ((size_t)nnz + 4 * N) / CHUNK_NNZ);      // partial records
  return b;
}

}  // namespace

struct aapdhg_server {
  aapdhg_options opt{};
  size_t budget = 0;
  int max_slots = 0;
  int device = 0;
  hipStream_t compute = nullptr, copy = nullptr;
  bool own_compute = false, own_copy = false;
  std::thread worker, admitter;
  std::mutex mu;
  std::condition_variable cv;    // epoch thread: ready requests or stop
  std::condition_variable cv_a;  // admission thread: queued requests, freed budget or stop
  bool stopping = false;
  std::deque<Request*> queue;
  std::deque<Request*> ready;  // created, init step enqueued, waiting for an epoch boundary
  std::unordered_map<uint64_t, std::unique_ptr<Request>> tickets;
  std::vector<Request*> resident;  // epoch thread only
  uint64_t next_id = 1;
  int64_t n_submitted = 0, n_admitted = 0, n_finished = 0, n_epochs = 0;
  size_t held_bytes = 0;  // estimated footprint of the admitted requests (being created, ready, resident)
  int held_slots = 0;
  std::chrono::steady_clock::time_point t0;
  std::string fatal;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  void run();
  void admit_loop();
  // The epoch thread cannot go on: release the device state of every
  // admitted request, fail them and the queued ones, stop the admission
  // thread; later submissions are refused with the message.
  void die(aapdhg_status code, const std::string& msg) {
    for (Request* r : resident) r->prob.reset();
    std::lock_guard<std::mutex> lk(mu);
    fatal = msg;
    stopping = true;
    cv_a.notify_all();
    for (Request* r : resident) fail(r, code, msg);
    resident.clear();
    for (Request* r : ready) {
      if (r->ready_ev) (void)hipEventDestroy(r->ready_ev);
      r->ready_ev = nullptr;
      r->prob.reset();
      fail(r, code, msg);
    }
    ready.clear();
    for (Request* r : queue) fail(r, code, msg);
    queue.clear();
  }
  void fail(Request* r, aapdhg_status e, const std::string& msg) {  // with mu held
    r->state = RQ_FAILED;
    r->err = e;
    r->errmsg = msg;
    r->t_done = now();
  }
};

// Admission thread: create queued requests on the copy stream.
void aapdhg_server::admit_loop() {
  try {
    hip_check(hipSetDevice(device), "server device");
  } catch (const Error& e) {
    std::lock_guard<std::mutex> lk(mu);
    fatal = e.msg;
    return;
  }
  g_setup_stream = copy;
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        if (stopping) return;
        while (!queue.empty() && queue.front()->est_bytes > budget) {  // can never fit
          Request* q = queue.front();
          queue.pop_front();
          fail(q, AAPDHG_E_NOMEM, "request does not fit in the server's device-memory budget");
        }
        if (!queue.empty() && held_slots < max_slots && held_bytes + queue.front()->est_bytes <= budget) break;
        cv_a.wait_for(lk, std::chrono::milliseconds(20));
      }
      r = queue.front();
      queue.pop_front();
      r->state = RQ_ADMITTING;
      held_bytes += r->est_bytes;
      ++held_slots;
    }
    aapdhg_status err = AAPDHG_OK;
    std::string msg;
    try {
      r->prob = std::make_unique<Problem>();
      r->prob->create(r->m, r->n, r->nnz, r->rowptr.data(), r->colidx.data(), r->val.data(), r->c.data(),
                      r->q.data(), r->l.data(), r->u.data(), r->rowtype.data(), &opt);
      r->prob->enqueue_reset(copy);
      r->prob->enqueue_init(copy);
      hip_check(hipEventCreateWithFlags(&r->ready_ev, hipEventDisableTiming), "ready event");
      hip_check(hipEventRecord(r->ready_ev, copy), "ready event");
    } catch (const Error& e) {
      err = e.status;
      msg = e.msg;
    } catch (const std::bad_alloc&) {
      err = AAPDHG_E_NOMEM;
      msg = "host allocation failed";
    } catch (const std::exception& e) {
      err = AAPDHG_E_ARG;
      msg = e.what();
    }
    if (err != AAPDHG_OK) {
      r->prob.reset();
      if (r->ready_ev) (void)hipEventDestroy(r->ready_ev);
      r->ready_ev = nullptr;
    }
    // the host copies of the inputs are no longer needed
    std::vector<int64_t>().swap(r->rowptr);
    std::vector<int32_t>().swap(r->colidx);
    std::vector<double>().swap(r->val);
    std::lock_guard<std::mutex> lk(mu);  // r may be released by a poll once its state is final
    if (err == AAPDHG_OK && !fatal.empty()) {  // the epoch thread has stopped for good
      (void)hipEventDestroy(r->ready_ev);
      r->ready_ev = nullptr;
      r->prob.reset();
      held_bytes -= r->est_bytes;
      --held_slots;
      fail(r, AAPDHG_E_STATE, fatal);
    } else if (err == AAPDHG_OK) {
      ready.push_back(r);
      cv.notify_one();
    } else {
      held_bytes -= r->est_bytes;
      --held_slots;
      fail(r, err, msg);
    }
  }
}

void aapdhg_server::run() {
  hipStream_t st = compute;
  try {
    hip_check(hipSetDevice(device), "server device");
    LaunchSet set;
    bool dirty = false;
    for (;;) {
      // ---- take the ready requests in ----
      std::vector<Request*> cand;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (resident.empty() && ready.empty() && !stopping)
          cv.wait_for(lk, std::chrono::milliseconds(20), [&] { return stopping || !ready.empty(); });
        if (stopping) break;
        cand.assign(ready.begin(), ready.end());
        ready.clear();
      }
      for (Request* r : cand) {
        hip_check(hipStreamWaitEvent(st, r->ready_ev, 0), "wait for admission");
        (void)hipEventDestroy(r->ready_ev);
        r->ready_ev = nullptr;
        std::lock_guard<std::mutex> lk(mu);
        r->state = RQ_RESIDENT;
        r->t_admit = now();
        resident.push_back(r);
        ++n_admitted;
        dirty = true;
      }
      if (resident.empty()) continue;
      // ---- one epoch for every resident LP ----
      TraceRange tr("aapdhg serving epoch");
      if (dirty) {
        std::vector<Problem*> ps;
        for (Request* r : resident) ps.push_back(r->prob.get());
        set.build(ps);
        dirty = false;
      }
      set.enqueue_passes(st, opt.epoch);
      hip_check(launch_gather_status(set.t.lps, set.t.nlps, (int*)set.d_status.p, st), "status gather");
      hip_check(hipMemcpyAsync(set.h_status, set.d_status.p, set.t.nlps * 4, hipMemcpyDeviceToHost, st), "status copy");
      hip_check(hipStreamSynchronize(st), "epoch sync");
      {
        std::lock_guard<std::mutex> lk(mu);
        ++n_epochs;
      }
      // ---- retire ----
      std::vector<Request*> keep;
      for (size_t i = 0; i < resident.size(); ++i) {
        Request* r = resident[i];
        if (set.h_status[i] == ST_RUNNING) {
          keep.push_back(r);
          continue;
        }
        r->x.resize(r->n);
        r->y.resize(r->m);
        r->prob->result(r->x.data(), r->y.data(), nullptr, &r->info, true);
        r->prob.reset();
        std::lock_guard<std::mutex> lk(mu);
        r->state = RQ_DONE;
        r->t_done = now();
        held_bytes -= r->est_bytes;
        --held_slots;
        ++n_finished;
        dirty = true;
        cv_a.notify_one();
      }
      resident.swap(keep);
    }
  } catch (const Error& e) {
    die(e.status, e.msg);
  } catch (const std::bad_alloc&) {
    die(AAPDHG_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    die(AAPDHG_E_ARG, e.what());
  }
  for (Request* r : resident) r->prob.reset();  // stopped: requests stay resident until the server is freed
  resident.clear();
}

extern "C" {

aapdhg_status aapdhg_server_start(size_t hbm_budget_bytes, int32_t max_slots, const aapdhg_options* opt,
                                  void* compute_stream, void* copy_stream, aapdhg_server_t* out) {
  if (!out) {
    g_thread_error = "out is NULL";
    return AAPDHG_E_ARG;
  }
  *out = nullptr;
  if (max_slots < 1 || max_slots > LaunchSet::MAX_STATUS) {
    g_thread_error = "max_slots out of range";
    return AAPDHG_E_ARG;
  }
  auto* s = new (std::nothrow) aapdhg_server;
  if (!s) return AAPDHG_E_NOMEM;
  if (opt) s->opt = *opt; else default_options(&s->opt);
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    g_thread_error = "hipGetDevice failed";
    return AAPDHG_E_HIP;
  }
  s->compute = (hipStream_t)compute_stream;
  s->copy = (hipStream_t)copy_stream;
  if (!s->compute) {
    s->own_compute = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) == hipSuccess;
    if (!s->own_compute) s->compute = nullptr;
  }
  if (!s->copy) {
    s->own_copy = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) == hipSuccess;
    if (!s->own_copy) s->copy = nullptr;
  }
  if (!s->compute || !s->copy || s->compute == s->copy) {
    const bool same = s->compute && s->compute == s->copy;
    if (s->own_compute) (void)hipStreamDestroy(s->compute);
    if (s->own_copy) (void)hipStreamDestroy(s->copy);
    delete s;
    g_thread_error = same ? "the compute and copy streams must differ" : "stream creation failed";
    return same ? AAPDHG_E_ARG : AAPDHG_E_HIP;
  }
  try {
    s->worker = std::thread([s] { s->run(); });
    s->admitter = std::thread([s] { s->admit_loop(); });
  } catch (const std::exception&) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stopping = true;
    }
    s->cv.notify_all();
    s->cv_a.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->own_compute) (void)hipStreamDestroy(s->compute);
    if (s->own_copy) (void)hipStreamDestroy(s->copy);
    delete s;
    g_thread_error = "thread creation failed";
    return AAPDHG_E_NOMEM;
  }
  *out = s;
  return AAPDHG_OK;
}

aapdhg_status aapdhg_server_submit(aapdhg_server_t s, int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr,
                                   const int32_t* col_idx, const double* val, const double* c, const double* q,
                                   const double* l, const double* u, const uint8_t* row_type, uint64_t* ticket) {
  if (!s || !ticket || !row_ptr || !c || !q || !l || !u || !row_type || m < 1 || n < 1 || nnz < 0 ||
      ((!col_idx || !val) && nnz > 0)) {
    g_thread_error = "invalid submit arguments";
    return AAPDHG_E_ARG;
  }
  std::unique_ptr<Request> r;
  try {
    r = std::make_unique<Request>();
    r->m = m;
    r->n = n;
    r->nnz = nnz;
    r->rowptr.assign(row_ptr, row_ptr + m + 1);
    r->colidx.assign(col_idx, col_idx + nnz);
    r->val.assign(val, val + nnz);
    r->c.assign(c, c + n);
    r->q.assign(q, q + m);
    r->l.assign(l, l + n);
    r->u.assign(u, u + n);
    r->rowtype.assign(row_type, row_type + m);
    r->est_bytes = estimate_bytes(s->opt, m, n, nnz);
  } catch (const std::exception&) {
    g_thread_error = "host allocation failed while copying the request";
    return AAPDHG_E_NOMEM;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->fatal.empty()) {
    g_thread_error = s->fatal;
    return AAPDHG_E_STATE;
  }
  r->id = s->next_id++;
  r->t_submit = s->now();
  *ticket = r->id;
  s->queue.push_back(r.get());
  s->tickets[r->id] = std::move(r);
  ++s->n_submitted;
  s->cv_a.notify_one();
  return AAPDHG_OK;
}

aapdhg_status aapdhg_server_poll(aapdhg_server_t s, uint64_t ticket, aapdhg_info* info, double* x, double* y,
                                 double* t_admit, double* t_done) {
  if (!s) return AAPDHG_E_ARG;
  std::unique_ptr<Request> done;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
      g_thread_error = "unknown ticket";
      return AAPDHG_E_ARG;
    }
    Request* r = it->second.get();
    if (r->state == RQ_QUEUED || r->state == RQ_ADMITTING || r->state == RQ_RESIDENT) return AAPDHG_PENDING;
    done = std::move(it->second);
    s->tickets.erase(it);
  }
  if (t_admit) *t_admit = done->t_admit - done->t_submit >= 0 ? done->t_admit - done->t_submit : -1.0;
  if (t_done) *t_done = done->t_done - done->t_submit;
  if (done->state == RQ_FAILED) {
    g_thread_error = done->errmsg;
    return done->err;
  }
  if (info) *info = done->info;
  if (x) std::copy(done->x.begin(), done->x.end(), x);
  if (y) std::copy(done->y.begin(), done->y.end(), y);
  return AAPDHG_OK;
}

aapdhg_status aapdhg_server_stats(aapdhg_server_t s, int64_t* stats6) {
  if (!s || !stats6) return AAPDHG_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  stats6[0] = s->n_submitted;
  stats6[1] = s->n_admitted;
  stats6[2] = s->n_finished;
  stats6[3] = (int64_t)(s->n_admitted - s->n_finished);
  stats6[4] = s->n_epochs;
  stats6[5] = (int64_t)s->held_bytes;
  return AAPDHG_OK;
}

aapdhg_status aapdhg_server_stop(aapdhg_server_t s) {
  if (!s) return AAPDHG_E_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  s->cv_a.notify_all();
  if (s->admitter.joinable()) s->admitter.join();
  if (s->worker.joinable()) s->worker.join();
  // requests admitted but not yet taken in: release their device state
  for (Request* r : s->ready) {
    if (r->ready_ev) (void)hipEventDestroy(r->ready_ev);
    r->prob.reset();
  }
  s->ready.clear();
  if (s->own_compute) (void)hipStreamDestroy(s->compute);
  if (s->own_copy) (void)hipStreamDestroy(s->copy);
  delete s;
  return AAPDHG_OK;
}

}  // extern "C"
