// Serving form: a request loop with continuous batching.
//
// Requests (sparse-fit problems of different sizes) are submitted from host
// memory and queued.  The scheduler thread admits queued requests, in arrival
// order, while a slot is free and the request's device footprint fits the HBM
// budget, and hands them to a materialiser thread, which builds each admitted
// request's resident problem (data copied once, Gram and factorisation, zero
// state) on a stream of its own while the resident requests keep running.  A
// materialised request joins the resident set at the start of the next round.
// Every scheduler round advances ALL resident requests together -- one-class
// requests by `round_iters` outer iterations of the batched persistent launch,
// softmax requests by the same number of iterations of their own kernels,
// spread over two extra streams so that the kernels of different requests
// overlap -- then retires the finished ones (results copied to host, device
// memory released) so that waiting requests can enter.  A request's arithmetic
// never depends on the other requests it shares rounds with, so its result is
// the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "bca.h"
#include "bca_internal.h"

namespace {

enum { RQ_QUEUED = BCA_REQ_QUEUED, RQ_RUNNING = BCA_REQ_RUNNING, RQ_DONE = BCA_REQ_DONE,
       RQ_FAILED = BCA_REQ_FAILED, RQ_CANCELLED = BCA_REQ_CANCELLED };

double now_s() {
  using namespace std::chrono;
  return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

size_t esize(int dtype) { return dtype == BCA_F64 ? 8 : (dtype == BCA_F32 ? 4 : 2); }

struct Request {
  uint64_t ticket = 0;
  bca_params params{};
  std::vector<int64_t> rows;
  std::vector<std::vector<char>> A, b;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int state = RQ_QUEUED;
  std::atomic<bool> cancel{false};   // set by bca_server_cancel, read by the scheduler
  bca_problem prob = nullptr;
  int issued = 0;                    // outer iterations issued by the rounds so far
  size_t bytes = 0;
  std::vector<int32_t> support;
  std::vector<double> coef;
  double objective = 0;
  int iters = 0;
  std::string err;
};

// Device footprint of a request (what bca_create + bca_finalize + the batched
// form allocate), used for admission.
size_t footprint(const bca_params& p, const std::vector<int64_t>& rows) {
  const int64_t n = p.n_features, C = p.loss == BCA_LOSS_SOFTMAX ? p.n_classes : 1;
  const int64_t ld = (n + 63) / 64 * 64;
  int64_t m = 0;
  for (auto r : rows) m += r;
  const int64_t N = p.n_partitions, M = p.n_blocks;
  const int64_t nj = (n + M - 1) / M;
  size_t b = (size_t)m * ld * esize(p.a_dtype);       // A
  b += (size_t)m * 8 * (1 + 2 * C + (C > 1 ? C : 0));  // b, omega, nu (and the multi-class row buffer)
  const int64_t T = (nj + 63) / 64;
  b += (size_t)N * n * C * 8 * 3 + (size_t)N * ld * C * 8;   // x, u, rhs, xs
  b += (size_t)N * M * T * (T + 1) / 2 * 4096 * 8;   // tiled inverses K_ij^-1
  b += (size_t)N * M * T * T * 64 * C * 8;            // slots of the symmetric products
  b += (size_t)N * M * nj * nj * 8 * 2;               // finalize work space (released after)
  int64_t mx = 0;
  for (auto r : rows) mx = std::max(mx, r);
  b += (size_t)N * ((mx + 15) / 16) * ld * 8;                   // batched partial sums (16-row items)
  b += (size_t)std::min<int64_t>(1024, N * ((mx + 3) / 4)) * ld * C * 8;   // one-problem partial sums
  return b + (1 << 20);
}

}  // namespace

// Softmax requests run their own kernels; they are spread over two extra
// streams so that the kernels of different requests, each too small to fill the
// GPU, overlap.  The server's own streams (these and the materialiser's) are
// non-blocking, at the default priority: the rounds may run on the legacy
// default stream (the caller's), and a blocking stream would wait for each round
// launched before its every command (and each round for the stream's last
// command), which would leave the materialiser one command per round.  With the
// caller's stream, that makes four streams, one per hardware queue of a process.
//
// The batched launch is cooperative, with a grid sized to fill every CU, and its
// grid barriers need all of its workgroups resident at once: no other kernel may
// run beside it.  So the softmax kernels of a round finish before it starts, and
// the materialiser's device work (each library call, which returns with its
// stream drained) and the batched launch hold `gpu_mu` in turn.
constexpr int kSideStreams = 2;

struct bca_server_s {
  size_t budget = 0, used = 0;
  int max_slots = 1, round_iters = 1;
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t side[kSideStreams] = {nullptr, nullptr};
  hipStream_t mstream = nullptr;   // the materialiser's stream
  uint64_t side_next = 0;
  std::mutex mu;
  std::mutex gpu_mu;               // the batched launch, or one materialiser call
  std::condition_variable cv;      // wakes the scheduler
  std::condition_variable mcv;     // wakes the materialiser
  std::condition_variable rcv;     // wakes the releaser
  bool kick = false;               // something for the scheduler (submit, cancel, ready)
  std::deque<Request*> queue;      // submitted, not admitted
  std::deque<Request*> to_mat;     // admitted, waiting for the materialiser
  int materialising = 0;           // taken by the materialiser, not finished
  std::vector<Request*> ready;     // materialised, joining at the next round
  std::deque<Request*> to_free;    // retired, device memory not yet released
  std::vector<Request*> active;    // resident
  std::map<uint64_t, std::unique_ptr<Request>> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker, mat_worker, rel_worker;
  // statistics
  int64_t rounds = 0;
  double busy_s = 0;
  double times[BCA_SRV_TIMES] = {};   // guarded by mu
};

namespace {

// Release a request's device problem and host copy.  Called without the server
// lock (bca_destroy waits for the problem's stream and frees device memory).
void release(Request* r) {
  if (r->prob) {
    bca_destroy(r->prob);
    r->prob = nullptr;
  }
  r->A.clear();
  r->b.clear();
  r->A.shrink_to_fit();
  r->b.shrink_to_fit();
}

// Final state of a request; with the server lock held.  `freed`: its device
// memory is already released (else the materialiser releases it later and returns
// its bytes to the budget then).
void settle(bca_server_s* S, Request* r, int state, const std::string& err, bool freed = true) {
  r->state = state;
  r->err = err;
  r->t_done = now_s();
  if (freed) S->used -= r->bytes;
}

// Create, load and finalize the resident problem of an admitted request on the
// materialiser's stream, then move it to the stream its rounds run on.
void add_time(bca_server_s* S, int k, double dt) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->times[k] += dt;
}

// gpu_mu for one materialiser call, with the time spent waiting for it recorded
struct GpuTurn {
  bca_server_s* S;
  std::unique_lock<std::mutex> lk;
  explicit GpuTurn(bca_server_s* s, int wait_slot) : S(s), lk(s->gpu_mu, std::defer_lock) {
    const double t = now_s();
    lk.lock();
    add_time(S, wait_slot, now_s() - t);
  }
};

int materialise(bca_server_s* S, Request* r) {
  bca_params p = r->params;
  p.rows = r->rows.data();
  int rc = BCA_OK;
  {
    GpuTurn g(S, BCA_SRV_MAT_WAIT);
    rc = bca_create(&p, S->mstream, &r->prob);
  }
  if (rc != BCA_OK) return rc;
  for (int i = 0; i < p.n_partitions; ++i) {
    GpuTurn g(S, BCA_SRV_MAT_WAIT);
    rc = bca_set_data(r->prob, i, r->A[i].data(), p.n_features, r->b[i].data(), BCA_MEM_HOST);
    if (rc != BCA_OK) return rc;
  }
  {
    GpuTurn g(S, BCA_SRV_MAT_WAIT);
    rc = bca_finalize(r->prob);
    // one-class requests: the batched pass's tile shape, a fixed function of the
    // request's shape (a timed choice would make its rounding depend on timing
    // noise, so that the same request could give other bits on another server):
    // the most rows per tile the row length allows (R x chunks per lane <= 8), 64
    // rows per work item, 256 for rows of one 16-byte chunk per lane in tall
    // partitions (such items are small, and each costs a call)
    if (rc == BCA_OK && p.loss != BCA_LOSS_SOFTMAX) {
      const int vec = p.a_dtype == BCA_F64 ? 2 : (p.a_dtype == BCA_F32 ? 4 : 8);
      const int nvec = (p.n_features + vec - 1) / vec;
      int nc = 1;
      while (nc < 8 && 64 * nc < nvec) nc *= 2;
      int64_t mx = 0;
      for (int i = 0; i < p.n_partitions; ++i) mx = std::max<int64_t>(mx, p.rows[i]);
      const int rt = 8 / nc;
      const int ri = (nc == 1 && mx >= 4096) ? 256 : 64;
      rc = bca_batch_set_shape(r->prob, rt, ri);
    }
  }
  if (rc != BCA_OK) return rc;
  hipStream_t st = S->stream;
  if (p.loss == BCA_LOSS_SOFTMAX) st = S->side[S->side_next++ % kSideStreams];
  return bca::set_problem_stream(r->prob, st);
}

int collect(Request* r) {
  const bca_params& p = r->params;
  const int C = p.loss == BCA_LOSS_SOFTMAX ? p.n_classes : 1;
  r->support.resize(p.kappa);
  r->coef.resize((size_t)p.n_features * C);
  int rc = bca_get_support(r->prob, r->support.data(), nullptr);
  if (rc == BCA_OK) rc = bca_get_coef(r->prob, r->coef.data());
  if (rc == BCA_OK) rc = bca_get_objective(r->prob, &r->objective);
  if (rc == BCA_OK) rc = bca_get_residuals(r->prob, nullptr, nullptr, nullptr, &r->iters);
  return rc;
}

// Releases retired requests (device memory and host copies).  bca_destroy waits
// for the request's stream and hipFree for the whole device, i.e. for the round
// running at the time: on a thread of its own that wait holds up neither the
// scheduler nor the materialiser.  The bytes return to the budget once freed.
void releaser(bca_server_s* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    Request* f = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->rcv.wait(lk, [&] { return S->stop || !S->to_free.empty(); });
      if (S->stop) break;
      f = S->to_free.front();
      S->to_free.pop_front();
    }
    const double t = now_s();
    release(f);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->used -= f->bytes;
      S->times[BCA_SRV_RELEASE] += now_s() - t;
      S->kick = true;   // room in the budget for waiting requests
    }
    S->cv.notify_all();
  }
}

void materialiser(bca_server_s* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->mcv.wait(lk, [&] { return S->stop || !S->to_mat.empty(); });
      if (S->stop) break;
      r = S->to_mat.front();
      S->to_mat.pop_front();
      S->materialising += 1;
    }
    int rc = BCA_OK;
    std::string msg;
    if (!r->cancel) {
      const double t = now_s();
      rc = materialise(S, r);
      if (rc != BCA_OK) msg = bca_last_error();
      add_time(S, BCA_SRV_MATERIALISE, now_s() - t);
    }
    const bool drop = r->cancel || rc != BCA_OK;
    if (drop) release(r);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->materialising -= 1;
      if (r->cancel)
        settle(S, r, RQ_CANCELLED, "cancelled");
      else if (rc != BCA_OK)
        settle(S, r, RQ_FAILED, msg);
      else
        S->ready.push_back(r);
      S->kick = true;
    }
    S->cv.notify_all();
  }
}

void scheduler(bca_server_s* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    std::vector<Request*> act;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->active.empty() && S->ready.empty())
        S->cv.wait_for(lk, std::chrono::milliseconds(50), [&] { return S->stop || S->kick; });
      S->kick = false;
      if (S->stop) break;
      // cancelled requests still waiting leave the queue
      for (auto it = S->queue.begin(); it != S->queue.end();) {
        if ((*it)->cancel) {
          (*it)->state = RQ_CANCELLED;
          (*it)->t_done = now_s();
          it = S->queue.erase(it);
        } else {
          ++it;
        }
      }
      // admission in arrival order: a free slot and room in the HBM budget
      bool admitted = false;
      auto slots = [&] {
        return (int)(S->active.size() + S->ready.size() + S->to_mat.size()) + S->materialising;
      };
      while (!S->queue.empty() && slots() < S->max_slots) {
        Request* r = S->queue.front();
        if (S->used + r->bytes > S->budget) break;
        S->queue.pop_front();
        S->used += r->bytes;
        r->state = RQ_RUNNING;
        r->t_admit = now_s();
        S->to_mat.push_back(r);
        admitted = true;
      }
      if (admitted) S->mcv.notify_all();
      // materialised requests join the resident set
      for (Request* r : S->ready) S->active.push_back(r);
      S->ready.clear();
      act = S->active;
    }
    if (act.empty()) continue;
    const double t0 = now_s();
    // one round: every resident request advances by round_iters outer iterations
    std::vector<bca_problem> one_class;
    std::vector<Request*> oc_req;
    std::vector<std::pair<Request*, std::string>> failed;
    // (the iteration counts are tracked on the host: no device read-back, which
    // would wait for the request's stream, inside the round)
    double tm = now_s();
    for (Request* r : act) {
      if (r->cancel) continue;
      const int k = std::min(S->round_iters, r->params.max_iters - r->issued);
      if (r->params.loss == BCA_LOSS_SOFTMAX) {
        if (k > 0 && bca_step(r->prob, k, nullptr) != BCA_OK) failed.push_back({r, bca_last_error()});
      } else {
        one_class.push_back(r->prob);
        oc_req.push_back(r);
      }
      r->issued += std::max(k, 0);
    }
    for (int q = 0; q < kSideStreams; ++q)
      if (S->side[q]) (void)hipStreamSynchronize(S->side[q]);
    add_time(S, BCA_SRV_SOFTMAX, now_s() - tm);
    if (!one_class.empty()) {
      GpuTurn g(S, BCA_SRV_SCHED_WAIT);
      tm = now_s();
      if (bca_batch_step(one_class.data(), (int)one_class.size(), S->round_iters, S->stream) != BCA_OK) {
        const std::string msg = bca_last_error();
        for (Request* r : oc_req) failed.push_back({r, msg});
      }
      (void)hipStreamSynchronize(S->stream);
      add_time(S, BCA_SRV_BATCHED, now_s() - tm);
    }
    tm = now_s();
    // retire finished, failed and cancelled requests
    std::vector<Request*> keep, gone;
    std::vector<std::pair<int, std::string>> outcome;
    for (Request* r : act) {
      bool bad = false;
      std::string msg;
      for (auto& f : failed)
        if (f.first == r) {
          bad = true;
          msg = f.second;
        }
      const int it = r->issued;
      if (r->cancel) {
        outcome.push_back({RQ_CANCELLED, "cancelled"});
      } else if (bad) {
        outcome.push_back({RQ_FAILED, msg});
      } else if (it >= r->params.max_iters) {
        const int rc = collect(r);
        outcome.push_back({rc == BCA_OK ? RQ_DONE : RQ_FAILED, rc == BCA_OK ? "" : bca_last_error()});
      } else {
        keep.push_back(r);
        continue;
      }
      gone.push_back(r);
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (size_t q = 0; q < gone.size(); ++q) {
        settle(S, gone[q], outcome[q].first, outcome[q].second, false);
        S->to_free.push_back(gone[q]);
      }
      S->active = keep;
      S->rounds += 1;
      S->busy_s += now_s() - t0;
      S->times[BCA_SRV_RETIRE] += now_s() - tm;
    }
    if (!gone.empty()) S->rcv.notify_all();
    S->cv.notify_all();
  }
}

}  // namespace

extern "C" {

int bca_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t round_iters, void* hip_stream,
                      bca_server* out) {
  if (!out || max_slots < 1 || round_iters < 1 || hbm_budget_bytes == 0) return BCA_E_INVALID;
  bca_server S = new bca_server_s();
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  S->round_iters = round_iters;
  S->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return BCA_E_DEVICE;
  }
  hipStream_t* mine[kSideStreams + 1] = {&S->side[0], &S->side[1], &S->mstream};
  for (int q = 0; q <= kSideStreams; ++q) {
    if (hipStreamCreateWithFlags(mine[q], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < q; ++j) (void)hipStreamDestroy(*mine[j]);
      delete S;
      return BCA_E_DEVICE;
    }
  }
  S->worker = std::thread(scheduler, S);
  S->mat_worker = std::thread(materialiser, S);
  S->rel_worker = std::thread(releaser, S);
  *out = S;
  return BCA_OK;
}

int bca_server_submit(bca_server S, const bca_params* params, const void* const* A, const void* const* b,
                      uint64_t* ticket) {
  if (!S || !params || !A || !b || !ticket || !params->rows) return BCA_E_INVALID;
  const bca_params& p = *params;
  if (p.n_partitions < 1 || p.n_features < 1) return BCA_E_INVALID;
  if (p.flags != 0) return BCA_E_INVALID;  // requests run the batched form: no exact x-update
  auto r = std::make_unique<Request>();
  r->params = p;
  r->rows.assign(p.rows, p.rows + p.n_partitions);
  r->params.rows = nullptr;
  r->bytes = footprint(p, r->rows);
  if (r->bytes > S->budget) return BCA_E_BUDGET;
  const size_t es = esize(p.a_dtype);
  const size_t bs = p.loss == BCA_LOSS_SOFTMAX ? 4 : 8;
  r->A.resize(p.n_partitions);
  r->b.resize(p.n_partitions);
  for (int i = 0; i < p.n_partitions; ++i) {
    if (!A[i] || !b[i] || r->rows[i] < 1) return BCA_E_INVALID;
    r->A[i].resize((size_t)r->rows[i] * p.n_features * es);
    std::memcpy(r->A[i].data(), A[i], r->A[i].size());
    r->b[i].resize((size_t)r->rows[i] * bs);
    std::memcpy(r->b[i].data(), b[i], r->b[i].size());
  }
  std::lock_guard<std::mutex> lk(S->mu);
  r->ticket = S->next_ticket++;
  r->t_submit = now_s();
  *ticket = r->ticket;
  S->queue.push_back(r.get());
  S->all[r->ticket] = std::move(r);
  S->kick = true;
  S->cv.notify_all();
  return BCA_OK;
}

int bca_server_poll(bca_server S, uint64_t ticket, int32_t* state) {
  if (!S || !state) return BCA_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return BCA_E_NOTFOUND;
  *state = it->second->state;
  return BCA_OK;
}

int bca_server_fetch(bca_server S, uint64_t ticket, int32_t* idx, double* x, double* f, double* lat_s) {
  if (!S) return BCA_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return BCA_E_NOTFOUND;
  Request* r = it->second.get();
  if (r->state == RQ_CANCELLED) return BCA_E_CANCELLED;
  if (r->state == RQ_FAILED) return BCA_E_DEVICE;
  if (r->state != RQ_DONE) return BCA_E_STATE;
  if (idx) std::copy(r->support.begin(), r->support.end(), idx);
  if (x) std::copy(r->coef.begin(), r->coef.end(), x);
  if (f) *f = r->objective;
  if (lat_s) *lat_s = r->t_done - r->t_submit;
  return BCA_OK;
}

int bca_server_cancel(bca_server S, uint64_t ticket) {
  if (!S) return BCA_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return BCA_E_NOTFOUND;
  it->second->cancel = true;
  S->kick = true;
  S->cv.notify_all();
  return BCA_OK;
}

int bca_server_stats(bca_server S, int32_t* queued, int32_t* running, double* used_bytes, int64_t* rounds) {
  if (!S) return BCA_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  if (queued) *queued = (int32_t)S->queue.size();
  // admitted requests: resident, materialised, or being materialised
  if (running) *running = (int32_t)(S->active.size() + S->ready.size() + S->to_mat.size()) + S->materialising;
  if (used_bytes) *used_bytes = (double)S->used;
  if (rounds) *rounds = S->rounds;
  return BCA_OK;
}

int bca_server_timing(bca_server S, double* seconds, int32_t count) {
  if (!S || !seconds || count < 0 || count > BCA_SRV_TIMES) return BCA_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  for (int k = 0; k < count; ++k) seconds[k] = S->times[k];
  return BCA_OK;
}

int bca_server_destroy(bca_server S) {
  if (!S) return BCA_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  S->mcv.notify_all();
  S->rcv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  if (S->mat_worker.joinable()) S->mat_worker.join();
  if (S->rel_worker.joinable()) S->rel_worker.join();
  for (auto& kv : S->all)
    if (kv.second->prob) bca_destroy(kv.second->prob);
  for (int q = 0; q < kSideStreams; ++q)
    if (S->side[q]) (void)hipStreamDestroy(S->side[q]);
  if (S->mstream) (void)hipStreamDestroy(S->mstream);
  delete S;
  return BCA_OK;
}

}  // extern "C"
