// Serving form: a request loop with continuous batching.
//
// Requests (sparse-fit problems of different sizes) are submitted from host
// memory and queued.  A scheduler thread admits queued requests, in arrival
// order, while a slot is free and the request's device footprint fits the HBM
// budget; an admitted request gets a resident problem (data copied once, Gram
// and factorisation, zero state).  Every scheduler round advances ALL resident
// requests together -- one-class requests by `round_iters` outer iterations of
// the batched persistent launch, softmax requests by the same number of
// iterations of their own kernels, spread over three extra streams so that
// the kernels of different requests overlap -- then retires the finished ones (results
// copied to host, device memory released) so that waiting requests can enter
// between rounds.  A request's arithmetic never depends on the other requests
// it shares rounds with, so its result is the same alone and in any mix.
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
  b += (size_t)N * ((mx + 127) / 128) * 4 * ld * 8;             // batched partial sums
  b += (size_t)std::min<int64_t>(1024, N * ((mx + 3) / 4)) * ld * C * 8;   // one-problem partial sums
  return b + (1 << 20);
}

}  // namespace

// Softmax requests run their own kernels; they are spread over a few extra
// streams (default priority) so that the kernels of different requests, each
// too small to fill the GPU, overlap.
constexpr int kSideStreams = 3;

struct bca_server_s {
  size_t budget = 0, used = 0;
  int max_slots = 1, round_iters = 1;
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t side[kSideStreams] = {nullptr, nullptr, nullptr};
  uint64_t side_next = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<uint64_t, std::unique_ptr<Request>> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // statistics
  int64_t rounds = 0;
  double busy_s = 0;
};

namespace {

void finish(bca_server_s* S, Request* r, int state, const std::string& err) {
  if (r->prob) {
    bca_destroy(r->prob);
    r->prob = nullptr;
  }
  r->state = state;
  r->err = err;
  r->t_done = now_s();
  S->used -= r->bytes;
  r->A.clear();
  r->b.clear();
  r->A.shrink_to_fit();
  r->b.shrink_to_fit();
}

// Create, load and finalize the resident problem of an admitted request.
int materialise(bca_server_s* S, Request* r) {
  bca_params p = r->params;
  p.rows = r->rows.data();
  hipStream_t st = S->stream;
  if (p.loss == BCA_LOSS_SOFTMAX && S->side[0]) st = S->side[S->side_next++ % kSideStreams];
  int rc = bca_create(&p, st, &r->prob);
  if (rc != BCA_OK) return rc;
  for (int i = 0; i < p.n_partitions; ++i) {
    rc = bca_set_data(r->prob, i, r->A[i].data(), p.n_features, r->b[i].data(), BCA_MEM_HOST);
    if (rc != BCA_OK) return rc;
  }
  return bca_finalize(r->prob);
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

void scheduler(bca_server_s* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    std::vector<Request*> admitted;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait_for(lk, std::chrono::milliseconds(S->active.empty() && S->queue.empty() ? 50 : 0), [&] {
        return S->stop || !S->queue.empty() || !S->active.empty();
      });
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
      while (!S->queue.empty() && (int)(S->active.size() + admitted.size()) < S->max_slots) {
        Request* r = S->queue.front();
        if (S->used + r->bytes > S->budget) break;
        S->queue.pop_front();
        S->used += r->bytes;
        r->state = RQ_RUNNING;
        r->t_admit = now_s();
        admitted.push_back(r);
      }
    }
    const double t0 = now_s();
    for (Request* r : admitted) {
      const int rc = materialise(S, r);
      std::lock_guard<std::mutex> lk(S->mu);
      if (rc != BCA_OK) {
        finish(S, r, RQ_FAILED, bca_last_error());
      } else {
        S->active.push_back(r);
      }
    }
    std::vector<Request*> act;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      act = S->active;
    }
    if (act.empty()) continue;
    // one round: every resident request advances by round_iters outer iterations
    std::vector<bca_problem> one_class;
    std::vector<Request*> oc_req;
    std::vector<std::pair<Request*, std::string>> failed;
    for (Request* r : act) {
      if (r->cancel) continue;
      if (r->params.loss == BCA_LOSS_SOFTMAX) {
        int done_it = 0;
        bca_get_residuals(r->prob, nullptr, nullptr, nullptr, &done_it);
        const int k = std::min(S->round_iters, r->params.max_iters - done_it);
        if (k > 0 && bca_step(r->prob, k, nullptr) != BCA_OK) failed.push_back({r, bca_last_error()});
      } else {
        one_class.push_back(r->prob);
        oc_req.push_back(r);
      }
    }
    if (!one_class.empty()) {
      if (bca_batch_step(one_class.data(), (int)one_class.size(), S->round_iters, S->stream) != BCA_OK) {
        const std::string msg = bca_last_error();
        for (Request* r : oc_req) failed.push_back({r, msg});
      }
    }
    (void)hipStreamSynchronize(S->stream);
    for (int q = 0; q < kSideStreams; ++q)
      if (S->side[q]) (void)hipStreamSynchronize(S->side[q]);
    // retire finished, failed and cancelled requests
    std::vector<Request*> keep;
    for (Request* r : act) {
      bool bad = false;
      std::string msg;
      for (auto& f : failed)
        if (f.first == r) {
          bad = true;
          msg = f.second;
        }
      int it = 0;
      if (!bad && !r->cancel) bca_get_residuals(r->prob, nullptr, nullptr, nullptr, &it);
      std::lock_guard<std::mutex> lk(S->mu);
      if (r->cancel) {
        finish(S, r, RQ_CANCELLED, "cancelled");
      } else if (bad) {
        finish(S, r, RQ_FAILED, msg);
      } else if (it >= r->params.max_iters) {
        const int rc = collect(r);
        finish(S, r, rc == BCA_OK ? RQ_DONE : RQ_FAILED, rc == BCA_OK ? "" : bca_last_error());
      } else {
        keep.push_back(r);
      }
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      // requests admitted while this round ran are not in `act`; keep them
      std::vector<Request*> merged = keep;
      for (Request* r : S->active)
        if (std::find(act.begin(), act.end(), r) == act.end()) merged.push_back(r);
      S->active = merged;
      S->rounds += 1;
      S->busy_s += now_s() - t0;
    }
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
  for (int q = 0; q < kSideStreams; ++q) {
    if (hipStreamCreate(&S->side[q]) != hipSuccess) {
      for (int j = 0; j < q; ++j) (void)hipStreamDestroy(S->side[j]);
      delete S;
      return BCA_E_DEVICE;
    }
  }
  S->worker = std::thread(scheduler, S);
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
  S->cv.notify_all();
  return BCA_OK;
}

int bca_server_stats(bca_server S, int32_t* queued, int32_t* running, double* used_bytes, int64_t* rounds) {
  if (!S) return BCA_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  if (queued) *queued = (int32_t)S->queue.size();
  if (running) *running = (int32_t)S->active.size();
  if (used_bytes) *used_bytes = (double)S->used;
  if (rounds) *rounds = S->rounds;
  return BCA_OK;
}

int bca_server_destroy(bca_server S) {
  if (!S) return BCA_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (Request* r : S->active)
    if (r->prob) bca_destroy(r->prob);
  for (int q = 0; q < kSideStreams; ++q)
    if (S->side[q]) (void)hipStreamDestroy(S->side[q]);
  delete S;
  return BCA_OK;
}

}  // extern "C"
