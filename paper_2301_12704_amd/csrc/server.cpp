// Serving loop: factorizations stay resident on the device and solve requests (1..many right-
// hand sides each, any of the resident systems) are batched continuously.  The factorization
// is independent of the right-hand side (Sec. 3.4: the solve phase reuses the stored factors),
// so every request for a system is served by the same factors, and requests that wait while a
// batch runs are merged into that system's next batch.
//
// One worker thread per system, each on a stream of its own, so batches of different systems
// overlap on the device.  Memory admission charges what the systems actually hold: every
// system's right-hand-side workspaces (solve buffers, FGMRES and H^2 vectors) stay allocated
// between batches at the size of its largest batch, so they are charged to the budget while
// the system is resident and never refunded.  A batch needs only the growth of its system's
// workspaces beyond what it already holds (estimated from its columns); it is admitted when
// that growth fits in the device's free memory, read again at every admission decision, and in
// the budget next to everything charged (a batch with no other batch running may exceed the
// budget, so a small budget serializes batches instead of starving them).  A batch whose
// growth does not fit in the free memory even with no other batch running completes its
// requests with AIFMM_ERR_BUSY.  After a batch its system's charge is set to what it holds.
// Admitted batches run to completion (direct solve, or flexible GMRES to the server's residual
// target) and every request in one is completed with its own columns of the solution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "system.hpp"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
  int sys = 0;
  int64_t nrhs = 0;
  std::vector<double> b;  // N x nrhs column-major (copied at submission)
  std::vector<double> x;
  std::vector<int32_t> iters;
  std::vector<double> relres;
  clk::time_point t_submit, t_done;
  int batch_cols = 0;     // columns of the batch that served it
  aifmm_status status = AIFMM_OK;
  bool done = false;
};

}  // namespace

struct aifmm_server {
  std::vector<aifmm_system*> sys;
  std::vector<hipStream_t> own_streams, old_streams;
  size_t budget = 0, used = 0, peak = 0;
  std::vector<size_t> held;  // per system: right-hand-side workspace bytes charged to used
  int inflight = 0;          // batches admitted and not yet finished
  double rtol = 0.0;
  int max_cols = 64;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_mem;
  std::unordered_map<int64_t, Request> req;
  std::vector<std::deque<int64_t>> pending;
  int64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  int64_t batches = 0, batched_requests = 0;
  std::string err;

  // estimated right-hand-side workspace bytes of a system serving batches of nr columns
  size_t need(const aifmm_system& s, int nr) const {
    int restart = rtol > 0 ? 30 : 0;
    return (size_t)s.N * nr * sizeof(double) * (size_t)(8 + 2 * restart);
  }
  // the device's free memory now (AIFMM_DEBUG_FREE_BYTES replaces it, to force the busy path
  // from the host in tests)
  static size_t free_bytes() {
    if (const char* v = getenv("AIFMM_DEBUG_FREE_BYTES"); v && *v) return (size_t)strtoull(v, nullptr, 10);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return 0;
    return fr;
  }

  void worker(int i) {
    aifmm_system& s = *sys[i];
    (void)hipSetDevice(s.device);
    while (true) {
      std::vector<int64_t> take;
      int cols = 0;
      size_t bytes = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || !pending[i].empty(); });
        if (stop && pending[i].empty()) return;
        // FIFO, as many requests as fit in the column limit (at least one)
        while (!pending[i].empty()) {
          Request& r = req[pending[i].front()];
          if (!take.empty() && cols + r.nrhs > max_cols) break;
          cols += (int)r.nrhs;
          take.push_back(pending[i].front());
          pending[i].pop_front();
        }
        const size_t est = need(s, cols);
        bytes = est > held[i] ? est - held[i] : 0;  // growth beyond what the system holds
        bool busy = false;
        cv_mem.wait(lk, [&] {
          if (stop) return true;
          const bool fits_free = bytes == 0 || bytes <= free_bytes();
          if (fits_free && (inflight == 0 || used + bytes <= budget)) return true;
          if (inflight == 0) {  // nothing will free memory: the batch cannot run now
            busy = true;
            return true;
          }
          return false;
        });
        if (busy) {
          auto now = clk::now();
          for (int64_t t : take) {
            Request& r = req[t];
            r.t_done = now;
            r.batch_cols = cols;
            r.status = AIFMM_ERR_BUSY;
            r.done = true;
            r.b.clear();
            r.b.shrink_to_fit();
          }
          err = "serving: a batch of " + std::to_string(cols) + " columns needs " + std::to_string(bytes) +
                " more device bytes than are free";
          lk.unlock();
          cv_done.notify_all();
          continue;
        }
        used += bytes;
        ++inflight;
        peak = std::max(peak, used);
      }
      // pack the batch
      int64_t N = s.N;
      std::vector<double> B((size_t)N * cols), X((size_t)N * cols);
      std::vector<int32_t> its(cols, 0);
      std::vector<double> rel(cols, 0.0);
      {
        std::lock_guard<std::mutex> lk(mu);
        int64_t c = 0;
        for (int64_t t : take) {
          Request& r = req[t];
          std::memcpy(B.data() + c * N, r.b.data(), sizeof(double) * N * r.nrhs);
          c += r.nrhs;
        }
      }
      aifmm_status st = AIFMM_OK;
      std::string msg;
      size_t now_held = 0;
      {
        std::lock_guard<std::mutex> use(s.use);  // other calls on this system wait for the batch
        try {
          if (rtol > 0)
            aifmm::gmres_system(s, B.data(), cols, N, rtol, 30, 500, X.data(), N, its.data(), rel.data(), false, false);
          else
            aifmm::solve_system(s, B.data(), cols, N, X.data(), N, false, false);
        } catch (const aifmm::Error& e) {
          st = e.st;
          msg = e.msg;
        } catch (const std::exception& e) {
          st = AIFMM_ERR_DEVICE;
          msg = e.what();
        }
        now_held = aifmm::rhs_workspace_bytes(s);
      }
      auto now = clk::now();
      {
        std::lock_guard<std::mutex> lk(mu);
        // the reservation is replaced by the system's actual holdings
        used = used - bytes - held[i] + now_held;
        held[i] = now_held;
        peak = std::max(peak, used);
        --inflight;
        int64_t c = 0;
        for (int64_t t : take) {
          Request& r = req[t];
          r.x.assign(X.begin() + c * N, X.begin() + (c + r.nrhs) * N);
          r.iters.assign(its.begin() + c, its.begin() + c + r.nrhs);
          r.relres.assign(rel.begin() + c, rel.begin() + c + r.nrhs);
          r.t_done = now;
          r.batch_cols = cols;
          r.status = st;
          r.done = true;
          r.b.clear();
          r.b.shrink_to_fit();
          c += r.nrhs;
        }
        if (st != AIFMM_OK) err = msg;
        ++batches;
        batched_requests += (int64_t)take.size();
      }
      cv_mem.notify_all();
      cv_done.notify_all();
    }
  }
};

extern "C" {

aifmm_status aifmm_server_create(aifmm_system* const* systems, int32_t nsys, size_t hbm_budget, double rtol,
                                 int32_t max_cols, aifmm_server** out) {
  if (!out || !systems || nsys <= 0 || max_cols <= 0 || rtol < 0) return AIFMM_ERR_ARG;
  *out = nullptr;
  for (int i = 0; i < nsys; ++i) {
    if (!systems[i]) return AIFMM_ERR_ARG;
    if (!systems[i]->factored) return AIFMM_ERR_STATE;
    for (int j = 0; j < i; ++j)
      if (systems[j] == systems[i]) return AIFMM_ERR_ARG;
  }
  // what the systems already hold in right-hand-side workspaces is charged from the start
  size_t held0 = 0;
  std::vector<size_t> held(nsys);
  for (int i = 0; i < nsys; ++i) {
    std::lock_guard<std::mutex> use(systems[i]->use);
    held[i] = aifmm::rhs_workspace_bytes(*systems[i]);
    held0 += held[i];
  }
  if (hbm_budget == 0) {  // default: 90% of the device memory free now, plus what is already held
    size_t fr = 0, tot = 0;
    if (hipSetDevice(systems[0]->device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) return AIFMM_ERR_DEVICE;
    hbm_budget = fr / 10 * 9 + held0;
  }
  auto* srv = new aifmm_server();
  srv->sys.assign(systems, systems + nsys);
  srv->held = held;
  srv->used = held0;
  srv->peak = held0;
  srv->budget = hbm_budget;
  srv->rtol = rtol;
  srv->max_cols = max_cols;
  srv->pending.resize(nsys);
  for (int i = 0; i < nsys; ++i) {
    hipStream_t st = nullptr;
    if (hipSetDevice(srv->sys[i]->device) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (size_t j = 0; j < srv->own_streams.size(); ++j) {
        srv->sys[j]->stream = srv->old_streams[j];
        (void)hipStreamDestroy(srv->own_streams[j]);
      }
      delete srv;
      return AIFMM_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> use(srv->sys[i]->use);
    srv->old_streams.push_back(srv->sys[i]->stream);
    srv->own_streams.push_back(st);
    srv->sys[i]->stream = st;
  }
  for (int i = 0; i < nsys; ++i) srv->workers.emplace_back([srv, i] { srv->worker(i); });
  *out = srv;
  return AIFMM_OK;
}

aifmm_status aifmm_server_submit(aifmm_server* srv, int32_t sys, const double* b, int64_t nrhs, int64_t ldb,
                                 int64_t* ticket) {
  if (!srv || !b || !ticket || sys < 0 || sys >= (int32_t)srv->sys.size() || nrhs <= 0) return AIFMM_ERR_ARG;
  int64_t N = srv->sys[sys]->N;
  if (ldb < N || nrhs > srv->max_cols) return AIFMM_ERR_ARG;
  Request r;
  r.sys = sys;
  r.nrhs = nrhs;
  r.b.resize((size_t)N * nrhs);
  for (int64_t c = 0; c < nrhs; ++c) std::memcpy(r.b.data() + c * N, b + c * ldb, sizeof(double) * N);
  r.t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return AIFMM_ERR_STATE;
    *ticket = srv->next_ticket++;
    srv->req.emplace(*ticket, std::move(r));
    srv->pending[sys].push_back(*ticket);
  }
  srv->cv_work.notify_all();
  return AIFMM_OK;
}

aifmm_status aifmm_server_wait(aifmm_server* srv, int64_t ticket, double* x, int64_t ldx, double* latency_s,
                               int32_t* batch_cols, int32_t* iters, double* relres) {
  if (!srv || !x) return AIFMM_ERR_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->req.find(ticket);
  if (it == srv->req.end()) return AIFMM_ERR_ARG;
  Request* rp = &it->second;  // element addresses survive rehashing by other submissions
  int64_t N = srv->sys[rp->sys]->N;
  if (ldx < N) return AIFMM_ERR_ARG;
  srv->cv_done.wait(lk, [&] { return rp->done; });
  Request& r = *rp;
  aifmm_status st = r.status;
  if ((int64_t)r.x.size() == N * r.nrhs)  // a request refused as busy carries no solution
    for (int64_t c = 0; c < r.nrhs; ++c) std::memcpy(x + c * ldx, r.x.data() + c * N, sizeof(double) * N);
  if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
  if (batch_cols) *batch_cols = r.batch_cols;
  if (iters && (int64_t)r.iters.size() == r.nrhs) std::copy(r.iters.begin(), r.iters.end(), iters);
  if (relres && (int64_t)r.relres.size() == r.nrhs) std::copy(r.relres.begin(), r.relres.end(), relres);
  srv->req.erase(ticket);
  return st;
}

aifmm_status aifmm_server_stats(aifmm_server* srv, int64_t* batches, int64_t* requests, size_t* peak_bytes) {
  if (!srv) return AIFMM_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (batches) *batches = srv->batches;
  if (requests) *requests = srv->batched_requests;
  if (peak_bytes) *peak_bytes = srv->peak;
  return AIFMM_OK;
}

void aifmm_server_destroy(aifmm_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  srv->cv_mem.notify_all();
  for (auto& t : srv->workers) t.join();
  for (size_t i = 0; i < srv->sys.size(); ++i) {
    std::lock_guard<std::mutex> use(srv->sys[i]->use);
    (void)hipStreamSynchronize(srv->own_streams[i]);
    srv->sys[i]->stream = srv->old_streams[i];
    (void)hipStreamDestroy(srv->own_streams[i]);
  }
  delete srv;
}

}  // extern "C"
