// Continuous-batching request loop over the mu-mode Lawson2b path.
//
// A server owns one mm_ctx, a small pool of HIP streams (default priority) and one
// host thread. solve_submit copies a request into the pending queue. The loop
//   1. admits pending requests in arrival order while fewer than max_active are
//      running and the HBM budget covers the request's footprint (operator, factors,
//      scratch, state); admission runs mumode_setup and uploads u0;
//   2. enqueues a few Lawson2b steps for every running request, each request on the
//      stream of its slot, so kernels of different requests overlap on the device;
//   3. retires requests whose last step has completed (event query, no blocking):
//      checks the non-finite flag, copies the solution out, releases device memory.
// Each request runs the same kernels on the same shapes whether it is alone or in a
// mix, so its result does not depend on the other requests.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "mm_internal.h"

namespace {

constexpr int kStreams = 4;
constexpr int kStepsPerRound = 4;

struct Job {
  uint64_t id = 0;
  mm_request req{};
  std::vector<double> a, u0;
  int64_t est_bytes = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  // running state
  mm_op* op = nullptr;
  double* u = nullptr;
  int done_steps = 0;
  int slot = 0;
  hipEvent_t ev = nullptr;
  int64_t bytes = 0;
};

struct Result {
  int status = MM_OK;
  std::vector<double> u;
  mm_stats stats{};
};

int64_t footprint(const mm_request& r) {
  int64_t dof = 1, na = 1, fac = 0, nmax = 0;
  for (int mu = 0; mu < r.d; ++mu) {
    dof *= r.n[mu];
    na *= r.n[mu] + 2;
    fac += (int64_t)r.n[mu] * r.n[mu];
    nmax = std::max<int64_t>(nmax, r.n[mu]);
  }
  // a, u, 4 scratch grid functions, factors, Pade workspace (7 n^2)
  return 8 * (na + 5 * dof + fac + 7 * nmax * nmax) + 4096;
}

}  // namespace

struct mm_server {
  int device = 0;
  int max_active = 8;
  int64_t budget = 0;
  mm_ctx* ctx = nullptr;
  hipStream_t streams[kStreams] = {};
  std::thread thr;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_id = 1;
  std::deque<std::unique_ptr<Job>> pending;
  std::map<uint64_t, Result> results;
  std::map<uint64_t, int> state;   // 0 pending, 1 running
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  void finish(Job& j, int status) {
    Result r;
    r.status = status;
    if (status == MM_OK) {
      // the request's completion event has fired; a blocking copy on the null stream
      // does not wait for the (non-blocking) slot streams, which may hold other work
      r.u.resize(j.u0.size());
      if (hipMemcpy(r.u.data(), j.u, r.u.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        r.status = MM_EDEVICE;
    }
    j.t_done = now();
    r.stats.t_submit = j.t_submit;
    r.stats.t_admit = j.t_admit;
    r.stats.t_done = j.t_done;
    r.stats.bytes = j.bytes;
    r.stats.steps = j.done_steps;
    r.stats.status = r.status;
    release(j);
    std::lock_guard<std::mutex> lk(mu);
    state.erase(j.id);
    results[j.id] = std::move(r);
  }

  void release(Job& j) {
    if (j.op) mumode_destroy(j.op);
    j.op = nullptr;
    if (j.u) hipFree(j.u);
    j.u = nullptr;
    if (j.ev) hipEventDestroy(j.ev);
    j.ev = nullptr;
  }

  int admit(Job& j, int slot) {
    const mm_request& r = j.req;
    double* da = nullptr;
    const size_t abytes = j.a.size() * sizeof(double);
    if (hipMalloc((void**)&da, abytes) != hipSuccess) return MM_ENOMEM;
    if (hipMemcpy(da, j.a.data(), abytes, hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(da);
      return MM_EDEVICE;
    }
    mm_problem p{};
    p.d = r.d;
    for (int i = 0; i < 3; ++i) {
      p.n[i] = r.n[i];
      p.beta[i] = r.beta[i];
      p.beta_bar[i] = r.beta_bar[i];
    }
    for (int i = 0; i < 4; ++i) p.r[i] = r.r[i];
    p.lambda = r.lambda;
    p.a = da;
    int st = mumode_setup(ctx, &p, r.tau, MM_LAWSON, MM_LAWSON2B, 0, r.prec, 0, &j.op);
    hipFree(da);
    if (st != MM_OK) return st;
    const size_t ubytes = j.u0.size() * sizeof(double);
    if (hipMalloc((void**)&j.u, ubytes) != hipSuccess) return MM_ENOMEM;
    if (hipMemcpyAsync(j.u, j.u0.data(), ubytes, hipMemcpyHostToDevice, streams[slot]) != hipSuccess)
      return MM_EDEVICE;
    if (hipEventCreateWithFlags(&j.ev, hipEventDisableTiming) != hipSuccess) return MM_EDEVICE;
    j.slot = slot;
    j.bytes = j.op->bytes + (int64_t)ubytes;
    j.t_admit = now();
    return MM_OK;
  }

  void loop() {
    hipSetDevice(device);
    std::vector<std::unique_ptr<Job>> active;
    int64_t used = 0;
    int rr = 0;
    while (true) {
      std::deque<std::unique_ptr<Job>> admit_now;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (active.empty() && pending.empty()) cv.wait(lk, [&] { return stop || !pending.empty(); });
        if (stop && pending.empty() && active.empty()) break;
        // admission in arrival order: stop at the first request that does not fit
        while (!pending.empty() && (int)active.size() + (int)admit_now.size() < max_active &&
               used + pending.front()->est_bytes <= budget) {
          used += pending.front()->est_bytes;
          state[pending.front()->id] = 1;
          admit_now.push_back(std::move(pending.front()));
          pending.pop_front();
        }
      }
      for (auto& jp : admit_now) {
        const int slot = rr++ % kStreams;
        const int st = admit(*jp, slot);
        if (st != MM_OK) {
          used -= jp->est_bytes;
          finish(*jp, st);
          continue;
        }
        used += jp->bytes - jp->est_bytes;
        jp->est_bytes = jp->bytes;
        active.push_back(std::move(jp));
      }
      // one round: a few steps for every running request
      for (auto& jp : active) {
        Job& j = *jp;
        if (j.done_steps >= j.req.steps) continue;
        const int k = std::min(kStepsPerRound, j.req.steps - j.done_steps);
        if (lawson_step(ctx, j.op, j.u, k, streams[j.slot]) != MM_OK) {
          j.done_steps = -1;
          continue;
        }
        j.done_steps += k;
        if (j.done_steps >= j.req.steps) hipEventRecord(j.ev, streams[j.slot]);
      }
      // retire finished requests without blocking on the others
      for (size_t i = 0; i < active.size();) {
        Job& j = *active[i];
        bool fin = false;
        int status = MM_OK;
        if (j.done_steps < 0) {
          fin = true;
          status = MM_EDEVICE;
        } else if (j.done_steps >= j.req.steps) {
          const hipError_t q = hipEventQuery(j.ev);
          if (q == hipSuccess) {
            fin = true;
            int flag = 0;
            if (hipMemcpy(&flag, j.op->flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
              status = MM_EDEVICE;
            else if (flag)
              status = MM_EUNSTABLE;
          } else if (q != hipErrorNotReady) {
            fin = true;
            status = MM_EDEVICE;
          }
        }
        if (fin) {
          used -= j.bytes;
          finish(j, status);
          active.erase(active.begin() + i);
        } else {
          ++i;
        }
      }
      // nothing left to enqueue: wait for the device instead of spinning
      bool all_enqueued = !active.empty();
      for (auto& jp : active) all_enqueued = all_enqueued && jp->done_steps >= jp->req.steps;
      if (all_enqueued) {
        std::unique_lock<std::mutex> lk(mu);
        bool can_admit = !pending.empty() && (int)active.size() < max_active &&
                         used + pending.front()->est_bytes <= budget;
        lk.unlock();
        if (!can_admit) hipEventSynchronize(active.front()->ev);
      }
    }
  }
};

extern "C" {

mm_status mm_server_create(int device, int max_active, int64_t hbm_budget, mm_server** out) {
  if (!out || max_active < 1) return MM_EINVAL;
  *out = nullptr;
  auto* s = new mm_server();
  s->device = device;
  s->max_active = max_active;
  mm_status st = mm_ctx_create(device, &s->ctx);
  if (st != MM_OK) {
    delete s;
    return st;
  }
  if (hbm_budget <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      mm_ctx_destroy(s->ctx);
      delete s;
      return MM_EDEVICE;
    }
    hbm_budget = (int64_t)(0.9 * (double)fr);
  }
  s->budget = hbm_budget;
  for (int i = 0; i < kStreams; ++i)
    if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) {
      mm_ctx_destroy(s->ctx);
      delete s;
      return MM_EDEVICE;
    }
  s->t0 = std::chrono::steady_clock::now();
  s->thr = std::thread([s] { s->loop(); });
  *out = s;
  return MM_OK;
}

void mm_server_destroy(mm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->thr.joinable()) s->thr.join();
  for (int i = 0; i < kStreams; ++i)
    if (s->streams[i]) hipStreamDestroy(s->streams[i]);
  mm_ctx_destroy(s->ctx);
  delete s;
}

double mm_server_clock(const mm_server* s) { return s ? s->now() : 0.0; }

mm_status solve_submit(mm_server* s, const mm_request* r, uint64_t* id) {
  if (!s || !r || !id) return MM_EINVAL;
  if ((r->d != 2 && r->d != 3) || !r->a || !r->u0 || !(r->tau > 0) || r->steps < 0 ||
      r->prec < MM_FP64 || r->prec > MM_BF16X6)
    return MM_EINVAL;
  int64_t dof = 1, na = 1;
  for (int mu = 0; mu < r->d; ++mu) {
    if (r->n[mu] < 1 || r->n[mu] > 4096) return MM_EINVAL;
    dof *= r->n[mu];
    na *= r->n[mu] + 2;
  }
  auto j = std::make_unique<Job>();
  j->req = *r;
  for (int mu = r->d; mu < 3; ++mu) j->req.n[mu] = 1;
  j->a.assign(r->a, r->a + na);
  j->u0.assign(r->u0, r->u0 + dof);
  j->req.a = nullptr;
  j->req.u0 = nullptr;
  j->est_bytes = footprint(j->req);
  if (j->est_bytes > s->budget) return MM_ENOMEM;
  j->t_submit = s->now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    j->id = s->next_id++;
    *id = j->id;
    s->state[j->id] = 0;
    s->pending.push_back(std::move(j));
  }
  s->cv.notify_all();
  return MM_OK;
}

mm_status solve_poll(mm_server* s, uint64_t id, double* u_out, mm_stats* stats) {
  if (!s) return MM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->results.find(id);
  if (it == s->results.end()) return s->state.count(id) ? MM_NOT_READY : MM_ENOTFOUND;
  Result& r = it->second;
  if (u_out && r.status == MM_OK) std::memcpy(u_out, r.u.data(), r.u.size() * sizeof(double));
  if (stats) *stats = r.stats;
  const mm_status st = (mm_status)r.status;
  s->results.erase(it);
  return st;
}

}  // extern "C"
