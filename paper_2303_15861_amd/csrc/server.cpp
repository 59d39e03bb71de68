// Continuous-batching request loop over the mu-mode Lawson2b path.
//
// A server owns a few admission threads and one step thread, each with its own mm_ctx,
// and a pool of HIP streams (default priority):
//   admission threads: take submitted requests in arrival order while fewer than
//     max_active are admitted and the HBM budget covers the request's footprint; upload
//     a and u0 and run mumode_setup (operator, Pade factors) on their own streams, with
//     stream-ordered allocations, then hand the request to the step thread;
//   step thread: batches at the granularity of steps. Admitted finite-difference
//     requests are grouped into classes of equal (d, n, precision, digit count); a
//     class lives on one stream, and every tick the step thread enqueues the next few
//     steps of all its members together -- per pass one stencil launch and one grouped
//     mode product per axis for up to eight requests -- so a request that arrives while
//     others run joins their launches at the next tick, and one that finishes leaves.
//     At most two ticks per class are in flight, which bounds how long a newcomer
//     waits. Small 2D requests run whole in the one-workgroup solver, up to sixteen
//     per launch; periodic requests run their own step loops. Requests whose events
//     have fired are retired (non-finite flag, copy-out, release of memory and budget).
// Setup of new requests overlaps the steps of running ones. Every output of a grouped
// launch is computed by the same kernel code in the same order as for its request
// alone, so a result does not depend on the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include <cmath>

#include "mm_internal.h"

namespace {

constexpr int kStreams = 4;
constexpr int kAdmitThreads = 4;
constexpr int kTicksInFlight = 2;       // per class
constexpr int kMaxTickSteps = 32;

struct Job {
  uint64_t id = 0;
  mm_request req{};
  std::vector<double> a, u0, vel;
  int64_t est_bytes = 0;
  double work = 0;   // flop estimate for stream balancing
  double t_submit = 0, t_admit = 0, t_done = 0;
  mm_op* op = nullptr;
  double* u = nullptr;
  int slot = 0;              // stream index
  int remaining = 0;         // steps not yet enqueued (grouped requests)
  bool enqueued = false;     // every step is on a stream and ev follows the last one
  hipEvent_t ev = nullptr;
  int64_t bytes = 0;
};

// Requests that step together: equal d, n, precision, digit count and scheme.
struct Klass {
  int d = 0, n[3] = {0, 0, 0}, prec = 0, slices = 0, scheme = 0;
  int slot = 0;
  double load = 0;                      // work estimate of the members
  std::vector<Job*> members;            // arrival order, steps remaining
  std::deque<hipEvent_t> ticks;         // enqueued ticks not yet known complete
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
  // periodic: d diffusion fields (and the velocity copy), [D1 | D2 | A] per axis and the
  // remainder's three scratch grid functions per axis
  const bool periodic = r.bc[0] == MM_BC_PERIODIC;
  if (periodic) na = r.d * dof * (r.velocity ? 2 : 1) + 3 * r.d * dof + 3 * fac;
  // a, u, 4 scratch grid functions, factors (+ mixed copies), Pade workspace (7 n^2)
  return 8 * (na + 5 * dof + 2 * fac + 7 * nmax * nmax) + 4096;
}

// flops of one Lawson2b step (two actions of d mode products) plus the stencil passes
double step_work(const mm_request& r) {
  double dof = 1, nsum = 0;
  for (int mu = 0; mu < r.d; ++mu) {
    dof *= r.n[mu];
    nsum += r.n[mu];
  }
  return dof * (4.0 * nsum + 200.0);
}

}  // namespace

struct mm_server {
  int device = 0;
  int max_active = 8;
  int64_t budget = 0;
  mm_ctx* ctx = nullptr;                    // step thread
  mm_ctx* actx[kAdmitThreads] = {};         // admission threads
  hipStream_t streams[kStreams] = {};
  double stream_load[kStreams] = {};
  std::thread admit_thr[kAdmitThreads], step_thr;
  std::mutex mu;
  std::condition_variable cv_admit, cv_step;
  bool stop = false;
  uint64_t next_id = 1;
  std::deque<std::unique_ptr<Job>> pending;   // submitted
  std::deque<std::unique_ptr<Job>> ready;     // set up, not yet enqueued
  int64_t used = 0;                           // bytes held by admitted requests
  int admitted = 0;                           // in setup, ready or running
  std::map<uint64_t, Result> results;
  std::map<uint64_t, int> state;              // 0 pending, 1 admitted
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // record the outcome; called without the lock held
  void finish(Job& j, int status) {
    Result r;
    r.status = status;
    if (status == MM_OK) {
      // the completion event has fired; a blocking copy on the null stream does not
      // wait for the (non-blocking) slot streams, which may hold other requests' work
      r.u.resize(j.u0.size());
      if (hipMemcpy(r.u.data(), j.u, r.u.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        r.status = MM_EDEVICE;
    }
    j.t_done = now();
    r.stats.t_submit = j.t_submit;
    r.stats.t_admit = j.t_admit;
    r.stats.t_done = j.t_done;
    r.stats.bytes = j.bytes;
    r.stats.steps = (r.status == MM_OK) ? j.req.steps : 0;
    r.stats.status = r.status;
    release(j);
    std::lock_guard<std::mutex> lk(mu);
    state.erase(j.id);
    results[j.id] = std::move(r);
  }

  void release(Job& j) {
    if (j.op) {
      hipStream_t fs = j.op->ctx->stream;
      mumode_destroy(j.op);   // stream-ordered frees on the op's context stream
      if (j.u) hipFreeAsync(j.u, fs);
    } else if (j.u) {
      hipFreeAsync(j.u, ctx->stream);
    }
    j.op = nullptr;
    j.u = nullptr;
    if (j.ev) hipEventDestroy(j.ev);
    j.ev = nullptr;
  }

  // admission thread: upload and set up one request on the thread's own stream
  int admit(Job& j, mm_ctx* actx) {
    const mm_request& r = j.req;
    hipStream_t cs = actx->stream;
    double* da = nullptr;
    double* dv = nullptr;
    const size_t abytes = j.a.size() * sizeof(double);
    const size_t ubytes = j.u0.size() * sizeof(double);
    const size_t vbytes = j.vel.size() * sizeof(double);
    if (hipMallocAsync((void**)&da, abytes, cs) != hipSuccess) return MM_ENOMEM;
    if (vbytes && hipMallocAsync((void**)&dv, vbytes, cs) != hipSuccess) {
      hipFreeAsync(da, cs);
      return MM_ENOMEM;
    }
    auto free_inputs = [&] {
      hipFreeAsync(da, cs);
      if (dv) hipFreeAsync(dv, cs);
    };
    if (hipMallocAsync((void**)&j.u, ubytes, cs) != hipSuccess) {
      j.u = nullptr;
      free_inputs();
      return MM_ENOMEM;
    }
    if (hipMemcpyAsync(da, j.a.data(), abytes, hipMemcpyHostToDevice, cs) != hipSuccess ||
        (vbytes && hipMemcpyAsync(dv, j.vel.data(), vbytes, hipMemcpyHostToDevice, cs) != hipSuccess) ||
        hipMemcpyAsync(j.u, j.u0.data(), ubytes, hipMemcpyHostToDevice, cs) != hipSuccess) {
      free_inputs();
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
    for (int i = 0; i < 3; ++i) p.bc[i] = r.bc[i];
    p.form = r.form;
    p.lambda = r.lambda;
    p.a = da;
    for (int i = 0; i < 3; ++i) p.length[i] = r.length[i];
    p.velocity = dv;
    // mumode_setup ends with a synchronisation of actx's stream: a, u and the op are
    // ready for any stream afterwards
    const int st = mumode_setup(actx, &p, r.tau, MM_LAWSON, MM_LAWSON2B, 0, r.prec, r.slices, &j.op);
    free_inputs();
    if (st != MM_OK) {
      j.op = nullptr;
      return st;
    }
    if (hipEventCreateWithFlags(&j.ev, hipEventDisableTiming) != hipSuccess) return MM_EDEVICE;
    j.op->ctx = ctx;   // from here on the step thread owns the op
    j.bytes = j.op->bytes + (int64_t)ubytes;
    j.t_admit = now();
    return MM_OK;
  }

  void admission_loop(mm_ctx* actx) {
    hipSetDevice(device);
    while (true) {
      std::unique_ptr<Job> j;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_admit.wait(lk, [&] {
          if (pending.empty()) return stop;
          return admitted < max_active && used + pending.front()->est_bytes <= budget;
        });
        if (pending.empty()) return;   // stop requested and nothing left to admit
        j = std::move(pending.front());
        pending.pop_front();
        used += j->est_bytes;
        ++admitted;
        state[j->id] = 1;
      }
      const int st = admit(*j, actx);
      if (st != MM_OK && j->u) {   // free u on this thread's stream (no op took it over)
        if (!j->op) {
          hipFreeAsync(j->u, actx->stream);
          j->u = nullptr;
        }
      }
      if (st != MM_OK) {
        finish(*j, st);
        {
          std::lock_guard<std::mutex> lk(mu);
          used -= j->est_bytes;
          --admitted;
        }
        cv_step.notify_all();
        continue;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        used += j->bytes - j->est_bytes;
        ready.push_back(std::move(j));
      }
      cv_step.notify_all();
    }
  }

  void retire(Job& j, int status) {
    const int64_t b = j.bytes;
    finish(j, status);
    {
      std::lock_guard<std::mutex> lk(mu);
      used -= b;
      --admitted;
    }
    cv_admit.notify_all();
  }

  // ---------------------------------------------------------------- step thread
  std::vector<std::unique_ptr<Klass>> classes;
  std::vector<hipEvent_t> spare_events;
  mutable std::mutex cmu;                     // guards counters
  mm_server_counters counters{};

  hipEvent_t take_event() {
    if (!spare_events.empty()) {
      hipEvent_t e = spare_events.back();
      spare_events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  int least_loaded() const { return (int)(std::min_element(stream_load, stream_load + kStreams) - stream_load); }

  Klass* class_of(const mm_op* op) {
    for (auto& k : classes)
      if (k->d == op->d && k->n[0] == op->n[0] && k->n[1] == op->n[1] && k->n[2] == op->n[2] &&
          k->prec == op->prec && k->slices == op->slices && k->scheme == op->scheme) {
        if (k->members.empty() && k->ticks.empty()) k->slot = least_loaded();   // idle: may move
        return k.get();
      }
    auto k = std::make_unique<Klass>();
    k->d = op->d;
    for (int i = 0; i < 3; ++i) k->n[i] = op->n[i];
    k->prec = op->prec;
    k->slices = op->slices;
    k->scheme = op->scheme;
    k->slot = least_loaded();
    classes.push_back(std::move(k));
    return classes.back().get();
  }

  // Enqueue a request's whole solve on the least loaded stream (periodic problems)
  int enqueue_alone(Job& j) {
    const int s = least_loaded();
    j.slot = s;
    int st = lawson_step(ctx, j.op, j.u, j.req.steps, streams[s]);
    if (st == MM_OK && hipEventRecord(j.ev, streams[s]) != hipSuccess) st = MM_EDEVICE;
    if (st == MM_OK) {
      stream_load[s] += j.work;
      j.enqueued = true;
      std::lock_guard<std::mutex> lk(cmu);
      ++counters.single_solves;
    }
    return st;
  }

  // Small 2D requests: whole solves, up to kMaxSmallBatch per launch
  void enqueue_small(std::vector<Job*>& small, std::vector<Job*>& failed) {
    for (size_t i0 = 0; i0 < small.size(); i0 += mm::kMaxSmallBatch) {
      const int cnt = (int)std::min<size_t>(mm::kMaxSmallBatch, small.size() - i0);
      const mm_op* ops[mm::kMaxSmallBatch];
      double* us[mm::kMaxSmallBatch];
      int ns[mm::kMaxSmallBatch];
      double work = 0;
      for (int i = 0; i < cnt; ++i) {
        Job* j = small[i0 + i];
        ops[i] = j->op;
        us[i] = j->u;
        ns[i] = j->req.steps;
        work += j->work;
      }
      const int s = least_loaded();
      // one launch per scheme (Lawson-Euler and Lawson2b kernels differ); the server
      // serves Lawson2b only, so this is one launch
      int st = mm::enqueue_small2d_group(ctx, ops, us, ns, cnt, streams[s]);
      for (int i = 0; i < cnt; ++i) {
        Job* j = small[i0 + i];
        j->slot = s;
        if (st == MM_OK && hipEventRecord(j->ev, streams[s]) == hipSuccess) {
          j->enqueued = true;
        } else {
          failed.push_back(j);
        }
      }
      if (st == MM_OK) {
        stream_load[s] += work;
        std::lock_guard<std::mutex> lk(cmu);
        ++counters.small_launches;
        counters.small_solves += cnt;
      }
    }
    small.clear();
  }

  // One tick of a class: the next k steps of every member with steps left, in groups of
  // up to kMaxGroups per launch sequence, on the class's stream.
  void enqueue_tick(Klass& k, std::vector<Job*>& failed) {
    if (k.members.empty()) return;
    hipStream_t st = streams[k.slot];
    // steps per tick: about a millisecond of work at a few tens of TFLOP/s, so that
    // newcomers join quickly and the host keeps ahead of the device
    double wstep = 0;
    int kmin = kMaxTickSteps;
    for (Job* j : k.members) {
      wstep += j->work / std::max(1, j->req.steps);
      kmin = std::min(kmin, j->remaining);
    }
    const int ktarget = (int)std::max(1.0, std::min((double)kMaxTickSteps, 3e10 / std::max(wstep, 1.0)));
    const int ksteps = std::max(1, std::min(ktarget, kmin));
    for (size_t i0 = 0; i0 < k.members.size(); i0 += mm::kMaxGroups) {
      const int cnt = (int)std::min<size_t>(mm::kMaxGroups, k.members.size() - i0);
      const mm_op* ops[mm::kMaxGroups];
      double* us[mm::kMaxGroups];
      for (int i = 0; i < cnt; ++i) {
        ops[i] = k.members[i0 + i]->op;
        us[i] = k.members[i0 + i]->u;
      }
      const int rc = mm::enqueue_lawson_group(ctx, ops, us, cnt, ksteps, st);
      {
        std::lock_guard<std::mutex> lk(cmu);
        ++counters.group_launches;
        counters.problem_steps += (int64_t)cnt * ksteps;
        counters.group_steps += ksteps;
      }
      for (int i = 0; i < cnt; ++i) {
        Job* j = k.members[i0 + i];
        if (rc != MM_OK) {
          j->remaining = 0;
          failed.push_back(j);
          continue;
        }
        j->remaining -= ksteps;
        if (j->remaining == 0) {
          if (hipEventRecord(j->ev, st) == hipSuccess)
            j->enqueued = true;
          else
            failed.push_back(j);
        }
      }
    }
    {
      std::lock_guard<std::mutex> lk(cmu);
      ++counters.ticks;
    }
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, st) == hipSuccess) k.ticks.push_back(e);
    else if (e) spare_events.push_back(e);
    // members whose steps are all enqueued leave the class
    double gone = 0;
    std::vector<Job*> keep;
    for (Job* j : k.members)
      if (j->remaining > 0)
        keep.push_back(j);
      else
        gone += j->work;
    k.members.swap(keep);
    k.load -= gone;
  }

  void step_loop() {
    hipSetDevice(device);
    std::vector<std::unique_ptr<Job>> active;    // every admitted request not yet retired
    std::vector<Job*> small, failed;
    while (true) {
      std::deque<std::unique_ptr<Job>> fresh;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (active.empty()) {
          cv_step.wait(lk, [&] { return !ready.empty() || (stop && pending.empty() && admitted == 0); });
          if (ready.empty() && stop && pending.empty() && admitted == 0) break;
        }
        fresh.swap(ready);
      }
      bool progressed = !fresh.empty();
      for (auto& jp : fresh) {
        Job& j = *jp;
        if (j.req.steps == 0) {
          // nothing to enqueue: the request is done once its setup is
          if (hipEventRecord(j.ev, ctx->stream) == hipSuccess) j.enqueued = true;
          else failed.push_back(&j);
        } else if (mm::small2d_fusable(ctx, j.op)) {
          small.push_back(&j);
        } else if (mm::lawson_groupable(j.op)) {
          Klass* k = class_of(j.op);
          j.slot = k->slot;
          j.remaining = j.req.steps;
          k->members.push_back(&j);
          k->load += j.work;
          stream_load[k->slot] += j.work;
        } else if (enqueue_alone(j) != MM_OK) {
          failed.push_back(&j);
        }
        active.push_back(std::move(jp));
      }
      if (!small.empty()) enqueue_small(small, failed);
      for (auto& kp : classes) {
        Klass& k = *kp;
        while (!k.ticks.empty()) {
          const hipError_t q = hipEventQuery(k.ticks.front());
          if (q == hipErrorNotReady) break;
          spare_events.push_back(k.ticks.front());
          k.ticks.pop_front();
          progressed = true;
        }
        if (!k.members.empty() && (int)k.ticks.size() < kTicksInFlight) {
          enqueue_tick(k, failed);
          progressed = true;
        }
      }
      // retire: requests that failed to enqueue (after their stream has drained) and
      // requests whose last step has completed
      for (size_t i = 0; i < active.size();) {
        Job& j = *active[i];
        bool is_failed = std::find(failed.begin(), failed.end(), &j) != failed.end();
        int status = MM_OK;
        if (is_failed) {
          hipStreamSynchronize(streams[j.slot]);
          status = MM_EDEVICE;
        } else {
          if (!j.enqueued) {
            ++i;
            continue;
          }
          const hipError_t q = hipEventQuery(j.ev);
          if (q == hipErrorNotReady) {
            ++i;
            continue;
          }
          if (q != hipSuccess) {
            status = MM_EDEVICE;
          } else {
            int flag = 0;
            if (hipMemcpy(&flag, j.op->flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
              status = MM_EDEVICE;
            else if (flag)
              status = MM_EUNSTABLE;
          }
        }
        stream_load[j.slot] -= j.work;
        if (is_failed) {
          // take it out of its class, if it is still a member
          for (auto& kp : classes) {
            auto& m = kp->members;
            auto it = std::find(m.begin(), m.end(), &j);
            if (it != m.end()) {
              kp->load -= j.work;
              m.erase(it);
            }
          }
          failed.erase(std::find(failed.begin(), failed.end(), &j));
        }
        retire(j, status);
        active.erase(active.begin() + i);
        progressed = true;
      }
      if (!progressed && !active.empty()) {
        // nothing finished or enqueued: wait for new work or poll the events again shortly
        std::unique_lock<std::mutex> lk(mu);
        cv_step.wait_for(lk, std::chrono::microseconds(100), [&] { return !ready.empty(); });
      }
    }
    for (auto& kp : classes)
      for (hipEvent_t e : kp->ticks) hipEventDestroy(e);
    for (hipEvent_t e : spare_events) hipEventDestroy(e);
    classes.clear();
    spare_events.clear();
  }
};

extern "C" {

mm_status mm_server_create(int device, int max_active, int64_t hbm_budget, mm_server** out) {
  if (!out) return MM_EINVAL;
  *out = nullptr;
  if (max_active < 1) return MM_EINVAL;
  auto* s = new mm_server();
  s->device = device;
  s->max_active = max_active;
  mm_status st = mm_ctx_create(device, &s->ctx);
  for (int i = 0; i < kAdmitThreads && st == MM_OK; ++i) st = mm_ctx_create(device, &s->actx[i]);
  if (st != MM_OK) {
    for (int i = 0; i < kAdmitThreads; ++i) mm_ctx_destroy(s->actx[i]);
    mm_ctx_destroy(s->ctx);
    delete s;
    return st;
  }
  if (hbm_budget <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      for (int i = 0; i < kAdmitThreads; ++i) mm_ctx_destroy(s->actx[i]);
      mm_ctx_destroy(s->ctx);
      delete s;
      return MM_EDEVICE;
    }
    hbm_budget = (int64_t)(0.9 * (double)fr);
  }
  s->budget = hbm_budget;
  for (int i = 0; i < kStreams; ++i)
    if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) {
      for (int k = 0; k < i; ++k) hipStreamDestroy(s->streams[k]);
      for (int k = 0; k < kAdmitThreads; ++k) mm_ctx_destroy(s->actx[k]);
      mm_ctx_destroy(s->ctx);
      delete s;
      return MM_EDEVICE;
    }
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < kAdmitThreads; ++i) {
    mm_ctx* a = s->actx[i];
    s->admit_thr[i] = std::thread([s, a] { s->admission_loop(a); });
  }
  s->step_thr = std::thread([s] { s->step_loop(); });
  *out = s;
  return MM_OK;
}

void mm_server_destroy(mm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_admit.notify_all();
  s->cv_step.notify_all();
  for (int i = 0; i < kAdmitThreads; ++i)
    if (s->admit_thr[i].joinable()) s->admit_thr[i].join();
  s->cv_step.notify_all();
  if (s->step_thr.joinable()) s->step_thr.join();
  hipSetDevice(s->device);
  for (int i = 0; i < kStreams; ++i)
    if (s->streams[i]) hipStreamDestroy(s->streams[i]);
  for (int i = 0; i < kAdmitThreads; ++i) mm_ctx_destroy(s->actx[i]);
  mm_ctx_destroy(s->ctx);
  delete s;
}

double mm_server_clock(const mm_server* s) { return s ? s->now() : 0.0; }

mm_status mm_server_read_counters(mm_server* s, mm_server_counters* out) {
  if (!s || !out) return MM_EINVAL;
  std::lock_guard<std::mutex> lk(s->cmu);
  *out = s->counters;
  return MM_OK;
}

mm_status solve_submit(mm_server* s, const mm_request* r, uint64_t* id) {
  if (!s || !r || !id) return MM_EINVAL;
  if ((r->d != 2 && r->d != 3) || !r->a || !r->u0 || !(r->tau > 0) || r->steps < 0 ||
      r->prec < MM_FP64 || r->prec > MM_SLICED ||
      (r->prec == MM_SLICED && r->slices != 0 && (r->slices < mm::kMinSlices || r->slices > mm::kMaxSlices)))
    return MM_EINVAL;
  if (r->form != MM_FORM_FLUX && r->form != MM_FORM_NONDIV) return MM_EINVAL;
  int64_t dof = 1, na = 1;
  const bool periodic = r->bc[0] == MM_BC_PERIODIC;
  for (int mu = 0; mu < r->d; ++mu) {
    if (r->n[mu] < 1 || r->n[mu] > 4096) return MM_EINVAL;
    if (r->bc[mu] != MM_BC_DIRICHLET && r->bc[mu] != MM_BC_NEUMANN && r->bc[mu] != MM_BC_PERIODIC) return MM_EINVAL;
    if ((r->bc[mu] == MM_BC_PERIODIC) != periodic) return MM_EINVAL;
    if (periodic && !(r->length[mu] > 0.0 && std::isfinite(r->length[mu]))) return MM_EINVAL;
    dof *= r->n[mu];
    na *= r->n[mu] + 2;
  }
  if (periodic) na = r->d * dof;
  auto j = std::make_unique<Job>();
  j->req = *r;
  for (int mu = r->d; mu < 3; ++mu) {
    j->req.n[mu] = 1;
    j->req.bc[mu] = MM_BC_DIRICHLET;
  }
  j->a.assign(r->a, r->a + na);
  j->u0.assign(r->u0, r->u0 + dof);
  if (periodic && r->velocity) j->vel.assign(r->velocity, r->velocity + r->d * dof);
  j->req.a = nullptr;
  j->req.u0 = nullptr;
  j->est_bytes = footprint(j->req);
  j->work = step_work(j->req) * std::max(1, j->req.steps);
  j->req.velocity = nullptr;   // copied into j->vel
  if (j->est_bytes > s->budget) return MM_ENOMEM;
  j->t_submit = s->now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return MM_EBUSY;
    j->id = s->next_id++;
    *id = j->id;
    s->state[j->id] = 0;
    s->pending.push_back(std::move(j));
  }
  s->cv_admit.notify_all();
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
