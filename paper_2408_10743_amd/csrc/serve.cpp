// serve.cpp -- continuous-batching request engine (qd_engine_* in qdist.h).
//
// Requests are prepared on the submitting thread (input check, basis,
// generator matrices, plan).  A worker thread owns an executor and loops:
// admit waiting requests while the active set has free slots and the device
// footprint budget allows, run one step over every active code (their
// rounds share the kernel launches of the step), and move finished codes to
// the completion queue.  New requests therefore join between steps while
// earlier ones are still on the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/qdist.h"
#include "engine.hpp"

using namespace qd;

namespace {
double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

struct qd_engine {
  int device = 0;
  std::unique_ptr<Executor> ex;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Job>> pending;
  std::vector<std::unique_ptr<Job>> active;
  std::deque<std::unique_ptr<Job>> completed;
  size_t budget = 0, in_use = 0;
  int max_active = 0;
  bool stop = false;
  volatile int cancel_flag = 0;
  int outstanding = 0;  // submitted and not yet polled
  void run();
};

void qd_engine::run() {
  (void)hipSetDevice(device);
  hipStream_t s = ex->stream();
  std::vector<size_t> fp;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
      if (stop) cancel_flag = 1;
      if (stop && pending.empty() && active.empty()) break;
      // Admission: first come first served while slots and memory allow.
      while (!pending.empty() && int(active.size()) < max_active) {
        Job &j = *pending.front();
        const size_t need = Executor::footprint(j);
        if (!active.empty() && in_use + need > budget) break;
        in_use += need;
        j.t0 = now_ms();  // admission time; latency is measured from t_submit
        active.push_back(std::move(pending.front()));
        pending.pop_front();
        Job &a = *active.back();
        a.S.host_ms = 0;
        if (stop) a.opt.cancel = &cancel_flag;
        const int rc = ex->admit(a, s);
        if (rc) {
          a.status = rc;
          a.done = true;
        }
      }
      if (stop)
        for (auto &a : active) a->opt.cancel = &cancel_flag;
    }
    std::vector<Job *> v;
    for (auto &a : active)
      if (!a->done) v.push_back(a.get());
    if (!v.empty()) {
      const int rc = ex->step(v, s);
      if (rc)
        for (Job *j : v)
          if (!j->done) { j->status = rc; j->done = true; }
    }
    std::lock_guard<std::mutex> lk(mu);
    bool moved = false;
    for (size_t i = 0; i < active.size();) {
      if (active[i]->done) {
        ex->retire(*active[i]);
        in_use -= std::min(in_use, Executor::footprint(*active[i]));
        completed.push_back(std::move(active[i]));
        active.erase(active.begin() + long(i));
        moved = true;
      } else {
        ++i;
      }
    }
    if (moved) cv_done.notify_all();
  }
  cv_done.notify_all();
}

extern "C" {

qd_engine *qd_engine_create(size_t mem_budget, int max_active, void *stream) {
  auto e = std::make_unique<qd_engine>();
  if (hipGetDevice(&e->device) != hipSuccess) return nullptr;
  e->ex = std::make_unique<Executor>(static_cast<hipStream_t>(stream));
  if (!e->ex->ok()) return nullptr;
  // Short steps, so that new requests join the device work every few ms.
  e->ex->set_spec_combos(1ull << 24);
  // Tiles of 256 entries: a step ends with its last tile, and requests
  // that arrive meanwhile wait for it.
  e->ex->set_long_seg(256);
  e->ex->set_tuned(false);  // latency first: short tiles, whatever a throughput tuning chose
  e->ex->set_mfma_min_round(1ull << 26);  // and no table expansion for rounds of a few microseconds
  e->budget = mem_budget ? mem_budget : (size_t(8) << 30);
  e->max_active = max_active > 0 ? max_active : 512;
  qd_engine *raw = e.release();
  raw->worker = std::thread([raw] { raw->run(); });
  return raw;
}

int qd_engine_submit(qd_engine *e, const uint8_t *G, int m, int n, int field, unsigned long long tag,
                     const qd_options *opt) {
  if (!e) return QD_ERR_INVALID;
  auto job = std::make_unique<Job>();
  if (opt) {
    job->opt = *opt;
    job->opt.stream = nullptr;  // the engine's stream
    job->opt.timing = 0;
  }
  job->tag = tag;
  job->t_submit = now_ms();
  job->m = m;
  job->n = n;
  job->field = field;
  int rc = QD_OK;
  if (!G || m < 0 || n <= 0 || (field != QD_FIELD_F2 && field != QD_FIELD_F4)) rc = QD_ERR_INVALID;
  else if (n > kMaxN) rc = QD_ERR_TOO_LARGE;
  if (!rc) {
    job->G.assign(G, G + size_t(m) * (field == QD_FIELD_F2 ? 2 * n : n));
    Executor::prepare(*job);
    rc = job->status;
  }
  std::lock_guard<std::mutex> lk(e->mu);
  if (e->stop) return QD_ERR_INVALID;
  ++e->outstanding;
  if (rc) {
    job->status = rc;
    job->t0 = job->t_done = now_ms();
    e->completed.push_back(std::move(job));
    e->cv_done.notify_all();
    return rc;
  }
  e->pending.push_back(std::move(job));
  e->cv_work.notify_one();
  return QD_OK;
}

int qd_engine_poll(qd_engine *e, qd_result *out, uint8_t *witness, int max, int wait_ms) {
  if (!e || !out || max <= 0) return QD_ERR_INVALID;
  std::unique_lock<std::mutex> lk(e->mu);
  if (e->completed.empty() && wait_ms > 0)
    e->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !e->completed.empty(); });
  int k = 0;
  while (k < max && !e->completed.empty()) {
    std::unique_ptr<Job> j = std::move(e->completed.front());
    e->completed.pop_front();
    --e->outstanding;
    qd_result &r = out[k];
    std::memset(&r, 0, sizeof(r));
    r.tag = j->tag;
    r.status = j->status;
    r.n = j->n;
    r.d = j->status >= 0 ? j->U : -1;
    r.L = j->L;
    r.latency_ms = j->t_done - j->t_submit;
    r.queue_ms = j->t0 - j->t_submit;
    r.combinations = j->visited;
    if (witness && j->status >= 0) {
      uint8_t *w = witness + size_t(k) * 2 * QD_MAX_N;
      for (int q = 0; q < j->n; ++q) {
        w[q] = uint8_t((j->wit.x[q >> 6] >> (q & 63)) & 1);
        w[j->n + q] = uint8_t((j->wit.z[q >> 6] >> (q & 63)) & 1);
      }
    }
    ++k;
  }
  return k;
}

int qd_engine_outstanding(qd_engine *e) {
  if (!e) return QD_ERR_INVALID;
  std::lock_guard<std::mutex> lk(e->mu);
  return e->outstanding;
}

void qd_engine_destroy(qd_engine *e) {
  if (!e) return;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    e->stop = true;
  }
  e->cv_work.notify_all();
  if (e->worker.joinable()) e->worker.join();
  delete e;
}

}  // extern "C"
