// api.cpp -- C ABI of libqdist (include/qdist.h): argument checks and
// output marshalling around the step executor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/qdist.h"
#include "engine.hpp"
#include "host.hpp"
#include "kernels.hpp"

namespace qd {
hipError_t launch_valu(uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t s);
hipError_t launch_mix(int mix, uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t s);
}  // namespace qd

using namespace qd;

namespace {

void unpack(const BRow &r, int n, uint8_t *out) {
  for (int q = 0; q < n; ++q) {
    out[q] = uint8_t((r.x[q >> 6] >> (q & 63)) & 1);
    out[n + q] = uint8_t((r.z[q >> 6] >> (q & 63)) & 1);
  }
}

bool fill_job(Job &job, const uint8_t *G, int m, int n, int field, const qd_options *opt) {
  if (opt) job.opt = *opt;
  job.m = m;
  job.n = n;
  job.field = field;
  if (!G || m < 0 || n <= 0 || n > kMaxN || (field != QD_FIELD_F2 && field != QD_FIELD_F4)) {
    job.status = (n > kMaxN) ? QD_ERR_TOO_LARGE : QD_ERR_INVALID;
    return false;
  }
  const size_t bytes = size_t(m) * (field == QD_FIELD_F2 ? 2 * n : n);
  job.G.assign(G, G + bytes);
  return true;
}

// Host preparation of many jobs on a few threads.
void prepare_all(std::vector<Job> &jobs) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const size_t nt = std::min<size_t>(hw, jobs.size());
  if (nt <= 1) {
    for (Job &j : jobs)
      if (!j.status) Executor::prepare(j);
    return;
  }
  std::vector<std::thread> th;
  for (size_t w = 0; w < nt; ++w)
    th.emplace_back([&jobs, w, nt] {
      for (size_t i = w; i < jobs.size(); i += nt)
        if (!jobs[i].status) Executor::prepare(jobs[i]);
    });
  for (auto &t : th) t.join();
}

int finish(Job &job, int *d, uint8_t *witness, qd_stats *st) {
  if (st) *st = job.S;
  if (job.status < 0) {
    if (d) *d = -1;
    return job.status;
  }
  if (d) *d = job.U;
  if (witness) unpack(job.wit, job.n, witness);
  return job.status;
}

}  // namespace

namespace {
// Times `launch(blocks, iters)` after a short warm-up; lane-ops per second
// for `ops_per_iter` lane-ops per thread per iteration.
template <class F>
int time_probe(F launch, double ops_per_iter, double *lane_ops_per_s) {
  Executor *ex = nullptr;
  std::unique_lock<std::mutex> lk;
  int rc = default_executor(&ex, &lk);
  if (rc) return rc;
  hipStream_t s = ex->stream();
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return QD_ERR_DEVICE;
  const uint32_t blocks = uint32_t(cus) * 16, iters = 4096;
  uint32_t *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.f;
  rc = QD_ERR_DEVICE;
  if (hipMalloc(reinterpret_cast<void **>(&out), size_t(blocks) * 256 * 4) == hipSuccess &&
      hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
      launch(blocks, 64u, out, s) == hipSuccess && hipEventRecord(e0, s) == hipSuccess &&
      launch(blocks, iters, out, s) == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
      hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
    *lane_ops_per_s = double(blocks) * 256.0 * double(iters) * ops_per_iter / (double(ms) * 1e-3);
    rc = QD_OK;
  }
  if (out) (void)hipFree(out);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}
}  // namespace

namespace qd {

// One round over a caller-given package layout (qd_round_min,
// qd_round_census, qd_round_walk, qd_round_min_noalloc) on `arena_ex`, or on
// the device's default executor when it is NULL.
int one_round(const uint8_t *rows, const int *dims, int P, int n, int t, int partial_words, int walk, int *wmin,
              uint8_t *witness, unsigned long long *count, unsigned long long *weight_sum, int below,
              unsigned long long *census, Executor *arena_ex) {
  if (!rows || !dims || !wmin || !count || P <= 0 || P > 2 * kMaxN || t < 1 || n <= 0) return QD_ERR_INVALID;
  if (n > kMaxN) return QD_ERR_TOO_LARGE;
  if (partial_words < 0 || (partial_words > 0 && partial_words >= (n + 31) / 32)) return QD_ERR_INVALID;
  if (walk < 0 || walk > 4096) return QD_ERR_INVALID;
  Job job;
  job.n = n;
  job.single_round = true;
  job.t = t;
  job.opt.partial_weight = -1;
  job.opt.walk = walk;
  job.want_wsum = weight_sum != nullptr;
  job.force_words = partial_words;
  job.census_below = census ? std::min(below, n + 2) : 0;
  Gamma g;
  for (int i = 0; i < P; ++i) {
    if (dims[i] != 1 && dims[i] != 2) return QD_ERR_INVALID;
    Package pk;
    pk.dim = dims[i];
    pk.pivot = -1;
    std::vector<BRow> two;
    const int rc = load_rows(rows + size_t(2 * i) * 2 * n, 2, n, QD_FIELD_F2, two);
    if (rc) return rc;
    pk.r = two[0];
    if (pk.dim == 2) pk.s = two[1];
    g.pk.push_back(pk);
  }
  *wmin = n + 1;
  *count = 0;
  if (weight_sum) *weight_sum = 0;
  if (census) census[0] = census[1] = 0;
  if (t > P) return QD_OK;
  if (t > kTMax || (walk > 0 && t > kWalkMaxT)) return QD_ERR_TOO_LARGE;
  job.use.push_back(g);
  Executor::prepare_gammas(job);
  if (job.gd[0].prefix[size_t(P) * job.gd[0].R + t] >= kSat) return QD_ERR_TOO_LARGE;
  Executor *ex = arena_ex;
  std::unique_lock<std::mutex> lk;
  if (!ex) {
    const int rc = default_executor(&ex, &lk);
    if (rc) return rc;
  }
  std::vector<Job *> v{&job};
  run_jobs(*ex, v, ex->stream());
  if (job.status < 0) return job.status == QD_ERR_NOMEM && arena_ex ? QD_ERR_TOO_LARGE : job.status;
  *wmin = job.U;
  *count = job.visited;
  if (weight_sum) *weight_sum = job.wsum;
  if (census) {
    census[0] = job.census[0];
    census[1] = job.census[1];
  }
  if (witness && job.U <= n) unpack(job.wit, n, witness);
  return QD_OK;
}

}  // namespace qd

extern "C" {

int qd_distance_ex(const uint8_t *G, int m, int n, int field, const qd_options *opt, int *d, uint8_t *witness,
                   qd_stats *st) {
  if (d) *d = -1;
  if (!d) return QD_ERR_INVALID;
  Job job;
  if (fill_job(job, G, m, n, field, opt)) Executor::prepare(job);
  if (job.status) return finish(job, d, witness, st);
  Executor *ex = nullptr;
  std::unique_lock<std::mutex> lk;
  const int rc = default_executor(&ex, &lk);
  if (rc) {
    job.status = rc;
    return finish(job, d, witness, st);
  }
  hipStream_t s = job.opt.stream ? static_cast<hipStream_t>(job.opt.stream) : ex->stream();
  std::vector<Job *> v{&job};
  run_jobs(*ex, v, s);
  return finish(job, d, witness, st);
}

int qd_distance(const uint8_t *G, int m, int n, int field, int *d, uint8_t *witness) {
  return qd_distance_ex(G, m, n, field, nullptr, d, witness, nullptr);
}

int qd_distance_batch_ex(int count, const uint8_t *const *G, const int *m, const int *n, const int *field,
                         const qd_options *opt, int *d, uint8_t *const *witness, int *status, qd_stats *st) {
  if (count < 0 || (count > 0 && (!G || !m || !n || !field || !d || !status))) return QD_ERR_INVALID;
  std::vector<Job> jobs(count);
  for (int i = 0; i < count; ++i) fill_job(jobs[i], G[i], m[i], n[i], field[i], opt);
  prepare_all(jobs);
  int first = QD_OK;
  Executor *ex = nullptr;
  std::unique_lock<std::mutex> lk;
  const int rc = count ? default_executor(&ex, &lk) : QD_OK;
  if (rc) {
    for (Job &j : jobs)
      if (!j.status) j.status = rc;
  } else if (count) {
    hipStream_t s = (opt && opt->stream) ? static_cast<hipStream_t>(opt->stream) : ex->stream();
    std::vector<Job *> v;
    for (Job &j : jobs) v.push_back(&j);
    run_jobs(*ex, v, s);
  }
  for (int i = 0; i < count; ++i) {
    status[i] = finish(jobs[i], &d[i], witness ? witness[i] : nullptr, st ? &st[i] : nullptr);
    if (status[i] < 0 && first == QD_OK) first = status[i];
  }
  return first;
}

int qd_distance_batch(int count, const uint8_t *const *G, const int *m, const int *n, const int *field, int *d,
                      uint8_t *const *witness, int *status) {
  return qd_distance_batch_ex(count, G, m, n, field, nullptr, d, witness, status, nullptr);
}

int qd_plan(const uint8_t *G, int m, int n, int field, int diag, int max_gamma, qd_plan_info *out) {
  if (!out) return QD_ERR_INVALID;
  std::memset(out, 0, sizeof(*out));
  if (diag != QD_DIAG_AUTO && diag != QD_DIAG_F2 && diag != QD_DIAG_F4 && diag != QD_DIAG_ISO)
    return QD_ERR_INVALID;
  if (max_gamma < 0) return QD_ERR_INVALID;
  std::vector<BRow> rows;
  int rc = load_rows(G, m, n, field, rows);
  if (rc) return rc;
  const int k = make_basis(rows, n);
  if (k == 0) return QD_ERR_ZERO_CODE;
  const int hmax = max_gamma > 0 ? std::min(max_gamma, kMaxGamma) : kMaxGamma;
  std::vector<Gamma> f4 = build_f4(rows, n, hmax);
  Gamma f2 = build_f2(rows, n);
  for (const Gamma &g : f4)
    if (!check_gamma(g, n)) return QD_ERR_INTERNAL;
  if (!check_gamma(f2, n)) return QD_ERR_INTERNAL;
  std::vector<Gamma> iso = build_iso(rows, n, hmax);
  for (const Gamma &g : iso)
    if (!check_gamma_iso(g, n)) return QD_ERR_INTERNAL;
  const bool f4_scalar = field == QD_FIELD_F4 || alpha_closed(rows, n);
  PlanChoice pc = choose_plan(f4, f2, iso, n, k, diag, max_gamma, f4_scalar);
  // Mixed packages, as the automatic plan of qd_distance_ex takes them.
  std::vector<int> caps;
  if (!f4_scalar && k < n && pc.predicted_f4 >= kMixMinWork) {
    if (!try_mixed_f4(rows, n, k, pc.d_est, max_gamma, f4, caps)) return QD_ERR_INTERNAL;
    if (!caps.empty()) pc = choose_plan(f4, f2, iso, n, k, diag, max_gamma, f4_scalar);
  }
  for (int j = 0; j < QD_MAX_GAMMA; ++j) out->f4_two_row_cap[j] = j < int(caps.size()) ? caps[j] : -1;
  out->f4_scalar_classes = f4_scalar ? 1 : 0;
  out->n = n;
  out->rank = k;
  out->d_estimate = pc.d_est;
  out->predicted_f2 = pc.predicted_f2;
  out->predicted_f4 = pc.predicted_f4;
  out->predicted_iso = pc.predicted_iso;
  const int show = diag == QD_DIAG_AUTO ? pc.diag : diag;
  out->diag = show;
  std::vector<Gamma> gs;
  if (show == QD_DIAG_F2) gs.push_back(f2);
  else if (show == QD_DIAG_ISO) gs = iso;
  else gs = f4;
  out->h = int(gs.size());
  out->h_used = show == pc.diag ? pc.h_used : out->h;
  for (int j = 0; j < out->h; ++j) {
    out->P[j] = gs[j].P();
    out->delta[j] = gs[j].delta;
    for (int i = 0; i < gs[j].P(); ++i) {
      out->dims[j][i] = gs[j].pk[i].dim;
      out->pivot[j][i] = gs[j].pk[i].pivot;
    }
  }
  return QD_OK;
}


int qd_round_min(const uint8_t *rows, const int *dims, int P, int n, int t, int *wmin, uint8_t *witness,
                 unsigned long long *count, int partial_words) {
  return one_round(rows, dims, P, n, t, partial_words, 0, wmin, witness, count, nullptr, 0, nullptr, nullptr);
}

int qd_round_census(const uint8_t *rows, const int *dims, int P, int n, int t, int partial_words, int below,
                    int *wmin, uint8_t *witness, unsigned long long *count, unsigned long long *below_count,
                    unsigned long long *below_weight_sum) {
  if (below < 1 || !below_count || !below_weight_sum) return QD_ERR_INVALID;
  unsigned long long c[2] = {0, 0};
  const int rc = one_round(rows, dims, P, n, t, partial_words, 0, wmin, witness, count, nullptr, below, c, nullptr);
  *below_count = c[0];
  *below_weight_sum = c[1];
  return rc;
}

int qd_round_walk(const uint8_t *rows, const int *dims, int P, int n, int t, int per_lane, int *wmin,
                  uint8_t *witness, unsigned long long *count, unsigned long long *weight_sum) {
  if (per_lane < 1) return QD_ERR_INVALID;
  return one_round(rows, dims, P, n, t, 0, per_lane, wmin, witness, count, weight_sum, 0, nullptr, nullptr);
}

const char *qd_strerror(int status) {
  switch (status) {
    case QD_OK: return "ok";
    case QD_INCOMPLETE: return "incomplete: budget, cancel or walk depth reached before the bounds met";
    case QD_ERR_INVALID: return "invalid argument";
    case QD_ERR_ZERO_CODE: return "the rows span the zero code";
    case QD_ERR_TOO_LARGE: return "problem too large (n > 128 or round beyond the supported depth)";
    case QD_ERR_NOMEM: return "device memory allocation failed";
    case QD_ERR_DEVICE: return "no usable gfx950 device or a HIP call failed";
    case QD_ERR_INTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

int qd_device_check(char *name, int len) {
  if (name && len > 0) {
    name[0] = 0;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      std::strncpy(name, prop.gcnArchName, size_t(len - 1));
      name[len - 1] = 0;
    }
  }
  Executor *ex = nullptr;
  std::unique_lock<std::mutex> lk;
  return default_executor(&ex, &lk);
}

int qd_valu_peak(double *lane_ops_per_s) {
  if (!lane_ops_per_s) return QD_ERR_INVALID;
  return time_probe(launch_valu, 32.0, lane_ops_per_s);  // 8 chains x 4 ops
}

int qd_valu_mix(int mix, double *lane_ops_per_s) {
  if (!lane_ops_per_s || mix < 0 || mix > QD_MIX_XOR_SGPR) return QD_ERR_INVALID;
  return time_probe([mix](uint32_t b, uint32_t it, uint32_t *o, hipStream_t s) { return launch_mix(mix, b, it, o, s); },
                    24.0, lane_ops_per_s);  // 8 chains x 3 ops
}

}  // extern "C"
