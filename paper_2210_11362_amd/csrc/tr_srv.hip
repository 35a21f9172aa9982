// Serving runtime: a request loop that runs many TR-ALS jobs on one GPU with
// continuous admission.  One scheduler thread admits arrived jobs (arrival
// order, HBM-footprint admission into a device arena, bounded backfill of
// small jobs); every slot is a worker thread with two streams that runs its
// job from generation to fit, so admitted jobs overlap on the device.  Device
// memory comes from one arena allocated at creation: no hipMalloc/hipFree (and
// their device-wide synchronisation) while jobs run.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "runtime.h"

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator of job regions inside one device allocation.  Free
// ranges are kept by offset and merged with their neighbours on release.
class Arena {
 public:
  char* base = nullptr;
  size_t cap = 0, in_use = 0, peak = 0;

  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      in_use += bytes;
      peak = std::max(peak, in_use);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    in_use -= bytes;
    auto next = free_.lower_bound(off);
    size_t start = off, len = bytes;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + bytes == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }
  void reset(size_t bytes) {
    cap = bytes;
    free_.clear();
    free_[0] = bytes;
    in_use = peak = 0;
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Job {
  uint64_t id = 0;
  tr_job_desc d{};
  std::vector<const double*> init_ptrs;
  int64_t numel = 1;
  size_t bytes_x = 0, bytes_cores = 0, bytes_gen = 0, bytes_ctx = 0, footprint = 0;
  unsigned shadow_mask = 0;
  int state = TR_JOB_QUEUED;
  int status = TR_OK;
  double rel_err = NAN;
  double t_arrival = 0, t_admit = -1, t_done = -1;
  size_t off = 0;
  int slot = -1;
  std::vector<std::vector<double>> cores;
  std::string err;
};

struct Slot {
  std::thread th;
  hipStream_t s = nullptr, s2 = nullptr;
  Job* job = nullptr;
};

inline size_t esize(int dt) { return dt == TR_F64 ? 8 : 4; }

}  // namespace

struct tr_srv {
  int device = 0;
  Arena arena;
  std::vector<Slot> slots;
  std::thread sched;
  std::mutex mu;
  std::condition_variable cv_sched, cv_slot, cv_done;
  std::vector<Job*> pending;  // ordered by (arrival, id)
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_id = 1;
  bool stop = false;
  int flags = 0;
  int running = 0, max_running = 0;
  uint64_t n_done = 0, n_failed = 0;
  double head_block_since = -1;   // time the queue head was first refused memory
  uint64_t head_block_id = 0;
  Clock::time_point t0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

constexpr double HEAD_MAX_WAIT_S = 0.5;

// What a finished job hands back (committed to the Job under the lock).
struct JobOut {
  double rel_err = NAN;
  std::vector<std::vector<double>> cores;
  std::string err;
};

// One job on one slot: generate (or borrow) X and the initial cores, create a
// context in the job's arena region, run the mixed and finishing sweeps, fit,
// copy the final cores to the host.
int run_job(tr_srv* srv, const Job* j, hipStream_t s, hipStream_t s2, JobOut* out) {
  const tr_job_desc& d = j->d;
  char* base = srv->arena.base + j->off;
  size_t off = 0;
  auto carve = [&](size_t b) {
    char* p = base + off;
    off += trx_round(b);
    return p;
  };
  void* X = d.X ? const_cast<void*>(d.X) : (void*)carve(j->numel * esize(d.x_dtype));
  double* cores[TR_MAXN] = {nullptr};
  for (int k = 0; k < d.N; ++k)
    cores[k] = (double*)carve((size_t)d.ranks[k] * d.dims[k] * d.ranks[(k + 1) % d.N] * 8);
  // the generator's workspace and, after it in stream order, the context's
  char* shared = base + off;
  int rc = TR_OK;
  if (!d.X) {
    rc = trx_gen(d.N, d.dims, d.ranks, d.seed, d.eta, X, d.x_dtype, nullptr, d.init_cores ? nullptr : cores,
                 shared, j->bytes_gen, s, &out->err);
    if (rc) return rc;
  } else if (!d.init_cores) {
    for (int k = 0; k < d.N; ++k)
      if (launch_philox_normal(cores[k], (int64_t)d.ranks[k] * d.dims[k] * d.ranks[(k + 1) % d.N], d.seed,
                               GEN_SID_INIT + k, s) != hipSuccess) {
        out->err = "initial-core generation failed";
        return TR_EHIP;
      }
  }
  if (d.init_cores)
    for (int k = 0; k < d.N; ++k)
      if (hipMemcpyAsync(cores[k], j->init_ptrs[k], (size_t)d.ranks[k] * d.dims[k] * d.ranks[(k + 1) % d.N] * 8,
                         hipMemcpyDeviceToDevice, s) != hipSuccess) {
        out->err = "copy of the initial cores failed";
        return TR_EHIP;
      }
  TrxOpts o;
  o.region = shared;
  o.region_bytes = j->bytes_ctx;
  o.stream2 = s2;
  o.shadow_mask = j->shadow_mask;
  tr_als_ctx* ctx = nullptr;
  rc = trx_init(&ctx, d.N, d.dims, d.ranks, X, d.x_dtype, cores, d.variant, s, o);
  if (rc) {
    out->err = "context creation failed: " + std::string(tr_als_strerror(rc));
    return rc;
  }
  if (d.nsweeps_mixed > 0) rc = tr_als_sweep(ctx, d.nsweeps_mixed, d.prec_mixed, d.refine);
  if (rc == TR_OK && d.nsweeps_fin > 0) rc = tr_als_sweep(ctx, d.nsweeps_fin, d.prec_fin, d.refine);
  double fit = NAN;
  if (rc == TR_OK) rc = tr_als_fit(ctx, &fit);
  if (rc) out->err = tr_als_last_error(ctx);
  out->rel_err = fit;
  // final cores (the last good ones on a solve failure) to the host
  out->cores.resize(d.N);
  for (int k = 0; k < d.N; ++k) {
    const size_t n = (size_t)d.ranks[k] * d.dims[k] * d.ranks[(k + 1) % d.N];
    out->cores[k].resize(n);
    if (hipMemcpyAsync(out->cores[k].data(), cores[k], n * 8, hipMemcpyDeviceToHost, s) != hipSuccess && !rc) {
      out->err = "copy of the final cores failed";
      rc = TR_EHIP;
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess && !rc) {
    out->err = "stream synchronisation failed";
    rc = TR_EHIP;
  }
  tr_als_destroy(ctx);
  return rc;
}

void slot_main(tr_srv* srv, int k) {
  (void)hipSetDevice(srv->device);
  Slot& sl = srv->slots[k];
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    srv->cv_slot.wait(lk, [&] { return srv->stop || sl.job != nullptr; });
    if (!sl.job) return;
    Job* j = sl.job;
    lk.unlock();
    JobOut res;
    const int rc = run_job(srv, j, sl.s, sl.s2, &res);
    // nothing of the job may still run when its region is handed out again
    (void)hipStreamSynchronize(sl.s2);
    (void)hipStreamSynchronize(sl.s);
    lk.lock();
    srv->arena.release(j->off, j->footprint);
    j->rel_err = res.rel_err;
    j->cores = std::move(res.cores);
    j->err = std::move(res.err);
    j->status = rc;
    j->state = rc == TR_OK ? TR_JOB_DONE : TR_JOB_FAILED;
    j->t_done = srv->now();
    if (rc == TR_OK) srv->n_done++;
    else srv->n_failed++;
    srv->running--;
    sl.job = nullptr;
    srv->cv_sched.notify_one();
    srv->cv_done.notify_all();
  }
}

// Admission: arrived jobs in arrival order, each needing a free slot and one
// contiguous arena region of its footprint.  When the oldest arrived job does
// not fit, later jobs with footprint <= arena/64 may go first, for at most
// HEAD_MAX_WAIT_S seconds of the head's waiting.
void sched_main(tr_srv* srv) {
  std::unique_lock<std::mutex> lk(srv->mu);
  while (!srv->stop) {
    const double now = srv->now();
    double next_arrival = -1;
    bool head = true, backfill_ok = true, assigned = false;
    for (size_t q = 0; q < srv->pending.size();) {
      Job* j = srv->pending[q];
      if (j->t_arrival > now) { next_arrival = j->t_arrival; break; }
      int free_slot = -1;
      for (size_t k = 0; k < srv->slots.size(); ++k)
        if (!srv->slots[k].job) { free_slot = (int)k; break; }
      if (free_slot < 0) break;
      const bool small = j->footprint <= srv->arena.cap / 64;
      size_t off = 0;
      if ((!head && !(backfill_ok && small)) || !srv->arena.alloc(j->footprint, &off)) {
        if (head) {
          if (srv->head_block_id != j->id) { srv->head_block_id = j->id; srv->head_block_since = now; }
          backfill_ok = now - srv->head_block_since < HEAD_MAX_WAIT_S;
        }
        head = false;
        ++q;
        continue;
      }
      if (head) srv->head_block_id = 0;
      j->off = off;
      j->slot = free_slot;
      j->state = TR_JOB_RUNNING;
      j->t_admit = now;
      srv->slots[free_slot].job = j;
      srv->running++;
      srv->max_running = std::max(srv->max_running, srv->running);
      srv->pending.erase(srv->pending.begin() + q);
      assigned = true;
    }
    if (assigned) srv->cv_slot.notify_all();
    if (next_arrival >= 0)
      srv->cv_sched.wait_until(lk, srv->t0 + std::chrono::duration_cast<Clock::duration>(
                                                  std::chrono::duration<double>(next_arrival)));
    else if (!srv->stop)
      srv->cv_sched.wait(lk);
  }
}

int validate(const tr_job_desc& d) {
  if (d.N < 2 || d.N > TR_MAXN) return TR_EINVAL;
  for (int k = 0; k < d.N; ++k)
    if (d.dims[k] < 1 || d.ranks[k] < 1 || d.ranks[k] > TR_MAXR) return TR_EINVAL;
  if (d.variant != TR_NE && d.variant != TR_QR) return TR_EINVAL;
  if (d.prec_mixed < TR_F64 || d.prec_mixed > TR_FP8 || d.prec_fin < TR_F64 || d.prec_fin > TR_FP8) return TR_EINVAL;
  if (d.nsweeps_mixed < 0 || d.nsweeps_fin < 0 || d.refine < 0 || d.refine > 4) return TR_EINVAL;
  if (d.x_dtype != TR_F32 && d.x_dtype != TR_F64) return TR_EINVAL;
  if (!(d.eta >= 0.0) || !std::isfinite(d.eta) || !std::isfinite(d.t_arrival)) return TR_EINVAL;
  if (d.init_cores)
    for (int k = 0; k < d.N; ++k)
      if (!d.init_cores[k]) return TR_EINVAL;
  return TR_OK;
}

}  // namespace

extern "C" {

int tr_srv_create(tr_srv** out, size_t hbm_budget_bytes, int max_slots, int flags) {
  if (!out) return TR_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || max_slots > 64 || (flags & ~TR_SRV_BATCH)) return TR_EINVAL;
  auto srv = std::make_unique<tr_srv>();
  if (hipGetDevice(&srv->device) != hipSuccess) return TR_EHIP;
  size_t bytes = hbm_budget_bytes;
  if (bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return TR_EHIP;
    bytes = (size_t)(0.9 * (double)fr);
  }
  bytes = bytes / TRX_ALIGN * TRX_ALIGN;
  if (bytes == 0) return TR_EINVAL;
  void* base = nullptr;
  if (hipMalloc(&base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return TR_ENOMEM;
  }
  srv->arena.base = (char*)base;
  srv->arena.reset(bytes);
  srv->flags = flags;
  srv->slots.resize(max_slots);
  for (auto& sl : srv->slots)
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sl.s2, hipStreamNonBlocking) != hipSuccess) {
      for (auto& q : srv->slots) {
        if (q.s) (void)hipStreamDestroy(q.s);
        if (q.s2) (void)hipStreamDestroy(q.s2);
      }
      (void)hipFree(base);
      return TR_EHIP;
    }
  srv->t0 = Clock::now();
  tr_srv* p = srv.release();
  for (int k = 0; k < max_slots; ++k) p->slots[k].th = std::thread(slot_main, p, k);
  p->sched = std::thread(sched_main, p);
  *out = p;
  return TR_OK;
}

int tr_srv_submit(tr_srv* srv, const tr_job_desc* desc, uint64_t* job_id) {
  if (!srv || !desc || !job_id) return TR_EINVAL;
  int rc = validate(*desc);
  if (rc) return rc;
  auto j = std::make_unique<Job>();
  j->d = *desc;
  const tr_job_desc& d = j->d;
  if (d.init_cores) {
    j->init_ptrs.assign(d.init_cores, d.init_cores + d.N);
    j->d.init_cores = j->init_ptrs.data();
  }
  for (int k = 0; k < d.N; ++k) {
    if (j->numel > (int64_t(1) << 62) / d.dims[k]) return TR_EINVAL;
    j->numel *= d.dims[k];
  }
  auto bit = [](int p) { return (p == TR_BF16 || p == TR_FP8) ? (1u << p) : 0u; };
  if (d.nsweeps_mixed > 0) j->shadow_mask |= bit(d.prec_mixed);
  if (d.nsweeps_fin > 0) j->shadow_mask |= bit(d.prec_fin);
  j->bytes_x = d.X ? 0 : trx_round((size_t)j->numel * esize(d.x_dtype));
  for (int k = 0; k < d.N; ++k)
    j->bytes_cores += trx_round((size_t)d.ranks[k] * d.dims[k] * d.ranks[(k + 1) % d.N] * 8);
  j->bytes_gen = d.X ? 0 : trx_gen_workspace(d.N, d.dims, d.ranks, true);
  j->bytes_ctx = trx_footprint(d.N, d.dims, d.ranks, d.x_dtype, d.variant, j->shadow_mask);
  if (j->bytes_ctx == 0 || (!d.X && j->bytes_gen == 0)) return TR_EINVAL;
  j->footprint = j->bytes_x + j->bytes_cores + std::max(j->bytes_gen, j->bytes_ctx);
  if (j->footprint > srv->arena.cap) return TR_ENOMEM;
  std::lock_guard<std::mutex> lk(srv->mu);
  const double now = srv->now();
  j->t_arrival = std::max(d.t_arrival, now);
  j->id = srv->next_id++;
  Job* jp = j.get();
  srv->jobs[jp->id] = std::move(j);
  auto pos = std::upper_bound(srv->pending.begin(), srv->pending.end(), jp, [](const Job* a, const Job* b) {
    return a->t_arrival < b->t_arrival || (a->t_arrival == b->t_arrival && a->id < b->id);
  });
  srv->pending.insert(pos, jp);
  *job_id = jp->id;
  srv->cv_sched.notify_one();
  return TR_OK;
}

static void fill_info(const Job& j, tr_job_info* info) {
  info->state = j.state;
  info->status = j.status;
  info->rel_err = j.rel_err;
  info->t_arrival = j.t_arrival;
  info->t_admit = j.t_admit;
  info->t_done = j.t_done;
  info->footprint = j.footprint;
  info->slot = j.slot;
  info->batched = 0;
}

int tr_srv_poll(tr_srv* srv, uint64_t id, tr_job_info* info) {
  if (!srv || !info) return TR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(id);
  if (it == srv->jobs.end()) return TR_EINVAL;
  fill_info(*it->second, info);
  return TR_OK;
}

int tr_srv_wait(tr_srv* srv, uint64_t id, tr_job_info* info) {
  if (!srv || !info) return TR_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(id);
  if (it == srv->jobs.end()) return TR_EINVAL;
  Job* j = it->second.get();
  srv->cv_done.wait(lk, [&] { return j->state == TR_JOB_DONE || j->state == TR_JOB_FAILED; });
  fill_info(*j, info);
  return TR_OK;
}

int tr_srv_result(tr_srv* srv, uint64_t id, double* const* cores_host) {
  if (!srv || !cores_host) return TR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(id);
  if (it == srv->jobs.end()) return TR_EINVAL;
  const Job& j = *it->second;
  if (j.state != TR_JOB_DONE && j.state != TR_JOB_FAILED) return TR_EINVAL;
  if ((int)j.cores.size() != j.d.N) return TR_EINVAL;
  for (int k = 0; k < j.d.N; ++k) {
    if (!cores_host[k]) return TR_EINVAL;
    std::copy(j.cores[k].begin(), j.cores[k].end(), cores_host[k]);
  }
  return TR_OK;
}

int tr_srv_drain(tr_srv* srv) {
  if (!srv) return TR_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->pending.empty() && srv->running == 0; });
  return TR_OK;
}

int tr_srv_stats_read(tr_srv* srv, tr_srv_stats* out) {
  if (!srv || !out) return TR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  out->submitted = srv->next_id - 1;
  out->done = srv->n_done;
  out->failed = srv->n_failed;
  out->arena_bytes = srv->arena.cap;
  out->peak_in_use = srv->arena.peak;
  out->slots = (int)srv->slots.size();
  out->max_running = srv->max_running;
  return TR_OK;
}

const char* tr_srv_job_error(tr_srv* srv, uint64_t id) {
  if (!srv) return "null server";
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(id);
  if (it == srv->jobs.end()) return "unknown job";
  const Job& j = *it->second;
  if (j.state != TR_JOB_DONE && j.state != TR_JOB_FAILED) return "";
  return j.err.c_str();
}

int tr_srv_destroy(tr_srv* srv) {
  if (!srv) return TR_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    for (Job* j : srv->pending) {
      j->state = TR_JOB_FAILED;
      j->status = TR_EINVAL;
      j->err = "server destroyed before the job was admitted";
    }
    srv->pending.clear();
  }
  srv->cv_sched.notify_all();
  srv->cv_slot.notify_all();
  if (srv->sched.joinable()) srv->sched.join();
  for (auto& sl : srv->slots)
    if (sl.th.joinable()) sl.th.join();
  for (auto& sl : srv->slots) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    if (sl.s2) (void)hipStreamSynchronize(sl.s2);
    if (sl.s) (void)hipStreamDestroy(sl.s);
    if (sl.s2) (void)hipStreamDestroy(sl.s2);
  }
  if (srv->arena.base) (void)hipFree(srv->arena.base);
  delete srv;
  return TR_OK;
}

}  // extern "C"
