// Serving runtime: a request loop that runs many TR-ALS jobs on one GPU with
// continuous admission.  One executor thread is the only caller of HIP: it
// admits arrived jobs (arrival order, HBM-footprint admission into a device
// arena, bounded backfill of small jobs), enqueues each admitted job's whole
// work (generation, sweeps, fit, result copies) on its slot's streams without
// waiting, and polls the slots' completion events, so admitted jobs overlap on
// the device.  Device memory comes from one arena allocated at creation: no
// hipMalloc/hipFree (and their device-wide synchronisation) while jobs run.
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
#include "tiny.h"

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
  bool tiny = false;          // runs in a batch lane
  int state = TR_JOB_QUEUED;
  int status = TR_OK;
  double rel_err = NAN;
  double t_arrival = 0, t_admit = -1, t_done = -1;
  size_t off = 0;
  int slot = -1;
  std::vector<std::vector<double>> cores;
  std::string err;
};

// A slot runs one job at a time: its streams, the completion event of the job
// and pinned host memory for the job's results (status word, norms, cores).
struct Slot {
  hipStream_t s = nullptr, s2 = nullptr;
  hipEvent_t done = nullptr;
  Job* job = nullptr;
  tr_als_ctx* ctx = nullptr;
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  int rc = TR_OK;             // enqueue failure of the running job
  std::string err;
};

// A batch lane runs up to LANE_MAX small jobs as one persistent launch (one
// workgroup per job): its stream, completion event, descriptor arrays and
// pinned memory for the jobs' results.
constexpr int LANE_MAX = 64;
constexpr int NLANES = 2;

struct Lane {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  std::vector<Job*> jobs;
  TinyJob* h_desc = nullptr;   // pinned
  TinyJob* d_desc = nullptr;   // device
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  int rc = TR_OK;
  std::string err;
};

inline size_t esize(int dt) { return dt == TR_F64 ? 8 : 4; }

inline size_t core_elems(const tr_job_desc& d, int k) {
  return (size_t)d.ranks[k] * d.dims[k] * d.ranks[(k + 1) % d.N];
}

constexpr size_t PIN_HEAD = 64;              // status word, ||X||^2, residual^2
constexpr size_t PIN_DEFAULT = 8u << 20;     // per slot; grown on demand

}  // namespace

struct tr_srv {
  int device = 0;
  Arena arena;
  std::vector<Slot> slots;
  std::vector<Lane> lanes;
  std::vector<char*> old_pinned;   // outgrown pinned buffers, freed at destroy
  std::thread exec;
  std::mutex mu;
  std::condition_variable cv_exec, cv_done;
  std::vector<Job*> pending;  // ordered by (arrival, id)
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_id = 1;
  uint64_t gen = 0;           // bumped by every submit and by stop, under the lock
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
constexpr auto POLL = std::chrono::microseconds(50);
constexpr auto IDLE_MAX = std::chrono::milliseconds(10);

// Enqueue a whole job on its slot: generate (or borrow) X and the initial
// cores, create a context in the job's arena region, the mixed and finishing
// sweeps, the fit, the copies of the results to pinned memory and the
// completion event.  Nothing here waits on the device (FP8 contractions read
// their scale back).
int start_job(tr_srv* srv, Slot& sl) {
  const Job* j = sl.job;
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
  size_t core_bytes = 0;
  for (int k = 0; k < d.N; ++k) {
    cores[k] = (double*)carve(core_elems(d, k) * 8);
    core_bytes += core_elems(d, k) * 8;
  }
  if (PIN_HEAD + core_bytes > sl.pinned_bytes) {
    void* p = nullptr;
    const size_t want = std::max(PIN_HEAD + core_bytes, 2 * sl.pinned_bytes);
    if (hipHostMalloc(&p, want, 0) != hipSuccess) {
      (void)hipGetLastError();
      sl.err = "pinned host allocation failed";
      return TR_ENOMEM;
    }
    if (sl.pinned) srv->old_pinned.push_back(sl.pinned);
    sl.pinned = (char*)p;
    sl.pinned_bytes = want;
  }
  // the generator's workspace and, after it in stream order, the context's
  char* shared = base + off;
  hipStream_t s = sl.s;
  int rc = TR_OK;
  if (!d.X) {
    rc = trx_gen(d.N, d.dims, d.ranks, d.seed, d.eta, X, d.x_dtype, nullptr, d.init_cores ? nullptr : cores,
                 shared, j->bytes_gen, s, &sl.err);
    if (rc) return rc;
  } else if (!d.init_cores) {
    for (int k = 0; k < d.N; ++k)
      if (launch_philox_normal(cores[k], (int64_t)core_elems(d, k), d.seed, GEN_SID_INIT + k, s) != hipSuccess) {
        sl.err = "initial-core generation failed";
        return TR_EHIP;
      }
  }
  if (d.init_cores)
    for (int k = 0; k < d.N; ++k)
      if (hipMemcpyAsync(cores[k], j->init_ptrs[k], core_elems(d, k) * 8, hipMemcpyDeviceToDevice, s) !=
          hipSuccess) {
        sl.err = "copy of the initial cores failed";
        return TR_EHIP;
      }
  TrxOpts o;
  o.region = shared;
  o.region_bytes = j->bytes_ctx;
  o.stream2 = sl.s2;
  o.shadow_mask = j->shadow_mask;
  o.no_sync = true;
  rc = trx_init(&sl.ctx, d.N, d.dims, d.ranks, X, d.x_dtype, cores, d.variant, s, o);
  if (rc) {
    sl.err = "context creation failed: " + std::string(tr_als_strerror(rc));
    return rc;
  }
  rc = trx_run_async(sl.ctx, d.nsweeps_mixed, d.prec_mixed, d.nsweeps_fin, d.prec_fin, d.refine, (int*)sl.pinned,
                     (double*)(sl.pinned + 16));
  if (rc) {
    sl.err = tr_als_last_error(sl.ctx);
    return rc;
  }
  size_t po = PIN_HEAD;
  for (int k = 0; k < d.N; ++k) {
    if (hipMemcpyAsync(sl.pinned + po, cores[k], core_elems(d, k) * 8, hipMemcpyDeviceToHost, s) != hipSuccess) {
      sl.err = "copy of the final cores failed";
      return TR_EHIP;
    }
    po += core_elems(d, k) * 8;
  }
  if (hipEventRecord(sl.done, s) != hipSuccess) {
    sl.err = "event record failed";
    return TR_EHIP;
  }
  return TR_OK;
}

// Results of a finished (or failed-to-enqueue) job, read from the slot.
struct JobOut {
  int rc = TR_OK;
  double rel_err = NAN;
  std::vector<std::vector<double>> cores;
  std::string err;
};

JobOut finish_job(Slot& sl) {
  JobOut r;
  const tr_job_desc& d = sl.job->d;
  r.rc = sl.rc;
  r.err = sl.err;
  // nothing of the job may still run when its region is handed out again
  if (hipStreamSynchronize(sl.s2) != hipSuccess || hipStreamSynchronize(sl.s) != hipSuccess) {
    (void)hipGetLastError();
    if (r.rc == TR_OK) { r.rc = TR_EHIP; r.err = "stream synchronisation failed"; }
  }
  if (r.rc == TR_OK) {
    const int st = *(const int*)sl.pinned;
    const double* sc = (const double*)(sl.pinned + 16);
    if (st) {
      r.rc = (st & ST_SINGULAR) ? TR_ESINGULAR : TR_ENONFINITE;
      r.err = trx_status_text(st);
    } else {
      r.rel_err = sc[0] > 0 ? std::sqrt(std::max(0.0, sc[1])) / std::sqrt(sc[0]) : 0.0;
    }
    // final cores (the last good ones after a solve failure)
    r.cores.resize(d.N);
    size_t po = PIN_HEAD;
    for (int k = 0; k < d.N; ++k) {
      const double* src = (const double*)(sl.pinned + po);
      r.cores[k].assign(src, src + core_elems(d, k));
      po += core_elems(d, k) * 8;
    }
  }
  if (sl.ctx) tr_als_destroy(sl.ctx);
  sl.ctx = nullptr;
  sl.rc = TR_OK;
  sl.err.clear();
  return r;
}

// Admission: arrived jobs in arrival order, each needing one contiguous arena
// region of its footprint and a free slot (small jobs of a batching server: a
// place in a batch lane; the jobs admitted to an idle lane in one pass form its
// next batch).  When the oldest arrived regular job does not fit, later jobs
// with footprint <= arena/64 may go first, for at most HEAD_MAX_WAIT_S seconds
// of the head's waiting.  Called with the lock held; returns the slots and
// lanes that received work and the next future arrival (or -1).
void admit(tr_srv* srv, std::vector<int>* started, std::vector<int>* lanes_started, double* next_arrival) {
  const double now = srv->now();
  *next_arrival = -1;
  bool head = true, backfill_ok = true;
  int forming = -1;
  for (size_t q = 0; q < srv->pending.size();) {
    Job* j = srv->pending[q];
    if (j->t_arrival > now) { *next_arrival = j->t_arrival; break; }
    size_t off = 0;
    if (j->tiny) {
      if (forming < 0 || srv->lanes[forming].jobs.size() >= (size_t)LANE_MAX) {
        forming = -1;
        for (size_t k = 0; k < srv->lanes.size(); ++k)
          if (srv->lanes[k].jobs.empty()) { forming = (int)k; break; }
      }
      if (forming < 0 || !srv->arena.alloc(j->footprint, &off)) { ++q; continue; }
      // a lane is started only once it holds a job: an idle lane picked while
      // memory is full must not be launched with an empty batch
      if (srv->lanes[forming].jobs.empty()) lanes_started->push_back(forming);
      j->off = off;
      j->slot = forming;
      j->state = TR_JOB_RUNNING;
      j->t_admit = now;
      srv->lanes[forming].jobs.push_back(j);
      srv->running++;
      srv->max_running = std::max(srv->max_running, srv->running);
      srv->pending.erase(srv->pending.begin() + q);
      continue;
    }
    int free_slot = -1;
    for (size_t k = 0; k < srv->slots.size(); ++k)
      if (!srv->slots[k].job) { free_slot = (int)k; break; }
    if (free_slot < 0) { ++q; continue; }
    const bool small = j->footprint <= srv->arena.cap / 64;
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
    started->push_back(free_slot);
  }
}

// Generate (or borrow) each job's X and initial cores in its arena region and
// enqueue the lane's batch: descriptors to the device, one persistent launch,
// results to pinned memory, completion event.
int start_batch(tr_srv* srv, Lane& ln) {
  hipStream_t s = ln.s;
  if (ln.jobs.empty()) return TR_OK;
  size_t need = 0;
  for (const Job* j : ln.jobs) {
    need += PIN_HEAD;
    for (int k = 0; k < j->d.N; ++k) need += core_elems(j->d, k) * 8;
  }
  if (need > ln.pinned_bytes) {
    void* p = nullptr;
    const size_t want = std::max(need, 2 * ln.pinned_bytes);
    if (hipHostMalloc(&p, want, 0) != hipSuccess) {
      (void)hipGetLastError();
      ln.err = "pinned host allocation failed";
      return TR_ENOMEM;
    }
    if (ln.pinned) srv->old_pinned.push_back(ln.pinned);
    ln.pinned = (char*)p;
    ln.pinned_bytes = want;
  }
  std::vector<std::vector<double*>> cores_of(ln.jobs.size());
  for (size_t q = 0; q < ln.jobs.size(); ++q) {
    const Job* j = ln.jobs[q];
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
    for (int k = 0; k < d.N; ++k) cores[k] = (double*)carve(core_elems(d, k) * 8);
    char* shared = base + off;   // generator workspace, then the batch kernel's scratch
    if (!d.X) {
      const int rc = trx_gen(d.N, d.dims, d.ranks, d.seed, d.eta, X, d.x_dtype, nullptr,
                             d.init_cores ? nullptr : cores, shared, j->bytes_gen, s, &ln.err);
      if (rc) return rc;
    } else if (!d.init_cores) {
      for (int k = 0; k < d.N; ++k)
        if (launch_philox_normal(cores[k], (int64_t)core_elems(d, k), d.seed, GEN_SID_INIT + k, s) != hipSuccess) {
          ln.err = "initial-core generation failed";
          return TR_EHIP;
        }
    }
    if (d.init_cores)
      for (int k = 0; k < d.N; ++k)
        if (hipMemcpyAsync(cores[k], j->init_ptrs[k], core_elems(d, k) * 8, hipMemcpyDeviceToDevice, s) !=
            hipSuccess) {
          ln.err = "copy of the initial cores failed";
          return TR_EHIP;
        }
    tiny_fill(&ln.h_desc[q], d.N, d.dims, d.ranks, X, d.x_dtype, cores, (double*)shared, d.nsweeps_mixed,
              d.prec_mixed, d.nsweeps_fin, d.prec_fin, d.refine);
    cores_of[q].assign(cores, cores + d.N);
  }
  const int n = (int)ln.jobs.size();
  if (hipMemcpyAsync(ln.d_desc, ln.h_desc, n * sizeof(TinyJob), hipMemcpyHostToDevice, s) != hipSuccess ||
      launch_tiny_als(ln.d_desc, n, s) != hipSuccess) {
    ln.err = "batch launch failed";
    return TR_EHIP;
  }
  size_t po = 0;
  for (size_t q = 0; q < ln.jobs.size(); ++q) {
    const tr_job_desc& d = ln.jobs[q]->d;
    if (hipMemcpyAsync(ln.pinned + po, ln.h_desc[q].status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(ln.pinned + po + 16, ln.h_desc[q].scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess) {
      ln.err = "copy of the results failed";
      return TR_EHIP;
    }
    po += PIN_HEAD;
    for (int k = 0; k < d.N; ++k) {
      if (hipMemcpyAsync(ln.pinned + po, cores_of[q][k], core_elems(d, k) * 8, hipMemcpyDeviceToHost, s) !=
          hipSuccess) {
        ln.err = "copy of the final cores failed";
        return TR_EHIP;
      }
      po += core_elems(d, k) * 8;
    }
  }
  if (hipEventRecord(ln.done, s) != hipSuccess) {
    ln.err = "event record failed";
    return TR_EHIP;
  }
  return TR_OK;
}

std::vector<JobOut> finish_batch(Lane& ln) {
  std::vector<JobOut> out(ln.jobs.size());
  const bool sync_ok = hipStreamSynchronize(ln.s) == hipSuccess;
  if (!sync_ok) (void)hipGetLastError();
  size_t po = 0;
  for (size_t q = 0; q < ln.jobs.size(); ++q) {
    JobOut& r = out[q];
    const tr_job_desc& d = ln.jobs[q]->d;
    if (ln.rc != TR_OK || !sync_ok) {
      r.rc = ln.rc != TR_OK ? ln.rc : TR_EHIP;
      r.err = ln.rc != TR_OK ? ln.err : "stream synchronisation failed";
      continue;
    }
    const int st = *(const int*)(ln.pinned + po);
    const double* sc = (const double*)(ln.pinned + po + 16);
    if (st) {
      r.rc = (st & ST_SINGULAR) ? TR_ESINGULAR : TR_ENONFINITE;
      r.err = trx_status_text(st);
    } else {
      r.rel_err = sc[0] > 0 ? std::sqrt(std::max(0.0, sc[1])) / std::sqrt(sc[0]) : 0.0;
    }
    po += PIN_HEAD;
    r.cores.resize(d.N);
    for (int k = 0; k < d.N; ++k) {
      const double* src = (const double*)(ln.pinned + po);
      r.cores[k].assign(src, src + core_elems(d, k));
      po += core_elems(d, k) * 8;
    }
  }
  ln.rc = TR_OK;
  ln.err.clear();
  return out;
}

void commit_job(tr_srv* srv, Job* j, JobOut& r) {
  srv->arena.release(j->off, j->footprint);
  j->rel_err = r.rel_err;
  j->cores = std::move(r.cores);
  j->err = std::move(r.err);
  j->status = r.rc;
  j->state = r.rc == TR_OK ? TR_JOB_DONE : TR_JOB_FAILED;
  j->t_done = srv->now();
  if (r.rc == TR_OK) srv->n_done++;
  else srv->n_failed++;
  srv->running--;
}

// The executor: the only thread that calls HIP.  It admits jobs, enqueues each
// admitted job's whole work on its slot, and polls the slots' completion
// events; queued jobs are dropped and running ones finished when stopping.
void exec_main(tr_srv* srv) {
  (void)hipSetDevice(srv->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    if (srv->stop && srv->running == 0) break;
    std::vector<int> started, lanes_started;
    double next_arrival = -1;
    const uint64_t seen = srv->gen;
    if (!srv->stop) admit(srv, &started, &lanes_started, &next_arrival);
    lk.unlock();
    for (int k : started) {
      Slot& sl = srv->slots[k];
      sl.rc = start_job(srv, sl);
      if (sl.rc != TR_OK) (void)hipGetLastError();
    }
    for (int k : lanes_started) {
      Lane& ln = srv->lanes[k];
      ln.rc = start_batch(srv, ln);
      if (ln.rc != TR_OK) (void)hipGetLastError();
    }
    // completions
    std::vector<std::pair<int, JobOut>> finished;
    for (size_t k = 0; k < srv->slots.size(); ++k) {
      Slot& sl = srv->slots[k];
      if (!sl.job) continue;
      bool ready = sl.rc != TR_OK;
      if (!ready) {
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipSuccess) ready = true;
        else if (q != hipErrorNotReady) {
          (void)hipGetLastError();
          sl.rc = TR_EHIP;
          sl.err = "completion event failed";
          ready = true;
        }
      }
      if (ready) finished.emplace_back((int)k, finish_job(sl));
    }
    std::vector<std::pair<int, std::vector<JobOut>>> lanes_finished;
    for (size_t k = 0; k < srv->lanes.size(); ++k) {
      Lane& ln = srv->lanes[k];
      if (ln.jobs.empty()) continue;
      bool ready = ln.rc != TR_OK;
      if (!ready) {
        const hipError_t q = hipEventQuery(ln.done);
        if (q == hipSuccess) ready = true;
        else if (q != hipErrorNotReady) {
          (void)hipGetLastError();
          ln.rc = TR_EHIP;
          ln.err = "completion event failed";
          ready = true;
        }
      }
      if (ready) lanes_finished.emplace_back((int)k, finish_batch(ln));
    }
    lk.lock();
    for (auto& f : finished) {
      Slot& sl = srv->slots[f.first];
      commit_job(srv, sl.job, f.second);
      sl.job = nullptr;
    }
    for (auto& f : lanes_finished) {
      Lane& ln = srv->lanes[f.first];
      for (size_t q = 0; q < ln.jobs.size(); ++q) commit_job(srv, ln.jobs[q], f.second[q]);
      ln.jobs.clear();
    }
    if (!finished.empty() || !lanes_finished.empty()) srv->cv_done.notify_all();
    if (!started.empty() || !finished.empty() || !lanes_started.empty() || !lanes_finished.empty()) continue;
    // A submit (or stop) while the lock was released notified nobody: its job
    // is not in next_arrival, so admit again instead of waiting.
    if (srv->gen != seen) continue;
    if (srv->running > 0) {
      srv->cv_exec.wait_for(lk, POLL);
    } else {
      // idle: until the next arrival or a submit, and never longer than IDLE_MAX
      const auto until = std::min(Clock::now() + IDLE_MAX,
                                  next_arrival >= 0 ? srv->t0 + std::chrono::duration_cast<Clock::duration>(
                                                                    std::chrono::duration<double>(next_arrival))
                                                    : Clock::time_point::max());
      srv->cv_exec.wait_until(lk, until);
    }
  }
}

void release_slots(tr_srv* srv) {
  for (auto& sl : srv->slots) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    if (sl.s2) (void)hipStreamSynchronize(sl.s2);
    if (sl.s) (void)hipStreamDestroy(sl.s);
    if (sl.s2) (void)hipStreamDestroy(sl.s2);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    sl = Slot();
  }
  for (auto& ln : srv->lanes) {
    if (ln.s) (void)hipStreamSynchronize(ln.s);
    if (ln.s) (void)hipStreamDestroy(ln.s);
    if (ln.done) (void)hipEventDestroy(ln.done);
    if (ln.h_desc) (void)hipHostFree(ln.h_desc);
    if (ln.d_desc) (void)hipFree(ln.d_desc);
    if (ln.pinned) (void)hipHostFree(ln.pinned);
    ln = Lane();
  }
  for (char* p : srv->old_pinned) (void)hipHostFree(p);
  srv->old_pinned.clear();
}

int validate(const tr_job_desc& d) {
  if (d.N < 2 || d.N > TR_MAXN) return TR_EINVAL;
  for (int k = 0; k < d.N; ++k)
    if (d.dims[k] < 1 || d.ranks[k] < 1 || d.ranks[k] > TR_MAXR) return TR_EINVAL;
  if (d.variant != TR_NE && d.variant != TR_QR && d.variant != TR_QRNE) return TR_EINVAL;
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
  int rc = TR_OK;
  for (auto& sl : srv->slots) {
    void* pin = nullptr;
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sl.s2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      rc = TR_EHIP;
      break;
    }
    if (hipHostMalloc(&pin, PIN_DEFAULT, 0) != hipSuccess) {
      rc = TR_ENOMEM;
      break;
    }
    sl.pinned = (char*)pin;
    sl.pinned_bytes = PIN_DEFAULT;
  }
  if (rc == TR_OK && (flags & TR_SRV_BATCH)) {
    srv->lanes.resize(NLANES);
    for (auto& ln : srv->lanes) {
      void* h = nullptr;
      void* pin = nullptr;
      void* dd = nullptr;
      if (hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess) {
        rc = TR_EHIP;
        break;
      }
      if (hipHostMalloc(&h, LANE_MAX * sizeof(TinyJob), 0) != hipSuccess ||
          hipHostMalloc(&pin, PIN_DEFAULT, 0) != hipSuccess || hipMalloc(&dd, LANE_MAX * sizeof(TinyJob)) != hipSuccess) {
        if (h) (void)hipHostFree(h);
        if (pin) (void)hipHostFree(pin);
        rc = TR_ENOMEM;
        break;
      }
      ln.h_desc = (TinyJob*)h;
      ln.d_desc = (TinyJob*)dd;
      ln.pinned = (char*)pin;
      ln.pinned_bytes = PIN_DEFAULT;
    }
  }
  if (rc) {
    (void)hipGetLastError();
    release_slots(srv.get());
    (void)hipFree(base);
    return rc;
  }
  srv->t0 = Clock::now();
  tr_srv* p = srv.release();
  p->exec = std::thread(exec_main, p);
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
  auto lane_prec = [](int p) { return p == TR_F64 || p == TR_F32 || p == TR_BF16; };
  j->tiny = (srv->flags & TR_SRV_BATCH) && d.variant == TR_NE && tiny_eligible(d.N, d.dims, d.ranks) &&
            (d.nsweeps_mixed == 0 || lane_prec(d.prec_mixed)) && (d.nsweeps_fin == 0 || lane_prec(d.prec_fin));
  j->bytes_ctx = j->tiny ? trx_round(tiny_ws_bytes(d.N, d.dims, d.ranks))
                         : trx_footprint(d.N, d.dims, d.ranks, d.x_dtype, d.variant, j->shadow_mask);
  if (j->bytes_ctx == 0 || (!d.X && j->bytes_gen == 0)) return TR_EINVAL;
  j->footprint = j->bytes_x + j->bytes_cores + std::max(j->bytes_gen, j->bytes_ctx);
  if (j->footprint > srv->arena.cap) return TR_ENOMEM;
  std::lock_guard<std::mutex> lk(srv->mu);
  const double now = srv->now();
  j->t_arrival = std::max(d.t_arrival, now);
  j->id = srv->next_id++;
  Job* jp = j.get();
  srv->jobs[jp->id] = std::move(j);
  srv->gen++;
  auto pos = std::upper_bound(srv->pending.begin(), srv->pending.end(), jp, [](const Job* a, const Job* b) {
    return a->t_arrival < b->t_arrival || (a->t_arrival == b->t_arrival && a->id < b->id);
  });
  srv->pending.insert(pos, jp);
  *job_id = jp->id;
  srv->cv_exec.notify_one();
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
  info->batched = j.tiny ? 1 : 0;
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
    srv->gen++;
    for (Job* j : srv->pending) {
      j->state = TR_JOB_FAILED;
      j->status = TR_EINVAL;
      j->err = "server destroyed before the job was admitted";
    }
    srv->pending.clear();
  }
  srv->cv_exec.notify_all();
  srv->cv_done.notify_all();
  if (srv->exec.joinable()) srv->exec.join();
  release_slots(srv);
  if (srv->arena.base) (void)hipFree(srv->arena.base);
  delete srv;
  return TR_OK;
}

}  // extern "C"
