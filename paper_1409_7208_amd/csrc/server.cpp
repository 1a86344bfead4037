// Served form: a request loop that runs construction jobs concurrently on
// one device.
//
// Jobs are copied into pinned host memory at submit and wait in a FIFO
// queue.  A fixed set of workers, each with its own HIP stream, takes the
// head of the queue as soon as the device memory it needs fits the budget
// next to the jobs already running (a job that fits no budget runs alone),
// so jobs that arrive while others are on the device start as soon as a
// worker and memory are free and their kernels overlap with the running
// ones (continuous batching).  Device buffers come from the library's
// caching pool, so they stay resident between jobs instead of being
// allocated per job.  Each job runs exactly the single-call path
// (sdbg_count_solid, then sdbg_build), so its results do not depend on what
// else is running.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "abi_common.h"
#include "admission.h"

namespace {

using Clock = std::chrono::steady_clock;

enum { kWaiting = 1, kRunning = 2 };

struct Job {
  uint64_t id = 0;
  uint8_t* seq = nullptr;  // pinned host copies of the reads
  uint64_t* off = nullptr;
  uint64_t n_reads = 0, n_bases = 0;
  sdbg_params params{};
  uint64_t footprint = 0;
  bool alone = false;  // retry after running out of device memory: run alone
  uint64_t adm_seq = 0;     // admission bookkeeping (admission.h)
  bool adm_shared = false;
  const sdbg::Trace* trace = nullptr;  // the worker's record while running
  int status = kWaiting;
  std::string err;
  sdbg_job_stats stats{};
  sdbg_edges* edges = nullptr;
  sdbg_graph* graph = nullptr;
};

// Device bytes a job may need at its peak: per (k+1)-mer occurrence bound,
// the two key buffers and counts of the partition, the mercy lookup table
// and the edge-set merges (measured peaks of the library's pool, outputs
// included: about 12 bytes per occurrence for one-word keys, which are
// counted on one strand, and 42-51, 72-77 and 94-103 bytes for two-, three-
// and four-word keys), with a margin; plus the reads and a constant for
// small jobs.
uint64_t job_footprint(uint64_t occ, uint64_t bases, uint32_t k) {
  const uint64_t w = (uint64_t)sdbg::key_words((int)k);
  const uint64_t per_occ = w == 1 ? 24 : 28 * w + 16;
  return occ * per_occ + 3 * bases + (64ull << 20);
}

// Jobs whose footprint exceeds this run alone.  A replay of the serving
// workload with four jobs at once stalled for minutes on a job of 8.2M reads
// at k = 61 (53 GB footprint) that had started next to others, while the
// same job alone finishes in well under a second; until the cause is known,
// large jobs do not share the device.
constexpr uint64_t kExclusiveBytes = 8ull << 30;

// Pinned host staging, kept for reuse: freeing pinned memory can wait for
// the whole device, which would stall the jobs still running.
class PinnedPool {
 public:
  void* get(size_t bytes) {
    bytes = (bytes + 4095) & ~size_t(4095);
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = free_.lower_bound(bytes);
      if (it != free_.end() && it->first <= 2 * bytes + (1u << 20)) {
        void* p = it->second;
        free_.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      throw sdbg::Error(SDBG_E_NOMEM, "pinned host allocation failed");
    }
    std::lock_guard<std::mutex> lk(mu_);
    size_[p] = bytes;
    return p;
  }
  void put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.emplace(size_[p], p);
  }
  ~PinnedPool() {
    for (auto& kv : size_) (void)hipHostFree(kv.first);
  }

 private:
  std::mutex mu_;
  std::multimap<size_t, void*> free_;
  std::unordered_map<void*, size_t> size_;
};

}  // namespace

struct sdbg_server {
  sdbg_server_cfg cfg{};
  int device = 0;
  uint64_t budget = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  sdbg_sched::Admission<Job*> adm{0};  // guarded by mu
  std::unordered_map<uint64_t, Job*> jobs;
  uint64_t next_id = 1;
  bool stopping = false;
  std::vector<std::thread> workers;
  PinnedPool pinned;

  void free_pinned(Job* j) {
    pinned.put(j->seq);
    pinned.put(j->off);
    j->seq = nullptr;
    j->off = nullptr;
  }

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  void run_job(Job* j, hipStream_t s) {
    sdbg::EdgesOut eo;
    sdbg::GraphOut go;
    sdbg_edges* e = nullptr;
    int rc = sdbg_abi::guarded([&]() -> int {
      sdbg::Ctx c(s);
      {
        sdbg::DevReads R{};
        R.n_reads = j->n_reads;
        R.n_bases = j->n_bases;
        sdbg::DBuf<uint8_t> seq_d = c.buf<uint8_t>(j->n_bases + 16);
        sdbg::DBuf<uint64_t> off_d = c.buf<uint64_t>(j->n_reads + 1);
        c.h2d(seq_d.get(), j->seq, j->n_bases);
        c.h2d(off_d.get(), j->off, j->n_reads + 1);
        R.seq = seq_d.get();
        R.offsets = off_d.get();
        sdbg::CountParams P{(int)j->params.k, j->params.d, j->params.mercy != 0, (int)j->params.prefix_len,
                            j->params.mem_budget};
        // A job that shares the device plans its partition within the
        // memory it was admitted with, not within what is free right now.
        if (!P.mem_budget && !j->alone && j->footprint <= budget) P.mem_budget = j->footprint;
        sdbg::count_solid(R, P, c, &eo);
        c.sync();
      }
      e = sdbg_abi::wrap_edges(eo, j->params.k);
      if (cfg.build) {
        sdbg::build_graph(e->keys, e->count, e->n, (int)j->params.k, c, &go, false);
        c.sync();
        j->graph = sdbg_abi::wrap_graph(go, j->params.k);
      }
      return SDBG_OK;
    });
    j->edges = e;
    if (rc != SDBG_OK) {
      j->err = sdbg_abi::t_err;
      if (e) sdbg_free(e);
      j->edges = nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    j->trace = nullptr;
    if (adm.finish(j, rc == SDBG_E_NOMEM_DEVICE)) {
      // Device memory ran out next to other jobs: queued again at the head,
      // to run when the device is otherwise idle.
      j->status = kWaiting;
      j->err.clear();
    } else {
      j->stats.end_s = now();
      j->stats.n_occ = j->edges ? j->edges->n_occ : 0;
      j->status = rc;
      j->stats.status = rc;
      free_pinned(j);
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }

  void worker() {
    (void)hipSetDevice(device);
    sdbg::Trace trace;
    sdbg::current_trace() = &trace;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    for (;;) {
      Job* j = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stopping || adm.head_admissible(); });
        if (stopping) break;
        j = adm.start_head();
        j->status = kRunning;
        trace.stage.store("start");
        trace.activity.store("");
        j->trace = &trace;
        j->stats.status = kRunning;
        j->stats.start_s = now();
        cv_work.notify_all();  // the next head may fit too
      }
      run_job(j, s);
    }
    if (s) (void)hipStreamDestroy(s);
  }
};

extern "C" {

int sdbg_job_footprint(const sdbg_reads* reads, const sdbg_params* params, uint64_t* bytes) {
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(reads && params && bytes, SDBG_E_INVAL, "null argument");
    SDBG_CHECK(!reads->on_device, SDBG_E_INVAL, "the request loop takes host reads");
    sdbg_abi::check_params(params);
    SDBG_CHECK(reads->n_reads == 0 || reads->offsets, SDBG_E_INVAL, "null offsets");
    std::vector<uint64_t> o(reads->n_reads + 1, 0);
    if (reads->n_reads) std::memcpy(o.data(), reads->offsets, sizeof(uint64_t) * (reads->n_reads + 1));
    SDBG_CHECK(o[0] == 0, SDBG_E_INVAL, "offsets[0] must be 0");
    *bytes = job_footprint(sdbg_abi::occ_bound(o, params->k), o.back(), params->k);
    return SDBG_OK;
  });
}

int sdbg_server_trace(sdbg_server* sv, uint64_t job_id, const char** stage, const char** activity, double* seconds) {
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(sv && stage && activity && seconds, SDBG_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(job_id);
    SDBG_CHECK(it != sv->jobs.end(), SDBG_E_INVAL, "unknown job id");
    const sdbg::Trace* t = it->second->trace;
    *stage = t ? t->stage.load() : "";
    *activity = t ? t->activity.load() : "";
    const int64_t ns = std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
    *seconds = t ? (double)(ns - t->since_ns.load()) * 1e-9 : 0.0;
    return SDBG_OK;
  });
}

int sdbg_server_state(sdbg_server* sv, sdbg_server_info* info) {
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(sv && info, SDBG_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    info->budget = sv->adm.budget();
    info->mem_in_use = sv->adm.mem_in_use();
    info->queued = (uint32_t)sv->adm.queued();
    info->running = sv->adm.running();
    info->jobs = sv->jobs.size();
    info->uptime_s = sv->now();
    return SDBG_OK;
  });
}

int sdbg_server_start(const sdbg_server_cfg* cfg, sdbg_server** out) {
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(out, SDBG_E_INVAL, "null argument");
    *out = nullptr;
    SDBG_CHECK(!cfg || cfg->max_jobs <= 64, SDBG_E_INVAL, "max_jobs must be at most 64");
    sdbg_server* sv = new sdbg_server();
    if (cfg) sv->cfg = *cfg;
    if (!sv->cfg.max_jobs) sv->cfg.max_jobs = 4;
    if (!sv->cfg.queue_cap) sv->cfg.queue_cap = 4096;
    try {
      SDBG_HIP(hipGetDevice(&sv->device));
      sdbg_params p{};
      p.mem_budget = sv->cfg.mem_budget;
      sv->budget = sdbg_abi::device_budget(&p);
      sv->adm = sdbg_sched::Admission<Job*>(sv->budget, kExclusiveBytes);
      sv->t0 = Clock::now();
      for (uint32_t i = 0; i < sv->cfg.max_jobs; ++i) sv->workers.emplace_back([sv] { sv->worker(); });
    } catch (...) {
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
      }
      sv->cv_work.notify_all();
      for (auto& t : sv->workers) t.join();
      delete sv;
      throw;
    }
    *out = sv;
    return SDBG_OK;
  });
}

int sdbg_server_submit(sdbg_server* sv, const sdbg_reads* reads, const sdbg_params* params, uint64_t* job_id) {
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(sv && reads && params && job_id, SDBG_E_INVAL, "null argument");
    SDBG_CHECK(!reads->on_device, SDBG_E_INVAL, "the request loop takes host reads");
    sdbg_abi::check_params(params);
    SDBG_CHECK(reads->n_reads == 0 || reads->offsets, SDBG_E_INVAL, "null offsets");
    std::vector<uint64_t> o(reads->n_reads + 1, 0);
    if (reads->n_reads) {
      std::memcpy(o.data(), reads->offsets, sizeof(uint64_t) * (reads->n_reads + 1));
      SDBG_CHECK(o[0] == 0, SDBG_E_INVAL, "offsets[0] must be 0");
      for (uint64_t i = 0; i < reads->n_reads; ++i)
        SDBG_CHECK(o[i + 1] >= o[i], SDBG_E_INVAL, "offsets must be non-decreasing");
      SDBG_CHECK(o.back() == 0 || reads->seq, SDBG_E_INVAL, "null seq");
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      SDBG_CHECK(!sv->stopping, SDBG_E_INVAL, "server is stopping");
      if (sv->adm.queued() >= sv->cfg.queue_cap) throw sdbg::Error(SDBG_E_BUSY, "queue full");
    }
    Job* j = new Job();
    j->n_reads = reads->n_reads;
    j->n_bases = o.back();
    j->params = *params;
    j->params.stream = nullptr;
    j->footprint = job_footprint(sdbg_abi::occ_bound(o, params->k), j->n_bases, params->k);
    try {
      j->seq = static_cast<uint8_t*>(sv->pinned.get(j->n_bases + 16));
      j->off = static_cast<uint64_t*>(sv->pinned.get(sizeof(uint64_t) * (j->n_reads + 1)));
    } catch (...) {
      sv->free_pinned(j);
      delete j;
      throw;
    }
    if (j->n_bases) std::memcpy(j->seq, reads->seq, j->n_bases);
    std::memcpy(j->off, o.data(), sizeof(uint64_t) * (j->n_reads + 1));
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (sv->stopping || sv->adm.queued() >= sv->cfg.queue_cap) {
        const bool stop = sv->stopping;
        sv->free_pinned(j);
        delete j;
        throw sdbg::Error(stop ? SDBG_E_INVAL : SDBG_E_BUSY, stop ? "server is stopping" : "queue full");
      }
      j->id = sv->next_id++;
      j->stats.status = kWaiting;
      j->stats.submit_s = sv->now();
      j->stats.footprint = j->footprint;
      sv->jobs[j->id] = j;
      sv->adm.push(j);
      *job_id = j->id;
    }
    sv->cv_work.notify_all();
    return SDBG_OK;
  });
}

int sdbg_server_poll(sdbg_server* sv, uint64_t job_id, int wait, sdbg_edges** edges, sdbg_graph** graph,
                     sdbg_job_stats* stats) {
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(sv, SDBG_E_INVAL, "null argument");
    if (edges) *edges = nullptr;
    if (graph) *graph = nullptr;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(job_id);
    SDBG_CHECK(it != sv->jobs.end(), SDBG_E_INVAL, "unknown job id");
    Job* j = it->second;
    if (wait) sv->cv_done.wait(lk, [&] { return j->status <= 0; });
    if (stats) *stats = j->stats;
    if (j->status > 0) return j->status;
    sv->jobs.erase(it);
    lk.unlock();
    const int rc = j->status;
    const std::string err = j->err;
    if (edges)
      *edges = j->edges;
    else if (j->edges)
      sdbg_free(j->edges);
    if (graph)
      *graph = j->graph;
    else if (j->graph)
      sdbg_free(j->graph);
    delete j;
    if (rc != SDBG_OK) throw sdbg::Error(rc, err);
    return SDBG_OK;
  });
}

int sdbg_server_cancel(sdbg_server* sv, uint64_t job_id) {
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(sv, SDBG_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(job_id);
    SDBG_CHECK(it != sv->jobs.end(), SDBG_E_INVAL, "unknown job id");
    Job* j = it->second;
    if (j->status != kWaiting || !sv->adm.cancel(j)) return SDBG_E_BUSY;
    j->status = SDBG_E_CANCELLED;
    j->stats.status = SDBG_E_CANCELLED;
    j->stats.end_s = sv->now();
    j->err = "cancelled";
    sv->free_pinned(j);
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
    return SDBG_OK;
  });
}

int sdbg_server_stop(sdbg_server* sv) {
  return sdbg_abi::guarded([&]() -> int {
    if (!sv) return SDBG_OK;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      for (Job* j : sv->adm.drain()) {
        j->status = SDBG_E_CANCELLED;
        j->stats.status = SDBG_E_CANCELLED;
        sv->free_pinned(j);
      }
      sv->cv_done.wait(lk, [&] { return sv->adm.running() == 0; });
      sv->stopping = true;
    }
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
    for (auto& t : sv->workers) t.join();
    for (auto& kv : sv->jobs) {
      Job* j = kv.second;
      if (j->edges) sdbg_free(j->edges);
      if (j->graph) sdbg_free(j->graph);
      sv->free_pinned(j);
      delete j;
    }
    delete sv;
    return SDBG_OK;
  });
}

}  // extern "C"
