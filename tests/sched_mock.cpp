// Host-only replay of the request loop's admission policy (admission.h) with a
// mock executor: worker threads take jobs exactly as the server's workers
// do, and "run" them against a fake device of fixed memory, where a job
// whose true peak does not fit what is left fails with out-of-memory.
//
// Input (stdin): one line "budget device_bytes workers time_scale
// exclusive_above", then
// one line per job "arrival_s footprint true_peak duration_s", in
// submission order.  Output: one line per job "id status attempts
// first_start_rank", then "ok" — or, if the jobs do not all finish within
// the deadline, the scheduler state and exit code 3.  Exit code 2 flags a
// broken invariant (fake device over capacity, a job started out of FIFO
// order, a shared start over the budget).
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

#include "admission.h"

namespace {

struct MockJob {
  uint64_t id = 0;
  double arrival = 0, duration = 0;
  uint64_t footprint = 0, peak = 0;
  bool alone = false;
  uint64_t adm_seq = 0;
  bool adm_shared = false;
  int status = 1;  // 1 waiting, 2 running, 0 done, -3 out of memory
  int attempts = 0;
  int64_t first_start = -1;
};

struct FakeDevice {
  std::mutex mu;
  uint64_t cap = 0, used = 0, high = 0;
  bool take(uint64_t b) {
    std::lock_guard<std::mutex> lk(mu);
    if (used + b > cap) return false;
    used += b;
    high = std::max(high, used);
    return true;
  }
  void give(uint64_t b) {
    std::lock_guard<std::mutex> lk(mu);
    used -= b;
  }
};

void fail(const char* what) {
  std::printf("invariant broken: %s\n", what);
  std::fflush(stdout);
  std::_Exit(2);
}

}  // namespace

int main() {
  uint64_t budget = 0, device = 0;
  unsigned workers = 0;
  double scale = 1.0;
  uint64_t exclusive_above = 0;
  if (std::scanf("%lu %lu %u %lf %lu", &budget, &device, &workers, &scale, &exclusive_above) != 5) return 1;
  std::vector<MockJob> jobs;
  MockJob j;
  while (std::scanf("%lf %lu %lu %lf", &j.arrival, &j.footprint, &j.peak, &j.duration) == 4) {
    j.id = jobs.size();
    jobs.push_back(j);
  }

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  sdbg_sched::Admission<MockJob*> adm(budget, exclusive_above);
  FakeDevice dev;
  dev.cap = device;
  bool stopping = false;
  size_t done = 0;
  int64_t starts = 0;
  uint64_t next_first = 0;  // FIFO: first attempts start in submission order
  bool running_alone = false;

  auto worker = [&]() {
    for (;;) {
      MockJob* x = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stopping || adm.head_admissible(); });
        if (stopping) return;
        x = adm.start_head();
        if (x->attempts == 0) {
          if (x->id != next_first) fail("a job started before an earlier one");
          ++next_first;
          x->first_start = starts;
        }
        ++starts;
        ++x->attempts;
        x->status = 2;
        if (adm.running() > 1 && adm.mem_in_use() > adm.budget()) fail("shared start over the budget");
        if (adm.running() > 1 && (x->alone || running_alone))
          fail("a job that must run alone shares the device");
        if (adm.exclusive(x)) running_alone = true;
        cv_work.notify_all();
      }
      // mock executor: the job's true peak must fit what the device has left
      const bool fits = dev.take(x->peak);
      if (fits) {
        std::this_thread::sleep_for(std::chrono::duration<double>(x->duration * scale));
        dev.give(x->peak);
      } else {
        std::this_thread::sleep_for(std::chrono::duration<double>(x->duration * scale * 0.1));
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        if (adm.exclusive(x)) running_alone = false;
        if (!adm.finish(x, !fits)) {
          x->status = fits ? 0 : -3;
          ++done;
        } else {
          x->status = 1;
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  };
  std::vector<std::thread> ws;
  for (unsigned i = 0; i < workers; ++i) ws.emplace_back(worker);

  const auto t0 = std::chrono::steady_clock::now();
  std::thread submitter([&]() {
    for (auto& x : jobs) {
      std::this_thread::sleep_until(t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                             std::chrono::duration<double>(x.arrival * scale)));
      std::lock_guard<std::mutex> lk(mu);
      adm.push(&x);
      cv_work.notify_all();
    }
  });
  submitter.join();

  bool finished;
  {
    std::unique_lock<std::mutex> lk(mu);
    finished = cv_done.wait_for(lk, std::chrono::seconds(20), [&] { return done == jobs.size(); });
    if (!finished) {
      std::printf("deadline passed: %zu of %zu done, queued %zu, running %u, mem_in_use %lu of %lu\n", done,
                  jobs.size(), adm.queued(), adm.running(), adm.mem_in_use(), adm.budget());
      for (auto& x : jobs)
        std::printf("job %lu status %d attempts %d alone %d\n", x.id, x.status, x.attempts, (int)x.alone);
    }
    stopping = true;
  }
  cv_work.notify_all();
  for (auto& t : ws) t.join();
  if (!finished) return 3;
  if (dev.high > dev.cap) fail("fake device over capacity");
  for (auto& x : jobs) std::printf("%lu %d %d %ld\n", x.id, x.status, x.attempts, (long)x.first_start);
  std::printf("ok\n");
  return 0;
}
