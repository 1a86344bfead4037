// Admission policy of the request loop (server.cpp): a FIFO queue of jobs,
// each charged its device-memory footprint while it runs.  Pure host code
// with no HIP dependency, so that the policy can be driven by a mock
// executor on the CPU.  Not thread-safe: the caller holds its own lock
// around every call.
//
// Rules:
//   * only the head of the queue may start (FIFO, no overtaking);
//   * it starts when its footprint fits the budget next to the running jobs;
//   * a job larger than the whole budget, larger than the exclusive
//     threshold, or marked `alone` starts only when nothing else runs, and
//     nothing else starts while it runs;
//   * a job that ran out of device memory while another job ran at any time
//     during its run is marked `alone` and queued again at the head (the
//     others may have finished by the time it reports); out of memory when
//     it had the device to itself is final.
// Every waiting job eventually starts as long as running jobs finish: the
// head is admissible at the latest when nothing runs.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <vector>

namespace sdbg_sched {

// JobPtr: pointer to a job with `uint64_t footprint`, `bool alone` and
// `uint64_t adm_seq, adm_shared` (written here).
template <typename JobPtr>
class Admission {
 public:
  // exclusive_above: footprint above which a job runs alone (0 = none).
  explicit Admission(uint64_t budget, uint64_t exclusive_above = 0)
      : budget_(budget), exclusive_above_(exclusive_above) {}

  void push(JobPtr j) { q_.push_back(j); }

  bool head_admissible() const {
    if (q_.empty() || exclusive_) return false;
    const JobPtr j = q_.front();
    if (exclusive(j)) return running_ == 0;
    return mem_in_use_ + j->footprint <= budget_;
  }

  // Removes the head and charges its footprint (head_admissible() must hold).
  JobPtr start_head() {
    JobPtr j = q_.front();
    q_.pop_front();
    mem_in_use_ += j->footprint;
    ++running_;
    j->adm_seq = ++starts_;
    j->adm_shared = running_ > 1;
    exclusive_ = exclusive(j);
    return j;
  }

  // A running job ended.  Returns true if it was queued again (at the head)
  // to run alone, after running out of device memory next to other jobs.
  bool finish(JobPtr j, bool out_of_device_memory) {
    mem_in_use_ -= j->footprint;
    --running_;
    if (exclusive(j)) exclusive_ = false;
    // another job overlapped this one if one ran when it started, one still
    // runs, or one started after it
    const bool shared = j->adm_shared || running_ > 0 || starts_ != j->adm_seq;
    if (out_of_device_memory && !j->alone && shared) {
      j->alone = true;
      q_.push_front(j);
      return true;
    }
    return false;
  }

  // Removes a waiting job; false if it is not in the queue.
  bool cancel(JobPtr j) {
    auto it = std::find(q_.begin(), q_.end(), j);
    if (it == q_.end()) return false;
    q_.erase(it);
    return true;
  }

  // Removes and returns every waiting job.
  std::vector<JobPtr> drain() {
    std::vector<JobPtr> v(q_.begin(), q_.end());
    q_.clear();
    return v;
  }

  bool exclusive(const JobPtr j) const {
    return j->alone || j->footprint > budget_ || (exclusive_above_ && j->footprint > exclusive_above_);
  }

  size_t queued() const { return q_.size(); }
  uint32_t running() const { return running_; }
  uint64_t mem_in_use() const { return mem_in_use_; }
  uint64_t budget() const { return budget_; }

 private:
  std::deque<JobPtr> q_;
  uint64_t budget_;
  uint64_t exclusive_above_;
  uint64_t mem_in_use_ = 0;
  uint64_t starts_ = 0;
  uint32_t running_ = 0;
  bool exclusive_ = false;  // a job that must run alone is running
};

}  // namespace sdbg_sched
