#include "runtime.h"

#include <unordered_set>

#include "engine.h"

#include <algorithm>
#include <chrono>
#include <iterator>

namespace sdbg {

namespace {
constexpr int kMaxDevices = 64;
Pool g_pools[kMaxDevices];

size_t round_size(size_t b) {
  if (b <= (1u << 20)) return (b + 255) & ~size_t(255);
  return (b + (2u << 20) - 1) & ~size_t((2u << 20) - 1);
}
}  // namespace

Pool& Pool::get() {
  int dev = 0;
  SDBG_HIP(hipGetDevice(&dev));
  SDBG_CHECK(dev >= 0 && dev < kMaxDevices, -4, "device index out of range");
  return g_pools[dev];
}

void* Pool::alloc(size_t bytes, hipStream_t s) {
  size_t want = round_size(bytes);
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (fail_after_ >= 0 && fail_after_-- == 0)
      throw Error(-3, "device allocation of " + std::to_string(want) + " bytes failed (injected)");
    for (auto it = free_.lower_bound(want); it != free_.end() && it->first <= want + want / 2 + (4u << 20); ++it) {
      if (it->second.tagged && it->second.s != s) continue;
      void* p = it->second.p;
      cached_ -= it->first;
      in_use_ += it->first;
      peak_ = std::max(peak_, in_use_);
      if (it->second.tagged) tagged_at_.erase(p);
      free_.erase(it);
      return p;
    }
  }
  trace_activity("device allocation");
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
    const size_t reserve = std::max<size_t>(size_t(1) << 30, tot / 64);
    if (fr < want + reserve) trim();
  } else {
    (void)hipGetLastError();
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim();
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim_all();
      e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trace_activity("");
      throw Error(-3, "device allocation of " + std::to_string(want) + " bytes failed: " + hipGetErrorString(e));
    }
  }
  trace_activity("");
  std::lock_guard<std::mutex> lk(mu_);
  size_[p] = want;
  in_use_ += want;
  peak_ = std::max(peak_, in_use_);
  return p;
}

void Pool::release(void* p, hipStream_t s, bool tagged) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  auto it = size_.find(p);
  if (it == size_.end()) return;
  auto at = free_.emplace(it->second, Blk{p, s, tagged, ++releases_});
  if (tagged) {
    tags_[s].push_back(Tag{releases_, p});
    tagged_at_[p] = at;
  }
  cached_ += it->second;
  in_use_ -= it->second;
}

void Pool::untag(hipStream_t s, uint64_t upto) {
  std::lock_guard<std::mutex> lk(mu_);
  auto t = tags_.find(s);
  if (t == tags_.end()) return;
  std::vector<Tag>& L = t->second;
  size_t n = 0;  // release numbers grow along the list: untag a prefix
  for (; n < L.size() && L[n].id <= upto; ++n) {
    auto a = tagged_at_.find(L[n].p);
    if (a == tagged_at_.end() || a->second->second.id != L[n].id) continue;
    a->second->second.tagged = false;
    tagged_at_.erase(a);
  }
  L.erase(L.begin(), L.begin() + n);
  if (L.empty()) tags_.erase(t);
}

uint64_t Pool::release_mark() {
  std::lock_guard<std::mutex> lk(mu_);
  return releases_;
}

// Cached blocks no stream may still use are freed; hipFree can wait for the
// device, so it is called after the pool's lock is released.
void Pool::trim() {
  std::vector<void*> give;
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end();) {
      if (it->second.tagged) {
        ++it;
        continue;
      }
      give.push_back(it->second.p);
      size_.erase(it->second.p);
      cached_ -= it->first;
      it = free_.erase(it);
    }
  }
  if (give.empty()) return;
  trace_activity("releasing cached device memory");
  for (void* p : give) (void)hipFree(p);
  trace_activity("");
}

void Pool::trim_all() {
  std::unordered_set<uint64_t> snap;  // release numbers of the blocks cached now
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : free_) snap.insert(kv.second.id);
  }
  if (snap.empty()) return;
  trace_activity("device synchronisation to release cached memory");
  // work queued before this point is all the work that can use the blocks
  // released before it; a block handed out and released again since has a
  // new release number and is kept
  (void)hipDeviceSynchronize();
  std::vector<void*> give;
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end();) {
      if (!snap.count(it->second.id)) {
        ++it;
        continue;
      }
      give.push_back(it->second.p);
      size_.erase(it->second.p);
      tagged_at_.erase(it->second.p);
      cached_ -= it->first;
      it = free_.erase(it);
    }
  }
  for (void* p : give) (void)hipFree(p);
  trace_activity("");
}

void Pool::stats(uint64_t* in_use, uint64_t* peak, uint64_t* cached, bool reset_peak) {
  std::lock_guard<std::mutex> lk(mu_);
  if (reset_peak) peak_ = in_use_;
  if (in_use) *in_use = in_use_;
  if (peak) *peak = peak_;
  if (cached) *cached = cached_;
}

void Pool::fail_after(int64_t after) {
  std::lock_guard<std::mutex> lk(mu_);
  fail_after_ = after;
}

size_t Pool::cached_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  return cached_;
}

Arena::Arena(void* base, size_t bytes) : base_(static_cast<char*>(base)), cap_(bytes & ~size_t(255)) {
  if (cap_) free_.emplace(0, cap_);
}

void* Arena::alloc(size_t bytes) {
  const size_t want = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < want) continue;
    const size_t off = it->first, rest = it->second - want;
    free_.erase(it);
    if (rest) free_.emplace(off + want, rest);
    used_[off] = want;
    in_use_ += want;
    peak_ = std::max(peak_, in_use_);
    return base_ + off;
  }
  throw Error(-3, "fixed scratch of " + std::to_string(cap_) + " bytes cannot hold a further " +
                      std::to_string(want) + " bytes (" + std::to_string(in_use_) + " in use): input too large");
}

void Arena::release(void* p) {
  if (!p) return;
  const size_t off = static_cast<size_t>(static_cast<char*>(p) - base_);
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t sz = u->second;
  size_t start = off;
  used_.erase(u);
  in_use_ -= sz;
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && nx->first == off + sz) {  // merge with the next free range
    sz += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // and with the previous one
    auto pv = std::prev(nx);
    if (pv->first + pv->second == start) {
      start = pv->first;
      sz += pv->second;
      free_.erase(pv);
    }
  }
  free_.emplace(start, sz);
}

Trace*& current_trace() {
  thread_local Trace* t = nullptr;
  return t;
}

namespace {
int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
}  // namespace

void trace_stage(const char* stage) {
  if (Trace* t = current_trace()) {
    t->stage.store(stage);
    t->since_ns.store(now_ns());
  }
}

void trace_activity(const char* activity) {
  if (Trace* t = current_trace()) {
    t->activity.store(activity);
    t->since_ns.store(now_ns());
  }
}

Arena*& current_arena() {
  thread_local Arena* a = nullptr;
  return a;
}

}  // namespace sdbg

namespace sdbg {

namespace {
struct Pending {
  const char* name;
  uint64_t bytes;
  hipEvent_t a, b;
};
thread_local bool t_prof = false;
thread_local std::vector<Pending> t_pending;
thread_local std::vector<ProfRecord> t_records;
}  // namespace

void prof_enable(bool on) { t_prof = on; }
bool prof_enabled() { return t_prof; }
std::vector<ProfRecord>& prof_records() { return t_records; }

void prof_flush() {
  for (auto& p : t_pending) {
    float ms = 0;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess)
      t_records.push_back(ProfRecord{p.name, (double)ms, p.bytes});
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  t_pending.clear();
}

void prof_set_last_bytes(uint64_t bytes) {
  if (!t_pending.empty()) t_pending.back().bytes = bytes;
}

Stage::Stage(Ctx& c, const char* name, uint64_t bytes) : c_(c), name_(name), bytes_(bytes) {
  trace_stage(name);
  if (t_prof) {
    SDBG_HIP(hipEventCreate(&a_));
    SDBG_HIP(hipEventRecord(a_, c_.s));
  }
}

Stage::~Stage() {
  if (!a_) return;
  hipEvent_t b = nullptr;
  if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, c_.s) == hipSuccess) {
    t_pending.push_back(Pending{name_, bytes_, a_, b});
  } else {
    (void)hipEventDestroy(a_);
    if (b) (void)hipEventDestroy(b);
  }
}

}  // namespace sdbg
