// Host runtime for the SdBG library: error handling, a caching device
// memory pool, and a per-call context bound to one HIP stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <cstdio>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

namespace sdbg {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SDBG_HIP(expr)                                                                                  \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      throw ::sdbg::Error(-4, std::string(#expr) + ": " + hipGetErrorString(e_) + " at " + __FILE__ + \
                                  ":" + std::to_string(__LINE__));                                      \
  } while (0)

#define SDBG_CHECK(cond, code, msg)                     \
  do {                                                  \
    if (!(cond)) throw ::sdbg::Error((code), (msg));    \
  } while (0)

// Where a thread's call is, for diagnosis: the last kernel stage it entered
// and what it is waiting on, with the time it got there.  A thread points
// `current_trace()` at a record it owns (the request loop does, per worker);
// otherwise nothing is recorded.
struct Trace {
  std::atomic<const char*> stage{""}, activity{""};
  std::atomic<int64_t> since_ns{0};
};
Trace*& current_trace();
void trace_stage(const char* stage);
void trace_activity(const char* activity);  // "" when done waiting

// Caching allocator: device blocks are kept after release and handed out
// again to requests of similar size, so that repeated calls do not pay for
// hipMalloc/hipFree.  One pool per device.
//
// A released block may still be read or written by work queued on the
// stream that used it; it is tagged with that stream and handed out again
// only to the same stream (stream order makes that safe) until the stream
// has been synchronised, after which untag() makes it free for any stream.
//
// New device memory is taken only while a reserve stays free on the device
// (1/64 of it, at least 1 GiB) for the runtime's own needs (queues, kernel
// arguments) and other users of the device; cached blocks are given back
// first when an allocation would cut into it.
class Pool {
 public:
  void* alloc(size_t bytes, hipStream_t s);
  void release(void* p, hipStream_t s, bool tagged);
  // Makes the blocks released on s up to release number `upto` free for any
  // stream (call after s has been synchronised; release_mark() taken before
  // the synchronisation bounds what it covers).
  void untag(hipStream_t s, uint64_t upto = ~0ull);
  uint64_t release_mark();
  void trim();
  // Gives back every cached block, tagged ones included: the blocks cached
  // now are collected, the device is synchronised (so no stream still uses
  // them), and those still cached are freed.  The last resort before an
  // allocation fails.
  void trim_all();
  size_t cached_bytes();
  // Bytes handed out and not released, and the most at any time since the
  // last reset (reset_peak sets it to the current use).
  void stats(uint64_t* in_use, uint64_t* peak, uint64_t* cached, bool reset_peak);
  // Test hook: after `after` more allocations succeed, the next one fails
  // with an out-of-device-memory error (once); negative disables.
  void fail_after(int64_t after);
  static Pool& get();  // pool of the current device

 private:
  struct Blk {
    void* p;
    hipStream_t s;
    bool tagged;
    uint64_t id;  // release number (a block released again gets a new one)
  };
  struct Tag {
    uint64_t id;
    void* p;
  };
  std::mutex mu_;
  std::multimap<size_t, Blk> free_;
  // per stream, the blocks released tagged, in release order, and where
  // each tagged block sits in free_ (untag() walks only these; entries of
  // blocks handed out or given back since are skipped)
  std::unordered_map<hipStream_t, std::vector<Tag>> tags_;
  std::unordered_map<void*, std::multimap<size_t, Blk>::iterator> tagged_at_;
  std::unordered_map<void*, size_t> size_;
  size_t cached_ = 0;
  uint64_t in_use_ = 0, peak_ = 0, releases_ = 0;
  int64_t fail_after_ = -1;
};

// A fixed device region that stands in for the pool: while one is made
// current on a thread (ArenaScope), every DBuf that thread creates is carved
// out of it, and nothing is allocated from the device.  First fit over a
// sorted free list with coalescing; blocks are 256-byte aligned.  All users
// of one arena run on one stream, so a block freed by one step and handed
// to the next is reused in stream order.  Running out is an error (code -3)
// raised before any kernel touches the block.
class Arena {
 public:
  Arena(void* base, size_t bytes);
  void* alloc(size_t bytes);
  void release(void* p);
  size_t capacity() const { return cap_; }
  size_t peak() const { return peak_; }

 private:
  char* base_;
  size_t cap_;
  size_t in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;           // offset -> bytes
  std::unordered_map<size_t, size_t> used_;  // offset -> bytes
};

Arena*& current_arena();  // of the calling thread; nullptr = the pool

class ArenaScope {
 public:
  explicit ArenaScope(Arena* a) : prev_(current_arena()) { current_arena() = a; }
  ~ArenaScope() { current_arena() = prev_; }
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;

 private:
  Arena* prev_;
};

// Device buffer owned by the calling scope, returned to the pool (tagged
// with its stream) on destruction, or to the arena it was carved from.
template <typename T>
class DBuf {
 public:
  DBuf() = default;
  DBuf(size_t n, hipStream_t s) { reset(n, s); }
  ~DBuf() { free(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p_(o.p_), n_(o.n_), s_(o.s_), a_(o.a_) { o.p_ = nullptr; o.n_ = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      free();
      p_ = o.p_; n_ = o.n_; s_ = o.s_; a_ = o.a_;
      o.p_ = nullptr; o.n_ = 0;
    }
    return *this;
  }
  void reset(size_t n, hipStream_t s) {
    free();
    n_ = n;
    s_ = s;
    a_ = current_arena();
    if (a_)
      p_ = static_cast<T*>(a_->alloc(sizeof(T) * (n ? n : 1)));
    else
      p_ = static_cast<T*>(Pool::get().alloc(sizeof(T) * (n ? n : 1), s));
  }
  void free() noexcept {
    if (p_) {
      try {
        if (a_)
          a_->release(p_);
        else
          Pool::get().release(p_, s_, true);
      } catch (...) {
      }
    }
    p_ = nullptr;
    n_ = 0;
  }
  T* release_ownership() {
    T* p = p_;
    p_ = nullptr;
    n_ = 0;
    return p;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
  hipStream_t s_ = nullptr;
  Arena* a_ = nullptr;
};

// Per-call context.  Declared before any DBuf of the call, so that it is
// destroyed after them: its destructor waits for the stream (also on the
// error path) and then frees the call's released blocks for other streams.
struct Ctx {
  hipStream_t s;
  explicit Ctx(void* stream) : s(static_cast<hipStream_t>(stream)) {}
  ~Ctx() {
    (void)hipStreamSynchronize(s);
    try {
      Pool::get().untag(s);
    } catch (...) {
    }
  }
  Ctx(const Ctx&) = delete;
  Ctx& operator=(const Ctx&) = delete;
  template <typename T>
  DBuf<T> buf(size_t n) { return DBuf<T>(n, s); }
  void sync() {
    trace_activity("stream synchronisation");
    Pool& pool = Pool::get();
    const uint64_t mark = pool.release_mark();
    const hipError_t e = hipStreamSynchronize(s);
    trace_activity("");
    SDBG_HIP(e);
    pool.untag(s, mark);  // what the stream released so far is idle now
  }
  template <typename T>
  T d2h_one(const T* dev) {
    T v;
    SDBG_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    sync();
    return v;
  }
  template <typename T>
  void d2h(T* host, const T* dev, size_t n) {
    if (!n) return;
    SDBG_HIP(hipMemcpyAsync(host, dev, sizeof(T) * n, hipMemcpyDeviceToHost, s));
    sync();
  }
  // Host-to-device copy; waits for it, so `host` may be released at once.
  template <typename T>
  void h2d(T* dev, const T* host, size_t n) {
    if (!n) return;
    SDBG_HIP(hipMemcpyAsync(dev, host, sizeof(T) * n, hipMemcpyHostToDevice, s));
    sync();
  }
  template <typename T>
  void d2d(T* dst, const T* src, size_t n) {
    if (!n) return;
    SDBG_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
  }
  void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(-4, std::string("launch of ") + what + ": " + hipGetErrorString(e));
  }
};

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace sdbg
