// C ABI of the SdBG library (declared in include/sdbg.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "abi_common.h"
#include "prims.h"

namespace sdbg_abi {

thread_local std::string t_err;

// Edge sets the library computed itself are sorted and in range by
// construction; sdbg_build checks the others.
constexpr int kSortedByConstruction = 0x100;

// Every object handed out is registered with its kind, so that sdbg_free
// can release any of them and rejects unknown pointers.
std::mutex g_reg_mu;
std::unordered_map<void*, int>& registry() {
  static std::unordered_map<void*, int> r;
  return r;
}

void reg_add(void* p, int kind) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  registry()[p] = kind;
}

int reg_take(void* p) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  auto it = registry().find(p);
  if (it == registry().end()) return 0;
  int k = it->second;
  registry().erase(it);
  return k;
}

int reg_entry(const void* p) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  auto it = registry().find(const_cast<void*>(p));
  return it == registry().end() ? 0 : it->second;
}

int reg_kind(const void* p) { return reg_entry(p) & 0xFF; }

void pool_free(void* p) {
  if (p) sdbg::Pool::get().release(p, nullptr, false);
}

void check_k(uint32_t k) { SDBG_CHECK(k >= 2 && k <= 127, SDBG_E_INVAL, "k must be in [2, 127]"); }

void check_params(const sdbg_params* p) {
  check_k(p->k);
  SDBG_CHECK(p->d >= 1, SDBG_E_INVAL, "d must be >= 1");
  SDBG_CHECK(p->prefix_len <= 8, SDBG_E_INVAL, "prefix_len must be in [0, 8]");
}

sdbg_edges* wrap_edges(const sdbg::EdgesOut& eo, uint32_t k) {
  sdbg_edges* e = new sdbg_edges();
  e->k = k;
  e->w = (uint32_t)sdbg::key_words((int)k);
  e->n = eo.n;
  e->n_mercy = eo.n_mercy;
  e->n_occ = eo.n_occ;
  e->keys = eo.keys;
  e->count = eo.count;
  reg_add(e, kEdges | kSortedByConstruction);
  return e;
}

sdbg_graph* wrap_graph(const sdbg::GraphOut& go, uint32_t k) {
  sdbg_graph* g = new sdbg_graph();
  g->k = k;
  g->w = (uint32_t)sdbg::key_words((int)k);
  g->m = go.m;
  g->t = go.t;
  g->W = go.W;
  g->last = go.last;
  g->valid = go.valid;
  g->tip = go.tip;
  g->mult = go.mult;
  std::memcpy(g->F, go.F, sizeof(g->F));
  g->tip_seq = go.tip_seq;
  g->tip_words = go.tip_words;
  reg_add(g, kGraph);
  return g;
}

// Host copy of a read set's offsets (validated); device offsets are copied.
std::vector<uint64_t> host_offsets(sdbg::Ctx& c, const sdbg_reads* r) {
  std::vector<uint64_t> o(r->n_reads + 1, 0);
  if (r->n_reads == 0) return o;
  SDBG_CHECK(r->offsets, SDBG_E_INVAL, "null offsets");
  if (r->on_device)
    c.d2h(o.data(), r->offsets, r->n_reads + 1);
  else
    std::memcpy(o.data(), r->offsets, sizeof(uint64_t) * (r->n_reads + 1));
  SDBG_CHECK(o[0] == 0, SDBG_E_INVAL, "offsets[0] must be 0");
  for (uint64_t i = 0; i < r->n_reads; ++i) SDBG_CHECK(o[i + 1] >= o[i], SDBG_E_INVAL, "offsets must be non-decreasing");
  SDBG_CHECK(o[r->n_reads] == 0 || r->seq, SDBG_E_INVAL, "null seq");
  return o;
}

// (k+1)-mer occurrences of a read set if no byte splits a read (an upper
// bound otherwise): 2 * sum over reads of max(0, len - k).
uint64_t occ_bound(const std::vector<uint64_t>& o, uint32_t k) {
  uint64_t n = 0;
  for (size_t i = 0; i + 1 < o.size(); ++i) {
    const uint64_t len = o[i + 1] - o[i];
    if (len > k) n += 2 * (len - k);
  }
  return n;
}

// Device bytes per key of a batched pass: two key buffers, counts, solid
// output and its per-set copy, plus the reads' share.
uint64_t batch_bytes_per_key(uint32_t w) { return 32ull * w + 16; }

// Host threads (and streams) building the graphs of a batch.
constexpr unsigned kBuildThreads = 4;

uint64_t device_budget(const sdbg_params* p) {
  if (p->mem_budget) return p->mem_budget;
  size_t fr = 0, tot = 0;
  SDBG_HIP(hipMemGetInfo(&fr, &tot));
  return (uint64_t)(0.8 * (double)(fr + sdbg::Pool::get().cached_bytes()));
}

// Every field of the caller's sdbg_tune, and nothing past it.
void tune_to_abi(const sdbg::SortTune& x, sdbg_tune* t) {
  t->digit_bits = (uint32_t)x.digit_bits;
  t->tile_shift = (uint32_t)x.tile_shift;
  t->leaf_wg_per_cu = (uint32_t)x.leaf_wg_per_cu;
  t->leaf_cap_shift = (uint32_t)x.leaf_cap_shift;
  t->first_bits = (uint32_t)x.first_bits;
  t->mercy_shift = (uint32_t)x.mercy_shift;
  t->reserved[0] = t->reserved[1] = 0;
}

}  // namespace sdbg_abi

using namespace sdbg_abi;

extern "C" {

const char* sdbg_last_error(void) { return t_err.c_str(); }

void sdbg_profile_enable(int on) { sdbg::prof_enable(on != 0); }

void sdbg_profile_reset(void) {
  sdbg::prof_flush();
  sdbg::prof_records().clear();
}

uint32_t sdbg_profile_count(void) { return (uint32_t)sdbg::prof_records().size(); }

int sdbg_profile_get(uint32_t i, const char** name, double* ms, uint64_t* bytes) {
  auto& r = sdbg::prof_records();
  if (i >= r.size()) return SDBG_E_INVAL;
  if (name) *name = r[i].name;
  if (ms) *ms = r[i].ms;
  if (bytes) *bytes = r[i].bytes;
  return SDBG_OK;
}

int sdbg_pool_stats(uint64_t* in_use, uint64_t* peak, uint64_t* cached, int reset_peak) {
  return guarded([&]() -> int {
    sdbg::Pool::get().stats(in_use, peak, cached, reset_peak != 0);
    return SDBG_OK;
  });
}

int sdbg_fail_alloc_after(int64_t after) {
  return guarded([&]() -> int {
    sdbg::Pool::get().fail_after(after);
    return SDBG_OK;
  });
}

void sdbg_trim(void) {
  try {
    sdbg::Pool::get().trim();
  } catch (...) {
  }
}

int sdbg_count_solid(const sdbg_reads* reads, const sdbg_params* params, sdbg_edges** out) {
  return guarded([&]() -> int {
    SDBG_CHECK(reads && params && out, SDBG_E_INVAL, "null argument");
    *out = nullptr;
    check_k(params->k);
    SDBG_CHECK(params->d >= 1, SDBG_E_INVAL, "d must be >= 1");
    SDBG_CHECK(params->prefix_len <= 8, SDBG_E_INVAL, "prefix_len must be in [0, 8]");
    SDBG_CHECK(reads->n_reads == 0 || (reads->offsets != nullptr), SDBG_E_INVAL, "null offsets");
    sdbg::Ctx c(params->stream);
    sdbg::DevReads R{};
    R.n_reads = reads->n_reads;
    sdbg::DBuf<uint8_t> seq_d;
    sdbg::DBuf<uint64_t> off_d;
    if (reads->n_reads == 0) {
      off_d = c.buf<uint64_t>(1);
      uint64_t z = 0;
      c.h2d(off_d.get(), &z, 1);
      R.offsets = off_d.get();
      R.seq = nullptr;
      R.n_bases = 0;
    } else if (reads->on_device) {
      R.offsets = reads->offsets;
      R.seq = reads->seq;
      uint64_t first = c.d2h_one(reads->offsets);
      R.n_bases = c.d2h_one(reads->offsets + reads->n_reads);
      SDBG_CHECK(first == 0, SDBG_E_INVAL, "offsets[0] must be 0");
      // with offsets[0] = 0 and no decrease, every read lies in [0, n_bases)
      SDBG_CHECK(sdbg::nondecreasing(reads->offsets, reads->n_reads, c), SDBG_E_INVAL,
                 "offsets must be non-decreasing");
      SDBG_CHECK(R.n_bases == 0 || reads->seq, SDBG_E_INVAL, "null seq");
    } else {
      const uint64_t* o = reads->offsets;
      SDBG_CHECK(o[0] == 0, SDBG_E_INVAL, "offsets[0] must be 0");
      for (uint64_t i = 0; i < reads->n_reads; ++i)
        SDBG_CHECK(o[i + 1] >= o[i], SDBG_E_INVAL, "offsets must be non-decreasing");
      R.n_bases = o[reads->n_reads];
      SDBG_CHECK(R.n_bases == 0 || reads->seq, SDBG_E_INVAL, "null seq");
      seq_d = c.buf<uint8_t>(R.n_bases + 16);
      off_d = c.buf<uint64_t>(reads->n_reads + 1);
      c.h2d(seq_d.get(), reads->seq, R.n_bases);
      c.h2d(off_d.get(), o, reads->n_reads + 1);
      R.seq = seq_d.get();
      R.offsets = off_d.get();
    }
    sdbg::CountParams P{(int)params->k, params->d, params->mercy != 0, (int)params->prefix_len, params->mem_budget};
    sdbg::EdgesOut eo;
    sdbg::count_solid(R, P, c, &eo);
    c.sync();
    sdbg::prof_flush();
    *out = wrap_edges(eo, params->k);
    return SDBG_OK;
  });
}

int sdbg_build(const sdbg_edges* edges, const sdbg_params* params, sdbg_graph** out) {
  return guarded([&]() -> int {
    SDBG_CHECK(edges && out, SDBG_E_INVAL, "null argument");
    *out = nullptr;
    SDBG_CHECK(reg_kind(edges) == kEdges, SDBG_E_INVAL, "not an edge set returned by this library");
    check_k(edges->k);
    sdbg::Ctx c(params ? params->stream : nullptr);
    sdbg::GraphOut go;
    sdbg::build_graph(edges->keys, edges->count, edges->n, (int)edges->k, c, &go,
                      (reg_entry(edges) & kSortedByConstruction) == 0);
    c.sync();
    sdbg::prof_flush();
    sdbg_graph* g = new sdbg_graph();
    g->k = edges->k;
    g->w = edges->w;
    g->m = go.m;
    g->t = go.t;
    g->W = go.W;
    g->last = go.last;
    g->valid = go.valid;
    g->tip = go.tip;
    g->mult = go.mult;
    std::memcpy(g->F, go.F, sizeof(g->F));
    g->tip_seq = go.tip_seq;
    g->tip_words = go.tip_words;
    reg_add(g, kGraph);
    *out = g;
    return SDBG_OK;
  });
}

int sdbg_edges_union(const sdbg_edges* a, const sdbg_edges* b, const sdbg_params* params, sdbg_edges** out) {
  return guarded([&]() -> int {
    SDBG_CHECK(a && b && out, SDBG_E_INVAL, "null argument");
    *out = nullptr;
    SDBG_CHECK(reg_kind(a) == kEdges && reg_kind(b) == kEdges, SDBG_E_INVAL,
               "not an edge set returned by this library");
    SDBG_CHECK(a->k == b->k, SDBG_E_INVAL, "edge sets of different k");
    sdbg::Ctx c(params ? params->stream : nullptr);
    sdbg::EdgesOut eo;
    sdbg::edges_union(a->keys, a->count, a->n, b->keys, b->count, b->n, (int)a->k, c, &eo);
    c.sync();
    sdbg::prof_flush();
    eo.n_mercy = 0;
    eo.n_occ = a->n_occ + b->n_occ;
    *out = wrap_edges(eo, a->k);
    return SDBG_OK;
  });
}

int sdbg_multi_k(const sdbg_reads* reads, const uint32_t* ks, uint32_t n_k, const sdbg_params* params,
                 const sdbg_clean_params* clean, uint64_t* stats, sdbg_unitigs** out) {
  // Objects of the iteration in flight, released on every exit.
  struct Held {
    void* p[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    ~Held() {
      for (void* x : p) sdbg_free(x);
    }
  } h;
  enum { kReadEdges, kContigEdges, kEdgesAll, kGraphI, kIndexI, kPrev, kCur };
  const int rc = guarded([&]() -> int {
    SDBG_CHECK(reads && ks && params && clean && out && n_k > 0, SDBG_E_INVAL, "null argument");
    *out = nullptr;
    for (uint32_t i = 0; i < n_k; ++i) {
      check_k(ks[i]);
      SDBG_CHECK(i == 0 || ks[i] > ks[i - 1], SDBG_E_INVAL, "k values must ascend");
    }
    return SDBG_OK;
  });
  if (rc != SDBG_OK) return rc;
  for (uint32_t i = 0; i < n_k; ++i) {
    sdbg_params p = *params;
    p.k = ks[i];
    int r = sdbg_count_solid(reads, &p, reinterpret_cast<sdbg_edges**>(&h.p[kReadEdges]));
    if (r != SDBG_OK) return r;
    auto* re = static_cast<sdbg_edges*>(h.p[kReadEdges]);
    const uint64_t n_read_edges = re->n;
    auto* prev = static_cast<sdbg_unitigs*>(h.p[kPrev]);
    if (prev && prev->n) {  // the contigs of the previous k: all their (k+1)-mers
      sdbg_reads cr{prev->seq, prev->offsets, prev->n, 1, 0};
      sdbg_params pc = p;
      pc.d = 1;
      pc.mercy = 0;
      r = sdbg_count_solid(&cr, &pc, reinterpret_cast<sdbg_edges**>(&h.p[kContigEdges]));
      if (r != SDBG_OK) return r;
      r = sdbg_edges_union(re, static_cast<sdbg_edges*>(h.p[kContigEdges]), &p,
                           reinterpret_cast<sdbg_edges**>(&h.p[kEdgesAll]));
      if (r != SDBG_OK) return r;
      sdbg_free(h.p[kReadEdges]);
      sdbg_free(h.p[kContigEdges]);
      h.p[kReadEdges] = h.p[kContigEdges] = nullptr;
    } else {
      h.p[kEdgesAll] = h.p[kReadEdges];
      h.p[kReadEdges] = nullptr;
    }
    auto* e = static_cast<sdbg_edges*>(h.p[kEdgesAll]);
    const uint64_t n_edges = e->n;
    r = sdbg_build(e, &p, reinterpret_cast<sdbg_graph**>(&h.p[kGraphI]));
    if (r != SDBG_OK) return r;
    sdbg_free(h.p[kEdgesAll]);
    h.p[kEdgesAll] = nullptr;
    auto* g = static_cast<sdbg_graph*>(h.p[kGraphI]);
    r = sdbg_index_build(g, &p, reinterpret_cast<sdbg_index**>(&h.p[kIndexI]));
    if (r != SDBG_OK) return r;
    auto* ix = static_cast<sdbg_index*>(h.p[kIndexI]);
    uint64_t n_tips = 0, n_bubble = 0, n_low = 0;
    r = sdbg_remove_tips(g, ix, clean->tip_factor * ks[i], &n_tips, p.stream);
    if (r != SDBG_OK) return r;
    // bubbles, then low local coverage, each on the unitigs of the edges left
    for (int step = 0; step < 2; ++step) {
      const uint32_t f = step == 0 ? clean->bubble_factor : clean->low_cov_factor;
      if (f == 0) continue;
      r = sdbg_unitigs_build(g, ix, reinterpret_cast<sdbg_unitigs**>(&h.p[kCur]), p.stream);
      if (r != SDBG_OK) return r;
      auto* cu = static_cast<sdbg_unitigs*>(h.p[kCur]);
      r = step == 0 ? sdbg_merge_bubbles(g, ix, cu, f * ks[i], &n_bubble, p.stream)
                    : sdbg_remove_low_coverage(g, ix, cu, f * ks[i], clean->low_cov_permille, &n_low, p.stream);
      if (r != SDBG_OK) return r;
      sdbg_free(h.p[kCur]);
      h.p[kCur] = nullptr;
    }
    sdbg_unitigs* u = nullptr;
    r = sdbg_unitigs_build(g, ix, &u, p.stream);
    if (r != SDBG_OK) return r;
    sdbg_free(h.p[kIndexI]);
    sdbg_free(h.p[kGraphI]);
    sdbg_free(h.p[kPrev]);
    h.p[kIndexI] = h.p[kGraphI] = nullptr;
    h.p[kPrev] = u;
    if (stats) {
      uint64_t* st = stats + 6 * (uint64_t)i;
      st[0] = n_edges;
      st[1] = n_edges - n_read_edges;
      st[2] = n_tips;
      st[3] = n_bubble;
      st[4] = n_low;
      st[5] = u->n;
    }
  }
  *out = static_cast<sdbg_unitigs*>(h.p[kPrev]);
  h.p[kPrev] = nullptr;
  return SDBG_OK;
}

// Graph builders of a batch: a few host threads, each on a stream of its
// own, build the sets' graphs once every pass has counted, so that one
// set's size read-backs overlap the other sets' kernels.  (Building next to
// the counting passes was measured slower: the two compete for the device.)
// The destructor stops and joins the threads (also when the caller throws);
// errors are collected for finish_and_check().
class BatchBuilders {
 public:
  BatchBuilders(sdbg_edges** edges, sdbg_graph** graphs, uint64_t n_sets, uint32_t k) : edges_(edges), graphs_(graphs),
                                                                                        k_(k) {
    int dev = 0;
    SDBG_HIP(hipGetDevice(&dev));
    const unsigned nth = (unsigned)std::min<uint64_t>(kBuildThreads, n_sets);
    for (unsigned t = 0; t < nth; ++t) th_.emplace_back([this, dev] { work(dev); });
  }
  ~BatchBuilders() { finish(/*stop=*/true); }
  void push(uint64_t s0, uint64_t s1) {
    {
      std::lock_guard<std::mutex> g(mu_);
      for (uint64_t s = s0; s < s1; ++s) q_.push_back(s);
    }
    cv_.notify_all();
  }
  // All sets pushed: wait for the builds, rethrow the first error.
  void finish_and_check() {
    finish(false);
    if (!err_.empty()) throw sdbg::Error(err_rc_, err_);
  }

 private:
  void finish(bool stop) {
    {
      std::lock_guard<std::mutex> g(mu_);
      closed_ = true;
      if (stop) failed_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_)
      if (t.joinable()) t.join();
  }
  void work(int dev) {
    const int rc = guarded([&]() -> int {
      SDBG_HIP(hipSetDevice(dev));
      hipStream_t st = nullptr;
      SDBG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      try {
        sdbg::Ctx c2(st);
        for (;;) {
          uint64_t i;
          {
            std::unique_lock<std::mutex> g(mu_);
            cv_.wait(g, [&] { return failed_ || closed_ || !q_.empty(); });
            if (failed_ || q_.empty()) break;
            i = q_.front();
            q_.pop_front();
          }
          sdbg::GraphOut go;
          sdbg::build_graph(edges_[i]->keys, edges_[i]->count, edges_[i]->n, (int)k_, c2, &go, false);
          c2.sync();
          graphs_[i] = wrap_graph(go, k_);
        }
      } catch (...) {
        (void)hipStreamDestroy(st);
        throw;
      }
      (void)hipStreamDestroy(st);
      return SDBG_OK;
    });
    if (rc != SDBG_OK) {
      std::lock_guard<std::mutex> g(mu_);
      if (err_.empty()) {
        err_ = t_err.empty() ? "graph build failed" : t_err;
        err_rc_ = rc;
      }
      failed_ = true;
      cv_.notify_all();
    }
  }

  sdbg_edges** edges_;
  sdbg_graph** graphs_;
  uint32_t k_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<uint64_t> q_;
  bool closed_ = false, failed_ = false;
  std::string err_;
  int err_rc_ = SDBG_OK;
  std::vector<std::thread> th_;
};

int sdbg_batch_run(const sdbg_reads* sets, uint64_t n_sets, const sdbg_params* params, sdbg_edges** edges_out,
                   sdbg_graph** graphs_out) {
  std::vector<void*> made;
  int rc = guarded([&]() -> int {
    SDBG_CHECK(params && edges_out && (sets || n_sets == 0), SDBG_E_INVAL, "null argument");
    for (uint64_t s = 0; s < n_sets; ++s) {
      edges_out[s] = nullptr;
      if (graphs_out) graphs_out[s] = nullptr;
    }
    check_params(params);
    const uint32_t k = params->k, w = (uint32_t)sdbg::key_words((int)k);
    sdbg::Ctx c(params->stream);
    // Per set: bases and occurrence bound.  Host sets are checked on the
    // host; device sets on the device (one read-back for all of them), so
    // their offsets never travel to the host.
    std::vector<std::vector<uint64_t>> off(n_sets);  // host sets only
    std::vector<uint64_t> occ(n_sets, 0), nbases(n_sets, 0);
    {
      sdbg::DBuf<unsigned long long> st = c.buf<unsigned long long>(3 * n_sets);
      uint64_t n_dev = 0;
      for (uint64_t s = 0; s < n_sets; ++s) {
        if (sets[s].on_device && sets[s].n_reads) {
          SDBG_CHECK(sets[s].offsets, SDBG_E_INVAL, "null offsets");
          if (!n_dev++) sdbg::fill<uint64_t>(reinterpret_cast<uint64_t*>(st.get()), 3 * n_sets, 0, c);
          sdbg::offsets_summary(sets[s].offsets, sets[s].n_reads, k, st.get() + 3 * s, c);
        } else {
          off[s] = host_offsets(c, &sets[s]);
          occ[s] = occ_bound(off[s], k);
          nbases[s] = off[s].back();
        }
      }
      if (n_dev) {
        std::vector<unsigned long long> h(3 * n_sets);
        c.d2h(h.data(), st.get(), 3 * n_sets);
        for (uint64_t s = 0; s < n_sets; ++s) {
          if (!(sets[s].on_device && sets[s].n_reads)) continue;
          SDBG_CHECK(h[3 * s] == 0, SDBG_E_INVAL, "offsets[0] must be 0 and offsets must be non-decreasing");
          occ[s] = h[3 * s + 1];
          nbases[s] = h[3 * s + 2];
          SDBG_CHECK(nbases[s] == 0 || sets[s].seq, SDBG_E_INVAL, "null seq");
        }
      }
    }
    const bool shared = !(params->mercy && params->d >= 2);
    sdbg::CountParams P{(int)k, params->d, params->mercy != 0, (int)params->prefix_len, params->mem_budget};
    uint64_t s0 = 0;
    while (s0 < n_sets) {
      // the budget is taken again for every pass: the outputs of the
      // earlier passes stay on the device
      const uint64_t budget = device_budget(params);
      const uint64_t max_keys = std::min<uint64_t>(budget / batch_bytes_per_key(w), 0xFFFFFFFFull);
      if (std::getenv("SDBG_VERBOSE")) {
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        uint64_t iu = 0, pk = 0, ca = 0;
        sdbg::Pool::get().stats(&iu, &pk, &ca, false);
        std::fprintf(stderr, "[sdbg] batch pass from set %llu: budget %.2f GB, free %.2f GB, pool in use %.2f GB "
                             "cached %.2f GB\n",
                     (unsigned long long)s0, budget / 1e9, fr / 1e9, iu / 1e9, ca / 1e9);
      }
      if (!shared || occ[s0] > max_keys) {
        // one set alone on the single-set path (mercy, or larger than a pass)
        sdbg::EdgesOut eo;
        {
          sdbg::DevReads R{};
          R.n_reads = sets[s0].n_reads;
          R.n_bases = nbases[s0];
          sdbg::DBuf<uint8_t> seq_d = c.buf<uint8_t>(R.n_bases + 16);
          sdbg::DBuf<uint64_t> off_d = c.buf<uint64_t>(R.n_reads + 1);
          if (R.n_bases) {
            if (sets[s0].on_device)
              c.d2d(seq_d.get(), sets[s0].seq, R.n_bases);
            else
              c.h2d(seq_d.get(), sets[s0].seq, R.n_bases);
          }
          if (sets[s0].on_device && R.n_reads)
            c.d2d(off_d.get(), sets[s0].offsets, R.n_reads + 1);
          else
            c.h2d(off_d.get(), off[s0].data(), R.n_reads + 1);
          R.seq = seq_d.get();
          R.offsets = off_d.get();
          sdbg::count_solid(R, P, c, &eo);
          c.sync();
        }
        edges_out[s0] = wrap_edges(eo, k);
        made.push_back(edges_out[s0]);
        ++s0;
        continue;
      }
      // a wave: consecutive sets whose keys fit one pass
      uint64_t s1 = s0, keys = 0, bases = 0, reads = 0;
      while (s1 < n_sets && occ[s1] <= max_keys && keys + occ[s1] <= max_keys) {
        keys += occ[s1];
        bases += nbases[s1];
        reads += sets[s1].n_reads;
        ++s1;
      }
      std::vector<sdbg::EdgesOut> outs;
      {
        sdbg::DBuf<uint8_t> seq_d = c.buf<uint8_t>(bases + 16);
        sdbg::DBuf<uint64_t> off_d = c.buf<uint64_t>(reads + 1);
        std::vector<uint64_t> rb(s1 - s0 + 1);
        std::vector<std::vector<uint64_t>> ho;  // rebased offsets of host sets, kept until the copies are done
        uint64_t rp = 0, bp = 0;
        for (uint64_t s = s0; s < s1; ++s) {
          rb[s - s0] = rp;
          const uint64_t nb = nbases[s];
          const uint64_t nr = sets[s].n_reads;
          if (sets[s].on_device && nr) {
            sdbg::offsets_rebase(sets[s].offsets, nr, bp, off_d.get() + rp, c);
          } else if (nr) {
            ho.emplace_back(nr);
            for (uint64_t i = 0; i < nr; ++i) ho.back()[i] = bp + off[s][i];
            c.h2d(off_d.get() + rp, ho.back().data(), nr);
          }
          if (nb) {
            if (sets[s].on_device)
              c.d2d(seq_d.get() + bp, sets[s].seq, nb);
            else
              c.h2d(seq_d.get() + bp, sets[s].seq, nb);
          }
          rp += nr;
          bp += nb;
        }
        sdbg::fill<uint64_t>(off_d.get() + reads, 1, bp, c);
        rb[s1 - s0] = rp;
        sdbg::DevReads R{seq_d.get(), off_d.get(), reads, bases};
        try {
          sdbg::count_solid_sets(R, rb, P, c, &outs);
        } catch (...) {
          for (auto& o : outs) {
            pool_free(o.keys);
            pool_free(o.count);
          }
          throw;
        }
        c.sync();
      }
      for (uint64_t s = s0; s < s1; ++s) {
        edges_out[s] = wrap_edges(outs[s - s0], k);
        made.push_back(edges_out[s]);
      }
      s0 = s1;
    }
    if (graphs_out && n_sets) {
      c.sync();
      BatchBuilders builders(edges_out, graphs_out, n_sets, k);
      builders.push(0, n_sets);
      builders.finish_and_check();
    }
    sdbg::prof_flush();
    return SDBG_OK;
  });
  if (rc != SDBG_OK) {
    // (the builders are joined by now: the guarded lambda has returned)
    for (void* p : made) sdbg_free(p);
    for (uint64_t s = 0; edges_out && s < n_sets; ++s) {
      edges_out[s] = nullptr;
      if (graphs_out && graphs_out[s]) {
        sdbg_free(graphs_out[s]);
        graphs_out[s] = nullptr;
      }
    }
  }
  return rc;
}

int sdbg_tune_get(sdbg_tune* t) {
  return guarded([&]() -> int {
    SDBG_CHECK(t, SDBG_E_INVAL, "null argument");
    tune_to_abi(sdbg::sort_tune(), t);
    return SDBG_OK;
  });
}

int sdbg_tune_set(const sdbg_tune* t) {
  return guarded([&]() -> int {
    sdbg::SortTune x;
    if (t) {
      x.digit_bits = (int)t->digit_bits;
      x.tile_shift = (int)t->tile_shift;
      x.leaf_wg_per_cu = (int)t->leaf_wg_per_cu;
      x.leaf_cap_shift = (int)t->leaf_cap_shift;
      x.first_bits = (int)t->first_bits;
      x.mercy_shift = (int)t->mercy_shift;
    }
    sdbg::set_sort_tune(x);
    return SDBG_OK;
  });
}

int sdbg_autotune(const sdbg_reads* sets, uint64_t n_sets, const sdbg_params* params, uint32_t reps, sdbg_tune* best) {
  return guarded([&]() -> int {
    SDBG_CHECK(params && (sets || n_sets == 0), SDBG_E_INVAL, "null argument");
    check_params(params);
    if (!reps) reps = 3;
    std::vector<sdbg_edges*> eo(n_sets ? n_sets : 1);
    // Median wall time of reps batched counts of the sample (each call
    // waits for its stream, so the host clock brackets the device work).
    auto time_it = [&](const sdbg::SortTune& t) -> double {
      sdbg::set_sort_tune(t);
      std::vector<double> ts;
      for (uint32_t r = 0; r <= reps; ++r) {  // the first run warms the memory pool
        const auto a = std::chrono::steady_clock::now();
        const int rc = sdbg_batch_run(sets, n_sets, params, eo.data(), nullptr);
        const auto b = std::chrono::steady_clock::now();
        if (rc != SDBG_OK) throw sdbg::Error(rc, t_err);
        for (uint64_t s = 0; s < n_sets; ++s) sdbg_free(eo[s]);
        if (r) ts.push_back(std::chrono::duration<double>(b - a).count());
      }
      std::sort(ts.begin(), ts.end());
      return ts[ts.size() / 2];
    };
    const sdbg::SortTune start = sdbg::sort_tune();
    sdbg::SortTune cur = start;
    try {
      double best_t = time_it(cur);
      // coordinate descent over the three knobs
      const int digit_vals[] = {6, 7, 8}, shift_vals[] = {0, 1}, wpc_vals[] = {4, 8, 16, 32};
      for (int knob = 0; knob < 4; ++knob) {
        const int* vals = knob == 0 ? digit_vals : knob == 2 ? wpc_vals : shift_vals;
        const int nv = knob == 0 ? 3 : knob == 2 ? 4 : 2;
        for (int i = 0; i < nv; ++i) {
          sdbg::SortTune t = cur;
          int& f = knob == 0 ? t.digit_bits : knob == 1 ? t.tile_shift : knob == 2 ? t.leaf_wg_per_cu : t.leaf_cap_shift;
          if (f == vals[i]) continue;
          f = vals[i];
          const double x = time_it(t);
          if (x < best_t) {
            best_t = x;
            cur = t;
          }
        }
      }
    } catch (...) {
      sdbg::set_sort_tune(start);
      throw;
    }
    sdbg::set_sort_tune(cur);
    if (best) tune_to_abi(cur, best);
    return SDBG_OK;
  });
}

int sdbg_edges_from_host(const uint64_t* keys, const uint32_t* count, uint64_t n, uint32_t k, sdbg_edges** out) {
  return guarded([&]() -> int {
    SDBG_CHECK(out && (n == 0 || (keys && count)), SDBG_E_INVAL, "null argument");
    *out = nullptr;
    check_k(k);
    const uint32_t w = (uint32_t)sdbg::key_words((int)k);
    sdbg::Ctx c(nullptr);
    sdbg::DBuf<uint64_t> kd = c.buf<uint64_t>(n * w);
    sdbg::DBuf<uint32_t> cd = c.buf<uint32_t>(n);
    c.h2d(kd.get(), keys, n * w);
    c.h2d(cd.get(), count, n);
    sdbg_edges* e = new sdbg_edges();
    e->k = k;
    e->w = w;
    e->n = n;
    e->n_mercy = 0;
    e->n_occ = 0;
    e->keys = kd.release_ownership();
    e->count = cd.release_ownership();
    reg_add(e, kEdges);
    *out = e;
    return SDBG_OK;
  });
}

int sdbg_edges_to_host(const sdbg_edges* e, uint64_t* keys, uint32_t* count) {
  return guarded([&]() -> int {
    SDBG_CHECK(e && reg_kind(e) == kEdges, SDBG_E_INVAL, "not an edge set returned by this library");
    sdbg::Ctx c(nullptr);
    if (keys) c.d2h(keys, e->keys, e->n * e->w);
    if (count) c.d2h(count, e->count, e->n);
    return SDBG_OK;
  });
}

int sdbg_graph_to_host(const sdbg_graph* g, uint8_t* W, uint64_t* last, uint64_t* valid, uint64_t* tip, uint32_t* mult,
                       uint64_t* tip_seq) {
  return guarded([&]() -> int {
    SDBG_CHECK(g && reg_kind(g) == kGraph, SDBG_E_INVAL, "not a graph returned by this library");
    sdbg::Ctx c(nullptr);
    const uint64_t words = (g->m + 63) / 64;
    if (W) c.d2h(W, g->W, g->m);
    if (last) c.d2h(last, g->last, words);
    if (valid) c.d2h(valid, g->valid, words);
    if (tip) c.d2h(tip, g->tip, words);
    if (mult) c.d2h(mult, g->mult, g->m);
    if (tip_seq) c.d2h(tip_seq, g->tip_seq, g->tip_words);
    return SDBG_OK;
  });
}

void sdbg_free(void* obj) {
  if (!obj) return;
  int kind = reg_take(obj) & 0xFF;
  try {
    if (kind == kEdges) {
      sdbg_edges* e = static_cast<sdbg_edges*>(obj);
      pool_free(e->keys);
      pool_free(e->count);
      delete e;
    } else if (kind == kGraph) {
      sdbg_graph* g = static_cast<sdbg_graph*>(obj);
      pool_free(g->W);
      pool_free(g->last);
      pool_free(g->valid);
      pool_free(g->tip);
      pool_free(g->mult);
      pool_free(g->tip_seq);
      delete g;
    } else if (kind == kIndex) {
      free_index(obj);
    } else if (kind == kUnitigs) {
      free_unitigs(obj);
    } else if (kind == kBwt) {
      free_bwt(obj);
    }
  } catch (...) {
  }
}

}  // extern "C"
