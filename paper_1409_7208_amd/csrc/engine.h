// Internal interface between the C ABI and the device pipeline.
#pragma once

#include <stdint.h>

#include <vector>

#include "runtime.h"

namespace sdbg {

inline int key_words(int k) { return (2 * (k + 1) + 63) / 64; }

// Reads resident on the device (borrowed).
struct DevReads {
  const uint8_t* seq;
  const uint64_t* offsets;
  uint64_t n_reads;
  uint64_t n_bases;  // offsets[n_reads]
};

struct CountParams {
  int k;
  uint32_t d;
  bool mercy;
  int prefix_len;
  uint64_t mem_budget;  // bytes, 0 = auto
};

// Result of counting: device arrays owned by the caller afterwards.
struct EdgesOut {
  uint64_t* keys = nullptr;   // n * w words
  uint32_t* count = nullptr;  // n
  uint64_t n = 0, n_mercy = 0, n_occ = 0;
};

struct GraphOut {
  uint64_t m = 0, t = 0;
  uint8_t* W = nullptr;
  uint64_t* last = nullptr;
  uint64_t* valid = nullptr;
  uint64_t* tip = nullptr;
  uint32_t* mult = nullptr;
  uint64_t F[6] = {0, 0, 0, 0, 0, 0};
  uint64_t* tip_seq = nullptr;
  uint64_t tip_words = 0;
};

// Kernel timings for profiling: when enabled, kernels of the calling
// thread's calls are bracketed by HIP events on the call's stream (no extra
// synchronisation); elapsed times are read when the call completes.
struct ProfRecord {
  const char* name;
  double ms;
  uint64_t bytes;  // algorithmic bytes read + written by the launch
};
void prof_enable(bool on);
bool prof_enabled();
std::vector<ProfRecord>& prof_records();
void prof_flush();  // resolve pending events (stream must be complete)
void prof_set_last_bytes(uint64_t bytes);  // bytes of the most recent stage

class Stage {
 public:
  Stage(Ctx& c, const char* name, uint64_t bytes);
  ~Stage();
  Stage(const Stage&) = delete;
  Stage& operator=(const Stage&) = delete;

 private:
  Ctx& c_;
  const char* name_;
  uint64_t bytes_;
  hipEvent_t a_ = nullptr;
};

// Launch parameters of the partition/sort engine.  Results never depend on
// them; they only move work between passes and workgroups.
struct SortTune {
  int digit_bits = 7;       // most key bits one refinement pass cuts (4..8)
  int tile_shift = 0;       // refinement tile = the width's default tile >> tile_shift (0 or 1)
  int leaf_wg_per_cu = 16;  // persistent leaf workgroups per compute unit (1..32)
  int leaf_cap_shift = 0;   // largest leaf = the width's default >> leaf_cap_shift (0 or 1)
  int first_bits = 6;       // key bits of the first cut, taken from the packed reads (4..8)
  int mercy_shift = 0;      // mercy lookup table 2^mercy_shift times smaller than sized (0..8)
};
SortTune sort_tune();
void set_sort_tune(const SortTune& t);

void count_solid(const DevReads& r, const CountParams& p, Ctx& c, EdgesOut* out);
// Several read sets (reads [rb[s], rb[s+1]) of r) counted together, mercy
// off; outs[s] equals count_solid of set s alone.
void count_solid_sets(const DevReads& r, const std::vector<uint64_t>& rb, const CountParams& p, Ctx& c,
                      std::vector<EdgesOut>* outs);
// Union of two edge sets of the same k (ascending, unique): keys of either,
// counts summed (an error if a sum does not fit 32 bits).
void edges_union(const uint64_t* A, const uint32_t* Ac, uint64_t nA, const uint64_t* B, const uint32_t* Bc,
                 uint64_t nB, int k, Ctx& c, EdgesOut* out);
// check = false skips the order check for edge sets the library computed.
void build_graph(const uint64_t* keys, const uint32_t* count, uint64_t n, int k, Ctx& c, GraphOut* out,
                 bool check = true);

}  // namespace sdbg
