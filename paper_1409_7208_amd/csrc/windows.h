// Windows of the packed read stream: the arguments the extraction and
// mercy kernels share, and the walk from a window index to its read and
// stream position.  __host__ __device__, so host programs can replay them.
#pragma once

#include "kernels.h"

namespace sdbg {

struct ExArgs {
  const uint64_t* packed;
  const uint64_t* bad;
  const uint64_t* woff;     // n_reads + 1 window offsets
  const uint64_t* offsets;  // read offsets
  uint64_t n_reads, NW;
  int any_bad;
  int k, kb;
  int pb;             // prefix bits used by the group filter
  uint32_t glo, ghi;  // keep keys whose top pb bits are in [glo, ghi)
  int dlo, dbits;     // partition digit = bits [dlo, dlo + dbits)
  const uint64_t* tr; // tr[t] = read holding window t*TR_GRAIN (last entry: n_reads - 1)
  // Several read sets in one launch (null for a single set): the windows of
  // set s are [sw[s], sw[s+1]), its tiles [st[s], st[s+1]) (at least one),
  // tset[t] = set of tile t.  Tiles never straddle sets, and the histogram
  // table is set-major: set s owns columns [st[s]*2^dbits, st[s+1]*2^dbits),
  // digit-major within, so one scan orders keys by (set, digit, tile).
  const uint32_t* tset;
  const uint64_t* sw;
  const uint64_t* st;
  // 1: each window emits only its canonical key (the smaller of its two
  // strands' keys), twice if both are equal; 0: both keys.
  int canon;
};

// Granularity of the window -> read table.
constexpr uint64_t TR_GRAIN = 64;

DEV uint64_t find_read(const uint64_t* __restrict__ woff, uint64_t n_reads, uint64_t g) {
  uint64_t lo = 0, hi = n_reads;  // woff[lo] <= g < woff[hi]
  while (hi - lo > 1) {
    uint64_t mid = (lo + hi) >> 1;
    if (woff[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// First read lo <= r <= hi with woff[r] <= g < woff[r+1].
DEV uint64_t find_read_in(const uint64_t* __restrict__ woff, uint64_t lo, uint64_t hi, uint64_t g) {
  ++hi;  // woff[lo] <= g < woff[hi]
  while (hi - lo > 1) {
    uint64_t mid = (lo + hi) >> 1;
    if (woff[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

struct WinIter {
  uint64_t r, i, nw, rstart;
  // The read of window g lies between the reads of the first windows of its
  // granule and of the next granule.
  DEV void init(const ExArgs& a, uint64_t g) {
    const uint64_t t = g / TR_GRAIN;
    r = find_read_in(a.woff, a.tr[t], a.tr[t + 1], g);
    rstart = a.offsets[r];
    i = g - a.woff[r];
    nw = a.woff[r + 1] - a.woff[r];
  }

  DEV uint64_t pos() const { return rstart + i; }
  DEV void next(const ExArgs& a) {
    ++i;
    while (i >= nw && r + 1 < a.n_reads) {
      ++r;
      i = 0;
      rstart = a.offsets[r];
      nw = a.woff[r + 1] - a.woff[r];
    }
  }
};

// Are bits [j, j+len) of the flag stream all zero?  len <= 128.
DEV bool window_clean(const uint64_t* __restrict__ bad, uint64_t j, int len) {
  uint64_t q = j >> 6;
  int s = (int)(j & 63);
  uint64_t a = bad[q] >> s;
  int got = 64 - s;
  if (len <= got) return (len >= 64 ? a : (a & ((1ull << len) - 1))) == 0;
  if (a) return false;
  int need = len - got;
  uint64_t b = bad[q + 1];
  if (need <= 64) return (need >= 64 ? b : (b & ((1ull << need) - 1))) == 0;
  if (b) return false;
  need -= 64;
  return (bad[q + 2] & ((1ull << need) - 1)) == 0;
}

}  // namespace sdbg
