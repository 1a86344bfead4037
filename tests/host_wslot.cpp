// Host replay of the word-slot mercy table (paper_1409_7208_amd/csrc/
// wslots.h, windows.h; the per-thread bodies of the fill and lookup kernels
// are __host__ __device__): random reads with non-ACGT bases, a random
// solid set drawn from their window keys plus keys of no window, the table
// filled by every solid key's thread, then every window's flags from the
// lookup run with one, two and four windows per thread, against a binary
// search of the sorted set.  Key widths of two to four words, and a shrunk
// table whose buckets overflow.  Built with the undefined-behaviour
// sanitizer.  Prints "ok" or the first mismatch.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "wslots.h"

using namespace sdbg;

namespace {

struct Stream {
  std::vector<uint64_t> packed, bad, offsets, woff, tr;
  uint64_t n_reads = 0, NW = 0;
  bool any_bad = false;
};

// Reads of random length (some without a window) over ACGT with about one
// base in 100 replaced by N; base j of the stream at bits 2(j mod 32) of
// word j/32, non-ACGT bases flagged in a bit stream.
Stream make_stream(int k, int n_reads, std::mt19937_64& rng) {
  Stream st;
  st.n_reads = n_reads;
  std::vector<uint8_t> codes, isbad;
  st.offsets.push_back(0);
  st.woff.push_back(0);
  for (int r = 0; r < n_reads; ++r) {
    const int len = (int)(rng() % 80) + k - 10;
    for (int i = 0; i < len; ++i) {
      const bool b = rng() % 100 == 0;
      codes.push_back(b ? 0 : (uint8_t)(rng() & 3));
      isbad.push_back(b);
      st.any_bad = st.any_bad || b;
    }
    st.offsets.push_back(codes.size());
    st.woff.push_back(st.woff.back() + (len > k ? (uint64_t)(len - k) : 0));
  }
  st.NW = st.woff.back();
  const uint64_t nb = codes.size();
  st.packed.assign(nb / 32 + 8, 0);
  st.bad.assign(nb / 64 + 8, 0);
  for (uint64_t j = 0; j < nb; ++j) {
    st.packed[j / 32] |= (uint64_t)codes[j] << (2 * (j % 32));
    if (isbad[j]) st.bad[j / 64] |= 1ull << (j % 64);
  }
  // tr[t] = read holding window t * TR_GRAIN; the last entry is the last read
  const uint64_t ntr = (st.NW + TR_GRAIN - 1) / TR_GRAIN + 1;
  st.tr.assign(ntr, (uint64_t)n_reads - 1);
  for (uint64_t t = 0; t + 1 < ntr; ++t) {
    const uint64_t g = t * TR_GRAIN;
    st.tr[t] = (uint64_t)(std::upper_bound(st.woff.begin(), st.woff.end(), g) - st.woff.begin()) - 1;
  }
  return st;
}

template <int W>
bool less_key(const std::vector<uint64_t>& v, size_t a, size_t b) {
  return key_less<W>(key_load<W>(&v[a * W]), key_load<W>(&v[b * W]));
}

template <int W, int SWD, int IPT>
bool run_lookups(const ExArgs& a, const std::vector<uint64_t>& tab, int bb, int rbits, const SortedView& S,
                 const std::vector<uint8_t>& sfl, const std::vector<uint8_t>& want, int k, int shrink) {
  std::vector<uint8_t> wf(a.NW + 8, 0xEE);
  for (uint64_t g0 = 0; g0 < a.NW; g0 += IPT)
    wslot_window_flags<W, SWD, IPT>(a, tab.data(), bb, rbits, S, sfl.data(), wf.data(), g0);
  for (uint64_t g = 0; g < a.NW; ++g)
    if (wf[g] != want[g]) {
      std::printf("mismatch k=%d shrink=%d ipt=%d window=%llu got=%d want=%d\n", k, shrink, IPT,
                  (unsigned long long)g, wf[g], want[g]);
      return false;
    }
  return true;
}

template <int W, int SWD>
bool check_swd(const ExArgs& a, const std::vector<uint64_t>& keys, uint64_t nS, const std::vector<uint8_t>& sfl,
               const SortedView& S, const WordSlots& ws, const std::vector<uint8_t>& want, int k, int shrink) {
  if constexpr (SWD > W) {
    return false;
  } else {
    const uint64_t nb = 1ull << ws.bb;
    // every bucket must be written by the fill: start from a pattern
    std::vector<uint64_t> tab(nb * WS_SLOTS * SWD, 0xA5A5A5A5A5A5A5A5ull);
    for (uint64_t i = 0; i < nS; ++i)
      wslot_fill_one<W, SWD>(keys.data(), nS, sfl.data(), tab.data(), nb, ws.bb, ws.rbits, i);
    return run_lookups<W, SWD, 1>(a, tab, ws.bb, ws.rbits, S, sfl, want, k, shrink) &&
           run_lookups<W, SWD, 2>(a, tab, ws.bb, ws.rbits, S, sfl, want, k, shrink) &&
           run_lookups<W, SWD, 4>(a, tab, ws.bb, ws.rbits, S, sfl, want, k, shrink);
  }
}

template <int W>
bool check(int k, int shrink, std::mt19937_64& rng) {
  const int kb = 2 * (k + 1);
  const Stream st = make_stream(k, 700, rng);
  ExArgs a{};
  a.packed = st.packed.data();
  a.bad = st.bad.data();
  a.woff = st.woff.data();
  a.offsets = st.offsets.data();
  a.n_reads = st.n_reads;
  a.NW = st.NW;
  a.any_bad = st.any_bad ? 1 : 0;
  a.k = k;
  a.kb = kb;
  a.tr = st.tr.data();
  // window keys in window order (0x80 marks a window with a non-ACGT base)
  std::vector<uint64_t> wkeys(st.NW * W, 0);
  std::vector<uint8_t> clean(st.NW, 0);
  for (uint64_t r = 0, g = 0; r < st.n_reads; ++r)
    for (uint64_t i = 0; i < st.woff[r + 1] - st.woff[r]; ++i, ++g) {
      const uint64_t j = st.offsets[r] + i;
      bool ok = true;
      for (int t = 0; t <= k; ++t) ok = ok && !((st.bad[(j + t) / 64] >> ((j + t) % 64)) & 1);
      clean[g] = ok;
      key_store<W>(&wkeys[g * W], key_from_fwd<W>(stream_bits<W>(st.packed.data(), 2 * j, kb), kb));
    }
  // solid set: about 60% of the clean window keys and as many keys of no window
  std::vector<uint64_t> keys;
  for (uint64_t g = 0; g < st.NW; ++g)
    if (clean[g] && rng() % 10 < 6)
      for (int x = 0; x < W; ++x) keys.push_back(wkeys[g * W + x]);
  const uint64_t extra = keys.size() / W;
  for (uint64_t e = 0; e < extra; ++e) {
    Key<W> r;
    for (int x = 0; x < W; ++x) r.w[x] = rng();
    r = key_lowbits<W>(r, kb);
    for (int x = 0; x < W; ++x) keys.push_back(r.w[x]);
  }
  std::vector<size_t> ord(keys.size() / W);
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return less_key<W>(keys, x, y); });
  std::vector<uint64_t> sk;
  for (size_t i = 0; i < ord.size(); ++i)
    if (i == 0 || key_less<W>(key_load<W>(&keys[ord[i - 1] * W]), key_load<W>(&keys[ord[i] * W])))
      for (int x = 0; x < W; ++x) sk.push_back(keys[ord[i] * W + x]);
  const uint64_t nS = sk.size() / W;
  std::vector<uint8_t> sfl(nS);
  for (auto& f : sfl) f = (uint8_t)(1 | (rng() & 6));
  // directory over the top db bits
  const int db = std::min(kb, 10);
  std::vector<uint64_t> dir((1ull << db) + 1);
  for (uint64_t b = 0, i = 0; b <= (1ull << db); ++b) {
    while (i < nS && key_bits<W>(key_load<W>(&sk[i * W]), kb - db, db) < b) ++i;
    dir[b] = i;
  }
  const SortedView S{sk.data(), dir.data(), nS, kb, db};
  std::vector<uint8_t> want(st.NW);
  for (uint64_t g = 0; g < st.NW; ++g) {
    if (!clean[g]) {
      want[g] = 0x80;
      continue;
    }
    const Key<W> q = key_load<W>(&wkeys[g * W]);
    uint64_t lo = 0, hi = nS;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      if (key_less<W>(key_load<W>(&sk[mid * W]), q))
        lo = mid + 1;
      else
        hi = mid;
    }
    want[g] = lo < nS && key_eq<W>(key_load<W>(&sk[lo * W]), q) ? sfl[lo] : 0;
  }
  const WordSlots ws = word_slots_shape(kb, W, nS, shrink);
  switch (ws.swd) {
    case 1: return check_swd<W, 1>(a, sk, nS, sfl, S, ws, want, k, shrink);
    case 2: return check_swd<W, 2>(a, sk, nS, sfl, S, ws, want, k, shrink);
    case 3: return check_swd<W, 3>(a, sk, nS, sfl, S, ws, want, k, shrink);
    case 4: return check_swd<W, 4>(a, sk, nS, sfl, S, ws, want, k, shrink);
  }
  std::printf("bad slot width %d\n", ws.swd);
  return false;
}

}  // namespace

int main() {
  std::mt19937_64 rng(0x1409720801ull);
  for (int k : {32, 47, 62, 63, 64, 71, 80, 94, 95, 96, 110, 127})
    for (int shrink : {0, 4}) {
      const int w = (2 * (k + 1) + 63) / 64;
      const bool ok = w == 2 ? check<2>(k, shrink, rng) : w == 3 ? check<3>(k, shrink, rng) : check<4>(k, shrink, rng);
      if (!ok) return 1;
    }
  std::printf("ok\n");
  return 0;
}
