// Word-slot bucket table of the solid edge set (keys of two or more words):
// shape, fill (per solid key) and lookup (per window key).  The per-thread
// bodies of the fill and lookup kernels are __host__ __device__ functions,
// so host programs can replay them.
#pragma once

#include <algorithm>

#include "kernels.h"
#include "windows.h"

namespace sdbg {

// Solid set as a static bucket table for the per-window lookups of the
// mercy rule.  Window keys arrive in read order, i.e. at random places in
// key order, so a lookup should touch one short stretch of memory: random
// reads from a table of several GB are bound by the number of load
// requests and lines they make, so buckets are small and slots carry only
// what the bucket number does not.  Bucket b holds the solid keys whose top
// bb bits are b -- a contiguous range of the sorted solid set -- and is
// built from it by one pass without atomics.  Keys whose bucket holds more
// keys than slots are searched in the sorted set.
//
// Wider keys (two or more words): 4 slots of SWD words each.  A slot is the
// little-endian integer (key's low rbits bits) | (valid | dead-end flags) <<
// rbits; bit 64*SWD - 1 of slot 0 marks an overfull bucket.
constexpr int WS_SLOTS = 4;

struct WordSlots {
  int bb, rbits, swd;
};

inline WordSlots word_slots_shape(int kb, int W, uint64_t nS, int shrink) {
  WordSlots p{};
  const int bmin = std::max(1, kb + 5 - 64 * W);  // the slot must fit W words
  p.bb = bmin;
  while (p.bb < 30 && p.bb < kb && ((uint64_t)WS_SLOTS << p.bb) < 2 * nS) ++p.bb;
  p.bb = std::max(bmin, p.bb - shrink);
  p.rbits = kb - p.bb;
  p.swd = (p.rbits + 5 + 63) / 64;
  return p;
}

// Remainder bits of little-endian word i of a slot (0..64).
DEV int ws_bits(int rbits, int i) { return rbits - 64 * i >= 64 ? 64 : (rbits - 64 * i > 0 ? rbits - 64 * i : 0); }

DEV uint64_t ws_mask(int nbits) { return nbits >= 64 ? ~0ull : (nbits ? (~0ull >> (64 - nbits)) : 0ull); }

// One thread per solid key; the first key of each bucket (the sorted set
// holds a bucket's keys together) writes the whole bucket and clears the
// empty buckets between the previous key's bucket and its own (the last one
// also those after it), so every bucket is written exactly once.
template <int W, int SWD>
DEV void wslot_fill_one(const uint64_t* __restrict__ keys, uint64_t nS, const uint8_t* __restrict__ sfl,
                        uint64_t* __restrict__ tab, uint64_t nb, int bb, int rbits, uint64_t i) {
  if (i >= nS) return;
  const uint32_t b = key_bits<W>(key_load<W>(keys + i * W), rbits, bb);
  const uint64_t prev = i > 0 ? (uint64_t)key_bits<W>(key_load<W>(keys + (i - 1) * W), rbits, bb) : ~0ull;
  if (i > 0 && prev == b) return;
  const uint64_t lastb = key_bits<W>(key_load<W>(keys + (nS - 1) * W), rbits, bb);
  const uint64_t z1 = b == lastb ? nb : b;
  for (uint64_t e = prev + 1; e < z1; ++e)
    if (e != b)
      for (int x = 0; x < WS_SLOTS * SWD; ++x) tab[e * (WS_SLOTS * SWD) + x] = 0;
  const int fw = rbits >> 6, fs = rbits & 63;
  uint64_t* out = tab + (uint64_t)b * (WS_SLOTS * SWD);
  bool more = true;  // key i + j is still in bucket b
#pragma unroll
  for (int j = 0; j < WS_SLOTS; ++j) {
    uint64_t w[SWD];
#pragma unroll
    for (int x = 0; x < SWD; ++x) w[x] = 0;
    more = more && i + j < nS && (j == 0 || key_bits<W>(key_load<W>(keys + (i + j) * W), rbits, bb) == b);
    if (more) {
      const Key<W> k = key_load<W>(keys + (i + j) * W);
#pragma unroll
      for (int x = 0; x < SWD; ++x) w[x] = k.w[W - 1 - x] & ws_mask(ws_bits(rbits, x));
      const uint64_t fl = 8u | sfl[i + j];
#pragma unroll
      for (int x = 0; x < SWD; ++x) {
        if (x == fw) w[x] |= fl << fs;
        if (x == fw + 1 && fs > 60) w[x] |= fl >> (64 - fs);
      }
    }
    if (j == 0 && i + WS_SLOTS < nS && key_bits<W>(key_load<W>(keys + (i + WS_SLOTS) * W), rbits, bb) == b)
      w[SWD - 1] |= 1ull << 63;
#pragma unroll
    for (int x = 0; x < SWD; ++x) out[j * SWD + x] = w[x];
  }
}

template <int W, int SWD>
DEV uint8_t wslot_flags(const uint64_t* __restrict__ tab, const SortedView& S, const uint8_t* __restrict__ sfl,
                        const Key<W>& q, int bb, int rbits) {
  const uint64_t b = key_bits<W>(q, rbits, bb);
  const uint4* v = reinterpret_cast<const uint4*>(tab + b * (WS_SLOTS * SWD));
  uint64_t w[WS_SLOTS * SWD];
#pragma unroll
  for (int i = 0; i < WS_SLOTS * SWD / 2; ++i) {
    const uint4 x = v[i];
    w[2 * i] = x.x | ((uint64_t)x.y << 32);
    w[2 * i + 1] = x.z | ((uint64_t)x.w << 32);
  }
  const bool ovf = (w[SWD - 1] >> 63) != 0;
  const int fw = rbits >> 6, fs = rbits & 63;
  uint8_t f = 0;
#pragma unroll
  for (int j = 0; j < WS_SLOTS; ++j) {
    bool eq = true;
    uint64_t fl = 0;
#pragma unroll
    for (int i = 0; i < SWD; ++i) {
      const uint64_t m = ws_mask(ws_bits(rbits, i));
      eq = eq && ((w[j * SWD + i] ^ q.w[W - 1 - i]) & m) == 0;
      if (i == fw) fl |= w[j * SWD + i] >> fs;
      if (i == fw + 1 && fs > 60) fl |= w[j * SWD + i] << (64 - fs);
    }
    if (eq && (fl & 8)) f = (uint8_t)(fl & 7);
  }
  if (!f && ovf) {
    uint64_t ix;
    f = sv_find<W>(S, q, &ix) ? sfl[ix] : 0;
  }
  return f;
}

// Per forward-strand window: 0x80 if it holds a non-ACGT base, else the
// dead-end flags of its edge if solid, else 0.  Each thread takes IPT
// consecutive windows: their keys are built first, then all bucket lookups
// are issued together (independent loads in flight).  3-word keys are
// launched with IPT = 1: with two or more windows per thread the gfx950 code
// for that width lost lookups in every workgroup after the first one per CU
// (a loop-carried lane mask seeded from an undefined SGPR pair picked up the
// previous workgroup's register state), while the same functions replayed
// on the host are exact.
template <int W, int SWD, int IPT>
DEV void wslot_window_flags(const ExArgs& a, const uint64_t* __restrict__ tab, int bb, int rbits, const SortedView& S,
                            const uint8_t* __restrict__ sfl, uint8_t* __restrict__ wf, uint64_t g0) {
  if (g0 >= a.NW) return;
  WinIter it;
  it.init(a, g0);
  Key<W> key[IPT];
  bool ok[IPT];
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    ok[q] = false;
    key[q] = key_zero<W>();
    if (g0 + q < a.NW) {
      const uint64_t j = it.pos();
      if (!a.any_bad || window_clean(a.bad, j, a.k + 1)) {
        ok[q] = true;
        key[q] = key_from_fwd<W>(stream_bits<W>(a.packed, 2 * j, a.kb), a.kb);
      }
      it.next(a);
    }
  }
  uint8_t f[IPT];
#pragma unroll
  for (int q = 0; q < IPT; ++q) f[q] = ok[q] ? wslot_flags<W, SWD>(tab, S, sfl, key[q], bb, rbits) : (uint8_t)0x80;
#pragma unroll
  for (int q = 0; q < IPT; ++q)
    if (g0 + q < a.NW) wf[g0 + q] = f[q];
}

}  // namespace sdbg
