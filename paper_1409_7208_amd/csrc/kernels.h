// Kernel-side building blocks shared by the counting and graph stages.
#pragma once

#include "device.h"

namespace sdbg {

// Tile shapes per key width W (64-bit words per key).
//   IPT : windows per thread in the extraction partition (2 keys each)
//   TK  : keys per workgroup tile in the segment partition, a multiple of
//         512 (one word: 28 KB of keys, so five workgroups fit a CU's LDS)
//   CAP : most keys a leaf workgroup sorts in LDS
template <int W>
struct Tune;
template <>
struct Tune<1> {
  static constexpr int IPT = 6, TK = 3584, CAP = 2048;
};
template <>
struct Tune<2> {
  static constexpr int IPT = 4, TK = 2048, CAP = 1024;
};
template <>
struct Tune<3> {
  static constexpr int IPT = 2, TK = 1024, CAP = 1024;
};
template <>
struct Tune<4> {
  static constexpr int IPT = 2, TK = 1024, CAP = 1024;
};

// OR a 2-bit value into an even bit position.
template <int W>
DEV Key<W> key_or2(const Key<W>& a, int pos, uint64_t v) {
  Key<W> r = a;
  int li = pos >> 6, s = pos & 63;
#pragma unroll
  for (int j = 0; j < W; ++j)
    if (j == li) r.w[W - 1 - j] |= v << s;
  return r;
}

// n <= 64 bits starting at bit lo.
template <int W>
DEV uint64_t key_bits64(const Key<W>& k, int lo, int n) {
  int li = lo >> 6, s = lo & 63;
  uint64_t v = limb<W>(k, li) >> s;
  if (s && s + n > 64) v |= limb<W>(k, li + 1) << (64 - s);
  return n >= 64 ? v : (v & ((1ull << n) - 1));
}

// Sorted key array with a directory over its top `db` bits (of `kbits`
// significant bits): dir[b] = first index whose top bits are >= b, for
// b in [0, 2^db]; lookups binary-search one directory bucket.
struct SortedView {
  const uint64_t* keys;
  const uint64_t* dir;
  uint64_t n;
  int kbits, db;
};

template <int W>
DEV uint64_t sv_lower(const SortedView& v, const Key<W>& q) {
  uint32_t b = key_bits<W>(q, v.kbits - v.db, v.db);
  uint64_t lo = v.dir[b], hi = v.dir[b + 1];
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (key_less<W>(key_load<W>(v.keys + mid * W), q))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// First index whose key is > q.
template <int W>
DEV uint64_t sv_upper(const SortedView& v, const Key<W>& q) {
  uint32_t b = key_bits<W>(q, v.kbits - v.db, v.db);
  uint64_t lo = v.dir[b], hi = v.dir[b + 1];
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (!key_less<W>(q, key_load<W>(v.keys + mid * W)))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <int W>
DEV bool sv_find(const SortedView& v, const Key<W>& q, uint64_t* idx) {
  uint64_t i = sv_lower<W>(v, q);
  *idx = i;
  return i < v.n && key_eq<W>(key_load<W>(v.keys + i * W), q);
}

// Does some key x of the view have x[0..k-1] equal to node P (forward
// packing of a k-mer, 2k bits)?  The keys of the out-edges of P are
// P*4 + c, c in 0..3.
template <int W>
DEV bool sv_has_source(const SortedView& v, const Key<W>& P) {
  Key<W> q = key_shl<W>(P, 2);
  uint64_t i = sv_lower<W>(v, q);
  if (i >= v.n) return false;
  return key_eq<W>(key_shr<W>(key_load<W>(v.keys + i * W), 2), P);
}

// Does some key x of the view have x[1..k] equal to node P (2k bits)?  Such
// x = (c, P[0..k-2], P[k-1]) has key ((c + 4*P[0..k-2]) * 4 + P[k-1]) = base
// + 4c with base = P[0..k-2] * 16 + P[k-1]: at most 13 keys from base on.
template <int W>
DEV bool sv_has_target(const SortedView& v, const Key<W>& P, int k) {
  uint64_t last = key_bits<W>(P, 2 * k - 2, 2);
  Key<W> base = key_or_low<W>(key_shl<W>(key_lowbits<W>(P, 2 * k - 2), 4), last);
  Key<W> hi4 = key_shr<W>(base, 4);
  uint64_t i = sv_lower<W>(v, base);
  for (; i < v.n; ++i) {
    Key<W> x = key_load<W>(v.keys + i * W);
    if (!key_eq<W>(key_shr<W>(x, 4), hi4)) break;
    if ((x.w[W - 1] & 3) == last) return true;
  }
  return false;
}

// Edge key of the reverse complement of the (k+1)-mer with edge key x
// (kb = 2(k+1) bits): back to the forward packing (rotate right by one
// base), complement-reverse, rotate left again.
template <int W>
DEV Key<W> key_revcomp(const Key<W>& x, int kb) {
  const Key<W> F = key_or2<W>(key_shr<W>(x, 2), kb - 2, x.w[W - 1] & 3);
  return key_from_fwd<W>(revcomp_fwd<W>(F, kb), kb);
}

// Forward packing F and reverse-complement packing R of consecutive
// windows of a packed 2-bit stream (base j at bits 2(j mod 32) of word
// j/32), updated by one base per step instead of being rebuilt: the next
// window drops its first base from the bottom of F and takes the new base
// on top; R gains the new base's complement at the bottom.  A window that
// does not follow the one held (a new read, or the first window) is built
// from the stream.  kb = 2(k+1).
template <int W>
struct Roller {
  Key<W> F, R;
  uint64_t j = 0;     // stream position of the window held
  bool held = false;  // F and R hold the window at j
  DEV void at(const uint64_t* __restrict__ packed, int k, int kb, uint64_t pos) {
    if (held && pos == j + 1) {
      const uint64_t p = pos + (uint64_t)k;  // the new last base
      const uint64_t b = (packed[p >> 5] >> (2 * (p & 31))) & 3;
      F = key_or2<W>(key_shr<W>(F, 2), kb - 2, b);
      R = key_or_low<W>(key_lowbits<W>(key_shl<W>(R, 2), kb), 3 - b);
    } else {
      F = stream_bits<W>(packed, 2 * pos, kb);
      R = revcomp_fwd<W>(F, kb);
    }
    j = pos;
    held = true;
  }
  DEV Key<W> fwd_key(int kb) const { return key_from_fwd<W>(F, kb); }
  DEV Key<W> rc_key(int kb) const { return key_from_fwd<W>(R, kb); }
};

// Target node x[1..k] of edge key x (2k bits): (x >> 4) + x[k] * 4^(k-1).
template <int W>
DEV Key<W> edge_target(const Key<W>& x, int k) {
  return key_or2<W>(key_shr<W>(x, 4), 2 * k - 2, x.w[W - 1] & 3);
}

}  // namespace sdbg
