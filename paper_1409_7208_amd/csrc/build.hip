// SdBG arrays of a sorted edge set (Section 2, first paragraph: edge labels
// with minus flags, the last bit vector, F, the edge-validity bit vector
// and the 2kt-bit vector of zero-indegree vertex k-mers).
//
// Rows are the real edges E (already in key order), one '$' row per vertex
// with no outgoing edge (list Zout) and one dummy row per vertex with no
// incoming edge (list Zin).  Each list is produced in row order, and every
// row finds its final index as its index in its own list plus the number of
// rows of the two other lists that sort before it (directory lookups), so
// the merge is one scatter.  All row-order comparisons reduce to integer
// comparisons of edge keys and vertex packings:
//   real row of edge x, source v = x>>2 (a k-mer, forward packing P(v)):
//       after '$' rows whose vertex z has P(z) < P(v), after dummy rows with
//       v'[0..k-2] <= v[1..k-1];
//   '$' row of z: after real rows with key < P(z)*4, after dummy rows with
//       v'[0..k-2] <= z[1..k-1];
//   dummy row of v': after real rows with key < v'[0..k-2]*16, after '$'
//       rows with P(z) < v'[0..k-2]*4.
// A dummy row is stored by its "dummy key" v'[0..k-2]*4 + v'[k-1]; dummy
// rows sort by that key.

#include "engine.h"
#include "kernels.h"
#include "prims.h"

namespace sdbg {

namespace {

inline unsigned grid1(uint64_t n) {
  uint64_t g = ceil_div(n, SDBG_BLOCK);
  SDBG_CHECK(g < (1ull << 31), -1, "grid too large");
  return (unsigned)(g ? g : 1);
}

// First index in [lo, hi) whose key is >= q.
template <int W>
DEV uint64_t lower_in(const uint64_t* keys, uint64_t lo, uint64_t hi, const Key<W>& q) {
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (key_less<W>(key_load<W>(keys + mid * W), q))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Row flags in two passes over tiles of consecutive edges.  The target of
// an edge with label c and source v is the node c*4^(k-1) + (v div 4), so
// over a tile (sources ascending) the targets of its label-c edges ascend
// within one range, and the out-edges of those targets form one stretch of
// E per label.  A tile finds its four stretches (8 searches), stages them
// in LDS and answers every edge's "has my target an out-edge" there (in the
// stretch in global memory when they do not fit).  The same answer says
// that the found target has an in-edge: its first out-edge is marked in
// hin, and the second pass gives the dummy-row bit to every first edge of
// a source that no edge marked.  Final flags per edge: bit0 minus, bit1
// '$' row for its target (the target has no out-edge and this is the first
// edge into it), bit2 dummy row for its source (first edge of the source,
// and the source has no in-edge), bit3 last; the first pass keeps "first
// edge of its source" in bit4, which the second replaces by bit2.
template <int W>
struct RowTile {
  static constexpr int IPT = W == 1 ? 8 : (W == 2 ? 4 : 2);
  static constexpr int TILE = SDBG_BLOCK * IPT;
  static constexpr int RCAP = 2 * TILE;  // staged stretch keys (about TILE expected)
};

template <int W>
DEV uint64_t lds_lower(const uint64_t* R, uint32_t lo, uint32_t hi, const Key<W>& q) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (key_less<W>(key_load<W>(R + (uint64_t)mid * W), q))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <int W>
__global__ __launch_bounds__(SDBG_BLOCK) void k_row_out(SortedView E, int k, uint8_t* __restrict__ fl,
                                                        uint8_t* __restrict__ hin) {
  constexpr int IPT = RowTile<W>::IPT, TILE = RowTile<W>::TILE, RCAP = RowTile<W>::RCAP;
  __shared__ uint64_t R[RCAP * W];
  __shared__ uint64_t rg[8];
  const uint64_t i0 = blockIdx.x * (uint64_t)TILE;
  const uint64_t i1 = i0 + TILE < E.n ? i0 + TILE : E.n;
  if (threadIdx.x < 8) {
    // stretch of label c = threadIdx.x / 2: from the first key >= T(first
    // edge) * 4 (even threads) to the first key > T(last edge) * 4 + 3
    const uint32_t c = threadIdx.x >> 1;
    const bool hi = threadIdx.x & 1;
    const Key<W> xs = key_load<W>(E.keys + (hi ? i1 - 1 : i0) * W);
    const Key<W> T4 = key_shl<W>(key_or2<W>(key_shr<W>(xs, 4), 2 * k - 2, c), 2);
    rg[threadIdx.x] = hi ? sv_upper<W>(E, key_or_low<W>(T4, 3)) : sv_lower<W>(E, T4);
  }
  __syncthreads();
  uint64_t lo[4];
  uint32_t off[5];
  off[0] = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    lo[c] = rg[2 * c];
    const uint64_t len = rg[2 * c + 1] - rg[2 * c];
    off[c + 1] = off[c] + (uint32_t)(len < (uint64_t)RCAP ? len : (uint64_t)RCAP + 1);
  }
  const bool staged = off[4] <= (uint32_t)RCAP;
  if (staged) {
    for (uint32_t j = threadIdx.x; j < off[4]; j += SDBG_BLOCK) {
      int c = 0;
#pragma unroll
      for (int u = 1; u < 4; ++u)
        if (j >= off[u]) c = u;
      key_store<W>(R + (uint64_t)j * W, key_load_g<W>(E.keys + (lo[c] + (j - off[c])) * W));
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    const uint64_t i = i0 + (uint64_t)q * SDBG_BLOCK + threadIdx.x;
    if (i >= i1) continue;
    const Key<W> x = key_load<W>(E.keys + i * W);
    const uint32_t c = (uint32_t)(x.w[W - 1] & 3);
    const Key<W> T = edge_target<W>(x, k);
    const Key<W> T4 = key_shl<W>(T, 2);
    bool has_out;
    uint64_t io;
    if (staged) {
      uint32_t end = off[0], beg = off[0];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((uint32_t)u == c) {
          beg = off[u];
          end = off[u + 1];
        }
      const uint32_t j = (uint32_t)lds_lower<W>(R, beg, end, T4);
      has_out = j < end && key_eq<W>(key_shr<W>(key_load<W>(R + (uint64_t)j * W), 2), T);
      io = j - beg;
    } else {
      uint64_t l = 0, h = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((uint32_t)u == c) {
          l = rg[2 * u];
          h = rg[2 * u + 1];
        }
      const uint64_t j = lower_in<W>(E.keys, l, h, T4);
      has_out = j < h && key_eq<W>(key_shr<W>(key_load<W>(E.keys + j * W), 2), T);
      io = j - l;
    }
    if (has_out) {
      uint64_t l = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((uint32_t)u == c) l = lo[u];
      hin[l + io] = 1;
    }
    const Key<W> grp = key_shr<W>(x, 4), src = key_shr<W>(x, 2);
    bool minus = false;
    for (uint64_t j = i; j-- > 0;) {
      const Key<W> y = key_load<W>(E.keys + j * W);
      if (!key_eq<W>(key_shr<W>(y, 4), grp)) break;
      if ((y.w[W - 1] & 3) == c) {
        minus = true;
        break;
      }
    }
    const bool first = i == 0 || !key_eq<W>(key_shr<W>(key_load<W>(E.keys + (i - 1) * W), 2), src);
    const bool last = i + 1 == E.n || !key_eq<W>(key_shr<W>(key_load<W>(E.keys + (i + 1) * W), 2), src);
    fl[i] = (uint8_t)((minus ? 1 : 0) | (!minus && !has_out ? 2 : 0) | (last ? 8 : 0) | (first ? 16 : 0));
  }
}

// Second pass: eight edges per thread.
__global__ __launch_bounds__(SDBG_BLOCK) void k_row_in(uint8_t* __restrict__ fl, const uint8_t* __restrict__ hin,
                                                       uint64_t n) {
  const uint64_t b = (blockIdx.x * (uint64_t)SDBG_BLOCK + threadIdx.x) * 8;
  if (b >= n) return;
  if (b + 8 <= n) {
    uint64_t f = *reinterpret_cast<const uint64_t*>(fl + b);
    const uint64_t h = *reinterpret_cast<const uint64_t*>(hin + b);
    const uint64_t first = f & 0x1010101010101010ull;
    // a byte of h is 0 or 1: (h * 16) marks the bytes whose edge was found
    const uint64_t zin = first & ~(h << 4);
    f = (f & ~0x1010101010101010ull) | (zin >> 2);
    *reinterpret_cast<uint64_t*>(fl + b) = f;
  } else {
    for (uint64_t i = b; i < n; ++i) {
      const uint8_t f = fl[i];
      fl[i] = (uint8_t)((f & ~16) | ((f & 16) && !hin[i] ? 4 : 0));
    }
  }
}

// Split of the flagged edges into 4 classes, keeping edge order within a
// class.  mode 0: '$' rows, class = label, value = target vertex P(z);
// mode 1: dummy rows, class = last base of the source, value = dummy key.
constexpr int SPLIT_IPT = 32;  // four 8-byte words of flags per thread
constexpr int SPLIT_TILE = SDBG_BLOCK * SPLIT_IPT;

// The flag bytes of edges [base, base + 8) as one word (one load; byte by
// byte at the end of the array, zero past it).  base is a multiple of 8.
DEV uint64_t flags8(const uint8_t* __restrict__ fl, uint64_t n, uint64_t base) {
  if (base + 8 <= n) return *reinterpret_cast<const uint64_t*>(fl + base);
  uint64_t f = 0;
  for (uint64_t q = 0; base + q < n && q < 8; ++q) f |= (uint64_t)fl[base + q] << (8 * q);
  return f;
}

// Class and value of flagged edge i.
template <int W>
DEV void split_item(const SortedView& E, int mode, int k, uint64_t i, uint32_t* cls, Key<W>* val) {
  Key<W> x = key_load<W>(E.keys + i * W);
  if (mode == 0) {
    *cls = (uint32_t)(x.w[W - 1] & 3);
    *val = edge_target<W>(x, k);
  } else {
    Key<W> P = key_shr<W>(x, 2);
    uint64_t top = key_bits<W>(P, 2 * k - 2, 2);
    *cls = (uint32_t)top;
    *val = key_or_low<W>(key_shl<W>(key_lowbits<W>(P, 2 * k - 2), 2), top);
  }
}

template <int W>
__global__ __launch_bounds__(SDBG_BLOCK) void k_split_count(SortedView E, const uint8_t* __restrict__ fl, int mode,
                                                            int k, uint64_t ntiles, uint64_t* __restrict__ tc) {
  __shared__ uint32_t h[4];
  if (threadIdx.x < 4) h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = blockIdx.x * (uint64_t)SPLIT_TILE + threadIdx.x * SPLIT_IPT;
  const uint64_t bit = mode ? 4 : 2;
  uint64_t f8[SPLIT_IPT / 8];
#pragma unroll
  for (int u = 0; u < SPLIT_IPT / 8; ++u) f8[u] = flags8(fl, E.n, base + 8 * u);
#pragma unroll
  for (int q = 0; q < SPLIT_IPT; ++q) {
    if (!((f8[q >> 3] >> (8 * (q & 7))) & bit)) continue;
    uint32_t cl;
    Key<W> v;
    split_item<W>(E, mode, k, base + q, &cl, &v);
    atomicAdd(&h[cl], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 4) tc[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

template <int W>
__global__ __launch_bounds__(SDBG_BLOCK) void k_split_write(SortedView E, const uint8_t* __restrict__ fl, int mode,
                                                            int k, uint64_t ntiles, const uint64_t* __restrict__ tcs,
                                                            uint64_t* __restrict__ out) {
  __shared__ uint64_t sc[SDBG_WAVES + 1];
  const uint64_t base = blockIdx.x * (uint64_t)SPLIT_TILE + threadIdx.x * SPLIT_IPT;
  const uint64_t bit = mode ? 4 : 2;
  uint64_t f8[SPLIT_IPT / 8];
#pragma unroll
  for (int u = 0; u < SPLIT_IPT / 8; ++u) f8[u] = flags8(fl, E.n, base + 8 * u);
  uint64_t packed = 0;  // 4 x 16-bit per-class counts of this thread
#pragma unroll
  for (int q = 0; q < SPLIT_IPT; ++q) {
    if (!((f8[q >> 3] >> (8 * (q & 7))) & bit)) continue;
    uint32_t cl;
    Key<W> v;
    split_item<W>(E, mode, k, base + q, &cl, &v);
    packed += 1ull << (16 * cl);
  }
  uint64_t tot;
  uint64_t ex = block_excl_scan<uint64_t>(packed, sc, &tot);
  uint64_t pos[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) pos[c] = tcs[c * ntiles + blockIdx.x] + ((ex >> (16 * c)) & 0xFFFF);
#pragma unroll
  for (int q = 0; q < SPLIT_IPT; ++q) {
    if (!((f8[q >> 3] >> (8 * (q & 7))) & bit)) continue;
    uint32_t cl;
    Key<W> v;
    split_item<W>(E, mode, k, base + q, &cl, &v);
    {
      uint64_t p = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c == (int)cl) p = pos[c]++;
      key_store<W>(out + p * W, v);
    }
  }
}

// The dummy rows arrive as 4 runs (by the source's last base), each sorted
// by dummy key; merge them by rank.
template <int W>
__global__ void k_merge4(const uint64_t* __restrict__ in, uint64_t t, const uint64_t* __restrict__ run_start,
                         uint64_t* __restrict__ out) {
  uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (j >= t) return;
  int c = 0;
  while (c < 3 && j >= run_start[c + 1]) ++c;
  Key<W> x = key_load<W>(in + j * W);
  uint64_t r = j - run_start[c];
  for (int o = 0; o < 4; ++o)
    if (o != c) r += lower_in<W>(in, run_start[o], run_start[o + 1], x) - run_start[o];
  key_store<W>(out + r * W, x);
}

// Lower bound of q1 in v1 and lower (first key >= q2) or, with UPPER2,
// upper bound (first key > q2) of q2 in v2, searched in lockstep so that the
// loads of the two searches overlap.
template <int W, bool UPPER2>
DEV void sv_bounds2(const SortedView& v1, const Key<W>& q1, const SortedView& v2, const Key<W>& q2, uint64_t* r1,
                    uint64_t* r2) {
  const uint32_t b1 = key_bits<W>(q1, v1.kbits - v1.db, v1.db), b2 = key_bits<W>(q2, v2.kbits - v2.db, v2.db);
  uint64_t lo1 = v1.dir[b1], hi1 = v1.dir[b1 + 1], lo2 = v2.dir[b2], hi2 = v2.dir[b2 + 1];
  while (lo1 < hi1 || lo2 < hi2) {
    const bool a1 = lo1 < hi1, a2 = lo2 < hi2;
    const uint64_t m1 = (lo1 + hi1) >> 1, m2 = (lo2 + hi2) >> 1;
    Key<W> k1 = key_zero<W>(), k2 = key_zero<W>();
    if (a1) k1 = key_load<W>(v1.keys + m1 * W);
    if (a2) k2 = key_load<W>(v2.keys + m2 * W);
    if (a1) {
      if (key_less<W>(k1, q1))
        lo1 = m1 + 1;
      else
        hi1 = m1;
    }
    if (a2) {
      if (UPPER2 ? !key_less<W>(q2, k2) : key_less<W>(k2, q2))
        lo2 = m2 + 1;
      else
        hi2 = m2;
    }
  }
  *r1 = lo1;
  *r2 = lo2;
}

// Row placement.  rf: bit0 last, bit1 valid, bit2 tip.  A real row's
// index is its edge index plus the '$' rows before it (Zo keys below its
// source) and the dummy rows before it (Zi keys up to its source's top
// k-1 symbols, then 3): both counts grow with the edge index, so a tile of
// consecutive edges needs only the stretches of Zo and Zi between the
// counts of its first and last edges.  Those are staged in LDS (a search
// in global memory when they do not fit) and each edge's counts are found
// there.
template <int W>
struct PlaceTile {
  static constexpr int IPT = W == 1 ? 8 : (W == 2 ? 4 : 2);
  static constexpr int TILE = SDBG_BLOCK * IPT;
  static constexpr int RCAP = 1024 / W;  // staged keys of each list (a few per tile expected)
};

template <int W, bool UPPER>
DEV uint64_t lds_bound(const uint64_t* R, uint32_t lo, uint32_t hi, const Key<W>& q) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    const Key<W> k = key_load<W>(R + (uint64_t)mid * W);
    if (UPPER ? !key_less<W>(q, k) : key_less<W>(k, q))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <int W, bool UPPER>
DEV uint64_t glob_bound(const uint64_t* keys, uint64_t lo, uint64_t hi, const Key<W>& q) {
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    const Key<W> k = key_load<W>(keys + mid * W);
    if (UPPER ? !key_less<W>(q, k) : key_less<W>(k, q))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <int W>
DEV Key<W> place_hi3(const Key<W>& x) {
  return key_or_low<W>(key_shl<W>(key_shr<W>(x, 4), 2), 3);
}

template <int W>
__global__ __launch_bounds__(SDBG_BLOCK) void k_place_real(SortedView E, const uint32_t* __restrict__ cnt,
                                                           const uint8_t* __restrict__ fl, SortedView Zo,
                                                           SortedView Zi, uint8_t* __restrict__ Wb,
                                                           uint32_t* __restrict__ mult, uint8_t* __restrict__ rf) {
  constexpr int IPT = PlaceTile<W>::IPT, TILE = PlaceTile<W>::TILE, RCAP = PlaceTile<W>::RCAP;
  __shared__ uint64_t RO[RCAP * W], RI[RCAP * W];
  __shared__ uint64_t rg[4];
  const uint64_t i0 = blockIdx.x * (uint64_t)TILE;
  const uint64_t i1 = i0 + TILE < E.n ? i0 + TILE : E.n;
  if (threadIdx.x < 4) {
    // Zo lower bounds of the first and last sources, Zi upper bounds of
    // their hi3 keys
    const Key<W> x = key_load<W>(E.keys + ((threadIdx.x & 1) ? i1 - 1 : i0) * W);
    uint64_t r;
    if (threadIdx.x < 2) {
      uint64_t a, b;
      sv_bounds2<W, true>(Zo, key_shr<W>(x, 2), Zi, place_hi3<W>(x), &a, &b);
      r = a;
    } else {
      uint64_t a, b;
      sv_bounds2<W, true>(Zo, key_shr<W>(x, 2), Zi, place_hi3<W>(x), &a, &b);
      r = b;
    }
    rg[threadIdx.x] = r;
  }
  __syncthreads();
  const uint64_t o0 = rg[0], o1 = rg[1], z0 = rg[2], z1 = rg[3];
  const bool so = o1 - o0 <= (uint64_t)RCAP, si = z1 - z0 <= (uint64_t)RCAP;
  if (so)
    for (uint32_t j = threadIdx.x; j < (uint32_t)(o1 - o0); j += SDBG_BLOCK)
      key_store<W>(RO + (uint64_t)j * W, key_load_g<W>(Zo.keys + (o0 + j) * W));
  if (si)
    for (uint32_t j = threadIdx.x; j < (uint32_t)(z1 - z0); j += SDBG_BLOCK)
      key_store<W>(RI + (uint64_t)j * W, key_load_g<W>(Zi.keys + (z0 + j) * W));
  __syncthreads();
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    const uint64_t i = i0 + (uint64_t)q * SDBG_BLOCK + threadIdx.x;
    if (i >= i1) continue;
    const Key<W> x = key_load<W>(E.keys + i * W);
    const Key<W> src = key_shr<W>(x, 2), hi3 = place_hi3<W>(x);
    const uint64_t ro = so ? o0 + lds_bound<W, false>(RO, 0, (uint32_t)(o1 - o0), src)
                           : glob_bound<W, false>(Zo.keys, o0, o1, src);
    const uint64_t ri = si ? z0 + lds_bound<W, true>(RI, 0, (uint32_t)(z1 - z0), hi3)
                           : glob_bound<W, true>(Zi.keys, z0, z1, hi3);
    const uint64_t p = i + ro + ri;
    const uint8_t f = fl[i];
    Wb[p] = (uint8_t)(((x.w[W - 1] & 3) + 1) | ((f & 1) ? 8 : 0));
    mult[p] = cnt[i];
    rf[p] = (uint8_t)(((f & 8) ? 1 : 0) | 2);
  }
}

template <int W>
__global__ void k_place_zout(SortedView E, SortedView Zo, SortedView Zi, uint8_t* __restrict__ Wb,
                             uint32_t* __restrict__ mult, uint8_t* __restrict__ rf) {
  uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (j >= Zo.n) return;
  const Key<W> z = key_load<W>(Zo.keys + j * W);
  const Key<W> hi3 = key_or_low<W>(key_shl<W>(key_shr<W>(z, 2), 2), 3);
  uint64_t re, ri;
  sv_bounds2<W, true>(E, key_shl<W>(z, 2), Zi, hi3, &re, &ri);
  const uint64_t p = j + re + ri;
  Wb[p] = 0;
  mult[p] = 0;
  rf[p] = 1;
}

template <int W>
__global__ void k_place_zin(SortedView E, SortedView Zo, SortedView Zi, uint8_t* __restrict__ Wb,
                            uint32_t* __restrict__ mult, uint8_t* __restrict__ rf) {
  uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (j >= Zi.n) return;
  const Key<W> y = key_load<W>(Zi.keys + j * W);
  const Key<W> hv = key_shr<W>(y, 2);
  uint64_t re, ro;
  sv_bounds2<W, false>(E, key_shl<W>(hv, 4), Zo, key_shl<W>(hv, 2), &re, &ro);
  const uint64_t p = j + re + ro;
  const bool last = j + 1 == Zi.n || !key_eq<W>(key_shr<W>(key_load<W>(Zi.keys + (j + 1) * W), 2), hv);
  Wb[p] = (uint8_t)((y.w[W - 1] & 3) + 1);
  mult[p] = 0;
  rf[p] = (uint8_t)(4 | (last ? 1 : 0));
}

// Each thread takes 8 consecutive rows (one 8-byte load of their flags) and
// makes one byte of each bit vector; the 8 threads of a group of 64 rows
// OR their bytes together (3 shuffles), and the group's first thread
// writes the word.
__global__ __launch_bounds__(SDBG_BLOCK) void k_pack_bits(const uint8_t* __restrict__ rf, uint64_t m,
                                                          uint64_t* __restrict__ last, uint64_t* __restrict__ valid,
                                                          uint64_t* __restrict__ tip) {
  const uint64_t t = blockIdx.x * (uint64_t)SDBG_BLOCK + threadIdx.x;
  const uint64_t r0 = t * 8;
  uint64_t f = 0;
  if (r0 + 8 <= m) {
    f = *reinterpret_cast<const uint64_t*>(rf + r0);
  } else {
    for (uint64_t q = 0; r0 + q < m && q < 8; ++q) f |= (uint64_t)rf[r0 + q] << (8 * q);
  }
  uint64_t bl = 0, bv = 0, bt = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint64_t b = f >> (8 * q);
    bl |= (b & 1) << q;
    bv |= ((b >> 1) & 1) << q;
    bt |= ((b >> 2) & 1) << q;
  }
  const int sh = 8 * (int)(threadIdx.x & 7);
  bl <<= sh;
  bv <<= sh;
  bt <<= sh;
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    bl |= __shfl_xor(bl, o, 64);
    bv |= __shfl_xor(bv, o, 64);
    bt |= __shfl_xor(bt, o, 64);
  }
  if ((threadIdx.x & 7) == 0 && r0 < m) {
    last[r0 >> 6] = bl;
    valid[r0 >> 6] = bv;
    tip[r0 >> 6] = bt;
  }
}

// F: rows whose source ends in A, C, G (the last symbol of a source is the
// top base of the key, of P(z), and of the dummy key).
template <int W>
__global__ void k_F(SortedView E, SortedView Zo, SortedView Zi, int k, uint64_t* __restrict__ F) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint64_t m = E.n + Zo.n + Zi.n;
  F[0] = 0;
  F[1] = 0;
  for (int s = 1; s < 4; ++s) {
    Key<W> one = key_zero<W>();
    one.w[W - 1] = (uint64_t)s;
    F[s + 1] = sv_lower<W>(E, key_shl<W>(one, 2 * k)) + sv_lower<W>(Zo, key_shl<W>(one, 2 * k - 2)) +
               sv_lower<W>(Zi, key_shl<W>(one, 2 * k - 2));
  }
  F[5] = m;
}

// tip_seq word w gathers the 2k-bit packings of the dummy vertices that
// overlap bits [64w, 64w+64).
template <int W>
__global__ void k_tipseq(const uint64_t* __restrict__ zi, uint64_t t, int k, uint64_t words, uint64_t* __restrict__ out) {
  uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (w >= words) return;
  const uint64_t fb = 2ull * k, b0 = 64 * w, b1 = b0 + 64;
  uint64_t r0 = b0 / fb, r1 = (b1 - 1) / fb;
  if (r1 >= t) r1 = t - 1;
  uint64_t acc = 0;
  for (uint64_t r = r0; r <= r1; ++r) {
    const Key<W> y = key_load<W>(zi + r * W);
    const Key<W> P = key_or2<W>(key_shr<W>(y, 2), 2 * k - 2, y.w[W - 1] & 3);
    const uint64_t fs = fb * r;
    const uint64_t lo = fs > b0 ? fs : b0, hi = (fs + fb) < b1 ? (fs + fb) : b1;
    acc |= key_bits64<W>(P, (int)(lo - fs), (int)(hi - lo)) << (lo - b0);
  }
  out[w] = acc;
}

template <int W>
__global__ void k_check_sorted_b(const uint64_t* __restrict__ keys, uint64_t n, int kbits, uint32_t* flags) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  Key<W> x = key_load<W>(keys + i * W);
  if (!key_eq<W>(key_lowbits<W>(x, kbits), x)) atomicOr(flags, 2u);
  if (i > 0 && !key_less<W>(key_load<W>(keys + (i - 1) * W), x)) atomicOr(flags, 1u);
}

template <int W>
__global__ void k_dir_b(const uint64_t* __restrict__ keys, uint64_t n, int kbits, int db, uint64_t* __restrict__ dir) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i > n) return;
  uint64_t b = i < n ? key_bits<W>(key_load<W>(keys + i * W), kbits - db, db) : (1ull << db);
  uint64_t from = i == 0 ? 0 : (uint64_t)key_bits<W>(key_load<W>(keys + (i - 1) * W), kbits - db, db) + 1;
  for (uint64_t x = from; x <= b; ++x) dir[x] = i;
}

template <int W>
struct Builder {
  Ctx& c;
  explicit Builder(Ctx& c_) : c(c_) {}

  // Directory of about two keys per entry (at most 2^27 entries): the row
  // placement's lookups then take one or two steps after it.
  SortedView view(const uint64_t* keys, uint64_t n, int kbits, DBuf<uint64_t>& dir) {
    int db = 1;
    while (db < 27 && db < kbits && (n >> (db + 1)) > 0) ++db;
    dir = c.buf<uint64_t>((1ull << db) + 1);
    k_dir_b<W><<<grid1(n + 1), SDBG_BLOCK, 0, c.s>>>(keys, n, kbits, db, dir.get());
    c.check_launch("dir");
    return SortedView{keys, dir.get(), n, kbits, db};
  }

  // Compacts the flagged edges of one kind into `out` (row order within
  // each class); returns the 5 class boundaries.
  void split(const SortedView& E, const uint8_t* fl, int mode, int k, DBuf<uint64_t>& out, uint64_t bounds[5]) {
    const uint64_t ntiles = ceil_div(E.n, SPLIT_TILE);
    DBuf<uint64_t> tc = c.buf<uint64_t>(4 * ntiles + 1), tot = c.buf<uint64_t>(1);
    {
      Stage st_(c, "split_count", E.n);
      k_split_count<W><<<(unsigned)ntiles, SDBG_BLOCK, 0, c.s>>>(E, fl, mode, k, ntiles, tc.get());
      c.check_launch("split_count");
    }
    scan_excl<uint64_t, uint64_t>(tc.get(), tc.get(), 4 * ntiles, tc.get() + 4 * ntiles, c);
    uint64_t h[5];
    for (int q = 0; q < 4; ++q) h[q] = c.d2h_one(tc.get() + q * ntiles);
    h[4] = c.d2h_one(tc.get() + 4 * ntiles);
    for (int q = 0; q < 5; ++q) bounds[q] = h[q];
    out = c.buf<uint64_t>(h[4] * W);
    {
      Stage st_(c, "split_write", E.n + h[4] * 16 * W);
      k_split_write<W><<<(unsigned)ntiles, SDBG_BLOCK, 0, c.s>>>(E, fl, mode, k, ntiles, tc.get(), out.get());
      c.check_launch("split_write");
    }
  }

  void run(const uint64_t* keys, const uint32_t* count, uint64_t n, int k, GraphOut* g, bool check) {
    const int kb = 2 * (k + 1);
    *g = GraphOut{};
    if (n == 0) return;
    if (check) {
      DBuf<uint32_t> flags = c.buf<uint32_t>(1);
      fill<uint32_t>(flags.get(), 1, 0, c);
      k_check_sorted_b<W><<<grid1(n), SDBG_BLOCK, 0, c.s>>>(keys, n, kb, flags.get());
      c.check_launch("check_sorted");
      uint32_t f = c.d2h_one(flags.get());
      SDBG_CHECK(!(f & 2), -1, "edge key has bits above 2(k+1)");
      SDBG_CHECK(!(f & 1), -1, "edge keys are not strictly ascending");
    }
    DBuf<uint64_t> edir;
    SortedView E = view(keys, n, kb, edir);
    DBuf<uint8_t> fl = c.buf<uint8_t>(n);
    {
      DBuf<uint8_t> hin = c.buf<uint8_t>(n);
      fill<uint8_t>(hin.get(), n, 0, c);
      {
        // every edge key once, each stretch of targets once (about as many
        // keys), flags and marks
        Stage st_(c, "row_flags", n * (16 * W + 2));
        k_row_out<W><<<(unsigned)ceil_div(n, RowTile<W>::TILE), SDBG_BLOCK, 0, c.s>>>(E, k, fl.get(), hin.get());
        c.check_launch("row_flags");
      }
      {
        Stage st_(c, "row_in", n * 3);
        k_row_in<<<grid1(ceil_div(n, 8)), SDBG_BLOCK, 0, c.s>>>(fl.get(), hin.get(), n);
        c.check_launch("row_in");
      }
    }
    DBuf<uint64_t> zo, zi_runs, zi;
    uint64_t bo[5], bi[5];
    split(E, fl.get(), 0, k, zo, bo);
    split(E, fl.get(), 1, k, zi_runs, bi);
    const uint64_t nzo = bo[4], t = bi[4];
    zi = c.buf<uint64_t>(t * W);
    if (t) {
      DBuf<uint64_t> rs = c.buf<uint64_t>(5);
      c.h2d(rs.get(), bi, 5);
      k_merge4<W><<<grid1(t), SDBG_BLOCK, 0, c.s>>>(zi_runs.get(), t, rs.get(), zi.get());
      c.check_launch("merge4");
      c.sync();
    }
    zi_runs.free();
    DBuf<uint64_t> odir, idir;
    SortedView Zo = view(zo.get(), nzo, 2 * k, odir);
    SortedView Zi = view(zi.get(), t, 2 * k, idir);
    const uint64_t m = n + nzo + t;
    const uint64_t words = ceil_div(m, 64);
    DBuf<uint8_t> Wb = c.buf<uint8_t>(m), rf = c.buf<uint8_t>(m);
    DBuf<uint32_t> mult = c.buf<uint32_t>(m);
    {
      Stage st_(c, "place_real", n * (8 * W + 4 + 1) + n * 6);
      k_place_real<W><<<(unsigned)ceil_div(n, PlaceTile<W>::TILE), SDBG_BLOCK, 0, c.s>>>(E, count, fl.get(), Zo, Zi,
                                                                                        Wb.get(), mult.get(), rf.get());
      c.check_launch("place_real");
    }
    if (nzo) {
      k_place_zout<W><<<grid1(nzo), SDBG_BLOCK, 0, c.s>>>(E, Zo, Zi, Wb.get(), mult.get(), rf.get());
      c.check_launch("place_zout");
    }
    if (t) {
      k_place_zin<W><<<grid1(t), SDBG_BLOCK, 0, c.s>>>(E, Zo, Zi, Wb.get(), mult.get(), rf.get());
      c.check_launch("place_zin");
    }
    DBuf<uint64_t> last = c.buf<uint64_t>(words), valid = c.buf<uint64_t>(words), tip = c.buf<uint64_t>(words);
    {
      Stage st_(c, "pack_bits", m + 3 * words * 8);
      k_pack_bits<<<grid1(ceil_div(m, 8)), SDBG_BLOCK, 0, c.s>>>(rf.get(), m, last.get(), valid.get(), tip.get());
      c.check_launch("pack_bits");
    }
    DBuf<uint64_t> F = c.buf<uint64_t>(6);
    k_F<W><<<1, 64, 0, c.s>>>(E, Zo, Zi, k, F.get());
    c.check_launch("F");
    const uint64_t tw = ceil_div(2ull * k * t, 64);
    DBuf<uint64_t> ts = c.buf<uint64_t>(tw);
    if (tw) {
      k_tipseq<W><<<grid1(tw), SDBG_BLOCK, 0, c.s>>>(zi.get(), t, k, tw, ts.get());
      c.check_launch("tipseq");
    }
    c.d2h(g->F, F.get(), 6);
    g->m = m;
    g->t = t;
    g->tip_words = tw;
    g->W = Wb.release_ownership();
    g->mult = mult.release_ownership();
    g->last = last.release_ownership();
    g->valid = valid.release_ownership();
    g->tip = tip.release_ownership();
    g->tip_seq = ts.release_ownership();
  }
};

}  // namespace

void build_graph(const uint64_t* keys, const uint32_t* count, uint64_t n, int k, Ctx& c, GraphOut* out, bool check) {
  switch (key_words(k)) {
    case 1: Builder<1>(c).run(keys, count, n, k, out, check); break;
    case 2: Builder<2>(c).run(keys, count, n, k, out, check); break;
    case 3: Builder<3>(c).run(keys, count, n, k, out, check); break;
    case 4: Builder<4>(c).run(keys, count, n, k, out, check); break;
    default: throw Error(-1, "k out of range");
  }
}

}  // namespace sdbg
