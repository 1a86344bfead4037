// Navigation of a succinct de Bruijn graph on the device: rank directories
// over the arrays sdbg_build emits and batched queries (Section 2, first
// paragraph: the SdBG supports traversal in constant time per step through
// rank and select over W, last and F).
//
// Rows are grouped into nodes by the last bit vector; a node is identified
// by the index of its last row.  Block c of the rows (F[c] <= row < F[c+1])
// holds the nodes whose k-mer ends in base c.  The r-th unflagged row with
// label c (minus = 0) is the unique edge that enters the r-th non-dummy node
// of block c; flagged c-rows enter the same node as the nearest earlier
// unflagged c-row.  A dummy node (tip rows) stands before a vertex with no
// incoming edge, and tip_seq holds that vertex's k-mer.
//
// Index: per 64 rows, cumulative counts of last bits, of last bits of
// non-dummy nodes, of tip bits, and of each of the 8 row classes (label
// 1..4, minus 0/1), and select directories (the block of every 256th one)
// for the non-dummy node ends and the four unflagged classes.  rank is one
// cumulative count plus a popcount over at most 64 rows; select is a
// binary search over the cumulative counts between two directory samples,
// then a scan of one 64-row block; a row's node end and the previous node
// end are found by scanning the last bits word by word.
#include <hip/hip_runtime.h>

#include <cstring>

#include "abi_common.h"
#include "device.h"
#include "prims.h"

namespace sdbg {
namespace {

constexpr uint64_t NONE = ~0ull;

// Select directories: the 64-row block that holds every SEL_S-th one, so a
// select searches the cumulative counts between two samples only.
constexpr uint64_t SEL_S = 256;

struct Nav {
  uint64_t m, nb;  // rows, 64-row blocks
  int k;
  uint64_t F[6];
  const uint8_t* W;
  const uint64_t *last, *tip, *tip_seq;
  const uint64_t *c_last, *c_nt, *c_tip;  // nb + 1 cumulative counts each
  const uint64_t* c_cls;                  // class-major: c_cls[s * (nb + 1) + b]
  const uint32_t* sel_nt;                 // select directory of non-dummy node ends
  const uint32_t* sel_cls;                // of the unflagged classes 0..3, sel_stride entries each
  uint64_t sel_stride;
};

// Row class of a W byte: label c in 1..4 and minus f -> f * 4 + c - 1; -1 for '$'.
DEV int row_class(uint8_t w) {
  const int c = w & 7;
  return c == 0 ? -1 : ((w >> 3) & 1) * 4 + c - 1;
}

// Bytes of x equal to v (exact, no carries between bytes).
DEV int count_bytes_eq(uint64_t x, uint8_t v) {
  const uint64_t y = x ^ (0x0101010101010101ull * v);
  const uint64_t nz = ((y & 0x7F7F7F7F7F7F7F7Full) + 0x7F7F7F7F7F7F7F7Full) | y;  // high bit set iff byte nonzero
  return __popcll(~nz & 0x8080808080808080ull);
}

// A bit vector as the and-not of two stored ones (b & ~nb; nb may be
// null), with its cumulative counts per 64-bit word.
struct Bits {
  const uint64_t *b, *nb, *cum;
  uint64_t nw;
  const uint32_t* sel;  // select directory, or null
  DEV uint64_t word(uint64_t w) const { return nb ? (b[w] & ~nb[w]) : b[w]; }
  DEV uint64_t rank(uint64_t i) const {  // ones in [0, i)
    const uint64_t w = i >> 6, r = i & 63;
    return cum[w] + (r ? (uint64_t)__popcll(word(w) & ((1ull << r) - 1)) : 0);
  }
  DEV uint64_t select(uint64_t r) const {  // position of the one of 0-based rank r (r < total)
    uint64_t lo = 0, hi = nw;  // last word w with cum[w] <= r
    if (sel) {
      const uint64_t j = r / SEL_S;
      lo = sel[j];
      if ((j + 1) * SEL_S < cum[nw]) hi = (uint64_t)sel[j + 1] + 1;
    }
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (cum[mid] <= r)
        lo = mid;
      else
        hi = mid;
    }
    uint64_t x = word(lo);
    for (uint64_t left = r - cum[lo]; left; --left) x &= x - 1;
    return (lo << 6) + (uint64_t)__builtin_ctzll(x);
  }
};

DEV Bits node_bits(const Nav& v) { return Bits{v.last, v.tip, v.c_nt, v.nb, v.sel_nt}; }  // ends of non-dummy nodes
DEV Bits tip_bits(const Nav& v) { return Bits{v.tip, nullptr, v.c_tip, v.nb, nullptr}; }

// Smallest set position >= i of b (one exists), by a scan of its words.
DEV uint64_t next_one(const uint64_t* b, uint64_t i) {
  uint64_t w = i >> 6;
  uint64_t x = b[w] & (~0ull << (i & 63));
  while (!x) x = b[++w];
  return (w << 6) + (uint64_t)__builtin_ctzll(x);
}

// Largest set position < i of b, or NONE.
DEV uint64_t prev_one(const uint64_t* b, uint64_t i) {
  if (i == 0) return NONE;
  uint64_t w = (i - 1) >> 6;
  uint64_t x = b[w] & (~0ull >> (63 - ((i - 1) & 63)));
  while (!x) {
    if (w == 0) return NONE;
    x = b[--w];
  }
  return (w << 6) + 63 - (uint64_t)__builtin_clzll(x);
}

// Eight bytes of W from row p on; rows past m read as 0xFF (no class).
DEV uint64_t w8(const Nav& v, uint64_t p) {
  if (p + 8 <= v.m) return *reinterpret_cast<const uint64_t*>(v.W + p);
  uint64_t x = ~0ull;
  for (uint64_t q = 0; p + q < v.m && q < 8; ++q) x = (x & ~(0xFFull << (8 * q))) | ((uint64_t)v.W[p + q] << (8 * q));
  return x;
}

// Rows of class s in [0, i).
DEV uint64_t rank_cls(const Nav& v, int s, uint64_t i) {
  const uint64_t b = i >> 6;
  uint64_t n = v.c_cls[(uint64_t)s * (v.nb + 1) + b];
  const uint8_t want = (uint8_t)((s >> 2) << 3 | ((s & 3) + 1));
  const uint64_t r = i & 63;
  for (uint64_t q = 0; q * 8 < r; ++q) {
    uint64_t x = w8(v, (b << 6) + q * 8);
    const uint64_t take = r - q * 8 < 8 ? r - q * 8 : 8;
    if (take < 8) x |= ~0ull << (8 * take);  // bytes past i become 0xFF (no class)
    n += count_bytes_eq(x, want);
  }
  return n;
}

// Row of the 0-based r-th row of class s (r < total), else NONE.
DEV uint64_t select_cls(const Nav& v, int s, uint64_t r) {
  const uint64_t* c = v.c_cls + (uint64_t)s * (v.nb + 1);
  if (r >= c[v.nb]) return NONE;
  uint64_t lo = 0, hi = v.nb;
  if (s < 4) {  // unflagged classes have select directories
    const uint32_t* sel = v.sel_cls + (uint64_t)s * v.sel_stride;
    const uint64_t j = r / SEL_S;
    lo = sel[j];
    if ((j + 1) * SEL_S < c[v.nb]) hi = (uint64_t)sel[j + 1] + 1;
  }
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (c[mid] <= r)
      lo = mid;
    else
      hi = mid;
  }
  const uint8_t want = (uint8_t)((s >> 2) << 3 | ((s & 3) + 1));
  uint64_t left = r - c[lo];
  uint64_t i = lo << 6;
  for (;; i += 8) {  // eight rows at a time up to the word that holds it
    const uint64_t n = (uint64_t)count_bytes_eq(w8(v, i), want);
    if (n > left) break;
    left -= n;
  }
  for (;; ++i)
    if (v.W[i] == want && left-- == 0) return i;
}

DEV int block_of(const Nav& v, uint64_t row) {
  int c = 1;
  while (c < 4 && row >= v.F[c + 1]) ++c;
  return c;
}

DEV bool bit(const uint64_t* b, uint64_t i) { return (b[i >> 6] >> (i & 63)) & 1; }

// Last row of the node that holds row i (the next last bit).
DEV uint64_t node_of(const Nav& v, uint64_t i) { return next_one(v.last, i); }

// Unflagged row entering non-dummy node u (its last row), block c.
DEV uint64_t in_row(const Nav& v, uint64_t u, int c) {
  const Bits N = node_bits(v);
  return select_cls(v, c - 1, N.rank(u) - N.rank(v.F[c]));
}

// The k-mer of non-dummy node u: put(j, base) for j = 0..k-1.  Walks back
// one base per step through the entering rows until k bases are known or
// a node entered by its dummy row, whose k-mer is in tip_seq.
template <typename Put>
DEV void node_kmer(const Nav& v, uint64_t u, Put put) {
  uint64_t cur = u;
  for (int s = 0; s < v.k; ++s) {
    const int cc = block_of(v, cur);
    put(v.k - 1 - s, (uint64_t)(cc - 1));  // base k-1-s of the node
    if (s + 1 == v.k) break;
    const uint64_t j = in_row(v, cur, cc);
    if (bit(v.tip, j)) {  // cur has no incoming edge: its k-mer is stored
      const uint64_t tr = tip_bits(v).rank(j);
      for (int i = s; i < v.k; ++i) {  // node base i - s = base i of cur
        const uint64_t b = 2 * ((uint64_t)v.k * tr + i);
        put(i - s, (v.tip_seq[b >> 6] >> (b & 63)) & 3);
      }
      break;
    }
    cur = node_of(v, j);
  }
}

__global__ void k_counts(const uint8_t* __restrict__ W, const uint64_t* __restrict__ last,
                         const uint64_t* __restrict__ tip, uint64_t m, uint64_t nb, uint64_t* __restrict__ p_last,
                         uint64_t* __restrict__ p_nt, uint64_t* __restrict__ p_tip, uint64_t* __restrict__ p_cls) {
  const uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const uint64_t l = last[b], t = tip[b];
  p_last[b] = __popcll(l);
  p_nt[b] = __popcll(l & ~t);
  p_tip[b] = __popcll(t);
  uint32_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const uint64_t r0 = b << 6, r1 = r0 + 64 < m ? r0 + 64 : m;
  for (uint64_t i = r0; i < r1; ++i) {
    const int s = row_class(W[i]);
    if (s >= 0) ++cnt[s];
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) p_cls[(uint64_t)s * (nb + 1) + b] = cnt[s];
}

// Node entered by the edge of row x (NONE for a '$' row): unflagged c-rows
// before x; a flagged row enters the node of the nearest earlier unflagged one.
DEV uint64_t nav_forward(const Nav& v, uint64_t x) {
  const int c = v.W[x] & 7;
  if (c == 0) return NONE;
  uint64_t r = rank_cls(v, c - 1, x);
  if ((v.W[x] >> 3) & 1) --r;
  const Bits N = node_bits(v);
  return N.select(N.rank(v.F[c]) + r);
}

// Outgoing edges of node u (its last row): the rows of the node, 0 for a
// node whose only row is a '$' row.
DEV uint64_t nav_outdeg(const Nav& v, uint64_t u) {
  if ((v.W[u] & 7) == 0) return 0;
  const uint64_t p = prev_one(v.last, u);  // last row of the previous node
  return u - (p == NONE ? 0 : p + 1) + 1;
}

// Incoming edges of node u (dummy rows not counted): its unflagged entering
// row and the flagged rows of the same label up to the next unflagged one.
DEV uint64_t nav_indeg(const Nav& v, uint64_t u) {
  if (bit(v.tip, u)) return 0;
  const int c = block_of(v, u);
  const uint64_t j = in_row(v, u, c);
  if (bit(v.tip, j)) return 0;  // entered only by its dummy row
  // flagged c-rows after j up to the next unflagged c-row
  uint64_t n = 1;
  for (uint64_t p = j + 1; p < v.m; ++p) {
    const uint8_t w = v.W[p];
    if (w == (uint8_t)c) break;
    n += w == (uint8_t)(c | 8);
  }
  return n;
}

// sel[j] = block holding the one of rank j * SEL_S, from the cumulative
// counts cum[0..nb] (one thread per block).
__global__ void k_select_dir(const uint64_t* __restrict__ cum, uint64_t nb, uint32_t* __restrict__ sel) {
  const uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (b >= nb) return;
  for (uint64_t j = (cum[b] + SEL_S - 1) / SEL_S; j * SEL_S < cum[b + 1]; ++j) sel[j] = (uint32_t)b;
}

constexpr int OP_NODE = 1, OP_FORWARD = 2, OP_BACKWARD = 3, OP_OUTDEG = 4, OP_INDEG = 5, OP_LABEL = 6;

__global__ void k_nav(Nav v, int op, const uint64_t* __restrict__ q, uint64_t n, uint64_t* __restrict__ out) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t x = q[t];
  const int lw = (2 * v.k + 63) / 64;  // words of a LABEL result
  if (x >= v.m) {
    if (op == OP_LABEL)
      for (int j = 0; j < lw; ++j) out[t * lw + j] = NONE;
    else
      out[t] = NONE;
    return;
  }
  if (op == OP_NODE) {
    out[t] = node_of(v, x);
  } else if (op == OP_FORWARD) {
    out[t] = nav_forward(v, x);
  } else if (op == OP_OUTDEG) {
    out[t] = nav_outdeg(v, node_of(v, x));
  } else {
    const uint64_t u = node_of(v, x);
    const int c = block_of(v, u);
    if (op == OP_BACKWARD) {
      out[t] = bit(v.tip, u) ? NONE : node_of(v, in_row(v, u, c));
    } else if (op == OP_INDEG) {
      out[t] = nav_indeg(v, u);
    } else {  // OP_LABEL
      if (bit(v.tip, u)) {
        for (int j = 0; j < lw; ++j) out[t * lw + j] = NONE;
        return;
      }
      uint64_t w[4] = {0, 0, 0, 0};
      node_kmer(v, u, [&](int pos, uint64_t b) { w[(2 * pos) >> 6] |= b << ((2 * pos) & 63); });
      for (int j = 0; j < lw; ++j) out[t * lw + j] = w[j];
    }
  }
}


// Unitigs of the valid edges (the contigs that Section 2, fourth paragraph
// and Fig. 1, carry from one k to the next; the paper gives no
// construction, so this is the reading implemented): maximal paths whose
// inner nodes have in- and out-degree 1, degrees counted over valid edges.
// An edge continues the unitig of its predecessor iff its source node is
// (in 1, out 1); the predecessor is then that node's one valid entering
// edge.  Ranks along each unitig come from pointer jumping over the
// predecessor links (a link jumps to its link's link each round, in two
// buffers so that every round reads the previous one; a row whose link
// reaches a unitig's first edge is resolved: it holds that edge and its
// distance from it).  The jumping runs over splitters -- every first edge
// and about one row in 64 -- after each splitter has walked the rows up to
// the next one (below); only when the valid edges hold cycles of (in 1,
// out 1) nodes, which have no first edge, does it run over every row: once
// a round resolves nothing new, the remaining rows lie on cycles, each
// cycle is opened at its smallest row (the minimum over the cycle by
// doubling) and the jumping resumes.

constexpr uint64_t DONE = 1ull << 63;  // anc[i] flag: i resolved, anc = first edge of its unitig

// Valid rows of node u (its last row); *only = one of them.
DEV uint32_t valid_out(const Nav& v, const uint64_t* valid, uint64_t u, uint64_t* only) {
  const uint64_t p = prev_one(v.last, u);
  uint32_t n = 0;
  for (uint64_t r = p == NONE ? 0 : p + 1; r <= u; ++r)
    if (bit(valid, r)) {
      ++n;
      *only = r;
    }
  return n;
}

// Valid rows entering node u (its last row); *only = one of them.
DEV uint32_t valid_in(const Nav& v, const uint64_t* valid, uint64_t u, uint64_t* only) {
  if (bit(v.tip, u)) return 0;  // a dummy node
  const int c = block_of(v, u);
  const uint64_t j = in_row(v, u, c);
  if (bit(v.tip, j)) return 0;  // entered by its dummy row only
  uint32_t n = 0;
  if (bit(valid, j)) {
    n = 1;
    *only = j;
  }
  for (uint64_t p = j + 1; p < v.m; ++p) {  // flagged c-rows up to the next unflagged one
    const uint8_t w = v.W[p];
    if (w == (uint8_t)c) break;
    if (w == (uint8_t)(c | 8) && bit(valid, p)) {
      ++n;
      *only = p;
    }
  }
  return n;
}

// Predecessor of valid row i on its unitig, or NONE if i starts one.
DEV uint64_t unitig_pred(const Nav& v, const uint64_t* valid, uint64_t i) {
  const uint64_t u = node_of(v, i);
  uint64_t o = NONE, in = NONE;
  if (valid_out(v, valid, u, &o) != 1) return NONE;
  if (valid_in(v, valid, u, &in) != 1) return NONE;
  return in;
}

// Wave-aggregated add of x to *n.
DEV void wave_add(unsigned long long* n, uint64_t x) {
#pragma unroll
  for (int o = 32; o; o >>= 1) x += __shfl_xor(x, o);
  if ((threadIdx.x & 63) == 0 && x) atomicAdd(n, (unsigned long long)x);
}

// anc = predecessor (unresolved) or the row itself | DONE (a first edge);
// NONE for rows that are not valid edges.  *n_open += unresolved rows.
__global__ void k_ut_init(Nav v, const uint64_t* __restrict__ valid, uint64_t* __restrict__ anc,
                          uint64_t* __restrict__ dist, unsigned long long* __restrict__ n_open,
                          unsigned long long* __restrict__ n_valid) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t open = 0, ok = 0;
  if (i < v.m) {
    if (!bit(valid, i)) {
      anc[i] = NONE;
      dist[i] = 0;
    } else {
      const uint64_t p = unitig_pred(v, valid, i);
      anc[i] = p == NONE ? (i | DONE) : p;
      dist[i] = p == NONE ? 0 : 1;
      open = p != NONE;
      ok = 1;
    }
  }
  wave_add(n_open, open);
  wave_add(n_valid, ok);
}

// One round of pointer jumping from (a0, d0) into (a1, d1).
__global__ void k_ut_jump(uint64_t m, const uint64_t* __restrict__ a0, const uint64_t* __restrict__ d0,
                          uint64_t* __restrict__ a1, uint64_t* __restrict__ d1,
                          unsigned long long* __restrict__ n_open) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t open = 0;
  if (i < m) {
    const uint64_t x = a0[i];
    if (x == NONE || (x & DONE)) {
      a1[i] = x;
      d1[i] = d0[i];
    } else {
      const uint64_t y = a0[x];
      a1[i] = y;
      d1[i] = d0[i] + d0[x];
      open = !(y & DONE);
    }
  }
  wave_add(n_open, open);
}

// Ones of the bit vector hb before position h (hcum: its counts per word,
// exclusive scan).
DEV uint64_t head_rank(const uint64_t* hb, const uint64_t* hcum, uint64_t h) {
  const uint64_t w = h >> 6, r = h & 63;
  return hcum[w] + (r ? (uint64_t)__popcll(hb[w] & ((1ull << r) - 1)) : 0);
}

// Splitters shorten the jumping: every first edge and about one valid row
// in SPLIT_INV (by a hash of the row) is a splitter; each splitter walks the
// successor links to the next splitter, labelling the rows it passes with
// its index and their distance from it; pointer jumping then runs over the
// splitters alone, and every row adds its distance to its splitter's.
constexpr int SPLIT_SHIFT = 6;  // one row in 64

DEV bool hashed_splitter(uint64_t i) { return ((i * 0x9E3779B97F4A7C15ull) >> (64 - SPLIT_SHIFT)) == 0; }

// succ[pred[i]] = i for rows with a predecessor (succ filled with NONE).
__global__ void k_ut_succ(uint64_t m, const uint64_t* __restrict__ anc, uint64_t* __restrict__ succ) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t x = anc[i];
  if (x != NONE && !(x & DONE)) succ[x] = i;
}

// Splitter bits and counts per 64-row word (one wave per word).
__global__ void k_ut_split_mark(uint64_t m, const uint64_t* __restrict__ anc, uint64_t* __restrict__ sb,
                                uint64_t* __restrict__ sc) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  bool sp = false;
  if (i < m) {
    const uint64_t x = anc[i];
    sp = x != NONE && ((x & DONE) || hashed_splitter(i));
  }
  const uint64_t b = __ballot(sp);
  if ((threadIdx.x & 63) == 0 && i < m) {
    sb[i >> 6] = b;
    sc[i >> 6] = __popcll(b);
  }
}

// slist[rank] = splitter row.
__global__ void k_ut_split_list(uint64_t m, const uint64_t* __restrict__ sb, const uint64_t* __restrict__ scum,
                                uint64_t* __restrict__ slist) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m || !bit(sb, i)) return;
  slist[head_rank(sb, scum, i)] = i;
}

// Splitter j walks to the next splitter: rows passed get lab = j and their
// distance from it; the next splitter t gets spred[t] = j and sdist[t] = its
// distance.  Segment j (the splitter and the rows it labels) has seglen[j]
// rows (TAIL set if it ends its unitig), segsum[j] = their sum of mult and
// seglast[j] = its last row.
// *n_walked += rows labelled.
constexpr uint64_t TAIL = 1ull << 63;

__global__ void k_ut_split_walk(uint64_t ns, const uint64_t* __restrict__ slist, const uint64_t* __restrict__ sb,
                                const uint64_t* __restrict__ scum, const uint64_t* __restrict__ succ,
                                const uint32_t* __restrict__ mult, uint64_t* __restrict__ lab,
                                uint64_t* __restrict__ off, uint64_t* __restrict__ spred, uint64_t* __restrict__ sdist,
                                uint64_t* __restrict__ seglen, uint64_t* __restrict__ segsum,
                                uint64_t* __restrict__ seglast, unsigned long long* __restrict__ n_walked) {
  const uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t walked = 0;
  if (j < ns) {
    const uint64_t s0 = slist[j];
    uint64_t r = succ[s0], o = 1, sum = mult[s0], prev = s0;
    while (r != NONE && !bit(sb, r)) {
      lab[r] = j;
      off[r] = o;
      sum += mult[r];
      prev = r;
      r = succ[r];
      ++o;
      ++walked;
    }
    if (r != NONE) {
      const uint64_t t = head_rank(sb, scum, r);
      spred[t] = j;
      sdist[t] = o;
    }
    seglen[j] = o | (r == NONE ? TAIL : 0);
    segsum[j] = sum;
    seglast[j] = prev;
  }
  wave_add(n_walked, walked);
}

// Splitter-level start of the jumping: anc = spred or self | DONE.
__global__ void k_ut_split_init(uint64_t ns, const uint64_t* __restrict__ spred, const uint64_t* __restrict__ sdist,
                                uint64_t* __restrict__ anc, uint64_t* __restrict__ dist,
                                unsigned long long* __restrict__ n_open) {
  const uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t open = 0;
  if (j < ns) {
    const uint64_t p = spred[j];
    anc[j] = p == NONE ? (j | DONE) : p;
    dist[j] = p == NONE ? 0 : sdist[j];
    open = p != NONE;
  }
  wave_add(n_open, open);
}

// Per splitter (once ranked): its segment's mult into its unitig's sum;
// the tail segment sets the unitig's length and last row, the first one its
// first row.
__global__ void k_ut_split_sums(uint64_t ns, const uint64_t* __restrict__ slist, const uint64_t* __restrict__ sanc,
                                const uint64_t* __restrict__ sdst, const uint64_t* __restrict__ seglen,
                                const uint64_t* __restrict__ segsum, const uint64_t* __restrict__ seglast,
                                const uint64_t* __restrict__ hb, const uint64_t* __restrict__ hcum,
                                uint64_t* __restrict__ first, uint64_t* __restrict__ len,
                                unsigned long long* __restrict__ msum, uint64_t* __restrict__ last) {
  const uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (j >= ns) return;
  const uint64_t h = slist[sanc[j] & ~DONE];
  const uint64_t u = head_rank(hb, hcum, h);
  atomicAdd(msum + u, (unsigned long long)segsum[j]);
  if (seglen[j] & TAIL) {
    len[u] = sdst[j] + (seglen[j] & ~TAIL);
    last[u] = seglast[j];
  }
  if (sanc[j] == (j | DONE)) first[u] = slist[j];
}

// Base k + distance of each valid row's unitig, from its splitter.
__global__ void k_ut_split_bases(uint64_t m, uint32_t k, const uint8_t* __restrict__ W,
                                 const uint64_t* __restrict__ anc0, const uint64_t* __restrict__ sb,
                                 const uint64_t* __restrict__ scum, const uint64_t* __restrict__ slist,
                                 const uint64_t* __restrict__ sanc, const uint64_t* __restrict__ sdst,
                                 const uint64_t* __restrict__ lab, const uint64_t* __restrict__ offr,
                                 const uint64_t* __restrict__ hb, const uint64_t* __restrict__ hcum,
                                 const uint64_t* __restrict__ off, uint8_t* __restrict__ seq) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m || anc0[i] == NONE) return;
  const bool sp = bit(sb, i);
  const uint64_t j = sp ? head_rank(sb, scum, i) : lab[i];
  const uint64_t u = head_rank(hb, hcum, slist[sanc[j] & ~DONE]);
  seq[off[u] + k + sdst[j] + (sp ? 0 : offr[i])] = "ACGT"[(W[i] & 7) - 1];
}

// Unresolved rows (on cycles): link = predecessor, mn = the row itself.
__global__ void k_cyc_init(Nav v, const uint64_t* __restrict__ valid, const uint64_t* __restrict__ anc,
                           uint64_t* __restrict__ link, uint64_t* __restrict__ mn) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= v.m) return;
  const uint64_t x = anc[i];
  if (x == NONE || (x & DONE)) {
    link[i] = NONE;
    return;
  }
  link[i] = unitig_pred(v, valid, i);
  mn[i] = i;
}

// mn1 = min over the 2^(r+1) rows ending at i along the cycle.
__global__ void k_cyc_min(uint64_t m, const uint64_t* __restrict__ l0, const uint64_t* __restrict__ mn0,
                          uint64_t* __restrict__ l1, uint64_t* __restrict__ mn1) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t x = l0[i];
  if (x == NONE) {
    l1[i] = NONE;
    return;
  }
  const uint64_t a = mn0[i], b = mn0[x];
  mn1[i] = a < b ? a : b;
  l1[i] = l0[x];
}

// Each cycle's smallest row becomes its first edge; the others link to
// their predecessors again.
__global__ void k_cyc_open(uint64_t m, const uint64_t* __restrict__ link, const uint64_t* __restrict__ mn,
                           const Nav v, const uint64_t* __restrict__ valid, uint64_t* __restrict__ anc,
                           uint64_t* __restrict__ dist, unsigned long long* __restrict__ n_cycles) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t opened = 0;
  if (i < m && link[i] != NONE) {
    if (mn[i] == i) {
      anc[i] = i | DONE;
      dist[i] = 0;
      opened = 1;
    } else {
      anc[i] = unitig_pred(v, valid, i);
      dist[i] = 1;
    }
  }
  wave_add(n_cycles, opened);
}

// First edges per 64-row word (one wave per word): bits and counts.
__global__ void k_ut_heads(uint64_t m, const uint64_t* __restrict__ anc, uint64_t* __restrict__ hb,
                           uint64_t* __restrict__ hc) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const bool h = i < m && anc[i] == (i | DONE);
  const uint64_t b = __ballot(h);
  if ((threadIdx.x & 63) == 0 && i < m) {
    hb[i >> 6] = b;
    hc[i >> 6] = __popcll(b);
  }
}

// Per valid row: its unitig's first row, length (max distance + 1) and
// multiplicity (sum of mult).
__global__ void k_ut_sums(uint64_t m, const uint64_t* __restrict__ anc, const uint64_t* __restrict__ dist,
                          const uint32_t* __restrict__ mult, const uint64_t* __restrict__ hb,
                          const uint64_t* __restrict__ hcum, uint64_t* __restrict__ first,
                          unsigned long long* __restrict__ len, unsigned long long* __restrict__ msum) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t x = anc[i];
  if (x == NONE) return;
  const uint64_t h = x & ~DONE;
  const uint64_t u = head_rank(hb, hcum, h);
  if (h == i) first[u] = i;
  atomicMax(len + u, (unsigned long long)(dist[i] + 1));
  atomicAdd(msum + u, (unsigned long long)mult[i]);
}

// last[u] = the row at distance len[u] - 1 of unitig u (rows ranked by
// jumping over every row).
__global__ void k_ut_last(uint64_t m, const uint64_t* __restrict__ anc, const uint64_t* __restrict__ dist,
                          const uint64_t* __restrict__ hb, const uint64_t* __restrict__ hcum,
                          const uint64_t* __restrict__ len, uint64_t* __restrict__ last) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t x = anc[i];
  if (x == NONE) return;
  const uint64_t u = head_rank(hb, hcum, x & ~DONE);
  if (dist[i] + 1 == len[u]) last[u] = i;
}

// offsets[u] += k * u (offsets hold the exclusive scan of the lengths).
__global__ void k_ut_offsets(uint64_t n, uint32_t k, uint64_t* __restrict__ off) {
  const uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (u <= n) off[u] += (uint64_t)k * u;
}

// Base k + dist of a unitig is the label of its edge at that distance.
__global__ void k_ut_edge_bases(uint64_t m, uint32_t k, const uint8_t* __restrict__ W,
                                const uint64_t* __restrict__ anc, const uint64_t* __restrict__ dist,
                                const uint64_t* __restrict__ hb, const uint64_t* __restrict__ hcum,
                                const uint64_t* __restrict__ off, uint8_t* __restrict__ seq) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t x = anc[i];
  if (x == NONE) return;
  const uint64_t u = head_rank(hb, hcum, x & ~DONE);
  seq[off[u] + k + dist[i]] = "ACGT"[(W[i] & 7) - 1];
}

// The first k bases of a unitig: the k-mer of its first edge's source node.
__global__ void k_ut_node_bases(Nav v, uint64_t n, const uint64_t* __restrict__ first,
                                const uint64_t* __restrict__ off, uint8_t* __restrict__ seq) {
  const uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (u >= n) return;
  uint8_t* out = seq + off[u];
  node_kmer(v, node_of(v, first[u]), [&](int pos, uint64_t b) { out[pos] = "ACGT"[b]; });
}

// Bubble merging and low-local-coverage removal (Section 2, fourth
// paragraph, lists both among the cleaning steps, without definitions; the
// readings implemented).  Both take the unitigs of the current valid edges;
// unitig u runs from s(u), the source node of its first edge, to t(u), the
// node its last edge enters; cycles take part in neither.
//  * Bubbles: unitigs of at most max_len edges sharing s and t form a group;
//    all but the one of highest mean multiplicity (mult(a) * len(b) against
//    mult(b) * len(a); ties to the smaller first row) are removed.  The
//    unitigs leaving a branching node are exactly its valid rows, so each
//    unitig compares itself with the unitigs of its start node's other rows.
//  * Low local coverage: the neighbouring edges of a unitig of at most
//    max_len edges are the valid edges other than its first and last that
//    leave or enter s or t; it is removed if there is one and
//    mult * count * 1000 < ratio_permille * len * (sum of their mult).
// One thread per unitig decides from the graph as given (a flag per
// unitig); a second launch walks the flagged unitigs and clears their
// valid bits, so every removal of a call is decided before any is made.

// f(row) for each valid row leaving node x (its last row).
template <typename F>
DEV void for_valid_out(const Nav& v, const uint64_t* valid, uint64_t x, F f) {
  const uint64_t p = prev_one(v.last, x);
  for (uint64_t r = p == NONE ? 0 : p + 1; r <= x; ++r)
    if (bit(valid, r)) f(r);
}

// f(row) for each valid row entering node x.
template <typename F>
DEV void for_valid_in(const Nav& v, const uint64_t* valid, uint64_t x, F f) {
  if (bit(v.tip, x)) return;
  const int c = block_of(v, x);
  const uint64_t j = in_row(v, x, c);
  if (bit(v.tip, j)) return;
  if (bit(valid, j)) f(j);
  for (uint64_t p = j + 1; p < v.m; ++p) {
    const uint8_t w = v.W[p];
    if (w == (uint8_t)c) break;
    if (w == (uint8_t)(c | 8) && bit(valid, p)) f(p);
  }
}

// Node entered by the last of the n edges of the unitig whose first row is
// r (*last = that edge's row), or NONE if the valid edges do not form such
// a path (a unitig set of another state of the graph).
DEV uint64_t unitig_end(const Nav& v, const uint64_t* valid, uint64_t r, uint64_t n, uint64_t* last) {
  for (uint64_t j = 1; j < n; ++j) {
    const uint64_t x = nav_forward(v, r);
    if (x == NONE) return NONE;
    uint64_t o = NONE;
    if (valid_out(v, valid, x, &o) != 1) return NONE;
    r = o;
  }
  *last = r;
  return nav_forward(v, r);
}

// Start node of unitig u if it may take part (at most max_len edges, first
// row valid, not a cycle), else NONE.
DEV uint64_t cleaning_start(const Nav& v, const uint64_t* valid, uint64_t r0, uint64_t len, uint32_t max_len) {
  if (len == 0 || len > max_len || r0 >= v.m || !bit(valid, r0)) return NONE;
  const uint64_t s = node_of(v, r0);
  uint64_t o;
  if (valid_in(v, valid, s, &o) == 1 && valid_out(v, valid, s, &o) == 1) return NONE;  // a cycle
  return s;
}

// Index of the unitig whose first row is r (first[] ascending), or NONE.
DEV uint64_t unitig_of_first(const uint64_t* first, uint64_t n, uint64_t r) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (first[mid] < r)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < n && first[lo] == r ? lo : NONE;
}

typedef unsigned __int128 u128;

__global__ void k_bubble_flags(Nav v, const uint64_t* __restrict__ valid, const uint64_t* __restrict__ first,
                               const uint64_t* __restrict__ len, const uint64_t* __restrict__ umult, uint64_t n,
                               uint32_t max_len, uint8_t* __restrict__ flag) {
  const uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (u >= n) return;
  flag[u] = 0;
  const uint64_t r0 = first[u], L = len[u];
  const uint64_t s = cleaning_start(v, valid, r0, L, max_len);
  if (s == NONE) return;
  uint64_t last;
  const uint64_t t = unitig_end(v, valid, r0, L, &last);
  if (t == NONE) return;
  bool beaten = false;
  for_valid_out(v, valid, s, [&](uint64_t r) {
    if (beaten || r == r0) return;
    const uint64_t w = unitig_of_first(first, n, r);
    if (w == NONE || len[w] > max_len) return;
    uint64_t l2;
    if (unitig_end(v, valid, r, len[w], &l2) != t) return;
    const u128 a = (u128)umult[w] * L, b = (u128)umult[u] * len[w];
    beaten = a > b || (a == b && r < r0);
  });
  flag[u] = beaten ? 1 : 0;
}

__global__ void k_low_cov_flags(Nav v, const uint64_t* __restrict__ valid, const uint32_t* __restrict__ mult,
                                const uint64_t* __restrict__ first, const uint64_t* __restrict__ len,
                                const uint64_t* __restrict__ umult, uint64_t n, uint32_t max_len,
                                uint32_t ratio_permille, uint8_t* __restrict__ flag) {
  const uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (u >= n) return;
  flag[u] = 0;
  const uint64_t r0 = first[u], L = len[u];
  const uint64_t s = cleaning_start(v, valid, r0, L, max_len);
  if (s == NONE) return;
  uint64_t last;
  const uint64_t t = unitig_end(v, valid, r0, L, &last);
  if (t == NONE) return;
  uint64_t sum = 0, cnt = 0;
  auto add = [&](uint64_t r) {
    if (r == r0 || r == last) return;
    sum += mult[r];
    ++cnt;
  };
  for_valid_out(v, valid, s, add);
  for_valid_in(v, valid, s, add);
  if (t != s) {
    for_valid_out(v, valid, t, add);
    for_valid_in(v, valid, t, add);
  }
  flag[u] = cnt && (u128)umult[u] * cnt * 1000 < (u128)ratio_permille * L * sum ? 1 : 0;
}

// Clears the valid bits of the flagged unitigs' edges; the unitigs are
// those of the rows set in `walk` (valid itself, or every real row).
__global__ void k_clear_flagged(Nav v, const uint64_t* walk, uint64_t* valid, const uint64_t* __restrict__ first,
                                const uint64_t* __restrict__ len, const uint8_t* __restrict__ flag, uint64_t n,
                                unsigned long long* __restrict__ n_removed) {
  const uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t cleared = 0;
  if (u < n && flag[u]) {
    uint64_t r = first[u];
    for (uint64_t j = 0; j < len[u]; ++j) {
      const unsigned long long m = 1ull << (r & 63);
      const unsigned long long old = atomicAnd(reinterpret_cast<unsigned long long*>(valid + (r >> 6)), ~m);
      cleared += (old & m) ? 1 : 0;
      if (j + 1 == len[u]) break;
      const uint64_t x = nav_forward(v, r);  // an inner node: its one row of `walk` is the next edge
      uint64_t o = NONE;
      if (x == NONE || valid_out(v, walk, x, &o) != 1) break;
      r = o;
    }
  }
  wave_add(n_removed, cleared);
}

// Tip removal (Section 2, fourth paragraph, names it among the cleaning
// steps and gives no definition; the reading used here): on the graph as
// built, a forward tip is a path v0 -> ... -> vj (1 <= j <= max_len edges)
// from a node with no incoming edge through nodes of in- and out-degree 1
// (v0: out-degree 1) to a node vj with in-degree >= 2 or out-degree 0; a
// backward tip is its mirror image, from a node with no outgoing edge back
// to a node with out-degree >= 2 or in-degree 0.  Such a path is exactly a
// unitig of the graph as built (every real row) whose ends have those
// degrees, so the tips are found on the unitigs of the real rows: one
// thread per unitig looks at its two end nodes, and the flagged unitigs'
// edges are cleared from the validity vector.  Validity is not read, so
// every tip is found on the graph as built and all are removed at once.

// Rows that are real edges (a label and no tip bit), one wave per word.
__global__ void k_real_rows(Nav v, uint64_t* __restrict__ real) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const bool r = i < v.m && (v.W[i] & 7) != 0 && !bit(v.tip, i);
  const uint64_t b = __ballot(r);
  if ((threadIdx.x & 63) == 0 && i < v.m) real[i >> 6] = b;
}

// flag[u] = unitig u of the real rows is a tip of at most max_len edges.
__global__ void k_tip_flags(Nav v, const uint64_t* __restrict__ real, const uint64_t* __restrict__ first,
                            const uint64_t* __restrict__ last, const uint64_t* __restrict__ len, uint64_t n,
                            uint32_t max_len, uint8_t* __restrict__ flag) {
  const uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (u >= n) return;
  flag[u] = 0;
  if (len[u] > max_len) return;
  const uint64_t s = node_of(v, first[u]), t = nav_forward(v, last[u]);
  uint64_t o;
  const uint32_t out_s = valid_out(v, real, s, &o), in_s = valid_in(v, real, s, &o);
  if (in_s == 1 && out_s == 1) return;  // a cycle
  const uint32_t out_t = valid_out(v, real, t, &o), in_t = valid_in(v, real, t, &o);
  const bool fwd = in_s == 0 && out_s == 1 && (in_t >= 2 || out_t == 0);
  const bool bwd = out_t == 0 && in_t == 1 && (out_s >= 2 || in_s == 0);
  flag[u] = fwd || bwd ? 1 : 0;
}

}  // namespace

// The index borrows the graph's arrays and owns its counts.
struct NavIndex {
  Nav v;
  uint64_t* counts = nullptr;  // c_last, c_nt, c_tip, then c_cls
  uint32_t* sel = nullptr;     // select directories: node ends, then classes 0..3
};

}  // namespace sdbg

namespace sdbg {

// Unitigs of the rows set in `valid` (real rows of g; the graph's validity
// or every real row), ranked as described above; with_seq = false stops
// after the first rows, lengths, multiplicities and last rows.
struct UnitigCore {
  uint64_t n = 0, n_cycles = 0, n_bases = 0;
  DBuf<uint64_t> first, len, msum, last, off;
  DBuf<uint8_t> seq;
};

static void unitig_core(const NavIndex* ix, const sdbg_graph* g, const uint64_t* valid, bool with_seq, Ctx& c,
                        UnitigCore* out) {
  const Nav& v = ix->v;
  const uint64_t m = g->m, nw = ceil_div(m, 64);
  SDBG_CHECK(ceil_div(m, SDBG_BLOCK) < (1ull << 31), SDBG_E_INVAL, "graph too large");
  const unsigned grid = (unsigned)ceil_div(m ? m : 1, SDBG_BLOCK);
  DBuf<uint64_t> a0 = c.buf<uint64_t>(m), a1 = c.buf<uint64_t>(m), d0 = c.buf<uint64_t>(m),
                 d1 = c.buf<uint64_t>(m);
  uint64_t* A[2] = {a0.get(), a1.get()};
  uint64_t* D[2] = {d0.get(), d1.get()};
  DBuf<unsigned long long> cnt = c.buf<unsigned long long>(3);  // open rows, cycles, valid rows
  uint64_t* cnt64 = reinterpret_cast<uint64_t*>(cnt.get());
  fill<uint64_t>(cnt64, 3, 0, c);
  int cur = 0;
  uint64_t open = 0, n_cycles = 0, n_valid = 0;
  if (m) {
    k_ut_init<<<grid, SDBG_BLOCK, 0, c.s>>>(v, valid, A[0], D[0], cnt.get(), cnt.get() + 2);
    c.check_launch("unitig links");
    uint64_t h3[3];
    c.d2h(h3, cnt64, 3);
    open = h3[0];
    n_valid = h3[2];
  }
  // Splitter ranking, for valid edges without cycles.  A[1] holds the
  // successor links, D[1] each row's splitter and offr its distance from it.
  DBuf<uint64_t> sb, scum, slist, seglen, segsum, seglast, offr, sa[2], sd[2];
  uint64_t ns = 0;
  int sc = 0;
  bool by_splitters = false;
  if (open) {
    fill<uint64_t>(A[1], m, NONE, c);
    k_ut_succ<<<grid, SDBG_BLOCK, 0, c.s>>>(m, A[0], A[1]);
    sb = c.buf<uint64_t>(nw);
    scum = c.buf<uint64_t>(nw + 1);
    k_ut_split_mark<<<grid, SDBG_BLOCK, 0, c.s>>>(m, A[0], sb.get(), scum.get());
    c.check_launch("unitig splitters");
    scan_excl<uint64_t, uint64_t>(scum.get(), scum.get(), nw, scum.get() + nw, c);
    ns = c.d2h_one(scum.get() + nw);
  }
  if (open && ns) {  // (no splitter at all: the open rows lie on cycles)
    const unsigned sgrid = (unsigned)ceil_div(ns, SDBG_BLOCK);
    slist = c.buf<uint64_t>(ns);
    seglen = c.buf<uint64_t>(ns);
    segsum = c.buf<uint64_t>(ns);
    seglast = c.buf<uint64_t>(ns);
    offr = c.buf<uint64_t>(m);
    for (int q = 0; q < 2; ++q) {
      sa[q] = c.buf<uint64_t>(ns);
      sd[q] = c.buf<uint64_t>(ns);
    }
    DBuf<uint64_t> spred = c.buf<uint64_t>(ns), sdist = c.buf<uint64_t>(ns);
    k_ut_split_list<<<grid, SDBG_BLOCK, 0, c.s>>>(m, sb.get(), scum.get(), slist.get());
    fill<uint64_t>(spred.get(), ns, NONE, c);
    fill<uint64_t>(cnt64, 1, 0, c);
    k_ut_split_walk<<<sgrid, SDBG_BLOCK, 0, c.s>>>(ns, slist.get(), sb.get(), scum.get(), A[1], g->mult, D[1],
                                                   offr.get(), spred.get(), sdist.get(), seglen.get(),
                                                   segsum.get(), seglast.get(), cnt.get());
    c.check_launch("unitig splitter walks");
    const uint64_t walked = c.d2h_one(cnt64);
    if (walked + ns == n_valid) {  // every row reached: no cycle without a splitter
      fill<uint64_t>(cnt64, 1, 0, c);
      k_ut_split_init<<<sgrid, SDBG_BLOCK, 0, c.s>>>(ns, spred.get(), sdist.get(), sa[0].get(), sd[0].get(),
                                                     cnt.get());
      c.check_launch("unitig splitter links");
      uint64_t sopen = c.d2h_one(cnt64);
      while (sopen) {
        fill<uint64_t>(cnt64, 1, 0, c);
        k_ut_jump<<<sgrid, SDBG_BLOCK, 0, c.s>>>(ns, sa[sc].get(), sd[sc].get(), sa[sc ^ 1].get(),
                                                 sd[sc ^ 1].get(), cnt.get());
        c.check_launch("unitig splitter jump");
        sc ^= 1;
        const uint64_t now = c.d2h_one(cnt64);
        if (now == sopen) break;  // a cycle of splitters
        sopen = now;
      }
      by_splitters = sopen == 0;
    }
  }
  if (!by_splitters && open) {
    // Jumping over every row (the valid edges hold cycles), from the links
    // kernel's A[0] and D[0] ...
    auto jump = [&]() {
      while (open) {
        fill<uint64_t>(cnt64, 1, 0, c);
        k_ut_jump<<<grid, SDBG_BLOCK, 0, c.s>>>(m, A[cur], D[cur], A[cur ^ 1], D[cur ^ 1], cnt.get());
        c.check_launch("unitig jump");
        cur ^= 1;
        const uint64_t now = c.d2h_one(cnt64);
        if (now == open) break;  // only cycles are left
        open = now;
      }
    };
    jump();
    if (open) {  // ... then each cycle opened at its smallest row
      DBuf<uint64_t> l0 = c.buf<uint64_t>(m), l1 = c.buf<uint64_t>(m), n0 = c.buf<uint64_t>(m),
                     n1 = c.buf<uint64_t>(m);
      uint64_t* L[2] = {l0.get(), l1.get()};
      uint64_t* N[2] = {n0.get(), n1.get()};
      k_cyc_init<<<grid, SDBG_BLOCK, 0, c.s>>>(v, valid, A[cur], L[0], N[0]);
      c.check_launch("cycle links");
      int cc = 0;
      for (uint64_t span = 1; span < open; span <<= 1, cc ^= 1) {
        k_cyc_min<<<grid, SDBG_BLOCK, 0, c.s>>>(m, L[cc], N[cc], L[cc ^ 1], N[cc ^ 1]);
        c.check_launch("cycle minimum");
      }
      // the jumped links still mark the cycle rows (they never reach NONE)
      k_cyc_open<<<grid, SDBG_BLOCK, 0, c.s>>>(m, L[cc], N[cc], v, valid, A[cur], D[cur], cnt.get() + 1);
      c.check_launch("cycle open");
      n_cycles = c.d2h_one(cnt64 + 1);
      open -= n_cycles;
      jump();
      SDBG_CHECK(open == 0, SDBG_E_HIP, "unitig ranking did not converge");
    }
  }
  // first edges, ranked in row order (A[cur]: a first edge holds itself | DONE)
  DBuf<uint64_t> hb = c.buf<uint64_t>(nw ? nw : 1), hcum = c.buf<uint64_t>(nw + 1);
  if (nw) {
    k_ut_heads<<<grid, SDBG_BLOCK, 0, c.s>>>(m, A[cur], hb.get(), hcum.get());
    c.check_launch("unitig heads");
  }
  scan_excl<uint64_t, uint64_t>(hcum.get(), hcum.get(), nw, hcum.get() + nw, c);
  const uint64_t n = c.d2h_one(hcum.get() + nw);
  DBuf<uint64_t>& first = out->first;
  DBuf<uint64_t>& len = out->len;
  DBuf<uint64_t>& msum = out->msum;
  DBuf<uint64_t>& last = out->last;
  first = c.buf<uint64_t>(n ? n : 1);
  len = c.buf<uint64_t>(n ? n : 1);
  msum = c.buf<uint64_t>(n ? n : 1);
  last = c.buf<uint64_t>(n ? n : 1);
  fill<uint64_t>(len.get(), n, 0, c);
  fill<uint64_t>(msum.get(), n, 0, c);
  if (by_splitters) {
    k_ut_split_sums<<<(unsigned)ceil_div(ns, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(
        ns, slist.get(), sa[sc].get(), sd[sc].get(), seglen.get(), segsum.get(), seglast.get(), hb.get(),
        hcum.get(), first.get(), len.get(), reinterpret_cast<unsigned long long*>(msum.get()), last.get());
    c.check_launch("unitig sums");
  } else if (m) {
    k_ut_sums<<<grid, SDBG_BLOCK, 0, c.s>>>(m, A[cur], D[cur], g->mult, hb.get(), hcum.get(), first.get(),
                                            reinterpret_cast<unsigned long long*>(len.get()),
                                            reinterpret_cast<unsigned long long*>(msum.get()));
    c.check_launch("unitig sums");
    k_ut_last<<<grid, SDBG_BLOCK, 0, c.s>>>(m, A[cur], D[cur], hb.get(), hcum.get(), len.get(), last.get());
    c.check_launch("unitig last rows");
  }
  out->n = n;
  out->n_cycles = n_cycles;
  if (!with_seq) return;
  DBuf<uint64_t>& off = out->off;
  off = c.buf<uint64_t>(n + 1);
  scan_excl<uint64_t, uint64_t>(len.get(), off.get(), n, off.get() + n, c);
  k_ut_offsets<<<(unsigned)ceil_div(n + 1, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(n, g->k, off.get());
  c.check_launch("unitig offsets");
  const uint64_t n_bases = c.d2h_one(off.get() + n);
  out->n_bases = n_bases;
  DBuf<uint8_t>& seq = out->seq;
  seq = c.buf<uint8_t>(n_bases ? n_bases : 1);
  if (by_splitters) {
    k_ut_split_bases<<<grid, SDBG_BLOCK, 0, c.s>>>(m, g->k, g->W, A[0], sb.get(), scum.get(), slist.get(),
                                                   sa[sc].get(), sd[sc].get(), D[1], offr.get(), hb.get(),
                                                   hcum.get(), off.get(), seq.get());
    c.check_launch("unitig edge bases");
  } else if (m) {
    k_ut_edge_bases<<<grid, SDBG_BLOCK, 0, c.s>>>(m, g->k, g->W, A[cur], D[cur], hb.get(), hcum.get(),
                                                  off.get(), seq.get());
    c.check_launch("unitig edge bases");
  }
  if (n) {
    k_ut_node_bases<<<(unsigned)ceil_div(n, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(v, n, first.get(), off.get(),
                                                                              seq.get());
    c.check_launch("unitig node bases");
  }
}

}  // namespace sdbg

namespace sdbg_abi {
void free_index(void* p) {
  auto* ix = static_cast<sdbg::NavIndex*>(p);
  pool_free(ix->counts);
  pool_free(ix->sel);
  delete ix;
}

void free_unitigs(void* p) {
  auto* u = static_cast<sdbg_unitigs*>(p);
  pool_free(u->first_row);
  pool_free(u->len);
  pool_free(u->mult);
  pool_free(u->offsets);
  pool_free(u->seq);
  delete u;
}
}  // namespace sdbg_abi

extern "C" {

int sdbg_index_build(const sdbg_graph* g, const sdbg_params* params, sdbg_index** out) {
  using namespace sdbg;
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(g && out, SDBG_E_INVAL, "null argument");
    *out = nullptr;
    SDBG_CHECK(sdbg_abi::reg_kind(g) == 2, SDBG_E_INVAL, "not a graph returned by this library");
    Ctx c(params ? params->stream : nullptr);
    auto* ix = new NavIndex();
    try {
      Nav& v = ix->v;
      v.m = g->m;
      v.nb = ceil_div(g->m, 64);
      v.k = (int)g->k;
      std::memcpy(v.F, g->F, sizeof(v.F));
      v.W = g->W;
      v.last = g->last;
      v.tip = g->tip;
      v.tip_seq = g->tip_seq;
      const uint64_t nb = v.nb;
      DBuf<uint64_t> cnt = c.buf<uint64_t>(11 * (nb + 1));
      uint64_t* cl = cnt.get();
      uint64_t* cn = cl + (nb + 1);
      uint64_t* ct = cn + (nb + 1);
      uint64_t* cc = ct + (nb + 1);
      if (nb) {
        k_counts<<<(unsigned)ceil_div(nb, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(g->W, g->last, g->tip, g->m, nb, cl, cn,
                                                                          ct, cc);
        c.check_launch("nav counts");
      }
      for (int a = 0; a < 11; ++a) {  // each of the 11 arrays: exclusive scan, total at [nb]
        uint64_t* p = cl + (uint64_t)a * (nb + 1);
        scan_excl<uint64_t, uint64_t>(p, p, nb, p + nb, c);
      }
      v.c_last = cl;
      v.c_nt = cn;
      v.c_tip = ct;
      v.c_cls = cc;
      // select directories (at most m / SEL_S + 1 samples each)
      v.sel_stride = v.m / SEL_S + 2;
      DBuf<uint32_t> sel = c.buf<uint32_t>(5 * v.sel_stride);
      if (nb) {
        k_select_dir<<<(unsigned)ceil_div(nb, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(cn, nb, sel.get());
        for (int q = 0; q < 4; ++q)
          k_select_dir<<<(unsigned)ceil_div(nb, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(
              cc + (uint64_t)q * (nb + 1), nb, sel.get() + (uint64_t)(q + 1) * v.sel_stride);
        c.check_launch("nav select directories");
      }
      v.sel_nt = sel.get();
      v.sel_cls = sel.get() + v.sel_stride;
      c.sync();
      ix->counts = cnt.release_ownership();
      ix->sel = sel.release_ownership();
    } catch (...) {
      delete ix;
      throw;
    }
    sdbg_abi::reg_add(ix, sdbg_abi::kIndex);
    *out = reinterpret_cast<sdbg_index*>(ix);
    return SDBG_OK;
  });
}

int sdbg_navigate(const sdbg_index* index, int op, const uint64_t* rows, uint64_t n, uint64_t* out, void* stream) {
  using namespace sdbg;
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(index && (n == 0 || (rows && out)), SDBG_E_INVAL, "null argument");
    SDBG_CHECK(sdbg_abi::reg_kind(index) == sdbg_abi::kIndex, SDBG_E_INVAL, "not an index returned by this library");
    SDBG_CHECK(op >= OP_NODE && op <= OP_LABEL, SDBG_E_INVAL, "unknown navigation op");
    const NavIndex* ix = reinterpret_cast<const NavIndex*>(index);
    Ctx c(stream);
    if (n) {
      SDBG_CHECK(ceil_div(n, SDBG_BLOCK) < (1ull << 31), SDBG_E_INVAL, "too many queries");
      k_nav<<<(unsigned)ceil_div(n, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(ix->v, op, rows, n, out);
      c.check_launch("navigate");
    }
    c.sync();
    return SDBG_OK;
  });
}

int sdbg_remove_tips(sdbg_graph* g, const sdbg_index* index, uint32_t max_len, uint64_t* n_removed, void* stream) {
  using namespace sdbg;
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(g && index, SDBG_E_INVAL, "null argument");
    SDBG_CHECK(sdbg_abi::reg_kind(g) == sdbg_abi::kGraph, SDBG_E_INVAL, "not a graph returned by this library");
    SDBG_CHECK(sdbg_abi::reg_kind(index) == sdbg_abi::kIndex, SDBG_E_INVAL, "not an index returned by this library");
    const NavIndex* ix = reinterpret_cast<const NavIndex*>(index);
    SDBG_CHECK(ix->v.W == g->W && ix->v.m == g->m, SDBG_E_INVAL, "the index was not built on this graph");
    Ctx c(stream);
    DBuf<unsigned long long> cnt = c.buf<unsigned long long>(1);
    fill<uint64_t>(reinterpret_cast<uint64_t*>(cnt.get()), 1, 0, c);
    if (g->m && max_len) {
      SDBG_CHECK(ceil_div(g->m, SDBG_BLOCK) < (1ull << 31), SDBG_E_INVAL, "graph too large");
      DBuf<uint64_t> real = c.buf<uint64_t>(ceil_div(g->m, 64));
      k_real_rows<<<(unsigned)ceil_div(g->m, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(ix->v, real.get());
      c.check_launch("real rows");
      UnitigCore uc;
      unitig_core(ix, g, real.get(), false, c, &uc);
      if (uc.n) {
        const unsigned grid = (unsigned)ceil_div(uc.n, SDBG_BLOCK);
        DBuf<uint8_t> flag = c.buf<uint8_t>(uc.n);
        k_tip_flags<<<grid, SDBG_BLOCK, 0, c.s>>>(ix->v, real.get(), uc.first.get(), uc.last.get(), uc.len.get(),
                                                  uc.n, max_len, flag.get());
        c.check_launch("tip flags");
        k_clear_flagged<<<grid, SDBG_BLOCK, 0, c.s>>>(ix->v, real.get(), g->valid, uc.first.get(), uc.len.get(),
                                                      flag.get(), uc.n, cnt.get());
        c.check_launch("clear tips");
      }
    }
    unsigned long long h = 0;
    c.d2h(&h, cnt.get(), 1);
    if (n_removed) *n_removed = h;
    return SDBG_OK;
  });
}

int sdbg_unitigs_build(const sdbg_graph* g, const sdbg_index* index, sdbg_unitigs** out, void* stream) {
  using namespace sdbg;
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(g && index && out, SDBG_E_INVAL, "null argument");
    *out = nullptr;
    SDBG_CHECK(sdbg_abi::reg_kind(g) == sdbg_abi::kGraph, SDBG_E_INVAL, "not a graph returned by this library");
    SDBG_CHECK(sdbg_abi::reg_kind(index) == sdbg_abi::kIndex, SDBG_E_INVAL, "not an index returned by this library");
    const NavIndex* ix = reinterpret_cast<const NavIndex*>(index);
    SDBG_CHECK(ix->v.W == g->W && ix->v.m == g->m, SDBG_E_INVAL, "the index was not built on this graph");
    Ctx c(stream);
    UnitigCore uc;
    unitig_core(ix, g, g->valid, true, c, &uc);
    c.sync();
    auto* u = new sdbg_unitigs();
    u->k = g->k;
    u->n = uc.n;
    u->n_cycles = uc.n_cycles;
    u->n_bases = uc.n_bases;
    u->first_row = uc.first.release_ownership();
    u->len = uc.len.release_ownership();
    u->mult = uc.msum.release_ownership();
    u->offsets = uc.off.release_ownership();
    u->seq = uc.seq.release_ownership();
    sdbg_abi::reg_add(u, sdbg_abi::kUnitigs);
    *out = u;
    return SDBG_OK;
  });
}

int sdbg_unitigs_to_host(const sdbg_unitigs* u, uint64_t* first_row, uint64_t* len, uint64_t* mult,
                         uint64_t* offsets, uint8_t* seq) {
  using namespace sdbg;
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(u && sdbg_abi::reg_kind(u) == sdbg_abi::kUnitigs, SDBG_E_INVAL,
               "not a unitig set returned by this library");
    Ctx c(nullptr);
    if (first_row) c.d2h(first_row, u->first_row, u->n);
    if (len) c.d2h(len, u->len, u->n);
    if (mult) c.d2h(mult, u->mult, u->n);
    if (offsets) c.d2h(offsets, u->offsets, u->n + 1);
    if (seq) c.d2h(seq, u->seq, u->n_bases);
    return SDBG_OK;
  });
}

}  // extern "C"

// Shared body of the two unitig-based cleaning calls.
static int clean_by_unitigs(sdbg_graph* g, const sdbg_index* index, const sdbg_unitigs* u, uint32_t max_len,
                            int low_cov, uint32_t ratio_permille, uint64_t* n_removed, void* stream) {
  using namespace sdbg;
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(g && index && u, SDBG_E_INVAL, "null argument");
    SDBG_CHECK(sdbg_abi::reg_kind(g) == sdbg_abi::kGraph, SDBG_E_INVAL, "not a graph returned by this library");
    SDBG_CHECK(sdbg_abi::reg_kind(index) == sdbg_abi::kIndex, SDBG_E_INVAL, "not an index returned by this library");
    SDBG_CHECK(sdbg_abi::reg_kind(u) == sdbg_abi::kUnitigs, SDBG_E_INVAL,
               "not a unitig set returned by this library");
    const NavIndex* ix = reinterpret_cast<const NavIndex*>(index);
    SDBG_CHECK(ix->v.W == g->W && ix->v.m == g->m, SDBG_E_INVAL, "the index was not built on this graph");
    SDBG_CHECK(u->k == g->k, SDBG_E_INVAL, "unitigs of another k");
    Ctx c(stream);
    DBuf<unsigned long long> cnt = c.buf<unsigned long long>(1);
    fill<uint64_t>(reinterpret_cast<uint64_t*>(cnt.get()), 1, 0, c);
    if (u->n && max_len) {
      SDBG_CHECK(ceil_div(u->n, SDBG_BLOCK) < (1ull << 31), SDBG_E_INVAL, "too many unitigs");
      const unsigned grid = (unsigned)ceil_div(u->n, SDBG_BLOCK);
      DBuf<uint8_t> flag = c.buf<uint8_t>(u->n);
      if (low_cov)
        k_low_cov_flags<<<grid, SDBG_BLOCK, 0, c.s>>>(ix->v, g->valid, g->mult, u->first_row, u->len, u->mult, u->n,
                                                      max_len, ratio_permille, flag.get());
      else
        k_bubble_flags<<<grid, SDBG_BLOCK, 0, c.s>>>(ix->v, g->valid, u->first_row, u->len, u->mult, u->n, max_len,
                                                     flag.get());
      c.check_launch(low_cov ? "low coverage flags" : "bubble flags");
      k_clear_flagged<<<grid, SDBG_BLOCK, 0, c.s>>>(ix->v, g->valid, g->valid, u->first_row, u->len, flag.get(),
                                                    u->n, cnt.get());
      c.check_launch("clear flagged unitigs");
    }
    unsigned long long h = 0;
    c.d2h(&h, cnt.get(), 1);
    if (n_removed) *n_removed = h;
    return SDBG_OK;
  });
}

extern "C" {

int sdbg_merge_bubbles(sdbg_graph* g, const sdbg_index* index, const sdbg_unitigs* u, uint32_t max_len,
                       uint64_t* n_removed, void* stream) {
  return clean_by_unitigs(g, index, u, max_len, 0, 0, n_removed, stream);
}

int sdbg_remove_low_coverage(sdbg_graph* g, const sdbg_index* index, const sdbg_unitigs* u, uint32_t max_len,
                             uint32_t ratio_permille, uint64_t* n_removed, void* stream) {
  return clean_by_unitigs(g, index, u, max_len, 1, ratio_permille, n_removed, stream);
}

}  // extern "C"
