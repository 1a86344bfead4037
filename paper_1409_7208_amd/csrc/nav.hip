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
  for (uint64_t i = lo << 6;; ++i)
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
    } else {  // OP_LABEL: walk back, one base per step, until k bases or a dummy row
      uint64_t w[4] = {0, 0, 0, 0};
      auto put = [&](int pos, uint64_t b) { w[(2 * pos) >> 6] |= b << ((2 * pos) & 63); };
      if (bit(v.tip, u)) {
        for (int j = 0; j < lw; ++j) out[t * lw + j] = NONE;
        return;
      }
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
      for (int j = 0; j < lw; ++j) out[t * lw + j] = w[j];
    }
  }
}

// Tip removal (Section 2, fourth paragraph, names it among the cleaning
// steps and gives no definition; the reading used here): on the graph as
// built, a forward tip is a path v0 -> ... -> vj (1 <= j <= max_len edges)
// from a node with no incoming edge through nodes of in- and out-degree 1
// (v0: out-degree 1) to a node vj with in-degree >= 2 or out-degree 0; a
// backward tip is its mirror image, from a node with no outgoing edge back
// to a node with out-degree >= 2 or in-degree 0.  One thread per row: a
// dummy row starts a forward walk at the node it enters, a '$' row a
// backward walk at its node.  The walk is taken once to decide and, for a
// tip, again to clear the valid bits of its edges; validity is not read,
// so every tip is found on the graph as built and all are removed at once.
// n_removed counts the valid bits cleared.
__global__ void k_remove_tips(Nav v, uint64_t* __restrict__ valid, uint32_t max_len,
                              unsigned long long* __restrict__ n_removed) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= v.m) return;
  const bool fwd = bit(v.tip, i), bwd = (v.W[i] & 7) == 0;
  if (!fwd && !bwd) return;
  uint32_t len = 0;
  bool tip = false;
  if (fwd) {
    // a node of out-degree 1 has one row, its last row, which is its edge
    uint64_t cur = nav_forward(v, i);
    while (len < max_len && nav_outdeg(v, cur) == 1) {
      cur = nav_forward(v, cur);
      ++len;
      const uint64_t in = nav_indeg(v, cur);
      if (in >= 2 || nav_outdeg(v, cur) == 0) {
        tip = true;
        break;
      }
      if (in != 1) break;
    }
  } else {
    uint64_t cur = i;  // a node of out-degree 0 has one row, its '$' row
    while (len < max_len && nav_indeg(v, cur) == 1) {
      cur = node_of(v, in_row(v, cur, block_of(v, cur)));
      ++len;
      const uint64_t out = nav_outdeg(v, cur);
      if (out >= 2 || nav_indeg(v, cur) == 0) {
        tip = true;
        break;
      }
      if (out != 1) break;
    }
  }
  if (!tip) return;
  unsigned long long cleared = 0;
  uint64_t cur = fwd ? nav_forward(v, i) : i;
  for (uint32_t s = 0; s < len; ++s) {
    const uint64_t row = fwd ? cur : in_row(v, cur, block_of(v, cur));
    const unsigned long long bitm = 1ull << (row & 63);
    const unsigned long long old = atomicAnd(reinterpret_cast<unsigned long long*>(valid + (row >> 6)), ~bitm);
    cleared += (old & bitm) ? 1 : 0;
    cur = fwd ? nav_forward(v, cur) : node_of(v, row);
  }
  if (cleared) atomicAdd(n_removed, cleared);
}

}  // namespace

// The index borrows the graph's arrays and owns its counts.
struct NavIndex {
  Nav v;
  uint64_t* counts = nullptr;  // c_last, c_nt, c_tip, then c_cls
  uint32_t* sel = nullptr;     // select directories: node ends, then classes 0..3
};

}  // namespace sdbg

namespace sdbg_abi {
void free_index(void* p) {
  auto* ix = static_cast<sdbg::NavIndex*>(p);
  pool_free(ix->counts);
  pool_free(ix->sel);
  delete ix;
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
      k_remove_tips<<<(unsigned)ceil_div(g->m, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(ix->v, g->valid, max_len,
                                                                                  cnt.get());
      c.check_launch("remove_tips");
    }
    unsigned long long h = 0;
    c.d2h(&h, cnt.get(), 1);
    if (n_removed) *n_removed = h;
    return SDBG_OK;
  });
}

}  // extern "C"
