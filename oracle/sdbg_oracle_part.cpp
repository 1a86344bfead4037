// TEST INFRASTRUCTURE ONLY -- never linked into, loaded by, or called from
// the device library.  Only the tests, the scripts that write stored
// expected values, and the benchmark's CPU-baseline leg use it.
//
// Partitioned form of the oracle, for read sets too large for the
// string-based one (sdbg_oracle.cpp).  It computes the same things, from the
// same definitions (Section 2 of Li et al., MEGAHIT; the readings are the
// ones stated in sdbg_oracle.cpp), on packed integer keys instead of
// strings, one block of the key space at a time.  Section 2 (second
// paragraph) cuts the (k+1)-mers into blocks by their length-l colex prefix
// and processes consecutive blocks separately; here l = 4 (256 blocks, or
// one block when k < 8), and the blocks are handed to a pool of threads.
// Every step is the plain definition:
//   count     sort the keys of a block, count equal keys (both strands of
//             every window contribute one key each);
//   solid     count >= d;
//   mercy     per read, consecutive solid windows x, y with at least one
//             window between them, x with no solid out-edge and y with no
//             solid in-edge: the windows between and their reverse
//             complements; their counts are counted again over all reads;
//   rows      edges, one '$' row per vertex with no outgoing edge, one dummy
//             row per vertex with no incoming edge, ordered by source read
//             from its last symbol to its first, then label ($ < A < C < G < T);
//   arrays    W with minus flags, last, valid, tip, mult, F, tip_seq.
// It shares nothing with the device library.

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

namespace {

// Base-4 number of up to 256 bits, little-endian 64-bit limbs.
template <int W>
struct Big {
  std::array<uint64_t, W> v{};
  void push(int dgt) {  // *4 + dgt
    for (int i = W - 1; i > 0; --i) v[i] = (v[i] << 2) | (v[i - 1] >> 62);
    v[0] = (v[0] << 2) | (uint64_t)dgt;
  }
  int digit(int pos) const { return (int)((v[(2 * pos) / 64] >> ((2 * pos) % 64)) & 3); }
  Big shr_digits(int n) const {  // floor(x / 4^n), n < 32
    Big r;
    const int s = 2 * n;
    if (s == 0) return *this;
    for (int i = 0; i < W; ++i) r.v[i] = (v[i] >> s) | (i + 1 < W ? v[i + 1] << (64 - s) : 0);
    return r;
  }
  bool operator<(const Big& o) const {
    for (int i = W - 1; i >= 0; --i)
      if (v[i] != o.v[i]) return v[i] < o.v[i];
    return false;
  }
  bool operator==(const Big& o) const { return v == o.v; }
  bool operator!=(const Big& o) const { return !(v == o.v); }
};

int code_of(unsigned char c) {
  switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

int words_of(int k) { return (2 * (k + 1) + 63) / 64; }

// Blocks: the 4 most significant colex symbols of the key (8 bits), or a
// single block for k < 8.
int block_digits(int k) { return k >= 8 ? 4 : 0; }

// The ACGT stretches of read r as base codes.
template <typename F>
void for_each_segment(const uint8_t* seq, const uint64_t* off, uint64_t r, std::vector<int8_t>& buf, F&& f) {
  buf.clear();
  for (uint64_t p = off[r]; p < off[r + 1]; ++p) {
    const int c = code_of(seq[p]);
    if (c < 0) {
      if (!buf.empty()) f(buf);
      buf.clear();
    } else {
      buf.push_back((int8_t)c);
    }
  }
  if (!buf.empty()) f(buf);
}

// Digit j (most significant first, j = 0..k) of the key of window e =
// s[i..i+k]: e[k-1], e[k-2], ..., e[0], then e[k].
inline int fwd_digit(const int8_t* e, int k, int j) { return j < k ? e[k - 1 - j] : e[k]; }
// The same for the reverse complement of e: rc[m] = 3 - e[k-m], so the
// digits are 3-e[1], 3-e[2], ..., 3-e[k], then 3-e[0].
inline int rc_digit(const int8_t* e, int k, int j) { return j < k ? 3 - e[j + 1] : 3 - e[0]; }

template <int W, typename D>
Big<W> key_of(const int8_t* e, int k, D digit) {
  Big<W> x;
  for (int j = 0; j <= k; ++j) x.push(digit(e, k, j));
  return x;
}

template <typename D>
int block_of(const int8_t* e, int k, D digit) {
  int b = 0;
  for (int j = 0; j < block_digits(k); ++j) b = b * 4 + digit(e, k, j);
  return b;
}

template <int W>
int block_of_key(const Big<W>& x, int k) {
  int b = 0;
  for (int j = 0; j < block_digits(k); ++j) b = b * 4 + x.digit(k - j);
  return b;
}

void parallel_for(int threads, uint64_t n, const std::function<void(uint64_t, int)>& f) {
  std::atomic<uint64_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&, t] {
      for (uint64_t i; (i = next.fetch_add(1)) < n;) f(i, t);
    });
  for (auto& th : pool) th.join();
}

template <int W>
const Big<W>* find_key(const std::vector<Big<W>>& s, const std::vector<uint64_t>& bstart, int k, const Big<W>& x) {
  const int b = block_of_key(x, k);
  auto lo = s.begin() + (int64_t)bstart[b], hi = s.begin() + (int64_t)bstart[b + 1];
  auto it = std::lower_bound(lo, hi, x);
  return (it != hi && *it == x) ? &*it : nullptr;
}

template <int W>
int count_solid_w(const uint8_t* seq, const uint64_t* off, uint64_t n_reads, int k, uint32_t d, bool mercy,
                  int threads, uint64_t group_keys, uint64_t** keys_out, uint32_t** counts_out, uint64_t* n_out,
                  uint64_t* n_mercy_out, uint64_t* n_occ_out) {
  const int nb = 1 << (2 * block_digits(k));
  // keys of each block, for the grouping: 2 per window whose digits put it there
  std::vector<uint64_t> per_block(nb, 0);
  uint64_t n_occ = 0;
  {
    std::vector<std::vector<uint64_t>> part(threads, std::vector<uint64_t>(nb, 0));
    parallel_for(threads, n_reads, [&](uint64_t r, int t) {
      std::vector<int8_t> buf;
      for_each_segment(seq, off, r, buf, [&](const std::vector<int8_t>& s) {
        for (size_t i = 0; i + k + 1 <= s.size(); ++i) {
          part[t][block_of(&s[i], k, fwd_digit)] += 1;
          part[t][block_of(&s[i], k, rc_digit)] += 1;
        }
      });
    });
    for (int t = 0; t < threads; ++t)
      for (int b = 0; b < nb; ++b) per_block[b] += part[t][b];
    for (int b = 0; b < nb; ++b) n_occ += per_block[b];
  }

  // Count, one group of consecutive blocks at a time; keep solid keys.
  std::vector<std::vector<Big<W>>> S(nb);
  std::vector<std::vector<uint32_t>> Sc(nb);
  bool too_many = false;
  for (int b0 = 0; b0 < nb;) {
    int b1 = b0;
    uint64_t acc = 0;
    while (b1 < nb && (b1 == b0 || acc + per_block[b1] <= group_keys)) acc += per_block[b1++];
    std::vector<std::vector<std::vector<Big<W>>>> local(threads, std::vector<std::vector<Big<W>>>(b1 - b0));
    parallel_for(threads, n_reads, [&](uint64_t r, int t) {
      std::vector<int8_t> buf;
      for_each_segment(seq, off, r, buf, [&](const std::vector<int8_t>& s) {
        for (size_t i = 0; i + k + 1 <= s.size(); ++i) {
          const int bf = block_of(&s[i], k, fwd_digit), br = block_of(&s[i], k, rc_digit);
          if (bf >= b0 && bf < b1) local[t][bf - b0].push_back(key_of<W>(&s[i], k, fwd_digit));
          if (br >= b0 && br < b1) local[t][br - b0].push_back(key_of<W>(&s[i], k, rc_digit));
        }
      });
    });
    std::mutex mu;
    parallel_for(threads, (uint64_t)(b1 - b0), [&](uint64_t j, int) {
      std::vector<Big<W>> keys;
      for (int t = 0; t < threads; ++t) {
        keys.insert(keys.end(), local[t][j].begin(), local[t][j].end());
        std::vector<Big<W>>().swap(local[t][j]);
      }
      std::sort(keys.begin(), keys.end());
      std::vector<Big<W>> s;
      std::vector<uint32_t> c;
      for (size_t i = 0; i < keys.size();) {
        size_t e = i + 1;
        while (e < keys.size() && keys[e] == keys[i]) ++e;
        const uint64_t cnt = e - i;
        if (cnt >= d) {
          if (cnt > 0xffffffffull) {
            std::lock_guard<std::mutex> lk(mu);
            too_many = true;
          }
          s.push_back(keys[i]);
          c.push_back((uint32_t)cnt);
        }
        i = e;
      }
      S[b0 + j].swap(s);
      Sc[b0 + j].swap(c);
    });
    b0 = b1;
  }
  if (too_many) return -3;

  // All solid keys in key order (blocks are consecutive key ranges).
  std::vector<uint64_t> bstart(nb + 1, 0);
  for (int b = 0; b < nb; ++b) bstart[b + 1] = bstart[b] + S[b].size();
  std::vector<Big<W>> SA;
  std::vector<uint32_t> SC;
  SA.reserve(bstart[nb]);
  SC.reserve(bstart[nb]);
  for (int b = 0; b < nb; ++b) {
    SA.insert(SA.end(), S[b].begin(), S[b].end());
    SC.insert(SC.end(), Sc[b].begin(), Sc[b].end());
    std::vector<Big<W>>().swap(S[b]);
    std::vector<uint32_t>().swap(Sc[b]);
  }

  // Mercy: per read, on the forward strand, between consecutive solid windows.
  std::vector<Big<W>> M;
  std::vector<uint32_t> MC;
  if (mercy) {
    std::vector<std::vector<Big<W>>> local(threads);
    parallel_for(threads, n_reads, [&](uint64_t r, int t) {
      std::vector<int8_t> buf;
      for_each_segment(seq, off, r, buf, [&](const std::vector<int8_t>& s) {
        if (s.size() < (size_t)k + 1) return;
        const size_t nw = s.size() - k;
        std::vector<size_t> pos;
        for (size_t i = 0; i < nw; ++i)
          if (find_key(SA, bstart, k, key_of<W>(&s[i], k, fwd_digit))) pos.push_back(i);
        for (size_t a = 0; a + 1 < pos.size(); ++a) {
          const size_t p = pos[a], q = pos[a + 1];
          if (q - p < 2) continue;
          const int8_t* x = &s[p];
          const int8_t* y = &s[q];
          // x has an out-edge iff some edge x[1..k] c is solid; its key
          // digits are x[k], x[k-1], ..., x[1], then c
          bool x_out = false, y_in = false;
          for (int c = 0; c < 4 && !x_out; ++c) {
            Big<W> z;
            for (int j = 0; j < k; ++j) z.push(x[k - j]);
            z.push(c);
            x_out = find_key(SA, bstart, k, z) != nullptr;
          }
          // y has an in-edge iff some edge c y[0..k-1] is solid; its key
          // digits are y[k-2], ..., y[0], c, then y[k-1]
          for (int c = 0; c < 4 && !y_in; ++c) {
            Big<W> z;
            for (int j = k - 2; j >= 0; --j) z.push(y[j]);
            z.push(c);
            z.push(y[k - 1]);
            y_in = find_key(SA, bstart, k, z) != nullptr;
          }
          if (x_out || y_in) continue;
          for (size_t i = p + 1; i < q; ++i) {
            local[t].push_back(key_of<W>(&s[i], k, fwd_digit));
            local[t].push_back(key_of<W>(&s[i], k, rc_digit));
          }
        }
      });
    });
    for (auto& l : local) {
      M.insert(M.end(), l.begin(), l.end());
      std::vector<Big<W>>().swap(l);
    }
    std::sort(M.begin(), M.end());
    M.erase(std::unique(M.begin(), M.end()), M.end());
    // counts of the mercy edges, counted again over all windows
    std::vector<std::vector<uint32_t>> part(threads, std::vector<uint32_t>(M.size(), 0));
    std::vector<uint64_t> mstart(nb + 1, 0);
    for (const auto& x : M) mstart[block_of_key(x, k) + 1] += 1;
    for (int b = 0; b < nb; ++b) mstart[b + 1] += mstart[b];
    if (!M.empty())
      parallel_for(threads, n_reads, [&](uint64_t r, int t) {
        std::vector<int8_t> buf;
        for_each_segment(seq, off, r, buf, [&](const std::vector<int8_t>& s) {
          for (size_t i = 0; i + k + 1 <= s.size(); ++i) {
            for (int strand = 0; strand < 2; ++strand) {
              const int b = strand ? block_of(&s[i], k, rc_digit) : block_of(&s[i], k, fwd_digit);
              if (mstart[b] == mstart[b + 1]) continue;
              const Big<W> x = strand ? key_of<W>(&s[i], k, rc_digit) : key_of<W>(&s[i], k, fwd_digit);
              const Big<W>* f = find_key(M, mstart, k, x);
              if (f) part[t][f - M.data()] += 1;
            }
          }
        });
      });
    MC.assign(M.size(), 0);
    for (int t = 0; t < threads; ++t)
      for (size_t i = 0; i < M.size(); ++i) MC[i] += part[t][i];
  }

  // E = solid + mercy, merged in key order.
  const uint64_t n = SA.size() + M.size();
  uint64_t* keys = (uint64_t*)std::malloc(sizeof(uint64_t) * (n * W + 1));
  uint32_t* counts = (uint32_t*)std::malloc(sizeof(uint32_t) * (n + 1));
  if (!keys || !counts) {
    std::free(keys);
    std::free(counts);
    return -2;
  }
  size_t a = 0, b = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const bool from_s = b >= M.size() || (a < SA.size() && SA[a] < M[b]);
    const Big<W>& x = from_s ? SA[a] : M[b];
    for (int j = 0; j < W; ++j) keys[i * W + j] = x.v[W - 1 - j];
    counts[i] = from_s ? SC[a] : MC[b];
    if (from_s)
      ++a;
    else
      ++b;
  }
  *keys_out = keys;
  *counts_out = counts;
  *n_out = n;
  *n_mercy_out = M.size();
  *n_occ_out = n_occ;
  return 0;
}

// ------------------------------------------------------------------ build

// A row as its symbols, ranks $ = 0, A..T = 1..4, 3 bits each, most
// significant first: source[k-1], source[k-2], ..., source[0], label.
// Numeric order of the codes is the row order.
constexpr int kRowLimbs = 6;  // 3 * 128 bits
using RowCode = std::array<uint64_t, kRowLimbs>;

struct RowBuilder {
  int k;
  RowCode c{};
  int n = 0;
  void put(int rank) {  // appends a symbol (most significant first)
    const int pos = 3 * (kRowLimbs * 64 / 3 - 1 - n);  // bit position of this symbol's field
    c[kRowLimbs - 1 - pos / 64] |= (uint64_t)rank << (pos % 64);
    if (pos % 64 > 61) c[kRowLimbs - 2 - pos / 64] |= (uint64_t)rank >> (64 - pos % 64);
    ++n;
  }
};

// Field of symbol number idx (0 = source[k-1]) cleared.
RowCode without_symbol(RowCode c, int idx) {
  const int pos = 3 * (kRowLimbs * 64 / 3 - 1 - idx);
  c[kRowLimbs - 1 - pos / 64] &= ~((uint64_t)7 << (pos % 64));
  if (pos % 64 > 61) c[kRowLimbs - 2 - pos / 64] &= ~((uint64_t)7 >> (64 - pos % 64));
  return c;
}

struct Row {
  RowCode code;  // c[0] most significant limb
  uint8_t kind;  // 0 real, 1 '$' row, 2 dummy row
  uint8_t label;
  uint32_t mult;
  uint64_t node;  // index of the dummy row's vertex in the zero-indegree list
};

template <int W>
int build_w(const uint64_t* keys, const uint32_t* counts, uint64_t n, int k, int threads, void* gout);

}  // namespace

extern "C" {

// Same output as oracle_count_solid (sdbg_oracle.cpp), computed block by
// block on `threads` threads; consecutive blocks are counted together up to
// group_keys keys (0 = no limit) to bound memory.
int oracle_part_count_solid(const uint8_t* seq, const uint64_t* offsets, uint64_t n_reads, uint32_t k, uint32_t d,
                            uint32_t mercy, int threads, uint64_t group_keys, uint64_t** keys_out,
                            uint32_t** counts_out, uint64_t* n_out, uint64_t* n_mercy_out, uint64_t* n_occ_out) {
  if (k < 2 || k > 127 || d < 1) return -1;
  if (threads < 1) threads = 1;
  if (!group_keys) group_keys = ~0ull;
  switch (words_of((int)k)) {
    case 1:
      return count_solid_w<1>(seq, offsets, n_reads, (int)k, d, mercy != 0, threads, group_keys, keys_out, counts_out,
                              n_out, n_mercy_out, n_occ_out);
    case 2:
      return count_solid_w<2>(seq, offsets, n_reads, (int)k, d, mercy != 0, threads, group_keys, keys_out, counts_out,
                              n_out, n_mercy_out, n_occ_out);
    case 3:
      return count_solid_w<3>(seq, offsets, n_reads, (int)k, d, mercy != 0, threads, group_keys, keys_out, counts_out,
                              n_out, n_mercy_out, n_occ_out);
    default:
      return count_solid_w<4>(seq, offsets, n_reads, (int)k, d, mercy != 0, threads, group_keys, keys_out, counts_out,
                              n_out, n_mercy_out, n_occ_out);
  }
}

// Same output as oracle_build, computed block by block on `threads` threads.
// g points to an oracle_graph (sdbg_oracle.cpp); release with
// oracle_free_graph.
int oracle_part_build(const uint64_t* keys, const uint32_t* counts, uint64_t n, uint32_t k, int threads, void* g) {
  if (k < 2 || k > 127) return -1;
  if (threads < 1) threads = 1;
  switch (words_of((int)k)) {
    case 1: return build_w<1>(keys, counts, n, (int)k, threads, g);
    case 2: return build_w<2>(keys, counts, n, (int)k, threads, g);
    case 3: return build_w<3>(keys, counts, n, (int)k, threads, g);
    default: return build_w<4>(keys, counts, n, (int)k, threads, g);
  }
}

}  // extern "C"

namespace {

// Layout of oracle_graph in sdbg_oracle.cpp.
struct GraphOut {
  uint64_t m, t;
  uint8_t* W;
  uint64_t* last;
  uint64_t* valid;
  uint64_t* tip;
  uint32_t* mult;
  uint64_t F[6];
  uint64_t* tip_seq;
  uint64_t tip_words;
};

template <int W>
int build_w(const uint64_t* keys, const uint32_t* counts, uint64_t n, int k, int threads, void* gout) {
  GraphOut* g = static_cast<GraphOut*>(gout);
  std::memset(g, 0, sizeof(*g));
  const int nb = 1 << (2 * block_digits(k));
  std::vector<Big<W>> E(n);
  for (uint64_t i = 0; i < n; ++i)
    for (int j = 0; j < W; ++j) E[i].v[W - 1 - j] = keys[i * W + j];

  // Vertices.  A vertex v = v[0..k-1] is kept as the number with digits
  // v[k-1], ..., v[0] (its colex key).  Source of edge e: key / 4; target
  // e[1..k]: digits e[k], e[k-1], ..., e[1] = label * 4^(k-1) + key / 16.
  std::vector<Big<W>> P, Q;
  P.reserve(n);
  Q.reserve(n);
  for (uint64_t i = 0; i < n; ++i) {
    P.push_back(E[i].shr_digits(1));
    Big<W> t;
    t.push(E[i].digit(0));
    const Big<W> rest = E[i].shr_digits(2);
    for (int j = k - 2; j >= 0; --j) t.push(rest.digit(j));
    Q.push_back(t);
  }
  std::sort(P.begin(), P.end());
  P.erase(std::unique(P.begin(), P.end()), P.end());
  std::sort(Q.begin(), Q.end());
  Q.erase(std::unique(Q.begin(), Q.end()), Q.end());
  std::vector<Big<W>> Zout, Zin;  // Q \ P (no outgoing edge), P \ Q (no incoming edge)
  std::set_difference(Q.begin(), Q.end(), P.begin(), P.end(), std::back_inserter(Zout));
  std::set_difference(P.begin(), P.end(), Q.begin(), Q.end(), std::back_inserter(Zin));
  std::vector<Big<W>>().swap(P);
  std::vector<Big<W>>().swap(Q);

  // Symbols of a vertex, most significant key digit first: v[k-1], ..., v[0].
  auto vdigit = [&](const Big<W>& v, int j) { return v.digit(k - 1 - j); };
  // Block of a row: its source's 4 last symbols (the top of the row order).
  auto row_block_src = [&](const Big<W>& v) {
    int b = 0;
    for (int j = 0; j < block_digits(k); ++j) b = b * 4 + vdigit(v, j);
    return b;
  };
  auto row_block_dummy = [&](const Big<W>& v) {  // source $ v[0..k-2]: symbols v[k-2], v[k-3], ...
    int b = 0;
    for (int j = 0; j < block_digits(k); ++j) b = b * 4 + vdigit(v, j + 1);
    return b;
  };
  // E is in key order, so the edges of a block are a contiguous range
  std::vector<uint64_t> eb(nb + 1, 0);
  for (uint64_t i = 0; i < n; ++i) eb[row_block_src(E[i].shr_digits(1)) + 1] += 1;
  for (int b = 0; b < nb; ++b) eb[b + 1] += eb[b];
  std::vector<std::vector<uint64_t>> rZo(nb), rZi(nb);
  for (uint64_t i = 0; i < Zout.size(); ++i) rZo[row_block_src(Zout[i])].push_back(i);
  for (uint64_t i = 0; i < Zin.size(); ++i) rZi[row_block_dummy(Zin[i])].push_back(i);

  struct Block {
    std::vector<uint8_t> W8, flags;  // flags: 1 last, 2 valid, 4 tip
    std::vector<uint32_t> mult;
    std::vector<uint64_t> tips;  // vertex of each dummy row, in row order
    uint64_t first_sym[5] = {0, 0, 0, 0, 0};  // rows whose source[k-1] has rank c
  };
  std::vector<Block> blocks(nb);
  parallel_for(threads, (uint64_t)nb, [&](uint64_t b, int) {
    Block& B = blocks[b];
    std::vector<Row> rows;
    for (uint64_t i = eb[b]; i < eb[b + 1]; ++i) {
      RowBuilder rb{k};
      const Big<W> v = E[i].shr_digits(1);
      for (int j = 0; j < k; ++j) rb.put(vdigit(v, j) + 1);
      const int label = E[i].digit(0) + 1;
      rb.put(label);
      rows.push_back(Row{rb.c, 0, (uint8_t)label, counts[i], 0});
    }
    for (uint64_t i : rZo[b]) {
      RowBuilder rb{k};
      for (int j = 0; j < k; ++j) rb.put(vdigit(Zout[i], j) + 1);
      rb.put(0);
      rows.push_back(Row{rb.c, 1, 0, 0, 0});
    }
    for (uint64_t i : rZi[b]) {
      RowBuilder rb{k};
      for (int j = 1; j < k; ++j) rb.put(vdigit(Zin[i], j) + 1);  // source[k-1..1] = v[k-2..0]
      rb.put(0);                                                    // source[0] = $
      const int label = vdigit(Zin[i], 0) + 1;                      // v[k-1]
      rb.put(label);
      rows.push_back(Row{rb.c, 2, (uint8_t)label, 0, i});
    }
    std::sort(rows.begin(), rows.end(), [](const Row& a, const Row& c) { return a.code < c.code; });
    const size_t m = rows.size();
    B.W8.resize(m);
    B.flags.resize(m);
    B.mult.resize(m);
    std::set<RowCode> seen;  // (source[1..k-1], label) of the rows so far
    for (size_t i = 0; i < m; ++i) {
      const Row& r = rows[i];
      const RowCode group = without_symbol(r.code, k - 1);  // drop source[0]
      const bool minus = r.label != 0 && seen.count(group) > 0;
      seen.insert(group);
      B.W8[i] = (uint8_t)(r.label | (minus ? 8 : 0));
      // last: the next row has another source (rows of other blocks do)
      const bool last = i + 1 == m || without_symbol(rows[i + 1].code, k) != without_symbol(r.code, k);
      B.flags[i] = (uint8_t)((last ? 1 : 0) | (r.kind == 0 ? 2 : 0) | (r.kind == 2 ? 4 : 0));
      B.mult[i] = r.kind == 0 ? r.mult : 0;
      if (r.kind == 2) B.tips.push_back(r.node);
      // source[k-1]'s rank is the row code's first symbol
      const int pos = 3 * (kRowLimbs * 64 / 3 - 1);
      B.first_sym[(r.code[kRowLimbs - 1 - pos / 64] >> (pos % 64)) & 7] += 1;
    }
  });

  uint64_t m = 0, t = 0;
  for (const Block& B : blocks) m += B.W8.size();
  for (const auto& z : rZi) t += z.size();
  const uint64_t words = (m + 63) / 64;
  g->m = m;
  g->t = t;
  g->W = (uint8_t*)std::calloc(m + 1, 1);
  g->last = (uint64_t*)std::calloc(words + 1, 8);
  g->valid = (uint64_t*)std::calloc(words + 1, 8);
  g->tip = (uint64_t*)std::calloc(words + 1, 8);
  g->mult = (uint32_t*)std::calloc(m + 1, 4);
  g->tip_words = (2 * (uint64_t)k * t + 63) / 64;
  g->tip_seq = (uint64_t*)std::calloc(g->tip_words + 1, 8);
  if (!g->W || !g->last || !g->valid || !g->tip || !g->mult || !g->tip_seq) return -2;
  uint64_t row = 0, tip_rank = 0;
  uint64_t first_sym[5] = {0, 0, 0, 0, 0};
  for (int b = 0; b < nb; ++b) {
    Block& B = blocks[b];
    for (size_t i = 0; i < B.W8.size(); ++i, ++row) {
      g->W[row] = B.W8[i];
      if (B.flags[i] & 1) g->last[row / 64] |= 1ull << (row % 64);
      if (B.flags[i] & 2) g->valid[row / 64] |= 1ull << (row % 64);
      if (B.flags[i] & 4) g->tip[row / 64] |= 1ull << (row % 64);
      g->mult[row] = B.mult[i];
    }
    for (uint64_t node : B.tips) {
      const Big<W>& v = Zin[node];
      for (int j = 0; j < k; ++j) {  // base j of the vertex at bits 2(k r + j)
        const uint64_t bit = 2 * ((uint64_t)k * tip_rank + j);
        g->tip_seq[bit / 64] |= (uint64_t)v.digit(j) << (bit % 64);
      }
      ++tip_rank;
    }
    for (int c = 0; c < 5; ++c) first_sym[c] += B.first_sym[c];
    Block().W8.swap(B.W8);
    Block().flags.swap(B.flags);
    Block().mult.swap(B.mult);
  }
  uint64_t f = 0;
  for (int c = 0; c < 5; ++c) {
    g->F[c] = f;
    f += first_sym[c];
  }
  g->F[5] = m;
  return 0;
}

}  // namespace
