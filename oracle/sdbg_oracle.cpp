// TEST INFRASTRUCTURE ONLY -- never linked into, loaded by, or called from
// the device library.  Only the tests, the smoke check and the benchmark's
// CPU-baseline leg use it.
//
// Plain, slow CPU oracle for succinct de Bruijn graph (SdBG) construction
// from reads (Li et al., MEGAHIT, Section 2 "Methods"):
//   * every (k+1)-mer of every read, on both strands, is counted
//     (Section 2, third paragraph);
//   * (k+1)-mers seen at least d times are "solid" (same paragraph);
//   * mercy-kmers: between two solid (k+1)-mers x, y of one read, where x has
//     no outgoing and y no incoming solid edge and every (k+1)-mer between them
//     is non-solid, the in-between (k+1)-mers are added (same paragraph);
//   * the edges are ordered by the reverse-lexicographic (colex) order of
//     their length-k prefix (Section 2, second paragraph);
//   * the SdBG arrays: per-row label with a "minus" flag, the "last" bit, F,
//     an edge-validity bit per row and a 2kt-bit vector holding the k-mers of
//     the t zero-indegree vertices (Section 2, first paragraph).
//
// Everything is done on strings over "ACGT" (with '$' for the dummy symbol)
// and with std::sort / std::unordered_map, exactly in the order the
// definitions are stated, so it can be checked against the paper by eye.
// Readings taken where the paper is silent are listed in the design notes:
// both strands counted literally (a palindrome counts twice), ties between
// rows of one source broken by label with $ < A < C < G < T, one dummy row
// per zero-indegree vertex, one '$' row per zero-outdegree vertex, validity 1
// on real rows only.

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace {

int base_code(unsigned char c) {
  switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

const char kBase[4] = {'A', 'C', 'G', 'T'};

char complement(char c) {
  switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    default: return 'A';
  }
}

std::string revcomp(const std::string& s) {
  std::string r(s.rbegin(), s.rend());
  for (char& c : r) c = complement(c);
  return r;
}

// Reads split at every byte that is not A/C/G/T (either case); the pieces are
// upper-cased.  A piece shorter than k+1 holds no (k+1)-mer.
std::vector<std::string> segments(const uint8_t* seq, const uint64_t* offsets, uint64_t n_reads) {
  std::vector<std::string> out;
  for (uint64_t r = 0; r < n_reads; ++r) {
    std::string cur;
    for (uint64_t p = offsets[r]; p < offsets[r + 1]; ++p) {
      int c = base_code(seq[p]);
      if (c < 0) {
        if (!cur.empty()) out.push_back(cur);
        cur.clear();
      } else {
        cur.push_back(kBase[c]);
      }
    }
    if (!cur.empty()) out.push_back(cur);
  }
  return out;
}

int key_words(int k) { return (2 * (k + 1) + 63) / 64; }

// Sort key of edge e = e[0..k]: the digits e[k-1], e[k-2], ..., e[0], e[k]
// (most significant first) in base 4, i.e. colex order of the k-prefix and
// then the label.  Written right-aligned into w words, word 0 most
// significant.
void edge_key(const std::string& e, int k, uint64_t* out) {
  uint64_t limb[4] = {0, 0, 0, 0};  // little-endian 256-bit accumulator
  auto push_digit = [&](int dgt) {
    for (int i = 3; i > 0; --i) limb[i] = (limb[i] << 2) | (limb[i - 1] >> 62);
    limb[0] = (limb[0] << 2) | (uint64_t)dgt;
  };
  for (int j = k - 1; j >= 0; --j) push_digit(base_code(e[j]));
  push_digit(base_code(e[k]));
  int w = key_words(k);
  for (int i = 0; i < w; ++i) out[i] = limb[w - 1 - i];
}

std::string key_to_edge(const uint64_t* words, int k) {
  int w = key_words(k);
  uint64_t limb[4] = {0, 0, 0, 0};
  for (int i = 0; i < w; ++i) limb[w - 1 - i] = words[i];
  auto digit = [&](int pos) {  // base-4 digit at position pos (0 = least significant)
    return (int)((limb[(2 * pos) / 64] >> ((2 * pos) % 64)) & 3);
  };
  std::string e(k + 1, 'A');
  e[k] = kBase[digit(0)];
  for (int j = 0; j < k; ++j) e[j] = kBase[digit(j + 1)];
  return e;
}

struct KeyLess {
  int w;
  bool operator()(const std::vector<uint64_t>& a, const std::vector<uint64_t>& b) const {
    for (int i = 0; i < w; ++i)
      if (a[i] != b[i]) return a[i] < b[i];
    return false;
  }
};

int sym_rank(char c) {
  switch (c) {
    case '$': return 0;
    case 'A': return 1;
    case 'C': return 2;
    case 'G': return 3;
    case 'T': return 4;
    default: return 5;
  }
}

struct Row {
  std::string src;  // length k, may start with '$' (dummy row)
  char label;       // '$' or a base
  int kind;         // 0 real, 1 '$' row, 2 dummy row
  uint32_t mult;
  std::string tip;  // the zero-indegree k-mer of a dummy row
};

// Row order: source read from its last symbol to its first, then the label,
// with $ < A < C < G < T.
bool row_less(const Row& a, const Row& b) {
  int k = (int)a.src.size();
  for (int i = k - 1; i >= 0; --i) {
    int ra = sym_rank(a.src[i]), rb = sym_rank(b.src[i]);
    if (ra != rb) return ra < rb;
  }
  return sym_rank(a.label) < sym_rank(b.label);
}

}  // namespace

extern "C" {

typedef struct oracle_graph {
  uint64_t m, t;
  uint8_t* W;         // m bytes: label code ($=0, A..T=1..4) | 8 * minus
  uint64_t* last;     // ceil(m/64) words, bit i = row i
  uint64_t* valid;
  uint64_t* tip;
  uint32_t* mult;     // m
  uint64_t F[6];
  uint64_t* tip_seq;  // ceil(2kt/64) words
  uint64_t tip_words;
} oracle_graph;

void oracle_free(void* p) { std::free(p); }

// A (k+1)-mer count as reported (32 bits): 0 and *out = c if it fits, else
// -3 (the input has a (k+1)-mer seen 2^32 times or more; not clamped).
int oracle_narrow_count(uint64_t c, uint32_t* out) {
  if (c > 0xffffffffull) return -3;
  *out = (uint32_t)c;
  return 0;
}

// Counts of every (k+1)-mer over both strands, solid filter (count >= d) and,
// if mercy != 0, mercy-kmers.  Outputs the edge set E sorted by key with each
// edge's count; n_mercy = number of edges added by the mercy rule; n_occ =
// number of (k+1)-mer occurrences counted (both strands).  Returns -3 if an
// output edge's count does not fit 32 bits.
int oracle_count_solid(const uint8_t* seq, const uint64_t* offsets, uint64_t n_reads, uint32_t k, uint32_t d,
                       uint32_t mercy, uint64_t** keys_out, uint32_t** counts_out, uint64_t* n_out,
                       uint64_t* n_mercy_out, uint64_t* n_occ_out) {
  if (k < 2 || k > 127 || d < 1) return -1;
  const int K = (int)k;
  std::vector<std::string> segs = segments(seq, offsets, n_reads);

  // Count every (k+1)-mer and its reverse complement.
  std::unordered_map<std::string, uint64_t> count;
  uint64_t n_occ = 0;
  for (const std::string& s : segs) {
    if ((int)s.size() < K + 1) continue;
    for (size_t i = 0; i + K + 1 <= s.size(); ++i) {
      std::string x = s.substr(i, K + 1);
      count[x] += 1;
      count[revcomp(x)] += 1;
      n_occ += 2;
    }
  }

  // Solid (k+1)-mers.
  std::unordered_set<std::string> solid;
  for (const auto& kv : count)
    if (kv.second >= d) solid.insert(kv.first);

  // Mercy-kmers, with degrees taken on the solid set.
  std::unordered_set<std::string> mercy_set;
  if (mercy) {
    std::unordered_set<std::string> solid_src, solid_dst;  // k-long prefixes / suffixes of solid edges
    for (const std::string& x : solid) {
      solid_src.insert(x.substr(0, K));
      solid_dst.insert(x.substr(1, K));
    }
    for (const std::string& s : segs) {
      if ((int)s.size() < K + 1) continue;
      size_t nw = s.size() - K;
      std::vector<size_t> pos;  // positions of solid windows, ascending
      for (size_t i = 0; i < nw; ++i)
        if (solid.count(s.substr(i, K + 1))) pos.push_back(i);
      for (size_t a = 0; a + 1 < pos.size(); ++a) {
        size_t p = pos[a], q = pos[a + 1];
        if (q - p < 2) continue;
        std::string x = s.substr(p, K + 1), y = s.substr(q, K + 1);
        bool x_has_out = solid_src.count(x.substr(1, K)) > 0;
        bool y_has_in = solid_dst.count(y.substr(0, K)) > 0;
        if (x_has_out || y_has_in) continue;
        for (size_t i = p + 1; i < q; ++i) {
          std::string z = s.substr(i, K + 1);
          mercy_set.insert(z);
          mercy_set.insert(revcomp(z));
        }
      }
    }
  }

  // E = solid + mercy, sorted by key.  Counts are reported in 32 bits; a
  // count that does not fit is an error, never clamped.
  const int w = key_words(K);
  std::vector<std::pair<std::vector<uint64_t>, uint32_t>> edges;
  bool too_many = false;
  auto add = [&](const std::string& x) {
    std::vector<uint64_t> key(w);
    edge_key(x, K, key.data());
    uint32_t c32 = 0;
    if (oracle_narrow_count(count[x], &c32) != 0) too_many = true;
    edges.push_back({key, c32});
  };
  for (const std::string& x : solid) add(x);
  for (const std::string& x : mercy_set) add(x);
  if (too_many) return -3;
  KeyLess less{w};
  std::sort(edges.begin(), edges.end(), [&](const auto& a, const auto& b) { return less(a.first, b.first); });

  uint64_t n = edges.size();
  uint64_t* keys = (uint64_t*)std::malloc(sizeof(uint64_t) * (n * w + 1));
  uint32_t* counts = (uint32_t*)std::malloc(sizeof(uint32_t) * (n + 1));
  if (!keys || !counts) return -2;
  for (uint64_t i = 0; i < n; ++i) {
    for (int j = 0; j < w; ++j) keys[i * w + j] = edges[i].first[j];
    counts[i] = edges[i].second;
  }
  *keys_out = keys;
  *counts_out = counts;
  *n_out = n;
  *n_mercy_out = mercy_set.size();
  *n_occ_out = n_occ;
  return 0;
}

// SdBG arrays of an edge set given as sorted keys with counts.
int oracle_build(const uint64_t* keys, const uint32_t* counts, uint64_t n, uint32_t k, oracle_graph* g) {
  if (k < 2 || k > 127) return -1;
  const int K = (int)k;
  const int w = key_words(K);

  std::vector<std::string> E(n);
  for (uint64_t i = 0; i < n; ++i) E[i] = key_to_edge(keys + i * w, K);

  // Vertices: sources (k-prefixes) and targets (k-suffixes) of edges.
  std::set<std::string> P, Q;
  for (const std::string& e : E) {
    P.insert(e.substr(0, K));
    Q.insert(e.substr(1, K));
  }

  std::vector<Row> rows;
  for (uint64_t i = 0; i < n; ++i) rows.push_back(Row{E[i].substr(0, K), E[i][K], 0, counts[i], ""});
  for (const std::string& v : Q)  // zero outdegree: one '$' row
    if (!P.count(v)) rows.push_back(Row{v, '$', 1, 0, ""});
  for (const std::string& v : P)  // zero indegree: one dummy row entering v
    if (!Q.count(v)) rows.push_back(Row{"$" + v.substr(0, K - 1), v[K - 1], 2, 0, v});
  std::sort(rows.begin(), rows.end(), row_less);

  const uint64_t m = rows.size();
  const uint64_t words = (m + 63) / 64;
  g->m = m;
  g->W = (uint8_t*)std::calloc(m + 1, 1);
  g->last = (uint64_t*)std::calloc(words + 1, 8);
  g->valid = (uint64_t*)std::calloc(words + 1, 8);
  g->tip = (uint64_t*)std::calloc(words + 1, 8);
  g->mult = (uint32_t*)std::calloc(m + 1, 4);
  if (!g->W || !g->last || !g->valid || !g->tip || !g->mult) return -2;

  std::set<std::string> seen;  // (source[1..k-1], label) of rows so far
  uint64_t t = 0;
  for (uint64_t i = 0; i < m; ++i) {
    const Row& r = rows[i];
    std::string group = r.src.substr(1) + r.label;
    bool minus = r.label != '$' && seen.count(group) > 0;
    seen.insert(group);
    g->W[i] = (uint8_t)(sym_rank(r.label) | (minus ? 8 : 0));
    bool last = (i + 1 == m) || rows[i + 1].src != r.src;
    if (last) g->last[i / 64] |= 1ull << (i % 64);
    if (r.kind == 0) g->valid[i / 64] |= 1ull << (i % 64);
    if (r.kind == 2) {
      g->tip[i / 64] |= 1ull << (i % 64);
      ++t;
    }
    g->mult[i] = r.kind == 0 ? r.mult : 0;
  }
  for (int c = 0; c < 5; ++c) {
    uint64_t f = 0;
    for (const Row& r : rows)
      if (sym_rank(r.src[K - 1]) < c) ++f;
    g->F[c] = f;
  }
  g->F[5] = m;

  g->t = t;
  g->tip_words = (2 * (uint64_t)K * t + 63) / 64;
  g->tip_seq = (uint64_t*)std::calloc(g->tip_words + 1, 8);
  if (!g->tip_seq) return -2;
  uint64_t r_idx = 0;
  for (const Row& r : rows) {
    if (r.kind != 2) continue;
    for (int j = 0; j < K; ++j) {
      uint64_t bit = 2 * ((uint64_t)K * r_idx + j);
      g->tip_seq[bit / 64] |= (uint64_t)base_code(r.tip[j]) << (bit % 64);
    }
    ++r_idx;
  }
  return 0;
}

void oracle_free_graph(oracle_graph* g) {
  std::free(g->W);
  std::free(g->last);
  std::free(g->valid);
  std::free(g->tip);
  std::free(g->mult);
  std::free(g->tip_seq);
  std::memset(g, 0, sizeof(*g));
}

// Number of occurrences, over both strands of every read, of each query edge
// (given by key).  Used to check sampled outputs of large runs; one pass
// over the reads with a hash lookup per (k+1)-mer, split across threads.
int oracle_count_keys(const uint8_t* seq, const uint64_t* offsets, uint64_t n_reads, uint32_t k,
                      const uint64_t* qkeys, uint64_t nq, uint64_t* counts, int threads) {
  if (k < 2 || k > 127) return -1;
  const int K = (int)k;
  const int w = key_words(K);
  std::unordered_map<std::string, uint64_t> index;  // edge string -> query index
  for (uint64_t i = 0; i < nq; ++i) index[key_to_edge(qkeys + i * w, K)] = i;
  if (threads < 1) threads = 1;
  std::vector<std::vector<uint64_t>> part(threads, std::vector<uint64_t>(nq, 0));
  auto work = [&](int tid) {
    std::string x(K + 1, 'A');
    for (uint64_t r = tid; r < n_reads; r += threads) {
      uint64_t a = offsets[r], b = offsets[r + 1];
      uint64_t run = 0;  // ACGT bases ending at p
      for (uint64_t p = a; p < b; ++p) {
        run = base_code(seq[p]) < 0 ? 0 : run + 1;
        if (run < (uint64_t)K + 1) continue;
        for (int j = 0; j <= K; ++j) x[j] = kBase[base_code(seq[p - K + j])];
        auto it = index.find(x);
        if (it != index.end()) part[tid][it->second] += 1;
        it = index.find(revcomp(x));
        if (it != index.end()) part[tid][it->second] += 1;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) pool.emplace_back(work, t);
  for (auto& th : pool) th.join();
  for (uint64_t i = 0; i < nq; ++i) {
    uint64_t s = 0;
    for (int t = 0; t < threads; ++t) s += part[t][i];
    counts[i] = s;
  }
  return 0;
}

}  // extern "C"
