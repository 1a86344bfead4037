// Counting path (Section 2, third paragraph): reads -> 2-bit packing ->
// both-strand (k+1)-mer keys -> MSD radix partition in HBM -> per-leaf LDS
// sort + run-length count + solid filter -> mercy-kmers -> sorted edge set.
// Keys of up to three words are counted as canonical keys (one per window,
// see window_emit) and the counted set is expanded to both strands before
// the mercy step (expand_rc).
//
// Keys are the colex edge keys (Section 2, second paragraph): digits
// e[k-1], ..., e[0], e[k] of the (k+1)-mer e.  The partition cuts the key
// space by its most significant bits; the first cut is taken straight from
// the packed reads (keys are computed twice, once to histogram and once to
// scatter, instead of being written and re-read), the later cuts are
// segmented passes over the key buffers, and leaves small enough for LDS
// are sorted and counted there.  Consecutive blocks of the top-bit prefix
// space are grouped so that a group's key buffers fit the memory budget
// (the block-wise strategy of Section 2, second paragraph).

#include <algorithm>
#include <cmath>
#include <cstring>

#include "engine.h"
#include "kernels.h"
#include "prims.h"
#include "windows.h"
#include "wslots.h"

#include <cstdio>
#include <cstdlib>

namespace sdbg {

// ------------------------------------------------------------ packing
// Thread t packs bases [64t, 64t+64): two words of 2-bit codes (base j at
// bits 2(j mod 32) of word j/32) and one word of "not ACGT" flags.
__global__ __launch_bounds__(SDBG_BLOCK) void k_pack(const uint8_t* __restrict__ seq, uint64_t nb,
                                                     uint64_t* __restrict__ packed, uint64_t* __restrict__ bad,
                                                     uint32_t* __restrict__ any_bad) {
  uint64_t t = blockIdx.x * (uint64_t)SDBG_BLOCK + threadIdx.x;
  uint64_t base = t * 64;
  if (base >= nb) return;
  uint64_t p0 = 0, p1 = 0, bw = 0;
  if (base + 64 <= nb && ((reinterpret_cast<uintptr_t>(seq + base)) & 15) == 0) {
    const uint4* v = reinterpret_cast<const uint4*>(seq + base);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint4 x = v[q];
      uint32_t wd[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = q * 16 + e * 4 + b;
          bool ok;
          uint64_t code = base_code((wd[e] >> (8 * b)) & 0xFFu, &ok);
          if (i < 32)
            p0 |= code << (2 * i);
          else
            p1 |= code << (2 * (i - 32));
          bw |= (uint64_t)(!ok) << i;
        }
      }
    }
  } else {
    for (int i = 0; i < 64 && base + i < nb; ++i) {
      bool ok;
      uint64_t code = base_code(seq[base + i], &ok);
      if (i < 32)
        p0 |= code << (2 * i);
      else
        p1 |= code << (2 * (i - 32));
      bw |= (uint64_t)(!ok) << i;
    }
  }
  packed[2 * t] = p0;
  packed[2 * t + 1] = p1;
  bad[t] = bw;
  if (bw) atomicOr(any_bad, 1u);
}

// Windows (k+1-mer start positions) per read: max(0, len - k).
__global__ void k_nwin(const uint64_t* __restrict__ offsets, uint64_t n_reads, int k, uint64_t* __restrict__ nwin) {
  uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  uint64_t a = offsets[r], b = offsets[r + 1];
  uint64_t len = b > a ? b - a : 0;
  nwin[r] = len > (uint64_t)k ? len - k : 0;
}

// ------------------------------------------------------------ extraction
// Windows and histogram-table column of one extraction tile.
struct TileGeo {
  uint64_t g0, gend;    // first window of the tile, end of its set's windows
  uint64_t col, stride; // table entry of digit d: col + d * stride
};

template <int IPT>
DEV TileGeo tile_geo(const ExArgs& a, uint64_t t, uint64_t ntiles) {
  constexpr uint64_t WPT = (uint64_t)SDBG_BLOCK * IPT;
  TileGeo g;
  if (!a.tset) {
    g.g0 = t * WPT;
    g.gend = a.NW;
    g.col = t;
    g.stride = ntiles;
  } else {
    const uint32_t s = a.tset[t];
    const uint64_t t0 = a.st[s];
    g.g0 = a.sw[s] + (t - t0) * WPT;
    g.gend = a.sw[s + 1];
    g.col = (t0 << a.dbits) + (t - t0);
    g.stride = a.st[s + 1] - t0;
  }
  return g;
}

// tr[t] = read containing window t * TR_GRAIN; one thread per read.
__global__ void k_tile_reads(const uint64_t* __restrict__ woff, uint64_t n_reads, uint64_t* __restrict__ tr) {
  uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  const uint64_t a = woff[r], b = woff[r + 1];
  for (uint64_t t = (a + TR_GRAIN - 1) / TR_GRAIN; t * TR_GRAIN < b; ++t) tr[t] = r;
}

// Keys of window at stream position j: forward strand and reverse complement.
template <int W>
DEV void window_keys(const ExArgs& a, uint64_t j, Key<W>* kf, Key<W>* kr) {
  Key<W> F = stream_bits<W>(a.packed, 2 * j, a.kb);
  *kf = key_from_fwd<W>(F, a.kb);
  *kr = key_from_fwd<W>(revcomp_fwd<W>(F, a.kb), a.kb);
}

// Keys a window emits into the count: both strands' keys, or (canon) its
// canonical key, once, or twice when the window is its own reverse
// complement -- so every canonical key's count is the count of either of
// its strands' keys over both strands.  Returns how many (1 or 2).
template <int W>
DEV int window_emit(const ExArgs& a, Roller<W>& rl, uint64_t j, Key<W>* k0, Key<W>* k1) {
  rl.at(a.packed, a.k, a.kb, j);
  const Key<W> kf = rl.fwd_key(a.kb), kr = rl.rc_key(a.kb);
  if (!a.canon) {
    *k0 = kf;
    *k1 = kr;
    return 2;
  }
  *k0 = key_less<W>(kr, kf) ? kr : kf;
  *k1 = *k0;
  return key_eq<W>(kf, kr) ? 2 : 1;
}

template <int W>
DEV bool ex_pass(const ExArgs& a, const Key<W>& key) {
  uint32_t p = key_bits<W>(key, a.kb - a.pb, a.pb);
  return p >= a.glo && p < a.ghi;
}

// Histogram of the partition digit per tile of 256*IPT windows, written
// digit-major: tab[d * ntiles + tile].  If occ is given, occ[tile] = the
// tile's occurrences, two per clean window.
template <int W, int IPT>
__global__ __launch_bounds__(SDBG_BLOCK) void k_ex_hist(ExArgs a, uint32_t* __restrict__ tab, uint64_t ntiles,
                                                        uint64_t* __restrict__ occ) {
  __shared__ uint32_t h[256];
  __shared__ uint32_t wsum[SDBG_WAVES];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint32_t produced = 0;
  const TileGeo tg = tile_geo<IPT>(a, blockIdx.x, ntiles);
  const uint64_t g0 = tg.g0 + (uint64_t)threadIdx.x * IPT;
  if (g0 < tg.gend) {
    WinIter it;
    it.init(a, g0);
    Roller<W> rl;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      if (g0 + q < tg.gend) {
        uint64_t j = it.pos();
        if (!a.any_bad || window_clean(a.bad, j, a.k + 1)) {
          Key<W> k0, k1;
          const int ne = window_emit<W>(a, rl, j, &k0, &k1);
          produced += 2;
          if (ex_pass<W>(a, k0)) atomicAdd(&h[key_bits<W>(k0, a.dlo, a.dbits)], 1u);
          if (ne == 2 && ex_pass<W>(a, k1)) atomicAdd(&h[key_bits<W>(k1, a.dlo, a.dbits)], 1u);
        }
        it.next(a);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < (1u << a.dbits)) tab[tg.col + (uint64_t)threadIdx.x * tg.stride] = h[threadIdx.x];
  if (occ) {
    const uint32_t s = wave_sum(produced);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t t = 0;
#pragma unroll
      for (int i = 0; i < SDBG_WAVES; ++i) t += wsum[i];
      occ[blockIdx.x] = t;
    }
  }
}

// Scatter: recompute the tile's keys, counting-sort them by digit in LDS and
// write each digit's run to its place (tab holds the exclusive scan of the
// digit-major histogram, i.e. each (digit, tile) run's first position).
template <int W, int IPT>
__global__ __launch_bounds__(SDBG_BLOCK) void k_ex_scatter(ExArgs a, const uint32_t* __restrict__ tab, uint64_t ntiles,
                                                           uint64_t* __restrict__ out) {
  constexpr int NK = 2 * IPT;
  __shared__ uint64_t lk[NK * SDBG_BLOCK * W];
  __shared__ uint32_t cnt[256], lst[256], gb[256];
  __shared__ uint32_t sc[SDBG_WAVES + 1];
  const uint32_t nbins = 1u << a.dbits;
  const TileGeo tg = tile_geo<IPT>(a, blockIdx.x, ntiles);
  cnt[threadIdx.x] = 0;
  gb[threadIdx.x] = threadIdx.x < nbins ? tab[tg.col + (uint64_t)threadIdx.x * tg.stride] : 0;
  __syncthreads();
  Key<W> keys[NK];
  uint32_t pos[NK];
#pragma unroll
  for (int q = 0; q < NK; ++q) pos[q] = 0xFFFFFFFFu;
  const uint64_t g0 = tg.g0 + (uint64_t)threadIdx.x * IPT;
  if (g0 < tg.gend) {
    WinIter it;
    it.init(a, g0);
    Roller<W> rl;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      if (g0 + q < tg.gend) {
        uint64_t j = it.pos();
        if (!a.any_bad || window_clean(a.bad, j, a.k + 1)) {
          const int ne = window_emit<W>(a, rl, j, &keys[2 * q], &keys[2 * q + 1]);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if (h < ne && ex_pass<W>(a, keys[2 * q + h])) {
              uint32_t d = key_bits<W>(keys[2 * q + h], a.dlo, a.dbits);
              uint32_t s = atomicAdd(&cnt[d], 1u);
              pos[2 * q + h] = (d << 16) | s;
            }
          }
        }
        it.next(a);
      }
    }
  }
  __syncthreads();
  uint32_t total;
  uint32_t ex = block_excl_scan<uint32_t>(cnt[threadIdx.x], sc, &total);
  lst[threadIdx.x] = ex;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    if (pos[q] != 0xFFFFFFFFu) {
      uint32_t p = lst[pos[q] >> 16] + (pos[q] & 0xFFFFu);
      key_store<W>(&lk[p * W], keys[q]);
    }
  }
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < total; p += SDBG_BLOCK) {
    Key<W> key = key_load<W>(&lk[p * W]);
    uint32_t d = key_bits<W>(key, a.dlo, a.dbits);
    uint64_t dst = (uint64_t)gb[d] + (p - lst[d]);
    key_store<W>(out + dst * W, key);
  }
}

// 16-bit-prefix histogram with global atomics; only used to plan groups
// when the memory budget forces splitting a first-digit block.
template <int W, int IPT>
__global__ __launch_bounds__(SDBG_BLOCK) void k_ex_hist_prefix(ExArgs a, unsigned long long* __restrict__ h) {
  const uint64_t g0 = ((uint64_t)blockIdx.x * SDBG_BLOCK + threadIdx.x) * IPT;
  if (g0 >= a.NW) return;
  WinIter it;
  it.init(a, g0);
  Roller<W> rl;
  for (int q = 0; q < IPT && g0 + q < a.NW; ++q) {
    uint64_t j = it.pos();
    if (!a.any_bad || window_clean(a.bad, j, a.k + 1)) {
      Key<W> k0, k1;
      const int ne = window_emit<W>(a, rl, j, &k0, &k1);
      atomicAdd(&h[key_bits<W>(k0, a.kb - a.pb, a.pb)], 1ull);
      if (ne == 2) atomicAdd(&h[key_bits<W>(k1, a.kb - a.pb, a.pb)], 1ull);
    }
    it.next(a);
  }
}

// ------------------------------------------------------------ segments
// An ordered list of key ranges ("segments"); all keys of a segment share
// their bits above `bit`.  Segment s lives at [off, off+len) of buffer buf.
struct SegView {
  uint64_t* off;
  uint64_t* len;
  uint16_t* bit;  // key bits below the segment's common prefix
  uint8_t* buf;
  uint8_t* D;  // digit width of this level's cut (0 = not cut)
  uint64_t n;
};

// st[0] = oversized segments that still have key bits to cut, st[1] = their
// keys, st[2] = how many of them came whole out of their parent's cut (D
// flag set by k_seg_newwrite).
__global__ void k_seg_stats(SegView v, uint64_t cap, unsigned long long* st) {
  uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  unsigned long long n = 0, sum = 0, whole = 0;
  if (s < v.n && v.len[s] > cap && v.bit[s] > 0) {
    n = 1;
    sum = v.len[s];
    whole = v.D[s] != 0;
  }
  n = wave_sum(n);
  sum = wave_sum(sum);
  whole = wave_sum(whole);
  if ((threadIdx.x & 63) == 0 && n) {
    atomicAdd(&st[0], n);
    atomicAdd(&st[1], sum);
    if (whole) atomicAdd(&st[2], whole);
  }
}

// An oversized segment that a cut left whole (all its keys fell into one
// digit) may hold many copies of a few keys, for which cutting a few bits
// per level would take as many levels as the key has bits.  Its keys share
// every bit above the highest bit in which some key differs from the first
// one, so `bit` drops to that bit + 1; all keys equal -> 0 (the leaf then
// counts the run).  Workgroups stride over the segments.
template <int W>
__global__ __launch_bounds__(SDBG_BLOCK) void k_seg_squeeze(SegView v, uint64_t* const* __restrict__ bufs,
                                                            uint64_t cap) {
  __shared__ uint64_t red[SDBG_WAVES][W];
  for (uint64_t s = blockIdx.x; s < v.n; s += gridDim.x) {
    if (!v.D[s] || v.len[s] <= cap || v.bit[s] == 0) continue;  // uniform over the workgroup
    const uint64_t* src = bufs[v.buf[s]] + v.off[s] * W;
    const uint64_t len = v.len[s];
    const Key<W> k0 = key_load_g<W>(src);
    uint64_t x[W];
#pragma unroll
    for (int j = 0; j < W; ++j) x[j] = 0;
    for (uint64_t i = threadIdx.x; i < len; i += SDBG_BLOCK) {
      const Key<W> ki = key_load_g<W>(src + i * W);
#pragma unroll
      for (int j = 0; j < W; ++j) x[j] |= ki.w[j] ^ k0.w[j];
    }
#pragma unroll
    for (int j = 0; j < W; ++j)
      for (int o = 32; o > 0; o >>= 1) x[j] |= __shfl_xor(x[j], o, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int j = 0; j < W; ++j) red[threadIdx.x >> 6][j] = x[j];
    __syncthreads();
    if (threadIdx.x == 0) {
      int nb = 0;  // highest differing bit + 1 (word 0 is the most significant)
      for (int j = 0; j < W && !nb; ++j) {
        uint64_t o = 0;
        for (int q = 0; q < SDBG_WAVES; ++q) o |= red[q][j];
        if (o) nb = 64 * (W - 1 - j) + 64 - __clzll(o);
      }
      if (nb < (int)v.bit[s]) v.bit[s] = (uint16_t)nb;
      v.D[s] = 0;
    }
    __syncthreads();
  }
}

__global__ void k_seg_mark(SegView v, uint64_t cap, int D, int tk, uint64_t* __restrict__ ntiles,
                           uint64_t* __restrict__ tabsz) {
  uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (s >= v.n) return;
  int d = 0;
  if (v.len[s] > cap && v.bit[s] > 0) d = min(D, (int)v.bit[s]);
  v.D[s] = (uint8_t)d;
  uint64_t nt = d ? (v.len[s] + tk - 1) / tk : 0;
  ntiles[s] = nt;
  tabsz[s] = nt << d;
}

// Segment of each tile t < NT: the last segment whose first tile is <= t
// (tile_first is the exclusive scan of the tile counts, so a run of equal
// entries ends with the one segment of the run that has tiles).
__global__ void k_seg_tiles(SegView v, const uint64_t* __restrict__ tile_first, uint64_t NT,
                            uint32_t* __restrict__ tile_seg) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t >= NT) return;
  uint64_t lo = 0, hi = v.n;  // first segment whose first tile is > t
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (tile_first[mid] <= t)
      lo = mid + 1;
    else
      hi = mid;
  }
  tile_seg[t] = (uint32_t)(lo - 1);
}

template <int W, int TK>
__global__ __launch_bounds__(SDBG_BLOCK) void k_seg_hist(SegView v, uint64_t* const* __restrict__ bufs,
                                                         const uint32_t* __restrict__ tile_seg,
                                                         const uint64_t* __restrict__ tile_first,
                                                         const uint64_t* __restrict__ tab_base,
                                                         uint32_t* __restrict__ tab) {
  __shared__ uint32_t h[256];
  const uint64_t tile = blockIdx.x;
  const uint32_t s = tile_seg[tile];
  const uint64_t i = tile - tile_first[s];
  const uint64_t len = v.len[s];
  const uint64_t nt = (len + TK - 1) / TK;
  const int D = v.D[s], lo = (int)v.bit[s] - D;
  const uint64_t* src = bufs[v.buf[s]] + (v.off[s] + i * TK) * W;
  const uint32_t n = (uint32_t)min((uint64_t)TK, len - i * TK);
  h[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < n; p += SDBG_BLOCK)
    atomicAdd(&h[key_bits<W>(key_load_g<W>(src + (uint64_t)p * W), lo, D)], 1u);
  __syncthreads();
  if (threadIdx.x < (1u << D)) tab[tab_base[s] + (uint64_t)threadIdx.x * nt + i] = h[threadIdx.x];
}

template <int W, int TK>
__global__ __launch_bounds__(SDBG_BLOCK) void k_seg_scatter(SegView v, uint64_t* const* __restrict__ bufs,
                                                            const uint32_t* __restrict__ tile_seg,
                                                            const uint64_t* __restrict__ tile_first,
                                                            const uint64_t* __restrict__ tab_base,
                                                            const uint32_t* __restrict__ tabscan) {
  static_assert(TK % SDBG_BLOCK == 0, "whole keys per thread");
  constexpr int PER = TK / SDBG_BLOCK;
  __shared__ uint64_t lk[TK * W];
  __shared__ uint32_t cnt[256], lst[256], gb[256];
  __shared__ uint32_t sc[SDBG_WAVES + 1];
  const uint64_t tile = blockIdx.x;
  const uint32_t s = tile_seg[tile];
  const uint64_t i = tile - tile_first[s];
  const uint64_t len = v.len[s];
  const uint64_t nt = (len + TK - 1) / TK;
  const int D = v.D[s], lo = (int)v.bit[s] - D;
  const int b = v.buf[s];
  const uint64_t* src = bufs[b] + (v.off[s] + i * TK) * W;
  uint64_t* dst = bufs[b ^ 1] + v.off[s] * W;
  const uint32_t n = (uint32_t)min((uint64_t)TK, len - i * TK);
  const uint64_t tb = tab_base[s];
  const uint32_t seg0 = tabscan[tb];
  cnt[threadIdx.x] = 0;
  gb[threadIdx.x] = threadIdx.x < (1u << D) ? tabscan[tb + (uint64_t)threadIdx.x * nt + i] - seg0 : 0;
  __syncthreads();
  Key<W> keys[PER];
  uint32_t pos[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    uint32_t p = q * SDBG_BLOCK + threadIdx.x;
    pos[q] = 0xFFFFFFFFu;
    if (p < n) {
      keys[q] = key_load_g<W>(src + (uint64_t)p * W);
      uint32_t d = key_bits<W>(keys[q], lo, D);
      pos[q] = (d << 16) | atomicAdd(&cnt[d], 1u);
    }
  }
  __syncthreads();
  uint32_t total;
  lst[threadIdx.x] = block_excl_scan<uint32_t>(cnt[threadIdx.x], sc, &total);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q)
    if (pos[q] != 0xFFFFFFFFu) key_store<W>(&lk[(lst[pos[q] >> 16] + (pos[q] & 0xFFFFu)) * W], keys[q]);
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < total; p += SDBG_BLOCK) {
    Key<W> key = key_load<W>(&lk[p * W]);
    uint32_t d = key_bits<W>(key, lo, D);
    key_store_g<W>(dst + ((uint64_t)gb[d] + (p - lst[d])) * W, key);
  }
}


// Entries of the next segment list contributed by segment s: itself if not
// cut, else its non-empty children.
__device__ __forceinline__ void child_range(const SegView& v, uint64_t s, int tk, const uint64_t* tab_base,
                                            const uint32_t* tabscan, uint32_t d, uint64_t* start, uint64_t* end) {
  const int D = v.D[s];
  const uint64_t nt = (v.len[s] + tk - 1) / tk;
  const uint64_t tb = tab_base[s];
  const uint32_t s0 = tabscan[tb];
  *start = tabscan[tb + d * nt] - s0;
  *end = (d + 1 < (1u << D)) ? (uint64_t)(tabscan[tb + (uint64_t)(d + 1) * nt] - s0) : v.len[s];
}

// One wave per segment; its lanes take the children of a cut segment in
// turn (2^D <= 256 of them).
__global__ void k_seg_newcount(SegView v, int tk, const uint64_t* __restrict__ tab_base,
                               const uint32_t* __restrict__ tabscan, uint64_t* __restrict__ cnt) {
  const uint64_t s = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint32_t lane = threadIdx.x & 63;
  if (s >= v.n) return;  // whole waves
  const int D = v.D[s];
  if (!D) {
    if (lane == 0) cnt[s] = 1;
    return;
  }
  uint64_t c = 0;
  for (uint32_t d = lane; d < (1u << D); d += 64) {
    uint64_t a, b;
    child_range(v, s, tk, tab_base, tabscan, d, &a, &b);
    c += b > a;
  }
  c = wave_sum(c);
  if (lane == 0) cnt[s] = c;
}

__global__ void k_seg_newwrite(SegView v, int tk, const uint64_t* __restrict__ tab_base,
                               const uint32_t* __restrict__ tabscan, const uint64_t* __restrict__ newpos, SegView nv) {
  const uint64_t s = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint32_t lane = threadIdx.x & 63;
  if (s >= v.n) return;  // whole waves
  uint64_t p = newpos[s];
  const int D = v.D[s];
  if (!D) {
    if (lane == 0) {
      nv.off[p] = v.off[s];
      nv.len[p] = v.len[s];
      nv.bit[p] = v.bit[s];
      nv.buf[p] = v.buf[s];
      nv.D[p] = 0;
    }
    return;
  }
  for (uint32_t d0 = 0; d0 < (1u << D); d0 += 64) {
    const uint32_t d = d0 + lane;
    uint64_t a = 0, b = 0;
    if (d < (1u << D)) child_range(v, s, tk, tab_base, tabscan, d, &a, &b);
    const uint32_t ne = b > a ? 1u : 0u;
    const uint32_t incl = wave_incl_scan<uint32_t>(ne);
    if (ne) {
      const uint64_t q = p + incl - 1;
      nv.off[q] = v.off[s] + a;
      nv.len[q] = b - a;
      nv.bit[q] = (uint16_t)(v.bit[s] - D);
      nv.buf[q] = (uint8_t)(v.buf[s] ^ 1);
      nv.D[q] = (uint8_t)(b - a == v.len[s]);  // the cut left it whole
    }
    p += __shfl(incl, 63, 64);
  }
}

// ------------------------------------------------------------ leaves
// Persistent workgroups walk the leaf segments with a fixed stride (grid
// sized to the resident capacity), and each one loads the next segment's
// descriptor and keys into registers while it sorts the current one, so
// the global-memory latency of a segment overlaps the LDS work of the one
// before.  Per segment: duplicates are merged first with an LDS hash table
// (one slot per distinct key: owner element in the high 16 bits, count in
// the low 16 bits, updated with LDS atomics), so that a key seen hundreds
// of times costs one atomic per copy instead of a serial run for one
// thread.  Only the distinct keys that will be written (count >= dmin, or
// all when want_low) are then counting-sorted by their next B key bits;
// each thread finishes a contiguous range of bins with an insertion sort,
// and the keys with count >= dmin (then, if want_low, those below) are
// written back in place at the segment's start, counts into cnt[] at the
// same positions.  A segment longer than CAP has no key bits left to cut,
// so all its keys are equal.
template <int W>
DEV uint32_t leaf_hash(const Key<W>& k) {
  uint32_t h = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) h ^= (uint32_t)k.w[i] ^ (uint32_t)(k.w[i] >> 32) * 0x85EBCA6Bu;
  return h * 0x9E3779B1u;
}

template <int CAP>
struct LeafShape {
  static constexpr int PER = CAP / SDBG_BLOCK;
  static constexpr int H = 2 * CAP;  // hash slots, load <= 1/2
  static constexpr int MAXB = CAP >= 1024 ? 9 : 8;  // bins <= 512: a few output keys per bin at most
};

template <int W, int CAP>
__global__ __launch_bounds__(SDBG_BLOCK, 4) void k_leaf(SegView v, uint64_t* const* __restrict__ bufs,
                                                     uint32_t* __restrict__ cnt, uint32_t dmin, int want_low,
                                                     int distinct, const uint32_t* __restrict__ ids,
                                                     uint64_t* __restrict__ nsolid, uint64_t* __restrict__ nlow) {
  constexpr int PER = LeafShape<CAP>::PER, H = LeafShape<CAP>::H, MAXB = LeafShape<CAP>::MAXB;
  constexpr uint32_t EMPTY = 0xFFFFFFFFu;
  static_assert(CAP <= 4096 && H <= 65536, "leaf sizes");
  __shared__ uint64_t A[CAP * W];
  __shared__ uint32_t hs[H];
  __shared__ uint16_t idx[CAP];
  __shared__ uint32_t bins[(1 << MAXB) + 1];
  __shared__ uint32_t sc[SDBG_WAVES + 1];
  uint64_t* const buf0 = bufs[0];
  uint64_t* const buf1 = bufs[1];
  const uint64_t G = gridDim.x;

  // next segment, prefetched (the first PF keys of each thread; the largest
  // one-word leaf holds the rest back so that it needs no scratch memory)
  constexpr int PF = (W == 1 && CAP > 1024) ? PER - 2 : PER;
  uint64_t n_len = 0, n_off = 0;
  int n_buf = 0, n_bit = 0;
  Key<W> nk[PER];
  auto fetch = [&](uint64_t t) {
    if (t >= v.n) return;
    n_len = v.len[t];
    n_off = v.off[t];
    n_buf = v.buf[t];
    n_bit = v.bit[t];
    if (n_len <= CAP) {
      const uint64_t* src = (n_buf ? buf1 : buf0) + n_off * W;
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int i = q * SDBG_BLOCK + threadIdx.x;
        if (i < (int)n_len) nk[q] = key_load_g<W>(src + (uint64_t)i * W);
      }
    }
  };
  fetch(blockIdx.x);
  for (uint64_t s = blockIdx.x; s < v.n; s += G) {
    const uint64_t len = n_len;
    uint64_t* keys = (n_buf ? buf1 : buf0) + n_off * W;
    uint32_t* cn = cnt + n_off;
    const int bit = n_bit;
    if (len > CAP) {
      fetch(s + G);
      if (threadIdx.x == 0) {
        // a partition group holds fewer than 2^32 keys (checked on the host
        // before the keys are extracted), so a run's count fits 32 bits
        const uint32_t c = (uint32_t)len;
        const bool solid = len >= dmin;
        if (solid || want_low) cn[0] = c;
        const uint64_t id = ids ? ids[s] : s;
        nsolid[id] = solid;
        nlow[id] = !solid && want_low;
      }
      continue;
    }
    const int n = (int)len;
    // hash slots in use: a power of two >= 2n (load <= 1/2)
    int hb = 6;
    while ((1 << hb) < 2 * n) ++hb;
    const int Hs = 1 << hb;
    const uint32_t hshift = 32 - (uint32_t)hb;
    // keys to LDS, then start loading the next segment
    lds_barrier();  // the previous segment's LDS readers are done
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = q * SDBG_BLOCK + threadIdx.x;
      if (i < n) key_store<W>(&A[i * W], q < PF ? nk[q] : key_load_g<W>(keys + (uint64_t)i * W));
    }
    if (distinct) {
      // keys known to be distinct: each is its own slot, count 1
      for (int i = threadIdx.x; i < n; i += SDBG_BLOCK) hs[i] = ((uint32_t)i << 16) | 1u;
    } else {
      for (int i = threadIdx.x; i < Hs; i += SDBG_BLOCK) hs[i] = EMPTY;
    }
    fetch(s + G);
    lds_barrier();
    // 1. merge duplicates; the element that claims a slot represents its key
    uint32_t rep[PER];  // representative's hash slot (| digit << 16 once binned), else EMPTY
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      rep[q] = EMPTY;
      const int i = q * SDBG_BLOCK + threadIdx.x;
      if (i < n && distinct) {
        rep[q] = (uint32_t)i;
      } else if (i < n) {
        const Key<W> kx = key_load<W>(&A[i * W]);
        uint32_t h = leaf_hash<W>(kx) >> hshift;
        for (;;) {
          uint32_t cur = hs[h];
          if (cur == EMPTY) {
            cur = atomicCAS(&hs[h], EMPTY, ((uint32_t)i << 16) | 1u);
            if (cur == EMPTY) {
              rep[q] = h;
              break;
            }
          }
          if (key_eq<W>(key_load<W>(&A[(cur >> 16) * W]), kx)) {
            atomicAdd(&hs[h], 1u);
            break;
          }
          h = (h + 1) & (uint32_t)(Hs - 1);
        }
      }
    }
    lds_barrier();
    // 2. only keys that will be written are sorted: drop the others, count
    uint32_t nout = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      if (rep[q] != EMPTY && !want_low && (hs[rep[q]] & 0xFFFFu) < dmin) rep[q] = EMPTY;
      nout += rep[q] != EMPTY;
    }
    uint32_t T;
    (void)block_excl_scan<uint32_t>(nout, sc, &T);
    int B = 0;
    while ((1u << B) < T && B < MAXB) ++B;
    B = min(B, bit);
    const int lo = bit - B;
    const int nbins = 1 << B;
    for (int i = threadIdx.x; i <= nbins; i += SDBG_BLOCK) bins[i] = 0;
    lds_barrier();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      if (rep[q] != EMPTY) {
        const uint32_t dg = B ? key_bits<W>(key_load<W>(&A[(hs[rep[q]] >> 16) * W]), lo, B) : 0;
        atomicAdd(&bins[dg], 1u);
        rep[q] |= dg << 16;
      }
    }
    lds_barrier();
    // 3. bin offsets (each thread scans a contiguous run of bins)
    {
      const int per = (nbins + SDBG_BLOCK - 1) / SDBG_BLOCK;
      const int b0 = min(nbins, (int)threadIdx.x * per), b1 = min(nbins, b0 + per);
      uint32_t run = 0;
      for (int b = b0; b < b1; ++b) run += bins[b];
      uint32_t tot;
      uint32_t ex = block_excl_scan<uint32_t>(run, sc, &tot);
      for (int b = b0; b < b1; ++b) {
        uint32_t t = bins[b];
        bins[b] = ex;
        ex += t;
      }
      if (threadIdx.x == 0) bins[nbins] = tot;
    }
    lds_barrier();
    // output keys (as hash slots) grouped by bin, in any order within a bin
    // (each bin is sorted next); bins[d] ends as the end of bin d
#pragma unroll
    for (int q = 0; q < PER; ++q)
      if (rep[q] != EMPTY) idx[atomicAdd(&bins[rep[q] >> 16], 1u)] = (uint16_t)(rep[q] & 0xFFFFu);
    lds_barrier();
    // 4. finish each thread's bins: sort by key, count outputs, write
    const int b0 = (int)(((uint64_t)threadIdx.x * nbins) / SDBG_BLOCK);
    const int b1 = (int)(((uint64_t)(threadIdx.x + 1) * nbins) / SDBG_BLOCK);
    const int r0 = b0 ? (int)bins[b0 - 1] : 0, r1 = b1 ? (int)bins[b1 - 1] : 0;
    for (int i = r0 + 1; i < r1; ++i) {
      const uint16_t x = idx[i];
      const Key<W> kx = key_load<W>(&A[(hs[x] >> 16) * W]);
      int j = i - 1;
      while (j >= r0 && key_less<W>(kx, key_load<W>(&A[(hs[idx[j]] >> 16) * W]))) {
        idx[j + 1] = idx[j];
        --j;
      }
      idx[j + 1] = x;
    }
    uint32_t ns = 0, nl = 0;
    for (int i = r0; i < r1; ++i) {
      const uint32_t c = hs[idx[i]] & 0xFFFFu;
      if (c >= dmin)
        ++ns;
      else if (want_low)
        ++nl;
    }
    // both counts in one scan (each fits 16 bits)
    uint32_t tot2;
    const uint32_t ex2 = block_excl_scan<uint32_t>(ns | (nl << 16), sc, &tot2);
    const uint32_t NS = tot2 & 0xFFFFu, NL = tot2 >> 16;
    uint32_t bs = ex2 & 0xFFFFu, bl = ex2 >> 16;
    for (int i = r0; i < r1; ++i) {
      const uint32_t e = hs[idx[i]];
      const uint32_t c = e & 0xFFFFu;
      const Key<W> kx = key_load<W>(&A[(e >> 16) * W]);
      if (c >= dmin) {
        key_store_g<W>(keys + (uint64_t)bs * W, kx);
        cn[bs] = c;
        ++bs;
      } else if (want_low) {
        key_store_g<W>(keys + (uint64_t)(NS + bl) * W, kx);
        cn[NS + bl] = c;
        ++bl;
      }
    }
    if (threadIdx.x == 0) {
      const uint64_t id = ids ? ids[s] : s;
      nsolid[id] = NS;
      nlow[id] = NL;
    }
  }
}

// Gather the per-leaf outputs into dense arrays in leaf order (= key order).
template <int W>
__global__ __launch_bounds__(SDBG_BLOCK) void k_compact(SegView v, uint64_t* const* __restrict__ bufs,
                                                        const uint32_t* __restrict__ cnt,
                                                        const uint64_t* __restrict__ nsolid,
                                                        const uint64_t* __restrict__ spos,
                                                        const uint64_t* __restrict__ nlow,
                                                        const uint64_t* __restrict__ lpos, uint64_t* __restrict__ skeys,
                                                        uint32_t* __restrict__ scnt, uint64_t* __restrict__ lkeys,
                                                        uint32_t* __restrict__ lcnt) {
  // one wave per segment (a leaf writes a few hundred keys at most)
  const uint64_t s = (uint64_t)blockIdx.x * SDBG_WAVES + (threadIdx.x >> 6);
  if (s >= v.n) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t off = v.off[s];
  const uint64_t* src = bufs[v.buf[s]] + off * W;
  const uint64_t a = nsolid[s], b = nlow ? nlow[s] : 0;
  const uint64_t ps = spos[s];
  for (uint64_t i = lane; i < a; i += 64) {
    key_store<W>(skeys + (ps + i) * W, key_load_g<W>(src + i * W));
    scnt[ps + i] = cnt[off + i];
  }
  if (b) {
    const uint64_t pl = lpos[s];
    for (uint64_t i = lane; i < b; i += 64) {
      key_store<W>(lkeys + (pl + i) * W, key_load_g<W>(src + (a + i) * W));
      lcnt[pl + i] = cnt[off + a + i];
    }
  }
}

// ------------------------------------------------------------ directory
template <int W>
__global__ void k_dir(const uint64_t* __restrict__ keys, uint64_t n, int kbits, int db, uint64_t* __restrict__ dir) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i > n) return;
  uint64_t b = i < n ? key_bits<W>(key_load<W>(keys + i * W), kbits - db, db) : (1ull << db);
  uint64_t from = i == 0 ? 0 : (uint64_t)key_bits<W>(key_load<W>(keys + (i - 1) * W), kbits - db, db) + 1;
  for (uint64_t x = from; x <= b; ++x) dir[x] = i;
}

// Order check of a key array: flags[0] |= 1 if some key is not strictly
// greater than its predecessor, |= 2 if a key has bits above kbits.
template <int W>
__global__ void k_check_sorted(const uint64_t* __restrict__ keys, uint64_t n, int kbits, uint32_t* flags) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  Key<W> x = key_load<W>(keys + i * W);
  if (!key_eq<W>(key_lowbits<W>(x, kbits), x)) atomicOr(flags, 2u);
  if (i > 0 && !key_less<W>(key_load<W>(keys + (i - 1) * W), x)) atomicOr(flags, 1u);
}

// ------------------------------------------------------------ mercy
// Dead-end flags of solid edges: bit1 = no outgoing solid edge, bit2 = no
// incoming solid edge (degrees on the solid set), bit0 = solid.
template <int W>
__global__ void k_dead_ends(SortedView S, int k, uint8_t* __restrict__ fl) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  Key<W> x = key_load<W>(S.keys + i * W);
  bool out = sv_has_source<W>(S, edge_target<W>(x, k));
  bool in = sv_has_target<W>(S, key_shr<W>(x, 2), k);
  fl[i] = (uint8_t)(1 | (!out ? 2 : 0) | (!in ? 4 : 0));
}

// One-word keys (k <= 31) use a table of k-mer NODES instead of edges.  A
// node's entry holds its in-set (bit c: the solid edge c + node exists) and
// its out-set (bit 4 + c: node + c exists), so one lookup answers both
// windows of a read that meet at that node, and the dead-end flags of a
// window are empty sets of its end nodes (no pass over the solid set for
// them).  Node key NK (2k bits) of the k-mer b[0..k-1]: the digits b[k-2],
// ..., b[0], b[k-1], i.e. key_from_fwd of its forward packing.  For an edge
// key x (digits e[k-1], ..., e[0], e[k]):
//   source node e[0..k-1]: NK = (x mod 4^k) with its low digit replaced by
//                          e[k-1] = x div 4^k; contributes out-bit e[k];
//   target node e[1..k]:   NK = ((x div 16) * 4) + e[k]; contributes in-bit
//                          e[0] = (x div 4) mod 4.
// Bucket = NK >> rbits, BW 64-bit words: slot j holds bits [j*sb, (j+1)*sb)
// of the bucket read as one little-endian integer, (NK mod 2^rbits) | sets
// << rbits, sb = rbits + 8; the bucket's top bit marks a bucket with more
// nodes than slots.  The nodes that did not fit
// their bucket go to the spill line of their block of 2^s buckets (4 words,
// slots of NK mod 2^(rbits+s) | sets << (rbits+s), in bucket order); its top
// bit marks a block with more such nodes than the line holds, whose other
// nodes are then looked up in the sorted set.  Stored nodes have a
// non-empty set byte; absent nodes have none.
constexpr int NODE_BLOCK_SHIFT = 6;  // buckets per fill workgroup and spill line: one per thread
constexpr int NODE_FILL_THREADS = 1 << NODE_BLOCK_SHIFT;
constexpr int SPILL_WORDS = 4;
constexpr int NODE_BW = 2;           // bucket words
constexpr int NODE_LOAD = 2;         // slots per solid edge

struct NodeShape {
  int nkb, bw, bb, rbits, sb, slots;
  int s, ssb, sslots;  // block shift; spill slot bits and slots
};

// Smallest table with slots * buckets >= load * nS (at most 2 nS nodes).
inline NodeShape node_shape(int k, uint64_t nS, int shrink, int bw, int load) {
  NodeShape p{};
  p.nkb = 2 * k;
  p.bw = bw;
  const int bmin = std::max(1, p.nkb + NODE_BLOCK_SHIFT + 8 - 63);  // spill slots fit a word
  auto set = [&](int bb) {
    p.bb = bb;
    p.rbits = p.nkb - bb;
    p.sb = p.rbits + 8;
    p.slots = (64 * bw - 1) / p.sb;
    p.s = std::min(NODE_BLOCK_SHIFT, bb);
    p.ssb = p.rbits + p.s + 8;
    p.sslots = (64 * SPILL_WORDS - 1) / p.ssb;
  };
  for (int bb = bmin;; ++bb) {
    set(bb);
    if (bb >= 30 || bb >= p.nkb - 2 || ((uint64_t)p.slots << bb) >= (uint64_t)load * nS) break;
  }
  if (shrink) set(std::max(bmin, p.bb - shrink));
  return p;
}

struct NodeTab {
  const uint64_t* tab;
  const uint64_t* spill;
  SortedView S;  // the solid edge set
  int nkb, bw, rbits, sb, slots, s, ssb, sslots;
};

DEV uint64_t node_of_target(uint64_t x) { return ((x >> 4) << 2) | (x & 3); }
DEV uint64_t node_of_source(uint64_t x, int nkb) {
  return (x & (~0ull >> (64 - nkb)) & ~3ull) | (x >> nkb);
}

// Sets of node nk from the sorted solid set: out-edges are the keys F*4 + c
// (F = forward packing of the node), in-edges the keys (c + 4*F[0..k-2])*4
// + F[k-1], which lie among the keys sharing x div 16.
DEV uint32_t node_sets_sorted(const SortedView& S, uint64_t nk, int nkb) {
  const uint64_t F = (nk >> 2) | ((nk & 3) << (nkb - 2));
  uint32_t f = 0;
  Key<1> q;
  q.w[0] = F << 2;
  for (uint64_t i = sv_lower<1>(S, q); i < S.n; ++i) {
    const uint64_t x = S.keys[i];
    if ((x >> 2) != F) break;
    f |= 16u << (x & 3);
  }
  const uint64_t last = F >> (nkb - 2);
  const uint64_t base = ((F & (~0ull >> (66 - nkb))) << 4) | last;
  q.w[0] = base;
  for (uint64_t i = sv_lower<1>(S, q); i < S.n; ++i) {
    const uint64_t x = S.keys[i];
    if ((x >> 4) != (base >> 4)) break;
    if ((x & 3) == last) f |= 1u << ((x >> 2) & 3);
  }
  return f;
}

// Sets stored for q in a packed line of BW words (slots of sb bits: low
// rbits bits of the node key, then its sets); *ovf = the line's top bit.
template <int BW>
DEV uint32_t line_sets(const uint64_t* line, uint64_t q, int rbits, int sb, int slots, bool* ovf) {
  const uint4* v = reinterpret_cast<const uint4*>(line);
  uint64_t w[BW];
#pragma unroll
  for (int i = 0; i < BW / 2; ++i) {
    const uint4 x = v[i];
    w[2 * i] = x.x | ((uint64_t)x.y << 32);
    w[2 * i + 1] = x.z | ((uint64_t)x.w << 32);
  }
  *ovf = (w[BW - 1] >> 63) != 0;
  const uint64_t rmask = ~0ull >> (64 - rbits);
  const uint64_t smask = ~0ull >> (64 - sb);
  const uint64_t qr = q & rmask;
  uint32_t f = 0;
  for (int j = 0; j < slots; ++j) {
    const uint64_t x = w[0] & smask;
    const uint32_t sets = (uint32_t)(x >> rbits);
    if (sets && (x & rmask) == qr) f = sets;
#pragma unroll
    for (int i = 0; i < BW - 1; ++i) w[i] = (w[i] >> sb) | (w[i + 1] << (64 - sb));
    w[BW - 1] >>= sb;
  }
  return f;
}

template <int BW>
DEV uint32_t node_sets_bw(const NodeTab& t, uint64_t nk) {
  bool ovf;
  uint32_t f = line_sets<BW>(t.tab + (nk >> t.rbits) * BW, nk, t.rbits, t.sb, t.slots, &ovf);
  if (!f && ovf) {
    f = line_sets<SPILL_WORDS>(t.spill + (nk >> (t.rbits + t.s)) * SPILL_WORDS, nk, t.rbits + t.s, t.ssb, t.sslots,
                               &ovf);
    if (!f && ovf) f = node_sets_sorted(t.S, nk, t.nkb);
  }
  return f;
}

DEV uint32_t node_sets(const NodeTab& t, uint64_t nk) {
  return t.bw == 4 ? node_sets_bw<4>(t, nk) : node_sets_bw<2>(t, nk);
}

// First index of S whose key is >= key, for a key whose bits below its top
// p bits are zero: straight from the directory when p <= its bits.
DEV uint64_t sv_prefix_lower(const SortedView& S, uint64_t key, int p) {
  if (p <= S.db) return S.dir[key >> (S.kbits - S.db)];
  Key<1> q;
  q.w[0] = key;
  return sv_lower<1>(S, q);
}

// Sets a packed slot into words w at bit position pos.
template <int BW>
DEV void put_slot(uint64_t* w, uint64_t slot, int pos, int sb) {
  const int wd = pos >> 6, off = pos & 63;
#pragma unroll
  for (int x = 0; x < BW; ++x) {
    if (x == wd) w[x] |= slot << off;
    if (x == wd + 1 && off + sb > 64) w[x] |= slot >> (64 - off);
  }
}

// Table fill: persistent one-wave workgroups, each taking blocks of 2^s
// buckets in turn (one-wave workgroups keep many blocks' dependent loads in
// flight per compute unit; the next block's stretch bounds are loaded while
// the current one is processed).  A block's nodes come from five stretches
// of the sorted solid set: the edges whose target node falls in the block
// (keys sharing their top bb - s bits), and for each top digit c the edges
// whose source node falls in it (keys c, then the block's bb - s bits).
// Each contribution (node key, set bit) claims its node's entry in a list
// of NODE_LIST entries per bucket in LDS (compare-and-swap on the key, then
// OR of the bit); then one thread per bucket packs the first slots nodes of
// its list into the bucket and hands the rest to the block's spill line in
// bucket order.  The order of a bucket's nodes (first come, first placed)
// may differ between runs; lookups compare keys, so their results do not.
// A bucket with more nodes than its list marks itself and the spill line
// overfull.  The
// barriers order LDS only: no thread reads another's global data.
constexpr int NODE_LIST = 6;

DEV uint64_t node_stretch_bound(const SortedView& S, const NodeShape& p, uint64_t B, int r) {
  const uint64_t nblk = 1ull << (p.bb - p.s);
  const int t = r >> 1;
  const uint64_t v = B + (r & 1);
  if (v == nblk && (t == 0 || t == 4)) return S.n;  // past the last key (the bound would not fit the key width)
  if (t == 0)  // v << (rbits + 2 + s) with a shift of 64 only when v = 0 (one block)
    return sv_prefix_lower(S, v ? v << (p.rbits + 2 + p.s) : 0, p.bb - p.s);
  return sv_prefix_lower(S, ((uint64_t)(t - 1) << p.nkb) + (v << (p.rbits + p.s)), p.bb - p.s + 2);
}

template <int BW>
__global__ __launch_bounds__(NODE_FILL_THREADS) void k_node_fill(SortedView S, NodeShape p,
                                                                 uint64_t* __restrict__ tab,
                                                                 uint64_t* __restrict__ spill) {
  constexpr int NT = NODE_FILL_THREADS;
  constexpr uint64_t EMPTY = ~0ull;
  __shared__ unsigned long long lk[NT * NODE_LIST];
  __shared__ uint32_t lf[NT * NODE_LIST];
  __shared__ uint32_t lost[NT];
  __shared__ uint64_t rg[10];
  __shared__ unsigned long long sw[SPILL_WORDS];
  const int s = p.s;
  const uint64_t nblk = 1ull << (p.bb - s);
  const uint32_t nbk = 1u << s;
  const uint32_t lmask = nbk - 1;
  const uint64_t kmask = ~0ull >> (64 - (p.rbits + s));  // node key below the block
  const uint32_t j = threadIdx.x;
  uint64_t nxt = 0;
  if (j < 10 && blockIdx.x < nblk) nxt = node_stretch_bound(S, p, blockIdx.x, j);
  for (uint64_t B = blockIdx.x; B < nblk; B += gridDim.x) {
    if (j < 10) rg[j] = nxt;
#pragma unroll
    for (int r = 0; r < NODE_LIST; ++r) {
      lk[r * NT + j] = EMPTY;
      lf[r * NT + j] = 0;
    }
    lost[j] = 0;
    if (j < SPILL_WORDS) sw[j] = 0;
    lds_barrier();
    uint64_t lo[5], base[6];
    base[0] = 0;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      lo[t] = rg[2 * t];
      base[t + 1] = base[t] + (rg[2 * t + 1] - rg[2 * t]);
    }
    const uint64_t total = base[5];
    if (j < 10 && B + gridDim.x < nblk) nxt = node_stretch_bound(S, p, B + gridDim.x, j);
    // contributions i = 0 .. total-1 over the five stretches; each thread
    // loads four before it inserts them
    for (uint64_t i0 = 0; i0 < total; i0 += 4 * NT) {
      uint64_t x[4];
      uint32_t tt[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t i = i0 + q * NT + j;
        uint64_t src = 0;
        tt[q] = 5;
#pragma unroll
        for (int t = 0; t < 5; ++t)
          if (i >= base[t] && i < base[t + 1]) {
            src = lo[t] + (i - base[t]);
            tt[q] = t;
          }
        x[q] = tt[q] < 5 ? S.keys[src] : 0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (tt[q] == 5) continue;
        const uint64_t nk = tt[q] == 0 ? node_of_target(x[q]) : node_of_source(x[q], p.nkb);
        const uint32_t bit = tt[q] == 0 ? 1u << ((x[q] >> 2) & 3) : 16u << (x[q] & 3);
        const uint32_t b = (uint32_t)(nk >> p.rbits) & lmask;
        const unsigned long long key = (unsigned long long)(nk & kmask);
        bool done = false;
        for (int r = 0; r < NODE_LIST && !done; ++r) {
          const unsigned long long old = atomicCAS(&lk[r * NT + b], (unsigned long long)EMPTY, key);
          if (old == EMPTY || old == key) {
            atomicOr(&lf[r * NT + b], bit);
            done = true;
          }
        }
        if (!done) lost[b] = 1;
      }
    }
    lds_barrier();
    // thread j: bucket j's nodes, entries 0 .. nn-1 (a bucket's list fills
    // from its first entry on)
    uint32_t nn = 0;
    if (j < nbk)
      while (nn < (uint32_t)NODE_LIST && lk[nn * NT + j] != EMPTY) ++nn;
    const bool lst = j < nbk && lost[j] != 0;
    const uint32_t nsp = nn > (uint32_t)p.slots ? nn - (uint32_t)p.slots : 0;
    const uint32_t incl = wave_incl_scan<uint32_t>(nsp);
    const uint32_t total_sp = __shfl(incl, NT - 1, NT);
    const bool any_lost = __any(lst);
    uint32_t spos = incl - nsp;  // this bucket's first spill slot
    const uint64_t rmask = ~0ull >> (64 - p.rbits);
    uint64_t w[BW];
#pragma unroll
    for (int x = 0; x < BW; ++x) w[x] = 0;
    for (uint32_t r = 0; r < nn; ++r) {
      const uint64_t key = lk[r * NT + j];
      const uint64_t f = lf[r * NT + j];
      if (r < (uint32_t)p.slots) {
        put_slot<BW>(w, (key & rmask) | (f << p.rbits), (int)r * p.sb, p.sb);
      } else if (spos < (uint32_t)p.sslots) {
        const uint64_t slot = key | (f << (p.rbits + s));
        const int pos = (int)spos * p.ssb, wd = pos >> 6, off = pos & 63;
        atomicOr(&sw[wd], (unsigned long long)(slot << off));
        if (off + p.ssb > 64) atomicOr(&sw[wd + 1], (unsigned long long)(slot >> (64 - off)));
        ++spos;
      }
    }
    if (nn > (uint32_t)p.slots || lst) w[BW - 1] |= 1ull << 63;
    if (j < nbk) {
      uint64_t* out = tab + (uint64_t)BW * ((B << s) + j);
#pragma unroll
      for (int x = 0; x < BW; ++x) out[x] = w[x];
    }
    lds_barrier();
    if (j < SPILL_WORDS)
      spill[(uint64_t)SPILL_WORDS * B + j] =
          sw[j] | (j == SPILL_WORDS - 1 && (any_lost || total_sp > (uint32_t)p.sslots) ? 1ull << 63 : 0);
    lds_barrier();  // LDS is reused by the next block
  }
}

// Per forward-strand window: 0x80 if it holds a non-ACGT base, else its
// flags from one node: a window at an even index looks up its target node
// (which gives its solidity and its no-out flag; no-in is left unknown,
// 0x08), one at an odd index its source node (solidity and no-in; no-out
// unknown, 0x10).  The windows 2m, 2m+1 of one read share that node, so a
// thread's IPT windows (IPT even) need about IPT/2 lookups.  Non-solid
// windows get 0.
DEV uint8_t node_window_flag(uint64_t x, uint32_t sets, bool odd) {
  if (!odd) {
    if (!((sets >> ((x >> 2) & 3)) & 1)) return 0;
    return (uint8_t)(1 | ((sets >> 4) == 0 ? 2 : 0) | 0x08);
  }
  if (!((sets >> (4 + (x & 3))) & 1)) return 0;
  return (uint8_t)(1 | ((sets & 15) == 0 ? 4 : 0) | 0x10);
}

template <int BW, int IPT>
__global__ __launch_bounds__(SDBG_BLOCK) void k_node_window_flags(ExArgs a, NodeTab t, uint8_t* __restrict__ wf) {
  static_assert(IPT % 2 == 0, "windows come in pairs");
  const uint64_t g0 = ((uint64_t)blockIdx.x * SDBG_BLOCK + threadIdx.x) * IPT;
  if (g0 >= a.NW) return;
  WinIter it;
  it.init(a, g0);
  uint64_t key[IPT], nk[IPT];
  bool ok[IPT];
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    ok[q] = false;
    key[q] = 0;
    nk[q] = 0;
    if (g0 + q < a.NW) {
      const uint64_t j = it.pos();
      if (!a.any_bad || window_clean(a.bad, j, a.k + 1)) {
        ok[q] = true;
        key[q] = key_from_fwd<1>(stream_bits<1>(a.packed, 2 * j, a.kb), a.kb).w[0];
        nk[q] = (q & 1) ? node_of_source(key[q], t.nkb) : node_of_target(key[q]);
      }
      it.next(a);
    }
  }
  bool dup[IPT];
  uint32_t sets[IPT];
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    dup[q] = (q & 1) && ok[q] && ok[q - 1] && nk[q] == nk[q - 1];
    sets[q] = ok[q] && !dup[q] ? node_sets_bw<BW>(t, nk[q]) : 0u;
  }
#pragma unroll
  for (int q = 1; q < IPT; q += 2)
    if (dup[q]) sets[q] = sets[q - 1];
#pragma unroll
  for (int q = 0; q < IPT; ++q)
    if (g0 + q < a.NW) wf[g0 + q] = ok[q] ? node_window_flag(key[q], sets[q], q & 1) : (uint8_t)0x80;
}

template <int W, int SWD>
__global__ void k_wslot_fill(const uint64_t* __restrict__ keys, uint64_t nS, const uint8_t* __restrict__ sfl,
                             uint64_t* __restrict__ tab, uint64_t nb, int bb, int rbits) {
  wslot_fill_one<W, SWD>(keys, nS, sfl, tab, nb, bb, rbits, blockIdx.x * (uint64_t)blockDim.x + threadIdx.x);
}

template <int W, int SWD, int IPT>
__global__ __launch_bounds__(SDBG_BLOCK) void k_window_flags(ExArgs a, const uint64_t* __restrict__ tab, int bb,
                                                             int rbits, SortedView S, const uint8_t* __restrict__ sfl,
                                                             uint8_t* __restrict__ wf) {
  wslot_window_flags<W, SWD, IPT>(a, tab, bb, rbits, S, sfl, wf,
                                  ((uint64_t)blockIdx.x * SDBG_BLOCK + threadIdx.x) * IPT);
}

// 1 where x[i] != 0; then, at the scanned positions, the indices themselves.
__global__ void k_nonzero(const uint64_t* __restrict__ x, uint64_t n, uint64_t* __restrict__ f) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) f[i] = x[i] != 0;
}

__global__ void k_list_nonzero(const uint64_t* __restrict__ x, uint64_t n, const uint64_t* __restrict__ pos,
                               uint64_t* __restrict__ list) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n && x[i]) list[pos[i]] = i;
}

// Mercy rule along each read (forward strand): consecutive solid windows
// p < q of one ACGT stretch, q - p >= 2, p without outgoing and q without
// incoming solid edge: windows p+1..q-1 and their reverse complements are
// mercy edges.  Pass 0 counts keys per read, pass 1 writes them (only for
// reads with a count).  Flags are read eight at a time (wf is padded to a
// whole word).  A flag the node lookups left unknown (one-word keys: 0x10
// no-out, 0x08 no-in) is looked up in the node table when a pair needs it;
// pass 0 writes it back into wf (each thread only its own read's bytes).
template <int W>
__global__ void k_mercy(ExArgs a, uint8_t* __restrict__ wf, int pass, uint64_t* __restrict__ mcount,
                        const uint64_t* __restrict__ mpos, uint64_t* __restrict__ cand, NodeTab nt,
                        const uint64_t* __restrict__ rlist, uint64_t nlist) {
  uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (pass) {
    // pass 1 runs over the list of reads with candidates, so that its waves
    // are full
    if (r >= nlist) return;
    r = rlist[r];
  } else if (r >= a.n_reads) {
    return;
  }
  const uint64_t g0 = a.woff[r], g1 = a.woff[r + 1];
  const uint64_t rs = a.offsets[r];
  uint64_t out = pass ? mpos[r] : 0, c = 0;
  int64_t p = -1;
  uint8_t fp = 0;
  const uint64_t* wf64 = reinterpret_cast<const uint64_t*>(wf);
  uint64_t wi = g0 >> 3;
  uint64_t word = g0 < g1 ? wf64[wi] >> (8 * (g0 & 7)) : 0;
  int avail = 8 - (int)(g0 & 7);
  for (uint64_t g = g0; g < g1; ++g) {
    if (!avail) {
      word = wf64[++wi];
      avail = 8;
    }
    const uint8_t f = (uint8_t)word;
    word >>= 8;
    --avail;
    if (f & 0x80) {
      p = -1;
      continue;
    }
    if (!(f & 1)) continue;
    const int64_t q = (int64_t)(g - g0);
    bool fire = false;
    if (p >= 0 && q - p >= 2) {
      bool noout = (fp & 2) != 0, noin = (f & 4) != 0;
      if constexpr (W == 1) {
        // pass 0 stores what it looked up, so pass 1 finds the flags known
        if (fp & 0x10) {
          const uint64_t x = key_from_fwd<1>(stream_bits<1>(a.packed, 2 * (rs + (uint64_t)p), a.kb), a.kb).w[0];
          noout = (node_sets(nt, node_of_target(x)) >> 4) == 0;
          wf[g0 + (uint64_t)p] = (uint8_t)((fp & ~0x10) | (noout ? 2 : 0));
        }
        if (noout && (f & 0x08)) {
          const uint64_t x = key_from_fwd<1>(stream_bits<1>(a.packed, 2 * (rs + (uint64_t)q), a.kb), a.kb).w[0];
          noin = (node_sets(nt, node_of_source(x, nt.nkb)) & 15) == 0;
          wf[g] = (uint8_t)((f & ~0x08) | (noin ? 4 : 0));
        }
      }
      fire = noout && noin;
    }
    if (fire) {
      if (!pass) {
        c += 2 * (uint64_t)(q - p - 1);
      } else {
        for (int64_t i = p + 1; i < q; ++i) {
          Key<W> kf, kr;
          window_keys<W>(a, rs + (uint64_t)i, &kf, &kr);
          key_store<W>(cand + out * W, kf);
          key_store<W>(cand + (out + 1) * W, kr);
          out += 2;
        }
      }
    }
    p = q;
    fp = f;
  }
  if (!pass) mcount[r] = c;
}

// Counts of mercy edges from the low-count set (d > 2); with canon, the set
// holds canonical keys only and an edge is looked up by its canonical key.
template <int W>
__global__ void k_lookup_counts(const uint64_t* __restrict__ keys, uint64_t n, SortedView L,
                                const uint32_t* __restrict__ lcnt, int canon, int kb, uint32_t* __restrict__ out) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  Key<W> q = key_load<W>(keys + i * W);
  if (canon) {
    const Key<W> r = key_revcomp<W>(q, kb);
    if (key_less<W>(r, q)) q = r;
  }
  uint64_t ix;
  out[i] = sv_find<W>(L, q, &ix) ? lcnt[ix] : 0;
}

// Counted canonical keys (one to three words) -> the other strand's keys.
// Every key that is not its own reverse complement gives its reverse
// complement with the same count, packed as a (W+1)-word key (key << 32 |
// count) so that the partition engine sorts the pairs by key.  Pass 0
// counts such keys per block of SDBG_BLOCK, pass 1 writes them at the
// scanned block offsets.
template <int W>
__global__ __launch_bounds__(SDBG_BLOCK) void k_rc_pack(const uint64_t* __restrict__ S,
                                                        const uint32_t* __restrict__ Sc, uint64_t n, int kb, int pass,
                                                        uint64_t* __restrict__ bpos, uint64_t* __restrict__ R2) {
  __shared__ uint32_t wc[SDBG_WAVES];
  const uint64_t i = blockIdx.x * (uint64_t)SDBG_BLOCK + threadIdx.x;
  Key<W> r = key_zero<W>();
  bool emit = false;
  if (i < n) {
    const Key<W> x = key_load<W>(S + i * W);
    r = key_revcomp<W>(x, kb);
    emit = !key_eq<W>(r, x);
  }
  const uint64_t m = __ballot(emit);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wc[wid] = (uint32_t)__popcll(m);
  __syncthreads();
  if (pass == 0) {
    if (threadIdx.x == 0) {
      uint64_t t = 0;
#pragma unroll
      for (int w = 0; w < SDBG_WAVES; ++w) t += wc[w];
      bpos[blockIdx.x] = t;
    }
    return;
  }
  if (!emit) return;
  uint64_t pos = bpos[blockIdx.x] + (uint64_t)__popcll(m & ((1ull << lane) - 1));
  for (int w = 0; w < wid; ++w) pos += wc[w];
  Key<W + 1> t;
  t.w[0] = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) t.w[j + 1] = r.w[j];
  t = key_shl<W + 1>(t, 32);
  t.w[W] |= Sc[i];
  key_store<W + 1>(R2 + pos * (W + 1), t);
}

template <int W>
__global__ void k_rc_unpack(const uint64_t* __restrict__ R2, uint64_t n, uint64_t* __restrict__ keys,
                            uint32_t* __restrict__ cnt) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Key<W + 1> t = key_load<W + 1>(R2 + i * (W + 1));
  cnt[i] = (uint32_t)t.w[W];
  const Key<W + 1> k = key_shr<W + 1>(t, 32);
  Key<W> out;
#pragma unroll
  for (int j = 0; j < W; ++j) out.w[j] = k.w[j + 1];
  key_store<W>(keys + i * W, out);
}

// Merge of two sorted key sets (with their counts) along the merge path
// (equal keys, if any, come out next to each other, B's first): output tile t covers positions [t*T, (t+1)*T); the split of each
// tile boundary between A and B is found by one binary search on the
// cross diagonal, then a workgroup stages its A and B runs in LDS, each
// thread merges a stretch of the tile's output along the same path, and the
// merged tile is written out through LDS.
template <int W>
struct MergeTile {
  static constexpr int T = W == 1 ? 2048 : W == 2 ? 1024 : 512;
};

template <int W>
__global__ void k_merge_split(const uint64_t* __restrict__ A, uint64_t na, const uint64_t* __restrict__ B, uint64_t nb,
                              uint64_t ntiles, uint64_t* __restrict__ split) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  const uint64_t d = min(t * (uint64_t)MergeTile<W>::T, na + nb);
  // smallest i in [max(0, d - nb), min(d, na)] with A[i] > B[d - i - 1]
  uint64_t lo = d > nb ? d - nb : 0, hi = min(d, na);
  while (lo < hi) {
    const uint64_t i = (lo + hi) >> 1;
    if (key_less<W>(key_load<W>(A + i * W), key_load<W>(B + (d - i - 1) * W)))
      lo = i + 1;
    else
      hi = i;
  }
  split[t] = lo;
}

template <int W>
__global__ __launch_bounds__(SDBG_BLOCK) void k_merge_tile(const uint64_t* __restrict__ A, const uint32_t* __restrict__ Ac,
                                                           uint64_t na, const uint64_t* __restrict__ B,
                                                           const uint32_t* __restrict__ Bc, uint64_t nb,
                                                           const uint64_t* __restrict__ split, uint64_t* __restrict__ E,
                                                           uint32_t* __restrict__ Ec) {
  constexpr int T = MergeTile<W>::T;
  __shared__ uint64_t la[T * W], lb[T * W];
  const uint64_t t = blockIdx.x;
  const uint64_t d0 = t * (uint64_t)T, d1 = min(d0 + T, na + nb);
  const uint64_t a0 = split[t], a1 = split[t + 1];
  const uint64_t b0 = d0 - a0, b1 = d1 - a1;
  const int nA = (int)(a1 - a0), nB = (int)(b1 - b0);
  for (int i = threadIdx.x; i < nA; i += SDBG_BLOCK) key_store<W>(&la[i * W], key_load<W>(A + (a0 + i) * W));
  for (int i = threadIdx.x; i < nB; i += SDBG_BLOCK) key_store<W>(&lb[i * W], key_load<W>(B + (b0 + i) * W));
  lds_barrier();
  // each thread merges PT consecutive outputs of the tile into registers:
  // its start on the merge path by one search along its diagonal, then a
  // sequential merge (on equal keys B's goes first, as in the split) ...
  static_assert(T % SDBG_BLOCK == 0, "whole outputs per thread");
  constexpr int PT = T / SDBG_BLOCK;
  const int n = nA + nB;
  const int o0 = min((int)threadIdx.x * PT, n);
  int lo = max(0, o0 - nB), hi = min(o0, nA);
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (key_less<W>(key_load<W>(&la[m * W]), key_load<W>(&lb[(o0 - m - 1) * W])))
      lo = m + 1;
    else
      hi = m;
  }
  int ia = lo, ib = o0 - lo;
  Key<W> ok[PT];
  uint32_t oc[PT];
#pragma unroll
  for (int q = 0; q < PT; ++q) {
    if (o0 + q < n) {
      const bool ta = ib >= nB || (ia < nA && key_less<W>(key_load<W>(&la[ia * W]), key_load<W>(&lb[ib * W])));
      ok[q] = key_load<W>(ta ? &la[ia * W] : &lb[ib * W]);
      oc[q] = ta ? Ac[a0 + ia] : Bc[b0 + ib];
      ia += ta;
      ib += !ta;
    }
  }
  // ... then the tile goes back through LDS (keys over la, counts over lb)
  // so that the stores are coalesced
  lds_barrier();
  uint32_t* lc = reinterpret_cast<uint32_t*>(lb);
#pragma unroll
  for (int q = 0; q < PT; ++q)
    if (o0 + q < n) {
      key_store<W>(&la[(o0 + q) * W], ok[q]);
      lc[o0 + q] = oc[q];
    }
  lds_barrier();
  for (int i = threadIdx.x; i < n; i += SDBG_BLOCK) {
    key_store_g<W>(E + (d0 + i) * W, key_load<W>(&la[i * W]));
    Ec[d0 + i] = lc[i];
  }
}

// Union of two edge sets (each ascending and unique): the merge along the
// merge path above keeps equal keys next to each other (B's first), so
// each key of the union starts a run of one or two; the first of a run
// takes the run's summed count.
template <int W>
__global__ void k_union_heads(const uint64_t* __restrict__ E, uint64_t n, uint32_t* __restrict__ head) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = i == 0 || !key_eq<W>(key_load<W>(E + (i - 1) * W), key_load<W>(E + i * W)) ? 1u : 0u;
}

template <int W>
__global__ void k_union_scatter(const uint64_t* __restrict__ E, const uint32_t* __restrict__ Ec, uint64_t n,
                                const uint64_t* __restrict__ pos, uint64_t* __restrict__ O, uint32_t* __restrict__ Oc,
                                uint32_t* __restrict__ overflow) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Key<W> x = key_load<W>(E + i * W);
  if (i > 0 && key_eq<W>(key_load<W>(E + (i - 1) * W), x)) return;
  uint64_t sum = Ec[i];
  if (i + 1 < n && key_eq<W>(key_load<W>(E + (i + 1) * W), x)) sum += Ec[i + 1];
  if (sum > 0xFFFFFFFFull) {
    atomicOr(overflow, 1u);
    sum = 0xFFFFFFFFull;
  }
  key_store_g<W>(O + pos[i] * W, x);
  Oc[pos[i]] = (uint32_t)sum;
}

}  // namespace sdbg

// ================================================================ host side
namespace sdbg {
namespace {

// SDBG_VERBOSE=1 in the environment traces sizes of each stage to stderr.
bool verbose() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("SDBG_VERBOSE");
    v = (e && *e && *e != '0') ? 1 : 0;
  }
  return v == 1;
}
#define VLOG(...)                         \
  do {                                    \
    if (verbose()) {                      \
      std::fprintf(stderr, "[sdbg] " __VA_ARGS__); \
      std::fputc('\n', stderr);          \
    }                                     \
  } while (0)

inline unsigned grid1(uint64_t n) {
  uint64_t g = ceil_div(n, SDBG_BLOCK);
  SDBG_CHECK(g < (1ull << 31), -1, "grid too large");
  return (unsigned)(g ? g : 1);
}

std::mutex g_tune_mu;
SortTune g_tune;

int cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n = v;
    else
      n = 256;
  }
  return n;
}

// Resident grid of the persistent node-table fill.
template <int BW>
unsigned node_fill_grid(uint64_t nblk) {
  static int resident = 0;
  if (!resident) {
    int r = 0;
    SDBG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, reinterpret_cast<const void*>(&k_node_fill<BW>),
                                                          NODE_FILL_THREADS, 0));
    resident = std::max(1, std::min(r, 32));
  }
  return (unsigned)std::min<uint64_t>(nblk, (uint64_t)cu_count() * resident);
}

struct SegList {
  DBuf<uint64_t> off, len;
  DBuf<uint16_t> bit;
  DBuf<uint8_t> buf, D;
  uint64_t n = 0;
  void alloc(Ctx& c, uint64_t cnt) {
    n = cnt;
    off = c.buf<uint64_t>(cnt);
    len = c.buf<uint64_t>(cnt);
    bit = c.buf<uint16_t>(cnt);
    buf = c.buf<uint8_t>(cnt);
    D = c.buf<uint8_t>(cnt);
  }
  SegView view() const { return SegView{off.get(), len.get(), bit.get(), buf.get(), D.get(), n}; }
};

// Keys of at most this many words are counted as canonical keys (a key and
// its count then fit kCanonWords + 1 words for the reverse-complement sort).
constexpr int kCanonWords = 3;

// Leaf launches with at least this many segments are split by segment size.
constexpr uint64_t kLeafSplitMin = 16384;

// Segment list split by size: flags (1 = at most cap keys), then the
// entries copied to the small or the large list with their positions in
// the original one (pos = exclusive scan of the flags).
__global__ void k_seg_small(SegView v, uint64_t cap, uint64_t* __restrict__ f) {
  const uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (s < v.n) f[s] = v.len[s] <= cap;
}

__global__ void k_seg_split(SegView v, uint64_t cap, const uint64_t* __restrict__ pos, SegView a, uint32_t* __restrict__ ida,
                            SegView b, uint32_t* __restrict__ idb) {
  const uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (s >= v.n) return;
  const bool small = v.len[s] <= cap;
  const uint64_t p = small ? pos[s] : s - pos[s];
  const SegView& o = small ? a : b;
  o.off[p] = v.off[s];
  o.len[p] = v.len[s];
  o.bit[p] = v.bit[s];
  o.buf[p] = v.buf[s];
  o.D[p] = v.D[s];
  (small ? ida : idb)[p] = (uint32_t)s;
}

// Initial segments from the first cut: digit d covers [start_d, start_d+len_d).
__global__ void k_seg_init(const uint32_t* __restrict__ tabscan, uint64_t ntiles, uint32_t nbins, uint64_t total,
                           int bit, SegView v) {
  uint32_t d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= nbins) return;
  uint64_t a = tabscan[(uint64_t)d * ntiles];
  uint64_t b = d + 1 < nbins ? tabscan[(uint64_t)(d + 1) * ntiles] : total;
  v.off[d] = a;
  v.len[d] = b - a;
  v.bit[d] = (uint16_t)bit;
  v.buf[d] = 0;
  v.D[d] = 0;
}

// Initial segments of several read sets: segment s * nbins + d is digit d
// of set s (st = first tile of each set, at least one tile per set).
__global__ void k_seg_init_sets(const uint32_t* __restrict__ tabscan, const uint64_t* __restrict__ st, uint64_t nsets,
                                int dbits, uint64_t total, int bit, SegView v) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint32_t nbins = 1u << dbits;
  if (i >= nsets * nbins) return;
  const uint64_t s = i >> dbits;
  const uint32_t d = (uint32_t)(i & (nbins - 1));
  const uint64_t t0 = st[s], nt = st[s + 1] - t0, base = t0 << dbits;
  const uint64_t a = tabscan[base + d * nt];
  const uint64_t b = d + 1 < nbins ? tabscan[base + (d + 1) * nt] : (s + 1 < nsets ? tabscan[st[s + 1] << dbits] : total);
  v.off[i] = a;
  v.len[i] = b - a;
  v.bit[i] = (uint16_t)bit;
  v.buf[i] = 0;
  v.D[i] = 0;
}

__global__ void k_gather_idx(const uint64_t* __restrict__ src, const uint64_t* __restrict__ idx, uint64_t n,
                             uint64_t* __restrict__ dst) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

// Per set s (and s = nsets for the end): its first key position and its
// first output edge.  Leaf segments are in key order, so the set's output
// starts at the scanned output count of its first segment (the first one
// at or after the set's first key).
__global__ void k_set_bounds(const uint64_t* __restrict__ seg_off, uint64_t nseg, const uint64_t* __restrict__ spos,
                             const uint32_t* __restrict__ tabscan, const uint64_t* __restrict__ st, int dbits,
                             uint64_t nsets, uint64_t total, uint64_t* __restrict__ key_base,
                             uint64_t* __restrict__ out_base) {
  const uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (s > nsets) return;
  const uint64_t kb = s < nsets ? tabscan[st[s] << dbits] : total;
  uint64_t lo = 0, hi = nseg;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (seg_off[mid] < kb)
      lo = mid + 1;
    else
      hi = mid;
  }
  key_base[s] = kb;
  out_base[s] = spos[lo];
}

__global__ void k_gather_strided(const uint32_t* __restrict__ src, uint64_t stride, uint32_t n, uint64_t* dst) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[(uint64_t)i * stride];
}

// The two ping-pong buffer pointers, written on the stream (no host wait).
__global__ void k_set_bufs(uint64_t** db, uint64_t* a, uint64_t* b) {
  if (threadIdx.x == 0) {
    db[0] = a;
    db[1] = b;
  }
}

// A segment list of one segment: all n keys, in buffer 0, `bit` key bits.
__global__ void k_seg_single(SegView v, uint64_t n, int bit) {
  if (threadIdx.x == 0) {
    v.off[0] = 0;
    v.len[0] = n;
    v.bit[0] = (uint16_t)bit;
    v.buf[0] = 0;
    v.D[0] = 0;
  }
}

template <int W>
struct Counter {
  static constexpr int IPT = Tune<W>::IPT, TK = Tune<W>::TK, CAP = Tune<W>::CAP;
  Ctx& c;
  SortTune tune;
  explicit Counter(Ctx& c_) : c(c_), tune(sort_tune()) {}
  bool distinct_keys = false;  // the next leaves() call sorts keys known to be distinct

  // Largest segment a leaf sorts (the refinement cuts until segments fit).
  uint64_t leaf_cap() const { return (uint64_t)CAP >> tune.leaf_cap_shift; }

  // Persistent leaf launch: as many workgroups as can be resident (at most
  // leaf_wg_per_cu per compute unit), so that none waits for another.
  template <int CAPX>
  void launch_leaf(const SegList& L, uint64_t* const* d_bufs, uint32_t* cnt, uint32_t dmin, bool want_low,
                   uint64_t* ns, uint64_t* nl, const uint32_t* ids = nullptr) {
    static int resident = 0;
    if (!resident) {
      int r = 0;
      SDBG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, reinterpret_cast<const void*>(&k_leaf<W, CAPX>),
                                                            SDBG_BLOCK, 0));
      resident = std::max(1, r);
    }
    const int per_cu = std::max(1, std::min(resident, tune.leaf_wg_per_cu));
    const unsigned lgrid = (unsigned)std::min<uint64_t>(L.n, (uint64_t)cu_count() * per_cu);
    k_leaf<W, CAPX><<<lgrid, SDBG_BLOCK, 0, c.s>>>(L.view(), d_bufs, cnt, dmin, want_low ? 1 : 0,
                                                   distinct_keys ? 1 : 0, ids, ns, nl);
    c.check_launch("leaf");
  }

  // Histogram and scatter of one refinement level with tiles of TKX keys.
  template <int TKX>
  void seg_pass(SegList& L, uint64_t* const* d_bufs, uint64_t NT, uint64_t NTab, uint64_t moved, DBuf<uint32_t>& tile_seg,
                DBuf<uint64_t>& tile_first, DBuf<uint64_t>& tab_base, DBuf<uint32_t>& tab) {
    {
      Stage st_(c, "seg_hist", moved * 8 * W + NTab * 4);
      k_seg_hist<W, TKX><<<(unsigned)NT, SDBG_BLOCK, 0, c.s>>>(L.view(), d_bufs, tile_seg.get(), tile_first.get(),
                                                                 tab_base.get(), tab.get());
      c.check_launch("seg_hist");
    }
    scan_excl<uint32_t, uint32_t>(tab.get(), tab.get(), NTab, nullptr, c);
    {
      Stage st_(c, "seg_scatter", moved * 16 * W + NTab * 4);
      k_seg_scatter<W, TKX><<<(unsigned)NT, SDBG_BLOCK, 0, c.s>>>(L.view(), d_bufs, tile_seg.get(), tile_first.get(),
                                                                    tab_base.get(), tab.get());
      c.check_launch("seg_scatter");
    }
  }

  // Cut every segment longer than CAP (while it has key bits left) until
  // all fit a leaf; data ping-pongs between bufs[0] and bufs[1] at equal
  // offsets.
  // Every level takes at least one bit off each oversized segment, so
  // kbits (the segments' largest `bit`) levels always suffice.
  void refine(SegList& L, uint64_t* const* d_bufs, int kbits) {
    DBuf<unsigned long long> st = c.buf<unsigned long long>(3);
    for (int level = 0; level <= kbits; ++level) {
      if (L.n == 0) return;
      unsigned long long hs[3];
      if (level > 0) {
        // segments the last cut left whole: skip their common bits
        k_seg_squeeze<W><<<(unsigned)std::min<uint64_t>(L.n, 4096), SDBG_BLOCK, 0, c.s>>>(L.view(), d_bufs,
                                                                                          leaf_cap());
        c.check_launch("seg_squeeze");
      }
      fill<uint64_t>(reinterpret_cast<uint64_t*>(st.get()), 3, 0, c);
      k_seg_stats<<<grid1(L.n), SDBG_BLOCK, 0, c.s>>>(L.view(), leaf_cap(), st.get());
      c.check_launch("seg_stats");
      c.d2h(hs, st.get(), 3);
      if (hs[0] == 0) return;
      const uint64_t avg = hs[1] / hs[0];
      VLOG("refine level %d: %llu segments, %llu oversized holding %llu keys", level, (unsigned long long)L.n,
           hs[0], hs[1]);
      int D = 1;
      while (D < tune.digit_bits && (avg >> D) > leaf_cap() / 2) ++D;
      const int tk = TK >> tune.tile_shift;
      DBuf<uint64_t> ntiles = c.buf<uint64_t>(L.n), tabsz = c.buf<uint64_t>(L.n);
      DBuf<uint64_t> tile_first = c.buf<uint64_t>(L.n), tab_base = c.buf<uint64_t>(L.n);
      DBuf<uint64_t> tot = c.buf<uint64_t>(2);
      k_seg_mark<<<grid1(L.n), SDBG_BLOCK, 0, c.s>>>(L.view(), leaf_cap(), D, tk, ntiles.get(), tabsz.get());
      c.check_launch("seg_mark");
      scan_excl<uint64_t, uint64_t>(ntiles.get(), tile_first.get(), L.n, tot.get(), c);
      scan_excl<uint64_t, uint64_t>(tabsz.get(), tab_base.get(), L.n, tot.get() + 1, c);
      uint64_t ht[2];
      c.d2h(ht, tot.get(), 2);
      const uint64_t NT = ht[0], NTab = ht[1];
      SDBG_CHECK(NT < (1ull << 31), -3, "too many partition tiles");
      DBuf<uint32_t> tile_seg = c.buf<uint32_t>(NT), tab = c.buf<uint32_t>(NTab);
      k_seg_tiles<<<grid1(NT), SDBG_BLOCK, 0, c.s>>>(L.view(), tile_first.get(), NT, tile_seg.get());
      c.check_launch("seg_tiles");
      if (tk == TK)
        seg_pass<TK>(L, d_bufs, NT, NTab, hs[1], tile_seg, tile_first, tab_base, tab);
      else
        seg_pass<TK / 2>(L, d_bufs, NT, NTab, hs[1], tile_seg, tile_first, tab_base, tab);
      DBuf<uint64_t> ncnt = c.buf<uint64_t>(L.n), npos = c.buf<uint64_t>(L.n);
      k_seg_newcount<<<grid1(L.n * 64), SDBG_BLOCK, 0, c.s>>>(L.view(), tk, tab_base.get(), tab.get(), ncnt.get());
      c.check_launch("seg_newcount");
      scan_excl<uint64_t, uint64_t>(ncnt.get(), npos.get(), L.n, tot.get(), c);
      const uint64_t nn = c.d2h_one(tot.get());
      SegList N;
      N.alloc(c, nn);
      k_seg_newwrite<<<grid1(L.n * 64), SDBG_BLOCK, 0, c.s>>>(L.view(), tk, tab_base.get(), tab.get(), npos.get(),
                                                             N.view());
      c.check_launch("seg_newwrite");
      L = std::move(N);
    }
    throw Error(-4, "partition did not converge");
  }

  // Leaves -> dense sorted (key, count) arrays of the distinct keys with
  // count >= dmin, and (if want_low) of those below.
  // spos_keep (optional) receives each segment's first output position,
  // with the total at index L.n.
  void leaves(SegList& L, uint64_t nkeys, uint64_t* const* d_bufs, uint32_t* cnt, uint32_t dmin, bool want_low,
              DBuf<uint64_t>& skeys, DBuf<uint32_t>& scnt, uint64_t* ns_out, DBuf<uint64_t>& lkeys,
              DBuf<uint32_t>& lcnt, uint64_t* nl_out, DBuf<uint64_t>* spos_keep = nullptr) {
    DBuf<uint64_t> nsolid = c.buf<uint64_t>(L.n), nlow = c.buf<uint64_t>(L.n);
    DBuf<uint64_t> spos = c.buf<uint64_t>(L.n + 1), lpos = c.buf<uint64_t>(L.n), tot = c.buf<uint64_t>(2);
    if (verbose() && L.n) {
      // leaf sizes: segments and keys up to 256, 512, 1024, 2048 keys, longer (runs of one key)
      std::vector<uint64_t> len(L.n);
      c.d2h(len.data(), L.len.get(), L.n);
      uint64_t ns[5] = {}, nk[5] = {};
      for (uint64_t x : len) {
        const int b = x <= 256 ? 0 : x <= 512 ? 1 : x <= 1024 ? 2 : x <= 2048 ? 3 : 4;
        ++ns[b];
        nk[b] += x;
      }
      VLOG("leaves: %llu segments, %llu keys; by size <=256/512/1024/2048/longer: segments %llu %llu %llu %llu %llu, "
           "keys %llu %llu %llu %llu %llu",
           (unsigned long long)L.n, (unsigned long long)nkeys, (unsigned long long)ns[0], (unsigned long long)ns[1],
           (unsigned long long)ns[2], (unsigned long long)ns[3], (unsigned long long)ns[4], (unsigned long long)nk[0],
           (unsigned long long)nk[1], (unsigned long long)nk[2], (unsigned long long)nk[3], (unsigned long long)nk[4]);
    }
    if (L.n) {
      Stage st_(c, "leaf", nkeys * 8 * W);
      if (tune.leaf_cap_shift == 0 && L.n >= kLeafSplitMin) {
        // segments of at most CAP/2 keys go to the half-size leaf, which
        // keeps more workgroups on a CU; the others to the full-size one
        DBuf<uint64_t> pos = c.buf<uint64_t>(L.n + 1);
        k_seg_small<<<grid1(L.n), SDBG_BLOCK, 0, c.s>>>(L.view(), (uint64_t)CAP / 2, pos.get());
        scan_excl<uint64_t, uint64_t>(pos.get(), pos.get(), L.n, pos.get() + L.n, c);
        const uint64_t ns_small = c.d2h_one(pos.get() + L.n);
        SegList A, B;
        A.alloc(c, ns_small);
        B.alloc(c, L.n - ns_small);
        DBuf<uint32_t> ida = c.buf<uint32_t>(A.n), idb = c.buf<uint32_t>(B.n);
        k_seg_split<<<grid1(L.n), SDBG_BLOCK, 0, c.s>>>(L.view(), (uint64_t)CAP / 2, pos.get(), A.view(), ida.get(),
                                                        B.view(), idb.get());
        c.check_launch("seg_split");
        if (A.n) launch_leaf<CAP / 2>(A, d_bufs, cnt, dmin, want_low, nsolid.get(), nlow.get(), ida.get());
        if (B.n) launch_leaf<CAP>(B, d_bufs, cnt, dmin, want_low, nsolid.get(), nlow.get(), idb.get());
      } else if (tune.leaf_cap_shift == 0) {
        launch_leaf<CAP>(L, d_bufs, cnt, dmin, want_low, nsolid.get(), nlow.get());
      } else {
        launch_leaf<CAP / 2>(L, d_bufs, cnt, dmin, want_low, nsolid.get(), nlow.get());
      }
    }
    scan_excl<uint64_t, uint64_t>(nsolid.get(), spos.get(), L.n, spos.get() + L.n, c);
    scan_excl<uint64_t, uint64_t>(nlow.get(), lpos.get(), L.n, tot.get() + 1, c);
    c.d2d(tot.get(), spos.get() + L.n, 1);
    uint64_t ht[2];
    c.d2h(ht, tot.get(), 2);
    *ns_out = ht[0];
    *nl_out = want_low ? ht[1] : 0;
    const uint64_t outb = (*ns_out + *nl_out) * (8 * W + 4);
    if (L.n) prof_set_last_bytes(nkeys * 8 * W + outb);
    skeys = c.buf<uint64_t>(ht[0] * W);
    scnt = c.buf<uint32_t>(ht[0]);
    if (want_low) {
      lkeys = c.buf<uint64_t>(ht[1] * W);
      lcnt = c.buf<uint32_t>(ht[1]);
    }
    if (L.n) {
      Stage st_(c, "compact", 2 * outb + L.n * 32);
      k_compact<W><<<(unsigned)ceil_div(L.n, SDBG_WAVES), SDBG_BLOCK, 0, c.s>>>(L.view(), d_bufs, cnt, nsolid.get(),
                                                                             spos.get(),
                                                            want_low ? nlow.get() : nullptr, lpos.get(), skeys.get(),
                                                            scnt.get(), want_low ? lkeys.get() : nullptr,
                                                            want_low ? lcnt.get() : nullptr);
      c.check_launch("compact");
    }
    if (spos_keep) *spos_keep = std::move(spos);
  }

  // Sorted distinct keys of an arbitrary key array (consumed).
  // distinct: the keys are known to be pairwise different (the leaves skip
  // their duplicate merge).
  void sort_unique(DBuf<uint64_t>& keys, uint64_t n, int kb, DBuf<uint64_t>& out, uint64_t* nout,
                   bool distinct = false) {
    SDBG_CHECK(n < (1ull << 32), -3, "key array too large for one partition group");
    DBuf<uint64_t> other = c.buf<uint64_t>(n * W);
    DBuf<uint32_t> cnt = c.buf<uint32_t>(n);
    DBuf<uint64_t*> db = c.buf<uint64_t*>(2);
    k_set_bufs<<<1, 64, 0, c.s>>>(db.get(), keys.get(), other.get());
    c.check_launch("set_bufs");
    SegList L;
    L.alloc(c, 1);
    k_seg_single<<<1, 64, 0, c.s>>>(L.view(), n, kb);
    c.check_launch("seg_single");
    refine(L, db.get(), kb);
    DBuf<uint32_t> ocnt;
    DBuf<uint64_t> lk;
    DBuf<uint32_t> lc;
    uint64_t nl;
    distinct_keys = distinct;
    leaves(L, n, db.get(), cnt.get(), 1, false, out, ocnt, nout, lk, lc, &nl);
    distinct_keys = false;
    c.sync();
  }

  // Merge of two sorted key sets with their counts.
  void merge_sets(const char* name, const uint64_t* A, const uint32_t* Ac, uint64_t nA, const uint64_t* B,
                  const uint32_t* Bc, uint64_t nB, DBuf<uint64_t>& E, DBuf<uint32_t>& Ec) {
    E = c.buf<uint64_t>((nA + nB) * W);
    Ec = c.buf<uint32_t>(nA + nB);
    const uint64_t mt = ceil_div(nA + nB, MergeTile<W>::T);
    SDBG_CHECK(mt < (1ull << 31), -3, "merge too large");
    DBuf<uint64_t> split = c.buf<uint64_t>(mt + 1);
    k_merge_split<W><<<grid1(mt + 1), SDBG_BLOCK, 0, c.s>>>(A, nA, B, nB, mt, split.get());
    c.check_launch("merge_split");
    {
      Stage st_(c, name, 2 * (nA + nB) * (8 * W + 4));
      k_merge_tile<W><<<(unsigned)mt, SDBG_BLOCK, 0, c.s>>>(A, Ac, nA, B, Bc, nB, split.get(), E.get(), Ec.get());
      c.check_launch(name);
    }
    c.sync();
  }

  // Canonical counted keys -> both strands' keys: the reverse complements
  // (with the same counts) are sorted as two-word (key, count) keys and
  // merged in.  One-word keys only.
  void expand_rc(DBuf<uint64_t>& S, DBuf<uint32_t>& Sc, uint64_t* nS, int kb) {
    if constexpr (W <= kCanonWords) {
      const uint64_t n = *nS;
      const uint64_t nblk = ceil_div(n, SDBG_BLOCK);
      DBuf<uint64_t> bpos = c.buf<uint64_t>(nblk), tot = c.buf<uint64_t>(1);
      k_rc_pack<W><<<(unsigned)nblk, SDBG_BLOCK, 0, c.s>>>(S.get(), Sc.get(), n, kb, 0, bpos.get(), nullptr);
      c.check_launch("rc_count");
      scan_excl<uint64_t, uint64_t>(bpos.get(), bpos.get(), nblk, tot.get(), c);
      const uint64_t nR = c.d2h_one(tot.get());
      DBuf<uint64_t> R2 = c.buf<uint64_t>((W + 1) * nR);
      {
        Stage st_(c, "rc_pack", n * (8 * W + 4) + nR * 8 * (W + 1));
        k_rc_pack<W><<<(unsigned)nblk, SDBG_BLOCK, 0, c.s>>>(S.get(), Sc.get(), n, kb, 1, bpos.get(), R2.get());
        c.check_launch("rc_pack");
      }
      if (nR == 0) return;
      DBuf<uint64_t> R2s;
      uint64_t nR2 = 0;
      {
        Counter<W + 1> c2(c);
        c2.sort_unique(R2, nR, kb + 32, R2s, &nR2, true);
      }
      SDBG_CHECK(nR2 == nR, -4, "reverse complement keys are not distinct");
      R2.free();
      DBuf<uint64_t> Rk = c.buf<uint64_t>(nR * W);
      DBuf<uint32_t> Rc = c.buf<uint32_t>(nR);
      {
        Stage st_(c, "rc_unpack", nR * 8 * (W + 1) + nR * (8 * W + 4));
        k_rc_unpack<W><<<grid1(nR), SDBG_BLOCK, 0, c.s>>>(R2s.get(), nR, Rk.get(), Rc.get());
        c.check_launch("rc_unpack");
      }
      R2s.free();
      DBuf<uint64_t> E;
      DBuf<uint32_t> Ec;
      merge_sets("rc_merge", S.get(), Sc.get(), n, Rk.get(), Rc.get(), nR, E, Ec);
      S = std::move(E);
      Sc = std::move(Ec);
      *nS = n + nR;
    } else {
      (void)S;
      (void)Sc;
      (void)nS;
      (void)kb;
      throw Error(-4, "canonical counting is for keys of at most three words");
    }
  }

  SortedView make_view(const uint64_t* keys, uint64_t n, int kbits, DBuf<uint64_t>& dir) {
    int db = 1;
    while (db < 24 && db < kbits && (n >> (db + 3)) > 0) ++db;
    return make_view_db(keys, n, kbits, db, dir);
  }

  SortedView make_view_db(const uint64_t* keys, uint64_t n, int kbits, int db, DBuf<uint64_t>& dir) {
    dir = c.buf<uint64_t>((1ull << db) + 1);
    k_dir<W><<<grid1(n + 1), SDBG_BLOCK, 0, c.s>>>(keys, n, kbits, db, dir.get());
    c.check_launch("dir");
    return SortedView{keys, dir.get(), n, kbits, db};
  }

  // Packed reads, window offsets and the window -> read table.
  struct Prep {
    DBuf<uint64_t> packed, bad, woff, trd;
    uint64_t words = 0, NW = 0;
    uint32_t any_bad = 0;
    ExArgs ea{};
  };

  void prepare(const DevReads& R, int k, Prep& pr) {
    const int kb = 2 * (k + 1);
    const uint64_t nb = R.n_bases;
    // ---- pack
    const uint64_t words = ceil_div(nb, 64);
    pr.words = words;
    DBuf<uint64_t>& packed = pr.packed;
    DBuf<uint64_t>& bad = pr.bad;
    packed = c.buf<uint64_t>(2 * words + W + 8);
    bad = c.buf<uint64_t>(words + 8);
    DBuf<uint32_t> anyb = c.buf<uint32_t>(1);
    fill<uint64_t>(packed.get() + 2 * words, W + 8, 0, c);
    fill<uint64_t>(bad.get() + words, 8, 0, c);
    fill<uint32_t>(anyb.get(), 1, 0, c);
    if (words) {
      Stage st_(c, "pack", nb + 3 * words * 8);
      k_pack<<<grid1(words), SDBG_BLOCK, 0, c.s>>>(R.seq, nb, packed.get(), bad.get(), anyb.get());
      c.check_launch("pack");
    }
    // ---- windows per read
    DBuf<uint64_t>& woff = pr.woff;
    woff = c.buf<uint64_t>(R.n_reads + 1);
    {
      DBuf<uint64_t> nwin = c.buf<uint64_t>(R.n_reads);
      if (R.n_reads) {
        k_nwin<<<grid1(R.n_reads), SDBG_BLOCK, 0, c.s>>>(R.offsets, R.n_reads, k, nwin.get());
        c.check_launch("nwin");
      }
      scan_excl<uint64_t, uint64_t>(nwin.get(), woff.get(), R.n_reads, woff.get() + R.n_reads, c);
    }
    const uint64_t NW = c.d2h_one(woff.get() + R.n_reads);
    const uint32_t any_bad = c.d2h_one(anyb.get());
    pr.NW = NW;
    pr.any_bad = any_bad;
    if (NW == 0) return;

    ExArgs& ea = pr.ea;
    ea.packed = packed.get();
    ea.bad = bad.get();
    ea.woff = woff.get();
    ea.offsets = R.offsets;
    ea.n_reads = R.n_reads;
    ea.NW = NW;
    ea.any_bad = any_bad ? 1 : 0;
    ea.k = k;
    ea.kb = kb;
    ea.pb = std::min(16, kb);
    ea.glo = 0;
    ea.ghi = 1u << ea.pb;
    ea.dbits = std::min(tune.first_bits, kb);
    ea.dlo = kb - ea.dbits;
    const uint64_t ntr = ceil_div(NW, TR_GRAIN) + 1;
    DBuf<uint64_t>& trd = pr.trd;
    trd = c.buf<uint64_t>(ntr);
    fill<uint64_t>(trd.get() + ntr - 1, 1, R.n_reads - 1, c);
    k_tile_reads<<<grid1(R.n_reads), SDBG_BLOCK, 0, c.s>>>(woff.get(), R.n_reads, trd.get());
    c.check_launch("tile_reads");
    ea.tr = trd.get();
  }

  // Fill the word-slot table and probe it once per forward window.
  template <int SWD>
  void window_flags_sw(const ExArgs& ea, const WordSlots& ws, const SortedView& bv, const uint64_t* skeys,
                       const uint8_t* sfl, uint64_t* btab, uint64_t nb, uint64_t NW, uint64_t words, uint8_t* wf,
                       uint64_t nS) {
    if constexpr (SWD <= W) {
      {
        Stage st_(c, "bucket_fill", nS * (8 * W + 1) + nb * WS_SLOTS * SWD * 8);
        k_wslot_fill<W, SWD><<<grid1(nS), SDBG_BLOCK, 0, c.s>>>(skeys, nS, sfl, btab, nb, ws.bb, ws.rbits);
        c.check_launch("bucket_fill");
      }
      // each probe reads its bucket of 4 slots
      Stage st_(c, "window_flags", 3 * words * 8 + NW + NW * WS_SLOTS * SWD * 8);
      constexpr int WIPT = W == 2 ? 4 : W == 4 ? 2 : 1;
      k_window_flags<W, SWD, WIPT><<<grid1(ceil_div(NW, WIPT)), SDBG_BLOCK, 0, c.s>>>(ea, btab, ws.bb, ws.rbits, bv,
                                                                                    sfl, wf);
      c.check_launch("window_flags");
    } else {
      throw Error(-4, "slot wider than a key");
    }
  }

  void window_flags_ws(const ExArgs& ea, const WordSlots& ws, const SortedView& bv, const uint64_t* skeys,
                       const uint8_t* sfl, uint64_t* btab, uint64_t nb, uint64_t NW, uint64_t words, uint8_t* wf,
                       uint64_t nS) {
    switch (ws.swd) {
      case 1: window_flags_sw<1>(ea, ws, bv, skeys, sfl, btab, nb, NW, words, wf, nS); break;
      case 2: window_flags_sw<2>(ea, ws, bv, skeys, sfl, btab, nb, NW, words, wf, nS); break;
      case 3: window_flags_sw<3>(ea, ws, bv, skeys, sfl, btab, nb, NW, words, wf, nS); break;
      case 4: window_flags_sw<4>(ea, ws, bv, skeys, sfl, btab, nb, NW, words, wf, nS); break;
      default: throw Error(-4, "bad slot width");
    }
  }

  void run(const DevReads& R, const CountParams& P, EdgesOut* out) {
    const int k = P.k, kb = 2 * (k + 1);
    Prep pr;
    prepare(R, k, pr);
    *out = EdgesOut{};
    if (pr.NW == 0) return;
    const uint64_t NW = pr.NW, words = pr.words;
    ExArgs ea = pr.ea;
    // Keys of up to three words are counted on one strand (canonical keys)
    // and expanded to both strands afterwards: half the keys pass the
    // partition.
    ea.canon = W <= kCanonWords ? 1 : 0;
    const uint32_t nbins = 1u << ea.dbits;
    const uint64_t win_per_tile = (uint64_t)SDBG_BLOCK * IPT;
    const uint64_t ntiles = ceil_div(NW, win_per_tile);
    SDBG_CHECK(ntiles < (1ull << 31), -3, "too many reads for one launch");

    // ---- first-digit histogram over all keys
    // Every key passes the unfiltered histogram, so the scan total is the
    // number N of keys to sort; for a single group the scanned table is
    // also the scatter's offset table.  The occurrences (two per clean
    // window) are counted alongside.
    DBuf<uint32_t> tab = c.buf<uint32_t>(ntiles * nbins);
    DBuf<uint64_t> tot = c.buf<uint64_t>(1);
    DBuf<uint64_t> occ = c.buf<uint64_t>(ea.any_bad ? ntiles : 0);
    {
      Stage st_(c, "ex_hist", 3 * words * 8 + ntiles * nbins * 4);
      k_ex_hist<W, IPT><<<(unsigned)ntiles, SDBG_BLOCK, 0, c.s>>>(ea, tab.get(), ntiles,
                                                                  ea.any_bad ? occ.get() : nullptr);
      c.check_launch("ex_hist");
    }
    scan_excl<uint32_t, uint32_t>(tab.get(), tab.get(), ntiles * nbins, tot.get(), c);
    const uint64_t N = c.d2h_one(tot.get());
    if (ea.any_bad) {
      // (tot keeps N: a single group's scatter reads it again)
      DBuf<uint64_t> otot = c.buf<uint64_t>(1);
      scan_excl<uint64_t, uint64_t>(occ.get(), occ.get(), ntiles, otot.get(), c);
      out->n_occ = c.d2h_one(otot.get());
    } else {
      out->n_occ = 2 * NW;
    }
    occ.free();

    // ---- groups of consecutive prefix blocks within the memory budget
    uint64_t budget = P.mem_budget;
    if (!budget) {
      size_t fr = 0, totm = 0;
      SDBG_HIP(hipMemGetInfo(&fr, &totm));
      budget = (uint64_t)(0.8 * (double)(fr + Pool::get().cached_bytes()));
    }
    const uint64_t per_key = 16ull * W + 4;
    uint64_t max_keys = std::min<uint64_t>(budget / per_key, 0xFFFFFFFFull);
    std::vector<std::pair<uint32_t, uint32_t>> groups;
    if (N <= max_keys || P.prefix_len == 0) {
      SDBG_CHECK(N <= max_keys, -3, "memory budget cannot hold the keys and prefix_len is 0");
      groups.push_back({0u, 1u << ea.pb});
    } else {
      const int ub = std::max(0, ea.pb - 2 * P.prefix_len);  // block = 2^ub prefix values
      const uint32_t nvals = 1u << ea.pb;
      // Key counts per first-cut digit come from the scanned histogram table
      // already at hand; when every digit fits the budget and digit ranges
      // are unions of prefix blocks, groups are planned on digits and no
      // finer histogram is needed.
      const int dshift = ea.pb - ea.dbits;  // prefix values per digit = 2^dshift
      std::vector<uint64_t> dstart(nbins + 1);
      {
        DBuf<uint64_t> ds = c.buf<uint64_t>(nbins);
        k_gather_strided<<<grid1(nbins), SDBG_BLOCK, 0, c.s>>>(tab.get(), ntiles, nbins, ds.get());
        c.check_launch("gather_strided");
        c.d2h(dstart.data(), ds.get(), nbins);
        dstart[nbins] = N & 0xFFFFFFFFull;
      }
      // The table holds 32-bit positions, so starts are exact modulo 2^32;
      // the differences are the digit counts if they add up to N (no digit
      // holds 2^32 keys or more).
      std::vector<uint64_t> dcount(nbins);
      uint64_t dsum = 0;
      for (uint32_t d = 0; d < nbins; ++d) {
        dcount[d] = (uint32_t)(dstart[d + 1] - dstart[d]);
        dsum += dcount[d];
      }
      bool digits_fit = ub <= dshift && dsum == N;
      for (uint32_t d = 0; d < nbins && digits_fit; ++d) digits_fit = dcount[d] <= max_keys;
      std::vector<unsigned long long> h;
      uint32_t unit;
      if (digits_fit) {
        unit = 1u << dshift;
        h.assign(nvals, 0);
        for (uint32_t d = 0; d < nbins; ++d) h[(uint64_t)d << dshift] = dcount[d];
      } else {
        unit = 1u << ub;
        DBuf<unsigned long long> ph = c.buf<unsigned long long>(nvals);
        fill<uint64_t>(reinterpret_cast<uint64_t*>(ph.get()), nvals, 0, c);
        k_ex_hist_prefix<W, IPT><<<(unsigned)ntiles, SDBG_BLOCK, 0, c.s>>>(ea, ph.get());
        c.check_launch("ex_hist_prefix");
        h.resize(nvals);
        c.d2h(h.data(), ph.get(), h.size());
      }
      uint32_t g0 = 0;
      uint64_t acc = 0;
      for (uint32_t u = 0; u < nvals; u += unit) {
        uint64_t bs = 0;
        for (uint32_t x = u; x < u + unit; ++x) bs += h[x];
        SDBG_CHECK(bs <= max_keys, -3, "one prefix block exceeds the memory budget");
        if (acc + bs > max_keys) {
          groups.push_back({g0, u});
          g0 = u;
          acc = 0;
        }
        acc += bs;
      }
      groups.push_back({g0, nvals});
    }

    // ---- per group: partition, leaves, compaction
    std::vector<DBuf<uint64_t>> s_keys(groups.size()), l_keys(groups.size());
    std::vector<DBuf<uint32_t>> s_cnt(groups.size()), l_cnt(groups.size());
    std::vector<uint64_t> s_n(groups.size()), l_n(groups.size());
    const bool want_low = P.mercy && P.d > 2;
    {
      const uint64_t cap_keys = groups.size() == 1 ? N : max_keys;
      DBuf<uint64_t> bufA = c.buf<uint64_t>(cap_keys * W), bufB = c.buf<uint64_t>(cap_keys * W);
      DBuf<uint32_t> cnt = c.buf<uint32_t>(cap_keys);
      DBuf<uint64_t*> db = c.buf<uint64_t*>(2);
      k_set_bufs<<<1, 64, 0, c.s>>>(db.get(), bufA.get(), bufB.get());
      c.check_launch("set_bufs");
      for (size_t gi = 0; gi < groups.size(); ++gi) {
        ExArgs ga = ea;
        ga.glo = groups[gi].first;
        ga.ghi = groups[gi].second;
        if (groups.size() > 1) {
          k_ex_hist<W, IPT><<<(unsigned)ntiles, SDBG_BLOCK, 0, c.s>>>(ga, tab.get(), ntiles, nullptr);
          c.check_launch("ex_hist(group)");
          scan_excl<uint32_t, uint32_t>(tab.get(), tab.get(), ntiles * nbins, tot.get(), c);
        }
        const uint64_t NG = c.d2h_one(tot.get());
        SDBG_CHECK(NG <= cap_keys, -4, "group larger than planned");
        if (NG == 0) continue;
        {
          Stage st_(c, "ex_scatter", 3 * words * 8 + ntiles * nbins * 4 + NG * 8 * W);
          k_ex_scatter<W, IPT><<<(unsigned)ntiles, SDBG_BLOCK, 0, c.s>>>(ga, tab.get(), ntiles, bufA.get());
          c.check_launch("ex_scatter");
        }
        SegList L;
        L.alloc(c, nbins);
        k_seg_init<<<grid1(nbins), SDBG_BLOCK, 0, c.s>>>(tab.get(), ntiles, nbins, NG, kb - ea.dbits, L.view());
        c.check_launch("seg_init");
        refine(L, db.get(), kb - ea.dbits);
        leaves(L, NG, db.get(), cnt.get(), P.d, want_low, s_keys[gi], s_cnt[gi], &s_n[gi], l_keys[gi], l_cnt[gi],
               &l_n[gi]);
      }
    }
    tab.free();
    // ---- concatenate groups
    uint64_t nS = 0, nL = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      nS += s_n[gi];
      nL += l_n[gi];
    }
    DBuf<uint64_t> S, Lk;
    DBuf<uint32_t> Sc, Lc;
    if (groups.size() == 1) {
      S = std::move(s_keys[0]);
      Sc = std::move(s_cnt[0]);
      Lk = std::move(l_keys[0]);
      Lc = std::move(l_cnt[0]);
    } else {
      S = c.buf<uint64_t>(nS * W);
      Sc = c.buf<uint32_t>(nS);
      Lk = c.buf<uint64_t>(nL * W);
      Lc = c.buf<uint32_t>(nL);
      uint64_t ps = 0, pl = 0;
      for (size_t gi = 0; gi < groups.size(); ++gi) {
        c.d2d(S.get() + ps * W, s_keys[gi].get(), s_n[gi] * W);
        c.d2d(Sc.get() + ps, s_cnt[gi].get(), s_n[gi]);
        c.d2d(Lk.get() + pl * W, l_keys[gi].get(), l_n[gi] * W);
        c.d2d(Lc.get() + pl, l_cnt[gi].get(), l_n[gi]);
        ps += s_n[gi];
        pl += l_n[gi];
      }
      c.sync();
      s_keys.clear();
      s_cnt.clear();
      l_keys.clear();
      l_cnt.clear();
    }

    // ---- both strands
    if (ea.canon && nS > 0) expand_rc(S, Sc, &nS, kb);

    // ---- mercy-kmers
    DBuf<uint64_t> M;
    DBuf<uint32_t> Mc;
    uint64_t nM = 0;
    if (P.mercy && P.d >= 2 && nS > 0) {
      DBuf<uint64_t> sdir;
      SortedView sv = make_view(S.get(), nS, kb, sdir);
      DBuf<uint8_t> sfl;
      DBuf<uint8_t> wf = c.buf<uint8_t>(NW + 8);
      DBuf<uint64_t> btab, spill;
      NodeTab nt{};
      if constexpr (W == 1) {
        // node table, about slots/2 nodes per bucket
        const NodeShape ns = node_shape(k, nS, tune.mercy_shift, NODE_BW, NODE_LOAD);
        const uint64_t nb = 1ull << ns.bb, nblk = nb >> ns.s;
        btab = c.buf<uint64_t>(ns.bw * nb);
        spill = c.buf<uint64_t>(SPILL_WORDS * nblk);
        nt = NodeTab{btab.get(), spill.get(), sv, ns.nkb, ns.bw, ns.rbits, ns.sb, ns.slots, ns.s, ns.ssb, ns.sslots};
        VLOG("mercy node table: 2^%d buckets of %d words, %d slots of %d bits; spill lines of %d slots", ns.bb, ns.bw,
             ns.slots, ns.sb, ns.sslots);
        {
          // every solid edge is staged twice (as an in-edge and as an out-edge)
          Stage st_(c, "node_fill", nS * 16 + nb * 8 * ns.bw + nblk * 8 * SPILL_WORDS);
          if (ns.bw == 4)
            k_node_fill<4><<<node_fill_grid<4>(nblk), NODE_FILL_THREADS, 0, c.s>>>(sv, ns, btab.get(), spill.get());
          else
            k_node_fill<2><<<node_fill_grid<2>(nblk), NODE_FILL_THREADS, 0, c.s>>>(sv, ns, btab.get(), spill.get());
          c.check_launch("node_fill");
        }
        {
          // one bucket per pair of windows
          Stage st_(c, "window_flags", 3 * words * 8 + NW + ceil_div(NW, 2) * 8 * ns.bw);
          if (ns.bw == 4)
            k_node_window_flags<4, 12><<<grid1(ceil_div(NW, 12)), SDBG_BLOCK, 0, c.s>>>(ea, nt, wf.get());
          else
            k_node_window_flags<2, 12><<<grid1(ceil_div(NW, 12)), SDBG_BLOCK, 0, c.s>>>(ea, nt, wf.get());
          c.check_launch("window_flags");
        }
      } else {
        sfl = c.buf<uint8_t>(nS);
        {
          Stage st_(c, "dead_ends", nS * (8 * W + 1));
          k_dead_ends<W><<<grid1(nS), SDBG_BLOCK, 0, c.s>>>(sv, k, sfl.get());
          c.check_launch("dead_ends");
        }
        // word-slot buckets, about 2 solid keys per bucket of 4
        const WordSlots ws = word_slots_shape(kb, W, nS, tune.mercy_shift);
        const uint64_t nb = 1ull << ws.bb;
        btab = c.buf<uint64_t>(nb * WS_SLOTS * ws.swd);
        VLOG("mercy table: 2^%d buckets of %d x %d words", ws.bb, WS_SLOTS, ws.swd);
        window_flags_ws(ea, ws, sv, S.get(), sfl.get(), btab.get(), nb, NW, words, wf.get(), nS);
      }
      DBuf<uint64_t> mcount = c.buf<uint64_t>(R.n_reads), mpos = c.buf<uint64_t>(R.n_reads);
      {
        Stage st_(c, "mercy_count", NW + R.n_reads * 24);
        k_mercy<W><<<grid1(R.n_reads), SDBG_BLOCK, 0, c.s>>>(ea, wf.get(), 0, mcount.get(), nullptr, nullptr, nt,
                                                            nullptr, 0);
        c.check_launch("mercy_count");
      }
      scan_excl<uint64_t, uint64_t>(mcount.get(), mpos.get(), R.n_reads, tot.get(), c);
      const uint64_t NC = c.d2h_one(tot.get());
      VLOG("mercy: %llu solid edges, %llu candidate keys", (unsigned long long)nS, (unsigned long long)NC);
      if (NC) {
        DBuf<uint64_t> cand = c.buf<uint64_t>(NC * W);
        // reads with candidates, in read order
        DBuf<uint64_t> rpos = c.buf<uint64_t>(R.n_reads);
        k_nonzero<<<grid1(R.n_reads), SDBG_BLOCK, 0, c.s>>>(mcount.get(), R.n_reads, rpos.get());
        c.check_launch("mercy_reads");
        scan_excl<uint64_t, uint64_t>(rpos.get(), rpos.get(), R.n_reads, tot.get(), c);
        const uint64_t NR = c.d2h_one(tot.get());
        DBuf<uint64_t> rlist = c.buf<uint64_t>(NR);
        k_list_nonzero<<<grid1(R.n_reads), SDBG_BLOCK, 0, c.s>>>(mcount.get(), R.n_reads, rpos.get(), rlist.get());
        c.check_launch("mercy_reads");
        {
          Stage st_(c, "mercy_emit", NW + NR * 32 + NC * 8 * W);
          k_mercy<W><<<grid1(NR), SDBG_BLOCK, 0, c.s>>>(ea, wf.get(), 1, mcount.get(), mpos.get(), cand.get(), nt,
                                                        rlist.get(), NR);
          c.check_launch("mercy_emit");
        }
        wf.free();
        sort_unique(cand, NC, kb, M, &nM);
        VLOG("mercy: %llu distinct mercy edges", (unsigned long long)nM);
        Mc = c.buf<uint32_t>(nM);
        if (P.d <= 2) {
          fill<uint32_t>(Mc.get(), nM, 1u, c);
        } else {
          DBuf<uint64_t> ldir;
          SortedView lv = make_view(Lk.get(), nL, kb, ldir);
          k_lookup_counts<W><<<grid1(nM), SDBG_BLOCK, 0, c.s>>>(M.get(), nM, lv, Lc.get(), ea.canon, kb, Mc.get());
          c.check_launch("lookup_counts");
          c.sync();
        }
      }
    }
    // ---- E = S + M
    out->n_mercy = nM;
    out->n = nS + nM;
    if (nM == 0) {
      out->keys = S.release_ownership();
      out->count = Sc.release_ownership();
    } else {
      DBuf<uint64_t> E;
      DBuf<uint32_t> Ec;
      merge_sets("merge", S.get(), Sc.get(), nS, M.get(), Mc.get(), nM, E, Ec);
      out->keys = E.release_ownership();
      out->count = Ec.release_ownership();
    }
    c.sync();
  }

  // Several read sets in one pass, without mercy: R holds the sets' reads
  // back to back, set s owns reads [rb[s], rb[s+1]).  The first cut is
  // taken per set (tiles never straddle sets and the histogram table is
  // set-major), so every later segment lies inside one set, and the
  // refinement, leaf and compaction launches serve all sets at once.
  // Output: one edge set per read set, each equal to a single-set run.
  void run_sets(const DevReads& R, const std::vector<uint64_t>& rb, const CountParams& P, std::vector<EdgesOut>* outs) {
    const int k = P.k, kb = 2 * (k + 1);
    const uint64_t S = rb.size() - 1;
    outs->assign(S, EdgesOut{});
    Prep pr;
    prepare(R, k, pr);
    if (pr.NW == 0) return;
    ExArgs ea = pr.ea;
    // windows of each set
    DBuf<uint64_t> rbd = c.buf<uint64_t>(S + 1), swd = c.buf<uint64_t>(S + 1);
    c.h2d(rbd.get(), rb.data(), S + 1);
    k_gather_idx<<<grid1(S + 1), SDBG_BLOCK, 0, c.s>>>(pr.woff.get(), rbd.get(), S + 1, swd.get());
    c.check_launch("gather_idx");
    std::vector<uint64_t> sw(S + 1);
    c.d2h(sw.data(), swd.get(), S + 1);
    // tiles per set (at least one, so that every set has table columns)
    const uint64_t WPT = (uint64_t)SDBG_BLOCK * IPT;
    std::vector<uint64_t> st(S + 1);
    std::vector<uint32_t> tset;
    uint64_t NT = 0;
    for (uint64_t s = 0; s < S; ++s) {
      const uint64_t nt = std::max<uint64_t>(1, ceil_div(sw[s + 1] - sw[s], WPT));
      st[s] = NT;
      NT += nt;
      tset.insert(tset.end(), nt, (uint32_t)s);
    }
    st[S] = NT;
    SDBG_CHECK(NT < (1ull << 31), -3, "too many reads for one launch");
    DBuf<uint64_t> std_ = c.buf<uint64_t>(S + 1);
    DBuf<uint32_t> tsd = c.buf<uint32_t>(NT);
    c.h2d(std_.get(), st.data(), S + 1);
    c.h2d(tsd.get(), tset.data(), NT);
    ea.tset = tsd.get();
    ea.sw = swd.get();
    ea.st = std_.get();
    const uint32_t nbins = 1u << ea.dbits;
    DBuf<uint32_t> tab = c.buf<uint32_t>(NT * nbins);
    DBuf<uint64_t> tot = c.buf<uint64_t>(1);
    {
      Stage st_(c, "ex_hist", 3 * pr.words * 8 + NT * nbins * 4);
      k_ex_hist<W, IPT><<<(unsigned)NT, SDBG_BLOCK, 0, c.s>>>(ea, tab.get(), NT, nullptr);
      c.check_launch("ex_hist");
    }
    scan_excl<uint32_t, uint32_t>(tab.get(), tab.get(), NT * nbins, tot.get(), c);
    const uint64_t N = c.d2h_one(tot.get());
    SDBG_CHECK(N <= 0xFFFFFFFFull, -3, "read sets too large for one pass");
    DBuf<uint64_t> bufA = c.buf<uint64_t>(N * W), bufB = c.buf<uint64_t>(N * W);
    DBuf<uint32_t> cnt = c.buf<uint32_t>(N);
    DBuf<uint64_t*> db = c.buf<uint64_t*>(2);
    k_set_bufs<<<1, 64, 0, c.s>>>(db.get(), bufA.get(), bufB.get());
    c.check_launch("set_bufs");
    if (N) {
      Stage st_(c, "ex_scatter", 3 * pr.words * 8 + NT * nbins * 4 + N * 8 * W);
      k_ex_scatter<W, IPT><<<(unsigned)NT, SDBG_BLOCK, 0, c.s>>>(ea, tab.get(), NT, bufA.get());
      c.check_launch("ex_scatter");
    }
    SegList L;
    L.alloc(c, S * nbins);
    k_seg_init_sets<<<grid1(S * nbins), SDBG_BLOCK, 0, c.s>>>(tab.get(), std_.get(), S, ea.dbits, N, kb - ea.dbits,
                                                              L.view());
    c.check_launch("seg_init_sets");
    refine(L, db.get(), kb - ea.dbits);
    DBuf<uint64_t> Sk, Lk, spos;
    DBuf<uint32_t> Sc, Lc;
    uint64_t nS = 0, nL = 0;
    leaves(L, N, db.get(), cnt.get(), P.d, false, Sk, Sc, &nS, Lk, Lc, &nL, &spos);
    DBuf<uint64_t> kbase = c.buf<uint64_t>(S + 1), obase = c.buf<uint64_t>(S + 1);
    k_set_bounds<<<grid1(S + 1), SDBG_BLOCK, 0, c.s>>>(L.off.get(), L.n, spos.get(), tab.get(), std_.get(), ea.dbits,
                                                       S, N, kbase.get(), obase.get());
    c.check_launch("set_bounds");
    std::vector<uint64_t> hk(S + 1), ho(S + 1);
    c.d2h(hk.data(), kbase.get(), S + 1);
    c.d2h(ho.data(), obase.get(), S + 1);
    for (uint64_t s = 0; s < S; ++s) {
      EdgesOut& o = (*outs)[s];
      o.n_occ = hk[s + 1] - hk[s];
      o.n = ho[s + 1] - ho[s];
      DBuf<uint64_t> ok = c.buf<uint64_t>(o.n * W);
      DBuf<uint32_t> oc = c.buf<uint32_t>(o.n);
      c.d2d(ok.get(), Sk.get() + ho[s] * W, o.n * W);
      c.d2d(oc.get(), Sc.get() + ho[s], o.n);
      o.keys = ok.release_ownership();
      o.count = oc.release_ownership();
    }
    c.sync();
  }
};

}  // namespace

SortTune sort_tune() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tune;
}

void set_sort_tune(const SortTune& t) {
  SDBG_CHECK(t.digit_bits >= 4 && t.digit_bits <= 8, -1, "digit_bits must be in [4, 8]");
  SDBG_CHECK(t.tile_shift == 0 || t.tile_shift == 1, -1, "tile_shift must be 0 or 1");
  SDBG_CHECK(t.leaf_wg_per_cu >= 1 && t.leaf_wg_per_cu <= 32, -1, "leaf_wg_per_cu must be in [1, 32]");
  SDBG_CHECK(t.leaf_cap_shift == 0 || t.leaf_cap_shift == 1, -1, "leaf_cap_shift must be 0 or 1");
  SDBG_CHECK(t.first_bits >= 4 && t.first_bits <= 8, -1, "first_bits must be in [4, 8]");
  SDBG_CHECK(t.mercy_shift >= 0 && t.mercy_shift <= 8, -1, "mercy_shift must be in [0, 8]");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune = t;
}

void count_solid_sets(const DevReads& r, const std::vector<uint64_t>& rb, const CountParams& p, Ctx& c,
                      std::vector<EdgesOut>* outs) {
  switch (key_words(p.k)) {
    case 1: Counter<1>(c).run_sets(r, rb, p, outs); break;
    case 2: Counter<2>(c).run_sets(r, rb, p, outs); break;
    case 3: Counter<3>(c).run_sets(r, rb, p, outs); break;
    case 4: Counter<4>(c).run_sets(r, rb, p, outs); break;
    default: throw Error(-1, "k out of range");
  }
}

template <int W>
void edges_union_w(const uint64_t* A, const uint32_t* Ac, uint64_t nA, const uint64_t* B, const uint32_t* Bc,
                   uint64_t nB, Ctx& c, EdgesOut* out) {
  const uint64_t n = nA + nB;
  if (n == 0) {
    DBuf<uint64_t> O = c.buf<uint64_t>(W);
    DBuf<uint32_t> Oc = c.buf<uint32_t>(1);
    out->keys = O.release_ownership();
    out->count = Oc.release_ownership();
    out->n = 0;
    return;
  }
  Counter<W> ct(c);
  DBuf<uint64_t> E;
  DBuf<uint32_t> Ec;
  ct.merge_sets("union_merge", A, Ac, nA, B, Bc, nB, E, Ec);
  DBuf<uint32_t> head = c.buf<uint32_t>(n);
  DBuf<uint64_t> pos = c.buf<uint64_t>(n + 1);
  DBuf<uint32_t> ovf = c.buf<uint32_t>(1);
  fill<uint32_t>(ovf.get(), 1, 0u, c);
  {
    k_union_heads<W><<<(unsigned)ceil_div(n, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(E.get(), n, head.get());
    c.check_launch("union heads");
  }
  scan_excl<uint32_t, uint64_t>(head.get(), pos.get(), n, pos.get() + n, c);
  const uint64_t nu = c.d2h_one(pos.get() + n);
  DBuf<uint64_t> O = c.buf<uint64_t>((nu ? nu : 1) * W);
  DBuf<uint32_t> Oc = c.buf<uint32_t>(nu ? nu : 1);
  {
    k_union_scatter<W><<<(unsigned)ceil_div(n, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(E.get(), Ec.get(), n, pos.get(),
                                                                                O.get(), Oc.get(), ovf.get());
    c.check_launch("union scatter");
  }
  SDBG_CHECK(c.d2h_one(ovf.get()) == 0, -1, "a summed count does not fit 32 bits");
  out->keys = O.release_ownership();
  out->count = Oc.release_ownership();
  out->n = nu;
}

void edges_union(const uint64_t* A, const uint32_t* Ac, uint64_t nA, const uint64_t* B, const uint32_t* Bc,
                 uint64_t nB, int k, Ctx& c, EdgesOut* out) {
  switch (key_words(k)) {
    case 1: edges_union_w<1>(A, Ac, nA, B, Bc, nB, c, out); break;
    case 2: edges_union_w<2>(A, Ac, nA, B, Bc, nB, c, out); break;
    case 3: edges_union_w<3>(A, Ac, nA, B, Bc, nB, c, out); break;
    case 4: edges_union_w<4>(A, Ac, nA, B, Bc, nB, c, out); break;
    default: throw Error(-1, "k out of range");
  }
}

void count_solid(const DevReads& r, const CountParams& p, Ctx& c, EdgesOut* out) {
  switch (key_words(p.k)) {
    case 1: Counter<1>(c).run(r, p, out); break;
    case 2: Counter<2>(c).run(r, p, out); break;
    case 3: Counter<3>(c).run(r, p, out); break;
    case 4: Counter<4>(c).run(r, p, out); break;
    default: throw Error(-1, "k out of range");
  }
}

}  // namespace sdbg
