// The Burrows-Wheeler transform of a read set: every suffix of every read
// sorted (Section 2, second paragraph: the construction adapts CX1, whose
// core is this sort; the paper gives no details, so the multi-string BWT is
// the reading implemented).  Read r is followed by its own end marker $_r,
// smaller than every base, with $_r < $_s for r < s; the text of the read
// set is read 0, $_0, read 1, $_1, ..., so read r's suffix at offset j
// (0 <= j <= len) is text position offsets[r] + r + j.
//
// The sort is prefix doubling on the device: the suffixes are first sorted
// by their first 21 characters (3 bits each, $ = 0 and everything after it
// 0) into groups of equal prefixes, each named by the place of its first
// suffix in the order.  Each further round re-sorts only the suffixes of
// groups that still hold more than one, by (group of the first h
// characters, group of the next h) -- or, for a suffix whose end marker
// lies within its first h characters, (group, read index), which orders
// equal suffixes of different reads -- and splits their groups in place,
// until every group holds one suffix.  Each round sorts (key, position)
// pairs with a stable least-significant-digit radix sort (8-bit digits; per
// 2048-element tile, a digit histogram, then a scatter that ranks equal
// digits within each wave by ballots).
#include <hip/hip_runtime.h>

#include <vector>

#include "abi_common.h"
#include "prims.h"

namespace sdbg {
namespace {

constexpr int RADIX_TILE = 2048;  // elements per tile: 8 per thread
constexpr int FIRST_CHARS = 21;   // characters of the first ranking (3 bits each)

// err |= 1 for a byte that is not a base (either case).
__global__ void k_bwt_check(const uint8_t* __restrict__ seq, uint64_t n, uint32_t* __restrict__ err) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  bool bad = false;
  if (i < n) {
    const uint8_t b = seq[i] & 0xDF;  // upper case
    bad = !(b == 'A' || b == 'C' || b == 'G' || b == 'T');
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(err, 1u);
}

DEV uint64_t base_code(uint8_t b) {  // A, C, G, T -> 1..4 ($ is 0)
  b &= 0xDF;
  return b == 'A' ? 1 : b == 'C' ? 2 : b == 'G' ? 3 : 4;
}

// rid[p] = read of text position p (one thread per read).
__global__ void k_bwt_rid(const uint64_t* __restrict__ off, uint64_t n_reads, uint32_t* __restrict__ rid) {
  const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  const uint64_t s = off[r] + r, e = off[r + 1] + r;  // bases [s, e), $ at e
  for (uint64_t p = s; p <= e; ++p) rid[p] = (uint32_t)r;
}

// First ranking key: the suffix's first 21 characters, 3 bits each.
__global__ void k_bwt_first_keys(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ off,
                                 const uint32_t* __restrict__ rid, uint64_t N, uint64_t* __restrict__ key,
                                 uint64_t* __restrict__ val) {
  const uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (p >= N) return;
  const uint64_t r = rid[p];
  const uint64_t j = p - (off[r] + r), len = off[r + 1] - off[r];
  uint64_t k = 0;
  for (int t = 0; t < FIRST_CHARS; ++t) {
    const uint64_t c = j + t < len ? base_code(seq[off[r] + j + t]) : 0;
    k = (k << 3) | c;
  }
  key[p] = k;
  val[p] = p;
}

// Doubling key of unresolved suffix i (text position u[i]) from the group
// starts of the first h characters: (group, group of the next h) or, when
// its end marker lies within the first h, (group, read index).
__global__ void k_bwt_pair_keys(const uint64_t* __restrict__ u, uint64_t m, const uint64_t* __restrict__ off,
                                const uint32_t* __restrict__ rid, const uint64_t* __restrict__ grp, uint64_t N,
                                uint64_t n_reads, uint64_t h, uint64_t* __restrict__ key, uint64_t* __restrict__ val) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t p = u[i], r = rid[p];
  const uint64_t end = off[r + 1] + r;  // position of $_r
  const uint64_t second = end - p + 1 <= h ? r : n_reads + grp[p + h];
  key[i] = grp[p] * (N + n_reads) + second;
  val[i] = p;
}

// Digit counts of each tile, digit-major: hist[d * ntiles + tile].
__global__ void k_radix_hist(const uint64_t* __restrict__ key, uint64_t n, int shift, uint64_t ntiles,
                             uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t t0 = blockIdx.x * (uint64_t)RADIX_TILE;
  for (int q = 0; q < RADIX_TILE / SDBG_BLOCK; ++q) {
    const uint64_t i = t0 + (uint64_t)q * SDBG_BLOCK + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(key[i] >> shift) & 255], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one digit: an element's place is its digit's offset for
// the tile, plus the elements of the tile before it with the same digit
// (earlier sub-tiles, earlier waves, then earlier lanes found by ballots).
__global__ void k_radix_scatter(const uint64_t* __restrict__ key, const uint64_t* __restrict__ val, uint64_t n,
                                int shift, uint64_t ntiles, const uint32_t* __restrict__ hoff,
                                uint64_t* __restrict__ okey, uint64_t* __restrict__ oval) {
  __shared__ uint32_t cum[256];
  __shared__ uint32_t wc[SDBG_WAVES][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  cum[threadIdx.x] = hoff[(uint64_t)threadIdx.x * ntiles + blockIdx.x];
  for (int q = 0; q < SDBG_WAVES; ++q) wc[q][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t t0 = blockIdx.x * (uint64_t)RADIX_TILE;
  for (int q = 0; q < RADIX_TILE / SDBG_BLOCK; ++q) {
    const uint64_t i = t0 + (uint64_t)q * SDBG_BLOCK + threadIdx.x;
    const bool ok = i < n;
    const uint64_t k = ok ? key[i] : 0;
    const uint32_t d = (uint32_t)(k >> shift) & 255;
    uint64_t m = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot(ok && ((d >> b) & 1));
      m &= ((d >> b) & 1) ? bal : ~bal;
    }
    const uint32_t before = (uint32_t)__popcll(m & ((1ull << lane) - 1));
    if (ok && before == 0) wc[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (ok) {
      uint32_t at = cum[d] + before;
      for (int x = 0; x < w; ++x) at += wc[x][d];
      okey[at] = k;
      oval[at] = val[i];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int x = 0; x < SDBG_WAVES; ++x) {
      add += wc[x][threadIdx.x];
      wc[x][threadIdx.x] = 0;
    }
    cum[threadIdx.x] += add;
    __syncthreads();
  }
}

// head[i] = 1 where the sorted key changes (a new rank starts).
__global__ void k_bwt_heads(const uint64_t* __restrict__ key, uint64_t n, uint32_t* __restrict__ head) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) head[i] = i == 0 || key[i] != key[i - 1] ? 1u : 0u;
}

// hidx[g] = index of the g-th head (g = heads before it); hidx[total] = m.
__global__ void k_bwt_head_index(const uint32_t* __restrict__ head, const uint64_t* __restrict__ excl, uint64_t m,
                                 uint64_t* __restrict__ hidx) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  if (head[i]) hidx[excl[i]] = i;
  if (i == 0) hidx[excl[m]] = m;
}

// Sorted element i of the suffixes being refined (text position val[i];
// upos[i] = its place in the suffix order, i itself in the first round):
// its group starts at the place of its group's first element; it takes its
// place in sa; flag = its group still holds more than one suffix.
__global__ void k_bwt_refine(const uint64_t* __restrict__ val, const uint32_t* __restrict__ head,
                             const uint64_t* __restrict__ excl, const uint64_t* __restrict__ hidx,
                             const uint64_t* __restrict__ upos, uint64_t m, uint64_t* __restrict__ grp,
                             uint64_t* __restrict__ sa, uint32_t* __restrict__ flag) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t g = excl[i] + head[i] - 1;
  const uint64_t a = hidx[g], b = hidx[g + 1];
  const uint64_t p = val[i];
  grp[p] = upos ? upos[a] : a;
  sa[upos ? upos[i] : i] = p;
  flag[i] = b - a > 1 ? 1u : 0u;
}

// The suffixes of groups still shared, in order: positions and places.
__global__ void k_bwt_compact(const uint64_t* __restrict__ val, const uint64_t* __restrict__ upos,
                              const uint32_t* __restrict__ flag, const uint64_t* __restrict__ fpos, uint64_t m,
                              uint64_t* __restrict__ u_out, uint64_t* __restrict__ upos_out) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= m || !flag[i]) return;
  u_out[fpos[i]] = val[i];
  upos_out[fpos[i]] = upos ? upos[i] : i;
}

// BWT character of sorted suffix i: the character before it in its read, or
// '$' for a suffix that starts its read.
__global__ void k_bwt_chars(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ off,
                            const uint32_t* __restrict__ rid, const uint64_t* __restrict__ sa, uint64_t N,
                            uint8_t* __restrict__ out) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint64_t p = sa[i], r = rid[p];
  const uint64_t j = p - (off[r] + r);
  out[i] = j == 0 ? (uint8_t)'$' : (uint8_t)(seq[off[r] + j - 1] & 0xDF);
}

unsigned grid_of(uint64_t n) { return (unsigned)ceil_div(n ? n : 1, SDBG_BLOCK); }

// Sorts (key, val) pairs by the low `bits` bits of the keys (stable); the
// result is in k0/v0 (k1/v1 are the other buffers).
void radix_sort_pairs(uint64_t*& k0, uint64_t*& v0, uint64_t*& k1, uint64_t*& v1, uint64_t n, int bits, Ctx& c) {
  if (n == 0) return;
  const uint64_t ntiles = ceil_div(n, RADIX_TILE);
  SDBG_CHECK(ntiles < (1ull << 31) && 256 * ntiles < (1ull << 32), SDBG_E_INVAL, "too many suffixes");
  DBuf<uint32_t> hist = c.buf<uint32_t>(256 * ntiles);
  for (int shift = 0; shift < bits; shift += 8) {
    k_radix_hist<<<(unsigned)ntiles, SDBG_BLOCK, 0, c.s>>>(k0, n, shift, ntiles, hist.get());
    c.check_launch("radix hist");
    scan_excl<uint32_t, uint32_t>(hist.get(), hist.get(), 256 * ntiles, nullptr, c);
    k_radix_scatter<<<(unsigned)ntiles, SDBG_BLOCK, 0, c.s>>>(k0, v0, n, shift, ntiles, hist.get(), k1, v1);
    c.check_launch("radix scatter");
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
}

int bits_of(uint64_t x) {
  int b = 0;
  while (b < 64 && (x >> b)) ++b;
  return b;
}

}  // namespace
}  // namespace sdbg

namespace sdbg_abi {
void free_bwt(void* p) {
  auto* b = static_cast<sdbg_bwt*>(p);
  pool_free(b->bwt);
  pool_free(b->sa);
  delete b;
}
}  // namespace sdbg_abi

extern "C" {

int sdbg_read_bwt(const sdbg_reads* reads, const sdbg_params* params, sdbg_bwt** out) {
  using namespace sdbg;
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(reads && out, SDBG_E_INVAL, "null argument");
    *out = nullptr;
    Ctx c(params ? params->stream : nullptr);
    const std::vector<uint64_t> o = sdbg_abi::host_offsets(c, reads);
    const uint64_t n_reads = reads->n_reads, n_bases = o[n_reads];
    const uint64_t N = n_bases + n_reads;  // suffixes (each read: its bases and its end marker)
    // ranks and keys: N + n_reads < 2^32 keeps rank * (N + n_reads) + second below 2^64
    SDBG_CHECK(N + n_reads < (1ull << 32), SDBG_E_INVAL, "read set too large for 32-bit ranks");
    DBuf<uint8_t> seq_d;
    DBuf<uint64_t> off_d;
    const uint8_t* seq = reads->seq;
    const uint64_t* off = reads->offsets;
    if (!reads->on_device || n_reads == 0) {
      seq_d = c.buf<uint8_t>(n_bases ? n_bases : 1);
      off_d = c.buf<uint64_t>(n_reads + 1);
      if (n_bases) c.h2d(seq_d.get(), reads->seq, n_bases);
      c.h2d(off_d.get(), o.data(), n_reads + 1);
      seq = seq_d.get();
      off = off_d.get();
    }
    if (n_bases) {
      DBuf<uint32_t> err = c.buf<uint32_t>(1);
      fill<uint32_t>(err.get(), 1, 0u, c);
      k_bwt_check<<<grid_of(n_bases), SDBG_BLOCK, 0, c.s>>>(seq, n_bases, err.get());
      c.check_launch("bwt check");
      SDBG_CHECK(c.d2h_one(err.get()) == 0, SDBG_E_INVAL, "reads must hold only A, C, G, T");
    }
    DBuf<uint64_t> sa = c.buf<uint64_t>(N ? N : 1);
    DBuf<uint8_t> chars = c.buf<uint8_t>(N ? N : 1);
    if (N) {
      DBuf<uint32_t> rid = c.buf<uint32_t>(N);
      k_bwt_rid<<<grid_of(n_reads), SDBG_BLOCK, 0, c.s>>>(off, n_reads, rid.get());
      c.check_launch("bwt read of position");
      // keys and positions of the suffixes being sorted (two buffers each),
      // group start of every suffix, and the refinement's working arrays
      DBuf<uint64_t> ka = c.buf<uint64_t>(N), kb = c.buf<uint64_t>(N), va = c.buf<uint64_t>(N),
                     vb = c.buf<uint64_t>(N), grp = c.buf<uint64_t>(N), ulist = c.buf<uint64_t>(N),
                     upa = c.buf<uint64_t>(N), upb = c.buf<uint64_t>(N), excl = c.buf<uint64_t>(N + 1),
                     hidx = c.buf<uint64_t>(N + 1), fpos = c.buf<uint64_t>(N + 1);
      DBuf<uint32_t> head = c.buf<uint32_t>(N), flag = c.buf<uint32_t>(N);
      uint64_t *k0 = ka.get(), *k1 = kb.get(), *v0 = va.get(), *v1 = vb.get();
      uint64_t *up = nullptr, *up_next = upa.get(), *up_spare = upb.get();
      k_bwt_first_keys<<<grid_of(N), SDBG_BLOCK, 0, c.s>>>(seq, off, rid.get(), N, k0, v0);
      c.check_launch("bwt first keys");
      int bits = 3 * FIRST_CHARS;
      uint64_t h = FIRST_CHARS, m = N;  // m suffixes still to order (all, in the first round)
      for (int round = 0;; ++round) {
        SDBG_CHECK(round < 40, SDBG_E_HIP, "suffix ranking did not converge");
        radix_sort_pairs(k0, v0, k1, v1, m, bits, c);
        const unsigned g = grid_of(m);
        k_bwt_heads<<<g, SDBG_BLOCK, 0, c.s>>>(k0, m, head.get());
        c.check_launch("bwt heads");
        scan_excl<uint32_t, uint64_t>(head.get(), excl.get(), m, excl.get() + m, c);
        k_bwt_head_index<<<g, SDBG_BLOCK, 0, c.s>>>(head.get(), excl.get(), m, hidx.get());
        c.check_launch("bwt head index");
        k_bwt_refine<<<g, SDBG_BLOCK, 0, c.s>>>(v0, head.get(), excl.get(), hidx.get(), up, m, grp.get(), sa.get(),
                                                flag.get());
        c.check_launch("bwt refine");
        scan_excl<uint32_t, uint64_t>(flag.get(), fpos.get(), m, fpos.get() + m, c);
        const uint64_t nm = c.d2h_one(fpos.get() + m);
        if (nm == 0) break;  // every suffix has its own place
        k_bwt_compact<<<g, SDBG_BLOCK, 0, c.s>>>(v0, up, flag.get(), fpos.get(), m, ulist.get(), up_next);
        c.check_launch("bwt compact");
        k_bwt_pair_keys<<<grid_of(nm), SDBG_BLOCK, 0, c.s>>>(ulist.get(), nm, off, rid.get(), grp.get(), N, n_reads,
                                                            h, k0, v0);
        c.check_launch("bwt pair keys");
        if (!up) {
          up = up_next;
          up_next = up_spare;
        } else {
          std::swap(up, up_next);
        }
        m = nm;
        bits = bits_of((N - 1) * (N + n_reads) + (N + n_reads - 1));
        h *= 2;
      }
      k_bwt_chars<<<grid_of(N), SDBG_BLOCK, 0, c.s>>>(seq, off, rid.get(), sa.get(), N, chars.get());
      c.check_launch("bwt chars");
    }
    c.sync();
    auto* b = new sdbg_bwt();
    b->n = N;
    b->n_reads = n_reads;
    b->bwt = chars.release_ownership();
    b->sa = sa.release_ownership();
    sdbg_abi::reg_add(b, sdbg_abi::kBwt);
    *out = b;
    return SDBG_OK;
  });
}

int sdbg_bwt_to_host(const sdbg_bwt* b, uint8_t* bwt, uint64_t* sa) {
  using namespace sdbg;
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(b && sdbg_abi::reg_kind(b) == sdbg_abi::kBwt, SDBG_E_INVAL, "not a BWT returned by this library");
    Ctx c(nullptr);
    if (bwt) c.d2h(bwt, b->bwt, b->n);
    if (sa) c.d2h(sa, b->sa, b->n);
    return SDBG_OK;
  });
}

}  // extern "C"
