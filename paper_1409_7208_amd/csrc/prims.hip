// Generic device-wide primitives: fills and exclusive scans.
#include "prims.h"

namespace sdbg {

template <typename T>
__global__ void k_fill(T* p, uint64_t n, T v) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <typename T>
void fill(T* p, uint64_t n, T v, Ctx& c) {
  if (!n) return;
  uint64_t blocks = ceil_div(n, SDBG_BLOCK);
  if (blocks > 65536) blocks = 65536;
  k_fill<T><<<(unsigned)blocks, SDBG_BLOCK, 0, c.s>>>(p, n, v);
  c.check_launch("fill");
}
template void fill<uint64_t>(uint64_t*, uint64_t, uint64_t, Ctx&);
template void fill<uint32_t>(uint32_t*, uint64_t, uint32_t, Ctx&);
template void fill<uint8_t>(uint8_t*, uint64_t, uint8_t, Ctx&);

// Exclusive scan, reduce-then-scan.  Each workgroup covers SCAN_TILE
// consecutive elements staged through LDS so that global accesses are
// coalesced; the per-tile sums are scanned recursively.
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SDBG_BLOCK * SCAN_IPT;

template <typename Tin>
__global__ __launch_bounds__(SDBG_BLOCK) void k_scan_reduce(const Tin* __restrict__ in, uint64_t n, uint64_t* __restrict__ sums) {
  __shared__ uint64_t red[SDBG_WAVES];
  uint64_t base = blockIdx.x * (uint64_t)SCAN_TILE;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    uint64_t idx = base + i * SDBG_BLOCK + threadIdx.x;
    if (idx < n) s += (uint64_t)in[idx];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int i = 0; i < SDBG_WAVES; ++i) t += red[i];
    sums[blockIdx.x] = t;
  }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(SDBG_BLOCK) void k_scan_down(const Tin* in, Tout* out, uint64_t n, const uint64_t* __restrict__ tile_off,
                                                         uint64_t* total) {
  __shared__ uint64_t v[SCAN_TILE];
  __shared__ uint64_t sc[SDBG_WAVES + 1];
  uint64_t base = blockIdx.x * (uint64_t)SCAN_TILE;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    uint64_t idx = base + i * SDBG_BLOCK + threadIdx.x;
    v[i * SDBG_BLOCK + threadIdx.x] = idx < n ? (uint64_t)in[idx] : 0;
  }
  __syncthreads();
  uint64_t loc[SCAN_IPT];
  uint64_t run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    loc[i] = run;
    run += v[threadIdx.x * SCAN_IPT + i];
  }
  uint64_t tot;
  uint64_t ex = block_excl_scan<uint64_t>(run, sc, &tot);
  uint64_t off = (tile_off ? tile_off[blockIdx.x] : 0) + ex;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) v[threadIdx.x * SCAN_IPT + i] = off + loc[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    uint64_t idx = base + i * SDBG_BLOCK + threadIdx.x;
    if (idx < n) out[idx] = (Tout)v[i * SDBG_BLOCK + threadIdx.x];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SDBG_BLOCK - 1) {
    uint64_t last = base + SCAN_TILE - 1;
    (void)last;
    *total = (tile_off ? tile_off[blockIdx.x] : 0) + tot;
  }
}

template <typename Tin, typename Tout>
void scan_excl(const Tin* in, Tout* out, uint64_t n, uint64_t* d_total, Ctx& c) {
  if (n == 0) {
    if (d_total) fill<uint64_t>(d_total, 1, 0, c);
    return;
  }
  uint64_t tiles = ceil_div(n, SCAN_TILE);
  SDBG_CHECK(tiles < (1ull << 31), -1, "scan too large");
  if (tiles == 1) {
    k_scan_down<Tin, Tout><<<1, SDBG_BLOCK, 0, c.s>>>(in, out, n, nullptr, d_total);
    c.check_launch("scan_down");
    return;
  }
  DBuf<uint64_t> sums = c.buf<uint64_t>(tiles);
  k_scan_reduce<Tin><<<(unsigned)tiles, SDBG_BLOCK, 0, c.s>>>(in, n, sums.get());
  c.check_launch("scan_reduce");
  scan_excl<uint64_t, uint64_t>(sums.get(), sums.get(), tiles, nullptr, c);
  k_scan_down<Tin, Tout><<<(unsigned)tiles, SDBG_BLOCK, 0, c.s>>>(in, out, n, sums.get(), d_total);
  c.check_launch("scan_down");
}

__global__ void k_decreasing(const uint64_t* __restrict__ off, uint64_t n, uint32_t* __restrict__ flag) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (uint64_t j = i; j < n; j += stride) bad |= off[j + 1] < off[j];
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

bool nondecreasing(const uint64_t* off, uint64_t n, Ctx& c) {
  if (n == 0) return true;
  DBuf<uint32_t> flag = c.buf<uint32_t>(1);
  fill<uint32_t>(flag.get(), 1, 0u, c);
  uint64_t blocks = ceil_div(n, SDBG_BLOCK);
  if (blocks > 65536) blocks = 65536;
  k_decreasing<<<(unsigned)blocks, SDBG_BLOCK, 0, c.s>>>(off, n, flag.get());
  c.check_launch("offsets check");
  return c.d2h_one(flag.get()) == 0;
}

__global__ void k_off_summary(const uint64_t* __restrict__ off, uint64_t n, uint32_t k,
                              unsigned long long* __restrict__ st) {
  __shared__ unsigned long long part[2];
  if (threadIdx.x < 2) part[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long bad = 0, occ = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t a = off[i], b = off[i + 1];
    if (b < a) {
      bad = 1;
    } else if (b - a > k) {
      occ += 2 * (b - a - k);
    }
  }
  if (bad) atomicOr(&part[0], 1ull);
  if (occ) atomicAdd(&part[1], occ);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (part[0] || (blockIdx.x == 0 && off[0] != 0)) atomicOr(&st[0], 1ull);
    if (part[1]) atomicAdd(&st[1], part[1]);
    if (blockIdx.x == 0) st[2] = off[n];
  }
}

void offsets_summary(const uint64_t* off, uint64_t n, uint32_t k, unsigned long long* st, Ctx& c) {
  uint64_t blocks = ceil_div(n, SDBG_BLOCK);
  if (blocks > 1024) blocks = 1024;
  if (blocks == 0) blocks = 1;
  k_off_summary<<<(unsigned)blocks, SDBG_BLOCK, 0, c.s>>>(off, n, k, st);
  c.check_launch("offsets summary");
}

__global__ void k_off_rebase(const uint64_t* __restrict__ off, uint64_t n, uint64_t base, uint64_t* __restrict__ out) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = off[i] + base;
}

void offsets_rebase(const uint64_t* off, uint64_t n, uint64_t base, uint64_t* out, Ctx& c) {
  if (!n) return;
  k_off_rebase<<<(unsigned)ceil_div(n, SDBG_BLOCK), SDBG_BLOCK, 0, c.s>>>(off, n, base, out);
  c.check_launch("offsets rebase");
}

template void scan_excl<uint64_t, uint64_t>(const uint64_t*, uint64_t*, uint64_t, uint64_t*, Ctx&);
template void scan_excl<uint32_t, uint32_t>(const uint32_t*, uint32_t*, uint64_t, uint64_t*, Ctx&);
template void scan_excl<uint32_t, uint64_t>(const uint32_t*, uint64_t*, uint64_t, uint64_t*, Ctx&);

}  // namespace sdbg
