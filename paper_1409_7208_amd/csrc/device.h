// Device-side primitives for gfx950 (wave64): multiword keys, bit helpers,
// wave and workgroup scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SDBG_BLOCK 256
#define SDBG_WAVES (SDBG_BLOCK / 64)

// Host-callable as well, so that the key arithmetic can be checked on the CPU.
#define DEV __host__ __device__ __forceinline__

// A key of W 64-bit words; w[0] is the most significant word, the same
// order as in memory.  Indices into w[] are always compile-time constants
// (loops are unrolled and select with comparisons), so keys stay in VGPRs.
template <int W>
struct Key {
  uint64_t w[W];
};

template <int W>
DEV Key<W> key_load(const uint64_t* p) {
  Key<W> k;
#pragma unroll
  for (int i = 0; i < W; ++i) k.w[i] = p[i];
  return k;
}

template <int W>
DEV void key_store(uint64_t* p, const Key<W>& k) {
#pragma unroll
  for (int i = 0; i < W; ++i) p[i] = k.w[i];
}

// Key access through a pointer the compiler cannot place in global memory
// (one read from a table of buffers): as generic pointers these become flat
// accesses, which also count against the LDS wait counter, so a wait for LDS
// (a barrier) would wait for them too.  These access global memory.
typedef __attribute__((address_space(1))) uint64_t global_u64;

template <int W>
__device__ __forceinline__ Key<W> key_load_g(const uint64_t* p) {
  const global_u64* q = (const global_u64*)p;
  Key<W> k;
#pragma unroll
  for (int i = 0; i < W; ++i) k.w[i] = q[i];
  return k;
}

template <int W>
__device__ __forceinline__ void key_store_g(uint64_t* p, const Key<W>& k) {
  global_u64* q = (global_u64*)p;
#pragma unroll
  for (int i = 0; i < W; ++i) q[i] = k.w[i];
}

template <int W>
DEV bool key_less(const Key<W>& a, const Key<W>& b) {
#pragma unroll
  for (int i = 0; i < W; ++i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i];
  return false;
}

template <int W>
DEV bool key_eq(const Key<W>& a, const Key<W>& b) {
  bool e = true;
#pragma unroll
  for (int i = 0; i < W; ++i) e = e && (a.w[i] == b.w[i]);
  return e;
}

template <int W>
DEV Key<W> key_zero() {
  Key<W> k;
#pragma unroll
  for (int i = 0; i < W; ++i) k.w[i] = 0;
  return k;
}

// Limb j counted from the least significant end.
template <int W>
DEV uint64_t limb(const Key<W>& k, int j) {
  uint64_t v = 0;
#pragma unroll
  for (int t = 0; t < W; ++t)
    if (t == j) v = k.w[W - 1 - t];
  return v;
}

// n <= 32 bits starting at bit lo (bit 0 = least significant bit of the key).
template <int W>
DEV uint32_t key_bits(const Key<W>& k, int lo, int n) {
  int li = lo >> 6, s = lo & 63;
  uint64_t v = limb<W>(k, li) >> s;
  if (s + n > 64) v |= limb<W>(k, li + 1) << (64 - s);
  return (uint32_t)(v & ((n >= 64) ? ~0ull : ((1ull << n) - 1)));
}

template <int W>
DEV Key<W> key_shr(const Key<W>& a, int s) {
  Key<W> r;
  int q = s >> 6, b = s & 63;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    uint64_t lo = limb<W>(a, j + q), hi = limb<W>(a, j + q + 1);
    r.w[W - 1 - j] = b ? ((lo >> b) | (hi << (64 - b))) : lo;
  }
  return r;
}

template <int W>
DEV Key<W> key_shl(const Key<W>& a, int s) {
  Key<W> r;
  int q = s >> 6, b = s & 63;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    uint64_t hi = limb<W>(a, j - q), lo = limb<W>(a, j - q - 1);
    r.w[W - 1 - j] = b ? ((hi << b) | (lo >> (64 - b))) : hi;
  }
  return r;
}

// Keep the low n bits (0 <= n <= 64W).
template <int W>
DEV Key<W> key_lowbits(const Key<W>& a, int n) {
  Key<W> r;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    int keep = n - 64 * j;
    uint64_t m = keep >= 64 ? ~0ull : (keep <= 0 ? 0ull : ((1ull << keep) - 1));
    r.w[W - 1 - j] = a.w[W - 1 - j] & m;
  }
  return r;
}

template <int W>
DEV Key<W> key_or_low(const Key<W>& a, uint64_t v) {
  Key<W> r = a;
  r.w[W - 1] |= v;
  return r;
}

template <int W>
DEV Key<W> key_xor_mask(const Key<W>& a, int n) {  // complement the low n bits
  Key<W> r;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    int keep = n - 64 * j;
    uint64_t m = keep >= 64 ? ~0ull : (keep <= 0 ? 0ull : ((1ull << keep) - 1));
    r.w[W - 1 - j] = a.w[W - 1 - j] ^ m;
  }
  return r;
}

// Reverse the order of the 32 two-bit groups of a word.
DEV uint64_t rev2_64(uint64_t x) {
  x = ((x >> 2) & 0x3333333333333333ull) | ((x & 0x3333333333333333ull) << 2);
  x = ((x >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((x & 0x0F0F0F0F0F0F0F0Full) << 4);
  return __builtin_bswap64(x);
}

// nbits-bit little-endian value at bit position pos of a packed 2-bit
// stream (base j at bits 2(j mod 32) of word j/32).  Reads W+1 words from
// word pos/64 on; the stream carries zero padding for that.
template <int W>
DEV Key<W> stream_bits(const uint64_t* __restrict__ pw, uint64_t pos, int nbits) {
  uint64_t q = pos >> 6;
  int s = (int)(pos & 63);
  Key<W> r;
  uint64_t cur = pw[q];
#pragma unroll
  for (int j = 0; j < W; ++j) {
    uint64_t nxt = pw[q + j + 1];
    r.w[W - 1 - j] = s ? ((cur >> s) | (nxt << (64 - s))) : cur;
    cur = nxt;
  }
  return key_lowbits<W>(r, nbits);
}

// Edge key from the forward packing F of a (k+1)-mer (F = sum e[i] 4^i,
// kb = 2(k+1) bits): the base-4 digits e[k-1], ..., e[0], e[k], which is F
// rotated left by one base within kb bits.
template <int W>
DEV Key<W> key_from_fwd(const Key<W>& F, int kb) {
  uint64_t top = key_bits<W>(F, kb - 2, 2);
  Key<W> r = key_lowbits<W>(key_shl<W>(F, 2), kb);
  return key_or_low<W>(r, top);
}

// Forward packing of the reverse complement of the (k+1)-mer packed in F.
template <int W>
DEV Key<W> revcomp_fwd(const Key<W>& F, int kb) {
  Key<W> r;
#pragma unroll
  for (int i = 0; i < W; ++i) r.w[i] = rev2_64(F.w[W - 1 - i]);
  r = key_shr<W>(r, 64 * W - kb);
  return key_xor_mask<W>(r, kb);
}

// ---------------------------------------------------------------- scans
template <typename T>
DEV T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

template <typename T>
DEV T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup barrier for communication through LDS only: waits for this
// wave's LDS operations but not for its global loads and stores (the fence
// of __syncthreads would), so global traffic in flight keeps overlapping
// with the work after the barrier.  The memory clobber keeps the compiler
// from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Exclusive scan over the SDBG_BLOCK threads of a workgroup; *total gets the
// sum.  `scratch` holds SDBG_WAVES elements of LDS; the scan ends with a
// barrier, so the caller may reuse scratch at once.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* scratch, T* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) scratch[wid] = inc;
  lds_barrier();
  T base = 0, all = 0;
#pragma unroll
  for (int i = 0; i < SDBG_WAVES; ++i) {
    const T t = scratch[i];
    base += i < wid ? t : T(0);
    all += t;
  }
  *total = all;
  lds_barrier();  // scratch may be reused at once
  return base + inc - v;
}

// 2-bit code of an ASCII base; *ok = false for anything but A/C/G/T (any case).
DEV uint32_t base_code(uint32_t c, bool* ok) {
  uint32_t u = c & 0xDFu;  // upper-case letters
  *ok = (u == 'A') | (u == 'C') | (u == 'G') | (u == 'T');
  uint32_t x = (c >> 1) & 3u;  // A:0 C:1 G:3 T:2
  return x ^ (x >> 1);          // A:0 C:1 G:2 T:3
}
