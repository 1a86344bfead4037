// Device-wide helpers callable from host code.
#pragma once

#include "device.h"
#include "runtime.h"

namespace sdbg {

// p[0..n) = v, with a kernel (no memset nodes, so the call is safe inside
// captured graphs).
template <typename T>
void fill(T* p, uint64_t n, T v, Ctx& c);

// out[i] = sum of in[0..i) (in-place allowed).  If d_total is non-null,
// *d_total = sum of all n elements.
template <typename Tin, typename Tout>
void scan_excl(const Tin* in, Tout* out, uint64_t n, uint64_t* d_total, Ctx& c);

// True iff off[0..n] never decreases (n + 1 entries; one read-back).
bool nondecreasing(const uint64_t* off, uint64_t n, Ctx& c);

// Read offsets off[0..n] on the device, summarised into st[0..2] (device,
// zeroed by the caller; no read-back): st[0] != 0 if off[0] != 0 or the
// offsets ever decrease, st[1] += 2 * sum over reads of max(0, len - k)
// (the occurrence bound), st[2] = off[n] (bases).
void offsets_summary(const uint64_t* off, uint64_t n, uint32_t k, unsigned long long* st, Ctx& c);

// out[i] = off[i] + base for i < n (device arrays).
void offsets_rebase(const uint64_t* off, uint64_t n, uint64_t base, uint64_t* out, Ctx& c);

}  // namespace sdbg
