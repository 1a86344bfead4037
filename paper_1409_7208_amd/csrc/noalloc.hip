// Allocation-free form of sdbg_count_solid (declared in include/sdbg.h).
//
// Every working buffer of the counting pipeline is carved out of one fixed
// device array, `scratch`, instead of the caching pool, and the edge set is
// written into buffers the caller passes in, so a call allocates no device
// memory.  Each device holds its own copy of the array (at its own address)
// from the first use of the library's code object on that device until the
// process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "abi_common.h"
#include "prims.h"

static constexpr size_t kScratchBytes = size_t(SDBG_NOALLOC_SCRATCH_MB) << 20;

// The fixed scratch (one copy per device).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on each device, resolved once with that
// device current.  In host code the array's name is a host-side stand-in,
// never a device address: only these resolved pointers reach kernels.
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
// Calls on one device share its scratch; they take turns.
std::mutex g_dev_mu[kMaxDevices];

int current_device() {
  int dev = 0;
  SDBG_HIP(hipGetDevice(&dev));
  SDBG_CHECK(dev >= 0 && dev < kMaxDevices, SDBG_E_HIP, "device index out of range");
  return dev;
}

void* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    SDBG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SDBG_CHECK(p != nullptr, SDBG_E_HIP, "scratch has no device address");
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// Device bytes per (k+1)-mer occurrence bound that the input must leave room
// for: the two key buffers and counts of the partition (16w + 4), the
// extraction tables and mercy lookups (about 8 more), and the edge set with
// its reverse-complement expansion and merges (about 12w + 8 per solid
// edge, at most one per two occurrences).
uint64_t bytes_per_occ(uint32_t k) {
  const uint64_t w = (uint64_t)sdbg::key_words((int)k);
  return 24 * w + 16;
}

}  // namespace

extern "C" int sdbg_count_solid_noalloc(const sdbg_reads* reads, const sdbg_params* params, uint64_t* keys_out,
                                        uint32_t* count_out, uint64_t cap, uint64_t* n_out, uint64_t* n_mercy_out,
                                        uint64_t* n_occ_out, uint64_t* scratch_peak_out) {
  return sdbg_abi::guarded([&]() -> int {
    SDBG_CHECK(reads && params && n_out, SDBG_E_INVAL, "null argument");
    SDBG_CHECK(cap == 0 || (keys_out && count_out), SDBG_E_INVAL, "null output buffer");
    *n_out = 0;
    if (n_mercy_out) *n_mercy_out = 0;
    if (n_occ_out) *n_occ_out = 0;
    if (scratch_peak_out) *scratch_peak_out = 0;
    sdbg_abi::check_params(params);
    SDBG_CHECK(reads->n_reads == 0 || reads->offsets, SDBG_E_INVAL, "null offsets");
    const int dev = current_device();
    std::lock_guard<std::mutex> turn(g_dev_mu[dev]);
    sdbg::Arena arena(scratch_on(dev), kScratchBytes);
    sdbg::ArenaScope use(&arena);
    sdbg::Ctx c(params->stream);
    const uint32_t k = params->k, w = (uint32_t)sdbg::key_words((int)k);

    sdbg::DevReads R{};
    R.n_reads = reads->n_reads;
    sdbg::DBuf<uint8_t> seq_d;
    sdbg::DBuf<uint64_t> off_d;
    std::vector<uint64_t> ho;
    if (reads->on_device && reads->n_reads) {
      const uint64_t first = c.d2h_one(reads->offsets);
      R.n_bases = c.d2h_one(reads->offsets + reads->n_reads);
      SDBG_CHECK(first == 0, SDBG_E_INVAL, "offsets[0] must be 0");
    } else {
      ho = sdbg_abi::host_offsets(c, reads);
      R.n_bases = ho.back();
    }
    // Up-front size check: each base starts at most two occurrences.
    const uint64_t occ_max = reads->on_device ? 2 * R.n_bases : sdbg_abi::occ_bound(ho, k);
    const uint64_t staged = reads->on_device ? 0 : R.n_bases + 16 + 8 * (R.n_reads + 1);
    const uint64_t need = staged + R.n_bases / 2 + occ_max * bytes_per_occ(k) + (1ull << 20);
    SDBG_CHECK(need <= kScratchBytes, SDBG_E_NOMEM_DEVICE,
               "input too large for the allocation-free call: about " + std::to_string(need) +
                   " bytes of scratch needed, " + std::to_string(kScratchBytes) + " available");
    if (R.n_reads == 0) {
      off_d = c.buf<uint64_t>(1);
      const uint64_t z = 0;
      c.h2d(off_d.get(), &z, 1);
      R.offsets = off_d.get();
      R.seq = nullptr;
    } else if (reads->on_device) {
      R.offsets = reads->offsets;
      R.seq = reads->seq;
      SDBG_CHECK(sdbg::nondecreasing(reads->offsets, reads->n_reads, c), SDBG_E_INVAL,
                 "offsets must be non-decreasing");
      SDBG_CHECK(R.n_bases == 0 || reads->seq, SDBG_E_INVAL, "null seq");
    } else {
      seq_d = c.buf<uint8_t>(R.n_bases + 16);
      off_d = c.buf<uint64_t>(R.n_reads + 1);
      c.h2d(seq_d.get(), reads->seq, R.n_bases);
      c.h2d(off_d.get(), ho.data(), R.n_reads + 1);
      R.seq = seq_d.get();
      R.offsets = off_d.get();
    }
    const uint64_t budget = params->mem_budget ? std::min<uint64_t>(params->mem_budget, kScratchBytes) : kScratchBytes;
    sdbg::CountParams P{(int)k, params->d, params->mercy != 0, (int)params->prefix_len, budget};
    sdbg::EdgesOut eo;
    sdbg::count_solid(R, P, c, &eo);
    *n_out = eo.n;
    if (n_mercy_out) *n_mercy_out = eo.n_mercy;
    if (n_occ_out) *n_occ_out = eo.n_occ;
    if (eo.n > cap) {
      c.sync();
      throw sdbg::Error(SDBG_E_INVAL, "output capacity " + std::to_string(cap) + " is below the " +
                                          std::to_string(eo.n) + " edges of the result (returned in *n_out)");
    }
    c.d2d(keys_out, eo.keys, eo.n * w);
    c.d2d(count_out, eo.count, eo.n);
    c.sync();
    if (scratch_peak_out) *scratch_peak_out = arena.peak();
    sdbg::prof_flush();
    return SDBG_OK;
  });
}
