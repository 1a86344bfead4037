// Host replay of the device window-key helpers (paper_1409_7208_amd/csrc/
// kernels.h, device.h are __host__ __device__): the rolling update of the
// forward and reverse-complement packings must equal the packings built
// from the stream, for every key width, over random streams with read
// breaks.  Prints "ok" or the first mismatch.
#include <cstdio>
#include <random>
#include <vector>

#include "kernels.h"

using namespace sdbg;

template <int W>
bool check(int k, std::mt19937_64& rng) {
  const int kb = 2 * (k + 1);
  const uint64_t nbases = 4000;
  std::vector<uint64_t> packed(nbases / 32 + 8, 0);
  for (uint64_t j = 0; j < nbases; ++j) packed[j / 32] |= (rng() & 3) << (2 * (j % 32));
  Roller<W> rl;
  for (uint64_t pos = 0; pos + k + 1 <= nbases; ++pos) {
    if (rng() % 17 == 0) pos += rng() % 40;  // a jump, as at a read break or a skipped window
    if (pos + k + 1 > nbases) break;
    rl.at(packed.data(), k, kb, pos);
    const Key<W> F = stream_bits<W>(packed.data(), 2 * pos, kb);
    const Key<W> R = revcomp_fwd<W>(F, kb);
    if (!key_eq<W>(rl.F, F) || !key_eq<W>(rl.R, R) || !key_eq<W>(rl.fwd_key(kb), key_from_fwd<W>(F, kb)) ||
        !key_eq<W>(rl.rc_key(kb), key_from_fwd<W>(R, kb))) {
      std::printf("mismatch k=%d pos=%llu\n", k, (unsigned long long)pos);
      return false;
    }
  }
  return true;
}

int main() {
  std::mt19937_64 rng(0x14097208);
  for (int k = 2; k <= 127; ++k) {
    const int w = (2 * (k + 1) + 63) / 64;
    const bool ok = w == 1 ? check<1>(k, rng) : w == 2 ? check<2>(k, rng) : w == 3 ? check<3>(k, rng) : check<4>(k, rng);
    if (!ok) return 1;
  }
  std::printf("ok\n");
  return 0;
}
