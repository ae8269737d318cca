// k_tail instantiations for 2-bit + N mask sequences reporting per-final-state histograms (see
// tail.hpp); a translation unit of its own so the chunk-scan variants compile
// in parallel.
#include "tail.hpp"

namespace coex {

int tail_occupancy_2bit_hist(const TailKey& k, uint32_t lds) { return tail_occupancy_enc<ENC_2BIT, MODE_HIST>(k, lds); }

bool tail_launch_2bit_hist(const TailKey& k, uint32_t blocks, uint32_t lds, hipStream_t st, const ScanArgs& a) {
  return tail_launch_enc<ENC_2BIT, MODE_HIST>(k, blocks, lds, st, a);
}

}  // namespace coex
