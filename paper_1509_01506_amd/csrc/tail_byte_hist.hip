// k_tail instantiations for byte sequences reporting per-final-state histograms (see
// tail.hpp); a translation unit of its own so the chunk-scan variants compile
// in parallel.
#include "tail.hpp"

namespace coex {

int tail_occupancy_byte_hist(const TailKey& k, uint32_t lds) { return tail_occupancy_enc<ENC_BYTE, MODE_HIST>(k, lds); }

bool tail_launch_byte_hist(const TailKey& k, uint32_t blocks, uint32_t lds, hipStream_t st, const ScanArgs& a) {
  return tail_launch_enc<ENC_BYTE, MODE_HIST>(k, blocks, lds, st, a);
}

}  // namespace coex
