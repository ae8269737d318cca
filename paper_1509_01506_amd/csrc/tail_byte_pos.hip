// k_tail instantiations for byte sequences reporting appended match positions (see
// tail.hpp); a translation unit of its own so the chunk-scan variants compile
// in parallel.
#include "tail.hpp"

namespace coex {

int tail_occupancy_byte_pos(const TailKey& k, uint32_t lds) { return tail_occupancy_enc<ENC_BYTE, MODE_POS>(k, lds); }

bool tail_launch_byte_pos(const TailKey& k, uint32_t blocks, uint32_t lds, hipStream_t st, const ScanArgs& a) {
  return tail_launch_enc<ENC_BYTE, MODE_POS>(k, blocks, lds, st, a);
}

}  // namespace coex
