// The paper's own method on the host's cores (Section III, Algorithm 1): a
// reported CPU baseline beside the GPU scan, never a fallback for it.
//
// The sequence is cut into equal chunks (the last takes the remainder), one
// chunk at a time per worker thread.  For chunk t > 0 the possible starting
// states are the image of Q under the symbol before the chunk (Section III.A;
// {q0} after a reset symbol); chunk 0 starts at q0.  The first candidate's
// run R0 covers the whole chunk and keeps its state after each of the first
// `window` symbols (the per-step list of Algorithm 1).  Every other candidate
// runs until its state equals R0's state after the same number of symbols
// (the converging point, Section III.B.3); its record is R0's with the counts
// before that point replaced by its own (the count fix-up of Algorithm 1).  A
// run that has not met R0 inside the window continues to the chunk end on its
// own.  The join then walks the chunks in order: each chunk's true first state
// is its predecessor's last state, which selects that chunk's record.
//
// Counts are kept per accepting state (visits) and spread over the pattern
// ids each accepting state ends at the end.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "coex.h"
#include "dfa.hpp"

namespace coex {
namespace {

constexpr int kReset = 4;  // decoded symbol that resets to q0

struct HostSeq {
  const uint8_t* data;
  const uint8_t* nmask;
  uint64_t n;
  int enc;
  uint8_t byte_sym[256];
  void init() {
    std::memset(byte_sym, kReset, sizeof byte_sym);
    const char* up = "ACGT";
    const char* lo = "acgt";
    for (int i = 0; i < 4; ++i) {
      byte_sym[(uint8_t)up[i]] = (uint8_t)i;
      byte_sym[(uint8_t)lo[i]] = (uint8_t)i;
    }
  }
  template <int ENC>
  int at(uint64_t i) const {
    if (ENC == COEX_ENC_BYTE) return byte_sym[data[i]];
    if (nmask && ((nmask[i >> 3] >> (i & 7)) & 1u)) return kReset;
    return (data[i >> 2] >> (2 * (i & 3))) & 3;
  }
};

// One candidate's outcome over its chunk.
struct Record {
  uint32_t init = 0;
  uint32_t last = 0;
  int64_t meet = -1;             // symbols consumed when it met R0 (-1: never, full run)
  std::vector<uint64_t> visits;  // per accepting state: visits in [0, meet) or the whole chunk
};

struct ChunkOut {
  std::vector<Record> rec;                               // one per possible starting state, R0 first
  std::vector<std::pair<uint32_t, uint32_t>> r0_events;  // R0's (step, accepting index) inside the window
};

struct Ctx {
  const Dfa* d;
  HostSeq sq;
  std::vector<uint32_t> tab;  // [s * 5 + sym] = next | (acc + 1) << 16, sym 4 = reset
  uint64_t n_chunks, base_len, window;
  uint32_t n_acc;
};

inline uint32_t step(const Ctx& C, uint32_t s, int sym) { return C.tab[(size_t)s * 5 + (uint32_t)sym]; }

template <int ENC>
void run_chunk(const Ctx& C, uint64_t t, ChunkOut& out, std::vector<uint32_t>& r0_states) {
  const Dfa& d = *C.d;
  const uint64_t lo = t * C.base_len;
  const uint64_t hi = (t + 1 == C.n_chunks) ? C.sq.n : lo + C.base_len;
  const uint64_t len = hi - lo;
  const uint64_t win = std::min<uint64_t>(C.window, len);
  // possible starting states (Section III.A)
  std::vector<uint32_t> cand;
  if (lo == 0) {
    cand.push_back(d.q0);
  } else {
    const int c = C.sq.at<ENC>(lo - 1);
    if (c == kReset) {
      cand.push_back(d.q0);
    } else {
      const PssTable& P = d.pss[1];
      for (uint32_t i = P.off[c]; i < P.off[c + 1]; ++i) cand.push_back(P.states[i]);
    }
  }
  out.rec.assign(cand.size(), Record());
  out.r0_events.clear();
  r0_states.resize(std::max<uint64_t>(win, 1));
  // R0: the whole chunk, states and accepting visits of the window kept
  {
    Record& r = out.rec[0];
    r.init = cand[0];
    r.visits.assign(C.n_acc, 0);
    uint32_t s = cand[0];
    uint64_t j = 0;
    for (; j < len && j < win; ++j) {
      const uint32_t e = step(C, s, C.sq.at<ENC>(lo + j));
      s = e & 0xFFFFu;
      if (e >> 16) {
        r.visits[(e >> 16) - 1] += 1;
        out.r0_events.push_back({(uint32_t)j, (e >> 16) - 1});
      }
      r0_states[j] = s;
    }
    // the rest of the chunk: only the state and the visits
    uint64_t* visits = r.visits.data();
    const uint32_t* tab = C.tab.data();
    if (ENC == COEX_ENC_2BIT) {
      // eight bases (two code bytes, one mask byte) at a time once aligned
      for (; j < len && ((lo + j) & 7); ++j) {
        const uint32_t e = tab[(size_t)s * 5 + (uint32_t)C.sq.at<ENC>(lo + j)];
        s = e & 0xFFFFu;
        if (e >> 16) visits[(e >> 16) - 1] += 1;
      }
      for (; j + 8 <= len; j += 8) {
        const uint64_t q = lo + j;
        const uint32_t m = C.sq.nmask ? C.sq.nmask[q >> 3] : 0u;
        const uint32_t codes = (uint32_t)C.sq.data[q >> 2] | (uint32_t)C.sq.data[(q >> 2) + 1] << 8;
        for (int i = 0; i < 8; ++i) {
          const uint32_t sym = ((m >> i) & 1u) ? 4u : (codes >> (2 * i)) & 3u;
          const uint32_t e = tab[(size_t)s * 5 + sym];
          s = e & 0xFFFFu;
          if (e >> 16) visits[(e >> 16) - 1] += 1;
        }
      }
    }
    for (; j < len; ++j) {
      const uint32_t e = tab[(size_t)s * 5 + (uint32_t)C.sq.at<ENC>(lo + j)];
      s = e & 0xFFFFu;
      if (e >> 16) visits[(e >> 16) - 1] += 1;
    }
    r.last = s;
    r.meet = 0;
  }
  // the other candidates: until they meet R0 after the same number of symbols
  for (size_t k = 1; k < cand.size(); ++k) {
    Record& r = out.rec[k];
    r.init = cand[k];
    r.visits.assign(C.n_acc, 0);
    uint32_t s = cand[k];
    r.meet = -1;
    for (uint64_t j = 0; j < len; ++j) {
      const uint32_t e = step(C, s, C.sq.at<ENC>(lo + j));
      s = e & 0xFFFFu;
      if (e >> 16) r.visits[(e >> 16) - 1] += 1;
      if (j < win && s == r0_states[j]) {  // converging point: j + 1 symbols consumed
        r.meet = (int64_t)(j + 1);
        break;
      }
    }
    r.last = r.meet >= 0 ? out.rec[0].last : s;
  }
}

}  // namespace
}  // namespace coex

extern "C" int coex_count_host(const coex_dfa* dfa, const void* bases, const uint8_t* n_mask, uint64_t n_bases,
                               int32_t encoding, uint32_t threads, uint64_t n_chunks, uint64_t window,
                               uint64_t* counts) {
  using namespace coex;
  if (!dfa || !counts || (n_bases && !bases)) return COEX_EINVAL;
  if (encoding != COEX_ENC_BYTE && encoding != COEX_ENC_2BIT) return COEX_EINVAL;
  try {
    const Dfa& d = *reinterpret_cast<const Dfa*>(dfa);
    Ctx C;
    C.d = &d;
    C.sq = HostSeq{static_cast<const uint8_t*>(bases), encoding == COEX_ENC_2BIT ? n_mask : nullptr, n_bases,
                   encoding, {}};
    C.sq.init();
    C.n_acc = d.n_accepting;
    C.tab.resize((size_t)d.n_states * 5);
    for (uint32_t s = 0; s < d.n_states; ++s) {
      for (int c = 0; c < 4; ++c) {
        const uint32_t t = d.delta[s * 4 + c];
        C.tab[(size_t)s * 5 + c] = t | (uint32_t)(d.acc_index[t] + 1) << 16;
      }
      C.tab[(size_t)s * 5 + 4] = d.q0;  // a reset symbol: q0, no match
    }
    if (threads == 0) threads = std::max(1u, std::thread::hardware_concurrency());
    if (n_chunks == 0) n_chunks = threads;
    if (n_bases == 0) n_chunks = 1;
    n_chunks = std::min<uint64_t>(n_chunks, std::max<uint64_t>(1, n_bases));
    C.n_chunks = n_chunks;
    C.base_len = n_bases / n_chunks;
    C.window = window ? window : 4096;
    std::vector<ChunkOut> outs(n_chunks);
    std::atomic<uint64_t> next{0};
    auto worker = [&]() {
      std::vector<uint32_t> r0_states;
      for (uint64_t t = next.fetch_add(1); t < n_chunks; t = next.fetch_add(1)) {
        if (encoding == COEX_ENC_BYTE) run_chunk<COEX_ENC_BYTE>(C, t, outs[t], r0_states);
        else run_chunk<COEX_ENC_2BIT>(C, t, outs[t], r0_states);
      }
    };
    const uint32_t nt = (uint32_t)std::min<uint64_t>(threads, n_chunks);
    std::vector<std::thread> pool;
    for (uint32_t i = 1; i < nt; ++i) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    // the join: each chunk's true first state is its predecessor's last state
    std::vector<uint64_t> total(C.n_acc, 0);
    uint32_t s = d.q0;
    for (uint64_t t = 0; t < n_chunks; ++t) {
      const ChunkOut& o = outs[t];
      size_t k = 0;
      while (k < o.rec.size() && o.rec[k].init != s) ++k;
      if (k == o.rec.size()) return COEX_EINTERNAL;  // the true state is always a candidate
      const Record& r = o.rec[k];
      if (k == 0 || r.meet < 0) {
        for (uint32_t a = 0; a < C.n_acc; ++a) total[a] += r.visits[a];
      } else {
        // fix-up: R0's counts with its prefix before the converging point
        // replaced by this run's own
        const Record& r0 = o.rec[0];
        for (uint32_t a = 0; a < C.n_acc; ++a) total[a] += r0.visits[a] + r.visits[a];
        for (const auto& ev : o.r0_events)
          if ((int64_t)ev.first < r.meet) total[ev.second] -= 1;
      }
      s = r.last;
    }
    std::vector<uint64_t> per(d.n_patterns, 0);
    for (uint32_t a = 0; a < C.n_acc; ++a) {
      const uint32_t st = d.acc_state[a];
      for (uint32_t x = d.out_off[st]; x < d.out_off[st + 1]; ++x) per[d.out_ids[x]] += total[a];
    }
    std::memcpy(counts, per.data(), per.size() * 8);
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}
