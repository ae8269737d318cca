// Host-side automaton representation, compilers and analysis for libcoex.
//
// A Dfa is the quintuple (Q, Sigma, delta, q0, F) of Section II of the paper
// with Sigma = {A,C,G,T} (columns 0..3) and F carried as output sets: the
// pattern ids that end at each state.
#pragma once

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace coex {

constexpr uint32_t kMaxStates = 4096;      // device tables index rows with 16-bit byte offsets
constexpr uint32_t kMaxStatesStep2 = 1024; // two-symbol table rows are 64 B
constexpr uint32_t kMaxStatesStep3 = 1023; // three-symbol entries hold row * 64 + flag in 16 bits
constexpr uint32_t kMaxLookback = 8;
constexpr uint32_t kNoSync = 0xFFFFFFFFu;
// match_density above which three symbols per lookup lose: a flagged 48-base
// unit is replayed base by base (about 48 dependent lookups instead of 16),
// so with d the fraction of flagged three-symbol steps a unit is replayed
// with probability 1 - (1 - d)^16, and above d = 0.01 (16% of units) the
// replays cost more than the 8 lookups per unit that two symbols per lookup
// (exact counts, no replay) would add
constexpr double kDenseMatches = 0.01;

struct PssTable {              // possible starting states after a k-base lookback
  uint32_t k = 0;
  uint32_t max_size = 0;
  std::vector<uint32_t> off;   // 4^k + 1; k-gram index = sum code(b_i) * 4^i, oldest base first
  std::vector<uint16_t> states;
};

struct DeviceCopy;             // per-device tables (runtime)

struct Dfa {
  uint32_t n_states = 0;
  uint32_t q0 = 0;
  uint32_t n_patterns = 0;
  std::vector<uint32_t> delta;    // n_states * 4
  std::vector<uint32_t> out_off;  // n_states + 1
  std::vector<uint32_t> out_ids;  // ascending within a state

  // analysis (filled by analyze())
  uint32_t n_accepting = 0;
  uint32_t max_out = 0;
  uint32_t sync_depth = kNoSync;
  // three-symbol steps that visit an accepting state, as a fraction, on a
  // fixed pseudo-random sequence run from q0 (walks of three symbols per
  // lookup replay every 48-base unit that holds a match, so automata that
  // match often walk two symbols per lookup, whose entries count exactly)
  double match_density = 0.0;
  std::vector<int32_t> acc_index;  // state -> dense accepting index, -1 if not final
  std::vector<uint32_t> acc_state; // dense index -> state
  PssTable pss[kMaxLookback + 1];  // [1..8]

  std::mutex mu;                  // guards the lazy device copies
  std::vector<DeviceCopy*> dev;   // indexed by device ordinal; owned, freed in ~Dfa
  Dfa() = default;
  Dfa(const Dfa&) = delete;
  Dfa& operator=(const Dfa&) = delete;
  ~Dfa();
};

// Compilers: return COEX_* status.
int compile_kmers(const std::vector<std::string>& kmers, std::unique_ptr<Dfa>& out);
int compile_regex(const std::string& regex, std::unique_ptr<Dfa>& out);
int from_table(const uint32_t* delta, uint32_t n_states, uint32_t q0, const uint32_t* out_off,
               const uint32_t* out_ids, uint32_t n_patterns, std::unique_ptr<Dfa>& out);

// Fills the analysis fields (accepting index, sync depth, PSS tables).
void analyze(Dfa& d);

}  // namespace coex
