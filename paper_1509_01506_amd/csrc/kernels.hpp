// HIP kernels of libcoex (gfx950, wave64).
//
// The scan is the paper's input-based decomposition (Section III, Algorithm 1)
// laid out for CDNA4:
//   - a chunk of the sequence belongs to one lane; a wave owns 64 consecutive
//     chunks (a "tile");
//   - possible starting states (PSS) of each chunk come from a table indexed
//     by the k bases before it (Section III.A, with k >= 1 symbols instead of
//     one); the lanes of a group run the candidates of one chunk in lockstep
//     over the same symbols and stop at the converging point, detected with a
//     wave ballot against the group's first lane (Section III.B.3);
//   - the owner lane then scans the rest of its chunk once, from the
//     converged state, with the transition table in LDS: two symbols per
//     lookup, 128-byte loads per lane from HBM;
//   - a compose kernel joins each chunk's last state to the next chunk's first
//     state (the paper's join), and a fix-up kernel recounts each chunk's
//     prefix up to its converging point from the true starting state (the
//     count fix-up of Algorithm 1 in an equivalent form).
//
// Table formats (built on the host, copied to LDS):
//   state register value s = state_id << SHIFT (SHIFT = 6 with the two-symbol
//   table, 4 without);
//   T1 (one symbol) : u32[n][4]  = (succ << SHIFT) | (acc_index + 1) << 16
//   T2 (two symbols): u32[n][16] = (succ2 << 6) | count << 24, column
//                     g = c0 | c1 << 2 for symbols c0 then c1; count = number
//                     of pattern ends at the two visited states (or just 1 if
//                     any, when counts could overflow the 8-bit field).
//   T3 (three symbols, at most 1023 states): u16[n + 1][64] = succ3 << 6 |
//                     flag, column g = c0 | c1 << 2 | c2 << 4; flag = an
//                     accepting state is among the three visited ones.  The
//                     entry is the next state register value itself (flag in
//                     bit 0, which no row offset uses); row n repeats row 0,
//                     so a walk that carries a set flag into the next address
//                     still reads table entries (the word is replayed anyway).
//   Column order is the encoding's natural one: A,C,G,T for 2-bit codes and
//   A,C,T,G for bytes ((byte >> 1) & 3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Threads per block of the scan kernels.
#define COEX_SCAN_BLOCK 768
// Minimum waves per SIMD the chunk-scan kernel is compiled for (caps its
// registers at 512 / waves).
#define COEX_TAIL_WAVES 6

namespace coex {

constexpr int ENC_BYTE = 0;
constexpr int ENC_2BIT = 1;
constexpr uint32_t NONCONV = 0xFFFFFFFFu;
constexpr uint32_t FIXED = 0x40000000u;   // conv_t flag: prefix already recounted in the scan kernel
constexpr int TILE = 64;          // chunks per wave
constexpr int SPEC_WIN = 64;      // symbols examined for convergence

struct ScanArgs {
  // sequence
  const uint8_t* bases;
  const uint8_t* nmask;
  uint64_t n;                 // buffer position one past the sequence's last base
  uint64_t first;             // buffer position of the sequence's first base
  uint64_t chunk;
  uint64_t n_chunks;
  uint64_t n_tiles;
  // tables (global copies)
  const uint32_t* T2;
  const uint16_t* T3;
  const uint32_t* T1;
  const uint32_t* wtab;       // weight (number of patterns) per accepting index
  uint32_t n_states;
  uint32_t n_acc;
  uint32_t q0s;               // q0 << SHIFT
  uint32_t lds_t1_off;        // byte offset of T1 in LDS
  uint32_t lds_w_off;         // byte offset of weights in LDS
  uint32_t lds_hist_off;      // byte offset of the visit histogram in LDS
  // possible starting states
  const uint32_t* pss_off;
  const uint16_t* pss_states;
  uint32_t k;
  uint32_t group;             // lanes per chunk in the speculation (power of two)
  uint32_t max_cand;          // largest candidate list of any chunk
  uint32_t nc_group;          // lanes per non-converged chunk (power of two >= max_cand)
  // per-chunk outputs
  uint32_t* conv_t;           // symbols consumed to the converging point, NONCONV if none
  uint32_t* conv_s;           // state there
  uint32_t* end_s;            // state at the chunk end (converged chunks)
  uint32_t* tail_cnt;         // matches in [conv_t, end)
  uint32_t* fix_count;        // chunks left for the fix-up kernel besides the first chunk of every tile
  uint32_t* fix_list;
  uint64_t* front;            // per tile: the first SPEC_WIN symbols of its first chunk (3 words)
  uint32_t lds_red_off;       // LDS byte offset of the per-wave partial sums (scan kernel)
  uint32_t spec_pss_off;      // LDS byte offsets of the PSS table in the speculation kernel (0: not staged)
  uint32_t spec_pss_states;
  uint32_t pss_n_off;
  uint32_t pss_n_states;
  uint32_t* nc_count;         // number of non-converged chunks
  uint32_t* nc_chunk;         // slot -> chunk
  uint32_t* nc_slot;          // chunk -> slot
  uint32_t* nc_m;             // slot -> number of candidates
  uint32_t* nc_cand;          // slot * max_cand + i -> candidate state
  uint32_t* nc_end;           // slot * max_cand + i -> end state from that candidate
  uint32_t* nc_cnt;           // per slot and candidate: its run's weighted match count
  uint32_t* true_start;       // n_chunks + 1
  unsigned long long* pat_counts;  // per pattern (the caller's counts), or NULL
  unsigned long long* total;  // weighted total
  uint64_t* chunk_cnt;        // per chunk total (find / records)
  uint32_t* err;              // device consistency flag
  uint32_t* err_sticky;       // failures kept across calls until read (coex_errors_async), or NULL
  // outputs per accepting index
  const uint32_t* acc_out_off;
  const uint32_t* acc_out_ids;
  uint32_t n_patterns;
  // find / records
  const uint64_t* chunk_off;  // exclusive prefix of chunk_cnt
  int64_t* pos_out;
  uint32_t* pat_out;
  uint64_t pos_cap;
  uint64_t* rec_counts;       // n_chunks * n_patterns
  uint32_t* rec_init;
  uint32_t* rec_last;
  uint32_t shift;             // SHIFT (state register scale)
  // find in one pass: every match appended as end position << 24 | pattern id
  unsigned long long* app_count;
  uint64_t* app_keys;
  uint64_t app_cap;
};

// A failed device consistency check: the call's own word (read by checked
// calls) and the word kept until the caller reads it.
__device__ __forceinline__ void flag_error(const ScanArgs& a, uint32_t bits) {
  atomicOr(a.err, bits);
  if (a.err_sticky) atomicOr(a.err_sticky, bits);
}

// ------------------------------------------------------------------ symbols
// Column of the base at p for the table of encoding ENC, or -1 for a reset.
template <int ENC>
__device__ __forceinline__ int load_col(const ScanArgs& a, uint64_t p) {
  if constexpr (ENC == ENC_2BIT) {
    if (a.nmask && ((a.nmask[p >> 3] >> (p & 7)) & 1u)) return -1;
    return (a.bases[p >> 2] >> (2u * (uint32_t)(p & 3))) & 3u;
  } else {
    uint32_t b = a.bases[p];
    uint32_t t = (b >> 1) & 3u;
    uint32_t expect = (0x47544341u >> (8u * t)) & 0xFFu;  // 'A','C','T','G'
    return ((b & 0xDFu) == expect) ? (int)t : -1;
  }
}

// A,C,G,T code (for the PSS index) of a column.
template <int ENC>
__device__ __forceinline__ uint32_t col_to_code(uint32_t c) {
  if constexpr (ENC == ENC_2BIT) return c;
  else return c ^ (c >> 1);
}

// 16 bases starting at p (p % 16 == 0, p + 16 <= n): columns packed two bits
// per base (base i at bits 2i) and a reset bit per base.
template <int ENC>
__device__ __forceinline__ void load_word(const ScanArgs& a, uint64_t p, uint32_t& cols, uint32_t& rst) {
  if constexpr (ENC == ENC_2BIT) {
    cols = *reinterpret_cast<const uint32_t*>(a.bases + (p >> 2));
    rst = a.nmask ? (uint32_t)*reinterpret_cast<const uint16_t*>(a.nmask + (p >> 3)) : 0u;
  } else {
    uint4 v = *reinterpret_cast<const uint4*>(a.bases + p);
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
    cols = 0;
    rst = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uint32_t t = (w[i] >> 1) & 0x03030303u;
      uint32_t expect = __builtin_amdgcn_perm(0u, 0x47544341u, t);
      uint32_t bad = (w[i] & 0xDFDFDFDFu) ^ expect;  // nonzero byte = reset
      uint32_t u = t | (t >> 6);                     // nibbles in bytes 0 and 2
      uint32_t packed = (u & 0xFu) | ((u >> 12) & 0xF0u);
      cols |= packed << (8 * i);
      uint32_t r = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) r |= (((bad >> (8 * j)) & 0xFFu) != 0u) << j;
      rst |= r << (4 * i);
    }
  }
}

// ------------------------------------------------------------------ table access
// Table bases: LDS in the scan kernels, global memory elsewhere (the same
// byte layout either way).
struct Tab {
  const char* t2;   // two-symbol table (SHIFT == 6)
  const char* t1;   // one-symbol table
  uint32_t q0s;     // start state register value
};

template <int SHIFT>
__device__ __forceinline__ uint32_t t1_lookup(const Tab& tb, uint32_t s, uint32_t col) {
  return *reinterpret_cast<const uint32_t*>(tb.t1 + (s >> (SHIFT - 4)) + col * 4u);
}

__device__ __forceinline__ uint32_t t2_lookup(const Tab& tb, uint32_t s, uint32_t g) {
  return *reinterpret_cast<const uint32_t*>(tb.t2 + s + g * 4u);
}

// ------------------------------------------------------------------ sinks
// A sink receives the matches of a scanned range.  `hit(pos, a)` is called
// for every visit of an accepting state (dense index a) at base position
// pos; `word(cnt)` receives the exact weighted count of a 16-base word when
// the sink does not need per-position detail (kReplay == false).
struct SinkTotal {      // total weighted count from exact two-symbol counts
  static constexpr bool kReplay = false;
  static constexpr bool kOutline = false;
  const uint32_t* w;    // weight per accepting index
  uint32_t cnt = 0;
  __device__ void word(uint32_t c) { cnt += c; }
  __device__ void hit(uint64_t, uint32_t a) { cnt += w[a]; }
};

struct SinkHist {       // per accepting state visits in an LDS histogram
  static constexpr bool kReplay = true;
  static constexpr bool kOutline = false;
  const uint32_t* w;
  uint32_t* hist;
  uint32_t cnt = 0;
  __device__ void word(uint32_t) {}
  __device__ void hit(uint64_t, uint32_t a) {
    cnt += w[a];
    atomicAdd(hist + a, 1u);
  }
};

struct SinkGlobal {     // weighted count, and per-pattern counts straight to global memory
  static constexpr bool kReplay = true;
  static constexpr bool kOutline = false;
  const uint32_t* w;
  const uint32_t* out_off;     // per accepting index: its pattern ids
  const uint32_t* out_ids;
  unsigned long long* pat;     // NULL: count only
  unsigned long long* app_count = nullptr;  // non-NULL: append (position << 24 | id) keys
  uint64_t* app_keys = nullptr;
  uint64_t app_cap = 0;
  uint32_t cnt = 0;
  __device__ void word(uint32_t) {}
  __device__ void hit(uint64_t p, uint32_t a) {
    cnt += w[a];
    if (pat)
      for (uint32_t j = out_off[a]; j < out_off[a + 1]; ++j) atomicAdd(pat + out_ids[j], 1ull);
    if (app_count)
      for (uint32_t j = out_off[a]; j < out_off[a + 1]; ++j) {
        const unsigned long long i = atomicAdd(app_count, 1ull);
        if (i < app_cap) app_keys[i] = p << 24 | out_ids[j];
      }
  }
};

struct SinkPositions {  // end positions and pattern ids, in order
  static constexpr bool kReplay = true;
  static constexpr bool kOutline = false;
  const uint32_t* out_off;   // per accepting index
  const uint32_t* out_ids;
  int64_t* pos;
  uint32_t* pat;
  uint64_t at;
  uint64_t cap;              // writes stop at the buffer end whatever the count
  uint64_t first;            // buffer position of the sequence's first base
  uint32_t cnt = 0;
  __device__ void word(uint32_t) {}
  __device__ void hit(uint64_t p, uint32_t a) {
    for (uint32_t i = out_off[a]; i < out_off[a + 1]; ++i) {
      if (at < cap) {
        pos[at] = (int64_t)(p - first);
        if (pat) pat[at] = out_ids[i];
      }
      ++at;
      ++cnt;
    }
  }
};

struct SinkRecord {     // per chunk, per pattern counts
  static constexpr bool kReplay = true;
  static constexpr bool kOutline = false;
  const uint32_t* out_off;
  const uint32_t* out_ids;
  uint64_t* row;
  uint32_t cnt = 0;
  __device__ void word(uint32_t) {}
  __device__ void hit(uint64_t, uint32_t a) {
    for (uint32_t i = out_off[a]; i < out_off[a + 1]; ++i) {
      row[out_ids[i]] += 1;
      ++cnt;
    }
  }
};

// ------------------------------------------------------------------ scanning
// One symbol (col < 0: reset); returns the new state.
template <int SHIFT, class Sink>
__device__ __forceinline__ uint32_t step1(const Tab& tb, uint32_t s, int col, uint64_t p, Sink& sink) {
  if (col < 0) return tb.q0s;
  uint32_t e = t1_lookup<SHIFT>(tb, s, (uint32_t)col);
  uint32_t a = e >> 16;
  if (a) sink.hit(p, a - 1u);
  return e & 0xFFFFu;
}

// The bases of one 16-base word selected by `act` (bit i = base p+i), one
// at a time, resets honoured.
template <int SHIFT, class Sink>
__device__ __forceinline__ uint32_t word_slow(const Tab& tb, uint32_t s, uint32_t cols, uint32_t rst, uint32_t act,
                                              uint64_t p, Sink& sink) {
#pragma unroll 1
  for (int i = 0; i < 16; ++i) {
    if (!((act >> i) & 1u)) continue;
    int col = ((rst >> i) & 1u) ? -1 : (int)((cols >> (2 * i)) & 3u);
    s = step1<SHIFT>(tb, s, col, p + i, sink);
  }
  return s;
}

// A word one base at a time through the sink's own out-of-line routine when
// it has one (kOutline: keeps the rare path out of the unrolled hot loop).
template <int SHIFT, class Sink>
__device__ __forceinline__ uint32_t slow_word(const Tab& tb, uint32_t s, uint32_t cols, uint32_t rst, uint32_t act,
                                              uint64_t p, Sink& sink) {
  if constexpr (Sink::kOutline) return sink.template slow<SHIFT>(s, cols, rst, act, p);
  else return word_slow<SHIFT>(tb, s, cols, rst, act, p, sink);
}

// LDS read at a byte address.  The two-symbol table is staged at LDS
// address 0 (the kernels using it declare no other LDS), so a state value
// (row byte offset) plus a column offset is a complete LDS address.
typedef __attribute__((address_space(3))) const uint32_t lds_u32;
typedef __attribute__((address_space(3))) const char lds_c;
__device__ __forceinline__ uint32_t lds_at(uint32_t addr) { return *(lds_u32*)(uintptr_t)addr; }
typedef __attribute__((address_space(3))) const uint16_t lds_u16;
__device__ __forceinline__ uint32_t lds_u16_at(uint32_t addr) { return *(lds_u16*)(uintptr_t)addr; }

// (e & 0xFFFF) + byte B of x in one VALU instruction (sub-dword operand
// selection): the next row offset from a table entry plus a column offset.
template <int B>
__device__ __forceinline__ uint32_t row_plus_byte(uint32_t e, uint32_t x) {
  uint32_t r;
  if constexpr (B == 0)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:BYTE_0"
        : "=v"(r) : "v"(e), "v"(x));
  else if constexpr (B == 1)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:BYTE_1"
        : "=v"(r) : "v"(e), "v"(x));
  else if constexpr (B == 2)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:BYTE_2"
        : "=v"(r) : "v"(e), "v"(x));
  else
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:BYTE_3"
        : "=v"(r) : "v"(e), "v"(x));
  return r;
}

// 16 symbols without resets: eight two-symbol lookups (STEP 2, table in LDS
// at address 0), five three-symbol lookups and one one-symbol lookup (STEP 3,
// three-symbol table at LDS address 0), or sixteen one-symbol lookups.
// Returns the state after the word; `c` receives the number of pattern ends
// in the word (STEP 2, exact two-symbol counts) or a nonzero flag when any
// accepting state was visited (STEP 3: the returned state is then not
// meaningful and the caller replays the word).
// For STEP 2 the two-bit columns are spread into byte lanes once per word
// (columns of even grams times 4 in xa, odd grams in xb), so each lookup
// costs one address instruction.
template <int SHIFT, int STEP>
__device__ __forceinline__ uint32_t walk16(const Tab& tb, uint32_t s, uint32_t cols, uint32_t& c) {
  static_assert(STEP == 1 || SHIFT == 6, "two- and three-symbol tables need 64-byte state units");
  if constexpr (STEP == 3) {
    // entry = next state register (row * 64) | flag; address = 2 * (entry + column)
    const uint32_t e0 = lds_u16_at((s + (cols & 63u)) << 1);
    const uint32_t e1 = lds_u16_at((e0 + ((cols >> 6) & 63u)) << 1);
    const uint32_t e2 = lds_u16_at((e1 + ((cols >> 12) & 63u)) << 1);
    const uint32_t e3 = lds_u16_at((e2 + ((cols >> 18) & 63u)) << 1);
    const uint32_t e4 = lds_u16_at((e3 + ((cols >> 24) & 63u)) << 1);
    const uint32_t t = t1_lookup<SHIFT>(tb, e4, cols >> 30);  // e4 >> 2 drops the flag bit
    c = ((e0 | e1 | e2 | e3 | e4) & 1u) | (t >> 16);
    return t & 0xFFFFu;
  } else if constexpr (STEP == 2) {
    const uint32_t xa = (cols << 2) & 0x3C3C3C3Cu;
    const uint32_t xb = (cols >> 2) & 0x3C3C3C3Cu;
    const uint32_t e0 = lds_at(row_plus_byte<0>(s, xa));
    const uint32_t e1 = lds_at(row_plus_byte<0>(e0, xb));
    const uint32_t e2 = lds_at(row_plus_byte<1>(e1, xa));
    const uint32_t e3 = lds_at(row_plus_byte<1>(e2, xb));
    const uint32_t e4 = lds_at(row_plus_byte<2>(e3, xa));
    const uint32_t e5 = lds_at(row_plus_byte<2>(e4, xb));
    const uint32_t e6 = lds_at(row_plus_byte<3>(e5, xa));
    const uint32_t e7 = lds_at(row_plus_byte<3>(e6, xb));
    c = (e0 + e1 + e2 + e3 + e4 + e5 + e6 + e7) >> 24;
    return e7 & 0xFFFFu;
  } else {
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      uint32_t e = t1_lookup<SHIFT>(tb, s, (cols >> (2 * j)) & 3u);
      s = e & 0xFFFFu;
      acc |= e;
    }
    c = acc >> 16;
    return s;
  }
}

// What follows the table walk of a word without a reset boundary (rst is 0
// or all ones): a word inside an N run ends in q0 and reports nothing; a word
// with matches is replayed base by base when the sink needs the detail, when
// the step cannot count exactly (STEP 1) or when the walk's end state is not
// meaningful (STEP 3 with a flag).
template <int SHIFT, int STEP, class Sink>
__device__ __forceinline__ uint32_t finish_word(const Tab& tb, uint32_t s, uint32_t e, uint32_t c, uint32_t cols,
                                                uint32_t rst, uint64_t p, Sink& sink) {
  if (rst) {
    e = tb.q0s;
    c = 0;
  }
  if constexpr (STEP == 3) {
    if (__builtin_expect(c != 0u, 0)) e = slow_word<SHIFT>(tb, s, cols, 0u, 0xFFFFu, p, sink);
  } else if constexpr (Sink::kReplay || STEP == 1) {
    if (__builtin_expect(c != 0u, 0)) slow_word<SHIFT>(tb, s, cols, 0u, 0xFFFFu, p, sink);
  } else {
    sink.word(c);
  }
  return e;
}

// One 16-base word with reset bits `rst`.  Words without resets and words
// made only of resets (inside runs of N) take the table walk; the latter
// end in q0 and report nothing, so lanes inside N runs do not diverge from
// the others.  Words with a reset boundary go one base at a time.
template <int SHIFT, int STEP, class Sink>
__device__ __forceinline__ uint32_t run_word(const Tab& tb, uint32_t s, uint32_t cols, uint32_t rst, uint64_t p,
                                             Sink& sink) {
  if (rst == 0u || rst == 0xFFFFu) {
    uint32_t c;
    const uint32_t e = walk16<SHIFT, STEP>(tb, s, cols, c);
    return finish_word<SHIFT, STEP>(tb, s, e, c, cols, rst, p, sink);
  }
  return slow_word<SHIFT>(tb, s, cols, rst, 0xFFFFu, p, sink);
}

// Two independent words (two chunks of one lane) walked with their lookups
// interleaved, so two dependent chains of LDS reads are in flight per lane.
template <int SHIFT, int STEP>
__device__ __forceinline__ void walk16x2(const Tab& tb, uint32_t s0, uint32_t cols0, uint32_t& e0, uint32_t& c0,
                                         uint32_t s1, uint32_t cols1, uint32_t& e1, uint32_t& c1) {
  if constexpr (STEP == 3) {
    const uint32_t a0 = lds_u16_at((s0 + (cols0 & 63u)) << 1);
    const uint32_t b0 = lds_u16_at((s1 + (cols1 & 63u)) << 1);
    const uint32_t a1 = lds_u16_at((a0 + ((cols0 >> 6) & 63u)) << 1);
    const uint32_t b1 = lds_u16_at((b0 + ((cols1 >> 6) & 63u)) << 1);
    const uint32_t a2 = lds_u16_at((a1 + ((cols0 >> 12) & 63u)) << 1);
    const uint32_t b2 = lds_u16_at((b1 + ((cols1 >> 12) & 63u)) << 1);
    const uint32_t a3 = lds_u16_at((a2 + ((cols0 >> 18) & 63u)) << 1);
    const uint32_t b3 = lds_u16_at((b2 + ((cols1 >> 18) & 63u)) << 1);
    const uint32_t a4 = lds_u16_at((a3 + ((cols0 >> 24) & 63u)) << 1);
    const uint32_t b4 = lds_u16_at((b3 + ((cols1 >> 24) & 63u)) << 1);
    const uint32_t ta = t1_lookup<SHIFT>(tb, a4, cols0 >> 30);
    const uint32_t tb1 = t1_lookup<SHIFT>(tb, b4, cols1 >> 30);
    c0 = ((a0 | a1 | a2 | a3 | a4) & 1u) | (ta >> 16);
    c1 = ((b0 | b1 | b2 | b3 | b4) & 1u) | (tb1 >> 16);
    e0 = ta & 0xFFFFu;
    e1 = tb1 & 0xFFFFu;
  } else if constexpr (STEP == 2) {
    const uint32_t xa = (cols0 << 2) & 0x3C3C3C3Cu, xb = (cols0 >> 2) & 0x3C3C3C3Cu;
    const uint32_t ya = (cols1 << 2) & 0x3C3C3C3Cu, yb = (cols1 >> 2) & 0x3C3C3C3Cu;
    const uint32_t a0 = lds_at(row_plus_byte<0>(s0, xa)), b0 = lds_at(row_plus_byte<0>(s1, ya));
    const uint32_t a1 = lds_at(row_plus_byte<0>(a0, xb)), b1 = lds_at(row_plus_byte<0>(b0, yb));
    const uint32_t a2 = lds_at(row_plus_byte<1>(a1, xa)), b2 = lds_at(row_plus_byte<1>(b1, ya));
    const uint32_t a3 = lds_at(row_plus_byte<1>(a2, xb)), b3 = lds_at(row_plus_byte<1>(b2, yb));
    const uint32_t a4 = lds_at(row_plus_byte<2>(a3, xa)), b4 = lds_at(row_plus_byte<2>(b3, ya));
    const uint32_t a5 = lds_at(row_plus_byte<2>(a4, xb)), b5 = lds_at(row_plus_byte<2>(b4, yb));
    const uint32_t a6 = lds_at(row_plus_byte<3>(a5, xa)), b6 = lds_at(row_plus_byte<3>(b5, ya));
    const uint32_t a7 = lds_at(row_plus_byte<3>(a6, xb)), b7 = lds_at(row_plus_byte<3>(b6, yb));
    c0 = (a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7) >> 24;
    c1 = (b0 + b1 + b2 + b3 + b4 + b5 + b6 + b7) >> 24;
    e0 = a7 & 0xFFFFu;
    e1 = b7 & 0xFFFFu;
  } else {
    e0 = walk16<SHIFT, STEP>(tb, s0, cols0, c0);
    e1 = walk16<SHIFT, STEP>(tb, s1, cols1, c1);
  }
}

// One word of each of two chains.
template <int SHIFT, int STEP, class Sink>
__device__ __forceinline__ void run_word2(const Tab& tb, uint32_t& s0, uint32_t cols0, uint32_t rst0, uint64_t p0,
                                          Sink& k0, uint32_t& s1, uint32_t cols1, uint32_t rst1, uint64_t p1,
                                          Sink& k1) {
  if ((rst0 == 0u || rst0 == 0xFFFFu) && (rst1 == 0u || rst1 == 0xFFFFu)) {
    uint32_t e0, c0, e1, c1;
    walk16x2<SHIFT, STEP>(tb, s0, cols0, e0, c0, s1, cols1, e1, c1);
    s0 = finish_word<SHIFT, STEP>(tb, s0, e0, c0, cols0, rst0, p0, k0);
    s1 = finish_word<SHIFT, STEP>(tb, s1, e1, c1, cols1, rst1, p1, k1);
  } else {
    s0 = run_word<SHIFT, STEP>(tb, s0, cols0, rst0, p0, k0);
    s1 = run_word<SHIFT, STEP>(tb, s1, cols1, rst1, p1, k1);
  }
}

// A block of sequence held in registers: 512 bases (128 bytes of 2-bit codes
// and 64 bytes of N mask) or 128 bases (128 bytes).  Loaded with 16-byte
// loads per lane so each lane consumes whole 128-byte lines at once.
template <int ENC>
struct Block;

template <>
struct Block<ENC_2BIT> {
  static constexpr uint64_t BASES = 512;
  static constexpr int WORDS = (int)(BASES / 16);  // 16 bases per 32-bit word
  static constexpr int MW = WORDS / 2;             // 32 bases per 32-bit mask word
  uint32_t v[WORDS];
  uint32_t m[MW];
  __device__ __forceinline__ void word(int w, uint32_t& cols, uint32_t& rst) const {
    cols = v[w];
    rst = (m[w >> 1] >> (16 * (w & 1))) & 0xFFFFu;
  }
  __device__ __forceinline__ uint32_t any_reset() const {
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < MW; ++i) x |= m[i];
    return x;
  }
  __device__ __forceinline__ void load_codes(const ScanArgs& a, uint64_t base) {
    const uint4* src = reinterpret_cast<const uint4*>(a.bases + (base >> 2));
#pragma unroll
    for (int i = 0; i < WORDS / 4; ++i) {
      uint4 t = src[i];
      v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w;
    }
  }
  // Codes of this block and the N bits of this block and the next (one
  // 128-byte mask line for 1024 bases, read once): the second half goes to
  // `next` for the following block.  Whole pair inside the sequence, mask
  // present.
  __device__ __forceinline__ void load_pair_first(const ScanArgs& a, uint64_t base, uint32_t (&next)[MW]) {
    load_codes(a, base);
    const uint4* ms = reinterpret_cast<const uint4*>(a.nmask + (base >> 3));
#pragma unroll
    for (int i = 0; i < MW / 4; ++i) {
      uint4 t = ms[i];
      m[4 * i] = t.x; m[4 * i + 1] = t.y; m[4 * i + 2] = t.z; m[4 * i + 3] = t.w;
      uint4 u = ms[MW / 4 + i];
      next[4 * i] = u.x; next[4 * i + 1] = u.y; next[4 * i + 2] = u.z; next[4 * i + 3] = u.w;
    }
  }
  __device__ __forceinline__ void load_second(const ScanArgs& a, uint64_t base, const uint32_t (&mask)[MW]) {
    load_codes(a, base);
#pragma unroll
    for (int i = 0; i < MW; ++i) m[i] = mask[i];
  }
  // whole block inside the sequence
  __device__ __forceinline__ void load(const ScanArgs& a, uint64_t base) {
    load_codes(a, base);
    if (a.nmask) {
      const uint4* ms = reinterpret_cast<const uint4*>(a.nmask + (base >> 3));
#pragma unroll
      for (int i = 0; i < MW / 4; ++i) {
        uint4 t = ms[i];
        m[4 * i] = t.x; m[4 * i + 1] = t.y; m[4 * i + 2] = t.z; m[4 * i + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < MW; ++i) m[i] = 0;
    }
  }
  // block crossing the end of the sequence: only bytes below n are read
  __device__ void load_partial(const ScanArgs& a, uint64_t base) {
    const uint64_t nb = (a.n + 3) >> 2, nm = (a.n + 7) >> 3;
#pragma unroll
    for (int w = 0; w < WORDS; ++w) {
      const uint64_t b = (base >> 2) + 4 * w;
      uint32_t x = 0;
      if (b + 4 <= nb) x = *reinterpret_cast<const uint32_t*>(a.bases + b);
      else
        for (uint64_t j = b; j < nb && j < b + 4; ++j) x |= (uint32_t)a.bases[j] << (8 * (j - b));
      v[w] = x;
    }
#pragma unroll
    for (int i = 0; i < MW; ++i) {
      const uint64_t b = (base >> 3) + 4 * i;
      uint32_t x = 0;
      if (a.nmask) {
        if (b + 4 <= nm) x = *reinterpret_cast<const uint32_t*>(a.nmask + b);
        else
          for (uint64_t j = b; j < nm && j < b + 4; ++j) x |= (uint32_t)a.nmask[j] << (8 * (j - b));
      }
      m[i] = x;
    }
  }
};

template <>
struct Block<ENC_BYTE> {
  static constexpr uint64_t BASES = 128;
  static constexpr int WORDS = 8;
  uint4 r[8];
  // Columns: each byte's code sits in its bits 0-1; t | t >> 6 puts two
  // bases' codes in bytes 0 and 2, byte permutes gather those, and one more
  // shift-or and permute give four codes per byte.  Resets: the high bit of
  // every byte that is not A/C/G/T (either case), found without a per-byte
  // compare ((b & 0x7F) + 0x7F has its high bit set for b & 0x7F nonzero);
  // the per-base bits are only spread out for a word that mixes bases and
  // resets.
  __device__ __forceinline__ void word(int w, uint32_t& cols, uint32_t& rst) const {
    const uint32_t x[4] = {r[w].x, r[w].y, r[w].z, r[w].w};
    uint32_t p[4], nz[4], any = 0u, all = 0x80808080u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t t = (x[i] >> 1) & 0x03030303u;
      const uint32_t expect = __builtin_amdgcn_perm(0u, 0x47544341u, t);  // 'A','C','T','G' by t
      const uint32_t bad = (x[i] & 0xDFDFDFDFu) ^ expect;                 // nonzero byte: not ACGTacgt
      nz[i] = (((bad & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | bad) & 0x80808080u;
      any |= nz[i];
      all &= nz[i];
      p[i] = t | (t >> 6);
    }
    const uint32_t q01 = __builtin_amdgcn_perm(p[1], p[0], 0x06040200u);  // bytes 0, 2 of p0 then of p1
    const uint32_t q23 = __builtin_amdgcn_perm(p[3], p[2], 0x06040200u);
    cols = __builtin_amdgcn_perm(q23 | (q23 >> 4), q01 | (q01 >> 4), 0x06040200u);
    if (any == 0u) {
      rst = 0u;
    } else if (all == 0x80808080u) {
      rst = 0xFFFFu;
    } else {
      rst = 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t v = nz[i];
        rst |= (((v >> 7) & 1u) | ((v >> 14) & 2u) | ((v >> 21) & 4u) | ((v >> 28) & 8u)) << (4 * i);
      }
    }
  }
  __device__ __forceinline__ uint32_t any_reset() const { return 1u; }  // checked per word
  __device__ __forceinline__ void load(const ScanArgs& a, uint64_t base) {
    const uint4* src = reinterpret_cast<const uint4*>(a.bases + base);
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = src[i];
  }
  __device__ void load_partial(const ScanArgs& a, uint64_t base) {
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const uint64_t b = base + 16 * w;
      if (b + 16 <= a.n) {
        r[w] = *reinterpret_cast<const uint4*>(a.bases + b);
      } else {
        uint32_t x[4] = {0, 0, 0, 0};
        for (uint64_t j = b; j < a.n && j < b + 16; ++j) x[(j - b) >> 2] |= (uint32_t)a.bases[j] << (8 * ((j - b) & 3));
        r[w] = make_uint4(x[0], x[1], x[2], x[3]);
      }
    }
  }
};

template <int ENC>
__device__ __forceinline__ void load_block(const ScanArgs& a, uint64_t base, Block<ENC>& b) {
  if (base + Block<ENC>::BASES <= a.n) b.load(a, base);
  else b.load_partial(a, base);
}

// 48 symbols (three words, no resets) as sixteen three-symbol lookups: the
// triples run across the word boundaries (bits 6j..6j+5 of w0 | w1 << 32 |
// w2 << 64).  Returns the state after the unit; `c` is nonzero when an
// accepting state was visited (the state is then not meaningful and the unit
// is replayed).
__device__ __forceinline__ uint32_t walk48(uint32_t s, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t& c) {
  uint32_t g[16];
#pragma unroll
  for (int j = 0; j < 5; ++j) g[j] = (w0 >> (6 * j)) & 63u;
  g[5] = __builtin_amdgcn_alignbit(w1, w0, 30) & 63u;
#pragma unroll
  for (int j = 6; j < 10; ++j) g[j] = (w1 >> (6 * j - 32)) & 63u;
  g[10] = __builtin_amdgcn_alignbit(w2, w1, 28) & 63u;
#pragma unroll
  for (int j = 11; j < 16; ++j) g[j] = (w2 >> (6 * j - 64)) & 63u;
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    s = lds_u16_at((s + g[j]) << 1);
    acc |= s;
  }
  c = acc & 1u;
  return s;
}

// Runs the words of block `b` (first base `base`) that hold bases in
// [lo, hi).  CHECKED = false promises the whole block lies in [lo, hi).  BLK
// is any register block with WORDS words and word(w, cols, rst).
template <class BLK, int SHIFT, int STEP, bool CHECKED, class Sink>
__device__ __forceinline__ uint32_t run_words(const Tab& tb, uint32_t s, const BLK& b, uint64_t base, uint64_t lo,
                                              uint64_t hi, Sink& sink) {
  constexpr int W = BLK::WORDS;
  constexpr int U = (STEP == 3 && !CHECKED) ? W / 3 : 0;  // whole 48-base units
#pragma unroll
  for (int u = 0; u < U; ++u) {
    uint32_t c0, r0, c1, r1, c2, r2;
    b.word(3 * u, c0, r0);
    b.word(3 * u + 1, c1, r1);
    b.word(3 * u + 2, c2, r2);
    const uint64_t p = base + 48 * u;
    // units without resets and units inside an N run take the same walk (the
    // latter end in q0 and report nothing), so lanes in N runs do not diverge
    const bool all_n = (r0 & r1 & r2) == 0xFFFFu;
    if ((r0 | r1 | r2) == 0u || all_n) {
      uint32_t f;
      const uint32_t e = walk48(s, c0, c1, c2, f);
      if (all_n) {
        s = tb.q0s;
      } else if (__builtin_expect(f != 0u, 0)) {  // matches in the unit: replay it base by base
        s = slow_word<SHIFT>(tb, s, c0, 0u, 0xFFFFu, p, sink);
        s = slow_word<SHIFT>(tb, s, c1, 0u, 0xFFFFu, p + 16, sink);
        s = slow_word<SHIFT>(tb, s, c2, 0u, 0xFFFFu, p + 32, sink);
      } else {
        s = e;
      }
    } else {
      s = run_word<SHIFT, STEP>(tb, s, c0, r0, p, sink);
      s = run_word<SHIFT, STEP>(tb, s, c1, r1, p + 16, sink);
      s = run_word<SHIFT, STEP>(tb, s, c2, r2, p + 32, sink);
    }
  }
#pragma unroll
  for (int w = 3 * U; w < W; ++w) {
    uint32_t cols, rst;
    b.word(w, cols, rst);
    const uint64_t p = base + 16 * w;
    if (CHECKED) {
      const uint64_t a0 = lo > p ? lo - p : 0;
      const uint64_t a1 = hi < p + 16 ? (hi > p ? hi - p : 0) : 16;
      if (a1 <= a0) continue;
      const uint32_t act = (0xFFFFu >> (16 - a1)) & ~((1u << a0) - 1u);
      if (act != 0xFFFFu) {
        s = slow_word<SHIFT>(tb, s, cols, rst, act, p, sink);
        continue;
      }
    }
    s = run_word<SHIFT, STEP>(tb, s, cols, rst, p, sink);
  }
  return s;
}

template <int ENC, int SHIFT, int STEP, bool CHECKED, class Sink>
__device__ __forceinline__ uint32_t run_block(const Tab& tb, uint32_t s, const Block<ENC>& b, uint64_t base,
                                              uint64_t lo, uint64_t hi, Sink& sink) {
  return run_words<Block<ENC>, SHIFT, STEP, CHECKED>(tb, s, b, base, lo, hi, sink);
}

// Scans [p, hi) from state s.  With HAS_FIRST, `first` already holds the
// block containing p.  Each middle block is loaded just before it is scanned.
template <int ENC, int SHIFT, int STEP, bool HAS_FIRST, class Sink>
__device__ __forceinline__ uint32_t scan_blocks(const ScanArgs& a, const Tab& tb, uint32_t s, uint64_t p,
                                                uint64_t hi, Sink& sink, const Block<ENC>& first) {
  using B = Block<ENC>;
  if (p >= hi) return s;
  uint64_t base = p / B::BASES * B::BASES;
  if constexpr (HAS_FIRST) {
    s = run_block<ENC, SHIFT, STEP, true>(tb, s, first, base, p, hi, sink);
  } else {
    B blk;
    load_block<ENC>(a, base, blk);
    s = run_block<ENC, SHIFT, STEP, true>(tb, s, blk, base, p, hi, sink);
  }
  base += B::BASES;
  for (; base + B::BASES <= hi; base += B::BASES) {
    B cur;
    if constexpr (ENC == ENC_2BIT) {
      // two blocks under one 128-byte line of N bits: the line is read once
      if ((base & (2 * B::BASES - 1)) == 0 && base + 2 * B::BASES <= hi && a.nmask) {
        uint32_t next_mask[B::MW];
        cur.load_pair_first(a, base, next_mask);
        s = run_block<ENC, SHIFT, STEP, false>(tb, s, cur, base, base, base + B::BASES, sink);
        base += B::BASES;
        B nx;
        nx.load_second(a, base, next_mask);
        s = run_block<ENC, SHIFT, STEP, false>(tb, s, nx, base, base, base + B::BASES, sink);
        continue;
      }
    }
    cur.load(a, base);
    s = run_block<ENC, SHIFT, STEP, false>(tb, s, cur, base, base, base + B::BASES, sink);
  }
  if (base < hi) {
    B blk;
    load_block<ENC>(a, base, blk);
    s = run_block<ENC, SHIFT, STEP, true>(tb, s, blk, base, base, hi, sink);
  }
  return s;
}

// [p, hi) with every block loaded here.
template <int ENC, int SHIFT, int STEP, class Sink>
__device__ __forceinline__ uint32_t scan_range(const ScanArgs& a, const Tab& tb, uint32_t s, uint64_t p, uint64_t hi,
                                               Sink& sink) {
  Block<ENC> unused;
  return scan_blocks<ENC, SHIFT, STEP, false>(a, tb, s, p, hi, sink, unused);
}

// Two ranges [p0, h0) and [p1, h1) (two chunks of one lane) from s0 and s1:
// each range's first block alone, then the whole blocks of both in lockstep
// with their lookups interleaved, then what is left of each range alone.
template <int ENC, int SHIFT, int STEP, class Sink>
__device__ __forceinline__ void scan_range2(const ScanArgs& a, const Tab& tb, uint32_t& s0, uint64_t p0, uint64_t h0,
                                            Sink& k0, uint32_t& s1, uint64_t p1, uint64_t h1, Sink& k1) {
  using B = Block<ENC>;
  constexpr int W = B::WORDS;
  uint64_t b0 = h0, b1 = h1;  // first base of the next whole block of each range
  if (p0 < h0) {
    b0 = p0 / B::BASES * B::BASES;
    B blk;
    load_block<ENC>(a, b0, blk);
    s0 = run_block<ENC, SHIFT, STEP, true>(tb, s0, blk, b0, p0, h0, k0);
    b0 += B::BASES;
  }
  if (p1 < h1) {
    b1 = p1 / B::BASES * B::BASES;
    B blk;
    load_block<ENC>(a, b1, blk);
    s1 = run_block<ENC, SHIFT, STEP, true>(tb, s1, blk, b1, p1, h1, k1);
    b1 += B::BASES;
  }
  for (; b0 + B::BASES <= h0 && b1 + B::BASES <= h1; b0 += B::BASES, b1 += B::BASES) {
    B x0, x1;
    x0.load(a, b0);
    x1.load(a, b1);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      uint32_t c0, r0, c1, r1;
      x0.word(w, c0, r0);
      x1.word(w, c1, r1);
      run_word2<SHIFT, STEP>(tb, s0, c0, r0, b0 + 16 * w, k0, s1, c1, r1, b1 + 16 * w, k1);
    }
  }
  for (; b0 < h0; b0 += B::BASES) {
    B blk;
    load_block<ENC>(a, b0, blk);
    s0 = run_block<ENC, SHIFT, STEP, true>(tb, s0, blk, b0, b0, h0, k0);
  }
  for (; b1 < h1; b1 += B::BASES) {
    B blk;
    load_block<ENC>(a, b1, blk);
    s1 = run_block<ENC, SHIFT, STEP, true>(tb, s1, blk, b1, b1, h1, k1);
  }
}

// ------------------------------------------------------------------ chunk headers
// The 8 bases before `lo` (lo >= 8): table columns two bits per base (oldest
// first), A,C,G,T codes the same way, and a reset bit per base.
template <int ENC>
__device__ __forceinline__ void lookback8(const ScanArgs& a, uint64_t lo, uint32_t& cols, uint32_t& codes,
                                          uint32_t& rst) {
  if constexpr (ENC == ENC_2BIT) {
    if ((lo & 7) == 0) {
      cols = *reinterpret_cast<const uint16_t*>(a.bases + ((lo - 8) >> 2));
      rst = a.nmask ? a.nmask[(lo - 8) >> 3] : 0u;
      codes = cols;
      return;
    }
  } else {
    if ((lo & 7) == 0) {
      const uint2 v = *reinterpret_cast<const uint2*>(a.bases + lo - 8);
      const uint32_t x[2] = {v.x, v.y};
      cols = codes = rst = 0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint32_t b = (x[i >> 2] >> (8 * (i & 3))) & 0xFFu;
        const uint32_t t = (b >> 1) & 3u;
        const uint32_t expect = (0x47544341u >> (8u * t)) & 0xFFu;
        rst |= (uint32_t)((b & 0xDFu) != expect) << i;
        cols |= t << (2 * i);
        codes |= (t ^ (t >> 1)) << (2 * i);
      }
      return;
    }
  }
  cols = codes = rst = 0;
  for (int i = 0; i < 8; ++i) {
    const int col = load_col<ENC>(a, lo - 8 + i);
    if (col < 0) rst |= 1u << i;
    else {
      cols |= (uint32_t)col << (2 * i);
      codes |= col_to_code<ENC>((uint32_t)col) << (2 * i);
    }
  }
}

// First base of chunk c (buffer position): chunks are counted from the
// sequence's first base.
__device__ __forceinline__ uint64_t chunk_lo(const ScanArgs& a, uint64_t c) { return a.first + c * a.chunk; }

// Candidate list of the chunk starting at lo: either one exact state (chunk
// 0, a reset inside the lookback window, or a window that reaches the
// sequence start) or the PSS table entry of the k-gram before the chunk.
template <int ENC, int SHIFT>
__device__ __forceinline__ void chunk_header(const ScanArgs& a, const Tab& tb, const uint32_t* pss_off, uint64_t lo,
                                             uint32_t& m, uint32_t& cbase, uint32_t& exact, bool& is_exact) {
  m = 1;
  cbase = 0;
  exact = tb.q0s;
  is_exact = true;
  if (lo == a.first) return;
  const uint32_t k = a.k;
  if (lo - a.first < 8) {  // the window reaches the sequence start: run from q0
    uint32_t s = tb.q0s;
    for (uint64_t i = a.first; i < lo; ++i) {
      const int col = load_col<ENC>(a, i);
      s = col < 0 ? tb.q0s : (t1_lookup<SHIFT>(tb, s, (uint32_t)col) & 0xFFFFu);
    }
    exact = s;
    return;
  }
  uint32_t cols, codes, rst;
  lookback8<ENC>(a, lo, cols, codes, rst);
  const uint32_t sh = 8 - k;  // window = the last k of the 8 bases
  const uint32_t wr = (rst >> sh) & ((1u << k) - 1u);
  if (wr) {  // a reset inside the window: the state is exact after it
    uint32_t s = tb.q0s;
    for (uint32_t i = sh; i < 8; ++i)
      s = ((rst >> i) & 1u) ? tb.q0s : (t1_lookup<SHIFT>(tb, s, (cols >> (2 * i)) & 3u) & 0xFFFFu);
    exact = s;
    return;
  }
  const uint32_t idx = (codes >> (2 * sh)) & ((k == 16 ? 0u : (1u << (2 * k))) - 1u);
  is_exact = false;
  cbase = pss_off[idx];
  m = pss_off[idx + 1] - cbase;
}

}  // namespace coex
