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
//   Column order is the encoding's natural one: A,C,G,T for 2-bit codes and
//   A,C,T,G for bytes ((byte >> 1) & 3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace coex {

constexpr int ENC_BYTE = 0;
constexpr int ENC_2BIT = 1;
constexpr uint32_t NONCONV = 0xFFFFFFFFu;
constexpr int TILE = 64;          // chunks per wave
constexpr int SPEC_WIN = 64;      // symbols examined for convergence

struct ScanArgs {
  // sequence
  const uint8_t* bases;
  const uint8_t* nmask;
  uint64_t n;
  uint64_t chunk;
  uint64_t n_chunks;
  uint64_t n_tiles;
  // tables (global copies)
  const uint32_t* T2;
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
  // per-chunk outputs
  uint32_t* conv_t;           // symbols consumed to the converging point, NONCONV if none
  uint32_t* conv_s;           // state there
  uint32_t* end_s;            // state at the chunk end (converged chunks)
  uint32_t* tail_cnt;         // matches in [conv_t, end)
  uint32_t* nc_count;         // number of non-converged chunks
  uint32_t* nc_chunk;         // slot -> chunk
  uint32_t* nc_slot;          // chunk -> slot
  uint32_t* nc_m;             // slot -> number of candidates
  uint32_t* nc_cand;          // slot * max_cand + i -> candidate state
  uint32_t* nc_end;           // slot * max_cand + i -> end state from that candidate
  uint32_t* true_start;       // n_chunks + 1
  unsigned long long* visits; // per accepting index
  unsigned long long* total;  // weighted total
  uint64_t* chunk_cnt;        // per chunk total (find / records)
  uint32_t* err;              // device consistency flag
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
};

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
  const uint32_t* w;    // weight per accepting index
  uint32_t cnt = 0;
  __device__ void word(uint32_t c) { cnt += c; }
  __device__ void hit(uint64_t, uint32_t a) { cnt += w[a]; }
};

struct SinkHist {       // per accepting state visits in an LDS histogram
  static constexpr bool kReplay = true;
  const uint32_t* w;
  uint32_t* hist;
  uint32_t cnt = 0;
  __device__ void word(uint32_t) {}
  __device__ void hit(uint64_t, uint32_t a) {
    cnt += w[a];
    atomicAdd(hist + a, 1u);
  }
};

struct SinkGlobal {     // weighted count, and visits straight to global memory
  static constexpr bool kReplay = true;
  const uint32_t* w;
  unsigned long long* visits;  // NULL: count only
  uint32_t cnt = 0;
  __device__ void word(uint32_t) {}
  __device__ void hit(uint64_t, uint32_t a) {
    cnt += w[a];
    if (visits) atomicAdd(visits + a, 1ull);
  }
};

struct SinkPositions {  // end positions and pattern ids, in order
  static constexpr bool kReplay = true;
  const uint32_t* out_off;   // per accepting index
  const uint32_t* out_ids;
  int64_t* pos;
  uint32_t* pat;
  uint64_t at;
  uint64_t cap;              // writes stop at the buffer end whatever the count
  uint32_t cnt = 0;
  __device__ void word(uint32_t) {}
  __device__ void hit(uint64_t p, uint32_t a) {
    for (uint32_t i = out_off[a]; i < out_off[a + 1]; ++i) {
      if (at < cap) {
        pos[at] = (int64_t)p;
        if (pat) pat[at] = out_ids[i];
      }
      ++at;
      ++cnt;
    }
  }
};

struct SinkRecord {     // per chunk, per pattern counts
  static constexpr bool kReplay = true;
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

// 16 symbols of one word, one at a time (resets honoured).
template <int SHIFT, class Sink>
__device__ __forceinline__ uint32_t word_slow(const Tab& tb, uint32_t s, uint32_t cols, uint32_t rst, uint64_t p,
                                              Sink& sink) {
#pragma unroll 1
  for (int i = 0; i < 16; ++i) {
    int col = ((rst >> i) & 1u) ? -1 : (int)((cols >> (2 * i)) & 3u);
    s = step1<SHIFT>(tb, s, col, p + i, sink);
  }
  return s;
}

// 16 symbols without resets: eight two-symbol lookups (STEP 2), or sixteen
// one-symbol lookups; a word with matches is replayed one symbol at a time
// when the sink needs per-position detail.
template <int SHIFT, int STEP, class Sink>
__device__ __forceinline__ uint32_t word_fast(const Tab& tb, uint32_t s, uint32_t cols, uint64_t p, Sink& sink) {
  static_assert(STEP == 1 || SHIFT == 6, "two-symbol tables need 64-byte rows");
  const uint32_t s0 = s;
  if constexpr (STEP == 2) {
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t e = t2_lookup(tb, s, (cols >> (4 * j)) & 15u);
      s = e & 0xFFFFu;
      acc += e;
    }
    uint32_t c = acc >> 24;
    if constexpr (Sink::kReplay) {
      if (c) word_slow<SHIFT>(tb, s0, cols, 0u, p, sink);
    } else {
      sink.word(c);
    }
  } else {
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      uint32_t e = t1_lookup<SHIFT>(tb, s, (cols >> (2 * j)) & 3u);
      s = e & 0xFFFFu;
      acc |= e;
    }
    if (acc >> 16) word_slow<SHIFT>(tb, s0, cols, 0u, p, sink);
  }
  return s;
}

// Scans [p, hi) from state s, reporting matches to the sink; returns the
// state after base hi-1.  Single bases until p is 16-aligned, whole words
// until the block boundary, whole blocks (128 bytes of sequence per lane and
// load), then words and single bases again.
template <int ENC, int SHIFT, int STEP, class Sink>
__device__ __forceinline__ uint32_t scan_range(const ScanArgs& a, const Tab& tb, uint32_t s, uint64_t p, uint64_t hi, Sink& sink) {
  constexpr uint64_t BLOCK = (ENC == ENC_2BIT) ? 512 : 128;
  while (p < hi && (p & 15)) {
    s = step1<SHIFT>(tb, s, load_col<ENC>(a, p), p, sink);
    ++p;
  }
  while (p + 16 <= hi && (p & (BLOCK - 1))) {
    uint32_t cols, rst;
    load_word<ENC>(a, p, cols, rst);
    s = rst ? word_slow<SHIFT>(tb, s, cols, rst, p, sink) : word_fast<SHIFT, STEP>(tb, s, cols, p, sink);
    p += 16;
  }
  while (p + BLOCK <= hi) {
    if constexpr (ENC == ENC_2BIT) {
      const uint4* src = reinterpret_cast<const uint4*>(a.bases + (p >> 2));
      uint4 v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = src[i];
      uint4 m[4] = {};
      uint32_t any = 0;
      if (a.nmask) {
        const uint4* ms = reinterpret_cast<const uint4*>(a.nmask + (p >> 3));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          m[i] = ms[i];
          any |= m[i].x | m[i].y | m[i].z | m[i].w;
        }
      }
      const uint32_t vw[32] = {v[0].x, v[0].y, v[0].z, v[0].w, v[1].x, v[1].y, v[1].z, v[1].w,
                               v[2].x, v[2].y, v[2].z, v[2].w, v[3].x, v[3].y, v[3].z, v[3].w,
                               v[4].x, v[4].y, v[4].z, v[4].w, v[5].x, v[5].y, v[5].z, v[5].w,
                               v[6].x, v[6].y, v[6].z, v[6].w, v[7].x, v[7].y, v[7].z, v[7].w};
      if (!any) {
#pragma unroll
        for (int w = 0; w < 32; ++w) s = word_fast<SHIFT, STEP>(tb, s, vw[w], p + 16 * w, sink);
      } else {
        const uint32_t mw[16] = {m[0].x, m[0].y, m[0].z, m[0].w, m[1].x, m[1].y, m[1].z, m[1].w,
                                 m[2].x, m[2].y, m[2].z, m[2].w, m[3].x, m[3].y, m[3].z, m[3].w};
#pragma unroll
        for (int w = 0; w < 32; ++w) {
          uint32_t r = (mw[w >> 1] >> (16 * (w & 1))) & 0xFFFFu;
          s = r ? word_slow<SHIFT>(tb, s, vw[w], r, p + 16 * w, sink)
                : word_fast<SHIFT, STEP>(tb, s, vw[w], p + 16 * w, sink);
        }
      }
    } else {
#pragma unroll 2
      for (int w = 0; w < 8; ++w) {
        uint32_t cols, rst;
        load_word<ENC>(a, p + 16 * w, cols, rst);
        s = rst ? word_slow<SHIFT>(tb, s, cols, rst, p + 16 * w, sink)
                : word_fast<SHIFT, STEP>(tb, s, cols, p + 16 * w, sink);
      }
    }
    p += BLOCK;
  }
  while (p + 16 <= hi) {
    uint32_t cols, rst;
    load_word<ENC>(a, p, cols, rst);
    s = rst ? word_slow<SHIFT>(tb, s, cols, rst, p, sink) : word_fast<SHIFT, STEP>(tb, s, cols, p, sink);
    p += 16;
  }
  while (p < hi) {
    s = step1<SHIFT>(tb, s, load_col<ENC>(a, p), p, sink);
    ++p;
  }
  return s;
}

}  // namespace coex
