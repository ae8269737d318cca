// libcoex batched scans: many (sequence, automaton) pairs in one persistent
// launch, for a batch of uneven sequences crossed with a set of resident
// automata (or any list of pairs, as a serving loop forms them).
//
// The method per pair is the paper's (Section III, Algorithm 1): the sequence
// is cut into chunks; a chunk's possible starting states come from the k
// bases before it (Section III.A with a k-base lookback); the candidate runs
// advance in lockstep until they agree (the converging point,
// Section III.B.3); the rest of the chunk is scanned once from there; the
// join takes each chunk's true first state from its predecessor's last
// state; the counts before the converging point are fixed up when the
// candidates disagree on them.
//
// Layout on the GPU (one launch of k_bscan does all pairs):
//   - automata are packed into LDS groups: the rows of every automaton of a
//     group sit in one LDS image whose entries are absolute row offsets, so a
//     lane's state register addresses its own automaton's rows directly;
//     two-symbol rows (64 B) when every automaton's counts fit them, else
//     one-symbol rows (16 B);
//   - a lane owns one (chunk, automaton) pair; a wave holds one automaton
//     over 64 consecutive chunks, and the waves of a span hold the other
//     automata of the group over the same chunks, so a chunk is read from
//     HBM about once for all automata of its group (the other waves find its
//     lines in cache) while each wave walks a single table;
//   - blocks are persistent and take 768-lane tasks from a device counter;
//     a block restages LDS only when its task moves to another group.
// k_bcompose resolves chunks whose candidates never agreed (only automata
// without a finite synchronising depth, or one longer than the chunk), and
// k_bfix recounts the prefixes whose candidate counts differed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "coex.h"
#include "dfa.hpp"
#include "kernels.hpp"

namespace coex {
namespace batch {

constexpr int kBlock = COEX_SCAN_BLOCK;
constexpr uint32_t kPad = 0xFFFFFFFFu;      // pair slot without an automaton
constexpr uint32_t kGroupStates2 = 960;     // two-symbol rows (64 B, 16-bit row offsets) + one-symbol rows in LDS
constexpr uint32_t kGroupStates1 = 4096;    // one-symbol rows: 16-bit row offsets of 16 B rows

struct SeqD {
  const uint8_t* bases;
  const uint8_t* nmask;
  uint64_t n;
};
struct DfaD {
  uint32_t base;      // state register value of state 0 (its row offset in the group image)
  uint32_t q0s;       // state register value of q0
  uint32_t k;         // lookback of the possible-starting-state table
  uint32_t group;
  const uint32_t* pss_off;
  const uint16_t* pss_states;
};
struct EntryD {       // one sequence with the automata of one group paired to it
  uint32_t seq;
  uint32_t slot0;     // first of the group's D pair slots
  uint32_t n_chunks;
  uint32_t unit0;     // first unit (global index)
};
struct UnitD {
  uint32_t entry;
  uint32_t chunk;
};
struct GroupD {
  uint64_t lane0;     // first lane of the launch
  uint64_t n_lanes;   // units * D
  uint64_t unit0;     // first unit
  uint64_t n_units;
  uint32_t task0;     // first block task
  uint32_t D;         // pair slots per entry
  uint32_t tab_bytes; // LDS image bytes
  uint32_t step;      // symbols per LDS lookup (2: 64 B rows, state = row offset; 1: 16 B rows)
  uint32_t t1_lds_off;  // two-symbol groups: LDS offset of the one-symbol rows staged after the image
  uint32_t t1_bytes;    // 0 for one-symbol groups (their image is the one-symbol rows)
  const uint32_t* tab;   // LDS image
  const uint32_t* t1;    // one-symbol rows in global memory, same register values
  const uint32_t* wtab;  // weight (patterns) per accepting index of the group
};
struct Args {
  const SeqD* seqs;
  const DfaD* dfas;
  const EntryD* entries;
  const UnitD* units;
  const GroupD* groups;
  const uint32_t* slot_dfa;
  const uint32_t* slot_out;
  const uint32_t* slot_entry;
  uint32_t n_groups, n_tasks, n_slots, bcast_off;
  uint64_t chunk;
  unsigned long long* counts;
  uint32_t n_counts;
  uint32_t* task_ctr;
  uint32_t* fix_count;
  uint32_t* fix_list;
  uint32_t* err;
  uint32_t* rec_t;     // symbols to the converging point, NONCONV if the candidates never agreed
  uint32_t* rec_s;     // converged state
  uint32_t* rec_end;   // state at the chunk end
  uint32_t* rec_tail;  // matches after the converging point
  uint32_t* rec_ts;    // true first state (written by k_bcompose)
  uint32_t max_cand;   // largest candidate list of any automaton
  uint32_t nc_stride;  // entries per lane in the arrays below
  uint32_t* nc_m;      // non-converged chunks: candidates, their end states and counts
  uint32_t* nc_init;
  uint32_t* nc_end;
  uint32_t* nc_cnt;
};

__device__ __forceinline__ void stage(char* dst, const void* src, uint32_t bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  for (uint32_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

__global__ void k_binit(Args A) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *A.task_ctr = 0;
    *A.fix_count = 0;
    *A.err = 0;
  }
  for (uint32_t i = t; i < A.n_counts; i += gridDim.x * blockDim.x) A.counts[i] = 0;
}

constexpr int W = 8;  // candidate registers per lane

// Lanes of a group come in spans of 64 * D: in a span, the 64 lanes of slot
// j hold 64 consecutive units, so one wave walks one automaton's table
// (lanes often share rows) while the D waves of a span read the same
// sequence bytes, mostly from cache.
__host__ __device__ __forceinline__ uint64_t lane_of(uint64_t u, uint32_t j, uint32_t D) {
  return (u / 64) * 64 * D + (uint64_t)j * 64 + (u % 64);
}
__device__ __forceinline__ void unit_of(uint64_t L, uint32_t D, uint64_t& u, uint32_t& j) {
  const uint64_t span = 64ull * D;
  const uint64_t r = L % span;
  j = (uint32_t)(r / 64);
  u = (L / span) * 64 + (r % 64);
}

// Byte sequences are converted once per run to 2-bit codes and an N mask
// (the encoding of the genome scan): every automaton of a chunk then reads
// 0.375 B/base with no per-lane decoding.
struct ConvArgs {
  const SeqD* src;        // byte sequences
  const SeqD* dst;        // their 2-bit copies (codes, mask, n)
  const uint64_t* prefix; // n_seq + 1: first 64-base group of each sequence
  uint32_t n_seq;
  uint64_t total;         // 64-base groups in all
};

__global__ __launch_bounds__(256) void k_bconvert(ConvArgs C) {
  // each block converts one contiguous run of groups; a thread's groups are
  // 256 apart, so the index of the sequence holding them only moves forward
  const uint64_t per_block = (C.total + gridDim.x - 1) / gridDim.x;
  const uint64_t g0 = (uint64_t)blockIdx.x * per_block;
  const uint64_t g1 = g0 + per_block < C.total ? g0 + per_block : C.total;
  uint32_t lo = 0;  // last sequence whose first group is <= g
  if (g0 + threadIdx.x < g1) {
    uint32_t hi = C.n_seq;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (C.prefix[mid] <= g0 + threadIdx.x) lo = mid;
      else hi = mid;
    }
  }
  for (uint64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
    while (lo + 1 < C.n_seq && C.prefix[lo + 1] <= g) ++lo;
    const SeqD in = C.src[lo], out = C.dst[lo];
    const uint64_t base = (g - C.prefix[lo]) * 64;
    uint32_t x[16];
    if (base + 64 <= in.n) {
      const uint4* src = reinterpret_cast<const uint4*>(in.bases + base);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint4 v = src[i];
        x[4 * i] = v.x; x[4 * i + 1] = v.y; x[4 * i + 2] = v.z; x[4 * i + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = 0x41414141u;  // past the end: never read by the scan
      for (uint64_t j = base; j < in.n; ++j) {
        const uint32_t k = (uint32_t)(j - base);
        x[k >> 2] = (x[k >> 2] & ~(0xFFu << (8 * (k & 3)))) | ((uint32_t)in.bases[j] << (8 * (k & 3)));
      }
    }
    uint32_t codes[4];
    uint64_t rst = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t cw = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t v = x[4 * w + i];
        const uint32_t t = (v >> 1) & 0x03030303u;                      // table column A,C,T,G
        const uint32_t expect = __builtin_amdgcn_perm(0u, 0x47544341u, t);
        const uint32_t bad = (v & 0xDFDFDFDFu) ^ expect;                 // nonzero byte: not ACGTacgt
        const uint32_t code = t ^ ((t >> 1) & 0x01010101u);              // A,C,G,T = 0..3
        const uint32_t u = code | (code >> 6);
        cw |= ((u & 0xFu) | ((u >> 12) & 0xF0u)) << (8 * i);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          rst |= (uint64_t)(((bad >> (8 * j)) & 0xFFu) != 0u) << (16 * w + 4 * i + j);
      }
      codes[w] = cw;
    }
    *reinterpret_cast<uint4*>(const_cast<uint8_t*>(out.bases) + base / 4) = make_uint4(codes[0], codes[1], codes[2], codes[3]);
    *reinterpret_cast<uint2*>(const_cast<uint8_t*>(out.nmask) + base / 8) = make_uint2((uint32_t)rst, (uint32_t)(rst >> 32));
  }
}

// One symbol for the active candidate slots; returns whether all slots
// below n now hold the same state.
template <int ENC, int SHIFT>
__device__ __forceinline__ bool step_slots(const Tab& tg, const uint32_t* wtab, uint32_t q0s, int col, uint32_t n,
                                           uint32_t lo_slot, uint32_t (&cand)[W], uint32_t (&pc)[W]) {
  bool same = true;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    if (i < (int)n && i >= (int)lo_slot) {
      uint32_t s2 = q0s;
      if (col >= 0) {
        const uint32_t e = t1_lookup<SHIFT>(tg, cand[i], (uint32_t)col);
        s2 = e & 0xFFFFu;
        if (e >> 16) pc[i] += wtab[(e >> 16) - 1u];
      }
      cand[i] = s2;
    }
    if (i < (int)n) same = same && cand[i] == cand[0];
  }
  return same;
}

// One (chunk, automaton) pair: candidates, lockstep speculation, the scan
// after the converging point, and the chunk's records.
//
// The candidates run in batches of at most 8 registers.  The first batch
// runs from the chunk start until its states agree (the converging point
// of those runs); that state becomes the representative of every candidate
// seen so far and takes slot 0 of the next batch, which runs its new
// candidates from the chunk start and the representative from its
// converging point on, until all agree again.  After the last batch every
// candidate's run has reached one state: the chunk's converging point.
// Counts: the candidates agree on the prefix count iff every batch's slots
// agreed at its converging point (counts after a common state are common).
template <int ENC, int SHIFT, int STEP>
__device__ __forceinline__ void lane_scan(const Args& A, const GroupD& G, const char* lds, uint64_t gl, uint64_t L) {
  uint64_t ul;
  uint32_t j;
  unit_of(L, G.D, ul, j);
  if (ul >= G.n_units) return;  // padding of the last span
  const UnitD un = A.units[G.unit0 + ul];
  const EntryD en = A.entries[un.entry];
  const uint32_t slot = en.slot0 + j;
  const uint32_t d = A.slot_dfa[slot];
  if (d == kPad) return;
  const DfaD df = A.dfas[d];
  const SeqD sq = A.seqs[en.seq];
  ScanArgs sa{};
  sa.bases = sq.bases;
  sa.nmask = sq.nmask;
  sa.n = sq.n;
  sa.k = df.k;
  const uint64_t lo = (uint64_t)un.chunk * A.chunk;
  const uint64_t hi = (un.chunk + 1 == en.n_chunks) ? sq.n : lo + A.chunk;
  // one-symbol rows in LDS (after the two-symbol image, or the image itself)
  const char* t1l = STEP == 2 ? lds + G.t1_lds_off : lds;
  const Tab tg{nullptr, t1l, df.q0s};
  uint32_t m, cbase, exact;
  bool is_exact;
  chunk_header<ENC, SHIFT>(sa, tg, df.pss_off, lo, m, cbase, exact, is_exact);
  if (m == 0 || m > A.max_cand) {
    atomicOr(A.err, 1u);
    return;
  }
  uint32_t rep = exact, rep_cnt = 0;
  uint64_t T = lo;
  bool have_rep = is_exact, eq = true, conv = true;
  for (uint32_t next = is_exact ? m : 0u; next < m;) {
    const uint32_t off = have_rep ? 1u : 0u;
    const uint32_t k = min(m - next, (uint32_t)W - off);
    const uint32_t n = k + off;
    uint32_t cand[W], pc[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
      cand[i] = 0;
      pc[i] = 0;
      if (i < (int)off) {
        cand[i] = rep;
        pc[i] = rep_cnt;
      } else if (i < (int)n) {
        cand[i] = df.base + ((uint32_t)df.pss_states[cbase + next + (uint32_t)i - off] << SHIFT);
      }
    }
    uint64_t p = lo;
    conv = n == 1;  // a single run is its own converging point
    // new candidates alone up to the representative's position
    for (; p < T; ++p) step_slots<ENC, SHIFT>(tg, G.wtab, df.q0s, load_col<ENC>(sa, p), n, off, cand, pc);
    while (!conv && p < hi) {
      conv = step_slots<ENC, SHIFT>(tg, G.wtab, df.q0s, load_col<ENC>(sa, p), n, 0u, cand, pc);
      ++p;
    }
    if (!conv) break;
#pragma unroll
    for (int i = 1; i < W; ++i)
      if (i < (int)n) eq = eq && pc[i] == pc[0];
    rep = cand[0];
    rep_cnt = pc[0];
    T = p;
    have_rep = true;
    next += k;
  }
  if (!conv && !A.nc_m) {  // cannot happen when the chunk exceeds every synchronising depth
    atomicOr(A.err, 8u);
    A.rec_t[gl] = 0;
    A.rec_end[gl] = rep;
    return;
  }
  if (!conv) {  // the chunk's state map on its candidates: each run to the chunk end
    A.rec_t[gl] = NONCONV;
    A.nc_m[gl] = m;
    for (uint32_t next = 0; next < m; next += W) {
      const uint32_t n = min(m - next, (uint32_t)W);
      uint32_t cand[W], pc[W];
#pragma unroll
      for (int i = 0; i < W; ++i) {
        pc[i] = 0;
        cand[i] = i < (int)n ? df.base + ((uint32_t)df.pss_states[cbase + next + (uint32_t)i] << SHIFT) : 0u;
      }
      for (uint64_t p = lo; p < hi; ++p) step_slots<ENC, SHIFT>(tg, G.wtab, df.q0s, load_col<ENC>(sa, p), n, 0u, cand, pc);
#pragma unroll
      for (int i = 0; i < W; ++i) {
        if (i < (int)n) {
          const uint64_t x = gl * A.nc_stride + next + i;
          A.nc_init[x] = df.base + ((uint32_t)df.pss_states[cbase + next + (uint32_t)i] << SHIFT);
          A.nc_end[x] = cand[i];
          A.nc_cnt[x] = pc[i];
        }
      }
    }
    return;
  }
  const Tab tb{lds, t1l, df.q0s};
  SinkTotal sink{G.wtab};
  const uint32_t e_end = scan_range<ENC, SHIFT, STEP>(sa, tb, rep, T, hi, sink);
  A.rec_end[gl] = e_end;
  A.rec_t[gl] = (uint32_t)(T - lo);
  if (eq) {
    const uint64_t tot = (uint64_t)rep_cnt + sink.cnt;
    if (tot) atomicAdd(A.counts + A.slot_out[slot], (unsigned long long)tot);
  } else {
    A.rec_s[gl] = rep;
    A.rec_tail[gl] = sink.cnt;
    A.fix_list[atomicAdd(A.fix_count, 1u)] = (uint32_t)gl;
  }
}

// Persistent scan: every block takes 768-lane tasks until the counter passes
// the last one (every wave reaches the exit).  LDS holds the group image at
// address 0 and one broadcast word after it.
template <int ENC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(COEX_TAIL_WAVES, 8))) void k_bscan(Args A) {
  extern __shared__ __align__(16) char lds[];
  uint32_t* bc = reinterpret_cast<uint32_t*>(lds + A.bcast_off);
  if (threadIdx.x == 0 && (uint32_t)(uintptr_t)(lds_c*)lds != 0u) atomicOr(A.err, 64u);
  int staged = -1;
  for (;;) {
    if (threadIdx.x == 0) bc[0] = atomicAdd(A.task_ctr, 1u);
    __syncthreads();
    const uint32_t task = bc[0];
    if (task >= A.n_tasks) break;
    uint32_t g = 0;
    while (g + 1 < A.n_groups && A.groups[g + 1].task0 <= task) ++g;
    GroupD G = A.groups[g];
    // group fields are uniform over the block: keep them in scalar registers
    G.D = __builtin_amdgcn_readfirstlane(G.D);
    G.step = __builtin_amdgcn_readfirstlane(G.step);
    G.t1_lds_off = __builtin_amdgcn_readfirstlane(G.t1_lds_off);
    G.t1_bytes = __builtin_amdgcn_readfirstlane(G.t1_bytes);
    G.unit0 = uniform64(G.unit0);
    G.lane0 = uniform64(G.lane0);
    G.n_lanes = uniform64(G.n_lanes);
    G.n_units = uniform64(G.n_units);
    G.t1 = reinterpret_cast<const uint32_t*>(uniform64(reinterpret_cast<uint64_t>(G.t1)));
    G.wtab = reinterpret_cast<const uint32_t*>(uniform64(reinterpret_cast<uint64_t>(G.wtab)));
    if ((int)g != staged) {
      stage(lds, G.tab, G.tab_bytes);
      if (G.t1_bytes) stage(lds + G.t1_lds_off, G.t1, G.t1_bytes);
      staged = (int)g;
    }
    __syncthreads();
    const uint64_t L = (uint64_t)(task - G.task0) * kBlock + threadIdx.x;
    if (L < G.n_lanes) {
      if (G.step == 2) lane_scan<ENC, 6, 2>(A, G, lds, G.lane0 + L, L);
      else lane_scan<ENC, 4, 1>(A, G, lds, G.lane0 + L, L);
    }
    __syncthreads();
  }
}

// The join for pairs with non-converged chunks: one thread per pair slot
// walks its chunks in order, picking each non-converged chunk's map entry
// for the true first state and recording the true first state of the
// others for the fix-up.
__global__ void k_bcompose(Args A) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= A.n_slots) return;
  const uint32_t d = A.slot_dfa[x];
  if (d == kPad) return;
  const DfaD df = A.dfas[d];
  const EntryD en = A.entries[A.slot_entry[x]];
  const GroupD G = A.groups[df.group];
  const uint32_t j = x - en.slot0;
  uint32_t q = df.q0s;
  unsigned long long add = 0;
  for (uint32_t c = 0; c < en.n_chunks; ++c) {
    const uint64_t gl = G.lane0 + lane_of((uint64_t)(en.unit0 - G.unit0 + c), j, G.D);
    if (A.rec_t[gl] == NONCONV) {
      const uint32_t m = A.nc_m[gl];
      uint32_t i = 0;
      const uint64_t b0 = gl * A.nc_stride;
      while (i < m && A.nc_init[b0 + i] != q) ++i;
      if (i == m) {
        atomicOr(A.err, 4u);
        return;
      }
      add += A.nc_cnt[b0 + i];
      q = A.nc_end[b0 + i];
    } else {
      A.rec_ts[gl] = q;
      q = A.rec_end[gl];
    }
  }
  if (add) atomicAdd(A.counts + A.slot_out[x], add);
}

// Prefix recount of the chunks whose candidates disagreed on the count
// before the converging point: from the true first state (the predecessor's
// last state) to the converging point, which it must reach.
template <int ENC>
__global__ void k_bfix(Args A) {
  const uint32_t nf = *A.fix_count;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x) {
    const uint32_t gl = A.fix_list[i];
    uint32_t g = 0;
    while (g + 1 < A.n_groups && A.groups[g + 1].lane0 <= gl) ++g;
    const GroupD G = A.groups[g];
    const uint64_t L = gl - G.lane0;
    uint64_t ul;
    uint32_t j;
    unit_of(L, G.D, ul, j);
    const UnitD un = A.units[G.unit0 + ul];
    const EntryD en = A.entries[un.entry];
    const uint32_t slot = en.slot0 + j;
    const DfaD df = A.dfas[A.slot_dfa[slot]];
    const SeqD sq = A.seqs[en.seq];
    ScanArgs sa{};
    sa.bases = sq.bases;
    sa.nmask = sq.nmask;
    sa.n = sq.n;
    const char* t1 = reinterpret_cast<const char*>(G.t1);
    const uint32_t sh = G.step == 2 ? 2u : 0u;  // state register -> one-symbol row offset
    const uint64_t prev = G.lane0 + lane_of(ul - 1, j, G.D);  // the same entry's previous chunk
    uint32_t q = A.rec_t[prev] == NONCONV ? A.rec_ts[gl] : A.rec_end[prev];
    const uint64_t lo = (uint64_t)un.chunk * A.chunk;
    const uint32_t t = A.rec_t[gl];
    uint32_t cnt = 0;
    for (uint32_t s = 0; s < t; ++s) {
      const int col = load_col<ENC>(sa, lo + s);
      if (col < 0) {
        q = df.q0s;
        continue;
      }
      const uint32_t e = *reinterpret_cast<const uint32_t*>(t1 + (q >> sh) + (uint32_t)col * 4u);
      q = e & 0xFFFFu;
      if (e >> 16) cnt += G.wtab[(e >> 16) - 1u];
    }
    if (q != A.rec_s[gl]) atomicOr(A.err, 2u);
    const uint64_t tot = (uint64_t)cnt + A.rec_tail[gl];
    if (tot) atomicAdd(A.counts + A.slot_out[slot], (unsigned long long)tot);
  }
}

// ====================================================================== host
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

const int kOrd2bit[4] = {0, 1, 2, 3};  // column j holds the successor on code ord[j]
const int kOrdByte[4] = {0, 1, 3, 2};

struct DevBuf {
  char* p = nullptr;
  size_t bytes = 0;
  int device = -1;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      int cur = -1;
      if (hipGetDevice(&cur) == hipSuccess && cur != device) (void)hipSetDevice(device);
      (void)hipFree(p);
      if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    }
    p = nullptr;
    bytes = 0;
  }
  int reserve(size_t want, int dev) {
    if (bytes >= want && device == dev) return COEX_OK;
    release();
    want = std::max<size_t>(want, 4096);
    if (hipMalloc(&p, want) != hipSuccess) { p = nullptr; return COEX_ENOMEM; }
    bytes = want;
    device = dev;
    return COEX_OK;
  }
};

// Host image assembled part by part, then copied to one device buffer.
struct Image {
  std::vector<char> host;
  size_t add(const void* src, size_t bytes) {
    const size_t off = host.size();
    host.resize(align_up(off + std::max<size_t>(bytes, 16), 256), 0);
    if (bytes) std::memcpy(host.data() + off, src, bytes);
    return off;
  }
};

int device_cus(int dev, int& n_cu) {
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) { n_cu = it->second; return COEX_OK; }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return COEX_EDEVICE;
  cache[dev] = v;
  n_cu = v;
  return COEX_OK;
}

}  // namespace batch
}  // namespace coex

// Resident automata, grouped for LDS (the handle behind coex_dfa_set).
struct coex_dfa_set {
  int device = 0;
  uint32_t n_dfa = 0;
  uint32_t W = 8;
  bool any_step2 = false, any_step1 = false;
  bool may_not_converge_below = false;  // some automaton has no finite synchronising depth
  uint32_t max_sync = 0;                // largest finite synchronising depth (+ lookback)
  uint32_t wmax = 64;                   // cap on candidate lists given at creation
  std::vector<uint32_t> n_states, group_of, k_of;
  // per automaton: largest candidate list per lookback k, synchronising
  // depth, and the device offsets of the PSS tables uploaded (the lookbacks
  // some width cap up to wmax selects; SIZE_MAX where none)
  std::vector<std::array<uint32_t, coex::kMaxLookback + 1>> pss_max;
  std::vector<uint32_t> sync_of;
  std::vector<std::array<size_t, coex::kMaxLookback + 1>> pss_off_at, pss_states_at;
  struct Group {
    std::vector<uint32_t> members;
    uint32_t step = 2;
    uint32_t n_states = 0, n_acc = 0, tab_bytes = 0;
    size_t off_tab[2], off_t1[2], off_w;
  };
  std::vector<Group> groups;
  // per automaton device descriptors per encoding (byte, 2-bit)
  std::vector<coex::batch::DfaD> dfa_dev[2];
  std::vector<coex::batch::GroupD> group_dev[2];  // lane fields filled per batch
  coex::batch::DevBuf buf;
};

// A batch of pairs over one automaton set (the handle behind coex_batch).
struct coex_batch {
  const coex_dfa_set* set = nullptr;
  int device = 0, n_cu = 0, enc = 0;
  uint64_t chunk = 0, fixed_chunk = 0;
  uint32_t n_pairs = 0, flags = 0, blocks = 0, lds_bytes = 0;
  bool needs_nc = false;
  // width cap of this batch (the set's at creation, the tuner's after
  // coex_batch_tune): lookback per automaton, largest candidate list,
  // convergence bounds and the automaton descriptors they give
  uint32_t width_cap = 0, W = 1, max_sync = 0;
  bool may_nc = false;
  std::vector<coex::batch::DfaD> dfa_dev;
  // host descriptors (kept to rebuild with another chunk length)
  std::vector<coex::batch::SeqD> seqs;
  std::vector<uint32_t> pair_seq, pair_dfa;
  uint64_t n_lanes = 0, n_units = 0;
  uint32_t n_tasks = 0, n_slots = 0, max_D = 0;
  coex::batch::Args args{};
  coex::batch::DevBuf desc, recs;
  // byte input converted to 2-bit codes + N mask once per run
  bool convert = false;
  int scan_enc = 0;
  coex::batch::ConvArgs cargs{};
  coex::batch::DevBuf conv;
  // graph replay
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap_stream = nullptr;
  unsigned long long* graph_counts = nullptr;
  // timing of the last timed run
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed_pending = false;
  ~coex_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

namespace coex {
namespace batch {

using Set = coex_dfa_set;
using Batch = coex_batch;

// Lookback of an automaton under a cap w on its candidate lists (mx[k] =
// its largest list after k bases): the shortest whose lists fit one batch of
// registers (8) and the cap, else the one with the fewest candidates if
// that fits the cap; 0 if none does.
uint32_t lookback_for(const std::array<uint32_t, kMaxLookback + 1>& mx, uint32_t w) {
  for (uint32_t k = 1; k <= kMaxLookback; ++k)
    if (mx[k] <= std::min<uint32_t>(8, w)) return k;
  uint32_t best = kMaxLookback;
  for (uint32_t k = 1; k <= kMaxLookback; ++k)
    if (mx[k] < mx[best]) best = k;
  return mx[best] <= w ? best : 0u;
}

int build_set(const coex_dfa* const* hs, uint32_t n_dfa, const coex_opts* o, std::unique_ptr<Set>& out) {
  if (!hs || n_dfa == 0) return COEX_EINVAL;
  auto S = std::make_unique<Set>();
  if (hipGetDevice(&S->device) != hipSuccess) return COEX_EDEVICE;
  S->n_dfa = n_dfa;
  std::vector<const Dfa*> ds(n_dfa);
  std::vector<uint32_t> step_of(n_dfa, 2);
  const uint32_t wmax = (o && o->width) ? o->width : 64u;
  if (wmax > 64) return COEX_EINVAL;
  for (uint32_t i = 0; i < n_dfa; ++i) {
    if (!hs[i]) return COEX_EINVAL;
    ds[i] = reinterpret_cast<const Dfa*>(hs[i]);
    // two-symbol rows need 64 B rows addressable with 16 bits and exact
    // 8-bit counts over a 16-base word
    const bool t2_ok = ds[i]->max_out <= 15 && ds[i]->n_states <= kGroupStates2;
    if (ds[i]->n_states > kGroupStates1) return COEX_ETOOBIG;
    if (ds[i]->max_out > 255) return COEX_EUNSUPPORTED;
    if (o && o->step == 2 && !t2_ok) return COEX_EUNSUPPORTED;
    step_of[i] = (o && o->step == 1) ? 1u : (t2_ok ? 2u : 1u);
    (step_of[i] == 2 ? S->any_step2 : S->any_step1) = true;
  }
  S->wmax = wmax;
  S->k_of.resize(n_dfa);
  S->pss_max.resize(n_dfa);
  S->sync_of.resize(n_dfa);
  uint32_t W = 1;
  for (uint32_t i = 0; i < n_dfa; ++i) {
    const Dfa& d = *ds[i];
    for (uint32_t kk = 0; kk <= kMaxLookback; ++kk) S->pss_max[i][kk] = kk ? d.pss[kk].max_size : d.n_states;
    S->sync_of[i] = d.sync_depth;
    const uint32_t k = lookback_for(S->pss_max[i], wmax);
    if (!k) return COEX_EUNSUPPORTED;
    S->k_of[i] = k;
    W = std::max(W, d.pss[k].max_size);
    if (d.sync_depth == kNoSync) S->may_not_converge_below = true;
    else S->max_sync = std::max(S->max_sync, d.sync_depth + k);
  }
  S->W = W;  // largest candidate list
  // groups: first fit by decreasing size among automata of the same step
  std::vector<uint32_t> order(n_dfa);
  for (uint32_t i = 0; i < n_dfa; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return ds[a]->n_states > ds[b]->n_states; });
  S->group_of.assign(n_dfa, 0);
  S->n_states.resize(n_dfa);
  for (uint32_t i : order) {
    const uint32_t n = ds[i]->n_states;
    const uint32_t cap = step_of[i] == 2 ? kGroupStates2 : kGroupStates1;
    S->n_states[i] = n;
    uint32_t g = 0;
    while (g < S->groups.size() && (S->groups[g].step != step_of[i] || S->groups[g].n_states + n > cap)) ++g;
    if (g == S->groups.size()) {
      S->groups.emplace_back();
      S->groups.back().step = step_of[i];
    }
    S->groups[g].members.push_back(i);
    S->groups[g].n_states += n;
    S->group_of[i] = g;
  }
  // images
  Image img;
  std::vector<uint32_t> base(n_dfa), acc_base(n_dfa), shift_of(n_dfa);
  for (auto& G : S->groups) {
    const uint32_t SH = G.step == 2 ? 6u : 4u;
    const uint32_t row = G.step == 2 ? 64u : 16u;
    for (uint32_t i : G.members) shift_of[i] = SH;
    uint32_t st = 0, ac = 0;
    for (uint32_t i : G.members) {
      base[i] = st * row;
      acc_base[i] = ac;
      st += ds[i]->n_states;
      ac += ds[i]->n_accepting;
    }
    G.n_acc = ac;
    G.tab_bytes = (uint32_t)align_up((size_t)st * row, 16);
    std::vector<uint32_t> w(std::max<uint32_t>(ac, 1), 0);
    for (uint32_t i : G.members) {
      const Dfa& d = *ds[i];
      for (uint32_t a = 0; a < d.n_accepting; ++a) {
        const uint32_t s = d.acc_state[a];
        w[acc_base[i] + a] = d.out_off[s + 1] - d.out_off[s];
      }
    }
    G.off_w = img.add(w.data(), w.size() * 4);
    for (int e = 0; e < 2; ++e) {
      const int* ord = e == 1 ? kOrd2bit : kOrdByte;
      std::vector<uint32_t> t1((size_t)st * 4), t2;
      if (G.step == 2) t2.resize((size_t)st * 16);
      for (uint32_t i : G.members) {
        const Dfa& d = *ds[i];
        auto reg = [&](uint32_t s) { return base[i] + (s << SH); };
        auto wt = [&](uint32_t s) { return d.out_off[s + 1] - d.out_off[s]; };
        const uint32_t r0 = base[i] / row;
        for (uint32_t s = 0; s < d.n_states; ++s) {
          for (int c = 0; c < 4; ++c) {
            const uint32_t t = d.delta[s * 4 + ord[c]];
            const uint32_t a = d.acc_index[t] >= 0 ? acc_base[i] + (uint32_t)d.acc_index[t] + 1u : 0u;
            t1[(size_t)(r0 + s) * 4 + c] = reg(t) | (a << 16);
          }
          if (G.step == 2)
            for (int g = 0; g < 16; ++g) {
              const uint32_t s1 = d.delta[s * 4 + ord[g & 3]];
              const uint32_t s2 = d.delta[s1 * 4 + ord[g >> 2]];
              t2[(size_t)(r0 + s) * 16 + g] = reg(s2) | ((wt(s1) + wt(s2)) << 24);
            }
        }
      }
      G.off_t1[e] = img.add(t1.data(), t1.size() * 4);
      G.off_tab[e] = G.step == 2 ? img.add(t2.data(), t2.size() * 4) : G.off_t1[e];
    }
  }
  // PSS tables: every lookback some width cap up to wmax selects
  S->pss_off_at.assign(n_dfa, {});
  S->pss_states_at.assign(n_dfa, {});
  for (uint32_t i = 0; i < n_dfa; ++i) {
    S->pss_off_at[i].fill(SIZE_MAX);
    S->pss_states_at[i].fill(SIZE_MAX);
    for (uint32_t w = 1; w <= wmax; w <<= 1) {
      for (const uint32_t k : {lookback_for(S->pss_max[i], w), S->k_of[i]}) {
        if (!k || S->pss_off_at[i][k] != SIZE_MAX) continue;
        const PssTable& P = ds[i]->pss[k];
        S->pss_off_at[i][k] = img.add(P.off.data(), P.off.size() * 4);
        S->pss_states_at[i][k] = img.add(P.states.data(), P.states.size() * 2);
      }
    }
  }
  int rc = S->buf.reserve(img.host.size(), S->device);
  if (rc) return rc;
  if (hipMemcpy(S->buf.p, img.host.data(), img.host.size(), hipMemcpyHostToDevice) != hipSuccess) return COEX_EDEVICE;
  for (int e = 0; e < 2; ++e) {
    S->dfa_dev[e].resize(n_dfa);
    for (uint32_t i = 0; i < n_dfa; ++i) {
      DfaD& D = S->dfa_dev[e][i];
      D.base = base[i];
      D.q0s = base[i] + (ds[i]->q0 << shift_of[i]);
      D.k = S->k_of[i];
      D.group = S->group_of[i];
      D.pss_off = reinterpret_cast<const uint32_t*>(S->buf.p + S->pss_off_at[i][D.k]);
      D.pss_states = reinterpret_cast<const uint16_t*>(S->buf.p + S->pss_states_at[i][D.k]);
    }
    S->group_dev[e].resize(S->groups.size());
    for (size_t g = 0; g < S->groups.size(); ++g) {
      GroupD& G = S->group_dev[e][g];
      G = GroupD{};
      G.tab_bytes = S->groups[g].tab_bytes;
      G.step = S->groups[g].step;
      G.t1_lds_off = G.step == 2 ? G.tab_bytes : 0u;
      G.t1_bytes = G.step == 2 ? S->groups[g].n_states * 16u : 0u;
      G.tab = reinterpret_cast<const uint32_t*>(S->buf.p + S->groups[g].off_tab[e]);
      G.t1 = reinterpret_cast<const uint32_t*>(S->buf.p + S->groups[g].off_t1[e]);
      G.wtab = reinterpret_cast<const uint32_t*>(S->buf.p + S->groups[g].off_w);
    }
  }
  out = std::move(S);
  return COEX_OK;
}

template <int ENC>
int occupancy(uint32_t lds) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_bscan<ENC>, kBlock, lds) != hipSuccess) return 1;
  return std::max(1, b);
}

template <int ENC>
void launch(Batch& B, hipStream_t st, hipEvent_t e0, hipEvent_t e1, bool attrs_only) {
  Args& A = B.args;
  if (attrs_only) {
    (void)hipFuncSetAttribute((const void*)k_bscan<ENC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)B.lds_bytes);
    return;
  }
  if (B.convert && B.cargs.total)
    hipLaunchKernelGGL(k_bconvert, dim3((uint32_t)std::min<uint64_t>((B.cargs.total + 255) / 256, 8192)), dim3(256), 0,
                       st, B.cargs);
  hipLaunchKernelGGL(k_binit, dim3(std::max<uint32_t>(1, std::min<uint32_t>((B.n_pairs + 255) / 256, 1024))),
                     dim3(256), 0, st, A);
  if (B.n_tasks) {
    if (e0) (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL((k_bscan<ENC>), dim3(B.blocks), dim3(kBlock), B.lds_bytes, st, A);
    if (e1) (void)hipEventRecord(e1, st);
    if (B.needs_nc)
      hipLaunchKernelGGL(k_bcompose, dim3((B.n_slots + 255) / 256), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_bfix<ENC>, dim3(std::max(1, B.n_cu)), dim3(256), 0, st, A);
  }
}

// attrs_only: set the scan kernel's LDS limit (outside any graph capture).
void dispatch(Batch& B, hipStream_t st, hipEvent_t e0, hipEvent_t e1, bool attrs_only = false) {
  const Set& S = *B.set;
  const bool by = B.scan_enc == 0;
  const bool a = attrs_only;
  (void)S;
  by ? launch<ENC_BYTE>(B, st, e0, e1, a) : launch<ENC_2BIT>(B, st, e0, e1, a);
}

uint32_t blocks_per_cu(const Set& S, int enc, uint32_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, uint32_t, uint32_t>, int> cache;
  const auto key = std::make_tuple(enc, 0u, lds);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return (uint32_t)it->second;
  const bool by = enc == 0;
  (void)S;
  const int b = by ? occupancy<ENC_BYTE>(lds) : occupancy<ENC_2BIT>(lds);
  cache[key] = b;
  return (uint32_t)b;
}

// Chunk length when none is given: about three tasks' worth of lanes per
// resident lane of the GPU, between 4 KiB and 1 MiB, a multiple of 4 KiB.
uint64_t default_chunk(const Batch& B, uint64_t lane_bases) {
  const uint64_t resident = (uint64_t)std::max(1, B.n_cu) * 2 * kBlock;
  uint64_t c = lane_bases / std::max<uint64_t>(1, 3 * resident);
  c = std::max<uint64_t>(4096, std::min<uint64_t>(c, 1ull << 20));
  return align_up(c, 4096);
}

// Descriptors and records for the current chunk length.
// The batch's lookbacks under its width cap (a power of two up to the
// set's cap): descriptors, largest candidate list, convergence bounds.
int apply_width(Batch& B) {
  const Set& S = *B.set;
  const uint32_t cap = B.width_cap ? B.width_cap : S.wmax;
  B.dfa_dev = S.dfa_dev[B.scan_enc];
  B.W = 1;
  B.max_sync = 0;
  B.may_nc = false;
  for (uint32_t i = 0; i < S.n_dfa; ++i) {
    const uint32_t k = lookback_for(S.pss_max[i], cap);
    if (!k || S.pss_off_at[i][k] == SIZE_MAX) return COEX_EUNSUPPORTED;
    DfaD& D = B.dfa_dev[i];
    D.k = k;
    D.pss_off = reinterpret_cast<const uint32_t*>(S.buf.p + S.pss_off_at[i][k]);
    D.pss_states = reinterpret_cast<const uint16_t*>(S.buf.p + S.pss_states_at[i][k]);
    B.W = std::max(B.W, S.pss_max[i][k]);
    if (S.sync_of[i] == kNoSync) B.may_nc = true;
    else B.max_sync = std::max(B.max_sync, S.sync_of[i] + k);
  }
  return COEX_OK;
}

int layout(Batch& B) {
  const Set& S = *B.set;
  B.convert = B.enc == 0;
  B.scan_enc = 1;
  const int e = B.scan_enc;
  {
    const int rcw = apply_width(B);
    if (rcw) return rcw;
  }
  const uint64_t C = B.chunk;
  const size_t ng = S.groups.size();
  // entries: (group, sequence) with the pair slots of that group
  std::vector<std::vector<std::vector<uint32_t>>> by_group(ng, std::vector<std::vector<uint32_t>>(B.seqs.size()));
  for (uint32_t i = 0; i < B.n_pairs; ++i) by_group[S.group_of[B.pair_dfa[i]]][B.pair_seq[i]].push_back(i);
  std::vector<EntryD> entries;
  std::vector<UnitD> units;
  std::vector<uint32_t> slot_dfa, slot_out, slot_entry;
  std::vector<GroupD> groups = S.group_dev[e];
  uint64_t lane0 = 0;
  uint32_t task0 = 0;
  B.max_D = 0;
  for (size_t g = 0; g < ng; ++g) {
    uint32_t D = 0;
    for (auto& v : by_group[g]) D = std::max<uint32_t>(D, (uint32_t)v.size());
    GroupD& G = groups[g];
    G.D = std::max<uint32_t>(D, 1);
    G.unit0 = units.size();
    G.lane0 = lane0;
    G.task0 = task0;
    for (uint32_t s = 0; s < B.seqs.size(); ++s) {
      auto& v = by_group[g][s];
      if (v.empty()) continue;
      const uint64_t n = B.seqs[s].n;
      const uint64_t K = n == 0 ? 0 : std::max<uint64_t>(1, n / C);
      if (K > 0xFFFFFFFFull) return COEX_EINVAL;
      EntryD en{};
      en.seq = s;
      en.slot0 = (uint32_t)slot_dfa.size();
      en.n_chunks = (uint32_t)K;
      en.unit0 = (uint32_t)units.size();
      const uint32_t eid = (uint32_t)entries.size();
      for (uint32_t jj = 0; jj < G.D; ++jj) {
        slot_dfa.push_back(jj < v.size() ? B.pair_dfa[v[jj]] : kPad);
        slot_out.push_back(jj < v.size() ? v[jj] : 0u);
        slot_entry.push_back(eid);
      }
      for (uint64_t c = 0; c < K; ++c) units.push_back(UnitD{eid, (uint32_t)c});
      entries.push_back(en);
    }
    G.n_units = units.size() - G.unit0;
    G.n_lanes = (G.n_units + 63) / 64 * 64 * (uint64_t)G.D;
    lane0 += G.n_lanes;
    task0 += (uint32_t)((G.n_lanes + kBlock - 1) / kBlock);
    B.max_D = std::max(B.max_D, G.D);
  }
  if (units.size() > 0xFFFFFFFFull || lane0 > 0xFFFFFFFFull) return COEX_EINVAL;
  B.n_lanes = lane0;
  B.n_units = units.size();
  B.n_tasks = task0;
  B.n_slots = (uint32_t)slot_dfa.size();
  // chunks may fail to converge only when an automaton's synchronising depth
  // (plus its lookback) reaches the chunk length
  B.needs_nc = B.may_nc || B.max_sync >= C;
  // 2-bit copies of byte sequences: codes then mask per sequence, 16-byte aligned
  std::vector<SeqD> scan_seqs = B.seqs;
  std::vector<uint64_t> prefix(B.seqs.size() + 1, 0);
  if (B.convert) {
    size_t off = 0;
    std::vector<size_t> co(B.seqs.size()), mo(B.seqs.size());
    for (size_t i = 0; i < B.seqs.size(); ++i) {
      const uint64_t groups = (B.seqs[i].n + 63) / 64;
      prefix[i + 1] = prefix[i] + groups;
      co[i] = off;
      off = align_up(off + groups * 16, 256);
      mo[i] = off;
      off = align_up(off + groups * 8, 256);
    }
    int rc0 = B.conv.reserve(std::max<size_t>(off, 256), B.device);
    if (rc0) return rc0;
    for (size_t i = 0; i < B.seqs.size(); ++i)
      scan_seqs[i] = SeqD{reinterpret_cast<const uint8_t*>(B.conv.p + co[i]),
                          reinterpret_cast<const uint8_t*>(B.conv.p + mo[i]), B.seqs[i].n};
  }
  Image img;
  const size_t o_seq = img.add(scan_seqs.data(), scan_seqs.size() * sizeof(SeqD));
  const size_t o_src = img.add(B.seqs.data(), B.seqs.size() * sizeof(SeqD));
  const size_t o_pre = img.add(prefix.data(), prefix.size() * 8);
  const size_t o_dfa = img.add(B.dfa_dev.data(), B.dfa_dev.size() * sizeof(DfaD));
  const size_t o_ent = img.add(entries.data(), entries.size() * sizeof(EntryD));
  const size_t o_unit = img.add(units.data(), units.size() * sizeof(UnitD));
  const size_t o_grp = img.add(groups.data(), groups.size() * sizeof(GroupD));
  const size_t o_sd = img.add(slot_dfa.data(), slot_dfa.size() * 4);
  const size_t o_so = img.add(slot_out.data(), slot_out.size() * 4);
  const size_t o_se = img.add(slot_entry.data(), slot_entry.size() * 4);
  int rc = B.desc.reserve(img.host.size(), B.device);
  if (rc) return rc;
  if (hipMemcpy(B.desc.p, img.host.data(), img.host.size(), hipMemcpyHostToDevice) != hipSuccess) return COEX_EDEVICE;
  // records
  const uint64_t NL = std::max<uint64_t>(B.n_lanes, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o2 = off; off = align_up(off + std::max<size_t>(bytes, 8), 256); return o2; };
  const size_t r_ctr = take(4), r_fc = take(4), r_err = take(4);
  const size_t r_fl = take(NL * 4), r_t = take(NL * 4), r_s = take(NL * 4), r_end = take(NL * 4), r_tail = take(NL * 4);
  size_t r_ts = 0, r_m = 0, r_init = 0, r_ne = 0, r_nc = 0;
  if (B.needs_nc) {
    r_ts = take(NL * 4);
    r_m = take(NL * 4);
    r_init = take(NL * B.W * 4);
    r_ne = take(NL * B.W * 4);
    r_nc = take(NL * B.W * 4);
  }
  rc = B.recs.reserve(off, B.device);
  if (rc) return rc;
  Args& A = B.args;
  A = Args{};
  char* dp = B.desc.p;
  char* rp = B.recs.p;
  A.seqs = reinterpret_cast<const SeqD*>(dp + o_seq);
  B.cargs = ConvArgs{reinterpret_cast<const SeqD*>(dp + o_src), reinterpret_cast<const SeqD*>(dp + o_seq),
                     reinterpret_cast<const uint64_t*>(dp + o_pre), (uint32_t)B.seqs.size(), prefix.back()};
  A.dfas = reinterpret_cast<const DfaD*>(dp + o_dfa);
  A.entries = reinterpret_cast<const EntryD*>(dp + o_ent);
  A.units = reinterpret_cast<const UnitD*>(dp + o_unit);
  A.groups = reinterpret_cast<const GroupD*>(dp + o_grp);
  A.slot_dfa = reinterpret_cast<const uint32_t*>(dp + o_sd);
  A.slot_out = reinterpret_cast<const uint32_t*>(dp + o_so);
  A.slot_entry = reinterpret_cast<const uint32_t*>(dp + o_se);
  A.n_groups = (uint32_t)ng;
  A.n_tasks = B.n_tasks;
  A.n_slots = B.n_slots;
  uint32_t tab_max = 0;
  for (auto& G : S.groups) tab_max = std::max(tab_max, G.tab_bytes + (G.step == 2 ? G.n_states * 16u : 0u));
  A.bcast_off = tab_max;
  B.lds_bytes = tab_max + 16;
  A.chunk = C;
  A.max_cand = B.W;
  A.nc_stride = B.W;
  A.n_counts = B.n_pairs;
  A.task_ctr = reinterpret_cast<uint32_t*>(rp + r_ctr);
  A.fix_count = reinterpret_cast<uint32_t*>(rp + r_fc);
  A.err = reinterpret_cast<uint32_t*>(rp + r_err);
  A.fix_list = reinterpret_cast<uint32_t*>(rp + r_fl);
  A.rec_t = reinterpret_cast<uint32_t*>(rp + r_t);
  A.rec_s = reinterpret_cast<uint32_t*>(rp + r_s);
  A.rec_end = reinterpret_cast<uint32_t*>(rp + r_end);
  A.rec_tail = reinterpret_cast<uint32_t*>(rp + r_tail);
  if (B.needs_nc) {
    A.rec_ts = reinterpret_cast<uint32_t*>(rp + r_ts);
    A.nc_m = reinterpret_cast<uint32_t*>(rp + r_m);
    A.nc_init = reinterpret_cast<uint32_t*>(rp + r_init);
    A.nc_end = reinterpret_cast<uint32_t*>(rp + r_ne);
    A.nc_cnt = reinterpret_cast<uint32_t*>(rp + r_nc);
  }
  const uint32_t per_cu = blocks_per_cu(S, B.scan_enc, B.lds_bytes);
  B.blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)B.n_cu * per_cu, B.n_tasks));
  // a new layout invalidates a captured graph
  if (B.exec) { (void)hipGraphExecDestroy(B.exec); B.exec = nullptr; }
  if (B.graph) { (void)hipGraphDestroy(B.graph); B.graph = nullptr; }
  return COEX_OK;
}

// Validates sequences and pairs, then lays the batch out for them (a failed
// call leaves the batch as it was).
int set_work(Batch& B, const coex_seq* seqs, uint32_t n_seq, const uint32_t* pair_seq, const uint32_t* pair_dfa,
             uint32_t n_pairs) {
  const Set* S = B.set;
  if (n_seq && !seqs) return COEX_EINVAL;
  int enc = -1;
  std::vector<SeqD> sv(n_seq);
  for (uint32_t s = 0; s < n_seq; ++s) {
    const coex_seq& q = seqs[s];
    if (q.encoding != COEX_ENC_BYTE && q.encoding != COEX_ENC_2BIT) return COEX_EINVAL;
    const int e = q.encoding == COEX_ENC_2BIT ? 1 : 0;
    if (enc < 0) enc = e;
    else if (enc != e) return COEX_EINVAL;
    if (q.n_bases > 0 && !q.bases) return COEX_EINVAL;
    if (((uintptr_t)q.bases & 15) || ((uintptr_t)q.n_mask & 15) || q.first_base) return COEX_EINVAL;
    sv[s] = SeqD{reinterpret_cast<const uint8_t*>(q.bases), e == 1 ? q.n_mask : nullptr, q.n_bases};
  }
  std::vector<uint32_t> ps, pd;
  if (pair_seq || pair_dfa) {
    if (!pair_seq || !pair_dfa) return COEX_EINVAL;
    ps.assign(pair_seq, pair_seq + n_pairs);
    pd.assign(pair_dfa, pair_dfa + n_pairs);
  } else {  // every sequence with every automaton, pair s * n_dfa + d
    if ((uint64_t)n_seq * S->n_dfa > 0xFFFFFFFFull) return COEX_EINVAL;
    n_pairs = n_seq * S->n_dfa;
    ps.resize(n_pairs);
    pd.resize(n_pairs);
    for (uint32_t s = 0; s < n_seq; ++s)
      for (uint32_t d = 0; d < S->n_dfa; ++d) {
        ps[s * S->n_dfa + d] = s;
        pd[s * S->n_dfa + d] = d;
      }
  }
  uint64_t total = 0;
  for (uint32_t i = 0; i < n_pairs; ++i) {
    if (ps[i] >= n_seq || pd[i] >= S->n_dfa) return COEX_EINVAL;
    total += sv[ps[i]].n;
  }
  B.enc = enc < 0 ? 0 : enc;
  B.seqs.swap(sv);
  B.pair_seq.swap(ps);
  B.pair_dfa.swap(pd);
  B.n_pairs = n_pairs;
  B.chunk = B.fixed_chunk ? B.fixed_chunk : default_chunk(B, total);
  return layout(B);
}

int build_batch(const Set* S, const coex_seq* seqs, uint32_t n_seq, const uint32_t* pair_seq,
                const uint32_t* pair_dfa, uint32_t n_pairs, const coex_opts* o, std::unique_ptr<Batch>& out) {
  if (!S) return COEX_EINVAL;
  auto B = std::make_unique<Batch>();
  B->set = S;
  if (hipGetDevice(&B->device) != hipSuccess) return COEX_EDEVICE;
  if (B->device != S->device) return COEX_EINVAL;
  int rc = device_cus(B->device, B->n_cu);
  if (rc) return rc;
  B->flags = o ? o->flags : 0u;
  if (o && o->width) {
    // caps the set has PSS tables for: powers of two up to its own
    if (o->width > S->wmax || (o->width & (o->width - 1))) return COEX_EINVAL;
    B->width_cap = o->width;
  }
  if (o && o->chunk) {
    // per-chunk tail counters are 32-bit: the last chunk holds under two
    // chunks' bases, at most 255 pattern ends per base
    if (o->chunk < 64 || 2ull * o->chunk * 255 > 0xFFFFFFFFull) return COEX_EINVAL;
    B->fixed_chunk = o->chunk;
  }
  rc = set_work(*B, seqs, n_seq, pair_seq, pair_dfa, n_pairs);
  if (rc) return rc;
  out = std::move(B);
  return COEX_OK;
}

int run(Batch& B, uint64_t* counts, hipStream_t st) {
  if (!counts && B.n_pairs) return COEX_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return COEX_EDEVICE;
  if (dev != B.device) return COEX_EINVAL;
  B.args.counts = reinterpret_cast<unsigned long long*>(counts);
  const bool timed = B.flags & COEX_FLAG_TIME;
  dispatch(B, st, nullptr, nullptr, true);
  if (timed && !B.ev0) {
    if (hipEventCreate(&B.ev0) != hipSuccess || hipEventCreate(&B.ev1) != hipSuccess) return COEX_EDEVICE;
  }
  if (B.flags & COEX_FLAG_GRAPH) {
    if (B.exec && B.graph_counts != B.args.counts) {
      (void)hipGraphExecDestroy(B.exec);
      (void)hipGraphDestroy(B.graph);
      B.exec = nullptr;
      B.graph = nullptr;
    }
    if (!B.exec) {
      if (!B.cap_stream && hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking) != hipSuccess)
        return COEX_EDEVICE;
      if (hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return COEX_EDEVICE;
      dispatch(B, B.cap_stream, nullptr, nullptr);
      if (hipStreamEndCapture(B.cap_stream, &B.graph) != hipSuccess) return COEX_EDEVICE;
      if (hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0) != hipSuccess) return COEX_EDEVICE;
      B.graph_counts = B.args.counts;
    }
    if (timed) (void)hipEventRecord(B.ev0, st);
    if (hipGraphLaunch(B.exec, st) != hipSuccess) return COEX_EDEVICE;
    if (timed) (void)hipEventRecord(B.ev1, st);
  } else {
    dispatch(B, st, timed ? B.ev0 : nullptr, timed ? B.ev1 : nullptr);
  }
  if (hipPeekAtLastError() != hipSuccess) return COEX_EDEVICE;
  B.timed_pending = timed;
  if (B.flags & COEX_FLAG_CHECK) {
    uint32_t e = 0;
    if (hipMemcpyAsync(&e, B.args.err, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return COEX_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return COEX_EDEVICE;
    if (e) return COEX_EINTERNAL;
  }
  return COEX_OK;
}

}  // namespace batch
}  // namespace coex

// ====================================================================== C ABI
extern "C" {

int coex_dfa_set_create(const coex_dfa* const* dfas, uint32_t n_dfa, const coex_opts* opts, coex_dfa_set** out) {
  if (!out) return COEX_EINVAL;
  try {
    std::unique_ptr<coex_dfa_set> S;
    const int rc = coex::batch::build_set(dfas, n_dfa, opts, S);
    if (rc) return rc;
    *out = S.release();
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

void coex_dfa_set_free(coex_dfa_set* set) { delete set; }

int coex_batch_create(const coex_dfa_set* set, const coex_seq* seqs, uint32_t n_seq, const uint32_t* pair_seq,
                      const uint32_t* pair_dfa, uint32_t n_pairs, const coex_opts* opts, coex_batch** out) {
  if (!out) return COEX_EINVAL;
  try {
    std::unique_ptr<coex_batch> B;
    const int rc = coex::batch::build_batch(set, seqs, n_seq, pair_seq, pair_dfa, n_pairs, opts, B);
    if (rc) return rc;
    *out = B.release();
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_batch_update(coex_batch* b, const coex_seq* seqs, uint32_t n_seq, const uint32_t* pair_seq,
                      const uint32_t* pair_dfa, uint32_t n_pairs) {
  if (!b) return COEX_EINVAL;
  try {
    return coex::batch::set_work(*b, seqs, n_seq, pair_seq, pair_dfa, n_pairs);
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_batch_run(coex_batch* b, uint64_t* counts_dev, void* stream) {
  if (!b) return COEX_EINVAL;
  try {
    return coex::batch::run(*b, counts_dev, (hipStream_t)stream);
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_batch_tune(coex_batch* b, uint64_t* counts_dev, void* stream, uint64_t* chunk_out, uint32_t* width_out) {
  if (!b || !chunk_out) return COEX_EINVAL;
  try {
    hipStream_t st = (hipStream_t)stream;
    const coex_dfa_set& S = *b->set;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return COEX_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return COEX_EDEVICE; }
    const uint32_t keep_flags = b->flags;
    b->flags &= ~(COEX_FLAG_GRAPH | COEX_FLAG_TIME | COEX_FLAG_CHECK);
    // width caps 1, 2, 4, ... up to the set's: each distinct choice of
    // lookbacks once (caps that select the same lookbacks run the same work)
    std::vector<uint32_t> caps;
    std::vector<std::vector<uint32_t>> seen;
    for (uint32_t w = 1; w <= S.wmax; w <<= 1) {
      std::vector<uint32_t> ks(S.n_dfa);
      bool ok = true;
      for (uint32_t i = 0; i < S.n_dfa && ok; ++i) {
        ks[i] = coex::batch::lookback_for(S.pss_max[i], w);
        ok = ks[i] != 0;
      }
      if (!ok || std::find(seen.begin(), seen.end(), ks) != seen.end()) continue;
      seen.push_back(ks);
      caps.push_back(w);
    }
    uint64_t best = b->chunk;
    uint32_t best_w = b->width_cap;
    float best_ms = 1e30f;
    int rc = COEX_OK;
    for (const uint32_t w : caps) {
      for (uint64_t c = 4096; c <= (1ull << 20) && rc == COEX_OK; c *= 4) {
        b->width_cap = w;
        b->chunk = c;
        rc = coex::batch::layout(*b);
        if (rc) break;
        rc = coex::batch::run(*b, counts_dev, st);  // warm-up
        if (rc) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = COEX_EDEVICE; break; }
        rc = coex::batch::run(*b, counts_dev, st);
        if (rc) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = COEX_EDEVICE; break; }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = COEX_EDEVICE; break; }
        if (ms < best_ms) { best_ms = ms; best = c; best_w = w; }
      }
      if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->flags = keep_flags;
    b->chunk = best;
    b->fixed_chunk = best;
    b->width_cap = best_w;
    const int rc2 = coex::batch::layout(*b);
    if (rc) return rc;
    if (rc2) return rc2;
    *chunk_out = best;
    if (width_out) *width_out = best_w ? best_w : S.wmax;
    return COEX_OK;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_batch_info(const coex_batch* b, coex_batch_info_t* info) {
  if (!b || !info) return COEX_EINVAL;
  const coex_dfa_set& S = *b->set;
  info->chunk = b->chunk;
  info->width = b->W;
  info->step = S.any_step2 ? (S.any_step1 ? 3u : 2u) : 1u;
  info->n_groups = (uint32_t)S.groups.size();
  info->n_pairs = b->n_pairs;
  info->n_tasks = b->n_tasks;
  info->n_lanes = b->n_lanes;
  info->blocks = b->blocks;
  info->last_ms = -1.0;
  if (b->timed_pending && b->ev1) {
    if (hipEventSynchronize(b->ev1) != hipSuccess) return COEX_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, b->ev0, b->ev1) != hipSuccess) return COEX_EDEVICE;
    info->last_ms = ms;
  }
  return COEX_OK;
}

void coex_batch_free(coex_batch* b) { delete b; }

int coex_count_batched(const coex_dfa* const* dfas, uint32_t n_dfa, const coex_seq* seqs, uint32_t n_seq,
                       uint64_t* counts_dev, const coex_opts* opts, void* stream) {
  coex_dfa_set* S = nullptr;
  int rc = coex_dfa_set_create(dfas, n_dfa, opts, &S);
  if (rc) return rc;
  coex_batch* B = nullptr;
  coex_opts o = opts ? *opts : coex_opts{};
  o.flags &= ~COEX_FLAG_GRAPH;
  rc = coex_batch_create(S, seqs, n_seq, nullptr, nullptr, 0, &o, &B);
  if (rc == COEX_OK) {
    rc = coex_batch_run(B, counts_dev, stream);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && rc == COEX_OK) rc = COEX_EDEVICE;
  }
  coex_batch_free(B);
  coex_dfa_set_free(S);
  return rc;
}

}  // extern "C"
