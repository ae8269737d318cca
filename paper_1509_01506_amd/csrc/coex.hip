// libcoex: kernels, host runtime and the C ABI (include/coex.h).
//
// Pipeline of one scan (Section III of the paper, re-laid out for one MI355X):
//   k_init       clears the small device counters;
//   k_tail       per tile of 64 chunks (one wave): possible starting states
//                from the lookback table, lockstep speculative runs with
//                ballot convergence (Algorithm 1's converging point); then one
//                lane per chunk: one scan of the rest of the chunk from the
//                converged state, the join with the predecessor lane and the
//                prefix recount inside the wave;
//   k_nonconv    chunks that did not converge inside the window: every
//                candidate runs to the chunk end (the paper's non-converged
//                runs), giving the chunk's state map on its candidates;
//   k_join_*     the join: true first state of every chunk from its
//                predecessor's last state, as a scan over the non-converged
//                chunks' maps (composed kJoinFan at a time per level);
//   k_fixup      recounts [chunk start, converging point) from the true first
//                state and checks it reaches the converged state (count
//                fix-up of Algorithm 1 in an equivalent form).
// Per-pattern counts are added to the caller's buffer as they are found
// (visits of each final state, spread over the patterns it ends).
// Positions add an exclusive scan of per-chunk counts and a second pass per
// chunk from its true first state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <tuple>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "coex.h"
#include "dfa.hpp"
#include "kernels.hpp"
#include "tail.hpp"

namespace coex {

// sort.hip: ordering of appended match keys (end position << 24 | pattern id)
constexpr uint32_t kSmallSortKeys = 4096;
size_t sort_temp_bytes(uint64_t cap);
int sort_match_keys(const uint64_t* keys, uint64_t* tmp, uint64_t n, void* temp, size_t temp_bytes, int64_t* pos,
                    uint32_t* pat, uint64_t first, hipStream_t st);
int counts_from_ids(const uint32_t* ids, uint64_t n, uint32_t n_pat, uint64_t* counts, hipStream_t st);

// ====================================================================== kernels
// The kept failure words of a stream's calls and of the no-allocation calls,
// OR-ed into *out (device or host-mapped memory) and cleared.
__global__ void k_take_errors(uint32_t* ws, uint32_t* st, uint32_t* out) {
  if (threadIdx.x != 0) return;
  uint32_t e = atomicExch(st, 0u);
  if (ws) e |= atomicExch(ws, 0u);
  *out = e;
}

__global__ void k_init(ScanArgs a, uint64_t* counts, uint32_t n_counts) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *a.nc_count = 0;
    *a.fix_count = 0;
    *a.err = 0;
    *a.total = 0;
    if (a.app_count) *a.app_count = 0;
  }
  if (counts)
    for (uint32_t i = t; i < n_counts; i += gridDim.x * blockDim.x) counts[i] = 0;
}

// Weighted match count of one run: exact per-word counts from the
// two-symbol table, weights of single matches (one-symbol steps) otherwise.
struct SinkCount {
  static constexpr bool kReplay = false;
  static constexpr bool kOutline = false;
  const uint32_t* w;
  uint32_t cnt = 0;
  __device__ void word(uint32_t c) { cnt += c; }
  __device__ void hit(uint64_t, uint32_t acc) { cnt += w[acc]; }
};

// Non-converged chunks: every candidate runs to the chunk end (the paper's
// runs that never meet R0), giving the chunk's map on its candidates and each
// run's match count.  Lanes take (chunk, candidate) pairs, G = a power of two
// at least the largest candidate list per chunk.  STEP 2 (two symbols per
// lookup, exact counts in the entries) needs the two-symbol table at LDS
// address 0, the one-symbol table after it.
template <int ENC, int SHIFT, int STEP>
__global__ __launch_bounds__(256) void k_nonconv(ScanArgs a) {
  static_assert(STEP == 1 || STEP == 2, "one or two symbols per lookup");
  extern __shared__ __align__(16) char lds[];
  if (*a.nc_count == 0u) return;  // the common case: every chunk converged
  const uint32_t t1_at = STEP == 2 ? a.n_states * 64u : 0u;
  if (STEP == 2) copy_to_lds(lds, a.T2, a.n_states * 64u);
  copy_to_lds(lds + t1_at, a.T1, a.n_states * 16u);
  __syncthreads();
  if (STEP == 2 && threadIdx.x == 0 && (uint32_t)(uintptr_t)(lds_c*)lds != 0u) flag_error(a, 64u);
  const Tab tb{STEP == 2 ? lds : nullptr, lds + t1_at, a.q0s};
  const uint32_t G = a.nc_group;
  const uint64_t n_pairs = (uint64_t)*a.nc_count * G;
  const uint64_t lanes = (uint64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs the same number of rounds (wave-uniform bound)
  const uint64_t rounds = (n_pairs + lanes - 1) / lanes;
  for (uint64_t r = 0; r < rounds; ++r) {
    const uint64_t pair = r * lanes + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = pair < n_pairs;
    const uint32_t slot = in ? (uint32_t)(pair / G) : 0u;
    const uint32_t i = (uint32_t)(pair % G);
    const uint64_t c = in ? a.nc_chunk[slot] : 0;
    const uint64_t lo = chunk_lo(a, c);
    const uint64_t hi = in ? (lo + a.chunk < a.n ? lo + a.chunk : a.n) : 0;
    uint32_t m = 0, cbase = 0, exact = 0;
    bool is_exact = false;
    if (in) chunk_header<ENC, SHIFT>(a, tb, a.pss_off, lo, m, cbase, exact, is_exact);
    const bool live = in && i < m;
    if (in && i == 0) a.nc_m[slot] = m;
    uint32_t s = is_exact ? exact : ((uint32_t)a.pss_states[cbase + (live ? i : 0)] << SHIFT);
    const uint32_t s0 = s;
    SinkCount cnt{a.wtab};
    if (live) s = scan_range<ENC, SHIFT, STEP>(a, tb, s, lo, hi, cnt);
    if (live) {
      a.nc_cand[(uint64_t)slot * a.max_cand + i] = s0;
      a.nc_end[(uint64_t)slot * a.max_cand + i] = s;
      a.nc_cnt[(uint64_t)slot * a.max_cand + i] = cnt.cnt;
    }
  }
}

constexpr uint32_t kCountTile = 1024;

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(v, (unsigned)o);
    if (lane >= o) v += t;
  }
  return v;
}

// Inclusive scan over a block of kCountTile threads; `sh` holds 16 words.
__device__ __forceinline__ uint64_t block_incl_scan(uint64_t v, uint64_t* sh) {
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  v = wave_incl_scan(v);
  if (lane == 63) sh[w] = v;
  __syncthreads();
  if (w == 0) {
    uint64_t x = lane < (kCountTile >> 6) ? sh[lane] : 0;
    x = wave_incl_scan(x);
    if (lane < (kCountTile >> 6)) sh[lane] = x;
  }
  __syncthreads();
  return v + (w ? sh[w - 1] : 0);
}

// The join for chunks that did not converge (Section III.A: each chunk's
// first state is its predecessor's last state), as a scan over function
// composition.  Items are the non-converged chunks in sequence order (rank
// k); item k's map M0[k][x] takes the index x of its true first state in its
// candidate list to the index of the next item's true first state: the
// position of its end state in the next chunk's list when that chunk is the
// next item, else (a converged chunk in between absorbs the chain) the
// constant index of the next item's known first state, its converged
// predecessor's last state (0xFF in the map).  A map is a row of R bytes (R a
// power of two, at least the largest candidate list, at most 64).  Rows are
// composed kJoinFan at a time per level (one lane per row entry) until one
// level has at most kJoinFan items; that level is walked in order from item
// 0's known first index, and the indices are pushed back down.
constexpr uint32_t kJoinFan = 64;
constexpr uint32_t kJoinMaxLevels = 6;  // kJoinFan^6 items > 2^32 chunks

__device__ __forceinline__ uint32_t find_cand(const ScanArgs& a, uint32_t slot, uint32_t state) {
  const uint32_t* cand = a.nc_cand + (uint64_t)slot * a.max_cand;
  const uint32_t m = a.nc_m[slot];
  for (uint32_t i = 0; i < m; ++i)
    if (cand[i] == state) return i;
  flag_error(a, 1u);  // the true first state is always a candidate
  return 0;
}

// Rank of each non-converged chunk among them: the exclusive scan of the
// flags in three launches (sums per tile of kCountTile chunks, k_scan_partials
// over the sums, then each tile from its offset), the order list inverted.
__global__ __launch_bounds__(kCountTile) void k_rank_partials(ScanArgs a, uint64_t* part) {
  __shared__ uint64_t sh[kCountTile / 64];
  if (*a.nc_count == 0u) return;
  const uint64_t c = (uint64_t)blockIdx.x * kCountTile + threadIdx.x;
  const uint64_t v = c < a.n_chunks && a.conv_t[c] == NONCONV ? 1u : 0u;
  const uint64_t incl = block_incl_scan(v, sh);
  if (threadIdx.x == kCountTile - 1) part[blockIdx.x] = incl;
}

__global__ __launch_bounds__(kCountTile) void k_rank_offsets(ScanArgs a, const uint64_t* part, uint32_t* order) {
  __shared__ uint64_t sh[kCountTile / 64];
  if (*a.nc_count == 0u) return;
  const uint64_t c = (uint64_t)blockIdx.x * kCountTile + threadIdx.x;
  const bool nc = c < a.n_chunks && a.conv_t[c] == NONCONV;
  const uint64_t incl = block_incl_scan(nc ? 1u : 0u, sh);
  if (nc) order[part[blockIdx.x] + incl - 1] = (uint32_t)c;
}

// Level-0 maps and the known first index of every item whose predecessor
// converged (and of item 0).
__global__ void k_join_map0(ScanArgs a, const uint32_t* order, uint8_t* M0, uint8_t* known, uint32_t R) {
  const uint32_t N = *a.nc_count;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t c = order[k];
    const uint32_t slot = a.nc_slot[c];
    const uint32_t m = a.nc_m[slot];
    if (c == 0 || a.conv_t[c - 1] != NONCONV)
      known[k] = (uint8_t)find_cand(a, slot, c == 0 ? a.q0s : a.end_s[c - 1]);
    uint8_t* row = M0 + k * R;
    if (c + 1 < a.n_chunks && a.conv_t[c + 1] == NONCONV) {
      const uint32_t nslot = a.nc_slot[c + 1];
      for (uint32_t i = 0; i < m; ++i) row[i] = (uint8_t)find_cand(a, nslot, a.nc_end[(uint64_t)slot * a.max_cand + i]);
    } else {
      for (uint32_t i = 0; i < m; ++i) row[i] = 0xFFu;
    }
  }
}

// One step through map row y of item j (of a level whose items each cover
// `level_div` level-0 items, n_lvl of them): 0xFF (level 0 only) is the next
// item's known index.  Indices no candidate has stay inside the row.
__device__ __forceinline__ uint32_t join_step(uint32_t y, uint64_t j, uint64_t n_lvl, uint64_t level_div,
                                              const uint8_t* known, uint32_t R) {
  const uint32_t x = y == 0xFFu ? (j + 1 < n_lvl ? known[(j + 1) * level_div] : 0u) : y;
  return x < R ? x : 0u;
}

__device__ __forceinline__ uint64_t join_items(uint32_t n, uint64_t level_div) { return (n + level_div - 1) / level_div; }

// Composition of kJoinFan consecutive rows of the level below into one row
// of the level above: lane (K, x) follows index x through them.
__global__ void k_join_up(const uint32_t* n_dev, uint64_t level_div, const uint8_t* below, uint8_t* up,
                          const uint8_t* known, uint32_t R) {
  const uint64_t n_below = join_items(*n_dev, level_div);
  const uint64_t n_up = (n_below + kJoinFan - 1) / kJoinFan;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_up * R;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t K = t / R;
    uint32_t x = (uint32_t)(t % R);
    const uint64_t end = (K + 1) * kJoinFan < n_below ? (K + 1) * kJoinFan : n_below;
    for (uint64_t j = K * kJoinFan; j < end; ++j) x = join_step(below[j * R + x], j, n_below, level_div, known, R);
    up[t] = (uint8_t)x;
  }
}

// The top level walked in order by one thread from item 0's known index.
__global__ void k_join_top(const uint32_t* n_dev, uint64_t level_div, const uint8_t* top, const uint8_t* known,
                           uint8_t* x_top, uint32_t R) {
  const uint64_t n = join_items(*n_dev, level_div);
  if (n == 0) return;
  uint32_t x = known[0] < R ? known[0] : 0u;
  for (uint64_t K = 0; K < n; ++K) {
    x_top[K] = (uint8_t)x;
    x = join_step(top[K * R + x], K, n, level_div, known, R);
  }
}

// First index of every item of the level below from its parent's.
__global__ void k_join_down(const uint32_t* n_dev, uint64_t level_div, const uint8_t* below, const uint8_t* x_up,
                            uint8_t* x_below, const uint8_t* known, uint32_t R) {
  const uint64_t n_below = join_items(*n_dev, level_div);
  const uint64_t n_up = (n_below + kJoinFan - 1) / kJoinFan;
  for (uint64_t K = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; K < n_up; K += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t x = x_up[K];
    const uint64_t end = (K + 1) * kJoinFan < n_below ? (K + 1) * kJoinFan : n_below;
    for (uint64_t j = K * kJoinFan; j < end; ++j) {
      x_below[j] = (uint8_t)x;
      x = join_step(below[j * R + x], j, n_below, level_div, known, R);
    }
  }
}

// True first states: each non-converged chunk and the chunk after it from the
// item's index; a chunk after a converged chunk from that chunk's last state.
__global__ void k_join_finish(ScanArgs a, const uint32_t* order, const uint8_t* x0) {
  const uint32_t N = *a.nc_count;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t c = order[k];
    const uint32_t slot = a.nc_slot[c];
    const uint32_t x = x0[k] < a.nc_m[slot] ? x0[k] : 0u;
    a.true_start[c] = a.nc_cand[(uint64_t)slot * a.max_cand + x];
    a.true_start[c + 1] = a.nc_end[(uint64_t)slot * a.max_cand + x];
  }
  for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= a.n_chunks;
       c += (uint64_t)gridDim.x * blockDim.x)
    if (c == 0) {
      if (a.n_chunks == 0 || a.conv_t[0] != NONCONV) a.true_start[0] = a.q0s;
    } else if (a.conv_t[c - 1] != NONCONV) {
      a.true_start[c] = a.end_s[c - 1];
    }
}

// The join walked in order from each converged chunk (one thread per run of
// non-converged chunks): automata whose candidate lists are wider than the
// composed maps' rows (more than kJoinFan possible starting states).
__global__ void k_compose_serial(ScanArgs a) {
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > a.n_chunks) return;
  if (c > 0 && a.conv_t[c - 1] == NONCONV) return;
  uint32_t s = c == 0 ? a.q0s : a.end_s[c - 1];
  a.true_start[c] = s;
  for (uint64_t cc = c; cc < a.n_chunks && a.conv_t[cc] == NONCONV; ++cc) {
    const uint32_t slot = a.nc_slot[cc];
    s = a.nc_end[(uint64_t)slot * a.max_cand + find_cand(a, slot, s)];
    a.true_start[cc + 1] = s;
  }
}

// Count fix-up for the chunks the scan kernel could not join inside a wave
// (first lane of a tile, non-converged chunks and their successors):
// recount the prefix before the converging point from the true first state
// (the whole chunk if it did not converge), check the run lands on the
// converged state, and add the chunk's total.
template <int ENC, int SHIFT, int STEP>
__global__ __launch_bounds__(256) void k_fixup(ScanArgs a, int per_state, int direct) {
  static_assert(STEP == 1, "the fix-up walks one symbol per lookup");
  // one-symbol table in LDS: the recounts are chains of dependent lookups
  extern __shared__ __align__(16) char lds[];
  const uint64_t n_imp = a.n_tiles;  // the first chunk of every tile
  const uint64_t n_fix = n_imp + *a.fix_count;
  if ((uint64_t)blockIdx.x * blockDim.x >= n_fix) return;  // no item for this block
  copy_to_lds(lds, a.T1, a.n_states * 16u);
  __syncthreads();
  const Tab tb{nullptr, lds, a.q0s};
  uint64_t mine_sum = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_fix; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t c = i < n_imp ? i * TILE : a.fix_list[i - n_imp];
    const uint64_t lo = chunk_lo(a, c);
    const uint64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
    SinkGlobal sink{a.wtab, a.acc_out_off, a.acc_out_ids, per_state ? a.pat_counts : nullptr, a.app_count, a.app_keys,
                    a.app_cap};
    // direct: every chunk converged (no join kernels ran), so the true first
    // state is the predecessor's last state
    const uint32_t s0 = direct ? (c == 0 ? a.q0s : a.end_s[c - 1]) : a.true_start[c];
    uint64_t mine;
    const uint32_t ct = a.conv_t[c];
    if (direct && ct == NONCONV) {
      flag_error(a, 128u);
      mine = 0;
    } else if (ct == NONCONV && !per_state && !a.app_count) {
      // a weighted total only: the candidate runs counted the chunk
      const uint32_t slot = a.nc_slot[c];
      const uint64_t at = (uint64_t)slot * a.max_cand + find_cand(a, slot, s0);
      if (a.nc_end[at] != a.true_start[c + 1]) flag_error(a, 2u);
      mine = a.nc_cnt[at];
    } else if (ct == NONCONV) {
      const uint32_t e = scan_range<ENC, SHIFT, STEP>(a, tb, s0, lo, hi, sink);
      if (e != a.true_start[c + 1]) flag_error(a, 2u);
      mine = sink.cnt;
    } else {
      uint32_t e;
      if (i < n_imp) {  // symbols kept by the scan kernel
        const uint64_t* f = a.front + 3 * i;
        e = run_staged<SHIFT>(tb, s0, f[0], f[1], f[2], ct, lo, sink);
      } else {
        e = scan_range<ENC, SHIFT, STEP>(a, tb, s0, lo, lo + ct, sink);
      }
      if (e != a.conv_s[c]) flag_error(a, 4u);
      mine = (uint64_t)sink.cnt + a.tail_cnt[c];
    }
    if (a.chunk_cnt) a.chunk_cnt[c] = mine;
    mine_sum += mine;
  }
  for (int o = 32; o > 0; o >>= 1) mine_sum += __shfl_down(mine_sum, o);
  if ((threadIdx.x & 63) == 0 && mine_sum) atomicAdd(a.total, (unsigned long long)mine_sum);
}

// Exclusive prefix of per-chunk counts in three launches: a sum per tile of
// 1024 chunks (k_count_partials), an exclusive scan of those sums
// (k_scan_partials, one block), then a scan of every tile's own chunks from
// its tile offset (k_count_offsets).  The last tile writes the total to
// *a.total.
__global__ __launch_bounds__(kCountTile) void k_count_partials(ScanArgs a, uint64_t* part) {
  __shared__ uint64_t sh[kCountTile / 64];
  const uint64_t i = (uint64_t)blockIdx.x * kCountTile + threadIdx.x;
  const uint64_t v = i < a.n_chunks ? a.chunk_cnt[i] : 0;
  const uint64_t incl = block_incl_scan(v, sh);
  if (threadIdx.x == kCountTile - 1) part[blockIdx.x] = incl;
}

// Exclusive scan of the tile sums in place (one block, any number of tiles).
__global__ __launch_bounds__(kCountTile) void k_scan_partials(uint64_t* part, uint32_t n_tiles) {
  __shared__ uint64_t sh[kCountTile / 64];
  __shared__ uint64_t carry_sh;
  if (threadIdx.x == 0) carry_sh = 0;
  __syncthreads();
  for (uint32_t t0 = 0; t0 < n_tiles; t0 += kCountTile) {
    const uint32_t t = t0 + threadIdx.x;
    const uint64_t v = t < n_tiles ? part[t] : 0;
    const uint64_t carry = carry_sh;
    const uint64_t incl = block_incl_scan(v, sh);
    if (t < n_tiles) part[t] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == kCountTile - 1) carry_sh = carry + incl;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kCountTile) void k_count_offsets(ScanArgs a, const uint64_t* part, uint64_t* off) {
  __shared__ uint64_t sh[kCountTile / 64];
  const uint64_t base = part[blockIdx.x];
  const uint64_t i = (uint64_t)blockIdx.x * kCountTile + threadIdx.x;
  const uint64_t v = i < a.n_chunks ? a.chunk_cnt[i] : 0;
  const uint64_t incl = block_incl_scan(v, sh);
  if (i < a.n_chunks) off[i] = base + incl - v;
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kCountTile - 1) *a.total = base + incl;
}

// Second pass of "find": every chunk from its true first state, writing end
// positions at its offset (ordered within and across chunks).  MODE 1 writes
// per-chunk records instead.
template <int ENC, int SHIFT, int STEP, int MODE>
__global__ __launch_bounds__(kScanBlock) void k_emit(ScanArgs a) {
  extern __shared__ __align__(16) char lds[];
  if (STEP == 2) copy_to_lds(lds, a.T2, a.n_states * 64u);
  copy_to_lds(lds + a.lds_t1_off, a.T1, a.n_states * 16u);
  __syncthreads();
  const Tab tb{lds, lds + a.lds_t1_off, a.q0s};
  if (STEP == 2 && threadIdx.x == 0 && (uint32_t)(uintptr_t)(lds_c*)lds != 0u) flag_error(a, 64u);
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_chunks) return;
  const uint64_t lo = chunk_lo(a, c);
  const uint64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  const uint32_t s0 = a.true_start[c];
  if (MODE == 0) {
    SinkPositions sink{a.acc_out_off, a.acc_out_ids, a.pos_out, a.pat_out, a.chunk_off[c], a.pos_cap, a.first};
    scan_range<ENC, SHIFT, STEP>(a, tb, s0, lo, hi, sink);
    if (sink.cnt != a.chunk_cnt[c]) flag_error(a, 8u);
  } else {
    uint64_t* row = a.rec_counts + c * a.n_patterns;
    for (uint32_t p = 0; p < a.n_patterns; ++p) row[p] = 0;
    SinkRecord sink{a.acc_out_off, a.acc_out_ids, row};
    const uint32_t e = scan_range<ENC, SHIFT, STEP>(a, tb, s0, lo, hi, sink);
    a.rec_init[c] = s0 >> a.shift;
    a.rec_last[c] = e >> a.shift;
    if (e != a.true_start[c + 1]) flag_error(a, 16u);
  }
}

// ====================================================================== host runtime
// Scratch of coex_count_noalloc: one array per GPU, placed by the code object
// loader, held until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host it names a stand-in, not the device
// address): the address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
// The last 256 bytes of the array hold the failure word kept across
// coex_count_noalloc calls (zero at load, cleared when read).
constexpr size_t kStaticStickyAt = kStaticScratchBytes - 256;

struct DeviceCopy {
  int device = -1;
  char* buf = nullptr;
  size_t bytes = 0;
  uint32_t shift = 6;
  bool t2_exact = true;
  bool dense = false;  // accepting states are visited in many three-symbol steps (Dfa::match_density)
  // per encoding [0] = byte, [1] = 2-bit
  const uint32_t* T2[2] = {nullptr, nullptr};
  const uint16_t* T3[2] = {nullptr, nullptr};  // automata of at most kMaxStatesStep3 states
  const uint32_t* T1[2] = {nullptr, nullptr};
  const uint32_t* wtab = nullptr;
  const uint32_t* acc_out_off = nullptr;
  const uint32_t* acc_out_ids = nullptr;
  const uint32_t* pss_off[kMaxLookback + 1] = {};
  const uint16_t* pss_states[kMaxLookback + 1] = {};
  ~DeviceCopy() {
    if (buf) {
      int cur = -1;
      if (hipGetDevice(&cur) == hipSuccess && cur != device) (void)hipSetDevice(device);
      (void)hipFree(buf);
      if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    }
  }
};

Dfa::~Dfa() {
  for (DeviceCopy* d : dev) delete d;
}

namespace {

std::mutex g_mu;

struct Workspace {
  char* buf = nullptr;
  size_t bytes = 0;
  int device = -1;
  uint32_t* sticky = nullptr;  // failures of this stream's calls, kept until coex_errors_async reads them
  // event pairs around the scan kernel of calls made with COEX_FLAG_TIME
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t ev_used = 0;
};
constexpr size_t kMaxTimedLaunches = 4096;
std::map<std::pair<int, void*>, Workspace> g_ws;  // (device, stream) -> workspace

int dev_props(int dev, int& n_cu) {
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = cache.find(dev);
  if (it != cache.end()) { n_cu = it->second; return COEX_OK; }
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return COEX_EDEVICE;
  cache[dev] = p.multiProcessorCount;
  n_cu = p.multiProcessorCount;
  return COEX_OK;
}

// Column order of the device tables: column j holds the successor on code ord[j].
const int kOrd2bit[4] = {0, 1, 2, 3};  // A C G T
const int kOrdByte[4] = {0, 1, 3, 2};  // A C T G ((byte >> 1) & 3)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int upload(Dfa& d, int dev, DeviceCopy*& out) {
  std::lock_guard<std::mutex> lk(d.mu);
  if ((int)d.dev.size() > dev && d.dev[dev]) { out = d.dev[dev]; return COEX_OK; }
  const uint32_t n = d.n_states;
  auto dc = std::make_unique<DeviceCopy>();
  dc->device = dev;
  dc->shift = n <= kMaxStatesStep2 ? 6 : 4;
  dc->t2_exact = d.max_out <= 15;
  dc->dense = d.match_density > kDenseMatches;
  const uint32_t S = dc->shift;
  std::vector<uint32_t> w(d.n_accepting);
  for (uint32_t i = 0; i < d.n_accepting; ++i) {
    uint32_t s = d.acc_state[i];
    w[i] = d.out_off[s + 1] - d.out_off[s];
  }
  auto weight = [&](uint32_t s) -> uint32_t { return d.out_off[s + 1] - d.out_off[s]; };
  // host images
  std::vector<uint32_t> T1[2], T2[2];
  std::vector<uint16_t> T3[2];
  const bool has_t3 = S == 6 && n <= kMaxStatesStep3;
  for (int e = 0; e < 2; ++e) {
    const int* ord = e == 1 ? kOrd2bit : kOrdByte;
    T1[e].resize((size_t)n * 4);
    for (uint32_t s = 0; s < n; ++s)
      for (int j = 0; j < 4; ++j) {
        uint32_t t = d.delta[s * 4 + ord[j]];
        T1[e][s * 4 + j] = (t << S) | ((uint32_t)(d.acc_index[t] + 1) << 16);
      }
    if (S == 6) {
      T2[e].resize((size_t)n * 16);
      for (uint32_t s = 0; s < n; ++s)
        for (int g = 0; g < 16; ++g) {
          uint32_t s1 = d.delta[s * 4 + ord[g & 3]];
          uint32_t s2 = d.delta[s1 * 4 + ord[g >> 2]];
          uint32_t cnt = weight(s1) + weight(s2);
          if (!dc->t2_exact) cnt = cnt ? 1u : 0u;
          T2[e][s * 16 + g] = (s2 << 6) | (cnt << 24);
        }
    }
    if (has_t3) {
      // three symbols per entry: succ3 * 64 | (an accepting state among the
      // three visited); row n repeats row 0
      T3[e].resize((size_t)(n + 1) * 64);
      for (uint32_t s = 0; s < n; ++s)
        for (int g = 0; g < 64; ++g) {
          const uint32_t s1 = d.delta[s * 4 + ord[g & 3]];
          const uint32_t s2 = d.delta[s1 * 4 + ord[(g >> 2) & 3]];
          const uint32_t s3 = d.delta[s2 * 4 + ord[g >> 4]];
          const bool hit = d.acc_index[s1] >= 0 || d.acc_index[s2] >= 0 || d.acc_index[s3] >= 0;
          T3[e][(size_t)s * 64 + g] = (uint16_t)((s3 << 6) | (hit ? 1u : 0u));
        }
      std::copy(T3[e].begin(), T3[e].begin() + 64, T3[e].begin() + (size_t)n * 64);
    }
  }
  std::vector<uint32_t> aoff(d.n_accepting + 1, 0), aids;
  for (uint32_t i = 0; i < d.n_accepting; ++i) {
    uint32_t s = d.acc_state[i];
    aids.insert(aids.end(), d.out_ids.begin() + d.out_off[s], d.out_ids.begin() + d.out_off[s + 1]);
    aoff[i + 1] = (uint32_t)aids.size();
  }
  // layout
  struct Part { const void* src; size_t bytes; size_t off; };
  std::vector<Part> parts;
  size_t off = 0;
  auto add = [&](const void* src, size_t bytes) {
    parts.push_back({src, bytes, off});
    off = align_up(off + std::max<size_t>(bytes, 16), 256);
    return parts.size() - 1;
  };
  size_t iT2[2] = {0, 0}, iT3[2] = {0, 0}, iT1[2];
  for (int e = 0; e < 2; ++e) {
    if (S == 6) iT2[e] = add(T2[e].data(), T2[e].size() * 4);
    if (has_t3) iT3[e] = add(T3[e].data(), T3[e].size() * 2);
    iT1[e] = add(T1[e].data(), T1[e].size() * 4);
  }
  size_t iw = add(w.data(), w.size() * 4);
  size_t iao = add(aoff.data(), aoff.size() * 4);
  size_t iai = add(aids.data(), aids.size() * 4);
  size_t ipo[kMaxLookback + 1], ips[kMaxLookback + 1];
  for (uint32_t k = 1; k <= kMaxLookback; ++k) {
    ipo[k] = add(d.pss[k].off.data(), d.pss[k].off.size() * 4);
    ips[k] = add(d.pss[k].states.data(), d.pss[k].states.size() * 2);
  }
  dc->bytes = off;
  if (hipMalloc(&dc->buf, off) != hipSuccess) { dc->buf = nullptr; return COEX_ENOMEM; }
  std::vector<char> img(off, 0);
  for (auto& p : parts)
    if (p.bytes) std::memcpy(img.data() + p.off, p.src, p.bytes);
  if (hipMemcpy(dc->buf, img.data(), off, hipMemcpyHostToDevice) != hipSuccess) return COEX_EDEVICE;
  auto at = [&](size_t i) { return dc->buf + parts[i].off; };
  for (int e = 0; e < 2; ++e) {
    dc->T2[e] = S == 6 ? reinterpret_cast<const uint32_t*>(at(iT2[e])) : nullptr;
    dc->T3[e] = has_t3 ? reinterpret_cast<const uint16_t*>(at(iT3[e])) : nullptr;
    dc->T1[e] = reinterpret_cast<const uint32_t*>(at(iT1[e]));
  }
  dc->wtab = reinterpret_cast<const uint32_t*>(at(iw));
  dc->acc_out_off = reinterpret_cast<const uint32_t*>(at(iao));
  dc->acc_out_ids = reinterpret_cast<const uint32_t*>(at(iai));
  for (uint32_t k = 1; k <= kMaxLookback; ++k) {
    dc->pss_off[k] = reinterpret_cast<const uint32_t*>(at(ipo[k]));
    dc->pss_states[k] = reinterpret_cast<const uint16_t*>(at(ips[k]));
  }
  if ((int)d.dev.size() <= dev) d.dev.resize(dev + 1, nullptr);
  d.dev[dev] = dc.release();
  out = d.dev[dev];
  return COEX_OK;
}

// The device copy of an automaton's tables if it already exists (no upload).
int resident(Dfa& d, int dev, DeviceCopy*& out) {
  std::lock_guard<std::mutex> lk(d.mu);
  if ((int)d.dev.size() > dev && d.dev[dev]) { out = d.dev[dev]; return COEX_OK; }
  return COEX_ENOTRESIDENT;
}

// Device address of this GPU's static scratch array, looked up once per
// device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_at[kMaxDevices] = {};

int static_scratch(int dev, char*& out) {
  if (dev < 0 || dev >= kMaxDevices) return COEX_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return COEX_EDEVICE;
    g_scratch_at[dev] = static_cast<char*>(p);
  }
  out = g_scratch_at[dev];
  return COEX_OK;
}

// Grow-only scratch per (device, stream).
int workspace(int dev, void* stream, size_t bytes, char*& out, Workspace*& wsp) {
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace& w = g_ws[{dev, stream}];
  wsp = &w;
  if (!w.sticky) {
    if (hipMalloc(&w.sticky, 256) != hipSuccess) { w.sticky = nullptr; return COEX_ENOMEM; }
    if (hipMemset(w.sticky, 0, 256) != hipSuccess) return COEX_EDEVICE;
  }
  if (w.bytes < bytes) {
    if (w.buf) {
      if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return COEX_EDEVICE;
      (void)hipFree(w.buf);
      w.buf = nullptr;
      w.bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc(&w.buf, want) != hipSuccess) { w.buf = nullptr; return COEX_ENOMEM; }
    w.bytes = want;
    w.device = dev;
  }
  out = w.buf;
  return COEX_OK;
}

}  // namespace

// The kept failure word of the calls on (device, stream), creating the
// stream's workspace if it has none yet (for calls made on other streams on
// the caller's behalf).
int stream_sticky(int dev, void* stream, uint32_t** out) {
  char* buf = nullptr;
  Workspace* w = nullptr;
  const int rc = workspace(dev, stream, 0, buf, w);
  if (rc) return rc;
  *out = w->sticky;
  return COEX_OK;
}

namespace {

struct Plan {
  uint32_t shift, step, chains, block, k, group, max_cand, blocks, lds_bytes;
  uint32_t join_r;       // map row bytes of the parallel join (0: the serial join, more than kJoinFan candidates)
  uint32_t join_levels;  // composed levels above the level-0 maps
  bool t2_exact;         // two-symbol entries carry exact weighted counts
  bool all_conv;  // every chunk's candidates must agree inside the window (synchronising depth)
  bool direct;    // counts only and all_conv: no non-converged maps, no join kernels
  uint64_t chunk, n_chunks, n_tiles;
  bool hist;   // several patterns (or inexact two-symbol counts): visit histogram
  int mode;    // what the chunk scan reports: MODE_TOTAL, MODE_HIST or MODE_POS
  int enc;
};

// Bytes of LDS the chunk-scan kernel stages: two-symbol table (step 2),
// one-symbol table, weights and histogram.
constexpr uint32_t kPssLdsMax = 16 * 1024;  // larger PSS tables stay in global memory

uint32_t pss_lds_bytes(const Dfa& d, uint32_t k) {
  const uint32_t b = (uint32_t)align_up(d.pss[k].off.size() * 4, 16) + (uint32_t)align_up(d.pss[k].states.size() * 2, 16);
  return b <= kPssLdsMax ? b : 0u;
}

// Per-wave partial sums of the chunk-scan kernel (up to 16 waves per block).
constexpr uint32_t kTailRedBytes = 16 * 8;

// LDS bytes in front of the one-symbol table: the multi-symbol table.
uint32_t wide_table_bytes(uint32_t step, uint32_t n) { return step == 2 ? n * 64 : step == 3 ? (n + 1) * 128 : 0; }

uint32_t tail_lds_bytes(uint32_t step, const Dfa& d, uint32_t k) {
  const uint32_t n = d.n_states;
  const uint32_t acc = (uint32_t)align_up(d.n_accepting * 4, 16);
  return wide_table_bytes(step, n) + n * 16 + 2 * acc + pss_lds_bytes(d, k) + kTailRedBytes + 16;
}

TailKey tail_key(const Plan& P) { return TailKey{P.enc, (int)P.shift, (int)P.step, (int)P.chains, P.mode}; }

// Resident blocks per CU of the chunk-scan kernel the plan will launch.
uint32_t tail_blocks_per_cu(const Plan& P, const Dfa& d) {
  static std::mutex mu;
  static std::map<std::tuple<int, uint32_t, uint32_t, uint32_t, int, uint32_t>, int> cache;
  const uint32_t lds = tail_lds_bytes(P.step, d, P.k);
  const auto key = std::make_tuple(P.enc, P.shift, P.step, P.chains, P.mode, lds);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return (uint32_t)it->second;
  const int b = std::max(1, tail_occupancy(tail_key(P), lds));
  cache[key] = b;
  return (uint32_t)b;
}

int make_plan(const Dfa& d, const DeviceCopy& dc, const coex_seq& sq, const coex_opts* o, int n_cu, Plan& P,
              bool force_hist, bool positions = false) {
  P.enc = sq.encoding == COEX_ENC_2BIT ? 1 : 0;
  P.shift = dc.shift;
  P.t2_exact = dc.shift == 6 && dc.t2_exact;
  if (o && o->step > 3) return COEX_EINVAL;
  // default: three symbols per lookup when the automaton has a three-symbol
  // table (fewest dependent LDS reads per base) and matches rarely, else two,
  // else one
  const uint32_t dstep = dc.shift != 6 ? 1u : (dc.T3[0] && !dc.dense ? 3u : 2u);
  P.step = (o && o->step) ? o->step : dstep;
  if (P.step == 2 && dc.shift != 6) return COEX_EUNSUPPORTED;
  if (P.step == 3 && !dc.T3[0]) return COEX_EUNSUPPORTED;
  if (o && o->chains > 2) return COEX_EINVAL;
  P.chains = (o && o->chains) ? o->chains : 1u;
  if (P.chains == 2 && P.step == 1) return COEX_EUNSUPPORTED;
  // lookback
  if (o && o->lookback) {
    if (o->lookback > kMaxLookback) return COEX_EINVAL;
    P.k = o->lookback;
  } else {
    P.k = kMaxLookback;
    for (uint32_t k = 1; k <= kMaxLookback; ++k)
      if (d.pss[k].max_size <= 8) { P.k = k; break; }
    if (d.pss[P.k].max_size > 8)
      for (uint32_t k = 1; k <= kMaxLookback; ++k)
        if (d.pss[k].max_size <= 64) { P.k = k; break; }
  }
  const uint32_t mx = std::max<uint32_t>(1, d.pss[P.k].max_size);
  P.max_cand = mx;
  if (o && o->width) {
    if (o->width > 64 || (o->width & (o->width - 1))) return COEX_EINVAL;
    P.group = o->width;
  } else {
    uint32_t g = 1;
    while (g < mx && g < 64) g <<= 1;
    P.group = g;
  }
  const uint64_t n = sq.n_bases;
  P.hist = force_hist || d.n_patterns > 1 || (P.step == 2 && !dc.t2_exact);
  P.mode = positions ? MODE_POS : (P.hist ? MODE_HIST : MODE_TOTAL);
  P.block = (uint32_t)tail_block(tail_key(P));
  if (o && o->chunk) {
    P.chunk = o->chunk;
  } else {
    // one round of the chunk-scan kernel over the whole GPU: as many chunks
    // as lanes that can be resident at once (occupancy of the actual kernel
    // with its LDS), chunk length a multiple of 512 bases
    const uint64_t lanes = (uint64_t)n_cu * tail_blocks_per_cu(P, d) * P.block * P.chains;
    uint64_t c = (n + lanes - 1) / std::max<uint64_t>(1, lanes);
    c = std::max<uint64_t>(512, align_up(c, 512));
    // bound the non-converged scratch (chunks * candidates * 12 bytes) to 768 MiB
    while ((n / c + 1) * (uint64_t)mx * 12 > (768ull << 20)) c *= 2;
    P.chunk = c;
  }
  P.n_chunks = n == 0 ? 0 : (n + P.chunk - 1) / P.chunk;
  P.n_tiles = (P.n_chunks + TILE - 1) / TILE;
  // after d symbols any two runs agree (d = synchronising depth), so a chunk
  // whose window holds d symbols converges; chunk 0 starts exactly
  {
    const uint64_t last_len = P.n_chunks ? n - (P.n_chunks - 1) * P.chunk : 0;
    const uint64_t shortest = P.n_chunks > 1 ? std::min<uint64_t>(P.chunk, last_len) : (uint64_t)SPEC_WIN;
    // (a chunk with more candidates than lanes in its group is not speculated)
    P.all_conv = d.sync_depth != kNoSync && d.sync_depth <= std::min<uint64_t>(SPEC_WIN, shortest) &&
                 P.max_cand <= P.group;
  }
  return COEX_OK;
}

}  // namespace

int tail_block(const TailKey& k) {
  if (k.chains == 2) return k.step == 3 ? TailShape<3, 2>::kBlock : TailShape<2, 2>::kBlock;
  return k.step == 3 ? TailShape<3, 1>::kBlock : (k.step == 2 ? TailShape<2, 1>::kBlock : TailShape<1, 1>::kBlock);
}

int tail_occupancy(const TailKey& k, uint32_t lds) {
  if (k.enc == ENC_BYTE)
    return k.mode == MODE_POS ? tail_occupancy_byte_pos(k, lds)
           : k.mode == MODE_HIST ? tail_occupancy_byte_hist(k, lds) : tail_occupancy_byte_count(k, lds);
  return k.mode == MODE_POS ? tail_occupancy_2bit_pos(k, lds)
         : k.mode == MODE_HIST ? tail_occupancy_2bit_hist(k, lds) : tail_occupancy_2bit_count(k, lds);
}

bool tail_launch(const TailKey& k, uint32_t blocks, uint32_t lds, hipStream_t st, const ScanArgs& a) {
  if (k.enc == ENC_BYTE)
    return k.mode == MODE_POS ? tail_launch_byte_pos(k, blocks, lds, st, a)
           : k.mode == MODE_HIST ? tail_launch_byte_hist(k, blocks, lds, st, a)
                                 : tail_launch_byte_count(k, blocks, lds, st, a);
  return k.mode == MODE_POS ? tail_launch_2bit_pos(k, blocks, lds, st, a)
         : k.mode == MODE_HIST ? tail_launch_2bit_hist(k, blocks, lds, st, a)
                               : tail_launch_2bit_count(k, blocks, lds, st, a);
}

namespace {

// Events bracketing the scan kernel when the call asked for timing.
std::pair<hipEvent_t, hipEvent_t>* timing_slot(Workspace* w) {
  if (!w || w->ev_used >= kMaxTimedLaunches) return nullptr;
  if (w->ev_used == w->ev.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return nullptr;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return nullptr; }
    w->ev.push_back({a, b});
  }
  return &w->ev[w->ev_used++];
}

void launch_scan(const Plan& P, const ScanArgs& a, hipStream_t st, Workspace* timed) {
  // speculation and scan: one lane per chunk and chain, CH tiles of 64 chunks per wave
  const uint64_t tiles_per_block = (uint64_t)(P.block / 64) * P.chains;
  const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, (P.n_tiles + tiles_per_block - 1) / tiles_per_block);
  auto* ev = timed ? timing_slot(timed) : nullptr;
  if (ev) (void)hipEventRecord(ev->first, st);
  (void)tail_launch(tail_key(P), blocks, P.lds_bytes, st, a);
  if (ev) (void)hipEventRecord(ev->second, st);
}

// Buffers of the parallel join (level l: items of kJoinFan^l level-0 items).
struct JoinBufs {
  uint32_t* order = nullptr;  // rank -> chunk
  uint8_t* known = nullptr;   // known first index of items after a converged chunk
  uint64_t* part = nullptr;   // rank partial sums per tile of kCountTile chunks
  uint8_t* map[kJoinMaxLevels + 1] = {};
  uint8_t* x[kJoinMaxLevels + 1] = {};
};

uint32_t grid_for(uint64_t threads, int n_cu) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((threads + 255) / 256, (uint64_t)n_cu * 16));
}

void launch_join(const Plan& P, ScanArgs& a, const JoinBufs& J, int n_cu, hipStream_t st) {
  const uint64_t nc = P.n_chunks;
  if (!P.join_r) {
    hipLaunchKernelGGL(k_compose_serial, dim3(grid_for(nc + 1, n_cu)), dim3(256), 0, st, a);
    return;
  }
  const uint32_t R = P.join_r;
  const uint32_t tiles = (uint32_t)((nc + kCountTile - 1) / kCountTile);
  hipLaunchKernelGGL(k_rank_partials, dim3(tiles), dim3(kCountTile), 0, st, a, J.part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kCountTile), 0, st, J.part, tiles);
  hipLaunchKernelGGL(k_rank_offsets, dim3(tiles), dim3(kCountTile), 0, st, a, (const uint64_t*)J.part, J.order);
  hipLaunchKernelGGL(k_join_map0, dim3(grid_for(nc, n_cu)), dim3(256), 0, st, a, (const uint32_t*)J.order, J.map[0],
                     J.known, R);
  uint64_t div = 1;
  for (uint32_t l = 1; l <= P.join_levels; ++l, div *= kJoinFan) {
    const uint64_t n_up = (nc + div * kJoinFan - 1) / (div * kJoinFan);
    hipLaunchKernelGGL(k_join_up, dim3(grid_for(n_up * R, n_cu)), dim3(256), 0, st, (const uint32_t*)a.nc_count, div,
                       (const uint8_t*)J.map[l - 1], J.map[l], (const uint8_t*)J.known, R);
  }
  hipLaunchKernelGGL(k_join_top, dim3(1), dim3(1), 0, st, (const uint32_t*)a.nc_count, div,
                     (const uint8_t*)J.map[P.join_levels], (const uint8_t*)J.known, J.x[P.join_levels], R);
  for (uint32_t l = P.join_levels; l >= 1; --l) {
    div /= kJoinFan;
    const uint64_t n_up = (nc + div * kJoinFan - 1) / (div * kJoinFan);
    hipLaunchKernelGGL(k_join_down, dim3(grid_for(n_up, n_cu)), dim3(256), 0, st, (const uint32_t*)a.nc_count, div,
                       (const uint8_t*)J.map[l - 1], (const uint8_t*)J.x[l], J.x[l - 1], (const uint8_t*)J.known, R);
  }
  hipLaunchKernelGGL(k_join_finish, dim3(grid_for(nc + 1, n_cu)), dim3(256), 0, st, a, (const uint32_t*)J.order,
                     (const uint8_t*)J.x[0]);
}

template <int ENC, int SHIFT>
void launch_pipeline(const Plan& P, ScanArgs& a, const JoinBufs& J, int n_cu, hipStream_t st, uint64_t* counts,
                     bool emit_counts, Workspace* timed) {
  // counts go straight to the caller's buffer (zeroed here): per pattern from
  // the visit histograms, or the total of a one-pattern automaton
  a.pat_counts = emit_counts && P.hist ? reinterpret_cast<unsigned long long*>(counts) : nullptr;
  if (emit_counts && !P.hist && a.n_patterns > 0) a.total = reinterpret_cast<unsigned long long*>(counts);
  hipLaunchKernelGGL(k_init, dim3(64), dim3(256), 0, st, a, counts, emit_counts ? a.n_patterns : 0u);
  if (P.n_chunks == 0) return;
  launch_scan(P, a, st, timed);
  constexpr int DSTEP = 1;  // prefix recounts: one-symbol table staged in LDS
  // counts of an automaton that synchronises inside every chunk's window need
  // neither non-converged maps nor the true first state of every chunk (the
  // fix-up reads its predecessor's last state); positions and records do
  const bool direct = P.direct;
  if (!direct) {
    // one lane per (chunk, candidate) pair, up to 8 blocks per CU; two symbols
    // per lookup when the two-symbol table counts exactly
    const uint64_t pairs = P.n_chunks * a.nc_group;
    const uint32_t nb = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((pairs + 255) / 256, (uint64_t)n_cu * 8));
    auto go = [&](auto kern, uint32_t lds) {
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(kern, dim3(nb), dim3(256), lds, st, a);
    };
    if constexpr (SHIFT == 6) {
      if (P.t2_exact) go(k_nonconv<ENC, 6, 2>, a.n_states * 80u + 16u);
      else go(k_nonconv<ENC, 6, 1>, a.n_states * 16u + 16u);
    } else {
      go(k_nonconv<ENC, SHIFT, 1>, a.n_states * 16u + 16u);
    }
    launch_join(P, a, J, n_cu, st);
  }
  // every chunk of a tile's first lane and every chunk on the fix list: up to
  // 8 blocks per CU (blocks past the device's item count return at once)
  const uint32_t fb = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>((P.n_tiles + (direct ? 0 : P.n_chunks) + 255) / 256, (uint64_t)n_cu * 8));
  const uint32_t t1_lds = a.n_states * 16u + 16u;
  (void)hipFuncSetAttribute((const void*)k_fixup<ENC, SHIFT, DSTEP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)t1_lds);
  hipLaunchKernelGGL((k_fixup<ENC, SHIFT, DSTEP>), dim3(fb), dim3(256), t1_lds, st, a, (int)P.hist, (int)direct);
}

// Everything a scan call shares: validation, upload, plan, workspace, args.
struct Call {
  int dev = 0, n_cu = 0;
  Workspace* wsp = nullptr;
  bool timed = false;
  DeviceCopy* dc = nullptr;
  Plan P{};
  ScanArgs a{};
  hipStream_t st = nullptr;
  char* ws = nullptr;
  uint64_t* chunk_off = nullptr;
  uint64_t* count_part = nullptr;  // per tile of kCountTile chunks: its count
  JoinBufs join;
};

// emit_counts: the call returns counts only (direct mode possible).
// noalloc: tables must already be resident, scratch is the static array.
// positions: the chunk scan appends every match (find in one pass).
int prepare(const coex_dfa* h, const coex_seq* seq, const coex_opts* o, void* stream, bool force_hist,
            bool need_chunk_cnt, Call& C, bool emit_counts = false, bool noalloc = false, bool positions = false) {
  if (!h || !seq) return COEX_EINVAL;
  Dfa& d = *const_cast<Dfa*>(reinterpret_cast<const Dfa*>(h));
  if (seq->encoding != COEX_ENC_BYTE && seq->encoding != COEX_ENC_2BIT) return COEX_EINVAL;
  if (seq->n_bases > 0 && !seq->bases) return COEX_EINVAL;
  // where the sequence starts: byte sequences may start at any address (the
  // kernels read from the 16-byte boundary below it and skip the bases in
  // front); 2-bit buffers are 16-byte aligned and first_base picks the base.
  // Whole 128-base steps move the pointers (16-byte steps of codes and mask).
  const uint8_t* bases = static_cast<const uint8_t*>(seq->bases);
  const uint8_t* nmask = seq->encoding == COEX_ENC_2BIT ? seq->n_mask : nullptr;
  uint64_t first = seq->first_base;
  if (seq->encoding == COEX_ENC_BYTE) {
    const uintptr_t mis = (uintptr_t)bases & 15u;
    bases -= mis;
    first += mis;
  } else if (((uintptr_t)bases & 15u) || ((uintptr_t)nmask & 15u)) {
    return COEX_EINVAL;
  }
  if (first >= (1ull << 62) || seq->n_bases >= (1ull << 62)) return COEX_EINVAL;
  {
    const uint64_t skip = first & ~127ull;
    if (bases) bases += seq->encoding == COEX_ENC_BYTE ? skip : skip / 4;
    if (nmask) nmask += skip / 8;
    first -= skip;
  }
  if (hipGetDevice(&C.dev) != hipSuccess) return COEX_EDEVICE;
  int rc = dev_props(C.dev, C.n_cu);
  if (rc) return rc;
  if (noalloc && o && (o->flags & COEX_FLAG_TIME)) return COEX_EUNSUPPORTED;  // timing creates events
  rc = noalloc ? resident(d, C.dev, C.dc) : upload(d, C.dev, C.dc);
  if (rc) return rc;
  rc = make_plan(d, *C.dc, *seq, o, C.n_cu, C.P, force_hist, positions);
  if (rc) return rc;
  Plan& P = C.P;
  // counts and appended positions need no true first state of every chunk
  // when all chunks converge (the fix-up takes its predecessor's last state)
  P.direct = (emit_counts || positions) && P.all_conv;
  // chunk counts must fit the 32-bit per-chunk tail counter
  if (P.chunk > (0xFFFFFFFFull / std::max<uint32_t>(1, 2 * d.max_out + 1))) return COEX_EINVAL;
  const uint32_t S = P.shift;
  const uint32_t n = d.n_states;
  const uint32_t t1_off = wide_table_bytes(P.step, n);
  const uint32_t w_off = t1_off + n * 16;
  const uint32_t h_off = w_off + (uint32_t)align_up(d.n_accepting * 4, 16);
  uint32_t lds_end = h_off + (uint32_t)align_up(d.n_accepting * 4, 16);
  // the PSS table of the chosen lookback goes to LDS (after the histogram)
  // when it is small
  const uint32_t pss_n_off = (uint32_t)d.pss[P.k].off.size();
  const uint32_t pss_n_st = (uint32_t)d.pss[P.k].states.size();
  uint32_t spec_pss_off = 0, spec_pss_states = 0, a_red_off_tmp = 0;
  if (pss_lds_bytes(d, P.k)) {
    spec_pss_off = lds_end;
    spec_pss_states = lds_end + (uint32_t)align_up(pss_n_off * 4, 16);
    lds_end += pss_lds_bytes(d, P.k);
  }
  a_red_off_tmp = lds_end;  // per-wave partial sums of the scan kernel
  lds_end += kTailRedBytes;
  P.lds_bytes = lds_end + 16;
  // workspace layout
  const uint64_t nc = P.n_chunks;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o2 = off; off = align_up(off + std::max<size_t>(bytes, 8), 256); return o2; };
  size_t o_ct = take(nc * 4), o_cs = take(nc * 4), o_es = take(nc * 4), o_tc = take(nc * 4);
  size_t o_ncc = take(4), o_nch = take(nc * 4), o_nsl = take(nc * 4), o_nm = take(nc * 4);
  size_t o_fxc = take(4), o_fxl = take(nc * 4);
  // candidate maps of non-converged chunks: only when the join kernels run
  const uint64_t nc_maps = P.direct ? 0 : nc * P.max_cand;
  size_t o_nca = take(nc_maps * 4), o_nen = take(nc_maps * 4), o_ncn = take(nc_maps * 4);
  // the parallel join: order, known indices, rank partials, maps and indices per level
  P.join_r = 0;
  P.join_levels = 0;
  size_t o_jord = 0, o_jkn = 0, o_jpart = 0, o_jmap[kJoinMaxLevels + 1] = {}, o_jx[kJoinMaxLevels + 1] = {};
  if (!P.direct && P.max_cand <= kJoinFan) {
    uint32_t r = 1;
    while (r < P.max_cand) r <<= 1;
    P.join_r = r;
    uint64_t items = nc;
    while (items > kJoinFan) {
      items = (items + kJoinFan - 1) / kJoinFan;
      ++P.join_levels;
    }
    o_jord = take(nc * 4);
    o_jkn = take(nc);
    o_jpart = take((nc + kCountTile - 1) / kCountTile * 8);
    uint64_t n_l = nc;
    for (uint32_t l = 0; l <= P.join_levels; ++l) {
      o_jmap[l] = take(n_l * r);
      o_jx[l] = take(n_l);
      n_l = (n_l + kJoinFan - 1) / kJoinFan;
    }
  }
  size_t o_ts = take((nc + 1) * 4), o_tot = take(8), o_err = take(4), o_app = take(8);
  size_t o_front = take((size_t)P.n_tiles * 3 * 8);
  size_t o_cc = need_chunk_cnt ? take(nc * 8) : 0, o_co = need_chunk_cnt ? take(nc * 8) : 0;
  size_t o_part = need_chunk_cnt ? take((nc + kCountTile - 1) / kCountTile * 8) : 0;
  if (noalloc) {
    if (off > kStaticStickyAt) return COEX_ESCRATCH;
    rc = static_scratch(C.dev, C.ws);
    C.wsp = nullptr;
  } else {
    rc = workspace(C.dev, stream, off, C.ws, C.wsp);
  }
  if (rc) return rc;
  C.st = (hipStream_t)stream;
  C.timed = o && (o->flags & COEX_FLAG_TIME);
  ScanArgs& a = C.a;
  char* w = C.ws;
  a.bases = bases;
  a.nmask = nmask;
  a.first = first;
  a.n = first + seq->n_bases;
  a.chunk = P.chunk;
  a.n_chunks = P.n_chunks;
  a.n_tiles = P.n_tiles;
  const int e = P.enc;
  a.T2 = C.dc->T2[e];
  a.T3 = C.dc->T3[e];
  a.T1 = C.dc->T1[e];
  a.wtab = C.dc->wtab;
  a.n_states = n;
  a.n_acc = d.n_accepting;
  a.q0s = d.q0 << S;
  a.lds_t1_off = t1_off;
  a.lds_w_off = w_off;
  a.lds_hist_off = h_off;
  a.pss_off = C.dc->pss_off[P.k];
  a.pss_states = C.dc->pss_states[P.k];
  a.k = P.k;
  a.group = P.group;
  a.max_cand = P.max_cand;
  a.conv_t = reinterpret_cast<uint32_t*>(w + o_ct);
  a.conv_s = reinterpret_cast<uint32_t*>(w + o_cs);
  a.end_s = reinterpret_cast<uint32_t*>(w + o_es);
  a.tail_cnt = reinterpret_cast<uint32_t*>(w + o_tc);
  a.nc_count = reinterpret_cast<uint32_t*>(w + o_ncc);
  a.fix_count = reinterpret_cast<uint32_t*>(w + o_fxc);
  a.fix_list = reinterpret_cast<uint32_t*>(w + o_fxl);
  a.spec_pss_off = spec_pss_off;
  a.lds_red_off = a_red_off_tmp;
  a.spec_pss_states = spec_pss_states;
  a.pss_n_off = pss_n_off;
  a.pss_n_states = pss_n_st;
  a.nc_chunk = reinterpret_cast<uint32_t*>(w + o_nch);
  a.nc_slot = reinterpret_cast<uint32_t*>(w + o_nsl);
  a.nc_m = reinterpret_cast<uint32_t*>(w + o_nm);
  a.nc_cand = reinterpret_cast<uint32_t*>(w + o_nca);
  a.nc_end = reinterpret_cast<uint32_t*>(w + o_nen);
  a.nc_cnt = reinterpret_cast<uint32_t*>(w + o_ncn);
  {
    uint32_t g = 1;
    while (g < P.max_cand) g <<= 1;
    a.nc_group = g;
  }
  C.join = JoinBufs{};
  if (P.join_r) {
    C.join.order = reinterpret_cast<uint32_t*>(w + o_jord);
    C.join.known = reinterpret_cast<uint8_t*>(w + o_jkn);
    C.join.part = reinterpret_cast<uint64_t*>(w + o_jpart);
    for (uint32_t l = 0; l <= P.join_levels; ++l) {
      C.join.map[l] = reinterpret_cast<uint8_t*>(w + o_jmap[l]);
      C.join.x[l] = reinterpret_cast<uint8_t*>(w + o_jx[l]);
    }
  }
  a.true_start = reinterpret_cast<uint32_t*>(w + o_ts);
  a.total = reinterpret_cast<unsigned long long*>(w + o_tot);
  a.err = reinterpret_cast<uint32_t*>(w + o_err);
  a.err_sticky = noalloc ? reinterpret_cast<uint32_t*>(w + kStaticStickyAt) : C.wsp->sticky;
  a.app_count = positions ? reinterpret_cast<unsigned long long*>(w + o_app) : nullptr;
  a.app_keys = nullptr;
  a.app_cap = 0;
  a.front = reinterpret_cast<uint64_t*>(w + o_front);
  a.chunk_cnt = need_chunk_cnt ? reinterpret_cast<uint64_t*>(w + o_cc) : nullptr;
  C.chunk_off = need_chunk_cnt ? reinterpret_cast<uint64_t*>(w + o_co) : nullptr;
  C.count_part = need_chunk_cnt ? reinterpret_cast<uint64_t*>(w + o_part) : nullptr;
  a.chunk_off = C.chunk_off;
  a.acc_out_off = C.dc->acc_out_off;
  a.acc_out_ids = C.dc->acc_out_ids;
  a.n_patterns = d.n_patterns;
  a.shift = S;
  return COEX_OK;
}

void run_pipeline(Call& C, uint64_t* counts, bool emit_counts) {
  const bool b = C.P.enc == 0;
  const Plan& P = C.P;
  Workspace* t = C.timed ? C.wsp : nullptr;
  if (P.shift == 6) {
    if (b) launch_pipeline<ENC_BYTE, 6>(P, C.a, C.join, C.n_cu, C.st, counts, emit_counts, t);
    else launch_pipeline<ENC_2BIT, 6>(P, C.a, C.join, C.n_cu, C.st, counts, emit_counts, t);
  } else {
    if (b) launch_pipeline<ENC_BYTE, 4>(P, C.a, C.join, C.n_cu, C.st, counts, emit_counts, t);
    else launch_pipeline<ENC_2BIT, 4>(P, C.a, C.join, C.n_cu, C.st, counts, emit_counts, t);
  }
}

template <int MODE>
void launch_emit(Call& C) {
  const uint32_t blocks = (uint32_t)((C.P.n_chunks + kScanBlock - 1) / kScanBlock);
  // emit kernels always stage both tables (two-symbol table when it exists)
  C.a.lds_t1_off = C.P.shift == 6 ? C.a.n_states * 64u : 0u;
  const uint32_t lds = C.a.lds_t1_off + C.a.n_states * 16u + 16u;
  auto go = [&](auto kern) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(std::max(1u, blocks)), dim3(kScanBlock), lds, C.st, C.a);
  };
  const bool b = C.P.enc == 0;
  if (C.P.shift == 6) {
    if (b) go(k_emit<ENC_BYTE, 6, 2, MODE>); else go(k_emit<ENC_2BIT, 6, 2, MODE>);
  } else {
    if (b) go(k_emit<ENC_BYTE, 4, 1, MODE>); else go(k_emit<ENC_2BIT, 4, 1, MODE>);
  }
}

int check_err(Call& C) {
  uint32_t e = 0;
  if (hipMemcpyAsync(&e, C.a.err, 4, hipMemcpyDeviceToHost, C.st) != hipSuccess) return COEX_EDEVICE;
  if (hipStreamSynchronize(C.st) != hipSuccess) return COEX_EDEVICE;
  return e ? COEX_EINTERNAL : COEX_OK;
}

}  // namespace
}  // namespace coex

// ====================================================================== C ABI
using coex::Dfa;

extern "C" {

int coex_compile_kmers(const char* const* kmers, uint32_t n, coex_dfa** out) {
  if (!kmers || !out || n == 0) return COEX_EINVAL;
  try {
    std::vector<std::string> v;
    v.reserve(n);
    for (uint32_t i = 0; i < n; ++i) {
      if (!kmers[i]) return COEX_EINVAL;
      v.emplace_back(kmers[i]);
    }
    std::unique_ptr<Dfa> d;
    int rc = coex::compile_kmers(v, d);
    if (rc) return rc;
    *out = reinterpret_cast<coex_dfa*>(d.release());
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_compile_regex(const char* regex, coex_dfa** out) {
  if (!regex || !out) return COEX_EINVAL;
  try {
    std::unique_ptr<Dfa> d;
    int rc = coex::compile_regex(regex, d);
    if (rc) return rc;
    *out = reinterpret_cast<coex_dfa*>(d.release());
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_dfa_from_table(const uint32_t* delta, uint32_t n_states, uint32_t q0, const uint32_t* out_offsets,
                        const uint32_t* out_ids, uint32_t n_patterns, coex_dfa** out) {
  if (!out) return COEX_EINVAL;
  try {
    std::unique_ptr<Dfa> d;
    int rc = coex::from_table(delta, n_states, q0, out_offsets, out_ids, n_patterns, d);
    if (rc) return rc;
    *out = reinterpret_cast<coex_dfa*>(d.release());
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_dfa_info(const coex_dfa* h, coex_dfa_info_t* info) {
  if (!h || !info) return COEX_EINVAL;
  const Dfa& d = *reinterpret_cast<const Dfa*>(h);
  info->n_states = d.n_states;
  info->n_patterns = d.n_patterns;
  info->n_accepting = d.n_accepting;
  info->q0 = d.q0;
  info->sync_depth = d.sync_depth;
  info->max_out = d.max_out;
  info->max_pss[0] = d.n_states;
  for (uint32_t k = 1; k <= coex::kMaxLookback; ++k) info->max_pss[k] = d.pss[k].max_size;
  return COEX_OK;
}

int coex_dfa_export(const coex_dfa* h, uint32_t* delta, uint32_t* out_offsets, uint32_t* out_ids) {
  if (!h) return COEX_EINVAL;
  const Dfa& d = *reinterpret_cast<const Dfa*>(h);
  if (delta) std::memcpy(delta, d.delta.data(), d.delta.size() * 4);
  if (out_offsets) std::memcpy(out_offsets, d.out_off.data(), d.out_off.size() * 4);
  if (out_ids && !d.out_ids.empty()) std::memcpy(out_ids, d.out_ids.data(), d.out_ids.size() * 4);
  return COEX_OK;
}

void coex_dfa_free(coex_dfa* h) { delete reinterpret_cast<Dfa*>(h); }

int coex_count(const coex_dfa* dfa, const coex_seq* seq, uint64_t* counts_dev, const coex_opts* opts,
               void* stream) {
  if (!counts_dev) return COEX_EINVAL;
  try {
    coex::Call C;
    int rc = coex::prepare(dfa, seq, opts, stream, false, false, C, true);
    if (rc) return rc;
    coex::run_pipeline(C, counts_dev, true);
    if (hipGetLastError() != hipSuccess) return COEX_EDEVICE;
    if (opts && (opts->flags & COEX_FLAG_CHECK)) return coex::check_err(C);
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_count_noalloc(const coex_dfa* dfa, const coex_seq* seq, uint64_t* counts_dev, const coex_opts* opts,
                       void* stream) {
  if (!counts_dev) return COEX_EINVAL;
  try {
    coex::Call C;
    int rc = coex::prepare(dfa, seq, opts, stream, false, false, C, true, true);
    if (rc) return rc;
    coex::run_pipeline(C, counts_dev, true);
    if (hipGetLastError() != hipSuccess) return COEX_EDEVICE;
    if (opts && (opts->flags & COEX_FLAG_CHECK)) return coex::check_err(C);
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_errors_async(void* stream, uint32_t* flags_out) {
  if (!flags_out) return COEX_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return COEX_EDEVICE;
  uint32_t* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(coex::g_mu);
    auto it = coex::g_ws.find({dev, stream});
    if (it != coex::g_ws.end()) ws = it->second.sticky;
  }
  char* sp = nullptr;
  if (coex::static_scratch(dev, sp) != COEX_OK) return COEX_EDEVICE;
  hipLaunchKernelGGL(coex::k_take_errors, dim3(1), dim3(64), 0, (hipStream_t)stream, ws,
                     reinterpret_cast<uint32_t*>(sp + coex::kStaticStickyAt), flags_out);
  return hipGetLastError() == hipSuccess ? COEX_OK : COEX_EDEVICE;
}

}  // extern "C"

namespace coex {
namespace {

// find in one pass: the chunk scan and the fix-up append every match as a
// key (end position << 24 | pattern id) to the caller's position buffer
// (positions are final when found: the scan runs from converging points, the
// prefixes from true first states); one synchronisation reads the total,
// then the keys are sorted and split into positions and pattern ids.
int find_one_pass(const coex_dfa* dfa, const coex_seq* seq, int64_t* pos_dev, uint32_t* pattern_dev,
                  uint64_t capacity, uint64_t* n_found, const coex_opts* opts, void* stream) {
  Call C;
  int rc = prepare(dfa, seq, opts, stream, false, false, C, false, false, true);
  if (rc) return rc;
  C.a.app_keys = reinterpret_cast<uint64_t*>(pos_dev);
  C.a.app_cap = pos_dev ? capacity : 0;
  run_pipeline(C, nullptr, false);
  uint64_t total = 0;
  uint32_t e = 0;
  if (C.P.n_chunks) {
    if (hipMemcpyAsync(&total, C.a.app_count, 8, hipMemcpyDeviceToHost, C.st) != hipSuccess) return COEX_EDEVICE;
    if (hipMemcpyAsync(&e, C.a.err, 4, hipMemcpyDeviceToHost, C.st) != hipSuccess) return COEX_EDEVICE;
  }
  if (hipStreamSynchronize(C.st) != hipSuccess) return COEX_EDEVICE;
  if (e) return COEX_EINTERNAL;
  *n_found = total;
  if (total > capacity) return COEX_ECAPACITY;
  if (total == 0) return COEX_OK;
  char* tmp = nullptr;
  size_t temp_bytes = 0;
  if (total > kSmallSortKeys) {
    temp_bytes = sort_temp_bytes(total);
    Workspace* wsp = nullptr;
    rc = workspace(C.dev, stream, align_up(total * 8, 256) + temp_bytes, tmp, wsp);
    if (rc) return rc;
  }
  if (sort_match_keys(reinterpret_cast<const uint64_t*>(pos_dev), reinterpret_cast<uint64_t*>(tmp), total,
                      tmp ? tmp + align_up(total * 8, 256) : nullptr, temp_bytes, pos_dev, pattern_dev, C.a.first,
                      C.st))
    return COEX_EDEVICE;
  return COEX_OK;
}

// find in two passes (chunk counts, their prefix, then each chunk again from
// its true first state writing at its offset): automata with more than 2^24
// pattern ids, sequences of 2^40 bases or more, or two chains per lane.
int find_two_pass(const coex_dfa* dfa, const coex_seq* seq, int64_t* pos_dev, uint32_t* pattern_dev,
                  uint64_t capacity, uint64_t* n_found, const coex_opts* opts, void* stream) {
  Call C;
  int rc = prepare(dfa, seq, opts, stream, false, true, C);
  if (rc) return rc;
  run_pipeline(C, nullptr, false);
  uint64_t total = 0;
  if (C.P.n_chunks) {
    const uint32_t tiles = (uint32_t)((C.P.n_chunks + kCountTile - 1) / kCountTile);
    hipLaunchKernelGGL(k_count_partials, dim3(tiles), dim3(kCountTile), 0, C.st, C.a, C.count_part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kCountTile), 0, C.st, C.count_part, tiles);
    hipLaunchKernelGGL(k_count_offsets, dim3(tiles), dim3(kCountTile), 0, C.st, C.a, C.count_part, C.chunk_off);
  }
  if (hipMemcpyAsync(&total, C.a.total, 8, hipMemcpyDeviceToHost, C.st) != hipSuccess) return COEX_EDEVICE;
  uint32_t e = 0;
  if (hipMemcpyAsync(&e, C.a.err, 4, hipMemcpyDeviceToHost, C.st) != hipSuccess) return COEX_EDEVICE;
  if (hipStreamSynchronize(C.st) != hipSuccess) return COEX_EDEVICE;
  if (e) return COEX_EINTERNAL;
  *n_found = total;
  if (total > capacity) return COEX_ECAPACITY;
  if (total == 0) return COEX_OK;
  C.a.pos_out = pos_dev;
  C.a.pat_out = pattern_dev;
  C.a.pos_cap = capacity;
  launch_emit<0>(C);
  if (hipGetLastError() != hipSuccess) return COEX_EDEVICE;
  return check_err(C);
}

}  // namespace
}  // namespace coex

extern "C" {

int coex_find(const coex_dfa* dfa, const coex_seq* seq, int64_t* pos_dev, uint32_t* pattern_dev,
              uint64_t capacity, uint64_t* n_found, const coex_opts* opts, void* stream) {
  if (!n_found || (capacity && !pos_dev)) return COEX_EINVAL;
  if (!dfa || !seq) return COEX_EINVAL;
  try {
    const Dfa& d = *reinterpret_cast<const Dfa*>(dfa);
    const bool one_pass = d.n_patterns <= (1u << 24) && seq->n_bases < (1ull << 40) - 256 && (!opts || opts->chains <= 1);
    return one_pass ? coex::find_one_pass(dfa, seq, pos_dev, pattern_dev, capacity, n_found, opts, stream)
                    : coex::find_two_pass(dfa, seq, pos_dev, pattern_dev, capacity, n_found, opts, stream);
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_count_find(const coex_dfa* dfa, const coex_seq* seq, uint64_t* counts_dev, int64_t* pos_dev,
                    uint32_t* pattern_dev, uint64_t capacity, uint64_t* n_found, const coex_opts* opts, void* stream) {
  if (!dfa || !counts_dev) return COEX_EINVAL;
  try {
    const Dfa& d = *reinterpret_cast<const Dfa*>(dfa);
    if (d.n_patterns > 1 && capacity && !pattern_dev) return COEX_EINVAL;
    const int rc = coex_find(dfa, seq, pos_dev, pattern_dev, capacity, n_found, opts, stream);
    if (rc) return rc;
    // several patterns and no id buffer: capacity 0, so no match was found
    if (coex::counts_from_ids(d.n_patterns > 1 ? pattern_dev : nullptr, *n_found, d.n_patterns, counts_dev,
                              (hipStream_t)stream))
      return COEX_EDEVICE;
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_count_chunks(const coex_dfa* dfa, const coex_seq* seq, uint32_t chunk, uint32_t* init_dev,
                      uint32_t* last_dev, uint64_t* counts_dev, void* stream) {
  if (!init_dev || !last_dev || !counts_dev || chunk == 0) return COEX_EINVAL;
  try {
    coex_opts o{};
    o.chunk = chunk;
    coex::Call C;
    int rc = coex::prepare(dfa, seq, &o, stream, false, true, C);
    if (rc) return rc;
    coex::run_pipeline(C, nullptr, false);
    C.a.rec_counts = counts_dev;
    C.a.rec_init = init_dev;
    C.a.rec_last = last_dev;
    if (C.P.n_chunks == 0) {
      // one empty chunk: (q0, q0, zeros)
      const Dfa& d = *reinterpret_cast<const Dfa*>(dfa);
      uint32_t q = d.q0;
      if (hipMemcpyAsync(init_dev, &q, 4, hipMemcpyHostToDevice, C.st) != hipSuccess ||
          hipMemcpyAsync(last_dev, &q, 4, hipMemcpyHostToDevice, C.st) != hipSuccess)
        return COEX_EDEVICE;
      std::vector<uint64_t> z(std::max<uint32_t>(1, d.n_patterns), 0);
      if (d.n_patterns &&
          hipMemcpyAsync(counts_dev, z.data(), 8 * d.n_patterns, hipMemcpyHostToDevice, C.st) != hipSuccess)
        return COEX_EDEVICE;
      if (hipStreamSynchronize(C.st) != hipSuccess) return COEX_EDEVICE;
      return COEX_OK;
    }
    coex::launch_emit<1>(C);
    if (hipGetLastError() != hipSuccess) return COEX_EDEVICE;
    return coex::check_err(C);
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

const char* coex_strerror(int s) {
  switch (s) {
    case COEX_OK: return "ok";
    case COEX_EINVAL: return "invalid argument";
    case COEX_EALPHABET: return "pattern empty or outside A,C,G,T";
    case COEX_ETOOBIG: return "automaton too large for the device tables";
    case COEX_ENOMEM: return "out of memory";
    case COEX_ECAPACITY: return "result buffer too small";
    case COEX_EDEVICE: return "HIP runtime error";
    case COEX_EUNSUPPORTED: return "unsupported option combination";
    case COEX_ESYNTAX: return "regular expression syntax error or empty match";
    case COEX_EINTERNAL: return "device consistency check failed";
    case COEX_ESCRATCH: return "call needs more scratch than the static array of coex_count_noalloc holds";
    case COEX_ENOTRESIDENT: return "automaton tables not yet on this device (any allocating scan call puts them there)";
    default: return "unknown status";
  }
}

int coex_profile(void* stream, double* total_ms, uint64_t* launches, int reset) {
  if (!total_ms || !launches) return COEX_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return COEX_EDEVICE;
  std::lock_guard<std::mutex> lk(coex::g_mu);
  auto it = coex::g_ws.find({dev, stream});
  double sum = 0.0;
  uint64_t cnt = 0;
  if (it != coex::g_ws.end()) {
    coex::Workspace& w = it->second;
    for (size_t i = 0; i < w.ev_used; ++i) {
      if (hipEventSynchronize(w.ev[i].second) != hipSuccess) return COEX_EDEVICE;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, w.ev[i].first, w.ev[i].second) != hipSuccess) return COEX_EDEVICE;
      sum += ms;
      ++cnt;
    }
    if (reset) w.ev_used = 0;
  }
  *total_ms = sum;
  *launches = cnt;
  return COEX_OK;
}

const char* coex_version(void) { return "coex 0.1 gfx950"; }

}  // extern "C"
