// The chunk-scan kernel k_tail and the device helpers it shares with the
// other kernels of libcoex: symbol staging, the speculation of a tile and the
// scan/join of its chunks (Section III of the paper, Algorithm 1, laid out for
// one MI355X; see coex.hip for the whole pipeline).  k_tail is instantiated in
// one translation unit per sequence encoding and count kind
// (tail_<enc>_<kind>.hip), which also launch it.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace coex {

constexpr int kScanBlock = COEX_SCAN_BLOCK;

__device__ __forceinline__ void copy_to_lds(char* dst, const void* src, uint32_t bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  for (uint32_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

// First SPEC_WIN symbols of [lo, hi) for block-unaligned chunk starts
// (aligned starts take them from the chunk's first block).
template <int ENC>
__device__ __forceinline__ void stage_symbols(const ScanArgs& a, uint64_t lo, uint64_t hi, uint64_t& sy0,
                                              uint64_t& sy1, uint64_t& rs) {
  uint32_t c[4] = {0, 0, 0, 0}, r[4] = {0, 0, 0, 0};
  for (uint32_t i = 0; i < SPEC_WIN && lo + i < hi; ++i) {
    const int col = load_col<ENC>(a, lo + i);
    const uint32_t bit = col < 0 ? 0u : (uint32_t)col;
    const uint32_t w = i >> 4, sh = 2 * (i & 15), rb = col < 0 ? 1u << (i & 15) : 0u;
    c[0] |= w == 0 ? bit << sh : 0u;
    c[1] |= w == 1 ? bit << sh : 0u;
    c[2] |= w == 2 ? bit << sh : 0u;
    c[3] |= w == 3 ? bit << sh : 0u;
    r[0] |= w == 0 ? rb : 0u;
    r[1] |= w == 1 ? rb : 0u;
    r[2] |= w == 2 ? rb : 0u;
    r[3] |= w == 3 ? rb : 0u;
  }
  sy0 = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
  sy1 = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
  rs = (uint64_t)r[0] | ((uint64_t)r[1] << 16) | ((uint64_t)r[2] << 32) | ((uint64_t)r[3] << 48);
}

// First SPEC_WIN symbols of a chunk starting at lo with lo % 64 == 0 and
// lo + 64 <= n: one 16-byte load of codes and one 8-byte load of N bits
// (2-bit), or four 16-byte loads (bytes).
template <int ENC>
__device__ __forceinline__ void front_symbols(const ScanArgs& a, uint64_t lo, uint64_t& sy0, uint64_t& sy1,
                                              uint64_t& rs) {
  if constexpr (ENC == ENC_2BIT) {
    const uint4 v = *reinterpret_cast<const uint4*>(a.bases + (lo >> 2));
    sy0 = (uint64_t)v.x | ((uint64_t)v.y << 32);
    sy1 = (uint64_t)v.z | ((uint64_t)v.w << 32);
    if (a.nmask) {
      const uint2 mm = *reinterpret_cast<const uint2*>(a.nmask + (lo >> 3));
      rs = (uint64_t)mm.x | ((uint64_t)mm.y << 32);
    } else {
      rs = 0;
    }
  } else {
    Block<ENC_BYTE> b;
#pragma unroll
    for (int i = 0; i < 4; ++i) b.r[i] = *reinterpret_cast<const uint4*>(a.bases + lo + 16 * i);
    uint32_t c[4], r[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) b.word(w, c[w], r[w]);
    sy0 = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
    sy1 = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
    rs = (uint64_t)r[0] | ((uint64_t)r[1] << 16) | ((uint64_t)r[2] << 32) | ((uint64_t)r[3] << 48);
  }
}

// Runs `count` (<= SPEC_WIN) staged symbols from s.
template <int SHIFT, class Sink>
__device__ __forceinline__ uint32_t run_staged(const Tab& tb, uint32_t s, uint64_t sy0, uint64_t sy1, uint64_t rs,
                                               uint32_t count, uint64_t p, Sink& sink) {
  for (uint32_t t = 0; t < count; ++t) {
    const int col = (rs & 1u) ? -1 : (int)(sy0 & 3u);
    s = step1<SHIFT>(tb, s, col, p + t, sink);
    sy0 = (sy0 >> 2) | (sy1 << 62);
    sy1 >>= 2;
    rs >>= 1;
  }
  return s;
}

// Slots in a list for the lanes of a wave that set `take` (all lanes of the
// wave call it): one atomic add of the wave's count on the list's counter,
// each lane's slot = the old value + the lanes before it that take one.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool take) {
  const unsigned long long bm = __ballot(take);
  if (bm == 0) return 0;
  const int leader = __ffsll((long long)bm) - 1;
  const uint32_t lane = threadIdx.x & 63;
  uint32_t base = 0;
  if ((int)lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(bm));
  base = __shfl(base, leader);
  return base + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull));
}

// Speculation for one tile of 64 chunks (one wave): possible starting states
// from the lookback table, then rounds in which G lanes run the candidates
// of one chunk in lockstep over its first symbols until they agree (the
// converging point of Algorithm 1).  Writes conv_t / conv_s per chunk (and
// returns this lane's pair), or queues the chunk as non-converged.
template <int ENC, int SHIFT>
__device__ __forceinline__ void spec_tile(const ScanArgs& a, const Tab& tb, const uint32_t* pss_off,
                                          const uint16_t* pss_states, uint64_t tile_id, uint32_t& out_t,
                                          uint32_t& out_s) {
  const int lane = threadIdx.x & 63;
  const uint64_t c = tile_id * TILE + lane;
  const bool valid = c < a.n_chunks;
  const uint64_t lo = valid ? chunk_lo(a, c) : 0;
  const uint64_t hi = valid ? (lo + a.chunk < a.n ? lo + a.chunk : a.n) : 0;
  uint32_t m = 0, cbase = 0, exact = 0;
  bool is_exact = false;
  uint64_t sy0 = 0, sy1 = 0, rs = 0;
  if (valid) {
    if ((lo & 63) == 0 && lo + SPEC_WIN <= a.n) front_symbols<ENC>(a, lo, sy0, sy1, rs);
    else stage_symbols<ENC>(a, lo, hi, sy0, sy1, rs);
    chunk_header<ENC, SHIFT>(a, tb, pss_off, lo, m, cbase, exact, is_exact);
  }
  const uint32_t len = (uint32_t)((hi - lo) < SPEC_WIN ? (hi - lo) : SPEC_WIN);
  const uint32_t G = a.group;
  const uint32_t R = 64u / G;
  const uint32_t gidx = lane / G, gi = lane % G, gl = lane & ~(G - 1);
  const unsigned long long gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  uint32_t my_t = NONCONV, my_s = 0;
  for (uint32_t r = 0; r < G; ++r) {
    const int owner = (int)(r * R + gidx);
    const uint32_t om = __shfl(m, owner);
    const uint32_t ocb = __shfl(cbase, owner);
    const uint32_t oex = __shfl(exact, owner);
    const int oisx = __shfl((int)is_exact, owner);
    const uint32_t olen = __shfl(len, owner);
    uint64_t o0 = __shfl(sy0, owner), o1 = __shfl(sy1, owner), orr = __shfl(rs, owner);
    const bool act = om > 0 && om <= G;
    uint32_t s = tb.q0s;
    if (act) s = oisx ? oex : ((uint32_t)pss_states[ocb + (gi < om ? gi : om - 1)] << SHIFT);
    uint32_t res_t = NONCONV, res_s = 0;
    for (uint32_t t = 0; t <= (uint32_t)SPEC_WIN; ++t) {
      const uint32_t lead = __shfl(s, (int)gl);
      const unsigned long long ne = __ballot(act && s != lead);
      const bool gdone = ((ne >> gl) & gmask) == 0;
      if (act && gdone && res_t == NONCONV && t <= olen) { res_t = t; res_s = s; }
      const bool pending = act && res_t == NONCONV && t < olen;
      if (__ballot(pending) == 0) break;
      const int col = (orr & 1u) ? -1 : (int)(o0 & 3u);
      s = col < 0 ? tb.q0s : (t1_lookup<SHIFT>(tb, s, (uint32_t)col) & 0xFFFFu);
      o0 = (o0 >> 2) | (o1 << 62);
      o1 >>= 2;
      orr >>= 1;
    }
    const int src = (int)(((uint32_t)lane - r * R) * G) & 63;
    const uint32_t rt = __shfl(res_t, src);
    const uint32_t rv = __shfl(res_s, src);
    if ((uint32_t)lane >= r * R && (uint32_t)lane < r * R + R) {
      my_t = rt;
      my_s = rv;
    }
  }
  out_t = my_t;
  out_s = my_s;
  // queue the non-converged chunks: one counter update per wave
  const bool queue = valid && my_t == NONCONV;
  const uint32_t slot = wave_append(a.nc_count, queue);
  if (!valid) return;
  if (queue) {
    a.nc_chunk[slot] = (uint32_t)c;
    a.nc_slot[c] = slot;
  }
  a.conv_t[c] = my_t;
  a.conv_s[c] = my_s;
}

// Sinks of the chunk-scan kernel.  Its tables, weights and histogram sit in
// LDS at fixed offsets (the kernel declares no other LDS, so dynamic LDS
// starts at address 0), so the base-by-base path of a word (reset
// boundaries, replays of words with matches) is one out-of-line routine
// taking those offsets: the unrolled hot loop keeps one call per word
// instead of an inlined copy of the rare path.
typedef __attribute__((address_space(3))) uint32_t lds_u32_rw;

// What the chunk-scan kernel reports: a one-pattern weighted total, the
// per-final-state visit histogram (several patterns), or every match as an
// append of (end position, pattern id) keys, in no particular order (find).
constexpr int MODE_TOTAL = 0;
constexpr int MODE_HIST = 1;
constexpr int MODE_POS = 2;

// Where positions-mode matches go: the output sets (global memory) and the
// append buffer of keys end position << 24 | pattern id.
struct AppendTo {
  const uint32_t* out_off;
  const uint32_t* out_ids;
  unsigned long long* count;
  uint64_t* keys;
  uint64_t cap;
};

// Appends the matches ending at position p in accepting state `acc`.
__device__ __forceinline__ void append_matches(const uint32_t* out_off, const uint32_t* out_ids,
                                               unsigned long long* count, uint64_t* keys, uint64_t cap, uint64_t p,
                                               uint32_t acc) {
  for (uint32_t j = out_off[acc]; j < out_off[acc + 1]; ++j) {
    const unsigned long long i = atomicAdd(count, 1ull);
    if (i < cap) keys[i] = p << 24 | out_ids[j];
  }
}

// The base-by-base path of one word (reset boundaries, replays of words with
// matches), out of line; scalar arguments only (a pointer to the kernel's
// argument block would make the kernel copy it to private memory).
template <int SHIFT, int MODE>
__device__ __noinline__ uint64_t tail_word_slow(uint32_t t1_off, uint32_t q0s, uint32_t w_off, uint32_t hist_off,
                                                uint32_t s, uint32_t cols, uint32_t rst, uint32_t act, uint64_t p,
                                                const uint32_t* out_off, const uint32_t* out_ids,
                                                unsigned long long* count, uint64_t* keys, uint64_t cap) {
  uint32_t cnt = 0;
  for (int i = 0; i < 16; ++i) {
    if (!((act >> i) & 1u)) continue;
    if ((rst >> i) & 1u) {
      s = q0s;
      continue;
    }
    const uint32_t e = lds_at(t1_off + (s >> (SHIFT - 4)) + ((cols >> (2 * i)) & 3u) * 4u);
    const uint32_t acc = e >> 16;
    if (acc) {
      cnt += lds_at(w_off + 4u * (acc - 1u));
      if (MODE == MODE_HIST)
        __atomic_fetch_add((lds_u32_rw*)(uintptr_t)(hist_off + 4u * (acc - 1u)), 1u, __ATOMIC_RELAXED);
      if (MODE == MODE_POS) append_matches(out_off, out_ids, count, keys, cap, p + (uint64_t)i, acc - 1u);
    }
    s = e & 0xFFFFu;
  }
  return (uint64_t)s | ((uint64_t)cnt << 32);
}

template <int MODE>
struct SinkTail {
  static constexpr bool kReplay = MODE != MODE_TOTAL;  // one-pattern totals take exact multi-symbol counts
  static constexpr bool kOutline = true;
  uint32_t t1_off, q0s, w_off, hist_off;
  AppendTo app;  // MODE_POS
  uint32_t cnt = 0;
  __device__ void word(uint32_t c) {
    if (MODE == MODE_TOTAL) cnt += c;
  }
  __device__ void hit(uint64_t p, uint32_t acc) {
    cnt += lds_at(w_off + 4u * acc);
    if (MODE == MODE_HIST) __atomic_fetch_add((lds_u32_rw*)(uintptr_t)(hist_off + 4u * acc), 1u, __ATOMIC_RELAXED);
    if (MODE == MODE_POS) append_matches(app.out_off, app.out_ids, app.count, app.keys, app.cap, p, acc);
  }
  template <int SHIFT>
  __device__ uint32_t slow(uint32_t s, uint32_t cols, uint32_t rst, uint32_t act, uint64_t p) {
    uint64_t r;
    if constexpr (MODE == MODE_POS)
      r = tail_word_slow<SHIFT, MODE>(t1_off, q0s, w_off, hist_off, s, cols, rst, act, p, app.out_off, app.out_ids,
                                      app.count, app.keys, app.cap);
    else
      r = tail_word_slow<SHIFT, MODE>(t1_off, q0s, w_off, hist_off, s, cols, rst, act, p, nullptr, nullptr, nullptr,
                                      nullptr, 0);
    cnt += (uint32_t)(r >> 32);
    return (uint32_t)r;
  }
};

// Launch shape of the chunk-scan kernel.  The three-symbol table leaves room
// for one block per CU: 1024 threads with one chain per lane (4 waves per
// SIMD, up to 128 registers), 768 with two chains (3 waves per SIMD, up to
// 168 registers for two register blocks of sequence).  The other tables fit
// two blocks of 768 per CU (6 waves per SIMD, up to 85 registers).
template <int STEP, int CH>
struct TailShape {
  static constexpr int kBlock = (STEP == 3 && CH == 1) ? 1024 : kScanBlock;
  static constexpr int kMinWaves = CH == 2 ? 3 : (STEP == 3 ? 4 : COEX_TAIL_WAVES);
};

// Speculation, then the scan of each chunk from its converging point (one
// lane per chunk and chain), then the join inside the wave: the predecessor
// lane's last state is this chunk's true first state, from which the prefix
// before the converging point is recounted.  Each wave owns CH tiles of 64
// consecutive chunks (tiles CH*w .. CH*w + CH - 1 of global wave w) and first
// runs the speculation of each, with the one-symbol table and the PSS table
// in LDS; a lane then walks its CH chunks with their lookups interleaved (CH
// dependent chains of LDS reads in flight).  The first lane of a tile,
// non-converged chunks and their successors are left to the fix-up kernel.
// MODE: what is reported (MODE_TOTAL, MODE_HIST, MODE_POS).
template <int ENC, int SHIFT, int STEP, int MODE, int CH>
__global__ __launch_bounds__((TailShape<STEP, CH>::kBlock))
__attribute__((amdgpu_waves_per_eu(TailShape<STEP, CH>::kMinWaves, 8))) void k_tail(ScanArgs a) {
  static_assert(CH == 1 || CH == 2, "one or two chains per lane");
  extern __shared__ __align__(16) char lds[];
  if (STEP == 2) copy_to_lds(lds, a.T2, a.n_states * 64u);
  if (STEP == 3) copy_to_lds(lds, a.T3, (a.n_states + 1) * 128u);
  copy_to_lds(lds + a.lds_t1_off, a.T1, a.n_states * 16u);
  uint32_t* wl = reinterpret_cast<uint32_t*>(lds + a.lds_w_off);
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds + a.lds_hist_off);
  for (uint32_t i = threadIdx.x; i < a.n_acc; i += blockDim.x) {
    wl[i] = a.wtab[i];
    if (MODE == MODE_HIST) hist[i] = 0;
  }
  const uint32_t* pss_off = a.pss_off;
  const uint16_t* pss_states = a.pss_states;
  if (a.spec_pss_off) {
    uint32_t* po = reinterpret_cast<uint32_t*>(lds + a.spec_pss_off);
    uint16_t* ps = reinterpret_cast<uint16_t*>(lds + a.spec_pss_states);
    for (uint32_t i = threadIdx.x; i < a.pss_n_off; i += blockDim.x) po[i] = a.pss_off[i];
    for (uint32_t i = threadIdx.x; i < a.pss_n_states; i += blockDim.x) ps[i] = a.pss_states[i];
    pss_off = po;
    pss_states = ps;
  }
  __syncthreads();
  const Tab tb{lds, lds + a.lds_t1_off, a.q0s};
  if (threadIdx.x == 0 && (uint32_t)(uintptr_t)(lds_c*)lds != 0u) flag_error(a, 64u);
  using Sink = SinkTail<MODE>;
  const Sink sink0{a.lds_t1_off, a.q0s, a.lds_w_off, a.lds_hist_off,
                   AppendTo{a.acc_out_off, a.acc_out_ids, a.app_count, a.app_keys, a.app_cap}};
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;  // global wave
  uint64_t c[CH], lo[CH], hi[CH];
  bool valid[CH], conv[CH];
  uint32_t my_t[CH], my_s[CH], out_e[CH], out_cnt[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const uint64_t tile = gw * CH + j;
    c[j] = tile * TILE + lane;
    my_t[j] = NONCONV;
    my_s[j] = 0;
    if (tile < a.n_tiles) spec_tile<ENC, SHIFT>(a, Tab{nullptr, tb.t1, a.q0s}, pss_off, pss_states, tile, my_t[j], my_s[j]);
    valid[j] = c[j] < a.n_chunks;
    if (!valid[j]) my_t[j] = NONCONV;
    conv[j] = my_t[j] != NONCONV;
    lo[j] = chunk_lo(a, c[j]);
    hi[j] = valid[j] ? (lo[j] + a.chunk < a.n ? lo[j] + a.chunk : a.n) : 0;
    out_e[j] = 0;
    out_cnt[j] = 0;
  }
  // the scan from the converging points
  {
    Sink sk[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) sk[j] = sink0;
    if constexpr (CH == 2) {
      if (conv[0] && conv[1]) {
        out_e[0] = my_s[0];
        out_e[1] = my_s[1];
        scan_range2<ENC, SHIFT, STEP>(a, tb, out_e[0], lo[0] + my_t[0], hi[0], sk[0], out_e[1], lo[1] + my_t[1],
                                      hi[1], sk[1]);
      } else {
        if (conv[0]) out_e[0] = scan_range<ENC, SHIFT, STEP>(a, tb, my_s[0], lo[0] + my_t[0], hi[0], sk[0]);
        if (conv[1]) out_e[1] = scan_range<ENC, SHIFT, STEP>(a, tb, my_s[1], lo[1] + my_t[1], hi[1], sk[1]);
      }
    } else {
      if (conv[0]) out_e[0] = scan_range<ENC, SHIFT, STEP>(a, tb, my_s[0], lo[0] + my_t[0], hi[0], sk[0]);
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) out_cnt[j] = sk[j].cnt;
  }
  uint64_t fixed_total = 0;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    // the join inside the wave
    const uint32_t pe = __shfl_up(out_e[j], 1u);
    const int pconv = __shfl_up((int)conv[j], 1u);
    bool fixed = false;
    if (conv[j] && lane > 0 && pconv) {
      Sink sink = sink0;
      uint64_t sy0, sy1, rs;
      if ((lo[j] & 63) == 0 && lo[j] + SPEC_WIN <= a.n) front_symbols<ENC>(a, lo[j], sy0, sy1, rs);
      else stage_symbols<ENC>(a, lo[j], hi[j], sy0, sy1, rs);
      const uint32_t e = run_staged<SHIFT>(tb, pe, sy0, sy1, rs, my_t[j], lo[j], sink);
      if (e != my_s[j]) flag_error(a, 32u);
      out_cnt[j] += sink.cnt;
      fixed = true;
      fixed_total += out_cnt[j];
    }
    // the first chunk of every tile goes to the fix-up kernel without a list
    // entry (its symbols before the converging point are kept for it); the
    // others only when their join could not be done here
    const bool to_fix = valid[j] && !fixed && lane > 0;
    const uint32_t fix_at = wave_append(a.fix_count, to_fix);
    if (valid[j]) {
      if (to_fix) a.fix_list[fix_at] = (uint32_t)c[j];
      else if (fixed && a.chunk_cnt) a.chunk_cnt[c[j]] = out_cnt[j];
      if (lane == 0 && conv[j]) {
        uint64_t sy0, sy1, rs;
        if ((lo[j] & 63) == 0 && lo[j] + SPEC_WIN <= a.n) front_symbols<ENC>(a, lo[j], sy0, sy1, rs);
        else stage_symbols<ENC>(a, lo[j], hi[j], sy0, sy1, rs);
        uint64_t* f = a.front + 3 * (c[j] / TILE);
        f[0] = sy0;
        f[1] = sy1;
        f[2] = rs;
      }
      if (fixed) a.conv_t[c[j]] = my_t[j] | FIXED;
      a.end_s[c[j]] = out_e[j];
      a.tail_cnt[c[j]] = out_cnt[j];
    }
  }
  if constexpr (MODE == MODE_HIST) {
    // per-pattern counts: each final state's visits, added to the patterns it ends
    __syncthreads();
    if (a.pat_counts)
      for (uint32_t i = threadIdx.x; i < a.n_acc; i += blockDim.x)
        if (hist[i])
          for (uint32_t j = a.acc_out_off[i]; j < a.acc_out_off[i + 1]; ++j)
            atomicAdd(a.pat_counts + a.acc_out_ids[j], (unsigned long long)hist[i]);
  } else if constexpr (MODE == MODE_TOTAL) {
    // one atomic per block for the joined chunks' total
    for (int o = 32; o > 0; o >>= 1) fixed_total += __shfl_down(fixed_total, o);
    uint64_t* red = reinterpret_cast<uint64_t*>(lds + a.lds_red_off);
    if (lane == 0) red[threadIdx.x >> 6] = fixed_total;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t t = 0;
      for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) t += red[w];
      if (t) atomicAdd(a.total, (unsigned long long)t);
    }
  }
}

// Which k_tail instantiation a scan uses.
struct TailKey {
  int enc;     // ENC_BYTE or ENC_2BIT
  int shift;   // state register scale: 6 (tables of up to 1024 states) or 4
  int step;    // symbols per lookup in the main walk: 1, 2 or 3
  int chains;  // chunks walked per lane with interleaved lookups: 1 or 2
  int mode;    // MODE_TOTAL, MODE_HIST or MODE_POS
};

// Threads per block of the instantiation (TailShape<step, chains>::kBlock).
int tail_block(const TailKey& k);
// Resident blocks per CU with `lds` bytes of dynamic LDS (0: no instantiation).
int tail_occupancy(const TailKey& k, uint32_t lds);
// Launches k_tail on `st`; false if the key has no instantiation.
bool tail_launch(const TailKey& k, uint32_t blocks, uint32_t lds, hipStream_t st, const ScanArgs& a);

// The calls above for one (encoding, mode) pair each, defined in one
// translation unit per pair (tail_<enc>_<kind>.hip).
#define COEX_TAIL_DECL(NAME)                                                                   \
  int tail_occupancy_##NAME(const TailKey& k, uint32_t lds);                                   \
  bool tail_launch_##NAME(const TailKey& k, uint32_t blocks, uint32_t lds, hipStream_t st,      \
                          const ScanArgs& a);
COEX_TAIL_DECL(byte_count)
COEX_TAIL_DECL(byte_hist)
COEX_TAIL_DECL(byte_pos)
COEX_TAIL_DECL(2bit_count)
COEX_TAIL_DECL(2bit_hist)
COEX_TAIL_DECL(2bit_pos)
#undef COEX_TAIL_DECL

// The dispatch shared by the translation units: every (shift, step, chains)
// combination that is instantiated (positions: one chain per lane).
template <int ENC, int MODE, class F>
bool tail_dispatch(const TailKey& k, F&& f) {
  if (MODE == MODE_POS && k.chains != 1) return false;
  if (k.shift == 6) {
    if (k.step == 3) {
      if constexpr (MODE != MODE_POS)
        if (k.chains == 2) return f(k_tail<ENC, 6, 3, MODE, 2>, TailShape<3, 2>::kBlock);
      return f(k_tail<ENC, 6, 3, MODE, 1>, TailShape<3, 1>::kBlock);
    }
    if (k.step == 2) {
      if constexpr (MODE != MODE_POS)
        if (k.chains == 2) return f(k_tail<ENC, 6, 2, MODE, 2>, TailShape<2, 2>::kBlock);
      return f(k_tail<ENC, 6, 2, MODE, 1>, TailShape<2, 1>::kBlock);
    }
    return k.chains == 1 && f(k_tail<ENC, 6, 1, MODE, 1>, TailShape<1, 1>::kBlock);
  }
  return k.shift == 4 && k.step == 1 && k.chains == 1 && f(k_tail<ENC, 4, 1, MODE, 1>, TailShape<1, 1>::kBlock);
}

template <int ENC, int MODE>
int tail_occupancy_enc(const TailKey& k, uint32_t lds) {
  int blocks = 0;
  const bool ok = tail_dispatch<ENC, MODE>(k, [&](auto kern, int block) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, block, lds) != hipSuccess) blocks = 1;
    return true;
  });
  return ok ? std::max(1, blocks) : 0;
}

template <int ENC, int MODE>
bool tail_launch_enc(const TailKey& k, uint32_t blocks, uint32_t lds, hipStream_t st, const ScanArgs& a) {
  return tail_dispatch<ENC, MODE>(k, [&](auto kern, int block) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(block), lds, st, a);
    return true;
  });
}

}  // namespace coex
