/*
 * Seeded synthetic DNA inputs (shared by the oracle side and the GPU side).
 *
 * This file holds input generation only: random numbers, the Markov source,
 * runs of 'N', and the two storage formats (one ASCII byte per base; 2-bit
 * codes packed four to a byte plus a 1-bit N mask).  It contains no pattern
 * matching, no automaton and nothing the scan computes.
 *
 * Random numbers: SplitMix64 used as a counter-based generator.  Output number
 * i of stream (seed, tag) is mix64(key + (i + 1) * GAMMA) with
 * key = mix64(seed * GAMMA ^ tag), mix64 being SplitMix64's finaliser.  Every
 * base's draws depend only on its index, so blocks are generated in parallel.
 *
 * Markov source: transition matrix P = 0.9 * 1 pi^T + 0.1 * I over {A,C,G,T},
 * pi = (0.295, 0.205, 0.205, 0.295).  With probability 0.1 a base repeats its
 * predecessor, otherwise it is a fresh draw from pi; pi is stationary, so the
 * GC fraction is 0.41.
 *
 * N runs: alternating gaps and runs with geometric lengths (means 99,000 and
 * 1,000), so about 1% of bases are 'N'.
 *
 * 2-bit layout: A=0 C=1 G=2 T=3; base i sits in bits 2*(i%4)..2*(i%4)+1 of
 * byte i/4; the mask has bit i%8 of byte i/8 set where base i is 'N'.  Under a
 * set mask bit the 2-bit code is the Markov base it replaced (readers must
 * ignore it).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t tag) { return mix64(seed * GAMMA ^ tag); }
static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }

uint64_t synth_draw(uint64_t seed, uint64_t tag, uint64_t i) { return draw(stream_key(seed, tag), i); }

static const char ACGT[4] = {'A', 'C', 'G', 'T'};

/* pi thresholds on a 32-bit uniform: A < .295, C < .5, G < .705, else T */
static inline int pi_draw(uint32_t u) {
  const uint64_t two32 = 4294967296ULL;
  if (u < (uint32_t)(0.295 * two32)) return 0;
  if (u < (uint32_t)(0.500 * two32)) return 1;
  if (u < (uint32_t)(0.705 * two32)) return 2;
  return 3;
}

static inline int stays(uint64_t r) { return (uint32_t)(r >> 32) < (uint32_t)(0.1 * 4294967296.0); }

/* Markov base at index i (i >= 0): walk back to the latest fresh draw. */
static inline int markov_at(uint64_t key, uint64_t i) {
  for (;;) {
    uint64_t r = draw(key, i);
    if (i == 0 || !stays(r)) return pi_draw((uint32_t)r);
    --i;
  }
}

/* iid uniform bytes over ACGT */
void synth_iid_bytes(uint64_t seed, uint64_t n, uint8_t* out) {
  uint64_t key = stream_key(seed, 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) out[i] = (uint8_t)ACGT[draw(key, (uint64_t)i) >> 62];
}

/* Markov codes 0..3 for [0, n) */
static void markov_codes_range(uint64_t key, uint64_t lo, uint64_t hi, uint8_t* out /* indexed from lo */) {
  if (lo >= hi) return;
  int prev = markov_at(key, lo);
  out[0] = (uint8_t)prev;
  for (uint64_t i = lo + 1; i < hi; ++i) {
    uint64_t r = draw(key, i);
    int b = stays(r) ? prev : pi_draw((uint32_t)r);
    out[i - lo] = (uint8_t)b;
    prev = b;
  }
}

/* N runs: fills `runs` with [start, end) pairs, returns the count (<= cap). */
uint64_t synth_n_runs(uint64_t seed, uint64_t n, double mean_gap, double mean_run, uint64_t* runs, uint64_t cap) {
  uint64_t key = stream_key(seed, 3);
  uint64_t k = 0, pos = 0, cnt = 0;
  if (mean_run <= 0.0) return 0;
  double pg = 1.0 / mean_gap, pr = 1.0 / mean_run;
  for (;;) {
    /* geometric on {1,2,...} with the given mean, by inversion of a 53-bit uniform */
    double u1 = ((draw(key, k++) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double u2 = ((draw(key, k++) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    uint64_t gap = 1 + (uint64_t)floor(log(u1) / log1p(-pg));
    uint64_t len = 1 + (uint64_t)floor(log(u2) / log1p(-pr));
    pos += gap;
    if (pos >= n) break;
    uint64_t end = pos + len > n ? n : pos + len;
    if (cnt < cap) { runs[2 * cnt] = pos; runs[2 * cnt + 1] = end; }
    ++cnt;
    pos = end;
  }
  return cnt;
}

#define BLOCK ((uint64_t)1 << 20)

/* Markov bytes (ACGT) with optional N runs written as 'N' */
void synth_markov_bytes(uint64_t seed, uint64_t n, int with_n, uint8_t* out) {
  uint64_t key = stream_key(seed, 2);
  int64_t nblk = (int64_t)((n + BLOCK - 1) / BLOCK);
#pragma omp parallel
  {
    uint8_t* tmp = (uint8_t*)malloc(BLOCK);
#pragma omp for schedule(static)
    for (int64_t b = 0; b < nblk; ++b) {
      uint64_t lo = (uint64_t)b * BLOCK, hi = lo + BLOCK > n ? n : lo + BLOCK;
      markov_codes_range(key, lo, hi, tmp);
      for (uint64_t i = lo; i < hi; ++i) out[i] = (uint8_t)ACGT[tmp[i - lo]];
    }
    free(tmp);
  }
  if (with_n) {
    uint64_t cap = n / 1000 + 1024;
    uint64_t* runs = (uint64_t*)malloc(cap * 2 * sizeof(uint64_t));
    uint64_t cnt = synth_n_runs(seed, n, 99000.0, 1000.0, runs, cap);
    if (cnt > cap) cnt = cap;
    for (uint64_t r = 0; r < cnt; ++r) memset(out + runs[2 * r], 'N', runs[2 * r + 1] - runs[2 * r]);
    free(runs);
  }
}

/* Markov 2-bit packed + N mask.  packed: ceil(n/4) bytes, mask: ceil(n/8) bytes. */
void synth_markov_2bit(uint64_t seed, uint64_t n, int with_n, uint8_t* packed, uint8_t* mask) {
  uint64_t key = stream_key(seed, 2);
  int64_t nblk = (int64_t)((n + BLOCK - 1) / BLOCK); /* BLOCK is a multiple of 8 */
#pragma omp parallel
  {
    uint8_t* tmp = (uint8_t*)malloc(BLOCK);
#pragma omp for schedule(static)
    for (int64_t b = 0; b < nblk; ++b) {
      uint64_t lo = (uint64_t)b * BLOCK, hi = lo + BLOCK > n ? n : lo + BLOCK;
      markov_codes_range(key, lo, hi, tmp);
      for (uint64_t i = lo; i < hi; i += 4) {
        uint8_t v = 0;
        for (uint64_t j = 0; j < 4 && i + j < hi; ++j) v |= (uint8_t)(tmp[i + j - lo] << (2 * j));
        packed[i >> 2] = v;
      }
      memset(mask + (lo >> 3), 0, ((hi - lo) + 7) >> 3);
    }
    free(tmp);
  }
  if (with_n) {
    uint64_t cap = n / 1000 + 1024;
    uint64_t* runs = (uint64_t*)malloc(cap * 2 * sizeof(uint64_t));
    uint64_t cnt = synth_n_runs(seed, n, 99000.0, 1000.0, runs, cap);
    if (cnt > cap) cnt = cap;
    for (uint64_t r = 0; r < cnt; ++r)
      for (uint64_t i = runs[2 * r]; i < runs[2 * r + 1]; ++i) mask[i >> 3] |= (uint8_t)(1u << (i & 7));
    free(runs);
  }
}

/* Convert ASCII bases to the 2-bit + mask form (non-ACGT bytes become N).
   Used to store one sequence both ways. */
void synth_bytes_to_2bit(const uint8_t* in, uint64_t n, uint8_t* packed, uint8_t* mask) {
  int64_t nb = (int64_t)((n + 7) >> 3);
#pragma omp parallel for schedule(static)
  for (int64_t B = 0; B < nb; ++B) {
    uint8_t m = 0;
    uint8_t p[2] = {0, 0};
    for (int j = 0; j < 8; ++j) {
      uint64_t i = (uint64_t)B * 8 + (uint64_t)j;
      if (i >= n) break;
      int c;
      switch (in[i]) {
        case 'A': case 'a': c = 0; break;
        case 'C': case 'c': c = 1; break;
        case 'G': case 'g': c = 2; break;
        case 'T': case 't': c = 3; break;
        default: c = -1;
      }
      if (c < 0) { m |= (uint8_t)(1u << j); c = 0; }
      p[j >> 2] |= (uint8_t)(c << (2 * (j & 3)));
    }
    mask[B] = m;
    uint64_t i0 = (uint64_t)B * 8;
    packed[i0 >> 2] = p[0];
    if (i0 + 4 < n) packed[(i0 >> 2) + 1] = p[1];
  }
}
