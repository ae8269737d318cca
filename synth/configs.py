"""The five synthetic workloads (sizes, seeds, pattern recipes).

Each function returns host data only; nothing here matches patterns.

  small   1 MiB iid uniform ACGT bytes (seed 1); one random 8-mer (seed 101);
          chunk 64 KiB; counts and sorted end positions.
  mid     256 MiB Markov bytes (GC 0.41) with N runs, 1% N (seed 2); a random
          regex over ACGT with classes and bounded repeats.  The regex is the
          generator's draw for seed 212: the first seed at or after 202 whose
          minimal search automaton has 48-80 states (it has 60).
  genome  3.2e9 bases from the same Markov source (seed 3), 2-bit packed with
          an N mask; 64 distinct random 12-mers (seed 303).
  batched 512 log-normal lengths (sigma 1.5, clipped mean about 7.8e6, clipped
          to [1e4, 5e7], seed 4) of Markov bytes; 16 automata with log-uniform
          target sizes in [10, 500] states: 8 random k-mer sets, 8 random
          regexes (seed 404).
  serving Poisson arrivals; sizes log-uniform over [1e3, 1e8]; automaton ids
          uniform over 32 resident automata of 10-1000 states: 16 k-mer sets
          and 16 regexes (seeds 5 and 505).

Automaton sizes.  Each automaton of the batched and serving sets has a target
size, log-uniform over the stated range.  A k-mer set holds target / k random
k-mers; a regex slot takes the generator's draws seed*100 + 50 + i + 1000*j
for j = 0, 1, ... and keeps the first whose minimal search automaton has
between max(lo, target / 1.6) and min(hi, 1.6 * target) states.  Sizes are a
property of the compiled automaton, which this package does not build, so the
accepted draw index j of every slot is recorded below (REGEX_DRAWS) and the
size of every automaton is asserted by the workload tests; every k-mer set
takes its first draw, which already lands inside the range.
"""
from __future__ import annotations

import numpy as np

from . import (Stream, iid_bytes, lognormal_lengths, loguniform_ints, markov_2bit, markov_bytes, poisson_arrivals,
               random_kmers, random_regex, uniform_ids)

SMALL_N = 1 << 20
SMALL_CHUNK = 1 << 16
MID_N = 256 << 20
GENOME_N = 3_200_000_000
MID_REGEX_SEED = 212


def small(n: int = SMALL_N):
    return iid_bytes(1, n), random_kmers(101, 1, 8)


def mid_regex() -> str:
    return random_regex(MID_REGEX_SEED)


def mid(n: int = MID_N):
    return markov_bytes(2, n, with_n=True), mid_regex()


def genome_kmers():
    return random_kmers(303, 64, 12)


def genome(n: int = GENOME_N):
    packed, mask = markov_2bit(3, n, with_n=True)
    return packed, mask, genome_kmers()


# ---------------------------------------------------------------- batched
BATCH_SEQS = 512
BATCH_SEED = 4
BATCH_PATTERN_SEED = 404


def size_targets(seed: int, n_kmer_sets: int, n_regexes: int, lo: float, hi: float):
    """Target automaton sizes, log-uniform in [lo, hi]: k-mer sets first, then regexes."""
    return loguniform_ints(seed, 16, n_kmer_sets + n_regexes, lo, hi)


def kmer_sets(seed: int, count: int, lo: float, hi: float):
    """`count` random k-mer sets, k in 6..14, with about log-uniform target
    automaton sizes in [lo, hi] states (count of k-mers = target / k)."""
    targets = loguniform_ints(seed, 16, count, lo, hi)
    st = Stream(seed, 17)
    out = []
    for i, t in enumerate(targets):
        k = 6 + st.below(9)
        out.append(random_kmers(seed * 100 + i, max(1, round((t - 1) / k)), k))
    return out


def regex_candidate(seed: int, i: int, j: int) -> str:
    """Draw j for regex slot i of a pattern set."""
    return random_regex(seed * 100 + 50 + i + 1000 * j)


def regex_window(target: int, lo: float, hi: float):
    """States a regex drawn for `target` must have: within a factor 1.6 of it, inside [lo, hi]."""
    return max(lo, target / 1.6), min(hi, target * 1.6)


# accepted draw index j per regex slot (see the module docstring)
REGEX_DRAWS = {
    404: (9, 1, 22, 14, 0, 37, 0, 23),
    505: (0, 0, 10, 0, 0, 4, 0, 3, 67, 0, 0, 1, 36, 0, 9, 0),
}


def regexes(seed: int, count: int):
    draws = REGEX_DRAWS[seed]
    return [regex_candidate(seed, i, draws[i]) for i in range(count)]


def batched_patterns():
    """8 k-mer sets and 8 regexes, target sizes log-uniform in [10, 500] states."""
    return kmer_sets(BATCH_PATTERN_SEED, 8, 10, 500), regexes(BATCH_PATTERN_SEED, 8)


def packed_sequences(seed: int, lengths):
    """One Markov byte buffer (N runs included) holding the sequences back to
    back, each starting at a multiple of 128 bytes: (buffer, offsets)."""
    offs, total = [], 0
    for n in lengths:
        offs.append(total)
        total += max(128, (int(n) + 127) // 128 * 128)
    return markov_bytes(seed, total, with_n=True), offs


def batched(count: int = BATCH_SEQS, scale: float = 1.0):
    """Lengths (log-normal, sigma 1.5, clipped mean about 7.8e6, clipped to
    [1e4, 5e7]), the packed byte buffer and offsets, and the patterns."""
    lengths = lognormal_lengths(BATCH_SEED, count)
    if scale != 1.0:
        lengths = [max(1, int(n * scale)) for n in lengths]
    buf, offs = packed_sequences(BATCH_SEED, lengths)
    return lengths, buf, offs, batched_patterns()


# ---------------------------------------------------------------- serving
SERVE_SEED = 5
SERVE_PATTERN_SEED = 505
SERVE_POOL = 100_000_000


def serving_patterns():
    """32 resident automata: 16 k-mer sets and 16 regexes, target sizes log-uniform in [10, 1000] states."""
    return kmer_sets(SERVE_PATTERN_SEED, 16, 10, 1000), regexes(SERVE_PATTERN_SEED, 16)


def serving_requests(count: int, qps: float, max_size: float = 1e8):
    """Arrival times (s), sizes (log-uniform over [1e3, max_size]), automaton
    ids (uniform over 32) and start offsets into the request pool."""
    arrivals = poisson_arrivals(SERVE_SEED, count, qps)
    sizes = loguniform_ints(SERVE_SEED, 18, count, 1e3, max_size)
    ids = uniform_ids(SERVE_SEED, 19, count, 32)
    st = Stream(SERVE_SEED, 20)
    offs = [st.below(max(1, SERVE_POOL - n + 1)) // 16 * 16 for n in sizes]
    return arrivals, sizes, ids, offs


def serving_pool():
    """The bytes requests are cut from (Markov with N runs, seed 5)."""
    return markov_bytes(SERVE_SEED, SERVE_POOL + 128, with_n=True)
