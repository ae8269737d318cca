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
          uniform over 32 resident automata (seeds 5 and 505).
"""
from __future__ import annotations

from . import iid_bytes, markov_2bit, markov_bytes, random_kmers, random_regex

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
