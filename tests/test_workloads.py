"""CPU tests of the workload generators and the bench contract: the batched
and serving workloads have the sizes and distributions they are stated to
have, are reproducible, and bench.py refuses more than one GPU."""
import math
import os
import subprocess
import sys

import numpy as np

import synth
from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_batched_lengths_and_patterns():
    lengths = synth.lognormal_lengths(configs.BATCH_SEED, configs.BATCH_SEQS)
    assert len(lengths) == 512
    assert min(lengths) >= 10_000 and max(lengths) <= 50_000_000
    # the clipped mean is solved to about 7.8e6 (the sample of 512 varies)
    assert 5e6 < np.mean(lengths) < 1.1e7
    assert lengths == synth.lognormal_lengths(configs.BATCH_SEED, configs.BATCH_SEQS)
    sets, rxs = configs.batched_patterns()
    assert len(sets) == 8 and len(rxs) == 8
    for s in sets:
        k = len(s[0])
        assert 6 <= k <= 14 and all(len(w) == k and set(w) <= set("ACGT") for w in s)
        assert len(set(s)) == len(s)
    assert (sets, rxs) == configs.batched_patterns()


def test_packed_sequences_layout():
    lengths = [0, 1, 127, 128, 1000]
    buf, offs = configs.packed_sequences(9, lengths)
    assert all(o % 128 == 0 for o in offs)
    for o, n, nxt in zip(offs, lengths, offs[1:] + [buf.size]):
        assert o + n <= nxt
    assert set(np.unique(buf)) <= set(b"ACGTN")


def test_serving_requests():
    arr, sizes, ids, offs = configs.serving_requests(2000, 1000.0)
    assert len(arr) == len(sizes) == len(ids) == len(offs) == 2000
    assert all(b > a for a, b in zip(arr, arr[1:]))
    # Poisson arrivals at 1000/s: mean gap 1 ms
    assert abs(np.mean(np.diff(arr)) - 1e-3) < 1e-4
    assert min(sizes) >= 1000 and max(sizes) <= 1e8
    # log-uniform sizes: the mean of log10 is about 5.5
    assert abs(np.mean(np.log10(sizes)) - 5.5) < 0.1
    assert set(ids) <= set(range(32)) and len(set(ids)) == 32
    assert all(o % 16 == 0 and o + n <= configs.SERVE_POOL for o, n in zip(offs, sizes))
    sets, rxs = configs.serving_patterns()
    assert len(sets) == 16 and len(rxs) == 16


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _states(dfa_maker, pattern):
    return dfa_maker(pattern).info().n_states


def _check_set(seed, n_kmer_sets, n_regexes, lo, hi, sets, rxs):
    import paper_1509_01506_amd as coex
    targets = configs.size_targets(seed, n_kmer_sets, n_regexes, lo, hi)
    assert len(sets) == n_kmer_sets and len(rxs) == n_regexes
    for s in sets:
        n = _states(coex.Dfa.kmers, s)
        assert lo <= n <= hi, (s[:2], n)
    draws = configs.REGEX_DRAWS[seed]
    for i, r in enumerate(rxs):
        wlo, whi = configs.regex_window(targets[n_kmer_sets + i], lo, hi)
        n = _states(coex.Dfa.regex, r)
        assert wlo <= n <= whi and lo <= n <= hi, (i, r, n, targets[n_kmer_sets + i])
        # the recorded draw is the first one inside the window
        assert r == configs.regex_candidate(seed, i, draws[i])
        for j in range(draws[i]):
            try:
                m = _states(coex.Dfa.regex, configs.regex_candidate(seed, i, j))
            except Exception:
                continue  # a draw the compiler rejects (empty match) is skipped
            assert not (wlo <= m <= whi), (i, j, m)


def test_batched_automata_sizes_in_range():
    # 16 automata of 10-500 states (8 k-mer sets, 8 regexes)
    sets, rxs = configs.batched_patterns()
    _check_set(configs.BATCH_PATTERN_SEED, 8, 8, 10, 500, sets, rxs)


def test_serving_automata_sizes_in_range():
    # 32 resident automata of 10-1000 states (16 k-mer sets, 16 regexes)
    sets, rxs = configs.serving_patterns()
    _check_set(configs.SERVE_PATTERN_SEED, 16, 16, 10, 1000, sets, rxs)
