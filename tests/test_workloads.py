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
