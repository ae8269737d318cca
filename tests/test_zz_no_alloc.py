"""coex_count_noalloc (the entry point that allocates nothing; its scratch is
a static device array per GPU) against coex_count, through the C ABI: equal
per-pattern counts on two calls in a row, the second with a smaller input
(the static array keeps the first call's contents), plus the refusals."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def coex():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1509_01506_amd as m
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_equals_count_on_two_calls(coex):
    import torch
    kmers = synth.random_kmers(303, 64, 12)
    d = coex.Dfa.kmers(kmers)
    # first call: 2-bit codes + N mask over several million bases (many tiles,
    # a ragged last chunk)
    n1 = 48_000_000 + 777
    seq1 = synth.markov_bytes(31, n1, with_n=True)
    packed, mask = synth.bytes_to_2bit(seq1)
    s1 = coex.to_device(packed, n=n1, encoding=coex.ENC_2BIT, nmask=mask)
    ref1 = coex.count(d, s1, check=True).cpu().numpy().view(np.uint64).copy()
    out = torch.full((64,), -1, dtype=torch.int64, device="cuda")
    say("noalloc: first call, 2-bit, n", n1)
    got1 = coex.count_noalloc(d, s1, out, check=True).cpu().numpy().view(np.uint64).copy()
    assert got1.tolist() == ref1.tolist()
    assert int(ref1.sum()) > 0
    # second call, smaller and in bytes, with another automaton
    n2 = 3_000_001
    seq2 = synth.markov_bytes(32, n2, with_n=True)
    s2 = coex.to_device(seq2)
    d2 = coex.Dfa.kmers(synth.random_kmers(304, 16, 8))
    ref2 = coex.count(d2, s2, check=True).cpu().numpy().view(np.uint64).copy()
    out2 = torch.full((16,), -1, dtype=torch.int64, device="cuda")
    say("noalloc: second call, bytes, n", n2)
    got2 = coex.count_noalloc(d2, s2, out2, check=True).cpu().numpy().view(np.uint64).copy()
    assert got2.tolist() == ref2.tolist()
    # and the first input again, after the smaller call
    say("noalloc: third call, the first input again")
    got3 = coex.count_noalloc(d, s1, out, check=True).cpu().numpy().view(np.uint64).copy()
    assert got3.tolist() == ref1.tolist()


def test_noalloc_one_pattern_and_unsynchronised(coex):
    import torch
    # a one-pattern regex (weighted total in the output word) and an automaton
    # without a synchronising word (candidate maps and the join kernels)
    n = 2_000_003
    seq = synth.markov_bytes(41, n, with_n=True)
    s = coex.to_device(seq)
    for d in (coex.Dfa.regex("CG[CGT]{3,4}[AG]{3,6}C{5}G"),
              coex.Dfa.table(np.array([[0, 1, 0, 1], [1, 0, 1, 0]], dtype=np.uint32).ravel(), 0,
                             np.array([0, 1, 1], dtype=np.uint32), np.array([0], dtype=np.uint32), 1)):
        ref = coex.count(d, s, check=True).cpu().numpy().view(np.uint64).copy()
        out = torch.empty(1, dtype=torch.int64, device="cuda")
        got = coex.count_noalloc(d, s, out, check=True).cpu().numpy().view(np.uint64).copy()
        assert got.tolist() == ref.tolist()


def test_noalloc_refusals(coex):
    import torch
    n = 3_000_000
    seq = synth.markov_bytes(51, n, with_n=False)
    s = coex.to_device(seq)
    out = torch.empty(4, dtype=torch.int64, device="cuda")
    fresh = coex.Dfa.kmers(["ACGT", "GGA"])
    # tables not yet on this device: refused before anything runs
    with pytest.raises(coex.CoexError) as e:
        coex.count_noalloc(fresh, s, out)
    assert e.value.name == "ENOTRESIDENT"
    coex.count(fresh, s)  # uploads the tables
    got = coex.count_noalloc(fresh, s, out, check=True).cpu().numpy().tolist()
    assert got[:2] == coex.count(fresh, s, check=True).cpu().numpy().tolist()
    # a plan whose per-chunk scratch exceeds the static array (one-base
    # chunks: 3e6 chunks of about 36 scratch bytes plus candidate maps)
    with pytest.raises(coex.CoexError) as e:
        coex.count_noalloc(fresh, s, out, chunk=1)
    assert e.value.name == "ESCRATCH"
    # timing is refused (it would create events)
    with pytest.raises(coex.CoexError) as e:
        coex._check(coex._lib().coex_count_noalloc(fresh.handle, coex.ctypes.byref(s._c()), out.data_ptr(),
                                                   coex.ctypes.byref(coex._opts(timed=True)),
                                                   coex._stream(None)), "count_noalloc")
    assert e.value.name == "EUNSUPPORTED"
