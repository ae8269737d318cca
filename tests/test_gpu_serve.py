"""GPU tests of the serving loop (coex_server): every request's count equals
the CPU oracle's, the same when the request runs alone and when it is mixed
with others in continuous batches; admission respects the HBM budget; a
request that can never fit is refused."""
import sys
import threading

import numpy as np
import pytest

import oracle
import synth
from synth import configs

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


def _patterns():
    sets = [synth.random_kmers(81, 1, 8), synth.random_kmers(82, 20, 10), synth.random_kmers(83, 5, 6)]
    rxs = [configs.mid_regex(), "A[CG]{2,4}T|GG(A|T)C", synth.random_regex(84)]
    return sets, rxs


def _oracle(sets, rxs, idx, seq):
    h = oracle.byte_seq(seq)
    if idx < len(sets):
        return int(oracle.count_kmers(sets[idx], h)[0].sum())
    return int(oracle.Regex(rxs[idx - len(sets)]).scan(h)[0])


def _requests(n, seed, max_size):
    pool = synth.markov_bytes(seed, 2_000_000 + 128, with_n=True)
    sizes = synth.loguniform_ints(seed, 1, n, 1, max_size)
    st = synth.Stream(seed, 2)
    reqs = []
    for i, sz in enumerate(sizes):
        if i % 9 == 0:
            sz = 0 if i % 18 == 0 else 1       # empty and one-base requests
        off = st.below(pool.size - sz - 1)
        reqs.append((pool[off:off + sz].copy(), st.below(6)))
    return reqs


def test_alone_and_in_mix(coex):
    import torch
    sets, rxs = _patterns()
    dfas = [coex.Dfa.kmers(k) for k in sets] + [coex.Dfa.regex(r) for r in rxs]
    reqs = _requests(60, 85, 400_000)
    expect = [_oracle(sets, rxs, d, seq) for seq, d in reqs]
    # 64 KiB copy pieces: the larger requests are copied in several pieces,
    # interleaved with the pieces of smaller ones
    srv = coex.Server(dfas, hbm_budget=64 << 20, copy_piece=1 << 16)
    # in the mix: everything submitted at once from pinned buffers
    bufs = [torch.from_numpy(seq).pin_memory() if seq.size else torch.empty(0, dtype=torch.uint8)
            for seq, _ in reqs]
    tickets = [srv.submit(b, d) for b, (_, d) in zip(bufs, reqs)]
    mixed = [srv.wait(t) for t in tickets]
    st = srv.stats()
    say("mix stats", st, "largest batch", max(m[1]["batch_size"] for m in mixed))
    assert [m[0] for m in mixed] == expect
    assert st["n_done"] == len(reqs) and st["n_batches"] < len(reqs)
    assert max(m[1]["batch_size"] for m in mixed) > 1
    # alone: one request in flight at a time (numpy, pageable memory)
    alone = []
    for seq, d in reqs:
        c, s = srv.wait(srv.submit(seq, d))
        assert s["batch_size"] == 1
        alone.append(c)
    assert alone == expect
    srv.close()


def test_budget_and_refusal(coex):
    sets, rxs = _patterns()
    dfas = [coex.Dfa.kmers(k) for k in sets] + [coex.Dfa.regex(r) for r in rxs]
    budget = 1 << 20
    srv = coex.Server(dfas, hbm_budget=budget, max_batch=4)
    reqs = [(synth.markov_bytes(86 + i, 300_000 + 1000 * i, with_n=True), i % 6) for i in range(12)]
    expect = [_oracle(sets, rxs, d, seq) for seq, d in reqs]
    out = {}

    def submitter():  # all at once from another thread: admission waits for arena space
        for i, (seq, d) in enumerate(reqs):
            out[i] = srv.submit(seq, d)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    got = [srv.wait(out[i]) for i in range(len(reqs))]
    assert [g[0] for g in got] == expect
    st = srv.stats()
    say("budget stats", st)
    assert st["max_arena_bytes"] <= budget
    assert max(g[1]["batch_size"] for g in got) <= 4
    big = np.zeros(budget + 1, dtype=np.uint8) + ord("A")
    t = srv.submit(big, 0)
    with pytest.raises(coex.CoexError):
        srv.wait(t)
    # the server keeps working after a refusal
    assert srv.wait(srv.submit(reqs[0][0], reqs[0][1]))[0] == expect[0]
    srv.close()


def test_odd_copy_pieces(coex):
    # copy pieces of 1000 bytes (not a multiple of any alignment) and an arena
    # smaller than the sum of the requests: pieces of several requests
    # interleave, the shortest remaining first, and every count stays exact
    import torch
    sets, rxs = _patterns()
    dfas = [coex.Dfa.kmers(k) for k in sets] + [coex.Dfa.regex(r) for r in rxs]
    reqs = _requests(40, 87, 60_000)
    expect = [_oracle(sets, rxs, d, seq) for seq, d in reqs]
    srv = coex.Server(dfas, hbm_budget=512 << 10, copy_piece=1000)
    bufs = [torch.from_numpy(seq).pin_memory() if seq.size else torch.empty(0, dtype=torch.uint8)
            for seq, _ in reqs]
    tickets = [srv.submit(b, d) for b, (_, d) in zip(bufs, reqs)]
    got = [srv.wait(t) for t in tickets]
    say("odd pieces stats", srv.stats())
    assert [g[0] for g in got] == expect
    assert srv.stats()["max_arena_bytes"] <= 512 << 10
    srv.close()
