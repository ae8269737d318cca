"""GPU parity of the batched path (coex_dfa_set / coex_batch / coex_count_batched):
every (sequence, automaton) count equals the CPU oracle's, over uneven
sequence lengths (empty, shorter than a chunk, ragged tails), automata of
every kind (k-mer sets, regexes, tables without a synchronising depth, many
patterns per state), both encodings, explicit pair lists, graph replays and
the autotuner."""
import sys

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


class Pat:
    """One automaton, compiled for the GPU and described for the oracle."""

    def __init__(self, coex, kind, spec, n_patterns=0):
        self.kind, self.spec = kind, spec
        if kind == "kmers":
            self.dfa = coex.Dfa.kmers(spec)
        elif kind == "regex":
            self.dfa = coex.Dfa.regex(spec)
            self.rx = oracle.Regex(spec)
        else:
            dl, q0, off, ids = spec
            self.dfa = coex.Dfa.table(dl, q0, off, ids, n_patterns)
            self.table = oracle.make_table(dl, q0, off, ids, n_patterns)

    def total(self, seq: "oracle.Seq") -> int:
        if self.kind == "kmers":
            return int(oracle.count_kmers(self.spec, seq)[0].sum())
        if self.kind == "regex":
            return int(self.rx.scan(seq)[0])
        return int(oracle.scan_table(self.table, seq)[0].sum())


def _parity_table():
    # two states, no synchronising word: candidates never agree
    return (np.array([1, 0, 0, 0, 0, 1, 1, 1], np.uint32), 0, np.array([0, 0, 1], np.uint32),
            np.array([0], np.uint32))


def _many_out_table():
    # one state ends 20 patterns: two-symbol counts do not fit, one-symbol rows are used
    delta = np.array([1, 0, 0, 0, 1, 0, 0, 0], np.uint32)
    return delta, 0, np.array([0, 0, 20], np.uint32), np.arange(20, dtype=np.uint32)


def _pats(coex):
    out = [Pat(coex, "kmers", synth.random_kmers(61, 1, 8)),
           Pat(coex, "kmers", synth.random_kmers(62, 12, 6) + ["ACG", "ACGTA"]),
           Pat(coex, "kmers", synth.random_kmers(63, 30, 11)),
           Pat(coex, "regex", configs.mid_regex()),
           Pat(coex, "regex", "A[CG]{2,4}T|GG(A|T)C")]
    for seed in range(2):
        out.append(Pat(coex, "regex", synth.random_regex(640 + seed)))
    dl, q0, off, ids = synth.random_table(65, 30, 4)
    out.append(Pat(coex, "table", (dl, q0, off, ids), 4))
    return out


LENGTHS = [0, 1, 7, 100, 4095, 4096, 4097, 10_000, 50_001, 123_457, 200_000, 300_001]


def _seqs(coex, seed, lengths, enc):
    buf, offs = configs.packed_sequences(seed, lengths)
    dev, host = [], []
    for o, n in zip(offs, lengths):
        a = buf[o:o + n]
        host.append(oracle.byte_seq(a))
        if enc == coex.ENC_BYTE:
            dev.append(coex.to_device(a, encoding=coex.ENC_BYTE))
        else:
            packed, mask = synth.bytes_to_2bit(a)
            dev.append(coex.to_device(packed, n=n, encoding=coex.ENC_2BIT, nmask=mask))
    return dev, host


def _expect(pats, host):
    return np.array([[p.total(h) for p in pats] for h in host], dtype=np.uint64)


@pytest.mark.parametrize("enc", [0, 1])
def test_cross_product_chunks(coex, enc):
    pats = _pats(coex)
    dev, host = _seqs(coex, 70 + enc, LENGTHS, enc)
    exp = _expect(pats, host)
    dset = coex.DfaSet([p.dfa for p in pats])
    for chunk in [64, 100, 4096, 0]:
        say("batch cross enc", enc, "chunk", chunk)
        b = coex.Batch(dset, dev, chunk=chunk, check=True)
        got = b.run().cpu().numpy().view(np.uint64)
        assert got.tolist() == exp.tolist(), (chunk, b.info())


def test_nonconverging_and_many_outputs(coex):
    pats = _pats(coex)[:3] + [Pat(coex, "table", _parity_table(), 1), Pat(coex, "table", _many_out_table(), 20)]
    dev, host = _seqs(coex, 72, LENGTHS, coex.ENC_BYTE)
    exp = _expect(pats, host)
    dset = coex.DfaSet([p.dfa for p in pats])
    for chunk in [64, 1000, 0]:
        say("batch nonconv chunk", chunk)
        b = coex.Batch(dset, dev, chunk=chunk, check=True)
        assert b.info().step == 3   # the 20-output table takes one-symbol rows, the rest two
        assert b.run().cpu().numpy().view(np.uint64).tolist() == exp.tolist()


def test_widths_steps_and_groups(coex):
    # forced one-symbol rows, width 8 and an automaton set split over several LDS groups
    pats = _pats(coex) + [Pat(coex, "kmers", synth.random_kmers(66 + i, 60, 12)) for i in range(3)]
    dev, host = _seqs(coex, 73, LENGTHS[3:], coex.ENC_BYTE)
    exp = _expect(pats, host)
    for width, step in [(8, 0), (64, 1), (0, 2), (16, 0)]:
        # width 8 takes the automata whose candidate lists fit 8 at some lookback
        use = [i for i, p in enumerate(pats) if min(p.dfa.info().max_pss[1:]) <= (width or 64)]
        assert len(use) >= 5
        dset = coex.DfaSet([pats[i].dfa for i in use], width=width, step=step)
        b = coex.Batch(dset, dev, chunk=5000, check=True)
        inf = b.info()
        say("batch width", width, "step", step, inf)
        if step == 2:
            assert inf.n_groups >= 2 and inf.step == 2
        if step == 1:
            assert inf.step == 1
        assert b.run().cpu().numpy().view(np.uint64).tolist() == exp[:, use].tolist()
    wide = [p.dfa for p in pats if min(p.dfa.info().max_pss[1:]) > 8]
    assert wide
    with pytest.raises(coex.CoexError):
        coex.DfaSet(wide, width=8)


def test_pair_lists(coex):
    pats = _pats(coex)
    dev, host = _seqs(coex, 74, LENGTHS, coex.ENC_BYTE)
    st = synth.Stream(75, 1)
    pairs = [(st.below(len(dev)), st.below(len(pats))) for _ in range(40)] + [(11, 0), (11, 0), (0, 3)]
    dset = coex.DfaSet([p.dfa for p in pats])
    b = coex.Batch(dset, dev, pairs=pairs, chunk=4096, check=True)
    got = b.run().cpu().numpy().view(np.uint64)
    assert got.tolist() == [pats[d].total(host[s]) for s, d in pairs]


def test_graph_replays(coex):
    import torch
    pats = _pats(coex)
    dev, host = _seqs(coex, 76, LENGTHS, coex.ENC_BYTE)
    exp = _expect(pats, host)
    dset = coex.DfaSet([p.dfa for p in pats])
    b = coex.Batch(dset, dev, chunk=4096, graph=True, timed=True)
    out = torch.zeros(exp.size, dtype=torch.int64, device="cuda")
    for r in range(4):
        got = b.run(out=out)
        torch.cuda.synchronize()
        say("graph replay", r, b.info().last_ms)
        assert got.cpu().numpy().view(np.uint64).tolist() == exp.tolist()
        out.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()


def test_tuner_and_convenience(coex):
    pats = _pats(coex)
    dev, host = _seqs(coex, 77, LENGTHS, coex.ENC_BYTE)
    exp = _expect(pats, host)
    dset = coex.DfaSet([p.dfa for p in pats])
    b = coex.Batch(dset, dev, check=True)
    c, w = b.tune()
    say("tuned chunk", c, "width cap", w)
    assert 4096 <= c <= (1 << 20)
    assert w in (1, 2, 4, 8, 16, 32, 64)
    assert b.info().chunk == c
    assert b.run().cpu().numpy().view(np.uint64).tolist() == exp.tolist()
    # every width cap the set allows gives the same counts
    for cap in (1, 2, 4, 8, 16, 32, 64):
        try:
            bw = coex.Batch(dset, dev, check=True, width=cap, chunk=4096)
        except coex.CoexError as e:  # some automaton needs more candidates than the cap
            assert e.name == "EUNSUPPORTED", e
            continue
        say("width cap", cap, bw.info())
        assert bw.info().width <= cap
        assert bw.run().cpu().numpy().view(np.uint64).tolist() == exp.tolist()
        bw.free()
    got = coex.count_batched([p.dfa for p in pats], dev).cpu().numpy().view(np.uint64)
    assert got.tolist() == exp.tolist()


def _all_pair_totals(pats, buf, offs, lengths, threads=None):
    """Oracle totals of every (sequence, automaton) pair, pairs spread over the
    host cores (each pair one sequential oracle scan)."""
    jobs = [(s, d) for s in range(len(lengths)) for d in range(len(pats))]
    jobs.sort(key=lambda sd: -lengths[sd[0]])  # longest first: balanced pool

    def one(sd):
        s, d = sd
        return pats[d].total(oracle.byte_seq(buf[offs[s]:offs[s] + lengths[s]]))

    vals = oracle.pool_map(one, jobs, threads)
    exp = np.zeros((len(lengths), len(pats)), dtype=np.uint64)
    for (s, d), v in zip(jobs, vals):
        exp[s, d] = v
    return exp


@pytest.mark.timeout(1200)
def test_batched_config_all_pairs(coex):
    # the batched workload (512 sequences, about 4e9 bases, 16 automata of
    # 10-500 states) in the bench's launch configuration (tuned chunk, graph
    # replay); the oracle checks all 8,192 pairs
    import time
    import torch
    lengths, buf, offs, (sets, rxs) = configs.batched()
    say("batched: total bases", sum(lengths))
    pats = [Pat(coex, "kmers", k) for k in sets] + [Pat(coex, "regex", r) for r in rxs]
    states = [p.dfa.info().n_states for p in pats]
    say("batched: automaton states", states)
    assert all(10 <= n <= 500 for n in states)
    dbuf = torch.from_numpy(buf).to("cuda")
    seqs = [coex.DeviceSeq(dbuf[o:o + max(n, 1)], n, coex.ENC_BYTE) for o, n in zip(offs, lengths)]
    dset = coex.DfaSet([p.dfa for p in pats])
    tb = coex.Batch(dset, seqs)
    chunk, width = tb.tune()
    tb.free()
    b = coex.Batch(dset, seqs, chunk=chunk, width=width, graph=True, check=False)
    got = b.run().cpu().numpy().view(np.uint64).reshape(len(lengths), len(pats))
    got2 = b.run().cpu().numpy().view(np.uint64).reshape(len(lengths), len(pats))
    say("batched: gpu done", b.info())
    del dbuf, seqs, b
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    exp = _all_pair_totals(pats, buf, offs, lengths, threads=min(16, oracle.host_threads()))
    say("batched: oracle over %d pairs in %.1f s" % (exp.size, time.perf_counter() - t0))
    bad = np.argwhere(got != exp)
    assert bad.size == 0, [(int(s), int(d), int(got[s, d]), int(exp[s, d])) for s, d in bad[:10]]
    assert (got2 == got).all()
