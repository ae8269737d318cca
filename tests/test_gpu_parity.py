"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit-exact, on seeded inputs spanning several tiles and a ragged tail, the
edge cases of the method, and every option that must not change results."""
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


def dev_bytes(coex, arr):
    return coex.to_device(np.asarray(arr, dtype=np.uint8), encoding=coex.ENC_BYTE)


def dev_2bit(coex, seq_bytes):
    packed, mask = synth.bytes_to_2bit(seq_bytes)
    return coex.to_device(packed, n=seq_bytes.size, encoding=coex.ENC_2BIT, nmask=mask), packed, mask


def gpu_counts(coex, dfa, s, **kw):
    return coex.count(dfa, s, check=True, **kw).cpu().numpy().view(np.uint64)


def test_small_config_count_and_positions(coex):
    seq, kmers = configs.small()
    say("small: n", seq.size, "kmer", kmers)
    d = coex.Dfa.kmers(kmers)
    s = dev_bytes(coex, seq)
    c = gpu_counts(coex, d, s, chunk=configs.SMALL_CHUNK)
    ec, epos, epat = oracle.count_kmers(kmers, oracle.byte_seq(seq), positions=True)
    assert c.tolist() == ec.tolist()
    pos, pat = coex.find(d, s, chunk=configs.SMALL_CHUNK)
    assert pos.cpu().numpy().tolist() == epos.tolist()
    assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()


def _kmer_sets():
    out = []
    for seed in range(3):
        st = synth.Stream(seed, 5)
        pats = [synth.random_kmers(seed * 31 + j, 1, 2 + st.below(9))[0] for j in range(10)]
        pats += [pats[1], pats[3][-2:]]       # duplicate id, suffix pattern
        out.append(pats)
    out.append(["A", "AA", "AAA", "AAAA"])        # output sets of size up to 4
    return out


@pytest.mark.parametrize("enc", ["byte", "2bit"])
def test_invariance_over_options(coex, enc):
    n = 40_003
    seq = synth.markov_bytes(21, n, with_n=True)
    seq[5000:5003] = ord("N")
    seq[::977] = ord("n")
    if enc == "byte":
        seq[3::1013] = ord("a")
        s = dev_bytes(coex, seq)
    else:
        s, _, _ = dev_2bit(coex, seq)
    for pats in _kmer_sets():
        d = coex.Dfa.kmers(pats)
        expect = oracle.count_kmers(pats, oracle.byte_seq(seq))[0].tolist()
        for chunk in [1, 7, 16, 63, 64, 100, 512, 1000, 4096, n - 1, n, n + 5, 0]:
            for (width, lookback, step, chains) in [(0, 0, 0, 0), (1, 1, 1, 1), (2, 1, 2, 1), (8, 2, 0, 0),
                                                    (64, 1, 0, 0), (4, 8, 2, 0), (0, 0, 3, 1), (1, 2, 3, 1),
                                                    (16, 1, 3, 1), (0, 0, 3, 2), (2, 1, 2, 2), (8, 3, 3, 2)]:
                say("invariance", enc, pats[:2], chunk, width, lookback, step, chains)
                got = gpu_counts(coex, d, s, chunk=chunk, width=width, lookback=lookback, step=step, chains=chains)
                assert got.tolist() == expect, (pats, chunk, width, lookback, step, chains)


def test_positions_multi_pattern(coex):
    n = 100_000
    seq = synth.markov_bytes(22, n, with_n=True)
    pats = ["ACG", "CG", "G", "TTAGG", "AGG", "ACGT", "ACG"]
    d = coex.Dfa.kmers(pats)
    _, epos, epat = oracle.count_kmers(pats, oracle.byte_seq(seq), positions=True)
    for chunk in [0, 1000, 4097]:
        for enc in ["byte", "2bit"]:
            s = dev_bytes(coex, seq) if enc == "byte" else dev_2bit(coex, seq)[0]
            say("positions", enc, chunk)
            pos, pat = coex.find(d, s, chunk=chunk)
            assert pos.cpu().numpy().tolist() == epos.tolist()
            assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()
    # capacity too small reports the required size
    s = dev_bytes(coex, seq)
    with pytest.raises(coex.CoexError) as e:
        coex.find(d, s, capacity=3)
    assert e.value.name == "ECAPACITY"


def test_count_find(coex):
    # counts and end positions from one scan equal the oracle's, for several
    # patterns (counts from the pattern ids), one pattern (count = matches),
    # no match at all, and a capacity too small
    n = 100_000
    seq = synth.markov_bytes(23, n, with_n=True)
    cases = [["ACG", "CG", "G", "TTAGG", "AGG", "ACGT", "ACG"], ["GATTACA"], ["ACGTACGTACGTACGTACGT"],
             synth.random_kmers(24, 200, 9)]
    for pats in cases:
        d = coex.Dfa.kmers(pats)
        ec, epos, epat = oracle.count_kmers(pats, oracle.byte_seq(seq), positions=True)
        for chunk in [0, 1000]:
            for enc in ["byte", "2bit"]:
                s = dev_bytes(coex, seq) if enc == "byte" else dev_2bit(coex, seq)[0]
                say("count_find", pats[:2], len(pats), enc, chunk)
                c, pos, pat = coex.count_find(d, s, chunk=chunk)
                assert c.cpu().numpy().view(np.uint64).tolist() == ec.tolist()
                assert pos.cpu().numpy().tolist() == epos.tolist()
                assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()
    d = coex.Dfa.kmers(cases[0])
    s = dev_bytes(coex, seq)
    with pytest.raises(coex.CoexError) as e:
        coex.count_find(d, s, capacity=3)
    assert e.value.name == "ECAPACITY"
    # an empty sequence: zero counts, no positions
    c, pos, _ = coex.count_find(d, dev_bytes(coex, seq[:0]))
    assert c.cpu().numpy().tolist() == [0] * len(cases[0]) and pos.numel() == 0


def test_regex_mid_fraction(coex):
    n = configs.MID_N // 64
    seq, rx = configs.mid(n)
    say("mid/64 regex", rx, n)
    d = coex.Dfa.regex(rx)
    s = dev_bytes(coex, seq)
    m, epos = oracle.Regex(rx).scan(oracle.byte_seq(seq), positions=True)
    assert gpu_counts(coex, d, s).tolist() == [m]
    pos, _ = coex.find(d, s)
    assert pos.cpu().numpy().tolist() == epos.tolist()


def test_random_regexes(coex):
    n = 60_000
    seq = synth.markov_bytes(23, n, with_n=True)
    s = dev_bytes(coex, seq)
    s2 = dev_2bit(coex, seq)[0]
    for seed in range(12):
        rx = synth.random_regex(seed)
        try:
            d = coex.Dfa.regex(rx)
        except coex.CoexError:
            continue
        m, epos = oracle.Regex(rx).scan(oracle.byte_seq(seq), positions=True)
        for chunk in [0, 333, 2048]:
            say("regex", rx, chunk)
            assert gpu_counts(coex, d, s, chunk=chunk).tolist() == [m]
            assert gpu_counts(coex, d, s2, chunk=chunk).tolist() == [m]
            if d.info().n_states <= 1023:
                assert gpu_counts(coex, d, s, chunk=chunk, step=3).tolist() == [m]
                assert gpu_counts(coex, d, s2, chunk=chunk, step=3).tolist() == [m]
        pos, _ = coex.find(d, s, chunk=1000)
        assert pos.cpu().numpy().tolist() == epos.tolist()


def test_genome_fraction(coex):
    n = configs.GENOME_N // 64
    packed, mask, kmers = configs.genome(n)
    say("genome/64", n)
    d = coex.Dfa.kmers(kmers)
    s = coex.to_device(packed, n=n, encoding=coex.ENC_2BIT, nmask=mask)
    expect = oracle.count_kmers(kmers, oracle.twobit_seq(packed, mask, n))[0]
    assert gpu_counts(coex, d, s).tolist() == expect.tolist()
    assert gpu_counts(coex, d, s, chunk=1 << 16, lookback=1, width=64).tolist() == expect.tolist()
    assert gpu_counts(coex, d, s, step=3).tolist() == expect.tolist()
    assert gpu_counts(coex, d, s, step=3, chunk=5000).tolist() == expect.tolist()
    assert gpu_counts(coex, d, s, step=3, chains=2).tolist() == expect.tolist()
    assert gpu_counts(coex, d, s, step=2, chains=2, chunk=4099).tolist() == expect.tolist()


def _parity_table():
    return np.array([1, 0, 0, 0, 0, 1, 1, 1], np.uint32), 0, np.array([0, 0, 1], np.uint32), np.array([0], np.uint32)


def test_tables_and_nonconverging(coex):
    n = 30_011
    seq = synth.markov_bytes(24, n, with_n=True)
    s = dev_bytes(coex, seq)
    s2 = dev_2bit(coex, seq)[0]
    tables = [(_parity_table(), 1)]
    for seed in range(4):
        dl, q0, off, ids = synth.random_table(seed, 20 + 30 * seed, 5)
        tables.append(((dl, q0, off, ids), 5))
    for (dl, q0, off, ids), P in tables:
        d = coex.Dfa.table(dl, q0, off, ids, P)
        t = oracle.make_table(dl, q0, off, ids, P)
        ec, epos, epat, _ = oracle.scan_table(t, oracle.byte_seq(seq), positions=True)
        for chunk in [0, 50, 999]:
            say("table", dl.size // 4, chunk)
            assert gpu_counts(coex, d, s, chunk=chunk).tolist() == ec.tolist()
            assert gpu_counts(coex, d, s2, chunk=chunk, width=1).tolist() == ec.tolist()
        pos, pat = coex.find(d, s, chunk=777)
        assert pos.cpu().numpy().tolist() == epos.tolist()
        assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()


def test_join_levels(coex):
    # enough non-converged chunks for one, two and three composed levels of
    # the join (64, 4,096 and 262,144 maps per level): the parity automaton
    # (no synchronising word) and random tables, byte and 2-bit input
    n = 1_500_007
    seq = synth.markov_bytes(27, n, with_n=True)
    seq[100_000:100_050] = ord("N")
    s = dev_bytes(coex, seq)
    s2 = dev_2bit(coex, seq)[0]
    tables = [(_parity_table(), 1)] + [(synth.random_table(seed, 12 + 9 * seed, 2), 2) for seed in (40, 41)]
    for (dl, q0, off, ids), P in tables:
        d = coex.Dfa.table(dl, q0, off, ids, P)
        t = oracle.make_table(dl, q0, off, ids, P)
        ec = oracle.scan_table(t, oracle.byte_seq(seq))[0]
        for chunk in [8, 64, 512, 40_000]:
            say("join levels", dl.size // 4, chunk)
            assert gpu_counts(coex, d, s, chunk=chunk).tolist() == ec.tolist()
            assert gpu_counts(coex, d, s2, chunk=chunk, step=1).tolist() == ec.tolist()
        init, last, cnt = coex.count_chunks(d, s, 64)
        e, c0 = oracle.run_range(t, oracle.byte_seq(seq), 0, 64 * 700, t.q0)
        assert int(init.cpu().numpy()[0]) == t.q0
        assert int(last.cpu().numpy()[699]) == e
        assert cnt.cpu().numpy()[:700].sum(axis=0).tolist() == c0.tolist()


def test_join_wide_lists_and_inexact_counts(coex):
    # non-converged chunks of automata whose candidate lists are wider than a
    # join map row (more than 64 states: the join walks each run of them in
    # order), of one past the two-symbol limit (1,100 states: one-symbol
    # candidate runs) and of one with up to 20 patterns per state (two-symbol
    # entries cannot count exactly: one-symbol candidate runs)
    n = 300_007
    seq = synth.markov_bytes(28, n, with_n=True)
    s = dev_bytes(coex, seq)
    s2 = dev_2bit(coex, seq)[0]
    tables = [(synth.random_table(42, 300, 3), 3, 1), (synth.random_table(43, 1100, 2), 2, 0),
              (synth.random_table(44, 50, 30, accept_frac=0.3, max_out=20), 30, 0)]
    for (dl, q0, off, ids), P, lookback in tables:
        d = coex.Dfa.table(dl, q0, off, ids, P)
        t = oracle.make_table(dl, q0, off, ids, P)
        ec = oracle.scan_table(t, oracle.byte_seq(seq))[0]
        for chunk in [512, 9_999]:
            say("wide lists", dl.size // 4, chunk)
            assert gpu_counts(coex, d, s, chunk=chunk, lookback=lookback).tolist() == ec.tolist()
            assert gpu_counts(coex, d, s2, chunk=chunk, lookback=lookback).tolist() == ec.tolist()


def test_unaligned_starts(coex):
    # sequences starting at any base of their buffers (the text T[1..n] wherever
    # it lies): byte sequences by address (1..15 bytes past a 16-byte boundary,
    # and further) and by first_base, 2-bit sequences by first_base; counts and
    # positions of an automaton with a synchronising word and counts of one
    # without, against the oracle on the same bases
    n = 150_011
    seq = synth.markov_bytes(29, n, with_n=True)
    kmers = synth.random_kmers(30, 6, 7) + ["ACG"]
    d = coex.Dfa.kmers(kmers)
    dl, q0, off, ids = _parity_table()
    dp = coex.Dfa.table(dl, q0, off, ids, 1)
    tp = oracle.make_table(dl, q0, off, ids, 1)
    s = dev_bytes(coex, seq)
    s2 = dev_2bit(coex, seq)[0]
    for start in list(range(1, 16)) + [16, 17, 127, 128, 129, 1000, 4099]:
        m = n - start - (start % 7)
        sub = seq[start:start + m]
        ec, epos, epat = oracle.count_kmers(kmers, oracle.byte_seq(sub), positions=True)
        ep = oracle.scan_table(tp, oracle.byte_seq(sub))[0]
        views = {"address": s.sub(start, m, by_address=True), "first_base": s.sub(start, m),
                 "2bit": s2.sub(start, m)}
        for name, v in views.items():
            say("unaligned", start, name)
            assert gpu_counts(coex, d, v).tolist() == ec.tolist(), (start, name)
            assert gpu_counts(coex, d, v, chunk=64).tolist() == ec.tolist(), (start, name)
            assert gpu_counts(coex, dp, v, chunk=1000).tolist() == ep.tolist(), (start, name)
            pos, pat = coex.find(d, v, chunk=4096)
            assert pos.cpu().numpy().tolist() == epos.tolist(), (start, name)
            assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist(), (start, name)
        if start in (3, 129):
            init, last, cnt = coex.count_chunks(dp, views["2bit"], 777)
            e, c0 = oracle.run_range(tp, oracle.byte_seq(sub), 0, 777 * 5, tp.q0)
            assert int(last.cpu().numpy()[4]) == e
            assert cnt.cpu().numpy()[:5].sum(axis=0).tolist() == c0.tolist()


def test_errors_async(coex):
    # unchecked calls keep their device consistency failures until read: none
    # after correct scans, on the current stream, another stream and the
    # no-allocation path
    import torch
    seq = synth.markov_bytes(31, 100_000, with_n=True)
    s = dev_bytes(coex, seq)
    d = coex.Dfa.kmers(synth.random_kmers(32, 4, 8))
    dl, q0, off, ids = _parity_table()
    dp = coex.Dfa.table(dl, q0, off, ids, 1)
    for _ in range(3):
        coex.count(d, s)
        coex.count(dp, s, chunk=512)
        coex.find(d, s)
    out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    coex.errors_async(out)
    assert int(out.cpu()[0]) == 0
    st = torch.cuda.Stream()
    pinned = torch.full((1,), -1, dtype=torch.int32, pin_memory=True)
    with torch.cuda.stream(st):
        coex.count(dp, s, stream=st)
        coex.errors_async(pinned, stream=st)
    st.synchronize()
    assert int(pinned[0]) == 0
    buf = torch.empty(4, dtype=torch.int64, device="cuda")
    coex.count_noalloc(d, s, out=buf)
    assert coex.errors() == 0


def test_fasta_records(coex):
    # FASTA text (headers, line breaks of both kinds, soft-masked runs, an
    # empty record) parsed on the host and scanned on the device: each record
    # alone (first_base) and the whole output with one N between records,
    # byte and 2-bit, soft-masking on and off; the oracle runs on the records'
    # own bases as generated here
    import random
    rnd = random.Random(5)
    kmers = synth.random_kmers(33, 5, 6) + ["ACGTA"]
    d = coex.Dfa.kmers(kmers)
    bodies = []
    for r, n in enumerate([120_000, 0, 7, 250_003, 64, 90_000]):
        b = bytearray(synth.markov_bytes(300 + r, n, with_n=True).tobytes()) if n else bytearray()
        for _ in range(5):
            if n > 100:
                a = rnd.randrange(n - 50)
                b[a:a + 40] = b[a:a + 40].lower()
        bodies.append(bytes(b))
    parts = []
    for r, b in enumerate(bodies):
        eol = b"\r\n" if r % 2 else b"\n"
        parts.append(b">chr%d test record%s" % (r, eol))
        w = 60 + 20 * (r % 3)
        parts += [b[i:i + w] + eol for i in range(0, len(b), w)]
    text = b"".join(parts)
    for soft in (False, True):
        recs_bytes = [bytes(ord("N") if soft and 97 <= c <= 122 else c for c in b) for b in bodies]
        joined = b"N".join(recs_bytes)
        ec_all, epos, epat = oracle.count_kmers(kmers, oracle.byte_seq(np.frombuffer(joined, np.uint8)),
                                                positions=True)
        for enc in (coex.ENC_BYTE, coex.ENC_2BIT):
            seq, recs = coex.fasta_to_device(text, encoding=enc, softmask=soft, separate=True)
            assert [r.name for r in recs] == ["chr%d test record" % i for i in range(len(bodies))]
            assert seq.n == len(joined)
            total = np.zeros(len(kmers), np.uint64)
            for r, rb in enumerate(recs_bytes):
                say("fasta", soft, enc, r)
                assert recs[r].length == len(rb)
                ec = oracle.count_kmers(kmers, oracle.byte_seq(np.frombuffer(rb, np.uint8)))[0] if rb else \
                    np.zeros(len(kmers), np.uint64)
                if rb:
                    assert gpu_counts(coex, d, seq.sub(recs[r].start, recs[r].length)).tolist() == ec.tolist()
                total += ec
            assert total.tolist() == ec_all.tolist()  # the separators stop cross-record matches
            assert gpu_counts(coex, d, seq).tolist() == ec_all.tolist()
            pos, pat = coex.find(d, seq)
            assert pos.cpu().numpy().tolist() == epos.tolist()
            assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()


def test_partitioned_kmer_set(coex):
    # 1,000 12-mers, past the device tables as one automaton, split into parts
    # of at most 1,023 (three-symbol tables) or 300 states; per-pattern counts
    # against the oracle's own automaton of the whole set, on a long and a
    # short input, byte and 2-bit; unchecked calls leave no kept failure
    kmers = synth.random_kmers(61, 1000, 12)
    n = 1_000_003
    seq = synth.markov_bytes(62, n, with_n=True)
    for i in range(300):  # planted occurrences
        at = 1000 + i * 3301
        seq[at:at + 12] = np.frombuffer(kmers[(7 * i) % 1000].encode(), dtype=np.uint8)
    ec = oracle.count_kmers(kmers, oracle.byte_seq(seq))[0]
    short = seq[:5000].copy()
    es = oracle.count_kmers(kmers, oracle.byte_seq(short))[0]
    s, s2 = dev_bytes(coex, seq), dev_2bit(coex, seq)[0]
    ss = dev_bytes(coex, short)
    for budget in (0, 300):
        p = coex.Partition(kmers, max_states=budget)
        say("partitioned", budget, p.n_parts)
        got = lambda x, **kw: p.count(x, **kw).cpu().numpy().view(np.uint64).tolist()
        assert got(s, check=True) == ec.tolist()
        assert got(s2) == ec.tolist()
        assert got(ss) == es.tolist()
        assert got(s2.sub(1000, 5000)) == oracle.count_kmers(kmers, oracle.byte_seq(seq[1000:6000]))[0].tolist()
        p.free()
    assert coex.errors() == 0


def test_count_chunks_records(coex):
    n = 50_000
    seq = synth.markov_bytes(25, n, with_n=True)
    s = dev_bytes(coex, seq)
    # a table automaton keeps its numbering: records compare state by state
    dl, q0, off, ids = synth.random_table(7, 40, 3)
    d = coex.Dfa.table(dl, q0, off, ids, 3)
    t = oracle.make_table(dl, q0, off, ids, 3)
    for n_chunks in [1, 10, 50]:
        chunk = n // n_chunks
        say("records", n_chunks)
        init, last, cnt = coex.count_chunks(d, s, chunk)
        r = oracle.kcoex(t, oracle.byte_seq(seq), n_chunks)
        # the join's pick per chunk: the record whose init is the true state
        cur, picks = t.q0, []
        for c in range(n_chunks):
            idx = [i for i in range(len(r.cr_init)) if r.cr_chunk[i] == c and r.cr_init[i] == cur][0]
            picks.append(idx)
            cur = int(r.cr_last[idx])
        assert init.cpu().numpy().tolist() == [int(r.cr_init[i]) for i in picks]
        assert last.cpu().numpy().tolist() == [int(r.cr_last[i]) for i in picks]
        assert cnt.cpu().numpy().tolist() == [r.cr_counts[i].tolist() for i in picks]


def test_edge_cases(coex):
    k12 = synth.random_kmers(9, 1, 12)[0]
    d = coex.Dfa.kmers([k12, "ACGT"])
    cases = {
        "empty": b"",
        "one": b"A",
        "all_N": b"N" * 5000,
        "short": (k12 + "A").encode(),
        "spanning": ("TT" + k12 + "GG" + k12).encode(),
        "n_at_boundaries": ("ACGTN" * 200 + k12 * 3).encode(),
        "lowercase": (k12.lower() + "acgt" + "xyz" + k12).encode(),
        "all_bytes": bytes(range(256)) * 20 + k12.encode(),
    }
    for name, text in cases.items():
        arr = np.frombuffer(text, dtype=np.uint8).copy() if text else np.zeros(0, np.uint8)
        expect = oracle.count_kmers([k12, "ACGT"], oracle.byte_seq(arr))[0].tolist()
        s = dev_bytes(coex, arr) if arr.size else coex.to_device(np.zeros(16, np.uint8), n=0)
        for chunk in [0, 4, 5, 16, 64, 1000]:
            say("edge", name, chunk)
            assert gpu_counts(coex, d, s, chunk=chunk).tolist() == expect, (name, chunk)
        if arr.size:
            s2 = dev_2bit(coex, arr)[0]
            assert gpu_counts(coex, d, s2, chunk=4).tolist() == expect, name
    # a 100-mer: chunks shorter than the synchronising depth
    long = synth.random_kmers(10, 1, 100)[0]
    d = coex.Dfa.kmers([long, long[:30]])
    text = synth.markov_bytes(26, 20_000).tobytes().decode()
    text = text[:5000] + long + text[5000:9000] + long + long + text[9000:]
    arr = np.frombuffer(text.encode(), dtype=np.uint8).copy()
    expect = oracle.count_kmers([long, long[:30]], oracle.byte_seq(arr))[0].tolist()
    s = dev_bytes(coex, arr)
    for chunk in [16, 64, 99, 512]:
        say("long pattern", chunk)
        assert gpu_counts(coex, d, s, chunk=chunk).tolist() == expect


def test_full_small_and_mid(coex):
    # the small and mid workloads at full size, with the bench's launch choices
    seq, kmers = configs.small()
    d = coex.Dfa.kmers(kmers)
    s = dev_bytes(coex, seq)
    ec, epos, epat = oracle.count_kmers(kmers, oracle.byte_seq(seq), positions=True)
    assert gpu_counts(coex, d, s, chunk=configs.SMALL_CHUNK).tolist() == ec.tolist()
    # the bench step: counts and positions from one scan
    c, pos, pat = coex.count_find(d, s, chunk=configs.SMALL_CHUNK)
    assert c.cpu().numpy().view(np.uint64).tolist() == ec.tolist()
    assert pos.cpu().numpy().tolist() == epos.tolist()
    assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()
    seq, rx = configs.mid()
    say("mid full", rx)
    d = coex.Dfa.regex(rx)
    s = dev_bytes(coex, seq)
    m, epos = oracle.Regex(rx).scan(oracle.byte_seq(seq), positions=True)
    assert gpu_counts(coex, d, s).tolist() == [m]
    pos, _ = coex.find(d, s)
    assert pos.cpu().numpy().tolist() == epos.tolist()
    c, pos, _ = coex.count_find(d, s)
    assert c.cpu().numpy().view(np.uint64).tolist() == [m]
    assert pos.cpu().numpy().tolist() == epos.tolist()


def test_full_genome(coex):
    # the 3.2e9-base workload in the bench's launch configuration; the oracle
    # computes all 64 counts over the whole sequence
    import torch
    packed, mask, kmers = configs.genome()
    n = configs.GENOME_N
    say("genome full: generated")
    d = coex.Dfa.kmers(kmers)
    s = coex.to_device(packed, n=n, encoding=coex.ENC_2BIT, nmask=mask)
    got = gpu_counts(coex, d, s)
    got3 = gpu_counts(coex, d, s, step=3)
    got2 = gpu_counts(coex, d, s, step=2)
    got32 = gpu_counts(coex, d, s, step=3, chains=2)
    got22 = gpu_counts(coex, d, s, step=2, chains=2)
    pos, pat = coex.find(d, s)
    say("genome full: gpu done", int(got.sum()), "matches", pos.numel())
    expect, epos, epat = oracle.count_kmers(kmers, oracle.twobit_seq(packed, mask, n), positions=True)
    say("genome full: oracle done", int(expect.sum()))
    assert got.tolist() == expect.tolist()
    # per-pattern end positions of the whole sequence ("count and extract")
    assert pos.cpu().numpy().tolist() == epos.tolist()
    assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()
    assert got3.tolist() == expect.tolist()
    assert got2.tolist() == expect.tolist()
    assert got32.tolist() == expect.tolist()
    assert got22.tolist() == expect.tolist()
    del s
    torch.cuda.empty_cache()


def test_parity_automaton_genome(coex):
    # the 3.2e9-base workload through the parity automaton, which has no
    # synchronising word: no chunk converges, every chunk's map is built and
    # the join composes about half a million maps; the oracle runs the whole
    # sequence from q0
    import torch
    packed, mask, _ = configs.genome()
    n = configs.GENOME_N
    say("parity genome: generated")
    dl, q0, off, ids = _parity_table()
    d = coex.Dfa.table(dl, q0, off, ids, 1)
    s = coex.to_device(packed, n=n, encoding=coex.ENC_2BIT, nmask=mask)
    got = gpu_counts(coex, d, s)
    got1 = gpu_counts(coex, d, s, step=1, chunk=1 << 16)
    say("parity genome: gpu done", got.tolist(), got1.tolist())
    expect = oracle.scan_table(oracle.make_table(dl, q0, off, ids, 1), oracle.twobit_seq(packed, mask, n))[0]
    say("parity genome: oracle done", expect.tolist())
    assert got.tolist() == expect.tolist()
    assert got1.tolist() == expect.tolist()
    del s
    torch.cuda.empty_cache()


def test_beyond_4g_bases(coex):
    # 2^32 + 2^24 + 777 bases (byte and 2-bit input): chunk offsets, block
    # addresses and end positions past 2^32; a pattern planted at the very end
    import torch
    n = (1 << 32) + (1 << 24) + 777
    seq = synth.markov_bytes(91, n, with_n=True)
    kmers = synth.random_kmers(92, 8, 10)
    seq[-10:] = np.frombuffer(kmers[3].encode(), dtype=np.uint8)
    say("beyond 4G: generated", n)
    ec, epos, epat = oracle.count_kmers(kmers, oracle.byte_seq(seq), positions=True)
    assert epos[-1] == n - 1 and int((epos >= (1 << 32)).sum()) > 0
    say("beyond 4G: oracle done", int(ec.sum()))
    d = coex.Dfa.kmers(kmers)
    s = dev_bytes(coex, seq)
    assert gpu_counts(coex, d, s).tolist() == ec.tolist()
    pos, pat = coex.find(d, s)
    assert pos.cpu().numpy().tolist() == epos.tolist()
    assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()
    say("beyond 4G: bytes ok")
    del s
    packed, mask = synth.bytes_to_2bit(seq)
    del seq
    s2 = coex.to_device(packed, n=n, encoding=coex.ENC_2BIT, nmask=mask)
    assert gpu_counts(coex, d, s2).tolist() == ec.tolist()
    pos, _ = coex.find(d, s2)
    assert pos.cpu().numpy().tolist() == epos.tolist()
    say("beyond 4G: 2-bit ok")
    del s2, pos, pat
    torch.cuda.empty_cache()


def test_large_automaton(coex):
    # 460 random 12-mers: about 3,800 states, past the two-symbol limit (1,024):
    # one-symbol rows with 16-bit state offsets, lookback up to 8 and more
    # than 64 possible starting states at short lookbacks
    kmers = synth.random_kmers(95, 460, 12)
    d = coex.Dfa.kmers(kmers)
    assert 1024 < d.info().n_states <= 4096
    n = 2_000_003
    seq = synth.markov_bytes(96, n, with_n=True)
    for i in range(0, 40):  # planted occurrences, some across chunk boundaries
        at = 4093 + i * 49_999
        seq[at:at + 12] = np.frombuffer(kmers[i * 11].encode(), dtype=np.uint8)
    ec, epos, epat = oracle.count_kmers(kmers, oracle.byte_seq(seq), positions=True)
    s = dev_bytes(coex, seq)
    s2 = dev_2bit(coex, seq)[0]
    for chunk in [0, 4096, 100_000]:
        say("large automaton", d.info().n_states, chunk)
        assert gpu_counts(coex, d, s, chunk=chunk).tolist() == ec.tolist()
        assert gpu_counts(coex, d, s2, chunk=chunk).tolist() == ec.tolist()
    pos, pat = coex.find(d, s)
    assert pos.cpu().numpy().tolist() == epos.tolist()
    assert pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist()
    with pytest.raises(coex.CoexError):
        coex.count(d, s, step=2)  # two symbols per lookup need at most 1,024 states


def test_streams_and_threads(coex):
    # four host threads, each with its own stream, count concurrently over
    # shared automaton handles (device copies made on first use) and their own
    # workspaces; every result equals the oracle
    import threading
    import torch
    pats = [synth.random_kmers(97, 10, 8), synth.random_kmers(98, 30, 11)]
    dfas = [coex.Dfa.kmers(k) for k in pats]
    seqs = [synth.markov_bytes(99 + i, 300_000 + 777 * i, with_n=True) for i in range(4)]
    expect = [[oracle.count_kmers(k, oracle.byte_seq(sq))[0].tolist() for k in pats] for sq in seqs]
    devs = [dev_bytes(coex, sq) for sq in seqs]
    torch.cuda.synchronize()
    got = {}
    errors = []

    def worker(t):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for r in range(4):
                    for j, d in enumerate(dfas):
                        c = coex.count(d, devs[t], chunk=[0, 4096][r % 2], stream=st, check=True)
                        got[(t, r, j)] = c.cpu().numpy().view(np.uint64).tolist()
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    say("streams and threads:", len(got), "calls")
    for (t, r, j), v in got.items():
        assert v == expect[t][j], (t, r, j)
