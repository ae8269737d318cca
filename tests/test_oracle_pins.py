"""Pins of the CPU oracle against things other than itself: brute force,
Python's `re` on tiny inputs, closed forms, invariants and the paper's worked
examples (Tables I-III, Fig. 2, Table IV).  CPU only."""
import itertools
import os
import re

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RC = str.maketrans("ACGTacgt", "TGCAtgca")


def rc(s: str) -> str:
    return s.translate(RC)[::-1]


# ------------------------------------------------------------------ generator
def test_generator_python_twin_matches_c():
    L = synth._load()
    for seed, tag, i in [(0, 1, 0), (1, 2, 5), (303, 11, 1000), (2 ** 40 + 7, 3, 123456789)]:
        assert L.synth_draw(seed, tag, i) == synth.draw(seed, tag, i)


def test_generator_formats_agree():
    n = 300_001
    b = synth.markov_bytes(2, n, with_n=True)
    packed, mask = synth.markov_2bit(2, n, with_n=True)
    assert (oracle.decode(oracle.byte_seq(b)) == oracle.decode(oracle.twobit_seq(packed, mask, n))).all()
    p2, m2 = synth.bytes_to_2bit(b)
    assert (oracle.decode(oracle.twobit_seq(p2, m2, n)) == oracle.decode(oracle.byte_seq(b))).all()


def test_generator_statistics():
    n = 4_000_000
    b = synth.markov_bytes(7, n, with_n=True)
    s = oracle.decode(oracle.byte_seq(b))
    valid = s >= 0
    gc = np.isin(s[valid], [1, 2]).mean()
    assert abs(gc - 0.41) < 0.005
    nfrac = (~valid).mean()
    assert 0.003 < nfrac < 0.03
    # repeat probability: P(x_i == x_{i-1}) = 0.1 + 0.9 * sum(pi^2)
    pi = np.array([0.295, 0.205, 0.205, 0.295])
    both = valid[1:] & valid[:-1]
    rep = (s[1:][both] == s[:-1][both]).mean()
    assert abs(rep - (0.1 + 0.9 * (pi ** 2).sum())) < 0.005
    u = synth.iid_bytes(1, 1 << 20)
    freq = np.bincount(u, minlength=256)[[65, 67, 71, 84]] / u.size
    assert np.all(np.abs(freq - 0.25) < 0.005)


# ------------------------------------------------------------------ decoding
def test_decode_bytes():
    s = oracle.byte_seq(b"ACGTacgtNn-x\x00Z")
    assert oracle.decode(s).tolist() == [0, 1, 2, 3, 0, 1, 2, 3, -1, -1, -1, -1, -1, -1]


def test_decode_2bit_layout():
    # bases T,G,C,A,A,C -> codes 3,2,1,0,0,1; base i at bits 2*(i%4) of byte i/4
    packed = np.array([3 | (2 << 2) | (1 << 4) | (0 << 6), 0 | (1 << 2)], dtype=np.uint8)
    mask = np.array([0b000100], dtype=np.uint8)  # base 2 is N
    s = oracle.twobit_seq(packed, mask, 6)
    assert oracle.decode(s).tolist() == [3, 2, -1, 0, 0, 1]
    s2 = oracle.twobit_seq(packed, None, 6)
    assert oracle.decode(s2).tolist() == [3, 2, 1, 0, 0, 1]


# ------------------------------------------------------------------ k-mer brute force
def _py_overlapping(text: str, pats):
    """Overlapping occurrences via Python's re look-ahead (a library routine);
    'N' (and any non-ACGT) never matches because patterns are ACGT only."""
    up = text.upper()
    out = []
    for p in pats:
        out.append(len(re.findall("(?=%s)" % re.escape(p.upper()), up)))
    return out


def test_brute_closed_forms():
    s = oracle.byte_seq("AAAA")
    c, pos, pat = oracle.kmer_brute(["AA", "AAA", "A"], s, positions=True)
    assert c.tolist() == [3, 2, 4]
    # positions ascending, ties by pattern id
    assert list(zip(pos.tolist(), pat.tolist())) == [(0, 2), (1, 0), (1, 2), (2, 0), (2, 1), (2, 2), (3, 0),
                                                     (3, 1), (3, 2)]
    assert oracle.kmer_brute(["AC"], oracle.byte_seq("ANC"))[0].tolist() == [0]
    assert oracle.kmer_brute(["ac"], oracle.byte_seq("xACgtAc"))[0].tolist() == [2]


def test_brute_vs_python_re():
    for seed in range(8):
        st = synth.Stream(seed, 99)
        text = "".join("ACGTN"[st.below(5)] if st.below(10) else "acgt"[st.below(4)] for _ in range(800))
        pats = [synth.random_kmers(seed * 7 + k, 1, 1 + k % 5)[0] for k in range(6)]
        got = oracle.kmer_brute(pats, oracle.byte_seq(text))[0].tolist()
        assert got == _py_overlapping(text, pats)


# ------------------------------------------------------------------ Aho-Corasick
def _state_after(t: oracle.Table, text: str) -> int:
    return oracle.scan_table(t, oracle.byte_seq(text))[3]


def test_ac_single_pattern_is_kmp_size():
    for k in [1, 3, 8, 12]:
        w = synth.random_kmers(k, 1, k)[0]
        assert oracle.ac_build([w]).n_states == k + 1


def test_ac_fig2_transitions_by_label():
    # Fig. 2: patterns acg, cat, cta, tta; from the state reached by "ac",
    # reading a, c, t leads to the states of "ca", "c", "ct" respectively.
    t = oracle.ac_build(["acg", "cat", "cta", "tta"])
    assert t.n_states == 12  # root, a, ac, acg, c, ca, cat, ct, cta, t, tt, tta
    for nxt, label in [("a", "ca"), ("c", "c"), ("t", "ct")]:
        assert _state_after(t, "ac" + nxt) == _state_after(t, label)
    # accepting exactly at pattern ends
    c, pos, _, _ = oracle.scan_table(t, oracle.byte_seq("acgcatctatta"), positions=True)
    assert c.tolist() == [1, 1, 1, 1]


def test_ac_exhaustive_short_strings():
    sets = [["AC", "C", "CAC"], ["AAA", "AA"], ["ACGT", "CGTA", "GT"], ["G", "G"], ["TTAG", "TAG", "AG", "G"]]
    alphabet = "ACGTN"
    for pats in sets:
        t = oracle.ac_build(pats)
        for L in range(0, 6):
            for tup in itertools.product(alphabet, repeat=L):
                text = "".join(tup)
                s = oracle.byte_seq(text)
                a = oracle.scan_table(t, s, positions=True)
                b = oracle.kmer_brute(pats, s, positions=True)
                assert a[0].tolist() == b[0].tolist(), (pats, text)
                assert a[1].tolist() == b[1].tolist() and a[2].tolist() == b[2].tolist()


def test_ac_random_vs_brute():
    for seed in range(6):
        st = synth.Stream(seed, 98)
        n = 10_000
        seq = synth.markov_bytes(seed, n, with_n=True)
        seq[st.below(n)::97] = ord("N")
        pats = []
        for k in range(12):
            pats += synth.random_kmers(seed * 100 + k, 1, 1 + st.below(7))
        pats.append(pats[0])                  # duplicate pattern
        pats.append(pats[1][-1:])             # suffix of another pattern
        s = oracle.byte_seq(seq)
        a = oracle.count_kmers(pats, s, positions=True)
        b = oracle.kmer_brute(pats, s, positions=True)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        packed, mask = synth.bytes_to_2bit(seq)
        c = oracle.count_kmers(pats, oracle.twobit_seq(packed, mask, n), positions=True)
        for x, y in zip(a, c):
            assert np.array_equal(x, y)


def test_ac_rejects_bad_patterns():
    with pytest.raises(ValueError):
        oracle.ac_build(["ACN"])
    with pytest.raises(ValueError):
        oracle.ac_build([""])


# ------------------------------------------------------------------ regex
def _py_regex_ends(rx: str, text: str):
    """End positions i with some T[j..i] in L(rx), by Python's re.fullmatch
    over every window without a non-ACGT byte."""
    pat = re.compile(rx, re.IGNORECASE)
    out = []
    for i in range(len(text)):
        for j in range(i, -1, -1):
            if text[j].upper() not in "ACGT":
                break
            if pat.fullmatch(text, j, i + 1):
                out.append(i)
                break
    return out


TABLE4 = [
    "agggtaaa|tttaccct",
    "(c|g|t)gggtaaa|tttaccc(a|c|g)",
    "a(a|c|t)ggtaaa|tttacc(a|g|t)t",
    "ag(a|c|t)gtaaa|tttac(a|g|t)ct",
    "agg(a|c|t)taaa|ttta(a|g|t)cct",
    "aggg(a|c|g)aaa|ttt(c|g|t)ccct",
    "agggt(c|g|t)aa|tt(a|c|g)accct",
    "agggta(c|g|t)a|t(a|c|g)taccct",
    "agggtaa(c|g|t)|(a|c|g)ttaccct",
]


def test_regex_vs_python_re_random():
    for seed in range(20):
        rx = synth.random_regex(seed)
        st = synth.Stream(seed, 97)
        text = "".join("ACGTN"[st.below(5)] if st.below(20) == 0 else "ACGT"[st.below(4)] for _ in range(300))
        got = oracle.Regex(rx).scan(oracle.byte_seq(text), positions=True)[1].tolist()
        assert got == _py_regex_ends(rx, text), rx


def test_regex_language_exhaustive():
    for rx in ["A(C|G)*T", "[AC]{2,3}G?", "(AC|CA)+", "A.{1,2}T", "G{3}|C", "(A|T)(C?G){1,2}"]:
        R = oracle.Regex(rx)
        for L in range(1, 7):
            for tup in itertools.product("ACGT", repeat=L):
                text = "".join(tup)
                got = R.scan(oracle.byte_seq(text), positions=True)[1].tolist()
                assert got == _py_regex_ends(rx, text), (rx, text)


def test_regex_literal_alternation_equals_kmers():
    seq = oracle.byte_seq(synth.markov_bytes(11, 200_000))
    for rx in TABLE4[:1]:
        a, b = rx.split("|")
        assert oracle.Regex(rx).scan(seq)[0] == int(oracle.kmer_brute([a, b], seq)[0].sum())
    # a class expands to the union of its words
    words = ["CGGGTAAA", "GGGGTAAA", "TGGGTAAA", "TTTACCCA", "TTTACCCC", "TTTACCCG"]
    assert oracle.Regex(TABLE4[1]).scan(seq)[0] == int(oracle.count_kmers(words, seq)[0].sum())


def test_regex_reverse_complement_symmetry():
    # every Table IV expression is "word set | reverse complement of it" with
    # all words 8 long, so end positions in T and in rc(T) are equinumerous
    text = synth.markov_bytes(12, 300_000).tobytes().decode()
    rtext = rc(text)
    for rx in TABLE4:
        R = oracle.Regex(rx)
        assert R.scan(oracle.byte_seq(text))[0] == R.scan(oracle.byte_seq(rtext))[0]


def test_regex_rejects():
    for bad in ["", "A|", "(A", "A{3,2}", "N", "A*", "(A|C)?"]:
        with pytest.raises(ValueError):
            oracle.Regex(bad)


# ------------------------------------------------------------------ tables and invariants
def _parity_table():
    # state = parity of A's since the last reset; pattern 0 ends where it is odd
    delta = np.array([1, 0, 0, 0, 0, 1, 1, 1], dtype=np.uint32)
    return oracle.make_table(delta, 0, [0, 0, 1], [0], 1)


def test_scan_table_closed_form_parity():
    text = synth.markov_bytes(5, 50_000).tobytes().decode()
    t = _parity_table()
    _, pos, _, _ = oracle.scan_table(t, oracle.byte_seq(text), positions=True)
    # closed form: running parity of A counts, restarted after each N
    par, expect = 0, []
    for i, ch in enumerate(text):
        if ch == "N":
            par = 0
            continue
        par ^= ch == "A"
        if par:
            expect.append(i)
    assert pos.tolist() == expect


def test_concat_with_reset_is_additive():
    pats = synth.random_kmers(3, 5, 4)
    x = synth.markov_bytes(31, 5000).tobytes().decode()
    y = synth.markov_bytes(32, 7000).tobytes().decode()
    cx = oracle.count_kmers(pats, oracle.byte_seq(x))[0]
    cy = oracle.count_kmers(pats, oracle.byte_seq(y))[0]
    cxy = oracle.count_kmers(pats, oracle.byte_seq(x + "N" + y))[0]
    assert (cxy == cx + cy).all()


def test_iid_expected_count_sanity():
    # E[count] of one 8-mer in n iid uniform bases is (n-7)/4^8 (= 16 at 1 MiB)
    tot = 0
    for seed in range(8):
        seq = synth.iid_bytes(seed, 1 << 20)
        w = synth.random_kmers(100 + seed, 1, 8)
        tot += int(oracle.count_kmers(w, oracle.byte_seq(seq))[0][0])
    assert abs(tot / 8 - ((1 << 20) - 7) / 4 ** 8) < 6


# ------------------------------------------------------------------ the paper's method
def _read_traces():
    rows, expect = {}, {}
    with open(os.path.join(GOLDEN, "table1_traces.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "expect":
                expect[parts[1]] = [int(x) for x in parts[2:]]
            else:
                rows.setdefault(parts[0], []).append([int(x) for x in parts[2:]])
    return rows, expect


def test_table1_converging_points():
    rows, expect = _read_traces()
    for tab in ["b", "c"]:
        r0 = rows[tab][0]
        got = [oracle.first_meet(r0, ri) + 1 for ri in rows[tab][1:]]
        assert got == expect[tab]
    # same state at different positions is not a converging point (Table I.c:
    # state 11 is R0's 5th and R2's 7th state)
    r0, r2 = rows["c"][0], rows["c"][2]
    assert r0[4] == 11 and r2[6] == 11 and oracle.first_meet(r0, r2) == 8


def test_table2_3_fixup():
    vals = {}
    with open(os.path.join(GOLDEN, "table2_3_fixup.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            vals[k] = [int(x) for x in v]
    got = oracle.fixup(vals["own_prefix"], vals["r0_total"], vals["r0_prefix"])
    assert got.tolist() == vals["expect"]


def test_pss_contains_true_state_and_is_image():
    t = oracle.ac_build(synth.random_kmers(5, 10, 5))
    for c in range(4):
        img = sorted({int(t.delta[q * 4 + c]) for q in range(t.n_states)})
        assert oracle.pss(t, c).tolist() == img
    assert oracle.pss(t, -1).tolist() == [t.q0]


@pytest.mark.parametrize("kind", ["kmers", "table", "parity"])
def test_kcoex_equals_sequential(kind):
    for seed in range(4):
        n = 3000 + 37 * seed
        seq = synth.markov_bytes(40 + seed, n, with_n=True)
        seq[::211] = ord("N")
        s = oracle.byte_seq(seq)
        if kind == "kmers":
            t = oracle.ac_build(synth.random_kmers(seed, 6, 3 + seed))
        elif kind == "table":
            t = oracle.make_table(*synth.random_table(seed, 9 + seed, 3), 3)
        else:
            t = _parity_table()
        ref = oracle.scan_table(t, s)[0]
        for n_chunks in [1, 2, 7, 64, n // 3, n, n + 5]:
            for window in [0, 3, 10]:
                r = oracle.kcoex(t, s, n_chunks, window)
                assert np.array_equal(r.totals, ref), (kind, seed, n_chunks, window)
                # every record equals a direct run of its chunk from its init state
                base = n // n_chunks
                for i in range(0, len(r.cr_init), max(1, len(r.cr_init) // 50)):
                    c = int(r.cr_chunk[i])
                    lo, hi = c * base, (n if c + 1 == n_chunks else (c + 1) * base)
                    e, cnt = oracle.run_range(t, s, lo, hi, int(r.cr_init[i]))
                    assert e == r.cr_last[i] and np.array_equal(cnt, r.cr_counts[i])
