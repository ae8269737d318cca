"""Host-side checks of libcoex (no GPU needed): the C ABI exports, the
automaton compilers (checked against the oracle's brute-force matchers by
walking the exported tables), analysis results and error paths."""
import itertools
import os
import re

import numpy as np
import pytest

import oracle
import synth
from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CODE = {"A": 0, "C": 1, "G": 2, "T": 3, "a": 0, "c": 1, "g": 2, "t": 3}


@pytest.fixture(scope="module")
def coex():
    import paper_1509_01506_amd as m
    return m


def walk(dfa, text):
    """Plain walk of an exported table (test helper): end positions and ids."""
    delta, q0, off, ids = dfa.export()
    s, out = q0, []
    for i, ch in enumerate(text):
        c = CODE.get(ch, -1)
        if c < 0:
            s = q0
            continue
        s = int(delta[4 * s + c])
        for k in range(off[s], off[s + 1]):
            out.append((i, int(ids[k])))
    return out


def test_header_symbols_exported(coex):
    src = open(os.path.join(ROOT, "include", "coex.h")).read()
    names = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(coex_\w+)\s*\(", src, re.M))
    assert len(names) >= 12
    lib = coex._lib()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(coex.EXPORTED) == names


def test_struct_layouts_match_header(coex, tmp_path):
    # the binding's ctypes structures against the header's, as a C compiler
    # lays them out
    import ctypes
    import subprocess
    prog = tmp_path / "layout.c"
    prog.write_text("""#include <stddef.h>
#include <stdio.h>
#include "coex.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(coex_seq), offsetof(coex_seq, n_bases), offsetof(coex_seq, encoding),
         offsetof(coex_seq, first_base), sizeof(coex_opts), offsetof(coex_opts, chains));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(prog)])
    got = [int(x) for x in subprocess.check_output([str(exe)], text=True).split()]
    S, O = coex._Seq, coex._Opts
    assert got == [ctypes.sizeof(S), S.n_bases.offset, S.encoding.offset, S.first_base.offset, ctypes.sizeof(O),
                   O.chains.offset]


def test_sub_sequences(coex):
    # sub-sequence descriptors share the buffers: first_base or the pointer moves
    import types
    fake = types.SimpleNamespace(data_ptr=lambda: 4096)
    s = coex.DeviceSeq(fake, 100, coex.ENC_BYTE)
    a = s.sub(5, 90)
    assert (a.first, a.byte_offset, a.n) == (5, 0, 90)
    b = a.sub(3, by_address=True)
    assert (b.first, b.byte_offset, b.n) == (5, 3, 87)
    c = b._c()
    assert (c.bases, c.first_base, c.n_bases) == (4099, 5, 87)
    with pytest.raises(ValueError):
        s.sub(50, 51)
    with pytest.raises(ValueError):
        coex.DeviceSeq(fake, 100, coex.ENC_2BIT).sub(1, by_address=True)


def test_kmers_match_brute_force(coex):
    for seed in range(5):
        st = synth.Stream(seed, 77)
        pats = [synth.random_kmers(seed * 50 + j, 1, 1 + st.below(6))[0] for j in range(8)]
        pats += [pats[0], pats[2][1:] or "A"]
        d = coex.Dfa.kmers(pats)
        text = synth.markov_bytes(seed + 9, 3000).tobytes().decode()
        c, pos, pat = oracle.kmer_brute(pats, oracle.byte_seq(text), positions=True)
        assert walk(d, text) == list(zip(pos.tolist(), pat.tolist()))


def test_kmers_exhaustive_short(coex):
    pats = ["ACG", "CG", "G", "TTT", "TT"]
    d = coex.Dfa.kmers(pats)
    for L in range(0, 6):
        for tup in itertools.product("ACGTN", repeat=L):
            text = "".join(tup)
            _, pos, pat = oracle.kmer_brute(pats, oracle.byte_seq(text), positions=True)
            assert walk(d, text) == list(zip(pos.tolist(), pat.tolist())), text


def test_single_pattern_kmp_size(coex):
    for k in [1, 5, 8, 12]:
        w = synth.random_kmers(k + 40, 1, k)[0]
        assert coex.Dfa.kmers([w]).info().n_states == k + 1


def test_fig2_transitions(coex):
    d = coex.Dfa.kmers(["acg", "cat", "cta", "tta"])
    delta, q0, _, _ = d.export()

    def state(text):
        s = q0
        for ch in text:
            s = int(delta[4 * s + CODE[ch]])
        return s
    for nxt, label in [("a", "ca"), ("c", "c"), ("t", "ct")]:
        assert state("ac" + nxt) == state(label)


def _is_minimal(delta, q0, off, ids):
    n = delta.size // 4
    label = {s: tuple(ids[off[s]:off[s + 1]]) for s in range(n)}
    def renumber(d):
        ids_ = {v: i for i, v in enumerate(sorted(set(d.values())))}
        return {s: ids_[v] for s, v in d.items()}
    cls = renumber(label)
    while True:
        sig = renumber({s: (cls[s],) + tuple(cls[int(delta[4 * s + c])] for c in range(4)) for s in range(n)})
        if len(set(sig.values())) == len(set(cls.values())):
            return len(set(sig.values())) == n
        cls = sig


def test_regex_language_and_minimality(coex):
    for rx in ["A(C|G)*T", "[AC]{2,3}G?", "(AC|CA)+", "A.{1,2}T", "G{3}|C", configs.mid_regex()]:
        d = coex.Dfa.regex(rx)
        R = oracle.Regex(rx)
        for L in range(1, 7):
            for tup in itertools.product("ACGT", repeat=L):
                text = "".join(tup)
                got = [p for p, _ in walk(d, text)]
                assert got == R.scan(oracle.byte_seq(text), positions=True)[1].tolist(), (rx, text)
        assert _is_minimal(*d.export())


def test_regex_random_vs_oracle(coex):
    for seed in range(30):
        rx = synth.random_regex(seed)
        try:
            d = coex.Dfa.regex(rx)
        except coex.CoexError as e:
            assert e.name == "ETOOBIG"
            continue
        text = synth.markov_bytes(seed, 4000).tobytes().decode()
        got = [p for p, _ in walk(d, text)]
        assert got == oracle.Regex(rx).scan(oracle.byte_seq(text), positions=True)[1].tolist(), rx


def test_table4_regexes_compile(coex):
    from test_oracle_pins import TABLE4
    text = synth.markov_bytes(3, 20000).tobytes().decode()
    for rx in TABLE4:
        d = coex.Dfa.regex(rx)
        got = [p for p, _ in walk(d, text)]
        assert got == oracle.Regex(rx).scan(oracle.byte_seq(text), positions=True)[1].tolist()


def test_workload_automata(coex):
    assert coex.Dfa.regex(configs.mid_regex()).info().n_states == 60
    inf = coex.Dfa.kmers(configs.genome_kmers()).info()
    assert 600 <= inf.n_states <= 700
    assert inf.sync_depth == 12 and inf.max_out == 1 and inf.n_accepting == 64
    assert coex.Dfa.kmers(configs.small()[1]).info().n_states == 9


def test_sync_depth_and_pss(coex):
    # finite language: depth <= longest pattern
    for k in [3, 8, 12]:
        d = coex.Dfa.kmers(synth.random_kmers(k, 16, k))
        inf = d.info()
        assert inf.sync_depth <= k
        assert all(inf.max_pss[i] >= inf.max_pss[i + 1] for i in range(8))
    # parity of A's never synchronises
    par = coex.Dfa.table([1, 0, 0, 0, 0, 1, 1, 1], 0, [0, 0, 1], [0], 1)
    assert par.info().sync_depth is None
    assert par.info().max_pss[8] == 2


def test_pss_brute_force(coex):
    # the possible starting states after k bases are the image of Q
    d = coex.Dfa.kmers(synth.random_kmers(9, 5, 4))
    delta, _, _, _ = d.export()
    n = delta.size // 4
    for k in [1, 2, 3]:
        mx = 0
        for w in itertools.product(range(4), repeat=k):
            img = set(range(n))
            for c in w:
                img = {int(delta[4 * s + c]) for s in img}
            mx = max(mx, len(img))
        assert d.info().max_pss[k] == mx


def test_errors(coex):
    def status(fn):
        with pytest.raises(coex.CoexError) as e:
            fn()
        return e.value.name
    assert status(lambda: coex.Dfa.kmers(["ACN"])) == "EALPHABET"
    assert status(lambda: coex.Dfa.kmers([""])) == "EALPHABET"
    assert status(lambda: coex.Dfa.kmers([])) == "EINVAL"
    assert status(lambda: coex.Dfa.regex("A(")) == "ESYNTAX"
    assert status(lambda: coex.Dfa.regex("A*")) == "ESYNTAX"
    assert status(lambda: coex.Dfa.regex("")) == "ESYNTAX"
    assert status(lambda: coex.Dfa.table([0, 0, 0, 5], 0, [0, 0], [], 0)) == "EINVAL"
    assert status(lambda: coex.Dfa.table([0, 0, 0, 0], 1, [0, 0], [], 0)) == "EINVAL"
    assert status(lambda: coex.Dfa.table([0, 0, 0, 0], 0, [0, 2], [0, 0], 1)) == "EINVAL"
    assert status(lambda: coex.Dfa.table([0, 0, 0, 0], 0, [0, 1], [3], 1)) == "EINVAL"
    n = 4097
    assert status(lambda: coex.Dfa.table(np.zeros(4 * n, np.uint32), 0, np.zeros(n + 1, np.uint32), [], 0)) \
        == "ETOOBIG"


def test_table_roundtrip(coex):
    delta, q0, off, ids = synth.random_table(4, 50, 7)
    d = coex.Dfa.table(delta, q0, off, ids, 7)
    d2, q2, o2, i2 = d.export()
    assert np.array_equal(d2, delta) and q2 == q0 and np.array_equal(o2, off) and np.array_equal(i2, ids)
