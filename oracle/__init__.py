"""CPU ORACLE — test infrastructure only.

Python access to ``oracle.c``: plain sequential definitions of what the
chunked speculative DFA scan computes (counts and end positions of every
overlapping occurrence), built from the paper's problem statement (Section II),
its modified Aho-Corasick automaton (Section III.B.1) and its Algorithm 1.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the product
library in ``paper_1509_01506_amd``; the only common dependency is the seeded
input generator package ``synth``.

Pins: every function here is checked in ``tests/test_oracle_pins.py`` against
something other than itself (brute force, Python's ``re`` on tiny inputs,
closed forms, invariants, the paper's worked examples).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

ENC_BYTE = 0
ENC_2BIT = 1
RESET = -1


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, single thread)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, os.path.join(_HERE, "oracle.c")])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        p, u32, u64, i64, ci = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        L.or_decode.argtypes = [p, p, u64, ci, u64, u64, p]
        L.or_scan_table.restype = u64
        L.or_scan_table.argtypes = [p, u32, u32, p, p, p, p, u64, ci, p, p, p, u64, p]
        L.or_run_range.restype = u32
        L.or_run_range.argtypes = [p, u32, p, p, p, p, u64, ci, u64, u64, u32, p]
        L.or_ac_build.restype = i64
        L.or_ac_build.argtypes = [p, u32, u32, p, p, p, u64]
        L.or_kmer_brute.restype = u64
        L.or_kmer_brute.argtypes = [p, u32, p, p, u64, ci, p, p, p, u64]
        L.or_regex_build.restype = p
        L.or_regex_build.argtypes = [ctypes.c_char_p, ci, ctypes.POINTER(ci)]
        L.or_regex_positions.restype = ci
        L.or_regex_positions.argtypes = [p]
        L.or_regex_free.argtypes = [p]
        L.or_regex_scan.restype = u64
        L.or_regex_scan.argtypes = [p, p, p, u64, ci, p, u64]
        L.or_first_meet.restype = i64
        L.or_first_meet.argtypes = [p, p, u64]
        L.or_fixup.argtypes = [p, p, p, u32, p]
        L.or_pss.restype = u32
        L.or_pss.argtypes = [p, u32, u32, ci, p]
        L.or_kcoex.restype = i64
        L.or_kcoex.argtypes = [p, u32, u32, p, p, u32, p, p, u64, ci, u64, u64, p, p, p, p, p, u64, p]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def host_threads() -> int:
    """Host cores this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def pool_map(fn, items, threads: Optional[int] = None) -> list:
    """[fn(x) for x in items] on a thread pool.  Every oracle call is one
    sequential C function that releases the interpreter lock, so independent
    (sequence, automaton) pairs run on separate cores; each pair itself stays
    a single sequential scan."""
    items = list(items)
    threads = threads or host_threads()
    if threads <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


# ------------------------------------------------------------------ sequences
@dataclass
class Seq:
    """A sequence in one of the two formats.  For ENC_BYTE `data` holds one
    ASCII byte per base; for ENC_2BIT it holds packed codes and `nmask` the
    N bits (or None)."""
    data: np.ndarray
    n: int
    enc: int = ENC_BYTE
    nmask: Optional[np.ndarray] = None


def byte_seq(arr) -> Seq:
    if isinstance(arr, (bytes, str)):
        arr = np.frombuffer(arr.encode() if isinstance(arr, str) else arr, dtype=np.uint8)
    a = np.ascontiguousarray(arr, dtype=np.uint8)
    return Seq(a, a.size, ENC_BYTE, None)


def twobit_seq(packed: np.ndarray, mask: Optional[np.ndarray], n: int) -> Seq:
    return Seq(np.ascontiguousarray(packed, dtype=np.uint8), n, ENC_2BIT,
               None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8))


def decode(seq: Seq, lo: int = 0, hi: Optional[int] = None) -> np.ndarray:
    """Symbols 0..3 (A,C,G,T) or -1 (reset) for bases [lo, hi)."""
    hi = seq.n if hi is None else hi
    out = np.empty(max(hi - lo, 0), dtype=np.int8)
    if hi > lo:
        _load().or_decode(_ptr(seq.data), _ptr(seq.nmask), seq.n, seq.enc, lo, hi, _ptr(out))
    return out


# ------------------------------------------------------------------ automata
@dataclass
class Table:
    """A complete DFA over A,C,G,T with output sets (CSR)."""
    delta: np.ndarray      # uint32[n_states*4]
    q0: int
    out_off: np.ndarray    # uint32[n_states+1]
    out_ids: np.ndarray    # uint32[...]
    n_patterns: int

    @property
    def n_states(self) -> int:
        return self.delta.size // 4


def make_table(delta, q0, out_off, out_ids, n_patterns) -> Table:
    """Normalise a caller's table: output ids sorted within each state."""
    delta = np.ascontiguousarray(delta, dtype=np.uint32)
    out_off = np.ascontiguousarray(out_off, dtype=np.uint32)
    ids = np.array(out_ids, dtype=np.uint32)
    for s in range(out_off.size - 1):
        ids[out_off[s]:out_off[s + 1]] = np.sort(ids[out_off[s]:out_off[s + 1]])
    return Table(delta, int(q0), out_off, ids, int(n_patterns))


def ac_build(kmers: list[str]) -> Table:
    """The oracle's own Aho-Corasick automaton (complete transitions)."""
    L = _load()
    n_pat = len(kmers)
    max_states = sum(len(k) for k in kmers) + 1
    out_cap = max(1, sum(len(k) for k in kmers) * max(1, n_pat))
    out_cap = min(out_cap, max_states * max(1, n_pat))
    delta = np.zeros(max_states * 4, dtype=np.uint32)
    out_off = np.zeros(max_states + 1, dtype=np.uint32)
    out_ids = np.zeros(out_cap, dtype=np.uint32)
    enc = [k.encode("ascii") for k in kmers]
    arr = (ctypes.c_char_p * max(1, n_pat))(*enc)
    r = L.or_ac_build(ctypes.cast(arr, ctypes.c_void_p), n_pat, max_states, _ptr(delta), _ptr(out_off),
                      _ptr(out_ids), out_cap)
    if r == -1:
        raise ValueError("pattern empty or outside A/C/G/T")
    if r < 0:
        raise RuntimeError("oracle AC capacity")
    ns = int(r)
    return Table(delta[: ns * 4].copy(), 0, out_off[: ns + 1].copy(), out_ids[: out_off[ns]].copy(), n_pat)


def scan_table(t: Table, seq: Seq, positions: bool = False):
    """Sequential run from q0 (Section II).  Returns (counts uint64[P],
    positions int64[m] or None, pattern ids uint32[m] or None, end_state)."""
    L = _load()
    counts = np.zeros(max(1, t.n_patterns), dtype=np.uint64)
    end = ctypes.c_uint32(0)
    if not positions:
        L.or_scan_table(_ptr(t.delta), t.n_states, t.q0, _ptr(t.out_off), _ptr(t.out_ids), _ptr(seq.data),
                        _ptr(seq.nmask), seq.n, seq.enc, _ptr(counts), None, None, 0, ctypes.byref(end))
        return counts[: t.n_patterns], None, None, end.value
    m = int(L.or_scan_table(_ptr(t.delta), t.n_states, t.q0, _ptr(t.out_off), _ptr(t.out_ids), _ptr(seq.data),
                            _ptr(seq.nmask), seq.n, seq.enc, _ptr(counts), None, None, 0, ctypes.byref(end)))
    pos = np.zeros(max(1, m), dtype=np.int64)
    pat = np.zeros(max(1, m), dtype=np.uint32)
    counts[:] = 0
    L.or_scan_table(_ptr(t.delta), t.n_states, t.q0, _ptr(t.out_off), _ptr(t.out_ids), _ptr(seq.data),
                    _ptr(seq.nmask), seq.n, seq.enc, _ptr(counts), _ptr(pos), _ptr(pat), m, ctypes.byref(end))
    return counts[: t.n_patterns], pos[:m], pat[:m], end.value


def run_range(t: Table, seq: Seq, lo: int, hi: int, start: int):
    """Run over [lo, hi) from `start`; returns (end_state, counts)."""
    counts = np.zeros(max(1, t.n_patterns), dtype=np.uint64)
    e = _load().or_run_range(_ptr(t.delta), t.q0, _ptr(t.out_off), _ptr(t.out_ids), _ptr(seq.data),
                             _ptr(seq.nmask), seq.n, seq.enc, lo, hi, start, _ptr(counts))
    return int(e), counts[: t.n_patterns]


def kmer_brute(kmers: list[str], seq: Seq, positions: bool = False):
    """Direct comparison at every end position (Section II problem statement)."""
    L = _load()
    n_pat = len(kmers)
    enc = [k.encode("ascii") for k in kmers]
    arr = (ctypes.c_char_p * max(1, n_pat))(*enc)
    counts = np.zeros(max(1, n_pat), dtype=np.uint64)
    m = int(L.or_kmer_brute(ctypes.cast(arr, ctypes.c_void_p), n_pat, _ptr(seq.data), _ptr(seq.nmask), seq.n,
                            seq.enc, _ptr(counts), None, None, 0))
    if not positions:
        return counts[:n_pat], None, None
    pos = np.zeros(max(1, m), dtype=np.int64)
    pat = np.zeros(max(1, m), dtype=np.uint32)
    counts[:] = 0
    L.or_kmer_brute(ctypes.cast(arr, ctypes.c_void_p), n_pat, _ptr(seq.data), _ptr(seq.nmask), seq.n, seq.enc,
                    _ptr(counts), _ptr(pos), _ptr(pat), m)
    return counts[:n_pat], pos[:m], pat[:m]


def count_kmers(kmers: list[str], seq: Seq, positions: bool = False):
    """Counts (and positions) of every k-mer via the oracle's own AC automaton."""
    return scan_table(ac_build(kmers), seq, positions)[:3]


class Regex:
    """The oracle's Glushkov position automaton of one regular expression."""

    def __init__(self, text: str, max_positions: int = 4096):
        L = _load()
        err = ctypes.c_int(0)
        h = L.or_regex_build(text.encode("ascii"), max_positions, ctypes.byref(err))
        if not h:
            raise ValueError({1: "syntax", 2: "matches the empty string", 3: "too many positions"}.get(err.value,
                                                                                                      "error"))
        self._h = ctypes.c_void_p(h)
        self.text = text

    @property
    def n_positions(self) -> int:
        return _load().or_regex_positions(self._h)

    def scan(self, seq: Seq, positions: bool = False):
        """Returns (count, positions int64[count] or None)."""
        L = _load()
        m = int(L.or_regex_scan(self._h, _ptr(seq.data), _ptr(seq.nmask), seq.n, seq.enc, None, 0))
        if not positions:
            return m, None
        pos = np.zeros(max(1, m), dtype=np.int64)
        L.or_regex_scan(self._h, _ptr(seq.data), _ptr(seq.nmask), seq.n, seq.enc, _ptr(pos), m)
        return m, pos[:m]

    def __del__(self):
        try:
            _load().or_regex_free(self._h)
        except Exception:
            pass


# ------------------------------------------------------- the paper's method
def first_meet(r0_trace, ri_trace) -> int:
    a = np.ascontiguousarray(r0_trace, dtype=np.uint32)
    b = np.ascontiguousarray(ri_trace, dtype=np.uint32)
    n = min(a.size, b.size)
    return int(_load().or_first_meet(_ptr(a), _ptr(b), n))


def fixup(own_prefix, r0_total, r0_prefix) -> np.ndarray:
    a = np.ascontiguousarray(own_prefix, dtype=np.uint64)
    b = np.ascontiguousarray(r0_total, dtype=np.uint64)
    c = np.ascontiguousarray(r0_prefix, dtype=np.uint64)
    out = np.zeros(a.size, dtype=np.uint64)
    _load().or_fixup(_ptr(a), _ptr(b), _ptr(c), a.size, _ptr(out))
    return out


def pss(t: Table, sym: int) -> np.ndarray:
    out = np.zeros(max(1, t.n_states), dtype=np.uint32)
    k = _load().or_pss(_ptr(t.delta), t.n_states, t.q0, sym, _ptr(out))
    return out[:k]


@dataclass
class KcoexResult:
    cr_init: np.ndarray
    cr_last: np.ndarray
    cr_counts: np.ndarray   # [n_cr, P]
    cr_chunk: np.ndarray
    conv_steps: np.ndarray
    totals: np.ndarray


def kcoex(t: Table, seq: Seq, n_chunks: int, window: int = 0) -> KcoexResult:
    """Algorithm 1 on one CPU thread (chunks, PSS, R0 + fix-up, join)."""
    L = _load()
    P = max(1, t.n_patterns)
    cap = max(1, n_chunks * max(1, t.n_states))
    cr_init = np.zeros(cap, dtype=np.uint32)
    cr_last = np.zeros(cap, dtype=np.uint32)
    cr_counts = np.zeros(cap * P, dtype=np.uint64)
    cr_chunk = np.zeros(cap, dtype=np.uint32)
    conv = np.zeros(cap, dtype=np.int64)
    totals = np.zeros(P, dtype=np.uint64)
    r = int(L.or_kcoex(_ptr(t.delta), t.n_states, t.q0, _ptr(t.out_off), _ptr(t.out_ids), P, _ptr(seq.data),
                       _ptr(seq.nmask), seq.n, seq.enc, n_chunks, window, _ptr(cr_init), _ptr(cr_last),
                       _ptr(cr_counts), _ptr(cr_chunk), _ptr(conv), cap, _ptr(totals)))
    if r < 0:
        raise RuntimeError("kcoex failed (%d)" % r)
    return KcoexResult(cr_init[:r], cr_last[:r], cr_counts[: r * P].reshape(r, P)[:, : t.n_patterns],
                       cr_chunk[:r], conv[:r], totals[: t.n_patterns])
