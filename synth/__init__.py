"""Seeded synthetic inputs for the DNA scan (sequences, pattern sets, regexes,
batch shapes, request traces).

Only input generation lives here: nothing in this package matches patterns,
builds automata or counts anything.  The oracle side and the GPU side both
draw their inputs from these functions, so the two always see identical data.

Bulk sequences come from ``gen.c`` (OpenMP, counter-based SplitMix64, see the
header there for the exact recipe); small draws (k-mers, regexes, lengths,
arrival times) use the same counter-based generator written in Python.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def build(force: bool = False) -> str:
    """Compile gen.c into libsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               os.path.join(_HERE, "gen.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        lib.synth_draw.restype = u64
        lib.synth_draw.argtypes = [u64, u64, u64]
        lib.synth_iid_bytes.argtypes = [u64, u64, p]
        lib.synth_markov_bytes.argtypes = [u64, u64, ctypes.c_int, p]
        lib.synth_markov_2bit.argtypes = [u64, u64, ctypes.c_int, p, p]
        lib.synth_bytes_to_2bit.argtypes = [p, u64, p, p]
        lib.synth_n_runs.restype = u64
        lib.synth_n_runs.argtypes = [u64, u64, ctypes.c_double, ctypes.c_double, p, u64]
        _lib = lib
    return _lib


# ---------------------------------------------------------------- generator
def _mix64(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


class Stream:
    """Counter-based SplitMix64 stream: draw i = mix64(key + (i+1)*GAMMA)."""

    def __init__(self, seed: int, tag: int):
        self.key = _mix64(((seed * GAMMA) & M64) ^ tag)
        self.i = 0

    def u64(self) -> int:
        self.i += 1
        return _mix64((self.key + self.i * GAMMA) & M64)

    def uniform(self) -> float:
        return ((self.u64() >> 11) + 0.5) / 9007199254740992.0

    def below(self, n: int) -> int:
        return self.u64() % n

    def normal(self) -> float:
        u1, u2 = self.uniform(), self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def draw(seed: int, tag: int, i: int) -> int:
    """Python twin of gen.c's synth_draw (checked equal in tests)."""
    return _mix64((_mix64(((seed * GAMMA) & M64) ^ tag) + (i + 1) * GAMMA) & M64)


# ---------------------------------------------------------------- sequences
def iid_bytes(seed: int, n: int) -> np.ndarray:
    """n iid uniform bases as ASCII bytes 'A','C','G','T'."""
    out = np.empty(n, dtype=np.uint8)
    if n:
        _load().synth_iid_bytes(seed, n, out.ctypes.data)
    return out


def markov_bytes(seed: int, n: int, with_n: bool = True) -> np.ndarray:
    """First-order Markov bases (GC 0.41) as ASCII, with runs of 'N' (about 1%)."""
    out = np.empty(n, dtype=np.uint8)
    if n:
        _load().synth_markov_bytes(seed, n, int(with_n), out.ctypes.data)
    return out


def markov_2bit(seed: int, n: int, with_n: bool = True):
    """Same source as markov_bytes, stored 2-bit packed plus a 1-bit N mask.

    Returns (packed uint8[ceil(n/4)], mask uint8[ceil(n/8)]); for equal seeds the
    bases equal markov_bytes(seed, n, with_n) position by position."""
    packed = np.empty((n + 3) // 4, dtype=np.uint8)
    mask = np.empty((n + 7) // 8, dtype=np.uint8)
    if n:
        _load().synth_markov_2bit(seed, n, int(with_n), packed.ctypes.data, mask.ctypes.data)
    return packed, mask


def bytes_to_2bit(seq: np.ndarray):
    """Store an ASCII sequence in the 2-bit + N-mask form (non-ACGT -> N)."""
    seq = np.ascontiguousarray(seq, dtype=np.uint8)
    n = seq.size
    packed = np.zeros((n + 3) // 4, dtype=np.uint8)
    mask = np.zeros((n + 7) // 8, dtype=np.uint8)
    if n:
        _load().synth_bytes_to_2bit(seq.ctypes.data, n, packed.ctypes.data, mask.ctypes.data)
    return packed, mask


def n_runs(seed: int, n: int, mean_gap: float = 99000.0, mean_run: float = 1000.0) -> np.ndarray:
    cap = n // 1000 + 1024
    buf = np.zeros((cap, 2), dtype=np.uint64)
    cnt = _load().synth_n_runs(seed, n, mean_gap, mean_run, buf.ctypes.data, cap)
    return buf[: min(cnt, cap)]


def from_text(text: str) -> np.ndarray:
    return np.frombuffer(text.encode("ascii"), dtype=np.uint8).copy()


# ---------------------------------------------------------------- patterns
BASES = "ACGT"


def random_kmers(seed: int, count: int, k: int, distinct: bool = True) -> list[str]:
    """`count` random k-mers over ACGT (distinct unless told otherwise)."""
    st = Stream(seed, 11)
    out, seen = [], set()
    while len(out) < count:
        w = "".join(BASES[st.below(4)] for _ in range(k))
        if distinct and w in seen:
            continue
        seen.add(w)
        out.append(w)
    return out


def random_regex(seed: int, min_atoms: int = 3, max_atoms: int = 8) -> str:
    """Random regex over ACGT: 3-8 atoms, each a base or a class of 2-3 bases,
    some carrying a bounded repeat {m,n} with 2 <= m <= n <= 6."""
    st = Stream(seed, 12)
    n_atoms = min_atoms + st.below(max_atoms - min_atoms + 1)
    parts = []
    for _ in range(n_atoms):
        if st.below(2) == 0:
            atom = BASES[st.below(4)]
        else:
            size = 2 + st.below(2)
            pool = list(BASES)
            chosen = []
            for _ in range(size):
                chosen.append(pool.pop(st.below(len(pool))))
            atom = "[" + "".join(sorted(chosen)) + "]"
        if st.below(5) < 2:
            m = 2 + st.below(5)
            n = m + st.below(7 - m)
            atom += "{%d}" % m if m == n else "{%d,%d}" % (m, n)
        parts.append(atom)
    return "".join(parts)


def random_table(seed: int, n_states: int, n_patterns: int, accept_frac: float = 0.1,
                 max_out: int = 2):
    """Random complete DFA over 4 symbols: delta uint32[n_states*4], q0,
    output sets in CSR form (offsets uint32[n_states+1], ids uint32[...])."""
    st = Stream(seed, 13)
    delta = np.array([st.below(n_states) for _ in range(n_states * 4)], dtype=np.uint32)
    q0 = st.below(n_states)
    offs, ids = [0], []
    for _ in range(n_states):
        if n_patterns and st.uniform() < accept_frac:
            k = 1 + st.below(max_out)
            s = sorted({st.below(n_patterns) for _ in range(k)})
            ids.extend(s)
        offs.append(len(ids))
    return delta, q0, np.array(offs, dtype=np.uint32), np.array(ids, dtype=np.uint32)


# ---------------------------------------------------------------- batch / serve shapes
def lognormal_lengths(seed: int, count: int = 512, sigma: float = 1.5, target_mean: float = 7.8e6,
                      lo: float = 1e4, hi: float = 5e7) -> list[int]:
    """Log-normal lengths clipped to [lo, hi] with mu solved so the clipped mean
    is about target_mean (bisection on the analytic clipped mean)."""
    def clipped_mean(mu):
        # E[clip(X, lo, hi)] for X = exp(mu + sigma Z)
        def Phi(x):
            return 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))
        a = (math.log(lo) - mu) / sigma
        b = (math.log(hi) - mu) / sigma
        mid = math.exp(mu + sigma * sigma / 2) * (Phi(b - sigma) - Phi(a - sigma))
        return lo * Phi(a) + mid + hi * (1.0 - Phi(b))
    l, r = math.log(lo), math.log(hi)
    for _ in range(200):
        m = 0.5 * (l + r)
        if clipped_mean(m) < target_mean:
            l = m
        else:
            r = m
    mu = 0.5 * (l + r)
    st = Stream(seed, 14)
    return [int(min(hi, max(lo, math.exp(mu + sigma * st.normal())))) for _ in range(count)]


def loguniform_ints(seed: int, tag: int, count: int, lo: float, hi: float) -> list[int]:
    st = Stream(seed, tag)
    return [int(round(math.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * st.uniform())))
            for _ in range(count)]


def poisson_arrivals(seed: int, count: int, qps: float) -> list[float]:
    """Arrival times (seconds) of a Poisson process with rate qps."""
    st = Stream(seed, 15)
    t, out = 0.0, []
    for _ in range(count):
        t += -math.log(st.uniform()) / qps
        out.append(t)
    return out


def uniform_ids(seed: int, tag: int, count: int, n: int) -> list[int]:
    st = Stream(seed, tag)
    return [st.below(n) for _ in range(count)]
