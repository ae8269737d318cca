"""Python binding of libcoex (include/coex.h): the chunked speculative
finite-automaton scan of DNA sequences on MI355X.

Argument marshalling only: every step of the scan runs in the HIP kernels of
``libcoex.so``.  PyTorch supplies device memory and streams.  If the shared
library is missing, importing this package raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("COEX_LIBRARY") or os.path.join(_HERE, "libcoex.so")

ENC_BYTE = 0
ENC_2BIT = 1
FLAG_CHECK = 1
FLAG_TIME = 2
FLAG_GRAPH = 4

STATUS = {0: "OK", -1: "EINVAL", -2: "EALPHABET", -3: "ETOOBIG", -4: "ENOMEM", -5: "ECAPACITY",
          -6: "EDEVICE", -7: "EUNSUPPORTED", -8: "ESYNTAX", -9: "EINTERNAL", -10: "ESCRATCH",
          -11: "ENOTRESIDENT"}

EXPORTED = ["coex_compile_kmers", "coex_compile_regex", "coex_dfa_from_table", "coex_dfa_info",
            "coex_dfa_export", "coex_dfa_free", "coex_count", "coex_count_noalloc", "coex_find",
            "coex_count_chunks", "coex_count_host", "coex_errors_async", "coex_count_find", "coex_fasta_measure", "coex_fasta_read",
            "coex_partition_kmers", "coex_partition_info", "coex_partition_part", "coex_count_partitioned",
            "coex_partition_free",
            "coex_count_batched", "coex_dfa_set_create", "coex_dfa_set_free", "coex_batch_create",
            "coex_batch_update", "coex_batch_run", "coex_batch_tune", "coex_batch_info", "coex_batch_free",
            "coex_server_create", "coex_server_submit", "coex_server_wait", "coex_server_stats", "coex_server_free",
            "coex_profile", "coex_strerror", "coex_version"]


class CoexError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s%s (%s)" % (what + ": " if what else "", _lib().coex_strerror(status).decode(),
                                        self.name))


class _Seq(ctypes.Structure):
    _fields_ = [("bases", ctypes.c_void_p), ("n_mask", ctypes.c_void_p), ("n_bases", ctypes.c_uint64),
                ("encoding", ctypes.c_int32), ("first_base", ctypes.c_uint64)]


class _Opts(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint32), ("width", ctypes.c_uint32), ("lookback", ctypes.c_uint32),
                ("step", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("chains", ctypes.c_uint32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_uint32), ("n_patterns", ctypes.c_uint32), ("n_accepting", ctypes.c_uint32),
                ("q0", ctypes.c_uint32), ("sync_depth", ctypes.c_uint32), ("max_out", ctypes.c_uint32),
                ("max_pss", ctypes.c_uint32 * 9)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint64), ("width", ctypes.c_uint32), ("step", ctypes.c_uint32),
                ("n_groups", ctypes.c_uint32), ("n_pairs", ctypes.c_uint32), ("n_tasks", ctypes.c_uint32),
                ("blocks", ctypes.c_uint32), ("n_lanes", ctypes.c_uint64), ("last_ms", ctypes.c_double)]


_L = None
_VOID = ("coex_dfa_free", "coex_partition_free", "coex_strerror", "coex_version", "coex_dfa_set_free", "coex_batch_free",
         "coex_server_free")


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_batch", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("width", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("copy_piece", ctypes.c_uint64)]


class _ReqStats(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("h2d_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("launch_to_done_ms", ctypes.c_double),
                ("batch_size", ctypes.c_uint32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("n_submitted", ctypes.c_uint64), ("n_done", ctypes.c_uint64), ("n_batches", ctypes.c_uint64),
                ("bases_done", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("max_arena_bytes", ctypes.c_uint64), ("device_ms", ctypes.c_double)]


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcoex.so is not built (run __graft_entry__.build() or "
                              "python paper_1509_01506_amd/build.py)")
        # torch first: the HIP runtime it loads is then the one libcoex.so
        # binds to (the same soname), so the device memory and streams torch
        # hands over belong to the library's runtime too; loading libcoex.so
        # first would bring in a second HIP runtime beside torch's
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        p, u32, u64, ci = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.coex_compile_kmers.argtypes = [p, u32, p]
        L.coex_compile_regex.argtypes = [ctypes.c_char_p, p]
        L.coex_dfa_from_table.argtypes = [p, u32, u32, p, p, u32, p]
        L.coex_dfa_info.argtypes = [p, p]
        L.coex_dfa_export.argtypes = [p, p, p, p]
        L.coex_dfa_free.argtypes = [p]
        L.coex_dfa_free.restype = None
        L.coex_count.argtypes = [p, p, p, p, p]
        L.coex_count_noalloc.argtypes = [p, p, p, p, p]
        L.coex_errors_async.argtypes = [p, p]
        L.coex_count_find.argtypes = [p, p, p, p, p, u64, p, p, p]
        L.coex_fasta_measure.argtypes = [p, u64, u32, u32, p, p]
        L.coex_partition_kmers.argtypes = [p, u32, u32, p]
        L.coex_partition_info.argtypes = [p, p, p]
        L.coex_partition_part.argtypes = [p, u32, p, p, p]
        L.coex_count_partitioned.argtypes = [p, p, p, p, p]
        L.coex_partition_free.argtypes = [p]
        L.coex_partition_free.restype = None
        L.coex_fasta_read.argtypes = [p, u64, ctypes.c_int32, u32, u32, p, p, u64, p, p, p, u64, p, p]
        L.coex_count_host.argtypes = [p, p, p, u64, ctypes.c_int32, u32, u64, u64, p]
        L.coex_find.argtypes = [p, p, p, p, u64, p, p, p]
        L.coex_count_chunks.argtypes = [p, p, u32, p, p, p, p]
        L.coex_count_batched.argtypes = [p, u32, p, u32, p, p, p]
        L.coex_dfa_set_create.argtypes = [p, u32, p, p]
        L.coex_dfa_set_free.argtypes = [p]
        L.coex_dfa_set_free.restype = None
        L.coex_batch_create.argtypes = [p, p, u32, p, p, u32, p, p]
        L.coex_batch_update.argtypes = [p, p, u32, p, p, u32]
        L.coex_batch_run.argtypes = [p, p, p]
        L.coex_server_create.argtypes = [p, u32, p, p]
        L.coex_server_submit.argtypes = [p, p, u64, u32, p]
        L.coex_server_wait.argtypes = [p, u64, p, p]
        L.coex_server_stats.argtypes = [p, p]
        L.coex_server_free.argtypes = [p]
        L.coex_server_free.restype = None
        L.coex_batch_tune.argtypes = [p, p, p, p, p]
        L.coex_batch_info.argtypes = [p, p]
        L.coex_batch_free.argtypes = [p]
        L.coex_batch_free.restype = None
        L.coex_profile.argtypes = [p, p, p, ci]
        L.coex_strerror.argtypes = [ci]
        L.coex_strerror.restype = ctypes.c_char_p
        L.coex_version.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in _VOID:
                getattr(L, name).restype = ci
        _L = L
    return _L


_lib()  # fail loudly at import when the native library is absent


def _check(rc: int, what: str):
    if rc != 0:
        raise CoexError(rc, what)


# ------------------------------------------------------------------ automata
@dataclass
class Info:
    n_states: int
    n_patterns: int
    n_accepting: int
    q0: int
    sync_depth: Optional[int]
    max_out: int
    max_pss: list


class Dfa:
    """A compiled automaton (library handle)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    @staticmethod
    def kmers(kmers: Sequence[str]) -> "Dfa":
        """Aho-Corasick automaton; pattern id = index."""
        enc = [k.encode("ascii") for k in kmers]
        arr = (ctypes.c_char_p * max(1, len(enc)))(*enc)
        out = ctypes.c_void_p()
        _check(_lib().coex_compile_kmers(ctypes.cast(arr, ctypes.c_void_p), len(enc), ctypes.byref(out)),
               "compile_kmers")
        return Dfa(out.value)

    @staticmethod
    def regex(text: str) -> "Dfa":
        out = ctypes.c_void_p()
        _check(_lib().coex_compile_regex(text.encode("ascii"), ctypes.byref(out)), "compile_regex")
        return Dfa(out.value)

    @staticmethod
    def table(delta, q0: int, out_offsets, out_ids, n_patterns: int) -> "Dfa":
        d = np.ascontiguousarray(delta, dtype=np.uint32)
        o = np.ascontiguousarray(out_offsets, dtype=np.uint32)
        i = np.ascontiguousarray(out_ids, dtype=np.uint32)
        if i.size == 0:
            i = np.zeros(1, dtype=np.uint32)
        out = ctypes.c_void_p()
        _check(_lib().coex_dfa_from_table(d.ctypes.data, d.size // 4, int(q0), o.ctypes.data, i.ctypes.data,
                                          int(n_patterns), ctypes.byref(out)), "dfa_from_table")
        return Dfa(out.value)

    def info(self) -> Info:
        x = _Info()
        _check(_lib().coex_dfa_info(self._h, ctypes.byref(x)), "dfa_info")
        return Info(x.n_states, x.n_patterns, x.n_accepting, x.q0,
                    None if x.sync_depth == 0xFFFFFFFF else x.sync_depth, x.max_out, list(x.max_pss))

    def export(self):
        """(delta uint32[n*4], q0, out_offsets uint32[n+1], out_ids uint32[...])."""
        inf = self.info()
        d = np.zeros(inf.n_states * 4, dtype=np.uint32)
        o = np.zeros(inf.n_states + 1, dtype=np.uint32)
        _check(_lib().coex_dfa_export(self._h, d.ctypes.data, o.ctypes.data, None), "dfa_export")
        i = np.zeros(max(1, int(o[-1])), dtype=np.uint32)
        _check(_lib().coex_dfa_export(self._h, None, None, i.ctypes.data), "dfa_export")
        return d, inf.q0, o, i[: int(o[-1])]

    def free(self):
        if self._h is not None and self._h.value:
            _lib().coex_dfa_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------------ sequences
@dataclass
class DeviceSeq:
    """A sequence in device memory (torch tensors keep the buffers alive)."""
    bases: "object"           # torch.uint8 CUDA tensor
    n: int
    encoding: int = ENC_BYTE
    nmask: "object" = None    # torch.uint8 CUDA tensor or None
    first: int = 0            # bases of the buffers before the sequence's first base
    byte_offset: int = 0      # bytes added to the base pointer (byte encoding: any address)

    def _c(self) -> _Seq:
        return _Seq(self.bases.data_ptr() + self.byte_offset if self.n else 0,
                    self.nmask.data_ptr() if self.nmask is not None else 0, self.n, self.encoding, self.first)

    def sub(self, start: int, n: Optional[int] = None, by_address: bool = False) -> "DeviceSeq":
        """The n bases from `start` of this sequence (to its end by default),
        sharing its buffers: by first_base, or for byte sequences by moving
        the base pointer itself to that byte (any address)."""
        n = self.n - start if n is None else n
        if start < 0 or n < 0 or start + n > self.n:
            raise ValueError("sub-sequence out of range")
        if by_address:
            if self.encoding != ENC_BYTE:
                raise ValueError("by_address needs the byte encoding")
            return DeviceSeq(self.bases, n, self.encoding, self.nmask, self.first, self.byte_offset + start)
        return DeviceSeq(self.bases, n, self.encoding, self.nmask, self.first + start, self.byte_offset)


def _pad16(arr: np.ndarray) -> np.ndarray:
    n = arr.size
    padded = np.zeros(((n + 127) // 128) * 128 or 128, dtype=np.uint8)
    padded[:n] = arr
    return padded


# ------------------------------------------------------------------ pattern partitioning
class Partition:
    """Pattern-based partitioning of a k-mer set (coex_partition_kmers): parts
    of at most `max_states` states each (0 = 1023), every part scanning the
    same sequence; counts per global pattern id."""

    def __init__(self, kmers: Sequence[str], max_states: int = 0):
        enc = [k.encode("ascii") for k in kmers]
        arr = (ctypes.c_char_p * len(enc))(*enc)
        out = ctypes.c_void_p()
        _check(_lib().coex_partition_kmers(ctypes.cast(arr, ctypes.c_void_p), len(enc), max_states,
                                           ctypes.byref(out)), "partition_kmers")
        self._h = out
        n_parts, n_pat = ctypes.c_uint32(0), ctypes.c_uint32(0)
        _check(_lib().coex_partition_info(self._h, ctypes.byref(n_parts), ctypes.byref(n_pat)), "partition_info")
        self.n_parts, self.n_patterns = int(n_parts.value), int(n_pat.value)

    def part(self, i: int):
        """(n_states of part i's automaton, global ids of its patterns)."""
        d, ids, n = ctypes.c_void_p(), ctypes.POINTER(ctypes.c_uint32)(), ctypes.c_uint32(0)
        _check(_lib().coex_partition_part(self._h, i, ctypes.byref(d), ctypes.byref(ids), ctypes.byref(n)),
               "partition_part")
        info = _Info()
        _check(_lib().coex_dfa_info(d, ctypes.byref(info)), "dfa_info")
        return int(info.n_states), [int(ids[j]) for j in range(n.value)]

    def count(self, seq: "DeviceSeq", out=None, check: bool = False, stream=None, **kw):
        import torch
        if out is None:
            out = torch.empty(max(1, self.n_patterns), dtype=torch.int64, device=seq.bases.device)
        s = seq._c()
        o = _opts(check=check, **kw)
        _check(_lib().coex_count_partitioned(self._h, ctypes.byref(s), out.data_ptr(), ctypes.byref(o),
                                             _stream(stream)), "count_partitioned")
        return out[: self.n_patterns]

    def free(self):
        if self._h is not None and self._h.value:
            _lib().coex_partition_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------------ FASTA
FASTA_SOFTMASK = 1
FASTA_SEPARATE = 2


@dataclass
class FastaRecord:
    name: str     # header line without '>' ("" for bases before the first header)
    start: int    # first base in the parsed output
    length: int


def read_fasta(text: bytes, encoding: int = ENC_2BIT, softmask: bool = False, separate: bool = False,
               threads: int = 0):
    """Parses FASTA text on the host (coex_fasta_read): returns (bases, mask,
    n, records); bases are bytes or packed 2-bit codes with `mask` the N bits
    (None for bytes)."""
    text = bytes(text)
    flags = (FASTA_SOFTMASK if softmask else 0) | (FASTA_SEPARATE if separate else 0)
    nr, nb = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(_lib().coex_fasta_measure(text, len(text), flags, threads, ctypes.byref(nr), ctypes.byref(nb)),
           "fasta_measure")
    n, R = int(nb.value), int(nr.value)
    if encoding == ENC_BYTE:
        data, mask = np.zeros(max(1, n), np.uint8), None
    else:
        data, mask = np.zeros(max(1, (n + 3) // 4), np.uint8), np.zeros(max(1, (n + 7) // 8), np.uint8)
    start, length, head = (np.zeros(max(1, R), np.uint64) for _ in range(3))
    _check(_lib().coex_fasta_read(text, len(text), encoding, flags, threads, data.ctypes.data,
                                  None if mask is None else mask.ctypes.data, n, start.ctypes.data,
                                  length.ctypes.data, head.ctypes.data, R, ctypes.byref(nr), ctypes.byref(nb)),
           "fasta_read")
    recs = []
    for r in range(R):
        h = int(head[r])
        if h == (1 << 64) - 1:
            name = ""
        else:
            e = text.find(b"\n", h)
            name = text[h + 1: e if e >= 0 else len(text)].decode("latin-1").strip()
        recs.append(FastaRecord(name, int(start[r]), int(length[r])))
    return data, mask, n, recs


def fasta_to_device(text: bytes, encoding: int = ENC_2BIT, softmask: bool = False, separate: bool = False,
                    threads: int = 0, device: str = "cuda"):
    """read_fasta, then the bases to the device: (DeviceSeq of the whole
    output, records); record r alone is seq.sub(rec.start, rec.length)."""
    data, mask, n, recs = read_fasta(text, encoding, softmask, separate, threads)
    return to_device(data, n=n, encoding=encoding, nmask=mask, device=device), recs


def to_device(data: np.ndarray, n: Optional[int] = None, encoding: int = ENC_BYTE,
              nmask: Optional[np.ndarray] = None, device: str = "cuda") -> DeviceSeq:
    """Copies a host sequence to the GPU (buffers padded to 128 bytes)."""
    import torch
    data = np.ascontiguousarray(data, dtype=np.uint8)
    if n is None:
        n = data.size if encoding == ENC_BYTE else data.size * 4
    b = torch.from_numpy(_pad16(data)).to(device)
    m = torch.from_numpy(_pad16(np.ascontiguousarray(nmask, dtype=np.uint8))).to(device) if nmask is not None \
        else None
    return DeviceSeq(b, int(n), encoding, m)


def _opts(chunk=0, width=0, lookback=0, step=0, check=False, timed=False, graph=False, chains=0) -> _Opts:
    return _Opts(chunk, width, lookback, step,
                 (FLAG_CHECK if check else 0) | (FLAG_TIME if timed else 0) | (FLAG_GRAPH if graph else 0), chains)


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)


# ------------------------------------------------------------------ scans
def count(dfa: Dfa, seq: DeviceSeq, out=None, chunk: int = 0, width: int = 0, lookback: int = 0, step: int = 0,
          check: bool = False, timed: bool = False, stream=None, chains: int = 0):
    """Per-pattern match counts as an int64 CUDA tensor (the device buffer holds uint64)."""
    import torch
    P = dfa.info().n_patterns
    if out is None:
        out = torch.empty(max(1, P), dtype=torch.int64, device=seq.bases.device)
    if out.numel() < P or out.dtype != torch.int64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int64 tensor of at least %d elements" % P)
    s = seq._c()
    o = _opts(chunk, width, lookback, step, check, timed, chains=chains)
    _check(_lib().coex_count(dfa.handle, ctypes.byref(s), out.data_ptr(), ctypes.byref(o), _stream(stream)),
           "count")
    return out[:P]


def count_noalloc(dfa: Dfa, seq: DeviceSeq, out, chunk: int = 0, width: int = 0, lookback: int = 0,
                  step: int = 0, check: bool = False, stream=None, chains: int = 0):
    """count() through coex_count_noalloc: the library allocates nothing (its
    scratch is a static device array); `out` is the caller's int64 tensor."""
    P = dfa.info().n_patterns
    if out.numel() < P or str(out.dtype) != "torch.int64" or not out.is_contiguous():
        raise ValueError("out must be a contiguous int64 tensor of at least %d elements" % P)
    s = seq._c()
    o = _opts(chunk, width, lookback, step, check, chains=chains)
    _check(_lib().coex_count_noalloc(dfa.handle, ctypes.byref(s), out.data_ptr(), ctypes.byref(o),
                                     _stream(stream)), "count_noalloc")
    return out[:P]


def find(dfa: Dfa, seq: DeviceSeq, capacity: Optional[int] = None, chunk: int = 0, width: int = 0,
         lookback: int = 0, step: int = 0, stream=None, chains: int = 0):
    """(end positions int64, pattern ids int32) CUDA tensors, ascending."""
    import torch
    dev = seq.bases.device
    s = seq._c()
    o = _opts(chunk, width, lookback, step, chains=chains)
    n_found = ctypes.c_uint64(0)
    if capacity is None:
        # a first guess that holds most results, so the scan usually runs once
        # (the second call below reruns it with the exact size)
        cap = min(int(seq.n) * max(1, dfa.info().max_out), 1 << 20)
    else:
        cap = int(capacity)
    pos = torch.empty(max(1, cap), dtype=torch.int64, device=dev)
    pat = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    rc = _lib().coex_find(dfa.handle, ctypes.byref(s), pos.data_ptr(), pat.data_ptr(), cap, ctypes.byref(n_found),
                          ctypes.byref(o), _stream(stream))
    if rc == -5 and capacity is None:
        cap = int(n_found.value)
        pos = torch.empty(max(1, cap), dtype=torch.int64, device=dev)
        pat = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
        rc = _lib().coex_find(dfa.handle, ctypes.byref(s), pos.data_ptr(), pat.data_ptr(), cap,
                              ctypes.byref(n_found), ctypes.byref(o), _stream(stream))
    _check(rc, "find")
    m = int(n_found.value)
    return pos[:m], pat[:m]


def count_find(dfa: Dfa, seq: DeviceSeq, out=None, capacity: Optional[int] = None, chunk: int = 0, width: int = 0,
               lookback: int = 0, step: int = 0, timed: bool = False, stream=None, chains: int = 0):
    """Counts and end positions from one scan (coex_count_find): (per-pattern
    counts int64, end positions int64, pattern ids int32) CUDA tensors."""
    import torch
    dev = seq.bases.device
    P = dfa.info().n_patterns
    if out is None:
        out = torch.empty(max(1, P), dtype=torch.int64, device=dev)
    s = seq._c()
    o = _opts(chunk, width, lookback, step, timed=timed, chains=chains)
    n_found = ctypes.c_uint64(0)
    cap = min(int(seq.n) * max(1, dfa.info().max_out), 1 << 20) if capacity is None else int(capacity)
    for attempt in range(2):
        pos = torch.empty(max(1, cap), dtype=torch.int64, device=dev)
        pat = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
        rc = _lib().coex_count_find(dfa.handle, ctypes.byref(s), out.data_ptr(), pos.data_ptr(), pat.data_ptr(), cap,
                                    ctypes.byref(n_found), ctypes.byref(o), _stream(stream))
        if rc == -5 and capacity is None and attempt == 0:
            cap = int(n_found.value)
            continue
        break
    _check(rc, "count_find")
    m = int(n_found.value)
    return out[:P], pos[:m], pat[:m]


def count_host(dfa: Dfa, data: np.ndarray, n: Optional[int] = None, encoding: int = ENC_BYTE,
               nmask: Optional[np.ndarray] = None, threads: int = 0, chunks: int = 0, window: int = 0) -> np.ndarray:
    """The paper's method on host threads (coex_count_host): per-pattern
    counts (uint64 numpy array) of a host sequence."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    if n is None:
        n = data.size if encoding == ENC_BYTE else data.size * 4
    m = np.ascontiguousarray(nmask, dtype=np.uint8) if nmask is not None else None
    out = np.zeros(max(1, dfa.info().n_patterns), dtype=np.uint64)
    _check(_lib().coex_count_host(dfa.handle, data.ctypes.data if data.size else None,
                                  m.ctypes.data if m is not None else None, int(n), int(encoding), int(threads),
                                  int(chunks), int(window), out.ctypes.data), "count_host")
    return out[:dfa.info().n_patterns]


def errors_async(out, stream=None):
    """Enqueues on the stream the read-and-clear of the device consistency
    failures kept since the last read (0 = every check passed): `out` is an
    int32 tensor (device, or pinned host memory) whose first element receives
    them once the stream gets there."""
    _check(_lib().coex_errors_async(_stream(stream), out.data_ptr()), "errors_async")
    return out


def errors(stream=None) -> int:
    """errors_async into pinned host memory, then a wait for the stream."""
    import torch
    out = torch.zeros(1, dtype=torch.int32, pin_memory=True)
    errors_async(out, stream)
    if stream is None or isinstance(stream, int):
        torch.cuda.synchronize()
    else:
        stream.synchronize()
    return int(out[0])


def count_chunks(dfa: Dfa, seq: DeviceSeq, chunk: int, stream=None):
    """Per-chunk records (init state, last state, counts[P]) for the true start states."""
    import torch
    dev = seq.bases.device
    inf = dfa.info()
    nc = max(1, (seq.n + chunk - 1) // chunk)
    init = torch.empty(nc, dtype=torch.int32, device=dev)
    last = torch.empty(nc, dtype=torch.int32, device=dev)
    cnt = torch.empty(nc * max(1, inf.n_patterns), dtype=torch.int64, device=dev)
    s = seq._c()
    _check(_lib().coex_count_chunks(dfa.handle, ctypes.byref(s), int(chunk), init.data_ptr(), last.data_ptr(),
                                    cnt.data_ptr(), _stream(stream)), "count_chunks")
    return init, last, cnt[: nc * inf.n_patterns].view(nc, inf.n_patterns)


def count_batched(dfas: Sequence[Dfa], seqs: Sequence[DeviceSeq], out=None, chunk: int = 0, width: int = 0,
                  lookback: int = 0, step: int = 0, stream=None):
    """counts[s, d] = total matches of dfas[d] in seqs[s] (int64 CUDA tensor)."""
    import torch
    dev = seqs[0].bases.device
    hs = (ctypes.c_void_p * len(dfas))(*[d.handle.value for d in dfas])
    ss = (_Seq * len(seqs))(*[s._c() for s in seqs])
    if out is None:
        out = torch.empty((len(seqs), len(dfas)), dtype=torch.int64, device=dev)
    if out.numel() < len(seqs) * len(dfas) or out.dtype != torch.int64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int64 tensor of n_seq * n_dfa elements")
    o = _opts(chunk, width, lookback, step)
    _check(_lib().coex_count_batched(ctypes.cast(hs, ctypes.c_void_p), len(dfas), ctypes.cast(ss, ctypes.c_void_p),
                                     len(seqs), out.data_ptr(), ctypes.byref(o), _stream(stream)),
           "count_batched")
    return out


class DfaSet:
    """Resident automata packed into LDS groups (coex_dfa_set)."""

    def __init__(self, dfas: Sequence[Dfa], width: int = 0, step: int = 0):
        self.dfas = list(dfas)
        hs = (ctypes.c_void_p * len(self.dfas))(*[d.handle.value for d in self.dfas])
        o = _opts(width=width, step=step)
        out = ctypes.c_void_p()
        _check(_lib().coex_dfa_set_create(ctypes.cast(hs, ctypes.c_void_p), len(self.dfas), ctypes.byref(o),
                                          ctypes.byref(out)), "dfa_set_create")
        self._h = out

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h is not None and self._h.value:
            _lib().coex_dfa_set_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


@dataclass
class BatchInfo:
    chunk: int
    width: int
    step: int
    n_groups: int
    n_pairs: int
    n_tasks: int
    blocks: int
    n_lanes: int
    last_ms: float


class Batch:
    """(sequence, automaton) pairs over a DfaSet, run in one persistent launch
    (coex_batch).  pairs=None: every sequence with every automaton, result
    shaped [n_seq, n_dfa]; else a list of (seq index, dfa index), result [n]."""

    def __init__(self, dset: DfaSet, seqs: Sequence[DeviceSeq], pairs=None, chunk: int = 0, check: bool = False,
                 timed: bool = False, graph: bool = False, width: int = 0):
        self.dset = dset
        self.seqs = list(seqs)          # keeps the device buffers alive
        ss = (_Seq * max(1, len(self.seqs)))(*[s._c() for s in self.seqs])
        o = _opts(chunk=chunk, width=width, check=check, timed=timed, graph=graph)
        out = ctypes.c_void_p()
        if pairs is None:
            self.shape = (len(self.seqs), len(dset.dfas))
            ps = pd = None
            n = 0
        else:
            arr = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
            ps = np.ascontiguousarray(arr[:, 0])
            pd = np.ascontiguousarray(arr[:, 1])
            n = arr.shape[0]
            self.shape = (n,)
        _check(_lib().coex_batch_create(dset.handle, ctypes.cast(ss, ctypes.c_void_p), len(self.seqs),
                                        None if ps is None else ps.ctypes.data,
                                        None if pd is None else pd.ctypes.data, n, ctypes.byref(o),
                                        ctypes.byref(out)), "batch_create")
        self._h = out
        self.n_pairs = int(np.prod(self.shape))

    def _out(self, out):
        import torch
        if out is None:
            out = torch.empty(max(1, self.n_pairs), dtype=torch.int64, device=self.seqs[0].bases.device)
        return out

    def _checked(self, out):
        if out.numel() < self.n_pairs or out.dtype.itemsize != 8 or not out.is_contiguous():
            raise ValueError("out must be a contiguous 64-bit tensor of at least %d elements" % self.n_pairs)
        return out

    def run(self, out=None, stream=None):
        out = self._checked(self._out(out))
        _check(_lib().coex_batch_run(self._h, out.data_ptr(), _stream(stream)), "batch_run")
        return out[: self.n_pairs].view(self.shape)

    def tune(self, out=None, stream=None):
        """Autotunes chunk length and speculation width cap together; returns
        (chunk, width cap) and keeps them for later runs."""
        out = self._checked(self._out(out))
        c = ctypes.c_uint64(0)
        w = ctypes.c_uint32(0)
        _check(_lib().coex_batch_tune(self._h, out.data_ptr(), _stream(stream), ctypes.byref(c), ctypes.byref(w)),
               "batch_tune")
        return int(c.value), int(w.value)

    def info(self) -> BatchInfo:
        x = _BatchInfo()
        _check(_lib().coex_batch_info(self._h, ctypes.byref(x)), "batch_info")
        return BatchInfo(int(x.chunk), x.width, x.step, x.n_groups, x.n_pairs, x.n_tasks, x.blocks,
                         int(x.n_lanes), x.last_ms)

    def free(self):
        if self._h is not None and self._h.value:
            _lib().coex_batch_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Serving loop over resident automata (coex_server): submit host
    sequences (ASCII bytes; page-locked tensors copy asynchronously) with an
    automaton index, wait for counts and per-request latencies."""

    def __init__(self, dfas: Sequence[Dfa], hbm_budget: int = 0, max_batch: int = 0, chunk: int = 0,
                 width: int = 0, copy_piece: int = 0):
        hs = (ctypes.c_void_p * len(dfas))(*[d.handle.value for d in dfas])
        o = _ServerOpts(int(hbm_budget), int(max_batch), int(chunk), int(width), 0, int(copy_piece))
        out = ctypes.c_void_p()
        _check(_lib().coex_server_create(ctypes.cast(hs, ctypes.c_void_p), len(dfas), ctypes.byref(o),
                                         ctypes.byref(out)), "server_create")
        self._h = out
        self._keep = {}

    def submit(self, data, dfa: int) -> int:
        """data: a CPU torch.uint8 tensor or a numpy uint8 array (kept alive until wait)."""
        if isinstance(data, np.ndarray):
            arr = np.ascontiguousarray(data, dtype=np.uint8)
            ptr, n = arr.ctypes.data, arr.size
        else:
            arr = data.contiguous()
            ptr, n = arr.data_ptr(), arr.numel()
        t = ctypes.c_uint64(0)
        _check(_lib().coex_server_submit(self._h, ptr if n else None, n, int(dfa), ctypes.byref(t)), "server_submit")
        self._keep[t.value] = arr
        return int(t.value)

    def wait(self, ticket: int):
        """(count, stats dict) of a submitted request."""
        c = ctypes.c_uint64(0)
        st = _ReqStats()
        rc = _lib().coex_server_wait(self._h, int(ticket), ctypes.byref(c), ctypes.byref(st))
        self._keep.pop(int(ticket), None)
        _check(rc, "server_wait")
        return int(c.value), {"queue_ms": st.queue_ms, "h2d_ms": st.h2d_ms, "device_ms": st.device_ms,
                              "total_ms": st.total_ms, "launch_to_done_ms": st.launch_to_done_ms,
                              "batch_size": st.batch_size}

    def stats(self) -> dict:
        x = _ServerStats()
        _check(_lib().coex_server_stats(self._h, ctypes.byref(x)), "server_stats")
        return {k: getattr(x, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            _lib().coex_server_free(self._h)
            self._h = ctypes.c_void_p(0)
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile(stream=None, reset: bool = True):
    """(total ms, launches) of the scan kernel over timed calls on `stream`."""
    ms = ctypes.c_double(0.0)
    k = ctypes.c_uint64(0)
    _check(_lib().coex_profile(_stream(stream), ctypes.byref(ms), ctypes.byref(k), int(reset)), "profile")
    return ms.value, int(k.value)


def version() -> str:
    return _lib().coex_version().decode()
