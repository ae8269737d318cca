"""FASTA ingest (coex_fasta_measure / coex_fasta_read) against a plain Python
reading of the format: records, bases, soft masking, separators, both
encodings, any number of threads.  Runs on the CPU."""
import random

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def coex():
    import paper_1509_01506_amd as m
    return m


def reference(text: bytes, softmask: bool, separate: bool):
    """Records (name, bases) and the output bytes, line by line."""
    recs = []
    cur = None
    for line in text.split(b"\n"):
        if line.startswith(b">"):
            cur = [line[1:].decode("latin-1").strip(), bytearray()]
            recs.append(cur)
            continue
        body = bytes(c for c in line if c not in b" \t\r\v\f")
        if cur is None:
            if not body:
                continue
            cur = ["", bytearray()]
            recs.append(cur)
        cur[1] += body
    if text and not recs:
        recs.append(["", bytearray()])
    out = bytearray()
    starts = []
    for i, (_, b) in enumerate(recs):
        if separate and i:
            out += b"N"
        starts.append(len(out))
        out += bytes(ord("N") if softmask and 97 <= c <= 122 else c for c in b)
    return recs, starts, bytes(out)


def random_fasta(seed: int, n_records: int, mean_len: int) -> bytes:
    rnd = random.Random(seed)
    parts = []
    if rnd.random() < 0.5:  # bases before the first header
        parts.append(b"acgtNNAC\n")
    for r in range(n_records):
        eol = b"\r\n" if rnd.random() < 0.3 else b"\n"
        parts.append(b">rec%d some description%s" % (r, eol))
        n = rnd.randint(0, 2 * mean_len)
        seq = bytearray(synth.markov_bytes(seed * 100 + r, n, with_n=True).tobytes()) if n else bytearray()
        for _ in range(rnd.randint(0, 3)):  # soft-masked runs and IUPAC codes
            if n > 10:
                a = rnd.randrange(n - 5)
                seq[a:a + 5] = seq[a:a + 5].lower()
                seq[rnd.randrange(n)] = ord(rnd.choice("RYKMSWn"))
        width = rnd.choice([60, 61, 70, 80, 1000])
        for i in range(0, len(seq), width):
            parts.append(bytes(seq[i:i + width]) + eol)
            if rnd.random() < 0.02:
                parts.append(eol)  # blank line
    text = b"".join(parts)
    if text and rnd.random() < 0.5:
        text = text.rstrip(b"\r\n")  # no final line break
    return text


CASES = [b"", b">only header", b">a\n>b\n", b"ACGT", b"ACGT\n>x\nGG\n", b">x\nAC GT\tAC\r\nNNn\n>y\n\n>z\nacgt",
         b"\n\n>x\nA\n", b">x\nACGT\n>>y\nA>C\n"]


@pytest.mark.parametrize("enc", [0, 1])
def test_fasta_cases_and_random(coex, enc):
    texts = CASES + [random_fasta(s, 1 + s % 7, 3000) for s in range(12)]
    for text in texts:
        for soft in (False, True):
            for sep in (False, True):
                recs, starts, out = reference(text, soft, sep)
                data, mask, n, got = coex.read_fasta(text, encoding=enc, softmask=soft, separate=sep)
                assert n == len(out), (text[:40], soft, sep)
                assert [r.name for r in got] == [r[0] for r in recs]
                assert [r.start for r in got] == starts
                assert [r.length for r in got] == [len(r[1]) for r in recs]
                if enc == 0:
                    assert data[:n].tobytes() == out
                else:
                    arr = np.frombuffer(out, np.uint8)
                    codes, m = synth.bytes_to_2bit(arr) if n else (np.zeros(1, np.uint8), np.zeros(1, np.uint8))
                    assert data[: (n + 3) // 4].tolist() == codes[: (n + 3) // 4].tolist()
                    assert mask[: (n + 7) // 8].tolist() == m[: (n + 7) // 8].tolist()


def test_fasta_threads_and_pieces(coex):
    # a text of several MiB: several pieces, output bytes shared at their edges
    text = random_fasta(99, 40, 150_000)
    assert len(text) > 4 << 20
    for soft, sep in [(False, False), (True, True)]:
        recs, starts, out = reference(text, soft, sep)
        arr = np.frombuffer(out, np.uint8)
        codes, m = synth.bytes_to_2bit(arr)
        for threads in (1, 3, 8, 16):
            data, _, n, got = coex.read_fasta(text, encoding=coex.ENC_BYTE, softmask=soft, separate=sep,
                                              threads=threads)
            assert data[:n].tobytes() == out
            assert [r.start for r in got] == starts
            data, mask, n, got = coex.read_fasta(text, encoding=coex.ENC_2BIT, softmask=soft, separate=sep,
                                                 threads=threads)
            assert np.array_equal(data[: (n + 3) // 4], codes[: (n + 3) // 4])
            assert np.array_equal(mask[: (n + 7) // 8], m[: (n + 7) // 8])


def test_fasta_errors(coex):
    import ctypes
    L = coex._lib()
    nr, nb = ctypes.c_uint64(0), ctypes.c_uint64(0)
    text = b">a\nACGT\n>b\nAC\n"
    buf = np.zeros(16, np.uint8)
    rs = np.zeros(1, np.uint64)
    # one record slot for two records
    assert L.coex_fasta_read(text, len(text), 0, 0, 0, buf.ctypes.data, None, 16, rs.ctypes.data, None, None, 1,
                             ctypes.byref(nr), ctypes.byref(nb)) == -5
    assert (nr.value, nb.value) == (2, 6)
    # three bases of room for six
    assert L.coex_fasta_read(text, len(text), 0, 0, 0, buf.ctypes.data, None, 3, None, None, None, 0,
                             ctypes.byref(nr), ctypes.byref(nb)) == -5
    assert L.coex_fasta_read(text, len(text), 0, 8, 0, buf.ctypes.data, None, 16, None, None, None, 0,
                             ctypes.byref(nr), ctypes.byref(nb)) == -1
    assert L.coex_fasta_read(text, len(text), 5, 0, 0, buf.ctypes.data, None, 16, None, None, None, 0,
                             ctypes.byref(nr), ctypes.byref(nb)) == -1
