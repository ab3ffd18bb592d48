"""CPU oracle for canonical-Huffman coding of quantization codes (uint16
symbols, and uint8 / uint32 symbols through the width-generic routines).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything in this directory, and this directory uses nothing
from the product library.

The arithmetic lives in ``hdref.c`` (plain C, one obvious loop per
definition); this module compiles it with gcc and wraps it with ctypes over
numpy arrays.  See ``hdref.c`` for the passage each routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hdref.c")
_LIB = os.path.join(_HERE, "libhdref.so")

OK, EARG, EINFEASIBLE, ESYMBOL, ECORRUPT, ENOMEM = 0, -1, -2, -3, -4, -5


def build(force: bool = True) -> str:
    """Compile hdref.c into libhdref.so (gcc -O2, plain C11)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        p = C.c_void_p
        u32, u64 = C.c_uint32, C.c_uint64
        L.hdref_histogram.argtypes = [p, u64, u32, p]
        L.hdref_histogram_w.argtypes = [p, u32, u64, u32, p]
        L.hdref_encode_w.argtypes = [p, u32, u64, p, p, u32, u32, u32, p, u64, p, u64, p, u64, p]
        L.hdref_decode_w.argtypes = [p, u64, u64, u64, p, p, u32, p, u32]
        L.hdref_decode_from_w.argtypes = [p, u64, u64, u64, u64, p, p, u32, p, u32, p]
        L.hdref_code_lengths.argtypes = [p, u32, u32, p]
        L.hdref_canonical_codes.argtypes = [p, u32, p]
        L.hdref_encode.argtypes = [p, u64, p, p, u32, u32, u32, p, u64, p, u64, p, u64, p]
        L.hdref_decode.argtypes = [p, u64, u64, u64, p, p, u32, p]
        L.hdref_decode_prefix.argtypes = [p, u64, u64, u64, p, p, u32, p, p]
        L.hdref_decode_from.argtypes = [p, u64, u64, u64, u64, p, p, u32, p, p]
        L.hdref_selfsync.argtypes = [p, u64, u64, u64, p, p, u32, u32, p, p, p]
        L.hdref_gap_backward.argtypes = [p, u64, u64, u64, p, p, u32, u32, p, p]
        for f in ("hdref_histogram", "hdref_code_lengths", "hdref_canonical_codes", "hdref_encode",
                  "hdref_decode", "hdref_decode_prefix", "hdref_selfsync", "hdref_gap_backward",
                  "hdref_histogram_w", "hdref_encode_w", "hdref_decode_w", "hdref_decode_from_w"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"{what}: oracle status {rc}")
        self.rc = rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


_WIDTH_DTYPE = {1: np.uint8, 2: np.uint16, 4: np.uint32}


def _symbols(x: np.ndarray):
    """(contiguous symbol array, width in bytes): uint8 and uint32 arrays keep
    their width, anything else is taken as uint16."""
    x = np.asarray(x)
    if x.dtype == np.uint8:
        return np.ascontiguousarray(x), 1
    if x.dtype == np.uint32:
        return np.ascontiguousarray(x), 4
    return np.ascontiguousarray(x, dtype=np.uint16), 2


def histogram(x: np.ndarray, A: int) -> np.ndarray:
    x, w = _symbols(x)
    cnt = np.zeros(A, dtype=np.uint64)
    _check(lib().hdref_histogram_w(_ptr(x), w, x.size, A, _ptr(cnt)), "histogram")
    return cnt


def code_lengths(cnt: np.ndarray, L: int) -> np.ndarray:
    cnt = np.ascontiguousarray(cnt, dtype=np.uint64)
    ln = np.zeros(cnt.size, dtype=np.uint8)
    _check(lib().hdref_code_lengths(_ptr(cnt), cnt.size, L, _ptr(ln)), "code_lengths")
    return ln


def canonical_codes(lengths: np.ndarray) -> np.ndarray:
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    code = np.zeros(lengths.size, dtype=np.uint32)
    _check(lib().hdref_canonical_codes(_ptr(lengths), lengths.size, _ptr(code)), "canonical_codes")
    return code


@dataclass
class Encoded:
    words: np.ndarray          # uint32[n_words], MSB-first, zero tail and 2 guard units
    gap: np.ndarray            # uint8[K], forward gap in bits
    chunk_counts: np.ndarray   # uint32[M]
    n_symbols: int
    n_bits: int
    S: int
    C: int

    @property
    def n_subseq(self):
        return self.gap.size

    @property
    def n_chunks(self):
        return self.chunk_counts.size

    @property
    def chunk_offsets(self) -> np.ndarray:
        """uint64[M + 1]: the output index of each chunk's first codeword (the
        exclusive prefix sum of the chunk counts, Sec. III-B step 3), then n."""
        off = np.zeros(self.chunk_counts.size + 1, dtype=np.uint64)
        np.cumsum(self.chunk_counts, dtype=np.uint64, out=off[1:])
        return off


def encode(x: np.ndarray, lengths: np.ndarray, codes: np.ndarray, S: int = 128, C: int = 32) -> Encoded:
    """Encodes x (uint8 / uint32 arrays at their width, anything else as uint16)."""
    x, wid = _symbols(x)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    A = lengths.size
    info = np.zeros(4, dtype=np.uint64)
    L = lib()
    _check(L.hdref_encode_w(_ptr(x), wid, x.size, _ptr(lengths), _ptr(codes), A, S, C,
                            None, 0, None, 0, None, 0, _ptr(info)), "encode(size)")
    B, NW, K, M = (int(v) for v in info)
    words = np.zeros(NW, dtype=np.uint32)
    gap = np.zeros(K, dtype=np.uint8)
    cc = np.zeros(M, dtype=np.uint32)
    _check(L.hdref_encode_w(_ptr(x), wid, x.size, _ptr(lengths), _ptr(codes), A, S, C,
                            _ptr(words), NW, _ptr(gap), K, _ptr(cc), M, _ptr(info)), "encode")
    return Encoded(words, gap, cc, x.size, B, S, C)


def decode(words: np.ndarray, n_bits: int, n: int, lengths: np.ndarray, codes: np.ndarray,
           width: int = 2) -> np.ndarray:
    """Bit-serial decode of n symbols into an unsigned array of `width` bytes (1, 2 or 4)."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    out = np.zeros(n, dtype=_WIDTH_DTYPE[width])
    _check(lib().hdref_decode_w(_ptr(words), words.size, n_bits, n, _ptr(lengths), _ptr(codes),
                                lengths.size, _ptr(out), width), "decode")
    return out


def decode_prefix(words, n_bits, n, lengths, codes, out=None):
    """Decodes the first n symbols (no end check); returns (symbols, end bit)."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    if out is None:
        out = np.zeros(n, dtype=np.uint16)
    end = np.zeros(1, dtype=np.uint64)
    _check(lib().hdref_decode_prefix(_ptr(words), words.size, n_bits, n, _ptr(lengths), _ptr(codes),
                                     lengths.size, _ptr(out), _ptr(end)), "decode_prefix")
    return out, int(end[0])


def decode_from(words, n_bits, start, n, lengths, codes, out=None, width: int = 2):
    """Decodes n symbols from codeword start `start` (no end check) into an
    unsigned array of `width` bytes; returns (symbols, end bit)."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    if out is None:
        out = np.zeros(n, dtype=_WIDTH_DTYPE[width])
    assert out.dtype == _WIDTH_DTYPE[width] and out.flags.c_contiguous and out.size >= n
    end = np.zeros(1, dtype=np.uint64)
    _check(lib().hdref_decode_from_w(_ptr(words), words.size, n_bits, start, n, _ptr(lengths), _ptr(codes),
                                     lengths.size, _ptr(out), width, _ptr(end)), "decode_from")
    return out, int(end[0])


def decode_chunks_parallel(words, n_bits, n, lengths, codes, gap, chunk_offsets, S, C, threads, width: int = 2):
    """The bit-serial decoder run on `threads` host threads, one contiguous
    range of chunks each, every range starting at its first subsequence's gap
    entry and writing from its first chunk's offset (chunk_offsets: uint64[M + 1]).
    Returns the decoded symbols."""
    from concurrent.futures import ThreadPoolExecutor
    words = np.ascontiguousarray(words, dtype=np.uint32)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    out = np.zeros(n, dtype=_WIDTH_DTYPE[width])
    M = int(chunk_offsets.size) - 1
    off = np.ascontiguousarray(chunk_offsets, dtype=np.uint64)
    bounds = [M * i // threads for i in range(threads + 1)]

    def run(i):
        c0, c1 = bounds[i], bounds[i + 1]
        if c0 >= c1:
            return
        k0 = c0 * C
        start = k0 * S + int(gap[k0])
        o0, o1 = int(off[c0]), int(off[c1])
        decode_from(words, n_bits, start, o1 - o0, lengths, codes, out[o0:o1], width)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(threads)))
    return out


def selfsync(words, n_bits, n, lengths, codes, S):
    """(sync_gap uint8[K], counts uint32[K], sync_bits uint32[K]) -- see hdref.c."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    K = (n_bits + S - 1) // S
    g = np.zeros(K, dtype=np.uint8)
    c = np.zeros(K, dtype=np.uint32)
    b = np.zeros(K, dtype=np.uint32)
    _check(lib().hdref_selfsync(_ptr(words), words.size, n_bits, n, _ptr(lengths), _ptr(codes),
                                lengths.size, S, _ptr(g), _ptr(c), _ptr(b)), "selfsync")
    return g, c, b


def gap_backward(words, n_bits, n, lengths, codes, S):
    words = np.ascontiguousarray(words, dtype=np.uint32)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    K = (n_bits + S - 1) // S
    g = np.zeros(K, dtype=np.int32)
    c = np.zeros(K, dtype=np.uint32)
    _check(lib().hdref_gap_backward(_ptr(words), words.size, n_bits, n, _ptr(lengths), _ptr(codes),
                                    lengths.size, S, _ptr(g), _ptr(c)), "gap_backward")
    return g, c


def build_codebook(x: np.ndarray, A: int, L: int):
    """histogram -> package-merge lengths -> canonical codes."""
    ln = code_lengths(histogram(x, A), L)
    return ln, canonical_codes(ln)
