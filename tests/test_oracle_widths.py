"""Pins of the oracle's symbol widths (uint8 / uint16 / uint32).

The paper adapts the decoders from single-byte symbols to multi-byte
quantization codes (Sec. IV) and says the method carries over to
double-precision data (Sec. V-A-3).  The bitstream does not depend on the
width, so the 8- and 32-bit paths are pinned by reduction to the 16-bit path
(itself pinned by the paper's worked examples), by a hand-worked stream with
symbols above 2^16 (tests/golden/wide_symbols.txt), by library references
(np.bincount) and by order-preserving relabelling of the alphabet."""
import numpy as np
import pytest

import hdsynth
import oracle
from conftest import load_golden, pack_bits


def test_bitstream_does_not_depend_on_symbol_width():
    rng = np.random.default_rng(31)
    x = hdsynth.two_sided_geometric(rng, 50_001, 0.6, 200)
    ln = oracle.code_lengths(oracle.histogram(x, 200), 16)
    cd = oracle.canonical_codes(ln)
    ref = oracle.encode(x, ln, cd, 64, 4)
    for dt, w in ((np.uint8, 1), (np.uint32, 4)):
        xv = x.astype(dt)
        assert np.array_equal(oracle.histogram(xv, 200), oracle.histogram(x, 200))
        e = oracle.encode(xv, ln, cd, 64, 4)
        assert np.array_equal(e.words, ref.words)
        assert np.array_equal(e.gap, ref.gap)
        assert np.array_equal(e.chunk_counts, ref.chunk_counts)
        got = oracle.decode(e.words, e.n_bits, x.size, ln, cd, width=w)
        assert got.dtype == dt
        assert np.array_equal(got, xv)


def test_wide_symbols_hand_worked(golden):
    g = golden("wide_symbols.txt")
    A = int(g["A"][0][0])
    ln = np.zeros(A, np.uint8)
    for s, l in g["length"]:
        ln[int(s)] = int(l)
    cd = oracle.canonical_codes(ln)
    for s, bits in g["code"]:
        assert cd[int(s)] == int(bits, 2)
    msg = np.array([int(v) for v in g["message"][0]], np.uint32)
    e = oracle.encode(msg, ln, cd, 32, 1)
    bits = g["bits"][0][0]
    assert e.n_bits == len(bits)
    assert np.array_equal(e.words, pack_bits(bits, e.words.size))
    assert int(e.words[0]) == int(g["word0"][0][0], 16)
    assert np.array_equal(oracle.decode(e.words, e.n_bits, msg.size, ln, cd, width=4), msg)
    with pytest.raises(oracle.OracleError) as ei:          # 2^24 symbols do not fit 16 bits
        oracle.decode(e.words, e.n_bits, msg.size, ln, cd, width=2)
    assert ei.value.rc == oracle.EARG


def test_wide_histogram_matches_bincount():
    rng = np.random.default_rng(32)
    A = 1 << 18
    x = hdsynth.two_sided_geometric(rng, 200_000, 0.999, A, dtype=np.uint32)
    assert x.max() > 65535
    assert np.array_equal(oracle.histogram(x, A), np.bincount(x, minlength=A).astype(np.uint64))


def test_code_lengths_invariant_under_order_preserving_relabelling():
    """Spreading the used symbols over a 2^24 alphabet (keeping their order)
    changes nothing: package-merge ranks by (count, symbol)."""
    rng = np.random.default_rng(33)
    for trial in range(20):
        m = int(rng.integers(2, 300))
        cnt = rng.integers(1, 1000, m).astype(np.uint64)
        L = int(rng.integers(int(np.ceil(np.log2(m))) if m > 1 else 1, 25))
        L = max(L, 1)
        small = oracle.code_lengths(cnt, L)
        pos = np.sort(rng.choice(1 << 24, m, replace=False))
        wide = np.zeros(1 << 24, np.uint64)
        wide[pos] = cnt
        big = oracle.code_lengths(wide, L)
        assert np.array_equal(big[pos], small)
        assert big.sum() == small.sum()
        cs, cb = oracle.canonical_codes(small), oracle.canonical_codes(big)
        assert np.array_equal(cb[pos], cs)


def test_wide_round_trip():
    rng = np.random.default_rng(34)
    A = 1 << 18
    x = hdsynth.two_sided_geometric(rng, 300_000, 0.998, A, dtype=np.uint32)
    ln = oracle.code_lengths(oracle.histogram(x, A), 24)
    cd = oracle.canonical_codes(ln)
    e = oracle.encode(x, ln, cd, 128, 32)
    assert np.array_equal(oracle.decode(e.words, e.n_bits, x.size, ln, cd, width=4), x)


def test_width_alphabet_limits():
    x8 = np.arange(10, dtype=np.uint8)
    with pytest.raises(oracle.OracleError):
        oracle.histogram(x8, 257)                           # one byte holds 256 symbols
    assert oracle.histogram(x8, 256).sum() == 10
    x16 = np.arange(10, dtype=np.uint16)
    with pytest.raises(oracle.OracleError):
        oracle.histogram(x16, 65537)
    x32 = np.arange(10, dtype=np.uint32)
    with pytest.raises(oracle.OracleError):
        oracle.histogram(x32, (1 << 24) + 1)
    with pytest.raises(oracle.OracleError):
        oracle.code_lengths(np.ones((1 << 24) + 1, np.uint64), 32)
    # a symbol value at or above A
    with pytest.raises(oracle.OracleError) as ei:
        oracle.histogram(np.array([300], np.uint32), 256)
    assert ei.value.rc == oracle.ESYMBOL


@pytest.mark.parametrize("dt,w", [(np.uint8, 1), (np.uint32, 4)])
def test_chunk_parallel_decode_other_widths(dt, w):
    rng = np.random.default_rng(35)
    A = 256 if w == 1 else 1 << 18
    x = hdsynth.two_sided_geometric(rng, 123_457, 0.7 if w == 1 else 0.998, A, dtype=dt)
    ln = oracle.code_lengths(oracle.histogram(x, A), 24)
    cd = oracle.canonical_codes(ln)
    e = oracle.encode(x, ln, cd, 128, 8)
    got = oracle.decode_chunks_parallel(e.words, e.n_bits, x.size, ln, cd, e.gap, e.chunk_offsets, 128, 8, 5,
                                        width=w)
    assert got.dtype == dt and np.array_equal(got, x)
