"""Pins for the CPU oracle (oracle/hdref.c) against facts that do not come
from the oracle itself: the paper's worked examples (tests/golden/), closed
forms, brute force on tiny alphabets, a textbook heap Huffman, and
independent numpy recomputations of the stream layout."""
import heapq
import itertools
import math

import numpy as np
import pytest

import oracle
from conftest import load_golden, pack_bits, unpack_bits

UINT32_MAX = 0xFFFFFFFF


def _codebook(g):
    letters = [e[0] for e in g["code"]]
    lengths = np.array([len(e[1]) for e in g["code"]], np.uint8)
    codes = np.array([int(e[1], 2) for e in g["code"]], np.uint32)
    return letters, lengths, codes


# --------------------------------------------------------------------------
# Paper examples: Listing 1 (self-synchronization) and Fig. 1 (gap array)
# --------------------------------------------------------------------------

def test_listing1_decode():
    g = load_golden("listing1_selfsync.txt")
    letters, ln, cd = _codebook(g)
    bits = g["bits"][0][0]
    want = g["decoded"][0][0]
    out = oracle.decode(pack_bits(bits), len(bits), len(want), ln, cd)
    assert "".join(letters[s] for s in out) == want


def test_listing1_skipped_bit_decodes_wrong_then_resyncs():
    g = load_golden("listing1_selfsync.txt")
    letters, ln, cd = _codebook(g)
    bits = g["bits"][0][0][1:]
    want = g["skip1_decoded"][0][0]
    out, end = oracle.decode_prefix(pack_bits(bits), len(bits), len(want), ln, cd)
    assert "".join(letters[s] for s in out) == want
    assert end == len(bits)


def test_listing1_sync_distance_from_raw_boundary():
    """A raw 32-bit subsequence boundary placed on the listing's second bit
    must reach a true codeword boundary after exactly 8 bits."""
    g = load_golden("listing1_selfsync.txt")
    letters, ln, cd = _codebook(g)
    bits = g["bits"][0][0]
    prefix = "010" + "00" * 14                       # D + 14 x A = 31 bits
    assert len(prefix) == 31
    s = prefix + bits
    n = 1 + 14 + len(g["decoded"][0][0])
    sg, cnt, sb = oracle.selfsync(pack_bits(s), len(s), n, ln, cd, 32)
    assert sb[0] == 0
    assert sb[1] == int(g["skip1_sync_bits"][0][0])
    assert sg[1] == 1                                # next true start is bit 33
    assert cnt.sum() == n


def _fig1():
    g = load_golden("figure1_gap.txt")
    letters, ln, cd = _codebook(g)
    x = np.array([letters.index(ch) for ch in g["string"][0][0]], np.uint16)
    return g, letters, ln, cd, x


def test_figure1_encoder_bits_and_forward_gap():
    g, letters, ln, cd, x = _fig1()
    S = int(g["S"][0][0])
    e = oracle.encode(x, ln, cd, S=S, C=1)
    assert e.n_bits == 32
    assert unpack_bits(e.words, e.n_bits) == g["bits"][0][0]
    assert e.gap.tolist() == [int(v) for v in g["gap_forward"][0]]
    assert e.chunk_counts.tolist() == [int(v) for v in g["counts_forward"][0]]
    assert e.chunk_offsets.tolist() == [0, 4, 8, 12, 15]


def test_figure1_backward_gap_is_the_printed_one():
    g, letters, ln, cd, x = _fig1()
    S = int(g["S"][0][0])
    words = pack_bits(g["bits"][0][0])
    gb, cb = oracle.gap_backward(words, 32, x.size, ln, cd, S)
    assert gb.tolist() == [int(v) for v in g["gap_backward"][0]]
    assert cb.tolist() == [int(v) for v in g["counts_backward"][0]]
    assert [k * S + int(v) for k, v in enumerate(gb)] == [int(v) for v in g["sync_markers"][0]]


def test_figure1_sync_points():
    g, letters, ln, cd, x = _fig1()
    S = int(g["S"][0][0])
    words = pack_bits(g["bits"][0][0])
    sg, cnt, sb = oracle.selfsync(words, 32, x.size, ln, cd, S)
    assert sg.tolist() == [int(v) for v in g["gap_forward"][0]]
    assert cnt.tolist() == [int(v) for v in g["counts_forward"][0]]


# --------------------------------------------------------------------------
# Histogram
# --------------------------------------------------------------------------

def test_histogram_matches_bincount_and_rejects_out_of_range():
    rng = np.random.default_rng(7)
    x = rng.integers(0, 300, 10000).astype(np.uint16)
    h = oracle.histogram(x, 300)
    assert h.sum() == x.size
    assert np.array_equal(h, np.bincount(x, minlength=300).astype(np.uint64))
    with pytest.raises(oracle.OracleError) as ei:
        oracle.histogram(np.array([1, 2, 300], np.uint16), 300)
    assert ei.value.rc == oracle.ESYMBOL


# --------------------------------------------------------------------------
# Code lengths (package-merge)
# --------------------------------------------------------------------------

def _cost(counts, lengths):
    return sum(int(c) * int(l) for c, l in zip(counts, lengths))


def _brute_min_cost_all(ws, L):
    """Every length vector in [1, L]^m with Kraft sum <= 1."""
    best = None
    for lens in itertools.product(range(1, L + 1), repeat=len(ws)):
        if sum(1 << (L - l) for l in lens) <= (1 << L):
            c = sum(w * l for w, l in zip(ws, lens))
            best = c if best is None else min(best, c)
    return best


def _brute_min_cost_multisets(ws, L):
    """Every multiset of lengths with Kraft sum <= 1; the shortest lengths go
    to the largest counts (rearrangement inequality)."""
    ws = sorted(ws, reverse=True)
    best = None
    for lens in itertools.combinations_with_replacement(range(1, L + 1), len(ws)):
        if sum(1 << (L - l) for l in lens) <= (1 << L):
            c = sum(w * l for w, l in zip(ws, lens))
            best = c if best is None else min(best, c)
    return best


def _heap_huffman(ws):
    """Textbook Huffman: (cost, depth per leaf)."""
    h = [(w, i, [i]) for i, w in enumerate(ws)]
    heapq.heapify(h)
    depth = [0] * len(ws)
    cost = 0
    tie = len(ws)
    while len(h) > 1:
        w1, _, a = heapq.heappop(h)
        w2, _, b = heapq.heappop(h)
        for i in a + b:
            depth[i] += 1
        cost += w1 + w2
        heapq.heappush(h, (w1 + w2, tie, a + b))
        tie += 1
    return cost, depth


def _random_counts(rng, A, m, skew):
    counts = np.zeros(A, np.uint64)
    used = rng.choice(A, m, replace=False)
    counts[used] = np.maximum(1, (rng.pareto(skew, m) * 50).astype(np.uint64) + 1)
    return counts


@pytest.mark.parametrize("seed", range(40))
def test_package_merge_is_optimal_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.integers(2, 7))
    L = int(rng.integers(max(1, math.ceil(math.log2(m))), 7))
    A = m + int(rng.integers(0, 4))
    counts = _random_counts(rng, A, m, 0.7 + rng.random())
    ln = oracle.code_lengths(counts, L)
    used = counts > 0
    assert np.all(ln[~used] == 0)
    assert np.all((ln[used] >= 1) & (ln[used] <= L))
    assert sum(2.0 ** -int(l) for l in ln[used]) <= 1.0
    assert _cost(counts, ln) == _brute_min_cost_all([int(c) for c in counts[used]], L)


@pytest.mark.parametrize("seed", range(12))
def test_package_merge_is_optimal_eight_symbols(seed):
    rng = np.random.default_rng(2000 + seed)
    m = int(rng.integers(7, 9))
    L = int(rng.integers(3, 9))
    counts = _random_counts(rng, m, m, 0.5 + rng.random())
    ln = oracle.code_lengths(counts, L)
    assert ln.max() <= L
    assert _cost(counts, ln) == _brute_min_cost_multisets([int(c) for c in counts], L)


@pytest.mark.parametrize("seed", range(12))
def test_package_merge_equals_heap_huffman_when_limit_is_loose(seed):
    rng = np.random.default_rng(3000 + seed)
    m = int(rng.integers(2, 200))
    counts = _random_counts(rng, m + 10, m, 0.3 + rng.random())
    ws = [int(c) for c in counts if c > 0]
    hcost, depth = _heap_huffman(ws)
    L = max(depth)
    for LL in (L, L + 3, 32):
        ln = oracle.code_lengths(counts, LL)
        assert _cost(counts, ln) == hcost


@pytest.mark.parametrize("seed", range(8))
def test_kraft_equality_and_entropy_bounds(seed):
    rng = np.random.default_rng(4000 + seed)
    A = 1024
    x = rng.geometric(0.3, 20000) % A
    counts = np.bincount(x, minlength=A).astype(np.uint64)
    L = 24
    ln = oracle.code_lengths(counts, L)
    used = counts > 0
    kraft = sum(1 << (L - int(l)) for l in ln[used])
    assert kraft == 1 << L                     # integer Kraft equality
    p = counts[used] / counts.sum()
    H = float(-(p * np.log2(p)).sum())
    lbar = _cost(counts, ln) / counts.sum()
    assert H - 1e-12 <= lbar < H + 1


def test_dyadic_counts_give_minus_log2_p():
    m = 9
    counts = np.array([1 << (m - 1 - i) for i in range(m - 1)] + [1], np.uint64)
    ln = oracle.code_lengths(counts, 16)
    assert ln.tolist() == list(range(1, m)) + [m - 1]


@pytest.mark.parametrize("j", [1, 2, 3, 5, 8])
def test_equiprobable_power_of_two(j):
    counts = np.full(1 << j, 17, np.uint64)
    ln = oracle.code_lengths(counts, 16)
    assert np.all(ln == j)


def test_fibonacci_counts_force_depth_and_limit_binds():
    fib = [1, 1]
    while len(fib) < 8:
        fib.append(fib[-1] + fib[-2])
    counts = np.array(fib, np.uint64)
    ln = oracle.code_lengths(counts, 32)
    assert ln.max() == 7                      # unconstrained depth m - 1
    for L in (3, 4, 5, 6):
        ln = oracle.code_lengths(counts, L)
        assert ln.max() == L                  # the limit binds
        assert _cost(counts, ln) == _brute_min_cost_multisets(fib, L)


def test_degenerate_alphabets():
    A = 16
    assert np.all(oracle.code_lengths(np.zeros(A, np.uint64), 8) == 0)
    one = np.zeros(A, np.uint64)
    one[5] = 99
    ln = oracle.code_lengths(one, 8)
    assert ln[5] == 1 and ln.sum() == 1
    full = np.arange(1, 9, dtype=np.uint64)       # m = 8 = 2^3
    assert np.all(oracle.code_lengths(full, 3) == 3)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.code_lengths(np.arange(1, 10, dtype=np.uint64), 3)   # 9 > 2^3
    assert ei.value.rc == oracle.EINFEASIBLE


# --------------------------------------------------------------------------
# Canonical codes
# --------------------------------------------------------------------------

def test_canonical_rfc1951_example():
    g = load_golden("rfc1951_canonical.txt")
    ln = np.array([int(v) for v in g["lengths"][0]], np.uint8)
    want = [int(v, 2) for v in g["codes"][0]]
    assert oracle.canonical_codes(ln).tolist() == want


@pytest.mark.parametrize("seed", range(6))
def test_canonical_properties(seed):
    rng = np.random.default_rng(5000 + seed)
    A = 300
    counts = _random_counts(rng, A, int(rng.integers(2, A)), 0.5 + rng.random())
    L = 20
    ln = oracle.code_lengths(counts, L)
    cd = oracle.canonical_codes(ln)
    used = [s for s in range(A) if ln[s] > 0]
    order = sorted(used, key=lambda s: (int(ln[s]), s))
    lj = [int(cd[s]) << (32 - int(ln[s])) for s in order]
    assert all(a < b for a, b in zip(lj, lj[1:]))           # strictly increasing
    for a, b in zip(order, order[1:]):
        if ln[a] == ln[b]:
            assert cd[b] == cd[a] + 1                        # consecutive in symbol order
    assert cd[order[0]] == 0
    last = order[-1]
    assert cd[last] == (1 << int(ln[last])) - 1              # complete code ends in all ones
    strs = [format(int(cd[s]), f"0{int(ln[s])}b") for s in used]
    for a in strs:                                           # prefix-free, by brute force
        for b in strs:
            assert a == b or not b.startswith(a)


def test_canonical_rejects_oversubscribed_lengths():
    with pytest.raises(oracle.OracleError):
        oracle.canonical_codes(np.array([1, 1, 1], np.uint8))


# --------------------------------------------------------------------------
# Encoder layout
# --------------------------------------------------------------------------

def _layout_by_numpy(x, ln, S, C):
    lens = ln[x].astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]]) if x.size else np.zeros(0, np.int64)
    B = int(lens.sum())
    K = (B + S - 1) // S
    M = (K + C - 1) // C
    with_end = np.concatenate([starts, [B]])
    bounds = np.arange(K, dtype=np.int64) * S
    p = with_end[np.searchsorted(with_end, bounds, side="left")]
    gap = (p - bounds).astype(np.uint8)
    cnt = np.bincount(starts // S, minlength=K)[:K] if K else np.zeros(0, np.int64)
    cc = np.add.reduceat(cnt, np.arange(0, K, C)) if K else np.zeros(0, np.int64)
    return B, K, M, gap, cnt, cc


@pytest.mark.parametrize("S,C", [(32, 1), (64, 4), (128, 32), (256, 32), (96, 3)])
def test_encoder_layout_matches_independent_recomputation(S, C):
    rng = np.random.default_rng(S * 7 + C)
    A = 512
    x = (256 + rng.integers(-40, 41, 50000)).astype(np.uint16)
    ln, cd = oracle.build_codebook(x, A, 16)
    e = oracle.encode(x, ln, cd, S, C)
    B, K, M, gap, cnt, cc = _layout_by_numpy(x, ln, S, C)
    assert e.n_bits == B and e.gap.size == K and e.chunk_counts.size == M
    assert e.words.size == (K * S + 31) // 32 + 2
    assert np.array_equal(e.gap, gap)
    assert np.array_equal(e.chunk_counts.astype(np.int64), cc)
    assert e.chunk_counts.sum() == x.size
    # stored offsets: the output index of each chunk's first codeword = the
    # number of codeword starts before the chunk's first bit (brute force),
    # then n
    starts = np.concatenate([[0], np.cumsum(ln[x].astype(np.int64))])[:-1]
    want_off = [int((starts < c * C * S).sum()) for c in range(M)] + [x.size]
    assert e.chunk_offsets.tolist() == want_off
    assert e.gap[0] == 0 and int(e.gap.max()) < int(ln.max())
    tail = unpack_bits(e.words, e.words.size * 32)[B:]
    assert set(tail) <= {"0"}
    assert np.array_equal(oracle.decode(e.words, B, x.size, ln, cd), x)


def test_encoder_bits_are_the_concatenated_codewords():
    rng = np.random.default_rng(11)
    x = rng.integers(0, 40, 3000).astype(np.uint16)
    ln, cd = oracle.build_codebook(x, 40, 12)
    e = oracle.encode(x, ln, cd, 128, 32)
    want = "".join(format(int(cd[s]), f"0{int(ln[s])}b") for s in x)
    assert unpack_bits(e.words, e.n_bits) == want


def test_encoder_rejects_symbols_without_codeword():
    ln = np.array([1, 1, 0], np.uint8)
    cd = np.array([0, 1, 0], np.uint32)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.encode(np.array([0, 2], np.uint16), ln, cd)
    assert ei.value.rc == oracle.ESYMBOL


def test_empty_stream():
    ln = np.array([1, 1], np.uint8)
    cd = np.array([0, 1], np.uint32)
    e = oracle.encode(np.zeros(0, np.uint16), ln, cd)
    assert e.n_bits == 0 and e.gap.size == 0 and e.chunk_counts.size == 0 and e.words.size == 2
    assert e.chunk_offsets.tolist() == [0]
    assert oracle.decode(e.words, 0, 0, ln, cd).size == 0


def test_gap_array_overhead_matches_table4_ratio():
    """Table IV: the optimized gap-array CR is the self-sync CR divided by
    1 + 1/16 (one byte per 128-bit subsequence).  The rounding intervals of
    the eight printed ratio pairs intersect in a band that must hold the
    format's overhead."""
    g = load_golden("table4_cr.txt")
    ss = [float(v) for v in g["opt_selfsync"][0]]
    ga = [float(v) for v in g["opt_gaparray"][0]]
    lo = max((a - 0.005) / (b + 0.005) for a, b in zip(ss, ga))
    hi = min((a + 0.005) / (b - 0.005) for a, b in zip(ss, ga))
    S = int(g["subseq_bits"][0][0])
    rng = np.random.default_rng(12)
    x = (512 + rng.integers(-30, 31, 400000)).astype(np.uint16)
    ln, cd = oracle.build_codebook(x, 1024, 24)
    e = oracle.encode(x, ln, cd, S, 32)
    ratio = (e.n_bits / 8 + e.gap.size) / (e.n_bits / 8)
    assert lo <= ratio <= hi, (lo, ratio, hi)


# --------------------------------------------------------------------------
# Decoder error paths
# --------------------------------------------------------------------------

def test_decoder_detects_wrong_length_and_incomplete_code():
    rng = np.random.default_rng(13)
    x = rng.integers(0, 10, 500).astype(np.uint16)
    ln, cd = oracle.build_codebook(x, 10, 8)
    e = oracle.encode(x, ln, cd)
    for B in (e.n_bits - 1, e.n_bits + 1):
        with pytest.raises(oracle.OracleError):
            oracle.decode(e.words, B, x.size, ln, cd)
    # a single used symbol has the code '0'; a '1' bit leaves the tree
    ln1 = np.array([0, 1], np.uint8)
    cd1 = np.array([0, 0], np.uint32)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.decode(pack_bits("0010"), 4, 4, ln1, cd1)
    assert ei.value.rc == oracle.ECORRUPT
    assert oracle.decode(pack_bits("000"), 3, 3, ln1, cd1).tolist() == [1, 1, 1]


def test_decoder_rejects_non_prefix_code():
    ln = np.array([1, 2], np.uint8)
    cd = np.array([0b1, 0b10], np.uint32)      # '1' is a prefix of '10'
    with pytest.raises(oracle.OracleError):
        oracle.decode(pack_bits("110"), 3, 2, ln, cd)


# --------------------------------------------------------------------------
# Self-synchronization reference
# --------------------------------------------------------------------------

@pytest.mark.parametrize("S", [32, 128, 256])
def test_sync_points_equal_encoder_gap(S):
    rng = np.random.default_rng(S)
    x = (2048 + np.rint(40 * rng.standard_normal(60000))).astype(np.uint16)
    ln, cd = oracle.build_codebook(x, 4096, 27)
    e = oracle.encode(x, ln, cd, S, 32)
    sg, cnt, sb = oracle.selfsync(e.words, e.n_bits, x.size, ln, cd, S)
    assert np.array_equal(sg, e.gap)
    _, _, _, _, cnt_np, _ = _layout_by_numpy(x, ln, S, 32)
    assert np.array_equal(cnt.astype(np.int64), cnt_np)
    assert np.array_equal(sb == 0, sg == 0)       # raw boundary is a true start iff gap is 0
    synced = sb != UINT32_MAX
    assert synced.mean() > 0.99          # a skewed Huffman code resynchronizes


def test_fixed_length_code_never_resyncs_off_phase():
    """All codewords 3 bits: from raw boundary 32k the decoder walks in steps
    of 3 and lands on a true start exactly when 32k is a multiple of 3."""
    rng = np.random.default_rng(14)
    x = rng.integers(0, 8, 4000).astype(np.uint16)
    ln = np.full(8, 3, np.uint8)
    cd = oracle.canonical_codes(ln)
    e = oracle.encode(x, ln, cd, 32, 1)
    sg, cnt, sb = oracle.selfsync(e.words, e.n_bits, x.size, ln, cd, 32)
    for k in range(sg.size):
        if (32 * k) % 3 == 0:
            assert sb[k] == 0
        else:
            assert sb[k] == UINT32_MAX
        assert sg[k] == (-32 * k) % 3


@pytest.mark.parametrize("S,C", [(32, 1), (128, 32), (96, 3)])
def test_decode_from_codeword_starts_matches_suffix(S, C):
    """Started at any true codeword start (computed here by numpy from the
    code lengths alone), the decoder reproduces the input's suffix and ends
    on the codeword boundary after the last symbol."""
    rng = np.random.default_rng(S + C)
    x = (300 + np.rint(25 * rng.standard_normal(40000))).astype(np.uint16)
    ln, cd = oracle.build_codebook(x, 1024, 20)
    e = oracle.encode(x, ln, cd, S, C)
    lens = ln[x].astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    for i in [0, 1, 17, 12345, x.size - 1]:
        n = min(500, x.size - i)
        got, end = oracle.decode_from(e.words, e.n_bits, int(starts[i]), n, ln, cd)
        assert np.array_equal(got, x[i:i + n])
        assert end == int(starts[i]) + int(lens[i:i + n].sum())
    with pytest.raises(oracle.OracleError):
        oracle.decode_from(e.words, e.n_bits, e.n_bits + 1, 1, ln, cd)


@pytest.mark.parametrize("threads", [1, 5, 16])
def test_chunk_parallel_decode_round_trips(threads):
    rng = np.random.default_rng(threads)
    x = (512 + rng.integers(-60, 61, 70001)).astype(np.uint16)
    ln, cd = oracle.build_codebook(x, 1024, 16)
    e = oracle.encode(x, ln, cd, 128, 32)
    y = oracle.decode_chunks_parallel(e.words, e.n_bits, x.size, ln, cd, e.gap, e.chunk_offsets, 128, 32,
                                      threads)
    assert np.array_equal(y, x)
