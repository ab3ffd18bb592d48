"""CPU checks of the C-ABI boundary: the library loads, exports everything
include/hd.h declares, and its host routines (codebook builder, reference
encoder) agree byte for byte with the oracle.  No GPU work is issued."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import hdsynth
import oracle
from conftest import ROOT


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "hd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(hd_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2201_09118_amd import hd
    declared = _header_functions()
    assert declared, "no declarations parsed"
    out = subprocess.run(["nm", "-D", "--defined-only", hd.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (hd_[a-z_]+)\b", out))
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    assert sorted(hd.SIGNATURES) == declared     # the binding covers exactly the header
    L = ctypes.CDLL(hd.LIB_PATH)
    for n in declared:
        assert getattr(L, n) is not None


def test_status_strings():
    from paper_2201_09118_amd import hd
    for st in range(0, -8, -1):
        assert hd.status_str(st) and hd.status_str(st) != "unknown status"


def _hist_cases():
    rng = np.random.default_rng(99)
    cases = []
    for i in range(25):
        A = int(rng.choice([2, 5, 64, 256, 1024, 4096]))
        m = int(rng.integers(1, A + 1))
        h = np.zeros(A, np.uint64)
        used = rng.choice(A, m, replace=False)
        h[used] = (rng.pareto(0.5 + rng.random(), m) * 100).astype(np.uint64) + 1
        L = int(rng.integers(max(1, int(np.ceil(np.log2(max(m, 2))))), 28))
        cases.append((h, L))
    # ties everywhere: equal counts
    cases.append((np.full(300, 7, np.uint64), 12))
    cases.append((np.array([5, 5, 5, 5, 1, 1, 1, 1], np.uint64), 3))
    return cases


@pytest.mark.parametrize("idx", range(27))
def test_build_codebook_matches_oracle_byte_for_byte(idx):
    from paper_2201_09118_amd import hd
    h, L = _hist_cases()[idx]
    ln, cd = hd.build_codebook(h, L)
    oln = oracle.code_lengths(h, L)
    ocd = oracle.canonical_codes(oln)
    assert np.array_equal(ln, oln)
    assert np.array_equal(cd, ocd)


def test_build_codebook_degenerate_and_errors():
    from paper_2201_09118_amd import hd
    ln, cd = hd.build_codebook(np.zeros(10, np.uint64), 8)
    assert ln.sum() == 0
    h = np.zeros(10, np.uint64)
    h[3] = 5
    ln, cd = hd.build_codebook(h, 8)
    assert ln[3] == 1 and ln.sum() == 1 and cd[3] == 0
    with pytest.raises(hd.HDError) as ei:
        hd.build_codebook(np.ones(9, np.uint64), 3)
    assert ei.value.status == hd.ERR_INFEASIBLE
    with pytest.raises(hd.HDError):
        hd.build_codebook(np.ones(9, np.uint64), 33)
    ln, cd = hd.build_codebook(np.ones(8, np.uint64), 3)
    assert np.all(ln == 3)


@pytest.mark.parametrize("S,C", [(32, 1), (64, 2), (128, 32), (256, 32), (512, 64), (96, 3)])
def test_encode_ref_matches_oracle(S, C):
    from paper_2201_09118_amd import hd
    rng = np.random.default_rng(S + C)
    x = hdsynth.two_sided_geometric(rng, 200_000, 0.6, 1024)
    hist = oracle.histogram(x, 1024)
    ln, cd = hd.build_codebook(hist, 20)
    hs = hd.encode_ref(x, ln, cd, 20, S, C)
    e = oracle.encode(x, ln, cd, S, C)
    assert hs.n_bits == e.n_bits
    assert np.array_equal(hs.words, e.words)
    assert np.array_equal(hs.gap, e.gap)
    assert np.array_equal(hs.chunk_offsets, e.chunk_offsets)
    assert hs.info.n_subseq == e.gap.size and hs.info.n_chunks == e.chunk_counts.size


def test_encode_ref_edge_cases():
    from paper_2201_09118_amd import hd
    ln = np.array([1, 1], np.uint8)
    cd = np.array([0, 1], np.uint32)
    hs = hd.encode_ref(np.zeros(0, np.uint16), ln, cd, 4)
    assert hs.n_bits == 0 and hs.words.size == 2 and hs.gap.size == 0 and hs.chunk_offsets.tolist() == [0]
    with pytest.raises(hd.HDError) as ei:
        hd.encode_ref(np.array([0, 2], np.uint16), ln, cd, 4)
    assert ei.value.status == hd.ERR_SYMBOL
    for S, C in ((48, 1), (0, 1), (128, 0)):
        with pytest.raises(hd.HDError) as ei:
            hd.encode_ref(np.array([0, 1], np.uint16), ln, cd, 4, S, C)
        assert ei.value.status == hd.ERR_ARG
    # longest codes (L = 32) and a single used symbol
    x = np.zeros(1000, np.uint16)
    h = np.bincount(x, minlength=4).astype(np.uint64)
    ln1, cd1 = hd.build_codebook(h, 32)
    e = oracle.encode(x, ln1, cd1, 128, 32)
    hs = hd.encode_ref(x, ln1, cd1, 32, 128, 32)
    assert np.array_equal(hs.words, e.words) and np.array_equal(hs.gap, e.gap)
    fib = [1, 1]
    while len(fib) < 34:
        fib.append(fib[-1] + fib[-2])
    h = np.array(fib, np.uint64)
    ln2, cd2 = hd.build_codebook(h, 32)
    assert ln2.max() == 32
    x = np.repeat(np.arange(34, dtype=np.uint16), 3)
    rng = np.random.default_rng(5)
    rng.shuffle(x)
    e = oracle.encode(x, ln2, cd2, 64, 4)
    hs = hd.encode_ref(x, ln2, cd2, 32, 64, 4)
    assert np.array_equal(hs.words, e.words) and np.array_equal(hs.gap, e.gap)
    assert np.array_equal(hs.chunk_offsets, e.chunk_offsets)
    assert np.array_equal(oracle.decode(hs.words, hs.n_bits, x.size, ln2, cd2), x)


def test_reconstruction_workspace_sizes():
    # status word (256 B) + the carry table of the three-pass path: ni x (nj / R) x nk int32,
    # R = 32 rows per wavefront block (halved down to 8 while a field gives < 4096 wavefronts)
    from paper_2201_09118_amd import hd
    assert hd.lorenzo_workspace_size((512, 512, 512)) == 256 + 512 * 16 * 512 * 4
    assert hd.lorenzo_workspace_size((64, 64, 64)) == 256 + 64 * 8 * 64 * 4          # R = 8
    assert hd.lorenzo_workspace_size((4, 8, 100)) == 256                              # one block: no table
    # long 1-D fields: one uint32 per tile of 4096 values and per group of 1024 tiles
    nt = (280_000_000 + 4095) // 4096
    assert hd.lorenzo_workspace_size((1, 1, 280_000_000)) == 256 + nt * 4 + (nt + 1023) // 1024 * 4
    assert hd.lorenzo_workspace_size((1, 1, 4096)) == 256
    assert hd.lorenzo_workspace_size((0, 5, 5)) == 256


def test_reconstruction_argument_errors_before_any_launch():
    from paper_2201_09118_amd import hd
    f = hd.lib().hd_lorenzo_reconstruct
    dummy = ctypes.c_void_p(16)                        # never dereferenced: every call fails its checks
    # no workspace / short workspace / radius 0 / eb <= 0 / NaN eb
    assert f(dummy, 2, 2, 2, 512, None, None, 0, 1e-4, dummy, None, None, 0, None) == hd.ERR_ARG
    assert f(dummy, 2, 2, 2, 512, None, None, 0, 1e-4, dummy, None, dummy, 8, None) == hd.ERR_ARG
    assert f(dummy, 2, 2, 2, 0, None, None, 0, 1e-4, dummy, None, dummy, 256, None) == hd.ERR_ARG
    assert f(dummy, 2, 2, 2, 512, None, None, 0, 0.0, dummy, None, dummy, 256, None) == hd.ERR_ARG
    assert f(dummy, 2, 2, 2, 512, None, None, 0, float("nan"), dummy, None, dummy, 256, None) == hd.ERR_ARG
    # outliers announced without lists; NULL codes
    assert f(dummy, 2, 2, 2, 512, None, None, 3, 1e-4, dummy, None, dummy, 256, None) == hd.ERR_ARG
    assert f(None, 2, 2, 2, 512, None, None, 0, 1e-4, dummy, None, dummy, 256, None) == hd.ERR_ARG
    # rows beyond 4096 values in a 2-D/3-D field
    ws = hd.lib().hd_lorenzo_workspace_size(2, 1, 8192)
    assert f(dummy, 2, 1, 8192, 512, None, None, 0, 1e-4, dummy, None, dummy, ws, None) == hd.ERR_UNSUPPORTED


def test_encode_workspace_sizes_and_layout_errors():
    from paper_2201_09118_amd import hd
    L = hd.lib()
    lay = hd.Layout(128, 32)
    n = 134_217_728
    nblk = (n + 4095) // 4096
    # status/total header + per-block bits + per-block offsets (the chunk
    # offsets go straight to the caller's array)
    assert L.hd_encode_workspace_size(n, 24, ctypes.byref(lay)) == 256 + nblk * 4 + nblk * 8
    assert L.hd_encode_workspace_size(n, 0, ctypes.byref(lay)) == 0
    assert L.hd_encode_workspace_size(n, 33, ctypes.byref(lay)) == 0
    assert L.hd_encode_workspace_size(n, 24, ctypes.byref(hd.Layout(0, 32))) == 0
    assert L.hd_encode_workspace_size(n, 24, None) == 0
    dummy = ctypes.c_void_p(16)
    # write: bad layouts and inconsistent chunk counts fail before any launch
    for S, C_, K, M in [(48, 32, 10, 1), (128, 0, 10, 1), (128, 32, 100, 2), (128, 32, 100, 5)]:
        st = L.hd_encode_write(dummy, 10, dummy, dummy, 4, ctypes.byref(hd.Layout(S, C_)), dummy, 500, dummy, K,
                               dummy, M, dummy, 1 << 20, None)
        assert st == hd.ERR_ARG, (S, C_, K, M)
    # histogram: alphabet outside [1, 65536]
    assert L.hd_histogram(dummy, 10, 0, dummy, None) == hd.ERR_ARG
    assert L.hd_histogram(dummy, 10, 65537, dummy, None) == hd.ERR_ARG


def test_stream_layout_sizes_match_the_encoders():
    from paper_2201_09118_amd import hd
    rng = np.random.default_rng(21)
    for S, C in ((32, 1), (128, 32), (256, 32), (96, 3)):
        x = hdsynth.two_sided_geometric(rng, 30_001, 0.5, 1024)
        ln, cd = oracle.build_codebook(x, 1024, 20)
        e = oracle.encode(x, ln, cd, S, C)
        info = hd.stream_layout(x.size, e.n_bits, 1024, 20, S, C)
        assert (info.n_words, info.n_subseq, info.n_chunks) == (e.words.size, e.gap.size, e.chunk_counts.size)
        assert e.chunk_offsets.size == info.n_chunks + 1
    info = hd.stream_layout(0, 0, 2, 1)
    assert (info.n_words, info.n_subseq, info.n_chunks) == (2, 0, 0)
    for args, st in (((10, 9, 4, 4), hd.ERR_CORRUPT), ((10, 41, 4, 4), hd.ERR_CORRUPT),
                     ((10, 20, 0, 4), hd.ERR_ARG), ((10, 20, 4, 33), hd.ERR_ARG)):
        with pytest.raises(hd.HDError) as ei:
            hd.stream_layout(*args)
        assert ei.value.status == st
    with pytest.raises(hd.HDError):
        hd.stream_layout(10, 20, 4, 4, 48, 1)


def test_noalloc_scratch_size_matches_header():
    from paper_2201_09118_amd import hd
    txt = open(os.path.join(ROOT, "include", "hd.h")).read()
    m = re.search(r"#define HD_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", txt)
    assert m, "HD_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == hd.NOALLOC_SCRATCH_BYTES
