"""Corrupted inputs in both modes: flipped bits in the words, a truncated
n_bits, a wrong n_symbols, another codebook, corrupted gap bytes.  The
decoder's structural checks are complete: its status is clean exactly when
the oracle finds the (corrupted) input consistent -- the bit-serial decode
from bit 0 gives n_symbols codewords ending on n_bits and, in gap mode, the
true sync points and chunk offsets equal the stored ones -- and then the
output is the oracle's decode.  No write may land past the claimed output."""
import numpy as np
import pytest

import hdsynth
import oracle
from hdcase import flush, make_case

pytestmark = pytest.mark.gpu

GUARD = 512


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    yield


def _consistent(words, B, n, ln, cd, S, C, gap, off, mode):
    """(consistent?, oracle decode or None) of a possibly corrupted input."""
    try:
        y = oracle.decode(words, B, n, ln, cd)
    except oracle.OracleError:
        return False, None
    if mode == 1:
        return True, y
    sg, cnt, _ = oracle.selfsync(words, B, n, ln, cd, S)
    K = sg.size
    M = (K + C - 1) // C
    want = np.zeros(M + 1, np.uint64)
    if K:
        np.cumsum(np.add.reduceat(cnt.astype(np.uint64), np.arange(0, K, C)), out=want[1:])
    ok = gap.size == K and np.array_equal(gap, sg) and off.size == M + 1 and np.array_equal(off, want)
    return bool(ok), y


def _run(words, gap, off, info, ln, cd, L, mode, lut_bits=0):
    import torch
    from paper_2201_09118_amd import hd
    tab = hd.Table(ln, cd, L, lut_bits)
    g = torch.from_numpy(gap).cuda() if mode == 0 else None
    o = torch.from_numpy(off.view(np.int64)).cuda() if mode == 0 else None
    ds = hd.DeviceStream(torch.from_numpy(words.view(np.int32)).cuda(), g, o, info, tab)
    n = int(info.n_symbols)
    out = torch.full((n + GUARD,), -1, dtype=torch.int16, device="cuda")
    ws = hd.decode(ds, out, mode)
    bits = hd.decode_status_bits(ws)
    host = out.cpu().numpy()
    return host[:n].view(np.uint16), bits, host[n:]


def _check(case, words, B, n, gap, off, mode, ln=None, cd=None, tag=""):
    from paper_2201_09118_amd import hd
    ln = case.lengths if ln is None else ln
    cd = case.codes if cd is None else cd
    S, C = case.S, case.C
    info = hd.stream_layout(n, B, case.A, case.L, S, C)
    info.n_words = words.size
    K, M = int(info.n_subseq), int(info.n_chunks)
    gap, off = gap[:K].copy(), off[:M + 1].copy()
    ok, y = _consistent(words, B, n, ln, cd, S, C, gap, off, mode)
    flush(f"fault {tag} mode={mode}: oracle-consistent={ok}")
    got, bits, tail = _run(words, gap, off, info, ln, cd, case.L, mode)
    assert (tail == -1).all(), "write past the claimed output"
    if ok:
        assert bits == 0 and np.array_equal(got, y), tag
    else:
        assert bits != 0, tag
    return ok


def _case(seed=60, n=300_007, A=1024, S=128, C=32, r=0.6):
    x = hdsynth.two_sided_geometric(np.random.default_rng(seed), n, r, A)
    return make_case(x, A, 24, S, C)


@pytest.mark.parametrize("mode", [0, 1])
def test_flipped_bits(mode):
    case = _case(61 + mode)
    e = case.enc
    rng = np.random.default_rng(7 + mode)
    flagged = 0
    for trial in range(6):
        w = e.words.copy()
        nflip = [1, 3, 40, 200, 1, 17][trial]
        pos = rng.integers(0, e.n_bits, nflip)
        for p in pos.tolist():
            w[p // 32] ^= np.uint32(1 << (31 - p % 32))
        flagged += not _check(case, w, e.n_bits, e.n_symbols, e.gap, e.chunk_offsets, mode, tag=f"flip{nflip}")
    assert flagged >= 3          # most of these corruptions break the stream's structure


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("d", [1, 7, 129])
def test_truncated_n_bits(mode, d):
    case = _case(62)
    e = case.enc
    assert not _check(case, e.words, e.n_bits - d, e.n_symbols, e.gap, e.chunk_offsets, mode, tag=f"trunc{d}")


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("dn", [-1, 1, -1000])
def test_wrong_n_symbols(mode, dn):
    case = _case(63)
    e = case.enc
    assert not _check(case, e.words, e.n_bits, e.n_symbols + dn, e.gap, e.chunk_offsets, mode, tag=f"n{dn:+d}")


@pytest.mark.parametrize("mode", [0, 1])
def test_another_codebook(mode):
    case = _case(64)
    other = _case(65, r=0.3)
    e = case.enc
    assert not np.array_equal(other.lengths, case.lengths)
    assert not _check(case, e.words, e.n_bits, e.n_symbols, e.gap, e.chunk_offsets, mode,
                      ln=other.lengths, cd=other.codes, tag="codebook")


def test_corrupted_gap_bytes():
    case = _case(66)
    e = case.enc
    for k, v in ((0, 1), (10, None), (e.gap.size // 2, 31), (e.gap.size - 1, None)):
        g = e.gap.copy()
        g[k] = (int(g[k]) + 1) % 24 if v is None else v
        assert not _check(case, e.words, e.n_bits, e.n_symbols, g, e.chunk_offsets, 0, tag=f"gap[{k}]")
