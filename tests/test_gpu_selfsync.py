"""GPU parity of the self-synchronizing decode (no gap array, no chunk counts
read) against the CPU oracle; the sync points found must equal the gap array
the oracle's encoder emits (the true codeword starts), bit for bit."""
import numpy as np
import pytest

import hdsynth
import oracle
from hdcase import expected, flush, make_case, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2201_09118_amd import hd  # noqa: F401
    yield


def _check_ss(case, lut_bits=0, tune=None):
    import torch
    from paper_2201_09118_amd import hd
    ds = upload(case, lut_bits, with_gap=False)          # no gap array, no chunk counts on the device
    n = case.x.size
    out = torch.full((max(n, 1),), -1, dtype=torch.int16, device="cuda")
    ws = hd.decode(ds, out, hd.MODE_SELF_SYNC, tune)
    bits = hd.decode_status_bits(ws)
    got = out[:n].cpu().numpy().view(np.uint16)
    want = expected(case)
    assert bits == 0, f"status bits {bits:#x}"
    gap = torch.zeros(max(case.enc.gap.size, 1), dtype=torch.uint8, device="cuda")
    hd.decode_sync_points(ds, ws, gap)
    found = gap[:case.enc.gap.size].cpu().numpy()
    sg, _, _ = oracle.selfsync(case.enc.words, case.enc.n_bits, n, case.lengths, case.codes, case.S)
    assert np.array_equal(found, sg), f"{(found != sg).sum()} sync points differ"
    assert np.array_equal(found, case.enc.gap)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{bad.size} mismatches, first at {bad[:8]}")


def test_config1_selfsync():
    flush("config1 self-sync")
    _check_ss(make_case(hdsynth.config1_symbols(), 1024, 16, 128, 32))


@pytest.mark.parametrize("i", range(16))
def test_random_streams_selfsync(i):
    rng = np.random.default_rng(500 + i)
    S = [32, 64, 128, 256, 512][i % 5]
    n = [1, 63, 64, 65, 4097, 54321, 200_001, 1000][i % 8]
    A = int(rng.choice([2, 3, 256, 1024, 4096]))
    r = float(rng.uniform(0.1, 0.95))
    x = hdsynth.two_sided_geometric(rng, n, r, A)
    used = int((np.bincount(x, minlength=A) > 0).sum())
    L = max(int(np.ceil(np.log2(max(used, 2)))), int(rng.integers(8, 28)))
    flush(f"self-sync random i={i} S={S} n={n} A={A} L={L}")
    _check_ss(make_case(x, A, L, S, 32), lut_bits=int(rng.choice([0, 8, 12])))


def test_fixed_length_code_never_synchronizes():
    """3-bit fixed-length code: raw boundaries 128k are off phase for 2 of 3
    subsequences and never resynchronize; the result must still be exact."""
    rng = np.random.default_rng(3)
    x = rng.integers(0, 8, 300_000).astype(np.uint16)
    case = make_case(x, 8, 3, 128, 32)
    assert set(case.lengths.tolist()) == {3}
    _check_ss(case)


@pytest.mark.parametrize("S", [32, 96, 256, 512])
def test_unconverged_tiles_at_every_subsequence_size(S):
    """3-bit fixed-length code at several subsequence sizes and a ragged
    length: tiles stay unconverged after the sync kernel's round budget
    (three rounds for codes this short) and are finished from per-entry exit
    tables."""
    rng = np.random.default_rng(30 + S)
    x = rng.integers(0, 8, 200_003).astype(np.uint16)
    flush(f"unconverged tiles S={S}")
    _check_ss(make_case(x, 8, 3, S, 32))


def test_runs_of_one_long_codeword_selfsync():
    """Runs of one long codeword (19 bits: a symbol that is rare overall, as
    the clamped values at the edge of a Lorenzo field) inside ordinary
    short-code data: those tiles resynchronize slowly or not at all and walk
    long codes through the per-length limits."""
    rng = np.random.default_rng(31)
    base = hdsynth.two_sided_geometric(rng, 600_000, 0.6, 1024)
    hist = np.bincount(base, minlength=1024).astype(np.uint64) * 4096
    hist[0] = 1
    ln = oracle.code_lengths(hist, 24)
    cd = oracle.canonical_codes(ln)
    assert ln[0] == ln.max() and ln[0] >= 16
    parts = []
    for seg in np.array_split(base, 25):
        parts += [seg, np.zeros(int(rng.integers(40, 400)), np.uint16)]
    x = np.concatenate(parts)
    flush(f"runs of one long codeword: {x.size} symbols")
    _check_ss(make_case(x, 1024, 24, 128, 32, ln, cd))


def test_even_length_code_odd_entries():
    """All codewords 2 bits: paths from odd offsets never meet even ones."""
    x = np.repeat(np.arange(4, dtype=np.uint16), 20_000)
    np.random.default_rng(4).shuffle(x)
    _check_ss(make_case(x, 4, 2, 64, 32))


def test_interleaved_runs_of_entry_dependent_tiles():
    """Segments of the codewords 00 and 01 only (a path from an odd offset
    reads 00 or 10 there and never meets the even ones: every such tile is
    entry-dependent) alternate with segments that use the 3-bit codewords
    (which resynchronize), so one stream holds many separate runs of
    dependent tiles, several per 64-tile window."""
    rng = np.random.default_rng(8)
    # lengths: symbols 0..2 get 2 bits, 3..4 get 3 bits (Kraft: 3/4 + 2/8 = 1)
    hist = np.array([1000, 1000, 1000, 1, 1], np.uint64)
    ln, cd = oracle.build_codebook(np.repeat(np.arange(5, dtype=np.uint16), hist.astype(np.int64)), 5, 3)
    assert sorted(ln.tolist()) == [2, 2, 2, 3, 3]
    parts = []
    for i in range(160):
        n = int(rng.integers(2_000, 40_000))
        if i % 2 == 0:
            parts.append(rng.choice(np.flatnonzero((ln == 2) & (cd < 2)), n).astype(np.uint16))
        else:
            parts.append(rng.integers(0, 5, n // 8).astype(np.uint16))
    x = np.concatenate(parts)
    case = make_case(x, 5, 3, 64, 32, ln, cd)
    _, _, sb = oracle.selfsync(case.enc.words, case.enc.n_bits, x.size, ln, cd, 64)
    assert (sb > 64 * 64).sum() > 1000           # raw paths that stay off for more than a tile
    flush(f"interleaved dependent runs: {x.size} symbols, {case.enc.gap.size // 64} tiles")
    _check_ss(case)


@pytest.mark.parametrize("S,n", [(32, 200_000), (32, 77_777), (64, 150_001), (32, 1_234)])
def test_entries_meeting_several_subsequences_later(S, n):
    """Codes of about 8 bits with 32- and 64-bit subsequences: paths from
    different entries of a tile often meet only in its second to fourth
    subsequence, or later; stream sizes leave a ragged last tile."""
    rng = np.random.default_rng(31 + n)
    x = hdsynth.two_sided_geometric(rng, n, 0.98, 4096)
    case = make_case(x, 4096, 20, S, 32)
    _, _, sb = oracle.selfsync(case.enc.words, case.enc.n_bits, x.size, case.lengths, case.codes, S)
    if n > 10_000:
        assert ((sb > S) & (sb <= 4 * S)).sum() > sb.size // 10
        assert (sb > 4 * S).sum() > 0
    flush(f"entries meeting later: S={S} n={n} K={sb.size}")
    _check_ss(case)


@pytest.mark.parametrize("i", range(12))
def test_long_code_streams_selfsync(i):
    """Mean code lengths from 6.7 to 11.4 bits in 32- to 128-bit subsequences:
    all three round budgets of the sync kernel (below 7, 10 and above), many
    tiles listed for the pending-tile kernel (few and many per workgroup) and
    first tiles of groups that the entry probe leaves unsettled."""
    S = [32, 64, 96, 128][i % 4]
    A = [4096, 65536, 16384][i % 3]
    r = [0.95, 0.98, 0.995, 0.998][(i // 3) % 4]
    n = [3001, 54321, 200003, 99999][i % 4]
    x = hdsynth.two_sided_geometric(np.random.default_rng(1900 + i), n, r, A)
    used = int((np.bincount(x, minlength=A) > 0).sum())
    L = max(int(np.ceil(np.log2(max(used, 2)))), [18, 22, 27][i % 3])
    flush(f"long-code self-sync i={i} S={S} A={A} r={r} n={n} L={L}")
    _check_ss(make_case(x, A, L, S, 32))


def test_all_one_bit_codes_selfsync():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 2, 400_000).astype(np.uint16)
    _check_ss(make_case(x, 2, 4, 128, 32))


def test_long_codes_selfsync():
    fib = [1, 1]
    while len(fib) < 30:
        fib.append(fib[-1] + fib[-2])
    x = np.repeat(np.arange(30, dtype=np.uint16), fib)
    np.random.default_rng(6).shuffle(x)
    case = make_case(x, 30, 27, 256, 32)
    _check_ss(case, lut_bits=6)
    _check_ss(case, lut_bits=12)


def test_single_symbol_selfsync():
    _check_ss(make_case(np.full(50_000, 9, np.uint16), 16, 4, 128, 32))


def test_selfsync_ignores_gap_and_chunk_offsets():
    """Self-sync reads neither metadata array: garbage there changes nothing."""
    import torch
    from paper_2201_09118_amd import hd
    x = hdsynth.two_sided_geometric(np.random.default_rng(7), 100_000, 0.5, 1024)
    case = make_case(x, 1024, 20, 128, 32)
    ds = upload(case)
    ds.gap.fill_(255)
    ds.chunk_offsets.fill_(7)
    out = torch.empty(x.size, dtype=torch.int16, device="cuda")
    ws = hd.decode(ds, out, hd.MODE_SELF_SYNC)
    assert hd.decode_status(ws) == hd.OK
    assert np.array_equal(out.cpu().numpy().view(np.uint16), x)


@pytest.mark.slow
def test_config2_full_selfsync():
    flush("config2 self-sync full")
    _check_ss(make_case(hdsynth.config2_symbols(), 1024, 24, 128, 32))


@pytest.mark.slow
def test_config3_full_selfsync():
    flush("config3 self-sync full")
    _check_ss(make_case(hdsynth.config3_symbols(), 4096, 27, 256, 32))
