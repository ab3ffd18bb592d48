"""GPU check of the allocation-free decode (hd_decode_noalloc) against hd_decode
through the C-ABI: same output, same status, on consecutive calls whose second
input is smaller (the fixed scratch keeps the first call's contents), in both
modes; oversized self-sync streams are refused before any launch."""
import numpy as np
import pytest

import hdsynth
from hdcase import expected, flush, make_case, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2201_09118_amd import hd  # noqa: F401
    yield


def _pair(ds, mode):
    """(output, status) of hd_decode_noalloc and of hd_decode on one stream."""
    import torch
    from paper_2201_09118_amd import hd
    n = ds.n_symbols
    a = torch.full((max(n, 1),), -1, dtype=torch.int16, device="cuda")
    b = torch.full((max(n, 1),), -1, dtype=torch.int16, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    hd.decode_noalloc(ds, a, st, mode)
    torch.cuda.synchronize()
    bits_a = int(st.cpu().numpy().view(np.uint32)[0])
    ws = hd.decode(ds, b, mode)
    bits_b = hd.decode_status_bits(ws)
    torch.cuda.synchronize()
    return (a[:n].cpu().numpy().view(np.uint16), bits_a), (b[:n].cpu().numpy().view(np.uint16), bits_b)


@pytest.mark.parametrize("mode", [0, 1], ids=["gap", "selfsync"])
def test_noalloc_matches_decode_on_shrinking_inputs(mode):
    big = make_case(hdsynth.config1_symbols(n=3_000_017), 1024, 16, 128, 32)
    rng = np.random.default_rng(7)
    small = make_case(rng.integers(0, 300, 70_001).astype(np.uint16), 300, 12, 64, 8)
    for name, case in (("big", big), ("small", small)):
        flush(f"noalloc mode={mode} {name} n={case.x.size} S={case.S} C={case.C}")
        ds = upload(case)
        (ga, sa), (gb, sb) = _pair(ds, mode)
        want = expected(case)
        assert sa == sb == 0, (hex(sa), hex(sb))
        assert np.array_equal(ga, gb)
        assert np.array_equal(ga, want)


@pytest.mark.parametrize("mode", [0, 1], ids=["gap", "selfsync"])
def test_noalloc_reports_corruption_like_decode(mode):
    import torch
    rng = np.random.default_rng(11)
    case = make_case(rng.integers(0, 64, 200_003).astype(np.uint16), 64, 10, 128, 32)
    ds = upload(case)
    # a clean call first, then the same stream with its tail truncated: the
    # scratch's earlier (clean) status must not hide the new fault
    (_, s0), _ = _pair(ds, mode)
    assert s0 == 0
    bad = ds.info
    flush(f"noalloc corrupt mode={mode}")
    from paper_2201_09118_amd import hd
    info = hd.StreamInfo(bad.n_symbols - 5, bad.n_bits, bad.n_words, bad.n_subseq, bad.n_chunks,
                         bad.subseq_bits, bad.chunk_subseqs, bad.alphabet_size, bad.max_len)
    ds2 = hd.DeviceStream(ds.words, ds.gap, ds.chunk_offsets, info, ds.table)
    (ga, sa), (gb, sb) = _pair(ds2, mode)
    assert sa != 0 and sa == sb, (hex(sa), hex(sb))
    torch.cuda.synchronize()


def test_noalloc_refuses_streams_beyond_the_scratch():
    import torch
    from paper_2201_09118_amd import hd
    S = 32
    K = 16 << 20                      # self-sync workspace > 32 MiB at one byte + records per subsequence
    nw = K * S // 32 + 2
    words = torch.zeros(nw, dtype=torch.int32, device="cuda")
    lengths = np.zeros(4, dtype=np.uint8)
    lengths[:] = 2
    codes = np.arange(4, dtype=np.uint32)
    tab = hd.Table(lengths, codes, 2)
    info = hd.StreamInfo(K * S // 2, K * S, nw, K, (K + 31) // 32, S, 32, 4, 2)
    ds = hd.DeviceStream(words, None, None, info, tab)
    assert hd.decode_workspace_size(ds, 1) > hd.NOALLOC_SCRATCH_BYTES
    out = torch.empty(K * S // 2, dtype=torch.int16, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(hd.HDError) as ei:
        hd.decode_noalloc(ds, out, st, 1)
    assert ei.value.status == hd.ERR_UNSUPPORTED
