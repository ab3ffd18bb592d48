"""The tuner levels of the decode (row a8: per stream class, the layout at
encode time, the first-level table bits, waves per workgroup and LDS
staging), each driven on the GPU: whatever they pick, the stream re-encoded
or re-tabled with it must decode exactly to the oracle's result."""
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
    yield


def _decode(ds, n, mode, tune):
    import torch
    from paper_2201_09118_amd import hd
    out = torch.full((n + 64,), -1, dtype=torch.int16, device="cuda")
    ws = hd.decode(ds, out, mode, tune)
    bits = hd.decode_status_bits(ws)
    return out[:n].cpu().numpy().view(np.uint16), bits, out[n:].cpu().numpy()


@pytest.mark.parametrize("mode", [0, 1])
def test_hd_autotune_pick_decodes_exactly(mode):
    import torch
    from paper_2201_09118_amd import hd
    x = hdsynth.two_sided_geometric(np.random.default_rng(90 + mode), 1_000_003, 0.55, 1024)
    case = make_case(x, 1024, 24, 128, 32)
    ds = upload(case, with_gap=(mode == 0))
    out = torch.empty(x.size, dtype=torch.int16, device="cuda")
    flush(f"hd_autotune mode={mode}")
    best, ms = hd.autotune(ds, out, mode=mode)
    assert ms > 0
    assert 1 <= best.waves_per_group <= 16
    assert 256 <= best.stage_symbols <= 16384 and best.stage_symbols % 64 == 0
    got, bits, tail = _decode(ds, x.size, mode, best)
    assert bits == 0 and np.array_equal(got, expected(case)) and (tail == -1).all()


def test_decode_params_k1_sweep_pick_decodes_exactly():
    from paper_2201_09118_amd import autotune, hd
    x = hdsynth.two_sided_geometric(np.random.default_rng(93), 800_001, 0.75, 4096)
    case = make_case(x, 4096, 24, 128, 32)
    hs = hd.encode_ref(x, case.lengths, case.codes, 24, 128, 32)
    tuner = autotune.Autotuner(lut_candidates=(9, 11, 12))
    flush("decode_params k1 sweep")
    k1, tune = tuner.decode_params(case.lengths, case.codes, 24, hs, 4096)
    assert k1 in (9, 11, 12)
    tab = hd.Table(case.lengths, case.codes, 24, k1)
    assert tab.lds_bytes >= 4 << k1
    ds = hd.DeviceStream.from_host(hs, tab)
    got, bits, tail = _decode(ds, x.size, hd.MODE_GAP, tune)
    assert bits == 0 and np.array_equal(got, expected(case)) and (tail == -1).all()
    assert tuner.decode_params(case.lengths, case.codes, 24, hs, 4096)[0] == k1      # cached


def test_choose_layout_pick_reencoded_decodes_exactly(tmp_path):
    from paper_2201_09118_amd import autotune, hd
    x = hdsynth.two_sided_geometric(np.random.default_rng(94), 600_000, 0.4, 256)
    ln = oracle.code_lengths(oracle.histogram(x, 256), 24)
    cd = oracle.canonical_codes(ln)
    path = str(tmp_path / "tune.json")
    tuner = autotune.Autotuner(path)
    flush("choose_layout")
    cands = ((128, 32), (256, 32), (64, 64))
    S, C = tuner.choose_layout(x, ln, cd, 24, 256, candidates=cands, sample=1 << 18)
    assert (S, C) in cands
    # re-encoded with the chosen layout by the oracle's encoder, decoded by the library
    case = make_case(x, 256, 24, S, C, ln, cd)
    for mode in (hd.MODE_GAP, hd.MODE_SELF_SYNC):
        ds = upload(case, with_gap=(mode == hd.MODE_GAP))
        got, bits, _ = _decode(ds, x.size, mode, None)
        assert bits == 0 and np.array_equal(got, oracle.decode(case.enc.words, case.enc.n_bits, x.size, ln, cd))
    # the cache persists and is read back
    tuner.save()
    again = autotune.Autotuner(path)
    assert again.choose_layout(x, ln, cd, 24, 256, candidates=cands, sample=1 << 18) == (S, C)
