"""GPU parity of the batched persistent decode: every stream of a batch --
each with its own alphabet, code-length limit, layout and table format --
must equal the oracle's decode, and the single-stream decode, bit for bit."""
import numpy as np
import pytest

import hdsynth
from hdcase import expected, flush, make_case, run_decode, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2201_09118_amd import hd  # noqa: F401
    yield


def _mixed_cases(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        n = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        A = int(rng.choice([2, 256, 1024, 4096, 20000]))
        r = float(rng.uniform(0.2, 0.8))
        S = int(rng.choice([64, 128, 256]))
        C = int(rng.choice([1, 8, 32, 64]))
        x = hdsynth.two_sided_geometric(rng, n, r, A)
        used = int((np.bincount(x, minlength=A) > 0).sum())
        L = max(int(np.ceil(np.log2(max(used, 2)))), int(rng.choice([12, 16, 24])))
        cases.append(make_case(x, A, L, S, C))
    return cases


def _run_batch(cases, tunes=None, lut_bits=None):
    import torch
    from paper_2201_09118_amd import hd
    dss = [upload(c, 0 if lut_bits is None else lut_bits[i]) for i, c in enumerate(cases)]
    outs = [torch.full((max(c.x.size, 8),), -1, dtype=torch.int16, device="cuda") for c in cases]
    ws = hd.decode_batch(dss, outs, hd.MODE_GAP, tunes)
    bits = hd.decode_status_bits(ws)
    return dss, [o[:c.x.size].cpu().numpy().view(np.uint16) for o, c in zip(outs, cases)], bits


def test_mixed_batch_matches_oracle():
    cases = _mixed_cases(41, 24, 1, 300_000)
    cases.append(make_case(np.zeros(0, np.uint16), 4, 2, 128, 32, np.array([1, 1, 0, 0], np.uint8),
                           np.array([0, 1, 0, 0], np.uint32)))
    flush(f"batch of {len(cases)} streams")
    dss, got, bits = _run_batch(cases)
    assert bits == 0, f"status {bits:#x}"
    for c, g in zip(cases, got):
        assert np.array_equal(g, expected(c))


def test_batch_equals_single_decodes_and_tunes():
    cases = _mixed_cases(42, 12, 1000, 500_000)
    rng = np.random.default_rng(1)
    luts = [int(v) for v in rng.choice([0, 8, 11, 12], len(cases))]
    for wpg in (4, 8):
        tunes = [{"waves_per_group": wpg, "stage_symbols": int(rng.choice([512, 1024, 2048, 4096]))}
                 for _ in cases]
        flush(f"batch wpg={wpg}")
        dss, got, bits = _run_batch(cases, tunes, luts)
        assert bits == 0
        for c, g, ds in zip(cases, got, dss):
            solo, sb = run_decode(ds)
            assert sb == 0
            assert np.array_equal(g, solo)
            assert np.array_equal(g, expected(c))


@pytest.mark.parametrize("shape", [(0, 0), (4, 1), (8, 2), (12, 0)])
def test_batch_staging_and_launch_shapes(shape):
    """Per-stream staging sizes (several multi-pass) in one launch whose waves
    per workgroup and workgroups per CU come from the first tune (0: the
    occupancy choice); tiny streams interleaved with large ones."""
    cases = _mixed_cases(45, 18, 1, 400_000)
    rng = np.random.default_rng(2)
    tunes = [{"stage_symbols": int(rng.choice([256, 512, 2048]))} for _ in cases]
    tunes[0].update(waves_per_group=shape[0], groups_per_cu=shape[1])
    flush(f"batch with launch shape {shape}")
    dss, got, bits = _run_batch(cases, tunes)
    assert bits == 0, f"status {bits:#x}"
    for c, g in zip(cases, got):
        assert np.array_equal(g, expected(c))


def test_batch_reports_corrupt_stream():
    from paper_2201_09118_amd import hd
    cases = _mixed_cases(43, 4, 10_000, 50_000)
    import torch
    dss = [upload(c) for c in cases]
    dss[2].chunk_offsets[1] += 1
    outs = [torch.zeros(c.x.size + 64, dtype=torch.int16, device="cuda") for c in cases]
    ws = hd.decode_batch(dss, outs)
    assert hd.decode_status(ws) == hd.ERR_CORRUPT
    for i in (0, 1, 3):
        assert np.array_equal(outs[i][:cases[i].x.size].cpu().numpy().view(np.uint16), expected(cases[i]))


def test_batch_rejects_selfsync_and_misaligned_output():
    import torch
    from paper_2201_09118_amd import hd
    cases = _mixed_cases(44, 2, 1000, 2000)
    dss = [upload(c) for c in cases]
    outs = [torch.zeros(c.x.size + 8, dtype=torch.int16, device="cuda") for c in cases]
    with pytest.raises(hd.HDError) as ei:
        hd.decode_batch(dss, outs, hd.MODE_SELF_SYNC, workspace=torch.zeros(1 << 20, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == hd.ERR_UNSUPPORTED
    with pytest.raises(hd.HDError) as ei:
        hd.decode_batch(dss, [outs[0], outs[1][1:]])
    assert ei.value.status == hd.ERR_ARG


def test_config4_shaped_batch_small():
    """The batched workload's recipe (log-uniform sizes, alphabets 256/1024/4096,
    r ~ U[0.2, 0.8], own codebooks, L = 24) at 1/256 of its sizes."""
    specs = hdsynth.batch_stream_specs(n_streams=64, lo=1 << 8, hi=1 << 18)
    cases = [make_case(hdsynth.batch_stream_symbols(sp), sp["A"], 24, 128, 32) for sp in specs]
    flush(f"config4-shaped batch: {sum(c.x.size for c in cases)} symbols")
    dss, got, bits = _run_batch(cases)
    assert bits == 0
    for c, g in zip(cases, got):
        assert np.array_equal(g, expected(c))


def test_autotuned_batch_launch_shape_decodes_exactly():
    import torch
    from paper_2201_09118_amd import autotune, hd
    specs = hdsynth.batch_stream_specs(n_streams=12, lo=1 << 10, hi=1 << 17)
    cases = [make_case(hdsynth.batch_stream_symbols(sp), sp["A"], 24, 64, 64) for sp in specs]
    dss = [upload(c) for c in cases]
    outs = [torch.full((max(c.x.size, 8),), -1, dtype=torch.int16, device="cuda") for c in cases]
    ws = hd.alloc_workspace(hd.decode_batch_workspace_size(dss))
    tuner = autotune.Autotuner()
    tunes = [hd.Tune(0, 1024, 0, 0) for _ in cases]
    keys = [autotune.class_key(sp["A"], c.x.size, c.enc.n_bits, 64) for sp, c in zip(specs, cases)]
    flush("batch launch autotune")
    shaped, options = tuner.batch_launch(dss, outs, tunes, ws, keys, reps=1)
    assert options and len(shaped) == len(cases)
    for o in outs:
        o.fill_(-1)
    hd.decode_batch(dss, outs, hd.MODE_GAP, shaped, ws)
    assert hd.decode_status_bits(ws) == 0
    for c, o in zip(cases, outs):
        assert np.array_equal(o[:c.x.size].cpu().numpy().view(np.uint16), expected(c))
    again, _ = tuner.batch_launch(dss, outs, tunes, ws, keys)       # cached
    assert [t.waves_per_group for t in again] == [t.waves_per_group for t in shaped]


def test_batch_with_streams_above_the_solo_threshold():
    """Streams of 2^23 symbols and more get their own decode launch inside
    hd_decode_batch; they are interleaved here with small streams (shared
    persistent launch), with per-stream staging given for some of them, and
    every output must equal the oracle's and the single-stream decode's."""
    rng = np.random.default_rng(47)
    sizes = [(1 << 23) + 5, 3000, (1 << 23) + 70_001, 17, 250_000, 5_000_000]
    cases = []
    for i, n in enumerate(sizes):
        A = [1024, 256, 4096, 2, 20000, 1024][i]
        x = hdsynth.two_sided_geometric(rng, n, float(rng.uniform(0.3, 0.8)), A)
        used = int((np.bincount(x, minlength=A) > 0).sum())
        L = max(int(np.ceil(np.log2(max(used, 2)))), 20)
        cases.append(make_case(x, A, L, [128, 64, 256, 128, 128, 64][i], [32, 8, 32, 1, 64, 64][i]))
    for tunes in (None, [{"stage_symbols": [0, 512, 2048, 0, 1024, 4096][i]} for i in range(len(cases))]):
        flush(f"batch with large streams, tunes={tunes is not None}")
        dss, got, bits = _run_batch(cases, tunes)
        assert bits == 0, f"status {bits:#x}"
        for c, g, ds in zip(cases, got, dss):
            assert np.array_equal(g, expected(c))


def test_batch_reports_a_fault_in_a_large_stream():
    """A gap byte off by one in a stream above the solo threshold: the batch's
    status word must carry the fault although that stream ran in its own launch."""
    rng = np.random.default_rng(48)
    big = make_case(hdsynth.two_sided_geometric(rng, (1 << 23) + 9, 0.6, 1024), 1024, 20, 128, 32)
    small = make_case(hdsynth.two_sided_geometric(rng, 30_000, 0.6, 1024), 1024, 20, 128, 32)
    import torch
    from paper_2201_09118_amd import hd
    dss = [upload(big), upload(small)]
    dss[0].gap[1000] += 1
    outs = [torch.zeros(c.x.size + 64, dtype=torch.int16, device="cuda") for c in (big, small)]
    ws = hd.decode_batch(dss, outs, hd.MODE_GAP)
    bits = hd.decode_status_bits(ws)
    assert bits != 0
    assert np.array_equal(outs[1][:small.x.size].cpu().numpy().view(np.uint16), expected(small))
