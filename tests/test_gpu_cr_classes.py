"""The paper's Algorithm 2 (Sec. IV-C) as built by hd_decode_cr_classes:
tiles classified by compression ratio, histogrammed and sorted on the device,
one launch per class on separate streams.  Bit-exact against the oracle."""
import numpy as np
import pytest

import hdsynth
from hdcase import expected, flush, make_case, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    yield


def _mixed(seed, n_seg=12, seg=120_000, A=1024):
    rng = np.random.default_rng(seed)
    parts = [hdsynth.two_sided_geometric(rng, int(rng.integers(seg // 2, seg * 2)), float(r), A)
             for r in rng.uniform(0.05, 0.95, n_seg)]
    return np.concatenate(parts)


def _run(case, ds=None):
    import torch
    from paper_2201_09118_amd import hd
    ds = ds or upload(case)
    n = case.x.size
    out = torch.full((n + 64,), -1, dtype=torch.int16, device="cuda")
    ws, rep = hd.decode_cr_classes(ds, out)
    bits = hd.decode_status_bits(ws)
    h = out.cpu().numpy()
    return h[:n].view(np.uint16), bits, h[n:], rep


@pytest.mark.parametrize("S,C,A,L", [(128, 32, 1024, 24), (256, 32, 4096, 27), (64, 64, 256, 16), (32, 2, 70000 // 2, 24)])
def test_cr_classes_decode_exactly(S, C, A, L):
    x = _mixed(S + C, A=A)
    case = make_case(x, A, L, S, C)
    flush(f"cr classes S={S} C={C} A={A}: n={x.size}")
    got, bits, tail, rep = _run(case)
    ntiles = (case.enc.gap.size + 63) // 64
    assert bits == 0 and np.array_equal(got, expected(case)) and (tail == -1).all()
    assert sum(v["tiles"] for v in rep["classes"].values()) == ntiles
    assert 1 <= rep["t_high"] <= 16 and rep["launches"] == len(rep["classes"])
    assert all(1 <= c <= rep["t_high"] + 1 for c in rep["classes"])


def test_cr_classes_use_several_classes_and_report_corruption():
    x = _mixed(5, n_seg=20)
    case = make_case(x, 1024, 24, 128, 32)
    got, bits, _, rep = _run(case)
    assert bits == 0 and np.array_equal(got, expected(case))
    assert len(rep["classes"]) >= 3            # the segments span several ratio classes
    ds = upload(case)
    ds.chunk_offsets[-1] += 1
    _, bits, _, _ = _run(case, ds)
    assert bits & (1 << 4)
    ds = upload(case)
    ds.chunk_offsets[7] -= 1
    _, bits, _, _ = _run(case, ds)
    assert bits != 0


def test_cr_classes_empty_and_tiny():
    for n in (0, 1, 65):
        x = np.arange(n, dtype=np.uint16) % 3
        case = make_case(x, 3, 4, 128, 32)
        got, bits, tail, rep = _run(case)
        assert bits == 0 and np.array_equal(got, expected(case)) and (tail == -1).all()
