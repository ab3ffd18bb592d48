"""GPU parity of hd_lorenzo_reconstruct (SZ-style reconstruction after decode)
against the reconstruction oracle (oracle/sz.py).

Integer results (q) are compared bit for bit (tolerance 0).  The float32 values
are compared bit for bit too: both sides form the float64 product q * 2 eb and
round it once to float32, so IEEE arithmetic fixes every bit."""
import numpy as np
import pytest

import hdsynth
from conftest import load_golden
from hdcase import flush, make_case, upload
from oracle import sz

pytestmark = pytest.mark.gpu

ERR_NO_OUTLIER = 1 << 7


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2201_09118_amd import hd  # noqa: F401
    yield


def _run(codes, shape, radius, oidx, oval, eb, want_q=True):
    """Uploads, reconstructs on the device, returns (q, x, status bits)."""
    import torch
    from paper_2201_09118_amd import hd
    n = int(np.prod(shape))
    c = torch.from_numpy(np.ascontiguousarray(codes, np.uint16).view(np.int16)).cuda()
    oi = torch.from_numpy(np.ascontiguousarray(oidx, np.uint64).view(np.int64)).cuda() if len(oidx) else None
    ov = torch.from_numpy(np.ascontiguousarray(oval, np.int32)).cuda() if len(oval) else None
    out = torch.full((max(n, 1),), float("nan"), dtype=torch.float32, device="cuda")
    q = torch.full((max(n, 1),), 0x5A5A5A5A, dtype=torch.int32, device="cuda") if want_q else None
    ws = hd.lorenzo_reconstruct(c, shape, radius, oi, ov, eb, out, q)
    bits = hd.decode_status_bits(ws)
    torch.cuda.synchronize()
    qh = q[:n].cpu().numpy() if want_q else None
    return qh, out[:n].cpu().numpy(), bits


def _check_field(F, tag):
    flush(f"lorenzo {tag}: shape {F.shape}, {F.outlier_idx.size} outliers")
    q_ref, x_ref = sz.reconstruct(F.codes, F.shape, F.radius, F.outlier_idx, F.outlier_val, F.eb)
    q, x, bits = _run(F.codes, F.shape, F.radius, F.outlier_idx, F.outlier_val, F.eb)
    assert bits == 0
    assert np.array_equal(q, q_ref.reshape(-1).astype(np.int32)), tag
    assert np.array_equal(x.view(np.uint32), x_ref.reshape(-1).view(np.uint32)), tag


def test_hand_worked_2x2x2():
    g = load_golden("lorenzo_2x2x2.txt")
    idx, val = (int(v) for v in g["outlier"][0])
    q, x, bits = _run(np.array([int(v) for v in g["codes"][0]], np.uint16), (2, 2, 2), 512,
                      np.array([idx], np.uint64), np.array([val], np.int32), 0.25)
    assert bits == 0
    assert q.tolist() == [int(v) for v in g["q"][0]]
    assert x.tolist() == [float(v) for v in g["value"][0]]


# shapes span several wavefront row blocks, ragged row lengths (scalar path),
# 1-8 chunks of 512 along k, plane counts off the unroll of 8, and 2-D / 1-D fields
SHAPES = [(3, 37, 100), (4, 65, 512), (2, 33, 1030), (2, 40, 1032), (1, 70, 4096), (1, 1, 3000),
          (5, 1, 64), (130, 9, 24), (9, 300, 16), (17, 47, 777), (1, 1, 1), (2, 3, 5)]


def _more_outliers(F, frac, seed):
    """The same field with a random fraction of its in-band codes moved to the
    outlier list (code 0, residual code - radius): q is unchanged."""
    rng = np.random.default_rng(seed)
    pick = np.flatnonzero((rng.random(F.codes.size) < frac) & (F.codes != 0))
    codes = F.codes.copy()
    vals = codes[pick].astype(np.int64) - F.radius
    codes[pick] = 0
    idx = np.concatenate([F.outlier_idx, pick.astype(np.uint64)])
    val = np.concatenate([F.outlier_val, vals.astype(np.int32)])
    order = np.argsort(idx, kind="stable")
    return hdsynth.LorenzoField(F.shape, F.eb, F.radius, codes, idx[order], val[order], F.field)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_generator_fields(shape):
    F = hdsynth.lorenzo_field(shape, seed=sum(shape), n_waves=2, noise_sigma=1e-3, eb=1e-3, radius=512)
    _check_field(_more_outliers(F, 0.02, sum(shape)), "mixed")


@pytest.mark.parametrize("n", [4097, 8192, 100_003, (1 << 20) + 7, 5_000_011])
def test_long_1d_fields(n):
    # ni = nj = 1 beyond one wavefront's row: reduce-then-scan over tiles
    F = hdsynth.lorenzo_field((1, 1, n), seed=n % 97, n_waves=2, noise_sigma=1e-3, eb=1e-3, radius=512)
    _check_field(_more_outliers(F, 0.01, n), "1-D")


def test_long_1d_unaligned_codes():
    import torch
    from paper_2201_09118_amd import hd
    F = hdsynth.lorenzo_field((1, 1, 50_001), seed=7, n_waves=2, noise_sigma=1e-3, eb=1e-3, radius=512)
    F = _more_outliers(F, 0.02, 7)
    q_ref, x_ref = sz.reconstruct(F.codes, F.shape, F.radius, F.outlier_idx, F.outlier_val, F.eb)
    buf = torch.from_numpy(np.concatenate([[0], F.codes]).astype(np.uint16).view(np.int16)).cuda()
    out = torch.empty(F.codes.size, dtype=torch.float32, device="cuda")
    q = torch.empty(F.codes.size, dtype=torch.int32, device="cuda")
    oi = torch.from_numpy(F.outlier_idx.view(np.int64)).cuda()
    ov = torch.from_numpy(F.outlier_val).cuda()
    ws = hd.lorenzo_reconstruct(buf[1:], F.shape, F.radius, oi, ov, F.eb, out, q)
    assert hd.decode_status_bits(ws) == 0
    assert np.array_equal(q.cpu().numpy(), q_ref.reshape(-1))
    assert np.array_equal(out.cpu().numpy().view(np.uint32), x_ref.reshape(-1).view(np.uint32))


def test_every_code_an_outlier():
    F = hdsynth.lorenzo_field((6, 50, 136), seed=8, n_waves=4, noise_sigma=1e-2, eb=1e-4, radius=4)
    assert F.outlier_idx.size > 0.95 * F.codes.size
    _check_field(F, "all outliers")


def test_no_outliers():
    F = hdsynth.lorenzo_field((6, 64, 256), seed=9, n_waves=1, noise_sigma=1e-4, eb=1e-2, radius=512)
    assert F.outlier_idx.size == 0
    _check_field(F, "no outliers")


def test_random_residuals_wrap_modulo_2_32():
    # residuals anywhere in int32: partial sums overflow; q must still agree
    # with the exact box sums modulo 2^32
    rng = np.random.default_rng(21)
    shape = (11, 70, 264)
    n = int(np.prod(shape))
    codes = rng.integers(1, 1 << 16, size=n).astype(np.uint16)
    zero = rng.random(n) < 0.3
    codes[zero] = 0
    oidx = np.flatnonzero(zero).astype(np.uint64)
    oval = rng.integers(-(1 << 31), 1 << 31, size=oidx.size, dtype=np.int64).astype(np.int32)
    q_ref = sz.inverse_lorenzo(sz.residuals(codes, 1000, oidx, oval), shape).reshape(-1)
    q, _, bits = _run(codes, shape, 1000, oidx, oval, 1e-4)
    assert bits == 0
    assert np.array_equal(q.view(np.uint32), (q_ref & 0xFFFFFFFF).astype(np.uint32))


def test_outlier_list_entries_off_code_zero_ignored():
    F = hdsynth.lorenzo_field((3, 20, 40), seed=10, n_waves=2, noise_sigma=1e-3, eb=1e-3, radius=512)
    extra = np.setdiff1d(np.arange(0, F.codes.size, 7, dtype=np.uint64), F.outlier_idx)
    oidx = np.concatenate([F.outlier_idx, extra])
    oval = np.concatenate([F.outlier_val, np.full(extra.size, 123456, np.int32)])
    order = np.argsort(oidx)
    q_ref, x_ref = sz.reconstruct(F.codes, F.shape, F.radius, F.outlier_idx, F.outlier_val, F.eb)
    q, x, bits = _run(F.codes, F.shape, F.radius, oidx[order], oval[order], F.eb)
    assert bits == 0 and np.array_equal(q, q_ref.reshape(-1))


def test_missing_outlier_flags_status_and_next_call_clears_it():
    from paper_2201_09118_amd import hd
    F = hdsynth.lorenzo_field((4, 30, 72), seed=11, n_waves=2, noise_sigma=1e-3, eb=1e-3, radius=64)
    assert F.outlier_idx.size > 2
    _, _, bits = _run(F.codes, F.shape, F.radius, F.outlier_idx[1:], F.outlier_val[1:], F.eb)
    assert bits == ERR_NO_OUTLIER
    _check_field(F, "after a flagged call")
    assert hd.status_str(hd.ERR_CORRUPT)


def test_empty_fields_only_clear_status():
    for shape in [(0, 5, 5), (3, 0, 8), (2, 2, 0)]:
        q, x, bits = _run(np.zeros(0, np.uint16), shape, 512, [], [], 1e-4)
        assert bits == 0 and q.size == 0 and x.size == 0


def test_argument_errors():
    import torch
    from paper_2201_09118_amd import hd
    c = torch.zeros(64, dtype=torch.int16, device="cuda")
    out = torch.zeros(64, dtype=torch.float32, device="cuda")
    ws = hd.alloc_workspace(hd.lorenzo_workspace_size((1, 1, 64)))
    for kw, st in [(dict(radius=0), hd.ERR_ARG), (dict(eb=0.0), hd.ERR_ARG), (dict(eb=float("inf")), hd.ERR_ARG),
                   (dict(shape=(2, 1, 8192)), hd.ERR_UNSUPPORTED)]:
        args = dict(shape=(1, 1, 64), radius=512, eb=1e-4)
        args.update(kw)
        with pytest.raises(hd.HDError) as ei:
            hd.lorenzo_reconstruct(c, args["shape"], args["radius"], None, None, args["eb"], out, None,
                                   ws if "shape" not in kw else None)
        assert ei.value.status == st
    short = hd.alloc_workspace(16)
    assert hd.lorenzo_workspace_size((64, 64, 64)) > short.numel()
    c2 = torch.zeros(64 ** 3, dtype=torch.int16, device="cuda")
    o2 = torch.zeros(64 ** 3, dtype=torch.float32, device="cuda")
    with pytest.raises(hd.HDError) as ei:
        hd.lorenzo_reconstruct(c2, (64, 64, 64), 512, None, None, 1e-4, o2, None, short)
    assert ei.value.status == hd.ERR_ARG


def test_decode_then_reconstruct_end_to_end():
    import torch
    from paper_2201_09118_amd import hd
    F = hdsynth.lorenzo_field((40, 96, 128), seed=12, n_waves=3, noise_sigma=1e-3, eb=2e-4, radius=512,
                              keep_field=True)
    flush(f"decode + reconstruct (40, 96, 128): {F.outlier_idx.size} outliers")
    case = make_case(F.codes, 1024, 24, 128, 32)
    ds = upload(case)
    codes = torch.empty(F.codes.size, dtype=torch.int16, device="cuda")
    ws = hd.decode(ds, codes, hd.MODE_GAP)
    assert hd.decode_status_bits(ws) == 0
    out = torch.empty(F.codes.size, dtype=torch.float32, device="cuda")
    oi = torch.from_numpy(F.outlier_idx.view(np.int64)).cuda()
    ov = torch.from_numpy(F.outlier_val).cuda()
    ws2 = hd.lorenzo_reconstruct(codes, F.shape, F.radius, oi, ov, F.eb, out)
    assert hd.decode_status_bits(ws2) == 0
    x = out.cpu().numpy()
    _, x_ref = sz.reconstruct(F.codes, F.shape, F.radius, F.outlier_idx, F.outlier_val, F.eb)
    assert np.array_equal(x.view(np.uint32), x_ref.reshape(-1).view(np.uint32))
    f = F.field.reshape(-1).astype(np.float64)
    assert (np.abs(x.astype(np.float64) - f) <= F.eb * (1 + 1e-9) + 2 * np.spacing(np.abs(F.field.reshape(-1)))).all()


def test_config2_field_full_size():
    # the 512^3 field of the decode benchmark, bit-exact against the oracle,
    # and within the error bound of the original data
    F = hdsynth.config2_field(keep_field=True)
    _check_field(F, "512^3")
    _, x, _ = _run(F.codes, F.shape, F.radius, F.outlier_idx, F.outlier_val, F.eb, want_q=False)
    err = np.abs(x.astype(np.float64) - F.field.reshape(-1).astype(np.float64))
    assert err.max() <= F.eb * (1 + 1e-9) + 2 * float(np.spacing(np.abs(F.field).max()))
