"""GPU parity of the 1- and 4-byte symbol widths against the oracle.

The decoders the paper starts from took one-byte symbols; it adapts them to
multi-byte quantization codes (Sec. IV) and notes that the method applies to
double-precision data (Sec. V-A-3), whose codes can need more than 16 bits.
The same kernels decode every width; the width fixes the staging and output
element type.  Integer work: every comparison is bit-exact."""
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


def _check(case, ds=None, mode=0, tune=None, lut_bits=0):
    ds = ds or upload(case, lut_bits)
    got, bits = run_decode(ds, mode, tune)
    want = expected(case)
    assert want.dtype == case.x.dtype and np.array_equal(want, case.x)
    assert bits == 0, f"status bits {bits:#x}"
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{bad.size} mismatches, first at {bad[:8]}: got {got[bad[:8]]} want {want[bad[:8]]}")


def _cases(dtype):
    rng = np.random.default_rng(4040 + np.dtype(dtype).itemsize)
    Ss = [32, 64, 128, 256, 512]
    Cs = [1, 2, 4, 8, 16, 32, 64]
    ns = [1, 15, 16, 17, 63, 64, 65, 777, 4099, 54321, 300_001]
    if dtype == np.uint8:
        As = [2, 3, 17, 200, 256]
    else:
        As = [2, 256, 4096, 65536, 1 << 18, 1 << 24]
    out = []
    for i in range(24):
        S, C, n = Ss[i % len(Ss)], Cs[(i // 2) % len(Cs)], ns[i % len(ns)]
        A = int(As[i % len(As)])
        r = float(rng.uniform(0.3, 0.999 if A > 4096 else 0.95))
        lut = int(rng.choice([0, 6, 9, 12, 14]))
        out.append((i, S, C, n, A, r, lut))
    return out


def _run_case(dtype, case, modes=(0, 1)):
    i, S, C, n, A, r, lut = case
    rng = np.random.default_rng(9000 + i)
    x = hdsynth.two_sided_geometric(rng, n, r, A, dtype=dtype)
    used = int(np.unique(x).size)
    L = max(24, int(np.ceil(np.log2(max(used, 2)))))
    c = make_case(x, A, min(L, 32), S, C)
    ds = upload(c, lut)
    for mode in modes:
        flush(f"width={np.dtype(dtype).itemsize} case {case} mode={mode}")
        _check(c, ds, mode=mode)


@pytest.mark.parametrize("case", _cases(np.uint8), ids=lambda c: f"u8-i{c[0]}-S{c[1]}-C{c[2]}-n{c[3]}-A{c[4]}")
def test_random_streams_u8(case):
    _run_case(np.uint8, case)


@pytest.mark.parametrize("case", _cases(np.uint32), ids=lambda c: f"u32-i{c[0]}-S{c[1]}-C{c[2]}-n{c[3]}-A{c[4]}")
def test_random_streams_u32(case):
    _run_case(np.uint32, case)


def test_u8_multi_pass_staging_and_ragged_groups():
    """One-bit codes (128 symbols per subsequence) force several staging
    passes; a 16-symbol output group makes the head and tail partial groups
    span up to 15 symbols."""
    rng = np.random.default_rng(41)
    x = rng.integers(0, 2, 500_003).astype(np.uint8)
    case = make_case(x, 2, 8, 128, 32)
    ds = upload(case)
    for stage in (256, 512, 2048, 8192):
        for mode in (0, 1):
            flush(f"u8 one-bit codes stage={stage} mode={mode}")
            _check(case, ds, mode=mode, tune={"stage_symbols": stage})


def test_u32_long_codes_above_first_level():
    """Wide alphabet whose used symbols all sit above 2^16 and whose codes are
    mostly longer than a 9-bit first level (per-length limits + symbol list)."""
    rng = np.random.default_rng(42)
    A = 1 << 20
    x = hdsynth.two_sided_geometric(rng, 400_000, 0.995, A, centre=(1 << 19) + 77, dtype=np.uint32)
    assert x.min() > 65535
    case = make_case(x, A, 27, 256, 32)
    assert case.lengths[case.lengths > 0].min() > 6
    for lut in (6, 9, 11):
        for mode in (0, 1):
            flush(f"u32 long codes lut={lut} mode={mode}")
            _check(case, lut_bits=lut, mode=mode)


def test_width_argument_errors():
    import torch
    from paper_2201_09118_amd import hd
    rng = np.random.default_rng(43)
    x = hdsynth.two_sided_geometric(rng, 10_000, 0.5, 1024, dtype=np.uint32)
    case = make_case(x, 1024, 16, 128, 32)
    ds = upload(case)
    out16 = torch.zeros(x.size, dtype=torch.int16, device="cuda")
    with pytest.raises(ValueError):
        hd.decode(ds, out16)                 # the binding refuses a narrower output tensor
    # the library refuses an alphabet that does not fit the declared width
    ds.info.symbol_bytes = 1
    out8 = torch.zeros(x.size, dtype=torch.uint8, device="cuda")
    with pytest.raises(hd.HDError) as ei:
        hd.decode(ds, out8)
    assert ei.value.status == hd.ERR_ARG
    ds.info.symbol_bytes = 3
    with pytest.raises(hd.HDError) as ei:
        hd.decode_workspace_size(ds)
    assert ei.value.status == hd.ERR_ARG
    # batched decode takes 2-byte symbols only
    ds.info.symbol_bytes = 4
    with pytest.raises(hd.HDError) as ei:
        hd.decode_batch_workspace_size([ds])
    assert ei.value.status == hd.ERR_UNSUPPORTED


@pytest.mark.slow
def test_config2_u8_full():
    flush("config2 u8: 512^3 Lorenzo codes, radius 128, A=256 L=24 S=128 C=32")
    x = hdsynth.config2_symbols_u8()
    case = make_case(x, 256, 24, 128, 32)
    flush(f"u8 encoded: B={case.enc.n_bits} lbar={case.enc.n_bits / x.size:.3f}")
    ds = upload(case)
    for mode in (0, 1):
        _check(case, ds, mode=mode)


@pytest.mark.slow
def test_config2_u32_full():
    flush("config2 u32: 512^3 Lorenzo codes, eb 1e-6, radius 2^17, A=2^18 L=24 S=128 C=32")
    x = hdsynth.config2_symbols_u32()
    case = make_case(x, 1 << 18, 24, 128, 32)
    flush(f"u32 encoded: B={case.enc.n_bits} lbar={case.enc.n_bits / x.size:.3f}")
    ds = upload(case)
    for mode in (0, 1):
        _check(case, ds, mode=mode)
