"""GPU parity of the device codebook builder (hd_build_codebook_device)
against the oracle's package-merge + canonical codes and the host builder.

Byte outputs: lengths and codes must equal the oracle's exactly.  Cases are
the code-length pins of the oracle (brute-force-sized alphabets, ties, dyadic
and equiprobable counts, Fibonacci counts where the limit binds, one and two
symbols) plus random histograms up to the builder's 4096 used symbols, and
the data-dependent failures it reports through the status word."""
import numpy as np
import pytest

import hdsynth
import oracle
from hdcase import flush

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2201_09118_amd import hd  # noqa: F401
    yield


def _device_book(cnt, L, ws=None):
    import torch
    from paper_2201_09118_amd import hd
    h = torch.from_numpy(np.ascontiguousarray(cnt, dtype=np.uint64).view(np.int64)).cuda()
    ln, cd, ws = hd.build_codebook_device(h, L, workspace=ws)
    bits = hd.decode_status_bits(ws)
    torch.cuda.synchronize()
    return ln.cpu().numpy(), cd.cpu().numpy().view(np.uint32), bits


def _check(cnt, L, tag):
    from paper_2201_09118_amd import hd
    flush(f"codebook {tag}: A={cnt.size} used={int((cnt > 0).sum())} L={L}")
    want_ln = oracle.code_lengths(cnt, L)
    want_cd = oracle.canonical_codes(want_ln)
    host_ln, host_cd = hd.build_codebook(cnt, L)
    ln, cd, bits = _device_book(cnt, L)
    assert bits == 0, f"{tag}: status {bits:#x}"
    assert np.array_equal(host_ln, want_ln) and np.array_equal(host_cd, want_cd), tag
    assert np.array_equal(ln, want_ln), f"{tag}: lengths differ at {np.flatnonzero(ln != want_ln)[:8]}"
    assert np.array_equal(cd, want_cd), f"{tag}: codes differ at {np.flatnonzero(cd != want_cd)[:8]}"


def test_small_alphabets_and_ties():
    rng = np.random.default_rng(51)
    for trial in range(60):
        A = int(rng.integers(2, 9))
        cnt = rng.integers(0, 6, A).astype(np.uint64)          # many equal counts: the tie rule decides
        if (cnt > 0).sum() < 2:
            cnt[:2] = [1, 1]
        L = int(rng.integers(int(np.ceil(np.log2((cnt > 0).sum()))), 8))
        _check(cnt, max(L, 1), f"small{trial}")


def test_special_counts():
    _check(np.array([8, 4, 2, 1, 1], np.uint64), 8, "dyadic")
    _check(np.full(256, 7, np.uint64), 8, "equiprobable-256")
    _check(np.full(256, 7, np.uint64), 12, "equiprobable-256-loose")
    fib = [1, 1]
    while len(fib) < 30:
        fib.append(fib[-1] + fib[-2])
    for L in (27, 20, 12, 5):
        _check(np.array(fib, np.uint64), L, f"fibonacci-L{L}")
    _check(np.array([0, 5, 0, 0], np.uint64), 4, "one-symbol")
    _check(np.array([0, 0, 0], np.uint64), 4, "empty")
    _check(np.array([3, 9], np.uint64), 1, "two-symbols-L1")
    _check(np.array([0] * 100 + [1, 1] + [0] * 50, np.uint64), 32, "two-symbols-L32")


@pytest.mark.parametrize("A,used,L", [(1024, 400, 24), (1024, 1024, 16), (4096, 4096, 24), (65536, 4096, 27),
                                      (65536, 3000, 12), (4096, 2000, 32)])
def test_random_histograms(A, used, L):
    rng = np.random.default_rng(A + used + L)
    for trial in range(4):
        cnt = np.zeros(A, np.uint64)
        pos = rng.choice(A, used, replace=False)
        kind = trial % 4
        if kind == 0:
            cnt[pos] = rng.integers(1, 1 << 20, used)
        elif kind == 1:
            cnt[pos] = np.floor(np.exp(rng.uniform(0, 27, used))).astype(np.uint64) + 1   # heavy spread
        elif kind == 2:
            cnt[pos] = rng.integers(1, 4, used)                                       # ties everywhere
        else:
            g = hdsynth.two_sided_geometric(rng, 2_000_000, 0.9, A)
            cnt = np.bincount(g, minlength=A).astype(np.uint64)
            if (cnt > 0).sum() > (1 << L):
                continue
        _check(cnt, L, f"random A={A} used={used} L={L} kind={kind}")


def test_histogram_of_config2_codes():
    """The codebook of the headline stream: device histogram -> device codebook."""
    import torch
    from paper_2201_09118_amd import hd
    x = hdsynth.lorenzo_field_codes((128, 128, 128), seed=2)
    xs = torch.from_numpy(x.view(np.int16)).cuda()
    h = hd.histogram(xs, 1024)
    ln, cd, ws = hd.build_codebook_device(h, 24)
    assert hd.decode_status_bits(ws) == 0
    want_ln = oracle.code_lengths(oracle.histogram(x, 1024), 24)
    assert np.array_equal(ln.cpu().numpy(), want_ln)
    assert np.array_equal(cd.cpu().numpy().view(np.uint32), oracle.canonical_codes(want_ln))


def test_reported_failures():
    from paper_2201_09118_amd import hd
    ws = hd.alloc_workspace(int(hd.lib().hd_codebook_workspace_size(32)))
    # more used symbols than 2^L codewords
    ln, cd, bits = _device_book(np.ones(9, np.uint64), 3, ws)
    assert bits & (1 << 8) and not ln.any() and not cd.any()
    # more used symbols than one workgroup ranks
    ln, cd, bits = _device_book(np.ones(5000, np.uint64), 24, ws)
    assert bits & (1 << 9) and not ln.any()
    # a count of 2^40
    cnt = np.ones(8, np.uint64)
    cnt[3] = 1 << 40
    ln, cd, bits = _device_book(cnt, 8, ws)
    assert bits & (1 << 10) and not ln.any()
    # the same workspace then builds a clean codebook and reports nothing
    cnt = np.array([5, 3, 2, 1], np.uint64)
    ln, cd, bits = _device_book(cnt, 4, ws)
    assert bits == 0
    want = oracle.code_lengths(cnt, 4)
    assert np.array_equal(ln, want) and np.array_equal(cd, oracle.canonical_codes(want))
