"""GPU tests of the continuous-batching decode server (hd_server_*).

Integer outputs: every served result must equal the same stream decoded
alone, bit for bit (tolerance 0), and the oracle's decode."""
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


def _pool(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        n = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        A = int(rng.choice([1024, 4096]))
        x = hdsynth.two_sided_geometric(rng, n, float(rng.uniform(0.2, 0.8)), A)
        cases.append(make_case(x, A, 24, 128, 32))
    return cases


def test_burst_results_identical_alone_and_in_mix():
    from paper_2201_09118_amd import hd, serve
    cases = _pool(61, 8, 2_000, 400_000)
    dss = [upload(c) for c in cases]
    solo = []
    for c, ds in zip(cases, dss):
        got, bits = run_decode(ds)
        assert bits == 0 and np.array_equal(got, expected(c))
        solo.append(got)
    server = hd.Server(256 << 20, n_streams=4, max_batch=16)
    times, which = serve.burst_schedule(64, len(cases))
    mismatches = []

    def check(i, ptr, n):
        if not np.array_equal(serve.copy_from_device(ptr, n), solo[which[i]]):
            mismatches.append(i)

    flush("burst of 64 requests")
    res = serve.run_served(server, dss, times, which, check)
    st = server.stats()
    server.close()
    assert not mismatches, mismatches
    assert res["requests"] == 64
    assert st["done"] == 64 and st["batches"] < 64        # requests shared batches
    assert st["arena_peak"] <= 256 << 20


def test_tight_budget_queues_but_completes():
    from paper_2201_09118_amd import hd, serve
    cases = _pool(62, 6, 100_000, 300_000)
    dss = [upload(c) for c in cases]
    biggest = max(c.x.size for c in cases) * 2
    budget = int(biggest * 1.6) + (1 << 20)                 # room for about one request at a time
    server = hd.Server(budget, n_streams=3, max_batch=8)
    times, which = serve.burst_schedule(24, len(cases))
    bad = []

    def check(i, ptr, n):
        if not np.array_equal(serve.copy_from_device(ptr, n), cases[which[i]].x):
            bad.append(i)

    res = serve.run_served(server, dss, times, which, check, defer=False)
    st = server.stats()
    assert not bad
    assert st["done"] == 24 and st["arena_peak"] <= budget
    # a request that can never fit is refused up front
    huge = _pool(63, 1, 2_000_000, 2_000_001)[0]
    with pytest.raises(hd.HDError) as ei:
        server.submit(upload(huge))
    assert ei.value.status == hd.ERR_NOMEM
    server.close()


def test_poisson_schedule_short():
    from paper_2201_09118_amd import hd, serve
    cases = _pool(64, 6, 10_000, 200_000)
    dss = [upload(c) for c in cases]
    server = hd.Server(128 << 20)
    times, which = serve.poisson_schedule(400.0, 60, len(cases))
    bad = []
    res = serve.run_served(server, dss, times, which,
                           lambda i, p, n: bad.append(i) if not np.array_equal(serve.copy_from_device(p, n),
                                                                                 cases[which[i]].x) else None)
    server.close()
    assert not bad
    assert np.isfinite(res["p50_ms"]) and res["p99_ms"] >= res["p50_ms"] > 0


def test_table_cache_hit_and_miss():
    from paper_2201_09118_amd import serve
    cases = _pool(65, 2, 1000, 2000)
    cache = serve.TableCache()
    a = cache.get(cases[0].lengths, cases[0].codes, 24)
    b = cache.get(cases[0].lengths, cases[0].codes, 24)
    c = cache.get(cases[1].lengths, cases[1].codes, 24)
    assert a is b and a is not c
    assert cache.hits == 1 and cache.misses == 2 and len(cache) == 2
