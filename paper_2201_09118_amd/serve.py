"""Serving driver: request schedules, a device-resident table cache, and the
two servers compared by the serving benchmark.

* ``run_served``: requests are submitted to the library's continuous-batching
  server (``hd.Server`` / ``hd_server_*``) at their scheduled arrival times;
  completions are polled and outputs released as they finish.
* ``run_serial``: a plain decode server fed the same schedule -- one
  ``hd_decode`` at a time, each waited for before the next starts.

Latency is completion time minus *scheduled* arrival time (a late submit
counts against the server).  Both clocks are the monotonic clock.
"""
from __future__ import annotations

import ctypes
import hashlib
import time

import numpy as np

from . import hd

_hip = None


def _hiprt():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def copy_from_device(ptr: int, n_symbols: int) -> np.ndarray:
    """Host copy of n uint16 symbols at a raw device pointer (server outputs)."""
    out = np.empty(n_symbols, np.uint16)
    if n_symbols:
        rc = _hiprt().hipMemcpy(out.ctypes.data, ptr, 2 * n_symbols, 2)   # hipMemcpyDeviceToHost
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed: {rc}")
    return out


class TableCache:
    """Device-resident decode tables keyed by a hash of the codebook."""

    def __init__(self):
        self._t = {}
        self.hits = 0
        self.misses = 0

    @staticmethod
    def key(lengths, codes, L, lut_bits=0) -> str:
        h = hashlib.sha1()
        h.update(np.ascontiguousarray(lengths, np.uint8).tobytes())
        h.update(np.ascontiguousarray(codes, np.uint32).tobytes())
        h.update(f"{L}/{lut_bits}".encode())
        return h.hexdigest()

    def get(self, lengths, codes, L, lut_bits=0) -> hd.Table:
        k = self.key(lengths, codes, L, lut_bits)
        t = self._t.get(k)
        if t is None:
            self.misses += 1
            t = hd.Table(lengths, codes, L, lut_bits)
            self._t[k] = t
        else:
            self.hits += 1
        return t

    def __len__(self):
        return len(self._t)


def poisson_schedule(rate: float, n_requests: int, n_pool: int, seed: int = 5):
    """Arrival offsets (s) of a Poisson process and the pool stream of each request."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    return np.cumsum(gaps) - gaps[0], rng.integers(0, n_pool, n_requests)


def burst_schedule(n_requests: int, n_pool: int, seed: int = 6):
    rng = np.random.default_rng(seed)
    return np.zeros(n_requests), rng.integers(0, n_pool, n_requests)


def _percentiles(lat):
    lat = np.asarray(lat)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def run_served(server: hd.Server, pool, times, which, check=None, check_every: int = 1, defer: bool = True):
    """Feeds the schedule to the server.  check(i, ptr, n) inspects the output
    of every check_every-th request: with defer, after the timed run (those
    outputs are held until then, so checking never delays the schedule; the
    budget must leave room for them), else as each completes."""
    n_req = len(times)
    start = time.perf_counter() + 0.01
    sched = start + np.asarray(times)
    lat = np.zeros(n_req)
    rid_to_i = {}
    held = []
    nxt = 0
    done = 0
    symbols = 0
    while done < n_req:
        now = time.perf_counter()
        while nxt < n_req and sched[nxt] <= now:
            rid_to_i[server.submit(pool[which[nxt]])] = nxt
            nxt += 1
        for rid in server.poll():
            i = rid_to_i.pop(rid)
            ptr, st, t_sub, t_done = server.result(rid)
            if st != hd.OK:
                raise RuntimeError(f"request {i} failed with status {st}")
            lat[i] = t_done - sched[i]
            n = pool[which[i]].n_symbols
            symbols += n
            if check is not None and i % check_every == 0:
                if defer:
                    held.append((i, rid, ptr, n))
                    done += 1
                    continue
                check(i, ptr, n)
            server.release(rid)
            done += 1
        if nxt < n_req:
            # sleep only while the next arrival is far off, then spin, so that
            # requests are submitted on time (as the serial server's loop does)
            wait = sched[nxt] - time.perf_counter()
            if wait > 2e-3:
                time.sleep(wait - 1e-3)
        elif done < n_req:
            time.sleep(1e-4)       # latency is stamped by the server, not by this poll
    wall = time.perf_counter() - start
    for i, rid, ptr, n in held:
        check(i, ptr, n)
        server.release(rid)
    p50, p99 = _percentiles(lat)
    return {"requests": n_req, "symbols": symbols, "wall_s": wall, "gbs": 2.0 * symbols / wall / 1e9,
            "p50_ms": p50 * 1e3, "p99_ms": p99 * 1e3, "latency_s": lat}


def run_serial(pool, times, which, outs, workspaces):
    """Plain decode server: one hd_decode at a time, each waited for."""
    import torch
    n_req = len(times)
    start = time.perf_counter() + 0.01
    sched = start + np.asarray(times)
    lat = np.zeros(n_req)
    symbols = 0
    for i in range(n_req):
        while time.perf_counter() < sched[i]:
            pass
        ds = pool[which[i]]
        hd.decode(ds, outs[which[i]], hd.MODE_GAP, None, workspaces[which[i]])
        torch.cuda.synchronize()
        lat[i] = time.perf_counter() - sched[i]
        symbols += ds.n_symbols
    wall = time.perf_counter() - start
    p50, p99 = _percentiles(lat)
    return {"requests": n_req, "symbols": symbols, "wall_s": wall, "gbs": 2.0 * symbols / wall / 1e9,
            "p50_ms": p50 * 1e3, "p99_ms": p99 * 1e3, "latency_s": lat}
