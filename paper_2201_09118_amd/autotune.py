"""Per-stream-class tuning of layout and decode parameters.

The paper re-tunes the shared-memory buffer on every decode call from each
sequence's compression ratio (Sec. IV-C, Alg. 2) at a cost of ~220 us per
call (Table I).  Here tuning happens once per *stream class* and is cached:

* encode-time layout: the subsequence length S and chunk size C of a class
  are chosen by encoding a sample with each candidate layout and timing its
  tuned decode (time per symbol);
* decode time: waves per workgroup and LDS staging size come from
  ``hd_autotune`` (a measured sweep in the library); the first-level table
  size (LDS table budget) is swept here by building tables of several widths;
* batched launch: the one launch's waves per workgroup and staging cap are
  measured on the batch itself (per set of classes).

A class is (alphabet bucket, mean code length in half bits, S); results are
keyed additionally by the GPU architecture and can be persisted as JSON.
Callers should tune a class on one of its larger streams (tiny streams are
launch-bound and say little about the kernel).  Every measurement runs the library's kernels.
"""
from __future__ import annotations

import json
import math
import os
import threading

import numpy as np

from . import hd

ALPHABET_BUCKETS = (256, 1024, 4096, 65536)


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", None) or p.name


def class_key(A: int, n_symbols: int, n_bits: int, S: int | None = None) -> str:
    """Stream class: alphabet bucket, mean code length to half a bit, and S."""
    ab = next(b for b in ALPHABET_BUCKETS if A <= b) if A <= ALPHABET_BUCKETS[-1] else A
    lbar = n_bits / max(n_symbols, 1)
    lb = round(lbar * 2) / 2
    return f"A{ab}-l{lb:.1f}" + (f"-S{S}" if S else "")


class Autotuner:
    """Caches tuned parameters per stream class (and per GPU architecture)."""

    def __init__(self, path: str | None = None, lut_candidates=(10, 11, 12)):
        self.path = path
        self.lut_candidates = tuple(lut_candidates)
        self._mu = threading.Lock()
        self.cache: dict = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    def save(self):
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)

    def _key(self, k: str) -> str:
        return f"{_arch()}/{k}"

    # -- decode parameters -------------------------------------------------

    def decode_params(self, lengths, codes, L, hs: hd.HostStream, A: int):
        """(lut_bits, Tune) for a host-encoded stream of this class, measured once."""
        import torch
        key = self._key("dec-" + class_key(A, hs.n_symbols, hs.n_bits, int(hs.info.subseq_bits)))
        with self._mu:
            hit = self.cache.get(key)
        if hit:
            return hit["lut_bits"], hd.Tune(hit["wpg"], hit["stage"], 0, 0)
        best = None
        out = torch.empty(max(hs.n_symbols, 8), dtype=torch.int16, device="cuda")
        for k1 in self.lut_candidates:
            tab = hd.Table(lengths, codes, L, k1)
            ds = hd.DeviceStream.from_host(hs, tab)
            t, ms = hd.autotune(ds, out)
            if best is None or ms < best[0]:
                best = (ms, k1, t.waves_per_group, t.stage_symbols)
            tab.close()
        ms, k1, wpg, stage = best
        with self._mu:
            self.cache[key] = {"lut_bits": int(k1), "wpg": int(wpg), "stage": int(stage), "ms": ms,
                               "n": hs.n_symbols}
        return k1, hd.Tune(wpg, stage, 0, 0)

    # -- batch launch shape ----------------------------------------------------

    def batch_launch(self, streams, outs, tunes, workspace, class_keys, reps: int = 3):
        """Shape of one batched launch, measured on this batch: waves per
        workgroup (0 = the library's occupancy choice) times a cap on the
        staging the launch reserves (streams above the cap decode in passes).
        Returns (per-stream tunes with the chosen shape, {option: ms})."""
        import torch
        key = self._key("batch-" + ",".join(sorted(set(class_keys))))
        smax = max(t.stage_symbols for t in tunes)
        with self._mu:
            hit = self.cache.get(key)

        def shaped(w, cap):
            return [hd.Tune(w if i == 0 else 0, min(t.stage_symbols, cap), 0, 0) for i, t in enumerate(tunes)]

        if hit:
            return shaped(hit["wpg"], hit["stage_cap"]), hit["options"]
        options = {}
        best = None
        for f in (1.0, 0.75, 0.5):
            cap = max(256, int(smax * f) // 64 * 64)
            for w in (0, 4, 8, 12, 16):
                tu = shaped(w, cap)
                try:
                    hd.decode_batch(streams, outs, hd.MODE_GAP, tu, workspace)
                except hd.HDError:
                    continue                      # layout above a workgroup's LDS
                torch.cuda.synchronize()
                ts = []
                for _ in range(reps):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    hd.decode_batch(streams, outs, hd.MODE_GAP, tu, workspace)
                    b.record()
                    torch.cuda.synchronize()
                    ts.append(a.elapsed_time(b))
                ms = float(np.median(ts))
                options[f"wpg{w}-cap{cap}"] = round(ms, 4)
                if best is None or ms < best[0]:
                    best = (ms, w, cap)
        if best is None:
            raise RuntimeError("no batch launch shape fits")
        with self._mu:
            self.cache[key] = {"wpg": best[1], "stage_cap": best[2], "ms": best[0], "options": options}
        return shaped(best[1], best[2]), options

    # -- encode-time layout --------------------------------------------------

    def choose_layout(self, x: np.ndarray, lengths, codes, L, A: int,
                      candidates=((128, 32), (256, 32), (64, 64)), sample: int = 1 << 22):
        """(S, C) with the lowest tuned decode time per symbol on a sample of x."""
        import torch
        xs = np.ascontiguousarray(x[:sample])
        bits = int(lengths[xs].astype(np.int64).sum())
        key = self._key("layout-" + class_key(A, xs.size, bits))
        with self._mu:
            hit = self.cache.get(key)
        if hit:
            return hit["S"], hit["C"]
        best = None
        out = torch.empty(max(xs.size, 8), dtype=torch.int16, device="cuda")
        tab = hd.Table(lengths, codes, L)
        for S, Cc in candidates:
            hs = hd.encode_ref(xs, lengths, codes, L, S, Cc)
            ds = hd.DeviceStream.from_host(hs, tab)
            _, ms = hd.autotune(ds, out)
            per_sym = ms / max(xs.size, 1)
            if best is None or per_sym < best[0]:
                best = (per_sym, S, Cc)
        tab.close()
        _, S, Cc = best
        with self._mu:
            self.cache[key] = {"S": int(S), "C": int(Cc), "ns_per_symbol": best[0] * 1e6}
        return S, Cc
