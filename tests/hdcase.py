"""Test helpers: build a stream with the ORACLE (codebook + encoder), upload it,
run the library's decode, and compare with the oracle's decode."""
from __future__ import annotations

import sys
from dataclasses import dataclass

import numpy as np

import oracle


def flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@dataclass
class Case:
    x: np.ndarray
    A: int
    L: int
    S: int
    C: int
    lengths: np.ndarray
    codes: np.ndarray
    enc: oracle.Encoded

    @property
    def width(self) -> int:
        return self.x.dtype.itemsize

    def info(self):
        from paper_2201_09118_amd import hd
        e = self.enc
        return hd.StreamInfo(e.n_symbols, e.n_bits, e.words.size, e.gap.size, e.chunk_counts.size,
                             self.S, self.C, self.A, self.L, self.width)


def make_case(x, A, L, S=128, C=32, lengths=None, codes=None) -> Case:
    """uint8 and uint32 symbol arrays keep their width; anything else is uint16."""
    x = np.asarray(x)
    x = np.ascontiguousarray(x if x.dtype in (np.uint8, np.uint32) else x.astype(np.uint16))
    if lengths is None:
        lengths = oracle.code_lengths(oracle.histogram(x, A), L)
        codes = oracle.canonical_codes(lengths)
    enc = oracle.encode(x, lengths, codes, S, C)
    return Case(x, A, L, S, C, lengths, codes, enc)


def upload(case: Case, lut_bits=0, with_gap=True, device="cuda"):
    import torch
    from paper_2201_09118_amd import hd
    tab = hd.Table(case.lengths, case.codes, case.L, lut_bits)
    e = case.enc
    w = torch.from_numpy(e.words.view(np.int32)).to(device)
    g = torch.from_numpy(e.gap).to(device) if with_gap else None
    c = torch.from_numpy(e.chunk_offsets.view(np.int64)).to(device) if with_gap else None
    return hd.DeviceStream(w, g, c, case.info(), tab)


_TORCH_OF = {1: "uint8", 2: "int16", 4: "int32"}
_NUMPY_OF = {1: np.uint8, 2: np.uint16, 4: np.uint32}


def run_decode(ds, mode=0, tune=None, n_out=None):
    import torch
    from paper_2201_09118_amd import hd
    n = ds.n_symbols if n_out is None else n_out
    w = int(ds.info.symbol_bytes) or 2
    out = torch.full((max(n, 1),), -1 if w > 1 else 255, dtype=getattr(torch, _TORCH_OF[w]), device="cuda")
    ws = hd.decode(ds, out, mode, tune)
    bits = hd.decode_status_bits(ws)
    torch.cuda.synchronize()
    return out[:n].cpu().numpy().view(_NUMPY_OF[w]), bits


def expected(case: Case) -> np.ndarray:
    e = case.enc
    return oracle.decode(e.words, e.n_bits, e.n_symbols, case.lengths, case.codes, width=case.width)
