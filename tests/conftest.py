import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs the HIP path")
    config.addinivalue_line("markers", "slow: full-size workload")


def load_golden(name):
    """Parses a `key value...` fixture; repeated keys accumulate in a list."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out.setdefault(key, []).append(vals)
    return out


def pack_bits(bitstr: str, n_words: int | None = None) -> np.ndarray:
    """Packs a '0'/'1' string MSB-first into uint32 units (test helper)."""
    nw = (len(bitstr) + 31) // 32 + 2 if n_words is None else n_words
    w = np.zeros(nw, dtype=np.uint32)
    for i, ch in enumerate(bitstr):
        if ch == "1":
            w[i // 32] |= np.uint32(1 << (31 - i % 32))
    return w


def unpack_bits(words: np.ndarray, n_bits: int) -> str:
    b = np.unpackbits(np.ascontiguousarray(words, dtype=">u4").view(np.uint8))
    return "".join("1" if v else "0" for v in b[:n_bits])


@pytest.fixture(scope="session")
def golden():
    return load_golden
