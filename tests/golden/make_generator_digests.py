"""Writes tests/golden/generator_digests.txt: SHA-256 digests of the seeded
synthetic inputs (hdsynth only; no coding arithmetic is involved), so that a
change to any generator shows up as a failing CPU test.

    python tests/golden/make_generator_digests.py
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import hdsynth  # noqa: E402

PREFIX = 1 << 22


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def spec_digest(specs) -> str:
    rows = np.array([[s["n"], s["A"], int(round(s["r"] * 2 ** 40))] for s in specs], dtype=np.int64)
    return sha(rows)


def digests():
    out = []
    x = hdsynth.config1_symbols()
    out.append(("config1", x.size, sha(x), sha(x[:PREFIX])))
    x = hdsynth.config2_symbols()
    out.append(("config2", x.size, sha(x), sha(x[:PREFIX])))
    del x
    x = hdsynth.config3_symbols()
    out.append(("config3", x.size, sha(x), sha(x[:PREFIX])))
    del x
    specs = hdsynth.batch_stream_specs()
    x = hdsynth.batch_stream_symbols(specs[0])
    out.append(("config4_specs", len(specs), spec_digest(specs), sha(x[:PREFIX])))
    specs = hdsynth.serve_pool_specs()
    x = hdsynth.batch_stream_symbols(specs[0])
    out.append(("config5_specs", len(specs), spec_digest(specs), sha(x[:PREFIX])))
    return out


def main():
    rows = digests()
    with open(os.path.join(HERE, "generator_digests.txt"), "w") as f:
        f.write("# SHA-256 of the seeded synthetic inputs (hdsynth), written by\n"
                "# make_generator_digests.py.  Columns: name, element count (streams for the\n"
                "# spec lists), digest of the whole array (of the (n, A, round(r * 2^40)) int64\n"
                "# rows for spec lists), digest of the first 2^22 elements (of stream 0's\n"
                "# symbols for spec lists).  Arrays are hashed as their native little-endian\n"
                "# bytes (uint16 symbols).\n")
        for name, n, full, pre in rows:
            f.write(f"digest {name} {n} {full} {pre}\n")


if __name__ == "__main__":
    main()
