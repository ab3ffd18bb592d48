"""Seeded synthetic symbol streams for the Huffman-decode workloads.

This module only draws input symbols. It holds none of the coding arithmetic
(no histograms of codes, no code lengths, no bit packing): both the CPU oracle
and the GPU library take its output as plain unsigned arrays (uint16 by
default; uint8 and uint32 for the other symbol widths).

The paper evaluates on SZ quantization codes of eight scientific datasets
(Sec. V-A, Table III) that are not available here.  The generators below stand
in for them with the same element type (uint16 quantization codes), the same
shapes (the 512^3 Nyx grid, the ~281 M-element 1-D HACC field) and the same
structure (a prediction residual re-centred by a radius offset, with code 0
marking an unpredictable value, as in SZ-style quantization, Sec. II-A).

Every generator is a pure function of its seed: numpy PCG64 seeded through
SeedSequence(seed); sub-streams use SeedSequence.spawn().
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng_for",
    "two_sided_geometric",
    "config1_symbols",
    "LorenzoField",
    "lorenzo_field",
    "lorenzo_field_codes",
    "config2_symbols",
    "config2_field",
    "config2_symbols_u8",
    "config2_symbols_u32",
    "config3_symbols",
    "batch_stream_specs",
    "batch_stream_symbols",
    "serve_pool_specs",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def two_sided_geometric(rng: np.random.Generator, n: int, r: float, A: int,
                        centre: int | None = None, dtype=np.uint16) -> np.ndarray:
    """x = centre + (G1 - G2), G ~ Geometric on {0,1,...} with P(G=g) ∝ r^g.

    The difference of two i.i.d. geometrics has P(d = k) ∝ r^|k| exactly.
    Values outside [0, A) are replaced by 0 (the SZ outlier marker).
    """
    c = A // 2 if centre is None else int(centre)
    p = 1.0 - float(r)
    x = np.full(n, c, dtype=np.int64)
    # numpy's geometric counts trials (>= 1); subtract 1 to count failures.
    x += rng.geometric(p, n).astype(np.int64) - 1
    x -= rng.geometric(p, n).astype(np.int64) - 1
    x[(x < 0) | (x >= A)] = 0
    assert A - 1 <= np.iinfo(dtype).max, "alphabet does not fit the symbol type"
    return x.astype(dtype)


def config1_symbols(n: int = 1 << 20, seed: int = 1) -> np.ndarray:
    """1,048,576 i.i.d. two-sided geometric symbols, A = 1024, r = 0.35."""
    return two_sided_geometric(rng_for(seed), n, 0.35, 1024)


def _smooth_field(shape, n_waves: int, rng: np.random.Generator) -> np.ndarray:
    """Sum of n_waves random 3-D plane sinusoids on a periodic grid (float32).

    f(i,j,k) = sum_m a_m sin(2*pi*(u_m i + v_m j + w_m k)/N + phi_m) with
    a ~ U(0,1), (u,v,w) ~ U{1..8}^3, phi ~ U[0, 2*pi).  Evaluated separably
    (sin(x+y) = sin x cos y + cos x sin y) so the 512^3 case takes seconds.
    """
    import torch

    ni, nj, nk = shape
    a = rng.uniform(0.0, 1.0, n_waves)
    uvw = rng.integers(1, 9, size=(n_waves, 3))
    phi = rng.uniform(0.0, 2.0 * math.pi, n_waves)
    ii = np.arange(ni, dtype=np.float64)[:, None]
    jj = np.arange(nj, dtype=np.float64)[None, :]
    kk = np.arange(nk, dtype=np.float64)
    f = torch.zeros(shape, dtype=torch.float32)
    for m in range(n_waves):
        u, v, w = (int(t) for t in uvw[m])
        ang_ij = 2.0 * math.pi * (u * ii / ni + v * jj / nj) + phi[m]
        ang_k = 2.0 * math.pi * w * kk / nk
        s_ij = torch.from_numpy((a[m] * np.sin(ang_ij)).astype(np.float32))
        c_ij = torch.from_numpy((a[m] * np.cos(ang_ij)).astype(np.float32))
        s_k = torch.from_numpy(np.sin(ang_k).astype(np.float32))
        c_k = torch.from_numpy(np.cos(ang_k).astype(np.float32))
        f.add_(s_ij[:, :, None] * c_k[None, None, :])
        f.add_(c_ij[:, :, None] * s_k[None, None, :])
    return f.numpy()


@dataclass
class LorenzoField:
    """A quantized field as an SZ-style compressor leaves it for the decoder.

    codes        uint16[n], C order: Lorenzo residual + radius, 0 = outlier;
    outlier_idx  uint64[m], ascending flat index of every code-0 position;
    outlier_val  int32[m], the true residual at each of those positions;
    field        float32[shape] (the original data) when kept, else None.
    """
    shape: tuple
    eb: float
    radius: int
    codes: np.ndarray
    outlier_idx: np.ndarray
    outlier_val: np.ndarray
    field: np.ndarray | None


def lorenzo_field(shape=(512, 512, 512), seed: int = 2, n_waves: int = 16,
                  noise_sigma: float = 1e-3, eb: float = 1e-4, radius: int = 512,
                  keep_field: bool = False, dtype=np.uint16) -> LorenzoField:
    """SZ-style quantization codes of a seeded smooth float32 field.

    field = n_waves random plane sinusoids + N(0, noise_sigma^2), float32.
    q = floor(f / (2 eb) + 1/2) (float64 arithmetic on the float32 values);
    r = 3-D first-order Lorenzo residual of q with zeros outside the grid;
    code = r + radius when 0 <= r + radius < 2 radius, else 0.  Every code-0
    position (out-of-range residuals, and r = -radius) goes to the outlier
    list with its true residual.  Flattened in C order (last axis fastest).
    Codes are returned as `dtype`, which must hold 2 radius - 1.
    """
    assert 2 * radius - 1 <= np.iinfo(dtype).max, "radius does not fit the code type"
    import torch

    rng = rng_for(seed)
    f = _smooth_field(shape, n_waves, rng)
    f += rng.standard_normal(f.shape, dtype=np.float32) * np.float32(noise_sigma)
    ft = torch.from_numpy(f)
    q = torch.floor(ft.to(torch.float64) / (2.0 * eb) + 0.5).to(torch.int32)
    del ft
    if not keep_field:
        del f
        f = None
    # Lorenzo residual = product of backward differences along each axis.
    for ax in range(3):
        d = q.clone()
        sl_dst = [slice(None)] * 3
        sl_src = [slice(None)] * 3
        sl_dst[ax] = slice(1, None)
        sl_src[ax] = slice(0, -1)
        d[tuple(sl_dst)] -= q[tuple(sl_src)]
        q = d
    code = q + radius
    code[(code < 0) | (code >= 2 * radius)] = 0
    codes = code.to(torch.int32).numpy().astype(dtype).reshape(-1)
    idx = np.flatnonzero(codes == 0).astype(np.uint64)
    val = q.reshape(-1).numpy()[idx.astype(np.int64)].astype(np.int32)
    return LorenzoField(tuple(int(v) for v in shape), float(eb), int(radius), codes, idx, val, f)


def lorenzo_field_codes(shape=(512, 512, 512), seed: int = 2, n_waves: int = 16,
                        noise_sigma: float = 1e-3, eb: float = 1e-4,
                        radius: int = 512) -> np.ndarray:
    """The codes of lorenzo_field (same arguments)."""
    return lorenzo_field(shape, seed, n_waves, noise_sigma, eb, radius).codes


def config2_symbols(seed: int = 2) -> np.ndarray:
    """512^3 = 134,217,728 Lorenzo-residual codes, A = 1024."""
    return lorenzo_field_codes((512, 512, 512), seed=seed)


def config2_field(seed: int = 2, keep_field: bool = False) -> LorenzoField:
    """The 512^3 field behind config2_symbols, with its outliers (eb 1e-4, radius 512)."""
    return lorenzo_field((512, 512, 512), seed=seed, keep_field=keep_field)


def config2_symbols_u8(seed: int = 2) -> np.ndarray:
    """The 512^3 field of config2_symbols quantized into one-byte codes
    (radius 128, A = 256), like the 8-bit symbols of the decoders the paper
    starts from (its single-byte baseline trims codes to one byte)."""
    return lorenzo_field((512, 512, 512), seed=seed, radius=128, dtype=np.uint8).codes


def config2_symbols_u32(seed: int = 2) -> np.ndarray:
    """The same field at a 100x tighter bound (eb 1e-6) with radius 2^17
    (A = 2^18): codes wider than 16 bits, as tight double-precision bounds
    need; residual spread about 1400 bins."""
    return lorenzo_field((512, 512, 512), seed=seed, eb=1e-6, radius=1 << 17, dtype=np.uint32).codes


def config3_symbols(n: int = 280_000_000, seed: int = 3, A: int = 4096,
                    sigma: float = 40.0, outlier_p: float = 1e-3) -> np.ndarray:
    """Discretised Gaussian (centre A/2, sigma 40) with a 0.1% uniform tail."""
    rng = rng_for(seed)
    x = np.rint(A / 2 + sigma * rng.standard_normal(n)).astype(np.int64)
    mask = rng.random(n) < outlier_p
    x[mask] = rng.integers(0, A, size=int(mask.sum()))
    np.clip(x, 0, A - 1, out=x)
    return x.astype(np.uint16)


def batch_stream_specs(n_streams: int = 256, lo: int = 1 << 16, hi: int = 1 << 26,
                       alphabets=(256, 1024, 4096), r_lo: float = 0.2, r_hi: float = 0.8,
                       seed: int = 4):
    """Per-stream (n, A, r, child seed) for the batched workload.

    n = floor(exp(U(ln lo, ln hi))), A uniform over `alphabets`, r ~ U[r_lo, r_hi].
    """
    ss = np.random.SeedSequence(seed)
    rng = np.random.Generator(np.random.PCG64(ss))
    ns = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n_streams))).astype(np.int64)
    As = rng.choice(np.asarray(alphabets, dtype=np.int64), n_streams)
    rs = rng.uniform(r_lo, r_hi, n_streams)
    kids = ss.spawn(n_streams)
    return [dict(n=int(ns[i]), A=int(As[i]), r=float(rs[i]), seed_seq=kids[i]) for i in range(n_streams)]


def batch_stream_symbols(spec) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(spec["seed_seq"]))
    return two_sided_geometric(rng, spec["n"], spec["r"], spec["A"])


def serve_pool_specs(n_pool: int = 64, lo: int = 1 << 20, hi: int = 1 << 28,
                     alphabets=(1024, 4096), seed: int = 5):
    """Distinct pre-encoded request streams for the serving loop."""
    return batch_stream_specs(n_pool, lo, hi, alphabets, 0.2, 0.8, seed)
