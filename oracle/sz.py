"""CPU oracle for SZ-style reconstruction after Huffman decoding.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports or
runs this file, and this file uses nothing from the product library.

What is computed.  The decoded symbols are SZ quantization codes (Sec. II-A:
error-bounded lossy compression; Sec. V-B-2 evaluates the whole cuSZ
decompression around the decoder).  The paper states the pipeline only in
outline; the reading taken here is the first-order Lorenzo scheme with
prequantization that cuSZ uses:

* each point holds an integer q = round(f / (2 eb)), so |f - 2 eb q| <= eb;
* the compressor stores the Lorenzo prediction residual of q (the 3-D
  first-order predictor, points outside the grid counting as 0), shifted by a
  radius into [1, 2 radius), with code 0 marking a residual kept out of band
  (an "outlier", stored as index + true residual);
* reconstruction undoes the three steps in reverse: residual from code or
  outlier list, q from the residuals, value = q * 2 eb.

The predictor's inverse has a plain definition: q at (i, j, k) is the sum of
the residuals over the box [0, i] x [0, j] x [0, k] (an inclusive prefix sum
along every axis).  Integers are int64 here (exact); the dequantized value is
the product q * (2 eb) taken in float64 (one IEEE rounding) and then rounded to
float32.
"""
from __future__ import annotations

import numpy as np


class MissingOutlier(ValueError):
    """A code-0 position has no entry in the outlier list."""


def residuals(codes: np.ndarray, radius: int, outlier_idx: np.ndarray, outlier_val: np.ndarray) -> np.ndarray:
    """int64 residuals: code - radius, or the outlier list's value where code == 0.

    Entries of the list at positions whose code is not 0 are not consulted."""
    codes = np.asarray(codes).reshape(-1)
    r = codes.astype(np.int64) - int(radius)
    zero = np.flatnonzero(codes == 0)
    idx = np.asarray(outlier_idx, dtype=np.int64).reshape(-1)
    val = np.asarray(outlier_val, dtype=np.int64).reshape(-1)
    pos = np.searchsorted(idx, zero)
    ok = pos < idx.size
    ok[ok] = idx[pos[ok]] == zero[ok]
    if not ok.all():
        raise MissingOutlier(f"{int((~ok).sum())} code-0 positions have no outlier entry")
    r[zero] = val[pos]
    return r


def inverse_lorenzo(r: np.ndarray, shape) -> np.ndarray:
    """q = inclusive prefix sum of the residuals along each of the three axes (int64)."""
    q = np.asarray(r, dtype=np.int64).reshape(shape).copy()
    for ax in range(3):
        np.cumsum(q, axis=ax, out=q)
    return q


def dequantize(q: np.ndarray, eb: float) -> np.ndarray:
    """value = q * (2 eb): the float64 product, then rounded to float32."""
    return (np.asarray(q, dtype=np.int64).astype(np.float64) * (2.0 * float(eb))).astype(np.float32)


def reconstruct(codes, shape, radius, outlier_idx, outlier_val, eb):
    """(q as int64[shape], value as float32[shape]) from the decoded codes."""
    q = inverse_lorenzo(residuals(codes, radius, outlier_idx, outlier_val), shape)
    return q, dequantize(q, eb)
