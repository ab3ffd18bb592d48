"""Pins of the seeded synthetic inputs (the stand-ins for the paper's
datasets, Sec. V-A, Table III): recorded digests and the analytic residual
spread of the config-2 field.  CPU only; hdsynth holds no coding arithmetic."""
import os
import sys

import numpy as np

import hdsynth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_generator_digests as mgd  # noqa: E402


def test_generator_digests_match_the_recorded_ones(golden):
    g = golden("generator_digests.txt")
    want = {row[0]: (int(row[1]), row[2], row[3]) for row in g["digest"]}
    got = {name: (n, full, pre) for name, n, full, pre in mgd.digests()}
    assert set(got) == set(want) == {"config1", "config2", "config3", "config4_specs", "config5_specs"}
    for name in want:
        assert got[name] == want[name], name


def test_config2_residual_spread_matches_the_noise_level():
    """The 3-D first-order Lorenzo residual of i.i.d. noise of std s is a signed
    sum of 8 independent copies: std sqrt(8) s, i.e. sqrt(8) s / (2 eb) bins
    after prequantization (rounding adds variance 8/12, under 0.3 %).  With
    s = 1e-3 and eb = 1e-4 that is 14.14 bins; on the 512^3 grid the smooth
    part adds almost nothing.  Checked on a 128^3 block of the config-2 field
    within 3 %."""
    F = hdsynth.config2_field()
    r = F.codes.astype(np.int64) - F.radius
    r[F.outlier_idx.astype(np.int64)] = F.outlier_val
    block = r.reshape(F.shape)[1:129, 1:129, 1:129]     # every point has all seven neighbours
    sigma = float(block.std())
    want = np.sqrt(8.0) * 1e-3 / (2 * 1e-4)
    assert abs(sigma / want - 1.0) < 0.03, sigma


def test_two_sided_geometric_is_symmetric_with_the_stated_ratio():
    """P(d = k) is proportional to r^|k|: the ratio of neighbouring masses is r
    on both sides of the centre (config 1: r = 0.35)."""
    x = hdsynth.config1_symbols().astype(np.int64) - 512
    c = np.bincount(np.abs(x), minlength=4)[:4].astype(np.float64)
    pos = np.array([(x == k).sum() for k in range(1, 4)], np.float64)
    neg = np.array([(x == -k).sum() for k in range(1, 4)], np.float64)
    assert abs(pos[0] / c[0] - 0.35) < 0.01 and abs(neg[0] / c[0] - 0.35) < 0.01
    assert abs(pos[1] / pos[0] - 0.35) < 0.02 and abs(neg[1] / neg[0] - 0.35) < 0.02
