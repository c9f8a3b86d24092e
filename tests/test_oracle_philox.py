"""The oracle's counter-based noise generator (Philox4x32-10 + Box-Muller)
against the generator's published known-answer vectors and the standard
normal distribution.  The device library implements the same definition; the
GPU tests compare the two bit for bit."""
import math
import os

import numpy as np
from scipy import stats

from conftest import ROOT
from oracle import philox as PH


def kat_rows():
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    return rows


def test_known_answer_vectors():
    rows = kat_rows()
    assert len(rows) == 3
    for r in rows:
        ctr = [np.array([v], dtype=np.uint64) for v in r[:4]]
        out = PH.philox4x32_10(ctr, (r[4], r[5]))
        assert [int(v[0]) for v in out] == r[6:10]


def test_counter_layout():
    # element pair j of (stream, counter) is Philox at counter words (j, stream, k_lo, k_hi)
    seed, stream, counter = 0x0123456789ABCDEF, 2, (7 << 32) + 5
    w = PH.raw_words(seed, stream, counter, 3)
    for j in range(3):
        ctr = [np.array([v], dtype=np.uint64) for v in (j, stream, 5, 7)]
        ref = PH.philox4x32_10(ctr, (0x89ABCDEF, 0x01234567))
        assert [int(v[0]) for v in ref] == [int(v) for v in w[:, j]]


def test_normals_distribution():
    z = PH.normals(1709, PH.STREAM_W_GRID, 3, 2_000_001)
    n = z.size
    assert n == 2_000_001 and np.all(np.isfinite(z))
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(stats.kurtosis(z, fisher=False) - 3) < 5 * math.sqrt(24 / n)
    assert stats.kstest(z[:200_000], "norm").pvalue > 1e-3
    # the two members of a Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(z[0:-1:2], z[1::2])[0, 1]) < 5 / math.sqrt(n / 2)


def test_streams_and_draws_differ():
    a = PH.normals(1, 0, 0, 1000)
    for other in (PH.normals(1, 1, 0, 1000), PH.normals(1, 0, 1, 1000), PH.normals(2, 0, 0, 1000)):
        assert abs(np.corrcoef(a, other)[0, 1]) < 0.15
        assert not np.any(a == other)
    # a prefix of a longer draw is the shorter draw
    assert np.array_equal(PH.normals(1, 0, 0, 999), a[:999])
