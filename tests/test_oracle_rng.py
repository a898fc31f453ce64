"""Pins for the oracle's counter-based random numbers (Philox4x32-10) and Box-Muller noise.

The noise is the starting point x(0) ~ N(0, I) of the sampling ODE (paper eq. 8) and the
uniform variates feed the flight-length law of eq. 4 (xi in (0, 1]).
"""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(orc, ctr, key, expect):
    assert [int(x) for x in orc.philox4x32_10(ctr, key)] == expect


def test_u01_range_endpoints(orc):
    # xi must lie in (0, 1]: eq. 4 takes ln(xi)
    assert orc.u01(0) == 2.0 ** -24
    assert orc.u01(0xFFFFFFFF) == 1.0
    assert orc.u01(0x000000FF) == 2.0 ** -24          # low 8 bits are dropped
    assert orc.u01(0x00000100) == 2.0 * 2.0 ** -24


def test_philox_words_uniform(orc):
    # 4096 counters -> 16384 words; chi-square on 16 bins of the top 4 bits
    words = np.concatenate([orc.philox4x32_10((i, 0, 0, 7), (123, 456)) for i in range(4096)])
    counts = np.bincount((words >> 28).astype(np.int64), minlength=16)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, 15) > 1e-4


def test_noise_is_standard_normal(orc):
    n = 100_000
    z = orc.noise(seed=2, id_base=0, n=n)
    assert z.shape == (5, n)
    for d in range(5):
        assert abs(z[d].mean()) < 4.0 / np.sqrt(n)
        assert abs(z[d].var() - 1.0) < 4.0 * np.sqrt(2.0 / n)
        assert stats.kstest(z[d], "norm").pvalue > 1e-4
    corr = np.corrcoef(z)
    off = corr[~np.eye(5, dtype=bool)]
    assert np.abs(off).max() < 4.0 / np.sqrt(n)


def test_noise_depends_only_on_stream_id(orc):
    a = orc.noise(seed=9, id_base=1000, n=64)
    b = orc.noise(seed=9, id_base=1032, n=32)
    np.testing.assert_array_equal(a[:, 32:], b)
    c = orc.noise(seed=10, id_base=1000, n=64)
    assert not np.allclose(a, c)
