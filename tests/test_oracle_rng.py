"""Pins of the oracle's random-number pieces: the u-mapping, the hand-written
logarithm (exhaustive against float64 log), Philox statistics and the start
node. The logarithm replaces the exponentiation of A-Res keys (Sec. 4.2.2)."""
import numpy as np
import pytest
from scipy import stats


def all_u():
    k = np.arange(1 << 23, dtype=np.uint64)
    return ((2 * k + 1).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def test_u01_range_and_exactness(orc):
    x = np.array([0, 1, 511, 512, 0x80000000, 0xFFFFFFFF, 0xFFFFFE00, 0xFFFFFDFF], dtype=np.uint32)
    u = orc.u01_n(x).astype(np.float64)
    assert u.min() > 0.0 and u.max() < 1.0
    # u * 2^24 is the odd integer 2*(x >> 9) + 1, i.e. the mapping is exact
    assert np.array_equal(u * 2.0 ** 24, 2.0 * (x >> 9).astype(np.float64) + 1.0)
    assert u[0] == 2.0 ** -24 and u[5] == 1.0 - 2.0 ** -24


def test_logf_exhaustive_accuracy(orc):
    """All 2^23 possible u: within 1 ulp of the float64 logarithm, negative,
    monotone non-decreasing in u (so larger u never gets a smaller key)."""
    u = all_u()
    r = orc.logf_n(u)
    ref = np.log(u.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    err = np.abs(r.astype(np.float64) - ref) / ulp
    assert err.max() < 1.0, err.max()
    assert np.all(r < 0)
    assert np.all(np.diff(r) >= 0)


def test_logf_powers_of_two(orc):
    """ln(2^-k) for k = 1..24 to within one ulp (e*ln2 path, f = 0)."""
    for k in range(1, 25):
        u = np.float32(2.0 ** -k)
        r = float(orc.logf(u))
        ref = -k * np.log(2.0)
        assert abs(r - ref) <= float(np.spacing(np.float32(abs(ref))))


def test_philox_words_uniform_and_distinct(orc):
    """Philox words over a block of counters: chi-square uniform over 256
    bins of the top byte and of the low byte; no duplicate words among
    2^16 draws beyond what a uniform 32-bit generator would give."""
    steps = np.repeat(np.arange(1, 257, dtype=np.uint32), 256)
    slots = np.tile(np.arange(256, dtype=np.uint32), 256)
    w = orc.draw_words(12345, 3, 77, steps, slots)
    for byte in (w >> 24, w & 0xFF):
        obs = np.bincount(byte.astype(np.int64), minlength=256)
        p = stats.chisquare(obs).pvalue
        assert p > 1e-4, p
    assert np.unique(w).size >= w.size - 8


def test_draws_depend_on_every_counter_field(orc):
    base = orc.draw_word(1, 2, 3, 4, 5)
    assert orc.draw_word(2, 2, 3, 4, 5) != base
    assert orc.draw_word(1, 9, 3, 4, 5) != base
    assert orc.draw_word(1, 2, 9, 4, 5) != base
    assert orc.draw_word(1, 2, 3, 9, 5) != base
    assert orc.draw_word(1, 2, 3, 4, 6) != base
    # the four words of one Philox block serve slots 4q..4q+3
    blk = orc.philox([(5 >> 2) | (4 << 16), 3, 2, 0], [1, 0])
    assert blk[5 & 3] == base


def test_start_node_uniform(orc):
    n = 7
    s = np.array([orc.start_node(99, 0, a, n) for a in range(14000)])
    assert s.min() == 0 and s.max() == n - 1
    obs = np.bincount(s, minlength=n)
    assert stats.chisquare(obs).pvalue > 1e-3
