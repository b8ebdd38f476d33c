"""Pins for the oracle's random projection (Philox4x64-10 + Box-Muller)."""

import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x64_10, gaussian_omega, box_muller


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2002, 0), (2**63 + 12345, 2**64 - 1)])
@pytest.mark.parametrize("ctr0", [0, 1, 17, 2**40 + 3])
def test_philox_blocks_match_numpy(key, ctr0):
    # numpy's Philox (an independent implementation of Philox4x64-10)
    # advances the counter before each block: its k-th block is ours at ctr0 + k.
    bg = np.random.Philox(counter=ctr0, key=np.array(key, dtype=np.uint64))
    ref = bg.random_raw(4 * 6).reshape(6, 4)
    for b in range(6):
        ours = philox4x64_10((np.uint64(ctr0 + b + 1), 0, 0, 0), key)
        assert [int(x) for x in ours] == [int(x) for x in ref[b]]


def test_philox_counter_words_matter():
    # a mistake that ignored counter word 1 or the key's second word would collide
    a = philox4x64_10((3, 0, 0, 0), (1, 2))
    b = philox4x64_10((3, 1, 0, 0), (1, 2))
    c = philox4x64_10((3, 0, 0, 0), (1, 3))
    assert [int(x) for x in a] != [int(x) for x in b]
    assert [int(x) for x in a] != [int(x) for x in c]


def test_box_muller_extremes():
    # r >> 11 == 0 gives u1 = 2^-53: finite radius sqrt(-2 ln 2^-53) ~ 8.57
    z0, z1 = box_muller(np.uint64(0), np.uint64(0))
    assert np.isclose(z0, np.sqrt(-2.0 * np.log(2.0 ** -53)))
    assert z1 == 0.0
    # the largest word gives u1 = 1 exactly -> zero radius
    z0, z1 = box_muller(np.uint64(2**64 - 1), np.uint64(2**63))
    assert z0 == 0.0 and z1 == 0.0


def test_omega_moments_and_ks():
    om = gaussian_omega(4000, 50, seed=11, channel=3)
    x = om.ravel()
    assert abs(x.mean()) < 5 * 1 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / x.size)
    assert abs(stats.skew(x)) < 0.02
    assert abs(stats.kurtosis(x)) < 0.04
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # columns j mod 4 use different words; each must be N(0,1) on its own
    for r in range(4):
        assert stats.kstest(om[:, r::4].ravel(), "norm").pvalue > 1e-3
    # independence across the sine/cosine pair (same radius)
    c = np.corrcoef(om[:, 0], om[:, 1])[0, 1]
    assert abs(c) < 5 / np.sqrt(om.shape[0])


def test_omega_columns_stable_under_growth():
    a = gaussian_omega(37, 10, seed=3, channel=1)
    b = gaussian_omega(37, 23, seed=3, channel=1)
    assert np.array_equal(a, b[:, :10])
    c = gaussian_omega(37, 13, seed=3, channel=1, col0=10)
    assert np.array_equal(c, b[:, 10:23])


def test_omega_entry_definition():
    # entry (i, j) comes from the block at counter (i, j // 4) and key (seed, channel)
    om = gaussian_omega(9, 11, seed=77, channel=5)
    i, j = 6, 9
    r = philox4x64_10((i, j // 4, 0, 0), (77, 5))
    z = box_muller(r[0], r[1]) + box_muller(r[2], r[3])
    assert om[i, j] == z[j % 4]
    assert not np.array_equal(gaussian_omega(9, 11, 77, 6), om)
