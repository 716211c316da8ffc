"""Pins for the oracle's counter-based generator and focal-volume sampler.

Philox4x64-10 is checked against numpy's independent implementation of the
same published generator; the sampler against the moments and uniformity a
uniform cylinder fixes (Sec. 2.1: ions uniform in a cylinder about the axis).
"""
import numpy as np
import pytest
from scipy import stats


def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(123)
    for _ in range(50):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        ctr[0] = ctr[0] | np.uint64(1)  # numpy increments first: feed ctr-1
        bg = np.random.Philox(key=key, counter=ctr - np.array([1, 0, 0, 0], dtype=np.uint64))
        ref = bg.random_raw(4).astype(np.uint64)
        got = orc.philox(ctr, key)
        assert np.array_equal(got, ref)


def test_uniform_word_layout(orc):
    # u_j uses word j%4 of block j/4, top 53 bits, (m+1) 2^-53.
    seed, cfg, atom = 7, 3, 12345
    for j in range(16):
        out = orc.philox([atom, j // 4, 0, 0], [seed, cfg])
        m = int(out[j % 4]) >> 11
        assert orc.uniform(seed, cfg, [atom], j)[0] == (m + 1) * 2.0**-53


def test_uniform_range_and_independence_of_sharding(orc):
    atoms = np.arange(1000, 21000, dtype=np.uint64)
    u = orc.uniform(0, 1, atoms, 4)
    assert u.min() > 0.0 and u.max() <= 1.0
    # any subset of indices gives the same numbers
    sub = atoms[::37]
    assert np.array_equal(orc.uniform(0, 1, sub, 4), u[::37])
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_sampler_moments(orc):
    n, R, zh = 200_000, 6e-6, 35e-6
    x, y, z = orc.sample_atoms(0, 0, 0, n, R, zh)
    r = np.hypot(x, y)
    assert r.max() <= R * (1 + 1e-15) and np.abs(z).max() <= zh
    # uniform disk: r^2/R^2 ~ U(0,1); azimuth ~ U(-pi,pi); z ~ U(-zh, zh)
    assert stats.kstest((r / R) ** 2, "uniform").pvalue > 1e-3
    assert stats.kstest(np.arctan2(y, x), "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-3
    assert stats.kstest(z, "uniform", args=(-zh, 2 * zh)).pvalue > 1e-3
    assert abs(np.mean(r**2) / (R * R / 2) - 1) < 0.01


def test_sampler_offset_consistency(orc):
    x0, y0, z0 = orc.sample_atoms(5, 2, 0, 100, 1.0, 1.0)
    x1, y1, z1 = orc.sample_atoms(5, 2, 40, 60, 1.0, 1.0)
    assert np.array_equal(x0[40:], x1) and np.array_equal(z0[40:], z1)
