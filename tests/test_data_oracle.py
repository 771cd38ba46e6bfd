"""Pins of the sparse-detector data path and metrics oracle (oracle/data_oracle.py)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import data_oracle as D


def test_philox_matches_numpy_bit_generator():
    """numpy.random.Philox is Philox4x64-10; it increments its counter before each block,
    so its i-th block is ours at counter (c + 1 + i)."""
    key = (0x0123456789ABCDEF, 0xFEDCBA9876543210)
    for start in (0, 7, 2 ** 40 + 3):
        bg = np.random.Philox(key=np.array(key, np.uint64),
                              counter=np.array([start, 0, 0, 0], np.uint64))
        raw = bg.random_raw(4 * 5).reshape(5, 4)
        ctr = np.zeros((5, 4), np.uint64)
        ctr[:, 0] = np.arange(start + 1, start + 6, dtype=np.uint64)
        assert np.array_equal(D.philox4x64_10(ctr, key), raw)


def test_mulhilo_against_python_integers():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2 ** 63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    hi, lo = D._mulhilo64(a, b)
    for x, y, h, l in zip(a[:200], b[:200], hi[:200], lo[:200]):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


def test_normals_are_standard_normal_and_independent():
    z1, z2 = D.normals(200000, seed=5)
    for z in (z1, z2):
        assert abs(z.mean()) < 5 / math.sqrt(z.size)
        assert abs(z.var() - 1.0) < 0.02
        assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z1, z2)[0, 1]) < 0.01
    a, _ = D.normals(1000, seed=6)
    assert not np.array_equal(a, z1[:1000])


def test_upsample_reproduces_linear_data_and_kept_columns():
    cols, step = 37, 4
    c = np.arange(cols, dtype=np.float64)
    full = np.stack([3.0 + 0.25 * c, -1.0 + 2.0 * c])          # linear in the column index
    sp = D.sparse_sample(full, step)
    assert sp.shape[-1] == math.ceil(cols / step)
    up = D.sparse_upsample(sp, cols, step)
    last = (sp.shape[-1] - 1) * step
    assert np.allclose(up[:, :last + 1], full[:, :last + 1], rtol=0, atol=1e-12)
    assert np.all(up[:, last + 1:] == full[:, [last]])        # held beyond the last kept column
    assert np.array_equal(up[:, ::step], sp)


def test_noise_statistics_match_the_photon_model():
    """For constant g the noisy value's variance is M^2 (lambda + var) / lambda^2 to first
    order (delta method on M log(I0 / counts)); without photons or electrons noise (I0 huge,
    var 0) the data come back unchanged."""
    n = 200000
    g = np.full(n, 30.0)
    M, I0, var = 40.0, 1e5, 0.5
    gn = D.add_noise(g, M=M, I0=I0, var=var, seed=9)
    lam = I0 * math.exp(-30.0 / M)
    pred = M * M * (lam + var) / lam ** 2
    assert abs(gn.var() / pred - 1.0) < 0.02
    assert abs(gn.mean() - 30.0) < 6 * math.sqrt(pred / n)
    quiet = D.add_noise(g[:1000], M=M, I0=1e30, var=0.0, seed=9)
    assert np.allclose(quiet, 30.0, rtol=1e-9)


def test_rmse_ssim_hand_example():
    """f = (0, 1), ref = (0, 2): means 1/2 and 1, population variances 1/4 and 1,
    covariance 1/2, ref range 2 -> c1 = 0.02^2, c2 = 0.06^2."""
    f, ref = np.array([0.0, 1.0]), np.array([0.0, 2.0])
    c1, c2 = 0.02 ** 2, 0.06 ** 2
    expect = (2 * 0.5 * 1.0 + c1) * (2 * 0.5 + c2) / ((0.25 + 1.0 + c1) * (0.25 + 1.0 + c2))
    assert D.ssim(f, ref) == pytest.approx(expect, rel=1e-14)
    assert D.rmse(f, ref) == pytest.approx(math.sqrt(0.5), rel=1e-14)


def test_rmse_ssim_identities():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(7, 9))
    assert D.ssim(x, x) == pytest.approx(1.0, abs=1e-14)
    assert D.rmse(x, x) == 0.0
    assert D.rmse(x + 0.3, x) == pytest.approx(0.3, rel=1e-12)
    e = rng.normal(size=x.shape)
    s = [D.ssim(x + a * e, x) for a in (0.1, 0.5, 1.0)]
    assert 1.0 > s[0] > s[1] > s[2]


def test_normals_at_equals_the_sequence():
    z1, z2 = D.normals(1001, seed=8)
    idx = np.array([0, 1, 2, 999, 1000, 513, 514])
    a1, a2 = D.normals_at(idx, seed=8)
    assert np.array_equal(a1, z1[idx]) and np.array_equal(a2, z2[idx])
    g = np.linspace(0, 40, 1001)
    full = D.add_noise(g, M=50.0, seed=8)
    assert np.array_equal(D.add_noise_at(g[idx], idx, 50.0, seed=8), full[idx])
