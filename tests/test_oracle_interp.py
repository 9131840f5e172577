"""Pins of the oracle's omega-to-lag mapping and of its interpolation between
lag-grid points (a reading: the method itself yields chi only at omega = m d).

The interpolation is pinned by what a straight line through neighbouring grid
values must satisfy: it reproduces any affine sequence exactly, returns the
grid value at f = 0, and treats lag 0 and lags past the grid as zeros for Im
chi while Re chi keeps its Kramers-Kronig values there."""
import numpy as np
import pytest

import oracle


def test_omega_lags_on_and_off_grid():
    neps, emin, emax = 64, -2.0, 2.0
    d = (emax - emin) / neps
    m, f = oracle.omega_lags([0.0, d, 7 * d * (1 + 1e-12), 2.5 * d, 63.75 * d], neps, emin, emax, interp=True)
    assert list(m) == [0, 1, 7, 2, 63]
    assert f[0] == 0.0 and f[1] == 0.0 and f[2] == 0.0
    assert f[3] == pytest.approx(0.5, abs=1e-12) and f[4] == pytest.approx(0.75, abs=1e-12)
    with pytest.raises(ValueError):
        oracle.omega_lags([2.5 * d], neps, emin, emax, interp=False)
    with pytest.raises(ValueError):
        oracle.omega_lags([-0.3 * d], neps, emin, emax, interp=True)


def test_interpolation_reproduces_affine_sequences():
    rng = np.random.Generator(np.random.PCG64(5))
    neps = 32
    a, b = rng.normal(size=(2, 3, 1))
    k = np.arange(neps, dtype=np.float64)
    v = a + b * k  # three affine sequences over the lags
    v[..., 0] = 0.0  # the grid value at lag 0 is zero by definition
    ms = rng.integers(1, neps - 1, size=40)
    fs = rng.uniform(0.0, 1.0, size=40)
    got = oracle.lag_interp(v, ms, fs)
    assert np.allclose(got, a + b * (ms + fs), rtol=0, atol=1e-13)
    # f = 0 returns the grid value itself
    assert np.array_equal(oracle.lag_interp(v, ms, np.zeros(40)), v[..., ms])


def test_interpolation_ends_of_the_grid():
    neps = 16
    v = np.arange(neps, dtype=np.float64) + 10.0
    # between lag 0 (zero) and lag 1
    assert oracle.lag_interp(v, [0], [0.25])[0] == pytest.approx(0.25 * v[1], abs=1e-15)
    # between the last lag and one past the grid (zero)
    assert oracle.lag_interp(v, [neps - 1], [0.25])[0] == pytest.approx(0.75 * v[neps - 1], abs=1e-15)
    assert oracle.lag_interp(v, [neps + 3], [0.5])[0] == 0.0


def test_kk_interpolation_keeps_static_and_tail_values():
    """Re chi at lag 0 (the static response) and past the grid is the KK sum
    itself, nonzero: the interpolated Re uses it at both ends."""
    rng = np.random.Generator(np.random.PCG64(8))
    neps = 24
    im = np.zeros((2, neps))
    im[:, 1:] = -np.abs(rng.normal(size=(2, neps - 1)))
    re0 = oracle.kk_real(im, [0])[:, 0]
    re1 = oracle.kk_real(im, [1])[:, 0]
    tail = oracle.kk_real(im, [neps, neps + 1])
    assert np.all(np.abs(re0) > 0) and np.all(np.abs(tail) > 0)
    got = oracle.kk_real_interp(im, [0, neps], [0.3, 0.6])
    assert np.allclose(got[:, 0], 0.7 * re0 + 0.3 * re1, rtol=1e-15, atol=0)
    assert np.allclose(got[:, 1], 0.4 * tail[:, 0] + 0.6 * tail[:, 1], rtol=1e-15, atol=0)
    # the KK sum is linear in Im chi, so interpolating Re equals taking the KK
    # sum of the interpolated weights (what a one-pass implementation does)
    j = np.arange(neps)
    def w(i):
        return np.where((j >= 1) & ((j - i) % 2 == 1), (2 / np.pi) * 2 * j / (j * j - float(i) ** 2 + ((j - i) % 2 == 0)), 0.0)
    direct = im @ (0.7 * w(5) + 0.3 * w(6))
    assert np.allclose(oracle.kk_real_interp(im, [5], [0.3])[:, 0], direct, rtol=1e-13, atol=0)
