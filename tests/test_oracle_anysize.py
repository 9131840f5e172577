"""Pins of the oracle on grids whose sizes are not powers of two (the paper's
2049-point grids): a brute-force double sum on a tiny odd grid, and the
periodic-image identity that a table repeating with period N/2 on an N grid
gives chi of the N/2 grid at q mod N/2."""
import numpy as np
import pytest

import oracle
from paper_1208_3210_amd import workloads as W

NEPS, EMIN, EMAX, GAMMA = 24, -1.5, 1.5, 0.15


def test_brute_force_on_an_odd_grid():
    nkx, nky = 5, 3
    eps = oracle.band_tb(0.4, -0.1, 0.03, nkx, nky)
    xi = eps - 0.05
    d = (EMAX - EMIN) / NEPS
    e = EMIN + (np.arange(NEPS) + 0.5) * d
    occ = e <= 0.0

    def A(iy, ix, j):
        return (GAMMA / np.pi) / ((e[j] - xi[iy, ix]) ** 2 + GAMMA ** 2)

    qs = [(1, 2), (4, 0), (2, 1)]
    ms = [1, 5, 13]
    got = oracle.chi_grid(xi, NEPS, EMIN, EMAX, GAMMA, [q[0] for q in qs], [q[1] for q in qs], ms)
    for iq, (qx, qy) in enumerate(qs):
        for im, m in enumerate(ms):
            tot = sum(A(iy, ix, j) * A((iy + qy) % nky, (ix + qx) % nkx, j + m)
                      for iy in range(nky) for ix in range(nkx) for j in range(NEPS - m) if occ[j] and not occ[j + m])
            assert got[iq, im] == pytest.approx(-d / (nkx * nky) * tot, rel=1e-12)


def test_band_on_an_odd_grid_is_the_closed_form():
    nkx, nky = 7, 9
    eps = oracle.band_tb(0.4, -0.1, 0.03, nkx, nky)
    kx = 2 * np.pi * np.arange(nkx) / nkx
    ky = 2 * np.pi * np.arange(nky) / nky
    KX, KY = np.meshgrid(kx, ky)
    ref = -0.8 * (np.cos(KX) + np.cos(KY)) + 0.4 * np.cos(KX) * np.cos(KY) - 0.06 * (np.cos(2 * KX) + np.cos(2 * KY))
    assert np.allclose(eps, ref, rtol=0, atol=1e-15)


def test_periodic_image_identity():
    """A table repeating with index period n on a 2n grid (n = 6): every k of
    the small grid appears four times, so chi of the big grid at q equals
    chi of the small grid at q mod n."""
    n = 6
    small = oracle.band_tb(0.4, -0.1, 0.03, n, n) - 0.1
    big = np.tile(small, (2, 2))
    qx = np.array([0, 1, 7, 11, 6])
    qy = np.array([2, 9, 4, 1, 6])
    ms = [2, 7]
    a = oracle.chi_grid(big, NEPS, EMIN, EMAX, GAMMA, qx, qy, ms)
    b = oracle.chi_grid(small, NEPS, EMIN, EMAX, GAMMA, qx % n, qy % n, ms)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-15 * np.abs(b).max())
