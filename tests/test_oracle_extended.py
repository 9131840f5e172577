"""Pins of the oracle's extended-momentum form (CPU only): momentum-density
weights on the spectral function (A(p, e) = rho(p) A_band(p, e), Eq. (4))
and a momentum grid spanning several Brillouin zones (Eq. (9) integrates
over all p).  Checks: brute force with the weights written out, the
unweighted reduction, exact quadratic scaling, zone-periodic replication,
the weighted q-sum identity."""
import numpy as np
import pytest

import oracle


def lor(e, xi, g):
    return (g / np.pi) / ((e - xi) ** 2 + g * g)


def test_weighted_brute_force():
    rng = np.random.default_rng(11)
    nky, nkx, neps, emin, emax, g = 4, 6, 10, -0.6, 0.7, 0.09
    xi = rng.uniform(-1.0, 1.0, size=(nky, nkx))
    rho = rng.uniform(0.0, 2.0, size=(nky, nkx))
    d = (emax - emin) / neps
    e = emin + (np.arange(neps) + 0.5) * d
    ms = np.arange(0, neps + 1)
    got = oracle.chi_full(xi, neps, emin, emax, g, ms, rho=rho)
    for im, m in enumerate(ms):
        for qy in range(nky):
            for qx in range(nkx):
                tot = 0.0
                for ky in range(nky):
                    for kx in range(nkx):
                        k2y, k2x = (ky + qy) % nky, (kx + qx) % nkx
                        for j in range(neps):
                            j2 = j + m
                            if j2 >= neps or not (e[j] <= 0.0 < e[j2]):
                                continue
                            tot += (rho[ky, kx] * lor(e[j], xi[ky, kx], g)) * (rho[k2y, k2x] * lor(e[j2], xi[k2y, k2x], g))
                want = -d * tot / (nkx * nky)
                assert abs(got[im, qy, qx] - want) <= 1e-14 * max(abs(want), 1e-3)


def test_unit_weights_and_quadratic_scaling():
    rng = np.random.default_rng(12)
    xi = rng.uniform(-1.0, 1.0, size=(8, 8))
    rho = rng.uniform(0.1, 1.0, size=(8, 8))
    ms = np.arange(1, 12)
    plain = oracle.chi_full(xi, 16, -1.0, 1.0, 0.1, ms)
    ones = oracle.chi_full(xi, 16, -1.0, 1.0, 0.1, ms, rho=np.ones((8, 8)))
    assert np.array_equal(plain, ones)
    a = oracle.chi_full(xi, 16, -1.0, 1.0, 0.1, ms, rho=rho)
    b = oracle.chi_full(xi, 16, -1.0, 1.0, 0.1, ms, rho=2.0 * rho)
    assert np.array_equal(b, 4.0 * a)


@pytest.mark.parametrize("kz", [2, 4])
def test_zone_periodic_band_replicates_the_first_zone(kz):
    n = 8
    t = (0.42, -0.10, 0.05)
    e1 = oracle.band_tb(*t, n, n)
    ez = oracle.band_tb(*t, n * kz, n * kz, kzones=kz)
    iy, ix = np.meshgrid(np.arange(n * kz), np.arange(n * kz), indexing="ij")
    assert np.allclose(ez, e1[iy % n, ix % n], rtol=0, atol=1e-14)
    mu = 0.05
    ms = np.array([1, 3, 7, 12])
    chi1 = oracle.chi_full(e1 - mu, 16, -2.0, 2.0, 0.1, ms)
    qy, qx = np.array([0, 3, n + 1, 2 * n - 1, kz * n - 2]), np.array([0, 5, 2 * n - 3, n, 1])
    got = oracle.chi_grid(ez - mu, 16, -2.0, 2.0, 0.1, qx, qy, ms)
    want = np.stack([chi1[:, y % n, x % n] for x, y in zip(qx, qy)])
    assert np.allclose(got, want, rtol=1e-12, atol=1e-17)


def test_weighted_q_sum_identity():
    rng = np.random.default_rng(13)
    xi = rng.uniform(-1.2, 1.2, size=(8, 16))
    rho = rng.uniform(0.0, 1.5, size=(8, 16))
    ms = np.array([0, 1, 2, 9, 20, 31, 40])
    full = oracle.chi_full(xi, 32, -1.0, 1.2, 0.07, ms, rho=rho)
    got = oracle.chi_qmean(xi, 32, -1.0, 1.2, 0.07, ms, rho=rho)
    assert np.allclose(got, full.mean(axis=(1, 2)), rtol=1e-13, atol=1e-17)


@pytest.mark.parametrize("kz", [2, 4])
def test_extended_grid_momentum_of_the_output_points(kz):
    """On a grid spanning kz zones per axis one step is kz/n reciprocal-lattice
    units: the point n/kz grid steps left of the centre is the reciprocal
    lattice vector G = (-1, 0), where a one-zone grid repeated over three
    zones has its point h = -1.  The form factor (Eq. (3)) and the
    Coulomb interaction must agree at that common momentum."""
    n, w = 16, 0.6
    hx_k, _ = oracle.zone_axis(n, 1, kz)
    hx_1, _ = oracle.zone_axis(n, 3)
    Xk = n // 2 - n // kz          # G = (-1, 0) on the kz-zone grid
    X1 = 3 * n // 2 - n            # h = -1 on the three-zone grid
    assert hx_k[Xk] == -1.0 and hx_1[X1] == -1.0
    m2k = oracle.m2_extended(n, n, 1, 1, 1, w, kz)
    m23 = oracle.m2_extended(n, n, 3, 3, 1, w)
    assert m2k[n // 2, Xk] == m23[3 * n // 2, X1]
    # |M(G)|^2 from the Gaussian orbital: F(Q) = exp(-s Q^2)(1 - 2 s Q^2 + s^2 Q^4) at Q = 2 pi, s = w^2/4
    s, Q2 = w * w / 4.0, (2 * np.pi) ** 2
    F = np.exp(-s * Q2) * (1 - 2 * s * Q2 + s * s * Q2 * Q2)
    assert np.isclose(m2k[n // 2, Xk], F * F, rtol=1e-13)
    # the interaction sees the same |Q|
    hy_k, _ = oracle.zone_axis(n, 1, kz)
    V = oracle.coulomb_v(hx_k, hy_k, 1.0)
    assert np.isclose(V[n // 2, Xk] * Q2, 1.0, rtol=1e-15)
