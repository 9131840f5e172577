"""Pins of the oracle's several-band forms (Eq. (4): summed spectral
function; Eq. (2): band-pair sum) against facts that do not come from it:
reduction to the single-band oracle, scaling of identical bands, the
bilinearity that ties the two forms together, and a brute-force double sum on
a tiny grid."""
import numpy as np
import pytest

import oracle
from paper_1208_3210_amd import workloads as W

NEPS, EMIN, EMAX, GAMMA = 32, -1.5, 1.5, 0.12


def setup(nk=8, nb=2, rho=False):
    eps = W.multiband_tables(nk, nb, seed=3)
    mu = oracle.mu_solve_bands(eps, GAMMA, 1.1)
    r = None
    if rho:
        r = np.stack([W.momentum_density_dx2y2(nk, nk, 2, 0.6), W.density_s(nk, nk, 2, 0.5)][:nb])
    return eps - mu, r


def q_list(nk):
    qy, qx = np.meshgrid(np.arange(nk), np.arange(nk), indexing="ij")
    return qx.ravel(), qy.ravel()


LAGS = np.array([1, 2, 5, 9, 17, 31])


def test_one_band_reduces_to_the_single_band_oracle():
    xi, r = setup(nb=1, rho=True)
    qx, qy = q_list(8)
    a = oracle.chi_grid_mb(xi, NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS, rho=r)
    b = oracle.chi_grid(xi[0], NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS, rho=r[0])
    assert np.allclose(a, b, rtol=1e-13, atol=1e-15 * np.abs(b).max())
    c = oracle.chi_grid_mb(xi, NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS, rho=r, pair_weight=[[1.0]])
    assert np.allclose(c, b, rtol=1e-13, atol=1e-15 * np.abs(b).max())


def test_identical_bands_scale_by_four():
    xi, _ = setup(nb=1)
    two = np.concatenate([xi, xi])
    qx, qy = q_list(8)
    a = oracle.chi_grid_mb(two, NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS)
    b = oracle.chi_grid(xi[0], NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS)
    assert np.allclose(a, 4.0 * b, rtol=1e-13, atol=1e-15 * np.abs(b).max())


def test_pair_form_is_bilinear_in_the_bands():
    """All weights 1 gives the summed form; the identity gives the sum of the
    bands' own single-band results."""
    xi, r = setup(nb=3, rho=False)
    qx, qy = q_list(8)
    summed = oracle.chi_grid_mb(xi, NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS)
    ones = oracle.chi_grid_mb(xi, NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS, pair_weight=np.ones((3, 3)))
    sc = np.abs(summed).max()
    assert np.abs(ones - summed).max() <= 1e-13 * sc
    diag = oracle.chi_grid_mb(xi, NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS, pair_weight=np.eye(3))
    own = sum(oracle.chi_grid(xi[n], NEPS, EMIN, EMAX, GAMMA, qx, qy, LAGS) for n in range(3))
    assert np.abs(diag - own).max() <= 1e-13 * np.abs(own).max()


def test_pair_form_against_a_brute_force_double_sum():
    nk = 4
    xi, r = setup(nk=nk, nb=2, rho=True)
    w = np.array([[0.7, 0.2], [1.3, 0.4]])
    d = (EMAX - EMIN) / NEPS
    e = EMIN + (np.arange(NEPS) + 0.5) * d
    occ = e <= 0.0

    def A(n, iy, ix, j):
        return r[n, iy, ix] * (GAMMA / np.pi) / ((e[j] - xi[n, iy, ix]) ** 2 + GAMMA ** 2)

    got = oracle.chi_grid_mb(xi, NEPS, EMIN, EMAX, GAMMA, [1, 3], [2, 0], [1, 6, 20], rho=r, pair_weight=w)
    for iq, (qx, qy) in enumerate([(1, 2), (3, 0)]):
        for im, m in enumerate([1, 6, 20]):
            tot = 0.0
            for nu in range(2):
                for mu in range(2):
                    for iy in range(nk):
                        for ix in range(nk):
                            for j in range(NEPS - m):
                                if occ[j] and not occ[j + m]:
                                    tot += w[nu, mu] * A(nu, iy, ix, j) * A(mu, (iy + qy) % nk, (ix + qx) % nk, j + m)
            assert got[iq, im] == pytest.approx(-d / nk ** 2 * tot, rel=1e-12)


def test_common_chemical_potential_of_identical_bands():
    xi, _ = setup(nb=1)
    eps = xi + 0.3
    assert oracle.mu_solve_bands(np.concatenate([eps, eps]), GAMMA, 1.6) == pytest.approx(
        oracle.mu_solve(eps[0], GAMMA, 0.8), abs=1e-13)


# ---- band-pair maps |M^{nu,mu}(Q)|^2 (Eqs. (2), (3)) ---------------------
def _maps(nb, nk, zx, zy, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.5, size=(nb, nb, zy * nk, zx * nk))


def test_pair_maps_with_constant_maps_reduce_to_pair_weights():
    """Maps that do not vary with Q give the constant-weight pair sum,
    repeated over the zones."""
    xi, r = setup(nb=2, rho=True)
    w = np.array([[0.7, 0.2], [1.3, 0.4]])
    m2 = np.broadcast_to(w[:, :, None, None], (2, 2, 8, 24))
    got = oracle.chi_pair_maps(xi, NEPS, EMIN, EMAX, GAMMA, LAGS, m2, 3, 1, rho=r)
    ref = oracle.extend(oracle.chi_full_mb(xi, NEPS, EMIN, EMAX, GAMMA, LAGS, rho=r, pair_weight=w), 3, 1, 0, 0.0)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_pair_maps_of_one_band_reduce_to_the_orbital_form_factor():
    """One band with the d-wave orbital's |M(Q)|^2 tabulated gives the
    analytic form-factor path of ``extend``."""
    xi, _ = setup(nb=1)
    m2 = oracle.m2_extended(8, 8, 3, 5, 1, 0.6)[None, None]
    got = oracle.chi_pair_maps(xi, NEPS, EMIN, EMAX, GAMMA, LAGS, m2, 3, 5)
    ref = oracle.extend(oracle.chi_full(xi[0], NEPS, EMIN, EMAX, GAMMA, LAGS), 3, 5, 1, 0.6)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_pair_maps_are_linear_in_the_maps():
    xi, _ = setup(nb=2)
    a, b = _maps(2, 8, 1, 3, 5), _maps(2, 8, 1, 3, 6)
    fa = oracle.chi_pair_maps(xi, NEPS, EMIN, EMAX, GAMMA, LAGS, a, 1, 3)
    fb = oracle.chi_pair_maps(xi, NEPS, EMIN, EMAX, GAMMA, LAGS, b, 1, 3)
    fab = oracle.chi_pair_maps(xi, NEPS, EMIN, EMAX, GAMMA, LAGS, 0.3 * a + 1.7 * b, 1, 3)
    assert np.abs(fab - (0.3 * fa + 1.7 * fb)).max() <= 1e-13 * np.abs(fab).max()


def test_pair_maps_against_a_brute_force_double_sum():
    """Every extended point of a tiny grid (4 x 4 k, two bands, 3 x 3 zones)
    summed directly: pairs, k and the occupied energies, each term weighted by
    its pair's map at that Q."""
    nk, zx, zy = 4, 3, 3
    xi, r = setup(nk=nk, nb=2, rho=True)
    m2 = _maps(2, nk, zx, zy, 7)
    d = (EMAX - EMIN) / NEPS
    e = EMIN + (np.arange(NEPS) + 0.5) * d
    occ = e <= 0.0

    def A(n, iy, ix, j):
        return r[n, iy, ix] * (GAMMA / np.pi) / ((e[j] - xi[n, iy, ix]) ** 2 + GAMMA ** 2)

    lags = [1, 6, 20]
    got = oracle.chi_pair_maps(xi, NEPS, EMIN, EMAX, GAMMA, lags, m2, zx, zy, rho=r)
    for Y in (0, 5, 11):
        for X in (2, 7, 9):
            # first-zone point of the extended point (the output grid is centred)
            qx, qy = (X - zx * nk // 2) % nk, (Y - zy * nk // 2) % nk
            for im, m in enumerate(lags):
                tot = 0.0
                for nu in range(2):
                    for mu in range(2):
                        for iy in range(nk):
                            for ix in range(nk):
                                for j in range(NEPS - m):
                                    if occ[j] and not occ[j + m]:
                                        tot += m2[nu, mu, Y, X] * A(nu, iy, ix, j) * A(mu, (iy + qy) % nk,
                                                                                        (ix + qx) % nk, j + m)
                assert got[im, Y, X] == pytest.approx(-d / nk ** 2 * tot, rel=1e-12)
