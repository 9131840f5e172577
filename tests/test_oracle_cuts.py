"""Pins of the oracle's cuts (Fig. 2(a) high-symmetry path, Fig. 5 zone
envelope and its Lorentzian fit) against facts fixed independently of it:
exact Lorentzian data, planted maps with known maxima, the geometry of the
Gamma-X-M path, and scipy's general least-squares solver."""
import numpy as np
import pytest
from scipy.optimize import curve_fit

import oracle


def test_fit_recovers_k0_from_exact_lorentzian():
    q = np.array([0.3, 1.1, 2.4, 3.9, 5.2])
    for k0 in (0.4, 1.89, 7.5):
        y = 1.0 / (1.0 + (q / k0) ** 2)
        assert oracle.envelope_fit(q, y) == pytest.approx(k0, rel=1e-10)


def test_fit_matches_general_least_squares_on_noisy_data():
    rng = np.random.Generator(np.random.PCG64(17))
    q = np.sort(rng.uniform(0.1, 6.0, size=9))
    y = 1.0 / (1.0 + (q / 1.89) ** 2) * (1.0 + 0.1 * rng.normal(size=q.size))
    popt, _ = curve_fit(lambda qq, k0: 1.0 / (1.0 + (qq / k0) ** 2), q, y, p0=[1.0], xtol=1e-15, ftol=1e-15,
                        gtol=1e-15)
    assert oracle.envelope_fit(q, y) == pytest.approx(abs(popt[0]), rel=1e-7)


def test_fit_at_the_range_ends():
    q = np.array([1.0, 2.0, 3.0])
    # flat data: no decay, u -> 0, k0 at its upper end 1/sqrt(1e-8) = 1e4
    assert oracle.envelope_fit(q, np.ones(3)) == pytest.approx(1e4, rel=1e-9)


@pytest.mark.parametrize("direction", [0, 1])
def test_zone_envelope_on_a_planted_map(direction):
    nk, zx, zy, k0, qs = 16, 5, 5, 1.3, 0.7
    plane = np.zeros((zy * nk, zx * nk))
    gx, gy = zx * nk // 2, zy * nk // 2
    step = 2 * np.pi / nk * (np.sqrt(2) if direction else 1.0) * qs
    # one offset s inside each segment; the central one at q = 0, so that the
    # normalised maxima are exactly 1 / (1 + (q/k0)^2)
    planted = [0, nk // 2 + 5, nk // 2 + nk + 11]
    for s in planted:
        q = s * step
        X, Y = gx + s, (gy + s if direction else gy)
        plane[Y, X] = -2.5 / (1.0 + (q / k0) ** 2)
    # a tie later in segment 1 must lose to the first maximum
    s_tie = planted[1] + 2
    plane[gy + s_tie if direction else gy, gx + s_tie] = plane[gy + planted[1] if direction else gy, gx + planted[1]]
    env = oracle.zone_envelope(plane, nk, zx, zy, direction, qs)
    assert list(env["X"]) == [gx + s for s in planted]
    assert list(env["Y"]) == [gy + s if direction else gy for s in planted]
    assert env["c_max"] == 2.5
    assert env["k0"] == pytest.approx(k0, rel=1e-9)


def test_zone_envelope_with_zones_inside_the_grid():
    """k-grid spanning kzones zones: the zone width is nk / kzones steps and a
    half zone left at the grid edge is not used."""
    nk, kz = 32, 4
    plane = np.zeros((nk, nk))
    plane[nk // 2, nk // 2 + 1] = -1.0          # central half zone [0, 4)
    plane[nk // 2, nk // 2 + 4 + 3] = -0.5      # zone 1: [4, 12)
    plane[nk // 2, nk - 1] = -9.0               # the edge half zone: ignored
    env = oracle.zone_envelope(plane, nk, 1, 1, 0, 1.0, kzones=kz)
    assert list(env["X"]) == [nk // 2 + 1, nk // 2 + 7]
    assert env["c_max"] == 1.0 and list(env["y"]) == [1.0, 0.5]
    assert env["q"][1] == pytest.approx(7 * 2 * np.pi / (nk // kz), rel=1e-15)


@pytest.mark.parametrize("nk,zones,kz", [(16, 1, 1), (16, 3, 1), (32, 1, 4)])
def test_high_symmetry_path_geometry(nk, zones, kz):
    X, Y = oracle.high_symmetry_path(nk, zones, zones, kz)
    W = nk // kz
    n = zones * nk
    g = n // 2
    assert X.size == 3 * W // 2 + 1
    assert (X[0], Y[0]) == (g, g) and (X[-1], Y[-1]) == (g, g)          # Gamma at both ends
    assert (X[W // 2], Y[W // 2]) == ((g + W // 2) % n, g)             # X = (pi, 0)
    assert (X[W], Y[W]) == ((g + W // 2) % n, (g + W // 2) % n)        # M = (pi, pi)
    # unwrapped steps: unit along the axes, (1, 1) on the diagonal
    dx = (np.diff(X.astype(int)) + n // 2) % n - n // 2
    dy = (np.diff(Y.astype(int)) + n // 2) % n - n // 2
    assert np.all(np.abs(dx) + np.abs(dy) >= 1) and np.all(np.abs(dx) <= 1) and np.all(np.abs(dy) <= 1)
    assert np.all(dx[:W // 2] == 1) and np.all(dy[W // 2:W] == 1)
    assert np.all(dx[W:] == -1) and np.all(dy[W:] == -1)
