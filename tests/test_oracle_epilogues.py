"""Pins of the oracle's Coulomb RPA, structure factor and peak search
(CPU only).  Each check comes from mathematics that does not reuse the
oracle's own expression: limits, identities written in real arithmetic,
detailed balance, brute force."""
import numpy as np

import oracle


def _chi(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.uniform(-0.3, 0.1, size=shape)
    im = -rng.uniform(0.0, 0.2, size=shape)
    return re, im


def test_coulomb_v_is_inverse_square_of_the_zone_momentum():
    hx, ux = oracle.zone_axis(8, 3)
    hy, uy = oracle.zone_axis(4, 5)
    V = oracle.coulomb_v(hx, hy, 2.0)
    Y, X = 7, 5
    Q2 = (2 * np.pi * hx[X]) ** 2 + (2 * np.pi * hy[Y]) ** 2
    assert np.isclose(V[Y, X] * Q2, 2.0, rtol=1e-15)
    # Q = 0 sits at the centre of the extended grid
    assert np.isinf(V[10, 12]) and hx[12] == 0.0 and hy[10] == 0.0
    assert np.isfinite(V).sum() == V.size - 1


def test_coulomb_v_with_a_kz_component():
    """A kz plane of a 3D grid: |Q|^2 gains (2 pi hz)^2, so V is finite at
    the in-plane centre and V |Q|^2 = v everywhere; hz = 0 is the 2D map."""
    hx, _ = oracle.zone_axis(8, 3)
    hy, _ = oracle.zone_axis(4, 5)
    hz = -0.25
    V = oracle.coulomb_v(hx, hy, 2.0, hz)
    Q2 = (2 * np.pi) ** 2 * (hx[None, :] ** 2 + hy[:, None] ** 2 + hz ** 2)
    assert np.allclose(V * Q2, 2.0, rtol=1e-15, atol=0)
    assert np.isfinite(V).all() and V[10, 12] == 2.0 / (2 * np.pi * hz) ** 2
    assert np.array_equal(oracle.coulomb_v(hx, hy, 2.0, 0.0), oracle.coulomb_v(hx, hy, 2.0))
    re, im = _chi((3, 20, 24), 11)
    imr, rer = oracle.rpa_coulomb(re, im, hx, hy, 0.7, hz)
    # Dyson identity in real arithmetic: chi = chi_RPA (1 - V chi) component by component
    V = V * (0.7 / 2.0)
    a, b = 1.0 - V * re, V * im
    d = a * a + b * b
    assert np.allclose(imr, im / d, rtol=1e-13, atol=1e-16)
    assert np.allclose(rer, (re * a - V * im * im) / d, rtol=1e-13, atol=1e-16)


def test_rpa_coulomb_identities():
    hx, _ = oracle.zone_axis(8, 3)
    hy, _ = oracle.zone_axis(8, 3)
    re, im = _chi((4, 24, 24), 1)
    v = 0.7
    imr, rer = oracle.rpa_coulomb(re, im, hx, hy, v)
    V = oracle.coulomb_v(hx, hy, v)[None]
    fin = np.isfinite(V) & np.ones_like(re, dtype=bool)
    V = np.where(np.isfinite(V), V, 0.0)
    # |1 - V chi|^2 written in real arithmetic
    D = (1 - V * re) ** 2 + (V * im) ** 2
    assert np.allclose((imr * D)[fin], im[fin], rtol=1e-12, atol=0)
    assert np.allclose((rer * D)[fin], (re * (1 - V * re) - V * im * im)[fin], rtol=1e-12, atol=1e-15)
    # the Q = 0 column takes the infinite-interaction limit
    assert np.all(imr[~fin] == 0.0) and np.all(rer[~fin] == 0.0)
    # no interaction: chi itself
    i0, r0 = oracle.rpa_coulomb(re, im, hx, hy, 0.0)
    assert np.array_equal(i0[fin], im[fin]) and np.array_equal(r0[fin], re[fin])
    # screening: |chi_RPA| < |chi| for Re chi < 0 (repulsive V > 0)
    neg = fin & (re < 0)
    assert np.all(np.abs(rer + 1j * imr)[neg] < np.abs(re + 1j * im)[neg])


def test_rpa_coulomb_approaches_its_limit_near_q0():
    # V -> infinity: chi_RPA -> -1/V -> 0 continuously
    hx = np.array([0.0, 1e-4, 1e-3])
    hy = np.array([0.0])
    re = np.full((1, 1, 3), -0.2)
    im = np.full((1, 1, 3), -0.05)
    imr, rer = oracle.rpa_coulomb(re, im, hx, hy, 1.0)
    assert imr[0, 0, 0] == 0 and rer[0, 0, 0] == 0
    Vs = oracle.coulomb_v(hx, hy, 1.0)[0, 1:]
    assert np.allclose(rer[0, 0, 1:], -1.0 / Vs, rtol=1e-3)


def test_structure_factor_limits_and_detailed_balance():
    omega = np.array([0.0, 0.05, 0.2, 0.5, 1.0])
    rng = np.random.Generator(np.random.PCG64(3))
    im = -rng.uniform(0.01, 0.1, size=(5, 3, 4))
    im[0] = 0.0
    # zero temperature: -Im / pi for omega > 0
    s0 = oracle.structure_factor(im, omega, 0.0)
    assert np.allclose(s0[1:], -im[1:] / np.pi, rtol=4e-16, atol=0) and np.all(s0[0] == 0.0)
    # detailed balance: S(-w) = exp(-w/kT) S(w) with Im chi odd in w
    kT = 0.03
    sp = oracle.structure_factor(im[1:], omega[1:], kT)
    sm = oracle.structure_factor(-im[1:], -omega[1:], kT)
    ratio = np.exp(-omega[1:] / kT)[:, None, None]
    assert np.allclose(sm, ratio * sp, rtol=1e-12)
    # classical limit: S -> -Im kT / (pi w) for kT >> w
    big = 1e6
    sc = oracle.structure_factor(im[1:], omega[1:], big)
    assert np.allclose(sc * np.pi * omega[1:, None, None] / (big * -im[1:]), 1.0, rtol=1e-5)
    # S >= 0 whenever -Im chi >= 0 and omega > 0
    assert np.all(oracle.structure_factor(im, omega, 0.1)[1:] >= 0.0)


def test_peak_index_brute_force_first_on_ties():
    rng = np.random.Generator(np.random.PCG64(4))
    im = -np.round(rng.uniform(0, 1, size=(6, 5, 7)), 1)  # many ties
    got = oracle.peak_index(im)
    for y in range(5):
        for x in range(7):
            col = list(-im[:, y, x])
            best = max(col)
            assert got[y, x] == col.index(best)
    assert got.dtype == np.int32
