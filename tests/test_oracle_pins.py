"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: brute force
with explicit delta masks, exact discrete identities (q-sum, energy-sum),
closed forms (flat band, 2D free electrons, form-factor quadrature, pole-pair
Kramers-Kronig) and exact symmetries.  A plausible slip in the oracle (a
dropped term, a wrong sign, an off-by-one window edge, a transposed index, a
wrong constant) fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


def lor(e, xi, g):
    """Eq. (5): unit-area Lorentzian of half width g centred on xi."""
    return (g / np.pi) / ((e - xi) ** 2 + g * g)


def spectral_table(xi, neps, emin, emax, g):
    """A[k, j] written out by the test itself (not taken from the oracle)."""
    d = (emax - emin) / neps
    e = emin + (np.arange(neps) + 0.5) * d
    return lor(e[None, :], xi.reshape(-1, 1), g), e, d


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("shape,neps,emin,emax,g", [((4, 6), 12, -0.7, 0.5, 0.11),
                                                    ((8, 8), 16, -1.0, 1.0, 0.2),
                                                    ((2, 4), 6, -0.3, 0.9, 0.05)])
def test_brute_force_quadruple_loop(shape, neps, emin, emax, g):
    """Eq. (9) on a periodic grid, as a quadruple sum with explicit masks
    [k' = k + q], [j' = j + m], [e_j <= 0] and [e_j' > 0]."""
    rng = np.random.default_rng(7)
    nky, nkx = shape
    xi = rng.uniform(-1.0, 1.0, size=shape)
    A, e, d = spectral_table(xi, neps, emin, emax, g)
    A = A.reshape(nky, nkx, neps)
    ms = np.arange(-1, neps + 2)
    qy, qx = np.meshgrid(np.arange(nky), np.arange(nkx), indexing="ij")
    got = oracle.chi_grid(xi, neps, emin, emax, g, qx.ravel(), qy.ravel(), ms)
    nk = nkx * nky
    for iq in range(nk):
        Qx, Qy = qx.ravel()[iq], qy.ravel()[iq]
        for im, m in enumerate(ms):
            tot = 0.0
            for ky in range(nky):
                for kx in range(nkx):
                    for ky2 in range(nky):
                        for kx2 in range(nkx):
                            if (kx2 - kx - Qx) % nkx or (ky2 - ky - Qy) % nky:
                                continue
                            for j in range(neps):
                                for j2 in range(neps):
                                    if j2 != j + m or not (e[j] <= 0.0 < e[j2]):
                                        continue
                                    tot += A[ky, kx, j] * A[ky2, kx2, j2]
            want = -d / nk * tot
            assert abs(got[iq, im] - want) <= 1e-14 * max(1.0, abs(want)), (iq, m)


# ---------------------------------------------------------- exact identities
def _tb_case(nkx, nky, neps, emin, emax, g, fill=1.15, t=(0.42, -0.10, 0.05)):
    eps = oracle.band_tb(*t, nkx, nky)
    mu = oracle.mu_solve(eps, g, fill)
    return eps - mu


@pytest.mark.parametrize("nkx,nky,neps,emin,emax", [(16, 12, 24, -1.0, 1.0), (8, 16, 20, -0.6, 1.4)])
def test_q_sum_identity(nkx, nky, neps, emin, emax):
    """Fig. 2(b) quantity: (1/Nk) sum_q Im chi(q, m) = -d sum_j D_P(j) D_H(j + m),
    with D the k-averaged occupied / unoccupied spectral weight."""
    g = 0.07
    xi = _tb_case(nkx, nky, neps, emin, emax, g)
    ms = np.arange(0, neps + 1)
    full = oracle.chi_full(xi, neps, emin, emax, g, ms)
    A, e, d = spectral_table(xi, neps, emin, emax, g)
    D = A.mean(axis=0)
    occ = e <= 0
    DP = np.where(occ, D, 0.0)
    DH = np.where(~occ, D, 0.0)
    for im, m in enumerate(ms):
        want = -d * sum(DP[j] * DH[j + m] for j in range(neps) if j + m < neps)
        got = full[im].mean()
        assert abs(got - want) <= 1e-14 * max(abs(want), 1e-3), m


def test_chi_qmean_matches_the_q_average_of_the_full_grid():
    g = 0.07
    xi = _tb_case(16, 8, 32, -1.0, 1.2, g)
    ms = np.array([0, 1, 2, 5, 17, 31, 32, 40])
    full = oracle.chi_full(xi, 32, -1.0, 1.2, g, ms)
    got = oracle.chi_qmean(xi, 32, -1.0, 1.2, g, ms)
    want = full.mean(axis=(1, 2))
    assert np.allclose(got, want, rtol=1e-13, atol=1e-17)
    assert got[0] == 0 and got[-2] == 0 and got[-1] == 0 and np.all(got[1:-2] < 0)


def test_energy_sum_identity():
    """Summing over every lag pairs each occupied point with each unoccupied one:
    sum_m Im chi(q, m) = -(d/Nk) sum_k nP(k) nH(k + q)."""
    nkx, nky, neps, emin, emax, g = 12, 10, 18, -0.9, 0.8, 0.09
    xi = _tb_case(nkx, nky, neps, emin, emax, g)
    ms = np.arange(1, neps)
    full = oracle.chi_full(xi, neps, emin, emax, g, ms)
    A, e, d = spectral_table(xi, neps, emin, emax, g)
    occ = e <= 0
    nP = A[:, occ].sum(axis=1).reshape(nky, nkx)
    nH = A[:, ~occ].sum(axis=1).reshape(nky, nkx)
    for qy in range(nky):
        for qx in range(nkx):
            shifted = np.roll(np.roll(nH, -qy, axis=0), -qx, axis=1)  # nH(k + q)
            want = -d / (nkx * nky) * np.sum(nP * shifted)
            got = full[:, qy, qx].sum()
            assert abs(got - want) <= 1e-13 * abs(want)


def test_empty_lags_are_exact_zero_and_sign():
    """Im chi(q, 0) = 0 (no transitions, Sec. 4), lags beyond the window are 0,
    and every term is positive so Im chi < 0 for 1 <= m < Neps."""
    nkx, nky, neps = 8, 8, 16
    xi = _tb_case(nkx, nky, neps, -1.0, 1.0, 0.05)
    ms = np.array([-3, -1, 0, 1, 5, 15, 16, 17, 40])
    full = oracle.chi_full(xi, neps, -1.0, 1.0, 0.05, ms)
    for im, m in enumerate(ms):
        if 1 <= m < neps:
            assert np.all(full[im] < 0.0)
        else:
            assert np.all(full[im] == 0.0)


def test_c4v_and_inversion_symmetry():
    """The square-lattice band is C4v symmetric and so is chi (Figs. 3-4)."""
    n, neps = 16, 24
    xi = _tb_case(n, n, neps, -1.2, 1.2, 0.06)
    full = oracle.chi_full(xi, neps, -1.2, 1.2, 0.06, np.array([1, 4, 9, 17]))
    idx = np.arange(n)
    neg = (-idx) % n
    tol = 1e-12 * np.abs(full).max()
    for sl in full:
        assert np.abs(sl - sl.T).max() <= tol                 # qx <-> qy
        assert np.abs(sl - sl[:, neg]).max() <= tol           # qx -> -qx
        assert np.abs(sl - sl[neg, :]).max() <= tol           # qy -> -qy
        assert np.abs(sl - sl[neg][:, neg]).max() <= tol      # inversion


def test_reciprocal_lattice_periodicity_and_zone_replication():
    """With |M|^2 = 1 the extended map repeats the first zone exactly, and a q
    shifted by a reciprocal lattice vector gives the same chi."""
    nkx, nky, neps = 8, 6, 12
    xi = _tb_case(nkx, nky, neps, -1.0, 1.0, 0.08)
    a = oracle.chi_grid(xi, neps, -1.0, 1.0, 0.08, [3, 3 + nkx, 3 - 2 * nkx], [2, 2 - nky, 2 + 3 * nky], [3])
    assert a[0, 0] == a[1, 0] == a[2, 0]
    full = oracle.chi_full(xi, neps, -1.0, 1.0, 0.08, np.array([2, 5]))
    ext = oracle.extend(full, 5, 3, 0, 0.6)
    assert ext.shape == (2, 3 * nky, 5 * nkx)
    for zy in range(3):
        for zx in range(5):
            blk = ext[:, zy * nky:(zy + 1) * nky, zx * nkx:(zx + 1) * nkx]
            assert np.array_equal(blk, ext[:, :nky, :nkx])
    # Gamma-centred: X = Zx*Nkx/2 is h = 0, first-zone index u = 0.
    assert ext[0, 3 * nky // 2, 5 * nkx // 2] == full[0, 0, 0]
    h, u = oracle.zone_axis(nkx, 5)
    assert h[5 * nkx // 2] == 0.0 and u[5 * nkx // 2] == 0 and h[0] == -2.5


# ------------------------------------------------------------- closed forms
def test_flat_band_mu_closed_form():
    """Flat band (t = t' = t'' = 0): n(mu) = 1 + 2 atan(mu/G)/pi, so
    mu = G tan(pi (n - 1) / 2)."""
    g = 0.05
    eps = np.zeros((8, 8))
    for fill in (0.3, 1.0, 1.15, 1.7):
        want = g * math.tan(math.pi * (fill - 1.0) / 2.0)
        assert abs(oracle.mu_solve(eps, g, fill) - want) < 2e-14


def test_half_filling_mu_is_zero():
    """t-only band on an even grid: eps(k + (pi, pi)) = -eps(k), so n(0) = 1."""
    eps = oracle.band_tb(0.4, 0.0, 0.0, 32, 16)
    assert abs(oracle.mu_solve(eps, 0.03, 1.0)) < 1e-13
    mu = oracle.mu_solve(eps, 0.03, 1.2)
    assert abs(oracle.filling(eps, 0.03, mu) - 1.2) < 1e-12


def test_flat_band_energy_quadrature_converges():
    """Flat band: chi does not depend on q and is the midpoint rule of
    -int L(e - xi0) L(e + w - xi0) de over the occupied window (Eq. (A3));
    the error falls as d^2."""
    g, xi0, emin, emax, w = 0.05, -0.07, -1.0, 1.0, 0.25
    errs = []
    for neps in (128, 256, 512):
        d = (emax - emin) / neps
        m = int(round(w / d))
        xi = np.full((4, 4), xi0)
        c = oracle.chi_grid(xi, neps, emin, emax, g, [0, 1, 3], [0, 2, 1], [m])
        assert np.all(c == c[0, 0])
        lo, hi = max(-w, emin), min(0.0, emax - w)
        ref, _ = integrate.quad(lambda e: lor(e, xi0, g) * lor(e + w, xi0, g), lo, hi,
                                epsabs=1e-15, epsrel=1e-12, points=[xi0, xi0 - w], limit=400)
        errs.append(abs(c[0, 0] + ref))
    assert errs[0] < 2e-5 * ref
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5


@pytest.mark.slow
def test_free_electron_lindhard_limit():
    """Normalisation: near the band bottom the t-only band is a 2D electron gas
    with m* = 1/(2t); for small G the oracle approaches
    Im chi = -(m* kF / (2 pi^2 q)) [sqrt(1 - nu_-^2)_+ - sqrt(1 - nu_+^2)_+],
    nu_pm = (m* w / q +- q / 2) / kF, per site per spin."""
    t, n, neps, emin, emax, g = 1.0, 512, 256, -0.5, 0.5, 0.02
    eps = oracle.band_tb(t, 0.0, 0.0, n, n)
    kf = 0.5
    mu = -4.0 * t + t * kf * kf          # eps ~ -4t + t k^2
    xi = eps - mu
    mstar = 1.0 / (2.0 * t)
    qi = 24
    q = 2.0 * math.pi * qi / n
    d = (emax - emin) / neps
    ms = np.array([8, 16, 24, 32, 40])
    got = oracle.chi_pairs(xi, neps, emin, emax, g, [qi] * ms.size, [0] * ms.size, ms)
    for val, m in zip(got, ms):
        w = m * d
        num = mstar * w / q
        nm_, np_ = (num - q / 2) / kf, (num + q / 2) / kf
        sq = lambda v: math.sqrt(1.0 - v * v) if abs(v) < 1.0 else 0.0
        want = -(mstar * kf / (2.0 * math.pi ** 2 * q)) * (sq(nm_) - sq(np_))
        assert abs(val - want) < 0.12 * abs(want), (m, val, want)


def test_form_factor_matches_quadrature():
    """Eq. (3) for phi = (x^2 - y^2) exp(-r^2/(2 w^2)): closed form vs a 2D
    trapezoid quadrature of int |phi|^2 cos(Q.r) / int |phi|^2."""
    w = 0.6
    L, n = 12 * w, 801
    x = np.linspace(-L, L, n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    dens = ((X * X - Y * Y) ** 2) * np.exp(-(X * X + Y * Y) / (w * w))
    norm = np.trapezoid(np.trapezoid(dens, x, axis=1), x)
    for Qx, Qy in [(0.0, 0.0), (1.3, 0.0), (0.0, 2.2), (2.5, 1.1), (-3.9, 4.4), (6.28, 6.28), (9.4, -1.0)]:
        num = np.trapezoid(np.trapezoid(dens * np.cos(Qx * X + Qy * Y), x, axis=1), x)
        assert abs(oracle.form_factor(Qx, Qy, w) - num / norm) < 1e-12


def _pole_pair(wv, w0, eta):
    c = 1.0 / (wv - w0 + 1j * eta) - 1.0 / (wv + w0 + 1j * eta)
    return c.real, c.imag


def test_kramers_kronig_pole_pair_converges():
    """Sec. 4 real part: a causal pole pair chi = 1/(w - w0 + i eta) - 1/(w + w0 + i eta)
    has odd Im and even Re.  On the lag grid the alternate-point rule recovers
    Re to within the truncated tail of Im beyond the last lag, which falls as
    wmax^-3 (Im ~ w^-3)."""
    w0, eta, d = 1.0, 0.2, 0.01
    errs = []
    for wmax in (30.0, 60.0, 120.0):
        n = int(round(wmax / d))
        lag = np.arange(n)
        re_ex, im = _pole_pair(lag * d, w0, eta)
        sel = np.array([0, 50, 100, 150, 300, 777])
        re = oracle.kk_real(im, sel)
        errs.append(np.abs(re - re_ex[sel]).max())
    assert errs[1] < 2e-6
    assert errs[1] < errs[0] / 6 and errs[2] < errs[1] / 6


def test_kramers_kronig_static_sign():
    """Im chi <= 0 for w > 0 gives Re chi(q, 0) < 0 (static screening sign)."""
    nkx, nky, neps = 8, 8, 32
    xi = _tb_case(nkx, nky, neps, -1.0, 1.0, 0.05)
    full = oracle.chi_full(xi, neps, -1.0, 1.0, 0.05, np.arange(neps))
    re0 = oracle.kk_real(np.moveaxis(full, 0, -1), [0])
    assert np.all(re0 < 0.0)


def test_rpa_identities():
    """chi_RPA = chi / (1 - U chi): U = 0 is the identity, and in general
    1/chi_RPA - 1/chi = -U (the Dyson form of the same relation)."""
    rng = np.random.default_rng(3)
    re = rng.uniform(-0.2, 0.1, 50)
    im = -rng.uniform(1e-4, 0.1, 50)
    i0, r0 = oracle.rpa(re, im, 0.0)
    assert np.array_equal(i0, im) and np.array_equal(r0, re)
    for U in (0.5, 1.5, 2.0):
        ir, rr = oracle.rpa(re, im, U)
        lhs = 1.0 / (rr + 1j * ir) - 1.0 / (re + 1j * im)
        assert np.abs(lhs + U).max() < 1e-12
        D = (1 - U * re) ** 2 + (U * im) ** 2
        assert np.abs(ir * D - im).max() < 1e-15


def test_config_band_matches_paper_band_width():
    """The synthetic band stands in for the Cu-O band, which the paper gives as
    running from about -1.4 eV to 1.9 eV (Sec. 3); fixture tests/golden/band_range.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "band_range.txt")
    vals = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    eps = oracle.band_tb(0.42, -0.10, 0.05, 256, 256)
    assert abs(eps.min() - vals["band_min_eV"]) < 0.1
    assert abs(eps.max() - vals["band_max_eV"]) < 0.1
