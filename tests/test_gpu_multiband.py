"""Several bands through the C ABI against the FP64 oracle: the summed
spectral function of Eq. (4) and the band-pair sum of Eq. (2), on the even
path (mirror-symmetric tables, extended zones with the orbital form factor)
and on the general path (tables without symmetry), the RPA path of the pair
sum, and argument errors.  Normwise tolerances as for the hot path."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {LH.LINDHARD_FP64: 1e-11, LH.LINDHARD_FP32C: 1e-5}
PRECS = [LH.LINDHARD_FP64, LH.LINDHARD_FP32C]
PAIRS = np.array([[1.0, 0.35, 0.0], [0.8, 0.5, 0.2], [0.0, 1.1, 0.6]])


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def cfg_of(symmetric, nb=3, pairs=True, rho=False):
    nk = 32
    eps = W.multiband_tables(nk, nb, seed=11)
    if not symmetric:
        rng = np.random.Generator(np.random.PCG64(12))
        eps = eps + rng.uniform(-0.05, 0.05, size=eps.shape)
    cfg = dict(eps_table=eps, n_bands=nb, filling=1.2, nkx=nk, nky=nk, neps=64, emin=-1.5, emax=1.5, gamma=0.08,
               omega=np.arange(1, 40, 2) * (3.0 / 64))
    if symmetric:
        cfg.update(zones=(3, 3), ff_kind=1, ff_width=0.6)
    if pairs:
        cfg["pair_weight"] = PAIRS[:nb, :nb]
    if rho:
        cfg["rho_table"] = np.stack([W.momentum_density_dx2y2(nk, nk, 1, 0.6), W.density_s(nk, nk, 1, 0.4),
                                     np.ones((nk, nk))][:nb])
    return cfg


def oracle_map(cfg):
    eps = np.asarray(cfg["eps_table"])
    mu = oracle.mu_solve_bands(eps, cfg["gamma"], cfg["filling"])
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    lags = np.rint(np.asarray(cfg["omega"]) / d).astype(np.int64)
    full = oracle.chi_full_mb(eps - mu, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags,
                              rho=cfg.get("rho_table"), pair_weight=cfg.get("pair_weight"))
    zx, zy = cfg.get("zones", (1, 1))
    return mu, oracle.extend(full, zx, zy, cfg.get("ff_kind", 0), cfg.get("ff_width", 0.0))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("pairs", [False, True])
def test_multiband_against_oracle(prec, symmetric, pairs):
    cfg = cfg_of(symmetric, pairs=pairs, rho=symmetric)
    mu, ref = oracle_map(cfg)
    plan = LH.Plan(precision=prec, **cfg)
    sched = plan.info.schedule.decode()
    assert (" even " in sched) == symmetric
    assert plan.info.mu == pytest.approx(mu, abs=1e-11)
    got = plan.exec()
    torch.cuda.synchronize()
    err = normwise(got.double().cpu().numpy(), ref)
    print("multiband prec=%d sym=%d pairs=%d err=%.3e %s" % (prec, symmetric, pairs, err, sched))
    assert err <= TOL[prec]
    again = plan.exec()
    torch.cuda.synchronize()
    assert torch.equal(got, again)
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_pair_sum_with_unit_weights_equals_summed_bands(prec):
    base = cfg_of(True, nb=2, pairs=False)
    a = LH.Plan(precision=prec, **base)
    b = LH.Plan(precision=prec, **dict(base, pair_weight=np.ones((2, 2))))
    x, y = a.exec(), b.exec()
    torch.cuda.synchronize()
    assert normwise(y.double().cpu().numpy(), x.double().cpu().numpy()) <= TOL[prec]
    a.close()
    b.close()


@pytest.mark.parametrize("prec", PRECS)
def test_pair_sum_rpa_path(prec):
    cfg = cfg_of(True, nb=2, pairs=True)
    cfg["want_rpa"] = True
    eps = np.asarray(cfg["eps_table"])
    mu = oracle.mu_solve_bands(eps, cfg["gamma"], cfg["filling"])
    neps = cfg["neps"]
    full = oracle.chi_full_mb(eps - mu, neps, cfg["emin"], cfg["emax"], cfg["gamma"], np.arange(neps),
                              pair_weight=cfg["pair_weight"])
    d = (cfg["emax"] - cfg["emin"]) / neps
    lags = np.rint(np.asarray(cfg["omega"]) / d).astype(np.int64)
    im1 = full[lags]
    re1 = np.moveaxis(oracle.kk_real(np.moveaxis(full, 0, -1), lags), -1, 0)
    im_ext = oracle.extend(im1, 3, 3, 1, 0.6)
    re_ext = oracle.extend(re1, 3, 3, 1, 0.6)
    imr, rer = oracle.rpa(re_ext, im_ext, 1.2)
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    re, gimr, grer = plan.rpa(1.2)
    torch.cuda.synchronize()
    errs = [normwise(x.double().cpu().numpy(), r) for x, r in ((im, im_ext), (re, re_ext), (gimr, imr), (grer, rer))]
    print("multiband rpa prec=%d errs=%s" % (prec, ["%.2e" % e for e in errs]))
    assert max(errs) <= TOL[prec]
    plan.close()


def test_multiband_argument_errors():
    cfg = cfg_of(True, nb=2)
    for bad in (dict(eps_table=None), dict(pair_weight=np.zeros((2, 2))), dict(pair_weight=-np.ones((2, 2))),
                dict(n_bands=LH.LINDHARD_MAX_BANDS + 1, eps_table=np.zeros((LH.LINDHARD_MAX_BANDS + 1, 32, 32)),
                     pair_weight=None)):
        c = dict(cfg, **bad)
        if c.get("eps_table") is None:
            c.update(t=0.4, tp=-0.1, tpp=0.05)
        with pytest.raises(LH.LindhardError) as ei:
            LH.Plan(precision=LH.LINDHARD_FP32C, **c)
        assert ei.value.status == LH.LINDHARD_EINVAL
    # a table of the wrong size is refused before the call
    with pytest.raises(ValueError):
        LH.Plan(precision=LH.LINDHARD_FP32C, **dict(cfg, n_bands=3))


# ---- band-pair maps |M^{nu,mu}(Q)|^2 (Eqs. (2), (3)) ---------------------
def pair_maps(nb, nky, nkx, zx, zy, seed, zero=()):
    """Smooth positive maps over the extended grid, one per pair (distinct, not
    symmetric in X and Y), with the pairs in `zero` all zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Y, X = np.meshgrid(np.arange(zy * nky) / nky, np.arange(zx * nkx) / nkx, indexing="ij")
    m2 = np.empty((nb, nb, zy * nky, zx * nkx))
    for nu in range(nb):
        for mu in range(nb):
            a, b, c = rng.uniform(0.2, 1.5, 3)
            m2[nu, mu] = a * np.exp(-b * (X - 1.3) ** 2 - 0.5 * c * Y) * (1.0 + 0.5 * np.sin(3.0 * X + c * Y))
    for nu, mu in zero:
        m2[nu, mu] = 0.0
    return m2


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("symmetric", [True, False])
def test_pair_maps_against_oracle(prec, symmetric):
    """Three bands with a Q-dependent map per pair (one pair's map zero): the
    even path over 3 x 3 zones and the general path over 3 x 1 zones, against
    the oracle's per-pair sum."""
    cfg = cfg_of(symmetric, nb=3, pairs=False)
    cfg.pop("ff_kind", None)
    cfg.pop("ff_width", None)
    zx, zy = (3, 3) if symmetric else (3, 1)
    cfg["zones"] = (zx, zy)
    cfg["pair_m2"] = pair_maps(3, 32, 32, zx, zy, seed=5 + symmetric, zero=[(0, 2)])
    eps = np.asarray(cfg["eps_table"])
    mu = oracle.mu_solve_bands(eps, cfg["gamma"], cfg["filling"])
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    lags = np.rint(np.asarray(cfg["omega"]) / d).astype(np.int64)
    ref = oracle.chi_pair_maps(eps - mu, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags,
                               cfg["pair_m2"], zx, zy)
    plan = LH.Plan(precision=prec, **cfg)
    sched = plan.info.schedule.decode()
    assert (" even " in sched) == symmetric
    got = plan.exec()
    torch.cuda.synchronize()
    err = normwise(got.double().cpu().numpy(), ref)
    print("pair maps prec=%d sym=%d err=%.3e %s" % (prec, symmetric, err, sched))
    assert err <= TOL[prec]
    again = plan.exec()
    torch.cuda.synchronize()
    assert torch.equal(got, again)
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_pair_map_of_one_band_equals_the_orbital_form_factor(prec):
    """One band with the d-wave orbital's |M(Q)|^2 tabulated equals the
    analytic form-factor path, and both equal the oracle."""
    base = dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.1, nkx=64, nky=64, neps=64, emin=-1.5, emax=1.5, gamma=0.06,
                omega=np.arange(1, 30, 3) * (3.0 / 64), zones=(3, 5))
    a = LH.Plan(precision=prec, ff_kind=1, ff_width=0.6, **base)
    b = LH.Plan(precision=prec, pair_m2=oracle.m2_extended(64, 64, 3, 5, 1, 0.6), **base)
    x, y = a.exec(), b.exec()
    torch.cuda.synchronize()
    assert normwise(y.double().cpu().numpy(), x.double().cpu().numpy()) <= TOL[prec]
    a.close()
    b.close()


def test_pair_map_argument_errors():
    cfg = cfg_of(True, nb=2, pairs=False)
    cfg.pop("ff_kind")
    cfg.pop("ff_width")
    m2 = pair_maps(2, 32, 32, 3, 3, seed=1)
    for bad in (dict(pair_weight=np.ones((2, 2))), dict(ff_kind=1, ff_width=0.6), dict(want_rpa=True),
                dict(pair_m2=-m2), dict(pair_m2=np.where(m2 > 1.0, np.nan, m2))):
        c = dict(cfg, pair_m2=m2)
        c.update(bad)
        with pytest.raises(LH.LindhardError) as ei:
            LH.Plan(precision=LH.LINDHARD_FP32C, **c)
        assert ei.value.status == LH.LINDHARD_EINVAL
