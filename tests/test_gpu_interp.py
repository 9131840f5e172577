"""Omegas between lag-grid points (omega_interp) through the C ABI against the
FP64 oracle: the bare map on the even and the general path, Re chi and the
Coulomb RPA, and S(q, omega) with the Bose factor at the omega itself.
Normwise tolerances as for the hot path (FP64 <= 1e-11, FP32 <= 1e-5); on-grid
omegas must give the same bits with and without interpolation."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {LH.LINDHARD_FP64: 1e-11, LH.LINDHARD_FP32C: 1e-5}
PRECS = [LH.LINDHARD_FP64, LH.LINDHARD_FP32C]
V_COULOMB = 0.5


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def offgrid_omegas(neps, emin, emax):
    """Fractions 0 .. 0.9 at lags 0, 1, 5, 17, 30 and the last lag (whose upper
    neighbour lies beyond the grid), plus plain grid points."""
    d = (emax - emin) / neps
    ms = [0, 1, 5, 17, 30, neps - 1]
    fs = [0.0, 0.25, 0.5, 0.9]
    return np.array([(m + f) * d for m in ms for f in fs if m + f > 0] + [3 * d, 12 * d])


def small_cfg():
    """The extended-zone RPA workload (5x5 zones, orbital form factor) shrunk
    to 32x32 k and 64 energies on [-2, 2] eV, at off-grid omegas."""
    cfg = W.config2()
    cfg.update(nkx=32, nky=32, neps=64, gamma=0.08, want_rpa=False, omega_interp=True)
    cfg["omega"] = offgrid_omegas(64, cfg["emin"], cfg["emax"])
    return cfg


def oracle_maps(cfg, eps):
    """(Re chi_ext, Im chi_ext) at the cfg omegas, interpolated between lags."""
    mu = cfg.get("mu", float("nan"))
    if not np.isfinite(mu):
        mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    neps = cfg["neps"]
    full = oracle.chi_full(eps - mu, neps, cfg["emin"], cfg["emax"], cfg["gamma"], np.arange(neps))
    im_all = np.moveaxis(full, 0, -1)  # [qy][qx][lag]
    m, f = oracle.omega_lags(cfg["omega"], neps, cfg["emin"], cfg["emax"], interp=True)
    assert np.any(f > 0) and np.any(f == 0)
    im1 = np.moveaxis(oracle.lag_interp(im_all, m, f), -1, 0)
    re1 = np.moveaxis(oracle.kk_real_interp(im_all, m, f), -1, 0)
    zx, zy = cfg.get("zones", (1, 1))
    ffk, w = cfg.get("ff_kind", 0), cfg.get("ff_width", 0.0)
    return oracle.extend(re1, zx, zy, ffk, w), oracle.extend(im1, zx, zy, ffk, w)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("want_rpa", [False, True])
def test_offgrid_bare_map_even_path(prec, want_rpa):
    cfg = small_cfg()
    cfg["want_rpa"] = want_rpa
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"])
    _, ref = oracle_maps(cfg, eps)
    plan = LH.Plan(precision=prec, **cfg)
    assert " even " in plan.info.schedule.decode()
    got = plan.exec()
    torch.cuda.synchronize()
    err = normwise(got.double().cpu().numpy(), ref)
    print("offgrid even prec=%d rpa=%d err=%.3e" % (prec, want_rpa, err))
    assert err <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_offgrid_bare_map_general_path(prec):
    """A table without inversion symmetry runs the complex path (its own
    row-transform epilogue blends the two lags)."""
    rng = np.random.Generator(np.random.PCG64(31))
    tab = rng.uniform(-1.2, 1.5, size=(16, 32))
    cfg = dict(eps_table=tab, mu=0.1, nkx=32, nky=16, neps=64, emin=-1.5, emax=1.5, gamma=0.07,
               omega=offgrid_omegas(64, -1.5, 1.5), omega_interp=True)
    _, ref = oracle_maps(cfg, tab)
    plan = LH.Plan(precision=prec, **cfg)
    assert " even " not in plan.info.schedule.decode()
    got = plan.exec()
    torch.cuda.synchronize()
    err = normwise(got.double().cpu().numpy(), ref)
    print("offgrid general prec=%d err=%.3e" % (prec, err))
    assert err <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_offgrid_rpa_and_structure_factor(prec):
    cfg = small_cfg()
    cfg["want_rpa"] = True
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"])
    re_ext, im_ext = oracle_maps(cfg, eps)
    zx, zy = cfg["zones"]
    hx, _ = oracle.zone_axis(cfg["nkx"], zx)
    hy, _ = oracle.zone_axis(cfg["nky"], zy)
    imr, rer = oracle.rpa_coulomb(re_ext, im_ext, hx, hy, V_COULOMB)
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    re, gimr, grer = plan.rpa_coulomb(V_COULOMB)
    kT = 0.025
    s = plan.structure_factor(im, kT)
    torch.cuda.synchronize()
    errs = [normwise(x.double().cpu().numpy(), r) for x, r in ((re, re_ext), (gimr, imr), (grer, rer))]
    e_s = normwise(s.double().cpu().numpy(), oracle.structure_factor(im_ext, cfg["omega"], kT))
    print("offgrid rpa prec=%d errs=%s S %.2e" % (prec, ["%.2e" % e for e in errs], e_s))
    assert max(errs) <= TOL[prec] and e_s <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_ongrid_omegas_unchanged_by_interp(prec):
    cfg = small_cfg()
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    cfg["omega"] = np.arange(1, 33) * d
    outs = []
    for interp in (False, True):
        plan = LH.Plan(precision=prec, **dict(cfg, omega_interp=interp))
        outs.append(plan.exec())
        torch.cuda.synchronize()
        plan.close()
    assert torch.equal(outs[0], outs[1])


def test_offgrid_rejected_without_interp():
    cfg = small_cfg()
    cfg["omega_interp"] = False
    with pytest.raises(LH.LindhardError) as ei:
        LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert ei.value.status == LH.LINDHARD_EOFFGRID
    cfg["omega_interp"] = True
    cfg["omega"] = [-0.01]
    with pytest.raises(LH.LindhardError) as ei:
        LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert ei.value.status == LH.LINDHARD_EOFFGRID
