"""Parity of the extended-momentum form (momentum-density weights on the
spectral function, momentum grids spanning several zones; Eqs. (4), (9))
with the FP64 oracle, through the C ABI.  Normwise; FP64 <= 1e-11, FP32
<= 1e-5."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {LH.LINDHARD_FP64: 1e-11, LH.LINDHARD_FP32C: 1e-5}
PRECS = [LH.LINDHARD_FP64, LH.LINDHARD_FP32C]


@pytest.fixture
def window(request, monkeypatch):
    for v in ("LINDHARD_WINDOW", "LINDHARD_SYMMETRY", "LINDHARD_EVEN_WINDOW"):
        monkeypatch.delenv(v, raising=False)
    if request.param in ("direct", "fft"):
        monkeypatch.setenv("LINDHARD_SYMMETRY", "off")
        monkeypatch.setenv("LINDHARD_WINDOW", request.param)
    elif request.param.startswith("even-"):
        monkeypatch.setenv("LINDHARD_EVEN_WINDOW", request.param[5:])
    return request.param


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def lags_of(cfg):
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    return np.rint(np.asarray(cfg["omega"]) / d).astype(np.int64)


def small_cfg(kz=4, nk=32, neps=32):
    cfg = W.config_extended(nk=nk, k_zones=kz, neps=neps)
    cfg.update(gamma=0.08)
    return cfg


def oracle_xi(cfg):
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"], kzones=cfg["k_zones"])
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    return eps - mu, mu


@pytest.mark.parametrize("window", ["auto", "even-mfma", "even-mfma4", "even-direct", "direct", "fft"], indirect=True)
@pytest.mark.parametrize("prec", PRECS)
def test_extended_full_grid(prec, window):
    cfg = small_cfg()
    xi, mu = oracle_xi(cfg)
    full = oracle.chi_full(xi, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags_of(cfg),
                           rho=cfg["rho_table"])
    ref = oracle.extend(full, 1, 1, 0, 0.0)
    plan = LH.Plan(precision=prec, **cfg)
    assert abs(plan.info.mu - mu) < 1e-12
    got = plan.exec()
    qa = plan.q_average(got)
    torch.cuda.synchronize()
    sched = plan.info.schedule.decode()
    err = normwise(got.double().cpu().numpy(), ref)
    qref = oracle.chi_qmean(xi, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags_of(cfg),
                            rho=cfg["rho_table"])
    qerr = normwise(qa.cpu().numpy(), qref)
    print("extended prec=%d window=%s err=%.2e qavg %.2e schedule=%s" % (prec, window, err, qerr, sched))
    assert (" even " in sched) == (window not in ("direct", "fft"))
    assert err <= TOL[prec] and qerr <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_asymmetric_density_table_takes_the_general_path(prec):
    cfg = small_cfg(kz=2, nk=16, neps=16)
    rng = np.random.Generator(np.random.PCG64(31))
    cfg["rho_table"] = rng.uniform(0.0, 1.0, size=(16, 16))
    xi, _ = oracle_xi(cfg)
    full = oracle.chi_full(xi, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags_of(cfg),
                           rho=cfg["rho_table"])
    plan = LH.Plan(precision=prec, **cfg)
    got = plan.exec()
    torch.cuda.synchronize()
    assert " even " not in plan.info.schedule.decode()
    err = normwise(got.double().cpu().numpy(), oracle.extend(full, 1, 1, 0, 0.0))
    print("asymmetric rho prec=%d err=%.2e" % (prec, err))
    assert err <= TOL[prec]
    plan.close()


def test_extended_full_size_sampled():
    """2048^2 momentum grid over 16 x 16 zones with the d_{x2-y2} momentum
    density, FP32: sampled (q, m) and the q-average at every lag."""
    cfg = W.config_extended()
    n, neps = cfg["nkx"], cfg["neps"]
    xi, mu = oracle_xi(cfg)
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert abs(plan.info.mu - mu) < 1e-10
    out = plan.exec()
    qa = plan.q_average(out)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(35))
    samples = [(0, 0, 1), (128, 0, 100), (64, 64, 256), (5, 900, 40)]
    for _ in range(8):
        samples.append((int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(1, 257))))
    qx = np.array([s[0] for s in samples])
    qy = np.array([s[1] for s in samples])
    ms = np.array([s[2] for s in samples])
    ref = oracle.chi_pairs(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, ms, rho=cfg["rho_table"])
    got = np.array([out[m - 1, (b + n // 2) % n, (a + n // 2) % n].item() for a, b, m in samples])
    scale = out.abs().max().item()
    err = np.abs(got - ref).max() / scale
    qref = oracle.chi_qmean(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], lags_of(cfg), rho=cfg["rho_table"])
    qerr = normwise(qa.cpu().numpy(), qref)
    print("extended 2048^2 sampled err %.2e, q-average err %.2e, schedule %s" % (err, qerr,
                                                                           plan.info.schedule.decode()))
    assert err <= 1e-5 and qerr <= 1e-5
    plan.close()


@pytest.mark.parametrize("window", ["auto", "direct"], indirect=True)
@pytest.mark.parametrize("prec", PRECS)
def test_extended_grid_with_zones_form_factor_and_rpa(prec, window):
    """A momentum grid spanning two zones, repeated over 3 x 3 output zones,
    with the orbital form factor (Eq. (3)) and both RPA forms: |M(Q)|^2 and
    V(Q) are taken at Q = 2 pi k_zones (X - Zx nkx/2)/nkx, the momentum the
    grid point stands for."""
    kz = 2
    cfg = small_cfg(kz=kz, nk=16, neps=32)
    cfg.update(zones=(3, 3), ff_kind=1, ff_width=0.6, want_rpa=True)
    xi, mu = oracle_xi(cfg)
    neps = cfg["neps"]
    full = oracle.chi_full(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], np.arange(neps), rho=cfg["rho_table"])
    lags = lags_of(cfg)
    im1 = full[lags]
    re1 = np.moveaxis(oracle.kk_real(np.moveaxis(full, 0, -1), lags), -1, 0)
    im_ext = oracle.extend(im1, 3, 3, 1, 0.6, kzones=kz)
    re_ext = oracle.extend(re1, 3, 3, 1, 0.6, kzones=kz)
    U, v = 1.1, 0.8
    imr_u, rer_u = oracle.rpa(re_ext, im_ext, U)
    hx, _ = oracle.zone_axis(cfg["nkx"], 3, kz)
    hy, _ = oracle.zone_axis(cfg["nky"], 3, kz)
    imr_c, rer_c = oracle.rpa_coulomb(re_ext, im_ext, hx, hy, v)
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    re, gimr_u, grer_u = plan.rpa(U)
    got_u = [x.double().cpu().numpy() for x in (im, re, gimr_u, grer_u)]
    _, gimr_c, grer_c = plan.rpa_coulomb(v)
    torch.cuda.synchronize()
    errs = [normwise(g, r) for g, r in zip(got_u, (im_ext, re_ext, imr_u, rer_u))]
    errs += [normwise(gimr_c.double().cpu().numpy(), imr_c), normwise(grer_c.double().cpu().numpy(), rer_c)]
    print("k_zones=2 zones 3x3 ff+rpa prec=%d window=%s errs=%s" % (prec, window, ["%.2e" % e for e in errs]))
    assert max(errs) <= TOL[prec]
    plan.close()
