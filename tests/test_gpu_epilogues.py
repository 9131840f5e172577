"""Parity of the widened epilogues (through the C ABI) with the FP64 oracle:
RPA with the Coulomb interaction V(Q) = v/|Q|^2, the dynamical structure
factor of Eq. (1) and the peak search over omega.  Same metric and
tolerances as the hot path (normwise; FP64 <= 1e-11, FP32 <= 1e-5); the
peak indices are integers decided in the kernel's precision, so the oracle
decides on the same values and must agree exactly."""
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
V_COULOMB = 0.5  # eV a^2: no pole of 1 - V chi on these grids


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def lags_of(cfg):
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    return np.rint(np.asarray(cfg["omega"]) / d).astype(np.int64)


def small_cfg():
    """The extended-zone RPA workload (5x5 zones, orbital form factor) shrunk
    to 32x32 k and 64 energies on [-2, 2] eV."""
    cfg = W.config2()
    cfg.update(nkx=32, nky=32, neps=64, gamma=0.08, omega=np.arange(1, 33) * (4.0 / 64))
    return cfg


def oracle_chi_ext(cfg):
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"])
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    neps = cfg["neps"]
    full = oracle.chi_full(eps - mu, neps, cfg["emin"], cfg["emax"], cfg["gamma"], np.arange(neps))
    lags = lags_of(cfg)
    im1 = full[lags]
    re1 = np.moveaxis(oracle.kk_real(np.moveaxis(full, 0, -1), lags), -1, 0)
    zx, zy = cfg["zones"]
    return (oracle.extend(re1, zx, zy, 1, cfg["ff_width"]), oracle.extend(im1, zx, zy, 1, cfg["ff_width"]))


@pytest.mark.parametrize("prec", PRECS)
def test_coulomb_rpa_full_grid(prec):
    cfg = small_cfg()
    re_ext, im_ext = oracle_chi_ext(cfg)
    zx, zy = cfg["zones"]
    hx, _ = oracle.zone_axis(cfg["nkx"], zx)
    hy, _ = oracle.zone_axis(cfg["nky"], zy)
    imr, rer = oracle.rpa_coulomb(re_ext, im_ext, hx, hy, V_COULOMB)
    plan = LH.Plan(precision=prec, **cfg)
    plan.exec()
    re, gimr, grer = plan.rpa_coulomb(V_COULOMB)
    torch.cuda.synchronize()
    errs = [normwise(x.double().cpu().numpy(), r) for x, r in ((re, re_ext), (gimr, imr), (grer, rer))]
    print("coulomb rpa prec=%d errs=%s" % (prec, ["%.2e" % e for e in errs]))
    assert max(errs) <= TOL[prec]
    # Q = 0 (the centre of the extended grid) takes the limit 0 exactly
    Y0, X0 = zy * cfg["nky"] // 2, zx * cfg["nkx"] // 2
    assert hx[X0] == 0.0 and hy[Y0] == 0.0
    assert torch.all(gimr[:, Y0, X0] == 0) and torch.all(grer[:, Y0, X0] == 0)
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kT", [0.0, 0.025, 1.0])
def test_structure_factor_and_peaks(prec, kT):
    cfg = small_cfg()
    re_ext, im_ext = oracle_chi_ext(cfg)
    zx, zy = cfg["zones"]
    hx, _ = oracle.zone_axis(cfg["nkx"], zx)
    hy, _ = oracle.zone_axis(cfg["nky"], zy)
    imr, _ = oracle.rpa_coulomb(re_ext, im_ext, hx, hy, V_COULOMB)
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    omega = lags_of(cfg) * d
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    _, gimr, _ = plan.rpa_coulomb(V_COULOMB)
    s_bare = plan.structure_factor(im, kT)
    s_rpa = plan.structure_factor(gimr, kT)
    torch.cuda.synchronize()
    # end to end against the oracle's own chain
    e_bare = normwise(s_bare.double().cpu().numpy(), oracle.structure_factor(im_ext, omega, kT))
    e_rpa = normwise(s_rpa.double().cpu().numpy(), oracle.structure_factor(imr, omega, kT))
    # the epilogue alone, on the kernel's own input values
    e_own = normwise(s_rpa.double().cpu().numpy(), oracle.structure_factor(gimr.double().cpu().numpy(), omega, kT))
    print("S(q,w) prec=%d kT=%g errs %.2e %.2e %.2e" % (prec, kT, e_bare, e_rpa, e_own))
    assert max(e_bare, e_rpa) <= TOL[prec]
    assert e_own <= (1e-15 if prec == LH.LINDHARD_FP64 else 3e-7)
    assert torch.all(s_bare >= 0)
    # in place
    inplace = gimr.clone()
    plan.structure_factor(inplace, kT, out=inplace)
    torch.cuda.synchronize()
    assert torch.equal(inplace, s_rpa)
    # peaks of -Im chi_RPA (plasmon search) and of -Im chi: exact on the same values
    for arr in (gimr, im):
        pk = plan.peak_index(arr)
        torch.cuda.synchronize()
        ref = oracle.peak_index(arr.cpu().numpy())
        assert np.array_equal(pk.cpu().numpy(), ref)
    plan.close()


def test_epilogue_argument_errors():
    cfg = small_cfg()
    plan = LH.Plan(precision=LH.LINDHARD_FP64, **cfg)
    im = plan.exec()
    torch.cuda.synchronize()
    with pytest.raises(LH.LindhardError) as ei:
        plan.structure_factor(im, -0.01)
    assert ei.value.status == LH.LINDHARD_EINVAL
    with pytest.raises(LH.LindhardError) as ei:
        plan.structure_factor(im, float("nan"))
    assert ei.value.status == LH.LINDHARD_EINVAL
    with pytest.raises(LH.LindhardError) as ei:
        plan.rpa_coulomb(float("inf"))
    assert ei.value.status == LH.LINDHARD_EINVAL
    plan.close()
    # Coulomb RPA needs a plan built for the RPA epilogue
    base = W.config1()
    p2 = LH.Plan(precision=LH.LINDHARD_FP64, **base)
    p2.exec()
    torch.cuda.synchronize()
    with pytest.raises(LH.LindhardError) as ei:
        p2.rpa_coulomb(1.0)
    assert ei.value.status == LH.LINDHARD_ESTATE
    p2.close()


@pytest.mark.parametrize("prec", [LH.LINDHARD_FP32C])
def test_config2_coulomb_sampled(prec):
    """512^2 k, 256 energies, 5x5 zones: Coulomb RPA and S(q, omega) at
    sampled q (all zones), oracle over all 255 lags there."""
    cfg = W.config2()
    n, neps = cfg["nkx"], cfg["neps"]
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], n, n)
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    qs = [(0, 0), (1, 0), (n // 2, 0), (37, 5), (200, 311)]
    qx = np.array([q[0] for q in qs])
    qy = np.array([q[1] for q in qs])
    im_all = oracle.chi_grid(eps - mu, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, np.arange(neps))
    lags = lags_of(cfg)
    re_w = oracle.kk_real(im_all, lags)
    im_w = im_all[:, lags]
    d = (cfg["emax"] - cfg["emin"]) / neps
    plan = LH.Plan(precision=prec, **cfg)
    plan.exec()
    _, gimr, grer = plan.rpa_coulomb(V_COULOMB)
    s = plan.structure_factor(gimr, 0.025)
    torch.cuda.synchronize()
    zx, zy = cfg["zones"]
    hx, ux = oracle.zone_axis(n, zx)
    hy, uy = oracle.zone_axis(n, zy)
    gi, gr, gs, ri, rr, rs = ([] for _ in range(6))
    for iq, (a, b) in enumerate(qs):
        for Y in np.nonzero(uy == b)[0]:
            for X in np.nonzero(ux == a)[0]:
                m2 = oracle.form_factor(2 * np.pi * hx[X], 2 * np.pi * hy[Y], cfg["ff_width"]) ** 2
                e_im = (m2 * im_w[iq])[:, None, None]
                e_re = (m2 * re_w[iq])[:, None, None]
                o_im, o_re = oracle.rpa_coulomb(e_re, e_im, hx[X:X + 1], hy[Y:Y + 1], V_COULOMB)
                ri.append(o_im[:, 0, 0])
                rr.append(o_re[:, 0, 0])
                rs.append(oracle.structure_factor(o_im, lags * d, 0.025)[:, 0, 0])
                gi.append(gimr[:, Y, X].double().cpu().numpy())
                gr.append(grer[:, Y, X].double().cpu().numpy())
                gs.append(s[:, Y, X].double().cpu().numpy())
    errs = [normwise(np.array(g), np.array(r)) for g, r in ((gi, ri), (gr, rr), (gs, rs))]
    print("config2 coulomb errs=%s" % ["%.2e" % e for e in errs])
    assert max(errs) <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_q_average_is_the_q_integrated_jdos(prec):
    """The 32x32 workload: the q-average of every omega plane against the
    oracle's q-integrated joint density of states (no q-sum there), a plain
    mean of the same array, and bitwise repeatability."""
    cfg = W.config1()
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"])
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    ref = oracle.chi_qmean(eps - mu, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags_of(cfg))
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    a = plan.q_average(im)
    b = plan.q_average(im)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    err = normwise(a.cpu().numpy(), ref)
    own = normwise(a.cpu().numpy(), im.double().mean(dim=(1, 2)).cpu().numpy())
    print("q-average prec=%d err %.2e (own mean %.2e)" % (prec, err, own))
    assert err <= TOL[prec] and own <= 1e-13
    plan.close()


def test_q_average_extended_zones_and_full_size():
    # extended zones with the form factor: the mean of the array itself
    cfg = small_cfg()
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    im = plan.exec()
    qa = plan.q_average(im)
    torch.cuda.synchronize()
    assert normwise(qa.cpu().numpy(), im.double().mean(dim=(1, 2)).cpu().numpy()) <= 1e-13
    plan.close()
    # the 2048^2 x 512 instance: every lag against the oracle's JDOS
    cfg = W.config3()
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"])
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    ref = oracle.chi_qmean(eps - mu, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags_of(cfg))
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    im = plan.exec()
    qa = plan.q_average(im)
    torch.cuda.synchronize()
    err = normwise(qa.cpu().numpy(), ref)
    print("q-average 2048^2 err %.2e" % err)
    assert err <= 1e-5
    plan.close()
