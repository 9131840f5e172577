"""Three-dimensional k-grids through the C ABI against the FP64 oracle: the
general path with a third, kz, transform pass; several shapes (flat and
cubic-ish, two kz planes), an omega between lag-grid points, two summed bands,
in-plane extended zones with the form factor, Kramers-Kronig with the contact
and Coulomb RPA, the output layout [omega][Z][Y][X], and the argument errors.
Normwise tolerances as for the hot path."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {LH.LINDHARD_FP64: 1e-11, LH.LINDHARD_FP32C: 1e-5}
PRECS = [LH.LINDHARD_FP64, LH.LINDHARD_FP32C]


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def cfg3(nkx, nky, nkz, **kw):
    cfg = dict(eps_table=W.band3d_table(nkx, nky, nkz, seed=7, tz=0.15), nkz=nkz, filling=1.1, nkx=nkx, nky=nky,
               neps=64, emin=-1.5, emax=1.5, gamma=0.08, omega=np.arange(1, 40, 3) * (3.0 / 64))
    cfg.update(kw)
    return cfg


def oracle_3d(cfg):
    eps = np.asarray(cfg["eps_table"], dtype=np.float64)
    nb = cfg.get("n_bands", 1)
    eps4 = eps.reshape(nb, cfg["nkz"], cfg["nky"], cfg["nkx"])
    mu = oracle.mu_solve(eps4.reshape(-1), cfg["gamma"], cfg["filling"] / nb)
    m, f = oracle.omega_lags(cfg["omega"], cfg["neps"], cfg["emin"], cfg["emax"], interp=cfg.get("omega_interp", False))
    full = oracle.chi_full_3d(eps4 - mu, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], np.arange(cfg["neps"]))
    vals = np.moveaxis(oracle.lag_interp(np.moveaxis(full, 0, -1), m, f), -1, 0)
    return mu, oracle.centre_3d(vals)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(16, 8, 4), (8, 8, 8), (32, 16, 2)])
def test_3d_against_oracle(prec, shape):
    nkx, nky, nkz = shape
    cfg = cfg3(nkx, nky, nkz)
    mu, ref = oracle_3d(cfg)
    plan = LH.Plan(precision=prec, **cfg)
    assert plan.shape == (len(cfg["omega"]), nkz * nky, nkx)
    assert " even " not in plan.info.schedule.decode()
    assert plan.info.mu == pytest.approx(mu, abs=1e-11)
    got = plan.exec()
    torch.cuda.synchronize()
    g = got.double().cpu().numpy().reshape(len(cfg["omega"]), nkz, nky, nkx)
    err = normwise(g, ref)
    print("3d prec=%d shape=%s err=%.3e %s" % (prec, shape, err, plan.info.schedule.decode()))
    assert err <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_3d_offgrid_omega_and_two_bands(prec):
    nkx, nky, nkz = 16, 8, 4
    t1 = W.band3d_table(nkx, nky, nkz, seed=7, tz=0.15)
    t2 = W.band3d_table(nkx, nky, nkz, seed=8, tz=0.05) + 0.4
    d = 3.0 / 64
    cfg = cfg3(nkx, nky, nkz, eps_table=np.stack([t1, t2]), n_bands=2, omega_interp=True,
               omega=np.array([2.5, 7.0, 11.25, 30.9]) * d)
    mu, ref = oracle_3d(cfg)
    plan = LH.Plan(precision=prec, **cfg)
    got = plan.exec()
    torch.cuda.synchronize()
    err = normwise(got.double().cpu().numpy().reshape(ref.shape), ref)
    print("3d interp two bands prec=%d err=%.3e" % (prec, err))
    assert err <= TOL[prec]
    # the plane epilogues work on the flattened 3D planes
    qa = plan.q_average(got)
    torch.cuda.synchronize()
    assert np.allclose(qa.cpu().numpy(), ref.reshape(ref.shape[0], -1).mean(axis=1), rtol=0,
                       atol=TOL[prec] * np.abs(ref).max())
    plan.close()


def _oracle_full_3d(cfg):
    eps = np.asarray(cfg["eps_table"], dtype=np.float64).reshape(cfg["nkz"], cfg["nky"], cfg["nkx"])
    mu = oracle.mu_solve(eps.reshape(-1), cfg["gamma"], cfg["filling"])
    full = oracle.chi_full_3d(eps - mu, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], np.arange(cfg["neps"]))
    return mu, full  # (neps, nkz, nky, nkx), natural q order


def _extend_3d(maps, cfg):
    """kz planes centred, every plane extended over the in-plane zones with
    the in-plane form factor: (n, nkz * zy * nky, zx * nkx)."""
    zx, zy = cfg["zones"]
    rolled = np.roll(maps, cfg["nkz"] // 2, axis=-3)
    ext = oracle.extend(rolled, zx, zy, cfg.get("ff_kind", 0), cfg.get("ff_width", 0.0))
    return ext.reshape(ext.shape[0], -1, ext.shape[-1])


@pytest.mark.parametrize("prec", PRECS)
def test_3d_extended_zones_and_form_factor(prec):
    """3D grid with 3 x 5 in-plane zones and the orbital form factor: every kz
    plane becomes a block of zones_y * nky rows (output [omega][Z][Y][X])."""
    cfg = cfg3(16, 8, 4, zones=(3, 5), ff_kind=1, ff_width=0.6)
    mu, full = _oracle_full_3d(cfg)
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    lags = np.rint(np.asarray(cfg["omega"]) / d).astype(int)
    ref = _extend_3d(full[lags], cfg)
    plan = LH.Plan(precision=prec, **cfg)
    assert plan.shape == (len(lags), 4 * 5 * 8, 3 * 16)
    got = plan.exec()
    torch.cuda.synchronize()
    err = normwise(got.double().cpu().numpy(), ref)
    print("3d zones+ff prec=%d err=%.3e" % (prec, err))
    assert err <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_3d_rpa_contact_and_coulomb(prec):
    """Kramers-Kronig and RPA on a 3D grid (3 x 1 zones, form factor): Re chi
    from every lag, the contact RPA, and the Coulomb RPA whose |Q|^2 includes
    the kz of each plane (lattice constant a along z)."""
    cfg = cfg3(8, 8, 4, zones=(3, 1), ff_kind=1, ff_width=0.6, want_rpa=True)
    mu, full = _oracle_full_3d(cfg)
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    lags = np.rint(np.asarray(cfg["omega"]) / d).astype(int)
    re1 = np.moveaxis(oracle.kk_real(np.moveaxis(full, 0, -1), lags), -1, 0)
    im_ext = _extend_3d(full[lags], cfg)
    re_ext = _extend_3d(re1, cfg)
    U, v = 1.1, 0.4
    imr_c, rer_c = oracle.rpa(re_ext, im_ext, U)
    nkz, nky, nkx = cfg["nkz"], cfg["nky"], cfg["nkx"]
    zx, zy = cfg["zones"]
    hx, _ = oracle.zone_axis(nkx, zx)
    hy, _ = oracle.zone_axis(nky, zy)
    imr_v, rer_v = np.empty_like(im_ext), np.empty_like(im_ext)
    for Z in range(nkz):
        rows = slice(Z * zy * nky, (Z + 1) * zy * nky)
        hz = (Z - nkz // 2) / nkz
        imr_v[:, rows], rer_v[:, rows] = oracle.rpa_coulomb(re_ext[:, rows], im_ext[:, rows], hx, hy, v, hz)
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    re, imr, rer = plan.rpa(U)
    torch.cuda.synchronize()
    errs = [normwise(x.double().cpu().numpy(), r) for x, r in ((im, im_ext), (re, re_ext), (imr, imr_c), (rer, rer_c))]
    re2, imr2, rer2 = plan.rpa_coulomb(v)
    torch.cuda.synchronize()
    errs += [normwise(x.double().cpu().numpy(), r) for x, r in ((re2, re_ext), (imr2, imr_v), (rer2, rer_v))]
    print("3d rpa prec=%d errs=%s" % (prec, ["%.2e" % e for e in errs]))
    assert max(errs) <= TOL[prec]
    plan.close()


def test_3d_argument_errors():
    base = cfg3(8, 8, 4)
    for bad in (dict(nkz=3, eps_table=np.zeros((3, 8, 8))), dict(k_zones=2),
                dict(pair_m2=np.ones((1, 1, 8, 8))), dict(nkz=512, eps_table=np.zeros((512, 8, 8)))):
        with pytest.raises(LH.LindhardError) as ei:
            LH.Plan(precision=LH.LINDHARD_FP32C, **dict(base, **bad))
        assert ei.value.status == LH.LINDHARD_EINVAL
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **base)
    im = plan.exec()
    with pytest.raises(LH.LindhardError):
        plan.high_symmetry_path()
    with pytest.raises(LH.LindhardError):
        plan.zone_envelope(im, 0)
    plan.close()
