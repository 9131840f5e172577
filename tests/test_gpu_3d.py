"""Three-dimensional k-grids through the C ABI against the FP64 oracle: the
general path with a third, kz, transform pass; several shapes (flat and
cubic-ish, two kz planes), an omega between lag-grid points, two summed bands,
the output layout [omega][Z][Y][X], and the argument errors.  Normwise
tolerances as for the hot path."""
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


def test_3d_argument_errors():
    base = cfg3(8, 8, 4)
    for bad in (dict(nkz=3, eps_table=np.zeros((3, 8, 8))), dict(zones=(3, 1)), dict(ff_kind=1, ff_width=0.6),
                dict(want_rpa=True), dict(nkz=512, eps_table=np.zeros((512, 8, 8)))):
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
