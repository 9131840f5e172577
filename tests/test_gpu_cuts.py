"""Cuts through the extended maps through the C ABI: the high-symmetry path of
Fig. 2(a) (indices equal to the oracle's, values a bit-exact gather of the
map and within the hot-path tolerance of the oracle's map) and the zone
envelope with its Lorentzian fit of Fig. 5 (maxima decided in the map's
precision exactly as the oracle decides them on the same values; k0 equal to
the oracle's fit of the same points to 1e-9; against the oracle's own map,
each chosen point a segment maximum up to the tolerance and k0 equal to the
fit of the oracle's values there)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {LH.LINDHARD_FP64: 1e-11, LH.LINDHARD_FP32C: 1e-5}
PRECS = [LH.LINDHARD_FP64, LH.LINDHARD_FP32C]
Q_SCALE = 1.0 / 7.46  # 1/a for a = 3.95 A = 7.46 bohr: q in atomic units


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def small_cfg():
    """The extended-zone workload (5x5 zones, orbital form factor) at 32x32 k,
    64 energies on [-2, 2] eV, 32 omegas."""
    cfg = W.config2()
    cfg.update(nkx=32, nky=32, neps=64, gamma=0.08, want_rpa=False, omega=np.arange(1, 33) * (4.0 / 64))
    return cfg


def check_against_oracle_map(env, ref_plane, prec, **kw):
    """The oracle's map may break near-ties differently (its values differ by
    rounding): every chosen point must be a maximum of its segment in the
    oracle's map up to the tolerance, and k0 must match the fit of the
    oracle's values at the chosen points."""
    full = oracle.zone_envelope(ref_plane, **kw)
    scale = np.abs(ref_plane).max()
    vals = -ref_plane[env["Y"], env["X"]]
    assert np.all(vals >= full["y"] * full["c_max"] - TOL[prec] * scale)
    k0_ref = oracle.envelope_fit(env["q"], vals / vals.max())
    assert env["k0"] == pytest.approx(k0_ref, rel=1e-9 if prec == LH.LINDHARD_FP64 else 1e-4)
    return full


def oracle_map(cfg):
    kz = cfg.get("k_zones", 1)
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"], kz)
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    lags = np.rint(np.asarray(cfg["omega"]) / d).astype(np.int64)
    full = oracle.chi_full(eps - mu, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags,
                           rho=cfg.get("rho_table"))
    zx, zy = cfg["zones"]
    return oracle.extend(full, zx, zy, cfg["ff_kind"], cfg["ff_width"])


@pytest.mark.parametrize("prec", PRECS)
def test_high_symmetry_cut(prec):
    cfg = small_cfg()
    ref = oracle_map(cfg)
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    X, Y = plan.high_symmetry_path()
    oX, oY = oracle.high_symmetry_path(cfg["nkx"], *cfg["zones"])
    assert np.array_equal(X, oX) and np.array_equal(Y, oY)
    c = plan.cut(im, X, Y)
    torch.cuda.synchronize()
    got = c.cpu().numpy()
    assert got.shape == (len(cfg["omega"]), X.size)
    assert np.array_equal(got, im.cpu().numpy()[:, Y, X])
    err = normwise(got, ref[:, oY, oX])
    print("high-symmetry cut prec=%d err=%.2e" % (prec, err))
    assert err <= TOL[prec]
    # arbitrary points (corners, repeats), then points off the grid
    ny, nx = plan.shape[1:]
    Xa = np.array([0, nx - 1, 0, nx - 1, 7, 7], dtype=np.int32)
    Ya = np.array([0, 0, ny - 1, ny - 1, 3, 3], dtype=np.int32)
    ca = plan.cut(im, Xa, Ya)
    torch.cuda.synchronize()
    assert np.array_equal(ca.cpu().numpy(), im.cpu().numpy()[:, Ya, Xa])
    for bad in ((np.array([nx]), np.array([0])), (np.array([0]), np.array([-1]))):
        with pytest.raises(LH.LindhardError) as ei:
            plan.cut(im, *bad)
        assert ei.value.status == LH.LINDHARD_EINVAL
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("direction", [0, 1])
def test_zone_envelope(prec, direction):
    cfg = small_cfg()
    ref = oracle_map(cfg)
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    for w in (7, 25):
        env = plan.zone_envelope(im, w, direction, Q_SCALE)
        own = oracle.zone_envelope(im[w].cpu().numpy(), cfg["nkx"], *cfg["zones"], direction, Q_SCALE)
        assert env["X"].size == 3
        assert np.array_equal(env["X"], own["X"]) and np.array_equal(env["Y"], own["Y"])
        assert np.allclose(env["y"], own["y"], rtol=1e-15, atol=0)
        assert np.allclose(env["q"], own["q"], rtol=1e-15, atol=0)
        assert env["c_max"] == own["c_max"]
        assert env["k0"] == pytest.approx(own["k0"], rel=1e-9)
        full = check_against_oracle_map(env, ref[w], prec, nk=cfg["nkx"], zx=cfg["zones"][0], zy=cfg["zones"][1],
                                        direction=direction, q_scale=Q_SCALE)
        print("envelope prec=%d dir=%d w=%d k0 %.6f (oracle map %.6f) y=%s" % (prec, direction, w, env["k0"],
                                                                              full["k0"], np.round(env["y"], 4)))
        assert 0.0 < env["k0"] < 1e4
    with pytest.raises(LH.LindhardError):
        plan.zone_envelope(im, len(cfg["omega"]), direction, Q_SCALE)
    with pytest.raises(LH.LindhardError):
        plan.zone_envelope(im, 0, 2, Q_SCALE)
    with pytest.raises(LH.LindhardError):
        plan.zone_envelope(im, 0, direction, 0.0)
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_zone_envelope_extended_momentum(prec):
    """A momentum grid spanning 8 x 8 zones with the d(x2-y2) momentum density
    (the form of Fig. 5): zones 8 steps wide inside one grid."""
    cfg = small_cfg()
    nk, kz = 64, 8
    cfg.update(nkx=nk, nky=nk, zones=(1, 1), ff_kind=0, ff_width=0.0, k_zones=kz,
               rho_table=W.momentum_density_dx2y2(nk, nk, kz, 0.6), omega=np.arange(1, 17) * (4.0 / 64))
    ref = oracle_map(cfg)
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    X, Y = plan.high_symmetry_path()
    oX, oY = oracle.high_symmetry_path(nk, 1, 1, kz)
    assert np.array_equal(X, oX) and np.array_equal(Y, oY) and X.size == 3 * (nk // kz) // 2 + 1
    for direction in (0, 1):
        env = plan.zone_envelope(im, 10, direction, Q_SCALE)
        own = oracle.zone_envelope(im[10].cpu().numpy(), nk, 1, 1, direction, Q_SCALE, kzones=kz)
        assert env["X"].size == (kz + 1) // 2
        assert np.array_equal(env["X"], own["X"]) and np.array_equal(env["Y"], own["Y"])
        assert env["k0"] == pytest.approx(own["k0"], rel=1e-9)
        full = check_against_oracle_map(env, ref[10], prec, nk=nk, zx=1, zy=1, direction=direction, q_scale=Q_SCALE,
                                        kzones=kz)
        print("extended envelope prec=%d dir=%d k0 %.6f (oracle map %.6f)" % (prec, direction, env["k0"], full["k0"]))
    plan.close()
