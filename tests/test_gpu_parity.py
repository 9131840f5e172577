"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Error metric: normwise, max|gpu - oracle| / max|oracle| over each compared
array; FP64 path <= 1e-11, FP32 path (compensated energy window) <= 1e-5.
Small cases compare every output element; full-size cases compare outputs
sampled one by one with the oracle and properties that hold at any size.
"""
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
WINDOWS = ["auto", "direct", "fft", "even-direct", "even-mfma", "even-mfma4"]
EVEN_WINDOWS = ("auto", "even-direct", "even-mfma", "even-mfma4")


@pytest.fixture
def window(request, monkeypatch):
    """Pipeline chosen at plan time.  auto: the plan's own choice (the real
    even path for mirror-symmetric bands, window form timed); direct / fft:
    the general complex path with the direct or the energy-FFT window;
    even-direct / even-mfma / even-mfma4: the even path with the vector-ALU
    window, the Toeplitz-blocked matrix-core window or the rank-1 matrix-core
    window (FP32; each where its LDS tiles fit, else the vector form)."""
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


def oracle_xi(cfg):
    if cfg.get("eps_table") is not None:
        eps = np.asarray(cfg["eps_table"], dtype=np.float64)
    else:
        eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"])
    mu = cfg["mu"] if not math.isnan(cfg.get("mu", math.nan)) else oracle.mu_solve(eps, cfg["gamma"],
                                                                                     cfg["filling"])
    return eps - mu, mu


def oracle_extended(cfg):
    xi, mu = oracle_xi(cfg)
    full = oracle.chi_full(xi, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags_of(cfg))
    zx, zy = cfg.get("zones", (1, 1))
    return oracle.extend(full, zx, zy, cfg.get("ff_kind", 0), cfg.get("ff_width", 0.0)), mu


def run_gpu(cfg, prec):
    plan = LH.Plan(precision=prec, **cfg)
    out = plan.exec()
    torch.cuda.synchronize()
    return plan, out.double().cpu().numpy()


@pytest.mark.parametrize("window", WINDOWS, indirect=True)
@pytest.mark.parametrize("prec", PRECS)
def test_config1_full_grid(prec, window):
    cfg = W.config1()
    ref, mu = oracle_extended(cfg)
    plan, got = run_gpu(cfg, prec)
    assert abs(plan.info.mu - mu) < 1e-12
    err = normwise(got, ref)
    print("config1 prec=%d window=%s err=%.3e schedule=%s" % (prec, window, err, plan.info.schedule.decode()))
    sched = plan.info.schedule.decode()
    assert (" even " in sched) == (window in EVEN_WINDOWS)
    if window == "even-mfma":
        assert " P3 mfma " in sched
    if window == "even-mfma4":
        assert (" P3 mfma4 " in sched) == (prec == LH.LINDHARD_FP32C)
    if window == "even-direct":
        assert " P3 direct " in sched
    assert err <= TOL[prec]
    plan.close()


EDGE = [
    # tiny grid, lags 0 / >= neps / beyond
    dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.15, nkx=4, nky=4, neps=4, emin=-1.0, emax=1.0, gamma=0.2,
         omega=np.array([0, 1, 2, 3, 4, 7]) * 0.5),
    # non-square, asymmetric window, unsorted lags with duplicates and empties
    dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.05, nkx=64, nky=16, neps=32, emin=-0.7, emax=0.9, gamma=0.08,
         omega=np.array([3, 1, 1, 0, 17, 40, 31]) * (1.6 / 32)),
    # tall grid, strided lag list
    dict(t=0.40, tp=-0.12, tpp=0.03, filling=0.9, nkx=16, nky=128, neps=128, emin=-2.0, emax=1.0, gamma=0.05,
         omega=np.arange(1, 100, 7) * (3.0 / 128)),
    # wide grid with few energies
    dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.15, nkx=256, nky=8, neps=16, emin=-1.0, emax=1.0, gamma=0.1,
         omega=np.arange(1, 16) * (2.0 / 16)),
    # extended zones with the orbital form factor
    dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.15, nkx=32, nky=16, neps=32, emin=-2.0, emax=2.0, gamma=0.1,
         omega=np.arange(1, 17) * (4.0 / 32), zones=(3, 5), ff_kind=1, ff_width=0.6),
    # zone replication without a form factor
    dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.15, nkx=16, nky=32, neps=64, emin=-1.0, emax=1.0, gamma=0.05,
         omega=np.arange(1, 33) / 32.0, zones=(5, 3)),
    # the largest row length and energy count handled in one launch shape
    dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.15, nkx=2048, nky=4, neps=8, emin=-1.0, emax=1.0, gamma=0.2,
         omega=np.arange(1, 8) * 0.25),
    dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.15, nkx=8, nky=8, neps=2048, emin=-2.0, emax=2.0, gamma=0.05,
         omega=np.array([1, 2, 100, 1023, 1024, 1500, 2047]) * (4.0 / 2048)),
]


@pytest.mark.parametrize("window", WINDOWS, indirect=True)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", range(len(EDGE)))
def test_edge_cases_full_grid(case, prec, window):
    cfg = dict(EDGE[case])
    ref, mu = oracle_extended(cfg)
    plan, got = run_gpu(cfg, prec)
    assert got.shape == ref.shape
    err = normwise(got, ref)
    print("edge %d prec=%d window=%s err=%.3e schedule=%s" % (case, prec, window, err, plan.info.schedule.decode()))
    assert err <= TOL[prec]
    # empty windows are exact zeros
    lags = lags_of(cfg)
    for w, m in enumerate(lags):
        if m == 0 or m >= cfg["neps"]:
            assert np.all(got[w] == 0.0)
    plan.close()


@pytest.mark.parametrize("window", WINDOWS, indirect=True)
@pytest.mark.parametrize("prec", PRECS)
def test_caller_table_without_inversion_symmetry(prec, window):
    """A random eps table (no symmetry): complex real-space functions."""
    rng = np.random.Generator(np.random.PCG64(11))
    tab = rng.uniform(-1.2, 1.5, size=(16, 32))
    cfg = dict(eps_table=tab, mu=0.1, nkx=32, nky=16, neps=64, emin=-1.5, emax=1.5, gamma=0.07,
               omega=np.arange(1, 40, 3) * (3.0 / 64))
    ref, _ = oracle_extended(cfg)
    plan, got = run_gpu(cfg, prec)
    err = normwise(got, ref)
    print("table prec=%d window=%s err=%.3e schedule=%s" % (prec, window, err, plan.info.schedule.decode()))
    assert err <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("window", EVEN_WINDOWS, indirect=True)
@pytest.mark.parametrize("prec", PRECS)
def test_caller_table_with_mirror_symmetry_takes_even_path(prec, window):
    """A random table made mirror symmetric in both axes is detected bit for
    bit and runs on the real even path; it must still match the oracle."""
    rng = np.random.Generator(np.random.PCG64(12))
    nky, nkx = 32, 64
    base = rng.uniform(-1.2, 1.5, size=(nky, nkx))
    iy = np.minimum(np.arange(nky), (nky - np.arange(nky)) % nky)
    ix = np.minimum(np.arange(nkx), (nkx - np.arange(nkx)) % nkx)
    tab = base[iy[:, None], ix[None, :]]
    cfg = dict(eps_table=tab, mu=0.05, nkx=nkx, nky=nky, neps=64, emin=-1.5, emax=1.5, gamma=0.07,
               omega=np.arange(1, 40, 3) * (3.0 / 64), zones=(3, 1), ff_kind=1, ff_width=0.6)
    ref, _ = oracle_extended(cfg)
    plan, got = run_gpu(cfg, prec)
    assert " even " in plan.info.schedule.decode()
    err = normwise(got, ref)
    print("sym table prec=%d window=%s err=%.3e schedule=%s" % (prec, window, err, plan.info.schedule.decode()))
    assert err <= TOL[prec]
    plan.close()


def test_given_mu_and_repeatability():
    cfg = W.config1()
    cfg["mu"] = 0.0125
    ref, _ = oracle_extended(cfg)
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert plan.info.mu == 0.0125 and plan.info.mu_iterations == 0
    a = plan.exec()
    b = plan.exec()
    torch.cuda.synchronize()
    assert torch.equal(a, b), "runs must be bitwise identical"
    assert normwise(a.double().cpu().numpy(), ref) <= 1e-5
    plan.close()


def _config2_small():
    """The extended-zone + RPA workload shrunk to 32x32 k and 64 energies on
    [-2, 2] eV (full-grid comparison of the RPA path)."""
    cfg = W.config2()
    cfg.update(nkx=32, nky=32, neps=64, gamma=0.08, omega=np.arange(1, 33) * (4.0 / 64))
    return cfg


@pytest.mark.parametrize("window", WINDOWS, indirect=True)
@pytest.mark.parametrize("prec", PRECS)
def test_rpa_path_full_grid(prec, window):
    cfg = _config2_small()
    U = W.CONFIG2_U
    xi, mu = oracle_xi(cfg)
    neps = cfg["neps"]
    all_lags = np.arange(neps)
    full = oracle.chi_full(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], all_lags)  # (neps, ny, nx)
    lags = lags_of(cfg)
    im1 = full[lags]
    re1 = np.moveaxis(oracle.kk_real(np.moveaxis(full, 0, -1), lags), -1, 0)
    zx, zy = cfg["zones"]
    im_ext = oracle.extend(im1, zx, zy, 1, cfg["ff_width"])
    re_ext = oracle.extend(re1, zx, zy, 1, cfg["ff_width"])
    imr, rer = oracle.rpa(re_ext, im_ext, U)

    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    re, gimr, grer = plan.rpa(U)
    torch.cuda.synchronize()
    errs = [normwise(x.double().cpu().numpy(), r) for x, r in ((im, im_ext), (re, re_ext), (gimr, imr),
                                                               (grer, rer))]
    print("rpa prec=%d window=%s errs=%s" % (prec, window, ["%.2e" % e for e in errs]))
    assert max(errs) <= TOL[prec]
    plan.close()


def test_rpa_zero_U_is_identity_and_needs_want_rpa():
    cfg = _config2_small()
    plan = LH.Plan(precision=LH.LINDHARD_FP64, **cfg)
    im = plan.exec()
    re, imr, rer = plan.rpa(0.0)
    torch.cuda.synchronize()
    assert torch.equal(imr, im) and torch.equal(rer, re)
    plan.close()
    cfg["want_rpa"] = False
    plan = LH.Plan(precision=LH.LINDHARD_FP64, **cfg)
    plan.exec()
    with pytest.raises(LH.LindhardError) as ei:
        plan.rpa(1.0)
    assert ei.value.status == LH.LINDHARD_ESTATE
    torch.cuda.synchronize()
    plan.close()


@pytest.mark.parametrize("window", ["auto", "fft", "even-mfma", "even-mfma4"], indirect=True)
@pytest.mark.parametrize("prec", PRECS)
def test_config2_full_size_sampled(prec, window):
    """512^2 k, 256 energies, 5x5 zones, form factor, KK and RPA: every output
    component at sampled q (all zones), oracle over all 255 lags there."""
    cfg = W.config2()
    U = W.CONFIG2_U
    n, neps = cfg["nkx"], cfg["neps"]
    xi, mu = oracle_xi(cfg)
    rng = np.random.Generator(np.random.PCG64(22))
    qs = [(0, 0), (n // 2, 0), (n // 2, n // 2), (37, 5)] + [tuple(rng.integers(0, n, 2)) for _ in range(4)]
    qx = np.array([q[0] for q in qs])
    qy = np.array([q[1] for q in qs])
    allm = np.arange(neps)
    im_all = oracle.chi_grid(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, allm)  # (nq, neps)
    lags = lags_of(cfg)
    re_w = oracle.kk_real(im_all, lags)  # (nq, nw)
    im_w = im_all[:, lags]

    plan = LH.Plan(precision=prec, **cfg)
    assert abs(plan.info.mu - mu) < 1e-12
    im = plan.exec()
    re, imr, rer = plan.rpa(U)
    torch.cuda.synchronize()
    zx, zy = cfg["zones"]
    hx, ux = oracle.zone_axis(n, zx)
    hy, uy = oracle.zone_axis(n, zy)
    gi, gr, gir, grr, ri, rr, rir, rrr = ([] for _ in range(8))
    for iq, (a, b) in enumerate(qs):
        Xs = np.nonzero(ux == a)[0]
        Ys = np.nonzero(uy == b)[0]
        for Y in Ys:
            for X in Xs:
                m2 = oracle.form_factor(2 * np.pi * hx[X], 2 * np.pi * hy[Y], cfg["ff_width"]) ** 2
                e_im, e_re = m2 * im_w[iq], m2 * re_w[iq]
                e_imr, e_rer = oracle.rpa(e_re, e_im, U)
                ri.append(e_im)
                rr.append(e_re)
                rir.append(e_imr)
                rrr.append(e_rer)
                gi.append(im[:, Y, X].double().cpu().numpy())
                gr.append(re[:, Y, X].double().cpu().numpy())
                gir.append(imr[:, Y, X].double().cpu().numpy())
                grr.append(rer[:, Y, X].double().cpu().numpy())
    errs = [normwise(np.array(g), np.array(r)) for g, r in ((gi, ri), (gr, rr), (gir, rir), (grr, rrr))]
    print("config2 prec=%d window=%s errs=%s" % (prec, window, ["%.2e" % e for e in errs]))
    assert max(errs) <= TOL[prec]
    plan.close()


def q_sum_identity_rhs(xi, neps, emin, emax, gamma, lags):
    """-d sum_j D_P(j) D_H(j+m), D = k-average of the spectral weight."""
    d = (emax - emin) / neps
    e = emin + (np.arange(neps) + 0.5) * d
    D = np.zeros(neps)
    x = xi.ravel()
    for c in range(0, x.size, 1 << 16):
        xs = x[c:c + (1 << 16), None]
        D += ((gamma / np.pi) / ((e[None, :] - xs) ** 2 + gamma * gamma)).sum(axis=0)
    D /= x.size
    occ = e <= 0
    DP, DH = np.where(occ, D, 0.0), np.where(~occ, D, 0.0)
    out = []
    for m in lags:
        out.append(-d * sum(DP[j] * DH[j + m] for j in range(neps) if 0 <= j + m < neps) if m >= 1 else 0.0)
    return np.array(out)


@pytest.mark.parametrize("window", ["auto", "fft", "direct", "even-direct", "even-mfma", "even-mfma4"], indirect=True)
def test_config3_full_size_sampled_fp32_vs_oracle_and_fp64(window):
    """2048^2 k, 512 energies, 256 lags, G = 0.01 eV: FP32 (the benchmarked
    launch) against the oracle at sampled (q, m), the q-sum identity at every
    lag, C4v symmetry, and FP32 against the FP64 GPU path on the full grid."""
    cfg = W.config3()
    n, neps = cfg["nkx"], cfg["neps"]
    xi, mu = oracle_xi(cfg)
    lags = lags_of(cfg)
    plan32 = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert abs(plan32.info.mu - mu) < 1e-12
    print("config3 [%s] schedule %s" % (window, plan32.info.schedule.decode()))
    if window == "even-mfma":
        assert " P3 mfma " in plan32.info.schedule.decode()
    if window == "even-mfma4":
        assert " P3 mfma4 " in plan32.info.schedule.decode()
    out32 = plan32.exec()
    torch.cuda.synchronize()
    plan32.close()

    rng = np.random.Generator(np.random.PCG64(33))
    samples = [(0, 0, 1), (n // 2, 0, 128), (n // 2, n // 2, 256), (100, 7, 100), (0, n // 4, 200)]
    for _ in range(11):
        samples.append((int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(1, 257))))
    qx = np.array([s[0] for s in samples])
    qy = np.array([s[1] for s in samples])
    ms = np.array([s[2] for s in samples])
    ref = oracle.chi_pairs(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, ms)
    got = np.array([out32[m - 1, (b + n // 2) % n, (a + n // 2) % n].item() for a, b, m in samples])
    scale = out32.abs().max().item()
    err_s = np.abs(got - ref).max() / scale
    print("config3 [%s] sampled fp32 err (vs max|chi|) = %.3e" % (window, err_s))
    assert err_s <= 1e-5

    rhs = q_sum_identity_rhs(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], lags)
    lhs = out32.double().mean(dim=(1, 2)).cpu().numpy()
    err_q = normwise(lhs, rhs)
    print("config3 q-sum identity fp32 err = %.3e" % err_q)
    assert err_q <= 1e-5

    # C4v: transpose and mirror (exclude the first row / column of the centred map)
    core = out32[:, 1:, 1:]
    sym_t = (core - core.transpose(1, 2)).abs().max().item() / scale
    sym_m = (core - core.flip(2)).abs().max().item() / scale
    print("config3 symmetry %.2e %.2e" % (sym_t, sym_m))
    assert sym_t <= 1e-5 and sym_m <= 1e-5

    plan64 = LH.Plan(precision=LH.LINDHARD_FP64, **cfg)
    out64 = plan64.exec()
    torch.cuda.synchronize()
    plan64.close()
    got64 = np.array([out64[m - 1, (b + n // 2) % n, (a + n // 2) % n].item() for a, b, m in samples])
    err64 = np.abs(got64 - ref).max() / scale
    diff = (out32.double() - out64).abs().amax(dim=(1, 2))
    per_slice = (diff / out64.abs().amax(dim=(1, 2)).clamp_min(1e-300)).max().item()
    overall = diff.max().item() / out64.abs().max().item()
    print("config3 fp64 sampled err %.3e ; fp32 vs fp64 normwise %.3e (worst slice %.3e)"
          % (err64, overall, per_slice))
    assert err64 <= 1e-11
    assert overall <= 1e-5


def test_autotuner_times_once_per_shape_and_caches(tmp_path, monkeypatch):
    """The first plan of a shape times the window schedules; the next plan of
    the same shape reuses the decision (in process and through the cache file),
    and the tuned plan still matches the oracle."""
    monkeypatch.delenv("LINDHARD_WINDOW", raising=False)
    monkeypatch.delenv("LINDHARD_SYMMETRY", raising=False)
    monkeypatch.delenv("LINDHARD_AUTOTUNE", raising=False)
    monkeypatch.setenv("LINDHARD_TUNE_CACHE", str(tmp_path / "tune.txt"))
    cfg = W.config1()
    cfg.update(nkx=64, nky=32, neps=128, emin=-2.0, emax=2.0, omega=np.arange(1, 41) * (4.0 / 128))
    ref, _ = oracle_extended(cfg)
    first = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    second = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    s1, s2 = first.info.schedule.decode(), second.info.schedule.decode()
    print(s1, "|", s2)
    assert " cached " in s2 or s2.endswith(" cached")
    for plan in (first, second):
        got = plan.exec()
        torch.cuda.synchronize()
        assert normwise(got.double().cpu().numpy(), ref) <= 1e-5
        plan.close()
    # the general path tunes its own window form
    monkeypatch.setenv("LINDHARD_SYMMETRY", "off")
    gen = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert " even " not in gen.info.schedule.decode()
    got = gen.exec()
    torch.cuda.synchronize()
    assert normwise(got.double().cpu().numpy(), ref) <= 1e-5
    gen.close()
    assert (tmp_path / "tune.txt").exists()


@pytest.mark.parametrize("window", ["auto", "direct", "fft"], indirect=True)
@pytest.mark.parametrize("prec", PRECS)
def test_grid_4096_sampled_and_q_sum(prec, window):
    """The largest power-of-two grid, 4096^2 k (128 energies on [-2, 2] eV,
    lags 1..64, G = 0.02 eV): sampled (q, m) against the oracle's direct sum
    and the q-sum identity (the oracle's q-average from k-averaged spectral
    weights) at every lag, on the even and the general path."""
    cfg = W.config3(nk=4096, neps=128)
    cfg.update(gamma=0.02, omega=W.lag_omegas(128, -2.0, 2.0, range(1, 65)))
    n, neps = cfg["nkx"], cfg["neps"]
    xi, mu = oracle_xi(cfg)
    plan = LH.Plan(precision=prec, **cfg)
    assert abs(plan.info.mu - mu) < 1e-12
    sched = plan.info.schedule.decode()
    assert (" even " in sched) == (window == "auto")
    out = plan.exec()
    torch.cuda.synchronize()
    samples = [(0, 0, 1), (n // 2, 0, 32), (n // 2, n // 2, 64), (1234, 3001, 17), (4095, 1, 50), (7, 2048, 3)]
    qx = np.array([s[0] for s in samples])
    qy = np.array([s[1] for s in samples])
    ms = np.array([s[2] for s in samples])
    ref = oracle.chi_pairs(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, ms)
    got = np.array([out[m - 1, (b + n // 2) % n, (a + n // 2) % n].item() for a, b, m in samples])
    scale = out.abs().max().item()
    err_s = np.abs(got - ref).max() / scale
    qref = oracle.chi_qmean(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], lags_of(cfg))
    qgot = out.double().mean(dim=(1, 2)).cpu().numpy()
    err_q = normwise(qgot, qref)
    print("4096^2 prec=%d window=%s sampled err %.3e, q-sum err %.3e, %s" % (prec, window, err_s, err_q, sched))
    plan.close()
    assert err_s <= TOL[prec] and err_q <= TOL[prec]


@pytest.mark.parametrize("window", ["auto", "even-mfma4"], indirect=True)
def test_grid_4096_512_energies_sampled(window):
    """4096^2 k x 512 energies x 256 lags, FP32: the energy window's staged
    slices then span more than 4 GiB of byte offsets (the rank-1 matrix window
    switches to 64-bit addressing); sampled (q, m) against the oracle."""
    cfg = W.config3(nk=4096)
    n, neps = cfg["nkx"], cfg["neps"]
    xi, mu = oracle_xi(cfg)
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    sched = plan.info.schedule.decode()
    if window == "even-mfma4":
        assert " P3 mfma4 " in sched
    out = plan.exec()
    torch.cuda.synchronize()
    samples = [(0, 0, 1), (n // 2, n // 2, 256), (1234, 3001, 170), (4095, 1, 50), (7, 2048, 255), (999, 17, 128)]
    qx = np.array([s[0] for s in samples])
    qy = np.array([s[1] for s in samples])
    ms = np.array([s[2] for s in samples])
    ref = oracle.chi_pairs(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, ms)
    got = np.array([out[m - 1, (b + n // 2) % n, (a + n // 2) % n].item() for a, b, m in samples])
    err = np.abs(got - ref).max() / out.abs().max().item()
    print("4096^2 x 512 [%s] sampled err %.3e, %s" % (window, err, sched))
    plan.close()
    assert err <= 1e-5
