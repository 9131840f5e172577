"""The widened forms at the sizes and launch configurations the benchmark
times, against the oracle on sampled (q, omega) points (errors relative to
the largest |Im chi| of the GPU map, FP32 bar 1e-5): two bands as weighted
pairs and as a summed spectral function (2048^2 k, 512 energies), the 3D grid
(256 x 256 x 64 k) and the paper's 2049^2 grid over 16 x 16 zones."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pairs", [True, False])
def test_two_bands_full_size_sampled(pairs):
    cfg = W.config_multiband(pairs=pairs)
    n, neps = cfg["nkx"], cfg["neps"]
    eps = np.asarray(cfg["eps_table"])
    mu = oracle.mu_solve_bands(eps, cfg["gamma"], cfg["filling"])
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert abs(plan.info.mu - mu) < 1e-10
    out = plan.exec()
    torch.cuda.synchronize()
    qx, qy, ms = np.array([0, 300, 1500]), np.array([0, 77, 2000]), np.array([1, 90, 256])
    ref = oracle.chi_grid_mb(eps - mu, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, ms,
                             pair_weight=cfg.get("pair_weight"))
    got = np.array([[out[m - 1, (b + n // 2) % n, (a + n // 2) % n].item() for m in ms] for a, b in zip(qx, qy)])
    err = np.abs(got - ref).max() / out.abs().max().item()
    print("two bands pairs=%d 2048^2 sampled err %.2e" % (pairs, err))
    assert err <= 1e-5
    plan.close()


def test_3d_full_size_sampled():
    cfg = W.config_3d()
    nx, ny, nz, neps = cfg["nkx"], cfg["nky"], cfg["nkz"], cfg["neps"]
    eps = np.asarray(cfg["eps_table"])
    mu = oracle.mu_solve(eps.reshape(-1), cfg["gamma"], cfg["filling"])
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert abs(plan.info.mu - mu) < 1e-10
    out = plan.exec()
    torch.cuda.synchronize()
    qx, qy, qz = np.array([0, 100, 255]), np.array([0, 31, 128]), np.array([0, 7, 40])
    ms = np.array([1, 128, 256])
    ref = oracle.chi_grid_3d(eps - mu, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, qz, ms)
    got = np.array([[out[m - 1, ((c + nz // 2) % nz) * ny + (b + ny // 2) % ny, (a + nx // 2) % nx].item()
                     for m in ms] for a, b, c in zip(qx, qy, qz)])
    err = np.abs(got - ref).max() / out.abs().max().item()
    print("3d 256x256x64 sampled err %.2e" % err)
    assert err <= 1e-5
    plan.close()


def test_grid_2049_full_size_sampled():
    cfg = W.config_extended(nk=2049)
    n, neps = cfg["nkx"], cfg["neps"]
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], n, n, cfg["k_zones"])
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    assert abs(plan.info.mu - mu) < 1e-10
    out = plan.exec()
    torch.cuda.synchronize()
    samples = [(0, 0, 1), (128, 0, 100), (1024, 1025, 256), (2048, 5, 40), (77, 1500, 200), (1, 2048, 3)]
    qx = np.array([s[0] for s in samples])
    qy = np.array([s[1] for s in samples])
    ms = np.array([s[2] for s in samples])
    ref = oracle.chi_pairs(eps - mu, neps, cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, ms, rho=cfg["rho_table"])
    got = np.array([out[m - 1, (b + n // 2) % n, (a + n // 2) % n].item() for a, b, m in samples])
    err = np.abs(got - ref).max() / out.abs().max().item()
    print("2049^2 sampled err %.2e, schedule %s" % (err, plan.info.schedule.decode()))
    assert err <= 1e-5
    plan.close()
