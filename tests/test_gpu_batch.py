"""The batched workload (mixed grids, energies, dopings and broadenings, run
with lindhard_exec_batch) against the FP64 oracle, instance by instance.

Every instance of the 64-instance batch (k-grids 128^2..1024^2, 64..512
energies, 64 lags, seed 4) is compared with the oracle's direct double sum at
two q points over all 64 lags and with the q-sum identity (the oracle's
q-average from the k-averaged spectral weights) at every lag; a reduced batch
(128^2 and 256^2 grids) is compared on a 16 x 16 q subsample at every lag.
Normwise, FP32 with compensated energy sums <= 1e-5."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def lags_of(cfg):
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    return np.rint(np.asarray(cfg["omega"]) / d).astype(np.int64)


def xi_of(cfg):
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"])
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    return eps - mu, mu


def run_batch(cfgs):
    plans = [LH.Plan(precision=LH.LINDHARD_FP32C, **c) for c in cfgs]
    outs = [p.empty() for p in plans]
    LH.exec_batch(plans, outs)
    torch.cuda.synchronize()
    return plans, outs


def sample(out, qx, qy, n):
    X = torch.as_tensor((np.asarray(qx) + n // 2) % n, device=out.device, dtype=torch.long)
    Y = torch.as_tensor((np.asarray(qy) + n // 2) % n, device=out.device, dtype=torch.long)
    return out[:, Y, X].double().cpu().numpy().T  # (nq, nlag)


def _oracle_instance(cfg, qx, qy):
    xi, mu = xi_of(cfg)
    lags = lags_of(cfg)
    ref = oracle.chi_grid(xi, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, lags)
    qref = oracle.chi_qmean(xi, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], lags)
    return mu, ref, qref


def test_config4_every_instance_against_oracle():
    from concurrent.futures import ThreadPoolExecutor

    cfgs = W.config4()
    plans, outs = run_batch(cfgs)
    rng = np.random.Generator(np.random.PCG64(44))
    qs = [([int(rng.integers(0, c["nkx"])), c["nkx"] // 2], [int(rng.integers(0, c["nky"])), c["nky"] // 4])
          for c in cfgs]
    # the oracle's sums of different instances run side by side (ctypes and
    # numpy release the interpreter lock)
    with ThreadPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(lambda a: _oracle_instance(*a), [(c, q[0], q[1]) for c, q in zip(cfgs, qs)]))
    worst = 0.0
    for i, (cfg, p, out, (qx, qy), (mu, ref, qref)) in enumerate(zip(cfgs, plans, outs, qs, refs)):
        assert abs(p.info.mu - mu) < 1e-12
        got = sample(out, qx, qy, cfg["nkx"])
        err = np.abs(got - ref).max() / np.abs(ref).max()
        qgot = out.double().mean(dim=(1, 2)).cpu().numpy()
        qerr = np.abs(qgot - qref).max() / np.abs(qref).max()
        worst = max(worst, err, qerr)
        assert err <= TOL and qerr <= TOL, (i, cfg["nkx"], cfg["neps"], err, qerr)
    print("config4: 64 instances, worst normwise error %.3e" % worst)
    for p in plans:
        p.close()


def test_reduced_batch_on_a_q_subsample():
    rng = np.random.Generator(np.random.PCG64(404))
    cfgs = []
    for _ in range(12):
        nk = int(rng.choice([128, 256]))
        neps = int(rng.choice([64, 128, 256]))
        cfgs.append(dict(**W.BAND1, filling=1.0 + rng.uniform(0.0, 0.2), nkx=nk, nky=nk, neps=neps, emin=-2.0,
                         emax=2.0, gamma=rng.uniform(0.01, 0.08), omega=W.lag_omegas(neps, -2.0, 2.0, range(1, 65))))
    plans, outs = run_batch(cfgs)
    for i, (cfg, p, out) in enumerate(zip(cfgs, plans, outs)):
        n = cfg["nkx"]
        xi, _ = xi_of(cfg)
        g = np.arange(0, n, n // 16) + 3
        QY, QX = np.meshgrid(g % n, g % n, indexing="ij")
        lags = lags_of(cfg)
        ref = oracle.chi_grid(xi, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], QX.ravel(), QY.ravel(), lags)
        got = sample(out, QX.ravel(), QY.ravel(), n)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print("reduced batch %d: %d^2 k, %d energies, err %.3e" % (i, n, cfg["neps"], err))
        assert err <= TOL
    for p in plans:
        p.close()
