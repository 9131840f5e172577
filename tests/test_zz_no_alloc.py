"""lindhard_q_average_noalloc (the q-average with the library's per-device
scratch array, for callers that cannot allocate device memory) against
lindhard_q_average of a plan, through the C ABI: two calls in a row, the
second on a smaller input, and against the oracle's q-average (the
q-integrated joint density of states of Fig. 2(b))."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(nk, neps, nlag, prec):
    cfg = W.config1()
    cfg.update(nkx=nk, nky=nk, neps=neps, emin=-2.0, emax=2.0, gamma=0.08,
               omega=np.arange(1, nlag + 1) * (4.0 / neps))
    plan = LH.Plan(precision=prec, **cfg)
    im = plan.exec()
    ref = plan.q_average(im)
    torch.cuda.synchronize()
    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], nk, nk)
    xi = eps - plan.info.mu
    qref = oracle.chi_qmean(xi, neps, cfg["emin"], cfg["emax"], cfg["gamma"], np.arange(1, nlag + 1))
    return plan, im, ref, qref


def test_q_average_noalloc_matches_the_plan_form_twice():
    # The first call on a device looks up the scratch array's address; the
    # runtime may place the library's device arrays then.  After it, calls
    # must leave the device's free memory unchanged.
    warm = torch.ones((2, 8), dtype=torch.float32, device="cuda")
    wout = torch.zeros(2, dtype=torch.float64, device="cuda")
    LH.q_average_noalloc(warm, wout)
    torch.cuda.synchronize()
    assert torch.equal(wout, torch.ones(2, dtype=torch.float64, device="cuda"))
    # first call: 64^2 k, 128 energies, 96 planes, FP32; second: 16^2, 32 energies, 12 planes, FP64
    for nk, neps, nlag, prec, tol in ((64, 128, 96, LH.LINDHARD_FP32C, 1e-5), (16, 32, 12, LH.LINDHARD_FP64, 1e-11)):
        plan, im, ref, qref = _case(nk, neps, nlag, prec)
        out = torch.full((nlag,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        LH.q_average_noalloc(im, out)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0, "the call must not allocate device memory"
        assert torch.equal(out, ref), "same kernels and partition: bit-identical to lindhard_q_average"
        err = np.abs(out.cpu().numpy() - qref).max() / np.abs(qref).max()
        print("noalloc q-average nk=%d nw=%d prec=%d err vs oracle %.2e" % (nk, nlag, prec, err))
        assert err <= tol
        plan.close()


def test_q_average_noalloc_rejects_sizes_beyond_its_scratch():
    im = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    out = torch.zeros(LH.NOALLOC_MAX_PLANES + 1, dtype=torch.float64, device="cuda")
    big = torch.zeros((LH.NOALLOC_MAX_PLANES + 1, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(LH.LindhardError) as ei:
        LH.q_average_noalloc(big, out)
    assert ei.value.status == LH.LINDHARD_EINVAL
    with pytest.raises(LH.LindhardError) as ei:
        LH.lindhard_q_average_noalloc(im.data_ptr(), 4, 8, 2, out.data_ptr(), 0)
    assert ei.value.status == LH.LINDHARD_EINVAL
    torch.cuda.synchronize()
