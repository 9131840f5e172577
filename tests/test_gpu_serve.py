"""Serving: continuous batching through lindhard_serve_* (C ABI).

Each served result must equal the same problem run alone (bitwise: the
schedule is deterministic and uses no atomics), a sample must match the
oracle, admission must respect the HBM budget, and rejected, invalid or
cancelled jobs must not affect the others."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1208_3210_amd import lindhard as LH
from paper_1208_3210_amd import workloads as W

pytestmark = pytest.mark.gpu


def small_jobs(n=14, seed=9):
    """The served workload's recipe at test sizes: k-grids 32..256, energies 32..128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for i in range(n):
        nk = int(rng.choice([32, 64, 128, 256]))
        neps = int(rng.choice([32, 64, 128]))
        nw = int(rng.integers(4, neps // 2 + 1))
        band = W.seeded_band(rng)
        U = float(rng.uniform(0.0, 2.0)) if rng.uniform() < 0.5 else float("nan")
        prob = dict(**band, filling=1.0 + rng.uniform(0, 0.2), nkx=nk, nky=nk, neps=neps, emin=-2.0, emax=2.0,
                    gamma=float(rng.uniform(0.02, 0.08)),
                    omega=W.lag_omegas(neps, -2.0, 2.0, range(1, nw + 1)),
                    precision=LH.LINDHARD_FP32C if i % 3 else LH.LINDHARD_FP64)
        jobs.append((U, prob))
    return jobs


def run_alone(U, prob):
    kw = dict(prob)
    if math.isfinite(U):
        kw["want_rpa"] = True
    plan = LH.Plan(**kw)
    im = plan.exec()
    res = {"im_chi": im}
    if math.isfinite(U):
        re, imr, rer = plan.rpa(U)
        res.update(re_chi=re, im_rpa=imr, re_rpa=rer)
    torch.cuda.synchronize()
    plan.close()
    return res


def test_served_results_equal_alone_and_match_oracle():
    jobs = small_jobs()
    srv = LH.Server(hbm_budget_bytes=8 << 30, max_inflight=4, max_queue=64)
    tickets = [srv.submit(U, **prob) for U, prob in jobs]
    for t, _ in tickets:
        assert srv.wait(t, 120.0) == LH.LINDHARD_OK
    st = srv.stats()
    assert st.completed == len(jobs) and st.failed == 0
    assert 0 < st.p50_ms <= st.p99_ms and st.points_per_s > 0
    assert st.hbm_high_water <= 8 << 30
    for (U, prob), (t, outs) in zip(jobs, tickets):
        alone = run_alone(U, prob)
        for k, v in alone.items():
            assert torch.equal(outs[k], v), (t, k)
    # one served job against the oracle
    U, prob = jobs[0]
    outs = tickets[0][1]
    eps = oracle.band_tb(prob["t"], prob["tp"], prob["tpp"], prob["nkx"], prob["nky"])
    mu = oracle.mu_solve(eps, prob["gamma"], prob["filling"])
    d = (prob["emax"] - prob["emin"]) / prob["neps"]
    lags = np.rint(np.asarray(prob["omega"]) / d).astype(int)
    full = oracle.chi_full(eps - mu, prob["neps"], prob["emin"], prob["emax"], prob["gamma"], lags)
    ref = oracle.extend(full, 1, 1, 0, 0.0)
    got = outs["im_chi"].double().cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    tol = 1e-11 if prob["precision"] == LH.LINDHARD_FP64 else 1e-5
    print("served vs oracle err %.3e" % err)
    assert err <= tol
    srv.close()


def test_admission_budget_rejection_cancel_and_isolation():
    U, prob = small_jobs(1, seed=3)[0]
    prob = dict(prob, nkx=256, nky=256, neps=128, omega=W.lag_omegas(128, -2.0, 2.0, range(1, 33)))
    probe = LH.Plan(**prob)
    fp = probe.info.workspace_bytes
    probe.close()
    # budget for one job at a time: admission serialises them
    srv = LH.Server(hbm_budget_bytes=int(fp * 1.5), max_inflight=4, max_queue=16)
    good = [srv.submit(float("nan"), **prob) for _ in range(4)]
    # a job larger than the budget is refused at submission
    big = dict(prob, nkx=1024, nky=1024)
    with pytest.raises(LH.LindhardError) as ei:
        srv.submit(float("nan"), **big)
    assert ei.value.status == LH.LINDHARD_ETOOBIG
    # an invalid job (omega off the lag grid) is refused and poisons nothing
    with pytest.raises(LH.LindhardError) as ei:
        srv.submit(float("nan"), **dict(prob, omega=[0.0123]))
    assert ei.value.status == LH.LINDHARD_EOFFGRID
    last, _ = srv.submit(float("nan"), **prob)
    rc = srv.cancel(last)
    assert rc in (LH.LINDHARD_OK, LH.LINDHARD_EBUSY)
    for t, _ in good:
        assert srv.wait(t, 120.0) == LH.LINDHARD_OK
    st_last = srv.wait(last, 120.0)
    assert st_last == (LH.LINDHARD_ECANCELED if rc == LH.LINDHARD_OK else LH.LINDHARD_OK)
    st = srv.stats()
    assert st.hbm_high_water <= int(fp * 1.5)
    assert st.rejected == 2
    ref = run_alone(float("nan"), prob)["im_chi"]
    for _, outs in good:
        assert torch.equal(outs["im_chi"], ref)
    srv.close()


def test_exec_batch_equals_individual_runs():
    """Mixed-size instances run as one batch give the same bits as one by one;
    the batch is captured into a HIP graph on its first call and replayed
    afterwards, so it is replayed several times with eager work and clears in
    between, and every replay is checked."""
    jobs = small_jobs(8, seed=21)
    plans = [LH.Plan(**prob) for U, prob in jobs]
    dtypes = {p.dtype for p in plans}
    for dt in dtypes:
        group = [p for p in plans if p.dtype == dt]
        alone = []
        for p in group:
            alone.append(p.exec())
        torch.cuda.synchronize()
        outs = [p.empty() for p in group]
        for rep in range(4):
            for o in outs:
                o.fill_(float("nan"))
            LH.exec_batch(group, outs)
            torch.cuda.synchronize()
            for o, a in zip(outs, alone):
                assert torch.equal(o, a), rep
            # eager work on the same plans between replays
            again = group[rep % len(group)].exec()
            torch.cuda.synchronize()
            assert torch.equal(again, alone[rep % len(group)])
    for p in plans:
        p.close()


def test_served_extended_forms_equal_alone():
    """Jobs using the wider problem fields (several bands with pair weights,
    a 3D grid, a grid that is not a power of two, omegas between lags, band
    pairs with a |M(Q)|^2 map each) are
    copied whole at submission: served results equal the same problems run
    alone, bit for bit."""
    d = 3.0 / 64
    base = dict(neps=64, emin=-1.5, emax=1.5, gamma=0.08, filling=1.1, precision=LH.LINDHARD_FP32C)
    jobs = [
        dict(base, eps_table=W.multiband_tables(32, 2, seed=4), n_bands=2, nkx=32, nky=32,
             pair_weight=np.array([[1.0, 0.3], [0.7, 0.2]]), omega=np.arange(1, 30, 4) * d),
        dict(base, eps_table=W.band3d_table(16, 8, 4), nkz=4, nkx=16, nky=8, omega=np.arange(1, 30, 4) * d),
        dict(base, eps_table=np.random.Generator(np.random.PCG64(2)).uniform(-1.2, 1.5, size=(17, 33)), nkx=33,
             nky=17, omega=np.arange(1, 30, 4) * d),
        dict(base, t=0.4, tp=-0.1, tpp=0.05, nkx=32, nky=32, omega_interp=True, omega=[2.5 * d, 7.25 * d, 30.9 * d]),
        dict(base, eps_table=W.multiband_tables(32, 2, seed=5), n_bands=2, nkx=32, nky=32, zones=(3, 1),
             pair_m2=np.random.Generator(np.random.PCG64(6)).uniform(0.0, 1.0, size=(2, 2, 32, 96)),
             omega=np.arange(1, 30, 4) * d),
    ]
    srv = LH.Server(hbm_budget_bytes=4 << 30, max_inflight=4, max_queue=16)
    tickets = [srv.submit(float("nan"), **j) for j in jobs]
    for t, _ in tickets:
        assert srv.wait(t, 120.0) == LH.LINDHARD_OK
    for j, (t, outs) in zip(jobs, tickets):
        plan = LH.Plan(**j)
        alone = plan.exec()
        torch.cuda.synchronize()
        assert torch.equal(outs["im_chi"], alone), t
        plan.close()
    srv.close()


def _tb(seed):
    band = W.seeded_band(np.random.Generator(np.random.PCG64(seed)))
    return dict(**band, filling=1.05 + 0.01 * (seed % 7), gamma=0.03 + 0.005 * (seed % 5))


def test_cached_plans_rebound_across_lag_ranges_equal_alone():
    """Jobs of one class (grid, energy window, precision) with different bands
    and omega lists run on one cached plan, rebound in place: a small lag
    range first, then larger ones (the spectral buffers grow), then a small
    one again on the grown buffers, then an RPA job (its own class).  Each
    result equals the problem planned afresh, bit for bit, and the server
    reports the reuse."""
    neps, e0, e1 = 128, -2.0, 2.0
    lag_sets = [range(1, 9), range(1, 41), range(3, 64, 5), range(1, 17), range(20, 60)]
    jobs = []
    for i, lags in enumerate(lag_sets):
        for prec in (LH.LINDHARD_FP32C, LH.LINDHARD_FP64):
            jobs.append((float("nan"), dict(**_tb(i), nkx=64, nky=64, neps=neps, emin=e0, emax=e1,
                                            omega=W.lag_omegas(neps, e0, e1, lags), precision=prec)))
    jobs.append((0.7, dict(**_tb(9), nkx=64, nky=64, neps=neps, emin=e0, emax=e1,
                           omega=W.lag_omegas(neps, e0, e1, range(1, 33)), precision=LH.LINDHARD_FP32C)))
    jobs.append((1.3, dict(**_tb(10), nkx=64, nky=64, neps=neps, emin=e0, emax=e1,
                           omega=W.lag_omegas(neps, e0, e1, range(2, 50, 3)), precision=LH.LINDHARD_FP32C)))
    # one worker, one job at a time (no merging): each runs on the plan its
    # predecessor of the class left behind
    srv = LH.Server(hbm_budget_bytes=4 << 30, max_inflight=1, max_queue=64)
    tickets = []
    for U, prob in jobs:
        tickets.append(srv.submit(U, **prob))
        assert srv.wait(tickets[-1][0], 120.0) == LH.LINDHARD_OK
    st = srv.stats()
    assert st.plan_builds == 3 and st.plan_reuses == len(jobs) - 3, (st.plan_builds, st.plan_reuses)
    assert st.cached_plans == 3 and st.resident_bytes <= st.hbm_high_water <= 4 << 30
    for (U, prob), (t, outs) in zip(jobs, tickets):
        alone = run_alone(U, prob)
        for k, v in alone.items():
            assert torch.equal(outs[k], v), (t, k)
    srv.close()


def test_warm_problems_and_eviction():
    """Problems given at creation are planned before the first job, so a job
    of their class reuses a plan at once; under a budget that holds about one
    plan, idle plans of other classes are evicted least recently used first
    and every result still equals the problem run alone."""
    e0, e1 = -2.0, 2.0
    mk = lambda nk, neps, seed, lags: dict(**_tb(seed), nkx=nk, nky=nk, neps=neps, emin=e0, emax=e1,  # noqa: E731
                                           omega=W.lag_omegas(neps, e0, e1, lags), precision=LH.LINDHARD_FP32C)
    warm = [mk(128, 64, 0, range(1, 33)), mk(64, 128, 1, range(1, 33))]
    srv = LH.Server(hbm_budget_bytes=8 << 30, max_inflight=2, max_queue=16, warm=warm)
    st = srv.stats()
    assert st.plan_builds == 2 and st.cached_plans == 2 and st.completed == 0
    t, outs = srv.submit(float("nan"), **mk(128, 64, 5, range(1, 20)))
    assert srv.wait(t, 120.0) == LH.LINDHARD_OK
    st = srv.stats()
    assert st.plan_reuses == 1 and st.plan_builds == 2
    assert torch.equal(outs["im_chi"], run_alone(float("nan"), mk(128, 64, 5, range(1, 20)))["im_chi"])
    # a wait that reported the job finished released its ticket
    with pytest.raises(LH.LindhardError):
        srv.wait(t, 1.0)
    srv.close()

    # two classes of about one budget each: every job evicts the other's plan
    probs = [mk(256, 128, 2, range(1, 33)), mk(256, 64, 3, range(1, 33)), mk(256, 128, 4, range(1, 40))]
    fps = []
    for pr in probs:
        p = LH.Plan(**pr)
        fps.append(p.info.workspace_bytes)
        p.close()
    budget = int(max(fps) * 1.3)
    srv = LH.Server(hbm_budget_bytes=budget, max_inflight=1, max_queue=16)
    tickets = []
    for pr in probs:
        tickets.append(srv.submit(float("nan"), **pr))
        assert srv.wait(tickets[-1][0], 120.0) == LH.LINDHARD_OK
    st = srv.stats()
    assert st.plan_evictions == 2 and st.plan_builds == 3 and st.hbm_high_water <= budget
    for pr, (t, outs) in zip(probs, tickets):
        assert torch.equal(outs["im_chi"], run_alone(float("nan"), pr)["im_chi"]), t
    srv.close()


@pytest.mark.parametrize("window", ["mfma4", "direct"])
def test_grouped_batch_launches_equal_alone(window, monkeypatch):
    """Instances of one grid run each pass as one launch over the group (the
    grid spans the largest instance; smaller ones return early): energies,
    lag ranges, bands, fillings and broadenings differ inside a group, and
    each result equals the instance run alone, bit for bit.  Also with a
    group of FP64 instances and one instance that is batched on its own."""
    monkeypatch.setenv("LINDHARD_EVEN_WINDOW", window)
    e0, e1 = -2.0, 2.0
    probs = []
    for i, (nk, neps, lags, prec) in enumerate([
            (64, 64, range(1, 33), LH.LINDHARD_FP32C), (64, 128, range(1, 50), LH.LINDHARD_FP32C),
            (64, 128, range(5, 20), LH.LINDHARD_FP32C), (64, 256, range(1, 120, 3), LH.LINDHARD_FP32C),
            (128, 64, range(1, 17), LH.LINDHARD_FP32C), (128, 128, range(1, 65), LH.LINDHARD_FP32C),
            (64, 64, range(1, 33), LH.LINDHARD_FP64), (64, 128, range(2, 40, 2), LH.LINDHARD_FP64),
            (32, 64, range(1, 9), LH.LINDHARD_FP32C)]):
        band = W.seeded_band(np.random.Generator(np.random.PCG64(100 + i)))
        probs.append(dict(**band, filling=1.02 + 0.02 * i, gamma=0.02 + 0.005 * i, nkx=nk, nky=nk, neps=neps,
                          emin=e0, emax=e1, omega=W.lag_omegas(neps, e0, e1, lags), precision=prec,
                          zones=(3, 1) if i == 1 else (1, 1)))
    plans = [LH.Plan(**p) for p in probs]
    alone = [p.exec() for p in plans]
    torch.cuda.synchronize()
    for dt in (torch.float32, torch.float64):
        group = [(p, a) for p, a in zip(plans, alone) if p.dtype == dt]
        outs = [p.empty() for p, _ in group]
        for rep in range(3):
            for o in outs:
                o.fill_(float("nan"))
            LH.exec_batch([p for p, _ in group], outs)
            torch.cuda.synchronize()
            for o, (_, a) in zip(outs, group):
                assert torch.equal(o, a), rep
    for p in plans:
        p.close()


def test_queued_jobs_of_one_class_run_merged_and_equal_alone():
    """A burst of jobs of one class queued behind a busy worker is taken
    together and run as grouped launches (the server counts them as merged);
    every result equals the job run alone, bit for bit."""
    e0, e1, neps = -2.0, 2.0, 128
    probs = []
    for i in range(10):
        band = W.seeded_band(np.random.Generator(np.random.PCG64(300 + i)))
        lags = range(1, 17 + 3 * i)
        probs.append(dict(**band, filling=1.0 + 0.015 * i, gamma=0.03 + 0.004 * i, nkx=128, nky=128, neps=neps,
                          emin=e0, emax=e1, omega=W.lag_omegas(neps, e0, e1, lags), precision=LH.LINDHARD_FP32C))
    srv = LH.Server(hbm_budget_bytes=8 << 30, max_inflight=1, max_queue=64)
    tickets = [srv.submit(float("nan"), **p) for p in probs]
    for t, _ in tickets:
        assert srv.wait(t, 120.0) == LH.LINDHARD_OK
    st = srv.stats()
    print("merged %d of %d, builds %d reuses %d" % (st.merged_jobs, len(probs), st.plan_builds, st.plan_reuses))
    assert st.merged_jobs >= 2 and st.completed == len(probs)
    for p, (t, outs) in zip(probs, tickets):
        assert torch.equal(outs["im_chi"], run_alone(float("nan"), p)["im_chi"]), t
    srv.close()
