"""Benchmark of the Lindhard hot path on one MI355X.

Workload: 2048 x 2048 k-grid, 512 energy points on [-2, 2] eV, G = 0.01 eV,
256 omegas in (0, 2] eV, seeded t-t'-t'' band, filling 1.15, FP32 with the
compensated energy window.  One step = one lindhard_exec: the whole hot path
(spectral builder + row FFT, column FFT, energy window, inverse column FFT,
inverse row FFT + epilogue) with the band, twiddles and workspace resident in
HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PASS_NAMES = ["p1_build_rowfft", "p2_colfft", "p3_window", "p4_colifft", "p5_rowifft_epilogue"]
KERNEL_NAMES = ["k_p1", "k_col<float, false>", "k_p3", "k_col<float, true>", "k_p5"]


def algorithmic(cfg, lag_hi, even, fp_bytes=4):
    """Algorithmic HBM bytes per pass and flops of the energy window for one
    exec.  General path: complex half plane (nkx/2+1) x nky per slice.  Even
    path (mirror-symmetric band): real quarter plane (nkx/2+1) x (nky/2+1)."""
    n_x, n_y, neps = cfg["nkx"], cfg["nky"], cfg["neps"]
    nw = len(cfg["omega"])
    if even:
        pts = (n_x // 2 + 1) * (n_y // 2 + 1)
        vb = fp_bytes
        flops_per_mac = 2.0
    else:
        pts = (n_x // 2 + 1) * n_y
        vb = 2 * fp_bytes
        flops_per_mac = 8.0
    nS = neps  # every slice enters the window at this workload
    nL = lag_hi
    B = pts * nS * vb
    S = pts * nL * vb
    out = n_x * n_y * nw * fp_bytes
    by = [B, 2 * B, B + S, 2 * S, S + out]
    j0 = neps // 2
    macs = sum(min(m, j0, neps - m) for m in range(1, nL + 1))
    fl_win = flops_per_mac * pts * macs
    return by, fl_win


def src_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, kernel_src_hash):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter
    reads for a plain 1 GiB device copy), only if the counters were taken on
    the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_2048x2048x512_fp32c.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_src_hash") != kernel_src_hash:
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("traffic_bytes_per_launch")


def cpu_baseline(cfg, nsamples=128):
    import oracle

    eps = oracle.band_tb(cfg["t"], cfg["tp"], cfg["tpp"], cfg["nkx"], cfg["nky"])
    mu = oracle.mu_solve(eps, cfg["gamma"], cfg["filling"])
    xi = eps - mu
    rng = np.random.Generator(np.random.PCG64(77))
    n = cfg["nkx"]
    nlag = len(cfg["omega"])
    qx = rng.integers(0, n, nsamples)
    qy = rng.integers(0, n, nsamples)
    ms = rng.integers(1, nlag + 1, nsamples)
    t0 = time.perf_counter()
    oracle.chi_pairs(xi, cfg["neps"], cfg["emin"], cfg["emax"], cfg["gamma"], qx, qy, ms)
    dt = time.perf_counter() - t0
    return {"value": nsamples / dt, "unit": "chi(q,w) points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d (q, omega) points of the 2048^2 k x 512 energy workload, q uniform, lag uniform in "
                      "1..%d, FP64 direct double sum; %.1f s wall" % (nsamples, nlag, dt)}


def bench_batched(LH, W, torch, steps=3):
    """64 mixed instances (k-grids 128^2..1024^2, 64..512 energies, 64 lags,
    doping x in [0, 0.2], G in [0.01, 0.08] eV) run as one batch per step."""
    cfgs = W.config4()
    t0 = time.perf_counter()
    plans = [LH.Plan(precision=LH.LINDHARD_FP32C, **c) for c in cfgs]
    t_plan = time.perf_counter() - t0
    outs = [p.empty() for p in plans]
    LH.exec_batch(plans, outs)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        LH.exec_batch(plans, outs)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    points = sum(c["nkx"] * c["nky"] * len(c["omega"]) for c in cfgs)
    for p in plans:
        p.close()
    del outs
    return {"instances": len(cfgs), "ms_per_batch": ms, "points_per_batch": points,
            "points_per_s": points / (ms * 1e-3), "plan_s_total": t_plan}


def served_warm_set(LH, W):
    """One problem per plan class and window-schedule bucket of the served
    stream: every grid and energy count, RPA or not, and (without RPA) the
    highest lag of each 32-lag bucket that 16..128 omegas reach."""
    warm = []
    band = dict(t=0.4, tp=-0.1, tpp=0.04, filling=1.1, gamma=0.04)
    for nk in (128, 256, 512, 1024):
        for neps in (64, 128, 256, 512):
            base = dict(**band, nkx=nk, nky=nk, neps=neps, emin=-2.0, emax=2.0, zones=(1, 1), ff_kind=0,
                        ff_width=0.0, precision=LH.LINDHARD_FP32C)
            warm.append(dict(base, omega=W.lag_omegas(neps, -2.0, 2.0, range(1, 129)), want_rpa=True))
            for top in (32, 64, 96, 128):
                if top - 31 < neps:
                    warm.append(dict(base, omega=W.lag_omegas(neps, -2.0, 2.0, range(1, min(top, neps - 1) + 1))))
    return warm


def bench_served(LH, W, torch, n_warm=200, n_req=2000, rate_hz=200.0, n_iso=400):
    """Poisson stream (mean 200 req/s) of mixed jobs through the server, its
    plan classes planned at creation; latency = submit -> result ready,
    reported over the requests after warm-up.  Then every fifth measured job
    again, alone (submitted after the previous one finished), for its
    isolated latency: the ratio served / isolated per job shows what the mix
    adds to each job, apart from the spread of job sizes."""
    jobs = W.config5(n_req=n_warm + n_req, rate_hz=rate_hz)
    t_c = time.perf_counter()
    srv = LH.Server(hbm_budget_bytes=64 << 30, max_inflight=8, max_queue=4096, warm=served_warm_set(LH, W))
    t_create = time.perf_counter() - t_c
    live = {}
    lat = {}
    t0 = time.perf_counter()
    done_points = 0

    def reap(block=False):
        nonlocal done_points
        for t in list(live):
            fin, st = srv.poll(t)
            if fin:
                k, t_sub, pts = live.pop(t)
                if st == LH.LINDHARD_OK and k >= n_warm:
                    lat[k] = (time.perf_counter() - t_sub) * 1e3
                    done_points += pts
                srv._keep.pop(t, None)
    t_first = None
    for k, job in enumerate(jobs):
        while True:
            now = time.perf_counter() - t0
            if now >= job["arrival_s"]:
                break
            reap()
            time.sleep(min(0.0005, job["arrival_s"] - now))
        while len(live) > 256:  # back-pressure: queued jobs hold their outputs
            reap()
            time.sleep(0.0005)
        if k == n_warm:
            t_first = time.perf_counter()
        ticket, outs = srv.submit(job["U"], precision=LH.LINDHARD_FP32C, **job["problem"])
        pts = outs["im_chi"].numel()
        live[ticket] = (k, time.perf_counter(), pts)
    while live:
        reap()
        time.sleep(0.0005)
    wall = time.perf_counter() - t_first
    st = srv.stats()
    # isolated latencies of a sample of the same jobs
    iso = {}
    for k in sorted(lat)[::max(1, n_req // n_iso)]:
        job = jobs[k]
        t_sub = time.perf_counter()
        ticket, outs = srv.submit(job["U"], precision=LH.LINDHARD_FP32C, **job["problem"])
        while not srv.poll(ticket)[0]:
            time.sleep(0.00005)
        iso[k] = (time.perf_counter() - t_sub) * 1e3
        srv._keep.pop(ticket, None)
    st2 = srv.stats()
    srv.close()
    v = np.array(list(lat.values()))
    ks = sorted(iso)
    iv = np.array([iso[k] for k in ks])
    ratio = np.array([lat[k] / iso[k] for k in ks])
    pc = lambda a, q: float(np.percentile(a, q))  # noqa: E731
    return {"requests": n_req, "warmup_requests": n_warm, "rate_hz": rate_hz,
            "p50_ms": pc(v, 50), "p99_ms": pc(v, 99),
            "isolated_p50_ms": pc(iv, 50), "isolated_p99_ms": pc(iv, 99), "isolated_sample": len(ks),
            "served_over_isolated_p50": pc(ratio, 50), "served_over_isolated_p99": pc(ratio, 99),
            "points_per_s": done_points / wall, "completed": int(st.completed), "failed": int(st.failed),
            "plan_builds": int(st.plan_builds), "plan_reuses": int(st.plan_reuses),
            "plan_evictions": int(st.plan_evictions), "merged_jobs": int(st.merged_jobs), "warm_classes_s": t_create,
            "hbm_high_water_GB": st2.hbm_high_water / 1e9, "max_inflight": 8,
            "latency_note": "submit -> result ready, host clock, requests after warm-up; isolated: the same "
                            "jobs one at a time on the warm server"}


def bench_epilogues(LH, W, torch, reps=3):
    """The RPA-side epilogues on the extended-zone workload (512^2 k, 256
    energies, 5x5 zones, orbital form factor, 128 omegas, FP32): Kramers-
    Kronig + contact RPA, Coulomb RPA, S(q, omega), the peak search and the
    q-average, each timed with events on the launch stream against its
    algorithmic HBM bytes; then the cuts (high-symmetry path, zone envelope
    with its fit) and omegas between lag-grid points."""
    cfg = W.config2()
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    im = plan.exec()
    re, imr, rer = plan.empty(), plan.empty(), plan.empty()
    s_out = plan.empty()
    pk = torch.empty(plan.shape[1:], dtype=torch.int32, device="cuda")
    qa = torch.empty(plan.shape[0], dtype=torch.float64, device="cuda")
    h = plan.handle
    sp = lambda: LH._stream_ptr(None)  # noqa: E731
    n_out = im.numel() * 4
    nk = cfg["nkx"] * cfg["nky"]
    first_zone = nk * cfg["neps"] * 4 + 2 * nk * len(cfg["omega"]) * 4  # KK reads all lags, writes Re, RPA re-reads
    steps = {
        "rpa_contact": (lambda: LH.lindhard_rpa(h, W.CONFIG2_U, re.data_ptr(), imr.data_ptr(), rer.data_ptr(), sp()),
                        first_zone + 3 * n_out),
        "rpa_coulomb": (lambda: LH.lindhard_rpa_coulomb(h, 0.5, re.data_ptr(), imr.data_ptr(), rer.data_ptr(), sp()),
                        first_zone + 3 * n_out),
        "structure_factor": (lambda: LH.lindhard_structure_factor(h, 0.025, imr.data_ptr(), s_out.data_ptr(), sp()),
                             2 * n_out),
        "peak_index": (lambda: LH.lindhard_peak_index(h, imr.data_ptr(), pk.data_ptr(), sp()), n_out + pk.numel() * 4),
        "q_average": (lambda: LH.lindhard_q_average(h, im.data_ptr(), qa.data_ptr(), sp()), n_out),
    }
    out = {"workload": "512^2 k, 256 energies, 5x5 zones, d(x2-y2) form factor, 128 omegas, FP32",
           "points": int(im.numel())}
    for name, (fn, nbytes) in steps.items():
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "alg_GB": nbytes / 1e9, "GB/s": nbytes / (ms * 1e-3) / 1e9,
                     "frac_hbm": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    # cuts: the high-symmetry path of every plane (a gather), and the zone
    # envelope with its Lorentzian fit of one plane (synchronous, host clock)
    X, Y = plan.high_symmetry_path()
    cut_out = torch.empty((plan.shape[0], X.size), dtype=im.dtype, device="cuda")
    cut = lambda: LH.lindhard_cut(h, im.data_ptr(), X, Y, cut_out.data_ptr(), sp())  # noqa: E731
    cut()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        cut()
    e1.record()
    torch.cuda.synchronize()
    out["high_symmetry_cut"] = {"ms": e0.elapsed_time(e1) / reps, "points": int(X.size),
                                "note": "includes the host-to-device copy of the path indices"}
    plan.zone_envelope(im, 0, 0, 1.0)
    t0 = time.perf_counter()
    for _ in range(reps):
        env = plan.zone_envelope(im, len(cfg["omega"]) // 2, 0, 1.0 / 7.46)
    out["zone_envelope"] = {"ms_host": (time.perf_counter() - t0) * 1e3 / reps, "k0_au": env["k0"],
                            "segments": int(env["X"].size), "note": "one plane, [100], synchronous call"}
    plan.close()
    # omegas between lag-grid points: the row-transform pass reads two lag
    # slices per output plane and blends them (the other passes are unchanged)
    d = (cfg["emax"] - cfg["emin"]) / cfg["neps"]
    og = {}
    for label, extra in (("on_grid", {}),
                         ("between_lags", dict(omega_interp=True, omega=(np.arange(1, 129) + 0.5) * d))):
        p2 = LH.Plan(precision=LH.LINDHARD_FP32C, **dict(cfg, want_rpa=False, **extra))
        o2 = p2.empty()
        p2.exec_timed(o2)
        runs = [p2.exec_timed(o2) for _ in range(reps)]
        og[label] = {"exec_ms": float(np.mean([sum(r) for r in runs])), "p5_ms": float(np.mean([r[4] for r in runs]))}
        p2.close()
    out["omega_between_lags"] = og
    return out


def bench_extended(LH, W, torch, steps=5):
    """The extended-momentum form on its own instance: a 2048^2 momentum grid
    spanning 16 x 16 zones with the d_{x2-y2} momentum density inside the
    sums, 512 energies, 256 omegas, FP32 (same passes as the main step)."""
    cfg = W.config_extended()
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    out = plan.empty()
    plan.exec_timed(out)
    ms = [sum(plan.exec_timed(out)) for _ in range(steps)]
    pts = cfg["nkx"] * cfg["nky"] * len(cfg["omega"])
    res = {"workload": "2048^2 momentum grid over 16x16 zones, d(x2-y2) momentum density, 512 energies, "
                       "256 omegas, FP32", "ms_per_step": float(np.mean(ms)),
           "points_per_s": pts / (float(np.mean(ms)) * 1e-3), "schedule": plan.info.schedule.decode()}
    plan.close()
    return res


def bench_multiband(LH, W, torch, steps=3):
    """Two bands on the 2048^2 x 512 x 256 FP32 instance: the summed spectral
    function of Eq. (4) (one correlation, the row pass once per band) and the
    band-pair sum of Eq. (2) (four weighted pairs: forward passes once per
    band, then window, column and row inverse passes per pair)."""
    res = {}
    for form, pairs in (("summed", False), ("pairs", True)):
        cfg = W.config_multiband(pairs=pairs)
        plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
        out = plan.empty()
        plan.exec_timed(out)
        ms = [sum(plan.exec_timed(out)) for _ in range(steps)]
        pts = cfg["nkx"] * cfg["nky"] * len(cfg["omega"])
        res[form] = {"ms_per_step": float(np.mean(ms)), "points_per_s": pts / (float(np.mean(ms)) * 1e-3),
                     "bands": 2, "pairs": int(np.count_nonzero(cfg["pair_weight"])) if pairs else 0,
                     "schedule": plan.info.schedule.decode()}
        plan.close()
        del out
    res["workload"] = "two seeded bands, 2048^2 k, 512 energies, 256 omegas, FP32"
    return res


def bench_general(LH, W, torch, cfg, steps=3):
    """The same 2048^2 x 512 x 256 FP32 instance on the general complex path
    (mirror symmetry not used): complex half-plane slices, 52 bytes per chi
    point of algorithmic traffic (55.9 GB per step) against the even path's
    16 (17.2 GB); per-pass times, rates and the roofline of its dominant pass."""
    old = os.environ.get("LINDHARD_SYMMETRY")
    os.environ["LINDHARD_SYMMETRY"] = "off"
    try:
        plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    finally:
        if old is None:
            os.environ.pop("LINDHARD_SYMMETRY", None)
        else:
            os.environ["LINDHARD_SYMMETRY"] = old
    out = plan.empty()
    plan.exec_timed(out)
    runs = np.array([plan.exec_timed(out) for _ in range(steps)])
    pass_avg = runs.mean(axis=0)
    ms = float(pass_avg.sum())
    schedule = plan.info.schedule.decode()
    by, fl_win = algorithmic(cfg, plan.info.lag_hi, False)
    gbs = [b / (t * 1e-3) / 1e9 for b, t in zip(by, pass_avg)]
    fft_window = " P3 fft " in schedule
    names = ["k_p1", "k_col<float, false>", "k_p3f" if fft_window else "k_p3", "k_col<float, true>", "k_p5"]
    dom = int(np.argmax(pass_avg))
    if dom == 2 and not fft_window:
        ach = fl_win / (pass_avg[2] * 1e-3) / 1e12
        roof = {"kernel": names[2], "bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS / 2, "unit": "TFLOP/s",
                "frac": ach / (PEAK_FP32_TFLOPS / 2)}
    else:
        roof = {"kernel": names[dom], "bound": "hbm", "achieved": gbs[dom], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": gbs[dom] / PEAK_HBM_GBS}
    roof["avg_ms"] = float(pass_avg[dom])
    pts = cfg["nkx"] * cfg["nky"] * len(cfg["omega"])
    res = {"workload": "2048^2 k, 512 energies, 256 omegas, FP32, general complex path", "ms_per_step": ms,
           "points_per_s": pts / (ms * 1e-3), "alg_GB_per_step": sum(by) / 1e9,
           "GB/s_per_step": sum(by) / (ms * 1e-3) / 1e9, "frac_hbm_per_step": sum(by) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
           "passes": {n: {"ms": float(t), "alg_GB": b / 1e9, "GB/s": g, "frac_hbm": g / PEAK_HBM_GBS, "kernel": k}
                      for n, t, b, g, k in zip(PASS_NAMES, pass_avg, by, gbs, names)},
           "roofline": roof, "schedule": schedule}
    plan.close()
    return res


def bench_grid_4096(LH, W, torch, steps=3):
    """The largest power-of-two grid: 4096 x 4096 k, 512 energies, 256 omegas,
    FP32 (four times the points of the main instance; the staged slices of the
    energy window span more than 4 GiB)."""
    cfg = W.config3(nk=4096)
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    out = plan.empty()
    plan.exec_timed(out)
    runs = [plan.exec_timed(out) for _ in range(steps)]
    ms = float(np.mean([sum(r) for r in runs]))
    pts = cfg["nkx"] * cfg["nky"] * len(cfg["omega"])
    res = {"workload": "4096^2 k, 512 energies, 256 omegas, FP32", "ms_per_step": ms,
           "points_per_s": pts / (ms * 1e-3), "passes_ms": [float(np.mean([r[i] for r in runs])) for i in range(5)],
           "schedule": plan.info.schedule.decode()}
    plan.close()
    return res


def bench_3d(LH, W, torch, steps=3):
    """Three-dimensional k-grid with as many points as the main instance:
    256 x 256 x 64 k, 512 energies, 256 omegas, FP32 (general complex path
    with the kz transform pass)."""
    cfg = W.config_3d()
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    out = plan.empty()
    plan.exec_timed(out)
    runs = [plan.exec_timed(out) for _ in range(steps)]
    ms = float(np.mean([sum(r) for r in runs]))
    pts = cfg["nkx"] * cfg["nky"] * cfg["nkz"] * len(cfg["omega"])
    res = {"workload": "256x256x64 k (3D), 512 energies, 256 omegas, FP32", "ms_per_step": ms,
           "points_per_s": pts / (ms * 1e-3), "passes_ms": [float(np.mean([r[i] for r in runs])) for i in range(5)],
           "schedule": plan.info.schedule.decode()}
    plan.close()
    return res


def bench_grid_2049(LH, W, torch, steps=2):
    """The paper's own grid size: 2049 x 2049 momenta spanning 16 x 16 zones
    (128 points per zone plus the closing point) with the d(x2-y2) momentum
    density, 512 energies, 256 omegas, FP32 -- a size that is not a power of
    two, so every transform runs as a Bluestein convolution of length 4096
    (the chirp is even, so 2N - 2 points suffice)."""
    cfg = W.config_extended(nk=2049)
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    out = plan.empty()
    plan.exec_timed(out)
    runs = [plan.exec_timed(out) for _ in range(steps)]
    ms = float(np.mean([sum(r) for r in runs]))
    pts = cfg["nkx"] * cfg["nky"] * len(cfg["omega"])
    res = {"workload": "2049^2 momentum grid over 16x16 zones, d(x2-y2) density, 512 energies, 256 omegas, FP32",
           "ms_per_step": ms, "points_per_s": pts / (ms * 1e-3),
           "passes_ms": [float(np.mean([r[i] for r in runs])) for i in range(5)],
           "schedule": plan.info.schedule.decode()}
    plan.close()
    return res


def bench_copy_rates(torch, gib=4, reps=10):
    """Event-timed rates of plain device streams over `gib` GiB of FP32: a fill (writes
    only), a copy (one read and one write per byte moved; both counted) and a sum (reads
    only, torch's reduction).  They are the rates a stream of each kind reaches on this
    memory system, the measure beside which a pass's GB/s is read."""
    n = (gib << 30) // 4
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, fn, nbytes in (("fill", lambda: x.fill_(1.0), 4 * n), ("copy", lambda: y.copy_(x), 8 * n),
                             ("sum", lambda: x.sum(), 4 * n)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        out[name] = {"ms": ms, "bytes": nbytes, "TB/s": nbytes / ms / 1e9}
        print("bench: %s of %d GiB: %.3f ms, %.2f TB/s" % (name, gib, ms, nbytes / ms / 1e9), file=sys.stderr,
              flush=True)
    del x, y
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--nk", type=int, default=2048)
    ap.add_argument("--neps", type=int, default=512)
    ap.add_argument("--window", choices=["auto", "direct", "fft", "even-direct", "even-mfma", "even-mfma4"],
                    default="auto",
                    help="energy-window variant (auto: the plan's own choice; direct / fft: general path; "
                         "even-direct / even-mfma / even-mfma4: even path on the vector ALUs / the matrix cores "
                         "as Toeplitz blocks / as 4x4 rank-1 updates)")
    ap.add_argument("--general", action="store_true",
                    help="force the general complex path even for a mirror-symmetric band")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance batched run")
    ap.add_argument("--no-served", action="store_true", help="skip the served Poisson stream")
    ap.add_argument("--no-epilogues", action="store_true",
                    help="skip the RPA / structure-factor / peak epilogues on the extended-zone workload")
    ap.add_argument("--no-extended", action="store_true",
                    help="skip the extended-momentum instance (16x16 zones, momentum density weights)")
    ap.add_argument("--no-3d", action="store_true", help="skip the three-dimensional k-grid instance")
    ap.add_argument("--no-general", action="store_true",
                    help="skip the same instance on the general complex path (symmetry not used)")
    ap.add_argument("--no-2049", action="store_true", help="skip the 2049^2 (not a power of two) instance")
    ap.add_argument("--no-4096", action="store_true", help="skip the 4096^2 instance")
    ap.add_argument("--no-multiband", action="store_true",
                    help="skip the two-band instances (summed spectral function, band-pair sum)")
    ap.add_argument("--epilogues-only", action="store_true",
                    help="only time the extended-zone epilogues (for profiling them on their own)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--copy-rates", action="store_true",
                    help="only time a plain 4 GiB device fill, copy and sum (the HBM rates plain streams "
                         "reach, beside which the FFT passes are read)")
    args = ap.parse_args()
    if args.general:
        os.environ["LINDHARD_SYMMETRY"] = "off"
    if args.window in ("direct", "fft"):
        os.environ["LINDHARD_WINDOW"] = args.window
    elif args.window.startswith("even-"):
        os.environ["LINDHARD_EVEN_WINDOW"] = args.window[5:]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not supported (got --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1208_3210_amd import lindhard as LH
    from paper_1208_3210_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)
        return
    if args.copy_rates:
        print(json.dumps({"copy_rates": bench_copy_rates(torch)}), flush=True)
        return
    if args.epilogues_only:
        print(json.dumps({"epilogues": bench_epilogues(LH, W, torch)}), flush=True)
        return
    cfg = W.config3(nk=args.nk, neps=args.neps)
    print("bench: planning %dx%d k, %d energies, %d omegas" % (cfg["nkx"], cfg["nky"], cfg["neps"],
                                                             len(cfg["omega"])), file=sys.stderr, flush=True)
    plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
    out = plan.empty()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.exec_timed(out)
    torch.cuda.synchronize()
    step_ms, pass_ms = [], []
    t_start = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        p = plan.exec_timed(out)
        pass_ms.append(p)
        step_ms.append(sum(p))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_start) * 1e3
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    points = cfg["nkx"] * cfg["nky"] * len(cfg["omega"])
    value = points / (ms_per_step * 1e-3)
    pass_avg = np.mean(np.array(pass_ms), axis=0)
    print("bench: %.3f ms/step (wall %.3f), passes %s" % (ms_per_step, wall_ms / args.steps,
                                                        ", ".join("%.3f" % x for x in pass_avg)),
          file=sys.stderr, flush=True)

    schedule = plan.info.schedule.decode()
    even = " even " in schedule
    by, fl_win = algorithmic(cfg, plan.info.lag_hi, even)
    gbs = [b / (t * 1e-3) / 1e9 for b, t in zip(by, pass_avg)]
    dom = int(np.argmax(pass_avg))
    src = [os.path.join(ROOT, "paper_1208_3210_amd", "csrc", f) for f in ("lh_kernels.hip", "lh_fft.h",
                                                                           "lh_regfft.h", "lh_window.hip")]
    khash = src_hash(src)
    fft_window = " P3 fft " in schedule
    mfma_window = " P3 mfma " in schedule
    mfma4_window = " P3 mfma4 " in schedule
    if even:
        KERNEL_NAMES[:] = ["k_e1", "k_ecol<float, false>",
                           "k_e3q" if mfma4_window else "k_e3m" if mfma_window else "k_e3",
                           "k_ecol<float, true>", "k_e5"]
    elif fft_window:
        KERNEL_NAMES[2] = "k_p3f"
    if dom == 2 and not fft_window:
        # algorithmic flops (2 per multiply-add of the window sums) over the
        # event-timed duration; the matrix-core form runs on the FP32 MFMA
        # peak, the direct form on the FP32 vector peak
        ach = fl_win / (pass_avg[2] * 1e-3) / 1e12
        on_mfma = mfma_window or mfma4_window
        roof = {"kernel": KERNEL_NAMES[2], "bound": "mfma" if on_mfma else "alu", "achieved": ach,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
                "traffic": traffic_from_profiles(KERNEL_NAMES[2], khash),
                "count": "useful flops: 2 per multiply-add of the energy sums, %.3g per step" % fl_win}
    else:
        roof = {"kernel": KERNEL_NAMES[dom], "bound": "hbm", "achieved": gbs[dom], "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": gbs[dom] / PEAK_HBM_GBS,
                "traffic": traffic_from_profiles(KERNEL_NAMES[dom], khash)}
    roof["avg_ms"] = float(pass_avg[dom])
    passes = {n: {"ms": float(t), "alg_GB": b / 1e9, "GB/s": g} for n, t, b, g in zip(PASS_NAMES, pass_avg, by, gbs)}
    for n, k in zip(PASS_NAMES, KERNEL_NAMES):
        passes[n]["hbm_traffic_bytes"] = traffic_from_profiles(k, khash)
    passes["p3_window"]["TFLOP/s"] = fl_win / (pass_avg[2] * 1e-3) / 1e12
    if mfma_window:
        # the 16x16 Toeplitz blocks also multiply the zero upper triangle
        pts = (cfg["nkx"] // 2 + 1) * (cfg["nky"] // 2 + 1)
        passes["p3_window"]["mfma_issued_TFLOP/s"] = pts * 16 * 2 * 16 ** 3 / (pass_avg[2] * 1e-3) / 1e12
    if mfma4_window:
        # 4x4 rank-1 blocks, one point each: tile t of 16 lags takes 16 (t + 1)
        # steps, plus the zero-padded ends (T(T-1)/2 partial chunks per group skipped)
        pts = (cfg["nkx"] // 2 + 1) * (cfg["nky"] // 2 + 1)
        nT = (plan.info.lag_hi + 15) // 16
        steps4 = sum(16 * (t + 1) for t in range(nT))
        passes["p3_window"]["mfma_issued_TFLOP/s"] = pts * steps4 * 32 / (pass_avg[2] * 1e-3) / 1e12
    for n, k in zip(PASS_NAMES, KERNEL_NAMES):
        passes[n]["kernel"] = k
    lat = np.array(step_ms)

    # plain FP64 GPU form on the same workload, and the FP32 vs FP64 error
    fp64 = None
    if not args.no_fp64:
        del out
        plan.close()
        plan64 = LH.Plan(precision=LH.LINDHARD_FP64, **cfg)
        o64 = plan64.empty()
        plan64.exec_timed(o64)
        t64 = [sum(plan64.exec_timed(o64)) for _ in range(3)]
        ms64 = float(np.mean(t64))
        plan = LH.Plan(precision=LH.LINDHARD_FP32C, **cfg)
        o32 = plan.exec()
        torch.cuda.synchronize()
        diff = (o32.double() - o64).abs()
        err = diff.max().item() / o64.abs().max().item()
        per_slice = (diff.amax(dim=(1, 2)) / o64.abs().amax(dim=(1, 2))).max().item()
        fp64 = {"ms_per_step": ms64, "value": points / (ms64 * 1e-3), "fp32c_speedup": ms64 / ms_per_step,
                "fp32c_vs_fp64_normwise": err, "fp32c_vs_fp64_worst_slice": per_slice}
        del o64, o32, diff
        plan64.close()
    plan.close()

    batched = None if args.no_batched else bench_batched(LH, W, torch)
    if batched:
        print("bench: batched %.3f ms per 64 instances" % batched["ms_per_batch"], file=sys.stderr, flush=True)
    served = None if args.no_served else bench_served(LH, W, torch)
    if served:
        print("bench: served p50 %.2f ms p99 %.2f ms (isolated p50 %.2f p99 %.2f; served/isolated p50 %.2f "
              "p99 %.2f; %d builds, %d reuses)" % (served["p50_ms"], served["p99_ms"], served["isolated_p50_ms"],
                                                   served["isolated_p99_ms"], served["served_over_isolated_p50"],
                                                   served["served_over_isolated_p99"], served["plan_builds"],
                                                   served["plan_reuses"]), file=sys.stderr, flush=True)
    ext = None if args.no_extended else bench_extended(LH, W, torch)
    if ext:
        print("bench: extended momentum %.3f ms/step" % ext["ms_per_step"], file=sys.stderr, flush=True)
    mb = None if args.no_multiband else bench_multiband(LH, W, torch)
    if mb:
        print("bench: two bands summed %.3f ms, pairs %.3f ms" % (mb["summed"]["ms_per_step"],
                                                                 mb["pairs"]["ms_per_step"]), file=sys.stderr,
              flush=True)
    gen = None if args.no_general else bench_general(LH, W, torch, cfg)
    if gen:
        print("bench: general path %.3f ms/step (%.2f TB/s on its 55.9 GB)" % (gen["ms_per_step"],
                                                                           gen["GB/s_per_step"] / 1e3),
              file=sys.stderr, flush=True)
    k3 = None if args.no_3d else bench_3d(LH, W, torch)
    if k3:
        print("bench: 3d %.3f ms/step" % k3["ms_per_step"], file=sys.stderr, flush=True)
    g2049 = None if args.no_2049 else bench_grid_2049(LH, W, torch)
    if g2049:
        print("bench: 2049^2 grid %.3f ms/step" % g2049["ms_per_step"], file=sys.stderr, flush=True)
    g4096 = None if args.no_4096 else bench_grid_4096(LH, W, torch)
    if g4096:
        print("bench: 4096^2 grid %.3f ms/step" % g4096["ms_per_step"], file=sys.stderr, flush=True)
    epi = None if args.no_epilogues else bench_epilogues(LH, W, torch)
    if epi:
        print("bench: epilogues " + ", ".join("%s %.3f ms" % (k, v["ms"]) for k, v in epi.items()
                                               if isinstance(v, dict) and "ms" in v), file=sys.stderr, flush=True)
    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg)
    res = {
        "metric": "chi(q,w) points/s at 2048^2 k x 512 eps, FP32 vs FP64 at <=1e-5 rel",
        "value": value, "unit": "chi(q,w) points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded t-t'-t'' band, seed 12083210)",
        "config": {"workload": "lindhard_2048x2048k_512eps_256w_fp32c", "nkx": cfg["nkx"], "nky": cfg["nky"],
                   "neps": cfg["neps"], "nomega": len(cfg["omega"]), "gamma_eV": cfg["gamma"],
                   "points_per_step": points, "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "roofline": roof, "passes": passes,
        "traffic_basis": {"even_path_alg_GB_per_step": sum(by) / 1e9 if even else None,
                          "even_path_B_per_point": sum(by) / points if even else None,
                          "general_schedule_alg_GB_per_step": sum(algorithmic(cfg, plan.info.lag_hi, False)[0]) / 1e9,
                          "note": "pass rates use the bytes of the path that ran (the even path stores real quarter "
                                  "planes: 16 B per chi point; the general complex schedule moves 52 B per point)"},
        "general_path": gen, "fp64_gpu": fp64, "batched": batched, "served": served,
        "epilogues": epi, "extended_momentum": ext, "multiband": mb, "k3d": k3, "grid_2049": g2049,
        "grid_4096": g4096,
        "cpu_baseline": cpu,
        "kernel_src_hash": khash, "schedule": schedule,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
