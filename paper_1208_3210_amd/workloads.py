"""Seeded synthetic inputs of the benchmark and parity workloads.

Parameters only: band hoppings, grids, broadenings, fillings and omega lists.
Nothing here evaluates the method.  The paper's NCCO band (KKR-LDA) is
replaced by a square-lattice t-t'-t'' band whose width (-1.48 .. 1.88 eV for
t = 0.42, t' = -0.10, t'' = 0.05 eV) matches the -1.4 .. 1.9 eV Cu-O band of
Sec. 3; random draws use numpy's PCG64 with a fixed seed per workload.
"""
from __future__ import annotations

import numpy as np

BAND1 = dict(t=0.42, tp=-0.10, tpp=0.05)


def lag_omegas(neps: int, emin: float, emax: float, lags) -> np.ndarray:
    """omega = m * d on the cell-centred energy grid of the window."""
    d = (emax - emin) / neps
    return np.asarray(lags, dtype=np.float64) * d


def config1() -> dict:
    """Plain method, FP64: 32x32 k, 64 energies on [-1, 1] eV, G = 0.05 eV,
    32 omegas in (0, 1] eV, first zone only, |M|^2 = 1."""
    neps, emin, emax = 64, -1.0, 1.0
    return dict(**BAND1, filling=1.15, nkx=32, nky=32, neps=neps, emin=emin, emax=emax, gamma=0.05,
                omega=lag_omegas(neps, emin, emax, range(1, 33)), zones=(1, 1), ff_kind=0, ff_width=0.0)


def config2() -> dict:
    """Extended zones + RPA: 512x512 k, 256 energies on [-2, 2] eV, G = 0.03 eV,
    128 omegas in (0, 2] eV, 5x5 zones, Gaussian d_{x2-y2} orbital of width 0.6,
    U = 1.5 eV (passed separately)."""
    neps, emin, emax = 256, -2.0, 2.0
    return dict(**BAND1, filling=1.15, nkx=512, nky=512, neps=neps, emin=emin, emax=emax, gamma=0.03,
                omega=lag_omegas(neps, emin, emax, range(1, 129)), zones=(5, 5), ff_kind=1, ff_width=0.6,
                want_rpa=True)


CONFIG2_U = 1.5


def seeded_band(rng: np.random.Generator) -> dict:
    """t in [0.35, 0.45], t'/t in [-0.35, -0.15], t''/t in [0, 0.2] (eV)."""
    t = rng.uniform(0.35, 0.45)
    return dict(t=t, tp=t * rng.uniform(-0.35, -0.15), tpp=t * rng.uniform(0.0, 0.2))


def config3(nk: int = 2048, neps: int = 512) -> dict:
    """Large single instance: 2048x2048 k, 512 energies on [-2, 2] eV,
    G = 0.01 eV, 256 omegas in (0, 2] eV, seeded band (seed 12083210), filling 1.15."""
    rng = np.random.Generator(np.random.PCG64(12083210))
    emin, emax = -2.0, 2.0
    nlag = neps // 2
    return dict(**seeded_band(rng), filling=1.15, nkx=nk, nky=nk, neps=neps, emin=emin, emax=emax,
                gamma=0.01, omega=lag_omegas(neps, emin, emax, range(1, nlag + 1)), zones=(1, 1), ff_kind=0,
                ff_width=0.0)


def momentum_density_dx2y2(nkx: int, nky: int, k_zones: int, w: float) -> np.ndarray:
    """Synthetic momentum density [iy][ix] of a Gaussian d_{x2-y2}-like orbital
    (x^2 - y^2) exp(-r^2 / (2 w^2)) of width w (lattice constants), standing in
    for the KKR momentum densities the paper uses: |phi(p)|^2 is proportional to
    (px^2 - py^2)^2 exp(-w^2 |p|^2), here normalised to a peak of 1, on the grid
    p = 2 pi k_zones (ix/nkx, iy/nky) taken with folded (mirror-symmetric)
    indices so that the table is exactly even in px and py."""
    ix = np.minimum(np.arange(nkx), nkx - np.arange(nkx))
    iy = np.minimum(np.arange(nky), nky - np.arange(nky))
    px = 2.0 * np.pi * k_zones * ix / nkx
    py = 2.0 * np.pi * k_zones * iy / nky
    PX, PY = np.meshgrid(px, py)
    rho = (PX * PX - PY * PY) ** 2 * np.exp(-w * w * (PX * PX + PY * PY))
    return rho / rho.max()


def multiband_tables(nk: int, nb: int = 2, seed: int = 20121208, k_zones: int = 1):
    """Seeded synthetic bands for the multi-band forms: band n is
    offset_n + sum_{a,b <= 2} c_nab cos(a px) cos(b py) with c_nab uniform in
    [-0.25, 0.25] eV and offsets spread over [-0.3, 0.6] eV, on
    p = 2 pi k_zones (ix, iy)/nk taken with folded indices (exactly mirror
    symmetric).  Returns eps [nb][nk][nk]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    i = np.minimum(np.arange(nk), nk - np.arange(nk))
    p = 2.0 * np.pi * k_zones * i / nk
    eps = np.empty((nb, nk, nk))
    for n in range(nb):
        c = rng.uniform(-0.25, 0.25, size=(3, 3))
        off = -0.3 + 0.9 * n / max(1, nb - 1)
        cx = np.stack([np.cos(a * p) for a in range(3)])  # [a][ix]
        eps[n] = off + np.einsum("ab,by,ax->yx", c, cx, cx)
    return eps


def density_s(nkx: int, nky: int, k_zones: int, w: float) -> np.ndarray:
    """Momentum density of an s-like Gaussian orbital exp(-r^2/(2 w^2)):
    exp(-w^2 |p|^2) on folded indices (exactly mirror symmetric), peak 1."""
    ix = np.minimum(np.arange(nkx), nkx - np.arange(nkx))
    iy = np.minimum(np.arange(nky), nky - np.arange(nky))
    PX, PY = np.meshgrid(2.0 * np.pi * k_zones * ix / nkx, 2.0 * np.pi * k_zones * iy / nky)
    return np.exp(-w * w * (PX * PX + PY * PY))


def config_multiband(nk: int = 2048, neps: int = 512, pairs: bool = True) -> dict:
    """Two-band instance (2048^2 k, 512 energies on [-2, 2] eV, G = 0.01 eV,
    256 omegas, filling 1.15 over both bands): seeded bands of
    ``multiband_tables``; with ``pairs`` the band-pair sum of Eq. (2) with
    weights [[1, 0.5], [0.5, 1]], else the summed spectral function of Eq. (4)."""
    emin, emax = -2.0, 2.0
    cfg = dict(eps_table=multiband_tables(nk, 2), n_bands=2, filling=1.15, nkx=nk, nky=nk, neps=neps, emin=emin,
               emax=emax, gamma=0.01, omega=lag_omegas(neps, emin, emax, range(1, neps // 2 + 1)), zones=(1, 1),
               ff_kind=0, ff_width=0.0)
    if pairs:
        cfg["pair_weight"] = np.array([[1.0, 0.5], [0.5, 1.0]])
    return cfg


def band3d_table(nkx: int, nky: int, nkz: int, seed: int = 1208, tz: float = 0.08) -> np.ndarray:
    """Seeded synthetic three-dimensional band [iz][iy][ix] (eV): an in-plane
    cosine series sum_{a,b <= 2} c_ab cos(a kx) cos(b ky), c_ab uniform in
    [-0.3, 0.3], plus an interlayer term -2 tz cos(kz), and a seeded
    perturbation of 0.02 eV so that no symmetry is exact."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(-0.3, 0.3, size=(3, 3))
    kx = 2.0 * np.pi * np.arange(nkx) / nkx
    ky = 2.0 * np.pi * np.arange(nky) / nky
    kz = 2.0 * np.pi * np.arange(nkz) / nkz
    cx = np.stack([np.cos(a * kx) for a in range(3)])
    cy = np.stack([np.cos(b * ky) for b in range(3)])
    plane = np.einsum("ab,by,ax->yx", c, cy, cx)
    eps = plane[None, :, :] - 2.0 * tz * np.cos(kz)[:, None, None]
    return eps + rng.uniform(-0.02, 0.02, size=eps.shape)


def config_3d(nkx: int = 256, nky: int = 256, nkz: int = 64, neps: int = 512) -> dict:
    """Three-dimensional instance with as many k points as the 2048^2 one:
    256 x 256 x 64 k (``band3d_table``), 512 energies on [-2, 2] eV,
    G = 0.01 eV, 256 omegas, filling 1.15."""
    emin, emax = -2.0, 2.0
    return dict(eps_table=band3d_table(nkx, nky, nkz), nkz=nkz, filling=1.15, nkx=nkx, nky=nky, neps=neps,
                emin=emin, emax=emax, gamma=0.01, omega=lag_omegas(neps, emin, emax, range(1, neps // 2 + 1)),
                zones=(1, 1), ff_kind=0, ff_width=0.0)


def config_extended(nk: int = 2048, k_zones: int = 16, neps: int = 512) -> dict:
    """Extended-momentum instance (the form the paper computes for its
    extended-zone maps): a 2048^2 momentum grid spanning 16 x 16 Brillouin
    zones (128 points per zone), the band of config 1 (filling 1.15), the
    Gaussian d_{x2-y2} momentum density of width 0.6 on the spectral function,
    512 energies on [-2, 2] eV, G = 0.02 eV, 256 omegas in (0, 2] eV."""
    emin, emax = -2.0, 2.0
    return dict(**BAND1, filling=1.15, nkx=nk, nky=nk, neps=neps, emin=emin, emax=emax, gamma=0.02,
                omega=lag_omegas(neps, emin, emax, range(1, neps // 2 + 1)), zones=(1, 1), ff_kind=0,
                ff_width=0.0, k_zones=k_zones, rho_table=momentum_density_dx2y2(nk, nk, k_zones, 0.6))


def config4(n: int = 64, seed: int = 4) -> list:
    """Batched: 64 instances, k-grid uniform over {128,256,512,1024}^2, energies
    over {64,128,256,512} on [-2, 2] eV, doping x in [0, 0.2] (filling 1 + x),
    G in [0.01, 0.08] eV, 64 lags each, band of config 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        nk = int(rng.choice([128, 256, 512, 1024]))
        neps = int(rng.choice([64, 128, 256, 512]))
        x = rng.uniform(0.0, 0.2)
        g = rng.uniform(0.01, 0.08)
        out.append(dict(**BAND1, filling=1.0 + x, nkx=nk, nky=nk, neps=neps, emin=-2.0, emax=2.0, gamma=g,
                        omega=lag_omegas(neps, -2.0, 2.0, range(1, 65)), zones=(1, 1), ff_kind=0,
                        ff_width=0.0))
    return out


def config5(n_req: int = 2200, seed: int = 5, rate_hz: float = 200.0) -> list:
    """Served Poisson stream: exponential inter-arrival times of mean 1/rate,
    k-grid over {128..1024}^2, energies over {64..512}, 16..128 omegas, band
    and doping as config 3, RPA with probability 1/2 and U in [0, 2] eV."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    jobs = []
    for _ in range(n_req):
        t += rng.exponential(1.0 / rate_hz)
        nk = int(rng.choice([128, 256, 512, 1024]))
        neps = int(rng.choice([64, 128, 256, 512]))
        nw = int(rng.integers(16, 129))
        band = seeded_band(rng)
        x = rng.uniform(0.0, 0.2)
        rpa = bool(rng.uniform() < 0.5)
        U = float(rng.uniform(0.0, 2.0)) if rpa else float("nan")
        jobs.append(dict(arrival_s=t, U=U,
                         problem=dict(**band, filling=1.0 + x, nkx=nk, nky=nk, neps=neps, emin=-2.0, emax=2.0,
                                      gamma=float(rng.uniform(0.01, 0.08)),
                                      omega=lag_omegas(neps, -2.0, 2.0, range(1, nw + 1)), zones=(1, 1),
                                      ff_kind=0, ff_width=0.0, want_rpa=rpa)))
    return jobs
