"""FP64 CPU oracle for the Lindhard / RPA hot path of arXiv:1208.3210.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
GPU library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the library under
``paper_1208_3210_amd`` never imports it, shares no source with it, and fails
loudly instead of falling back to it.

The heavy double sum over k and energy lives in ``lindhard_oracle.c`` (plain
C, FP64, Neumaier-compensated, OpenMP over q).  The cheap epilogues (orbital
form factor, extended zones, Kramers-Kronig, RPA) are written here in numpy,
each following the passage it cites.

Conventions (the readings the paper leaves open):
  * energy grid is cell centred: e_j = emin + (j + 1/2) d, d = (emax-emin)/Neps;
  * occupied points are e_j <= 0, j < j0;
  * Im chi is per site and per spin with unit-area Lorentzians (Eq. (5)) and
    no extra 1/(2 pi) (Eqs. (2), (A3));
  * lag m stands for omega = m d; m <= 0 or m >= Neps give exactly 0;
  * extended output X maps to h = (X - Zx Nkx/2)/Nkx reciprocal-lattice units
    and to the first-zone index u = (X - Zx Nkx/2) mod Nkx (same for Y).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lindhard_oracle.c")
_SO = os.path.join(_HERE, "liblindhard_oracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP).  Returns the .so path."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            lib.oracle_band_tb.argtypes = [ctypes.c_double] * 3 + [ctypes.c_int, ctypes.c_int, _dp]
            lib.oracle_band_tb.restype = None
            lib.oracle_band_tb_z.argtypes = [ctypes.c_double] * 3 + [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
            lib.oracle_band_tb_z.restype = None
            lib.oracle_filling.argtypes = [_dp, ctypes.c_long, ctypes.c_double, ctypes.c_double]
            lib.oracle_filling.restype = ctypes.c_double
            lib.oracle_mu.argtypes = [_dp, ctypes.c_long, ctypes.c_double, ctypes.c_double]
            lib.oracle_mu.restype = ctypes.c_double
            lib.oracle_j0.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
            lib.oracle_j0.restype = ctypes.c_int
            lib.oracle_chi_grid_w.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int, _ip, _ip, ctypes.c_int, _ip, _dp]
            lib.oracle_chi_grid_w.restype = ctypes.c_int
            lib.oracle_chi_pairs_w.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_long, _ip, _ip, _ip, _dp]
            lib.oracle_chi_pairs_w.restype = ctypes.c_int
            lib.oracle_chi_grid_mb.argtypes = [_dp, _dp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_int, _ip, _ip, ctypes.c_int, _ip, _dp]
            lib.oracle_chi_grid_mb.restype = ctypes.c_int
            lib.oracle_chi_grid_3d.argtypes = [_dp, _dp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int, _ip, _ip, _ip, ctypes.c_int, _ip,
                                               _dp]
            lib.oracle_chi_grid_3d.restype = ctypes.c_int
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


# --------------------------------------------------------------------------
# Band and chemical potential (Sec. 3: single Cu-O band, rigid-band doping)
# --------------------------------------------------------------------------
def band_tb(t: float, tp: float, tpp: float, nkx: int, nky: int, kzones: int = 1) -> np.ndarray:
    """eps(k) of the square-lattice t-t'-t'' band on the periodic k-grid, [iy][ix];
    with kzones > 1 the grid spans kzones Brillouin zones per axis (extended
    momentum p = 2 pi kzones (ix/nkx, iy/nky), Eq. (9))."""
    out = np.empty((nky, nkx), dtype=np.float64)
    if kzones == 1:
        _load().oracle_band_tb(float(t), float(tp), float(tpp), int(nkx), int(nky), _d(out))
    else:
        _load().oracle_band_tb_z(float(t), float(tp), float(tpp), int(nkx), int(nky), int(kzones), _d(out))
    return out


def filling(eps: np.ndarray, gamma: float, mu: float) -> float:
    """Electrons per site (both spins) of the Lorentzian-broadened band (Eq. (5))."""
    e = np.ascontiguousarray(eps, dtype=np.float64).ravel()
    return float(_load().oracle_filling(_d(e), e.size, float(gamma), float(mu)))


def mu_solve(eps: np.ndarray, gamma: float, fill: float) -> float:
    """Rigid-band chemical potential: bisection of n(mu) = fill (Sec. 3)."""
    e = np.ascontiguousarray(eps, dtype=np.float64).ravel()
    return float(_load().oracle_mu(_d(e), e.size, float(gamma), float(fill)))


# --------------------------------------------------------------------------
# Energy grid
# --------------------------------------------------------------------------
def energy_step(neps: int, emin: float, emax: float) -> float:
    return (emax - emin) / neps


def energy_points(neps: int, emin: float, emax: float) -> np.ndarray:
    d = energy_step(neps, emin, emax)
    return emin + (np.arange(neps) + 0.5) * d


def j0(neps: int, emin: float, emax: float) -> int:
    """Number of occupied energy points (e_j <= 0)."""
    return int(_load().oracle_j0(int(neps), float(emin), float(emax)))


# --------------------------------------------------------------------------
# Bare susceptibility, Eqs. (2), (5), (9), (A3)
# --------------------------------------------------------------------------
def _rho(rho, shape):
    if rho is None:
        return None
    r = np.ascontiguousarray(rho, dtype=np.float64)
    assert r.shape == shape
    return r


def chi_grid(xi: np.ndarray, neps: int, emin: float, emax: float, gamma: float,
             qx, qy, ms, rho=None) -> np.ndarray:
    """Im chi_1BZ for every (q in the q-list) x (m in the lag list): shape (nq, nm).
    rho: optional momentum-density weights [iy][ix] on the spectral function
    (A(p, e) = rho(p) A_band(p, e), Eq. (4))."""
    x = np.ascontiguousarray(xi, dtype=np.float64)
    r = _rho(rho, x.shape)
    nky, nkx = x.shape
    qx = np.ascontiguousarray(qx, dtype=np.int32)
    qy = np.ascontiguousarray(qy, dtype=np.int32)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    assert qx.shape == qy.shape
    out = np.empty((qx.size, ms.size), dtype=np.float64)
    rc = _load().oracle_chi_grid_w(_d(x), _d(r) if r is not None else None, nkx, nky, int(neps), float(emin),
                                   float(emax), float(gamma), qx.size, _i(qx), _i(qy), ms.size, _i(ms), _d(out))
    if rc != 0:
        raise RuntimeError("oracle_chi_grid failed: %d" % rc)
    return out


def chi_pairs(xi: np.ndarray, neps: int, emin: float, emax: float, gamma: float,
              qx, qy, ms, rho=None) -> np.ndarray:
    """Im chi_1BZ at explicit samples (qx[i], qy[i], ms[i]); rho as in chi_grid."""
    x = np.ascontiguousarray(xi, dtype=np.float64)
    r = _rho(rho, x.shape)
    nky, nkx = x.shape
    qx = np.ascontiguousarray(qx, dtype=np.int32)
    qy = np.ascontiguousarray(qy, dtype=np.int32)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    assert qx.shape == qy.shape == ms.shape
    out = np.empty(qx.size, dtype=np.float64)
    rc = _load().oracle_chi_pairs_w(_d(x), _d(r) if r is not None else None, nkx, nky, int(neps), float(emin),
                                    float(emax), float(gamma), qx.size, _i(qx), _i(qy), _i(ms), _d(out))
    if rc != 0:
        raise RuntimeError("oracle_chi_pairs failed: %d" % rc)
    return out


def chi_full(xi: np.ndarray, neps: int, emin: float, emax: float, gamma: float, ms, rho=None) -> np.ndarray:
    """Im chi_1BZ on the whole q-grid, natural q order: shape (nm, nky, nkx)."""
    nky, nkx = xi.shape
    qy, qx = np.meshgrid(np.arange(nky), np.arange(nkx), indexing="ij")
    g = chi_grid(xi, neps, emin, emax, gamma, qx.ravel(), qy.ravel(), ms, rho=rho)
    return np.ascontiguousarray(g.T.reshape(len(ms), nky, nkx))


# --------------------------------------------------------------------------
# Orbital form factor and extended zones, Eqs. (2)-(3), Figs. 3-6
# --------------------------------------------------------------------------
def form_factor(Qx, Qy, w: float):
    """On-site matrix element of Eq. (3) for a d_{x2-y2}-like Gaussian orbital.

    With phi(r) = (x^2 - y^2) exp(-r^2 / (2 w^2)) and
    F(Q) = int |phi|^2 e^{iQ.r} / int |phi|^2, the Gaussian moment algebra gives
    F(Q) = exp(-s|Q|^2) [1 - 2 s |Q|^2 + s^2 (Qx^2 - Qy^2)^2] with s = w^2 / 4.
    |M(Q)|^2 = F(Q)^2.
    """
    Qx = np.asarray(Qx, dtype=np.float64)
    Qy = np.asarray(Qy, dtype=np.float64)
    s = w * w / 4.0
    q2 = Qx * Qx + Qy * Qy
    return np.exp(-s * q2) * (1.0 - 2.0 * s * q2 + s * s * (Qx * Qx - Qy * Qy) ** 2)


def zone_axis(n: int, zones: int, kzones: int = 1):
    """For extended index X in [0, zones*n): (h in r.l.u., first-zone index u).

    On a momentum grid spanning kzones Brillouin zones per axis (extended
    momentum p = 2 pi kzones ix / n, Eq. (9)) one grid step is kzones / n
    reciprocal-lattice units, so h = kzones (X - zones n / 2) / n."""
    X = np.arange(zones * n)
    off = X - zones * n // 2
    return kzones * off / n, np.mod(off, n)


def m2_extended(nkx: int, nky: int, zx: int, zy: int, ff_kind: int, w: float, kzones: int = 1) -> np.ndarray:
    """|M(Q)|^2 on the extended output grid [Y][X]; 1 when ff_kind == 0."""
    hx, _ = zone_axis(nkx, zx, kzones)
    hy, _ = zone_axis(nky, zy, kzones)
    if ff_kind == 0:
        return np.ones((zy * nky, zx * nkx))
    Qx = 2.0 * np.pi * hx[None, :]
    Qy = 2.0 * np.pi * hy[:, None]
    return form_factor(Qx, Qy, w) ** 2


def extend(im1bz: np.ndarray, zx: int, zy: int, ff_kind: int, w: float, kzones: int = 1) -> np.ndarray:
    """Extended-zone map out[..., Y, X] = |M(Q)|^2 chi_1BZ[..., v, u], Q = 2 pi (h, l)
    with h, l from ``zone_axis`` (grid step kzones / n r.l.u.)."""
    nky, nkx = im1bz.shape[-2:]
    _, ux = zone_axis(nkx, zx)
    _, uy = zone_axis(nky, zy)
    base = im1bz[..., uy[:, None], ux[None, :]]
    return base * m2_extended(nkx, nky, zx, zy, ff_kind, w, kzones)


# --------------------------------------------------------------------------
# Kramers-Kronig real part (Sec. 4) and RPA (Sec. 4)
# --------------------------------------------------------------------------
def kk_real(im_all: np.ndarray, lags) -> np.ndarray:
    """Re chi at the given lags from Im chi at every lag 0..Neps-1 (last axis).

    Im chi is odd in omega; the principal-value integral
    Re chi(w) = (2/pi) P int_0^inf w' Im chi(w') / (w'^2 - w^2) dw'
    is taken with the alternate-point rule on the lag grid: only lags j with
    j - i odd enter, each with weight 2 d, so
    Re(i) = (2/pi) sum_{j=1..Neps-1, j-i odd} Im(j) 2 j / (j^2 - i^2).
    Im chi is zero beyond the energy window by definition, so there is no tail.
    """
    im_all = np.asarray(im_all, dtype=np.float64)
    neps = im_all.shape[-1]
    lags = np.asarray(lags, dtype=np.int64)
    out = np.zeros(im_all.shape[:-1] + (lags.size,), dtype=np.float64)
    for a, i in enumerate(lags):
        js = np.array([j for j in range(1, neps) if (j - i) % 2 != 0], dtype=np.int64)
        if js.size == 0:
            continue
        wts = (2.0 / np.pi) * 2.0 * js / (js.astype(np.float64) ** 2 - float(i) ** 2)
        out[..., a] = im_all[..., js] @ wts
    return out


def rpa(re_chi, im_chi, U: float):
    """chi_RPA = chi / (1 - U chi) in FP64 complex arithmetic (Sec. 4).

    Returns (Im chi_RPA, Re chi_RPA)."""
    chi = np.asarray(re_chi, dtype=np.float64) + 1j * np.asarray(im_chi, dtype=np.float64)
    r = chi / (1.0 - U * chi)
    return r.imag, r.real


def coulomb_v(hx, hy, v: float, hz: float = 0.0) -> np.ndarray:
    """Coulomb interaction V(Q) = v / |Q|^2 on the extended grid, the form
    the paper gives for the RPA denominator (Sec. 4: V_q decays as 1/q^2),
    with Q = 2 pi (h, l, hz) in units of 1/a (h, l in reciprocal-lattice units,
    see ``zone_axis``; hz that of a kz plane of a three-dimensional grid, the
    lattice constant along z taken as a).  Shape (len(hy), len(hx)); +inf at
    Q = 0."""
    hx = np.asarray(hx, dtype=np.float64)
    hy = np.asarray(hy, dtype=np.float64)
    q2 = (2.0 * np.pi) ** 2 * (hx[None, :] ** 2 + hy[:, None] ** 2 + float(hz) ** 2)
    with np.errstate(divide="ignore"):
        return np.where(q2 > 0.0, v / np.where(q2 > 0.0, q2, 1.0), np.inf)


def rpa_coulomb(re_chi, im_chi, hx, hy, v: float, hz: float = 0.0):
    """chi_RPA = chi / (1 - V(Q) chi) with the Coulomb V of ``coulomb_v``,
    diagonal in G (no local fields), in FP64 complex arithmetic.  Arrays are
    [..., Y, X] on the extended grid (one kz plane, hz, of a 3D grid).  At
    Q = 0 the interaction is infinite and chi_RPA takes its limit, 0.
    Returns (Im chi_RPA, Re chi_RPA)."""
    chi = np.asarray(re_chi, dtype=np.float64) + 1j * np.asarray(im_chi, dtype=np.float64)
    V = coulomb_v(hx, hy, v, hz)
    fin = np.isfinite(V)
    Vf = np.where(fin, V, 0.0)
    r = np.where(fin, chi / (1.0 - Vf * chi), 0.0)
    return r.imag, r.real


def structure_factor(im_chi, omega, kT: float) -> np.ndarray:
    """Dynamical structure factor from Im chi by the fluctuation-dissipation
    relation, Eq. (1): S = -(1/pi) Im chi / (1 - exp(-omega / kT)), omega and
    kT in eV, axis 0 of ``im_chi`` running over ``omega``.  kT = 0 is the
    zero-temperature limit (factor 1 for omega > 0, 0 for omega < 0); at
    omega = 0 the discrete Im chi is exactly 0 and S is set to 0."""
    im = np.asarray(im_chi, dtype=np.float64)
    om = np.asarray(omega, dtype=np.float64).reshape((-1,) + (1,) * (im.ndim - 1))
    if kT > 0.0:
        safe = np.where(om == 0.0, 1.0, om)
        bose = np.where(om == 0.0, 0.0, 1.0 / (-np.expm1(-safe / kT)))
    else:
        bose = np.where(om > 0.0, 1.0, 0.0) + 0.0 * om
    return -(1.0 / np.pi) * im * bose


def peak_index(im_chi) -> np.ndarray:
    """Index along axis 0 of the largest -Im chi (the RPA plasmon peaks,
    Sec. 4), the first one on ties."""
    im = np.asarray(im_chi)
    return np.argmin(im, axis=0).astype(np.int32)


def chi_qmean(xi: np.ndarray, neps: int, emin: float, emax: float, gamma: float, lags, rho=None) -> np.ndarray:
    """q-average of Im chi_1BZ at each lag (the q-integrated joint density of
    states of Fig. 2(b), with the sign of Im chi), computed without any
    q-sum: (1/Nk) sum_q Im chi(q, m) = -d sum_j D_P(j) D_H(j + m), where D is
    the k-averaged spectral weight of Eq. (5) (times rho(k) when momentum
    density weights are given) restricted to the occupied (j < j0) or
    unoccupied points.  O(Nk Neps + Neps Nomega)."""
    d = energy_step(neps, emin, emax)
    e = energy_points(neps, emin, emax)
    x = np.asarray(xi, dtype=np.float64).ravel()
    wt = None if rho is None else np.asarray(rho, dtype=np.float64).ravel()
    D = np.zeros(neps)
    for c in range(0, x.size, 1 << 16):
        xs = x[c:c + (1 << 16), None]
        a = (gamma / np.pi) / ((e[None, :] - xs) ** 2 + gamma * gamma)
        if wt is not None:
            a = a * wt[c:c + (1 << 16), None]
        D += a.sum(axis=0)
    D /= x.size
    occ = e <= 0.0
    DP, DH = np.where(occ, D, 0.0), np.where(~occ, D, 0.0)
    out = []
    for m in np.asarray(lags).ravel():
        m = int(m)
        if m < 1 or m >= neps:
            out.append(0.0)
        else:
            out.append(-d * float(np.dot(DP[:neps - m], DH[m:])))
    return np.array(out)


# --------------------------------------------------------------------------
# Omegas between lag-grid points (a reading: the method computes chi only at
# omega = m d, the energy step of the spectral-function grid)
# --------------------------------------------------------------------------
def omega_lags(omega, neps: int, emin: float, emax: float, interp: bool = False):
    """Lag m and fraction f of each omega, omega = (m + f) d, 0 <= f < 1.

    An omega within 1e-9 d of a grid point is on it (f = 0).  Off the grid
    the omega is rejected (ValueError) unless ``interp``."""
    d = energy_step(neps, emin, emax)
    ms, fs = [], []
    for om in np.asarray(omega, dtype=np.float64).ravel():
        r = om / d
        m = int(np.rint(r))
        if m >= 0 and abs(om - m * d) <= 1e-9 * d:
            ms.append(m)
            fs.append(0.0)
        elif interp and r > 0.0:
            m = int(np.floor(r))
            ms.append(m)
            fs.append(r - m)
        else:
            raise ValueError("omega %r is not on the lag grid" % om)
    return np.array(ms, dtype=np.int64), np.array(fs)


def lag_interp(values, m, f):
    """Value at omega = (m + f) d from values on the lag grid (last axis,
    lags 0 .. Neps-1): the straight line through the two neighbouring grid
    values, (1 - f) V(m) + f V(m + 1), where V is 0 at lag 0 and at lags
    beyond the grid (the discrete Im chi vanishes there)."""
    v = np.asarray(values, dtype=np.float64)
    neps = v.shape[-1]

    def at(k):
        if 1 <= k < neps:
            return v[..., k]
        return np.zeros(v.shape[:-1])

    return np.stack([(1.0 - fi) * at(int(mi)) + fi * at(int(mi) + 1) if fi > 0.0 else at(int(mi))
                     for mi, fi in zip(np.asarray(m).ravel(), np.asarray(f).ravel())], axis=-1)


def kk_real_interp(im_all: np.ndarray, m, f) -> np.ndarray:
    """Re chi at omega = (m + f) d: the straight line through ``kk_real`` at
    lags m and m + 1 (Re chi does not vanish at lag 0 or beyond the grid, so
    both ends come from the Kramers-Kronig sum itself)."""
    m = np.asarray(m, dtype=np.int64).ravel()
    f = np.asarray(f, dtype=np.float64).ravel()
    lo = kk_real(im_all, m)
    hi = kk_real(im_all, m + 1)
    return np.where(f > 0.0, (1.0 - f) * lo + f * hi, lo)


# --------------------------------------------------------------------------
# Cuts through the extended maps (Fig. 2(a) and Fig. 5)
# --------------------------------------------------------------------------
def high_symmetry_path(nk: int, zx: int, zy: int, kzones: int = 1):
    """Extended-grid indices of Gamma -> X -> M -> Gamma in the central zone,
    one point per grid step (the central zone is nk / kzones steps wide;
    indices wrap on a one-zone grid, where the zone boundary is the grid edge)."""
    W = nk // kzones
    nx, ny = zx * nk, zy * nk
    gx, gy = nx // 2, ny // 2
    pts = [(gx + s, gy) for s in range(W // 2)]                       # Gamma -> X
    pts += [(gx + W // 2, gy + s) for s in range(W // 2)]             # X -> M
    pts += [(gx + W // 2 - s, gy + W // 2 - s) for s in range(W // 2 + 1)]  # M -> Gamma
    X = np.array([p[0] % nx for p in pts], dtype=np.int32)
    Y = np.array([p[1] % ny for p in pts], dtype=np.int32)
    return X, Y


def envelope_fit(q, y, ulo: float = 1e-8, uhi: float = 1e8, nscan: int = 200001):
    """Least-squares k0 of y ~ 1 / (1 + (q/k0)^2) (the envelope model of
    Fig. 5): minimise F(u) = sum (y - 1/(1 + q^2 u))^2 over u = 1/k0^2 in
    [ulo, uhi] -- a dense log-spaced scan, then the root of dF/du inside the
    best scan cell (brentq); a minimum at the range end returns that end."""
    from scipy.optimize import brentq
    q = np.asarray(q, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)

    def F(u):
        u = np.asarray(u, dtype=np.float64)
        g = 1.0 / (1.0 + q[:, None] ** 2 * u[None, :])
        return ((y[:, None] - g) ** 2).sum(axis=0)

    def dF(u):
        g = 1.0 / (1.0 + q ** 2 * u)
        return 2.0 * float(np.sum((y - g) * q ** 2 * g * g))

    s = np.linspace(np.log(ulo), np.log(uhi), nscan)
    f = F(np.exp(s))
    i = int(np.argmin(f))
    a, b = s[max(i - 1, 0)], s[min(i + 1, nscan - 1)]
    sx = s[i]
    if dF(np.exp(a)) < 0.0 < dF(np.exp(b)):
        sx = brentq(lambda t: dF(np.exp(t)), a, b, xtol=1e-15, rtol=1e-15, maxiter=500)
    return float(np.exp(-0.5 * sx))


def zone_envelope(plane, nk: int, zx: int, zy: int, direction: int, q_scale: float, kzones: int = 1):
    """Envelope of one extended map ``plane`` [Y][X] of Im chi along [100]
    (direction 0) or [110] (1) from the grid centre: the central half zone and
    every further zone crossed give the point of largest -Im chi (the first
    on ties), normalised by the largest of them, at |q| = |Q| q_scale with
    Q = 2 pi (h, l); then ``envelope_fit``.  Returns a dict (k0, c_max, X, Y,
    q, y)."""
    plane = np.asarray(plane)
    W = nk // kzones
    zones = (zx if direction == 0 else min(zx, zy)) * kzones
    nseg = (zones + 1) // 2
    gx, gy = plane.shape[1] // 2, plane.shape[0] // 2
    Xs, Ys, cs, ss = [], [], [], []
    for k in range(nseg):
        lo = 0 if k == 0 else W // 2 + (k - 1) * W
        hi = W // 2 if k == 0 else lo + W
        best, bs = None, None
        for s in range(lo, hi):
            X, Y = gx + s, (gy + s if direction else gy)
            c = -plane[Y, X]
            if best is None or c > best:
                best, bs = c, s
        Xs.append(gx + bs)
        Ys.append(gy + bs if direction else gy)
        cs.append(float(best))
        ss.append(bs)
    cmax = max(cs)
    y = np.array(cs) / cmax
    step = 2.0 * np.pi / W * (np.sqrt(2.0) if direction else 1.0)
    q = np.array(ss, dtype=np.float64) * step * q_scale
    return {"k0": envelope_fit(q, y), "c_max": cmax, "X": np.array(Xs), "Y": np.array(Ys), "q": q, "y": y}


# --------------------------------------------------------------------------
# Several bands, Eqs. (2) and (4)
# --------------------------------------------------------------------------
def mu_solve_bands(eps_bands: np.ndarray, gamma: float, fill: float) -> float:
    """Common chemical potential of nb bands: electrons per site summed over
    the bands.  ``filling`` normalises by the number of values it is given, so
    on all nb planes at once it returns the per-site count divided by nb."""
    e = np.ascontiguousarray(eps_bands, dtype=np.float64)
    return mu_solve(e.reshape(-1), gamma, fill / e.shape[0])


def chi_grid_mb(xi_bands: np.ndarray, neps: int, emin: float, emax: float, gamma: float, qx, qy, ms,
                rho=None, pair_weight=None) -> np.ndarray:
    """Im chi_1BZ of several bands, xi_bands [band][iy][ix]: with no pair
    weights the spectral function sums the bands (Eq. (4), rho_n on band n);
    with weights w[nu][mu], sum w chi_{nu,mu} (Eq. (2)), band nu occupied and
    band mu empty.  Shape (nq, nm)."""
    x = np.ascontiguousarray(xi_bands, dtype=np.float64)
    nb, nky, nkx = x.shape
    r = None if rho is None else np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(x.shape))
    pw = None if pair_weight is None else np.ascontiguousarray(np.asarray(pair_weight, dtype=np.float64).reshape(nb, nb))
    qx = np.ascontiguousarray(qx, dtype=np.int32)
    qy = np.ascontiguousarray(qy, dtype=np.int32)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    out = np.empty((qx.size, ms.size), dtype=np.float64)
    rc = _load().oracle_chi_grid_mb(_d(x), _d(r) if r is not None else None, nb, _d(pw) if pw is not None else None,
                                    nkx, nky, int(neps), float(emin), float(emax), float(gamma), qx.size, _i(qx),
                                    _i(qy), ms.size, _i(ms), _d(out))
    if rc != 0:
        raise RuntimeError("oracle_chi_grid_mb failed: %d" % rc)
    return out


def chi_full_mb(xi_bands: np.ndarray, neps: int, emin: float, emax: float, gamma: float, ms, rho=None,
                pair_weight=None) -> np.ndarray:
    """``chi_grid_mb`` on the whole q-grid, natural q order: (nm, nky, nkx)."""
    _, nky, nkx = np.asarray(xi_bands).shape
    qy, qx = np.meshgrid(np.arange(nky), np.arange(nkx), indexing="ij")
    g = chi_grid_mb(xi_bands, neps, emin, emax, gamma, qx.ravel(), qy.ravel(), ms, rho, pair_weight)
    return np.moveaxis(g.reshape(nky, nkx, -1), -1, 0)


def chi_pair_maps(xi_bands: np.ndarray, neps: int, emin: float, emax: float, gamma: float, ms, m2,
                  zx: int, zy: int, rho=None) -> np.ndarray:
    """Eq. (2) with a matrix element per band pair that varies with Q (Eq. (3)):
    out[m, Y, X] = sum_{nu,mu} m2[nu, mu, Y, X] chi_{nu,mu}(q, m), where
    chi_{nu,mu} is the first-zone map of the pair alone (band nu occupied,
    band mu empty: ``chi_full_mb`` with the weight 1 on that pair and 0
    elsewhere) and q = (u, v) the first-zone point of the extended point
    (X, Y) (``zone_axis``).  m2 has shape (nb, nb, zy*nky, zx*nkx)."""
    x = np.asarray(xi_bands, dtype=np.float64)
    nb, nky, nkx = x.shape
    m2 = np.asarray(m2, dtype=np.float64).reshape(nb, nb, zy * nky, zx * nkx)
    out = np.zeros((len(np.atleast_1d(ms)), zy * nky, zx * nkx))
    for nu in range(nb):
        for mu in range(nb):
            w = np.zeros((nb, nb))
            w[nu, mu] = 1.0
            pair = chi_full_mb(x, neps, emin, emax, gamma, ms, rho=rho, pair_weight=w)
            out += extend(pair, zx, zy, 0, 0.0) * m2[nu, mu]
    return out


# --------------------------------------------------------------------------
# Three-dimensional k-grids (the d^3p of Eq. (9))
# --------------------------------------------------------------------------
def chi_grid_3d(xi3: np.ndarray, neps: int, emin: float, emax: float, gamma: float, qx, qy, qz, ms,
                rho=None, pair_weight=None) -> np.ndarray:
    """Im chi on a 3D periodic k-grid, xi3 [band][iz][iy][ix] (or [iz][iy][ix]
    for one band), bands as in ``chi_grid_mb``; shape (nq, nm)."""
    x = np.asarray(xi3, dtype=np.float64)
    if x.ndim == 3:
        x = x[None]
    x = np.ascontiguousarray(x)
    nb, nkz, nky, nkx = x.shape
    r = None if rho is None else np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(x.shape))
    pw = None if pair_weight is None else np.ascontiguousarray(np.asarray(pair_weight, dtype=np.float64).reshape(nb, nb))
    qx, qy, qz = (np.ascontiguousarray(a, dtype=np.int32) for a in (qx, qy, qz))
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    out = np.empty((qx.size, ms.size), dtype=np.float64)
    rc = _load().oracle_chi_grid_3d(_d(x), _d(r) if r is not None else None, nb, _d(pw) if pw is not None else None,
                                    nkx, nky, nkz, int(neps), float(emin), float(emax), float(gamma), qx.size,
                                    _i(qx), _i(qy), _i(qz), ms.size, _i(ms), _d(out))
    if rc != 0:
        raise RuntimeError("oracle_chi_grid_3d failed: %d" % rc)
    return out


def chi_full_3d(xi3: np.ndarray, neps: int, emin: float, emax: float, gamma: float, ms, rho=None,
                pair_weight=None) -> np.ndarray:
    """``chi_grid_3d`` on the whole q-grid, natural order: (nm, nkz, nky, nkx)."""
    sh = np.asarray(xi3).shape[-3:]
    qz, qy, qx = np.meshgrid(*(np.arange(n) for n in sh), indexing="ij")
    g = chi_grid_3d(xi3, neps, emin, emax, gamma, qx.ravel(), qy.ravel(), qz.ravel(), ms, rho, pair_weight)
    return np.moveaxis(g.reshape(sh + (-1,)), -1, 0)


def centre_3d(full: np.ndarray) -> np.ndarray:
    """Natural q order -> the output order of the maps: index (q + n/2) mod n
    on each of the last three axes."""
    return np.roll(full, [n // 2 for n in full.shape[-3:]], axis=(-3, -2, -1))
