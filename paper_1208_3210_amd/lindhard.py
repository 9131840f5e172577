"""Python binding of the C ABI in include/lindhard.h (argument marshalling only).

Every step of the computation runs in the gfx950 kernels of liblindhard.so.
PyTorch is used for device memory and streams: outputs are torch tensors on the
GPU and the current torch stream is passed to the library.  If the shared
library is missing this module raises; there is no fallback path.

torch is imported before the library is loaded so that the process holds a
single HIP runtime (the library's libamdhip64 dependency resolves to the one
torch has already loaded).
"""
from __future__ import annotations

import ctypes
import math
import os
import threading
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (must precede the CDLL load, see module docstring)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblindhard.so")

LINDHARD_OK = 0
LINDHARD_EINVAL = -1
LINDHARD_EOFFGRID = -2
LINDHARD_ENOMEM = -3
LINDHARD_ETOOBIG = -4
LINDHARD_EBUSY = -5
LINDHARD_EDEVICE = -6
LINDHARD_ENOCONV = -7
LINDHARD_ECANCELED = -8
LINDHARD_ESTATE = -9

LINDHARD_FP32C = 1
LINDHARD_FP64 = 2
LINDHARD_FF_NONE = 0
LINDHARD_FF_GAUSS_DX2Y2 = 1


class LindhardError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, strerror(status) if _lib_obj else "error", status))


class Problem(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("tp", ctypes.c_double), ("tpp", ctypes.c_double),
        ("eps_table", ctypes.POINTER(ctypes.c_double)),
        ("mu", ctypes.c_double), ("filling", ctypes.c_double), ("gamma", ctypes.c_double),
        ("nkx", ctypes.c_int32), ("nky", ctypes.c_int32),
        ("neps", ctypes.c_int32), ("emin", ctypes.c_double), ("emax", ctypes.c_double),
        ("nomega", ctypes.c_int32), ("omega", ctypes.POINTER(ctypes.c_double)),
        ("zones_x", ctypes.c_int32), ("zones_y", ctypes.c_int32),
        ("ff_kind", ctypes.c_int32), ("ff_width", ctypes.c_double),
        ("precision", ctypes.c_int32), ("want_rpa", ctypes.c_int32),
        ("k_zones", ctypes.c_int32), ("rho_table", ctypes.POINTER(ctypes.c_double)),
        ("omega_interp", ctypes.c_int32),
        ("n_bands", ctypes.c_int32), ("pair_weight", ctypes.POINTER(ctypes.c_double)),
        ("nkz", ctypes.c_int32), ("pair_m2", ctypes.POINTER(ctypes.c_double)),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("mu", ctypes.c_double), ("deps", ctypes.c_double), ("j0", ctypes.c_int32),
        ("out_nx", ctypes.c_int32), ("out_ny", ctypes.c_int32), ("nomega", ctypes.c_int32),
        ("lag_lo", ctypes.c_int32), ("lag_hi", ctypes.c_int32), ("mu_iterations", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_size_t), ("out_elems", ctypes.c_size_t),
        ("elem_bytes", ctypes.c_size_t), ("schedule", ctypes.c_char * 96),
    ]


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("warm", ctypes.POINTER(Problem)), ("n_warm", ctypes.c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
        ("rejected", ctypes.c_uint64), ("canceled", ctypes.c_uint64),
        ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("points_per_s", ctypes.c_double),
        ("hbm_high_water", ctypes.c_size_t), ("queue_depth", ctypes.c_int32), ("inflight", ctypes.c_int32),
        ("plan_reuses", ctypes.c_uint64), ("plan_builds", ctypes.c_uint64), ("plan_evictions", ctypes.c_uint64),
        ("cached_plans", ctypes.c_int32), ("resident_bytes", ctypes.c_size_t), ("merged_jobs", ctypes.c_uint64),
    ]


ENVELOPE_MAX = 64
LINDHARD_MAX_BANDS = 8


class Envelope(ctypes.Structure):
    _fields_ = [
        ("k0", ctypes.c_double), ("c_max", ctypes.c_double), ("nseg", ctypes.c_int32),
        ("X", ctypes.c_int32 * ENVELOPE_MAX), ("Y", ctypes.c_int32 * ENVELOPE_MAX),
        ("q", ctypes.c_double * ENVELOPE_MAX), ("y", ctypes.c_double * ENVELOPE_MAX),
    ]


EXPORTS = [
    "lindhard_plan", "lindhard_plan_info", "lindhard_exec", "lindhard_exec_timed", "lindhard_rpa",
    "lindhard_rpa_coulomb", "lindhard_structure_factor", "lindhard_q_average", "lindhard_q_average_noalloc",
    "lindhard_peak_index",
    "lindhard_cut", "lindhard_high_symmetry_path", "lindhard_zone_envelope", "lindhard_exec_batch",
    "lindhard_problem_shape",
    "lindhard_plan_destroy", "lindhard_serve_create", "lindhard_serve_submit", "lindhard_serve_poll",
    "lindhard_serve_wait", "lindhard_serve_cancel", "lindhard_serve_stats_get", "lindhard_serve_destroy",
    "lindhard_strerror",
]

_lib_obj = None
_lib_lock = threading.Lock()
_vp = ctypes.c_void_p
_st = ctypes.c_int


def lib() -> ctypes.CDLL:
    """Load liblindhard.so (raises if it has not been built)."""
    global _lib_obj
    with _lib_lock:
        if _lib_obj is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("liblindhard.so not found at %s; build it with "
                                   "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            L.lindhard_plan.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(_vp)]
            L.lindhard_plan_info.argtypes = [_vp, ctypes.POINTER(Info)]
            L.lindhard_exec.argtypes = [_vp, _vp, _vp]
            L.lindhard_exec_timed.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_float)]
            L.lindhard_rpa.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp]
            L.lindhard_rpa_coulomb.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp]
            L.lindhard_structure_factor.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp]
            L.lindhard_peak_index.argtypes = [_vp, _vp, _vp, _vp]
            L.lindhard_q_average.argtypes = [_vp, _vp, _vp, _vp]
            L.lindhard_q_average_noalloc.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _vp, _vp]
            L.lindhard_problem_shape.argtypes = [ctypes.POINTER(Problem)] + [ctypes.POINTER(ctypes.c_int32)] * 4
            _i32p = ctypes.POINTER(ctypes.c_int32)
            L.lindhard_cut.argtypes = [_vp, _vp, _i32p, _i32p, ctypes.c_int32, _vp, _vp]
            L.lindhard_high_symmetry_path.argtypes = [_vp, _i32p, _i32p, ctypes.c_int32, _i32p]
            L.lindhard_zone_envelope.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                                 ctypes.POINTER(Envelope), _vp]
            L.lindhard_exec_batch.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(_vp), _vp]
            L.lindhard_plan_destroy.argtypes = [_vp]
            L.lindhard_serve_create.argtypes = [ctypes.POINTER(ServeConfig), ctypes.POINTER(_vp)]
            L.lindhard_serve_submit.argtypes = [_vp, ctypes.POINTER(Problem), ctypes.c_double, _vp, _vp, _vp,
                                                _vp, ctypes.POINTER(ctypes.c_uint64)]
            L.lindhard_serve_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(_st)]
            L.lindhard_serve_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(_st)]
            L.lindhard_serve_cancel.argtypes = [_vp, ctypes.c_uint64]
            L.lindhard_serve_stats_get.argtypes = [_vp, ctypes.POINTER(ServeStats)]
            L.lindhard_serve_destroy.argtypes = [_vp]
            L.lindhard_strerror.argtypes = [_st]
            L.lindhard_strerror.restype = ctypes.c_char_p
            for name in EXPORTS:
                if name != "lindhard_strerror":
                    getattr(L, name).restype = _st
            _lib_obj = L
    return _lib_obj


def strerror(status: int) -> str:
    return lib().lindhard_strerror(int(status)).decode()


def _check(status: int, where: str):
    if status != LINDHARD_OK:
        raise LindhardError(status, where)


def make_problem(*, nkx: int, nky: int, neps: int, emin: float, emax: float, gamma: float,
                 omega: Sequence[float], t: float = 0.0, tp: float = 0.0, tpp: float = 0.0,
                 eps_table: Optional[np.ndarray] = None, mu: float = float("nan"), filling: float = 1.0,
                 zones: tuple = (1, 1), ff_kind: int = LINDHARD_FF_NONE, ff_width: float = 0.0,
                 precision: int = LINDHARD_FP32C, want_rpa: bool = False, k_zones: int = 1,
                 rho_table: Optional[np.ndarray] = None, omega_interp: bool = False, n_bands: int = 1,
                 pair_weight: Optional[np.ndarray] = None, nkz: int = 1, pair_m2: Optional[np.ndarray] = None):
    """Fill a Problem; returns (problem, keepalive) -- keep `keepalive` until the call."""
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
    keep = [om]
    nb = max(1, int(n_bands))
    nk3 = nkx * nky * max(1, int(nkz))
    n_m2 = nb * nb * int(zones[0]) * nkx * int(zones[1]) * nky
    for name, tab, n in (("eps_table", eps_table, nb * nk3), ("rho_table", rho_table, nb * nk3),
                         ("pair_weight", pair_weight, nb * nb), ("pair_m2", pair_m2, n_m2)):
        if tab is not None and np.asarray(tab).size != n:
            raise ValueError("%s holds %d values, %d expected" % (name, np.asarray(tab).size, n))
    p = Problem()
    p.t, p.tp, p.tpp = float(t), float(tp), float(tpp)
    if eps_table is not None:
        tab = np.ascontiguousarray(np.asarray(eps_table, dtype=np.float64))
        keep.append(tab)
        p.eps_table = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.mu, p.filling, p.gamma = float(mu), float(filling), float(gamma)
    p.nkx, p.nky, p.neps = int(nkx), int(nky), int(neps)
    p.emin, p.emax = float(emin), float(emax)
    p.nomega = int(om.size)
    p.omega = om.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.zones_x, p.zones_y = int(zones[0]), int(zones[1])
    p.ff_kind, p.ff_width = int(ff_kind), float(ff_width)
    p.precision, p.want_rpa = int(precision), int(bool(want_rpa))
    p.k_zones = int(k_zones)
    p.omega_interp = int(bool(omega_interp))
    p.n_bands = int(n_bands)
    p.nkz = int(nkz)
    if pair_weight is not None:
        pw = np.ascontiguousarray(np.asarray(pair_weight, dtype=np.float64))
        keep.append(pw)
        p.pair_weight = pw.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if rho_table is not None:
        rt = np.ascontiguousarray(np.asarray(rho_table, dtype=np.float64))
        keep.append(rt)
        p.rho_table = rt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if pair_m2 is not None:
        pm = np.ascontiguousarray(np.asarray(pair_m2, dtype=np.float64))
        keep.append(pm)
        p.pair_m2 = pm.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return p, keep


def lindhard_plan(problem: Problem) -> int:
    h = _vp()
    _check(lib().lindhard_plan(ctypes.byref(problem), ctypes.byref(h)), "lindhard_plan")
    return h.value


def lindhard_plan_info(plan: int) -> Info:
    info = Info()
    _check(lib().lindhard_plan_info(_vp(plan), ctypes.byref(info)), "lindhard_plan_info")
    return info


def lindhard_exec(plan: int, im_chi_ptr: int, stream_ptr: int) -> None:
    _check(lib().lindhard_exec(_vp(plan), _vp(im_chi_ptr), _vp(stream_ptr)), "lindhard_exec")


def lindhard_exec_timed(plan: int, im_chi_ptr: int, stream_ptr: int):
    """Run the hot path once and return the five pass durations (ms)."""
    ms = (ctypes.c_float * 5)()
    _check(lib().lindhard_exec_timed(_vp(plan), _vp(im_chi_ptr), _vp(stream_ptr), ms), "lindhard_exec_timed")
    return [float(x) for x in ms]


def lindhard_rpa(plan: int, U: float, re_ptr: int, imr_ptr: int, rer_ptr: int, stream_ptr: int) -> None:
    _check(lib().lindhard_rpa(_vp(plan), float(U), _vp(re_ptr), _vp(imr_ptr), _vp(rer_ptr), _vp(stream_ptr)),
           "lindhard_rpa")


def lindhard_rpa_coulomb(plan: int, v: float, re_ptr: int, imr_ptr: int, rer_ptr: int, stream_ptr: int) -> None:
    _check(lib().lindhard_rpa_coulomb(_vp(plan), float(v), _vp(re_ptr), _vp(imr_ptr), _vp(rer_ptr),
                                      _vp(stream_ptr)), "lindhard_rpa_coulomb")


def lindhard_structure_factor(plan: int, kT: float, im_ptr: int, s_ptr: int, stream_ptr: int) -> None:
    _check(lib().lindhard_structure_factor(_vp(plan), float(kT), _vp(im_ptr), _vp(s_ptr), _vp(stream_ptr)),
           "lindhard_structure_factor")


def lindhard_q_average(plan: int, im_ptr: int, out_ptr: int, stream_ptr: int) -> None:
    _check(lib().lindhard_q_average(_vp(plan), _vp(im_ptr), _vp(out_ptr), _vp(stream_ptr)), "lindhard_q_average")


NOALLOC_MAX_PLANES = 4096


def lindhard_q_average_noalloc(im_ptr: int, nomega: int, plane_elems: int, elem_bytes: int, out_ptr: int,
                               stream_ptr: int) -> None:
    _check(lib().lindhard_q_average_noalloc(_vp(im_ptr), int(nomega), int(plane_elems), int(elem_bytes),
                                            _vp(out_ptr), _vp(stream_ptr)), "lindhard_q_average_noalloc")


def q_average_noalloc(im: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """Mean of every plane of im ([nomega, ...] float32 or float64, contiguous,
    on the GPU) into the caller's float64 tensor `out` (nomega values), with
    the library's per-device scratch: no device memory is allocated."""
    if not (im.is_cuda and im.is_contiguous() and im.dtype in (torch.float32, torch.float64)):
        raise ValueError("im must be a contiguous float32/float64 GPU tensor")
    if not (out.is_cuda and out.is_contiguous() and out.dtype == torch.float64 and out.numel() == im.shape[0]):
        raise ValueError("out must be a contiguous float64 GPU tensor of im.shape[0] values")
    plane = im.numel() // im.shape[0]
    lindhard_q_average_noalloc(im.data_ptr(), im.shape[0], plane, im.element_size(), out.data_ptr(),
                               _stream_ptr(stream))
    return out


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def lindhard_cut(plan: int, im_ptr: int, X: np.ndarray, Y: np.ndarray, out_ptr: int, stream_ptr: int) -> None:
    X = np.ascontiguousarray(X, dtype=np.int32)
    Y = np.ascontiguousarray(Y, dtype=np.int32)
    if X.shape != Y.shape:
        raise ValueError("X and Y differ in length")
    _check(lib().lindhard_cut(_vp(plan), _vp(im_ptr), _i32(X), _i32(Y), int(X.size), _vp(out_ptr), _vp(stream_ptr)),
           "lindhard_cut")


def lindhard_high_symmetry_path(plan: int):
    n = ctypes.c_int32(0)
    dummy = np.zeros(1, dtype=np.int32)
    st = lib().lindhard_high_symmetry_path(_vp(plan), _i32(dummy), _i32(dummy), 0, ctypes.byref(n))
    if n.value <= 0:
        _check(st, "lindhard_high_symmetry_path")
    X = np.zeros(n.value, dtype=np.int32)
    Y = np.zeros(n.value, dtype=np.int32)
    _check(lib().lindhard_high_symmetry_path(_vp(plan), _i32(X), _i32(Y), n.value, ctypes.byref(n)),
           "lindhard_high_symmetry_path")
    return X, Y


def lindhard_zone_envelope(plan: int, im_ptr: int, omega_index: int, direction: int, q_scale: float,
                           stream_ptr: int) -> Envelope:
    env = Envelope()
    _check(lib().lindhard_zone_envelope(_vp(plan), _vp(im_ptr), int(omega_index), int(direction), float(q_scale),
                                        ctypes.byref(env), _vp(stream_ptr)), "lindhard_zone_envelope")
    return env


def lindhard_peak_index(plan: int, im_ptr: int, peak_ptr: int, stream_ptr: int) -> None:
    _check(lib().lindhard_peak_index(_vp(plan), _vp(im_ptr), _vp(peak_ptr), _vp(stream_ptr)), "lindhard_peak_index")


def lindhard_exec_batch(plans: Sequence[int], outs: Sequence[int], stream_ptr: int) -> None:
    n = len(plans)
    pa = (_vp * n)(*plans)
    oa = (_vp * n)(*outs)
    _check(lib().lindhard_exec_batch(pa, n, oa, _vp(stream_ptr)), "lindhard_exec_batch")


def lindhard_plan_destroy(plan: int) -> None:
    _check(lib().lindhard_plan_destroy(_vp(plan)), "lindhard_plan_destroy")


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dtype(precision: int):
    return torch.float64 if precision == LINDHARD_FP64 else torch.float32


class Plan:
    """One planned susceptibility problem; outputs are torch tensors on the GPU."""

    def __init__(self, **kw):
        self.kw = dict(kw)
        self.problem, keep = make_problem(**kw)
        self.handle = lindhard_plan(self.problem)
        del keep
        self.info = lindhard_plan_info(self.handle)
        self.dtype = _dtype(self.problem.precision)
        self.shape = (self.info.nomega, self.info.out_ny, self.info.out_nx)

    def empty(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=self.dtype, device="cuda")

    def exec(self, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if out is None:
            out = self.empty()
        assert out.is_cuda and out.dtype == self.dtype and tuple(out.shape) == self.shape and out.is_contiguous()
        lindhard_exec(self.handle, out.data_ptr(), _stream_ptr(stream))
        return out

    def exec_timed(self, out: torch.Tensor, stream=None):
        assert out.is_cuda and out.dtype == self.dtype and tuple(out.shape) == self.shape and out.is_contiguous()
        return lindhard_exec_timed(self.handle, out.data_ptr(), _stream_ptr(stream))

    def rpa(self, U: float, stream=None):
        re, imr, rer = self.empty(), self.empty(), self.empty()
        lindhard_rpa(self.handle, U, re.data_ptr(), imr.data_ptr(), rer.data_ptr(), _stream_ptr(stream))
        return re, imr, rer

    def rpa_coulomb(self, v: float, stream=None):
        """RPA with V(Q) = v / |Q|^2 (eV a^2); returns (Re chi, Im chi_RPA, Re chi_RPA)."""
        re, imr, rer = self.empty(), self.empty(), self.empty()
        lindhard_rpa_coulomb(self.handle, v, re.data_ptr(), imr.data_ptr(), rer.data_ptr(), _stream_ptr(stream))
        return re, imr, rer

    def structure_factor(self, im: torch.Tensor, kT: float, out: Optional[torch.Tensor] = None, stream=None):
        """S(q, omega) from an Im chi array of this plan's output layout (Eq. (1))."""
        assert im.is_cuda and im.dtype == self.dtype and tuple(im.shape) == self.shape and im.is_contiguous()
        if out is None:
            out = self.empty()
        assert out.is_cuda and out.dtype == self.dtype and tuple(out.shape) == self.shape and out.is_contiguous()
        lindhard_structure_factor(self.handle, kT, im.data_ptr(), out.data_ptr(), _stream_ptr(stream))
        return out

    def q_average(self, im: torch.Tensor, stream=None) -> torch.Tensor:
        """Mean over the output q grid of every omega plane (FP64, [nomega])."""
        assert im.is_cuda and im.dtype == self.dtype and tuple(im.shape) == self.shape and im.is_contiguous()
        out = torch.empty(self.shape[0], dtype=torch.float64, device="cuda")
        lindhard_q_average(self.handle, im.data_ptr(), out.data_ptr(), _stream_ptr(stream))
        return out

    def peak_index(self, im: torch.Tensor, stream=None) -> torch.Tensor:
        """Index into the omega list of the largest -Im at every extended point (int32 [out_ny, out_nx])."""
        assert im.is_cuda and im.dtype == self.dtype and tuple(im.shape) == self.shape and im.is_contiguous()
        out = torch.empty(self.shape[1:], dtype=torch.int32, device="cuda")
        lindhard_peak_index(self.handle, im.data_ptr(), out.data_ptr(), _stream_ptr(stream))
        return out

    def cut(self, im: torch.Tensor, X, Y, stream=None) -> torch.Tensor:
        """Every omega plane at the extended points (X[p], Y[p]): [nomega, npts]."""
        assert im.is_cuda and im.dtype == self.dtype and tuple(im.shape) == self.shape and im.is_contiguous()
        out = torch.empty((self.shape[0], len(X)), dtype=self.dtype, device="cuda")
        lindhard_cut(self.handle, im.data_ptr(), X, Y, out.data_ptr(), _stream_ptr(stream))
        return out

    def high_symmetry_path(self):
        """(X, Y) of the Gamma -> X -> M -> Gamma path of the central zone."""
        return lindhard_high_symmetry_path(self.handle)

    def zone_envelope(self, im: torch.Tensor, omega_index: int, direction: int = 0, q_scale: float = 1.0,
                      stream=None) -> dict:
        """Per-zone maxima of -Im chi along [100] (0) or [110] (1) from the
        grid centre and the fitted decay momentum k0 of 1/(1 + (q/k0)^2)."""
        assert im.is_cuda and im.dtype == self.dtype and tuple(im.shape) == self.shape and im.is_contiguous()
        e = lindhard_zone_envelope(self.handle, im.data_ptr(), omega_index, direction, q_scale, _stream_ptr(stream))
        n = e.nseg
        return {"k0": e.k0, "c_max": e.c_max, "X": np.array(e.X[:n]), "Y": np.array(e.Y[:n]),
                "q": np.array(e.q[:n]), "y": np.array(e.y[:n])}

    def close(self):
        if getattr(self, "handle", None):
            lindhard_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exec_batch(plans: Sequence[Plan], outs: Optional[Sequence[torch.Tensor]] = None, stream=None):
    if outs is None:
        outs = [p.empty() for p in plans]
    lindhard_exec_batch([p.handle for p in plans], [o.data_ptr() for o in outs], _stream_ptr(stream))
    return outs


def nan() -> float:
    return math.nan


class Server:
    """Continuous-batching server (lindhard_serve_*); outputs are torch tensors."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 4, max_queue: int = 1024, warm=()):
        """warm: problems (keyword dicts as for make_problem, want_rpa set for
        RPA jobs) planned before the first job is taken."""
        made = [make_problem(**w) for w in warm]
        arr = (Problem * max(1, len(made)))(*[m[0] for m in made])
        cfg = ServeConfig(int(hbm_budget_bytes), int(max_inflight), int(max_queue),
                          ctypes.cast(arr, ctypes.POINTER(Problem)) if made else None, len(made))
        h = _vp()
        _check(lib().lindhard_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "lindhard_serve_create")
        del made, arr
        self.handle = h.value
        self._keep = {}

    def submit(self, U: float = float("nan"), **problem):
        """Queue one job; returns (ticket, outputs dict of torch tensors)."""
        kw = dict(problem)
        if math.isfinite(U):
            kw["want_rpa"] = True
        p, keep = make_problem(**kw)
        try:
            info_probe = problem_shape(p)
        except LindhardError:
            # an invalid problem: the server refuses it itself (and counts the
            # refusal) before it touches the output, so a placeholder will do
            info_probe = (1,)
        dtype = _dtype(p.precision)
        outs = {"im_chi": torch.empty(info_probe, dtype=dtype, device="cuda")}
        if math.isfinite(U):
            for k in ("re_chi", "im_rpa", "re_rpa"):
                outs[k] = torch.empty(info_probe, dtype=dtype, device="cuda")
        ptr = lambda k: outs[k].data_ptr() if k in outs else None
        t = ctypes.c_uint64()
        _check(lib().lindhard_serve_submit(_vp(self.handle), ctypes.byref(p), float(U), _vp(ptr("im_chi")),
                                           _vp(ptr("re_chi")), _vp(ptr("im_rpa")), _vp(ptr("re_rpa")),
                                           ctypes.byref(t)), "lindhard_serve_submit")
        self._keep[t.value] = (outs, keep)
        return t.value, outs

    def poll(self, ticket: int):
        done = ctypes.c_int32()
        st = _st()
        _check(lib().lindhard_serve_poll(_vp(self.handle), ctypes.c_uint64(ticket), ctypes.byref(done),
                                         ctypes.byref(st)), "lindhard_serve_poll")
        return bool(done.value), int(st.value)

    def wait(self, ticket: int, timeout_s: float = -1.0) -> int:
        st = _st()
        _check(lib().lindhard_serve_wait(_vp(self.handle), ctypes.c_uint64(ticket), float(timeout_s),
                                         ctypes.byref(st)), "lindhard_serve_wait")
        return int(st.value)

    def cancel(self, ticket: int) -> int:
        return int(lib().lindhard_serve_cancel(_vp(self.handle), ctypes.c_uint64(ticket)))

    def stats(self) -> ServeStats:
        s = ServeStats()
        _check(lib().lindhard_serve_stats_get(_vp(self.handle), ctypes.byref(s)), "lindhard_serve_stats_get")
        return s

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().lindhard_serve_destroy(_vp(self.handle)), "lindhard_serve_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def problem_shape(problem: Problem) -> tuple:
    """(nomega, out_ny, out_nx) of the output arrays of a problem (the library's own answer)."""
    v = [ctypes.c_int32(0) for _ in range(4)]
    _check(lib().lindhard_problem_shape(ctypes.byref(problem), *[ctypes.byref(x) for x in v]), "lindhard_problem_shape")
    return (v[0].value, v[1].value, v[2].value)
