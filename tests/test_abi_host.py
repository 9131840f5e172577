"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/lindhard.h, and rejects invalid problems
during validation (before any device call)."""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBPATH = os.path.join(ROOT, "paper_1208_3210_amd", "liblindhard.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIBPATH), reason="liblindhard.so not built")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lindhard.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lindhard_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_function():
    from paper_1208_3210_amd import lindhard as LH

    lib = LH.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(LH.EXPORTS)


def test_strerror_covers_every_status():
    from paper_1208_3210_amd import lindhard as LH

    for s in range(0, -10, -1):
        assert LH.strerror(s) != "unknown status"
    assert LH.strerror(-99) == "unknown status"


def _base(**over):
    kw = dict(t=0.42, tp=-0.1, tpp=0.05, filling=1.15, nkx=32, nky=32, neps=64, emin=-1.0, emax=1.0,
              gamma=0.05, omega=np.arange(1, 33) / 32.0, precision=2)
    kw.update(over)
    return kw


@pytest.mark.parametrize("over,status", [
    (dict(nkx=48, zones=(2, 1)), -1), (dict(nkx=2050), -1), (dict(nkx=3), -1), (dict(nky=2), -1),
    (dict(nkx=8192), -1), (dict(nky=8192), -1), (dict(nkx=48, nkz=2), -1), (dict(neps=100), -1),
    (dict(neps=2), -1), (dict(omega=np.arange(65536) / 32.0 % 1.0), -1),
    (dict(nky=4096, zones=(1, 17)), -1),
    (dict(emin=0.1), -1), (dict(emax=-0.1), -1), (dict(gamma=0.0), -1), (dict(gamma=math.nan), -1),
    (dict(precision=3), -1), (dict(zones=(2, 1)), -1), (dict(zones=(1, 0)), -1), (dict(ff_kind=7), -1),
    (dict(ff_kind=1, ff_width=0.0), -1), (dict(filling=2.5), -1), (dict(mu=math.inf), -1),
    (dict(t=math.nan), -1), (dict(omega=[]), -1),
    (dict(omega=[1.5 / 32.0]), -2), (dict(omega=[-1.0 / 32.0]), -2), (dict(omega=[math.nan]), -2),
    (dict(omega=[1.0 / 32.0 + 1e-6]), -2),
])
def test_validation_rejects(over, status):
    from paper_1208_3210_amd import lindhard as LH

    p, keep = LH.make_problem(**_base(**over))
    with pytest.raises(LH.LindhardError) as ei:
        LH.lindhard_plan(p)
    assert ei.value.status == status


def test_validation_rejects_nonfinite_table():
    from paper_1208_3210_amd import lindhard as LH

    tab = np.zeros((32, 32))
    tab[3, 4] = math.inf
    p, keep = LH.make_problem(**_base(eps_table=tab, mu=0.0))
    with pytest.raises(LH.LindhardError) as ei:
        LH.lindhard_plan(p)
    assert ei.value.status == -1


def test_null_handles_are_rejected():
    import ctypes

    from paper_1208_3210_amd import lindhard as LH

    L = LH.lib()
    assert L.lindhard_exec(None, None, None) == -1
    assert L.lindhard_rpa(None, 1.0, None, None, None, None) == -1
    assert L.lindhard_rpa_coulomb(None, 1.0, None, None, None, None) == -1
    assert L.lindhard_structure_factor(None, 0.01, None, None, None) == -1
    assert L.lindhard_peak_index(None, None, None, None) == -1
    assert L.lindhard_q_average(None, None, None, None) == -1
    assert L.lindhard_cut(None, None, None, None, 1, None, None) == -1
    n = ctypes.c_int32(0)
    assert L.lindhard_high_symmetry_path(None, None, None, 0, ctypes.byref(n)) == -1
    assert L.lindhard_zone_envelope(None, None, 0, 0, 1.0, None, None) == -1
    assert L.lindhard_problem_shape(None, None, None, None, None) == -1
    assert L.lindhard_plan_destroy(None) == -1
    assert L.lindhard_plan_info(None, None) == -1
    assert L.lindhard_serve_create(None, ctypes.byref(ctypes.c_void_p())) == -1
    assert L.lindhard_serve_destroy(None) == -1


def test_problem_shape_is_host_only():
    """The output shape of a problem comes from the library without a device:
    extended zones, a 3D grid (nkz blocks of rows), a grid of any size."""
    from paper_1208_3210_amd import lindhard as LH

    p, keep = LH.make_problem(**_base(zones=(3, 5)))
    assert LH.problem_shape(p) == (32, 5 * 32, 3 * 32)
    tab = np.zeros((4, 8, 16))
    p, keep = LH.make_problem(**_base(nkx=16, nky=8, nkz=4, eps_table=tab))
    assert LH.problem_shape(p) == (32, 4 * 8, 16)
    p, keep = LH.make_problem(**_base(nkx=33, nky=17, eps_table=np.zeros((17, 33))))
    assert LH.problem_shape(p) == (32, 17, 33)
    p, keep = LH.make_problem(**_base(zones=(2, 1)))
    with pytest.raises(LH.LindhardError):
        LH.problem_shape(p)


@pytest.mark.parametrize("over", [
    dict(n_bands=2),                                                   # several bands need a table
    dict(n_bands=2, eps_table=np.zeros((2, 32, 32)), pair_weight=np.zeros((2, 2))),
    dict(n_bands=2, eps_table=np.zeros((2, 32, 32)), pair_weight=-np.ones((2, 2))),
    dict(n_bands=9, eps_table=np.zeros((9, 32, 32))),
    dict(nkz=3, eps_table=np.zeros((3, 32, 32))),                      # kz count not a power of two
    dict(nkz=4, eps_table=np.zeros((4, 32, 32)), k_zones=2),           # 3D: first-zone k-grid
    dict(nkz=4, eps_table=np.zeros((4, 32, 32)), pair_m2=np.ones((1, 1, 32, 32))),
    dict(nkx=33, eps_table=np.zeros((2, 32, 33)), n_bands=2),            # any size: one band
    dict(nkx=2050, eps_table=np.zeros((32, 2050))),                    # FP64 any size up to 2049
    dict(omega=[1.5 / 32.0], omega_interp=False),
    dict(omega=[-1.0 / 32.0], omega_interp=True),
])
def test_widened_forms_validated_on_the_host(over):
    """The several-band, 3D, any-size and off-grid rules are checked before any
    device work (the output-shape query runs the same validation)."""
    from paper_1208_3210_amd import lindhard as LH

    p, keep = LH.make_problem(**_base(**over))
    with pytest.raises(LH.LindhardError) as ei:
        LH.problem_shape(p)
    assert ei.value.status in (-1, -2)


def test_3d_extended_shapes_on_the_host():
    """A 3D grid with in-plane zones reports nkz blocks of zones_y * nky rows."""
    from paper_1208_3210_amd import lindhard as LH

    p, keep = LH.make_problem(**_base(nkz=4, eps_table=np.zeros((4, 32, 32)), zones=(3, 5), ff_kind=1,
                                      ff_width=0.6, want_rpa=True))
    assert LH.problem_shape(p) == (32, 4 * 5 * 32, 3 * 32)


def test_offgrid_omega_accepted_with_interp_on_the_host():
    from paper_1208_3210_amd import lindhard as LH

    p, keep = LH.make_problem(**_base(omega=[1.5 / 32.0, 2.0 / 32.0], omega_interp=True))
    assert LH.problem_shape(p) == (2, 32, 32)


def test_shape_limits_match_the_header():
    """Powers of two up to 4096 per axis, up to 65535 omegas, zones_y * nky
    up to 65535 (host-side validation through lindhard_problem_shape)."""
    import ctypes

    from paper_1208_3210_amd import lindhard as LH

    def shape(**over):
        p, keep = LH.make_problem(**_base(**over))
        v = [ctypes.c_int32() for _ in range(4)]
        st = LH.lib().lindhard_problem_shape(ctypes.byref(p), *[ctypes.byref(x) for x in v])
        return st, tuple(x.value for x in v)

    assert shape(nkx=4096, nky=4096) == (0, (32, 4096, 4096, 8))
    assert shape(nkx=4096, nky=4096, precision=1) == (0, (32, 4096, 4096, 4))
    assert shape(nkx=8192)[0] == -1
    assert shape(omega=np.arange(65535) % 32 / 32.0)[0] == 0
    assert shape(nky=4096, zones=(1, 15))[0] == 0
    assert shape(nkx=4096, zones=(15, 1)) == (0, (32, 32, 15 * 4096, 8))


def test_pair_maps_validated_on_the_host():
    """Band-pair |M(Q)|^2 maps: accepted on their own (the output shape is the
    extended grid's), refused with pair weights, the analytic form factor,
    RPA, a 3D grid, a grid of any size, or a negative or non-finite value."""
    from paper_1208_3210_amd import lindhard as LH

    tab = np.zeros((2, 32, 32))
    m2 = np.ones((2, 2, 32, 3 * 32))
    ok = dict(eps_table=tab, n_bands=2, zones=(3, 1), pair_m2=m2)
    p, keep = LH.make_problem(**_base(**ok))
    assert LH.problem_shape(p) == (32, 32, 96)
    bad = [dict(pair_weight=np.ones((2, 2))), dict(ff_kind=1, ff_width=0.6), dict(want_rpa=True),
           dict(pair_m2=-m2), dict(pair_m2=np.where(np.arange(m2.size).reshape(m2.shape) == 7, np.inf, m2))]
    for b in bad:
        p, keep = LH.make_problem(**_base(**dict(ok, **b)))
        with pytest.raises(LH.LindhardError) as ei:
            LH.problem_shape(p)
        assert ei.value.status == -1
    p, keep = LH.make_problem(**_base(eps_table=np.zeros((4, 32, 32)), nkz=4, pair_m2=np.ones((1, 1, 32, 32))))
    with pytest.raises(LH.LindhardError):
        LH.problem_shape(p)
    p, keep = LH.make_problem(**_base(nkx=33, eps_table=np.zeros((32, 33)), pair_m2=np.ones((1, 1, 32, 33))))
    with pytest.raises(LH.LindhardError):
        LH.problem_shape(p)
