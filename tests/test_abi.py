"""The C ABI: library loads, exports every declared symbol, validates arguments
before touching the device (CPU only; no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2204_13241_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "xs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(xs_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("xs_intensity_direct", "xs_intensity_grad", "xs_g2_rings", "xs_xsvs_contrast"):
        assert required in names
    assert set(names) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.xs_version() >= 100


def _status(rc):
    return rc, _lib.load().xs_last_error().decode()


def test_validation_errors_without_device_work():
    lib = _lib.load()
    rc, msg = _status(lib.xs_intensity_direct(None, None, None, None, 0, None, None, None))
    assert rc == _lib.XS_EINVAL and "NULL" in msg
    # g2: n_tau out of range
    edges = (ctypes.c_double * 3)(0.0, 1.0, 2.0)
    rc, msg = _status(lib.xs_g2_rings(None, 4, 0, None, edges, 2, 0, ctypes.c_void_p(1), None, None))
    assert rc == _lib.XS_EINVAL and "n_tau" in msg
    # non-increasing edges
    bad = (ctypes.c_double * 3)(0.0, 1.0, 1.0)
    rc, msg = _status(lib.xs_g2_rings(None, 4, 0, None, bad, 2, 1, ctypes.c_void_p(1), None, None))
    assert rc == _lib.XS_EINVAL and "increase" in msg
    # too many rings
    many = (ctypes.c_double * 1000)(*range(1000))
    rc, msg = _status(lib.xs_g2_rings(None, 4, 0, None, many, 999, 1, ctypes.c_void_p(1), None, None))
    assert rc == _lib.XS_ENOTSUP
    # xsvs: window longer than the series
    rc, msg = _status(lib.xs_xsvs_contrast(None, 4, 0, None, edges, 2, 4, ctypes.c_void_p(1), None, None))
    assert rc == _lib.XS_EINVAL and "n_levels" in msg
    # roofline probe: unknown kind
    rate = ctypes.c_double(0.0)
    rc, msg = _status(lib.xs_roofline_probe(7, 0, ctypes.byref(rate), None))
    assert rc == _lib.XS_EINVAL and "kind" in msg


def test_batch_validation():
    import numpy as np
    from paper_2204_13241_amd.api import make_batch
    lib = _lib.load()
    b = make_batch([10], [5], [0], 10.0)    # zero frames
    st = b.struct()
    rc, msg = _status(lib.xs_intensity_direct(ctypes.byref(st), None, None, None, 0, None, None, None))
    assert rc == _lib.XS_EINVAL and "n_frames" in msg
    b = make_batch([10], [5], [1], [0.0, 1.0, 1.0])   # bad box for FP32C
    st = b.struct()
    p = ctypes.c_void_p(8)
    rc, msg = _status(lib.xs_intensity_direct(ctypes.byref(st), p, p, p, 1, p, None, None))
    assert rc == _lib.XS_EINVAL and "box" in msg
    rc, msg = _status(lib.xs_intensity_direct(ctypes.byref(st), p, p, p, 7, p, None, None))
    assert rc == _lib.XS_EINVAL and "precision" in msg
    rc, msg = _status(lib.xs_intensity_grad(ctypes.byref(st), p, p, p, p, p, 0, None, None, None))
    assert rc == _lib.XS_EINVAL and "NULL" in msg


def test_tile_shape_roundtrip_and_limits():
    from paper_2204_13241_amd import api
    old = api.get_tile_shape(0)
    api.set_tile_shape(0, 64, 2, 16, 8192, 0)
    assert api.get_tile_shape(0)["q_per_lane"] == 2
    with pytest.raises(_lib.XsError):
        api.set_tile_shape(0, 64, 3, 16, 8192)
    with pytest.raises(_lib.XsError):
        api.set_tile_shape(1, 64, 4, 16, 100)
    # register-bound variants exist only where they are built
    api.set_tile_shape(0, 64, 32, 32, 0, 3)
    assert api.get_tile_shape(0)["waves_per_simd"] == 3
    api.set_tile_shape(0, 64, 8, 64, 0, 3)
    assert api.get_tile_shape(0)["waves_per_simd"] == 3
    for kind, ql, occ in ((0, 4, 3), (1, 8, 3), (1, 32, 3), (1, 32, 5), (0, 32, 4)):
        with pytest.raises(_lib.XsError):
            api.set_tile_shape(kind, 64, ql, 32, 8192, occ)
    old_g = api.get_tile_shape(1)
    api.set_tile_shape(1, 64, 32, 128, 8192, 0)
    assert api.get_tile_shape(1)["q_per_lane"] == 32
    api.set_tile_shape(1, **old_g)
    api.set_tile_shape(0, **old)


def test_plan_validation_without_device_work():
    import numpy as np
    from paper_2204_13241_amd.api import make_batch
    lib = _lib.load()
    out = ctypes.c_void_p()
    p = ctypes.c_void_p(8)
    coef = np.zeros((2, 9))
    cptr = coef.ctypes.data_as(ctypes.c_void_p)
    b = make_batch([10], [5], [1], 10.0)
    st = b.struct()
    rc, msg = _status(lib.xs_plan_create_species(ctypes.byref(st), p, p, 2, cptr, None, None))
    assert rc == _lib.XS_EINVAL and "NULL" in msg
    rc, msg = _status(lib.xs_plan_create_species(ctypes.byref(st), p, p, 0, cptr, ctypes.byref(out), None))
    assert rc == _lib.XS_EINVAL and "n_species" in msg and not out.value
    coef[1, 3] = np.nan
    rc, msg = _status(lib.xs_plan_create_species(ctypes.byref(st), p, p, 2, cptr, ctypes.byref(out), None))
    assert rc == _lib.XS_EINVAL and "finite" in msg
    bad = make_batch([10], [5], [1], [0.0, 1.0, 1.0])
    sb = bad.struct()
    rc, msg = _status(lib.xs_plan_create_species(ctypes.byref(sb), p, p, 2, cptr, ctypes.byref(out), None))
    assert rc == _lib.XS_EINVAL and "box" in msg
    for fn, args in ((lib.xs_plan_intensity_species, (None, p, p, None, None)),
                     (lib.xs_plan_grad_species, (None, p, p, p, 1, p, None, None)),
                     (lib.xs_plan_intensity, (None, p, p, p, None, None))):
        rc, msg = _status(fn(*args))
        assert rc == _lib.XS_EINVAL and "plan is NULL" in msg
    assert lib.xs_plan_destroy(None) == _lib.XS_OK
