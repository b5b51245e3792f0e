"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
validates arguments with the documented error codes before touching a device.

No compute call is made here (there is no GPU on this host)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT, has_gpu

import paper_2004_05962_amd as bsi
from paper_2004_05962_amd import _lib

HEADER = os.path.join(ROOT, "include", "bsi.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bsi_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 19
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_version_and_error_string():
    assert bsi.bsi_version() == 10000
    assert isinstance(bsi.bsi_last_error(), str)


@pytest.mark.parametrize("dims,spacing,expect", [
    ((64, 64, 64), (5, 5, 5), (16, 16, 16)),
    ((512, 512, 256), (3, 3, 3), (174, 174, 89)),
    ((512, 512, 256), (5, 5, 5), (106, 106, 55)),
    ((512, 512, 256), (8, 8, 8), (67, 67, 35)),
    ((256, 256, 160), (5, 5, 5), (55, 55, 35)),
    ((12, 12, 12), (5, 5, 5), (6, 6, 6)),
    ((1, 1, 1), (64, 64, 64), (4, 4, 4)),
])
def test_grid_dims(dims, spacing, expect):
    assert bsi.bsi_grid_dims(dims, spacing) == expect


@pytest.mark.parametrize("dims,spacing,code", [
    ((0, 4, 4), (1, 1, 1), _lib.BSI_ERR_INVALID_ARG),
    ((4, -1, 4), (1, 1, 1), _lib.BSI_ERR_INVALID_ARG),
    ((4, 4, 4), (1, 0, 1), _lib.BSI_ERR_INVALID_ARG),
    ((4, 4, 4), (1, 1, 65), _lib.BSI_ERR_UNSUPPORTED),
    ((1 << 21, 4, 4), (1, 1, 1), _lib.BSI_ERR_UNSUPPORTED),
    ((1 << 20, 1 << 11, 1), (1, 1, 1), _lib.BSI_ERR_UNSUPPORTED),   # a voxel plane of 2^32 * 3/2 floats
])
def test_bad_geometry(dims, spacing, code):
    with pytest.raises(bsi.BSIError) as e:
        bsi.bsi_grid_dims(dims, spacing)
    assert e.value.code == code
    assert bsi.bsi_last_error()


def _call(name, *args):
    return getattr(_lib.lib(), name)(*args)


def _t(v):
    return _lib._triple(v, "t")


P = ctypes.c_void_p(256)  # a non-null placeholder; never dereferenced by the checks below
NULL = ctypes.c_void_p(0)


def test_null_pointers_rejected_before_device():
    d, s = _t((8, 8, 8)), _t((2, 2, 2))
    assert _call("bsi_forward", NULL, d, s, P, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_forward", P, d, s, NULL, NULL) == _lib.BSI_ERR_INVALID_ARG
    for name in ("bsi_forward_lerp", "bsi_forward_scalar"):
        assert _call(name, NULL, d, s, P, NULL) == _lib.BSI_ERR_INVALID_ARG
        assert _call(name, P, d, s, NULL, NULL) == _lib.BSI_ERR_INVALID_ARG
        assert _call(name, P, d, _t((0, 1, 1)), P, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_adjoint", P, d, s, P, NULL, 1 << 30, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_adjoint_partials", NULL, d, s, P, 1 << 30, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_adjoint_partials", P, d, s, NULL, 1 << 30, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_adjoint_reduce", P, 1 << 30, d, s, NULL, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_adjoint_reduce", NULL, 1 << 30, d, s, P, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_warp", NULL, P, d, P, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_ssd_grad", P, P, P, d, P, NULL, P, 1 << 30, NULL) == _lib.BSI_ERR_INVALID_ARG
    for k in range(6):
        args = [P, P, P, d, s, P, P, P, 1 << 30, NULL]
        args[[0, 1, 2, 5, 6, 7][k]] = NULL
        assert _call("bsi_ssd_fused", *args) == _lib.BSI_ERR_INVALID_ARG
    for k in range(6):
        args = [P, P, P, d, s, ctypes.c_float(0.5), P, P, P, 1 << 30, NULL]
        args[[0, 1, 2, 6, 7, 8][k]] = NULL
        assert _call("bsi_ssd_fused_descent", *args) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_ssd_fused_descent", P, P, P, d, s, ctypes.c_float(float("inf")), P, P, P, 1 << 30,
                 NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_descent_step", NULL, P, ctypes.c_float(1.0), 4, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_descent_step", P, P, ctypes.c_float(1.0), -1, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert "non-null" in bsi.bsi_last_error() or "count" in bsi.bsi_last_error()


def test_workspace_size_checked_before_device():
    d, s = _t((40, 30, 20)), _t((5, 5, 5))
    need = bsi.bsi_adjoint_workspace_size((40, 30, 20), (5, 5, 5))
    assert need > 0
    assert _call("bsi_adjoint", P, d, s, P, P, need - 1, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert "workspace too small" in bsi.bsi_last_error()
    assert _call("bsi_adjoint_partials", P, d, s, P, need - 1, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_adjoint_reduce", P, need - 1, d, s, P, NULL) == _lib.BSI_ERR_INVALID_ARG
    fused = bsi.bsi_ssd_fused_workspace_size((40, 30, 20), (5, 5, 5))
    assert fused > 0
    assert _call("bsi_ssd_fused", P, P, P, d, s, P, P, P, fused - 1, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_ssd_fused_descent", P, P, P, d, s, ctypes.c_float(0.5), P, P, P, fused - 1,
                 NULL) == _lib.BSI_ERR_INVALID_ARG
    ssd = bsi.bsi_ssd_workspace_size((40, 30, 20))
    assert _call("bsi_ssd_grad", P, P, P, d, P, P, P, ssd - 1, NULL) == _lib.BSI_ERR_INVALID_ARG


def test_batch_argument_checks():
    plan = ctypes.c_void_p()
    n = ctypes.c_int32 * 3
    assert _call("bsi_batch_create", 0, n(4, 4, 4), n(1, 1, 1), ctypes.byref(plan)) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_batch_create", 1, n(0, 4, 4), n(1, 1, 1), ctypes.byref(plan)) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_batch_run", NULL, NULL) == _lib.BSI_ERR_INVALID_ARG
    assert _call("bsi_batch_launch", NULL, NULL) == _lib.BSI_ERR_INVALID_ARG
    buf = ctypes.create_string_buffer(16)
    assert _call("bsi_batch_describe", NULL, buf, 16) == _lib.BSI_ERR_INVALID_ARG
    _call("bsi_batch_destroy", NULL)  # NULL is ignored


@pytest.mark.skipif(has_gpu(), reason="checks the no-device path")
def test_no_device_reported():
    d, s = _t((8, 8, 8)), _t((2, 2, 2))
    assert _call("bsi_forward", P, d, s, P, NULL) == _lib.BSI_ERR_NO_DEVICE
    assert "no HIP device" in bsi.bsi_last_error()
    plan = ctypes.c_void_p()
    assert _call("bsi_batch_create", 1, d, s, ctypes.byref(plan)) == _lib.BSI_ERR_NO_DEVICE


def test_workspace_sizes_follow_brick_geometry():
    # the adjoint's partials cost a few % of the dfield at the benchmark sizes
    for dims, sp in (((512, 512, 256), (5, 5, 5)), ((256, 256, 256), (5, 5, 5)), ((512, 512, 256), (8, 8, 8))):
        field_bytes = 12 * dims[0] * dims[1] * dims[2]
        assert bsi.bsi_adjoint_workspace_size(dims, sp) < 0.06 * field_bytes


def test_every_export_has_a_package_binding():
    """Each C entry point is callable from the package under the same name."""
    missing = [n for n in _lib.EXPORTS if not callable(getattr(bsi, n, None))]
    assert not missing, missing


@pytest.mark.parametrize("dims,spacing", [((40000, 20000, 1), (1, 1, 1)), ((30000, 30000, 2), (1, 1, 1))])
def test_oversized_control_plane_rejected(dims, spacing):
    # a voxel plane under 2^32 floats whose control plane (gx * gy * 3 floats)
    # reaches 2^31: the kernels' signed 32-bit staging offsets would wrap
    with pytest.raises(bsi.BSIError) as e:
        bsi.bsi_grid_dims(dims, spacing)
    assert e.value.code == _lib.BSI_ERR_UNSUPPORTED
    with pytest.raises(bsi.BSIError) as e:
        bsi.bsi_general_grid_dims(dims, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    assert e.value.code == _lib.BSI_ERR_UNSUPPORTED


def test_batch_bind_checks_list_length_before_the_library():
    # a plan's geometry is known to the binding; a short list raises before any
    # pointer reaches the library (no device is needed for this check)
    fake = ctypes.c_void_p(0x1000)
    _lib._PLANS[fake.value] = ([(8, 8, 8), (9, 9, 9)], [(2, 2, 2), (3, 3, 3)])
    try:
        with pytest.raises(ValueError, match="2 volumes"):
            _lib.bsi_batch_bind(fake, grids=[None], fields=[None])
    finally:
        _lib._PLANS.pop(fake.value)
    with pytest.raises(ValueError, match="live batched plan"):
        _lib.bsi_batch_bind(ctypes.c_void_p(0x2000), grids=[], fields=[])


def test_general_window_start_is_the_exact_floor():
    # The library decides floor((x - o)/s) with FP32 error-free arithmetic (the
    # same routine on host and device); g = floor((n - 1 - o)/s) + 4 exercises it
    # on the host.  Checked against exact rationals: random geometries, quotients
    # that are exact integers, and origins far below one ulp of x.
    from oracle import general
    rng = np.random.default_rng(17)
    cases = []
    for _ in range(400):
        s = float(np.float32(rng.uniform(1.0, 64.0)))
        o = float(np.float32(-rng.uniform(0.0, 1.0) * s * 0.999999))
        n = int(rng.integers(1, 1 << 20))
        cases.append((n, s, o))
    for k in range(1, 40):
        cases += [(int(1.5 * (2 * k - 1) + 1.5), 1.5, -0.5), (2 * k + 1, 2.0, 0.0), (3 * k + 1, 3.0, -1e-30),
                  (5 * k + 1, 5.0, -np.float32(2.0) ** -40)]
    for n, s, o in cases:
        got = bsi.bsi_general_grid_dims((n, 1, 1), (s, 1.0, 1.0), (o, 0.0, 0.0))[0]
        assert got == general.grid_dims((n, 1, 1), (s, 1.0, 1.0), (o, 0.0, 0.0))[0], (n, s, o)


def test_noalloc_rejects_geometry_beyond_its_scratch_before_device():
    """bsi_adjoint_noalloc checks the partials' size against its fixed scratch
    (BSI_ADJOINT_NOALLOC_MAX_BYTES) on the host, before any device call."""
    text = open(HEADER).read()
    m = re.search(r"#define BSI_ADJOINT_NOALLOC_MAX_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "the header states the scratch size"
    cap = int(m.group(1)) << int(m.group(2))
    assert cap == _lib.BSI_ADJOINT_NOALLOC_MAX_BYTES
    P = ctypes.c_void_p(16)  # never dereferenced: rejected before any device use
    big = (512, 512, 256), (2, 2, 2)
    assert bsi.bsi_adjoint_workspace_size(*big) > cap
    rc = _call("bsi_adjoint_noalloc", P, _t(big[0]), _t(big[1]), P, NULL)
    assert rc == _lib.BSI_ERR_UNSUPPORTED
    assert "scratch" in bsi.bsi_last_error()
    # the benchmark geometry fits
    assert bsi.bsi_adjoint_workspace_size((512, 512, 256), (5, 5, 5)) <= cap
    assert _call("bsi_adjoint_noalloc", NULL, _t((8, 8, 8)), _t((2, 2, 2)), P, NULL) == _lib.BSI_ERR_INVALID_ARG
