"""ctypes binding of libbsi (include/bsi.h): argument marshalling only.

Each function has the name of the C entry point it calls.  Buffers are torch
tensors on the current HIP device; their checks (dtype, device, contiguity,
shape) happen here, the arithmetic in the library.  Every call is enqueued on
``stream`` (default: torch's current stream) and returns without synchronising.
A non-zero return code raises ``BSIError`` with the library's message.

The library must be built in-tree (``paper_2004_05962_amd/libbsi.so``); there is
no fallback: without it every call raises.
"""
import ctypes
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbsi.so")

BSI_OK = 0
BSI_ERR_INVALID_ARG = -1
BSI_ERR_UNSUPPORTED = -2
BSI_ERR_HIP = -3
BSI_ERR_NO_DEVICE = -4
BSI_ERR_NOMEM = -5
BSI_MAX_SPACING = 64

EXPORTS = (
    "bsi_version", "bsi_last_error", "bsi_grid_dims", "bsi_forward", "bsi_forward_lerp", "bsi_forward_scalar",
    "bsi_adjoint_workspace_size",
    "bsi_adjoint", "bsi_adjoint_partials", "bsi_adjoint_reduce", "bsi_adjoint_noalloc", "bsi_general_grid_dims",
    "bsi_forward_general", "bsi_adjoint_general_workspace_size", "bsi_adjoint_general", "bsi_warp", "bsi_ssd_workspace_size", "bsi_ssd_grad", "bsi_ssd_fused_workspace_size", "bsi_ssd_fused",
    "bsi_ssd_fused_descent", "bsi_descent_step",
    "bsi_batch_create", "bsi_batch_bind", "bsi_batch_tune", "bsi_batch_config", "bsi_batch_describe", "bsi_batch_run",
    "bsi_batch_run_separate", "bsi_batch_capture", "bsi_batch_launch", "bsi_batch_destroy",
)


class BSIError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"libbsi error {code}: {message}")
        self.code = code


_LIB = None
_I32x3 = ctypes.c_int32 * 3
_VP = ctypes.c_void_p


def lib():
    """Load libbsi.so (once) and declare its signatures."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    p3 = ctypes.POINTER(ctypes.c_int32)
    pf3 = ctypes.POINTER(ctypes.c_float)
    sig = {
        "bsi_version": ([], i32),
        "bsi_last_error": ([], ctypes.c_char_p),
        "bsi_grid_dims": ([p3, p3, p3], i32),
        "bsi_forward": ([_VP, p3, p3, _VP, _VP], i32),
        "bsi_forward_scalar": ([_VP, p3, p3, _VP, _VP], i32),
        "bsi_forward_lerp": ([_VP, p3, p3, _VP, _VP], i32),
        "bsi_adjoint_workspace_size": ([p3, p3, ctypes.POINTER(sz)], i32),
        "bsi_adjoint": ([_VP, p3, p3, _VP, _VP, sz, _VP], i32),
        "bsi_adjoint_partials": ([_VP, p3, p3, _VP, sz, _VP], i32),
        "bsi_adjoint_noalloc": ([_VP, p3, p3, _VP, _VP], i32),
        "bsi_general_grid_dims": ([p3, pf3, pf3, p3], i32),
        "bsi_forward_general": ([_VP, p3, pf3, pf3, _VP, _VP], i32),
        "bsi_adjoint_general_workspace_size": ([p3, pf3, pf3, ctypes.POINTER(sz)], i32),
        "bsi_adjoint_general": ([_VP, p3, pf3, pf3, _VP, _VP, sz, _VP], i32),
        "bsi_adjoint_reduce": ([_VP, sz, p3, p3, _VP, _VP], i32),
        "bsi_warp": ([_VP, _VP, p3, _VP, _VP], i32),
        "bsi_ssd_workspace_size": ([p3, ctypes.POINTER(sz)], i32),
        "bsi_ssd_grad": ([_VP, _VP, _VP, p3, _VP, _VP, _VP, sz, _VP], i32),
        "bsi_ssd_fused_workspace_size": ([p3, p3, ctypes.POINTER(sz)], i32),
        "bsi_ssd_fused": ([_VP, _VP, _VP, p3, p3, _VP, _VP, _VP, sz, _VP], i32),
        "bsi_ssd_fused_descent": ([_VP, _VP, _VP, p3, p3, ctypes.c_float, _VP, _VP, _VP, sz, _VP], i32),
        "bsi_descent_step": ([_VP, _VP, ctypes.c_float, i64, _VP], i32),
        "bsi_batch_create": ([i32, p3, p3, ctypes.POINTER(_VP)], i32),
        "bsi_batch_bind": ([_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                            ctypes.POINTER(_VP)], i32),
        "bsi_batch_tune": ([_VP, _VP], i32),
        "bsi_batch_config": ([_VP, p3, p3], i32),
        "bsi_batch_describe": ([_VP, ctypes.c_char_p, i32], i32),
        "bsi_batch_run": ([_VP, _VP], i32),
        "bsi_batch_run_separate": ([_VP, _VP], i32),
        "bsi_batch_capture": ([_VP, _VP], i32),
        "bsi_batch_launch": ([_VP, _VP], i32),
        "bsi_batch_destroy": ([_VP], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = L
    return L


def _check(rc):
    if rc != BSI_OK:
        msg = lib().bsi_last_error()
        raise BSIError(rc, msg.decode() if msg else "")


def _triple(v, name):
    t = tuple(int(a) for a in v)
    if len(t) != 3:
        raise ValueError(f"{name} must have three entries")
    return _I32x3(*t)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return _VP(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t, name, shape=None):
    if t is None:
        return _VP(0)
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _VP(t.data_ptr())


def _raw(t):
    return _VP(t.data_ptr()) if t is not None else _VP(0)


# ------------------------------------------------------------------- geometry
def bsi_version():
    return int(lib().bsi_version())


def bsi_last_error():
    m = lib().bsi_last_error()
    return m.decode() if m else ""


def bsi_grid_dims(dims, spacing):
    """(gx, gy, gz) = ceil(n/d) + 3 per axis."""
    out = _I32x3()
    _check(lib().bsi_grid_dims(_triple(dims, "dims"), _triple(spacing, "spacing"), out))
    return tuple(out)


def grid_shape(dims, spacing):
    gx, gy, gz = bsi_grid_dims(dims, spacing)
    return (gz, gy, gx, 3)


def field_shape(dims):
    nx, ny, nz = (int(v) for v in dims)
    return (nz, ny, nx, 3)


# ------------------------------------------------------------- forward/adjoint
def bsi_forward(grid, dims, spacing, field, stream=None):
    """Eq. 1 into ``field`` (nz, ny, nx, 3) from ``grid`` (gz, gy, gx, 3)."""
    g = _ptr(grid, "grid", grid_shape(dims, spacing))
    f = _ptr(field, "field", field_shape(dims))
    _check(lib().bsi_forward(g, _triple(dims, "dims"), _triple(spacing, "spacing"), f, _stream(stream)))


def bsi_forward_lerp(grid, dims, spacing, field, stream=None):
    """Eq. 1 in the paper's lerp form (ablation; same result up to rounding, far more arithmetic)."""
    g = _ptr(grid, "grid", grid_shape(dims, spacing))
    f = _ptr(field, "field", field_shape(dims))
    _check(lib().bsi_forward_lerp(g, _triple(dims, "dims"), _triple(spacing, "spacing"), f, _stream(stream)))


def bsi_forward_scalar(grid, dims, spacing, image, stream=None):
    """Scalar Eq. 1 (B-spline upsampling): ``image`` (nz, ny, nx) from ``grid`` (gz, gy, gx)."""
    gx, gy, gz = bsi_grid_dims(dims, spacing)
    nx, ny, nz = (int(v) for v in dims)
    g = _ptr(grid, "grid", (gz, gy, gx))
    o = _ptr(image, "image", (nz, ny, nx))
    _check(lib().bsi_forward_scalar(g, _triple(dims, "dims"), _triple(spacing, "spacing"), o, _stream(stream)))


def upsample(grid, spacing, dims=None, out=None, stream=None):
    """Cubic B-spline upsampling of a coarse scalar volume ``grid`` (gz, gy, gx) by the
    integer factors ``spacing`` (x, y, z); ``dims`` defaults to the largest volume
    the grid covers, (g - 3) * spacing per axis."""
    gz, gy, gx = (int(v) for v in grid.shape)
    if dims is None:
        dims = tuple((g - 3) * int(d) for g, d in zip((gx, gy, gz), spacing))
    if out is None:
        nx, ny, nz = (int(v) for v in dims)
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=grid.device)
    bsi_forward_scalar(grid, dims, spacing, out, stream)
    return out


def bsi_adjoint_workspace_size(dims, spacing):
    n = ctypes.c_size_t()
    _check(lib().bsi_adjoint_workspace_size(_triple(dims, "dims"), _triple(spacing, "spacing"), ctypes.byref(n)))
    return int(n.value)


def bsi_adjoint(dfield, dims, spacing, grid_grad, workspace, stream=None):
    """Transpose of Eq. 1: ``grid_grad`` (overwritten) from ``dfield``.

    ``workspace`` is a device tensor of at least bsi_adjoint_workspace_size bytes."""
    d = _ptr(dfield, "dfield", field_shape(dims))
    g = _ptr(grid_grad, "grid_grad", grid_shape(dims, spacing))
    w, nbytes = _workspace(workspace)
    _check(lib().bsi_adjoint(d, _triple(dims, "dims"), _triple(spacing, "spacing"), g, w, nbytes,
                             _stream(stream)))


def bsi_adjoint_partials(dfield, dims, spacing, workspace, stream=None):
    """Pass 1 of bsi_adjoint: per-brick partial sums of ``dfield`` into ``workspace``."""
    d = _ptr(dfield, "dfield", field_shape(dims))
    w, nbytes = _workspace(workspace)
    _check(lib().bsi_adjoint_partials(d, _triple(dims, "dims"), _triple(spacing, "spacing"), w, nbytes,
                                      _stream(stream)))


def bsi_adjoint_reduce(workspace, dims, spacing, grid_grad, stream=None):
    """Pass 2 of bsi_adjoint: fixed-order sum of the partials into ``grid_grad`` (overwritten)."""
    g = _ptr(grid_grad, "grid_grad", grid_shape(dims, spacing))
    w, nbytes = _workspace(workspace)
    _check(lib().bsi_adjoint_reduce(w, nbytes, _triple(dims, "dims"), _triple(spacing, "spacing"), g,
                                    _stream(stream)))


def bsi_adjoint_noalloc(dfield, dims, spacing, grid_grad, stream=None):
    """bsi_adjoint without a workspace and without allocating: the partials go to
    the library's fixed per-device scratch array (BSI_ADJOINT_NOALLOC_MAX_BYTES);
    calls that may overlap on one GPU race on it."""
    d = _ptr(dfield, "dfield", field_shape(dims))
    g = _ptr(grid_grad, "grid_grad", grid_shape(dims, spacing))
    _check(lib().bsi_adjoint_noalloc(d, _triple(dims, "dims"), _triple(spacing, "spacing"), g, _stream(stream)))


BSI_ADJOINT_NOALLOC_MAX_BYTES = 64 << 20


def _workspace(workspace):
    if not isinstance(workspace, torch.Tensor) or workspace.device.type != "cuda" or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    return _raw(workspace), workspace.numel() * workspace.element_size()


# ------------------------------------------------- real spacing, origin offset
_F32x3 = ctypes.c_float * 3


def _ftriple(v, name):
    vals = [float(x) for x in v]
    if len(vals) != 3:
        raise ValueError(f"{name} must have 3 entries (x, y, z)")
    return _F32x3(*vals)


def bsi_general_grid_dims(dims, spacing, origin):
    """(gx, gy, gz) = floor((n - 1 - o) / s) + 4 per axis."""
    out = _I32x3()
    _check(lib().bsi_general_grid_dims(_triple(dims, "dims"), _ftriple(spacing, "spacing"),
                                       _ftriple(origin, "origin"), out))
    return tuple(out)


def general_grid_shape(dims, spacing, origin):
    gx, gy, gz = bsi_general_grid_dims(dims, spacing, origin)
    return (gz, gy, gx, 3)


def bsi_forward_general(grid, dims, spacing, origin, field, stream=None):
    """Eq. 1 for real spacing and an origin offset (control point c at o + (c - 1) s)."""
    g = _ptr(grid, "grid", general_grid_shape(dims, spacing, origin))
    f = _ptr(field, "field", field_shape(dims))
    _check(lib().bsi_forward_general(g, _triple(dims, "dims"), _ftriple(spacing, "spacing"),
                                     _ftriple(origin, "origin"), f, _stream(stream)))


def bsi_adjoint_general_workspace_size(dims, spacing, origin):
    n = ctypes.c_size_t()
    _check(lib().bsi_adjoint_general_workspace_size(_triple(dims, "dims"), _ftriple(spacing, "spacing"),
                                                    _ftriple(origin, "origin"), ctypes.byref(n)))
    return int(n.value)


def bsi_adjoint_general(dfield, dims, spacing, origin, grid_grad, workspace, stream=None):
    """Transpose of bsi_forward_general; ``grid_grad`` overwritten."""
    d = _ptr(dfield, "dfield", field_shape(dims))
    g = _ptr(grid_grad, "grid_grad", general_grid_shape(dims, spacing, origin))
    w, nbytes = _workspace(workspace)
    _check(lib().bsi_adjoint_general(d, _triple(dims, "dims"), _ftriple(spacing, "spacing"),
                                     _ftriple(origin, "origin"), g, w, nbytes, _stream(stream)))


# ---------------------------------------------------------------- registration
def bsi_warp(field, image, dims, out, stream=None):
    nx, ny, nz = (int(v) for v in dims)
    f = _ptr(field, "field", field_shape(dims))
    i = _ptr(image, "image", (nz, ny, nx))
    o = _ptr(out, "out", (nz, ny, nx))
    _check(lib().bsi_warp(f, i, _triple(dims, "dims"), o, _stream(stream)))


def bsi_ssd_workspace_size(dims):
    n = ctypes.c_size_t()
    _check(lib().bsi_ssd_workspace_size(_triple(dims, "dims"), ctypes.byref(n)))
    return int(n.value)


def bsi_ssd_grad(field, moving, fixed, dims, dfield, loss, workspace, stream=None):
    nx, ny, nz = (int(v) for v in dims)
    f = _ptr(field, "field", field_shape(dims))
    m = _ptr(moving, "moving", (nz, ny, nx))
    x = _ptr(fixed, "fixed", (nz, ny, nx))
    d = _ptr(dfield, "dfield", field_shape(dims))
    l = _ptr(loss, "loss", (1,))
    w, nbytes = _workspace(workspace)
    _check(lib().bsi_ssd_grad(f, m, x, _triple(dims, "dims"), d, l, w, nbytes, _stream(stream)))


def bsi_ssd_fused_workspace_size(dims, spacing):
    n = ctypes.c_size_t()
    _check(lib().bsi_ssd_fused_workspace_size(_triple(dims, "dims"), _triple(spacing, "spacing"), ctypes.byref(n)))
    return int(n.value)


def bsi_ssd_fused(grid, moving, fixed, dims, spacing, grid_grad, loss, workspace, stream=None):
    """Loss and control-grid gradient of the SSD step in one pass (field never stored)."""
    nx, ny, nz = (int(v) for v in dims)
    g = _ptr(grid, "grid", grid_shape(dims, spacing))
    m = _ptr(moving, "moving", (nz, ny, nx))
    x = _ptr(fixed, "fixed", (nz, ny, nx))
    o = _ptr(grid_grad, "grid_grad", grid_shape(dims, spacing))
    l = _ptr(loss, "loss", (1,))
    w, nbytes = _workspace(workspace)
    _check(lib().bsi_ssd_fused(g, m, x, _triple(dims, "dims"), _triple(spacing, "spacing"), o, l, w, nbytes,
                               _stream(stream)))


def bsi_ssd_fused_descent(grid, moving, fixed, dims, spacing, eta, grid_grad, loss, workspace, stream=None):
    """One fused registration iteration: loss and gradient at `grid`, then grid -= eta * grad in place."""
    nx, ny, nz = (int(v) for v in dims)
    g = _ptr(grid, "grid", grid_shape(dims, spacing))
    m = _ptr(moving, "moving", (nz, ny, nx))
    x = _ptr(fixed, "fixed", (nz, ny, nx))
    o = _ptr(grid_grad, "grid_grad", grid_shape(dims, spacing))
    l = _ptr(loss, "loss", (1,))
    w, nbytes = _workspace(workspace)
    _check(lib().bsi_ssd_fused_descent(g, m, x, _triple(dims, "dims"), _triple(spacing, "spacing"),
                                       ctypes.c_float(float(eta)), o, l, w, nbytes, _stream(stream)))


def bsi_descent_step(grid, grad, eta, stream=None):
    g = _ptr(grid, "grid")
    d = _ptr(grad, "grad", tuple(grid.shape))
    _check(lib().bsi_descent_step(g, d, ctypes.c_float(float(eta)), grid.numel(), _stream(stream)))


# --------------------------------------------------------------------- batched
# Geometry of every live plan (keyed by its handle), so that bind can check each
# bound tensor against its volume before the library stores the pointers.
_PLANS = {}


def _ptr_array(tensors, name, shapes):
    if tensors is None:
        return None
    tensors = list(tensors)
    if len(tensors) != len(shapes):
        raise ValueError(f"{name} holds {len(tensors)} tensors; the plan has {len(shapes)} volumes")
    arr = (_VP * len(tensors))()
    for i, (t, shape) in enumerate(zip(tensors, shapes)):
        arr[i] = _ptr(t, f"{name}[{i}]", shape).value
    return arr


def bsi_batch_create(dims_list, spacing_list):
    n = len(dims_list)
    if n != len(spacing_list) or n < 1:
        raise ValueError("need one spacing per volume and at least one volume")
    dims = [tuple(int(v) for v in t) for t in dims_list]
    spacing = [tuple(int(v) for v in t) for t in spacing_list]
    if any(len(t) != 3 for t in dims + spacing):
        raise ValueError("every dims and spacing entry must have three values")
    d = (ctypes.c_int32 * (3 * n))(*[v for t in dims for v in t])
    s = (ctypes.c_int32 * (3 * n))(*[v for t in spacing for v in t])
    plan = _VP()
    _check(lib().bsi_batch_create(n, d, s, ctypes.byref(plan)))
    _PLANS[plan.value] = (dims, spacing)
    return plan


def bsi_batch_bind(plan, grids=None, fields=None, dfields=None, grid_grads=None):
    """Bind per-volume buffers; each list must hold exactly one tensor per volume, of
    that volume's grid or field shape (checked here, before the library sees them)."""
    if plan is None or not plan.value or plan.value not in _PLANS:
        raise ValueError("not a live batched plan")
    dims, spacing = _PLANS[plan.value]
    gshapes = [grid_shape(d, s) for d, s in zip(dims, spacing)]
    fshapes = [field_shape(d) for d in dims]
    arrs = [_ptr_array(grids, "grids", gshapes), _ptr_array(fields, "fields", fshapes),
            _ptr_array(dfields, "dfields", fshapes), _ptr_array(grid_grads, "grid_grads", gshapes)]
    _check(lib().bsi_batch_bind(plan, *arrs))


def bsi_batch_tune(plan, stream=None):
    _check(lib().bsi_batch_tune(plan, _stream(stream)))


def bsi_batch_config(plan):
    i, n = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().bsi_batch_config(plan, ctypes.byref(i), ctypes.byref(n)))
    return int(i.value), int(n.value)


def bsi_batch_describe(plan):
    buf = ctypes.create_string_buffer(512)
    _check(lib().bsi_batch_describe(plan, buf, 512))
    return buf.value.decode()


def bsi_batch_run(plan, stream=None):
    _check(lib().bsi_batch_run(plan, _stream(stream)))


def bsi_batch_run_separate(plan, stream=None):
    _check(lib().bsi_batch_run_separate(plan, _stream(stream)))


def bsi_batch_capture(plan, stream=None):
    _check(lib().bsi_batch_capture(plan, _stream(stream)))


def bsi_batch_launch(plan, stream=None):
    _check(lib().bsi_batch_launch(plan, _stream(stream)))


def bsi_batch_destroy(plan):
    if plan:
        _PLANS.pop(plan.value, None)
        lib().bsi_batch_destroy(plan)
