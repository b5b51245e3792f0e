"""CPU check of the kernels' index arithmetic.

``libbsi_check.so`` runs, on the host, the same geometry functions and address
helpers the kernels use, over every workgroup, lane and control point of a
launch, and checks that every load and store stays inside its buffer (and pass 2
reads only partials pass 1 wrote).  Geometries: the benchmark's volumes, every
spacing up to the 64 maximum, ragged and extreme shapes, and all 32 volumes of
the batched workload."""
import ctypes
import os

import pytest

import workloads
from conftest import ROOT

LIB = os.path.join(ROOT, "paper_2004_05962_amd", "libbsi_check.so")


@pytest.fixture(scope="module")
def check():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is not built: run __graft_entry__.build()")
    L = ctypes.CDLL(LIB)
    L.bsi_check_indices.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.c_char_p, ctypes.c_int]
    L.bsi_check_indices.restype = ctypes.c_int

    def run(dims, spacing):
        msg = ctypes.create_string_buffer(512)
        rc = L.bsi_check_indices((ctypes.c_int32 * 3)(*dims), (ctypes.c_int32 * 3)(*spacing), msg, 512)
        return rc, msg.value.decode()
    return run


GEOMS = [((512, 512, 256), (d, d, d)) for d in (3, 4, 5, 8)] + [
    ((256, 256, 256), (5, 5, 5)), ((256, 256, 160), (5, 5, 5)), ((64, 64, 64), (5, 5, 5)),
    ((1, 1, 1), (1, 1, 1)), ((1, 1, 1), (64, 64, 64)), ((7, 3, 2), (2, 3, 1)), ((130, 9, 11), (5, 4, 3)),
    ((65, 70, 33), (64, 7, 10)), ((33, 40, 129), (8, 33, 6)), ((510, 6, 7), (5, 5, 5)),
    ((91, 20, 12), (13, 2, 3)), ((200, 33, 9), (12, 12, 2)), ((65536, 3, 2), (7, 1, 2)),
    ((2, 65536, 3), (1, 5, 1)), ((3, 2, 65536), (2, 1, 6)), ((97, 300, 41), (17, 40, 33)),
]


@pytest.mark.parametrize("dims,spacing", GEOMS)
def test_index_arithmetic_in_bounds(check, dims, spacing):
    rc, msg = check(dims, spacing)
    assert rc == 0, msg


@pytest.mark.parametrize("d", range(1, 65))
def test_every_spacing(check, d):
    dims = (3 * d + 5, 2 * d + 7, d + 9)
    rc, msg = check(dims, (d, max(1, d // 2), min(64, d + 3)))
    assert rc == 0, msg


def test_batched_workload_volumes(check):
    dims, spac = workloads.cfg5_geometry()
    for d, s in zip(dims, spac):
        rc, msg = check(tuple(int(v) for v in d), tuple(int(v) for v in s))
        assert rc == 0, (tuple(d), tuple(s), msg)


def test_batched_item_loops_end_and_cover():
    """The batched kernels' item loops: each item once, every loop ends (a grid
    of one workgroup per item takes exactly its own item)."""
    L = ctypes.CDLL(LIB)
    L.bsi_check_batch_items.argtypes = [ctypes.c_char_p, ctypes.c_int]
    L.bsi_check_batch_items.restype = ctypes.c_int
    msg = ctypes.create_string_buffer(512)
    assert L.bsi_check_batch_items(msg, 512) == 0, msg.value.decode()


GENERAL = [
    ((64, 48, 40), (4.7, 5.3, 5.1), (-1.5, 0.0, -2.25)),
    ((37, 29, 23), (2.5, 3.25, 1.75), (-0.5, -3.0, -1.25)),
    ((130, 9, 11), (1.0, 2.2, 3.3), (0.0, -1.1, -0.2)),
    ((70, 45, 20), (63.5, 7.75, 10.0), (-63.0, -2.5, -9.5)),
    ((20, 20, 20), (4.0, 4.0, 4.0), (0.0, 0.0, 0.0)),
    ((192, 9, 7), (5.5, 2.0, 3.0), (-1.0, 0.0, -0.5)),
    ((96, 80, 72), (4.3, 5.6, 3.1), (-2.0, -0.7, -1.0)),
    ((512, 512, 256), (5.3, 4.7, 5.1), (-2.5, -0.25, -4.0)),
    ((1, 1, 1), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0)),
    ((300, 3, 200), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0)),
    ((65, 17, 50), (64.0, 64.0, 64.0), (-63.9, -0.5, 0.0)),
    ((257, 130, 97), (4.31, 1.07, 12.9), (-4.3, -1.0, -0.01)),
]


@pytest.mark.parametrize("dims,spacing,origin", GENERAL)
def test_general_adjoint_indices(dims, spacing, origin):
    """The real-spacing adjoint's bricks, LDS request, table reads, partial
    offsets and pass-2 spans, over geometries with unit, fractional and coarse
    spacings (host tables from the device's own window-start function)."""
    L = ctypes.CDLL(LIB)
    f3 = ctypes.c_float * 3
    L.bsi_check_general_indices.argtypes = [ctypes.POINTER(ctypes.c_int32), f3, f3, ctypes.c_char_p, ctypes.c_int]
    L.bsi_check_general_indices.restype = ctypes.c_int
    msg = ctypes.create_string_buffer(512)
    rc = L.bsi_check_general_indices((ctypes.c_int32 * 3)(*dims), f3(*spacing), f3(*origin), msg, 512)
    assert rc == 0, msg.value.decode()
