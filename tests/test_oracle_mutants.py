"""Planted mistakes in the oracle must be caught by the pins (CPU only).

Each mutant is a copy of the oracle's C source with one plausible slip
(a dropped neighbour, an off-by-one label, a transposed index, the pitch
used as the raster stride, ...).  It is compiled into a temporary library
and run through the same pins as the real oracle; every mutant has to fail
at least one of them.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "ccl_oracle.c")

MUTANTS = {
    "drop_right_neighbour": ("dx[8] = {0, -1, 1, 0,", "dx[8] = {0, -1, 0, 0,"),
    "ignore_8_connectivity": ("const int nnb = conn;", "const int nnb = 4;"),
    "label_off_by_one": ("(uint32_t)(p + 1)", "(uint32_t)(p)"),
    "pitch_as_raster_stride": ("const int64_t r = ny * W + nx;", "const int64_t r = ny * pitch + nx;"),
    "transposed_index": ("const int64_t qy = q / W, qx = q % W;", "const int64_t qy = q % W, qx = q / W;"),
    "equal_instead_of_nonzero": ("(mode == 0) ? (w != 0)", "(mode == 0) ? (w == v)"),
    "wrong_diagonal": ("dy[8] = {-1, 0, 0, 1, -1, -1, 1, 1}", "dy[8] = {-1, 0, 0, 1, -1, -1, 1, 0}"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor for %s not found exactly once" % name
    c = tmp_path / (name + ".c")
    c.write_text(src.replace(old, new))
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", str(c), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    fn = lib.oracle_label_2d
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                   ctypes.c_void_p]

    def label(img, conn):
        img = np.asarray(img)
        if img.strides[1] != 1:
            img = np.ascontiguousarray(img)
        H, W = img.shape
        pitch = img.strides[0] if H > 1 else W
        out = np.zeros((H, W), np.uint32)
        rc = fn(img.ctypes.data, H, W, pitch, conn, out.ctypes.data)
        if rc != 0:
            raise AssertionError("mutant returned %d" % rc)
        return out

    return label


def _pins_pass(label):
    try:
        for conn in (4, 8):
            pins.check_exhaustive(label, 3, 3, conn)
            pins.check_exhaustive(label, 2, 4, conn)
        pins.check_closed_forms(label, shapes=((5, 9), (9, 5), (16, 16)))
        pins.check_pitch(label, label)
        pins.check_mixed_values(label)
    except AssertionError:
        return False
    return True


def test_real_oracle_passes_the_mutant_pins(tmp_path):
    label = _build(tmp_path, "identity", "const int nnb = conn;", "const int nnb = conn;")
    assert _pins_pass(label)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    label = _build(tmp_path, name, old, new)
    assert not _pins_pass(label), "planted mistake %s survived every pin" % name
