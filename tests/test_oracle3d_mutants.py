"""Planted mistakes in the 3D oracle must be caught by its pins (CPU only)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests.test_oracle3d import closure3d

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "ccl_oracle.c")

MUTANTS = {
    "18_takes_corners": ("(conn == 18 && steps > 2)", "(conn == 18 && steps > 3)"),
    "6_takes_edges": ("(conn == 6 && steps > 1)", "(conn == 6 && steps > 2)"),
    "slice_stride_dropped": ("const int64_t r = nz * HW + ny * W + nx;", "const int64_t r = nz * W + ny * W + nx;"),
    "label_off_by_one_3d": ("const uint32_t lab = (uint32_t)p + 1u;", "const uint32_t lab = (uint32_t)p;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor for %s not found exactly once" % name
    c = tmp_path / (name + ".c")
    c.write_text(src.replace(old, new))
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", str(c), "-o", str(so)])
    fn = ctypes.CDLL(str(so)).oracle_label_3d
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                   ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]

    def label3d(vol, conn):
        vol = np.ascontiguousarray(vol)
        D, H, W = vol.shape
        out = np.zeros(vol.shape, np.uint32)
        if fn(vol.ctypes.data, D, H, W, W, H * W, conn, out.ctypes.data) != 0:
            raise AssertionError("mutant failed")
        return out

    return label3d


def _pins_pass(label3d):
    n = 8
    codes = np.arange(1 << n, dtype=np.uint32)
    vols = ((codes[:, None] >> np.arange(n, dtype=np.uint32)[None]) & 1).astype(np.uint8).reshape(-1, 2, 2, 2)
    for conn in (6, 18, 26):
        want = closure3d(vols, conn)
        for k in range(len(vols)):
            if not np.array_equal(label3d(vols[k], conn), want[k]):
                return False
    return True


def test_real_3d_oracle_passes(tmp_path):
    assert _pins_pass(_build(tmp_path, "identity", "(conn == 6 && steps > 1)", "(conn == 6 && steps > 1)"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_3d_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert not _pins_pass(_build(tmp_path, name, old, new))
