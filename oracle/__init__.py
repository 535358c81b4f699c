"""CPU oracle for connected-components labeling -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

The arithmetic lives in ``ccl_oracle.c`` (a plain single-threaded flood
fill, compiled with gcc).  This module only compiles it and marshals numpy
arrays through ctypes.

Definition computed (Introduction; Sec. II-A-2 and the atomicMin merge of
Sec. II-A-3, which make every root the smallest index of its set):

    label[y, x] = 0                                   for background
    label[y, x] = 1 + min raster index (y' * W + x')  over the component

Parity pins: the tests check this against a brute-force transitive closure
on every tiny image, against ``scipy.ndimage.label`` after renumbering, and
against closed forms of hand-built patterns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccl_oracle.c")
_LIB = os.path.join(_HERE, "libccl_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libccl_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-Wall", "-Werror", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _get():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        for name in ("oracle_label_2d", "oracle_label_2d_equal"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                           ctypes.c_int, ctypes.c_void_p]
        lib.oracle_label_3d.restype = ctypes.c_int
        lib.oracle_label_3d.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_void_p]
        lib.oracle_stats_2d.restype = ctypes.c_int
        lib.oracle_stats_2d.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        _lib = lib
    return _lib


def _run2d(name: str, img: np.ndarray, conn: int) -> np.ndarray:
    img = np.asarray(img)
    if img.ndim != 2:
        raise ValueError("expected a 2D image")
    if img.dtype != np.uint8:
        raise ValueError("expected uint8 pixels")
    if img.strides[1] != 1:
        img = np.ascontiguousarray(img)
    H, W = img.shape
    out = np.empty((H, W), dtype=np.uint32)
    if H == 0 or W == 0:
        return out
    # numpy may report any stride for a dimension of extent 1
    pitch = img.strides[0] if H > 1 else W
    if pitch < W:
        img = np.ascontiguousarray(img)
        pitch = W
    rc = getattr(_get(), name)(img.ctypes.data, H, W, pitch, int(conn), out.ctypes.data)
    if rc != 0:
        raise ValueError("%s failed with code %d (H=%d W=%d conn=%r)" % (name, rc, H, W, conn))
    return out


def label(img: np.ndarray, conn: int = 8) -> np.ndarray:
    """Canonical binary labels: nonzero pixels are foreground, background is 0."""
    return _run2d("oracle_label_2d", img, conn)


def label_equal(img: np.ndarray, conn: int = 8) -> np.ndarray:
    """Labels of every equal-value class (background included): 1 + min raster index."""
    return _run2d("oracle_label_2d_equal", img, conn)


# One record per component (layout of the C struct oracle_component).
STATS_DTYPE = np.dtype([("label", "<u4"), ("area", "<u4"), ("x_min", "<u4"), ("y_min", "<u4"),
                        ("x_max", "<u4"), ("y_max", "<u4"), ("sum_x", "<u8"), ("sum_y", "<u8")])


def stats(img: np.ndarray, conn: int = 8, equal: bool = False) -> np.ndarray:
    """Per-component statistics in increasing label order: label, area,
    inclusive bounding box, and the sums of column and row indices
    (centroid = sum / area).  equal=True uses equal-value components."""
    img = np.asarray(img)
    if img.ndim != 2 or img.dtype != np.uint8:
        raise ValueError("expected a 2D uint8 image")
    img = np.ascontiguousarray(img)
    H, W = img.shape
    lib = _get()
    n = ctypes.c_int64(0)
    rc = lib.oracle_stats_2d(img.ctypes.data, H, W, W, int(conn), 1 if equal else 0, None, 0,
                             ctypes.byref(n))
    if rc != 0:
        raise ValueError("oracle_stats_2d failed with code %d" % rc)
    out = np.zeros(n.value, dtype=STATS_DTYPE)
    rc = lib.oracle_stats_2d(img.ctypes.data, H, W, W, int(conn), 1 if equal else 0,
                             out.ctypes.data if n.value else None, n.value, ctypes.byref(n))
    if rc != 0:
        raise ValueError("oracle_stats_2d failed with code %d" % rc)
    return out


def label3d(vol: np.ndarray, conn: int = 26) -> np.ndarray:
    """Canonical 3D labels (conn 6, 18 or 26): 1 + the smallest raster index
    z*H*W + y*W + x of each voxel's component, 0 for background."""
    vol = np.ascontiguousarray(np.asarray(vol))
    if vol.ndim != 3 or vol.dtype != np.uint8:
        raise ValueError("expected a 3D uint8 volume")
    D, H, W = vol.shape
    out = np.empty((D, H, W), dtype=np.uint32)
    rc = _get().oracle_label_3d(vol.ctypes.data, D, H, W, W, H * W, int(conn), out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_label_3d failed with code %d" % rc)
    return out
