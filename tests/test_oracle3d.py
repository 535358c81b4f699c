"""Pins of the 3D oracle (conn 6 / 18 / 26): transitive closure of the voxel
adjacency on every tiny volume, scipy.ndimage.label with the matching 3D
structuring element, and closed forms."""
import itertools

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1708_08180_amd import workloads as wl

STEPS = {6: 1, 18: 2, 26: 3}


def neighbours3d(D, H, W, conn):
    n = D * H * W
    nb = np.zeros((n, n), bool)
    for p in range(n):
        z, y, x = p // (H * W), (p // W) % H, p % W
        for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
            k = (dz != 0) + (dy != 0) + (dx != 0)
            if k == 0 or k > STEPS[conn]:
                continue
            nz, ny, nx = z + dz, y + dy, x + dx
            if 0 <= nz < D and 0 <= ny < H and 0 <= nx < W:
                nb[p, (nz * H + ny) * W + nx] = True
    return nb


def closure3d(vols, conn):
    B, D, H, W = vols.shape
    n = D * H * W
    fg = vols.reshape(B, n) != 0
    reach = (fg[:, :, None] & fg[:, None, :] & neighbours3d(D, H, W, conn)[None]) | np.eye(n, dtype=bool)[None]
    reach &= fg[:, :, None]
    r = reach.astype(np.float32)
    for _ in range(max(1, int(np.ceil(np.log2(n))))):
        r = (np.matmul(r, r) > 0).astype(np.float32)
    first = np.argmax(r > 0, axis=2)
    return np.where(fg, first + 1, 0).astype(np.uint32).reshape(B, D, H, W)


def scipy3d(vol, conn):
    lab, n = ndimage.label(vol != 0, structure=ndimage.generate_binary_structure(3, STEPS[conn]))
    out = np.zeros(vol.shape, np.uint32)
    if n:
        flat = lab.ravel()
        first = np.full(n + 1, -1, np.int64)
        idx = np.nonzero(flat)[0]
        # first occurrence of each label in raster order
        u, pos = np.unique(flat[idx], return_index=True)
        first[u] = idx[pos]
        out = np.where(lab > 0, first[lab] + 1, 0).astype(np.uint32)
    return out


@pytest.mark.parametrize("conn", [6, 18, 26])
@pytest.mark.parametrize("shape", [(2, 2, 2), (2, 2, 3), (3, 2, 2), (2, 3, 2)])
def test_exhaustive_tiny_volumes(conn, shape):
    D, H, W = shape
    n = D * H * W
    codes = np.arange(1 << n, dtype=np.uint32)
    vols = ((codes[:, None] >> np.arange(n, dtype=np.uint32)[None]) & 1).astype(np.uint8).reshape(-1, D, H, W)
    want = closure3d(vols, conn)
    for k in range(len(vols)):
        assert np.array_equal(oracle.label3d(vols[k], conn), want[k]), (shape, conn, k)


@pytest.mark.parametrize("conn", [6, 18, 26])
@pytest.mark.parametrize("p", [0.2, 0.35, 0.5])
def test_matches_scipy(conn, p):
    rng = wl.rng_for(int(p * 100) + conn)
    vol = (rng.random((17, 23, 70)) < p).astype(np.uint8)
    assert np.array_equal(oracle.label3d(vol, conn), scipy3d(vol, conn))


def test_closed_forms():
    D, H, W = 5, 6, 7
    zz, yy, xx = np.indices((D, H, W))
    cb = (((zz + yy + xx) % 2) == 0).astype(np.uint8)
    raster = (zz * H + yy) * W + xx
    assert np.array_equal(oracle.label3d(cb, 6), np.where(cb > 0, raster + 1, 0))  # singletons
    for conn in (18, 26):  # edge neighbours keep the parity: one component
        assert np.array_equal(oracle.label3d(cb, conn), np.where(cb > 0, 1, 0))
    # a body diagonal: joined only through corners
    diag = np.zeros((D, D, D), np.uint8)
    for i in range(D):
        diag[i, i, i] = 1
    assert (oracle.label3d(diag, 26)[diag > 0] == 1).all()
    for conn in (6, 18):
        assert len(np.unique(oracle.label3d(diag, conn)[diag > 0])) == D
    # a 2D image repeated along z: 6-conn = 4-conn slices, 18 / 26 = 8-conn slices
    img = wl.bernoulli(H * 3, W * 4, 0.5, 3)
    vol = np.repeat(img[None], 4, axis=0)
    for conn, c2 in ((6, 4), (18, 8), (26, 8)):
        lab2 = oracle.label(img, c2)
        assert np.array_equal(oracle.label3d(vol, conn), np.repeat(lab2[None], 4, axis=0))
