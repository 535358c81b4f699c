"""GPU parity of 3D volume labeling (6 / 18 / 26-connectivity) against the
3D oracle, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import workloads as wl
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def gpu_label3d(vol, conn, pad=0):
    import torch
    from paper_1708_08180_amd import binding

    D, H, W = vol.shape
    if pad:
        big = torch.full((D, H + 1, W + pad), 3, dtype=torch.uint8, device="cuda")
        big[:, :H, :W] = torch.from_numpy(np.ascontiguousarray(vol)).cuda()
        d = big[:, :H, :W]
    else:
        d = torch.from_numpy(np.ascontiguousarray(vol)).cuda()
    out = binding.label3d(d, conn)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def _cmp(vol, conn, pad=0, what=""):
    say("3d %s %s conn=%d pad=%d" % (what, vol.shape, conn, pad))
    got = gpu_label3d(vol, conn, pad)
    want = oracle.label3d(vol, conn)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        z, y, x = bad[0]
        raise AssertionError("%s: %d mismatches, first at (%d,%d,%d): got %d want %d"
                             % (what, len(bad), z, y, x, got[z, y, x], want[z, y, x]))


def noise(shape, p, seed):
    return (wl.rng_for(seed).random(shape) < p).astype(np.uint8)


@pytest.mark.parametrize("conn", [6, 18, 26])
def test_3d_noise_ragged(conn):
    for k, (shape, p) in enumerate((((8, 32, 128), 0.3), ((5, 19, 70), 0.5), ((9, 33, 65), 0.25),
                                    ((1, 1, 1), 1.0), ((13, 1, 200), 0.5), ((4, 16, 64), 0.6),
                                    ((17, 40, 130), 0.2))):
        _cmp(noise(shape, p, 2100 + k), conn, what="noise p=%.2f" % p)


@pytest.mark.parametrize("conn", [6, 18, 26])
def test_3d_pitched(conn):
    _cmp(noise((6, 21, 77), 0.35, 2200), conn, pad=9, what="pitched")


@pytest.mark.parametrize("conn", [6, 18, 26])
def test_3d_closed_forms(conn):
    D, H, W = 9, 35, 70
    zz, yy, xx = np.indices((D, H, W))
    _cmp((((zz + yy + xx) % 2) == 0).astype(np.uint8), conn, what="checkerboard")
    diag = np.zeros((20, 20, 20), np.uint8)
    for i in range(20):
        diag[i, i, i] = 1
    _cmp(diag, conn, what="body diagonal")
    img = wl.bernoulli(40, 130, 0.5, 7)
    _cmp(np.repeat(img[None], 7, axis=0), conn, what="stacked 2D")
    _cmp(np.ones((6, 20, 70), np.uint8), conn, what="full")


def test_3d_full_size():
    # 256^3 voxels: a percolating component (26-conn at p=0.3) and smoothed blobs
    from scipy import ndimage

    _cmp(noise((256, 256, 256), 0.3, 2300), 26, what="noise 256^3")
    z = ndimage.gaussian_filter(wl.rng_for(2301).standard_normal((128, 256, 256), dtype=np.float32), 3.0)
    _cmp((z > np.median(z)).astype(np.uint8), 6, what="smoothed 128x256x256")
