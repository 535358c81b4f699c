"""GPU parity: libccl's labels must equal the CPU oracle's bit for bit.

Integer graph work, so the bar is exact equality on every pixel.  Every
call goes through the C ABI (ctypes binding); the oracle runs on the host.
"""
import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import workloads as wl
from tests import pins
from tests.gpu_util import CONFIGS, gpu_label, mosaic, say

pytestmark = pytest.mark.gpu


def _cmp(img, conn, config=None, pad=0, plain=False, what=""):
    say("case %s %dx%d conn=%d config=%s pad=%d" % (what, img.shape[0], img.shape[1], conn, config, pad))
    got = gpu_label(img, conn, config=config, pad=pad, plain=plain)
    want = oracle.label(img, conn)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("%s: %d mismatches, first at (%d,%d): got %d want %d"
                             % (what, len(bad), y, x, got[y, x], want[y, x]))


@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("seed", range(10))
def test_bernoulli_256(seed, conn):
    # the small configuration: 256x256, p = 0.5
    img = wl.bernoulli(256, 256, 0.5, seed)
    _cmp(img, conn, what="bern256 seed=%d" % seed)


@pytest.mark.parametrize("config", CONFIGS)
@pytest.mark.parametrize("conn", [8, 4])
def test_every_tile_config(config, conn):
    for seed, (H, W) in enumerate(((256, 256), (200, 333), (65, 129))):
        img = wl.bernoulli(H, W, 0.5, 100 + seed)
        _cmp(img, conn, config=config, what="cfg")
    img = wl.bernoulli(300, 260, 0.6, 7, g=3)
    _cmp(img, conn, config=config, what="cfg-g3")


@pytest.mark.parametrize("conn", [8, 4])
def test_all_tiny_images_mosaic(conn):
    # all 2^16 binary 4x4 images laid out with blank separators: every tiny
    # pattern lands at many tile offsets and straddles tile edges
    tiles = pins.all_images(4, 4)
    img = mosaic(tiles, gap=1)
    _cmp(img, conn, what="mosaic4x4")
    for config in ((16, 4), (32, 2)):
        _cmp(img, conn, config=config, what="mosaic4x4")
    # and the dense variant: gap 0 means patterns touch each other
    _cmp(mosaic(tiles[::7], gap=0), conn, what="mosaic4x4-dense")


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (200, 1), (17, 33), (64, 64), (65, 65),
                                   (63, 127), (1080, 1920), (2160, 3840), (1, 4096), (4096, 1),
                                   (3, 70000)])
def test_ragged_shapes(shape):
    H, W = shape
    for conn in (8, 4):
        img = wl.bernoulli(H, W, 0.55, H * 7 + W)
        _cmp(img, conn, what="ragged")


def test_pitch_and_values():
    img = wl.bernoulli(333, 517, 0.5, 3)
    for conn in (4, 8):
        _cmp(img, conn, pad=13, what="pitch")
        _cmp(img * 255, conn, what="fg255")
    rng = wl.rng_for(4)
    mixed = (rng.integers(1, 256, size=img.shape) * img).astype(np.uint8)
    for conn in (4, 8):
        _cmp(mixed, conn, what="mixed")


def test_closed_forms_on_gpu():
    def fn(img, conn):
        return gpu_label(img, conn)

    pins.check_closed_forms(fn, shapes=((1, 1), (5, 9), (64, 64), (65, 130), (130, 65), (257, 300)))


@pytest.mark.parametrize("conn", [8, 4])
def test_tile_corner_patterns(conn):
    # one pixel at every tile corner, diagonal contacts across every corner,
    # and 2x2 blocks centred on the corners
    for th in (16, 32, 64):
        H, W = 5 * th + 3, 5 * 64 + 5
        a = np.zeros((H, W), np.uint8)
        a[th - 1::th, 63::64] = 1
        a[th::th, 64::64] = 1          # (x0, y0) touches (x0-1, y0-1) diagonally
        b = np.zeros((H, W), np.uint8)
        b[th - 1::th, 64::64] = 1
        b[th::th, 63::64] = 1          # anti-diagonal contact across the corner
        c = np.zeros((H, W), np.uint8)
        for y in range(th, H, th):
            for x in range(64, W, 64):
                c[y - 1:y + 1, x - 1:x + 1] = 1
        d = np.zeros((H, W), np.uint8)
        d[::th, :] = 1
        d[:, ::64] = 1                 # grid lines on the first row/column of tiles
        for img in (a, b, c, d, 1 - d):
            _cmp(img.astype(np.uint8), conn, config=(th, 4 if th >= 4 else 1), what="corners")


@pytest.mark.parametrize("config", [c for c in CONFIGS if c[0] == 16] + [(64, 4), (128, 8)])
def test_most_flagged_roots_per_link_wavefront(config):
    """Under 4-connectivity a checkerboard makes every pixel its own
    component, so every foreground edge cell is a flagged local root.  A
    16-row link wavefront that holds both the top and the bottom row of a
    16-row tile then has 32 + 32 + 7 + 7 = 78 of them, more than one per
    lane (two rounds of walks); taller tiles give each wavefront at most
    one of those rows."""
    for phase in (0, 1):
        img = wl.checkerboard(16 * 5 + 3, 64 * 3 + 7, phase)
        _cmp(img, 4, config=config, what="checker%d-flagged" % phase)
        _cmp(img, 8, config=config, what="checker%d-flagged" % phase)


@pytest.mark.parametrize("conn", [8, 4])
def test_long_chains(conn):
    for (H, W) in ((512, 512), (1000, 777)):
        for name, img in (("serp", wl.serpentine(H, W)), ("colserp", wl.column_serpentine(H, W)),
                          ("spiral", wl.spiral(H, W)), ("rings", wl.rings(H, W))):
            _cmp(img, conn, what=name)


def test_smoothed_and_granular():
    for conn in (8, 4):
        _cmp(wl.smoothed_noise(700, 900, 4.0, 31), conn, what="smoothed")
        for g in (2, 4, 8, 16):
            _cmp(wl.bernoulli(1024, 1024, 0.5, wl.sweep_seed(0.5, g), g), conn, what="g%d" % g)


def test_deterministic_repeats():
    img = wl.bernoulli(1024, 1024, 0.5, 5)
    first = gpu_label(img, 8)
    for _ in range(20):
        assert np.array_equal(gpu_label(img, 8), first)
    assert np.array_equal(first, oracle.label(img, 8))


def test_plain_entry_point():
    img = wl.bernoulli(777, 1234, 0.5, 77)
    for conn in (4, 8):
        _cmp(img, conn, plain=True, what="plain")


@pytest.mark.parametrize("config", CONFIGS + [(16, 8), (32, 16), (64, 2)])
def test_repeated_runs_are_exact(config):
    # races in concurrent unions show up as run-to-run differences; every
    # configuration must give the oracle's labels on every repetition
    imgs = [wl.bernoulli(300, 260, 0.6, 7, g=3), wl.bernoulli(512, 512, 0.5, 3)]
    for conn in (4, 8):
        for img in imgs:
            want = oracle.label(img, conn)
            for rep in range(8):
                got = gpu_label(img, conn, config=config)
                assert np.array_equal(got, want), "config %s conn %d rep %d" % (config, conn, rep)


def test_stream_ordering_with_torch_work():
    # the library's kernels must run in order with torch work on the same
    # (non-default) stream: torch writes the image right before the call and
    # reads the labels right after, with no synchronization in between
    import torch

    img = wl.bernoulli(1024, 1536, 0.5, 21)
    want = oracle.label(img, 8)
    host = torch.from_numpy(img).pin_memory()
    from paper_1708_08180_amd import binding

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d = torch.zeros((1024, 1536), dtype=torch.uint8, device="cuda")
        out = torch.full((1024, 1536), -7, dtype=torch.int32, device="cuda")
        for _ in range(3):
            d.zero_()
            d.copy_(host, non_blocking=True)
            binding.label_plain(d, 8, out=out, stream=s)
            res = out.to("cpu", non_blocking=True)
            s.synchronize()
            assert np.array_equal(res.numpy().view(np.uint32), want)
