"""GPU parity of labels and component statistics in one call
(ccl_label_2d_stats): the labels against the oracle's pixel by pixel, the
records against the oracle's statistics field by field, and both against
the two-step path (ccl_label_2d, then ccl_component_stats)."""
import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import workloads as wl
from tests.gpu_util import CONFIGS, say, to_dev

pytestmark = pytest.mark.gpu

FIELDS = ("label", "area", "x_min", "y_min", "x_max", "y_max", "sum_x", "sum_y")
STATS_CONFIGS = [c for c in CONFIGS if c[0] <= 64]


def fused(img, conn, capacity=None, config=None, pad=0):
    import torch
    from paper_1708_08180_amd import binding

    lab, rec = binding.label_stats(to_dev(img, pad), conn, capacity=capacity, config=config)
    torch.cuda.synchronize()
    return lab.cpu().numpy().view(np.uint32), rec


def _cmp_records(got, want, what):
    assert len(got) == len(want), "%s: %d records, want %d" % (what, len(got), len(want))
    for f in FIELDS:
        g, w = got[f].astype(np.uint64), want[f].astype(np.uint64)
        if not np.array_equal(g, w):
            k = int(np.argmax(g != w))
            raise AssertionError("%s: field %s differs first at record %d (label %d): got %d want %d"
                                 % (what, f, k, want["label"][k], got[f][k], want[f][k]))


def _check(img, conn, what, config=None, pad=0):
    say("label+stats %s %dx%d conn=%d config=%s" % (what, img.shape[0], img.shape[1], conn, config))
    lab, rec = fused(img, conn, config=config, pad=pad)
    want_lab = oracle.label(img, conn)
    if not np.array_equal(lab, want_lab):
        y, x = np.argwhere(lab != want_lab)[0]
        raise AssertionError("%s: label differs at (%d, %d): got %d want %d" % (what, y, x, lab[y, x], want_lab[y, x]))
    _cmp_records(rec, oracle.stats(img, conn), what)


@pytest.mark.parametrize("conn", [8, 4])
def test_label_stats_small_and_ragged(conn):
    cases = ((256, 256, 0.5, 1), (300, 257, 0.45, 1), (1, 1, 1.0, 1), (1, 1, 0.0, 1), (3, 1000, 0.5, 1),
             (129, 65, 0.6, 3), (70, 70, 0.2, 1), (65, 64, 0.5, 1), (64, 65, 0.5, 1), (1000, 3, 0.5, 1),
             (200, 130, 0.9, 1))
    for seed, (H, W, p, g) in enumerate(cases):
        _check(wl.bernoulli(H, W, p, 2200 + seed, g), conn, "bern p=%.2f g=%d" % (p, g))


@pytest.mark.parametrize("conn", [8, 4])
def test_label_stats_closed_forms(conn):
    _check(np.zeros((50, 70), np.uint8), conn, "empty")
    _check(np.ones((50, 70), np.uint8), conn, "full")
    _check(np.ones((300, 200), np.uint8), conn, "full, many tiles")
    _check(wl.checkerboard(130, 190, 0), conn, "checkerboard")
    _check(wl.rings(97, 131), conn, "rings")
    _check(wl.serpentine(128, 200), conn, "serpentine")
    _check(wl.spiral(257, 300), conn, "spiral")


@pytest.mark.parametrize("conn", [8, 4])
def test_label_stats_most_components_per_tile(conn):
    """The most tile-local components a tile can hold: every pixel alone
    (4-connectivity checkerboard) or one pixel per 2 x 2 block
    (8-connectivity), over whole 64 x 64 tiles and a ragged edge."""
    img = np.zeros((128 + 9, 192 + 5), np.uint8)
    if conn == 4:
        img[:] = wl.checkerboard(*img.shape, 0)
    else:
        img[::2, ::2] = 1
    _check(img, conn, "densest components")


@pytest.mark.parametrize("config", STATS_CONFIGS)
def test_label_stats_every_config(config):
    img = wl.bernoulli(333, 450, 0.5, 2300)
    for conn in (8, 4):
        _check(img, conn, "bern 333x450", config=config)


def test_label_stats_pitched_rows():
    _check(wl.bernoulli(200, 333, 0.5, 2301), 8, "pitched", pad=29)


def test_label_stats_matches_two_step_path():
    """The same labels and records as ccl_label_2d then ccl_component_stats."""
    import torch
    from paper_1708_08180_amd import binding

    img = wl.bernoulli(1024, 1536, 0.5, 2302)
    for conn in (8, 4):
        lab, rec = fused(img, conn)
        d = to_dev(img)
        lab2 = binding.label(d, conn)
        rec2 = binding.component_stats(lab2)
        torch.cuda.synchronize()
        assert np.array_equal(lab, lab2.cpu().numpy().view(np.uint32))
        _cmp_records(rec, rec2, "two-step conn=%d" % conn)


def test_label_stats_capacity():
    img = wl.bernoulli(200, 300, 0.4, 2303)
    want = oracle.stats(img, 8)
    assert len(want) > 20
    lab, got = fused(img, 8, capacity=10)
    assert len(got) == 10
    _cmp_records(got, want[:10], "capacity 10")
    assert np.array_equal(lab, oracle.label(img, 8))
    # capacity 0 counts only
    import torch
    from paper_1708_08180_amd import binding

    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    d = to_dev(img)
    out = torch.empty(d.shape, dtype=torch.int32, device="cuda")
    lib = binding.load_library()
    rc = lib.ccl_label_2d_stats(d.data_ptr(), 200, 300, 300, 8, out.data_ptr(), None, 0, n.data_ptr(),
                                None, binding._stream_handle(None))
    assert rc == 0
    torch.cuda.synchronize()
    assert int(n.item()) == len(want)


def test_label_stats_repeated_calls_are_exact():
    """Back-to-back calls on one stream reuse the workspace: every call is
    exact (the records' accumulators and counters start clean)."""
    imgs = [wl.bernoulli(512, 700, p, 2310 + i) for i, p in enumerate((0.5, 0.3, 0.7, 0.5))]
    want = [(oracle.label(im, 8), oracle.stats(im, 8)) for im in imgs]
    for rep in range(3):
        for k, im in enumerate(imgs):
            lab, rec = fused(im, 8)
            assert np.array_equal(lab, want[k][0]), "rep %d image %d" % (rep, k)
            _cmp_records(rec, want[k][1], "rep %d image %d" % (rep, k))


def test_label_stats_full_size():
    # a percolating component crossing every tile, and many small ones
    _check(wl.bernoulli(4096, 4096, 0.5, wl.sweep_seed(0.5, 1)), 8, "bern 4096")
    _check(wl.bernoulli(4096, 4096, 0.3, wl.sweep_seed(0.3, 1)), 4, "bern 4096 p=0.3")
    _check(wl.smoothed_noise(2048, 2048, 4.0, 2304), 4, "smoothed 2048")
    _check(wl.spiral(2048, 2048), 8, "spiral 2048")
