"""GPU test of the entry point that allocates nothing (ccl_label_2d_noalloc):
its labels must equal those of ccl_label_2d on the same image, bit for bit,
on two calls in a row, the second with a smaller image (the fixed array keeps
the first call's contents), and the smaller image must also equal the
oracle."""
import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import binding
from paper_1708_08180_amd import workloads as wl
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _both(img, conn, pad=0):
    import torch

    d = to_dev(img, pad)
    a = binding.label_noalloc(d, conn)
    b = binding.label_plain(d, conn)
    torch.cuda.synchronize()
    return a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("conn", [8, 4])
def test_noalloc_matches_plain_large_then_small(conn):
    # the largest image the fixed array serves, then a smaller ragged one
    # with a row pitch that is not the width
    big = wl.bernoulli(4096, 4096, 0.5, 20501)
    say("noalloc conn=%d 4096x4096 Bernoulli(0.5) seed=20501" % conn)
    got, ref = _both(big, conn)
    assert np.array_equal(got, ref), "4096^2: %d pixels differ" % int(np.count_nonzero(got != ref))
    small = wl.smoothed_noise(777, 1029, 3.0, 77)
    say("noalloc conn=%d 777x1029 smoothed seed=77 pad=5" % conn)
    got, ref = _both(small, conn, pad=5)
    assert np.array_equal(got, ref), "777x1029: %d pixels differ" % int(np.count_nonzero(got != ref))
    want = oracle.label(small, conn)
    assert np.array_equal(got, want)


def test_noalloc_repeated_shapes():
    # back-to-back calls of shrinking and growing sizes on one stream
    shapes = [(1080, 1920), (240, 320), (1, 1), (65, 129), (2160, 3840)]
    for i, (H, W) in enumerate(shapes):
        img = wl.bernoulli(H, W, 0.45, 900 + i)
        say("noalloc sequence %dx%d" % (H, W))
        got, ref = _both(img, 8)
        assert np.array_equal(got, ref), "%dx%d: %d pixels differ" % (H, W, int(np.count_nonzero(got != ref)))
