"""GPU parity at the full workload sizes (4096^2 sweep, 8192^2 structured
cases), in the launch configuration the benchmark times (library defaults
through ccl_label_2d).  Bit-exact against the oracle on every pixel."""
import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import workloads as wl
from tests.gpu_util import gpu_label, say

pytestmark = pytest.mark.gpu


def _full(img, conn, what):
    say("full %s %dx%d conn=%d" % (what, img.shape[0], img.shape[1], conn))
    got = gpu_label(img, conn, plain=True)
    want = oracle.label(img, conn)
    n_bad = int(np.count_nonzero(got != want))
    assert n_bad == 0, "%s conn=%d: %d mismatching pixels" % (what, conn, n_bad)


@pytest.mark.parametrize("g", wl.SWEEP_G)
@pytest.mark.parametrize("p", wl.SWEEP_P)
def test_sweep_4096(p, g):
    img = wl.bernoulli(4096, 4096, p, wl.sweep_seed(p, g), g)
    for conn in (8, 4):
        _full(img, conn, "sweep p=%.1f g=%d" % (p, g))


@pytest.mark.parametrize("case", ["smoothed", "serpentine", "spiral"])
def test_structured_8192(case):
    if case == "smoothed":
        img = wl.smoothed_noise(8192, 8192, 4.0, 30001)
    elif case == "serpentine":
        img = wl.serpentine(8192, 8192)
    else:
        img = wl.spiral(8192, 8192)
    _full(img, 8, case)
    if case != "smoothed":
        _full(img, 4, case)
