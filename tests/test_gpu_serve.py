"""GPU tests of the served form: every frame's labels are the same in the mix
as alone (and equal the oracle), under small HBM budgets that force slot
reuse, in batched and in plain mode."""
import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import binding, serve
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

SMALL_CAMS = ((240, 320), (240, 320), (480, 640), (480, 640))


@pytest.fixture(scope="module")
def rings():
    return serve.make_rings(SMALL_CAMS, ring=4, seed_base=50100)


def _checker(conn, seen):
    import torch

    def check(tag, frame_h, labels):
        want = oracle.label(frame_h, conn)
        assert np.array_equal(labels, want), "frame %d differs from the oracle" % tag
        alone = binding.label_plain(torch.from_numpy(frame_h).cuda(), conn)
        torch.cuda.synchronize()
        assert np.array_equal(labels, alone.cpu().numpy().view(np.uint32)), "frame %d: mix != alone" % tag
        seen.append(tag)
    return check


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("conn", [8, 4])
def test_serve_frames_exact(rings, plain, conn):
    seen = []
    res = serve.run(rings, rate=3000.0, duration_s=0.15, plain=plain, conn=conn,
                    check=_checker(conn, seen))
    say("serve %s conn=%d: %d frames, %.0f fps, p99 %.3f ms" % (res.mode, conn, res.frames, res.fps, res.p99_ms))
    assert res.frames > 100 and len(seen) >= 3


def test_serve_tiny_budget_recycles_slots(rings):
    seen = []
    px = max(h * w for h, w in SMALL_CAMS)
    res = serve.run(rings, rate=5000.0, duration_s=0.1, plain=False, conn=8, n_workers=2,
                    max_batch=4, hbm_budget=3 * px * 4, check=_checker(8, seen))
    assert res.frames > 100


def test_serve_shutdown_with_frames_in_flight(rings):
    srv = binding.Server(480 * 640, 8 * 480 * 640 * 4, n_workers=2, max_batch=4)
    for i in range(50):
        assert srv.submit(rings[i % 4][0][1], i) == 0
    srv.close()   # drops frames still waiting for a slot, waits for the rest


def test_serve_rejects_oversized_frame(rings):
    srv = binding.Server(240 * 320, 4 * 240 * 320 * 4, n_workers=1, max_batch=2)
    assert srv.submit(rings[2][0][1], 0) == 6       # 480x640 > max_frame_pixels
    srv.close()
