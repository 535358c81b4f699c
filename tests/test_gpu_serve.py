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

    # ring frames repeat: the oracle and the stand-alone call run once per
    # distinct frame
    cache = {}

    def check(tag, frame_h, labels):
        key = id(frame_h)
        if key not in cache:
            alone = binding.label_plain(torch.from_numpy(frame_h).cuda(), conn)
            torch.cuda.synchronize()
            cache[key] = (oracle.label(frame_h, conn), alone.cpu().numpy().view(np.uint32))
        want, alone = cache[key]
        assert np.array_equal(labels, want), "frame %d differs from the oracle" % tag
        assert np.array_equal(labels, alone), "frame %d: mix != alone" % tag
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


@pytest.fixture(scope="module")
def camera_rings():
    # the served workload's cameras: 2 x 1920x1080 and 2 x 3840x2160
    return serve.make_rings(ring=3, seed_base=50000)


@pytest.mark.parametrize("plain", [False, True])
def test_serve_full_size_cameras_every_frame(camera_rings, plain):
    """Every completed 1080p and 2160p frame equals the oracle and the same
    frame labeled alone, in the batched mix and in the per-frame loop."""
    seen = []
    res = serve.run(camera_rings, rate=800.0, duration_s=0.05, plain=plain, conn=8,
                    check=_checker(8, seen), check_all=True)
    say("serve full-size %s: %d frames, all %d checked" % (res.mode, res.frames, len(seen)))
    assert res.frames >= 10 and len(seen) == res.frames
    sizes = {camera_rings[c][0][0].shape for c in range(4)}
    assert sizes == {(1080, 1920), (2160, 3840)}


def test_serve_release_rejects_bad_slots(rings):
    """Only a held slot can be released, once."""
    srv = binding.Server(480 * 640, 2 * 480 * 640 * 4, n_workers=1, max_batch=2)
    assert srv.n_slots == 2
    assert srv.submit(rings[2][0][1], 5) == 0
    got = []
    while not got:
        got = srv.poll()
    slot = got[0][2]
    for bad in (-1, 2, 1000, 1 - slot):    # out of range, or the slot no frame holds
        with pytest.raises(binding.CclError):
            srv.release(bad)
    srv.release(slot)
    with pytest.raises(binding.CclError):   # second release of the same slot
        srv.release(slot)
    # the pool still works: both slots admit frames again
    for t in (6, 7):
        assert srv.submit(rings[2][0][1], t) == 0
    done = []
    while len(done) < 2:
        done += srv.poll()
    assert sorted(r[2] for r in done) == [0, 1]
    for r in done:
        srv.release(r[2])
    srv.close()
