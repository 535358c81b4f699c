"""GPU parity of the batched form: every image of a batch must equal the
oracle and the single-image entry point bit for bit, across repeated calls
(graph replays and node updates, calls queued back to back) and ragged
image sets."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import binding
from paper_1708_08180_amd import workloads as wl
from tests.gpu_util import CONFIGS, say

pytestmark = pytest.mark.gpu

SMALL_SIZES = ((1, 1), (3, 70), (70, 3), (64, 64), (65, 129), (240, 320), (100, 333), (480, 640))


def _mixed_images(n, seed, sizes=SMALL_SIZES):
    rng = wl.rng_for(seed)
    imgs = []
    for i in range(n):
        H, W = sizes[int(rng.integers(len(sizes)))]
        if i % 3 == 0:
            imgs.append(wl.bernoulli(H, W, float(rng.uniform(0.2, 0.8)), seed * 1000 + i))
        elif i % 3 == 1:
            imgs.append(wl.smoothed_noise(H, W, float(rng.uniform(2, 8)), seed * 1000 + i))
        else:
            imgs.append(wl.bernoulli(H, W, 0.5, seed * 1000 + i, g=3))
    return imgs


def _run(ctx, imgs, conn):
    import torch

    d = [torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in imgs]
    outs = ctx.label(d, conn)
    torch.cuda.synchronize()
    return [o.cpu().numpy().view(np.uint32) for o in outs]


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("conn", [8, 4])
def test_batch_matches_oracle(conn, use_graph):
    ctx = binding.BatchContext(64, 64 * 480 * 640, use_graph=use_graph)
    for call, seed in enumerate((1, 2, 3)):       # several calls: graph replay and node updates
        imgs = _mixed_images(40 + 7 * call, seed)
        say("batch call %d conn=%d graph=%s n=%d" % (call, conn, use_graph, len(imgs)))
        got = _run(ctx, imgs, conn)
        for k, (im, g) in enumerate(zip(imgs, got)):
            want = oracle.label(im, conn)
            assert np.array_equal(g, want), "image %d (%dx%d) differs" % (k, im.shape[0], im.shape[1])
    ctx.close()


@pytest.mark.parametrize("config", CONFIGS)
def test_batch_tile_configs(config):
    ctx = binding.BatchContext(16, 16 * 480 * 640, config=config)
    imgs = _mixed_images(16, 9)
    for conn in (8, 4):
        got = _run(ctx, imgs, conn)
        for im, g in zip(imgs, got):
            assert np.array_equal(g, oracle.label(im, conn))
    ctx.close()


def test_batch_equals_single_image_path():
    import torch

    imgs = _mixed_images(24, 5, sizes=((720, 1280), (1080, 1920), (240, 320)))
    ctx = binding.BatchContext(24, sum(im.size for im in imgs))
    got = _run(ctx, imgs, 8)
    for im, g in zip(imgs, got):
        single = binding.label_plain(torch.from_numpy(im).cuda(), 8)
        torch.cuda.synchronize()
        assert np.array_equal(g, single.cpu().numpy().view(np.uint32))
    ctx.close()


def test_batch_single_image_and_sizes_change():
    ctx = binding.BatchContext(8, 8 * 1080 * 1920)
    for seed, n in ((11, 1), (12, 8), (13, 2), (14, 1)):
        imgs = _mixed_images(n, seed, sizes=((1080, 1920), (17, 33), (1, 1)))
        for conn in (8, 4):
            got = _run(ctx, imgs, conn)
            for im, g in zip(imgs, got):
                assert np.array_equal(g, oracle.label(im, conn))
    ctx.close()


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_back_to_back_calls_with_changing_shapes(use_graph):
    """Calls queued without a host synchronization in between, alternating
    batch shapes (so graph nodes are updated while earlier calls may still
    be queued) and repeating one shape (pure replays); every call has its
    own outputs and is checked after one final synchronization."""
    import torch

    ctx = binding.BatchContext(48, 48 * 480 * 640, use_graph=use_graph)
    plan = [(21, 5), (22, 40), (21, 5), (21, 5), (23, 1), (24, 17), (22, 40)]
    sets = {}
    for seed, n in set(plan):
        sets[seed] = _mixed_images(n, seed)
    dev = {seed: [torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in imgs]
           for seed, imgs in sets.items()}
    torch.cuda.synchronize()
    results = []
    for k, (seed, n) in enumerate(plan):
        conn = 8 if k % 2 == 0 else 4
        say("queued call %d seed=%d n=%d conn=%d graph=%s" % (k, seed, n, conn, use_graph))
        results.append((seed, conn, ctx.label(dev[seed], conn)))
    torch.cuda.synchronize()
    for seed, conn, outs in results:
        for im, o in zip(sets[seed], outs):
            assert np.array_equal(o.cpu().numpy().view(np.uint32), oracle.label(im, conn))
    ctx.close()


def test_batch_capacity_errors():
    import torch

    ctx = binding.BatchContext(2, 64 * 64)
    d = [torch.zeros((64, 64), dtype=torch.uint8, device="cuda") for _ in range(3)]
    with pytest.raises(binding.CclError) as e:
        ctx.label(d, 8)
    assert e.value.status == 6
    big = [torch.zeros((1024, 1024), dtype=torch.uint8, device="cuda")]
    with pytest.raises(binding.CclError) as e:
        ctx.label(big, 8)
    assert e.value.status == 6
    ctx.close()


def test_autotune_records_a_supported_config():
    import torch

    img = wl.bernoulli(512, 512, 0.5, 3)
    d = torch.from_numpy(img).cuda()
    binding.tuning_clear()
    best, ms = binding.autotune(d, 8, reps=2)
    assert best in {(t, w) for t in (16, 32, 64) for w in (1, 2, 4, 8, 16)}
    assert ms > 0
    assert binding.tuning_get(512, 512, 8) == best
    out = binding.label_plain(d, 8)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.label(img, 8))
    binding.tuning_clear()


@pytest.mark.parametrize("conn", [8, 4])
def test_batch_mixed_workload_sizes(conn):
    """Images of the batched workload's recipe and all its sizes, 3840x2160
    included, checked one by one against the oracle."""
    specs = wl.batch_spec(10, 40000)
    sizes = wl.BATCH_SIZES
    # the recipe's draws, with the sizes set so that every size appears twice
    specs = [dataclasses.replace(s, H=sizes[k % 5][0], W=sizes[k % 5][1]) for k, s in enumerate(specs)]
    imgs = wl.batch_images(specs)
    assert {im.shape for im in imgs} == set(sizes)
    ctx = binding.BatchContext(len(imgs), sum(im.size for im in imgs))
    got = _run(ctx, imgs, conn)
    for k, (im, g) in enumerate(zip(imgs, got)):
        say("batch mixed image %d %dx%d conn=%d" % (k, im.shape[0], im.shape[1], conn))
        want = oracle.label(im, conn)
        assert np.array_equal(g, want), "image %d (%dx%d) differs" % (k, im.shape[0], im.shape[1])
    ctx.close()


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_autotune_per_connectivity(use_graph):
    """ccl_ctx_autotune times every configuration on the batch, keeps the
    fastest per connectivity, and the context's later calls (switched
    kernels, rebuilt graphs) still equal the oracle on every image."""
    import torch

    ctx = binding.BatchContext(48, 48 * 480 * 640, use_graph=use_graph)
    imgs = _mixed_images(40, 21)
    d = [torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in imgs]
    for conn in (8, 4):
        before = ctx.config(conn)
        best, ms = ctx.autotune(d, conn, reps=2)
        say("autotune conn=%d graph=%s: %s -> %s (%.3f ms)" % (conn, use_graph, before, best, ms))
        assert ms > 0 and ctx.config(conn) == best
        assert best in {(t, w) for t in (16, 32, 64, 128) for w in (1, 2, 4, 8, 16)}
        for seed in (22, 23):
            batch = _mixed_images(30 + seed % 7, seed)
            got = _run(ctx, batch, conn)
            for k, (im, g) in enumerate(zip(batch, got)):
                assert np.array_equal(g, oracle.label(im, conn)), "conn %d image %d differs" % (conn, k)
    ctx.close()


def test_batch_autotune_keeps_a_fixed_config():
    import torch

    ctx = binding.BatchContext(8, 8 * 240 * 320, config=(32, 4))
    d = [torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in _mixed_images(4, 24)]
    with pytest.raises(binding.CclError):
        ctx.autotune(d, 8)
    assert ctx.config(8) == (32, 4) and ctx.config(4) == (32, 4)
    ctx.close()
