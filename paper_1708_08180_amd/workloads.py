"""Seeded synthetic input generators (numpy only).

This module makes images and nothing else: it holds no labeling
arithmetic, and both the GPU path's tests and the CPU oracle's tests take
their inputs from it.  Every generator draws from
``numpy.random.Generator(PCG64(seed))`` so a (recipe, seed) pair names one
image exactly; ``digest`` gives its SHA-256 for logs.

The paper measures on binarized photographs (Sec. III); those are replaced
here by synthetic masks with the same role: noise fields of controlled
density and grain, smoothed blobs, and adversarial long-chain structures.

Recipes
-------
* ``bernoulli(H, W, p, seed, g)``: a (ceil(H/g) x ceil(W/g)) field of
  i.i.d. Bernoulli(p) cells, each cell repeated over a g x g block, cropped.
* ``smoothed_noise(H, W, sigma, seed)``: float32 standard normal noise,
  Gaussian-filtered (``scipy.ndimage.gaussian_filter``, reflect borders),
  thresholded at its own median (about half foreground).
* ``serpentine(H, W)``: even rows fully set; odd row y holds a single
  connector pixel at x = W-1 when (y // 2) is even, else at x = 0.  One
  component under 4- and 8-connectivity.
* ``spiral(H, W)``: one inward square spiral of path width 1 and gap 1
  starting at (0, 0).  One component.
* ``rings(H, W)``: nested one-pixel square rings with a one-pixel gap; each
  ring is its own component.
* ``batch_spec`` / ``batch_images``: the mixed batch workload (sizes drawn
  from five camera resolutions, half noise and half smoothed masks).
* ``CameraStream``: moving filled ellipses plus 1% salt noise, one frame at
  a time, for the served workload.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np

FG = 1  # value written for foreground pixels


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def digest(img: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(img).tobytes()).hexdigest()


def bernoulli(H: int, W: int, p: float, seed: int, g: int = 1, fg: int = FG) -> np.ndarray:
    rng = rng_for(seed)
    hb, wb = -(-H // g), -(-W // g)
    field = (rng.random((hb, wb)) < p).astype(np.uint8)
    if g > 1:
        field = np.repeat(np.repeat(field, g, axis=0), g, axis=1)
    out = field[:H, :W] * np.uint8(fg)
    return np.ascontiguousarray(out)


def sweep_seed(p: float, g: int) -> int:
    """Seed of one cell of the 4096^2 density x granularity sweep."""
    return 20000 + 100 * int(round(10 * p)) + int(g)


SWEEP_P = (0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9)
SWEEP_G = (1, 2, 4, 8, 16)


def smoothed_noise(H: int, W: int, sigma: float, seed: int, fg: int = FG) -> np.ndarray:
    from scipy import ndimage

    rng = rng_for(seed)
    z = rng.standard_normal((H, W), dtype=np.float32)
    z = ndimage.gaussian_filter(z, sigma, mode="reflect")
    thr = np.median(z)
    return ((z > thr).astype(np.uint8) * np.uint8(fg))


def serpentine(H: int, W: int, fg: int = FG) -> np.ndarray:
    img = np.zeros((H, W), dtype=np.uint8)
    img[0::2, :] = fg
    for y in range(1, H, 2):
        img[y, W - 1 if (y // 2) % 2 == 0 else 0] = fg
    return img


def column_serpentine(H: int, W: int, fg: int = FG) -> np.ndarray:
    return np.ascontiguousarray(serpentine(W, H, fg).T)


def spiral(H: int, W: int, fg: int = FG) -> np.ndarray:
    img = np.zeros((H, W), dtype=np.uint8)
    t = 0
    while True:
        top, left, bottom, right = t, t, H - 1 - t, W - 1 - t
        if top > bottom or left > right:
            break
        img[top, left:right + 1] = fg
        if bottom == top:
            break
        img[top:bottom + 1, right] = fg
        if right == left:
            break
        img[bottom, left:right + 1] = fg
        if bottom - top < 2:
            break
        img[top + 2:bottom + 1, left] = fg
        if top + 2 > bottom - 2 or left + 2 > right - 2:
            break
        img[top + 2, left + 1] = fg  # connector into the next inner layer
        t += 2
    return img


def rings(H: int, W: int, fg: int = FG) -> np.ndarray:
    img = np.zeros((H, W), dtype=np.uint8)
    t = 0
    while True:
        top, left, bottom, right = t, t, H - 1 - t, W - 1 - t
        if top > bottom or left > right:
            break
        img[top, left:right + 1] = fg
        img[bottom, left:right + 1] = fg
        img[top:bottom + 1, left] = fg
        img[top:bottom + 1, right] = fg
        t += 2
    return img


def ring_corners(H: int, W: int):
    """Top-left corners (y, x) of the rings drawn by ``rings``."""
    out = []
    t = 0
    while t <= H - 1 - t and t <= W - 1 - t:
        out.append((t, t))
        t += 2
    return out


def checkerboard(H: int, W: int, parity: int = 0, fg: int = FG) -> np.ndarray:
    yy, xx = np.indices((H, W))
    return (((yy + xx) % 2 == parity).astype(np.uint8) * np.uint8(fg))


# ---------------------------------------------------------------- batches

BATCH_SIZES = ((240, 320), (480, 640), (720, 1280), (1080, 1920), (2160, 3840))  # (H, W)


@dataclass(frozen=True)
class ImageSpec:
    index: int
    H: int
    W: int
    kind: str      # "bernoulli" or "smoothed"
    param: float   # p for bernoulli, sigma for smoothed
    seed: int


def batch_spec(n: int = 512, seed: int = 40000, sizes=BATCH_SIZES):
    """Mixed batch: sizes uniform over ``sizes``; even indices Bernoulli(p~U[0.2,0.8]),
    odd indices smoothed noise with sigma~U[2,8] thresholded at its median."""
    rng = rng_for(seed)
    specs = []
    for i in range(n):
        H, W = sizes[int(rng.integers(len(sizes)))]
        if i % 2 == 0:
            specs.append(ImageSpec(i, H, W, "bernoulli", float(rng.uniform(0.2, 0.8)), seed + 1 + i))
        else:
            specs.append(ImageSpec(i, H, W, "smoothed", float(rng.uniform(2.0, 8.0)), seed + 1 + i))
    return specs


def make_image(spec: ImageSpec) -> np.ndarray:
    if spec.kind == "bernoulli":
        return bernoulli(spec.H, spec.W, spec.param, spec.seed)
    return smoothed_noise(spec.H, spec.W, spec.param, spec.seed)


def batch_images(specs, workers: int = 0):
    """Render a list of ``ImageSpec``; ``workers`` > 1 spreads them over processes."""
    if workers and workers > 1 and len(specs) > 1:
        import multiprocessing
        from concurrent.futures import ProcessPoolExecutor

        # spawn: the workers must not inherit a parent's GPU state
        with ProcessPoolExecutor(max_workers=workers,
                                 mp_context=multiprocessing.get_context("spawn")) as ex:
            return list(ex.map(make_image, specs, chunksize=4))
    return [make_image(s) for s in specs]


# ---------------------------------------------------------------- cameras

class CameraStream:
    """Binary foreground masks of moving filled ellipses plus salt noise.

    ``n_blobs`` ~ U{20..200}; semi-axes ~ U[5, 80] px; centres and angles
    follow seeded random walks (reflecting at the frame border); each pixel
    is additionally set with probability ``salt``.
    """

    def __init__(self, H: int, W: int, seed: int, salt: float = 0.01):
        self.H, self.W, self.salt = H, W, salt
        self.rng = rng_for(seed)
        n = int(self.rng.integers(20, 201))
        self.a = self.rng.uniform(5, 80, n)
        self.b = self.rng.uniform(5, 80, n)
        self.cy = self.rng.uniform(0, H, n)
        self.cx = self.rng.uniform(0, W, n)
        self.th = self.rng.uniform(0, math.pi, n)
        self.n = n

    def step(self) -> np.ndarray:
        rng, H, W = self.rng, self.H, self.W
        self.cy += rng.normal(0, 3.0, self.n)
        self.cx += rng.normal(0, 3.0, self.n)
        self.th += rng.normal(0, 0.05, self.n)
        self.cy = np.where(self.cy < 0, -self.cy, np.where(self.cy >= H, 2 * (H - 1) - self.cy, self.cy))
        self.cx = np.where(self.cx < 0, -self.cx, np.where(self.cx >= W, 2 * (W - 1) - self.cx, self.cx))
        img = (rng.random((H, W), dtype=np.float32) < self.salt).astype(np.uint8)
        for k in range(self.n):
            r = max(self.a[k], self.b[k])
            y0, y1 = max(0, int(self.cy[k] - r)), min(H, int(self.cy[k] + r) + 1)
            x0, x1 = max(0, int(self.cx[k] - r)), min(W, int(self.cx[k] + r) + 1)
            if y0 >= y1 or x0 >= x1:
                continue
            yy = np.arange(y0, y1, dtype=np.float32)[:, None] - np.float32(self.cy[k])
            xx = np.arange(x0, x1, dtype=np.float32)[None, :] - np.float32(self.cx[k])
            c, s = math.cos(self.th[k]), math.sin(self.th[k])
            u = (xx * c + yy * s) / self.a[k]
            v = (-xx * s + yy * c) / self.b[k]
            img[y0:y1, x0:x1] |= (u * u + v * v <= 1.0).astype(np.uint8)
        return img


CAMERA_SHAPES = ((1080, 1920), (1080, 1920), (2160, 3840), (2160, 3840))


def camera_streams(seed_base: int = 50000, shapes=CAMERA_SHAPES):
    return [CameraStream(H, W, seed_base + i) for i, (H, W) in enumerate(shapes)]
