"""Independent pins for connected-components labels.

Nothing here runs a flood fill or a union-find: the references are a
boolean transitive closure of the pixel adjacency matrix (brute force, tiny
images only), closed forms of hand-built patterns, invariants that any
canonical labeling must satisfy, and ``scipy.ndimage.label`` renumbered to
the canonical form.  Every check takes the labeling function under test as
an argument so the same pins serve the oracle, planted oracle mutants and
the GPU path.

Canonical form (Introduction; the smaller-index-wins merge of Sec. II-A-3):
label = 0 for background, else 1 + the smallest raster index y*W + x in the
pixel's component.
"""
from __future__ import annotations

import itertools

import numpy as np


# ------------------------------------------------------------ brute force

def neighbour_matrix(H: int, W: int, conn: int) -> np.ndarray:
    """n x n boolean matrix: True where two distinct pixels are neighbours."""
    n = H * W
    ys, xs = np.divmod(np.arange(n), W)
    dy = np.abs(ys[:, None] - ys[None, :])
    dx = np.abs(xs[:, None] - xs[None, :])
    if conn == 4:
        adj = (dy + dx) == 1
    elif conn == 8:
        adj = (np.maximum(dy, dx) == 1)
    else:
        raise ValueError(conn)
    return adj


def closure_labels(imgs: np.ndarray, conn: int, mode: str = "binary") -> np.ndarray:
    """Canonical labels of a stack of tiny images by transitive closure.

    imgs: (B, H, W) uint8.  mode "binary": nonzero pixels join nonzero
    neighbours; mode "equal": pixels join neighbours of equal value.
    """
    B, H, W = imgs.shape
    n = H * W
    flat = imgs.reshape(B, n)
    nb = neighbour_matrix(H, W, conn)
    if mode == "binary":
        fg = flat != 0
        same = fg[:, :, None] & fg[:, None, :]
        active = fg
    else:
        same = flat[:, :, None] == flat[:, None, :]
        active = np.ones_like(flat, dtype=bool)
    reach = (same & nb[None]) | np.eye(n, dtype=bool)[None]
    reach &= active[:, :, None]
    r = reach.astype(np.float32)
    steps = max(1, int(np.ceil(np.log2(max(n, 2)))))
    for _ in range(steps):
        r = (np.matmul(r, r) > 0).astype(np.float32)
    rb = r > 0
    first = np.argmax(rb, axis=2)  # smallest reachable index
    lab = np.where(active, first + 1, 0).astype(np.uint32)
    return lab.reshape(B, H, W)


def all_images(H: int, W: int) -> np.ndarray:
    n = H * W
    codes = np.arange(1 << n, dtype=np.uint32)
    bits = (codes[:, None] >> np.arange(n, dtype=np.uint32)[None, :]) & 1
    return bits.astype(np.uint8).reshape(-1, H, W)


def check_exhaustive(label_fn, H: int, W: int, conn: int, fg: int = 1):
    imgs = all_images(H, W) * np.uint8(fg)
    want = closure_labels(imgs, conn)
    for k in range(imgs.shape[0]):
        got = label_fn(imgs[k], conn)
        if not np.array_equal(got, want[k]):
            raise AssertionError(
                "mismatch on %dx%d image #%d conn=%d\nimg=\n%s\ngot=\n%s\nwant=\n%s"
                % (H, W, k, conn, imgs[k], got, want[k]))


# ------------------------------------------------------------ invariants

def check_invariants(img: np.ndarray, lab: np.ndarray):
    """Properties every canonical labeling has, whatever the connectivity."""
    H, W = img.shape
    fg = img != 0
    assert lab.shape == img.shape and lab.dtype == np.uint32
    assert np.all(lab[~fg] == 0), "background must be 0"
    assert np.all(lab[fg] >= 1), "foreground must be >= 1"
    idx = np.arange(H * W, dtype=np.int64).reshape(H, W)
    l64 = lab.astype(np.int64)
    assert np.all(l64[fg] <= idx[fg] + 1), "label exceeds 1 + own index"
    roots = l64[fg] - 1
    # the root pixel carries its own label (idempotence)
    assert np.all(lab.reshape(-1)[roots] == lab[fg]), "root not self-labeled"
    assert np.all(fg.reshape(-1)[roots]), "root is not foreground"


def component_count(lab: np.ndarray) -> int:
    H, W = lab.shape
    idx = np.arange(H * W, dtype=np.int64).reshape(H, W)
    return int(np.count_nonzero(lab.astype(np.int64) == idx + 1))


def check_neighbour_consistency(img: np.ndarray, lab: np.ndarray, conn: int):
    """Adjacent foreground pixels share a label (labels constant on components)."""
    fg = img != 0
    shifts = [(0, 1), (1, 0)] if conn == 4 else [(0, 1), (1, 0), (1, 1), (1, -1)]
    H, W = img.shape
    for dy, dx in shifts:
        y0, y1 = 0, H - dy
        xa0, xa1 = max(0, -dx), W - max(0, dx)
        a_fg = fg[y0:y1, xa0:xa1]
        b_fg = fg[y0 + dy:y1 + dy, xa0 + dx:xa1 + dx]
        a_l = lab[y0:y1, xa0:xa1]
        b_l = lab[y0 + dy:y1 + dy, xa0 + dx:xa1 + dx]
        both = a_fg & b_fg
        assert np.array_equal(a_l[both], b_l[both]), "adjacent pixels disagree (shift %r)" % ((dy, dx),)


# ------------------------------------------------------------ library

def scipy_canonical(img: np.ndarray, conn: int) -> np.ndarray:
    """scipy.ndimage.label renumbered to 1 + min raster index."""
    from scipy import ndimage

    st = ndimage.generate_binary_structure(2, 1 if conn == 4 else 2)
    lab, n = ndimage.label(img != 0, structure=st)
    H, W = img.shape
    flat = lab.reshape(-1)
    mins = np.full(n + 1, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(mins, flat, np.arange(H * W, dtype=np.int64))
    mapped = np.where(flat > 0, mins[flat] + 1, 0).astype(np.uint32)
    return mapped.reshape(H, W)


# ------------------------------------------------------------ closed forms

def closed_form_cases(H: int, W: int):
    """Yield (name, img, conn, expected_labels) for patterns with closed forms."""
    from paper_1708_08180_amd import workloads as wl

    idx = np.arange(H * W, dtype=np.int64).reshape(H, W)
    yy, xx = np.indices((H, W))
    z = np.zeros((H, W), dtype=np.uint32)
    for conn in (4, 8):
        yield "zeros", np.zeros((H, W), np.uint8), conn, z.copy()
        yield "ones", np.ones((H, W), np.uint8), conn, np.ones((H, W), np.uint32)
    # checkerboard with (x+y) even: singletons under 4, one component (label 1) under 8
    cb0 = wl.checkerboard(H, W, 0)
    yield "checker0", cb0, 4, np.where(cb0 != 0, idx + 1, 0).astype(np.uint32)
    if H >= 2 and W >= 2:
        yield "checker0", cb0, 8, np.where(cb0 != 0, 1, 0).astype(np.uint32)
        cb1 = wl.checkerboard(H, W, 1)
        yield "checker1", cb1, 8, np.where(cb1 != 0, 2, 0).astype(np.uint32)
    # horizontal stripes on even rows: label 1 + y*W
    hs = ((yy % 2) == 0).astype(np.uint8)
    vs = ((xx % 2) == 0).astype(np.uint8)
    dots = (((yy % 2) == 0) & ((xx % 2) == 0)).astype(np.uint8)
    for conn in (4, 8):
        yield "hstripes", hs, conn, np.where(hs != 0, yy * W + 1, 0).astype(np.uint32)
        yield "vstripes", vs, conn, np.where(vs != 0, xx + 1, 0).astype(np.uint32)
        yield "dots", dots, conn, np.where(dots != 0, idx + 1, 0).astype(np.uint32)
    # main diagonal: one component under 8 (label 1), singletons under 4
    dg = (yy == xx).astype(np.uint8)
    yield "diag", dg, 8, np.where(dg != 0, 1, 0).astype(np.uint32)
    yield "diag", dg, 4, np.where(dg != 0, idx + 1, 0).astype(np.uint32)
    # anti-diagonal x + y == W - 1: under 8 one component whose minimum pixel is (0, W-1)
    ad = (xx + yy == W - 1).astype(np.uint8)
    if ad.any():
        first = int(np.flatnonzero(ad.reshape(-1))[0])
        yield "antidiag", ad, 8, np.where(ad != 0, first + 1, 0).astype(np.uint32)
        yield "antidiag", ad, 4, np.where(ad != 0, idx + 1, 0).astype(np.uint32)
    # serpentine, column serpentine and spiral: one component with label 1
    for name, img in (("serpentine", wl.serpentine(H, W)),
                      ("colserpentine", wl.column_serpentine(H, W)),
                      ("spiral", wl.spiral(H, W))):
        for conn in (4, 8):
            yield name, img, conn, np.where(img != 0, 1, 0).astype(np.uint32)
    # nested rings: each ring labeled 1 + raster index of its top-left corner
    rg = wl.rings(H, W)
    want = np.zeros((H, W), np.uint32)
    t = 0
    for (cy, cx) in wl.ring_corners(H, W):
        top, left, bottom, right = cy, cx, H - 1 - cy, W - 1 - cx
        lab = cy * W + cx + 1
        want[top, left:right + 1] = lab
        want[bottom, left:right + 1] = lab
        want[top:bottom + 1, left] = lab
        want[top:bottom + 1, right] = lab
        t += 1
    for conn in (4, 8):
        yield "rings", rg, conn, want.copy()


def check_closed_forms(label_fn, shapes=((1, 1), (1, 7), (7, 1), (5, 9), (9, 5), (16, 16), (17, 33), (64, 70))):
    for (H, W) in shapes:
        for name, img, conn, want in closed_form_cases(H, W):
            got = label_fn(img, conn)
            if not np.array_equal(got, want):
                bad = np.argwhere(got != want)[:5]
                raise AssertionError("closed form %s %dx%d conn=%d differs at %s" % (name, H, W, conn, bad.tolist()))


def check_pitch(label_fn_pitched, label_fn, H=13, W=29, pad=7, seed=5):
    """Labels must not depend on the row pitch: raster index uses W."""
    from paper_1708_08180_amd import workloads as wl

    img = wl.bernoulli(H, W, 0.55, seed)
    big = np.full((H, W + pad), 255, dtype=np.uint8)
    big[:, :W] = img
    view = big[:, :W]
    for conn in (4, 8):
        a = label_fn_pitched(view, conn)
        b = label_fn(np.ascontiguousarray(img), conn)
        if not np.array_equal(a, b):
            raise AssertionError("pitch changes labels (conn=%d)" % conn)


def shapes_upto(n: int):
    for h, w in itertools.product(range(1, n + 1), repeat=2):
        if h * w <= n:
            yield h, w


def check_mixed_values(label_fn, H=24, W=31, seed=9):
    """Any nonzero value is foreground: pixels of different nonzero values join."""
    from paper_1708_08180_amd import workloads as wl

    rng = wl.rng_for(seed)
    vals = rng.integers(1, 256, size=(H, W)).astype(np.uint8)
    mask = wl.bernoulli(H, W, 0.6, seed + 1)
    img = (vals * mask).astype(np.uint8)
    for conn in (4, 8):
        got = label_fn(img, conn)
        want = label_fn(mask, conn)
        if not np.array_equal(got, want):
            raise AssertionError("labels depend on the nonzero value (conn=%d)" % conn)
        ref = closure_labels(mask[None, :8, :8], conn)[0]
        if not np.array_equal(label_fn(np.ascontiguousarray(img[:8, :8]), conn), ref):
            raise AssertionError("mixed-value 8x8 crop differs from closure (conn=%d)" % conn)
