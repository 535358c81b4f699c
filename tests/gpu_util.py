"""Helpers shared by the GPU tests: numpy image in, numpy uint32 labels out,
always through the C ABI of libccl (never through the oracle)."""
from __future__ import annotations

import sys

import numpy as np

# every compiled tile configuration (tile_h, waves)
CONFIGS = [(64, 4), (64, 8), (64, 16), (64, 1), (64, 2), (128, 8), (128, 4), (128, 16), (128, 2), (32, 1), (32, 2), (32, 4), (32, 8),
           (32, 16), (16, 1), (16, 2), (16, 4), (16, 8)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(img: np.ndarray, pad: int = 0):
    """Upload an image; with pad > 0 the rows get a pitch of W + pad bytes."""
    import torch

    H, W = img.shape
    if pad:
        big = torch.full((H, W + pad), 7, dtype=torch.uint8, device="cuda")
        big[:, :W] = torch.from_numpy(np.ascontiguousarray(img)).cuda()
        return big[:, :W]
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def gpu_label(img: np.ndarray, conn: int, config=None, pad: int = 0, plain: bool = False) -> np.ndarray:
    import torch
    from paper_1708_08180_amd import binding

    d = to_dev(img, pad)
    if plain:
        out = binding.label_plain(d, conn)
    else:
        out = binding.label(d, conn, config=config)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def mosaic(tiles: np.ndarray, gap: int = 1) -> np.ndarray:
    """Lay (B, h, w) tiny images on a grid separated by blank rows/columns."""
    B, h, w = tiles.shape
    cols = int(np.ceil(np.sqrt(B)))
    rows = -(-B // cols)
    out = np.zeros((rows * (h + gap), cols * (w + gap)), dtype=np.uint8)
    for k in range(B):
        r, c = divmod(k, cols)
        out[r * (h + gap):r * (h + gap) + h, c * (w + gap):c * (w + gap) + w] = tiles[k]
    return out
