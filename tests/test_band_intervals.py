"""The local merge takes a tile two rows at a time and treats every
connected component of such a band as one interval of columns, found from
the two row masks alone: under 8-connectivity the runs of (top | bottom);
under 4-connectivity those runs split wherever neither row continues across
a column boundary.  Checked here exhaustively on every 2 x 8 binary image,
against the CPU oracle's components, with the same mask formula the kernels
evaluate (written out in integers)."""
import numpy as np
import pytest

import oracle

W = 8


def band_interval_ids(top: int, bot: int, conn8: bool) -> np.ndarray:
    """Interval number of every column of the band (-1: empty column)."""
    m = top | bot
    starts = m & ~(m << 1)
    if not conn8:
        starts |= m & (m << 1) & ~(top & (top << 1)) & ~(bot & (bot << 1))
    ids = np.full(W, -1)
    k = -1
    for c in range(W):
        if (m >> c) & 1:
            k += starts >> c & 1
            ids[c] = k
    return ids


@pytest.mark.parametrize("conn", [8, 4])
def test_band_components_are_mask_intervals(conn):
    bits = ((np.arange(1 << W)[:, None] >> np.arange(W)) & 1).astype(np.uint8)
    for top in range(1 << W):
        for bot in range(1 << W):
            img = np.stack([bits[top], bits[bot]])
            lab = oracle.label(img, conn)
            ids = np.broadcast_to(band_interval_ids(top, bot, conn == 8), (2, W))
            fg = img != 0
            # the component -> interval map and its inverse are both functions
            pairs = set(zip(lab[fg].tolist(), ids[fg].tolist()))
            assert len(pairs) == len({p[0] for p in pairs}) == len({p[1] for p in pairs}), (top, bot, conn)
