"""Host checks of the seeded patch placement of the refined workload: it
delivers the requested number of boxes, every box is a valid hierarchy box
(4-aligned, inside the margin, no overlap) and lies on a flagged block or,
once the flagged blocks are full, on the buffer layers grown around them."""
import numpy as np
import pytest

import lbm_inputs


def _dilate(mask, k):
    out = mask.copy()
    for _ in range(k):
        g = out.copy()
        for ax in range(3):
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax], hi[ax] = slice(1, None), slice(None, -1)
            g[tuple(lo)] |= out[tuple(hi)]
            g[tuple(hi)] |= out[tuple(lo)]
        out = g
    return out


def _check(boxes, mask, n, edges, count):
    assert len(boxes) == count
    taken = np.zeros((n[2], n[1], n[0]), dtype=np.int32)
    grown = 0
    for lo, hi in boxes:
        e = hi[0] - lo[0]
        assert hi[1] - lo[1] == e and hi[2] - lo[2] == e and 2 * e in edges
        assert all(v % 4 == 0 for v in lo) and all(lo[a] >= 1 and hi[a] <= n[a] - 1 for a in range(3))
        taken[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += 1
        # blocks the box overlaps
        sl = tuple(slice(lo[a] // 8, (hi[a] - 1) // 8 + 1) for a in (2, 1, 0))
        k = 0
        while not _dilate(mask, k)[sl].any():
            k += 1
        grown = max(grown, k)
    assert taken.max() == 1, "boxes overlap"
    return grown


def test_place_patches_delivers_count_on_flagged_blocks():
    """The full-size test's mask: 20% of the blocks below z = 96 flagged;
    399 boxes, all within the flagged blocks' neighbourhood."""
    n = (256, 256, 256)
    nb = 32
    mask = (lbm_inputs.uniform(11, nb ** 3) < 0.2).reshape(nb, nb, nb)
    mask[12:] = False
    boxes = lbm_inputs.place_patches(mask, 8, n, count=399, seed=7)
    grown = _check(boxes, mask, n, (16, 24, 32, 48), 399)
    assert grown == 0, "a sparse 20% mask has room next to its flagged blocks"
    fine = 8 * sum(np.prod([hi[a] - lo[a] for a in range(3)]) for lo, hi in boxes)
    assert 14e6 < fine < 19e6          # ~400 x the mean volume of cubes of edge 16..48
    assert boxes == lbm_inputs.place_patches(mask, 8, n, count=399, seed=7)   # seeded


def test_place_patches_grows_the_mask_when_full():
    """A single flagged block cannot take 60 boxes: the placement grows the
    mask block by block and still delivers them, each as close as the
    buffer layers allow."""
    n = (128, 128, 128)
    mask = np.zeros((16, 16, 16), dtype=bool)
    mask[8, 8, 8] = True
    boxes = lbm_inputs.place_patches(mask, 8, n, count=60, seed=3)
    grown = _check(boxes, mask, n, (16, 24, 32, 48), 60)
    assert grown >= 1


def test_place_patches_reports_a_grid_too_small():
    mask = np.ones((2, 2, 2), dtype=bool)
    with pytest.raises(ValueError):
        lbm_inputs.place_patches(mask, 8, (16, 16, 16), count=50, seed=1)
