"""The neighbour table's size counted on the host (what set_scene allocates
while a batch runs, checked there against the device's own count) against
its definition written out in numpy: per pixel, the depths within dzmm of the
valid readings of its clipped window, [min - dzmm, max + dzmm] inside
[1, 65534].  CPU only (the count is host code)."""
import numpy as np
import pytest

import paper_2008_00326_amd as pk


def brute(depth, wx, wy, dzmm):
    H, W = depth.shape
    total = 0
    for j in range(H):
        for i in range(W):
            win = depth[max(j - wy, 0):j + wy + 1, max(i - wx, 0):i + wx + 1]
            v = win[win > 0]
            if v.size:
                total += min(65534, int(v.max()) + dzmm) - max(1, int(v.min()) - dzmm) + 1
    return total


@pytest.mark.parametrize("seed", range(6))
def test_host_count_matches_the_definition(seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1, 40)), int(rng.integers(1, 50))
    depth = rng.integers(0, 3000, size=(H, W)).astype(np.uint16)
    depth[rng.random((H, W)) < 0.3] = 0                    # missing readings
    if seed == 1:
        depth[:] = 0                                       # nothing observed
    if seed == 2:
        depth[rng.random((H, W)) < 0.5] = 65535            # the top of the range
        depth[0, 0] = 1                                    # and the bottom
    wx, wy, dzmm = int(rng.integers(0, 9)), int(rng.integers(0, 9)), int(rng.integers(0, 40))
    assert pk.table_entries(depth, wx, wy, dzmm) == brute(depth, wx, wy, dzmm)


def test_windows_wider_than_the_image_and_the_refusal():
    depth = np.array([[0, 500, 0], [700, 0, 0]], np.uint16)
    assert pk.table_entries(depth, 40, 40, 10) == 6 * ((700 + 10) - (500 - 10) + 1)
    assert pk.table_entries(depth, 49, 0, 10) == -1        # too wide: set_scene lets the device count
    with pytest.raises(pk.PerchError):
        pk.table_entries(depth, -1, 0, 10)
