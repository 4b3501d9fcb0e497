"""Grid-to-tile maps of the symmetric-product kernels, checked on the host for every size the launchers
accept: every upper-triangle tile of every block is computed by exactly one workgroup, workgroups
beyond the last tile map to nothing (the kernel returns at once), and every index lies inside the
block's tile grid."""
import numpy as np
import pytest

from paper_2106_02682_amd import vemb


def _check(grid, m, count, tiles):
    live = m[m[:, 0] == 1]
    assert np.all(m[m[:, 0] == 0, 1:] == -1)
    b, ti, tj = live[:, 1], live[:, 2], live[:, 3]
    assert np.all((b >= 0) & (b < count))
    assert np.all((ti >= 0) & (ti <= tj) & (tj < tiles))
    keys = (b.astype(np.int64) * tiles + ti) * tiles + tj
    assert len(np.unique(keys)) == len(keys) == count * tiles * (tiles + 1) // 2


def test_single_matrix_products_every_size():
    for n in range(16, 4097, 16):
        grid, m = vemb.tile_map(0, n)
        tiles = n // 16
        assert grid == tiles * (tiles + 1) // 2
        _check(grid, m, 1, tiles)


@pytest.mark.parametrize("n", [64, 128, 192, 256])
def test_batched_products_every_count(n):
    tiles = n // 64
    for count in list(range(1, 70)) + [127, 1029, 1100, 2999]:
        grid, m = vemb.tile_map(1, n, count)
        assert grid == count * tiles * (tiles + 1) // 2
        _check(grid, m, count, tiles)


def test_rejects_sizes_the_kernels_do_not_take():
    for kind, n, count in [(0, 40, 1), (0, 4112, 1), (1, 96, 3), (1, 320, 3), (1, 256, 0), (2, 64, 1)]:
        with pytest.raises(vemb.VembError):
            vemb.tile_map(kind, n, count)
