"""Pins of the frame-classification oracle (oracle/classify.py; Sec. 4,
Algorithm 1): hand-built frames with known answers and the invariants the
lists must satisfy on random frames."""
import numpy as np
import pytest

import ntc_inputs as I
from oracle import classify as C

BG = 0xFFFF


def test_one_material_everywhere_gives_simple_tiles():
    mat = np.full((8, 16), 3, np.uint16)
    lst, off, simple, cls = C.classify(mat, 5)
    assert list(cls) == [C.SIMPLE] * 4
    assert list(off) == [0, 0, 0, 0, 128, 128] and list(simple) == [0, 0, 0, 128, 0]
    # tile order, row-major inside a tile
    exp = [y * 16 + x for ty in range(2) for tx in range(2) for y in range(4 * ty, 4 * ty + 4)
           for x in range(8 * tx, 8 * tx + 8)]
    assert list(lst) == exp


@pytest.mark.parametrize("n_valid,expect", [(16, C.MIXED), (17, C.SIMPLE), (32, C.SIMPLE), (1, C.MIXED)])
def test_simple_needs_more_than_16_pixels(n_valid, expect):
    mat = np.full((4, 8), BG, np.uint16)
    mat.reshape(-1)[:n_valid] = 2
    lst, off, simple, cls = C.classify(mat, 3)
    assert cls[0] == expect
    assert list(lst) == list(range(n_valid))
    assert simple[2] == (n_valid if expect == C.SIMPLE else 0)


def test_mixed_tile_splits_by_material_in_pixel_order():
    mat = np.full((4, 8), BG, np.uint16)
    mat[0, 0], mat[0, 5], mat[1, 2], mat[3, 7], mat[2, 1] = 1, 0, 1, 0, 1
    lst, off, simple, cls = C.classify(mat, 2)
    assert cls[0] == C.MIXED
    assert list(lst) == [5, 31, 0, 10, 17] and list(off) == [0, 2, 5] and list(simple) == [0, 0]


def test_empty_and_all_background():
    mat = np.full((5, 9), BG, np.uint16)
    lst, off, simple, cls = C.classify(mat, 4)
    assert lst.size == 0 and list(off) == [0] * 5 and np.all(cls == C.NONE)
    assert cls.size == 2 * 2   # 9 x 5 pixels: 2 x 2 clipped tiles


def test_ids_at_or_above_n_mats_are_not_neural():
    mat = np.array([[0, 1, 2, 3, 4, 5, 6, 7]] * 4, np.uint16)
    lst, off, simple, cls = C.classify(mat, 4)
    assert sorted(int(i) % 8 for i in lst) == [0] * 4 + [1] * 4 + [2] * 4 + [3] * 4
    assert off[-1] == 16


@pytest.mark.parametrize("w,h,n_mats,noise", [(64, 32, 3, 0.0), (37, 22, 5, 0.05), (96, 64, 40, 0.02)])
def test_invariants_on_random_frames(w, h, n_mats, noise):
    rng = np.random.default_rng(w + h + n_mats)
    mat = I.material_frame(rng, w, h, n_mats, noise=noise)
    lst, off, simple, cls = C.classify(mat, n_mats)
    flat = mat.reshape(-1)
    valid = np.nonzero(flat < n_mats)[0]
    # the lists partition the valid pixels
    assert np.array_equal(np.sort(lst), valid)
    tw = (w + 7) // 8
    tile = (lst // w) // 4 * tw + (lst % w) // 8
    key = tile * 32 + ((lst // w) % 4) * 8 + (lst % w) % 8
    for m in range(n_mats):
        part = lst[off[m]:off[m + 1]]
        assert np.all(flat[part] == m)
        s = int(simple[m])
        assert np.all(cls[tile[off[m]:off[m] + s]] == C.SIMPLE)
        assert np.all(cls[tile[off[m] + s:off[m + 1]]] == C.MIXED)
        for a, b in ((off[m], off[m] + s), (off[m] + s, off[m + 1])):
            assert np.all(np.diff(key[a:b]) > 0)
    # a simple tile holds one material on more than 16 pixels
    for t in np.nonzero(cls == C.SIMPLE)[0]:
        ty, tx = divmod(int(t), tw)
        blk = mat[4 * ty:4 * ty + 4, 8 * tx:8 * tx + 8]
        ids = blk[blk < n_mats]
        assert ids.size > 16 and np.all(ids == ids[0])
