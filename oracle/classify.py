"""Frame classification by material, plain Python (the oracle of ntc_classify).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the GPU library
or its Python binding.

Sec. 4 ("Tile-based classification", Algorithm 1): the screen is cut into
8x4-pixel tiles; a tile is "simple" when all its pixels that carry a neural
material use the same one and there are more than 16 of them, it has no
neural pixel, or it is "mixed" (anything else, which includes a single
material on 16 pixels or fewer); the pixels of non-simple tiles are
regrouped by material. Readings: a pixel carries a neural material when its
id is below n_mats; tiles are numbered row-major and clipped at the frame
edge; the lists give, per material in material order, the pixels of its
simple tiles and then its other pixels, each part in tile order and
row-major inside a tile (the paper appends with atomics, so it fixes no
order).
"""
from __future__ import annotations

import numpy as np

NONE, SIMPLE, MIXED = 0, 1, 2


def tiles_of(width: int, height: int):
    return (width + 7) // 8, (height + 3) // 4


def classify(mat_ids: np.ndarray, n_mats: int):
    """(pixel_list int64 [valid], mat_offsets int64 [n_mats + 1],
    mat_simple int64 [n_mats], tile_class uint8 [tiles])."""
    mat = np.asarray(mat_ids)
    height, width = mat.shape
    tw, th = tiles_of(width, height)
    tile_class = np.zeros(tw * th, np.uint8)
    simple = [[] for _ in range(n_mats)]
    other = [[] for _ in range(n_mats)]
    for t in range(tw * th):
        tx, ty = t % tw, t // tw
        valid = []
        for y in range(4 * ty, min(4 * ty + 4, height)):
            for x in range(8 * tx, min(8 * tx + 8, width)):
                m = int(mat[y, x])
                if m < n_mats:
                    valid.append((y * width + x, m))
        if not valid:
            tile_class[t] = NONE
            continue
        ids = {m for _, m in valid}
        if len(ids) == 1 and len(valid) > 16:
            tile_class[t] = SIMPLE
            for idx, m in valid:
                simple[m].append(idx)
        else:
            tile_class[t] = MIXED
            for idx, m in valid:
                other[m].append(idx)
    lists, offsets, n_simple = [], [0], []
    for m in range(n_mats):
        lists += simple[m] + other[m]
        offsets.append(len(lists))
        n_simple.append(len(simple[m]))
    return (np.array(lists, np.int64), np.array(offsets, np.int64), np.array(n_simple, np.int64), tile_class)
