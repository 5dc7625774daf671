"""Pins of the oracle's BC1 texel decode (Sec. 3.1, latent BC1 compression).

* hand-built blocks with closed-form palettes (tests/golden/bc1_blocks.txt);
* block addressing on a multi-block texture with solid-colour blocks;
* an independent numpy decoder written from the blend form (1-a) e0 + a e1
  with the a values of the two BC1 modes, on many random blocks;
* invariants: indices 0 and 1 reproduce the endpoints, blends stay on the
  segment between them, three-colour index 3 is black.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from conftest import load_golden_blocks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bc1_blocks.txt")


def _word(c0, c1, idx):
    return np.uint64(c0 | (c1 << 16) | (idx << 32))


def test_golden_blocks(oracle_lib):
    O = oracle_lib
    blocks = load_golden_blocks(GOLDEN)
    assert len(blocks) >= 8
    for c0, c1, idx, rows in blocks:
        arr = np.array([[_word(c0, c1, idx)]], dtype=np.uint64)
        num, den, val = O.bc1_level(arr)
        for y in range(4):
            for x in range(4):
                for ch in range(3):
                    got = Fraction(int(num[y, x, ch]), int(den[y, x, ch]))
                    assert got == rows[y][x][ch], (hex(c0), hex(c1), hex(idx), x, y, ch)
                    assert val[y, x, ch] == float(rows[y][x][ch])


def test_block_addressing(oracle_lib):
    """8x8 texture = 2x2 blocks, block-row-major; each block a solid colour."""
    O = oracle_lib
    red, green, blue, white = 0xF800, 0x07E0, 0x001F, 0xFFFF
    # index word 0: every texel takes e0; c1 = 0 keeps four-colour mode.
    arr = np.array([[_word(red, 0, 0), _word(green, 0, 0)],
                    [_word(blue, 0, 0), _word(white, 0, 0)]], dtype=np.uint64)
    num, den, val = O.bc1_level(arr)
    expect = {(0, 0): (1, 0, 0), (1, 0): (0, 1, 0), (0, 1): (0, 0, 1), (1, 1): (1, 1, 1)}
    for j in range(8):
        for i in range(8):
            assert tuple(val[j, i]) == expect[(i // 4, j // 4)], (i, j)


def _numpy_bc1(words):
    """Independent decode: value * (6 * (2^b - 1)) as an exact integer, [n][16][3].

    Written from the blend form T = (1 - a) e0 + a e1 with a in
    {0, 1, 1/3, 2/3} (c0 > c1) or {0, 1, 1/2} and black for index 3."""
    words = words.astype(np.uint64)
    c0 = (words & np.uint64(0xFFFF)).astype(np.int64)
    c1 = ((words >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
    ind = (words >> np.uint64(32)).astype(np.int64)
    four = c0 > c1
    out = np.zeros((words.size, 16, 3), np.int64)
    fields = [(11, 31), (5, 63), (0, 31)]
    # a * 6 for each index, per mode
    a6_four = np.array([0, 6, 2, 4])
    a6_three = np.array([0, 6, 3, 0])
    for p in range(16):
        idx = (ind >> (2 * p)) & 3
        a6 = np.where(four, a6_four[idx], a6_three[idx])
        black = (~four) & (idx == 3)
        for ch, (sh, _) in enumerate(fields):
            e0 = (c0 >> sh) & (31 if ch != 1 else 63)
            e1 = (c1 >> sh) & (31 if ch != 1 else 63)
            v = (6 - a6) * e0 + a6 * e1  # = 6 * ((1-a) e0 + a e1)
            out[:, p, ch] = np.where(black, 0, v)
    return out


def test_random_blocks_vs_independent_decoder(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(1234)
    n_side = 128  # 16384 blocks, every mode and index appears
    c0 = rng.integers(0, 1 << 16, size=(n_side, n_side), dtype=np.uint64)
    c1 = rng.integers(0, 1 << 16, size=(n_side, n_side), dtype=np.uint64)
    c1[:4] = c0[:4]  # equal endpoints present too
    idx = rng.integers(0, 1 << 32, size=(n_side, n_side), dtype=np.uint64)
    words = c0 | (c1 << np.uint64(16)) | (idx << np.uint64(32))
    num, den, val = O.bc1_level(words)
    ref6 = _numpy_bc1(words.reshape(-1))  # [blocks][16][3], over 6 (2^b - 1)
    maxv = np.array([31, 63, 31], np.int64)
    H = W = 4 * n_side
    # texel (i, j) -> block (j//4, i//4), position 4 (j%4) + (i%4)
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    b = (j // 4) * n_side + (i // 4)
    p = 4 * (j % 4) + (i % 4)
    ref = ref6[b, p]  # [H][W][3]
    # cross-multiplied exact comparison: num/den == ref / (6 maxv)
    assert np.array_equal(num.astype(np.int64) * 6 * maxv, ref * den.astype(np.int64))
    # the float value is the correctly rounded quotient
    assert np.array_equal(val, num.astype(np.float64) / den.astype(np.float64))


def test_invariants(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(99)
    words = rng.integers(0, 1 << 63, size=(64, 64), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=(64, 64), dtype=np.uint64)
    num, den, val = O.bc1_level(words)
    w = words.reshape(-1)
    c0 = (w & np.uint64(0xFFFF)).astype(np.int64)
    c1 = ((w >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
    ind = (w >> np.uint64(32)).astype(np.int64)
    e0 = np.stack([(c0 >> 11) / 31.0, ((c0 >> 5) & 63) / 63.0, (c0 & 31) / 31.0], -1)
    e1 = np.stack([(c1 >> 11) / 31.0, ((c1 >> 5) & 63) / 63.0, (c1 & 31) / 31.0], -1)
    for bi in range(w.size):
        by, bx = divmod(bi, 64)
        for p in range(16):
            y, x = divmod(p, 4)
            t = val[4 * by + y, 4 * bx + x]
            k = (ind[bi] >> (2 * p)) & 3
            if k == 0:
                assert np.array_equal(t, e0[bi])
            elif k == 1:
                assert np.array_equal(t, e1[bi])
            elif k == 3 and c0[bi] <= c1[bi]:
                assert np.array_equal(t, np.zeros(3))
            else:
                lo = np.minimum(e0[bi], e1[bi]) - 1e-15
                hi = np.maximum(e0[bi], e1[bi]) + 1e-15
                assert np.all(t >= lo) and np.all(t <= hi)
    # denominators are the ones the two modes allow
    assert set(np.unique(den)) <= {1, 62, 93, 126, 189}
