"""Pins of the oracle's latent sampling (Sec. 3.3 bilinear filtering, Sec. 3.1
concatenation x = [c_0 .. c_3, u, v] and half-texel shift of textures 2 and 4).

Closed forms: constant textures, texel-centre exactness, reproduction of a
linear ramp, clamp and wrap edges, a half-texel shift equals the mean of two
neighbours, and BC1 texel centres return the decoded texel.
"""
import numpy as np

import ntc_inputs as I


def _grid(rng, w, h):
    return rng.random((h, w, 3))


def test_constant_texture(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(0)
    levels = [np.full((h, w, 3), c) for (w, h), c in zip([(8, 4), (16, 16), (4, 4), (12, 8)], [0.25, 0.5, 0.75, 0.125])]
    for addr in (O.CLAMP, O.WRAP):
        lat = O.Latents(levels, shift=I.PAPER_SHIFT, address=addr)
        uv = rng.random((500, 2)) * 1.4 - 0.2  # includes outside [0,1]
        x = O.features(lat, uv)
        for k, c in enumerate([0.25, 0.5, 0.75, 0.125]):
            assert np.allclose(x[:, 3 * k:3 * k + 3], c, rtol=0, atol=1e-15)
        assert np.array_equal(x[:, 12:14], uv)


def test_texel_centres_exact(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(1)
    sizes = [(16, 8), (8, 8), (4, 16), (8, 4)]
    levels = [_grid(rng, w, h) for (w, h) in sizes]
    lat = O.Latents(levels, shift=I.NO_SHIFT)
    for k, (w, h) in enumerate(sizes):
        i = rng.integers(0, w, 200)
        j = rng.integers(0, h, 200)
        uv = np.stack([(i + 0.5) / w, (j + 0.5) / h], 1)
        x = O.features(lat, uv)
        assert np.array_equal(x[:, 3 * k:3 * k + 3], levels[k][j, i])


def test_linear_ramp_reproduced(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(2)
    w, h = 32, 16
    i = np.arange(w)[None, :, None]
    j = np.arange(h)[:, None, None]
    a = np.array([0.01, -0.02, 0.03])
    b = np.array([0.05, 0.01, -0.04])
    grid = 0.3 + a * i + b * j
    lat = O.Latents([grid], shift=[(0.0, 0.0)])
    # interior: x = u w - 1/2 in [0, w-1]
    u = (rng.random(1000) * (w - 1) + 0.5) / w
    v = (rng.random(1000) * (h - 1) + 0.5) / h
    x = O.features(lat, np.stack([u, v], 1))
    px, py = u * w - 0.5, v * h - 0.5
    expect = 0.3 + a[None] * px[:, None] + b[None] * py[:, None]
    assert np.allclose(x[:, 0:3], expect, atol=1e-12)


def test_clamp_and_wrap_edges(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(3)
    w, h = 8, 8
    grid = _grid(rng, w, h)
    # left of the first centre: clamp returns column 0 (row blend only)
    u = np.full(50, 0.25 / w)
    jj = rng.integers(0, h, 50)
    v = (jj + 0.5) / h
    uv = np.stack([u, v], 1)
    xc = O.features(O.Latents([grid], address=O.CLAMP), uv)
    assert np.allclose(xc[:, 0:3], grid[jj, 0], atol=1e-15)
    # wrap: x = -0.25 -> taps at columns w-1 and 0 with weights 0.25 / 0.75
    xw = O.features(O.Latents([grid], address=O.WRAP), uv)
    assert np.allclose(xw[:, 0:3], 0.25 * grid[jj, w - 1] + 0.75 * grid[jj, 0], atol=1e-15)
    # past the last centre: clamp returns the last column
    uv2 = np.stack([np.full(50, (w - 0.1) / w), v], 1)
    xc2 = O.features(O.Latents([grid], address=O.CLAMP), uv2)
    assert np.allclose(xc2[:, 0:3], grid[jj, w - 1], atol=1e-15)


def test_half_texel_shift(oracle_lib):
    """A shift of (1/2, 1/2) texel at a texel centre averages the 2x2 texels
    (i, j) .. (i+1, j+1)."""
    O = oracle_lib
    rng = np.random.default_rng(4)
    w, h = 16, 16
    grid = _grid(rng, w, h)
    lat = O.Latents([grid, grid], shift=[(0.0, 0.0), (0.5, 0.5)])
    i = rng.integers(0, w - 1, 100)
    j = rng.integers(0, h - 1, 100)
    uv = np.stack([(i + 0.5) / w, (j + 0.5) / h], 1)
    x = O.features(lat, uv)
    assert np.array_equal(x[:, 0:3], grid[j, i])
    mean4 = 0.25 * (grid[j, i] + grid[j, i + 1] + grid[j + 1, i] + grid[j + 1, i + 1])
    assert np.allclose(x[:, 3:6], mean4, atol=1e-15)


def test_bc1_texel_centre_returns_decoded_texel(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(5)
    sizes = [(32, 32), (16, 16), (8, 8), (4, 4)]
    levels = I.bc1_pyramid(rng, sizes)
    lat = O.Latents(levels, shift=I.NO_SHIFT)
    for k, (w, h) in enumerate(sizes):
        _, _, val = O.bc1_level(levels[k])
        i = rng.integers(0, w, 100)
        j = rng.integers(0, h, 100)
        x = O.features(lat, np.stack([(i + 0.5) / w, (j + 0.5) / h], 1))
        assert np.array_equal(x[:, 3 * k:3 * k + 3], val[j, i])


def test_weights_sum_to_one_bc1(oracle_lib):
    """Bilinear sampling of a BC1 texture stays inside the per-channel range
    of the four taps; a block with one solid colour gives that colour."""
    O = oracle_lib
    solid = np.full((4, 4), np.uint64(0x5285), dtype=np.uint64)  # c0 = 0x5285, c1 = 0, indices 0
    lat = O.Latents([solid], shift=[(0.5, 0.5)])
    rng = np.random.default_rng(6)
    x = O.features(lat, rng.random((300, 2)))
    assert np.allclose(x[:, 0:3], [10 / 31, 20 / 63, 5 / 31], atol=1e-15)
