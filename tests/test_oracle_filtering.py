"""Pins of the filtering oracle (oracle/filtering.py; Sec. 3.2 mip chains,
Sec. 3.3 trilinear / anisotropic fetches)."""
import numpy as np
import pytest

import ntc_inputs as I
import oracle as O
from oracle import filtering as F

SH = (0.5, 0.5)


def _solid_chain(sizes, colours):
    """One BC1 mip per size, every block both endpoints = colour (565)."""
    return [np.full((h // 4, w // 4), np.uint64(c | (c << 16)), np.uint64) for (w, h), c in zip(sizes, colours)]


def _value565(c):
    return np.array([(c >> 11) / 31.0, ((c >> 5) & 63) / 63.0, (c & 31) / 31.0])


def test_zero_derivatives_give_bilinear_of_mip0():
    rng = np.random.default_rng(1)
    chain = I.bc1_mip_chain(rng, 64, 32)
    uv = rng.random((500, 2))
    ref = O.features(O.Latents([chain[0]], shift=[SH]), uv)[:, :3]
    for filt in ("trilinear", "anisotropic"):
        got = F.level_features(chain, SH, uv, np.zeros((500, 4)), filt)
        assert np.array_equal(got, ref), filt


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_power_of_two_footprint_selects_one_mip(m):
    rng = np.random.default_rng(2)
    chain = I.bc1_mip_chain(rng, 64, 64)
    uv = rng.random((300, 2))
    d = 2.0 ** m / 64  # 2^m texels of mip 0 per pixel along x and y
    duv = np.tile([d, 0.0, 0.0, d], (300, 1))
    got = F.level_features(chain, SH, uv, duv, "trilinear")
    ref = O.features(O.Latents([chain[m]], shift=[SH]), uv)[:, :3]
    assert np.allclose(got, ref, rtol=0, atol=1e-15)


def test_trilinear_weights_on_solid_mips():
    """Constant mips: the filtered value is the lod-weighted blend of the two
    constants, lod = log2 of the longer footprint axis, clamped."""
    sizes = [(64 >> m, 64 >> m) for m in range(5)]
    cols = [0xF800, 0x07E0, 0x001F, 0xFFE0, 0x0000]
    chain = _solid_chain(sizes, cols)
    vals = [_value565(c) for c in cols]
    uv = np.full((6, 2), 0.37)
    px = np.array([0.25, 1.0, 1.5, 2.0 ** 2.3, 2.0 ** 3.75, 100.0])  # texels of mip 0
    duv = np.stack([px / 64, np.zeros(6), np.zeros(6), 0.5 * px / 64], axis=1)
    got = F.level_features(chain, SH, uv, duv, "trilinear")
    for r, p in enumerate(px):
        lod = min(max(np.log2(p), 0.0), 4.0)
        m0 = int(np.floor(lod))
        t = lod - m0
        exp = vals[m0] if m0 == 4 else (1 - t) * vals[m0] + t * vals[m0 + 1]
        assert np.allclose(got[r], exp, rtol=0, atol=1e-12), r


def test_anisotropic_count_and_lod():
    # footprint 8 x 2 texels: N = 4, lod = log2(8 / 4) = 1 -> mip 1 exactly
    sizes = [(64 >> m, 64 >> m) for m in range(5)]
    cols = [0xF800, 0x07E0, 0x001F, 0xFFE0, 0x0000]
    chain = _solid_chain(sizes, cols)
    duv = np.array([[0.0, 2.0 / 64, 8.0 / 64, 0.0]])
    px2, py2 = F.axes_sq(duv, 64, 64)
    assert F.aniso_count(px2, py2, 16)[0] == 4
    assert F.aniso_count(px2, py2, 3)[0] == 3
    got = F.level_features(chain, SH, np.array([[0.5, 0.5]]), duv, "anisotropic")
    assert np.allclose(got[0], _value565(cols[1]), atol=1e-12)


def test_anisotropic_taps_average_trilinear_samples():
    """Isotropic footprint: one tap, equal to trilinear. Ratio 2 (equal
    squared terms): two taps at uv -/+ d/6, averaged."""
    rng = np.random.default_rng(3)
    chain = I.bc1_mip_chain(rng, 64, 64)
    uv = rng.random((200, 2)) * 0.8 + 0.1
    iso = np.tile([3.0 / 64, 0.0, 0.0, 3.0 / 64], (200, 1))
    assert np.array_equal(F.level_features(chain, SH, uv, iso, "anisotropic"),
                          F.level_features(chain, SH, uv, iso, "trilinear"))
    an = np.tile([4.0 / 64, 0.0, 0.0, 2.0 / 64], (200, 1))
    lod = np.full(200, 1.0)  # log2(4 / 2)
    d = np.array([4.0 / 64, 0.0])
    ref = 0.5 * (F.trilinear(chain, SH, lod, uv - d / 6) + F.trilinear(chain, SH, lod, uv + d / 6))
    ref_mip1 = 0.5 * (O.features(O.Latents([chain[1]], shift=[SH]), uv - d / 6)[:, :3] +
                      O.features(O.Latents([chain[1]], shift=[SH]), uv + d / 6)[:, :3])
    got = F.level_features(chain, SH, uv, an, "anisotropic")
    assert np.allclose(got, ref, rtol=0, atol=1e-15)
    assert np.allclose(got, ref_mip1, rtol=0, atol=1e-15)


def test_count_is_ceil_of_ratio():
    """N = min(ceil(Pmax / Pmin), max_aniso) against exact rational
    arithmetic: derivatives on a 1/64 grid (squared lengths exact), including
    axes whose ratio is exactly an integer (3-4-5 right triangles), where the
    count must be that integer and not the next."""
    from fractions import Fraction
    rng = np.random.default_rng(4)
    ints = rng.integers(-40, 41, (4000, 4)).astype(np.float64)
    exact_pairs = np.array([[3, 4, 0, 5], [6, 8, 3, 4], [0, 9, 3, 0], [12, 16, 0, 5], [5, 0, 0, 1],
                            [0, 0, 0, 0], [0, 0, 7, 0], [16, 0, 0, 1], [17, 0, 0, 1], [30, 40, 3, 4]], np.float64)
    ints = np.concatenate([exact_pairs, ints])
    duv = ints / 64.0
    px2, py2 = F.axes_sq(duv, 64, 64)
    for max_aniso in (16, 4):
        n = F.aniso_count(px2, py2, max_aniso)
        for r in range(ints.shape[0]):
            a = [Fraction(int(v)) for v in ints[r]]
            p2 = a[0] ** 2 + a[1] ** 2
            q2 = a[2] ** 2 + a[3] ** 2
            hi, lo = max(p2, q2), min(p2, q2)
            k = 1
            while k < max_aniso and k * k * lo < hi:
                k += 1
            assert n[r] == k, (ints[r], max_aniso, n[r], k)
    n16 = F.aniso_count(px2, py2, 16)
    assert list(n16[:10]) == [1, 2, 3, 4, 5, 1, 16, 16, 16, 10]


def test_count_is_ceil_of_ratio_random():
    """On random derivatives the count is ceil of the FP64 axis ratio,
    capped (integer ratios do not occur there)."""
    rng = np.random.default_rng(5)
    duv = rng.standard_normal((20000, 4)) * 0.05
    px2, py2 = F.axes_sq(duv, 256, 128)
    n = F.aniso_count(px2, py2, 16)
    r = F.aniso_ratio(px2, py2)
    assert np.array_equal(n, np.minimum(np.ceil(r), 16))
