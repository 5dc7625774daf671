"""Checks of the FP32 error bound that the GPU backward tests use to leave
out samples on ReLU kinks (tests/fp32_bounds.py)."""
import numpy as np

import ntc_inputs as I
import oracle as O
from fp32_bounds import U32, feature_error_bound, gamma, relu_ambiguous, relu_bounds


def _fma32(a, b, c):
    """Fused multiply-add rounded to FP32 (the FP64 product of two FP32
    values is exact; the FP64 sum adds at most 2^-53 before the final
    rounding)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def test_gamma():
    assert gamma(1) == U32 / (1 - U32)
    assert abs(gamma(64) / (64 * 2.0 ** -24) - 1) < 1e-5


def test_bound_holds_for_an_fp32_chain_and_is_not_loose_by_orders():
    """An FP32 evaluation (features rounded to FP32, every layer a chain of
    FP32 fused multiply-adds) stays within the bound on every unit of every
    sample, and the bound is within a few hundred times the largest error
    seen (it is a worst case, not a guess)."""
    rng = np.random.default_rng(11)
    sizes = [(128, 128), (64, 64), (32, 32), (16, 16)]
    lat_np = I.f32_pyramid(rng, sizes)
    Ws, bs = I.xavier_mlp(rng, (14, 64, 64, 8), bias="normal")
    uv = I.random_uv(rng, 4000)
    olat = O.Latents(lat_np, shift=I.PAPER_SHIFT)
    x = O.features(olat, uv)
    dx = np.broadcast_to(feature_error_bound(olat, lat_np, uv), x.shape)
    bounds = relu_bounds(x, dx, Ws, bs)
    h32 = x.astype(np.float32)
    worst = 0.0
    for l, (z, bound) in enumerate(bounds):
        W = Ws[l].astype(np.float32)
        z32 = np.broadcast_to(bs[l].astype(np.float32), z.shape).copy()
        for j in range(W.shape[1]):
            z32 = _fma32(h32[:, j:j + 1], W[None, :, j], z32)
        err = np.abs(z32.astype(np.float64) - z)
        assert np.all(err <= bound), l
        worst = max(worst, float(np.max(err / bound)))
        h32 = np.maximum(z32, np.float32(0.0))
    assert worst > 1e-3


def test_ambiguous_samples_are_near_kinks():
    """Samples flagged ambiguous have some |z| below 1e-4 (the bound is of
    order 1e-5 here); the rest keep every |z| above the bound."""
    rng = np.random.default_rng(12)
    sizes = [(64, 64), (32, 32), (16, 16), (8, 8)]
    lat_np = I.f32_pyramid(rng, sizes)
    Ws, bs = I.xavier_mlp(rng, (14, 64, 64, 8), bias="normal")
    uv = I.random_uv(rng, 20000)
    olat = O.Latents(lat_np, shift=I.PAPER_SHIFT)
    amb = relu_ambiguous(olat, Ws, bs, uv, lat_np)
    margin = O.relu_margin(olat, O.Mlp(Ws, bs), uv)
    assert amb.sum() < 0.01 * uv.shape[0]
    assert np.all(margin[amb] < 1e-4)
