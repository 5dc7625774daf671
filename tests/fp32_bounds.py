"""Rounding-error bounds used by the GPU tests to decide which samples the
FP32 kernels may branch on differently from the FP64 oracle (test helper,
not a test module)."""
import numpy as np

import oracle as O

U32 = 2.0 ** -24  # unit roundoff of FP32


def gamma(n):
    """gamma_n = n u / (1 - n u): the relative error bound of n rounded
    operations (Higham, "Accuracy and Stability of Numerical Algorithms",
    Sec. 3.1)."""
    return n * U32 / (1.0 - n * U32)


def relu_bounds(x, dx, Ws, bs):
    """Per hidden layer, (z, bound) for features x [n][d0] (FP64) whose FP32
    evaluation is off by at most dx: layer l's pre-activation
    z = b + sum_j W_j h_j evaluated by n = fan-in fused multiply-adds is off by
    at most gamma_n (|b| + sum |W_j h_j|) + sum |W_j| |dh_j|, and ReLU is
    1-Lipschitz, so |dh| <= the bound of the layer below."""
    out = []
    h, dh = x, dx
    for l in range(len(Ws) - 1):
        W = np.asarray(Ws[l], np.float64)
        b = np.asarray(bs[l], np.float64)
        aW = np.abs(W)
        z = h @ W.T + b
        bound = gamma(W.shape[1]) * (np.abs(h) @ aW.T + np.abs(b)) + dh @ aW.T
        out.append((z, bound))
        h, dh = np.maximum(z, 0.0), bound
    return out


def feature_error_bound(olat, lat_np, uv):
    """Bound on |x_fp32 - x| of the bilinear features of float latents: with
    power-of-two level sizes W <= 2^14 and |u| < 2, u W is exact in FP32, and
    so is u W - 1/2 + shift except where |u W| < 1/2, where it is off by at
    most 2^-25 texel (the result then lies within one texel of 0); the
    bilinear weights (products of 1 - f and f) and the 4-term blend add at
    most 6 roundings of the blended magnitude: |dx| <= 8 u max|latent|.
    u and v enter exactly."""
    for w, h in olat.sizes:
        assert w & (w - 1) == 0 and h & (h - 1) == 0, "the feature bound needs power-of-two level sizes"
        assert w <= 16384 and h <= 16384
    assert np.all(np.abs(uv) < 2)
    lat_max = max(float(np.max(np.abs(a))) for a in lat_np)
    d = np.full(3 * olat.n + 2, 8 * U32 * lat_max)
    d[-2:] = 0.0
    return d


def relu_ambiguous(olat, Ws, bs, uv, lat_np):
    """Samples whose ReLU pattern an FP32 evaluation may take differently:
    some hidden unit has |z| (FP64, from the oracle's features) at or below
    its FP32 error bound."""
    x = O.features(olat, uv)
    dx = np.broadcast_to(feature_error_bound(olat, lat_np, uv), x.shape)
    amb = np.zeros(uv.shape[0], bool)
    for z, bound in relu_bounds(x, dx, Ws, bs):
        amb |= np.any(np.abs(z) <= bound, axis=1)
    return amb
