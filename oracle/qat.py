"""Trainable BC1 latents in FP64 (numpy): the oracle of ntc_qat_*.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the GPU library
or its Python binding.

Sec. 3.2, Eqs. 1-3: the BC1 endpoints and the per-texel interpolation
weight are kept as floats; their BC1 values are a sigmoid followed by
quantisation to the field width (5, 6, 5 bits for an endpoint's r, g, b and
2 bits for the weight), and the quantisation lets gradients through
unchanged. Readings (the paper gives the formulas only):
  * quant(s, b) rounds s (2^b - 1) to the nearest integer code (ties to
    even; only s = 1/2 is a tie, and every field width puts the even code
    above it);
  * the texel is the four-colour BC1 palette entry of its weight code,
    ((3 - w) E0 + w E1) / (3 (2^b - 1)) per channel;
  * one level is an array [H/4][W/4][22] of logits per block: e0 (r, g, b),
    e1 (r, g, b), then the 16 texel weights, texel (x, y) at 4 y + x;
  * the exported block puts the larger RGB565 endpoint first (four-colour
    mode), mirroring the weights (w -> 3 - w) when the endpoints swap; equal
    endpoints give every texel index 0.
"""
from __future__ import annotations

import numpy as np

BITS = (5, 6, 5)
N_PARAMS = 22


def sigmoid(x):
    x = np.asarray(x, np.float64)
    return 1.0 / (1.0 + np.exp(-x))


def quant_code(x, bits: int) -> np.ndarray:
    """Code of quant(sigmoid(x), bits): round(sigmoid(x) (2^bits - 1))."""
    m = (1 << bits) - 1
    return np.rint(sigmoid(x) * m).astype(np.int64)


def codes(params: np.ndarray):
    """Endpoint codes E0, E1 [bh][bw][3] and weight codes w [bh][bw][16]."""
    p = np.asarray(params, np.float64)
    e0 = np.stack([quant_code(p[..., c], BITS[c]) for c in range(3)], axis=-1)
    e1 = np.stack([quant_code(p[..., 3 + c], BITS[c]) for c in range(3)], axis=-1)
    w = quant_code(p[..., 6:22], 2)
    return e0, e1, w


def _per_texel(a: np.ndarray) -> np.ndarray:
    """[bh][bw][16] (texel 4y + x of each block) -> [H][W]."""
    bh, bw = a.shape[:2]
    return a.reshape(bh, bw, 4, 4).transpose(0, 2, 1, 3).reshape(bh * 4, bw * 4)


def _per_block(a: np.ndarray) -> np.ndarray:
    """[bh][bw][c] -> [H][W][c] (each block's value on its 16 texels)."""
    return np.repeat(np.repeat(a, 4, axis=0), 4, axis=1)


def texels(params: np.ndarray):
    """(num, den, value): the texel value num / den per channel, [H][W][3]
    (den = 3 (2^b - 1)) and as float64."""
    e0, e1, w = codes(params)
    wt = _per_texel(w)[..., None]
    num = (3 - wt) * _per_block(e0) + wt * _per_block(e1)
    den = np.broadcast_to(np.array([3 * ((1 << b) - 1) for b in BITS], np.int64), num.shape)
    return num, den, num / den


def export_bc1(params: np.ndarray) -> np.ndarray:
    """uint64 BC1 blocks [bh][bw] whose decode is texels(params)."""
    e0, e1, w = codes(params)
    c0 = (e0[..., 0] << 11) | (e0[..., 1] << 5) | e0[..., 2]
    c1 = (e1[..., 0] << 11) | (e1[..., 1] << 5) | e1[..., 2]
    bh, bw = c0.shape
    out = np.zeros((bh, bw), np.uint64)
    index_of_weight = (0, 2, 3, 1)  # four-colour palette: E0, E1, (2E0+E1)/3, (E0+2E1)/3
    for by in range(bh):
        for bx in range(bw):
            a, b = int(c0[by, bx]), int(c1[by, bx])
            ws = [int(v) for v in w[by, bx]]
            if a < b:
                a, b = b, a
                ws = [3 - v for v in ws]
            idx = 0
            if a != b:
                for t, v in enumerate(ws):
                    idx |= index_of_weight[v] << (2 * t)
            out[by, bx] = np.uint64(a | (b << 16) | (idx << 32))
    return out


def backward(params: np.ndarray, grad_texels: np.ndarray) -> np.ndarray:
    """dL/dparams [bh][bw][22] for dL/dtexels [H][W][3], the quantisation
    passed through (straight-through): texel_c = (1 - a) E0_c + a E1_c with
    E = code / (2^b - 1) and a = w / 3, each the quantised sigmoid of its
    logit."""
    p = np.asarray(params, np.float64)
    g = np.asarray(grad_texels, np.float64)
    bh, bw = p.shape[:2]
    e0, e1, w = codes(p)
    m = np.array([(1 << b) - 1 for b in BITS], np.float64)
    v0, v1, a = e0 / m, e1 / m, w / 3.0
    # the block's 16 texels as [bh][bw][16][3]
    gb = g.reshape(bh, 4, bw, 4, 3).transpose(0, 2, 1, 3, 4).reshape(bh, bw, 16, 3)
    dv0 = ((1.0 - a)[..., None] * gb).sum(axis=2)
    dv1 = (a[..., None] * gb).sum(axis=2)
    da = ((v1 - v0)[:, :, None, :] * gb).sum(axis=3)
    s = sigmoid(p)
    ds = s * (1.0 - s)
    out = np.empty_like(p)
    out[..., 0:3] = ds[..., 0:3] * dv0
    out[..., 3:6] = ds[..., 3:6] * dv1
    out[..., 6:22] = ds[..., 6:22] * da
    return out
