"""Trilinear and anisotropic filtering of BC1 mip chains, FP64 (the oracle
of ntc_decode_filtered).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the GPU library
or its Python binding.

Sec. 3.2 keeps each mip of a latent texture as its own BC1 texture and
Sec. 3.3 fetches the latents with the texture unit's trilinear or
anisotropic filtering without naming the filter. Readings (the common
texture-filtering definitions):
  * footprint axes in texels of mip 0 of level k: Px = |(du/dx W, dv/dx H)|,
    Py = |(du/dy W, dv/dy H)|;
  * trilinear: lod = log2 max(Px, Py) clamped to [0, n_mips - 1]; the
    bilinear samples (clamp to edge, the level's shift in texels of each
    mip) of mips floor(lod) and floor(lod) + 1 are blended by lod's fraction;
  * anisotropic: N = min(ceil(Pmax / Pmin), max_aniso) trilinear samples at
    lod = log2(Pmax / N) along the longer axis, at uv + (i/(N + 1) - 1/2) d
    for i = 1..N, averaged;
  * N is the smallest integer n >= 1 with n Pmin >= Pmax (so ceil of the
    axis ratio, 1 for a zero footprint and max_aniso for a degenerate one),
    decided in FP64 like everything else here: the squared lengths of the
    FP32 derivatives times power-of-two sizes are exact in FP64 up to one
    rounding of their sum, so the decision is the mathematical one except
    for ratios within about 1e-16 of an integer. A kernel that decides N in
    FP32 can only differ from it where the ratio lies within FP32 rounding
    of an integer.
"""
from __future__ import annotations

import numpy as np

import oracle as O


def axes_sq(duv: np.ndarray, w0: int, h0: int):
    """(Px^2, Py^2) in FP64: squared footprint axes in texels of mip 0."""
    d = np.asarray(duv, np.float64)
    ax, bx, ay, by = d[:, 0] * w0, d[:, 1] * h0, d[:, 2] * w0, d[:, 3] * h0
    return ax * ax + bx * bx, ay * ay + by * by


def aniso_count(px2: np.ndarray, py2: np.ndarray, max_aniso: int) -> np.ndarray:
    """N = min(ceil(Pmax / Pmin), max_aniso): the smallest n >= 1 with
    n^2 Pmin^2 >= Pmax^2 (1 when both axes are 0, max_aniso when only Pmin
    is), compared in FP64."""
    px2 = np.asarray(px2, np.float64)
    py2 = np.asarray(py2, np.float64)
    pmax2, pmin2 = np.maximum(px2, py2), np.minimum(px2, py2)
    n = np.full(px2.shape, max_aniso, np.int64)
    for i in range(max_aniso - 1, 0, -1):
        n = np.where(float(i * i) * pmin2 >= pmax2, i, n)
    return n


def aniso_ratio(px2: np.ndarray, py2: np.ndarray) -> np.ndarray:
    """Pmax / Pmin in FP64 (inf for Pmin = 0, nan for a zero footprint)."""
    pmax2 = np.maximum(px2, py2).astype(np.float64)
    pmin2 = np.minimum(px2, py2).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.sqrt(pmax2 / pmin2)


def _log2(x):
    with np.errstate(divide="ignore"):
        return np.log2(np.asarray(x, np.float64))


def mip_sample(blocks: np.ndarray, shift, uv: np.ndarray) -> np.ndarray:
    """Bilinear sample (clamp to edge) of one BC1 mip, float64 [n][3]."""
    if uv.shape[0] == 0:
        return np.zeros((0, 3))
    return O.features(O.Latents([blocks], shift=[shift]), uv)[:, :3]


def trilinear(chain, shift, lod: np.ndarray, uv: np.ndarray) -> np.ndarray:
    nm = len(chain)
    m0 = np.clip(np.floor(lod).astype(np.int64), 0, nm - 1)
    t = lod - m0
    out = np.zeros((uv.shape[0], 3))
    for m in range(nm):
        sel = m0 == m
        if sel.any():
            out[sel] = mip_sample(chain[m], shift, uv[sel])
    for m in range(nm - 1):
        sel = (m0 == m) & (t > 0)
        if sel.any():
            c1 = mip_sample(chain[m + 1], shift, uv[sel])
            out[sel] += t[sel, None] * (c1 - out[sel])
    return out


def level_features(chain, shift, uv: np.ndarray, duv: np.ndarray, filt: str, max_aniso: int = 16) -> np.ndarray:
    """Filtered features [n][3] of one level (chain[m]: BC1 blocks of mip m)."""
    uv = np.asarray(uv, np.float64)
    duv = np.asarray(duv, np.float64)
    h0, w0 = chain[0].shape[0] * 4, chain[0].shape[1] * 4
    top = len(chain) - 1
    px2, py2 = axes_sq(duv, w0, h0)
    if filt == "trilinear":
        lod = np.clip(0.5 * _log2(np.maximum(px2, py2)), 0.0, top)
        return trilinear(chain, shift, lod, uv)
    n = aniso_count(px2, py2, max_aniso)
    lod = np.clip(0.5 * _log2(np.maximum(px2, py2)) - _log2(n), 0.0, top)
    major_x = px2 >= py2
    d = np.where(major_x[:, None], duv[:, 0:2], duv[:, 2:4])
    out = np.zeros((uv.shape[0], 3))
    for nv in np.unique(n):
        sel = n == nv
        acc = np.zeros((int(sel.sum()), 3))
        for i in range(1, int(nv) + 1):
            t = i / (nv + 1) - 0.5
            acc += trilinear(chain, shift, lod[sel], uv[sel] + t * d[sel])
        out[sel] = acc / nv
    return out


def features(levels, shifts, uv: np.ndarray, duv: np.ndarray, filt: str, max_aniso: int = 16) -> np.ndarray:
    """[n][3K + 2]: filtered features of the K levels, then (u, v)."""
    uv = np.asarray(uv, np.float64)
    cols = [level_features(chain, shifts[k], uv, duv, filt, max_aniso) for k, chain in enumerate(levels)]
    return np.concatenate(cols + [uv], axis=1)


def decode(levels, shifts, mlp, uv, duv, filt: str, max_aniso: int = 16) -> np.ndarray:
    return O.mlp_forward(mlp, features(levels, shifts, uv, duv, filt, max_aniso))
