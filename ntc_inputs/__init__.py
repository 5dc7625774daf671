"""Seeded synthetic inputs for the neural BC1 texture decode.

This module only draws numbers: BC1 block words, continuous latent grids,
MLP weights, sample coordinates and training targets. It contains none of
the decode's arithmetic (no BC1 palette decode, no filtering, no MLP), so
both the FP64 CPU oracle and the HIP path can be fed from it without
sharing any of the method's code.

Every generator takes a ``numpy.random.Generator``; ``streams(seed)`` splits
a seed into independent streams with ``SeedSequence(seed).spawn``:
stream 0 = latents, 1 = MLP, 2 = sample coordinates, 3 = targets / extras.

The shapes follow the paper's workloads: four latent textures per material
(Sec. 3.1, resolution table, VarB-shaped pyramid), 4096^2 textures and a
small MLP (Sec. 5, Tables 1 and 2). The Polyhaven texture sets and the
trained latents/MLPs used in Sec. 5 are not available; random BC1 words
and Xavier-initialised MLPs of the same shapes stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "streams", "bc1_level", "bc1_pyramid", "f32_pyramid", "xavier_mlp",
    "pixel_uv", "pixel_uv_subset", "random_uv", "value_noise_texture",
    "point_sample", "Workload", "WORKLOADS", "make_workload", "material_specs",
    "MaterialSpec", "make_material", "TILE", "tiled_to_rowmajor",
]

# Pixels are laid out in square tiles of TILE x TILE screen pixels (row-major
# tiles, row-major inside a tile) when order == "tiled": one 8x8 tile is one
# 64-pixel group, the analogue of the paper's 8x4 screen tiles (Sec. 4).
TILE = 8


def streams(seed: int, n: int = 4) -> List[np.random.Generator]:
    """Independent generators for (latents, mlp, uv, extra)."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


# ----------------------------------------------------------------------------
# Latents
# ----------------------------------------------------------------------------
def bc1_level(rng: np.random.Generator, width: int, height: int) -> np.ndarray:
    """Uniform random BC1 blocks for one W x H texture.

    Returns uint64 [(H/4), (W/4)], block-row-major. Bits 0-15 are the first
    RGB565 endpoint, 16-31 the second, 32-63 the sixteen 2-bit indices; the
    three fields are drawn independently and uniformly.
    """
    if width % 4 or height % 4 or width <= 0 or height <= 0:
        raise ValueError("BC1 textures need positive sizes that are multiples of 4")
    bh, bw = height // 4, width // 4
    c0 = rng.integers(0, 1 << 16, size=(bh, bw), dtype=np.uint64)
    c1 = rng.integers(0, 1 << 16, size=(bh, bw), dtype=np.uint64)
    idx = rng.integers(0, 1 << 32, size=(bh, bw), dtype=np.uint64)
    return (c0 | (c1 << np.uint64(16)) | (idx << np.uint64(32))).astype(np.uint64)


def bc1_pyramid(rng: np.random.Generator, sizes: Sequence[Tuple[int, int]]) -> List[np.ndarray]:
    """One BC1 level per (width, height), drawn level 0 first."""
    return [bc1_level(rng, w, h) for (w, h) in sizes]


def f32_pyramid(rng: np.random.Generator, sizes: Sequence[Tuple[int, int]]) -> List[np.ndarray]:
    """Continuous latent grids, float32 [H][W][3], uniform in [0, 1)."""
    return [rng.random((h, w, 3), dtype=np.float64).astype(np.float32) for (w, h) in sizes]


# ----------------------------------------------------------------------------
# MLP
# ----------------------------------------------------------------------------
def xavier_mlp(rng: np.random.Generator, dims: Sequence[int],
               bias: str = "zero") -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """Xavier-normal weights W[l] = float32 [dims[l+1]][dims[l]].

    std = sqrt(2 / (fan_in + fan_out)), drawn in float64 then rounded to
    float32. ``bias`` is "zero" (the workloads' setting) or "normal"
    (N(0, 0.1^2), used by tests so that every bias term is exercised).
    """
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        fi, fo = dims[l], dims[l + 1]
        std = math.sqrt(2.0 / (fi + fo))
        Ws.append((rng.standard_normal((fo, fi)) * std).astype(np.float32))
        if bias == "zero":
            bs.append(np.zeros(fo, dtype=np.float32))
        elif bias == "normal":
            bs.append((rng.standard_normal(fo) * 0.1).astype(np.float32))
        else:
            raise ValueError(bias)
    return Ws, bs


# ----------------------------------------------------------------------------
# Sample coordinates
# ----------------------------------------------------------------------------
def _pixel_xy(width: int, height: int, order: str) -> Tuple[np.ndarray, np.ndarray]:
    n = width * height
    k = np.arange(n, dtype=np.int64)
    if order == "rowmajor":
        return k % width, k // width
    if order == "tiled":
        if width % TILE or height % TILE:
            raise ValueError("tiled order needs sizes that are multiples of the tile")
        tiles_x = width // TILE
        t, r = k // (TILE * TILE), k % (TILE * TILE)
        return (t % tiles_x) * TILE + r % TILE, (t // tiles_x) * TILE + r // TILE
    raise ValueError(order)


def tiled_to_rowmajor(width: int, height: int) -> np.ndarray:
    """int64 [W*H]: the row-major index y W + x of the k-th pixel in tiled
    order (so ``a_rowmajor[perm] = a_tiled`` reorders per-pixel arrays)."""
    x, y = _pixel_xy(width, height, "tiled")
    return y * width + x


def pixel_uv(width: int, height: int, order: str = "rowmajor",
             jitter_rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """float32 [W*H][2] uv of every screen pixel.

    u = (x + 0.5 + j_x) / W, v = (y + 0.5 + j_y) / H with j = 0 (pixel
    centres) or, when ``jitter_rng`` is given, j uniform in [-0.5, 0.5] in
    output-pixel units, drawn x then y for all pixels in ``order``.
    """
    x, y = _pixel_xy(width, height, order)
    fx = x.astype(np.float64) + 0.5
    fy = y.astype(np.float64) + 0.5
    if jitter_rng is not None:
        j = jitter_rng.random((x.size, 2)) - 0.5
        fx += j[:, 0]
        fy += j[:, 1]
    uv = np.empty((x.size, 2), dtype=np.float32)
    uv[:, 0] = fx / width
    uv[:, 1] = fy / height
    return uv


def pixel_uv_subset(width: int, height: int, order: str, index: np.ndarray,
                    jitter_seed_rng_factory=None) -> np.ndarray:
    """uv of the pixels ``index`` of ``pixel_uv(width, height, order)``.

    Only valid without jitter (pixel centres): the full array need not be
    materialised for very large batches.
    """
    if jitter_seed_rng_factory is not None:
        raise ValueError("subset sampling is only defined for pixel-centre uv")
    n = width * height
    index = np.asarray(index, dtype=np.int64)
    if index.size and (index.min() < 0 or index.max() >= n):
        raise IndexError("pixel index out of range")
    if order == "rowmajor":
        x, y = index % width, index // width
    else:
        tiles_x = width // TILE
        t, r = index // (TILE * TILE), index % (TILE * TILE)
        x, y = (t % tiles_x) * TILE + r % TILE, (t // tiles_x) * TILE + r // TILE
    uv = np.empty((index.size, 2), dtype=np.float32)
    uv[:, 0] = (x.astype(np.float64) + 0.5) / width
    uv[:, 1] = (y.astype(np.float64) + 0.5) / height
    return uv


def random_uv(rng: np.random.Generator, n: int) -> np.ndarray:
    """float32 [n][2], u and v uniform in [0, 1)."""
    return rng.random((n, 2), dtype=np.float64).astype(np.float32)


# ----------------------------------------------------------------------------
# Training targets (value noise)
# ----------------------------------------------------------------------------
def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def value_noise_texture(rng: np.random.Generator, size: int, channels: int = 8,
                        octaves: int = 4) -> np.ndarray:
    """float32 [size][size][channels] fractal value noise in [0, 1].

    Octave o has a lattice of 4 * 2^o cells per side with U[0,1) values at
    the lattice points, smoothstep-weighted interpolation between them, and
    amplitude 2^-o; the sum is divided by the total amplitude. Each channel
    draws its own lattices, channel 0 first, octave 0 first. Evaluated at
    texel centres (i + 0.5) / size.
    """
    t = (np.arange(size, dtype=np.float64) + 0.5) / size
    out = np.zeros((size, size, channels), dtype=np.float64)
    total = sum(2.0 ** -o for o in range(octaves))
    for c in range(channels):
        acc = np.zeros((size, size), dtype=np.float64)
        for o in range(octaves):
            cells = 4 * (1 << o)
            lat = rng.random((cells + 1, cells + 1))
            p = t * cells
            i = np.minimum(np.floor(p).astype(np.int64), cells - 1)
            f = _smoothstep(p - i)
            # rows are y, columns are x
            a = lat[i[:, None], i[None, :]]
            b = lat[i[:, None], i[None, :] + 1]
            cc = lat[i[:, None] + 1, i[None, :]]
            d = lat[i[:, None] + 1, i[None, :] + 1]
            fx = f[None, :]
            fy = f[:, None]
            acc += (2.0 ** -o) * ((a * (1 - fx) + b * fx) * (1 - fy) + (cc * (1 - fx) + d * fx) * fy)
        out[:, :, c] = acc / total
    return out.astype(np.float32)


def point_sample(texture: np.ndarray, uv: np.ndarray) -> np.ndarray:
    """Nearest-texel lookup: texel (min(floor(u*W), W-1), min(floor(v*H), H-1))."""
    h, w = texture.shape[:2]
    u = uv[:, 0].astype(np.float64)
    v = uv[:, 1].astype(np.float64)
    i = np.clip(np.floor(u * w).astype(np.int64), 0, w - 1)
    j = np.clip(np.floor(v * h).astype(np.int64), 0, h - 1)
    return texture[j, i].astype(np.float32)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
PAPER_SHIFT = ((0.0, 0.0), (0.5, 0.5), (0.0, 0.0), (0.5, 0.5))
NO_SHIFT = ((0.0, 0.0),) * 4


@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    out_w: int
    out_h: int
    latent_sizes: Tuple[Tuple[int, int], ...]
    dims: Tuple[int, ...]
    latent_format: str          # "bc1" | "f32"
    uv_kind: str                # "centre" | "jitter" | "random"
    order: str = "tiled"
    n_samples: int = 0          # for uv_kind == "random"
    shift: Tuple[Tuple[float, float], ...] = PAPER_SHIFT

    @property
    def n(self) -> int:
        return self.n_samples if self.uv_kind == "random" else self.out_w * self.out_h

    @property
    def mlp_macs(self) -> int:
        return sum(self.dims[i] * self.dims[i + 1] for i in range(len(self.dims) - 1))


WORKLOADS = {
    # 256^2 output, 4 BC1 levels 128..16, MLP 14-32-32-8, pixel-centre uv.
    "c1": Workload("c1", 1, 256, 256, ((128, 128), (64, 64), (32, 32), (16, 16)),
                   (14, 32, 32, 8), "bc1", "centre"),
    # 4096^2 output, 4 BC1 levels 2048..256, MLP 14-64-64-64-8, jittered uv.
    "c2": Workload("c2", 2, 4096, 4096, ((2048, 2048), (1024, 1024), (512, 512), (256, 256)),
                   (14, 64, 64, 64, 8), "bc1", "jitter"),
    # backward: float latents 1024..128, MLP 14-64-64-8, 2^20 random uv.
    "c3": Workload("c3", 3, 0, 0, ((1024, 1024), (512, 512), (256, 256), (128, 128)),
                   (14, 64, 64, 8), "f32", "random", n_samples=1 << 20),
    # FP8 decode: same inputs as c2 (seed 2).
    "c4": Workload("c4", 2, 4096, 4096, ((2048, 2048), (1024, 1024), (512, 512), (256, 256)),
                   (14, 64, 64, 64, 8), "bc1", "jitter"),
}


def make_workload(wl: Workload, bias: str = "zero", order: Optional[str] = None):
    """Draw (latents, Ws, bs, uv) for a workload.

    latents: list of uint64 block arrays (bc1) or float32 grids (f32).
    """
    s_lat, s_mlp, s_uv, _ = streams(wl.seed)
    if wl.latent_format == "bc1":
        lat = bc1_pyramid(s_lat, wl.latent_sizes)
    else:
        lat = f32_pyramid(s_lat, wl.latent_sizes)
    Ws, bs = xavier_mlp(s_mlp, wl.dims, bias=bias)
    order = order or wl.order
    if wl.uv_kind == "centre":
        uv = pixel_uv(wl.out_w, wl.out_h, order)
    elif wl.uv_kind == "jitter":
        uv = pixel_uv(wl.out_w, wl.out_h, order, jitter_rng=s_uv)
    else:
        uv = random_uv(s_uv, wl.n_samples)
    return lat, Ws, bs, uv


def c3_targets(size: int = 2048, seed: int = 3) -> np.ndarray:
    """The 8-channel value-noise target texture of the backward workload."""
    return value_noise_texture(streams(seed)[3], size)


def calibration_uv(n: int = 65536, seed: int = 4) -> np.ndarray:
    """FP8 activation-range calibration samples, uniform in [0,1)^2."""
    return random_uv(streams(seed)[2], n)


# ----------------------------------------------------------------------------
# Many materials in one batch
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class MaterialSpec:
    index: int
    side: int
    width: int      # hidden width
    depth: int      # number of hidden layers
    seed: int

    @property
    def latent_sizes(self):
        s = self.side
        return ((s // 2, s // 2), (s // 4, s // 4), (s // 8, s // 8), (s // 16, s // 16))

    @property
    def dims(self):
        return (14,) + (self.width,) * self.depth + (8,)

    @property
    def n(self):
        return self.side * self.side


def material_specs(n_materials: int = 64, seed: int = 5) -> List[MaterialSpec]:
    """Sides 64 * round(2^U(9,12) / 64), hidden width in {32, 64}, depth in {2, 3}."""
    rng = streams(seed)[3]
    specs = []
    child_seeds = np.random.SeedSequence(seed).spawn(n_materials + 4)[4:]
    for m in range(n_materials):
        e = rng.uniform(9.0, 12.0)
        side = int(64 * round((2.0 ** e) / 64.0))
        side = min(max(side, 512), 4096)
        width = int(rng.choice([32, 64]))
        depth = int(rng.choice([2, 3]))
        specs.append(MaterialSpec(m, side, width, depth, int(child_seeds[m].generate_state(1)[0])))
    return specs


def make_material(spec: MaterialSpec, bias: str = "zero"):
    """(bc1 latents, Ws, bs) of one material; uv are pixel centres in tiled order."""
    s_lat, s_mlp, _, _ = streams(spec.seed)
    lat = bc1_pyramid(s_lat, spec.latent_sizes)
    Ws, bs = xavier_mlp(s_mlp, spec.dims, bias=bias)
    return lat, Ws, bs


def bc1_mip_chain(rng: np.random.Generator, width: int, height: int, n_mips: int = 0) -> List[np.ndarray]:
    """BC1 mips of one latent level, mip m of (width >> m) x (height >> m)
    texels, each drawn independently like bc1_level (the mips of a trained
    level are separate textures); n_mips = 0: down to 4 texels on the short side."""
    if not n_mips:
        n_mips = int(np.log2(min(width, height) // 4)) + 1
    return [bc1_level(rng, width >> m, height >> m) for m in range(n_mips)]


def perspective_plane(width: int, height: int, far: float = 20.0):
    """(uv float32 [W*H][2], duv float32 [W*H][4]) of a textured ground plane
    seen in perspective, pixels row-major: row y is at distance
    z = 1 / (1/far + (1 - 1/far) (y + 1/2) / height) (far at the top),
    u = 1/2 + (x + 1/2 - width/2) z / (width far), v = (far - z) / (far - 1);
    duv = (du/dx, dv/dx, du/dy, dv/dy) analytically. Near rows are isotropic,
    far rows stretched along v by up to `far` : 1."""
    x = (np.arange(width, dtype=np.float64) + 0.5)[None, :]
    t = (np.arange(height, dtype=np.float64) + 0.5)[:, None] / height
    a = 1.0 / far
    z = 1.0 / (a + (1.0 - a) * t)
    dzdy = -(1.0 - a) / height * z * z
    cx = (x - width / 2) / (width * far)
    u = 0.5 + cx * z
    v = (far - z) / (far - 1.0) + 0.0 * x
    dudx = z / (width * far) + 0.0 * x
    dudy = cx * dzdy
    dvdx = np.zeros_like(u)
    dvdy = -dzdy / (far - 1.0) + 0.0 * x
    uv = np.stack([u, v], axis=-1).reshape(-1, 2).astype(np.float32)
    duv = np.stack([dudx, dvdx, dudy, dvdy], axis=-1).reshape(-1, 4).astype(np.float32)
    return uv, duv


def material_frame(rng: np.random.Generator, width: int, height: int, n_mats: int, n_cells: int = 0,
                   background: float = 0.15, noise: float = 0.0) -> np.ndarray:
    """uint16 [height][width] material ids of a synthetic frame: Voronoi cells
    around n_cells seeds (default 2 n_mats), each cell one material (drawn
    uniformly) or, with probability ``background``, no neural material
    (id 0xFFFF); a fraction ``noise`` of pixels then gets a random id (or
    background), which makes isolated mixed tiles."""
    n_cells = n_cells or 2 * n_mats
    sx = rng.random(n_cells) * width
    sy = rng.random(n_cells) * height
    cell_mat = rng.integers(0, n_mats, n_cells).astype(np.uint16)
    cell_mat[rng.random(n_cells) < background] = 0xFFFF
    out = np.empty((height, width), np.uint16)
    xs = np.arange(width, dtype=np.float64) + 0.5
    for y0 in range(0, height, 64):
        ys = np.arange(y0, min(y0 + 64, height), dtype=np.float64)[:, None] + 0.5
        best = np.full((ys.shape[0], width), np.inf)
        arg = np.zeros((ys.shape[0], width), np.int64)
        for c in range(n_cells):
            d = (xs[None, :] - sx[c]) ** 2 + (ys - sy[c]) ** 2
            closer = d < best
            best[closer] = d[closer]
            arg[closer] = c
        out[y0:y0 + ys.shape[0]] = cell_mat[arg]
    if noise > 0:
        hit = rng.random((height, width)) < noise
        ids = rng.integers(0, n_mats + 1, int(hit.sum()))
        out[hit] = np.where(ids == n_mats, 0xFFFF, ids).astype(np.uint16)
    return out


def pixel_uv_torch(width: int, height: int, order: str = "tiled", device="cuda"):
    """Pixel-centre uv of every screen pixel as a float32 [W*H][2] torch tensor
    built on `device` (same values as pixel_uv without jitter)."""
    import torch
    n = width * height
    k = torch.arange(n, dtype=torch.int64, device=device)
    if order == "rowmajor":
        x, y = k % width, k // width
    else:
        tiles_x = width // TILE
        t, r = k // (TILE * TILE), k % (TILE * TILE)
        x = (t % tiles_x) * TILE + r % TILE
        y = (t // tiles_x) * TILE + r // TILE
    uv = torch.empty((n, 2), dtype=torch.float32, device=device)
    uv[:, 0] = ((x.to(torch.float64) + 0.5) / width).to(torch.float32)
    uv[:, 1] = ((y.to(torch.float64) + 0.5) / height).to(torch.float32)
    return uv
