"""FP64 CPU oracle of the neural BC1 texture decode (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the GPU library or its
Python binding. The arithmetic lives in ``ntc_oracle.c`` (plain C, IEEE
double); this module only marshals numpy arrays.

Paper: Belcour & Benyoub, "Hardware Accelerated Neural Block Texture
Compression with Cooperative Vectors". Sec. 3.1 (architecture, latent BC1
compression, variants), Sec. 3.2 (gradients into MLP and latents), Sec. 3.3
(bilinear filtering of the latents).

Pins: every function here is checked in ``tests/test_oracle_*.py`` against
something other than itself (hand-built BC1 blocks, a second numpy BC1
decoder, closed forms of bilinear filtering, numpy matrix products,
numpy/torch narrow-format casts, finite differences, torch FP64 autograd).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ntc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libntc_oracle.so")

MAX_LEVELS = 8
MAX_LAYERS = 8

CLAMP, WRAP = 0, 1
EXACT, FP16, FP8, FP8_F16 = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile ntc_oracle.c with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Level(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("format", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("data", ctypes.c_void_p),
                ("shift_x", ctypes.c_double), ("shift_y", ctypes.c_double)]


class _Mlp(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32),
                ("dims", ctypes.c_int32 * (MAX_LAYERS + 1)),
                ("W", ctypes.c_void_p * MAX_LAYERS),
                ("b", ctypes.c_void_p * MAX_LAYERS),
                ("precision", ctypes.c_int32),
                ("w_scale", ctypes.c_void_p),
                ("a_scale", ctypes.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_round_f16.restype = ctypes.c_double
        lib.oracle_round_f16.argtypes = [ctypes.c_double]
        lib.oracle_round_e4m3_sat.restype = ctypes.c_double
        lib.oracle_round_e4m3_sat.argtypes = [ctypes.c_double]
        lib.oracle_max_threads.restype = ctypes.c_int32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Latents:
    """Latent pyramid for the oracle. ``levels`` are uint64 BC1 block arrays
    [(H/4)][(W/4)] or float grids [H][W][3]; ``shift`` per level in texels."""

    def __init__(self, levels: Sequence[np.ndarray], shift=None, address: int = CLAMP,
                 fmt: Optional[str] = None):
        self.arrays: List[np.ndarray] = []
        self.sizes = []
        fmts = []
        for a in levels:
            if a.dtype == np.uint64:
                a = np.ascontiguousarray(a)
                h, w = a.shape[0] * 4, a.shape[1] * 4
                fmts.append(0)
            else:
                a = np.ascontiguousarray(a, dtype=np.float64)
                h, w = a.shape[0], a.shape[1]
                assert a.shape[2] == 3
                fmts.append(1)
            self.arrays.append(a)
            self.sizes.append((w, h))
        if fmt is not None:
            assert all(f == (0 if fmt == "bc1" else 1) for f in fmts)
        shift = shift if shift is not None else [(0.0, 0.0)] * len(levels)
        self.n = len(levels)
        assert 1 <= self.n <= MAX_LEVELS
        self.c = (_Level * self.n)()
        for k, a in enumerate(self.arrays):
            w, h = self.sizes[k]
            self.c[k] = _Level(w, h, fmts[k], 0, a.ctypes.data, float(shift[k][0]), float(shift[k][1]))
        self.address = address


class Mlp:
    """MLP for the oracle: W[l] [dims[l+1]][dims[l]], b[l] [dims[l+1]] (any float dtype,
    widened to float64). precision: EXACT, FP16 (round inputs and weights to binary16),
    FP8 (scale and round to E4M3; needs w_scale and a_scale) or FP8_F16 (as FP8, but
    the scaled hidden activations are clamped to [0, 256] and reach E4M3 through
    binary16: 256 * round_f16(min(a s / 256, 1)), then E4M3)."""

    def __init__(self, Ws, bs, precision: int = EXACT, w_scale=None, a_scale=None):
        self.W = [np.ascontiguousarray(w, dtype=np.float64) for w in Ws]
        self.b = [np.ascontiguousarray(b, dtype=np.float64) for b in bs]
        L = len(self.W)
        assert 1 <= L <= MAX_LAYERS
        dims = [self.W[0].shape[1]] + [w.shape[0] for w in self.W]
        for l in range(L):
            assert self.W[l].shape == (dims[l + 1], dims[l])
            assert self.b[l].shape == (dims[l + 1],)
        self.dims = dims
        self.c = _Mlp()
        self.c.n_layers = L
        for i, d in enumerate(dims):
            self.c.dims[i] = d
        for l in range(L):
            self.c.W[l] = self.W[l].ctypes.data
            self.c.b[l] = self.b[l].ctypes.data
        self.c.precision = precision
        self._ws = self._as = None
        if precision in (FP8, FP8_F16):
            self._ws = np.ascontiguousarray(w_scale, dtype=np.float64)
            self._as = np.ascontiguousarray(a_scale, dtype=np.float64)
            assert self._ws.shape == (L,) and self._as.shape == (L,)
            self.c.w_scale = self._ws.ctypes.data
            self.c.a_scale = self._as.ctypes.data


def default_threads() -> int:
    return int(_load().oracle_max_threads())


def round_f16(x: float) -> float:
    return _load().oracle_round_f16(float(x))


def round_e4m3_sat(x: float) -> float:
    return _load().oracle_round_e4m3_sat(float(x))


def bc1_level(blocks: np.ndarray):
    """(num, den, value) of every texel: int32 [H][W][3] x2 and float64 [H][W][3]."""
    blocks = np.ascontiguousarray(blocks, dtype=np.uint64)
    h, w = blocks.shape[0] * 4, blocks.shape[1] * 4
    num = np.empty((h, w, 3), np.int32)
    den = np.empty((h, w, 3), np.int32)
    val = np.empty((h, w, 3), np.float64)
    _load().oracle_bc1_level(_ptr(blocks), ctypes.c_int32(w), ctypes.c_int32(h),
                             _ptr(num), _ptr(den), _ptr(val))
    return num, den, val


def features(lat: Latents, uv: np.ndarray, threads: int = 0) -> np.ndarray:
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    n = uv.shape[0]
    x = np.empty((n, 3 * lat.n + 2), np.float64)
    _load().oracle_features(lat.c, ctypes.c_int32(lat.n), ctypes.c_int32(lat.address), _ptr(uv),
                            ctypes.c_int64(n), _ptr(x), ctypes.c_int32(threads or default_threads()))
    return x


def mlp_forward(mlp: Mlp, x: np.ndarray, threads: int = 0) -> np.ndarray:
    """f(x) for given feature vectors x [n][dims[0]], float64 [n][C]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    assert x.shape[1] == mlp.dims[0]
    out = np.empty((n, mlp.dims[-1]), np.float64)
    _load().oracle_mlp_forward(ctypes.byref(mlp.c), _ptr(x), ctypes.c_int64(n), _ptr(out),
                               ctypes.c_int32(threads or default_threads()))
    return out


def decode(lat: Latents, mlp: Mlp, uv: np.ndarray, threads: int = 0) -> np.ndarray:
    """p(uv) = f(x(uv)) for every sample, float64 [n][C]."""
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    n = uv.shape[0]
    out = np.empty((n, mlp.dims[-1]), np.float64)
    _load().oracle_decode(lat.c, ctypes.c_int32(lat.n), ctypes.c_int32(lat.address), ctypes.byref(mlp.c), _ptr(uv),
                          ctypes.c_int64(n), _ptr(out), ctypes.c_int32(threads or default_threads()))
    return out


def decode_index(lat: Latents, mlp: Mlp, uv: np.ndarray, index: np.ndarray, threads: int = 0) -> np.ndarray:
    """p(uv[index[r]]) for the given sample indices, float64 [len(index)][C]."""
    uv = np.ascontiguousarray(uv, dtype=np.float64) if uv.dtype != np.float64 else np.ascontiguousarray(uv)
    index = np.ascontiguousarray(index, dtype=np.int64)
    assert index.size == 0 or (index.min() >= 0 and index.max() < uv.shape[0])
    out = np.empty((index.size, mlp.dims[-1]), np.float64)
    _load().oracle_decode_index(lat.c, ctypes.c_int32(lat.n), ctypes.c_int32(lat.address), ctypes.byref(mlp.c),
                                _ptr(uv), _ptr(index), ctypes.c_int64(index.size), _ptr(out),
                                ctypes.c_int32(threads or default_threads()))
    return out


def layer_amax(lat: Latents, mlp: Mlp, uv: np.ndarray) -> np.ndarray:
    """Largest |input| of each layer over the samples (float64 [n_layers])."""
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    amax = np.zeros(len(mlp.W), np.float64)
    _load().oracle_layer_amax(lat.c, ctypes.c_int32(lat.n), ctypes.c_int32(lat.address), ctypes.byref(mlp.c),
                              _ptr(uv), ctypes.c_int64(uv.shape[0]), _ptr(amax))
    return amax


def fp8_scales(Ws, amax_act, pow2: bool = False):
    """Per-layer E4M3 scales: s = 448 / max|.| computed in float32, as float64
    values. With pow2, the power-of-two form the matrix-core path stores:
    weights 2^floor(log2(448 / max|W_l|)); first-layer inputs
    2^floor(log2(448 / max(amax_0, 1))) (BC1 latent values reach 1 whatever
    the calibration saw); hidden activations 2^floor(log2(256 / amax_l)),
    whose scaled values are clamped to [0, 256] (precision FP8_F16)."""
    if pow2:
        def p2(x):
            return float(np.ldexp(1.0, np.frexp(np.float64(x))[1] - 1))
        w_scale = np.array([p2(448.0 / np.max(np.abs(np.asarray(w, np.float32)))) for w in Ws], dtype=np.float64)
        a_scale = np.array([p2(448.0 / max(float(a), 1.0)) if l == 0 else (p2(256.0 / float(a)) if a > 0 else 1.0)
                            for l, a in enumerate(amax_act)], dtype=np.float64)
        return w_scale, a_scale
    w_scale = np.array([np.float32(448.0) / np.float32(np.max(np.abs(np.asarray(w, np.float32))))
                        for w in Ws], dtype=np.float64)
    a_scale = np.array([np.float32(448.0) / np.float32(a) for a in amax_act], dtype=np.float64)
    return w_scale, a_scale


def relu_margin(lat: Latents, mlp: Mlp, uv: np.ndarray, threads: int = 0) -> np.ndarray:
    """Per sample, the smallest |pre-activation| over all hidden units."""
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    out = np.empty(uv.shape[0], np.float64)
    _load().oracle_relu_margin(lat.c, ctypes.c_int32(lat.n), ctypes.c_int32(lat.address), ctypes.byref(mlp.c),
                               _ptr(uv), ctypes.c_int64(uv.shape[0]), _ptr(out),
                               ctypes.c_int32(threads or default_threads()))
    return out


def backward(lat: Latents, mlp: Mlp, uv: np.ndarray, grad_out: np.ndarray, threads: int = 0):
    """Gradients of sum(grad_out * p(uv)) w.r.t. W, b and float latent grids.

    Returns (gW list, gb list, glat list), float64."""
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    g = np.ascontiguousarray(grad_out, dtype=np.float64)
    n = uv.shape[0]
    assert g.shape == (n, mlp.dims[-1])
    gW = [np.zeros_like(w) for w in mlp.W]
    gb = [np.zeros_like(b) for b in mlp.b]
    glat = [np.zeros((h, w, 3), np.float64) for (w, h) in lat.sizes]
    L = len(gW)
    pW = (ctypes.c_void_p * L)(*[a.ctypes.data for a in gW])
    pb = (ctypes.c_void_p * L)(*[a.ctypes.data for a in gb])
    pl = (ctypes.c_void_p * lat.n)(*[a.ctypes.data for a in glat])
    _load().oracle_backward(lat.c, ctypes.c_int32(lat.n), ctypes.c_int32(lat.address), ctypes.byref(mlp.c), _ptr(uv),
                            ctypes.c_int64(n), _ptr(g), pW, pb, pl,
                            ctypes.c_int32(threads or default_threads()))
    return gW, gb, glat
