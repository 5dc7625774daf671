"""Python face of libntc: torch tensors in, torch tensors out.

PyTorch provides device memory and the current stream; every computation is
one of libntc's HIP kernels, called through the C ABI declared in
include/ntc.h. Names follow the paper (Belcour & Benyoub): latents T_k
(Sec. 3.1), the MLP f (Sec. 3.1), the decode p(uv) = f(x(uv)).
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi as A
from ._abi import NtcError, check

PAPER_SHIFT = ((0.0, 0.0), (0.5, 0.5), (0.0, 0.0), (0.5, 0.5))
NO_SHIFT = ((0.0, 0.0),) * 4

COMPUTE = {"f32": A.F32, "f16": A.F16, "bf16": A.BF16, "fp8": A.FP8_E4M3}
OUT_DTYPES = {torch.float32: A.F32, torch.float16: A.F16}


def _stream_handle(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _require_cuda(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Latents:
    """Latent pyramid T_0..T_{K-1} (Sec. 3.1) on the device.

    levels: BC1 block arrays (int64 / uint64 [(H/4)][(W/4)], the 64-bit block
    words) or float32 grids [H][W][3]; numpy arrays are copied to `device`.
    shift: per-level sampling offset in texels (paper: half a texel on the
    second and fourth textures). address: "clamp" or "wrap".
    """

    def __init__(self, levels: Sequence, shift=PAPER_SHIFT, address: str = "clamp", device="cuda"):
        if not 1 <= len(levels) <= A.MAX_LEVELS:
            raise ValueError("1..4 latent levels")
        self.tensors: List[torch.Tensor] = []
        fmt = None
        sizes = []
        for lv in levels:
            if isinstance(lv, np.ndarray):
                if lv.dtype == np.uint64:
                    lv = torch.from_numpy(np.ascontiguousarray(lv).view(np.int64))
                else:
                    lv = torch.from_numpy(np.ascontiguousarray(lv, dtype=np.float32))
                lv = lv.to(device)
            if lv.dtype in (torch.int64, torch.uint64):
                f = A.LATENT_BC1
                h, w = lv.shape[0] * 4, lv.shape[1] * 4
            elif lv.dtype == torch.float32:
                f = A.LATENT_F32
                h, w = lv.shape[0], lv.shape[1]
                if lv.dim() != 3 or lv.shape[2] != 3:
                    raise ValueError("float latents are [H][W][3]")
            else:
                raise ValueError(f"unsupported latent dtype {lv.dtype}")
            if fmt is not None and f != fmt:
                raise ValueError("all levels must share one format")
            fmt = f
            _require_cuda(lv, "latent level")
            self.tensors.append(lv)
            sizes.append((w, h))
        self.format = fmt
        self.sizes = sizes
        self.shift = tuple(tuple(map(float, s)) for s in shift[:len(levels)])
        self.address = {"clamp": A.CLAMP, "wrap": A.WRAP}[address]
        c = A.ntc_latents()
        c.n_levels = len(levels)
        c.format = fmt
        c.address = self.address
        c.reserved = 0
        for k, t in enumerate(self.tensors):
            c.width[k], c.height[k] = sizes[k]
            c.shift[k][0], c.shift[k][1] = self.shift[k]
            c.data[k] = t.data_ptr()
        self.c = c

    @property
    def n_levels(self) -> int:
        return len(self.tensors)


class Mlp:
    """MLP f (Sec. 3.1): W[l] float32 [dims[l+1]][dims[l]], b[l] float32 [dims[l+1]]."""

    def __init__(self, Ws, bs, device="cuda"):
        self.W = [torch.as_tensor(np.asarray(w) if isinstance(w, np.ndarray) else w).to(device, torch.float32).contiguous()
                  for w in Ws]
        self.b = [torch.as_tensor(np.asarray(b) if isinstance(b, np.ndarray) else b).to(device, torch.float32).contiguous()
                  for b in bs]
        if not 2 <= len(self.W) <= A.MAX_LAYERS:
            raise ValueError("2..5 layers")
        self.dims = [self.W[0].shape[1]] + [w.shape[0] for w in self.W]
        c = A.ntc_mlp()
        c.n_layers = len(self.W)
        for i, d in enumerate(self.dims):
            c.dims[i] = d
        for l in range(len(self.W)):
            c.W[l] = self.W[l].data_ptr()
            c.b[l] = self.b[l].data_ptr()
        self.c = c

    @classmethod
    def shape_only(cls, dims):
        m = cls.__new__(cls)
        m.W, m.b, m.dims = [], [], list(dims)
        c = A.ntc_mlp()
        c.n_layers = len(dims) - 1
        for i, d in enumerate(dims):
            c.dims[i] = d
        m.c = c
        return m

    @property
    def n_out(self) -> int:
        return self.dims[-1]


def pack_size(mlp: Mlp, compute: str) -> int:
    n = ctypes.c_size_t(0)
    check(A.lib().ntc_mlp_pack_size(ctypes.byref(mlp.c), COMPUTE[compute], ctypes.byref(n)))
    return n.value


def pack(mlp: Mlp, compute: str, act_amax: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Packed weight image for `compute` ("f32", "f16" or "fp8")."""
    nbytes = pack_size(mlp, compute)
    dev = mlp.W[0].device
    buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    check(A.lib().ntc_mlp_pack(ctypes.byref(mlp.c), COMPUTE[compute], _ptr(act_amax), _ptr(buf),
                               ctypes.c_size_t(nbytes), _stream_handle()))
    return buf


def calibrate_fp8(lat: Latents, mlp: Mlp, uv: torch.Tensor, packed_f32: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Largest |input| of every layer over the calibration samples uv."""
    _require_cuda(uv, "uv")
    if packed_f32 is None:
        packed_f32 = pack(mlp, "f32")
    amax = torch.empty(len(mlp.W), dtype=torch.float32, device=uv.device)
    check(A.lib().ntc_calibrate_fp8(ctypes.byref(lat.c), ctypes.byref(mlp.c), _ptr(packed_f32), _ptr(uv),
                                    ctypes.c_int64(uv.shape[0]), _ptr(amax), _stream_handle()))
    return amax


def tile_cfg(waves_per_cu: int = 0, stage_capacity: int = 0, tiles_per_iter: int = 0) -> A.ntc_tile_cfg:
    c = A.ntc_tile_cfg()
    c.waves_per_cu = waves_per_cu
    c.tiles_per_iter = tiles_per_iter
    c.stage_capacity = stage_capacity
    c.reserved = 0
    return c


def decode(lat: Latents, mlp: Mlp, uv: torch.Tensor, compute: str = "f16", packed: Optional[torch.Tensor] = None,
           out_dtype=torch.float32, cfg: Optional[A.ntc_tile_cfg] = None, out: Optional[torch.Tensor] = None,
           stream=None) -> torch.Tensor:
    """p(uv) = f(x(uv)) for every row of uv (float32 [n][2]); returns [n][C]."""
    _require_cuda(uv, "uv")
    if uv.dtype != torch.float32 or uv.dim() != 2 or uv.shape[1] != 2:
        raise ValueError("uv must be float32 [n][2]")
    if packed is None:
        packed = pack(mlp, compute)
    n = uv.shape[0]
    if out is None:
        out = torch.empty((n, mlp.n_out), dtype=out_dtype, device=uv.device)
    check(A.lib().ntc_decode(ctypes.byref(lat.c), ctypes.byref(mlp.c), COMPUTE[compute], _ptr(packed), _ptr(uv),
                             ctypes.c_int64(n), _ptr(out), OUT_DTYPES[out.dtype],
                             ctypes.byref(cfg) if cfg is not None else None, _stream_handle(stream)))
    return out


def bc1_decode_texels(lat: Latents, level: int):
    """(value float32 [H][W][3], numerator int32 [H][W][3]) of one BC1 level."""
    w, h = lat.sizes[level]
    dev = lat.tensors[level].device
    val = torch.empty((h, w, 3), dtype=torch.float32, device=dev)
    num = torch.empty((h, w, 3), dtype=torch.int16, device=dev)
    check(A.lib().ntc_bc1_decode_texels(ctypes.byref(lat.c), level, _ptr(val), _ptr(num), _stream_handle()))
    return val, num.to(torch.int32) & 0xFFFF


# ---------------------------------------------------------------------------
# Backward (Sec. 3.2)
# ---------------------------------------------------------------------------
def backward_workspace_size(lat: Latents, mlp: Mlp, n: int) -> int:
    b = ctypes.c_size_t(0)
    check(A.lib().ntc_decode_backward_workspace(ctypes.byref(lat.c), ctypes.byref(mlp.c), ctypes.c_int64(n),
                                                 ctypes.byref(b)))
    return b.value


def decode_backward(lat: Latents, mlp: Mlp, uv: torch.Tensor, grad_out: torch.Tensor,
                    workspace: Optional[torch.Tensor] = None):
    """Gradients (grad_W list, grad_b list, grad_latents list) of
    sum(grad_out * p(uv)) for float latents."""
    _require_cuda(uv, "uv")
    grad_out = grad_out.contiguous()
    _require_cuda(grad_out, "grad_out")
    if grad_out.dtype != torch.float32 or grad_out.shape != (uv.shape[0], mlp.n_out):
        raise ValueError("grad_out must be float32 [n][C]")
    n = uv.shape[0]
    dev = uv.device
    gW = [torch.empty_like(w) for w in mlp.W]
    gb = [torch.empty_like(b) for b in mlp.b]
    gl = [torch.empty_like(t) for t in lat.tensors]
    nbytes = backward_workspace_size(lat, mlp, n)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    L = len(gW)
    pW = (ctypes.c_void_p * L)(*[t.data_ptr() for t in gW])
    pb = (ctypes.c_void_p * L)(*[t.data_ptr() for t in gb])
    pl = (ctypes.c_void_p * len(gl))(*[t.data_ptr() for t in gl])
    check(A.lib().ntc_decode_backward(ctypes.byref(lat.c), ctypes.byref(mlp.c), _ptr(uv), ctypes.c_int64(n),
                                      _ptr(grad_out), pW, pb, pl, _ptr(workspace), ctypes.c_size_t(nbytes),
                                      _stream_handle()))
    return gW, gb, gl


class NtcDecodeFn(torch.autograd.Function):
    """out = p(uv) for float latents with the plain FP32 decode; backward by
    the hand-written gradient kernel. Only the inputs are saved: activations
    are recomputed per tile in the backward kernel.

    apply(uv, shift, address, n_levels, latent_0..latent_{K-1}, W_0, b_0, ..., W_{L-1}, b_{L-1})
    """

    @staticmethod
    def forward(ctx, uv, shift, address, n_levels, *params):
        lat_t = list(params[:n_levels])
        wb = params[n_levels:]
        Ws, bs = list(wb[0::2]), list(wb[1::2])
        lat = Latents([t.detach().contiguous() for t in lat_t], shift=shift, address=address)
        mlp = Mlp([w.detach() for w in Ws], [b.detach() for b in bs])
        out = decode(lat, mlp, uv.detach().contiguous(), compute="f32")
        ctx.save_for_backward(uv, *params)
        ctx.meta = (shift, address, n_levels)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        shift, address, n_levels = ctx.meta
        saved = ctx.saved_tensors
        uv, params = saved[0], saved[1:]
        lat_t = list(params[:n_levels])
        wb = params[n_levels:]
        lat = Latents([t.detach().contiguous() for t in lat_t], shift=shift, address=address)
        mlp = Mlp([w.detach() for w in wb[0::2]], [b.detach() for b in wb[1::2]])
        gW, gb, gl = decode_backward(lat, mlp, uv.detach().contiguous(), grad_out.float())
        grads = list(gl)
        for w, b in zip(gW, gb):
            grads += [w, b]
        return (None, None, None, None) + tuple(grads)


def decode_fn(uv, latents: Sequence[torch.Tensor], Ws: Sequence[torch.Tensor], bs: Sequence[torch.Tensor],
              shift=PAPER_SHIFT, address: str = "clamp"):
    """Differentiable decode of float latents (see NtcDecodeFn)."""
    params = list(latents)
    for w, b in zip(Ws, bs):
        params += [w, b]
    return NtcDecodeFn.apply(uv, tuple(shift[:len(latents)]), address, len(latents), *params)


# ---------------------------------------------------------------------------
# Trainable BC1 latents (Sec. 3.2, Eqs. 1-3)
# ---------------------------------------------------------------------------
QAT_PARAMS = 22  # per block: e0 (r, g, b), e1 (r, g, b), 16 texel weights


def _qat_check(params: torch.Tensor, width: int, height: int):
    _require_cuda(params, "params")
    if params.dtype != torch.float32 or not params.is_contiguous():
        raise ValueError("params must be contiguous float32")
    if tuple(params.shape) != (height // 4, width // 4, QAT_PARAMS):
        raise ValueError(f"params shape {tuple(params.shape)} != {(height // 4, width // 4, QAT_PARAMS)}")


def qat_texels(params: torch.Tensor, width: int, height: int) -> torch.Tensor:
    """Quantised texel values [height][width][3] of a trainable BC1 level."""
    _qat_check(params, width, height)
    out = torch.empty((height, width, 3), dtype=torch.float32, device=params.device)
    A.check(A.lib().ntc_qat_texels(_ptr(params), width, height, _ptr(out), _stream_handle()))
    return out


def qat_backward(params: torch.Tensor, width: int, height: int, grad_texels: torch.Tensor) -> torch.Tensor:
    """Gradient w.r.t. the logits, the quantisation passed through."""
    _qat_check(params, width, height)
    g = grad_texels.float().contiguous()
    if tuple(g.shape) != (height, width, 3):
        raise ValueError("grad_texels must be [height][width][3]")
    out = torch.empty_like(params)
    A.check(A.lib().ntc_qat_backward(_ptr(params), width, height, _ptr(g), _ptr(out), _stream_handle()))
    return out


def qat_export_bc1(params: torch.Tensor, width: int, height: int) -> torch.Tensor:
    """BC1 blocks [height/4][width/4] (uint64 bit patterns in an int64 tensor)
    whose decode equals qat_texels."""
    _qat_check(params, width, height)
    out = torch.empty((height // 4, width // 4), dtype=torch.int64, device=params.device)
    A.check(A.lib().ntc_qat_export_bc1(_ptr(params), width, height, _ptr(out), _stream_handle()))
    return out


class QatTexelsFn(torch.autograd.Function):
    """texels = qat_texels(params); backward by ntc_qat_backward."""

    @staticmethod
    def forward(ctx, params, width, height):
        p = params.detach().contiguous()
        ctx.save_for_backward(p)
        ctx.size = (width, height)
        return qat_texels(p, width, height)

    @staticmethod
    def backward(ctx, grad):
        (p,) = ctx.saved_tensors
        w, h = ctx.size
        return qat_backward(p, w, h, grad), None, None


def qat_texels_fn(params: torch.Tensor, width: int, height: int) -> torch.Tensor:
    """Differentiable quantised texels of a trainable BC1 level."""
    return QatTexelsFn.apply(params, width, height)


# ---------------------------------------------------------------------------
# Many materials in one launch (Sec. 4 grouping by MLP)
# ---------------------------------------------------------------------------
class Material:
    """One material of a batch: BC1 latents, its MLP (FP16 image packed on
    construction), its uv and an output buffer. With pixel_index (int32 [n]),
    uv and out are whole images ([P][2], [P][C]) and sample s is pixel
    pixel_index[s] of them."""

    def __init__(self, lat: Latents, mlp: Mlp, uv: torch.Tensor, out: Optional[torch.Tensor] = None,
                 out_dtype=torch.float32, packed: Optional[torch.Tensor] = None,
                 pixel_index: Optional[torch.Tensor] = None):
        _require_cuda(uv, "uv")
        self.lat, self.mlp, self.uv = lat, mlp, uv
        self.pixel_index = pixel_index
        self.packed = packed if packed is not None else pack(mlp, "f16")
        self.out = out if out is not None else torch.empty((uv.shape[0], mlp.n_out), dtype=out_dtype,
                                                           device=uv.device)
        c = A.ntc_material()
        c.lat = lat.c
        c.mlp = mlp.c
        c.packed = self.packed.data_ptr()
        c.uv = uv.data_ptr()
        c.out = self.out.data_ptr()
        c.out_dtype = OUT_DTYPES[self.out.dtype]
        c.reserved = 0
        if pixel_index is None:
            c.n = uv.shape[0]
            c.pixel_index = None
            c.image_pixels = 0
        else:
            if pixel_index.dtype != torch.int32 or not pixel_index.is_contiguous():
                raise ValueError("pixel_index must be contiguous int32")
            c.n = pixel_index.shape[0]
            c.pixel_index = pixel_index.data_ptr()
            c.image_pixels = uv.numel() // 2
        self.c = c


def batch_cfg(item_pixels: int = 0, waves_per_cu: int = 0, stage_capacity: int = 0, n_cus: int = 0):
    c = A.ntc_batch_cfg()
    c.item_pixels, c.waves_per_cu, c.stage_capacity, c.n_cus = item_pixels, waves_per_cu, stage_capacity, n_cus
    return c


class BatchPlan:
    """Host plan image + its device copy for ntc_decode_batched."""

    def __init__(self, materials: Sequence[Material], cfg=None, device="cuda"):
        self.materials = list(materials)
        arr = (A.ntc_material * len(self.materials))(*[m.c for m in self.materials])
        self._arr = arr
        self.cfg = cfg if cfg is not None else batch_cfg(n_cus=_device_cus(device))
        n = ctypes.c_size_t(0)
        check(A.lib().ntc_batched_plan_size(arr, len(self.materials), ctypes.byref(self.cfg), ctypes.byref(n)))
        self.nbytes = n.value
        self.host = np.zeros(self.nbytes, dtype=np.uint8)
        check(A.lib().ntc_batched_plan(arr, len(self.materials), ctypes.byref(self.cfg),
                                       self.host.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(self.nbytes)))
        self.dev = torch.from_numpy(self.host).to(device)
        torch.cuda.synchronize(device)

    def header(self):
        h = self.host[:64].view(np.int32)
        return dict(n_mats=int(h[2]), n_items=int(h[3]), n_waves=int(h[4]), stage_cap=int(h[5]))

    def launch(self, stream=None):
        check(A.lib().ntc_decode_batched(self.host.ctypes.data_as(ctypes.c_void_p), _ptr(self.dev),
                                         ctypes.c_size_t(self.nbytes), _stream_handle(stream)))


def _device_cus(device="cuda") -> int:
    return torch.cuda.get_device_properties(torch.device(device)).multi_processor_count


# ---------------------------------------------------------------------------
# Frame classification by material and the frame decode it feeds
# (Sec. 4 "Tile-based classification", Algorithm 1)
# ---------------------------------------------------------------------------
def classify(mat_ids: torch.Tensor, n_mats: int, tile_class: bool = True):
    """Classify the 8x4 tiles of a frame (uint16 material ids [H][W]; ids >=
    n_mats are not neural). Returns (pixel_list int32 [valid], mat_offsets
    int32 [n_mats + 1], mat_simple int32 [n_mats], tile_class uint8 [tiles]
    or None); pixel_list is sliced to the valid count, which takes one
    device-to-host copy of mat_offsets[n_mats]."""
    _require_cuda(mat_ids, "mat_ids")
    if mat_ids.dtype not in (torch.uint16, torch.int16) or mat_ids.dim() != 2 or not mat_ids.is_contiguous():
        raise ValueError("mat_ids must be a contiguous [H][W] uint16 (or int16 bit pattern) tensor")
    h, w = mat_ids.shape
    dev = mat_ids.device
    ws = ctypes.c_size_t(0)
    check(A.lib().ntc_classify_workspace(w, h, n_mats, ctypes.byref(ws)))
    work = torch.empty(max(ws.value, 1), dtype=torch.uint8, device=dev)
    lst = torch.empty(w * h, dtype=torch.int32, device=dev)
    off = torch.empty(n_mats + 1, dtype=torch.int32, device=dev)
    simple = torch.empty(n_mats, dtype=torch.int32, device=dev)
    tiles = ((w + 7) // 8) * ((h + 3) // 4)
    tcls = torch.empty(tiles, dtype=torch.uint8, device=dev) if tile_class else None
    check(A.lib().ntc_classify(_ptr(mat_ids), w, h, n_mats, _ptr(lst), _ptr(off), _ptr(simple), _ptr(tcls),
                               _ptr(work), ctypes.c_size_t(ws.value), _stream_handle()))
    n = int(off[n_mats].item())
    return lst[:n], off, simple, tcls


def gather_uv(uv_image: torch.Tensor, pixel_list: torch.Tensor) -> torch.Tensor:
    """uv of the listed pixels: uv_image float [H*W][2] (or [H][W][2])."""
    _require_cuda(uv_image, "uv_image")
    uvi = uv_image.reshape(-1, 2)
    if uvi.dtype != torch.float32 or not uvi.is_contiguous():
        raise ValueError("uv_image must be contiguous float32")
    n = pixel_list.shape[0]
    out = torch.empty((n, 2), dtype=torch.float32, device=uv_image.device)
    check(A.lib().ntc_gather_uv(_ptr(uvi), _ptr(pixel_list), n, _ptr(out), _stream_handle()))
    return out


def scatter_rows(rows: torch.Tensor, pixel_list: torch.Tensor, image: torch.Tensor) -> None:
    """image[pixel_list[i]] = rows[i]; image [H*W][C] (or [H][W][C]) of the rows' dtype."""
    _require_cuda(rows, "rows")
    img = image.reshape(-1, rows.shape[1])
    if img.data_ptr() != image.data_ptr() or not image.is_contiguous() or image.dtype != rows.dtype:
        raise ValueError("image must be contiguous with the rows' dtype")
    check(A.lib().ntc_scatter_rows(_ptr(rows), _ptr(pixel_list), rows.shape[0], rows.shape[1],
                                   OUT_DTYPES[rows.dtype], _ptr(img), _stream_handle()))


class FrameDecoder:
    """Decode a frame whose pixels use several neural materials: classify
    the tiles, gather the uv of every material's pixels, decode them with
    one batched launch (FP16 matrix cores) and scatter the outputs back.
    materials: sequence of (Latents, Mlp) with a common output width."""

    def __init__(self, materials, cfg=None, out_dtype=torch.float32, device="cuda"):
        self.materials = list(materials)
        widths = {m.n_out for _, m in self.materials}
        if len(widths) != 1:
            raise ValueError("materials must share the output width")
        self.n_out = widths.pop()
        self.packed = [pack(m, "f16") for _, m in self.materials]
        self.cfg, self.out_dtype, self.device = cfg, out_dtype, device

    def plan(self, mat_ids: torch.Tensor, uv_image: torch.Tensor, out: Optional[torch.Tensor] = None,
             indexed: bool = True):
        """Classification and the batch plan of one frame. indexed: the
        decode reads uv from uv_image and writes `out` ([H][W][C]) through
        the pixel lists; otherwise uv is gathered into per-material arrays
        and the rows are decoded into a separate buffer (to be scattered)."""
        lst, off, simple, tcls = classify(mat_ids, len(self.materials))
        offs = off.cpu().tolist()
        mats = []
        if indexed:
            if out is None:
                out = torch.zeros((mat_ids.shape[0], mat_ids.shape[1], self.n_out), dtype=self.out_dtype,
                                  device=self.device)
            uv = uv_image.reshape(-1, 2)
            rows = out.reshape(-1, self.n_out)
            for m, (lat, mlp) in enumerate(self.materials):
                a, b = offs[m], offs[m + 1]
                if b > a:
                    mats.append(Material(lat, mlp, uv, out=rows, packed=self.packed[m], pixel_index=lst[a:b]))
        else:
            uv = gather_uv(uv_image, lst)
            rows = torch.empty((lst.shape[0], self.n_out), dtype=self.out_dtype, device=self.device)
            for m, (lat, mlp) in enumerate(self.materials):
                a, b = offs[m], offs[m + 1]
                if b > a:
                    mats.append(Material(lat, mlp, uv[a:b], out=rows[a:b], packed=self.packed[m]))
        cfg = self.cfg
        if cfg is None and mats:
            # about two work items per persistent wave: a frame's materials
            # cover very different pixel counts, and longest-first packing
            # balances only when items outnumber waves
            n_cus = _device_cus(self.device)
            waves = n_cus * 8
            item = int(min(65536, max(64, (lst.shape[0] // (2 * waves)) // 64 * 64)))
            cfg = batch_cfg(item_pixels=item, waves_per_cu=8, n_cus=n_cus)
        plan = BatchPlan(mats, cfg, device=self.device) if mats else None
        return dict(pixel_list=lst, mat_offsets=off, mat_simple=simple, tile_class=tcls, uv=uv, rows=rows,
                    plan=plan, materials=mats, indexed=indexed)

    def decode(self, mat_ids: torch.Tensor, uv_image: torch.Tensor, out: Optional[torch.Tensor] = None,
               indexed: bool = True):
        """Output image [H][W][C]; pixels without a neural material keep the
        value of `out` (zero when it is not given)."""
        h, w = mat_ids.shape
        if out is None:
            out = torch.zeros((h, w, self.n_out), dtype=self.out_dtype, device=self.device)
        if not out.is_contiguous() or out.dtype != self.out_dtype or tuple(out.shape) != (h, w, self.n_out):
            raise ValueError("out must be a contiguous [H][W][C] image of the decoder's dtype")
        p = self.plan(mat_ids, uv_image, out=out, indexed=indexed)
        if p["plan"] is not None:
            p["plan"].launch()
            if not indexed:
                scatter_rows(p["rows"], p["pixel_list"], out)
        return out


# ---------------------------------------------------------------------------
# Mip-mapped latents and filtered sampling (Sec. 3.2 mip chains, Sec. 3.3)
# ---------------------------------------------------------------------------
FILTERS = {"trilinear": A.FILTER_TRILINEAR, "anisotropic": A.FILTER_ANISOTROPIC}


class LatentMips:
    """Latent levels with a BC1 mip chain each: levels[k][m] is the block
    array (uint64 / int64 [(H_k >> m)/4][(W_k >> m)/4]) of mip m of level k.
    shift: per-level sampling offset in texels of each mip."""

    def __init__(self, levels: Sequence[Sequence], shift=PAPER_SHIFT, device="cuda"):
        if not 1 <= len(levels) <= A.MAX_LEVELS:
            raise ValueError("1..4 latent levels")
        self.tensors = []
        c = A.ntc_latent_mips()
        c.n_levels = len(levels)
        self.shift = tuple(tuple(map(float, s)) for s in shift[:len(levels)])
        self.sizes = []
        for k, chain in enumerate(levels):
            if not 1 <= len(chain) <= A.MAX_MIPS:
                raise ValueError(f"level {k}: 1..{A.MAX_MIPS} mips")
            ts = []
            for b in chain:
                t = torch.from_numpy(np.ascontiguousarray(b).view(np.int64)) if isinstance(b, np.ndarray) else b
                ts.append(t.to(device))
            self.tensors.append(ts)
            h, w = ts[0].shape[0] * 4, ts[0].shape[1] * 4
            self.sizes.append((w, h))
            c.n_mips[k] = len(ts)
            c.width[k], c.height[k] = w, h
            c.shift[k][0], c.shift[k][1] = self.shift[k]
            for m, t in enumerate(ts):
                c.data[k][m] = t.data_ptr()
        self.c = c

    @property
    def n_levels(self) -> int:
        return len(self.tensors)


def decode_filtered(lat: LatentMips, mlp: Mlp, uv: torch.Tensor, duv: torch.Tensor, filter: str = "trilinear",
                    max_aniso: int = 16, packed: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                    out_dtype=torch.float32) -> torch.Tensor:
    """FP16 matrix-core decode with trilinear or anisotropic filtering of the
    latents over their mip chains; duv [n][4] = (du/dx, dv/dx, du/dy, dv/dy)."""
    _require_cuda(uv, "uv")
    _require_cuda(duv, "duv")
    n = uv.shape[0]
    if uv.dim() != 2 or uv.shape[1] != 2 or uv.dtype != torch.float32 or not uv.is_contiguous():
        raise ValueError("uv must be contiguous float32 [n][2]")
    if tuple(duv.shape) != (n, 4) or duv.dtype != torch.float32 or not duv.is_contiguous():
        raise ValueError("duv must be contiguous float32 [n][4]")
    if packed is None:
        packed = pack(mlp, "f16")
    if out is None:
        out = torch.empty((n, mlp.n_out), dtype=out_dtype, device=uv.device)
    check(A.lib().ntc_decode_filtered(ctypes.byref(lat.c), ctypes.byref(mlp.c), _ptr(packed), _ptr(uv), _ptr(duv), n,
                                      _ptr(out), OUT_DTYPES[out.dtype], FILTERS[filter], max_aniso,
                                      _stream_handle()))
    return out
