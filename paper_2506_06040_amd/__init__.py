"""MI355X (gfx950) neural BC1 texture decode.

Hot path of Belcour & Benyoub, "Hardware Accelerated Neural Block Texture
Compression with Cooperative Vectors": BC1 latent fetch and integer decode,
bilinear filtering, concatenation and a small MLP, as hand-written HIP
kernels behind the C ABI of include/ntc.h (libntc.so, built in-tree).
"""
from ._abi import NtcError  # noqa: F401
from .api import (  # noqa: F401
    NO_SHIFT, PAPER_SHIFT, BatchPlan, Latents, Material, Mlp, NtcDecodeFn, batch_cfg, bc1_decode_texels,
    calibrate_fp8, decode, decode_backward, decode_fn, pack, pack_size, tile_cfg,
    QAT_PARAMS, QatTexelsFn, qat_backward, qat_export_bc1, qat_texels, qat_texels_fn,
    FrameDecoder, classify, gather_uv, scatter_rows, LatentMips, decode_filtered,
)
from . import autotune  # noqa: F401,E402
