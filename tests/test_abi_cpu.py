"""The C-ABI library loads on a host without a GPU, exports every symbol that
include/ntc.h declares, and rejects bad arguments on the host (before any
HIP call) with the documented status codes. No compute call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntc.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ntc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def A():
    from paper_2506_06040_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libntc.so is not built; build it with python paper_2506_06040_amd/build.py")
    _abi.lib()
    return _abi


def test_exports_every_declared_symbol(A):
    names = _declared_functions()
    assert len(names) >= 12
    L = ctypes.CDLL(A.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(A.SIGNATURES), set(names) ^ set(A.SIGNATURES)


def test_status_strings(A):
    L = A.lib()
    for s in range(7):
        assert L.ntc_status_string(s).decode().startswith("NTC_")
    assert L.ntc_version() > 0


def _lat(A, fmt=0, n_levels=4, sizes=((64, 64), (32, 32), (16, 16), (8, 8)), data=0x1000):
    c = A.ntc_latents()
    c.n_levels = n_levels
    c.format = fmt
    c.address = 0
    c.reserved = 0
    for k in range(n_levels):
        c.width[k], c.height[k] = sizes[k]
        c.data[k] = data
    return c


def _mlp(A, dims=(14, 32, 32, 8), ptr=0x1000):
    c = A.ntc_mlp()
    c.n_layers = len(dims) - 1
    for i, d in enumerate(dims):
        c.dims[i] = d
    for l in range(len(dims) - 1):
        c.W[l] = ptr
        c.b[l] = ptr
    return c


def _decode(A, lat, mlp, compute=1, packed=0x1000, uv=0x1000, n=100, out=0x1000, out_dtype=0, cfg=None):
    return A.lib().ntc_decode(ctypes.byref(lat), ctypes.byref(mlp), compute, packed, uv, n, out, out_dtype,
                              ctypes.byref(cfg) if cfg else None, None)


def test_decode_validation(A):
    lat, mlp = _lat(A), _mlp(A)
    assert A.lib().ntc_decode(None, ctypes.byref(mlp), 1, 0x1000, 0x1000, 10, 0x1000, 0, None, None) == A.E_NULL
    assert _decode(A, lat, mlp, compute=7) == A.E_UNSUPPORTED
    assert _decode(A, lat, mlp, n=-1) == A.E_SHAPE
    assert _decode(A, lat, mlp, packed=0) == A.E_NULL
    assert _decode(A, lat, mlp, packed=0x1010) == A.E_ALIGN
    assert _decode(A, lat, mlp, uv=0x1004) == A.E_ALIGN
    assert _decode(A, lat, mlp, out=0x1008) == A.E_ALIGN
    assert _decode(A, lat, mlp, out_dtype=A.FP8_E4M3) == A.E_UNSUPPORTED
    assert _decode(A, lat, _mlp(A, dims=(12, 32, 8))) == A.E_SHAPE          # dims[0] != 3K+2
    assert _decode(A, lat, _mlp(A, dims=(14, 48, 48, 8))) == A.E_UNSUPPORTED  # width not in {16,32,64}
    assert _decode(A, lat, _mlp(A, dims=(14, 32, 64, 8))) == A.E_UNSUPPORTED  # unequal widths
    assert _decode(A, lat, _mlp(A, dims=(14, 32, 17))) == A.E_SHAPE
    assert _decode(A, lat, _mlp(A, dims=(14, 8))) == A.E_SHAPE               # one layer
    assert _decode(A, _lat(A, sizes=((62, 64),) * 4), mlp) == A.E_SHAPE     # not a multiple of 4
    assert _decode(A, _lat(A, n_levels=0), mlp) == A.E_SHAPE
    assert _decode(A, _lat(A, data=0), mlp) == A.E_NULL
    assert _decode(A, _lat(A, data=0x1004), mlp) == A.E_ALIGN
    assert _decode(A, _lat(A, fmt=1), mlp, compute=A.F16) == A.E_UNSUPPORTED  # MFMA path needs BC1
    bad = _lat(A)
    bad.shift[1][0] = 3.0
    assert _decode(A, bad, mlp) == A.E_SHAPE
    cfg = A.ntc_tile_cfg()
    cfg.waves_per_cu = 2000
    assert _decode(A, lat, mlp, cfg=cfg) == A.E_SHAPE
    cfg.waves_per_cu, cfg.stage_capacity = 8, 10
    assert _decode(A, lat, mlp, cfg=cfg) == A.E_SHAPE
    cfg.stage_capacity, cfg.tiles_per_iter = 1024, 1
    assert _decode(A, lat, mlp, cfg=cfg) == A.E_UNSUPPORTED
    # n == 0 enqueues nothing and succeeds without touching the GPU
    assert _decode(A, lat, mlp, n=0) == A.OK
    assert b"dims[0]" in (A.lib().ntc_decode(ctypes.byref(lat), ctypes.byref(_mlp(A, dims=(11, 32, 8))), 1,
                                             0x1000, 0x1000, 5, 0x1000, 0, None, None) and A.lib().ntc_last_error())


def test_span_length_per_shape(A):
    """tiles_per_iter must name the span compiled for the network shape and
    precision: 4 tiles for 64-wide networks of four or more layers and for
    the 64-wide BF16 / E4M3 decodes, 8 otherwise (n = 0: validated, nothing
    enqueued)."""
    lat = _lat(A)
    cfg = A.ntc_tile_cfg()
    cases = [((14, 32, 32, 8), A.F16, 8), ((14, 64, 64, 8), A.F16, 8), ((14, 64, 64, 64, 8), A.F16, 4),
             ((14, 64, 64, 8), A.BF16, 4), ((14, 32, 32, 8), A.BF16, 8), ((14, 64, 64, 8), A.FP8_E4M3, 4),
             ((14, 16, 16, 16, 16, 8), A.F16, 8)]
    for dims, compute, span in cases:
        mlp = _mlp(A, dims=dims)
        cfg.tiles_per_iter = span
        assert _decode(A, lat, mlp, compute=compute, n=0, cfg=cfg) == A.OK, (dims, compute)
        cfg.tiles_per_iter = 12 - span
        assert _decode(A, lat, mlp, compute=compute, n=0, cfg=cfg) == A.E_UNSUPPORTED, (dims, compute)


def test_pack_validation(A):
    L = A.lib()
    mlp = _mlp(A)
    n = ctypes.c_size_t(0)
    assert L.ntc_mlp_pack_size(ctypes.byref(mlp), A.F16, ctypes.byref(n)) == A.OK and n.value > 0
    n32 = ctypes.c_size_t(0)
    assert L.ntc_mlp_pack_size(ctypes.byref(mlp), A.F32, ctypes.byref(n32)) == A.OK
    assert L.ntc_mlp_pack_size(ctypes.byref(mlp), A.BF16, ctypes.byref(n)) == A.OK
    assert L.ntc_mlp_pack_size(ctypes.byref(mlp), 7, ctypes.byref(n)) == A.E_UNSUPPORTED
    assert L.ntc_mlp_pack(ctypes.byref(mlp), A.F16, None, 0x1000, 10, None) == A.E_WORKSPACE
    assert L.ntc_mlp_pack(ctypes.byref(mlp), A.F16, None, 0x1010, 1 << 20, None) == A.E_ALIGN
    assert L.ntc_mlp_pack(ctypes.byref(mlp), A.FP8_E4M3, None, 0x1000, 1 << 20, None) == A.E_NULL
    m0 = _mlp(A, ptr=0)
    assert L.ntc_mlp_pack(ctypes.byref(m0), A.F16, None, 0x1000, 1 << 20, None) == A.E_NULL


def test_backward_and_texel_validation(A):
    L = A.lib()
    lat_f, lat_b, mlp = _lat(A, fmt=1), _lat(A, fmt=0), _mlp(A, dims=(14, 64, 64, 8))
    n = ctypes.c_size_t(0)
    assert L.ntc_decode_backward_workspace(ctypes.byref(lat_f), ctypes.byref(mlp), 1 << 20, ctypes.byref(n)) == A.OK
    assert n.value > 0
    ptrs = (ctypes.c_void_p * 5)(*([0x1000] * 5))
    # BC1 latents have no continuous texel values to differentiate
    assert L.ntc_decode_backward(ctypes.byref(lat_b), ctypes.byref(mlp), 0x1000, 100, 0x1000, ptrs, ptrs, ptrs,
                                 0x1000, n.value, None) == A.E_UNSUPPORTED
    assert L.ntc_decode_backward(ctypes.byref(lat_f), ctypes.byref(mlp), 0x1000, 100, 0x1000, ptrs, ptrs, ptrs,
                                 0x1000, 16, None) == A.E_WORKSPACE
    assert L.ntc_decode_backward(ctypes.byref(lat_f), ctypes.byref(mlp), 0x1000, 100, 0x1000, None, ptrs, ptrs,
                                 0x1000, n.value, None) == A.E_NULL
    assert L.ntc_bc1_decode_texels(ctypes.byref(lat_b), 4, 0x1000, None, None) == A.E_SHAPE
    assert L.ntc_bc1_decode_texels(ctypes.byref(lat_b), 0, None, None, None) == A.E_NULL
    assert L.ntc_bc1_decode_texels(ctypes.byref(lat_f), 0, 0x1000, None, None) == A.E_UNSUPPORTED


def test_qat_validation(A):
    L = A.lib()
    p = 0x1000
    assert L.ntc_qat_texels(None, 16, 16, p, None) == A.E_NULL
    assert L.ntc_qat_texels(p, 16, 16, None, None) == A.E_NULL
    assert L.ntc_qat_texels(p, 18, 16, p, None) == A.E_SHAPE      # not a multiple of 4
    assert L.ntc_qat_texels(p, 0, 16, p, None) == A.E_SHAPE
    assert L.ntc_qat_texels(p, 16, 32768, p, None) == A.E_SHAPE   # above 16384
    assert L.ntc_qat_texels(p + 2, 16, 16, p, None) == A.E_ALIGN
    assert L.ntc_qat_backward(p, 16, 16, None, p, None) == A.E_NULL
    assert L.ntc_qat_export_bc1(p, 16, 16, p + 4, None) == A.E_ALIGN
    assert L.ntc_qat_export_bc1(p, 16, 12, None, None) == A.E_NULL


def test_classify_validation(A):
    L = A.lib()
    p = 0x1000
    n = ctypes.c_size_t(0)
    assert L.ntc_classify_workspace(64, 32, 3, ctypes.byref(n)) == A.OK and n.value > 0
    assert L.ntc_classify_workspace(64, 32, 3, None) == A.E_NULL
    assert L.ntc_classify_workspace(0, 32, 3, ctypes.byref(n)) == A.E_SHAPE
    assert L.ntc_classify_workspace(64, 32, 0, ctypes.byref(n)) == A.E_SHAPE
    assert L.ntc_classify_workspace(64, 32, 5000, ctypes.byref(n)) == A.E_SHAPE
    assert L.ntc_classify_workspace(40000, 32, 3, ctypes.byref(n)) == A.E_SHAPE
    need = n.value
    assert L.ntc_classify(p, 64, 32, 3, p, p, p, None, p, need - 1, None) == A.E_WORKSPACE
    assert L.ntc_classify(None, 64, 32, 3, p, p, p, None, p, need, None) == A.E_NULL
    assert L.ntc_classify(p, 64, 32, 3, p, p, p, None, p + 64, need, None) == A.E_ALIGN
    assert L.ntc_gather_uv(p, p, -1, p, None) == A.E_SHAPE
    assert L.ntc_gather_uv(None, p, 0, None, None) == A.OK     # nothing to do
    assert L.ntc_gather_uv(None, p, 10, p, None) == A.E_NULL
    assert L.ntc_scatter_rows(p, p, 10, 17, A.F32, p, None) == A.E_SHAPE
    assert L.ntc_scatter_rows(p, p, 10, 8, A.FP8_E4M3, p, None) == A.E_UNSUPPORTED
    assert L.ntc_scatter_rows(p + 2, p, 10, 8, A.F32, p, None) == A.E_ALIGN


def test_filtered_validation(A):
    L = A.lib()
    mlp = A.ntc_mlp()
    mlp.n_layers = 3
    for i, d in enumerate((14, 32, 32, 8)):
        mlp.dims[i] = d
    lat = A.ntc_latent_mips()
    lat.n_levels = 4
    for k, s in enumerate((64, 32, 16, 8)):
        lat.width[k] = lat.height[k] = s
        lat.n_mips[k] = 2
        for m in range(2):
            lat.data[k][m] = 0x1000
    p = 0x1000

    def call(n=100, filt=A.FILTER_TRILINEAR, aniso=16, uv=p, duv=p, out=p, packed=p):
        return L.ntc_decode_filtered(ctypes.byref(lat), ctypes.byref(mlp), packed, uv, duv, n, out, A.F32, filt,
                                     aniso, None)

    assert L.ntc_decode_filtered(None, ctypes.byref(mlp), p, p, p, 10, p, A.F32, 1, 16, None) == A.E_NULL
    assert call(filt=3) == A.E_UNSUPPORTED
    assert call(aniso=0) == A.E_SHAPE and call(aniso=17) == A.E_SHAPE
    assert call(duv=None) == A.E_NULL
    assert call(duv=p + 8) == A.E_ALIGN
    assert call(n=-1) == A.E_SHAPE
    assert call(n=0, uv=None, duv=None, out=None, packed=None) == A.OK
    lat.n_mips[3] = 3   # 8 >> 2 = 2 texels: too small
    lat.data[3][2] = p
    assert call() == A.E_SHAPE
    lat.n_mips[3] = 2
    lat.data[2][1] = 0
    assert call() == A.E_NULL
    lat.data[2][1] = p
    lat.shift[0][0] = 2.0
    assert call() == A.E_SHAPE


def test_classify_noalloc_limits(A):
    """The allocation-free classification rejects frames whose counts exceed
    its 8 MiB scratch, and bad arguments, before any HIP call."""
    L = A.lib()
    # 4096 x 4096 with 300 materials needs 600 * 4097 * 4 bytes > 8 MiB
    assert L.ntc_classify_noalloc(0x1000, 4096, 4096, 300, 0x1000, 0x1000, 0x1000, 0, None) == A.E_WORKSPACE
    assert b"8388608" in L.ntc_last_error()
    assert L.ntc_classify_noalloc(None, 64, 64, 3, 0x1000, 0x1000, 0x1000, 0, None) == A.E_NULL
    assert L.ntc_classify_noalloc(0x1001, 64, 64, 3, 0x1000, 0x1000, 0x1000, 0, None) == A.E_ALIGN
    assert L.ntc_classify_noalloc(0x1000, 0, 64, 3, 0x1000, 0x1000, 0x1000, 0, None) == A.E_SHAPE
    assert L.ntc_classify_noalloc(0x1000, 64, 64, 0, 0x1000, 0x1000, 0x1000, 0, None) == A.E_SHAPE
