"""Filtered decode over BC1 mip chains (ntc_decode_filtered; Sec. 3.2 mip
chains, Sec. 3.3 trilinear / anisotropic fetches) against the FP64 oracle
(oracle/filtering.py). The tap count N is an integer: the oracle takes the
exact N = min(ceil(Pmax / Pmin), max_aniso) (FP64), the kernel decides it
with FP32 squared lengths, so the two can differ only for samples whose axis
ratio lies within FP32 rounding of an integer below max_aniso. Those
samples (counted and printed, at most 0.1 %) are left out of the comparison;
everything else is continuous in the inputs and held to the FP16 gate."""
import numpy as np
import pytest
import torch

import ntc_inputs as I
import oracle as O
from oracle import filtering as F

pytestmark = pytest.mark.gpu

TOL_F16_ABS = 2e-3
# relative distance of the axis ratio from an integer within which the FP32
# decision of N may differ from the exact one: the FP32 squared lengths carry
# at most 3 roundings each (2 products, 1 sum: 3u), their product with i^2
# one more, so the compared ratio^2 is off by < 8u and the ratio by < 4u
# (u = 2^-24); 1e-6 leaves a factor 4 of headroom
RATIO_TOL = 1e-6


def _ambiguous(levels_wh, duv, max_aniso):
    """Samples whose tap count the FP32 decision may take differently on
    some level: ratio within RATIO_TOL of an integer 1 .. max_aniso - 1."""
    amb = np.zeros(duv.shape[0], bool)
    for (w, h) in levels_wh:
        r = F.aniso_ratio(*F.axes_sq(duv, w, h))
        k = np.round(r)
        with np.errstate(invalid="ignore"):
            amb |= (k >= 1) & (k <= max_aniso - 1) & (np.abs(r - k) <= RATIO_TOL * k)
    return amb


def _ntc():
    import paper_2506_06040_amd as ntc
    return ntc


def _case(seed, sizes, dims=(14, 64, 64, 64, 8)):
    rng = np.random.default_rng(seed)
    chains = [I.bc1_mip_chain(rng, w, h) for (w, h) in sizes]
    Ws, bs = I.xavier_mlp(rng, dims, bias="normal")
    return rng, chains, Ws, bs


def test_zero_derivatives_equal_bilinear_decode():
    ntc = _ntc()
    rng, chains, Ws, bs = _case(1, [(64, 64), (32, 32), (16, 16), (8, 8)])
    uv = rng.random((5000, 2)).astype(np.float32)
    mlp = ntc.Mlp(Ws, bs)
    lm = ntc.LatentMips(chains, shift=I.PAPER_SHIFT)
    uvt = torch.from_numpy(uv).cuda()
    zero = torch.zeros((uv.shape[0], 4), device="cuda")
    ref = ntc.decode(ntc.Latents([c[0] for c in chains], shift=I.PAPER_SHIFT), mlp, uvt, compute="f16")
    for filt in ("trilinear", "anisotropic"):
        got = ntc.decode_filtered(lm, mlp, uvt, zero, filter=filt)
        assert torch.equal(got, ref), filt


@pytest.mark.parametrize("filt,max_aniso", [("trilinear", 16), ("anisotropic", 16), ("anisotropic", 4)])
def test_perspective_plane_parity(filt, max_aniso):
    ntc = _ntc()
    sizes = [(256, 256), (128, 128), (64, 64), (32, 32)]
    rng, chains, Ws, bs = _case(2, sizes)
    uv, duv = I.perspective_plane(160, 96, far=24.0)
    # the plane seen at 4x the latent texel density: level 0 spans 0.1 .. 5 texels per pixel
    duv = duv * np.float32(0.625 * 4)
    out = ntc.decode_filtered(ntc.LatentMips(chains, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs),
                              torch.from_numpy(uv).cuda(), torch.from_numpy(duv).cuda(), filter=filt,
                              max_aniso=max_aniso).cpu().numpy()
    ref = F.decode(chains, I.PAPER_SHIFT, O.Mlp(Ws, bs), uv, duv, filt, max_aniso)
    keep = ~_ambiguous(sizes, duv, max_aniso) if filt == "anisotropic" else np.ones(uv.shape[0], bool)
    err = np.abs(out - ref)[keep].max()
    px2, py2 = F.axes_sq(duv, 256, 256)
    n = F.aniso_count(px2, py2, max_aniso)
    print(f"\n[filtered {filt} {max_aniso}] n={uv.shape[0]} taps {np.bincount(n)} "
          f"left out {int((~keep).sum())} max err {err:.2e}", flush=True)
    assert (~keep).sum() <= 1e-3 * uv.shape[0]
    assert err <= TOL_F16_ABS


def test_random_derivatives_parity():
    ntc = _ntc()
    rng, chains, Ws, bs = _case(3, [(128, 64), (64, 32), (32, 16), (16, 8)], dims=(14, 32, 32, 8))
    n = 3001
    uv = (rng.random((n, 2)) * 1.2 - 0.1).astype(np.float32)
    duv = (rng.standard_normal((n, 4)) * np.exp(rng.uniform(-8, 1, (n, 1)))).astype(np.float32)
    duv[:50] = 0.0
    duv[50:100, 2:] = 0.0           # degenerate footprint: one axis of length 0
    duv[100:150] *= 1e4             # far beyond the last mip
    for filt in ("trilinear", "anisotropic"):
        out = ntc.decode_filtered(ntc.LatentMips(chains, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs),
                                  torch.from_numpy(uv).cuda(), torch.from_numpy(duv).cuda(), filter=filt,
                                  max_aniso=8).cpu().numpy()
        ref = F.decode(chains, I.PAPER_SHIFT, O.Mlp(Ws, bs), uv, duv, filt, 8)
        keep = ~_ambiguous([(128, 64), (64, 32), (32, 16), (16, 8)], duv, 8) if filt == "anisotropic" \
            else np.ones(n, bool)
        err = np.abs(out - ref)[keep].max()
        print(f"[random duv {filt}] left out {int((~keep).sum())} max err {err:.2e}", flush=True)
        assert (~keep).sum() <= 1e-3 * n
        assert err <= TOL_F16_ABS, filt


@pytest.mark.parametrize("filt", ["trilinear", "anisotropic"])
def test_staged_footprints_equal_direct(filt):
    """A pixel's result does not depend on its span: coherent rows of a
    perspective plane (footprints staged in LDS) against the same pixels
    shuffled (spans whose footprints cover whole levels fetch directly),
    bit for bit, and against the oracle."""
    ntc = _ntc()
    sizes = [(128, 128), (64, 64), (32, 32), (16, 16)]
    rng, chains, Ws, bs = _case(4, sizes)
    uv, duv = I.perspective_plane(128, 96, far=12.0)
    duv = duv * np.float32(1.5)
    lm, mlp = ntc.LatentMips(chains, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs)
    perm = rng.permutation(uv.shape[0])

    def run(u, d):
        return ntc.decode_filtered(lm, mlp, torch.from_numpy(np.ascontiguousarray(u)).cuda(),
                                   torch.from_numpy(np.ascontiguousarray(d)).cuda(), filter=filt, max_aniso=8)

    coherent = run(uv, duv)
    shuffled = run(uv[perm], duv[perm])
    assert torch.equal(shuffled, coherent[torch.from_numpy(perm).cuda()])
    ref = F.decode(chains, I.PAPER_SHIFT, O.Mlp(Ws, bs), uv, duv, filt, 8)
    keep = ~_ambiguous(sizes, duv, 8) if filt == "anisotropic" else np.ones(uv.shape[0], bool)
    err = np.abs(coherent.cpu().numpy() - ref)[keep].max()
    print(f"[staged {filt}] left out {int((~keep).sum())} max err {err:.2e}", flush=True)
    assert (~keep).sum() <= 1e-3 * uv.shape[0]
    assert err <= TOL_F16_ABS


@pytest.mark.parametrize("filt", ["trilinear", "anisotropic"])
def test_unrelated_level_sizes(filt):
    """Levels that are not powers of two of each other (96^2 with 4 mips,
    64x32, 40^2 with 2 mips): each level takes its own level of detail."""
    ntc = _ntc()
    rng = np.random.default_rng(6)
    specs = [(96, 96, 4), (64, 32, 0), (40, 40, 2)]
    chains = [I.bc1_mip_chain(rng, w, h, m) for (w, h, m) in specs]
    sizes = [(w, h) for (w, h, _) in specs]
    Ws, bs = I.xavier_mlp(rng, (11, 32, 32, 8), bias="normal")
    n = 4000
    uv = (rng.random((n, 2)) * 1.2 - 0.1).astype(np.float32)
    duv = (rng.standard_normal((n, 4)) * np.exp(rng.uniform(-7, -1, (n, 1)))).astype(np.float32)
    shift = I.PAPER_SHIFT[:3]
    out = ntc.decode_filtered(ntc.LatentMips(chains, shift=shift), ntc.Mlp(Ws, bs), torch.from_numpy(uv).cuda(),
                              torch.from_numpy(duv).cuda(), filter=filt, max_aniso=8).cpu().numpy()
    ref = F.decode(chains, shift, O.Mlp(Ws, bs), uv, duv, filt, 8)
    keep = ~_ambiguous(sizes, duv, 8) if filt == "anisotropic" else np.ones(n, bool)
    err = np.abs(out - ref)[keep].max()
    print(f"[unrelated sizes {filt}] left out {int((~keep).sum())} max err {err:.2e}", flush=True)
    assert (~keep).sum() <= 1e-3 * n
    assert err <= TOL_F16_ABS


@pytest.mark.parametrize("n", [1, 63, 65, 255, 257, 1023, 1025, 2049])
def test_ragged_span_lengths(n):
    """Pixel counts around the 64-pixel sub-spans and the 256- and
    1024-pixel staged spans: the last span is partly filled, its missing
    pixels repeat the last one and are never stored."""
    ntc = _ntc()
    sizes = [(128, 128), (64, 64), (32, 32), (16, 16)]
    rng, chains, Ws, bs = _case(7, sizes)
    uv, duv = I.perspective_plane(64, 48, far=12.0)
    sel = rng.choice(uv.shape[0], size=n, replace=n > uv.shape[0])
    uv, duv = np.ascontiguousarray(uv[sel]), np.ascontiguousarray(duv[sel] * np.float32(2.0))
    lm, mlp = ntc.LatentMips(chains, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs)
    for filt in ("trilinear", "anisotropic"):
        out = torch.full((n + 7, 8), -7.0, device="cuda")
        ntc.decode_filtered(lm, mlp, torch.from_numpy(uv).cuda(), torch.from_numpy(duv).cuda(), filter=filt,
                            max_aniso=8, out=out[:n])
        got = out.cpu().numpy()
        assert np.all(got[n:] == -7.0), filt  # nothing written past the end
        ref = F.decode(chains, I.PAPER_SHIFT, O.Mlp(Ws, bs), uv, duv, filt, 8)
        keep = ~_ambiguous(sizes, duv, 8) if filt == "anisotropic" else np.ones(n, bool)
        err = np.abs(got[:n] - ref)[keep].max() if keep.any() else 0.0
        assert err <= TOL_F16_ABS, (filt, n, err)


@pytest.mark.parametrize("filt", ["trilinear", "anisotropic"])
def test_level_larger_than_level0(filt):
    """Power-of-two levels where level 1 is twice level 0's size: the level
    of detail is still shared (shift -1 for level 1) but not every shift is
    a non-negative integer, so the selection takes the general form."""
    ntc = _ntc()
    sizes = [(64, 64), (128, 128), (32, 32), (16, 16)]
    rng, chains, Ws, bs = _case(8, sizes)
    uv, duv = I.perspective_plane(96, 64, far=16.0)
    duv = duv * np.float32(3.0)
    out = ntc.decode_filtered(ntc.LatentMips(chains, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs),
                              torch.from_numpy(uv).cuda(), torch.from_numpy(duv).cuda(), filter=filt,
                              max_aniso=8).cpu().numpy()
    ref = F.decode(chains, I.PAPER_SHIFT, O.Mlp(Ws, bs), uv, duv, filt, 8)
    keep = ~_ambiguous(sizes, duv, 8) if filt == "anisotropic" else np.ones(uv.shape[0], bool)
    err = np.abs(out - ref)[keep].max()
    print(f"[larger level 1 {filt}] left out {int((~keep).sum())} max err {err:.2e}", flush=True)
    assert (~keep).sum() <= 1e-3 * uv.shape[0]
    assert err <= TOL_F16_ABS


@pytest.mark.parametrize("filt", ["trilinear", "anisotropic"])
def test_f16_output_is_rounded_f32_output(filt):
    """FP16 outputs are the FP32 outputs rounded to nearest even, bit for
    bit (the sigmoid is evaluated in FP32 either way)."""
    ntc = _ntc()
    rng, chains, Ws, bs = _case(9, [(128, 128), (64, 64), (32, 32), (16, 16)])
    uv, duv = I.perspective_plane(80, 70, far=10.0)
    lm, mlp = ntc.LatentMips(chains, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs)
    uvt, duvt = torch.from_numpy(uv).cuda(), torch.from_numpy(duv * np.float32(2.0)).cuda()
    o32 = ntc.decode_filtered(lm, mlp, uvt, duvt, filter=filt, max_aniso=8)
    o16 = ntc.decode_filtered(lm, mlp, uvt, duvt, filter=filt, max_aniso=8, out_dtype=torch.float16)
    assert o16.dtype == torch.float16
    assert torch.equal(o16, o32.half())


@pytest.mark.parametrize("n_out", [5, 12])
def test_output_widths(n_out):
    """Output widths that are not 8 (not a multiple of 4, and more than 8)
    take the other store paths of the filtered decode."""
    ntc = _ntc()
    sizes = [(128, 128), (64, 64), (32, 32), (16, 16)]
    rng, chains, Ws, bs = _case(10, sizes, dims=(14, 32, 32, n_out))
    uv, duv = I.perspective_plane(72, 40, far=10.0)
    duv = duv * np.float32(2.0)
    lm, mlp = ntc.LatentMips(chains, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs)
    for filt in ("trilinear", "anisotropic"):
        out = ntc.decode_filtered(lm, mlp, torch.from_numpy(uv).cuda(), torch.from_numpy(duv).cuda(), filter=filt,
                                  max_aniso=8).cpu().numpy()
        assert out.shape == (uv.shape[0], n_out)
        ref = F.decode(chains, I.PAPER_SHIFT, O.Mlp(Ws, bs), uv, duv, filt, 8)
        keep = ~_ambiguous(sizes, duv, 8) if filt == "anisotropic" else np.ones(uv.shape[0], bool)
        err = np.abs(out - ref)[keep].max()
        assert (~keep).sum() <= 1e-3 * uv.shape[0]
        assert err <= TOL_F16_ABS, (filt, n_out, err)
