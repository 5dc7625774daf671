"""Trainable BC1 latents on the GPU (ntc_qat_*; Sec. 3.2, Eqs. 1-3) against
the FP64 oracle (oracle/qat.py).

Codes and texels are bit-exact: a GPU code compares the FP32 logit with the
FP32 logit of each rounding midpoint, which decides exactly as rounding the
FP64 sigmoid except for a logit equal to one of those 97 constants (random
normal logits never are). Texel values are the FP32 value nearest the
rational code value on both sides.
"""
import numpy as np
import pytest
import torch

import ntc_inputs as I
import oracle as O
from fp32_bounds import relu_ambiguous
from oracle import qat as Q

pytestmark = pytest.mark.gpu


def _ntc():
    import paper_2506_06040_amd as ntc
    return ntc


def _params(rng, bh, bw, scale=2.5):
    p = rng.standard_normal((bh, bw, Q.N_PARAMS)) * scale
    p[0, 0, 3:6] = p[0, 0, 0:3]
    if bw > 1:
        p[0, 1, 0:3] = -np.abs(p[0, 1, 0:3]) - 1.0
        p[0, 1, 3:6] = np.abs(p[0, 1, 3:6]) + 1.0
    p[-1, -1, :] = 0.0  # every logit on the sigmoid's midpoint
    return p.astype(np.float32)


@pytest.mark.parametrize("w,h", [(64, 64), (128, 32), (4, 4), (36, 20)])
def test_qat_texels_and_export_bitexact(w, h):
    ntc = _ntc()
    rng = np.random.default_rng(w * 1000 + h)
    p = _params(rng, h // 4, w // 4)
    pt = torch.from_numpy(p).cuda()
    tex = ntc.qat_texels(pt, w, h).cpu().numpy()
    _, _, val = Q.texels(p)
    assert np.array_equal(tex, val.astype(np.float32))
    blk = ntc.qat_export_bc1(pt, w, h).cpu().numpy().view(np.uint64)
    assert np.array_equal(blk, Q.export_bc1(p))
    # the library's BC1 decoder reads the exported blocks back as the same texels
    dec, _ = ntc.bc1_decode_texels(ntc.Latents([blk]), 0)
    assert np.array_equal(dec.cpu().numpy(), tex)


def test_qat_backward_parity():
    ntc = _ntc()
    rng = np.random.default_rng(41)
    w, h = 96, 64
    p = _params(rng, h // 4, w // 4)
    g = rng.standard_normal((h, w, 3)).astype(np.float32)
    got = ntc.qat_backward(torch.from_numpy(p).cuda(), w, h, torch.from_numpy(g).cuda()).cpu().numpy()
    ref = Q.backward(p, g)
    # FP32 sums of at most 16 terms against FP64: error far below 1e-5 of the
    # largest gradient of each group (endpoints, weights)
    for name, sl in (("endpoints", slice(0, 6)), ("weights", slice(6, 22))):
        err = np.max(np.abs(got[..., sl] - ref[..., sl]))
        scale = np.max(np.abs(ref[..., sl]))
        print(f"\n[qat backward {name}] max err {err:.3g} of max {scale:.3g}", flush=True)
        assert err <= 1e-5 * scale, name


def test_qat_training_chain():
    """params -> quantised texels -> FP32 decode -> loss -> gradients into the
    logits (autograd through QatTexelsFn and NtcDecodeFn) against the oracle:
    decode backward on the float texels, then the straight-through map."""
    ntc = _ntc()
    rng = np.random.default_rng(43)
    sizes = [(64, 64), (32, 32), (16, 16), (8, 8)]
    params = [_params(rng, hh // 4, ww // 4) for (ww, hh) in sizes]
    Ws, bs = I.xavier_mlp(rng, (14, 64, 64, 8), bias="normal")
    uv = I.random_uv(rng, 3001)
    # texels exactly as both sides see them
    tex64 = [Q.texels(p)[2] for p in params]
    olat, omlp = O.Latents([t.astype(np.float32) for t in tex64], shift=I.PAPER_SHIFT), O.Mlp(Ws, bs)
    # samples on a ReLU kink within FP32 rounding are left out (the FP32 error
    # bound of tests/fp32_bounds.py)
    amb = relu_ambiguous(olat, Ws, bs, uv, [t.astype(np.float32) for t in tex64])
    print(f"[qat chain] ambiguous samples: {int(amb.sum())} of {uv.shape[0]}", flush=True)
    assert amb.sum() <= 5e-3 * uv.shape[0]
    uv = uv[~amb]
    tgt = rng.random((uv.shape[0], 8)).astype(np.float32)

    p_t = [torch.from_numpy(p).cuda().requires_grad_(True) for p in params]
    lat_t = [ntc.qat_texels_fn(pt, ww, hh) for pt, (ww, hh) in zip(p_t, sizes)]
    W_t = [torch.from_numpy(x).cuda() for x in Ws]
    b_t = [torch.from_numpy(x).cuda() for x in bs]
    out = ntc.decode_fn(torch.from_numpy(uv).cuda(), lat_t, W_t, b_t, shift=I.PAPER_SHIFT)
    loss = torch.mean((out - torch.from_numpy(tgt).cuda()) ** 2)
    loss.backward()

    of = O.decode(olat, omlp, uv)
    _, _, ol = O.backward(olat, omlp, uv, 2.0 * (of - tgt) / of.size)
    for k, (p, gl) in enumerate(zip(params, ol)):
        ref = Q.backward(p, gl)
        got = p_t[k].grad.cpu().numpy()
        rel = np.max(np.abs(got - ref)) / (np.max(np.abs(ref)) + 1e-30)
        print(f"[qat chain level {k}] max |err| / max |ref| = {rel:.2e}", flush=True)
        assert rel <= 1e-4, k
