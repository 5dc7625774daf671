"""GPU backward (Sec. 3.2) against the FP64 oracle's analytic gradient and
central finite differences of the oracle loss (h = 1e-3).

Where floating point takes a branch (the ReLU derivative), the FP32 kernel
and the FP64 oracle can disagree for samples whose pre-activation lies
within FP32 rounding distance of zero. Those samples are found with a
rigorous bound on |z_fp32 - z| per hidden unit (tests/fp32_bounds.py) and
given a zero upstream gradient on both sides (or left out), so every
remaining contribution is unique. On the C3 workload the bound leaves out
about 0.17 % of the samples (1,752 of 2^20); the tests print the count and
assert that it stays below 0.5 %.
"""
import numpy as np
import pytest
import torch

import ntc_inputs as I
import oracle as O
from fp32_bounds import relu_ambiguous

pytestmark = pytest.mark.gpu

AMBIGUOUS_MAX_FRACTION = 5e-3


def _ntc():
    import paper_2506_06040_amd as ntc
    return ntc


def _close(name, got, ref, rtol=1e-4):
    scale = np.max(np.abs(ref)) + 1e-30
    err = np.max(np.abs(got - ref)) / scale
    print(f"[{name}] max |err| / max |ref| = {err:.2e}", flush=True)
    assert err <= rtol, name


def _gpu_autograd(lat_np, Ws, bs, uv, tgt, shift):
    ntc = _ntc()
    lat_t = [torch.from_numpy(a).cuda().requires_grad_(True) for a in lat_np]
    W_t = [torch.from_numpy(w).cuda().requires_grad_(True) for w in Ws]
    b_t = [torch.from_numpy(b).cuda().requires_grad_(True) for b in bs]
    out = ntc.decode_fn(torch.from_numpy(uv).cuda(), lat_t, W_t, b_t, shift=shift)
    loss = torch.mean((out - torch.from_numpy(tgt).cuda()) ** 2)
    loss.backward()
    return ([t.grad.cpu().numpy() for t in W_t], [t.grad.cpu().numpy() for t in b_t],
            [t.grad.cpu().numpy() for t in lat_t], out.detach().cpu().numpy())


def _gpu_direct(lat_np, Ws, bs, uv, g, shift, address="clamp"):
    ntc = _ntc()
    lat = ntc.Latents(lat_np, shift=shift, address=address)
    mlp = ntc.Mlp(Ws, bs)
    gW, gb, gl = ntc.decode_backward(lat, mlp, torch.from_numpy(uv).cuda(),
                                     torch.from_numpy(g.astype(np.float32)).cuda())
    return [t.cpu().numpy() for t in gW], [t.cpu().numpy() for t in gb], [t.cpu().numpy() for t in gl]


def test_backward_autograd_small():
    rng = np.random.default_rng(31)
    sizes = [(64, 64), (32, 32), (16, 16), (8, 8)]
    lat_np = I.f32_pyramid(rng, sizes)
    Ws, bs = I.xavier_mlp(rng, (14, 64, 64, 8), bias="normal")
    uv = I.random_uv(rng, 4099)
    olat, omlp = O.Latents(lat_np, shift=I.PAPER_SHIFT), O.Mlp(Ws, bs)
    amb = relu_ambiguous(olat, Ws, bs, uv, lat_np)
    print(f"[small] ambiguous samples: {int(amb.sum())} of {uv.shape[0]}", flush=True)
    assert amb.sum() <= AMBIGUOUS_MAX_FRACTION * uv.shape[0]
    uv = uv[~amb]
    tgt = rng.random((uv.shape[0], 8)).astype(np.float32)
    gW, gb, gl, f = _gpu_autograd(lat_np, Ws, bs, uv, tgt, I.PAPER_SHIFT)
    of = O.decode(olat, omlp, uv)
    assert np.all(np.abs(f - of) <= 1e-5 * np.abs(of))
    oW, ob, ol = O.backward(olat, omlp, uv, 2.0 * (of - tgt) / of.size)
    for l in range(3):
        _close(f"dW{l}", gW[l], oW[l])
        _close(f"db{l}", gb[l], ob[l])
    for k in range(4):
        _close(f"dlat{k}", gl[k], ol[k])


def test_backward_wrap_addressing():
    """Wrap addressing with uv in [-0.5, 1.5): taps that leave a level wrap
    around, and their gradients land on the texels of the opposite edge;
    against the oracle's wrap-mode backward."""
    rng = np.random.default_rng(37)
    sizes = [(32, 32), (16, 16), (8, 8), (4, 4)]
    lat_np = I.f32_pyramid(rng, sizes)
    Ws, bs = I.xavier_mlp(rng, (14, 32, 32, 8), bias="normal")
    uv = (rng.random((6000, 2)) * 2.0 - 0.5).astype(np.float32)
    olat = O.Latents(lat_np, shift=I.PAPER_SHIFT, address=O.WRAP)
    omlp = O.Mlp(Ws, bs)
    amb = relu_ambiguous(olat, Ws, bs, uv, lat_np)
    print(f"[wrap] ambiguous samples: {int(amb.sum())} of {uv.shape[0]}", flush=True)
    assert amb.sum() <= AMBIGUOUS_MAX_FRACTION * uv.shape[0]
    g = rng.standard_normal((uv.shape[0], 8)) * 1e-3
    g[amb] = 0.0
    g = g.astype(np.float32).astype(np.float64)
    gW, gb, gl = _gpu_direct(lat_np, Ws, bs, uv, g, I.PAPER_SHIFT, address="wrap")
    oW, ob, ol = O.backward(olat, omlp, uv, g)
    for l in range(3):
        _close(f"wrap dW{l}", gW[l], oW[l])
        _close(f"wrap db{l}", gb[l], ob[l])
    for k in range(4):
        _close(f"wrap dlat{k}", gl[k], ol[k])
    # every edge texel of level 0 receives gradient from wrapped taps
    assert np.all(ol[0][0] != 0) and np.all(ol[0][:, 0] != 0)


def test_backward_clustered_samples():
    """Most samples inside one spatial bin of the latent-gradient scatter (its
    samples are sorted in several rounds), the rest spread: against the
    oracle."""
    rng = np.random.default_rng(41)
    sizes = [(128, 128), (64, 64), (32, 32), (16, 16)]
    lat_np = I.f32_pyramid(rng, sizes)
    Ws, bs = I.xavier_mlp(rng, (14, 32, 32, 8), bias="normal")
    hot = 0.3 + rng.random((12000, 2)) * (30.0 / 128.0)
    uv = np.concatenate([hot, rng.random((3000, 2))]).astype(np.float32)
    uv = uv[rng.permutation(uv.shape[0])]
    olat = O.Latents(lat_np, shift=I.PAPER_SHIFT)
    omlp = O.Mlp(Ws, bs)
    amb = relu_ambiguous(olat, Ws, bs, uv, lat_np)
    print(f"[clustered] ambiguous samples: {int(amb.sum())} of {uv.shape[0]}", flush=True)
    assert amb.sum() <= AMBIGUOUS_MAX_FRACTION * uv.shape[0]
    g = rng.standard_normal((uv.shape[0], 8)) * 1e-3
    g[amb] = 0.0
    g = g.astype(np.float32).astype(np.float64)
    gW, gb, gl = _gpu_direct(lat_np, Ws, bs, uv, g, I.PAPER_SHIFT)
    oW, ob, ol = O.backward(olat, omlp, uv, g)
    for l in range(3):
        _close(f"clustered dW{l}", gW[l], oW[l])
        _close(f"clustered db{l}", gb[l], ob[l])
    for k in range(4):
        _close(f"clustered dlat{k}", gl[k], ol[k])


@pytest.fixture(scope="module")
def c3():
    wl = I.WORKLOADS["c3"]
    lat_np, Ws, bs, uv = I.make_workload(wl)
    tgt = I.point_sample(I.c3_targets(), uv)
    olat, omlp = O.Latents(lat_np, shift=wl.shift), O.Mlp(Ws, bs)
    amb = relu_ambiguous(olat, Ws, bs, uv, lat_np)
    return dict(wl=wl, lat_np=lat_np, Ws=Ws, bs=bs, uv=uv, tgt=tgt, olat=olat, omlp=omlp, amb=amb)


def test_backward_c3_full_size(c3):
    """2^20 samples, latents 1024^2..128^2, MLP 14-64-64-8: the same upstream
    gradient of the L2 loss on both sides (zero on ambiguous samples)."""
    uv, tgt = c3["uv"], c3["tgt"]
    f = O.decode(c3["olat"], c3["omlp"], uv)
    g = (2.0 * (f - tgt) / f.size).astype(np.float32).astype(np.float64)
    amb = c3["amb"]
    print(f"[c3] ambiguous samples: {int(amb.sum())} of {uv.shape[0]}", flush=True)
    assert amb.sum() <= AMBIGUOUS_MAX_FRACTION * uv.shape[0]
    g[amb] = 0.0
    gW, gb, gl = _gpu_direct(c3["lat_np"], c3["Ws"], c3["bs"], uv, g, c3["wl"].shift)
    oW, ob, ol = O.backward(c3["olat"], c3["omlp"], uv, g)
    for l in range(3):
        _close(f"c3 dW{l}", gW[l], oW[l])
        _close(f"c3 db{l}", gb[l], ob[l])
    for k in range(4):
        _close(f"c3 dlat{k}", gl[k], ol[k])


def test_backward_c3_finite_differences(c3):
    """Central differences (h = 1e-3) of the FP64 oracle loss on 64 random
    parameters (weights, biases, touched latent texels) of the C3 shapes,
    against the GPU gradient from the autograd path, on 16384 of the samples."""
    rng = np.random.default_rng(33)
    sel = np.sort(rng.choice(c3["uv"].shape[0], 16384, replace=False))
    sel = sel[~c3["amb"][sel]]
    uv, tgt = c3["uv"][sel], c3["tgt"][sel]
    lat_np, Ws, bs = c3["lat_np"], c3["Ws"], c3["bs"]
    shift = c3["wl"].shift
    gW, gb, gl, _ = _gpu_autograd(lat_np, Ws, bs, uv, tgt, shift)
    olat = O.Latents(lat_np, shift=shift)
    of = O.decode(olat, c3["omlp"], uv)
    oW, ob, ol = O.backward(olat, c3["omlp"], uv, 2.0 * (of - tgt) / of.size)

    def loss(Ws_, bs_, lat_):
        ff = O.decode(O.Latents(lat_, shift=shift), O.Mlp(Ws_, bs_), uv)
        return np.mean((ff - tgt) ** 2)

    h = 1e-3
    checked = tried = 0
    while checked < 64 and tried < 160:
        tried += 1
        kind = tried % 3
        W2 = [w.astype(np.float64) for w in Ws]
        b2 = [b.astype(np.float64) for b in bs]
        l2 = list(lat_np)
        if kind == 0:
            l = int(rng.integers(3)); idx = tuple(int(rng.integers(s)) for s in W2[l].shape)
            arr, got, ref = W2, gW[l][idx], oW[l][idx]
        elif kind == 1:
            l = int(rng.integers(3)); idx = (int(rng.integers(b2[l].shape[0])),)
            arr, got, ref = b2, gb[l][idx], ob[l][idx]
        else:
            l = int(rng.integers(4)); nz = np.argwhere(ol[l] != 0); idx = tuple(nz[rng.integers(len(nz))])
            l2 = [a.astype(np.float64) for a in lat_np]
            arr, got, ref = l2, gl[l][idx], ol[l][idx]
        base = arr[l][idx]
        arr[l][idx] = base + h
        lp = loss(W2, b2, l2)
        arr[l][idx] = base - h
        lm = loss(W2, b2, l2)
        arr[l][idx] = base
        fd = (lp - lm) / (2 * h)
        # a +-h step across a ReLU kink of some sample breaks the central
        # difference; such parameters show up as the FD disagreeing with the
        # FP64 analytic gradient and are skipped
        if abs(fd - ref) > 1e-4 * max(abs(ref), 1e-7) + 1e-10:
            continue
        assert abs(got - fd) <= 1e-3 * max(abs(fd), 1e-7) + 1e-10, (kind, l, idx, got, fd)
        checked += 1
    print(f"[fd] {checked} parameters checked in {tried} tries", flush=True)
    assert checked >= 64


def test_backward_empty_batch_gives_zero():
    ntc = _ntc()
    rng = np.random.default_rng(2)
    lat = ntc.Latents(I.f32_pyramid(rng, [(16, 16), (8, 8), (8, 8), (4, 4)]))
    Ws, bs = I.xavier_mlp(rng, (14, 32, 32, 8), bias="normal")
    mlp = ntc.Mlp(Ws, bs)
    gW, gb, gl = ntc.decode_backward(lat, mlp, torch.zeros((0, 2), device="cuda"),
                                     torch.zeros((0, 8), device="cuda"))
    torch.cuda.synchronize()
    assert all(float(t.abs().max()) == 0.0 for t in gW + gb + gl)


def test_backward_weight_gradients_repeatable():
    """Weight and bias gradients are sums of per-workgroup FP32 partials added
    in FP64 in a fixed order, so two calls give the same bits (300k samples:
    all 1024 workgroups hold partials). Latent gradients come from FP32
    atomics, whose order varies: equal up to that rounding."""
    rng = np.random.default_rng(35)
    sizes = [(256, 256), (128, 128), (64, 64), (32, 32)]
    lat_np = I.f32_pyramid(rng, sizes)
    Ws, bs = I.xavier_mlp(rng, (14, 64, 64, 8), bias="normal")
    uv = I.random_uv(rng, 300_000)
    g = rng.standard_normal((uv.shape[0], 8)) * 1e-3
    a = _gpu_direct(lat_np, Ws, bs, uv, g, I.PAPER_SHIFT)
    b = _gpu_direct(lat_np, Ws, bs, uv, g, I.PAPER_SHIFT)
    for l in range(3):
        assert np.array_equal(a[0][l], b[0][l]), f"dW{l}"
        assert np.array_equal(a[1][l], b[1][l]), f"db{l}"
    for k in range(4):
        _close(f"repeat dlat{k}", a[2][k], b[2][k], rtol=1e-5)


@pytest.mark.parametrize("dims,sizes,address", [
    ((14, 64, 64, 8), [(64, 64), (32, 32), (16, 16), (8, 8)], "clamp"),
    ((14, 32, 32, 32, 8), [(48, 40), (24, 20), (12, 10), (8, 8)], "wrap"),
    ((11, 16, 5), [(40, 40), (20, 20), (16, 8)], "clamp"),
    ((5, 64, 64, 64, 16), [(32, 32)], "clamp"),
    ((8, 32, 3), [(16, 16), (8, 8)], "wrap"),
])
def test_forward_float_latents(dims, sizes, address):
    """FP32 decode of float latents (the training forward, on the FP32
    matrix cores) against the oracle: FP32 out within 1e-5 relative of every
    value, FP16 out within FP16 rounding of it; ragged and tiny batches."""
    ntc = _ntc()
    rng = np.random.default_rng(37 + dims[1] + len(dims))
    lat_np = I.f32_pyramid(rng, sizes)
    Ws, bs = I.xavier_mlp(rng, dims, bias="normal")
    shift = I.PAPER_SHIFT[:len(sizes)]
    lat = ntc.Latents(lat_np, shift=shift, address=address)
    mlp = ntc.Mlp(Ws, bs)
    olat = O.Latents(lat_np, shift=shift, address=O.WRAP if address == "wrap" else O.CLAMP)
    omlp = O.Mlp(Ws, bs)
    for n in (1, 33, 5003):
        uv = (rng.random((n, 2)) * 1.4 - 0.2).astype(np.float32)
        ref = O.decode(olat, omlp, uv)
        out = ntc.decode(lat, mlp, torch.from_numpy(uv).cuda(), compute="f32").cpu().numpy()
        assert out.shape == ref.shape
        assert np.all(np.abs(out - ref) <= 1e-5 * np.abs(ref)), (n, float(np.max(np.abs(out - ref) / np.abs(ref))))
        o16 = ntc.decode(lat, mlp, torch.from_numpy(uv).cuda(), compute="f32",
                         out_dtype=torch.float16).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(o16 - ref) <= 2.0 ** -11 * np.abs(ref) + 1e-7), n
    print(f"[forward float latents {dims} {address}] ok", flush=True)
