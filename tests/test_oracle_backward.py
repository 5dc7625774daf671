"""Pins of the oracle's analytic gradient (Sec. 3.2: gradients flow through
the MLP into every latent element).

* central finite differences in FP64 (h = 1e-3) of the oracle loss on random
  weights, biases and latent texels, skipping a parameter whose +-h step
  flips a ReLU (the loss is then not differentiable across the step);
* torch FP64 autograd of an independent torch forward on the CPU;
* structure: the latent gradient of a sample sits only on its 4x4 taps and
  sums, per channel, to dx of that channel (bilinear weights sum to one).
"""
import numpy as np
import torch

import ntc_inputs as I


def _setup(seed=11, n=256, dims=(14, 16, 12, 8), sizes=((16, 16), (8, 8), (8, 4), (4, 4))):
    rng = np.random.default_rng(seed)
    lat = [rng.random((h, w, 3)) for (w, h) in sizes]
    Ws = [rng.standard_normal((dims[l + 1], dims[l])) * 0.5 for l in range(len(dims) - 1)]
    bs = [rng.standard_normal(dims[l + 1]) * 0.2 for l in range(len(dims) - 1)]
    uv = rng.random((n, 2)) * 1.2 - 0.1   # some samples clamp at the edges
    tgt = rng.random((n, dims[-1]))
    return lat, Ws, bs, uv, tgt


def _loss(O, lat, Ws, bs, uv, tgt, shift):
    f = O.decode(O.Latents(lat, shift=shift), O.Mlp(Ws, bs), uv, threads=4)
    return np.mean((f - tgt) ** 2), f


def _relu_pattern(O, lat, Ws, bs, uv, shift):
    x = O.features(O.Latents(lat, shift=shift), uv)
    pats = []
    h = x.T
    for l in range(len(Ws) - 1):
        z = Ws[l] @ h + bs[l][:, None]
        pats.append(z > 0)
        h = np.maximum(z, 0)
    return np.concatenate([p.ravel() for p in pats])


def test_backward_vs_finite_differences(oracle_lib):
    O = oracle_lib
    lat, Ws, bs, uv, tgt = _setup()
    shift = I.PAPER_SHIFT
    L0, f = _loss(O, lat, Ws, bs, uv, tgt, shift)
    n, C = f.shape
    g = 2.0 * (f - tgt) / (n * C)
    gW, gb, glat = O.backward(O.Latents(lat, shift=shift), O.Mlp(Ws, bs), uv, g, threads=3)
    rng = np.random.default_rng(12)
    h = 1e-3
    base = _relu_pattern(O, lat, Ws, bs, uv, shift)
    checked = 0
    for trial in range(120):
        kind = trial % 3
        if kind == 0:
            l = rng.integers(len(Ws)); idx = tuple(rng.integers(s) for s in Ws[l].shape)
            arrs, ga = Ws, gW[l][idx]
            target = (l, idx)
        elif kind == 1:
            l = rng.integers(len(bs)); idx = (rng.integers(bs[l].shape[0]),)
            arrs, ga = bs, gb[l][idx]
            target = (l, idx)
        else:
            l = rng.integers(len(lat)); idx = tuple(rng.integers(s) for s in lat[l].shape)
            arrs, ga = lat, glat[l][idx]
            target = (l, idx)
        vals = []
        flipped = False
        for sgn in (+1, -1):
            a2 = [a.copy() for a in arrs]
            a2[target[0]][target[1]] += sgn * h
            args = {0: (lat, a2, bs), 1: (lat, Ws, a2), 2: (a2, Ws, bs)}[kind]
            if not np.array_equal(_relu_pattern(O, args[0], args[1], args[2], uv, shift), base):
                flipped = True
                break
            vals.append(_loss(O, args[0], args[1], args[2], uv, tgt, shift)[0])
        if flipped:
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        # central differences carry an O(h^2) truncation error of ~1e-6 relative here
        assert abs(fd - ga) <= 2e-5 * max(1e-3, abs(ga)) + 1e-8, (kind, target, fd, ga)
        checked += 1
    assert checked >= 64


def test_backward_vs_torch_autograd(oracle_lib):
    O = oracle_lib
    dims = (14, 16, 12, 8)
    lat, Ws, bs, uv, tgt = _setup(seed=13, n=300, dims=dims)
    shift = I.PAPER_SHIFT
    rng = np.random.default_rng(14)
    g = rng.standard_normal((uv.shape[0], dims[-1]))
    gW, gb, glat = O.backward(O.Latents(lat, shift=shift), O.Mlp(Ws, bs), uv, g, threads=2)

    tl = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in lat]
    tW = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in Ws]
    tb = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in bs]
    tuv = torch.tensor(uv, dtype=torch.float64)
    feats = []
    for k, grid in enumerate(tl):
        H, W = grid.shape[0], grid.shape[1]
        x = tuv[:, 0] * W - 0.5 + shift[k][0]
        y = tuv[:, 1] * H - 0.5 + shift[k][1]
        x0, y0 = torch.floor(x), torch.floor(y)
        fx, fy = x - x0, y - y0
        i0, j0 = x0.long(), y0.long()
        acc = 0
        for di in (0, 1):
            for dj in (0, 1):
                ii = (i0 + di).clamp(0, W - 1)
                jj = (j0 + dj).clamp(0, H - 1)
                w = (fx if di else 1 - fx) * (fy if dj else 1 - fy)
                acc = acc + w[:, None] * grid[jj, ii]
        feats.append(acc)
    feats.append(tuv)
    h = torch.cat(feats, 1)
    for l in range(len(tW)):
        z = h @ tW[l].T + tb[l]
        h = torch.relu(z) if l + 1 < len(tW) else torch.sigmoid(z)
    (h * torch.tensor(g)).sum().backward()
    for l in range(len(Ws)):
        assert np.allclose(gW[l], tW[l].grad.numpy(), rtol=1e-11, atol=1e-13)
        assert np.allclose(gb[l], tb[l].grad.numpy(), rtol=1e-11, atol=1e-13)
    for k in range(len(lat)):
        assert np.allclose(glat[k], tl[k].grad.numpy(), rtol=1e-11, atol=1e-13)


def test_latent_gradient_structure(oracle_lib):
    """One sample: the latent gradient of level k is non-zero only on its taps
    and sums (per channel) to dx; weight gradients factor as outer products."""
    O = oracle_lib
    dims = (14, 16, 8)
    lat, Ws, bs, _, _ = _setup(seed=15, dims=dims)
    uv = np.array([[0.37, 0.61]])
    g = np.random.default_rng(16).standard_normal((1, 8))
    gW, gb, glat = O.backward(O.Latents(lat, shift=I.PAPER_SHIFT), O.Mlp(Ws, bs), uv, g, threads=1)
    # dW_last = d_L h^T: rank one with row factor db_last
    assert np.linalg.matrix_rank(gW[-1], tol=1e-12) <= 1
    # dx = W_0^T d_0 with d_0 = db_0
    dx = Ws[0].T @ gb[0]
    for k in range(4):
        nz = np.argwhere(np.any(glat[k] != 0, axis=2))
        assert len(nz) <= 4
        assert np.allclose(glat[k].sum(axis=(0, 1)), dx[3 * k:3 * k + 3], rtol=1e-12, atol=1e-14)


def test_relu_margin(oracle_lib):
    """The margin is the smallest |z| of the hidden layers, checked against
    pre-activations built from the oracle's features and numpy matmul."""
    O = oracle_lib
    dims = (14, 16, 12, 8)
    lat, Ws, bs, uv, _ = _setup(seed=17, n=200, dims=dims)
    olat = O.Latents(lat, shift=I.PAPER_SHIFT)
    mg = O.relu_margin(olat, O.Mlp(Ws, bs), uv)
    x = O.features(olat, uv)
    z1 = x @ Ws[0].T + bs[0]
    z2 = np.maximum(z1, 0) @ Ws[1].T + bs[1]
    ref = np.minimum(np.abs(z1).min(1), np.abs(z2).min(1))
    assert np.allclose(mg, ref, rtol=1e-12, atol=1e-15)
