"""Pins of the oracle's MLP f(x) (Sec. 3.1) and of its narrow-format rounding.

MLP: zero weights give sigmoid(b_L); unit inputs expose single weights
(catches transposed operands); a ReLU layer with negative pre-activations is
cut to zero; one-hot pass-through networks give closed forms; random
networks agree with the composition of library routines (numpy matmul,
scipy expit). Rounding: binary16 against numpy's float16 cast, E4M3 against
torch's float8_e4m3fn cast and the 256 codes of the format.
"""
import numpy as np
import pytest
import torch
from scipy.special import expit

import ntc_inputs as I


def _one_level_lat(O):
    """A latent set whose features are irrelevant (tests feed x directly through
    a one-layer identity front)."""
    return O.Latents([np.zeros((4, 4, 3))])


def _run_mlp(O, Ws, bs, x, precision=0, ws=None, as_=None):
    """Evaluate the oracle MLP on given feature vectors x [n][d0].

    The oracle only exposes full decodes; a constant grid per feature makes the
    sampled features equal to x exactly (weights sum to one), so one level
    per 3 features is built; the extra features u, v are the sample uv."""
    n, d = x.shape
    # features come as 3 channels per level + u, v; build d0 = 3K+2 inputs
    assert (d - 2) % 3 == 0
    K = (d - 2) // 3
    outs = []
    for s in range(n):
        levels = [np.broadcast_to(x[s, 3 * k:3 * k + 3], (4, 4, 3)).copy() for k in range(K)]
        lat = O.Latents(levels)
        mlp = O.Mlp(Ws, bs, precision=precision, w_scale=ws, a_scale=as_)
        outs.append(O.decode(lat, mlp, x[s:s + 1, 3 * K:3 * K + 2], threads=1)[0])
    return np.array(outs)


def test_zero_weights_give_sigmoid_bias(oracle_lib):
    O = oracle_lib
    dims = (14, 32, 32, 8)
    Ws = [np.zeros((dims[l + 1], dims[l])) for l in range(3)]
    bs = [np.zeros(32), np.zeros(32), np.linspace(-3, 3, 8)]
    rng = np.random.default_rng(0)
    lat = O.Latents(I.bc1_pyramid(rng, [(16, 16), (8, 8), (8, 8), (4, 4)]))
    out = O.decode(lat, O.Mlp(Ws, bs), rng.random((64, 2)))
    assert np.allclose(out, 1.0 / (1.0 + np.exp(-np.linspace(-3, 3, 8)))[None], rtol=0, atol=0)


def test_unit_inputs_expose_single_weights(oracle_lib):
    """One layer: f_o(e_k) = sigmoid(W[o, k] + b[o]) for a unit feature vector e_k."""
    O = oracle_lib
    rng = np.random.default_rng(1)
    W = rng.standard_normal((5, 8))
    b = rng.standard_normal(5)
    for k in range(6):  # the 6 latent features (2 levels); u = v = 0 via uv input
        x = np.zeros((1, 8))
        x[0, k] = 1.0
        f = _run_mlp(O, [W], [b], x)[0]
        assert np.allclose(f, 1.0 / (1.0 + np.exp(-(W[:, k] + b))), rtol=1e-15, atol=0)
    # u and v enter as features 6 and 7
    f = _run_mlp(O, [W], [b], np.array([[0, 0, 0, 0, 0, 0, 0.5, 0.25]]))[0]
    assert np.allclose(f, 1.0 / (1.0 + np.exp(-(0.5 * W[:, 6] + 0.25 * W[:, 7] + b))), rtol=1e-15)


def test_relu_cuts_negative(oracle_lib):
    O = oracle_lib
    W0 = -np.ones((4, 8))          # all pre-activations negative for x >= 0
    b0 = np.full(4, -0.1)
    W1 = np.arange(12.0).reshape(3, 4)
    b1 = np.array([0.2, -0.3, 0.4])
    x = np.random.default_rng(2).random((3, 8))
    f = _run_mlp(O, [W0, W1], [b0, b1], x)
    assert np.array_equal(f, np.broadcast_to(1.0 / (1.0 + np.exp(-b1)), f.shape))


def test_one_hot_pass_through(oracle_lib):
    """Two ReLU layers that copy feature k (x_k >= 0) to output o: f_o = sigmoid(x_k),
    other outputs sigmoid(0) = 1/2. Non-square matrices catch transposition."""
    O = oracle_lib
    x = np.array([[0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8]])
    for k, o in [(0, 2), (5, 0), (7, 1)]:
        W0 = np.zeros((6, 8)); W0[3, k] = 1.0
        W1 = np.zeros((5, 6)); W1[4, 3] = 1.0
        W2 = np.zeros((3, 5)); W2[o, 4] = 1.0
        f = _run_mlp(O, [W0, W1, W2], [np.zeros(6), np.zeros(5), np.zeros(3)], x)[0]
        expect = np.full(3, 0.5)
        expect[o] = 1.0 / (1.0 + np.exp(-x[0, k]))
        assert np.allclose(f, expect, rtol=1e-15, atol=0)


def test_random_networks_vs_library_composition(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(3)
    for dims in [(8, 5, 3), (14, 7, 9, 4), (14, 64, 64, 64, 8)]:
        Ws = [rng.standard_normal((dims[l + 1], dims[l])) * 0.5 for l in range(len(dims) - 1)]
        bs = [rng.standard_normal(dims[l + 1]) * 0.3 for l in range(len(dims) - 1)]
        x = rng.random((7, dims[0]))
        f = _run_mlp(O, Ws, bs, x)
        h = x.T
        for l in range(len(Ws) - 1):
            h = np.maximum(np.matmul(Ws[l], h) + bs[l][:, None], 0.0)
        ref = expit(np.matmul(Ws[-1], h) + bs[-1][:, None]).T
        assert np.allclose(f, ref, rtol=1e-13, atol=1e-15)


def test_full_decode_matches_features_then_layers(oracle_lib):
    """decode == MLP applied to features (composition), on a BC1 pyramid."""
    O = oracle_lib
    wl = I.WORKLOADS["c1"]
    lat_np, Ws, bs, uv = I.make_workload(wl, bias="normal")
    lat = O.Latents(lat_np, shift=wl.shift)
    sel = np.random.default_rng(4).integers(0, uv.shape[0], 300)
    out = O.decode_index(lat, O.Mlp(Ws, bs), uv, sel)
    x = O.features(lat, uv[sel])
    h = x.T
    for l in range(len(Ws) - 1):
        h = np.maximum(Ws[l].astype(np.float64) @ h + bs[l][:, None], 0.0)
    ref = expit(Ws[-1].astype(np.float64) @ h + bs[-1][:, None]).T
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# Narrow formats
# ---------------------------------------------------------------------------
def test_round_f16_vs_numpy(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(5)
    xs = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 5, 20000),
        (np.arange(-3000, 3000) + 0.5) * 2.0 ** -24,           # subnormal ties
        np.array([65504.0, 65519.99, 65520.0, -65520.0, 1e6, 2.0 ** -25, 2.0 ** -26, 0.0, -0.0]),
        1.0 + (np.arange(1, 200) + 0.5) * 2.0 ** -10,          # ties in [1, 2)
    ])
    ref = xs.astype(np.float16).astype(np.float64)
    got = np.array([O.round_f16(v) for v in xs])
    assert np.array_equal(got, ref)


def test_round_e4m3_codes_and_torch(oracle_lib):
    O = oracle_lib
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    finite = codes[np.isfinite(codes)]
    assert finite.size == 254 and np.max(np.abs(finite)) == 448.0
    for v in finite:  # every code is a fixed point
        assert O.round_e4m3_sat(v) == v
    rng = np.random.default_rng(6)
    xs = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * np.float32(2.0) ** rng.integers(-12, 9, 20000).astype(np.float32),
        ((finite[:-1] + finite[1:]) / 2).astype(np.float32),  # midpoints between codes
    ]).astype(np.float32)
    xs = xs[np.abs(xs) <= 448.0]
    ref = torch.from_numpy(xs).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([O.round_e4m3_sat(float(v)) for v in xs])
    assert np.array_equal(got, ref)
    # saturation
    assert O.round_e4m3_sat(1e6) == 448.0 and O.round_e4m3_sat(-500.0) == -448.0
    assert O.round_e4m3_sat(464.0) == 448.0 and O.round_e4m3_sat(470.0) == 448.0


def test_fp16_emulation_is_layerwise_rounding(oracle_lib):
    """precision FP16 equals the exact MLP applied to inputs/weights rounded by
    numpy's float16 cast (bias and accumulation exact)."""
    O = oracle_lib
    rng = np.random.default_rng(7)
    dims = (8, 16, 16, 4)
    Ws = [rng.standard_normal((dims[l + 1], dims[l])) * 0.4 for l in range(3)]
    bs = [rng.standard_normal(dims[l + 1]) * 0.1 for l in range(3)]
    x = rng.random((5, 8))
    f = _run_mlp(O, Ws, bs, x, precision=O.FP16)
    r16 = lambda a: a.astype(np.float16).astype(np.float64)
    h = x.T
    for l in range(3):
        z = r16(Ws[l]) @ r16(h) + bs[l][:, None]
        h = np.maximum(z, 0) if l < 2 else expit(z)
    assert np.allclose(f, h.T, rtol=1e-13, atol=1e-15)


def test_fp8_emulation_is_scaled_rounding(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(8)
    dims = (8, 16, 4)
    Ws = [rng.standard_normal((dims[l + 1], dims[l])) * 0.4 for l in range(2)]
    bs = [rng.standard_normal(dims[l + 1]) * 0.1 for l in range(2)]
    x = rng.random((5, 8))
    ws = np.array([300.0, 250.0])
    as_ = np.array([400.0, 120.0])
    f = _run_mlp(O, Ws, bs, x, precision=O.FP8, ws=ws, as_=as_)

    def q(a, s):
        t = torch.from_numpy(np.clip(a * s, -448, 448).astype(np.float32))
        # scaled values are float64 here; round via float32 only where exact
        return t.to(torch.float8_e4m3fn).to(torch.float64).numpy()

    h = x.T
    for l in range(2):
        a = h * as_[l]
        w = Ws[l] * ws[l]
        qa = np.vectorize(O.round_e4m3_sat)(a)
        qw = np.vectorize(O.round_e4m3_sat)(w)
        z = (qw @ qa) / (ws[l] * as_[l]) + bs[l][:, None]
        h = np.maximum(z, 0) if l < 1 else expit(z)
    assert np.allclose(f, h.T, rtol=1e-13, atol=1e-15)
    # the rounding used above agrees with torch where the scaled value is a float32
    a32 = (x * 400.0).astype(np.float32)
    assert np.array_equal(np.vectorize(O.round_e4m3_sat)(a32.astype(np.float64)),
                          torch.from_numpy(np.clip(a32, -448, 448)).to(torch.float8_e4m3fn).to(torch.float64).numpy())


def test_fp8_f16_emulation_is_two_step_rounding(oracle_lib):
    """FP8_F16: first-layer inputs as in FP8; hidden activations h scaled by
    s, clamped to [0, 256], rounded to binary16 at 1/256 of that value and
    then to E4M3. Reference: numpy's float16 cast and torch's float8_e4m3fn
    cast (exact inputs only), not the oracle's rounding functions."""
    O = oracle_lib
    rng = np.random.default_rng(18)
    dims = (8, 16, 16, 4)
    Ws = [rng.standard_normal((dims[l + 1], dims[l])) * 0.5 for l in range(3)]
    bs = [rng.standard_normal(dims[l + 1]) * 0.2 for l in range(3)]
    x = rng.random((7, 8)).astype(np.float32).astype(np.float64)
    ws = np.array([128.0, 256.0, 64.0])
    as_ = np.array([256.0, 512.0, 16.0])  # the third clamps some activations at 256 / 16
    f = _run_mlp(O, Ws, bs, x, precision=O.FP8_F16, ws=ws, as_=as_)

    def e4m3(v32):
        return torch.from_numpy(np.asarray(v32, np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()

    h = x.T
    clamped = 0
    for l in range(3):
        qw = np.vectorize(O.round_e4m3_sat)(Ws[l] * ws[l])
        if l == 0:
            qa = e4m3(h * as_[l])  # x * 256 is exact in float32 and below 448
        else:
            t = np.clip(h * as_[l] / 256.0, 0.0, 1.0)
            clamped += int((h * as_[l] > 256.0).sum())
            qa = e4m3(t.astype(np.float16).astype(np.float32) * np.float32(256.0))
        z = (qw @ qa) / (ws[l] * as_[l]) + bs[l][:, None]
        h = np.maximum(z, 0) if l < 2 else expit(z)
    assert clamped > 0
    assert np.allclose(f, h.T, rtol=1e-13, atol=1e-15)
    # the two-step rounding differs from one E4M3 rounding somewhere
    f1 = _run_mlp(O, Ws, bs, x, precision=O.FP8, ws=ws, as_=as_)
    assert not np.allclose(f, f1, rtol=1e-13, atol=1e-15)


def test_layer_amax(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(9)
    wl = I.WORKLOADS["c1"]
    lat_np, Ws, bs, uv = I.make_workload(wl)
    lat = O.Latents(lat_np, shift=wl.shift)
    mlp = O.Mlp(Ws, bs)
    sel = rng.integers(0, uv.shape[0], 500)
    am = O.layer_amax(lat, mlp, uv[sel])
    x = O.features(lat, uv[sel])
    assert am[0] == np.max(np.abs(x))
    h1 = np.maximum(Ws[0].astype(np.float64) @ x.T + bs[0][:, None], 0)
    assert np.isclose(am[1], np.max(h1), rtol=1e-14)


def test_mlp_forward_batch_vs_brute_force(oracle_lib):
    """oracle.mlp_forward on a batch of several samples with odd widths: every
    row against plain Python dot-product loops (one sample at a time) and the
    whole batch against numpy composition. Distinct rows with distinct values
    catch a wrong row stride of the input or output arrays."""
    import math
    O = oracle_lib
    rng = np.random.default_rng(10)
    for dims in [(5, 7, 3), (14, 9, 11, 6), (8, 13, 13, 13, 16)]:
        Ws = [rng.standard_normal((dims[l + 1], dims[l])) * 0.6 for l in range(len(dims) - 1)]
        bs = [rng.standard_normal(dims[l + 1]) * 0.3 for l in range(len(dims) - 1)]
        x = rng.random((9, dims[0])) * 2.0 - 0.5
        got = O.mlp_forward(O.Mlp(Ws, bs), x, threads=3)
        assert got.shape == (9, dims[-1])
        for s in range(9):
            h = [float(v) for v in x[s]]
            for l in range(len(Ws)):
                z = [float(bs[l][i]) + sum(float(Ws[l][i, j]) * h[j] for j in range(len(h)))
                     for i in range(dims[l + 1])]
                h = [max(v, 0.0) for v in z] if l + 1 < len(Ws) else [1.0 / (1.0 + math.exp(-v)) for v in z]
            assert np.allclose(got[s], h, rtol=1e-13, atol=1e-15), (dims, s)
        hh = x.T
        for l in range(len(Ws) - 1):
            hh = np.maximum(Ws[l] @ hh + bs[l][:, None], 0.0)
        assert np.allclose(got, expit(Ws[-1] @ hh + bs[-1][:, None]).T, rtol=1e-13, atol=1e-15)
        # the rows differ, so a stride error could not hide behind equal rows
        assert len({tuple(np.round(r, 12)) for r in got}) == 9


def test_fp8_scales_closed_forms(oracle_lib):
    """Per-layer E4M3 scales s = 448 / max|.| (weights: largest magnitude of
    the layer's matrix, negative entries included; activations: the
    calibrated amax), and their power-of-two form: 2^floor(log2(448 / max))
    for the weights and the first layer's inputs (whose range always
    includes [0, 1]), 2^floor(log2(256 / amax)) for hidden activations."""
    O = oracle_lib
    Ws = [np.array([[0.5, -1.0], [0.25, 0.125]]), np.array([[448.0, 1.0]]), np.array([[-2.0, 500.0]]),
          np.array([[3.0, -7.0]])]
    amax = [0.7, 1.0, 448.0, 0.001]
    ws, as_ = O.fp8_scales(Ws, amax)
    assert ws[0] == 448.0 and ws[1] == 1.0
    assert ws[2] == np.float64(np.float32(448.0) / np.float32(500.0))
    assert ws[3] == 64.0
    assert as_[0] == np.float64(np.float32(448.0) / np.float32(0.7))
    assert abs(as_[0] - 640.0) <= 640.0 * 2.0 ** -23
    assert as_[1] == 448.0 and as_[2] == 1.0
    assert as_[3] == np.float64(np.float32(448.0) / np.float32(0.001))
    w2, a2 = O.fp8_scales(Ws, amax, pow2=True)
    assert list(w2) == [256.0, 1.0, 0.5, 64.0]
    # first layer: 448 / max(0.7, 1) = 448 -> 256; hidden: 256 / 1, 256 / 448, 256 / 0.001
    assert list(a2) == [256.0, 256.0, 0.5, 131072.0]
    # a power of two never exceeds the plain scale and is at least half of it
    assert np.all(w2 <= ws) and np.all(w2 > ws / 2)
    # hidden scales map the calibrated amax into [128, 256]
    hid = np.array(amax[1:]) * a2[1:]
    assert np.all(hid <= 256.0) and np.all(hid > 128.0)
    # a first layer calibrated at or above 1 keeps the 448 form
    _, a3 = O.fp8_scales(Ws, [1.5, 1.0, 1.0, 1.0], pow2=True)
    assert a3[0] == 256.0 and 1.5 * a3[0] <= 448.0
    _, a4 = O.fp8_scales(Ws, [3.0, 1.0, 1.0, 1.0], pow2=True)
    assert a4[0] == 128.0
