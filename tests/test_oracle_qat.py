"""Pins of the trainable-BC1 oracle (oracle/qat.py; Sec. 3.2, Eqs. 1-3)."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import qat as Q


def _params(rng, bh, bw, scale=2.5):
    p = rng.standard_normal((bh, bw, Q.N_PARAMS)) * scale
    p[0, 0, 3:6] = p[0, 0, 0:3]            # equal endpoints
    if bw > 1:
        p[0, 1, 0:3] = -np.abs(p[0, 1, 0:3]) - 1.0   # endpoint 0 below endpoint 1: swapped on export
        p[0, 1, 3:6] = np.abs(p[0, 1, 3:6]) + 1.0
    return p.astype(np.float32)


def test_export_decodes_to_the_quantised_texels():
    """The oracle's own BC1 decoder (pinned by hand-built blocks) maps the
    exported blocks to exactly the quantised texel values."""
    rng = np.random.default_rng(11)
    for bh, bw in ((8, 16), (1, 1), (3, 5)):
        p = _params(rng, bh, bw)
        num, den, _ = Q.texels(p)
        onum, oden, _ = O.bc1_level(Q.export_bc1(p))
        assert np.array_equal(onum.astype(np.int64) * den, num * oden.astype(np.int64)), (bh, bw)


def test_codes_closed_forms():
    for bits in (2, 5, 6):
        m = (1 << bits) - 1
        # sigmoid(0) = 1/2 lies on a midpoint; ties go to the even code, the upper one here
        assert Q.quant_code(np.zeros(1), bits)[0] == (m + 1) // 2
        k = np.arange(m + 1)
        p = np.clip(k / m, 1e-300, 1 - 1e-16)
        x = np.log(p) - np.log1p(-p)
        assert np.array_equal(Q.quant_code(x, bits), k)
        assert Q.quant_code(np.array([-60.0]), bits)[0] == 0
        assert Q.quant_code(np.array([60.0]), bits)[0] == m
        xs = np.linspace(-12, 12, 5001)
        assert np.all(np.diff(Q.quant_code(xs, bits)) >= 0)


def test_weights_at_one_end_select_an_endpoint():
    rng = np.random.default_rng(12)
    p = _params(rng, 2, 3).astype(np.float64)
    p[..., 6:] = 30.0  # w = 3 everywhere: texels are endpoint 1
    num, den, val = Q.texels(p)
    e0, e1, w = Q.codes(p)
    m = np.array([31, 63, 31], np.float64)
    assert np.allclose(val, np.repeat(np.repeat(e1 / m, 4, 0), 4, 1), rtol=0, atol=1e-15)
    g = rng.standard_normal((8, 12, 3))
    gp = Q.backward(p, g)
    assert np.all(gp[..., 0:3] == 0.0)   # endpoint 0 carries no weight


def test_backward_equals_autograd_of_straight_through_forward():
    """torch FP64 autograd of an independently written forward in which the
    quantisation is s + (round(s m) / m - s).detach()."""
    rng = np.random.default_rng(13)
    bh, bw = 4, 6
    p = _params(rng, bh, bw).astype(np.float64)
    g = rng.standard_normal((4 * bh, 4 * bw, 3))
    pt = torch.tensor(p, requires_grad=True)
    s = torch.sigmoid(pt)

    def q(v, m):
        return v + (torch.round(v * m) / m - v).detach()

    ms = torch.tensor([31.0, 63.0, 31.0], dtype=torch.float64)
    e0 = q(s[..., 0:3], ms)
    e1 = q(s[..., 3:6], ms)
    a = q(s[..., 6:22], 3.0)                      # [bh][bw][16]
    tex = torch.zeros((4 * bh, 4 * bw, 3), dtype=torch.float64)
    for t in range(16):
        y, x = t // 4, t % 4
        at = a[..., t:t + 1]
        tex[y::4, x::4, :] = (1 - at) * e0 + at * e1
    loss = (tex * torch.tensor(g)).sum()
    loss.backward()
    ref = pt.grad.numpy()
    got = Q.backward(p, g)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13)
    # and the forward values agree with the rational texels
    assert np.allclose(tex.detach().numpy(), Q.texels(p)[2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("bits", [2, 5, 6])
def test_quant_code_is_round_of_scaled_sigmoid(bits):
    rng = np.random.default_rng(14)
    x = rng.standard_normal(20000) * 4
    m = (1 << bits) - 1
    c = Q.quant_code(x, bits)
    s = 1.0 / (1.0 + np.exp(-x)) * m
    assert np.all(np.abs(s - c) <= 0.5)
