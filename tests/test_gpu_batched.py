"""Many materials in one persistent launch: equal to per-material decodes,
within the FP16 bound of the oracle, and identical under HIP-graph replay."""
import numpy as np
import pytest
import torch

import ntc_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu


def _ntc():
    import paper_2506_06040_amd as ntc
    return ntc


def _materials(specs, device="cuda"):
    ntc = _ntc()
    mats, raw = [], []
    for sp in specs:
        lat_np, Ws, bs = I.make_material(sp, bias="normal")
        lat = ntc.Latents(lat_np, shift=I.PAPER_SHIFT)
        mlp = ntc.Mlp(Ws, bs)
        uv = I.pixel_uv_torch(sp.side, sp.side, "tiled", device)
        mats.append(ntc.Material(lat, mlp, uv))
        raw.append((lat_np, Ws, bs))
    return mats, raw


def _small_specs():
    sp = []
    for i, (side, w, d) in enumerate([(64, 32, 2), (128, 64, 3), (192, 16, 1), (256, 32, 3), (64, 64, 2), (128, 64, 1)]):
        sp.append(I.MaterialSpec(i, side, w, d, 1000 + i))
    return sp


def test_batched_equals_single_and_oracle():
    ntc = _ntc()
    mats, raw = _materials(_small_specs())
    plan = ntc.BatchPlan(mats, cfg=ntc.batch_cfg(item_pixels=256, waves_per_cu=2, n_cus=8))
    plan.launch()
    torch.cuda.synchronize()
    for m, (lat_np, Ws, bs) in zip(mats, raw):
        single = ntc.decode(m.lat, m.mlp, m.uv, compute="f16", packed=m.packed)
        assert torch.equal(single, m.out)
        uv = m.uv.cpu().numpy()
        ref = O.decode(O.Latents(lat_np, shift=I.PAPER_SHIFT), O.Mlp(Ws, bs), uv)
        assert np.max(np.abs(m.out.cpu().numpy() - ref)) <= 2e-3


def test_batched_graph_replay():
    ntc = _ntc()
    mats, raw = _materials(_small_specs()[:4])
    plan = ntc.BatchPlan(mats, cfg=ntc.batch_cfg(item_pixels=512))
    plan.launch()
    torch.cuda.synchronize()
    eager = [m.out.clone() for m in mats]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        for m in mats:
            m.out.zero_()
        with torch.cuda.graph(g, stream=s):
            plan.launch(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for m in mats:
            m.out.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for m, e in zip(mats, eager):
            assert torch.equal(m.out, e), rep


def test_c5_64_materials_equal_per_material():
    """The 64-material workload: one launch equals 64 single launches (all
    pixels), and sampled pixels of a few materials match the oracle."""
    ntc = _ntc()
    specs = I.material_specs()
    mats, raw = _materials(specs)
    plan = ntc.BatchPlan(mats)
    plan.launch()
    torch.cuda.synchronize()
    for i, m in enumerate(mats):
        single = ntc.decode(m.lat, m.mlp, m.uv, compute="f16", packed=m.packed)
        assert torch.equal(single, m.out), i
        del single
    rng = np.random.default_rng(55)
    for i in (0, 17, 63):
        lat_np, Ws, bs = raw[i]
        sp = specs[i]
        idx = np.unique(rng.integers(0, sp.n, 4000))
        uv = I.pixel_uv_subset(sp.side, sp.side, "tiled", idx)
        ref = O.decode(O.Latents(lat_np, shift=I.PAPER_SHIFT), O.Mlp(Ws, bs), uv)
        got = mats[i].out[torch.from_numpy(idx).cuda()].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 2e-3, i


def test_autotuned_plan_equals_per_material(tmp_path):
    """The autotuner times its candidates, caches the winner, and the plan it
    builds decodes exactly like per-material launches."""
    ntc = _ntc()
    mats, _ = _materials(_small_specs())
    cache = str(tmp_path / "tune.json")
    cands = [dict(item_pixels=4096, waves_per_cu=8, stage_capacity=512),
             dict(item_pixels=16384, waves_per_cu=4, stage_capacity=1024)]
    best, table = ntc.autotune.tune_batched(mats, candidates=cands, cache=cache, reps=2)
    assert best in cands and len(table) == 2 and all(ms > 0 for _, ms in table)
    again, _ = ntc.autotune.tune_batched(mats, candidates=cands[:1], cache=cache)
    assert again == best  # served from the cache
    plan = ntc.autotune.tuned_batch_plan(mats, cache=cache, candidates=cands)
    for m in mats:
        m.out.fill_(-1.0)
    plan.launch()
    torch.cuda.synchronize()
    got = [m.out.clone() for m in mats]
    for m, g in zip(mats, got):
        ref = ntc.decode(m.lat, m.mlp, m.uv, compute="f16", packed=m.packed)
        assert torch.equal(g, ref)
