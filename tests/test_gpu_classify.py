"""Frame classification (ntc_classify; Sec. 4, Algorithm 1) and the frame
decode it feeds, against the oracle (oracle/classify.py, FP64 decode).
Lists, offsets and tile classes are integer results in a fixed order:
bit-exact."""
import numpy as np
import pytest
import torch

import ntc_inputs as I
import oracle as O
from oracle import classify as C

pytestmark = pytest.mark.gpu


def _ntc():
    import paper_2506_06040_amd as ntc
    return ntc


FRAMES = [
    dict(w=64, h=32, n=3, noise=0.0, seed=1),
    dict(w=37, h=22, n=5, noise=0.05, seed=2),
    dict(w=256, h=128, n=40, noise=0.02, seed=3),
    dict(w=200, h=120, n=1, noise=0.0, seed=4),
    dict(w=1024, h=512, n=64, noise=0.01, seed=5),
    dict(w=9, h=5, n=2, noise=0.0, seed=6, background=1.0),
    dict(w=130, h=66, n=300, noise=0.3, seed=7),
]


@pytest.mark.parametrize("f", FRAMES, ids=lambda f: f"{f['w']}x{f['h']}_m{f['n']}")
def test_classify_bitexact(f):
    ntc = _ntc()
    rng = np.random.default_rng(f["seed"])
    mat = I.material_frame(rng, f["w"], f["h"], f["n"], noise=f["noise"], background=f.get("background", 0.15))
    print(f"[classify] {f}", flush=True)
    lst, off, simple, tcls = ntc.classify(torch.from_numpy(mat).cuda(), f["n"])
    olst, ooff, osimple, otcls = C.classify(mat, f["n"])
    assert np.array_equal(off.cpu().numpy(), ooff)
    assert np.array_equal(simple.cpu().numpy(), osimple)
    assert np.array_equal(tcls.cpu().numpy(), otcls)
    assert np.array_equal(lst.cpu().numpy(), olst)
    # the same input gives the same lists
    lst2 = ntc.classify(torch.from_numpy(mat).cuda(), f["n"])[0]
    assert torch.equal(lst, lst2)


def test_gather_and_scatter():
    ntc = _ntc()
    rng = np.random.default_rng(8)
    h, w = 48, 80
    uv_img = rng.random((h, w, 2)).astype(np.float32)
    idx = rng.permutation(h * w)[:1000].astype(np.int32)
    uv = ntc.gather_uv(torch.from_numpy(uv_img).cuda(), torch.from_numpy(idx).cuda()).cpu().numpy()
    assert np.array_equal(uv, uv_img.reshape(-1, 2)[idx])
    for dt in (torch.float32, torch.float16):
        rows = torch.from_numpy(rng.random((1000, 9)).astype(np.float32)).to(dt).cuda()
        img = torch.zeros((h, w, 9), dtype=dt, device="cuda")
        ntc.scatter_rows(rows, torch.from_numpy(idx).cuda(), img)
        ref = np.zeros((h * w, 9), np.float32)
        ref[idx] = rows.float().cpu().numpy()
        assert np.array_equal(img.float().cpu().numpy().reshape(-1, 9), ref)


def test_frame_decode_equals_per_material_and_oracle():
    ntc = _ntc()
    rng = np.random.default_rng(9)
    h, w, n_mats = 192, 256, 6
    mat = I.material_frame(rng, w, h, n_mats, noise=0.02)
    uv_img = I.pixel_uv(w, h).reshape(h, w, 2)
    dims = [(14, 64, 64, 64, 8), (14, 32, 32, 8), (14, 64, 8), (14, 16, 16, 16, 8), (14, 64, 64, 8), (14, 32, 8)]
    mats, omats = [], []
    for m in range(n_mats):
        lat_np = I.bc1_pyramid(rng, [(128, 128), (64, 64), (32, 32), (16, 16)])
        Ws, bs = I.xavier_mlp(rng, dims[m], bias="normal")
        mats.append((ntc.Latents(lat_np, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs)))
        omats.append((O.Latents(lat_np, shift=I.PAPER_SHIFT), O.Mlp(Ws, bs)))
    fd = ntc.FrameDecoder(mats)
    mat_t = torch.from_numpy(mat).cuda()
    uv_t = torch.from_numpy(np.ascontiguousarray(uv_img)).cuda()
    out_t = fd.decode(mat_t, uv_t)
    # the decode through the pixel lists equals gather + decode + scatter
    assert torch.equal(out_t, fd.decode(mat_t, uv_t, indexed=False))
    out = out_t.cpu().numpy().reshape(-1, 8)
    lst, off, _, _ = ntc.classify(mat_t, n_mats)
    lst, off = lst.cpu().numpy(), off.cpu().numpy()
    flat_uv = uv_img.reshape(-1, 2)
    invalid = np.nonzero(mat.reshape(-1) >= n_mats)[0]
    assert np.all(out[invalid] == 0.0)
    for m, ((lat, mlp), (olat, omlp)) in enumerate(zip(mats, omats)):
        pix = lst[off[m]:off[m + 1]]
        if pix.size == 0:
            continue
        single = ntc.decode(lat, mlp, torch.from_numpy(flat_uv[pix]).cuda(), compute="f16").cpu().numpy()
        assert np.array_equal(out[pix], single), m
        ref = O.decode(olat, omlp, flat_uv[pix])
        err = np.abs(out[pix] - ref).max()
        print(f"[frame decode] material {m}: {pix.size} px, max err {err:.2e}", flush=True)
        assert err <= 2e-3, m


def test_batched_indexed_ignores_invalid_indices():
    """Indices outside the image read uv (0, 0) and write nothing; valid ones
    equal the plain decode of the same uv."""
    ntc = _ntc()
    rng = np.random.default_rng(10)
    h, w = 64, 96
    lat_np = I.bc1_pyramid(rng, [(64, 64), (32, 32), (16, 16), (8, 8)])
    Ws, bs = I.xavier_mlp(rng, (14, 32, 32, 8), bias="normal")
    lat, mlp = ntc.Latents(lat_np, shift=I.PAPER_SHIFT), ntc.Mlp(Ws, bs)
    uv_img = torch.from_numpy(rng.random((h * w, 2)).astype(np.float32)).cuda()
    idx = rng.permutation(h * w)[:2000].astype(np.int32)
    idx[::97] = -1
    idx[5::97] = h * w + 3
    out = torch.full((h * w, 8), 7.0, device="cuda")
    m = ntc.Material(lat, mlp, uv_img, out=out, pixel_index=torch.from_numpy(idx).cuda())
    ntc.BatchPlan([m]).launch()
    torch.cuda.synchronize()
    good = idx[(idx >= 0) & (idx < h * w)]
    ref = ntc.decode(lat, mlp, uv_img[torch.from_numpy(good).long().cuda()].contiguous(), compute="f16")
    got = out.cpu().numpy()
    assert np.array_equal(got[good], ref.cpu().numpy())
    untouched = np.setdiff1d(np.arange(h * w), good)
    assert np.all(got[untouched] == 7.0)
