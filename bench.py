#!/usr/bin/env python3
"""Throughput of the fused BC1 + MLP decode on one MI355X.

Workload (the headline configuration): 4096 x 4096 output pixels, four BC1
latent levels of 2048^2, 1024^2, 512^2 and 256^2 texels (random blocks,
seed 2), MLP 14-64-64-64-8 (Xavier-normal, zero biases), uv at pixel
centres plus uniform jitter of +-1/2 pixel, pixels in 8x8-tile order,
FP32 output. One step = one ntc_decode launch over all 16.7 M pixels with
inputs resident in HBM. value = pixels x steps / time of the timed steps,
in Gtexel/s, for the FP16 matrix-core path; the plain FP32 and the E4M3
paths, the backward and the batched decode are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gtexels/s fused BC1+MLP decode at 4096², FP16/FP8 MFMA vs FP32 plain at stated err"
PEAK_FP16_TFLOPS = 2500.0      # MI355X dense FP16 matrix peak
PEAK_FP8_TFLOPS = 5000.0
PEAK_FP32_VALU_TFLOPS = 157.3  # FP32 vector peak
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_2506_06040_amd/csrc/ntc_mfma.hip", "paper_2506_06040_amd/csrc/ntc_mfma_tile.hpp",
                  "paper_2506_06040_amd/csrc/ntc_device.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_decode_f16_c2.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def settle(fn, seconds=0.5):
    """Run fn until `seconds` have passed: the engine clock ramps up under a
    sustained load, and the warm-up steps alone are too short for it. Not
    part of any timed region."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()


def algorithmic_flops_per_px(dims):
    return 2 * sum(dims[i] * dims[i + 1] for i in range(len(dims) - 1))


def time_launches(fn, steps, warmup, settle_s=0.3):
    """Average milliseconds per call of fn (launches on the current stream),
    measured with HIP events around `steps` calls after the clock has
    settled under fn (settle_s seconds) and `warmup` calls."""
    import torch
    if settle_s > 0:
        settle(fn, settle_s)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def cpu_baseline(lat_np, Ws, bs, uv, shift, gpu_out, target_s=10.0):
    """The FP64 oracle timed on this host's cores on a bounded prefix of the
    pixels; also yields the GPU's error on that prefix."""
    import numpy as np

    import oracle as O
    olat = O.Latents(lat_np, shift=shift)
    omlp = O.Mlp(Ws, bs)
    threads = O.default_threads()
    probe = 65536
    t0 = time.perf_counter()
    O.decode(olat, omlp, uv[:probe], threads=threads)
    rate = probe / (time.perf_counter() - t0)
    n = int(min(uv.shape[0], max(probe, rate * target_s)))
    n -= n % 64
    t0 = time.perf_counter()
    ref = O.decode(olat, omlp, uv[:n], threads=threads)
    dt = time.perf_counter() - t0
    errs = {}
    for name, out in gpu_out.items():
        d = np.abs(out[:n].astype(np.float64) - ref)
        errs[name] = {"max": [float(f"{v:.3g}") for v in d.max(0)],
                      "rms": [float(f"{v:.3g}") for v in np.sqrt((d ** 2).mean(0))],
                      "max_all": float(f"{d.max():.3g}")}
    return {"value": n / dt / 1e9, "unit": "Gtexel/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of {uv.shape[0]} pixels (8x8-tile order) of the same workload, FP64, "
                      f"{dt:.1f} s"}, errs


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["f16", "f32", "fp8", "bf16", "rowmajor", "varA", "out9", "filtered", "bwd", "qat",
                                       "batched", "copy"],
                    default=None,
                    help="run only one leg (for profiling); 'copy' runs a plain 1 GiB device copy that "
                         "calibrates the HBM byte counters")
    ap.add_argument("--no-extras", action="store_true", help="skip backward and batched legs")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the decode has no cross-GPU step "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import ntc_inputs as I
    import paper_2506_06040_amd as ntc

    dev = "cuda"
    torch.cuda.set_device(0)
    if args.only == "copy":
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        ms = time_launches(lambda: dst.copy_(src), 5, 1)
        log(json.dumps({"leg": "copy", "bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
                        "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}))
        return
    wl = I.WORKLOADS["c2"]
    log("[bench] generating the 4096^2 workload")
    lat_np, Ws, bs, uv = I.make_workload(wl)
    N = uv.shape[0]
    lat = ntc.Latents(lat_np, shift=wl.shift, device=dev)
    mlp = ntc.Mlp(Ws, bs, device=dev)
    uvt = torch.from_numpy(uv).to(dev)
    out = torch.empty((N, 8), dtype=torch.float32, device=dev)
    flops = algorithmic_flops_per_px(wl.dims) * N
    result = {}

    def leg(compute, packed, steps, warmup):
        fn = lambda: ntc.decode(lat, mlp, uvt, compute=compute, packed=packed, out=out)
        ms = time_launches(fn, steps, warmup)
        return ms

    gpu_out = {}
    p16 = ntc.pack(mlp, "f16")
    if args.only in (None, "f16"):
        log("[bench] FP16 matrix-core decode")
        settle(lambda: ntc.decode(lat, mlp, uvt, compute="f16", packed=p16, out=out))
        ms16 = leg("f16", p16, args.steps, args.warmup)
        gpu_out["f16"] = out.cpu().numpy()
        result["f16_ms"] = ms16
    if args.only in (None, "f32"):
        log("[bench] FP32 plain decode")
        p32 = ntc.pack(mlp, "f32")
        ms32 = leg("f32", p32, max(2, args.steps // 5), 1)
        gpu_out["f32"] = out.cpu().numpy()
        result["f32_ms"] = ms32
    if args.only in (None, "fp8"):
        log("[bench] FP8 matrix-core decode")
        cal = torch.from_numpy(I.calibration_uv()).to(dev)
        amax = ntc.calibrate_fp8(lat, mlp, cal)
        p8 = ntc.pack(mlp, "fp8", act_amax=amax)
        ms8 = leg("fp8", p8, args.steps, args.warmup)
        gpu_out["fp8"] = out.cpu().numpy()
        result["fp8_ms"] = ms8
    if args.only in (None, "bf16"):
        log("[bench] BF16 matrix-core decode")
        pb = ntc.pack(mlp, "bf16")
        msb = leg("bf16", pb, args.steps, args.warmup)
        gpu_out["bf16"] = out.cpu().numpy()
        result["bf16_ms"] = msb

    extras = {}
    if args.only in (None, "rowmajor"):
        # the same samples in row-major pixel order: spans are 256-pixel runs
        # of one image row instead of four 8x8 tiles
        log("[bench] FP16 matrix-core decode, row-major pixel order")
        perm = I.tiled_to_rowmajor(wl.out_w, wl.out_h)
        uv_rm = np.empty_like(uv)
        uv_rm[perm] = uv
        uvt_rm = torch.from_numpy(uv_rm).to(dev)
        ms_rm = time_launches(lambda: ntc.decode(lat, mlp, uvt_rm, compute="f16", packed=p16, out=out), args.steps,
                              args.warmup)
        extras["rowmajor_f16"] = {"Gtexel_per_s": N / (ms_rm * 1e-3) / 1e9, "ms": ms_rm,
                                  "frac_fp16_mfma": flops / (ms_rm * 1e-3) / 1e12 / PEAK_FP16_TFLOPS,
                                  "order": "row-major (same uv per pixel as the tiled headline)"}
        del uvt_rm
    if args.only in (None, "varA") and not args.no_extras:
        # latent layout variant A of the paper: levels at W, W, W/2, W/2
        log("[bench] FP16 decode, latent layout variant A (4096^2, 4096^2, 2048^2, 2048^2)")
        sizes_a = [(4096, 4096), (4096, 4096), (2048, 2048), (2048, 2048)]
        lat_a = ntc.Latents(I.bc1_pyramid(I.streams(wl.seed + 100)[0], sizes_a), shift=wl.shift, device=dev)
        fa = lambda: ntc.decode(lat_a, mlp, uvt, compute="f16", packed=p16, out=out)
        ms_a = time_launches(fa, args.steps, args.warmup)
        extras["varA_f16"] = {"Gtexel_per_s": N / (ms_a * 1e-3) / 1e9, "ms": ms_a,
                              "frac_fp16_mfma": flops / (ms_a * 1e-3) / 1e12 / PEAK_FP16_TFLOPS,
                              "latents": sizes_a}
        del lat_a
    if args.only in (None, "out9") and not args.no_extras:
        # nine output channels: the same network with one more output row
        # (Xavier-normal like the others, zero bias)
        log("[bench] FP16 decode, 9 output channels")
        r9 = I.streams(wl.seed + 300)[1]
        fan = Ws[-1].shape[1]
        row = (r9.standard_normal((1, fan)) * np.sqrt(2.0 / (fan + 9))).astype(np.float32)
        mlp9 = ntc.Mlp(list(Ws[:-1]) + [np.concatenate([Ws[-1], row], 0)],
                       list(bs[:-1]) + [np.concatenate([bs[-1], np.zeros(1, np.float32)])], device=dev)
        p9 = ntc.pack(mlp9, "f16")
        out9 = torch.empty((N, 9), dtype=torch.float32, device=dev)
        ms9 = time_launches(lambda: ntc.decode(lat, mlp9, uvt, compute="f16", packed=p9, out=out9), args.steps,
                            args.warmup)
        flops9 = algorithmic_flops_per_px(tuple(wl.dims[:-1]) + (9,)) * N
        extras["out9_f16"] = {"Gtexel_per_s": N / (ms9 * 1e-3) / 1e9, "ms": ms9,
                              "frac_fp16_mfma": flops9 / (ms9 * 1e-3) / 1e12 / PEAK_FP16_TFLOPS}
        del out9, mlp9, p9
    if args.only in (None, "filtered") and not args.no_extras:
        # mip-mapped latents (2048^2 .. 256^2 levels, full BC1 mip chains),
        # a 4096^2 perspective ground plane with its screen derivatives
        log("[bench] filtered decode: 4096^2 perspective plane, trilinear and 16x anisotropic")
        rf = I.streams(wl.seed + 200)[0]
        chains = [I.bc1_mip_chain(rf, w, h) for (w, h) in wl.latent_sizes]
        lm = ntc.LatentMips(chains, shift=wl.shift, device=dev)
        uvp, duvp = I.perspective_plane(4096, 4096, far=24.0)
        uvp_t, duvp_t = torch.from_numpy(uvp).to(dev), torch.from_numpy(duvp).to(dev)
        res_f = {}
        for filt, ma in (("trilinear", 1), ("anisotropic", 16)):
            ff = lambda: ntc.decode_filtered(lm, mlp, uvp_t, duvp_t, filter=filt, max_aniso=max(ma, 1), packed=p16,
                                             out=out)
            ms_f = time_launches(ff, max(2, args.steps // 4), 2)
            res_f[filt] = {"ms": ms_f, "Gtexel_per_s": N / (ms_f * 1e-3) / 1e9}
        extras["filtered_c2"] = res_f
        del lm, uvp_t, duvp_t, chains
    if args.only in (None, "bwd") and not args.no_extras:
        log("[bench] backward (2^20 samples)")
        w3 = I.WORKLOADS["c3"]
        l3, W3, b3, uv3 = I.make_workload(w3)
        lat3 = [torch.from_numpy(a).to(dev).requires_grad_(True) for a in l3]
        Wt = [torch.from_numpy(w).to(dev).requires_grad_(True) for w in W3]
        bt = [torch.from_numpy(b).to(dev).requires_grad_(True) for b in b3]
        uv3t = torch.from_numpy(uv3).to(dev)
        tgt = torch.from_numpy(I.point_sample(I.c3_targets(), uv3)).to(dev)

        def step():
            o = ntc.decode_fn(uv3t, lat3, Wt, bt, shift=w3.shift)
            loss = torch.mean((o - tgt) ** 2)
            loss.backward()

        ms_b = time_launches(step, 5, 2)
        extras["backward_c3"] = {"ms_per_step": ms_b, "samples": int(uv3.shape[0]),
                                 "Msample_per_s": uv3.shape[0] / ms_b / 1e3,
                                 "step": "forward + L2 loss + backward (weights, biases, 1024^2..128^2 float latents)"}
        del lat3, Wt, bt, uv3t, tgt
    if args.only in (None, "qat") and not args.no_extras:
        log("[bench] trainable BC1 latents (2^20 samples)")
        w3 = I.WORKLOADS["c3"]
        _, W3, b3, uv3 = I.make_workload(w3)
        sizes = [(w, h) for (w, h) in w3.latent_sizes]
        rq = np.random.default_rng(6)
        params = [torch.from_numpy((rq.standard_normal((h // 4, w // 4, ntc.QAT_PARAMS)) * 1.5)
                                   .astype(np.float32)).to(dev).requires_grad_(True) for (w, h) in sizes]
        Wt = [torch.from_numpy(w).to(dev).requires_grad_(True) for w in W3]
        bt = [torch.from_numpy(b).to(dev).requires_grad_(True) for b in b3]
        uv3t = torch.from_numpy(uv3).to(dev)
        tgt = torch.from_numpy(I.point_sample(I.c3_targets(), uv3)).to(dev)

        def qstep():
            lat = [ntc.qat_texels_fn(p, w, h) for p, (w, h) in zip(params, sizes)]
            o = ntc.decode_fn(uv3t, lat, Wt, bt, shift=w3.shift)
            loss = torch.mean((o - tgt) ** 2)
            loss.backward()

        ms_q = time_launches(qstep, 5, 2)
        pd = [p.detach() for p in params]
        gt = [torch.randn((h, w, 3), device=dev) for (w, h) in sizes]
        ms_fwd = time_launches(lambda: [ntc.qat_texels(p, w, h) for p, (w, h) in zip(pd, sizes)], 20, 3)
        ms_bwd = time_launches(lambda: [ntc.qat_backward(p, w, h, g) for p, (w, h), g in zip(pd, sizes, gt)], 20, 3)
        texels = sum(w * h for (w, h) in sizes)
        # algorithmic bytes per texel: 88 B of logits per 16 texels, 12 B of
        # texels (forward) or texel gradients (backward), 88 B / 16 of logit
        # gradients written (backward)
        fb, bb = texels * (5.5 + 12), texels * (12 + 5.5 + 5.5)
        extras["qat_c3"] = {"ms_per_step": ms_q, "samples": int(uv3.shape[0]), "texels": texels,
                            "qat_texels_ms": ms_fwd, "qat_backward_ms": ms_bwd,
                            "qat_texels_GBs": fb / ms_fwd / 1e6, "qat_backward_GBs": bb / ms_bwd / 1e6,
                            "step": "quantised texels from logits + forward + L2 loss + backward into the "
                                    "logits, MLP weights and biases (1024^2..128^2 trainable BC1 levels)"}
        del params, Wt, bt, uv3t, tgt, pd, gt
    if args.only in (None, "batched") and not args.no_extras:
        log("[bench] batched: 64 materials")
        specs = I.material_specs()
        mats = []
        for sp in specs:
            lnp, Wm, bm = I.make_material(sp)
            m = ntc.Material(ntc.Latents(lnp, device=dev), ntc.Mlp(Wm, bm, device=dev),
                             I.pixel_uv_torch(sp.side, sp.side, "tiled", dev))
            mats.append(m)
        # tile shapes (work-item size, waves per CU, staging capacity) from
        # the autotuner; the tuning launches are not part of the timing
        best, table = ntc.autotune.tune_batched(mats, cache=None)
        plan = ntc.BatchPlan(mats, ntc.batch_cfg(n_cus=ntc.api._device_cus(dev), **best))
        npx = sum(sp.n for sp in specs)
        flops_b = sum(algorithmic_flops_per_px(sp.dims) * sp.n for sp in specs)
        ms_one = time_launches(plan.launch, 5, 2)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                plan.launch(stream=s)
        torch.cuda.current_stream().wait_stream(s)
        ms_graph = time_launches(g.replay, 5, 2)

        def per_material():
            for m in mats:
                ntc.decode(m.lat, m.mlp, m.uv, compute="f16", packed=m.packed, out=m.out)

        ms_many = time_launches(per_material, 3, 1)
        extras["batched_c5"] = {"materials": len(specs), "pixels": int(npx),
                                "one_launch_ms": ms_one, "graph_replay_ms": ms_graph,
                                "per_material_launches_ms": ms_many,
                                "Gtexel_per_s": npx / ms_graph / 1e6,
                                "per_material_Gtexel_per_s": npx / ms_many / 1e6,
                                "flops": flops_b,
                                "frac_fp16_mfma": flops_b / (ms_graph * 1e-3) / 1e12 / PEAK_FP16_TFLOPS,
                                "per_material_frac_fp16_mfma": flops_b / (ms_many * 1e-3) / 1e12 / PEAK_FP16_TFLOPS,
                                "waves": plan.header()["n_waves"], "autotuned": best,
                                "autotune_ms": {json.dumps(c, sort_keys=True): round(ms, 3) for c, ms in table}}
        del plan

        # a 4096^2 frame over the same 64 materials: classification of its
        # 8x4 tiles, uv gather, one batched decode, output scatter
        log("[bench] frame: 4096^2, 64 materials, classification + batched decode")
        fw = fh = 4096
        mat_ids = torch.from_numpy(I.material_frame(np.random.default_rng(7), fw, fh, len(mats),
                                                    noise=0.002)).to(dev)
        uv_img = torch.from_numpy(I.pixel_uv(fw, fh)).to(dev)
        fd = ntc.FrameDecoder([(m.lat, m.mlp) for m in mats])
        out_img = torch.zeros((fh, fw, 8), dtype=torch.float32, device=dev)
        fp = fd.plan(mat_ids, uv_img, out=out_img, indexed=True)
        fg = fd.plan(mat_ids, uv_img, indexed=False)
        n_valid = int(fp["pixel_list"].shape[0])
        A = ntc.api.A
        ws = ctypes.c_size_t(0)
        A.check(A.lib().ntc_classify_workspace(fw, fh, len(mats), ctypes.byref(ws)))
        cw = torch.empty(ws.value, dtype=torch.uint8, device=dev)
        cl = torch.empty(fw * fh, dtype=torch.int32, device=dev)
        co = torch.empty(len(mats) + 1, dtype=torch.int32, device=dev)
        cs = torch.empty(len(mats), dtype=torch.int32, device=dev)
        ct = torch.empty(((fw + 7) // 8) * ((fh + 3) // 4), dtype=torch.uint8, device=dev)
        sh = ntc.api._stream_handle()

        def classify_only():
            A.check(A.lib().ntc_classify(mat_ids.data_ptr(), fw, fh, len(mats), cl.data_ptr(), co.data_ptr(),
                                         cs.data_ptr(), ct.data_ptr(), cw.data_ptr(), ws.value, sh))

        ms_cls = time_launches(classify_only, 20, 3)
        ms_idx = time_launches(fp["plan"].launch, 10, 2)
        ms_gat = time_launches(lambda: ntc.gather_uv(uv_img, fg["pixel_list"]), 20, 3)
        ms_dec = time_launches(fg["plan"].launch, 10, 2)
        ms_sca = time_launches(lambda: ntc.scatter_rows(fg["rows"], fg["pixel_list"], out_img), 20, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            fd.decode(mat_ids, uv_img, out=out_img)
        torch.cuda.synchronize()
        ms_e2e = (time.perf_counter() - t0) / 3 * 1e3
        gpu_ms = ms_cls + ms_idx
        tcls = fp["tile_class"].cpu().numpy()
        extras["frame_c5"] = {"pixels": fw * fh, "neural_pixels": n_valid,
                              "tiles": {"none": int((tcls == 0).sum()), "simple": int((tcls == 1).sum()),
                                        "mixed": int((tcls == 2).sum())},
                              "classify_ms": ms_cls, "indexed_decode_ms": ms_idx, "gpu_ms": gpu_ms,
                              "Gtexel_per_s": n_valid / gpu_ms / 1e6,
                              "gathered": {"gather_ms": ms_gat, "decode_ms": ms_dec, "scatter_ms": ms_sca,
                                           "gpu_ms": ms_cls + ms_gat + ms_dec + ms_sca},
                              "classify_GBs": (2 * 2 * fw * fh + 4 * n_valid) / ms_cls / 1e6,
                              "end_to_end_ms": ms_e2e,
                              "note": "indexed: the batched decode reads uv and writes the image through the "
                                      "pixel lists; end_to_end includes the host batch plan of each frame"}
        del mats, fd, fp, fg, mat_ids, uv_img, out_img, cw, cl

    cpu = None
    errs = {}
    if args.only is None and not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle)")
        cpu, errs = cpu_baseline(lat_np, Ws, bs, uv, wl.shift, gpu_out)

    if args.only not in (None, "f16"):
        log(json.dumps({"leg": args.only, **result, **extras}))
        return

    ms16 = result["f16_ms"]
    value = N / (ms16 * 1e-3) / 1e9
    achieved = flops / (ms16 * 1e-3) / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_sha") == kernel_sha():
            traffic = tr.get("hbm_bytes_per_launch")
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gtexel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms16, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": "4096x4096 decode, BC1 latents 2048^2/1024^2/512^2/256^2, MLP 14-64-64-64-8, "
                               "jittered pixel-centre uv in 8x8-tile order, FP16 MFMA, FP32 out",
                   "pixels": N, "mlp": list(wl.dims)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP16_TFLOPS, 4), "traffic": traffic,
                     "kernel": "decode_mfma_kernel<PrecF16,64,4,1>",
                     "flops_per_launch": flops,
                     "hbm_algorithmic_GBs": round(N * 40 / (ms16 * 1e-3) / 1e9, 1)},
        "cpu_baseline": cpu,
    }
    if "f32_ms" in result:
        g32 = N / (result["f32_ms"] * 1e-3) / 1e9
        line["fp32_plain"] = {"Gtexel_per_s": round(g32, 3), "ms": round(result["f32_ms"], 3),
                              "frac_fp32_valu": round(flops / (result["f32_ms"] * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4)}
        line["speedup_f16_vs_f32"] = round(value / g32, 2)
    if "fp8_ms" in result:
        g8 = N / (result["fp8_ms"] * 1e-3) / 1e9
        line["fp8"] = {"Gtexel_per_s": round(g8, 3), "ms": round(result["fp8_ms"], 4),
                       "frac_fp8_mfma": round(flops / (result["fp8_ms"] * 1e-3) / 1e12 / PEAK_FP8_TFLOPS, 4)}
    if "bf16_ms" in result:
        gb = N / (result["bf16_ms"] * 1e-3) / 1e9
        line["bf16"] = {"Gtexel_per_s": round(gb, 3), "ms": round(result["bf16_ms"], 4),
                        "frac_bf16_mfma": round(flops / (result["bf16_ms"] * 1e-3) / 1e12 / PEAK_FP16_TFLOPS, 4)}
    if errs:
        line["err_vs_oracle"] = errs
    line.update(extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
