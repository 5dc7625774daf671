"""Tile-shape autotuner for the matrix-core decode and the batched launch.

Each candidate configuration is launched on the current stream and timed with
HIP events (best of a few repetitions after a warm-up launch). The winner per
(device, library version, problem signature) is kept in a JSON cache, so a
process tunes a given problem once and later processes reuse the result.

Tuned knobs:
  * single decode: persistent waves per compute unit and the LDS staging
    capacity per wave (texels);
  * batched decode: the work-item size (pixels per item handed to a wave),
    waves per compute unit and the staging capacity.
The span length of the staging loop and the register budget are fixed when
the library is compiled and are not tuned here.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import torch

from . import _abi as A
from . import api

DECODE_CANDIDATES = [dict(waves_per_cu=w, stage_capacity=c) for w in (4, 8, 12) for c in (512, 1024)]
BATCH_CANDIDATES = [dict(item_pixels=p, waves_per_cu=w, stage_capacity=c)
                    for p in (2048, 4096, 8192, 16384) for w in (8, 12) for c in (512, 1024)]


def default_cache_path() -> str:
    base = os.environ.get("NTC_AUTOTUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "ntc", "autotune.json")


def _device_key(device="cuda") -> str:
    p = torch.cuda.get_device_properties(torch.device(device))
    return f"{p.name}|{p.multi_processor_count}|lib{A.lib().ntc_version()}"


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: Dict) -> None:
    d = _load(path)
    d[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_ms(fn, reps: int = 3, warmup: int = 1) -> float:
    """Best of `reps` event-timed calls of fn on the current stream."""
    for _ in range(warmup):
        fn()
    best = float("inf")
    for _ in range(reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        e.synchronize()
        best = min(best, s.elapsed_time(e))
    return best


def _sig(parts: Iterable) -> str:
    return hashlib.sha1(json.dumps(list(parts), sort_keys=True).encode()).hexdigest()[:16]


def decode_signature(lat: api.Latents, mlp: api.Mlp, n: int, compute: str) -> str:
    return "decode:" + _sig([list(lat.sizes), int(lat.c.address), [int(d) for d in mlp.dims], int(n), compute])


def batched_signature(materials: Sequence[api.Material]) -> str:
    rows = sorted([list(m.lat.sizes), [int(d) for d in m.mlp.dims], int(m.uv.shape[0])] for m in materials)
    return "batched:" + _sig(rows)


def tune_decode(lat: api.Latents, mlp: api.Mlp, uv: torch.Tensor, compute: str = "f16",
                packed: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                candidates: Sequence[Dict] = DECODE_CANDIDATES, cache: Optional[str] = "default",
                reps: int = 3) -> Tuple[Dict, List[Tuple[Dict, float]]]:
    """Best tile configuration for ntc_decode on these inputs, and the timing table."""
    path = default_cache_path() if cache == "default" else cache
    key = _device_key(uv.device) + "|" + decode_signature(lat, mlp, uv.shape[0], compute)
    if path:
        hit = _load(path).get(key)
        if hit:
            return hit["best"], [(r["cfg"], r["ms"]) for r in hit["table"]]
    if packed is None:
        packed = api.pack(mlp, compute)
    if out is None:
        out = torch.empty((uv.shape[0], mlp.n_out), dtype=torch.float32, device=uv.device)
    table = []
    for c in candidates:
        cfg = api.tile_cfg(**c)
        ms = time_ms(lambda: api.decode(lat, mlp, uv, compute=compute, packed=packed, cfg=cfg, out=out), reps)
        table.append((dict(c), ms))
    best = min(table, key=lambda t: t[1])[0]
    if path:
        _store(path, key, {"best": best, "table": [{"cfg": c, "ms": ms} for c, ms in table]})
    return best, table


def tune_batched(materials: Sequence[api.Material], candidates: Sequence[Dict] = BATCH_CANDIDATES,
                 cache: Optional[str] = "default", reps: int = 3) -> Tuple[Dict, List[Tuple[Dict, float]]]:
    """Best batch configuration (item size, waves per CU, staging capacity)
    for one persistent launch over these materials, and the timing table."""
    dev = materials[0].uv.device
    path = default_cache_path() if cache == "default" else cache
    key = _device_key(dev) + "|" + batched_signature(materials)
    if path:
        hit = _load(path).get(key)
        if hit:
            return hit["best"], [(r["cfg"], r["ms"]) for r in hit["table"]]
    n_cus = api._device_cus(dev)
    table = []
    for c in candidates:
        plan = api.BatchPlan(materials, api.batch_cfg(n_cus=n_cus, **c), device=dev)
        table.append((dict(c), time_ms(plan.launch, reps)))
        del plan
    best = min(table, key=lambda t: t[1])[0]
    if path:
        _store(path, key, {"best": best, "table": [{"cfg": c, "ms": ms} for c, ms in table]})
    return best, table


def tuned_batch_plan(materials: Sequence[api.Material], cache: Optional[str] = "default",
                     candidates: Sequence[Dict] = BATCH_CANDIDATES) -> api.BatchPlan:
    """BatchPlan built with the autotuned configuration."""
    best, _ = tune_batched(materials, candidates=candidates, cache=cache)
    dev = materials[0].uv.device
    return api.BatchPlan(materials, api.batch_cfg(n_cus=api._device_cus(dev), **best), device=dev)
