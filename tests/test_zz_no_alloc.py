"""Allocation-free classification (ntc_classify_noalloc): the same lists as
ntc_classify with a caller workspace, bit for bit, on two calls in a row
(the second on a smaller frame, over the scratch the first one filled).
The size limit is checked on the host (tests/test_abi_cpu.py)."""
import ctypes

import numpy as np
import pytest
import torch

import ntc_inputs as I

pytestmark = pytest.mark.gpu


def _abi():
    from paper_2506_06040_amd import _abi
    return _abi


def _outputs(w, h, n_mats):
    tiles = ((w + 7) // 8) * ((h + 3) // 4)
    return (torch.full((w * h,), -7, dtype=torch.int32, device="cuda"),
            torch.full((n_mats + 1,), -7, dtype=torch.int32, device="cuda"),
            torch.full((n_mats,), -7, dtype=torch.int32, device="cuda"),
            torch.full((tiles,), 9, dtype=torch.uint8, device="cuda"))


def _with_workspace(A, mat, w, h, n_mats):
    ws = ctypes.c_size_t(0)
    A.check(A.lib().ntc_classify_workspace(w, h, n_mats, ctypes.byref(ws)))
    work = torch.empty(ws.value, dtype=torch.uint8, device="cuda")
    lst, off, sim, tc = _outputs(w, h, n_mats)
    A.check(A.lib().ntc_classify(mat.data_ptr(), w, h, n_mats, lst.data_ptr(), off.data_ptr(), sim.data_ptr(),
                                 tc.data_ptr(), work.data_ptr(), ws.value, None))
    return lst, off, sim, tc


def _no_alloc(A, mat, w, h, n_mats):
    lst, off, sim, tc = _outputs(w, h, n_mats)
    A.check(A.lib().ntc_classify_noalloc(mat.data_ptr(), w, h, n_mats, lst.data_ptr(), off.data_ptr(),
                                         sim.data_ptr(), tc.data_ptr(), None))
    return lst, off, sim, tc


def test_noalloc_equals_workspace_entry_point():
    A = _abi()
    frames = [dict(w=1024, h=512, n=64, noise=0.01, seed=5),   # 1 MiB of counts
              dict(w=130, h=66, n=300, noise=0.3, seed=7)]     # smaller, on the same scratch
    for f in frames:
        print(f"[no-alloc classify] {f}", flush=True)
        rng = np.random.default_rng(f["seed"])
        mat_np = I.material_frame(rng, f["w"], f["h"], f["n"], noise=f["noise"])
        mat = torch.from_numpy(mat_np).cuda()
        a = _no_alloc(A, mat, f["w"], f["h"], f["n"])
        b = _with_workspace(A, mat, f["w"], f["h"], f["n"])
        torch.cuda.synchronize()
        for x, y, name in zip(a, b, ("pixel_list", "mat_offsets", "mat_simple", "tile_class")):
            assert torch.equal(x, y), (f, name)
        assert int(a[1][-1]) == int(((mat_np < f["n"])).sum())
