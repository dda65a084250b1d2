"""The allocation-free entry point (qnep_compute_static) against qnep_compute.

Both run the same kernels; the static variant takes its workspace from the
library's fixed device array.  Two calls in a row, the second on a smaller
structure, must each match qnep_compute on the same inputs (FP32 bar: the same
kernels in the same order give the same bits, so the comparison is exact), and
a structure whose workspace exceeds the array is rejected before any launch.
"""
import math
import sys

import numpy as np
import pytest

from paper_2601_19034_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("energy", "forces", "virial", "charges", "charges_naked", "bec", "polarization", "energy_terms")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _alloc(torch, n, dev):
    shapes = {"energy": ((1,), torch.float64), "forces": ((3, n), torch.float32), "virial": ((9,), torch.float64),
              "charges": ((n,), torch.float32), "charges_naked": ((n,), torch.float32),
              "bec": ((9, n), torch.float32), "polarization": ((3,), torch.float64),
              "energy_terms": ((8,), torch.float64)}
    return {k: torch.full(shp, float("nan"), dtype=dt, device=dev) for k, (shp, dt) in shapes.items()}


def _outs(B, out):
    return B.qnep_outputs(*[out[k].data_ptr() for k in KEYS])


def _run_both(torch, B, model, w):
    dev = torch.device("cuda:0")
    s = w.system
    pos = torch.from_numpy(s.pos_f32_soa()).to(dev)
    types = torch.from_numpy(s.types.astype(np.int32)).to(dev)
    th = torch.from_numpy(np.asarray(w.theta, dtype=np.float32)).to(dev)
    es = B.make_es(w.es)
    sysm = B.make_system(s.n, pos.data_ptr(), types.data_ptr(), s.cell)
    stream = torch.cuda.current_stream(dev).cuda_stream
    need = B.qnep_workspace_size(model, es, sysm)
    assert need <= B.QNEP_STATIC_WORKSPACE_BYTES, need
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ref = _alloc(torch, s.n, dev)
    B.qnep_compute(model, th.data_ptr(), es, sysm, _outs(B, ref), ws.data_ptr(), ws.numel(), stream)
    assert B.qnep_check_status(ws.data_ptr(), stream) == 0
    got = _alloc(torch, s.n, dev)
    flags = torch.full((1,), -1, dtype=torch.int32, device=dev)
    B.qnep_compute_static(model, th.data_ptr(), es, sysm, _outs(B, got), flags.data_ptr(), stream)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    return {k: v.cpu().numpy() for k, v in ref.items()}, {k: v.cpu().numpy() for k, v in got.items()}


def test_static_matches_compute_two_calls():
    import torch
    from paper_2601_19034_amd import binding as B

    assert torch.cuda.is_available()
    B.load()
    # first the 3,000-atom water crop with PPPM, then the 192-atom water box with Ewald
    cases = [inputs.workload(1, "crop"), inputs.workload(0)]
    for w in cases:
        model = B.qnep_model_create(w.hp, B.QNEP_MLP_FP32)
        try:
            _say(f"[static] {w.name} N={w.system.n} method={w.es.method}")
            ref, got = _run_both(torch, B, model, w)
            for k in KEYS:
                assert np.all(np.isfinite(got[k])), k
                np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        finally:
            B.qnep_model_destroy(model)


def test_static_rejects_oversized_structure():
    import torch
    from paper_2601_19034_amd import binding as B

    B.load()
    w = inputs.workload(1)  # 24,000 atoms: about 114 MiB of workspace
    model = B.qnep_model_create(w.hp, B.QNEP_MLP_FP32)
    try:
        es = B.make_es(w.es)
        sysm = B.make_system(w.system.n, 0, 0, w.system.cell)
        assert B.qnep_workspace_size(model, es, sysm) > B.QNEP_STATIC_WORKSPACE_BYTES
        # positions are never read: the size check fails before anything is enqueued
        dummy = torch.zeros(1, device="cuda:0")
        sysm = B.make_system(w.system.n, dummy.data_ptr(), dummy.data_ptr(), w.system.cell)
        out = B.qnep_outputs(*([None] * len(KEYS)))
        with pytest.raises(B.QnepError, match="static workspace"):
            B.qnep_compute_static(model, dummy.data_ptr(), es, sysm, out, 0,
                                  torch.cuda.current_stream().cuda_stream)
    finally:
        B.qnep_model_destroy(model)
