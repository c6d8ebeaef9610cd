"""The allocation-free entry point (ldpcx_decode_noalloc) against ldpcx_decode.

Every decoder family that needs a workspace takes it from the library's static device
array; two calls in a row (the second with a smaller batch, so it runs on what the
first left in the array) must give bit for bit what ldpcx_decode gives on the same
inputs.  Batches are sized so that the first call runs as several chunks.
"""
import numpy as np
import pytest
import torch

from paper_2508_03567_amd import ldpcx as L
from paper_2508_03567_amd import synth as S

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _same(a, b, what):
    for x, y, name in zip(a[:3], b[:3], ("hard", "ok", "iters")):
        assert torch.equal(x, y), f"{what}: {name} differs"


def _pair(h, prm, llr, what):
    ref = L.decode(h, prm, llr)
    got = L.decode_noalloc(h, prm, llr)
    torch.cuda.synchronize()
    _same(got, ref, what)
    assert got[3] == ref[3]


@pytest.mark.parametrize("cfg,plan,sizes", [
    (2, None, (600, 100)),                      # interleaved binary, n = 64800: 256-codeword slices
    (3, ("minmax_interleaved", 64, 256), (2600, 300)),  # interleaved Min-Max, GF(64): two chunks, then one
    (3, None, (2600, 300)),                     # default: one codeword per workgroup, alpha-free, no workspace
    (3, ("spa_wave",), (2600, 300)),            # FFT-SPA wave kernels, GF(64)
    (1, None, (300, 70)),                       # QC packed: no workspace at all
])
def test_noalloc_matches_decode(cfg, plan, sizes):
    w = S.workload(cfg, batch=max(sizes))
    rule = "spa" if plan and plan[0].startswith("spa") else w.rule
    _, x = S.make_inputs(w)
    llr = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    h = L.Code(w.code)
    iters = min(w.max_iters, 6)
    for early in (False, True):
        prm = L.params(rule, w.schedule, iters, early_stop=early, nms_num=w.nms_num, nms_shift=w.nms_shift,
                       oms_offset=w.oms_offset, msg_max=w.msg_max)
        for b in sizes:
            if plan:
                L.plan_set(h, prm, b, *plan)
            print(f"noalloc: workload {w.name} rule {rule} early_stop {early} batch {b}", flush=True)
            _pair(h, prm, llr[:b].contiguous(), f"{w.name} {rule} batch {b} early_stop {early}")


def test_noalloc_rejects_bad_arguments():
    w = S.workload(0, batch=4)
    h = L.Code(w.code)
    prm = L.params(w.rule, w.schedule, 3)
    llr = torch.zeros((4, w.code.n), dtype=torch.int8, device=DEV)
    with pytest.raises(L.LdpcxError) as ei:
        L.ldpcx_decode_noalloc(h.handle, prm, -1, llr.data_ptr(), 0, 0, 0)
    assert ei.value.status == L.E_INVAL
    with pytest.raises(L.LdpcxError) as ei:
        L.ldpcx_decode_noalloc(h.handle, prm, 4, llr.data_ptr(), 0, 0, 0)
    assert ei.value.status == L.E_INVAL
