"""GPU tests of the continuous-batching server.

Every request must get exactly what a plain decode of that request alone gives
(bit-exact decisions, flags and iteration counts), whatever else is in flight,
however the budget splits it and in both serving modes; cancellation, budget
rejection and the counters are checked too.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2508_03567_amd import ldpcx as L
from paper_2508_03567_amd import synth as S

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

_CODES = {}
_POOL = {}


def _code(cfg):
    if cfg not in _CODES:
        _CODES[cfg] = L.Code(S.workload(cfg).code)
    return _CODES[cfg]


def _pool(cfg, size):
    """Seeded inputs of one configuration (requests take slices of it)."""
    if cfg not in _POOL or _POOL[cfg][1].shape[0] < size:
        w = S.workload(cfg, batch=size)
        _, llr = S.make_inputs(w, seed_offset=77)
        _POOL[cfg] = (w, np.ascontiguousarray(llr))
    return _POOL[cfg]


def _prm(w, max_iters=None):
    return L.params(rule=w.rule, schedule=w.schedule, max_iters=w.max_iters if max_iters is None else max_iters,
                    early_stop=True, nms_num=w.nms_num, nms_shift=w.nms_shift, oms_offset=w.oms_offset,
                    msg_max=w.msg_max)


def _requests(n_req, seed, max_size=300):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_req):
        cfg = int(rng.choice([0, 1, 2, 3], p=[0.4, 0.3, 0.1, 0.2]))
        size = int(np.exp(rng.uniform(0, np.log(max_size + 1))))
        if cfg == 2:
            size = min(size, 3)
        w, pool = _pool(cfg, 512 if cfg != 2 else 8)
        off = int(rng.integers(0, pool.shape[0] - size + 1))
        iters = {0: None, 1: None, 2: 12, 3: None}[cfg]
        reqs.append((cfg, _prm(w, iters), np.ascontiguousarray(pool[off:off + size])))
    return reqs


def _alone(cfg, prm, llr):
    hard, ok, it, _ = L.decode(_code(cfg), prm, torch.from_numpy(llr).to(DEV))
    torch.cuda.synchronize()
    return hard.cpu().numpy(), ok.cpu().numpy(), it.cpu().numpy()


@pytest.mark.parametrize("mode,budget,inflight,cap", [
    ("continuous", 256 << 20, 4, 0),
    ("continuous", 160 << 20, 3, 96),  # small budget and launch cap: requests are split across launches
    ("per_request", 256 << 20, 1, 0),
])
def test_results_alone_and_in_mix(mode, budget, inflight, cap):
    reqs = _requests(36, seed=5)
    with L.Server(hbm_budget=budget, max_inflight=inflight, mode=mode, max_launch_cw=cap) as srv:
        tickets = [srv.submit(_code(cfg), prm, llr) for cfg, prm, llr in reqs]
        outs = [srv.wait(t, timeout_ms=120000) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["codewords"] == sum(llr.shape[0] for _, _, llr in reqs)
    assert st["peak_bytes"] <= budget
    if cap:
        assert st["launches"] > 1
    for (cfg, prm, llr), (hard, ok, it, (ts, ta, td)) in zip(reqs, outs):
        h2, ok2, it2 = _alone(cfg, prm, llr)
        assert (hard == h2).all() and (ok == ok2).all() and (it == it2).all()
        assert ts <= ta <= td


def test_mix_matches_oracle():
    reqs = [r for r in _requests(12, seed=9, max_size=40) if r[0] != 2]
    with L.Server(hbm_budget=64 << 20, max_inflight=2) as srv:
        tickets = [srv.submit(_code(cfg), prm, llr) for cfg, prm, llr in reqs]
        outs = [srv.wait(t, timeout_ms=120000) for t in tickets]
    for (cfg, prm, llr), (hard, ok, it, _) in zip(reqs, outs):
        w = S.workload(cfg)
        d = dict(rule=w.rule, schedule=w.schedule, max_iters=prm.max_iters, early_stop=True, nms_num=w.nms_num,
                 nms_shift=w.nms_shift, oms_offset=w.oms_offset, msg_max=w.msg_max)
        ref = (O.decode_binary if w.code.g == 2 else O.decode_nb)(w.code, O.params(**d), llr)
        hh = L.unpack_bits(hard, w.code.n) if w.code.g == 2 else hard
        assert (hh == ref["hard"]).all() and (ok == ref["ok"]).all() and (it == ref["iters"]).all()


def test_cancel_and_zero_batch():
    w3, pool3 = _pool(3, 512)
    w0, pool0 = _pool(0, 512)
    with L.Server(hbm_budget=64 << 20, max_inflight=2, max_launch_cw=64) as srv:
        big = srv.submit(_code(3), _prm(w3), np.ascontiguousarray(pool3[:512]))
        small = srv.submit(_code(0), _prm(w0), np.ascontiguousarray(pool0[:10]))
        empty = srv.submit(_code(0), _prm(w0), np.ascontiguousarray(pool0[:0]))
        srv.cancel(big)
        with pytest.raises(L.LdpcxError) as ei:
            srv.wait(big, timeout_ms=60000)
        assert ei.value.status == L.E_CANCELLED
        hard, ok, it, _ = srv.wait(small, timeout_ms=60000)
        h2, ok2, it2 = _alone(0, _prm(w0), np.ascontiguousarray(pool0[:10]))
        assert (hard == h2).all() and (it == it2).all()
        hard, ok, it, (ts, ta, td) = srv.wait(empty, timeout_ms=1000)
        assert hard.shape[0] == 0
        with pytest.raises(L.LdpcxError) as ei:
            srv.poll(small)  # released by wait
        assert ei.value.status == L.E_NOTFOUND


def test_budget_rejection():
    w0, pool0 = _pool(0, 512)
    with L.Server(hbm_budget=512, max_inflight=1) as srv:
        with pytest.raises(L.LdpcxError) as ei:
            srv.submit(_code(0), _prm(w0), np.ascontiguousarray(pool0[:1]))
        assert ei.value.status == L.E_BUDGET


@pytest.mark.parametrize("mode,budget", [("continuous", 256 << 20), ("continuous", 4 << 20), ("per_request", 256 << 20)])
def test_layered_minmax_requests(mode, budget):
    """Min-Max requests of either schedule and any size join the ragged launches as
    one-codeword items (split across launches when the budget is small; launches of
    their own in per-request mode); each result equals a plain decode of the request
    alone."""
    w3, pool3 = _pool(3, 512)
    w0, pool0 = _pool(0, 512)
    lay = L.params("minmax", "layered", 8, True)
    reqs = [(3, lay, np.ascontiguousarray(pool3[:100])), (0, _prm(w0), np.ascontiguousarray(pool0[:30])),
            (3, lay, np.ascontiguousarray(pool3[100:103])), (3, _prm(w3, 8), np.ascontiguousarray(pool3[200:240])),
            (3, _prm(w3, 6), np.ascontiguousarray(pool3[:512])), (3, lay, np.ascontiguousarray(pool3[:300]))]
    with L.Server(hbm_budget=budget, max_inflight=3, mode=mode) as srv:
        tickets = [srv.submit(_code(cfg), prm, llr) for cfg, prm, llr in reqs]
        outs = [srv.wait(t, timeout_ms=120000) for t in tickets]
        st = srv.stats()
    assert st["peak_bytes"] <= budget
    if budget < (8 << 20):
        assert st["launches"] >= 3  # 812 Min-Max codewords of 24 KB input each
    for (cfg, prm, llr), (hard, ok, it, _) in zip(reqs, outs):
        h2, ok2, it2 = _alone(cfg, prm, llr)
        assert (hard == h2).all() and (ok == ok2).all() and (it == it2).all()


@pytest.mark.parametrize("mode,fail_at", [("per_request", 3), ("continuous", 2)])
def test_failed_launch_fails_only_its_requests(mode, fail_at, monkeypatch):
    """LDPCX_FAULT_INJECT=launch:N makes the server's N-th launch report a device error
    without touching the device: exactly the requests of that launch fail with
    LDPCX_E_DEVICE, and every request before and after it still completes with what a
    plain decode of it alone gives (the server keeps serving)."""
    monkeypatch.setenv("LDPCX_FAULT_INJECT", f"launch:{fail_at}")
    reqs = [r for r in _requests(10, seed=21, max_size=60) if r[0] != 2][:6]
    results = []
    with L.Server(hbm_budget=256 << 20, max_inflight=2, mode=mode) as srv:
        for cfg, prm, llr in reqs:  # one request in flight at a time: launch k decodes request k
            t = srv.submit(_code(cfg), prm, llr)
            try:
                results.append(srv.wait(t, timeout_ms=120000))
            except L.LdpcxError as ex:
                results.append(ex.status)
        st = srv.stats()
    for k, ((cfg, prm, llr), res) in enumerate(zip(reqs, results), start=1):
        if k == fail_at:
            assert res == L.E_DEVICE, f"request {k} should have failed"
            continue
        hard, ok, it, _ = res
        h2, ok2, it2 = _alone(cfg, prm, llr)
        assert (hard == h2).all() and (ok == ok2).all() and (it == it2).all()
    assert st["completed"] == len(reqs) - 1
    assert st["launches"] == len(reqs)


def test_chunks_run_the_plan_of_their_size():
    """A request whose chunks fall in different batch classes runs each chunk on the plan
    of its own size (here pinned differently per class), charges that plan's memory and
    still gives what a plain decode gives."""
    w1, pool1 = _pool(1, 512)
    h = L.Code(w1.code)
    prm = _prm(w1, 6)
    L.plan_set(h, prm, 512, "bin_qc_packed", 2)      # the class of the whole request
    L.plan_set(h, prm, 64, "bin_lds", 2, 256)         # the class of its 64-codeword chunks
    llr = np.ascontiguousarray(pool1[:300])
    with L.Server(hbm_budget=256 << 20, max_inflight=2, max_launch_cw=64) as srv:
        hard, ok, it, _ = srv.wait(srv.submit(h, prm, llr), timeout_ms=120000)
        assert srv.stats()["launches"] >= 5
    ref = L.decode(h, prm, torch.from_numpy(llr).to(DEV))
    torch.cuda.synchronize()
    assert (hard == ref[0].cpu().numpy()).all() and (ok == ref[1].cpu().numpy()).all()
    assert (it == ref[2].cpu().numpy()).all()
