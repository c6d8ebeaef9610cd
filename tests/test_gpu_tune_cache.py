"""Persisted autotuning: with LDPCX_TUNE_CACHE naming a file, ldpcx_tune merges its choice
into that file and every code handle created afterwards loads the entries of its code and
device, so a new process need not tune again."""
import json

import numpy as np
import pytest
import torch

import oracle as O
from paper_2508_03567_amd import ldpcx as L
from paper_2508_03567_amd import synth as S

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_tuned_plan_persists_and_loads(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("LDPCX_TUNE_CACHE", str(path))
    w = S.workload(0, batch=1000)
    prm = L.params(w.rule, w.schedule, 6, early_stop=True)
    h = L.Code(w.code)
    L.tune(h, prm, w.batch)
    tuned = L.plan_info(h, prm, w.batch)
    entries = json.loads(path.read_text())
    assert len(entries) == 1 and entries[0]["cw_per_wg"] == tuned["cw_per_wg"]
    # tuning another batch class adds an entry, re-tuning the same one replaces it
    L.tune(h, prm, 40)
    L.tune(h, prm, w.batch)
    assert len(json.loads(path.read_text())) == 2
    # a new handle of the same code loads the stored choice: edit it to a plan the tuner
    # would not pick by itself and check that the new handle reports exactly that plan
    for e in entries:
        e.update(family=0, cw_per_wg=3, threads=192)
    path.write_text(json.dumps(entries, indent=1))  # reformatted: the loader reads any layout
    h2 = L.Code(w.code)
    assert L.plan_info(h2, prm, w.batch) == dict(family="bin_lds", cw_per_wg=3, threads=192)
    cw, llr = S.make_inputs(w)
    hard, ok, it, _ = L.decode(h2, prm, torch.from_numpy(llr).to(DEV))
    torch.cuda.synchronize()
    ref = O.decode_binary(w.code, O.params(w.rule, w.schedule, 6, True), llr)
    assert (L.unpack_bits(hard.cpu().numpy(), w.code.n) == ref["hard"]).all()
    assert (it.cpu().numpy() == ref["iters"]).all() and (ok.cpu().numpy() == ref["ok"]).all()
    # another code does not pick up this code's entries
    other = L.Code(S.workload(1).code)
    assert L.plan_info(other, prm, w.batch)["family"] == "bin_qc_packed"
    # without the variable nothing is loaded
    monkeypatch.delenv("LDPCX_TUNE_CACHE")
    h3 = L.Code(w.code)
    assert L.plan_info(h3, prm, w.batch) != dict(family="bin_lds", cw_per_wg=3, threads=192)
