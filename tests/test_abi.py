"""The C-ABI library: it loads, exports every symbol include/ldpcx.h declares, and
rejects malformed codes on the host (no GPU needed for these paths)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2508_03567_amd import ldpcx as L
from paper_2508_03567_amd import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ldpcx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ldpcx_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = L.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTED)


def test_version_and_no_error_initially():
    assert "gfx950" in L.ldpcx_version()


def _desc(code, **over):
    d = dict(g=code.g, prim_poly=code.prim_poly, n=code.n, m=code.m, z=code.z)
    d.update(over)
    rp = np.ascontiguousarray(over.pop("row_ptr", code.row_ptr), dtype=np.int32)
    ci = np.ascontiguousarray(over.pop("col_idx", code.col_idx), dtype=np.int32)
    hv = code.h_val if "h_val" not in over else over["h_val"]
    hv = None if hv is None else np.ascontiguousarray(hv, dtype=np.uint8)
    keep = (rp, ci, hv)
    desc = L.CodeDesc(d["g"], d["prim_poly"], d["n"], d["m"],
                      rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      None if hv is None else hv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), d["z"],
                      code.n - code.m)
    return desc, keep


def _expect(desc, status):
    with pytest.raises(L.LdpcxError) as ei:
        L.ldpcx_code_create(desc)
    assert ei.value.status == status


def test_validation_rejects_malformed_codes():
    c0 = S.workload(0).code
    c3 = S.workload(3).code
    # unsorted columns
    ci = c0.col_idx.copy()
    ci[0], ci[1] = ci[1], ci[0]
    d, k = _desc(c0, col_idx=ci)
    _expect(d, L.E_INVAL)
    # column out of range
    ci = c0.col_idx.copy()
    ci[5] = c0.n
    d, k = _desc(c0, col_idx=ci)
    _expect(d, L.E_INVAL)
    # a layer whose rows share a column
    d, k = _desc(c0, z=96)
    _expect(d, L.E_INVAL)
    # layer size not dividing m
    d, k = _desc(c0, z=7)
    _expect(d, L.E_INVAL)
    # zero GF coefficient
    hv = c3.h_val.copy()
    hv[3] = 0
    d, k = _desc(c3, h_val=hv)
    _expect(d, L.E_INVAL)
    # non-primitive polynomial for GF(64): x^6 + 1 is reducible
    d, k = _desc(c3, prim_poly=0x41)
    _expect(d, L.E_INVAL)
    # field size not a power of two
    d, k = _desc(c3, g=48)
    _expect(d, L.E_INVAL)
    # check degree 1
    code1 = S.code_from_pairs("d1", 2, 3, 4, 2, [0, 1, 1], [0, 1, 2])
    d, k = _desc(code1)
    _expect(d, L.E_INVAL)
    # check degree above the binary limit
    code15 = S.code_from_pairs("d15", 2, 3, 20, 1, [0] * 15, list(range(15)))
    d, k = _desc(code15)
    _expect(d, L.E_UNSUPPORTED)
    assert L.ldpcx_last_error() != ""


def test_server_config_validation():
    """Bad server configurations are rejected on the host before any device call."""
    for cfg in (L.ServerConfig(0, 2, 0, 0), L.ServerConfig(1 << 20, 0, 0, 0), L.ServerConfig(1 << 20, 2, 7, 0),
                L.ServerConfig(1 << 20, 2, 0, -1), L.ServerConfig(1 << 20, 65, 0, 0)):
        with pytest.raises(L.LdpcxError) as ei:
            L.ldpcx_server_create(cfg)
        assert ei.value.status == L.E_INVAL
    for fn, args in ((L.lib().ldpcx_server_poll, (None, 1, None)), (L.lib().ldpcx_server_cancel, (None, 1)),
                     (L.lib().ldpcx_server_destroy, (None,)), (L.lib().ldpcx_decode_ragged, (None, -1, None))):
        assert fn(*args) == L.E_INVAL


def test_valu_probe_validation():
    """The measurement probe rejects non-positive sizes on the host."""
    for blocks, iters in ((0, 1), (1, 0), (-3, 5)):
        with pytest.raises(L.LdpcxError) as ei:
            L.ldpcx_valu_probe(blocks, iters)
        assert ei.value.status == L.E_INVAL
