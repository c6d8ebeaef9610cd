"""CPU oracle for the batched LDPC decoders -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``ldpc_oracle.c`` (plain C, OpenMP over codewords
only).  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product library never does.  It shares
no code with the GPU path: it builds its own GF(2^p) arithmetic by polynomial
multiplication and decodes with naive loops (see the C file's header for the
exact readings it implements).

Codes are passed duck-typed: any object with ``g, prim_poly, n, m, row_ptr,
col_idx, h_val`` attributes (CSR by check, ascending columns).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldpc_oracle.c")
_SO = os.path.join(_HERE, "libldpc_oracle.so")

RULES = {"ms": 0, "nms": 1, "oms": 2, "minmax": 3, "spa": 4}
SCHEDULES = {"flooding": 0, "layered": 1}


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.orc_gf_mul.restype = ctypes.c_int
        L.orc_gf_mul.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int]
        L.orc_gf_inv.restype = ctypes.c_int
        L.orc_gf_inv.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int]
        L.orc_gf_permute.restype = None
        L.orc_gf_permute.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, i32p, i32p]
        L.orc_syndrome_ok.restype = ctypes.c_int
        L.orc_binary_cn.restype = None
        L.orc_minmax_cn.restype = None
        L.orc_decode_binary.restype = ctypes.c_int
        L.orc_decode_nb.restype = ctypes.c_int
        L.orc_nb_layers.restype = ctypes.c_int
        L.orc_spa_weight.restype = ctypes.c_int
        L.orc_spa_weight.argtypes = [ctypes.c_int]
        L.orc_wht.restype = None
        L.orc_wht.argtypes = [ctypes.c_int, i32p, i32p]
        L.orc_spa_cn.restype = None
        L.orc_spa_qmul.restype = ctypes.c_int32
        L.orc_spa_qmul.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.orc_spa_norm.restype = ctypes.c_int
        L.orc_spa_norm.argtypes = [ctypes.c_int, i32p, i32p]
        L.orc_decode_spa.restype = ctypes.c_int
        _lib = L
    return _lib


class Params(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("early_stop", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("nms_num", ctypes.c_int32), ("nms_shift", ctypes.c_int32),
                ("oms_offset", ctypes.c_int32), ("msg_max", ctypes.c_int32),
                ("nb_msg_max", ctypes.c_int32)]


def params(rule="nms", schedule="flooding", max_iters=10, early_stop=True, nms_num=3,
           nms_shift=2, oms_offset=1, msg_max=127, nb_msg_max=0) -> Params:
    return Params(max_iters, int(bool(early_stop)), SCHEDULES[schedule], RULES[rule], nms_num,
                  nms_shift, oms_offset, msg_max, nb_msg_max)


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _nthreads(nthreads):
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return int(nthreads)


# ----------------------------------------------------------------- GF helpers
def gf_mul(g: int, poly: int, a: int, b: int) -> int:
    return lib().orc_gf_mul(g, poly, int(a), int(b))


def gf_inv(g: int, poly: int, a: int) -> int:
    return lib().orc_gf_inv(g, poly, int(a))


def gf_permute(g: int, poly: int, h: int, v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.int32)
    out = np.empty(g, dtype=np.int32)
    lib().orc_gf_permute(g, poly, int(h), _p(v, ctypes.c_int32), _p(out, ctypes.c_int32))
    return out


def syndrome_ok(code, symbols: np.ndarray) -> bool:
    c = np.ascontiguousarray(symbols, dtype=np.uint8)
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    hv = None if code.h_val is None else np.ascontiguousarray(code.h_val, dtype=np.uint8)
    return bool(lib().orc_syndrome_ok(
        ctypes.c_int(code.g), ctypes.c_uint32(code.prim_poly), ctypes.c_int(code.m),
        _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32),
        None if hv is None else _p(hv, ctypes.c_uint8), _p(c, ctypes.c_uint8)))


# ------------------------------------------------------------ check-node rules
def binary_cn(q: np.ndarray, prm: Params) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.int32)
    r = np.empty_like(q)
    lib().orc_binary_cn(ctypes.c_int(len(q)), _p(q, ctypes.c_int32), _p(r, ctypes.c_int32), ctypes.byref(prm))
    return r


def minmax_cn(g: int, poly: int, h: np.ndarray, alpha: np.ndarray):
    """beta [dc][g] from alpha [dc][g]; also returns (F&B pairs, middle-beta pairs)."""
    h = np.ascontiguousarray(h, dtype=np.uint8)
    a = np.ascontiguousarray(alpha, dtype=np.int32)
    dc = len(h)
    beta = np.empty((dc, g), dtype=np.int32)
    pfb, pb = ctypes.c_int64(0), ctypes.c_int64(0)
    lib().orc_minmax_cn(ctypes.c_int(g), ctypes.c_uint32(poly), ctypes.c_int(dc), _p(h, ctypes.c_uint8),
                        _p(a, ctypes.c_int32), _p(beta, ctypes.c_int32), ctypes.byref(pfb), ctypes.byref(pb))
    return beta, pfb.value, pb.value


def nb_layers(code) -> np.ndarray:
    """Layer index of every check for the layered Min-Max schedule (greedy colouring in
    ascending check order: the lowest layer holding no check that shares a variable)."""
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    out = np.empty(code.m, dtype=np.int32)
    lib().orc_nb_layers(ctypes.c_int(code.m), _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32),
                        _p(out, ctypes.c_int32))
    return out


# ------------------------------------------------------------------- decoders
def decode_binary(code, prm: Params, llr: np.ndarray, dump: bool = False, nthreads=None) -> dict:
    """llr int8 [B, n] -> dict(hard [B, n] u8, ok [B] u8, iters [B] i16, and q/r/lam dumps)."""
    llr = np.ascontiguousarray(llr, dtype=np.int8)
    B, n = llr.shape
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    E = int(rp[-1])
    hard = np.empty((B, n), dtype=np.uint8)
    ok = np.empty(B, dtype=np.uint8)
    it = np.empty(B, dtype=np.int16)
    dq = np.empty((B, E), dtype=np.int32) if dump else None
    dr = np.empty((B, E), dtype=np.int32) if dump else None
    dl = np.empty((B, n), dtype=np.int32) if dump else None
    rc = lib().orc_decode_binary(
        ctypes.c_int(n), ctypes.c_int(code.m), _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32),
        ctypes.byref(prm), ctypes.c_int(B), _p(llr, ctypes.c_int8), _p(hard, ctypes.c_uint8),
        _p(ok, ctypes.c_uint8), _p(it, ctypes.c_int16),
        None if dq is None else _p(dq, ctypes.c_int32), None if dr is None else _p(dr, ctypes.c_int32),
        None if dl is None else _p(dl, ctypes.c_int32), ctypes.c_int(_nthreads(nthreads)))
    if rc == -2:
        raise ValueError("oracle: the fixed-point FFT-SPA covers fields up to GF(256)")
    if rc != 0:
        raise ValueError("oracle: every check must have degree >= 2")
    out = dict(hard=hard, ok=ok, iters=it)
    if dump:
        out.update(q=dq, r=dr, lam=dl)
    return out


def decode_nb(code, prm: Params, gamma: np.ndarray, dump: bool = False, nthreads=None) -> dict:
    """gamma int16 [B, n, g] -> dict(hard, ok, iters, pairs, and alpha/beta dumps [B, E, g]).

    Schedule "flooding" is the two-phase Alg. 2; "layered" processes one check at a time
    in the order of nb_layers (alpha of eq. (14) formed from the current betas)."""
    gamma = np.ascontiguousarray(gamma, dtype=np.int16)
    B, n, g = gamma.shape
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    hv = np.ascontiguousarray(code.h_val if code.h_val is not None else np.ones(len(ci)), dtype=np.uint8)
    E = int(rp[-1])
    hard = np.empty((B, n), dtype=np.uint8)
    ok = np.empty(B, dtype=np.uint8)
    it = np.empty(B, dtype=np.int16)
    da = np.empty((B, E, g), dtype=np.int32) if dump else None
    db = np.empty((B, E, g), dtype=np.int32) if dump else None
    pairs = np.zeros(2, dtype=np.int64)
    rc = lib().orc_decode_nb(
        ctypes.c_int(g), ctypes.c_uint32(code.prim_poly), ctypes.c_int(n), ctypes.c_int(code.m),
        _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32), _p(hv, ctypes.c_uint8), ctypes.byref(prm),
        ctypes.c_int(B), _p(gamma, ctypes.c_int16), _p(hard, ctypes.c_uint8), _p(ok, ctypes.c_uint8),
        _p(it, ctypes.c_int16), None if da is None else _p(da, ctypes.c_int32),
        None if db is None else _p(db, ctypes.c_int32), _p(pairs, ctypes.c_int64),
        ctypes.c_int(_nthreads(nthreads)))
    if rc != 0:
        raise ValueError("oracle: every check must have degree >= 2")
    out = dict(hard=hard, ok=ok, iters=it, pairs=pairs)
    if dump:
        out.update(alpha=da, beta=db)
    return out


# ------------------------------------------------------------ fixed-point FFT-SPA
def spa_weight(c: int) -> int:
    """round(2^24 exp(-c / 4)): channel weight of a symbol with cost c."""
    return lib().orc_spa_weight(int(c))


def spa_qmul(a: int, b: int) -> int:
    """Product of two Q24 numbers as the fixed-point FFT-SPA takes it."""
    return int(lib().orc_spa_qmul(int(a), int(b)))


def spa_norm(z) -> Optional[np.ndarray]:
    """Normalisation of a non-negative vector to a Q24 distribution (None when sum z = 0)."""
    z = np.ascontiguousarray(z, dtype=np.int32)
    out = np.empty_like(z)
    ok = lib().orc_spa_norm(ctypes.c_int(len(z)), _p(z, ctypes.c_int32), _p(out, ctypes.c_int32))
    return out if ok else None


def wht(x) -> np.ndarray:
    """Walsh-Hadamard transform of an integer vector (length g)."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    out = np.empty_like(x)
    lib().orc_wht(ctypes.c_int(len(x)), _p(x, ctypes.c_int32), _p(out, ctypes.c_int32))
    return out


def spa_cn(g: int, poly: int, h, u) -> np.ndarray:
    """Check node of the fixed-point FFT-SPA: u int [dc, g] (Q24) -> v' [dc, g]."""
    h = np.ascontiguousarray(h, dtype=np.uint8)
    u = np.ascontiguousarray(u, dtype=np.int32)
    dc = len(h)
    v = np.empty((dc, g), dtype=np.int32)
    lib().orc_spa_cn(ctypes.c_int(g), ctypes.c_uint32(poly), ctypes.c_int(dc), _p(h, ctypes.c_uint8),
                     _p(u, ctypes.c_int32), _p(v, ctypes.c_int32))
    return v


def decode_spa(code, prm: Params, gamma: np.ndarray, dump: bool = False, nthreads=None) -> dict:
    """gamma int16 [B, n, g], g <= 256 -> dict(hard, ok, iters, and u/v dumps [B, E, g] in Q24)."""
    gamma = np.ascontiguousarray(gamma, dtype=np.int16)
    B, n, g = gamma.shape
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    hv = np.ascontiguousarray(code.h_val if code.h_val is not None else np.ones(len(ci)), dtype=np.uint8)
    E = int(rp[-1])
    hard = np.empty((B, n), dtype=np.uint8)
    ok = np.empty(B, dtype=np.uint8)
    it = np.empty(B, dtype=np.int16)
    du = np.empty((B, E, g), dtype=np.int32) if dump else None
    dv = np.empty((B, E, g), dtype=np.int32) if dump else None
    rc = lib().orc_decode_spa(
        ctypes.c_int(g), ctypes.c_uint32(code.prim_poly), ctypes.c_int(n), ctypes.c_int(code.m),
        _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32), _p(hv, ctypes.c_uint8), ctypes.byref(prm),
        ctypes.c_int(B), _p(gamma, ctypes.c_int16), _p(hard, ctypes.c_uint8), _p(ok, ctypes.c_uint8),
        _p(it, ctypes.c_int16), None if du is None else _p(du, ctypes.c_int32),
        None if dv is None else _p(dv, ctypes.c_int32), ctypes.c_int(_nthreads(nthreads)))
    if rc == -2:
        raise ValueError("oracle: the fixed-point FFT-SPA covers fields up to GF(256)")
    if rc != 0:
        raise ValueError("oracle: every check must have degree >= 2")
    out = dict(hard=hard, ok=ok, iters=it)
    if dump:
        out.update(u=du, v=dv)
    return out
