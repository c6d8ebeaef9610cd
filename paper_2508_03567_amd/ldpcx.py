"""Thin ctypes binding of libldpcx (include/ldpcx.h).

Argument marshalling only: every decoding step runs in the HIP library.  The
functions named ``ldpcx_*`` mirror the C entry points one to one and take raw
integers (device pointers, stream handles); the small helpers below them
(`Code`, `params`, `decode`, ...) only allocate torch tensors for the outputs
and pass their data pointers.  If the library is not built, importing this
module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldpcx.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_BUDGET, E_CANCELLED, E_TIMEOUT, E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7, -8
SCHED = {"flooding": 0, "layered": 1, "auto": 2}
SCHED_NAME = {v: k for k, v in SCHED.items()}
RULE = {"ms": 0, "nms": 1, "oms": 2, "minmax": 3, "spa": 4}
FAMILY_NAME = {0: "bin_lds", 1: "bin_interleaved", 2: "minmax_interleaved", 3: "bin_qc_packed", 4: "spa_wave",
               5: "minmax_lds", 6: "spa_lds", 7: "minmax_cw"}


class LdpcxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ldpcx status {status}: {msg}")
        self.status = status


class CodeDesc(ctypes.Structure):
    _fields_ = [("g", ctypes.c_int32), ("prim_poly", ctypes.c_uint32), ("n", ctypes.c_int32),
                ("m", ctypes.c_int32), ("row_ptr", ctypes.POINTER(ctypes.c_int32)),
                ("col_idx", ctypes.POINTER(ctypes.c_int32)), ("h_val", ctypes.POINTER(ctypes.c_uint8)),
                ("z", ctypes.c_int32), ("k_info", ctypes.c_int32)]


class DecodeParams(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("early_stop", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("nms_num", ctypes.c_int32), ("nms_shift", ctypes.c_int32),
                ("oms_offset", ctypes.c_int32), ("msg_max", ctypes.c_int32), ("nb_msg_max", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("max_launch_cw", ctypes.c_int32)]


SERVE = {"continuous": 0, "per_request": 1}


class Job(ctypes.Structure):
    _fields_ = [("code", ctypes.c_void_p), ("params", DecodeParams), ("batch", ctypes.c_int32),
                ("llr", ctypes.c_void_p), ("hard", ctypes.c_void_p), ("syndrome_ok", ctypes.c_void_p),
                ("iters", ctypes.c_void_p)]


_lib = None

_SIGS = {
    "ldpcx_code_create": [ctypes.POINTER(CodeDesc), ctypes.POINTER(ctypes.c_void_p)],
    "ldpcx_code_destroy": [ctypes.c_void_p],
    "ldpcx_code_info": [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int32)] * 6,
    "ldpcx_decode": [ctypes.c_void_p, ctypes.POINTER(DecodeParams), ctypes.c_int32, ctypes.c_void_p,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                     ctypes.c_void_p],
    "ldpcx_debug_dump": [ctypes.c_void_p, ctypes.POINTER(DecodeParams), ctypes.c_int32] + [ctypes.c_void_p] * 8,
    "ldpcx_decode_noalloc": [ctypes.c_void_p, ctypes.POINTER(DecodeParams), ctypes.c_int32, ctypes.c_void_p,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                             ctypes.c_void_p],
    "ldpcx_decode_ragged": [ctypes.POINTER(Job), ctypes.c_int32, ctypes.c_void_p],
    "ldpcx_tune": [ctypes.c_void_p, ctypes.POINTER(DecodeParams), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                   ctypes.POINTER(ctypes.c_float), ctypes.c_void_p],
    "ldpcx_plan_info": [ctypes.c_void_p, ctypes.POINTER(DecodeParams), ctypes.c_int32] +
                       [ctypes.POINTER(ctypes.c_int32)] * 3,
    "ldpcx_plan_set": [ctypes.c_void_p, ctypes.POINTER(DecodeParams), ctypes.c_int32, ctypes.c_int32,
                       ctypes.c_int32, ctypes.c_int32],
    "ldpcx_valu_probe": [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p],
    "ldpcx_server_create": [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)],
    "ldpcx_server_submit": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(DecodeParams), ctypes.c_int32,
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.POINTER(ctypes.c_uint64)],
    "ldpcx_server_poll": [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)],
    "ldpcx_server_wait": [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32] + [ctypes.POINTER(ctypes.c_double)] * 3,
    "ldpcx_server_cancel": [ctypes.c_void_p, ctypes.c_uint64],
    "ldpcx_server_stats": [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_uint64)] * 4,
    "ldpcx_server_destroy": [ctypes.c_void_p],
    "ldpcx_last_error": [],
    "ldpcx_version": [],
}

EXPORTED = tuple(_SIGS)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        # PyTorch ships its own HIP runtime under the same soname as the system one the
        # library links; loading torch first makes the whole process use torch's copy
        # (a second copy loaded first leaves torch without devices).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name in ("ldpcx_last_error", "ldpcx_version") else ctypes.c_int
        _lib = L
    return _lib


def _check(st: int) -> None:
    if st != OK:
        raise LdpcxError(st, lib().ldpcx_last_error().decode())


# ---------------------------------------------------------------- raw entry points
def ldpcx_version() -> str:
    return lib().ldpcx_version().decode()


def ldpcx_last_error() -> str:
    return lib().ldpcx_last_error().decode()


def ldpcx_code_create(desc: CodeDesc) -> int:
    h = ctypes.c_void_p()
    _check(lib().ldpcx_code_create(ctypes.byref(desc), ctypes.byref(h)))
    return h.value


def ldpcx_code_destroy(code: int) -> None:
    _check(lib().ldpcx_code_destroy(code))


def ldpcx_code_info(code: int) -> dict:
    vals = [ctypes.c_int32() for _ in range(6)]
    _check(lib().ldpcx_code_info(code, *[ctypes.byref(v) for v in vals]))
    return dict(zip(("n", "m", "nnz", "g", "max_dc", "max_dv"), (v.value for v in vals)))


def ldpcx_decode(code: int, prm: DecodeParams, batch: int, llr: int, hard: int, syndrome_ok: int, iters: int,
                 stream: int = 0) -> int:
    used = ctypes.c_int32(-1)
    _check(lib().ldpcx_decode(code, ctypes.byref(prm), batch, llr, hard, syndrome_ok, iters, ctypes.byref(used),
                              stream))
    return used.value


def ldpcx_decode_noalloc(code: int, prm: DecodeParams, batch: int, llr: int, hard: int, syndrome_ok: int,
                         iters: int, stream: int = 0) -> int:
    used = ctypes.c_int32(-1)
    _check(lib().ldpcx_decode_noalloc(code, ctypes.byref(prm), batch, llr, hard, syndrome_ok, iters,
                                      ctypes.byref(used), stream))
    return used.value


def ldpcx_debug_dump(code: int, prm: DecodeParams, batch: int, llr: int, hard: int, syndrome_ok: int, iters: int,
                     msg_a: int, msg_b: int, msg_c: int, stream: int = 0) -> None:
    _check(lib().ldpcx_debug_dump(code, ctypes.byref(prm), batch, llr, hard, syndrome_ok, iters, msg_a, msg_b,
                                  msg_c, stream))


def ldpcx_decode_ragged(jobs, stream: int = 0) -> None:
    arr = (Job * len(jobs))(*jobs)
    _check(lib().ldpcx_decode_ragged(arr, len(jobs), stream))


def ldpcx_tune(code: int, prm: DecodeParams, batch: int, stream: int = 0):
    sched = ctypes.c_int32(-1)
    us = ctypes.c_float(0)
    _check(lib().ldpcx_tune(code, ctypes.byref(prm), batch, ctypes.byref(sched), ctypes.byref(us), stream))
    return sched.value, us.value


def ldpcx_plan_info(code: int, prm: DecodeParams, batch: int) -> dict:
    vals = [ctypes.c_int32() for _ in range(3)]
    _check(lib().ldpcx_plan_info(code, ctypes.byref(prm), batch, *[ctypes.byref(v) for v in vals]))
    return dict(family=FAMILY_NAME[vals[0].value], cw_per_wg=vals[1].value, threads=vals[2].value)


def ldpcx_plan_set(code: int, prm: DecodeParams, batch: int, family: int, cw_per_wg: int = 1,
                   threads: int = 256) -> None:
    _check(lib().ldpcx_plan_set(code, ctypes.byref(prm), batch, family, cw_per_wg, threads))


def ldpcx_server_create(cfg: ServerConfig) -> int:
    h = ctypes.c_void_p()
    _check(lib().ldpcx_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def ldpcx_server_submit(srv: int, code: int, prm: DecodeParams, batch: int, llr: int, hard: int, ok: int,
                        iters: int) -> int:
    t = ctypes.c_uint64()
    _check(lib().ldpcx_server_submit(srv, code, ctypes.byref(prm), batch, llr, hard, ok, iters, ctypes.byref(t)))
    return t.value


def ldpcx_server_poll(srv: int, ticket: int) -> bool:
    d = ctypes.c_int32()
    _check(lib().ldpcx_server_poll(srv, ticket, ctypes.byref(d)))
    return bool(d.value)


def ldpcx_server_wait(srv: int, ticket: int, timeout_ms: int = -1):
    ts, ta, td = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = lib().ldpcx_server_wait(srv, ticket, timeout_ms, ctypes.byref(ts), ctypes.byref(ta), ctypes.byref(td))
    return st, ts.value, ta.value, td.value


def ldpcx_server_cancel(srv: int, ticket: int) -> None:
    _check(lib().ldpcx_server_cancel(srv, ticket))


def ldpcx_server_stats(srv: int) -> dict:
    vals = [ctypes.c_uint64() for _ in range(4)]
    _check(lib().ldpcx_server_stats(srv, *[ctypes.byref(v) for v in vals]))
    return dict(zip(("completed", "codewords", "launches", "peak_bytes"), (v.value for v in vals)))


def ldpcx_server_destroy(srv: int) -> None:
    _check(lib().ldpcx_server_destroy(srv))


# ---------------------------------------------------------------- convenience
def params(rule="nms", schedule="flooding", max_iters=10, early_stop=True, nms_num=3, nms_shift=2, oms_offset=1,
           msg_max=127, nb_msg_max=0) -> DecodeParams:
    return DecodeParams(int(max_iters), int(bool(early_stop)), SCHED[schedule], RULE[rule], nms_num, nms_shift,
                        oms_offset, msg_max, nb_msg_max)


class Code:
    """Device code handle built from any object with g, prim_poly, n, m, row_ptr, col_idx, h_val, z."""

    def __init__(self, code):
        self.g, self.n, self.m = int(code.g), int(code.n), int(code.m)
        self._rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
        self._ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
        self.nnz = int(self._rp[-1])
        self._hv = None if code.h_val is None else np.ascontiguousarray(code.h_val, dtype=np.uint8)
        desc = CodeDesc(self.g, int(code.prim_poly), self.n, self.m,
                        self._rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        self._ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        None if self._hv is None else self._hv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                        int(getattr(code, "z", 0) or 0), int(getattr(code, "k_info", self.n - self.m)))
        self.handle = ldpcx_code_create(desc)

    def close(self):
        if getattr(self, "handle", None):
            ldpcx_code_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hard_shape(self, batch):
        return (batch, (self.n + 7) // 8) if self.g == 2 else (batch, self.n)


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _outputs(code: Code, batch: int, device):
    import torch
    hard = torch.empty(code.hard_shape(batch), dtype=torch.uint8, device=device)
    ok = torch.empty(batch, dtype=torch.uint8, device=device)
    it = torch.empty(batch, dtype=torch.int16, device=device)
    return hard, ok, it


def _check_llr(code: Code, llr) -> None:
    import torch
    want = torch.int8 if code.g == 2 else torch.int16
    shape = (code.n,) if code.g == 2 else (code.n, code.g)
    if llr.dtype != want or not llr.is_contiguous() or tuple(llr.shape[1:]) != shape:
        raise ValueError(f"llr must be a contiguous {want} tensor of shape [B, {', '.join(map(str, shape))}]")


def decode(code: Code, prm: DecodeParams, llr, stream=None, out=None):
    """llr: device tensor int8 [B, n] (g == 2) or int16 [B, n, g].  Returns (hard, ok, iters, schedule)."""
    _check_llr(code, llr)
    batch = int(llr.shape[0])
    hard, ok, it = out if out is not None else _outputs(code, batch, llr.device)
    used = ldpcx_decode(code.handle, prm, batch, llr.data_ptr(), hard.data_ptr(), ok.data_ptr(), it.data_ptr(),
                        _stream_ptr(stream))
    return hard, ok, it, SCHED_NAME.get(used, used)


def decode_noalloc(code: Code, prm: DecodeParams, llr, stream=None, out=None):
    """As decode(), through the allocation-free entry point (caller-provided outputs via `out`)."""
    _check_llr(code, llr)
    batch = int(llr.shape[0])
    hard, ok, it = out if out is not None else _outputs(code, batch, llr.device)
    used = ldpcx_decode_noalloc(code.handle, prm, batch, llr.data_ptr(), hard.data_ptr(), ok.data_ptr(),
                                it.data_ptr(), _stream_ptr(stream))
    return hard, ok, it, SCHED_NAME.get(used, used)


def debug_dump(code: Code, prm: DecodeParams, llr, stream=None):
    """Decode and return the final messages: binary (hard, ok, iters, q, r, lam); GF(g) (..., alpha, beta),
    for rule SPA (..., u, v') in Q24."""
    import torch
    _check_llr(code, llr)
    batch = int(llr.shape[0])
    hard, ok, it = _outputs(code, batch, llr.device)
    if code.g == 2:
        a = torch.empty((batch, code.nnz), dtype=torch.int8, device=llr.device)
        b = torch.empty((batch, code.nnz), dtype=torch.int8, device=llr.device)
        c = torch.empty((batch, code.n), dtype=torch.int16, device=llr.device)
        cp = c.data_ptr()
    else:
        dt = torch.int32 if prm.rule == RULE["spa"] else torch.int16
        a = torch.empty((batch, code.nnz, code.g), dtype=dt, device=llr.device)
        b = torch.empty((batch, code.nnz, code.g), dtype=dt, device=llr.device)
        c, cp = None, 0
    ldpcx_debug_dump(code.handle, prm, batch, llr.data_ptr(), hard.data_ptr(), ok.data_ptr(), it.data_ptr(),
                     a.data_ptr(), b.data_ptr(), cp, _stream_ptr(stream))
    return (hard, ok, it, a, b, c) if code.g == 2 else (hard, ok, it, a, b)


class RaggedBatch:
    """A ragged batch marshalled once: the output tensors and the C job array are built
    here, and run() hands the same array to ldpcx_decode_ragged again (the inputs are read
    from the llr tensors' memory at each run)."""

    def __init__(self, items):
        self.items = list(items)  # keeps the codes and input tensors alive
        self.outs, jobs = [], []
        for code, prm, llr in self.items:
            _check_llr(code, llr)
            batch = int(llr.shape[0])
            hard, ok, it = _outputs(code, batch, llr.device)
            self.outs.append((hard, ok, it))
            jobs.append(Job(code.handle, prm, batch, llr.data_ptr(), hard.data_ptr(), ok.data_ptr(), it.data_ptr()))
        self.arr = (Job * len(jobs))(*jobs)

    def run(self, stream=None):
        _check(lib().ldpcx_decode_ragged(self.arr, len(self.arr), _stream_ptr(stream)))
        return self.outs


def decode_ragged(items, stream=None):
    """items: list of (Code, DecodeParams, llr tensor).  Returns a list of (hard, ok, iters)."""
    return RaggedBatch(items).run(stream)


def tune(code: Code, prm: DecodeParams, batch: int, stream=None):
    s, us = ldpcx_tune(code.handle, prm, batch, _stream_ptr(stream))
    return SCHED_NAME.get(s, s), us


def plan_info(code: Code, prm: DecodeParams, batch: int) -> dict:
    return ldpcx_plan_info(code.handle, prm, batch)


def plan_set(code: Code, prm: DecodeParams, batch: int, family: str, cw_per_wg: int = 1, threads: int = 256):
    fam = {v: k for k, v in FAMILY_NAME.items()}[family]
    ldpcx_plan_set(code.handle, prm, batch, fam, cw_per_wg, threads)


def ldpcx_valu_probe(blocks: int, iters: int, stream: int = 0) -> None:
    _check(lib().ldpcx_valu_probe(blocks, iters, ctypes.c_void_p(stream)))


def valu_probe(blocks: int, iters: int, stream=None) -> None:
    """Enqueue the packed 16-bit VALU issue-rate probe (16 wave instructions per round)."""
    ldpcx_valu_probe(blocks, iters, _stream_ptr(stream))


def unpack_bits(hard_packed: np.ndarray, n: int) -> np.ndarray:
    """[B, ceil(n/8)] LSB-first packed decisions -> [B, n] bits."""
    return np.unpackbits(np.asarray(hard_packed, dtype=np.uint8), axis=1, count=n, bitorder="little")


class Server:
    """Continuous-batching server over host buffers (ldpcx_server_*).

    submit() takes a host numpy array of channel LLRs (int8 [B, n] or int16 [B, n, g]),
    allocates the host outputs and keeps every buffer alive until the request is waited
    on; wait() returns (hard, ok, iters, (t_submit_us, t_admit_us, t_done_us)).
    """

    def __init__(self, hbm_budget: int = 8 << 30, max_inflight: int = 4, mode: str = "continuous",
                 max_launch_cw: int = 0):
        self.handle = ldpcx_server_create(ServerConfig(int(hbm_budget), int(max_inflight), SERVE[mode],
                                                       int(max_launch_cw)))
        self._live = {}

    def submit(self, code: Code, prm: DecodeParams, llr: np.ndarray) -> int:
        want = np.int8 if code.g == 2 else np.int16
        if llr.dtype != want or not llr.flags["C_CONTIGUOUS"]:
            raise ValueError(f"llr must be a C-contiguous {np.dtype(want).name} array")
        batch = int(llr.shape[0])
        hard = np.empty(code.hard_shape(batch), dtype=np.uint8)
        ok = np.empty(batch, dtype=np.uint8)
        it = np.empty(batch, dtype=np.int16)
        t = ldpcx_server_submit(self.handle, code.handle, prm, batch, llr.ctypes.data, hard.ctypes.data,
                                ok.ctypes.data, it.ctypes.data)
        self._live[t] = (llr, hard, ok, it)
        return t

    def poll(self, ticket: int) -> bool:
        return ldpcx_server_poll(self.handle, ticket)

    def wait(self, ticket: int, timeout_ms: int = -1):
        st, ts, ta, td = ldpcx_server_wait(self.handle, ticket, timeout_ms)
        if st == E_TIMEOUT:
            raise TimeoutError(ldpcx_last_error())
        bufs = self._live.pop(ticket, None)
        if st != OK:
            raise LdpcxError(st, ldpcx_last_error())
        _, hard, ok, it = bufs
        return hard, ok, it, (ts, ta, td)

    def cancel(self, ticket: int) -> None:
        ldpcx_server_cancel(self.handle, ticket)

    def stats(self) -> dict:
        return ldpcx_server_stats(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            ldpcx_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
