"""Seeded synthetic workloads for the batched LDPC decoders.

Builds what both the GPU decoder and the CPU oracle consume: parity-check
matrices (quasi-cyclic binary, long irregular binary with a staircase parity
part, random regular non-binary over GF(2^p), and the GF(4) example matrix of
eq. (1)), systematic encoders, and the BPSK/AWGN channel with integer
quantisation.

Nothing here decodes: there is no check-node or variable-node rule and no
syndrome test.  The small GF(2^p) multiply below exists only to encode
codewords and is written independently of the decoders' own field arithmetic.

Randomness: every draw comes from numpy's Philox4x32-10 counter-based
generator.  Codewords are generated in fixed chunks of ``CHUNK`` codewords,
each chunk with its own key derived from (seed, chunk index, purpose), so a
batch of B codewords is a prefix of any larger batch drawn with the same seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

CHUNK = 256

# Purposes used to separate random streams.
_P_INFO, _P_NOISE = 1, 2


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(k) for k in key])))


# --------------------------------------------------------------------------
# Code container
# --------------------------------------------------------------------------
@dataclass
class Code:
    """A sparse parity-check matrix H (m x n) over GF(g), g = 2^p.

    Stored by check (CSR): the nonzeros of row i are ``col_idx[row_ptr[i]:row_ptr[i+1]]``
    in ascending column order with GF coefficients ``h_val`` (None when g == 2).
    ``z`` is the number of consecutive rows that form one layer (rows inside a
    layer touch disjoint columns), or 0 when the code has no layer structure.
    ``k_info`` = n - m is the information length used for throughput accounting.
    """

    name: str
    g: int
    prim_poly: int
    n: int
    m: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    h_val: Optional[np.ndarray]
    z: int = 0
    k_info: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def p(self) -> int:
        return int(self.g).bit_length() - 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def col_degrees(self) -> np.ndarray:
        return np.bincount(self.col_idx, minlength=self.n)

    def dense(self) -> np.ndarray:
        H = np.zeros((self.m, self.n), dtype=np.int64)
        rows = np.repeat(np.arange(self.m), self.row_degrees())
        H[rows, self.col_idx] = 1 if self.h_val is None else self.h_val
        return H


def code_from_pairs(name, g, prim_poly, n, m, rows, cols, vals=None, z=0) -> Code:
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    if vals is not None:
        vals = np.asarray(vals, dtype=np.uint8)[order]
    key = rows * n + cols
    if np.any(key[1:] == key[:-1]):
        raise ValueError("repeated (row, col) entry")
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    return Code(name=name, g=g, prim_poly=prim_poly, n=n, m=m, row_ptr=row_ptr,
                col_idx=cols.astype(np.int32), h_val=vals, z=z, k_info=n - m)


def code_from_dense(H, g=2, prim_poly=0x3, z=0, name="dense") -> Code:
    H = np.asarray(H)
    rows, cols = np.nonzero(H)
    vals = None if g == 2 else H[rows, cols]
    return code_from_pairs(name, g, prim_poly, H.shape[1], H.shape[0], rows, cols, vals, z=z)


# --------------------------------------------------------------------------
# Quasi-cyclic binary codes
# --------------------------------------------------------------------------
def qc_code(shifts: np.ndarray, Z: int, name="qc") -> Code:
    """Expand a base matrix of circulant shifts (-1 = zero block).

    Circulant convention: row i of the Z x Z block with shift s has its one in
    column (i + s) mod Z.  Each base row becomes one layer of Z rows.
    """
    shifts = np.asarray(shifts)
    mb, nb = shifts.shape
    rows, cols = [], []
    i = np.arange(Z)
    for r in range(mb):
        for c in range(nb):
            s = int(shifts[r, c])
            if s < 0:
                continue
            rows.append(r * Z + i)
            cols.append(c * Z + (i + s) % Z)
    code = code_from_pairs(name, 2, 0x3, nb * Z, mb * Z, np.concatenate(rows), np.concatenate(cols), z=Z)
    code.meta["shifts"] = shifts.copy()
    code.meta["Z"] = Z
    return code


def cfg0_code(seed: int = 1) -> Code:
    """(3,6)-regular QC code, Z = 32, all 18 base entries nonzero, n = 192."""
    shifts = _rng(seed, 0).integers(0, 32, size=(3, 6))
    return qc_code(shifts, 32, name="qc_n192_z32")


def _place_base(col_w: np.ndarray, row_w: np.ndarray, rng, max_tries=100000) -> np.ndarray:
    """Random 0/1 base pattern with given column and row weights and no repeated entry.

    Columns are placed heaviest first; each picks distinct rows at random with
    probability proportional to the rows' remaining capacity.  A dead end restarts.
    """
    order = np.argsort(-col_w, kind="stable")
    for _ in range(max_tries):
        cap = row_w.astype(np.int64).copy()
        B = np.zeros((len(row_w), len(col_w)), dtype=bool)
        ok = True
        for c in order:
            w = int(col_w[c])
            avail = np.flatnonzero(cap > 0)
            if len(avail) < w:
                ok = False
                break
            p = cap[avail] / cap[avail].sum()
            rows = rng.choice(avail, size=w, replace=False, p=p)
            B[rows, c] = True
            cap[rows] -= 1
        if ok and not cap.any():
            return B
    raise RuntimeError("base placement failed")


def cfg1_code(seed: int = 2) -> Code:
    """Irregular QC code, 12 x 24 base, Z = 96, n = 2304.

    Column weights: 5 columns of weight 6, 8 of weight 3, 11 of weight 2 (76
    nonzeros); row weights 6 (8 rows) and 7 (4 rows).  Column and row weight
    orders are shuffled by the seed; shifts are uniform in [0, 96).
    """
    rng = _rng(seed, 0)
    col_w = np.array([6] * 5 + [3] * 8 + [2] * 11)
    row_w = np.array([6] * 8 + [7] * 4)
    rng.shuffle(col_w)
    rng.shuffle(row_w)
    B = _place_base(col_w, row_w, rng)
    shifts = np.where(B, rng.integers(0, 96, size=B.shape), -1)
    return qc_code(shifts, 96, name="qc_n2304_z96")


def cfg2_code(seed: int = 3) -> Code:
    """Long irregular code n = 64800, k = 32400 with Z = 360 group structure.

    Information columns come in 90 groups of 360: 36 groups of degree 8 and 54
    groups of degree 3 (12960 + 19440 columns, the split that gives check
    degree 7).  A group owns one address x_a per unit of degree; the 450
    addresses have residues mod 90 balanced (5 per residue, seeded shuffle) and
    x_a = r_a + 90 u_a with u_a uniform in [0, 360), distinct within a group.
    Column j of a group connects to checks (x_a + 90 j) mod 32400.  Parity
    column i (staircase) connects to checks i and i + 1.
    """
    rng = _rng(seed, 0)
    Zg, q, M, K = 360, 90, 32400, 32400
    degs = [8] * 36 + [3] * 54
    residues = np.repeat(np.arange(q), 5)
    rng.shuffle(residues)
    rows, cols = [], []
    j = np.arange(Zg)
    pos = 0
    addrs = []
    for gi, d in enumerate(degs):
        res = residues[pos:pos + d]
        pos += d
        while True:
            u = rng.integers(0, Zg, size=d)
            x = res + q * u
            if len(np.unique(x)) == d:
                break
        addrs.append(x)
        for xa in x:
            rows.append((xa + q * j) % M)
            cols.append(gi * Zg + j)
    ip = np.arange(M)
    rows += [ip, ip[1:]]
    cols += [K + ip, K + ip[:-1]]
    code = code_from_pairs("irr_n64800", 2, 0x3, K + M, M, np.concatenate(rows), np.concatenate(cols), z=0)
    code.meta["addresses"] = addrs
    code.meta["staircase_from"] = K
    return code


def random_regular_nb_code(n: int, m: int, dv: int, dc: int, g: int, prim_poly: int, seed: int,
                           name="nb") -> Code:
    """(dv, dc)-regular code over GF(g) by seeded socket matching without multi-edges.

    Coefficients are uniform over the nonzero field elements.
    """
    assert n * dv == m * dc
    rng = _rng(seed, 0)
    for _ in range(100000):
        vs = np.repeat(np.arange(n), dv)
        rng.shuffle(vs)
        rows = np.repeat(np.arange(m), dc)
        key = np.sort(rows * n + vs)
        if np.all(key[1:] != key[:-1]):
            break
    else:
        raise RuntimeError("socket matching failed")
    vals = rng.integers(1, g, size=n * dv)
    return code_from_pairs(name, g, prim_poly, n, m, rows, vs, vals)


def cfg3_code(seed: int = 4) -> Code:
    """(2,4)-regular code over GF(64), primitive polynomial x^6 + x + 1, n = 192 symbols."""
    return random_regular_nb_code(192, 96, 2, 4, 64, 0x43, seed, name="gf64_n192")


def eq1_code() -> Code:
    """The 3 x 6 example matrix over GF(4) of eq. (1), polynomial basis, alpha = 2, alpha^2 = 3."""
    a, a2 = 2, 3
    H = [[a, 0, 1, a, 0, 1],
         [a2, a, 0, 1, 1, 0],
         [0, a, a2, 0, a2, 1]]
    return code_from_dense(H, g=4, prim_poly=0x7, name="eq1_gf4")


# Primitive polynomials for the GF-size sweep (bit i = coefficient of x^i).
PRIM_POLY = {2: 0x3, 4: 0x7, 8: 0xB, 16: 0x13, 32: 0x25, 64: 0x43, 128: 0x89, 256: 0x11D}


# --------------------------------------------------------------------------
# Encoders (generator-side GF arithmetic, independent of the decoders)
# --------------------------------------------------------------------------
class _GFEnc:
    def __init__(self, g: int, poly: int):
        self.g = g
        p = g.bit_length() - 1
        exp = np.zeros(2 * g, dtype=np.int64)
        log = np.zeros(g, dtype=np.int64)
        v = 1
        for i in range(g - 1):
            exp[i] = v
            log[v] = i
            v <<= 1
            if v >> p:
                v ^= poly
        exp[g - 1:2 * g - 2] = exp[:g - 1]
        self.exp, self.log = exp, log

    def mul(self, a, b):
        a = np.asarray(a, dtype=np.int64)
        b = np.asarray(b, dtype=np.int64)
        r = self.exp[(self.log[a] + self.log[b]) % (self.g - 1)]
        return np.where((a == 0) | (b == 0), 0, r)

    def inv(self, a):
        a = np.asarray(a, dtype=np.int64)
        return self.exp[(self.g - 1 - self.log[a]) % (self.g - 1)]


def _rref_gf2(H: np.ndarray):
    """Reduced row echelon form over GF(2) with bit-packed rows.  Returns (R, pivots)."""
    m, n = H.shape
    P = np.packbits(H.astype(np.uint8), axis=1)
    pivots = []
    r = 0
    for c in range(n):
        if r == m:
            break
        byte, bit = c >> 3, 7 - (c & 7)
        colbits = (P[r:, byte] >> bit) & 1
        nz = np.flatnonzero(colbits)
        if len(nz) == 0:
            continue
        piv = r + nz[0]
        if piv != r:
            P[[r, piv]] = P[[piv, r]]
        hit = ((P[:, byte] >> bit) & 1).astype(bool)
        hit[r] = False
        P[hit] ^= P[r]
        pivots.append(c)
        r += 1
    R = np.unpackbits(P[:r], axis=1, count=n)
    return R, np.array(pivots, dtype=np.int64)


def _rref_gfq(H: np.ndarray, gf: _GFEnc):
    m, n = H.shape
    A = H.astype(np.int64).copy()
    pivots = []
    r = 0
    for c in range(n):
        if r == m:
            break
        nz = np.flatnonzero(A[r:, c])
        if len(nz) == 0:
            continue
        piv = r + nz[0]
        if piv != r:
            A[[r, piv]] = A[[piv, r]]
        A[r] = gf.mul(A[r], gf.inv(A[r, c]))
        for i in range(m):
            if i != r and A[i, c]:
                A[i] ^= gf.mul(A[r], A[i, c])
        pivots.append(c)
        r += 1
    return A[:r], np.array(pivots, dtype=np.int64)


class Encoder:
    """Systematic encoder from H by Gaussian elimination (or a staircase accumulator).

    Free (non-pivot) positions carry uniformly random symbols; pivot positions
    are solved from H c = 0.  For codes whose H is rank deficient the number of
    free positions exceeds n - m; all of them are random.
    """

    def __init__(self, code: Code):
        self.code = code
        self.staircase_from = code.meta.get("staircase_from")
        if self.staircase_from is not None:
            return
        H = code.dense()
        if code.g == 2:
            R, piv = _rref_gf2(H)
            self.gf = None
        else:
            self.gf = _GFEnc(code.g, code.prim_poly)
            R, piv = _rref_gfq(H, self.gf)
        free = np.setdiff1d(np.arange(code.n), piv)
        self.pivots, self.free = piv, free
        self.Rf = R[:, free]  # pivot symbol i = sum_f Rf[i, f] * c_f  (characteristic 2)

    def encode(self, free_symbols: np.ndarray) -> np.ndarray:
        code = self.code
        B = free_symbols.shape[0]
        if self.staircase_from is not None:
            K = self.staircase_from
            u = free_symbols.astype(np.uint8)
            rp, ci = code.row_ptr, code.col_idx
            info_deg = np.add.reduceat((ci < K).astype(np.int64), rp[:-1])
            # each check's information columns are its first info_deg entries (ascending columns)
            s = np.zeros((B, code.m), dtype=np.uint8)
            maxd = int(info_deg.max())
            for t in range(maxd):
                rows = np.flatnonzero(info_deg > t)
                s[:, rows] ^= u[:, ci[rp[rows] + t]]
            par = np.bitwise_xor.accumulate(s, axis=1)
            return np.concatenate([u, par], axis=1)
        c = np.zeros((B, code.n), dtype=np.uint8)
        c[:, self.free] = free_symbols
        if code.g == 2:
            par = (free_symbols.astype(np.float32) @ self.Rf.T.astype(np.float32))
            c[:, self.pivots] = (par.astype(np.int64) & 1).astype(np.uint8)
        else:
            acc = np.zeros((B, len(self.pivots)), dtype=np.int64)
            for j in range(len(self.free)):
                acc ^= self.gf.mul(self.Rf[None, :, j], free_symbols[:, j:j + 1].astype(np.int64))
            c[:, self.pivots] = acc.astype(np.uint8)
        return c

    @property
    def n_free(self) -> int:
        if self.staircase_from is not None:
            return self.staircase_from
        return len(self.free)


_ENC_CACHE: dict = {}


def encoder_for(code: Code) -> Encoder:
    key = id(code)
    enc = _ENC_CACHE.get(key)
    if enc is None or enc.code is not code:
        enc = Encoder(code)
        _ENC_CACHE[key] = enc
    return enc


def random_codewords(code: Code, batch: int, seed: int) -> np.ndarray:
    """[batch, n] uint8 codewords (symbols in [0, g)) with random information symbols."""
    enc = encoder_for(code)
    out = np.empty((batch, code.n), dtype=np.uint8)
    for c0 in range(0, batch, CHUNK):
        b = min(CHUNK, batch - c0)
        rng = _rng(seed, c0 // CHUNK, _P_INFO)
        free = rng.integers(0, code.g, size=(b, enc.n_free), dtype=np.int64).astype(np.uint8)
        out[c0:c0 + b] = enc.encode(free)
    return out


# --------------------------------------------------------------------------
# Channel: BPSK over AWGN, quantised
# --------------------------------------------------------------------------
def sigma2_for(ebn0_db: float, rate: float = 0.5) -> float:
    """Noise variance for BPSK at Eb/N0 (dB) and code rate R: 1 / (2 R 10^(Eb/N0/10))."""
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def _noise(seed: int, batch: int, width: int) -> np.ndarray:
    out = np.empty((batch, width), dtype=np.float64)
    for c0 in range(0, batch, CHUNK):
        b = min(CHUNK, batch - c0)
        out[c0:c0 + b] = _rng(seed, c0 // CHUNK, _P_NOISE).standard_normal((b, width))
    return out


def channel_bit_llr(bits: np.ndarray, ebn0_db: float, seed: int, rate: float = 0.5,
                    noiseless: bool = False) -> np.ndarray:
    """Real channel LLRs L = 2 y / sigma^2 for BPSK (bit 0 -> +1, bit 1 -> -1) over AWGN."""
    s2 = sigma2_for(ebn0_db, rate)
    x = 1.0 - 2.0 * bits.astype(np.float64)
    if not noiseless:
        x = x + np.sqrt(s2) * _noise(seed, bits.shape[0], bits.shape[1])
    return 2.0 * x / s2


def quantize(L: np.ndarray, scale: float, clip: int) -> np.ndarray:
    """Round half away from zero after scaling, then saturate to [-clip, clip]."""
    return np.clip(round_half_away(scale * L), -clip, clip)


def binary_llr_int8(codewords: np.ndarray, ebn0_db: float, seed: int, rate: float = 0.5,
                    scale: float = 2.0, clip: int = 31, noiseless: bool = False) -> np.ndarray:
    """int8 [batch, n] quantised channel LLRs (positive favours bit 0)."""
    return quantize(channel_bit_llr(codewords, ebn0_db, seed, rate, noiseless), scale, clip).astype(np.int8)


def symbol_bits(symbols: np.ndarray, p: int) -> np.ndarray:
    """[..., p] bits of GF(2^p) symbols; bit i is the coefficient of x^i."""
    return ((symbols[..., None].astype(np.int64) >> np.arange(p)) & 1).astype(np.uint8)


def nb_gamma_int16(symbols: np.ndarray, g: int, ebn0_db: float, seed: int, rate: float = 0.5,
                   scale: float = 4.0, clip: int = 127, noiseless: bool = False) -> np.ndarray:
    """int16 [batch, n, g] per-symbol channel log-likelihood ratio vectors, min 0 per symbol.

    Each symbol's p bits are sent as BPSK; per-bit LLRs are quantised to
    Lq = clip(round(scale * L), +-clip).  With independent bits, the cost of
    symbol x relative to the most likely symbol eta (the bitwise hard decision)
    is the sum of |Lq_i| over the bits where x differs from eta.
    """
    p = g.bit_length() - 1
    B, n = symbols.shape
    bits = symbol_bits(symbols, p).reshape(B, n * p)
    Lq = quantize(channel_bit_llr(bits, ebn0_db, seed, rate, noiseless), scale, clip).reshape(B, n, p)
    eta = (Lq < 0)
    mag = np.abs(Lq).astype(np.int16)
    xb = symbol_bits(np.arange(g), p).astype(bool)  # [g, p]
    gamma = np.zeros((B, n, g), dtype=np.int16)
    for i in range(p):
        diff = xb[None, None, :, i] != eta[:, :, None, i]
        gamma += np.where(diff, mag[:, :, None, i], np.int16(0)).astype(np.int16)
    return gamma


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    code: Code
    rule: str          # "nms" | "oms" | "ms" | "minmax"
    schedule: str      # "flooding" | "layered"
    max_iters: int
    batch: int
    ebn0_db: float
    data_seed: int
    nms_num: int = 3
    nms_shift: int = 2
    oms_offset: int = 1
    msg_max: int = 127

    @property
    def info_bits_per_cw(self) -> int:
        return self.code.k_info * self.code.p


_CODE_CACHE: dict = {}


def _cached(key, fn):
    c = _CODE_CACHE.get(key)
    if c is None:
        c = fn()
        _CODE_CACHE[key] = c
    return c


def workload(cfg: int, batch: Optional[int] = None, ebn0_db: Optional[float] = None) -> Workload:
    """The four decoder workloads (code seed = index + 1, data seed = 1000 + index)."""
    if cfg == 0:
        code = _cached(0, cfg0_code)
        w = Workload("qc_n192_nms_flood_i10", code, "nms", "flooding", 10, 1000, 2.5, 1000)
    elif cfg == 1:
        code = _cached(1, cfg1_code)
        w = Workload("qc_n2304_oms_layered_i20", code, "oms", "layered", 20, 65536, 2.0, 1001)
    elif cfg == 2:
        code = _cached(2, cfg2_code)
        w = Workload("irr_n64800_nms_flood_i50", code, "nms", "flooding", 50, 1024, 1.0, 1002)
    elif cfg == 3:
        code = _cached(3, cfg3_code)
        w = Workload("gf64_n192_minmax_i20", code, "minmax", "flooding", 20, 8192, 2.0, 1003)
    else:
        raise ValueError(cfg)
    if batch is not None:
        w.batch = batch
    if ebn0_db is not None:
        w.ebn0_db = ebn0_db
    return w


def make_inputs(w: Workload, seed_offset: int = 0, noiseless: bool = False):
    """(codewords, channel input) for a workload: int8 [B, n] LLRs or int16 [B, n, g] vectors."""
    seed = w.data_seed + seed_offset
    cw = random_codewords(w.code, w.batch, seed)
    if w.code.g == 2:
        llr = binary_llr_int8(cw, w.ebn0_db, seed, noiseless=noiseless)
    else:
        llr = nb_gamma_int16(cw, w.code.g, w.ebn0_db, seed, noiseless=noiseless)
    return cw, llr
