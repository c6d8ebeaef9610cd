"""Structure of the seeded synthetic workloads (codes, encoders, channel)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2508_03567_amd import synth as S


def _binary_syndrome_zero(code, cw):
    H = sp.csr_matrix((np.ones(code.nnz), code.col_idx, code.row_ptr), shape=(code.m, code.n))
    return ((H @ cw.T.astype(np.float64)).astype(np.int64) % 2 == 0).all(axis=0)


def test_cfg0_structure():
    c = S.workload(0).code
    assert (c.n, c.m, c.nnz, c.z) == (192, 96, 576, 32)
    assert (c.row_degrees() == 6).all() and (c.col_degrees() == 3).all()


def test_cfg1_structure():
    c = S.workload(1).code
    assert (c.n, c.m, c.nnz, c.z) == (2304, 1152, 7296, 96)
    shifts = c.meta["shifts"]
    assert shifts.shape == (12, 24) and (shifts >= 0).sum() == 76
    colw = (shifts >= 0).sum(axis=0)
    assert sorted(colw.tolist()) == [2] * 11 + [3] * 8 + [6] * 5
    roww = (shifts >= 0).sum(axis=1)
    assert sorted(roww.tolist()) == [6] * 8 + [7] * 4


@pytest.mark.parametrize("cfg", [0, 1])
def test_layers_touch_disjoint_columns(cfg):
    c = S.workload(cfg).code
    for layer in range(c.m // c.z):
        cols = c.col_idx[c.row_ptr[layer * c.z]:c.row_ptr[(layer + 1) * c.z]]
        assert len(np.unique(cols)) == len(cols)


def test_cfg2_structure():
    c = S.workload(2).code
    assert (c.n, c.m, c.nnz) == (64800, 32400, 226799)
    rd = c.row_degrees()
    assert rd[0] == 6 and (rd[1:] == 7).all()
    cd = c.col_degrees()
    assert (cd[:12960] == 8).all() and (cd[12960:32400] == 3).all()
    assert (cd[32400:-1] == 2).all() and cd[-1] == 1


def test_cfg3_structure():
    c = S.workload(3).code
    assert (c.g, c.prim_poly, c.n, c.m, c.nnz) == (64, 0x43, 192, 96, 384)
    assert (c.row_degrees() == 4).all() and (c.col_degrees() == 2).all()
    assert c.h_val.min() >= 1 and c.h_val.max() <= 63


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_binary_encoders_produce_codewords(cfg):
    w = S.workload(cfg, batch=64)
    cw = S.random_codewords(w.code, 64, seed=5)
    assert _binary_syndrome_zero(w.code, cw).all()
    assert 0.4 < cw.mean() < 0.6


def test_nb_encoder_produces_codewords():
    w = S.workload(3, batch=16)
    cw = S.random_codewords(w.code, 16, seed=5)
    assert all(O.syndrome_ok(w.code, c) for c in cw)
    assert len(np.unique(cw)) > 40


def test_batches_are_prefixes():
    w = S.workload(1, batch=300)
    cw1, l1 = S.make_inputs(w)
    w.batch = 40
    cw2, l2 = S.make_inputs(w)
    assert (cw1[:40] == cw2).all() and (l1[:40] == l2).all()


def test_channel_quantisation():
    bits = np.zeros((4, 1000), dtype=np.uint8)
    llr = S.binary_llr_int8(bits, 2.5, seed=1)
    assert llr.dtype == np.int8 and llr.min() >= -31 and llr.max() <= 31
    assert (llr > 0).mean() > 0.85
    # noiseless: L = 2/sigma^2 exactly, quantised with scale 2
    s2 = S.sigma2_for(2.5)
    llr0 = S.binary_llr_int8(np.ones((1, 3), dtype=np.uint8), 2.5, seed=1, noiseless=True)
    assert (llr0 == -min(31, int(np.floor(4.0 / s2 + 0.5)))).all()
    assert S.round_half_away(np.array([0.5, -0.5, 1.5, -2.5])).tolist() == [1, -1, 2, -3]


def test_nb_gamma_is_symbol_cost():
    sym = np.array([[0, 5, 63]], dtype=np.uint8)
    gam = S.nb_gamma_int16(sym, 64, 2.0, seed=3)
    assert gam.shape == (1, 3, 64) and (gam.min(axis=2) == 0).all()
    # the noiseless vector is minimal exactly at the sent symbol, and costs add per differing bit
    gam0 = S.nb_gamma_int16(sym, 64, 2.0, seed=3, noiseless=True)
    assert (gam0.argmin(axis=2) == sym).all()
    per_bit = gam0[0, 0, 1]
    pop = np.array([bin(x).count("1") for x in range(64)])
    assert (gam0[0, 0] == per_bit * pop).all()
