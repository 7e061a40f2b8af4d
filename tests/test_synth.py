"""Seeded input generators: code structure, channel statistics, determinism."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("n", [12, 32, 64, 128, 256])
def test_regular_code_structure(n):
    c = synth.regular_ldpc(n, seed=1000 + n)
    assert c.H.shape == (n // 2, n)
    assert (c.H.sum(axis=0) == 3).all() and (c.H.sum(axis=1) == 6).all()
    assert synth.rank_gf2(c.H) == n // 2 and c.k == n // 2
    assert ((c.H.astype(int) @ c.G.T.astype(int)) % 2 == 0).all()
    assert synth.rank_gf2(c.G) == c.k
    # CSR and its transpose describe the same edges, ascending
    edges = {(j, int(v)) for j in range(c.m) for v in c.col_idx[c.row_ptr[j]:c.row_ptr[j + 1]]}
    edges_t = {(int(j), v) for v in range(c.n) for j in c.var_idx[c.var_ptr[v]:c.var_ptr[v + 1]]}
    assert edges == edges_t == {(int(j), int(v)) for j, v in zip(*np.nonzero(c.H))}
    for j in range(c.m):
        seg = c.col_idx[c.row_ptr[j]:c.row_ptr[j + 1]]
        assert (np.diff(seg) > 0).all()


def test_code_is_deterministic():
    a = synth.regular_ldpc(64, seed=7)
    b = synth.regular_ldpc(64, seed=7)
    assert np.array_equal(a.H, b.H) and np.array_equal(a.G, b.G)


def test_channel_statistics():
    c = synth.regular_ldpc(128, seed=1128)
    bins = synth.make_bins(c, 4, 400, 4.0, seed=5)
    assert ((bins.codewords.astype(int) @ c.H.T.astype(int)) % 2 == 0).all()
    x = 1.0 - 2.0 * bins.codewords.astype(np.float64)
    resid = bins.y.astype(np.float64) - x.sum(axis=1)
    s2 = synth.ebn0_to_sigma2(4.0, 0.5)
    assert abs(resid.mean()) < 0.01
    assert abs(resid.var() / s2 - 1.0) < 0.02
    for b in range(bins.info.shape[0]):
        assert len({r.tobytes() for r in bins.info[b]}) == 4


def test_sigma2_values():
    assert abs(synth.ebn0_to_sigma2(2.0, 0.5) - 0.6310) < 1e-4
    assert abs(synth.ebn0_to_sigma2(5.0, 0.5) - 0.3162) < 1e-4


def test_weights_layout_and_seed():
    cfg = synth.ModelCfg(2, 64, 4)
    w1 = synth.make_weights(cfg, 11)
    w2 = synth.make_weights(cfg, 11)
    assert np.array_equal(w1, w2) and w1.dtype == np.float32
    u = synth.unpack_weights(w1, cfg)
    assert u["l1.W2"].shape == (64, 256) and np.all(u["lnf_g"] == 1.0) and np.all(u["bg1"] == 0)
    assert abs(u["P"].std() - 0.02) < 0.001
