"""Pins for the oracle's denoiser: library special cases (torch float64 CPU
ops, an implementation independent of the oracle's NumPy code), closed-form
special cases of Module A, and row-permutation equivariance."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import synth
from oracle import denoiser as D
from oracle.evidence import evidence

torch.set_default_dtype(torch.float64)


def _w(cfg, seed=3, **kw):
    return synth.unpack_weights(synth.make_weights(cfg, seed, **kw), cfg)


def test_layer_norm_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.normal(0.3, 2.0, size=(5, 7, 64))
    g, b = rng.normal(1, 0.1, 64), rng.normal(0, 0.1, 64)
    ref = F.layer_norm(torch.tensor(x), (64,), torch.tensor(g), torch.tensor(b), eps=1e-5).numpy()
    np.testing.assert_allclose(D.layer_norm(x, g, b), ref, rtol=1e-12, atol=1e-12)


def test_gelu_matches_torch_erf():
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(D.gelu(x), F.gelu(torch.tensor(x)).numpy(), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("heads,S", [(4, 9), (8, 3), (1, 5)])
def test_mha_matches_torch(heads, S):
    rng = np.random.default_rng(heads)
    d = 32
    x = rng.normal(0, 1, size=(6, S, d))
    Wqkv, bqkv = rng.normal(0, 0.3, (3 * d, d)), rng.normal(0, 0.1, 3 * d)
    Wo, bo = rng.normal(0, 0.3, (d, d)), rng.normal(0, 0.1, d)
    ours = D.mha(x, Wqkv, bqkv, Wo, bo, heads)
    xt = torch.tensor(x).transpose(0, 1)                      # [S][B][d]
    ref, _ = F.multi_head_attention_forward(
        xt, xt, xt, d, heads, torch.tensor(Wqkv), torch.tensor(bqkv), None, None, False, 0.0,
        torch.tensor(Wo), torch.tensor(bo), training=False, need_weights=False)
    np.testing.assert_allclose(ours, ref.transpose(0, 1).numpy(), rtol=1e-11, atol=1e-12)


def _torch_layer(Z, w, l, heads):
    """The same block assembled from torch's own attention/LN/GELU routines."""
    p = f"l{l}."
    T = lambda a: torch.tensor(a)
    K, n, d = Z.shape
    z = T(Z)

    def attn(x, wq, bq, wo, bo):           # x [B][S][d] -> attention over S
        xt = x.transpose(0, 1)
        o, _ = F.multi_head_attention_forward(xt, xt, xt, d, heads, T(wq), T(bq), None, None, False,
                                              0.0, T(wo), T(bo), training=False, need_weights=False)
        return o.transpose(0, 1)
    z = z + attn(F.layer_norm(z, (d,), T(w[p + "ln1_g"]), T(w[p + "ln1_b"])),
                 w[p + "Wqkv_r"], w[p + "bqkv_r"], w[p + "Wo_r"], w[p + "bo_r"])
    zt = z.transpose(0, 1)
    zt = zt + attn(F.layer_norm(zt, (d,), T(w[p + "ln2_g"]), T(w[p + "ln2_b"])),
                   w[p + "Wqkv_u"], w[p + "bqkv_u"], w[p + "Wo_u"], w[p + "bo_u"])
    z = zt.transpose(0, 1)
    h = F.gelu(F.linear(F.layer_norm(z, (d,), T(w[p + "ln3_g"]), T(w[p + "ln3_b"])), T(w[p + "W1"]), T(w[p + "b1"])))
    return (z + F.linear(h, T(w[p + "W2"]), T(w[p + "b2"]))).numpy()


def test_layer_matches_torch_composition():
    cfg = synth.ModelCfg(1, 64, 4, n_max=64)
    w = _w(cfg, bias_std=0.05, ln_std=0.1)
    rng = np.random.default_rng(5)
    Z = rng.normal(0, 1, size=(3, 10, 64))
    np.testing.assert_allclose(D.layer(Z, w, 0, 4), _torch_layer(Z, w, 0, 4), rtol=1e-10, atol=1e-11)


def test_single_key_attention_reduces_to_value_path():
    """With one row (K=1) user attention is softmax over one key = 1, so the
    block adds (LN(z) Wv^T + bv) Wo^T + bo exactly."""
    cfg = synth.ModelCfg(1, 32, 4, n_max=16)
    w = _w(cfg, bias_std=0.05, ln_std=0.1)
    rng = np.random.default_rng(6)
    x = rng.normal(0, 1, size=(7, 1, 32))
    o = D.mha(x, w["l0.Wqkv_u"], w["l0.bqkv_u"], w["l0.Wo_u"], w["l0.bo_u"], 4)
    v = x @ w["l0.Wqkv_u"][64:96].T + w["l0.bqkv_u"][64:96]
    np.testing.assert_allclose(o, v @ w["l0.Wo_u"].T + w["l0.bo_u"], rtol=1e-12, atol=1e-13)


def test_embedding_terms():
    cfg = synth.ModelCfg(1, 16, 2, n_max=8)
    w = _w(cfg)
    X = np.array([[0, 1, 2, 2], [2, 2, 1, 0]], np.uint8)
    Z = D.embed(X, 0.25, w)
    assert Z.shape == (2, 4, 16)
    np.testing.assert_allclose(Z[1, 2], w["E"][1] + w["P"][2] + 0.25 * w["u"], rtol=1e-15)


def test_module_a_closed_forms():
    cfg = synth.ModelCfg(1, 8, 2, n_max=4)
    w = _w(cfg)
    d = 8
    # w_0 = unit vector e_0, w_1 = unit vector e_1; row 0 has Z[0] = log 3 -> r = (3/4, 1/4)
    w["W"] = np.zeros((2, d)); w["W"][0, 0] = 1.0; w["W"][1, 1] = 1.0
    w["Wg1"] = np.zeros((d, 2 * d)); w["Wg2"] = np.zeros((d, d)); w["bg2"] = np.zeros(d)
    w["v"] = np.zeros((2, d)); w["v"][0, 2] = 1.0; w["v"][1, 3] = 1.0
    Z = np.zeros((2, 1, d)); Z[0, 0, 0] = math.log(3.0)
    p = np.array([[0.8, 0.2]])
    zt, parts = D.module_a(Z, p, w)
    np.testing.assert_allclose(parts["r"][:, 0, 0], [0.75, 0.25], rtol=1e-14)
    np.testing.assert_allclose(parts["r"][:, 0, 1], [0.5, 0.5], rtol=1e-14)
    # e[0] = 0.75*0.8*v0 + 0.5*0.2*v1 ; e[1] = 0.25*0.8*v0 + 0.5*0.2*v1
    np.testing.assert_allclose(parts["e"][0, 0, 2:4], [0.6, 0.1], rtol=1e-14)
    np.testing.assert_allclose(parts["e"][1, 0, 2:4], [0.2, 0.1], rtol=1e-14)
    # zero gate MLP -> g = 1/2 -> Z~ = (Z + e) / 2
    np.testing.assert_allclose(zt, 0.5 * (Z + parts["e"]), rtol=1e-14)
    # huge positive gate bias -> g -> 1 -> Z~ = Z
    w["bg2"] = np.full(d, 60.0)
    zt2, _ = D.module_a(Z, p, w)
    np.testing.assert_allclose(zt2, Z, atol=1e-20)


def test_module_a_responsibilities_sum_to_one_and_uniform_for_equal_rows():
    cfg = synth.ModelCfg(1, 16, 2, n_max=8)
    w = _w(cfg, seed=8)
    rng = np.random.default_rng(1)
    Z = rng.normal(0, 1, size=(5, 6, 16))
    _, p = evidence(rng.normal(0, 2, size=6), 0.5, 5)
    _, parts = D.module_a(Z, p, w)
    np.testing.assert_allclose(parts["r"].sum(axis=0), 1.0, rtol=1e-14)
    Zs = np.repeat(Z[:1], 5, axis=0)
    _, parts = D.module_a(Zs, p, w)
    np.testing.assert_allclose(parts["r"], 0.2, rtol=1e-14)
    _, parts1 = D.module_a(Z[:1], p, w)
    np.testing.assert_allclose(parts1["r"], 1.0)
    np.testing.assert_allclose(parts1["e"][0], p @ w["v"], rtol=1e-14)


def test_responsibilities_depend_only_on_the_column_symbols():
    """The rows of a slot share P[l] + gamma u, which cancels in the softmax
    over rows: r[k, l, a] is the softmax over k of <E[X[k, l]], w_a> / tau
    whatever P and gamma are (the identity the fused GPU kernel computes r
    from, checked here on the oracle's own Module A)."""
    cfg = synth.ModelCfg(1, 16, 2, n_max=8)
    w = _w(cfg, seed=12)
    rng = np.random.default_rng(4)
    X = rng.integers(0, 3, size=(5, 7)).astype(np.uint8)
    _, p = evidence(rng.normal(0, 2, size=7), 0.5, 5)
    tau = 0.7
    _, a = D.module_a(D.embed(X, 0.3, w), p, w, tau)
    w2 = dict(w)
    w2["P"] = rng.normal(0, 1.0, size=w["P"].shape)
    w2["u"] = rng.normal(0, 1.0, size=w["u"].shape)
    _, b = D.module_a(D.embed(X, 0.9, w2), p, w2, tau)
    np.testing.assert_allclose(a["r"], b["r"], rtol=1e-12)
    table = w["E"] @ w["W"].T                            # [3 symbols][2 logits]
    lt = table[X] / tau                                  # [K][n][2]
    r = np.exp(lt - lt.max(axis=0)) / np.exp(lt - lt.max(axis=0)).sum(axis=0)
    np.testing.assert_allclose(a["r"], r, rtol=1e-12)
    # and the intermediate logits themselves do depend on P and gamma
    assert np.max(np.abs(a["lbar"] - b["lbar"])) > 1e-3


def test_denoiser_row_permutation_equivariance():
    cfg = synth.ModelCfg(2, 32, 4, n_max=32)
    w = _w(cfg, bias_std=0.02, ln_std=0.05)
    code = synth.regular_ldpc(32, seed=1032)
    rng = np.random.default_rng(2)
    X = rng.integers(0, 3, size=(4, 32)).astype(np.uint8)
    _, p = evidence(rng.normal(0, 2, size=32), 0.4, 4)
    out = D.denoise(X, p, code, w, 2, 4, gamma=float((X == 2).mean()))
    perm = np.array([2, 0, 3, 1])
    out_p = D.denoise(X[perm], p, code, w, 2, 4, gamma=float((X == 2).mean()))
    np.testing.assert_allclose(out_p["logits"], out["logits"][perm], rtol=1e-11, atol=1e-12)


def test_projection_uses_final_layernorm_and_shared_w():
    cfg = synth.ModelCfg(1, 16, 2, n_max=8)
    w = _w(cfg, ln_std=0.1)
    rng = np.random.default_rng(4)
    Z = rng.normal(0, 1, size=(2, 3, 16))
    ref = F.linear(F.layer_norm(torch.tensor(Z), (16,), torch.tensor(w["lnf_g"]), torch.tensor(w["lnf_b"])),
                   torch.tensor(w["W"])).numpy()
    np.testing.assert_allclose(D.project(Z, w), ref, rtol=1e-12)
