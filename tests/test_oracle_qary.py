"""Pins of the Q-ary (GF(2^m)) decode in the oracle: the check message
against exhaustive enumeration of the c2v rule, the whole denoiser at Q = 2
against the binary oracle, the reveal rule at Q = 2 against the binary
reveal, and the refinement loop with a genie denoiser against brute-force
joint MAP on a tiny GF(8) code with K = 2."""
import math

import numpy as np
import pytest

import synth
from oracle import denoiser as D
from oracle import gf, metrics, parity, qary
from oracle.schedule import reveal as reveal_bin


def _rand_dists(rng, Q, k, peak=None):
    out = []
    for _ in range(k):
        p = rng.random(Q) ** 4
        if peak is not None:
            p[rng.integers(Q)] += peak
        out.append(p / p.sum())
    return out


@pytest.mark.parametrize("m,deg", [(3, 2), (3, 3), (3, 4), (3, 5)])
def test_check_message_equals_exhaustive_c2v(m, deg):
    rng = np.random.default_rng(m * 10 + deg)
    Q = 1 << m
    p = _rand_dists(rng, Q, deg - 1)
    al = [int(a) for a in rng.integers(1, Q, deg - 1)]
    ao = int(rng.integers(1, Q))
    np.testing.assert_allclose(qary.check_message(p, al, ao, m), gf.check_message_brute(p, al, ao, m), rtol=1e-12)


def test_check_message_equals_the_transform_form_at_q64():
    rng = np.random.default_rng(3)
    p = _rand_dists(rng, 64, 4, peak=50.0)
    al = [int(a) for a in rng.integers(1, 64, 4)]
    np.testing.assert_allclose(qary.check_message(p, al, 37, 6), gf.check_message_wht(p, al, 37, 6),
                               rtol=1e-9, atol=1e-15)


def test_xor_convolution_of_point_masses_and_uniform():
    a = np.zeros(8)
    a[5] = 1.0
    b = np.zeros(8)
    b[3] = 1.0
    out = qary.xor_convolve(a, b)
    assert out[5 ^ 3] == 1.0 and out.sum() == 1.0
    u = np.full(8, 1 / 8)
    np.testing.assert_allclose(qary.xor_convolve(u, _rand_dists(np.random.default_rng(1), 8, 1)[0]), u)


class _Gf2Code:
    """A binary code seen as a GF(2) code: every coefficient 1."""
    def __init__(self, code):
        self.n, self.m = code.n, code.m
        self.row_ptr, self.col_idx = code.row_ptr, code.col_idx
        self.var_ptr, self.var_idx = code.var_ptr, code.var_idx
        self.coef = np.ones(code.col_idx.shape[0], dtype=np.uint8)
        self.q_bits = 1


def test_denoiser_at_q2_equals_the_binary_oracle():
    """Embedding, Module A, layers, projection and Module B at Q = 2 reduce to
    the binary path (the binary lam_min floor set below every input)."""
    cfg = synth.ModelCfg(2, 32, 4, n_max=32)
    w = synth.unpack_weights(synth.make_weights(cfg, 9, bias_std=0.02, ln_std=0.05), cfg)
    code = synth.regular_ldpc(32, seed=1032)
    rng = np.random.default_rng(2)
    X = rng.integers(0, 2, size=(3, 32)).astype(np.uint8)
    X[rng.random((3, 32)) < 0.5] = 2
    p = D.softmax(rng.standard_normal((32, 2)), axis=1)
    ref = D.denoise(X, p, code, w, 2, 4, 0.4, lam_min=1e-300)
    got = qary.denoise_q(X, p, _Gf2Code(code), w, 2, 4, 0.4)
    np.testing.assert_allclose(got["lbar"], ref["lbar"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(got["logits"], ref["logits"], rtol=1e-9, atol=1e-9)


def test_module_b_at_q2_equals_the_binary_logit_bias():
    code = synth.regular_ldpc(64, seed=1064)
    rng = np.random.default_rng(4)
    lbar = rng.standard_normal((2, 64, 2)) * 3
    X = rng.integers(0, 2, size=(2, 64)).astype(np.uint8)
    X[rng.random((2, 64)) < 0.6] = 2
    ref = parity.module_b(lbar, X, code, eta=0.7, lam_max=20.0, lam_min=1e-300)
    got = qary.module_b_q(lbar, X, _Gf2Code(code), eta=0.7, lam_max=20.0)
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("first", [False, True])
def test_reveal_at_q2_equals_the_binary_reveal(first):
    rng = np.random.default_rng(5 + first)
    logits = rng.standard_normal((4, 40, 2))
    X = rng.integers(0, 2, size=(4, 40)).astype(np.uint8)
    X[rng.random((4, 40)) < 0.7] = 2
    Xb, Xq = X.copy(), X.copy()
    ib = reveal_bin(Xb, logits, 9, first)
    iq = qary.reveal_q(Xq, logits, 9, first, 1.0, 2)
    assert ib["selected"] == iq["selected"] and np.array_equal(Xb, Xq)


def test_uncertainty_is_minus_log_max_probability():
    rng = np.random.default_rng(6)
    L = rng.standard_normal((3, 5, 64)) * 4
    for tau in (0.5, 1.0, 2.0):
        e = np.exp(L / tau - (L / tau).max(-1, keepdims=True))
        np.testing.assert_allclose(qary.uncertainty(L, tau), -np.log((e / e.sum(-1, keepdims=True)).max(-1)),
                                   rtol=1e-12, atol=1e-15)


def test_temperature_reorders_sites_only_beyond_two_symbols():
    """Two sites with equal top-two gaps but different tails: at low tau the
    tails vanish and the gaps tie, at high tau the flatter tail loses."""
    L = np.zeros((1, 2, 8))
    L[0, 0] = [3.0, 1.0] + [-8.0] * 6
    L[0, 1] = [3.05, 1.0] + [-0.5] * 6
    hi = qary.uncertainty(L, 4.0)
    lo = qary.uncertainty(L, 0.25)
    assert hi[0, 0] < hi[0, 1] and lo[0, 1] < lo[0, 0]


def _tiny_gf8():
    return synth.qary_ldpc(6, 3, dv=2, dc=3, seed=8)


def test_tiny_gf8_codebook_by_search_matches_the_generator():
    code = _tiny_gf8()
    C = qary.codebook_q(code)
    assert C.shape == (8 ** code.k, 6)
    info = np.stack(np.meshgrid(*[np.arange(8)] * code.k, indexing="ij"), -1).reshape(-1, code.k)
    enc = code.encode(info)
    assert {r.tobytes() for r in C} == {r.tobytes() for r in enc}


def test_genie_refinement_recovers_the_map_set_on_gf8():
    """With exact conditional marginals as the denoiser, the Q-ary refinement
    (uncertainty ranking, first-reveal, linear schedule) ends on the
    brute-force joint-MAP pair whenever it holds >= 0.99 of the posterior."""
    code = _tiny_gf8()
    C = qary.codebook_q(code)
    rng = np.random.default_rng(11)
    checked = 0
    for trial in range(30):
        i, j = rng.choice(C.shape[0], 2, replace=False)
        s2 = [0.15, 0.25, 0.35][trial % 3]
        y = np.zeros((6, 8))
        for l in range(6):
            y[l, C[i, l]] += 1.0
            y[l, C[j, l]] += 1.0
        y += rng.standard_normal((6, 8)) * math.sqrt(s2)
        (a, b), mass = qary.map_pair_q(C, y, s2)
        if mass < 0.99:
            continue
        den = qary.genie_denoiser_q(C, y, s2)
        res = qary.decode_grid_q(2, 6, 8, code, den, T=12)
        assert metrics.same_multiset(res.X, C[[a, b]]), trial
        assert res.row_valid.all()
        checked += 1
    assert checked >= 8


def test_decode_invariants_counts_and_hold_fixed():
    code = _tiny_gf8()
    cfg = synth.ModelCfg(1, 32, 4, q=8, n_max=8)
    w = synth.unpack_weights(synth.make_weights(cfg, 3), cfg)
    S = np.random.default_rng(7).standard_normal((6, 8))
    res = qary.decode_bin_q(S, code, 3, w, 1, 4, T=5, keep=True)
    assert (res.X < 8).all()
    total = 0
    for s in res.steps:
        before = s["X_in"]
        rev = before != 8
        total += len(s["selected"])
        # revealed tokens never change
        nxt = res.steps[s["t"]]["X_in"] if s["t"] < len(res.steps) else res.X
        assert np.array_equal(nxt[rev], before[rev])
    assert total == 3 * 6
    assert [len(s["selected"]) for s in res.steps] == [3, 4, 3, 4, 4]


def test_q_ary_denoiser_is_row_permutation_equivariant():
    code = _tiny_gf8()
    cfg = synth.ModelCfg(2, 32, 4, q=8, n_max=8)
    w = synth.unpack_weights(synth.make_weights(cfg, 4, bias_std=0.02), cfg)
    rng = np.random.default_rng(8)
    X = rng.integers(0, 9, size=(3, 6)).astype(np.uint8)
    p = D.softmax(rng.standard_normal((6, 8)), axis=1)
    perm = [2, 0, 1]
    a = qary.denoise_q(X, p, code, w, 2, 4, 0.5)["logits"]
    b = qary.denoise_q(X[perm], p, code, w, 2, 4, 0.5)["logits"]
    np.testing.assert_allclose(b, a[perm], rtol=1e-12, atol=1e-12)
