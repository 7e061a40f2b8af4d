"""Pins of the PRISM-style quality head and the multi-threshold remask rule
in the oracle (Appendix, PRISM-style quality head and remasking plug-in)."""
import math

import numpy as np

import synth
from oracle import quality as Qh
from oracle.decode import DecodeOpts, decode_bin


def _model(d=64):
    cfg = synth.ModelCfg(1, d, 4, n_max=64)
    return cfg, synth.unpack_weights(synth.make_weights(cfg, 5, bias_std=0.02, ln_std=0.05), cfg)


def test_zero_first_layer_gives_the_closed_form():
    cfg, w = _model()
    H = 8
    psi = synth.make_quality_head(cfg.d, H, seed=1).astype(np.float64)
    psi[:H * cfg.d + H] = 0.0                     # W1 = 0, b1 = 0: the hidden LayerNorm sees a constant
    head = Qh.unpack_head(psi, cfg.d, H)
    Z = np.random.default_rng(0).standard_normal((2, 5, cfg.d))
    gel = [0.5 * b * (1 + math.erf(b / math.sqrt(2))) for b in head["b"]]
    want = 1 / (1 + math.exp(-(float(head["b2"]) + sum(a * c for a, c in zip(head["w2"], gel)))))
    np.testing.assert_allclose(Qh.token_quality(Z, w, head), want, rtol=1e-12)


def test_head_reads_the_normalised_latent():
    """LN_f makes omega blind to a shift of every feature and to a scaling."""
    cfg, w = _model()
    head = Qh.unpack_head(synth.make_quality_head(cfg.d, 16, seed=2), cfg.d, 16)
    Z = np.random.default_rng(1).standard_normal((3, 7, cfg.d))
    base = Qh.token_quality(Z, w, head)
    np.testing.assert_allclose(Qh.token_quality(Z + 3.7, w, head), base, rtol=1e-9)
    np.testing.assert_allclose(Qh.token_quality(Z * 50.0, w, head), base, rtol=1e-6)
    assert np.all((base > 0) & (base < 1))


def _decode(b2, phi):
    cfg, w = _model()
    code = synth.regular_ldpc(32, seed=1032)
    bins = synth.make_bins(code, 2, 1, 4.0, seed=9)
    H = 8
    psi = synth.make_quality_head(cfg.d, H, seed=3, b2=b2)
    head = Qh.unpack_head(psi, cfg.d, H)
    opts = DecodeOpts(remask=True, row_conf=lambda out: Qh.row_confidence(out["z"], w, head), phi=phi)
    return decode_bin(bins.y[0], float(bins.sigma2[0]), code, 2, w, 1, 4, 6, opts, keep=True)


def test_confident_head_never_remasks():
    res = _decode(30.0, (0.96, 0.90, 0.85))
    assert res.rounds == 0 and len(res.finals) == 1 and not res.finals[0]["low"].any()


def test_doubtful_head_uses_every_stage_with_every_row():
    phi = (0.96, 0.90, 0.85)
    res = _decode(-30.0, phi)
    assert res.rounds == len(phi) and len(res.finals) == len(phi) + 1
    assert all(f["low"].all() for f in res.finals[:-1])
    # each remask pass over all K rows runs T_rm = T = 6 steps after the initial 6
    assert len(res.steps) == 6 * (1 + len(phi))


def _head_with(d, H, seed, w1_scale, b1_std=0.3, ln_std=0.4):
    """A head whose hidden layer is live: nonzero W1 and b1, LN_H gain away
    from 1 and bias away from 0."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H, d)) * w1_scale
    b1 = rng.standard_normal(H) * b1_std * w1_scale
    g = 1.0 + rng.standard_normal(H) * ln_std
    b = rng.standard_normal(H) * ln_std
    w2 = rng.standard_normal(H) * 0.7
    psi = np.concatenate([W1.ravel(), b1, g, b, w2, [0.3]])
    return Qh.unpack_head(psi, d, H)


def _torch_quality(Z, w, head):
    """The head as a composition of torch float64 modules: LayerNorm over d
    (LN_f), Linear d -> H, LayerNorm over H, exact GELU, Linear H -> 1, sigmoid."""
    import torch
    F = torch.nn.functional
    t = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64)
    d = Z.shape[-1]
    H = head["W1"].shape[0]
    zhat = F.layer_norm(t(Z), (d,), t(w["lnf_g"]), t(w["lnf_b"]), eps=1e-5)
    h = F.linear(zhat, t(head["W1"]), t(head["b1"]))
    h = F.gelu(F.layer_norm(h, (H,), t(head["g"]), t(head["b"]), eps=1e-5), approximate="none")
    return torch.sigmoid(F.linear(h, t(head["w2"])[None, :], t(np.atleast_1d(head["b2"])))[..., 0]).numpy()


def test_hidden_layer_matches_a_torch_fp64_composition():
    """Nonzero W1 and b1, LN_H gain and bias; H != d and H == d both, and a
    small-variance hidden layer where the LayerNorm epsilon is visible."""
    cfg, w = _model()
    Z = np.random.default_rng(4).standard_normal((3, 9, cfg.d))
    for H, scale in ((16, 0.1), (cfg.d, 0.1), (24, 2e-3)):
        head = _head_with(cfg.d, H, seed=H, w1_scale=scale)
        got = Qh.token_quality(Z, w, head)
        np.testing.assert_allclose(got, _torch_quality(Z, w, head), rtol=1e-12, atol=1e-14)
        assert np.ptp(got) > 1e-3, "the hidden layer must move omega"


def test_rank_one_first_layer_gives_a_closed_form():
    """W1 = c s^T with c of zero mean and unit variance over the H hidden units
    and b1 = 0: the hidden pre-activation of a token is u * c with the scalar
    u = s . LN_f(z), so LN over H gives c * u / sqrt(u^2 + eps) whatever the
    token; omega follows in closed form.  A LayerNorm over the wrong axis, a
    wrong epsilon or W1 taken transposed all break it."""
    cfg, w = _model()
    H = cfg.d                                     # square, so a transposed W1 still runs
    rng = np.random.default_rng(7)
    c = rng.standard_normal(H)
    c = (c - c.mean()) / c.std()
    s = rng.standard_normal(cfg.d) * 1e-3         # u^2 comparable with eps
    head = _head_with(cfg.d, H, seed=8, w1_scale=1.0)
    head["W1"] = np.outer(c, s)
    head["b1"] = np.zeros(H)
    Z = np.random.default_rng(9).standard_normal((2, 6, cfg.d))
    mu = Z.mean(-1, keepdims=True)
    zhat = (Z - mu) / np.sqrt(((Z - mu) ** 2).mean(-1, keepdims=True) + 1e-5) * w["lnf_g"] + w["lnf_b"]
    want = np.empty(Z.shape[:2])
    for k in range(Z.shape[0]):
        for l in range(Z.shape[1]):
            u = float(s @ zhat[k, l])
            acc = float(head["b2"])
            for j in range(H):
                x = head["g"][j] * c[j] * u / math.sqrt(u * u + 1e-5) + head["b"][j]
                acc += head["w2"][j] * 0.5 * x * (1.0 + math.erf(x / math.sqrt(2.0)))
            want[k, l] = 1.0 / (1.0 + math.exp(-acc))
    np.testing.assert_allclose(Qh.token_quality(Z, w, head), want, rtol=1e-11)
    assert np.ptp(want) > 1e-2
