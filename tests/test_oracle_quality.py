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
