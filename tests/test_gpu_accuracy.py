"""Oracle agreement of whole decodes at the c2 workload's size, over the
3072 stored FP64 oracle grids of tests/golden/c2_oracle_grids.npz (written by
tests/golden/make_c2_oracle_grids.py, which calls only the oracle).

A decode is a chain of integer decisions (the reveal cut, each revealed
site's argmax, the first-reveal row choice: refinement loop and
confidence-ranked reveal, method section).  Once the GPU takes one of them
differently from the FP64 oracle the two trajectories part, so whether a bin
can match depends on how close its closest decision is to a tie.  Each stored
bin carries its smallest nonzero decision gap relative to the logits the
decision is made of (a margin difference of two sites over 4 max(1, |L|) of
both, an argmax margin over 2 max(1, |L|)): a relative logit error below it
cannot turn any decision.  Exact zeros are ties between identical user rows,
which carry bit-identical logits in any precision and are broken by index on
both sides.

For each precision the test measures the relative logit error of one
teacher-forced step against the oracle, max |dL| / max(1, |L|), then asserts
that every bin whose smallest relative gap exceeds twice that error is
decoded bit-identically, and reports the match rate over all bins with its
Clopper-Pearson 95% interval.  BF16 runs in the benchmark's launch
configuration (packed batches of 256 bins, graph replay); FP32 is the plain
path, one cider_decode call per bin.
"""
import os

import numpy as np
import pytest

import synth
from oracle.denoiser import denoise
from oracle.evidence import evidence

from gpu_common import code_handle, lib, prec_id, say, torch_cuda, weights_handle

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle_grids.npz")


def clopper_pearson(k, n, alpha=0.05):
    from scipy.stats import beta
    lo = 0.0 if k == 0 else float(beta.ppf(alpha / 2, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - alpha / 2, k + 1, n - k))
    return lo, hi


def _setup():
    g = np.load(GOLD)
    shape = tuple(int(v) for v in g["shape"])
    X = np.unpackbits(g["X_packed"], axis=-1, count=shape[-1]).reshape(shape)
    wl = synth.workload("c2")
    cfg = wl.model
    wh, w = weights_handle(cfg, wl.weight_seed)
    code = synth.regular_ldpc(wl.n, seed=wl.code_seed)
    bins = synth.make_bins(code, wl.K, shape[0], wl.ebn0_db, wl.bin_seed)
    assert float(np.sum(bins.y, dtype=np.float64)) == float(g["y_sum"][0]), "stored grids are for other inputs"
    return wl, cfg, wh, w, code, code_handle(code), bins, X, g["min_rel_gap"]


def _logit_error(prec, wl, cfg, wh, w, code, ch, bins):
    """max |L_gpu - L_oracle| / max(1, |L_oracle|) over teacher-forced steps
    of eight bins at four mask fractions."""
    torch = torch_cuda()
    P = lib()
    opts = P.cider_opts_default(precision=P.CIDER_FP64 if prec == "fp64" else prec_id(prec))
    fdt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(2024)
    K, n = wl.K, wl.n
    err = 0.0
    for b in range(8):
        y, s2 = bins.y[b], float(bins.sigma2[b])
        _, p = evidence(y.astype(np.float64), s2, K)
        for frac in (1.0, 0.75, 0.5, 0.25):
            X = rng.integers(0, 2, size=(K, n)).astype(np.uint8)
            X[rng.random((K, n)) < frac] = 2
            gamma = float(np.float32((X == 2).mean()))
            ref = denoise(X, p, code, w, cfg.n_layers, cfg.heads, gamma)["logits"]
            lg = torch.zeros(K, n, 2, dtype=fdt, device="cuda")
            P.cider_step_debug(torch.from_numpy(X).cuda(), None, torch.from_numpy(y).cuda(), s2, ch, K, n, wh,
                               gamma, 0, 0, opts, out_logits=lg)
            torch.cuda.synchronize()
            g = lg.cpu().numpy().astype(np.float64)
            err = max(err, float(np.max(np.abs(g - ref) / np.maximum(1.0, np.abs(ref)))))
    return err


def _report(name, got, X, rel_gap, err):
    B = X.shape[0]
    same = np.array([np.array_equal(got[b], X[b]) for b in range(B)])
    decidable = rel_gap > 2.0 * err
    sym = float(np.mean(got == X))
    lo, hi = clopper_pearson(int(same.sum()), B)
    dl, _ = clopper_pearson(int(same[decidable].sum()), int(decidable.sum())) if decidable.any() else (0.0, 1.0)
    print(f"  {name}: relative logit error {err:.3e}; bins matching {same.sum()}/{B} = {same.mean():.4f} "
          f"(95% CI {lo:.4f}..{hi:.4f}), symbols {sym:.5f}; decidable (relative gap > {2 * err:.2e}) "
          f"{decidable.sum()}/{B}, "
          f"matching {same[decidable].sum()} (lower bound {dl:.4f}); mismatches with gap above the bound: "
          f"{int((decidable & ~same).sum())}")
    bad = np.nonzero(decidable & ~same)[0]
    assert bad.size == 0, f"{name}: bins {bad[:10].tolist()} decode differently with every relative decision gap above 2x the error"
    return same, decidable


def test_c2_bf16_batched_agreement_over_stored_oracle_grids():
    torch = torch_cuda()
    P = lib()
    wl, cfg, wh, w, code, ch, bins, X, rel_gap = _setup()
    B, K, n = X.shape
    err = _logit_error("bf16", wl, cfg, wh, w, code, ch, bins)
    say(f"c2 BF16 batched over {B} stored oracle grids, 256 bins per call, graph replay")
    opts = P.cider_opts_default(precision=P.CIDER_BF16, use_graph=1)
    y = torch.from_numpy(bins.y).cuda()
    out = torch.full((B, K, n), 9, dtype=torch.uint8, device="cuda")
    for b0 in range(0, B, 256):
        P.cider_decode_batch([{"y": y[b], "sigma2": float(bins.sigma2[b]), "code": ch, "K": K, "n": n,
                               "out_symbols": out[b]} for b in range(b0, min(B, b0 + 256))], wh, wl.T, opts)
    torch.cuda.synchronize()
    _report("bf16 batched", out.cpu().numpy(), X, rel_gap, err)


def test_c2_fp32_plain_agreement_over_stored_oracle_grids():
    torch = torch_cuda()
    P = lib()
    wl, cfg, wh, w, code, ch, bins, X, rel_gap = _setup()
    B, K, n = X.shape
    err = _logit_error("fp32", wl, cfg, wh, w, code, ch, bins)
    say(f"c2 FP32 plain over {B} stored oracle grids, one call per bin, eager launches")
    opts = P.cider_opts_default(precision=P.CIDER_FP32, use_graph=0)
    y = torch.from_numpy(bins.y).cuda()
    out = torch.full((B, K, n), 9, dtype=torch.uint8, device="cuda")
    for b in range(B):
        P.cider_decode(y[b], float(bins.sigma2[b]), ch, K, n, wh, wl.T, out[b], opts)
        if b % 512 == 511:
            torch.cuda.synchronize()
            say(f"  {b + 1}/{B} bins decoded")
    torch.cuda.synchronize()
    same, decidable = _report("fp32 plain", out.cpu().numpy(), X, rel_gap, err)
    assert decidable.sum() >= B // 2, "FP32 should resolve most bins' decisions"


def test_c2_fp64_batched_agreement_over_stored_oracle_grids():
    """The FP64 mode in the benchmark's launch configuration: every stored bin
    is decidable at its error, and every one must equal the oracle's grid."""
    torch = torch_cuda()
    P = lib()
    wl, cfg, wh, w, code, ch, bins, X, rel_gap = _setup()
    B, K, n = X.shape
    err = _logit_error("fp64", wl, cfg, wh, w, code, ch, bins)
    say(f"c2 FP64 batched over {B} stored oracle grids, 256 bins per call, graph replay")
    opts = P.cider_opts_default(precision=P.CIDER_FP64, use_graph=1)
    y = torch.from_numpy(bins.y).cuda()
    out = torch.full((B, K, n), 9, dtype=torch.uint8, device="cuda")
    for b0 in range(0, B, 256):
        P.cider_decode_batch([{"y": y[b], "sigma2": float(bins.sigma2[b]), "code": ch, "K": K, "n": n,
                               "out_symbols": out[b]} for b in range(b0, min(B, b0 + 256))], wh, wl.T, opts)
    torch.cuda.synchronize()
    same, decidable = _report("fp64 batched", out.cpu().numpy(), X, rel_gap, err)
    assert decidable.all() and same.all()
