"""GPU parity of the GF(Q) decode -- the paper's main setting: Q-ary LDPC
codes over GF(64) with K = 2 users, evidence from the slot-wise AMP-MMSE
detector -- against the FP64 oracle, through the C ABI.

Inputs are the paper's Tiny scale (dataset scales and model sizing tables:
L = 12 slots, P = 8 checks, rate 1/3; D = 128, 4 layers, 4 heads, T = 12
steps) with a (2,3)-regular GF(64) code and seeded weights.  Each frame's
slots go through the GPU AMP-MMSE detector (cider_amp_evidence), and the
decoder and the oracle both read that evidence, so the tests cover the
detector -> decoder chain:
- teacher-forced steps: logits before and after Module B within the FP32
  (1e-5) and BF16 (2e-2) tolerances relative to max(1, |oracle|); the FP32
  reveal equals the oracle's where its decisions are clear of ties, the BF16
  reveal is a valid one;
- free-running FP32 decodes equal the oracle's on every bin whose decisions
  are clear of ties, and every row-valid flag equals H x = 0 over GF(64)
  recomputed from the grid;
- a packed batch of bins of different K and code length equals each bin
  decoded alone, bit for bit (symbols and logits).
"""
import numpy as np
import pytest

import synth
from oracle import qary
from oracle.denoiser import softmax

from gpu_common import TOL, lib, rel_err, say, torch_cuda

pytestmark = pytest.mark.gpu

Q_BITS, Q = 6, 64
N_S, AMP_ITERS = 24, 20


def _model(L=4, d=128, h=4, seed=21):
    P = lib()
    cfg = synth.ModelCfg(L, d, h, q=Q, n_max=64)
    blob = synth.make_weights(cfg, seed, bias_std=0.02, ln_std=0.05)
    return cfg, P.Weights(P.make_cfg(L, d, h, 4, 64, Q), blob), synth.unpack_weights(blob, cfg)


_codes = {}


def _code(n):
    P = lib()
    if n not in _codes:
        c = synth.qary_ldpc(n, Q_BITS, dv=2, dc=3, seed=2000 + n)
        _codes[n] = (c, P.CodeQ(c.n, c.m, c.row_ptr, c.col_idx, c.coef, Q_BITS))
    return _codes[n]


def _evidence(code, K, frames, ebn0, seed):
    """GPU AMP-MMSE evidence of coded frames: device [frames * n][Q] and its host copy."""
    torch = torch_cuda()
    P = lib()
    fr = synth.make_qary_frames(code, K, frames, N_S, ebn0, seed)
    sl = fr.slots
    S = torch.empty(sl.y.shape[0], Q, dtype=torch.float32, device="cuda")
    P.cider_amp_evidence(torch.from_numpy(sl.y).cuda(), torch.from_numpy(sl.rows).cuda(), sl.y.shape[0], N_S, Q,
                         K / Q, float(sl.p_sym[0]), AMP_ITERS, S)
    torch.cuda.synchronize()
    return fr, S, S.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_teacher_forced_step_at_tiny_scale(prec):
    torch = torch_cuda()
    P = lib()
    cfg, wh, w = _model()
    code, ch = _code(12)
    K, n = 2, 12
    fr, S, S_h = _evidence(code, K, 1, 4.0, seed=5)
    p = softmax(S_h, axis=1)
    opts = P.cider_opts_default(precision=P.CIDER_FP32 if prec == "fp32" else P.CIDER_BF16)
    tol = TOL[prec]
    rng = np.random.default_rng(3)
    for frac, first in ((1.0, 1), (0.5, 0), (0.15, 0)):
        X = rng.integers(0, Q, size=(K, n)).astype(np.uint8)
        X[rng.random((K, n)) < frac] = Q
        gamma = float((X == Q).mean())
        say(f"GF(64) teacher-forced {prec} K={K} n={n} mask={frac} first={first}")
        ref = qary.denoise_q(X, p, code, w, cfg.n_layers, cfg.heads, gamma)
        lbar = torch.zeros(K, n, Q, dtype=torch.float32, device="cuda")
        logits = torch.zeros_like(lbar)
        Xo = torch.zeros(K, n, dtype=torch.uint8, device="cuda")
        ncand = int((X == Q).any(axis=0).sum()) if first else int((X == Q).sum())
        r = max(1, ncand // 3)
        P.cider_step_debug_q(torch.from_numpy(X).cuda(), Xo, S[:n], ch, K, n, wh, gamma, r, first, opts,
                             out_lbar=lbar, out_logits=logits)
        torch.cuda.synchronize()
        e_lbar = rel_err(lbar.cpu().numpy(), ref["lbar"])
        e_log = rel_err(logits.cpu().numpy(), ref["logits"])
        print(f"  err lbar={e_lbar:.2e} logits={e_log:.2e}")
        assert e_lbar <= tol and e_log <= tol, (e_lbar, e_log)
        got = Xo.cpu().numpy()
        changed = got != X
        assert np.all(X[changed] == Q) and changed.sum() == min(r, ncand) and got.max() <= Q
        Xr = X.copy()
        info = qary.reveal_q(Xr, ref["logits"], r, bool(first), 1.0, Q)
        if prec == "fp32" and min(info["gaps"]["cut"], info["gaps"]["slot"], info["gaps"]["sel"]) > 1e-4:
            assert np.array_equal(got, Xr), "FP32 reveal differs from the oracle's"


def _free(K, frames, ebn0, seed, T=12):
    torch = torch_cuda()
    P = lib()
    cfg, wh, w = _model()
    code, ch = _code(12)
    n = code.n
    fr, S, S_h = _evidence(code, K, frames, ebn0, seed)
    out = torch.full((frames, K, n), 99, dtype=torch.uint8, device="cuda")
    valid = torch.zeros(frames, K, dtype=torch.uint8, device="cuda")
    opts = P.cider_opts_default(precision=P.CIDER_FP32, use_graph=1)
    say(f"GF(64) free-running FP32: {frames} frames, K={K}, n={n}, T={T}, packed")
    P.cider_decode_q_batch([{"S": S[f * n:(f + 1) * n], "code": ch, "K": K, "n": n, "out_symbols": out[f],
                             "out_row_valid": valid[f]} for f in range(frames)], wh, T, opts)
    torch.cuda.synchronize()
    X, V = out.cpu().numpy(), valid.cpu().numpy()
    match = safe = 0
    for f in range(frames):
        assert X[f].max() < Q
        assert np.array_equal(V[f], qary.gf_syndrome_ok(X[f], code)), f"frame {f}: row-valid flags"
        res = qary.decode_bin_q(S_h[f * n:(f + 1) * n], code, K, w, cfg.n_layers, cfg.heads, T)
        gaps = [s["gaps"][k] for s in res.steps for k in ("cut", "sel", "slot")]
        same = np.array_equal(X[f], res.X)
        if min(gaps) > 1e-4:
            safe += 1
            assert same, f"frame {f}: decoded differently although every decision is clear of ties"
        match += same
    print(f"  exact grid match {match}/{frames}, decidable {safe}/{frames}")
    return match, safe


def test_free_running_fp32_tiny_matches_oracle():
    match, safe = _free(2, 16, 4.0, seed=11)
    assert safe >= 4


def test_free_running_fp32_more_users_and_cosine_free():
    match, safe = _free(3, 8, 6.0, seed=12, T=9)
    assert safe >= 2


def test_packed_batch_equals_bins_alone_bitwise():
    torch = torch_cuda()
    P = lib()
    cfg, wh, w = _model()
    items = []
    for i, (K, n) in enumerate([(2, 12), (1, 18), (3, 12), (5, 18)]):
        code, ch = _code(n)
        fr, S, _ = _evidence(code, K, 1, 3.0 + i, seed=40 + i)
        items.append((K, n, ch, S))
    opts = P.cider_opts_default(precision=P.CIDER_BF16, use_graph=1)

    def run(sel):
        outs = {i: (torch.full((items[i][0], items[i][1]), 99, dtype=torch.uint8, device="cuda"),
                    torch.zeros(items[i][0], items[i][1], Q, dtype=torch.float32, device="cuda")) for i in sel}
        P.cider_decode_q_batch([{"S": items[i][3], "code": items[i][2], "K": items[i][0], "n": items[i][1],
                                 "out_symbols": outs[i][0], "out_logits": outs[i][1]} for i in sel], wh, 12, opts)
        torch.cuda.synchronize()
        return outs

    say("GF(64) packed batch vs alone, BF16, graph replay")
    mixed = run(list(range(len(items))))
    for i in range(len(items)):
        alone = run([i])[i]
        assert torch.equal(alone[0], mixed[i][0]) and torch.equal(alone[1], mixed[i][1]), f"bin {i}"


def test_gf_path_rejects_binary_mixups():
    torch = torch_cuda()
    P = lib()
    cfg, wh, w = _model(L=1)
    code, ch = _code(12)
    S = torch.zeros(12, Q, dtype=torch.float32, device="cuda")
    out = torch.zeros(2, 12, dtype=torch.uint8, device="cuda")
    say("GF(64) argument checks")
    with pytest.raises(P.CiderError) as e:                          # binary entry point, GF(64) weights
        P.cider_decode(S[:, 0].contiguous(), 1.0, ch, 2, 12, wh, 4, out)
    assert e.value.status == P.abi.CIDER_EINVAL
    with pytest.raises(P.CiderError) as e:                          # remasking is binary only
        P.cider_decode_q_batch([{"S": S, "code": ch, "K": 2, "n": 12, "out_symbols": out}], wh, 4,
                               P.cider_opts_default(remask=1))
    assert e.value.status == P.abi.CIDER_EUNSUPPORTED
