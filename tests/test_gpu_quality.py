"""GPU parity of the PRISM-style quality head as the remask criterion
(Appendix, PRISM-style quality head and remasking plug-in), through the C ABI.

- FP32 free-running decodes with the head against the oracle's decode with the
  same head (row confidence = mean token omega, thresholds phi_s after pass s):
  the decoded grids are equal on every bin whose reveal and threshold decisions
  the oracle takes with a safe margin, and some of those bins remask only part
  of their rows;
- the control flow at the extremes, bit for bit against the library's other
  paths: a head that is always sure (b2 = +30) never remasks, so the decode
  equals the one without remasking; a head that always doubts (b2 = -30)
  remasks every row after every stage, as the fixed criterion does with a
  threshold above 1 and as many rounds; in FP32, BF16 (fused blocks) and FP8;
- options that do not describe a head are rejected before any launch.
"""
import numpy as np
import pytest

import synth
from oracle import quality as Qh
from oracle.decode import DecodeOpts, decode_bin

from gpu_common import code_handle, code_of, lib, prec_id, say, torch_cuda, weights_handle

pytestmark = pytest.mark.gpu

MIN_GAP = 2e-5     # the FP32 decodes' decision margin


def _setup(d, h, n, K, B, L=2, ln_std=0.05, bias_std=0.02):
    torch_cuda()      # torch's device runtime first, before the library's own HIP calls
    cfg = synth.ModelCfg(L, d, h, n_max=max(n, 64))
    wh, w = weights_handle(cfg, seed=31 + d, bias_std=bias_std, ln_std=ln_std)
    code = code_of(n, 1000 + n)
    bins = synth.make_bins(code, K, B, [2.0, 4.0, 6.0], seed=77 + K + n)
    return cfg, wh, w, code, code_handle(code), bins


def _decode(wh, ch, bins, K, n, T, opts):
    torch = torch_cuda()
    P = lib()
    B = bins.y.shape[0]
    out = torch.full((B, K, n), 9, dtype=torch.uint8, device="cuda")
    valid = torch.zeros(B, K, dtype=torch.uint8, device="cuda")
    y = torch.from_numpy(np.ascontiguousarray(bins.y)).cuda()
    P.cider_decode_batch([{"y": y[b], "sigma2": float(bins.sigma2[b]), "code": ch, "K": K, "n": n,
                           "out_symbols": out[b], "out_row_valid": valid[b]} for b in range(B)], wh, T, opts)
    torch.cuda.synchronize()
    return out.cpu().numpy(), valid.cpu().numpy()


def _head(d, H, std, b2):
    torch = torch_cuda()
    psi = synth.make_quality_head(d, H, seed=5, std=std, b2=b2)
    return psi, torch.from_numpy(psi).cuda()


def _gaps(res):
    out = []
    for s in res.steps:
        out += [s["gaps"][k] for k in ("cut", "sel", "slot")]
    out += [f["gap_q"] for f in res.finals]
    return out


def test_quality_head_fp32_matches_oracle():
    P = lib()
    K, n, L, d, h, T, B, H = 4, 32, 2, 64, 4, 8, 12, 16
    cfg, wh, w, code, ch, bins = _setup(d, h, n, K, B, L)
    psi, dpsi = _head(d, H, std=1.0, b2=1.5)
    head = Qh.unpack_head(psi, d, H)

    def rc(out):
        return Qh.row_confidence(out["z"], w, head)

    # phi_0 in the widest gap of the middle half of the first final pass's row
    # confidences (that pass does not depend on phi), so that it splits rows
    first = np.sort(np.concatenate([
        decode_bin(bins.y[b], float(bins.sigma2[b]), code, K, w, L, h, T,
                   DecodeOpts(remask=True, row_conf=rc, phi=(0.0,))).finals[0]["q"] for b in range(B)]))
    lo, hi = len(first) // 4, 3 * len(first) // 4
    i = lo + int(np.argmax(np.diff(first[lo:hi + 1])))
    phi = (float(0.5 * (first[i] + first[i + 1])), 0.90, 0.85)
    say(f"quality head FP32 K={K} n={n} L={L} d={d} H={H} B={B} phi={phi}")
    opts = P.cider_opts_default(precision=prec_id("fp32"), remask=1, qhead=dpsi, qhead_hidden=H,
                                remask_stages=3, remask_phi=phi)
    Xg, Vg = _decode(wh, ch, bins, K, n, T, opts)
    oo = DecodeOpts(remask=True, row_conf=rc, phi=phi)
    safe = match = partial = 0
    for b in range(B):
        res = decode_bin(bins.y[b], float(bins.sigma2[b]), code, K, w, L, h, T, oo)
        same = np.array_equal(Xg[b], res.X)
        if all(g > MIN_GAP or g == 0.0 for g in _gaps(res)):
            safe += 1
            assert same, f"bin {b}: decidable bin decoded differently"
            assert np.array_equal(Vg[b], res.row_valid)
            partial += int(0 < res.finals[0]["low"].sum() < K)
        match += same
    print(f"  exact grid match {match}/{B}, decidable {safe}/{B}, decidable with part of the rows remasked {partial}")
    assert safe >= B // 3 and partial >= 1


@pytest.mark.parametrize("prec,d,h", [("fp32", 64, 4), ("bf16", 128, 8), ("fp8", 128, 8)])
def test_quality_head_extremes(prec, d, h):
    P = lib()
    K, n, T, B, H = 4, 64, 8, 6, 8
    cfg, wh, w, code, ch, bins = _setup(d, h, n, K, B)
    say(f"quality head extremes {prec} K={K} n={n} d={d} H={H}")
    _, sure = _head(d, H, std=0.05, b2=30.0)
    _, doubt = _head(d, H, std=0.05, b2=-30.0)
    base = dict(precision=prec_id(prec))
    plain = _decode(wh, ch, bins, K, n, T, P.cider_opts_default(remask=0, **base))
    got = _decode(wh, ch, bins, K, n, T, P.cider_opts_default(remask=1, qhead=sure, qhead_hidden=H, **base))
    assert np.array_equal(got[0], plain[0]) and np.array_equal(got[1], plain[1])
    for stages in (1, 3):
        fixed = _decode(wh, ch, bins, K, n, T, P.cider_opts_default(remask=1, remask_thr=2.0,
                                                                    remask_max_rounds=stages, **base))
        got = _decode(wh, ch, bins, K, n, T, P.cider_opts_default(remask=1, qhead=doubt, qhead_hidden=H,
                                                                  remask_stages=stages, **base))
        assert np.array_equal(got[0], fixed[0]) and np.array_equal(got[1], fixed[1]), stages


def test_quality_head_options_rejected():
    P = lib()
    K, n, T, B, H = 2, 32, 4, 1, 8
    cfg, wh, w, code, ch, bins = _setup(64, 4, n, K, B)
    _, psi = _head(64, H, std=0.05, b2=0.0)
    bad = [dict(remask=0, qhead=psi, qhead_hidden=H), dict(remask=1, qhead=psi, qhead_hidden=0),
           dict(remask=1, qhead=psi, qhead_hidden=65), dict(remask=1, qhead=psi, qhead_hidden=H, remask_stages=0),
           dict(remask=1, qhead=psi, qhead_hidden=H, remask_stages=5),
           dict(remask=1, qhead=psi, qhead_hidden=H, remask_phi=(float("nan"), 0.9, 0.85))]
    for kw in bad:
        with pytest.raises(P.CiderError) as e:
            _decode(wh, ch, bins, K, n, T, P.cider_opts_default(precision=prec_id("fp32"), **kw))
        assert e.value.status == P.abi.CIDER_EINVAL, kw
