"""GPU checks of the allocation-free decode (cider_decode_noalloc) against
cider_decode, through the C ABI: bit-identical symbols on two calls in a
row, the second on a smaller bin (the shared scratch keeps the first call's
contents), at BF16 and FP32; a bin too large for the scratch is rejected
before anything runs."""
import numpy as np
import pytest

import synth

from gpu_common import code_handle, code_of, lib, say, torch_cuda, weights_handle

pytestmark = pytest.mark.gpu


def _pair(P, torch, wh, cfg, K, n, T, prec, seed, remask=0):
    code = code_of(n, 1000 + n)
    ch = code_handle(code)
    bins = synth.make_bins(code, K, 1, 3.0, seed=seed)
    y = torch.from_numpy(bins.y[0]).cuda()
    s2 = float(bins.sigma2[0])
    opts = P.cider_opts_default(precision=prec, remask=remask)
    ref = torch.full((K, n), 9, dtype=torch.uint8, device="cuda")
    got = torch.full((K, n), 7, dtype=torch.uint8, device="cuda")
    say(f"noalloc vs decode: K={K} n={n} d={cfg.d} T={T} prec={prec} remask={remask}")
    P.cider_decode(y, s2, ch, K, n, wh, T, ref, opts)
    P.cider_decode_noalloc(y, s2, ch, K, n, wh, T, got, opts)
    torch.cuda.synchronize()
    assert torch.equal(got, ref), f"K={K} n={n}: allocation-free decode differs"
    assert set(np.unique(got.cpu().numpy())) <= {0, 1}


@pytest.mark.parametrize("prec_name", ["bf16", "fp32"])
def test_noalloc_matches_decode_then_smaller_bin(prec_name):
    torch = torch_cuda()
    P = lib()
    prec = P.CIDER_BF16 if prec_name == "bf16" else P.CIDER_FP32
    cfg = synth.ModelCfg(4, 128, 8, n_max=256)
    wh, _ = weights_handle(cfg, seed=12)
    _pair(P, torch, wh, cfg, 8, 256, 16, prec, seed=3)         # first call: 2048 tokens
    _pair(P, torch, wh, cfg, 3, 64, 8, prec, seed=4)           # second, smaller: 192 tokens
    _pair(P, torch, wh, cfg, 4, 128, 16, prec, seed=5, remask=1)


def test_noalloc_rejects_a_bin_beyond_the_scratch():
    torch = torch_cuda()
    P = lib()
    cfg = synth.ModelCfg(1, 384, 12, n_max=1024)
    wh, _ = weights_handle(cfg, seed=15)
    code = code_of(1024, 2024)
    y = torch.zeros(1024, dtype=torch.float32, device="cuda")
    out = torch.zeros(16, 1024, dtype=torch.uint8, device="cuda")
    say("noalloc: K=16 n=1024 d=384 must be rejected")
    with pytest.raises(P.CiderError) as ei:
        P.cider_decode_noalloc(y, 1.0, code_handle(code), 16, 1024, wh, 32, out)
    assert ei.value.status == P.abi.CIDER_EINVAL and "scratch" in str(ei.value)
