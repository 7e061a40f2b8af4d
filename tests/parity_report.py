"""Per-precision agreement with the FP64 oracle (GPU; not collected by pytest).

Teacher-forced: logits of one step on chosen grids (mask fractions 1, 0.5,
0), max |gpu - oracle| / max(1, |oracle|), for workload-shaped models (c1,
c2, and the c3 and c5 widths at two layers).  Free-running: whole decodes of
seeded c1 / c2 bins, the fraction of bins whose grid equals the oracle's and
the fraction of symbols that agree.

    python tests/parity_report.py      # writes gpurun_out/parity_report.json
"""
import sys, os, json
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT); sys.path.insert(0, os.path.join(ROOT, "tests"))
import numpy as np, torch, synth
from gpu_common import code_handle, code_of, lib, rel_err, weights_handle, prec_id
from oracle.denoiser import denoise
from oracle.evidence import evidence
from oracle.decode import DecodeOpts, decode_bin
P = lib()
out = {"teacher_forced": [], "free_running": []}
for (K, n, L, d, h, name) in [(2, 32, 2, 64, 4, "c1"), (4, 128, 4, 128, 8, "c2"), (8, 256, 2, 256, 8, "c3-like L=2"),
                               (4, 256, 2, 384, 12, "c5-like L=2")]:
    cfg = synth.ModelCfg(L, d, h, n_max=max(n, 64))
    wh, w = weights_handle(cfg, seed=12)
    code = code_of(n, 1000 + n); ch = code_handle(code)
    b = synth.make_bins(code, K, 1, 4.0, seed=9)
    y, s2 = b.y[0], float(b.sigma2[0])
    _, p = evidence(y.astype(np.float64), s2, K)
    rng = np.random.default_rng(1)
    for frac in (1.0, 0.5, 0.0):
        X = rng.integers(0, 2, size=(K, n)).astype(np.uint8); X[rng.random((K, n)) < frac] = 2
        g = float((X == 2).mean())
        ref = denoise(X, p, code, w, L, h, g)
        for prec in ("fp32", "bf16", "fp8"):
            if prec == "fp8" and d % 128: continue
            lg = torch.zeros(K, n, 2, dtype=torch.float32, device="cuda")
            lb = torch.zeros_like(lg)
            P.cider_step_debug(torch.from_numpy(X).cuda(), None, torch.from_numpy(y).cuda(), s2, ch, K, n, wh, g, 0, 0,
                               P.cider_opts_default(precision=prec_id(prec)), out_lbar=lb, out_logits=lg)
            torch.cuda.synchronize()
            e = rel_err(lg.cpu().numpy(), ref["logits"]); eb = rel_err(lb.cpu().numpy(), ref["lbar"])
            out["teacher_forced"].append(dict(case=name, mask=frac, prec=prec, logits_err=e, lbar_err=eb))
            print(name, frac, prec, f"{e:.2e} {eb:.2e}", flush=True)
# free running on c1 and c2 shapes
for (K, n, L, d, h, T, B, name) in [(2, 32, 2, 64, 4, 8, 32, "c1"), (4, 128, 4, 128, 8, 16, 16, "c2")]:
    cfg = synth.ModelCfg(L, d, h, n_max=max(n, 64))
    blob = synth.make_weights(cfg, 11 if name == "c1" else 12)
    w = synth.unpack_weights(blob, cfg)
    wh = P.Weights(P.make_cfg(L, d, h, 4, cfg.n_max), blob)
    code = code_of(n, 1032 if name == "c1" else 1128); ch = code_handle(code)
    bins = synth.make_bins(code, K, B, [4.0] if name == "c1" else [2.0, 4.0, 6.0], 101 if name == "c1" else 102)
    refs = [decode_bin(bins.y[i], float(bins.sigma2[i]), code, K, w, L, h, T, DecodeOpts()).X for i in range(B)]
    for prec in ("fp32", "bf16", "fp8"):
        if prec == "fp8" and d % 128: continue
        o = torch.zeros(B, K, n, dtype=torch.uint8, device="cuda")
        yy = torch.from_numpy(bins.y).cuda()
        P.cider_decode_batch([{"y": yy[i], "sigma2": float(bins.sigma2[i]), "code": ch, "K": K, "n": n, "out_symbols": o[i]}
                              for i in range(B)], wh, T, P.cider_opts_default(precision=prec_id(prec)))
        torch.cuda.synchronize()
        g = o.cpu().numpy()
        bm = float(np.mean([np.array_equal(g[i], refs[i]) for i in range(B)]))
        sm = float(np.mean([np.mean(g[i] == refs[i]) for i in range(B)]))
        out["free_running"].append(dict(case=name, prec=prec, bins=B, bin_match=bm, symbol_match=sm))
        print(name, prec, "bins", bm, "symbols", round(sm, 4), flush=True)
os.makedirs("gpurun_out", exist_ok=True)
json.dump(out, open("gpurun_out/parity_report.json", "w"), indent=1)
