"""Throughput benchmark of the CIDER refinement path on one MI355X.

One benchmark step = one complete decode (all refinement steps, final pass)
of a batch of synthetic bins through cider_decode_batch.  Default workload
(c2): K=4 users, binary (3,6)-regular LDPC n=128, Eb/N0 cycling {2,4,6} dB,
denoiser L=4 d=128 h=8 with seeded N(0, 0.02) weights, T=16, 256 bins per
batch, BF16 operands with FP32 accumulation.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "decoded bins/sec + p99 latency, BF16 batched vs FP32 plain, >=99.9% oracle symbol match"
PEAK = {"bf16": 2500.0, "fp32": 157.3, "fp8": 5000.0}   # dense TFLOP/s, MI355X published
HBM_PEAK = 8000.0                                        # GB/s


def _oracle_worker(args):
    """CPU baseline task: decode one bin with the FP64 oracle (single thread)."""
    name, b = args
    import synth
    from oracle.decode import DecodeOpts, decode_bin
    wl = synth.workload(name)
    code = synth.regular_ldpc(wl.n, seed=wl.code_seed)
    bins = synth.make_bins(code, wl.K, wl.batch, wl.ebn0_db, wl.bin_seed)
    w = synth.unpack_weights(synth.make_weights(wl.model, wl.weight_seed), wl.model)
    t0 = time.perf_counter()
    res = decode_bin(bins.y[b], float(bins.sigma2[b]), code, wl.K, w, wl.model.n_layers, wl.model.heads, wl.T,
                     DecodeOpts(remask=wl.remask, remask_thr=wl.remask_thr, remask_max_rounds=wl.remask_max_rounds))
    gaps = [g for s in res.steps for g in s["gaps"].values()] + [f["gap_q"] for f in res.finals]
    return b, res.X, time.perf_counter() - t0, min([g for g in gaps if g > 0] + [float("inf")])


def cpu_baseline(name: str, n_bins: int, workers: int):
    import multiprocessing as mp
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        out = pool.map(_oracle_worker, [(name, b) for b in range(n_bins)])
    wall = time.perf_counter() - t0
    return out, wall


def algorithmic(wl, es: int):
    """Per token and per forward: model FLOP, and FLOP / algorithmic HBM bytes
    of each kernel role (es = bytes per element of the compute type)."""
    d, L, F = wl.model.d, wl.model.n_layers, wl.model.d_ff
    n, K = wl.n, wl.K
    per_tok = L * (32 * d * d + 4 * n * d + 4 * K * d) + 6 * d * d + 12 * d
    flop = {
        "gemm_gate1": 2 * d * 2 * d, "gemm_gate2": 2 * d * d,
        "gemm_qkv_row": 2 * d * 3 * d, "gemm_o_row": 2 * d * d,
        "gemm_qkv_user": 2 * d * 3 * d, "gemm_o_user": 2 * d * d,
        "gemm_mlp_up": 2 * d * F, "gemm_mlp_down": 2 * F * d,
        "attn_row": 4 * n * d, "attn_user": 4 * K * d,
    }
    # bytes each kernel must move at minimum (inputs read once, outputs written once);
    # residual updates read and write the FP32 stream and, with the next LayerNorm
    # fused, also write its compute-type copy
    byt = {
        "gemm_gate1": (2 * d + d) * es, "gemm_gate2": d * es + 3 * 4 * d + d * es,
        "gemm_qkv_row": (d + 3 * d) * es, "gemm_qkv_user": (d + 3 * d) * es,
        "gemm_o_row": d * es + 8 * d + d * es, "gemm_o_user": d * es + 8 * d + d * es,
        "gemm_mlp_up": (d + F) * es, "gemm_mlp_down": F * es + 8 * d + d * es,
        "attn_row": (3 * d + d) * es, "attn_user": (3 * d + d) * es,
        "layernorm": 4 * d + d * es,
    }
    return per_tok, flop, byt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--cpu-bins", type=int, default=16)
    ap.add_argument("--plain-bins", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              "bins are independent, so N GPUs would each run this engine on a disjoint bin stream.",
              file=sys.stderr)
        sys.exit(2)

    import synth
    wl = synth.workload(args.workload)
    if wl.ragged_K is not None:
        raise SystemExit("bench.py times the fixed-shape workloads c1..c3")

    # ---- CPU baseline first, before the GPU is initialised (spawned workers)
    cpu = None
    oracle_out = {}
    if not args.no_cpu:
        workers = max(1, min(args.cpu_bins, os.cpu_count() or 1, 16))
        print(f"[bench] oracle cpu baseline: {args.cpu_bins} bins on {workers} workers", file=sys.stderr, flush=True)
        res, wall = cpu_baseline(args.workload, args.cpu_bins, workers)
        for b, X, secs, gap in res:
            oracle_out[b] = (X, secs, gap)
        cpu = {"value": args.cpu_bins / wall, "unit": "bins/s", "cores": workers, "kind": "oracle",
               "sample": f"first {args.cpu_bins} bins of the {args.workload} batch, FP64 NumPy oracle, "
                         f"one single-threaded worker process per core, wall {wall:.1f} s, "
                         f"{sum(r[2] for r in res):.1f} s CPU"}

    import torch
    import paper_2605_26580_amd as P
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    cfg = wl.model
    code = synth.regular_ldpc(wl.n, seed=wl.code_seed)
    bins = synth.make_bins(code, wl.K, wl.batch, wl.ebn0_db, wl.bin_seed)
    blob = synth.make_weights(cfg, wl.weight_seed)
    wh = P.Weights(P.make_cfg(cfg.n_layers, cfg.d, cfg.heads, cfg.mlp_mult, cfg.n_max), blob)
    ch = P.Code(code.n, code.m, code.row_ptr, code.col_idx)
    B, K, n = wl.batch, wl.K, wl.n
    y = torch.from_numpy(bins.y).to(dev)
    out = torch.zeros(B, K, n, dtype=torch.uint8, device=dev)
    prec = P.CIDER_BF16 if args.precision == "bf16" else P.CIDER_FP32
    opts = P.cider_opts_default(precision=prec, remask=int(wl.remask), remask_thr=wl.remask_thr,
                                remask_max_rounds=wl.remask_max_rounds, use_graph=1)
    blist = [{"y": y[b], "sigma2": float(bins.sigma2[b]), "code": ch, "K": K, "n": n, "out_symbols": out[b]}
             for b in range(B)]
    stream = torch.cuda.Stream()
    print(f"[bench] {args.workload}: {B} bins K={K} n={n} L={cfg.n_layers} d={cfg.d} T={wl.T} "
          f"{args.precision}, warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            P.cider_decode_batch(blist, wh, wl.T, opts, stream=stream)
        stream.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(args.steps):
            P.cider_decode_batch(blist, wh, wl.T, opts, stream=stream)
            ev[i + 1].record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    total = t1 - t0
    value = B * args.steps / total
    gpu_X = out.cpu().numpy()
    print(f"[bench] {value:.1f} bins/s", file=sys.stderr, flush=True)

    # ---- plain FP32 per-bin path on a subset (the comparison baseline)
    nplain = min(args.plain_bins, B)
    po = P.cider_opts_default(precision=P.CIDER_FP32, use_graph=0, remask=int(wl.remask),
                              remask_thr=wl.remask_thr, remask_max_rounds=wl.remask_max_rounds)
    plain_out = torch.zeros(nplain, K, n, dtype=torch.uint8, device=dev)
    with torch.cuda.stream(stream):
        P.cider_decode(y[0], float(bins.sigma2[0]), ch, K, n, wh, wl.T, plain_out[0], po, stream=stream)
        stream.synchronize()
        tp0 = time.perf_counter()
        for b in range(nplain):
            P.cider_decode(y[b], float(bins.sigma2[b]), ch, K, n, wh, wl.T, plain_out[b], po, stream=stream)
        stream.synchronize()
        tp1 = time.perf_counter()
    plain_value = nplain / (tp1 - tp0)
    plain_X = plain_out.cpu().numpy()
    print(f"[bench] fp32 plain {plain_value:.1f} bins/s", file=sys.stderr, flush=True)

    # ---- live per-kernel timing (HIP events around each launch, one decode)
    prof_opts = P.cider_opts_default(precision=prec, remask=int(wl.remask), remask_thr=wl.remask_thr,
                                     remask_max_rounds=wl.remask_max_rounds, profile=1)
    with torch.cuda.stream(stream):
        P.cider_profile_read(wh, reset=True)
        P.cider_decode_batch(blist, wh, wl.T, prof_opts, stream=stream)
        stream.synchronize()
    prof = P.cider_profile_read(wh, reset=True)
    tokens = B * K * n
    kind = "fp32" if args.precision == "fp32" else "bf16"
    per_tok, flop_role, byte_role = algorithmic(wl, 4 if kind == "fp32" else 2)
    dom_name, (dom_launches, dom_ms) = max(prof.items(), key=lambda kv: kv[1][1])
    dom_avg_ms = dom_ms / dom_launches
    roof = None
    if dom_name in byte_role:
        secs = dom_avg_ms * 1e-3
        fl = flop_role.get(dom_name, 0) * tokens
        by = byte_role[dom_name] * tokens
        if kind == "fp32" and dom_name.startswith("attn"):
            bound, peak, unit, ach = "alu", PEAK["fp32"], "TFLOP/s", fl / secs / 1e12
        elif fl / by >= PEAK[kind] * 1e12 / (HBM_PEAK * 1e9):
            bound, peak, unit, ach = "mfma", PEAK[kind], "TFLOP/s", fl / secs / 1e12
        else:
            bound, peak, unit, ach = "hbm", HBM_PEAK, "GB/s", by / secs / 1e9
        roof = {"bound": bound, "kernel": dom_name, "achieved": round(ach, 2), "peak": peak, "unit": unit,
                "frac": round(ach / peak, 4), "traffic": None, "avg_launch_ms": round(dom_avg_ms, 4),
                "flop_per_launch": fl, "bytes_per_launch": by,
                "tflops": round(fl / secs / 1e12, 2)}
    kernel_table = {k: {"launches": v[0], "avg_ms": round(v[1] / v[0], 4), "total_ms": round(v[1], 3)}
                    for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}

    # ---- agreement with the oracle on the CPU sample
    match = None
    if oracle_out:
        bm = sum(np.array_equal(gpu_X[b], oracle_out[b][0]) for b in oracle_out)
        sm = float(np.mean([np.mean(gpu_X[b] == oracle_out[b][0]) for b in oracle_out]))
        pm = [b for b in oracle_out if b < nplain]
        pbm = sum(np.array_equal(plain_X[b], oracle_out[b][0]) for b in pm)
        match = {"bins": len(oracle_out), "bf16_bin_match": bm / len(oracle_out), "bf16_symbol_match": round(sm, 5),
                 "fp32_plain_bin_match": (pbm / len(pm)) if pm else None}

    flop_batch = per_tok * tokens * (wl.T + 1)
    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "bins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": kind,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: K={K}, (3,6)-regular binary LDPC n={n}, BPSK sum + AWGN at "
                               f"Eb/N0 {list(wl.ebn0_db)} dB, denoiser L={cfg.n_layers} d={cfg.d} h={cfg.heads} "
                               f"seeded N(0,0.02) weights, T={wl.T}, {B} bins per batch",
                   "bins_per_batch": B, "K": K, "n": n, "T": wl.T, "remask": wl.remask},
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "symbols_per_s": round(value * K * n, 1),
        "model_tflops": round(flop_batch * args.steps / total / 1e12, 2),
        "fp32_plain": {"value": round(plain_value, 2), "unit": "bins/s", "bins": nplain,
                       "path": "cider_decode per bin, FP32, eager launches"},
        "speedup_vs_fp32_plain": round(value / plain_value, 2),
        "oracle_match": match,
        "roofline": roof,
        "kernels": kernel_table,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
