"""Throughput benchmark of the CIDER refinement path on one MI355X.

One benchmark step = one complete decode (every refinement step, the final
pass and any remask rounds) of one batch of synthetic bins through
cider_decode_batch.  Default workload (c2): K=4 users, binary (3,6)-regular
LDPC n=128, Eb/N0 cycling {2,4,6} dB, denoiser L=4 d=128 h=8 with seeded
N(0, 0.02) weights, T=16, 256 bins per batch, BF16 operands with FP32
accumulation.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --workload c1 --precision fp32     (small FP32 case)
    python bench.py --workload c3                      (K=8, n=256, remasking)
    python bench.py --workload c4                      (4096 ragged bins, one packed pass)
    python bench.py --workload c5 --load 0.5,0.9       (served: Poisson arrivals)
    python bench.py --workload amp                     (AMP-MMSE slot detector, 4096 frames)
    python bench.py --workload protocol                (stochastic binning: 160 frames, 100 users, 25 bins)
    python bench.py --workload gf64                    (GF(64) check-node update, 2^17 checks of degree 6)
    python bench.py --workload tiny64                  (GF(64) decoding at the paper's Tiny scale, 4096 frames)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "decoded bins/sec + p99 latency, BF16 batched vs FP32 plain, >=99.9% oracle symbol match"
PEAK = {"bf16": 2500.0, "fp32": 157.3, "fp8": 5000.0, "fp64": 78.6}   # dense TFLOP/s, MI355X published
HBM_PEAK = 8000.0                                        # GB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle, one single-threaded worker process per core

def _oracle_worker(args):
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
    return b, res.X, time.perf_counter() - t0


def _oracle_step_worker(args):
    """One denoiser forward of one bin (for workloads whose full decode is too
    long to time on the host): returns seconds per forward."""
    K, n, model, weight_seed, code_seed = args
    import synth
    from oracle.denoiser import denoise
    from oracle.evidence import evidence
    code = synth.regular_ldpc(n, seed=code_seed)
    b = synth.make_bins(code, K, 1, 4.0, seed=7)
    w = synth.unpack_weights(synth.make_weights(model, weight_seed), model)
    _, p = evidence(b.y[0].astype(np.float64), float(b.sigma2[0]), K)
    X = np.full((K, n), 2, np.uint8)
    t0 = time.perf_counter()
    denoise(X, p, code, w, model.n_layers, model.heads, 1.0)
    return time.perf_counter() - t0


# The slot-wise AMP-MMSE detector (the non-binary evidence front end): the
# paper's moderate scale, Q = 64 signatures, L = 24 slots per frame, n_s = 24
# measurements per slot, K = 2 users, a 48-bit payload, I_AMP = 20.
AMP = dict(Q=64, L=24, n_s=24, K=2, payload_bits=48, iters=20, ebn0_db=4.0, seed=106)


def _amp_slots(frames):
    import synth
    return synth.make_amp_slots(frames=frames, L=AMP["L"], Q=AMP["Q"], n_s=AMP["n_s"], K=AMP["K"],
                                payload_bits=AMP["payload_bits"], ebn0_db=AMP["ebn0_db"], seed=AMP["seed"])


def _amp_oracle_worker(args):
    from oracle.amp import amp_evidence_batch
    lo, hi, frames = args
    sl = _amp_slots(frames)
    t0 = time.perf_counter()
    S = amp_evidence_batch(sl.y[lo:hi], sl.rows[lo:hi], AMP["Q"], AMP["K"] / AMP["Q"], float(sl.p_sym[0]),
                           AMP["iters"])
    return lo, S, time.perf_counter() - t0


def run_amp(args):
    """AMP-MMSE evidence for a batch of frames; value = slots per second."""
    frames = args.bins or 4096
    sl = _amp_slots(frames)
    S_slots = sl.y.shape[0]
    Q, n_s, iters = AMP["Q"], AMP["n_s"], AMP["iters"]
    rho, su2 = AMP["K"] / Q, float(sl.p_sym[0])
    cpu, oracle_S = None, {}
    if not args.no_cpu:
        workers = max(1, min(16, os.cpu_count() or 1))
        per = 600                                  # slots per worker: about 0.7 s of oracle time each
        tasks = [(w * per, (w + 1) * per, frames) for w in range(workers)]
        log(f"oracle cpu baseline: {workers * per} slots on {workers} workers")
        out, wall = _pool(_amp_oracle_worker, tasks, workers)
        for lo, S, _ in out:
            oracle_S[lo] = S
        cpu = {"value": round(workers * per / wall, 2), "unit": "slots/s", "cores": workers, "kind": "oracle", "cpu_model": _cpu_model(),
               "sample": f"first {workers * per} slots of the batch, FP64 NumPy oracle, one single-threaded worker "
                         f"process per core ({per} slots each), wall {wall:.1f} s including start-up"}
    import torch
    import paper_2605_26580_amd as P
    torch.cuda.set_device(0)
    y = torch.from_numpy(sl.y).cuda()
    rows = torch.from_numpy(sl.rows).cuda()
    out = torch.empty(S_slots, Q, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            P.cider_amp_evidence(y, rows, S_slots, n_s, Q, rho, su2, iters, out, stream=stream)
        stream.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(args.steps):
            P.cider_amp_evidence(y, rows, S_slots, n_s, Q, rho, su2, iters, out, stream=stream)
            ev[i + 1].record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    value = S_slots * args.steps / (t1 - t0)
    # one launch per call: the kernel's own average duration from the events
    avg_ms = float(np.mean(lat))
    # operations the kernel performs: at Q = 64 each partial-DFT product is a
    # 64-point radix-2 FFT across the wave (per lane and stage one complex add
    # or subtract-and-twiddle, 5 FLOP on average), plus the MMSE denoiser (about
    # 20 FLOP per coordinate, a transcendental counted as one) and the residual,
    # Onsager and noise-estimate updates (9 FLOP per measurement); other Q take
    # the two dense complex products (8 Q n_s FLOP each)
    if Q == 64:
        fft = 5 * Q * 6
        flop = S_slots * (iters * (2 * fft + 20 * Q + 9 * n_s) + fft + 20 * Q)
    else:
        flop = S_slots * (iters * 16 + 8) * Q * n_s
    ach = flop / (avg_ms * 1e-3) / 1e12
    res = {"metric": "AMP-MMSE slot evidence/sec (non-binary detector front end)", "value": round(value, 1),
           "unit": "slots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round((t1 - t0) / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "frames_per_s": round(value / AMP["L"], 1),
           "config": {"workload": f"amp: Q={Q}, L={AMP['L']} slots per frame, n_s={n_s}, K={AMP['K']}, "
                                  f"{AMP['payload_bits']}-bit payload, Eb/N0 {AMP['ebn0_db']} dB, "
                                  f"I_AMP={iters}, {frames} frames per batch",
                      "slots_per_batch": S_slots},
           "roofline": {"bound": "alu", "kernel": "amp_evidence", "achieved": round(ach, 2), "peak": 157.3,
                        "unit": "TFLOP/s", "frac": round(ach / 157.3, 4), "traffic": None,
                        "avg_launch_ms": round(avg_ms, 4), "flop_per_launch": flop},
           "cpu_baseline": cpu}
    if oracle_S:
        got = out.cpu().numpy()
        err = 0.0
        for lo, S in oracle_S.items():
            g = got[lo:lo + S.shape[0]].astype(np.float64)
            err = max(err, float(np.max(np.abs(g - S) / np.maximum(1.0, np.abs(S)))))
        res["oracle_match"] = {"slots": int(sum(S.shape[0] for S in oracle_S.values())), "max_rel_err": err}
    log(f"{value:.1f} slots/s, kernel {avg_ms:.3f} ms per batch")
    return res


def _gf64_checks(C, dc, seed):
    rng = np.random.default_rng(seed)
    row_ptr = (np.arange(C + 1) * dc).astype(np.int32)
    coef = rng.integers(1, 64, C * dc).astype(np.uint8)
    p = rng.random((C * dc, 64)) ** 3
    p /= p.sum(axis=1, keepdims=True)
    return row_ptr, coef, p.astype(np.float32)


def _gf64_oracle_worker(args):
    from oracle import gf
    lo, hi, C, dc = args
    row_ptr, coef, p = _gf64_checks(C, dc, 7)
    p64 = p.astype(np.float64)
    t0 = time.perf_counter()
    out = {}
    for j in range(lo, hi):
        e0 = j * dc
        for o in range(e0, e0 + dc):
            others = [i for i in range(e0, e0 + dc) if i != o]
            out[o] = gf.check_message_wht([p64[i] for i in others], [int(coef[i]) for i in others], int(coef[o]))
    return out, time.perf_counter() - t0


def run_gf64(args):
    """GF(64) check-node update over 2^17 checks of degree 6; value = edges per second."""
    C, dc = args.bins or (1 << 17), 6
    E = C * dc
    row_ptr, coef, p = _gf64_checks(C, dc, 7)
    cpu, oracle = None, {}
    if not args.no_cpu:
        workers = max(1, min(16, os.cpu_count() or 1))
        per = 64
        tasks = [(w * per, (w + 1) * per, C, dc) for w in range(workers)]
        log(f"oracle cpu baseline: {workers * per} checks on {workers} workers")
        out, wall = _pool(_gf64_oracle_worker, tasks, workers)
        for o, _ in out:
            oracle.update(o)
        cpu = {"value": round(workers * per * dc / wall, 1), "unit": "edges/s", "cores": workers, "kind": "oracle", "cpu_model": _cpu_model(),
               "sample": f"first {workers * per} checks ({workers * per * dc} edges), FP64 NumPy oracle "
                         f"(Walsh-Hadamard form), one single-threaded worker process per core, wall {wall:.1f} s"}
    import torch
    import paper_2605_26580_amd as P
    torch.cuda.set_device(0)
    dp, dr, dcf = (torch.from_numpy(x).cuda() for x in (p, row_ptr, coef))
    out = torch.empty((E, 64), dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            P.cider_gf64_check_update(dp, dr, dcf, C, E, out, stream=stream)
        stream.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(args.steps):
            P.cider_gf64_check_update(dp, dr, dcf, C, E, out, stream=stream)
            ev[i + 1].record(stream)
        stream.synchronize()
        t1 = time.perf_counter()
    avg_ms = float(np.mean([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]))
    value = E * args.steps / (t1 - t0)
    byt = E * (64 * 4 * 2 + 1) + (C + 1) * 4          # distributions in and messages out, coefficients, row offsets
    ach = byt / (avg_ms * 1e-3) / 1e9
    res = {"metric": "GF(64) check-node messages/sec (non-binary parity layer)", "value": round(value, 1),
           "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round((t1 - t0) / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"gf64: {C} checks of degree {dc} ({E} edges), random nonzero coefficients, "
                                  f"random input distributions", "checks": C, "edges": E},
           "roofline": {"bound": "hbm", "kernel": "gf64_check", "achieved": round(ach, 1), "peak": HBM_PEAK,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK, 4), "traffic": None,
                        "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": byt},
           "cpu_baseline": cpu}
    if oracle:
        got = out.cpu().numpy()
        res["oracle_match"] = {"edges": len(oracle),
                               "max_abs_err": float(max(np.max(np.abs(got[o] - v)) for o, v in oracle.items()))}
    log(f"{value / 1e6:.1f} M edges/s, kernel {avg_ms:.3f} ms per call")
    return res


# The paper's main setting at its Tiny scale (dataset scales and model sizing
# tables): GF(64), K = 2 users, L = 12 slots (P = 8 checks, rate 1/3), denoiser
# D = 128, 4 layers, 4 heads, T = 12 refinement steps; evidence from the slot
# AMP-MMSE detector (n_s = 24, I_AMP = 20) at 4 dB.
TINY64 = dict(q_bits=6, n=12, K=2, L=4, d=128, heads=4, T=12, n_s=24, iters=20, ebn0_db=4.0, code_seed=2012,
              weight_seed=21, frame_seed=107)


def _tiny64_inputs(frames):
    import synth
    t = TINY64
    code = synth.qary_ldpc(t["n"], t["q_bits"], dv=2, dc=3, seed=t["code_seed"])
    fr = synth.make_qary_frames(code, t["K"], frames, t["n_s"], t["ebn0_db"], t["frame_seed"])
    cfg = synth.ModelCfg(t["L"], t["d"], t["heads"], q=1 << t["q_bits"], n_max=64)
    return code, fr, cfg


def _tiny64_oracle_worker(args):
    from oracle import qary
    from oracle.amp import amp_evidence_batch
    lo, hi, frames = args
    import synth
    t = TINY64
    code, fr, cfg = _tiny64_inputs(frames)
    w = synth.unpack_weights(synth.make_weights(cfg, t["weight_seed"]), cfg)
    Q, n = 1 << t["q_bits"], t["n"]
    sl = fr.slots
    t0 = time.perf_counter()
    out = {}
    for f in range(lo, hi):
        S = amp_evidence_batch(sl.y[f * n:(f + 1) * n], sl.rows[f * n:(f + 1) * n], Q, t["K"] / Q,
                               float(sl.p_sym[f * n]), t["iters"])
        out[f] = qary.decode_bin_q(S, code, t["K"], w, t["L"], t["heads"], t["T"]).X
    return out, time.perf_counter() - t0


def run_tiny64(args):
    """GF(64) decoding at the paper's Tiny scale: AMP-MMSE evidence and the
    refinement loop for a batch of frames; value = decoded frames (bins) per second."""
    t = TINY64
    if args.precision not in ("bf16", "fp32"):
        raise SystemExit("the GF(Q) decoder runs in bf16 or fp32")
    kind = args.precision
    frames = args.bins or 4096
    Q, n, K = 1 << t["q_bits"], t["n"], t["K"]
    cpu, oracle_X = None, {}
    if not args.no_cpu:
        workers = max(1, min(16, os.cpu_count() or 1))
        per = 24                                  # frames per worker: about 10 s of oracle time each
        tasks = [(w * per, (w + 1) * per, frames) for w in range(workers)]
        log(f"oracle cpu baseline: {workers * per} frames on {workers} workers")
        out, wall = _pool(_tiny64_oracle_worker, tasks, workers)
        for o, _ in out:
            oracle_X.update(o)
        cpu = {"value": round(workers * per / wall, 2), "unit": "bins/s", "cores": workers, "kind": "oracle",
               "cpu_model": _cpu_model(),
               "sample": f"first {workers * per} frames: FP64 AMP-MMSE evidence and FP64 decode per frame, one "
                         f"single-threaded worker process per core ({per} frames each), wall {wall:.1f} s"}
    import torch
    import synth
    import paper_2605_26580_amd as P
    torch.cuda.set_device(0)
    code, fr, cfg = _tiny64_inputs(frames)
    wh = P.Weights(P.make_cfg(t["L"], t["d"], t["heads"], 4, 64, Q), synth.make_weights(cfg, t["weight_seed"]))
    ch = P.CodeQ(code.n, code.m, code.row_ptr, code.col_idx, code.coef, t["q_bits"])
    sl = fr.slots
    y = torch.from_numpy(sl.y).cuda()
    rows = torch.from_numpy(sl.rows).cuda()
    S = torch.empty(frames * n, Q, dtype=torch.float32, device="cuda")
    out = torch.zeros(frames, K, n, dtype=torch.uint8, device="cuda")
    prec = {"bf16": P.CIDER_BF16, "fp32": P.CIDER_FP32}[kind]
    opts = P.cider_opts_default(precision=prec, use_graph=1)
    blist = [{"S": S[f * n:(f + 1) * n], "code": ch, "K": K, "n": n, "out_symbols": out[f]} for f in range(frames)]
    stream = torch.cuda.Stream()

    def one():
        P.cider_amp_evidence(y, rows, frames * n, t["n_s"], Q, K / Q, float(sl.p_sym[0]), t["iters"], S,
                             stream=stream)
        P.cider_decode_q_batch(blist, wh, t["T"], opts, stream=stream)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            one()
        stream.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(args.steps):
            one()
            ev[i + 1].record(stream)
        stream.synchronize()
        t1 = time.perf_counter()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    value = frames * args.steps / (t1 - t0)
    gpu_X = out.cpu().numpy()
    # the dominant kernel: one profiled decode (HIP events around every launch)
    po = P.cider_opts_default(precision=prec, profile=1)
    with torch.cuda.stream(stream):
        P.cider_profile_read(wh, reset=True)
        P.cider_decode_q_batch(blist, wh, t["T"], po, stream=stream)
        stream.synchronize()
    prof = P.cider_profile_read(wh, reset=True)
    kernels = {k: {"launches": v[0], "avg_ms": round(v[1] / v[0], 4), "total_ms": round(v[1], 3)}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    tokens = frames * K * n
    roof = roofline(prof, cfg, n, K, tokens, kind, "tiny64")
    res = {"metric": "decoded bins/sec, GF(64) Tiny scale (AMP-MMSE evidence + CIDER refinement)",
           "value": round(value, 1), "unit": "bins/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round((t1 - t0) / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": kind, "data": "synthetic",
           "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "latency_scope": "per bin: the frames of a batch are submitted and complete together",
           "symbols_per_s": round(value * K * n, 1),
           "config": {"workload": f"tiny64: GF(64) (2,3)-regular LDPC L={n} (P={code.m}, rate 1/3), K={K}, slot "
                                  f"channel n_s={t['n_s']} at {t['ebn0_db']} dB, AMP I={t['iters']}, denoiser "
                                  f"D={t['d']} {t['L']} layers {t['heads']} heads seeded N(0,0.02) weights, "
                                  f"T={t['T']}, {frames} frames per batch", "frames_per_batch": frames},
           "paper_context": {"ms_per_sample": 1.26, "hardware": "RTX 3090 + i5-14500 (paper's own, trained model; "
                                                                 "batching not stated)"},
           "roofline": roof, "kernels": kernels, "cpu_baseline": cpu}
    if oracle_X:
        fs = sorted(oracle_X)
        res["oracle_match"] = {"bins": len(fs),
                               "bin_match": round(float(np.mean([np.array_equal(gpu_X[f], oracle_X[f]) for f in fs])), 4),
                               "symbol_match": round(float(np.mean([np.mean(gpu_X[f] == oracle_X[f]) for f in fs])), 5)}
    log(f"{value:.1f} bins/s, batch {np.median(lat):.3f} ms")
    return res


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _pool(fn, tasks, workers):
    import multiprocessing as mp
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        out = pool.map(fn, tasks)
    return out, time.perf_counter() - t0


# ---------------------------------------------------------------------------
# algorithmic FLOP and bytes per token of each kernel role

def algorithmic(model, n, K, es: int):
    d, L, F = model.d, model.n_layers, model.d_ff
    per_tok = L * (32 * d * d + 4 * n * d + 4 * K * d) + 6 * d * d + 12 * d
    flop = {
        "gemm_gate1": 2 * d * 2 * d, "gemm_gate2": 2 * d * d,
        "gemm_qkv_row": 2 * d * 3 * d, "gemm_o_row": 2 * d * d,
        "gemm_qkv_user": 2 * d * 3 * d, "gemm_o_user": 2 * d * d,
        "gemm_mlp_up": 2 * d * F, "gemm_mlp_down": 2 * F * d, "mlp_fused": 4 * d * F,
        "attn_row": 4 * n * d, "attn_user": 4 * K * d,
        "attn_block_row": 8 * d * d + 4 * n * d, "attn_block_user": 8 * d * d + 4 * K * d,
        "gate_fused": 6 * d * d, "embed_gate": 6 * d * d, "user_block": 8 * d * d + 4 * K * d, "user_mlp": 8 * d * d + 4 * K * d + 4 * d * F,
        "oproj_mlp": 2 * d * d + 4 * d * F, "oproj_user_attn": 8 * d * d + 4 * K * d,
        "row_block": 8 * d * d + 4 * n * d,
        "qkv_attn_user": 6 * d * d + 4 * K * d, "qkv_attn_row": 6 * d * d + 4 * n * d,
    }
    # minimum bytes: inputs read once, outputs written once; residual updates read and
    # write the FP32 stream and (BF16) write the next LayerNorm's compute-type copy
    byt = {
        "gemm_gate1": (2 * d + d) * es, "gemm_gate2": d * es + 3 * 4 * d + d * es,
        "gemm_qkv_row": (d + 3 * d) * es, "gemm_qkv_user": (d + 3 * d) * es,
        "gemm_o_row": d * es + 8 * d + d * es, "gemm_o_user": d * es + 8 * d + d * es,
        "gemm_mlp_up": (d + F) * es, "gemm_mlp_down": F * es + 8 * d + d * es,
        "mlp_fused": d * es + 8 * d + d * es,
        "attn_row": (3 * d + d) * es, "attn_user": (3 * d + d) * es,
        "layernorm": 4 * d + d * es,
        # fused attention sublayer: XN in, FP32 residual read and written, next XN out
        "attn_block_row": 2 * d * es + 8 * d, "attn_block_user": 2 * d * es + 8 * d,
        "user_block": 2 * d * es + 8 * d, "row_block": 2 * d * es + 8 * d,
        # user sublayer + MLP: XN and R in, R and XN out once for both
        "user_mlp": 2 * d * es + 8 * d,
        # output projection + MLP: O and R in, R and XN out
        "oproj_mlp": 2 * d * es + 8 * d,
        # row output projection + user QKV + attention: O_row, R in; R, O_user out
        "oproj_user_attn": 2 * d * es + 8 * d,
        # QKV projection + user attention: XN in, O out
        "qkv_attn_user": 2 * d * es, "qkv_attn_row": 2 * d * es,
        # gate MLP: [Z ; e] in, residual stream and e read, residual and first XN written
        "gate_fused": 3 * d * es + 12 * d,
        # embedding + Module A + first LayerNorm: the symbol in (the weights and the
        # per-slot tables stay in cache), residual stream and first XN out
        "embed_gate": 1 + 4 * d + d * es,
    }
    return per_tok, flop, byt


def _measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if it was
    taken on the kernel source as it stands (the summary names that source file
    and records its SHA-1)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{kernel}_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_s = re.search(r"source_sha1:\s*([0-9a-f]{40})", txt)
    m_f = re.search(r"^source:\s*(\S+)", txt, re.M)
    if not m_b or not m_s or not m_f:
        return None
    src = os.path.join(ROOT, m_f.group(1))
    if not os.path.exists(src) or hashlib.sha1(open(src, "rb").read()).hexdigest() != m_s.group(1):
        return None
    return float(m_b.group(1))


def roofline(prof, model, n, K, tokens, kind, workload):
    per_tok, flop_role, byte_role = algorithmic(model, n, K, {"fp32": 4, "fp64": 8}.get(kind, 2))
    if kind == "fp8":   # the LayerNorm-fed GEMMs read 1-byte activations
        d = model.d
        byte_role["gemm_qkv_row"] = byte_role["gemm_qkv_user"] = d + 3 * d * 2 + 4
        byte_role["mlp_fused"] = d + 4 + 8 * d + d + 4
    dom_name, (dom_launches, dom_ms) = max(prof.items(), key=lambda kv: kv[1][1])
    dom_avg_ms = dom_ms / dom_launches
    if dom_name not in byte_role:
        return None
    secs = dom_avg_ms * 1e-3
    fl = flop_role.get(dom_name, 0) * tokens
    by = byte_role[dom_name] * tokens
    # the denoiser's dense contractions are the path's bound: the dominant kernel is
    # reported as GEMM FLOP/s against the dense MFMA peak of its operand type, with
    # its algorithmic HBM rate beside it
    if kind in ("fp32", "fp64") and dom_name.startswith("attn"):
        bound, peak, unit = "alu", PEAK[kind], "TFLOP/s"
    elif kind == "fp8" and dom_name == "oproj_mlp":
        # the token-resident d = 256 kernel runs only its MLP up projection in
        # e4m3: the peak is the time-weighted blend of the two MFMA rates
        d, F = model.d, model.d_ff
        f8 = 2 * d * F
        b16 = flop_role[dom_name] - f8
        bound, peak, unit = "mfma", round(flop_role[dom_name] / (f8 / PEAK["fp8"] + b16 / PEAK["bf16"]), 1), "TFLOP/s"
    else:
        bound, peak, unit = "mfma", PEAK[kind], "TFLOP/s"
    ach = fl / secs / 1e12
    gbs = by / secs / 1e9
    return {"bound": bound, "kernel": dom_name, "achieved": round(ach, 2), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4), "traffic": _measured_traffic(workload, dom_name),
            "avg_launch_ms": round(dom_avg_ms, 4), "flop_per_launch": fl, "bytes_per_launch": by,
            "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK, "unit": "GB/s", "frac": round(gbs / HBM_PEAK, 4)}}


# ---------------------------------------------------------------------------

def run_batched(args, wl, P, torch):
    """Fixed-shape (c1..c3) or ragged (c4) batch; returns the JSON dict."""
    import synth
    dev = torch.device("cuda", 0)
    cfg = wl.model
    ragged = wl.ragged_K is not None
    blob = synth.make_weights(cfg, wl.weight_seed)
    wh = P.Weights(P.make_cfg(cfg.n_layers, cfg.d, cfg.heads, cfg.mlp_mult, cfg.n_max, cfg.q), blob)
    if ragged:
        codes = {n: synth.regular_ldpc(n, seed=1000 + n) for n in wl.ragged_n}
        if wl.binning:
            # every decodable bin of the frames, in one packed call (as decode_frames issues it)
            K_tot, zeta, K_max = wl.binning
            frames = synth.make_protocol_frames(codes[wl.ragged_n[0]], args.bins or wl.batch, K_tot, zeta, K_max,
                                                wl.ebn0_range, wl.bin_seed)
            rb = [b for fr in frames for _, b in fr.bins]
            erased = sum(len(fr.overflow) for fr in frames)
        else:
            rb = synth.make_ragged_bins(codes, args.bins or wl.batch, wl.ragged_K, wl.ragged_n, wl.ebn0_range,
                                        wl.bin_seed)
        handles = {n: P.Code(c.n, c.m, c.row_ptr, c.col_idx) for n, c in codes.items()}
        shapes = [(b.K, b.n) for b in rb]
        ys = [torch.from_numpy(b.y).to(dev) for b in rb]
        s2 = [b.sigma2 for b in rb]
        chs = [handles[b.n] for b in rb]
    else:
        code = synth.regular_ldpc(wl.n, seed=wl.code_seed)
        B = args.bins or wl.batch
        bins = synth.make_bins(code, wl.K, B, wl.ebn0_db, wl.bin_seed)
        ch = P.Code(code.n, code.m, code.row_ptr, code.col_idx)
        shapes = [(wl.K, wl.n)] * B
        yall = torch.from_numpy(bins.y).to(dev)
        ys = [yall[b] for b in range(B)]
        s2 = [float(bins.sigma2[b]) for b in range(B)]
        chs = [ch] * B
    B = len(shapes)
    tokens = sum(K * n for K, n in shapes)
    outs = [torch.zeros(K, n, dtype=torch.uint8, device=dev) for K, n in shapes]
    rounds = torch.zeros(len(shapes), dtype=torch.int32, device=dev)
    prec = {"bf16": P.CIDER_BF16, "fp32": P.CIDER_FP32, "fp8": P.CIDER_FP8, "fp64": P.CIDER_FP64}[args.precision]
    kind = args.precision
    ro = dict(remask=int(wl.remask), remask_thr=wl.remask_thr, remask_max_rounds=wl.remask_max_rounds)
    if args.qhead:
        # quality head as the remask criterion: a seeded head that is always sure
        # (b2 = +30, no row remasked), so the run costs the head's evaluation at
        # every final pass and nothing more
        psi = synth.make_quality_head(cfg.d, args.qhead, seed=7, b2=30.0)
        qbuf = torch.from_numpy(psi).to(dev)
        ro = dict(remask=1, qhead=qbuf, qhead_hidden=args.qhead)
    opts = P.cider_opts_default(precision=prec, use_graph=1, autotune=args.autotune, **ro)
    blist = [{"y": ys[i], "sigma2": s2[i], "code": chs[i], "K": shapes[i][0], "n": shapes[i][1],
              "out_symbols": outs[i], "out_rounds": rounds[i:i + 1]} for i in range(B)]
    stream = torch.cuda.Stream()
    log(f"{wl.name}: {B} bins, {tokens} tokens, L={cfg.n_layers} d={cfg.d} h={cfg.heads} T={wl.T} "
        f"remask={wl.remask} {kind}, warmup {args.warmup}, steps {args.steps}")
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
            log(f"step {i + 1}/{args.steps} enqueued")
        stream.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    total = t1 - t0
    value = B * args.steps / total
    gpu_X = [o.cpu().numpy() for o in outs]
    rounds_hist = {int(k): int(v) for k, v in zip(*np.unique(rounds.cpu().numpy(), return_counts=True))}
    log(f"{value:.1f} bins/s")

    # plain FP32 per-bin path on a subset of the same bins (the comparison baseline)
    nplain = min(args.plain_bins, B)
    plain_value, plain_X = None, []
    if nplain > 0:
        po = P.cider_opts_default(precision=P.CIDER_FP32, use_graph=0, **ro)
        pouts = [torch.zeros(*shapes[i], dtype=torch.uint8, device=dev) for i in range(nplain)]
        with torch.cuda.stream(stream):
            P.cider_decode(ys[0], s2[0], chs[0], *shapes[0], wh, wl.T, pouts[0], po, stream=stream)
            stream.synchronize()
            tp0 = time.perf_counter()
            for i in range(nplain):
                P.cider_decode(ys[i], s2[i], chs[i], *shapes[i], wh, wl.T, pouts[i], po, stream=stream)
            stream.synchronize()
            tp1 = time.perf_counter()
        plain_value = nplain / (tp1 - tp0)
        plain_X = [p.cpu().numpy() for p in pouts]
        log(f"fp32 plain {plain_value:.2f} bins/s over {nplain} bins")

    # live per-kernel timing: HIP events around each launch during one decode
    prof_opts = P.cider_opts_default(precision=prec, profile=1, **ro)
    with torch.cuda.stream(stream):
        P.cider_profile_read(wh, reset=True)
        P.cider_decode_batch(blist, wh, wl.T, prof_opts, stream=stream)
        stream.synchronize()
    prof = P.cider_profile_read(wh, reset=True)
    mean_n = tokens / max(1, sum(K for K, _ in shapes))
    mean_K = tokens / max(1, sum(n for _, n in shapes))
    roof = roofline(prof, cfg, mean_n, mean_K, tokens, kind, wl.name)
    kernel_table = {k: {"launches": v[0], "avg_ms": round(v[1] / v[0], 4), "total_ms": round(v[1], 3)}
                    for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    tuning = [{"role": t[0], "N": t[1], "Kd": t[2], "bucket": t[3], "tile": t[4], "best_ms": round(t[5], 4),
               "default_ms": round(t[6], 4)} for t in P.cider_tuning_read(wh)]
    per_tok, _, _ = algorithmic(cfg, mean_n, mean_K, 2)
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "bins/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * total / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": kind, "data": "synthetic",
        "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "symbols_per_s": round(value * tokens / B, 1),
        "model_tflops_lower_bound": round(per_tok * tokens * (wl.T + 1) * args.steps / total / 1e12, 2),
        "fp32_plain": ({"value": round(plain_value, 3), "unit": "bins/s", "bins": nplain,
                        "path": "cider_decode per bin, FP32, eager launches"} if plain_value else None),
        "speedup_vs_fp32_plain": round(value / plain_value, 2) if plain_value else None,
        "latency_scope": "per bin: every bin of a batch is submitted with it and completes with it, so a bin's "
                         "latency is its batch's decode time (HIP events on the decode stream)",
        "remask_rounds": rounds_hist if wl.remask or args.qhead else None,
        "roofline": roof, "kernels": kernel_table, "tuning": tuning,
    }
    if args.qhead:
        res["quality_head"] = {"hidden": args.qhead, "b2": 30.0, "remask": "head criterion, no row below phi"}
    if wl.binning:
        K_tot, zeta, K_max = wl.binning
        nf = len(frames)
        res["users_per_s"] = round(nf * K_tot * args.steps / total, 1)
        res["config"] = {"workload": f"{wl.name}: {nf} frames of K_tot={K_tot} users, uniform preamble choice over "
                                     f"zeta={zeta} bins, bins with K_chi > {K_max} erased ({erased} of {nf * zeta}), "
                                     f"the other {B} bins (K_chi 1..{K_max}) decoded in one packed pass per step; "
                                     f"(3,6)-regular binary LDPC n={wl.ragged_n[0]}, Eb/N0 uniform "
                                     f"{list(wl.ebn0_range)} dB, L={cfg.n_layers} d={cfg.d} h={cfg.heads} "
                                     f"seeded N(0,0.02) weights, T={wl.T}",
                         "frames": nf, "bins_per_batch": B, "erased_bins": erased, "tokens": tokens, "T": wl.T,
                         "remask": wl.remask}
    elif ragged:
        res["config"] = {"workload": f"{wl.name}: {B} bins, K uniform {list(wl.ragged_K)}, n uniform "
                                     f"{list(wl.ragged_n)} (3,6)-regular binary LDPC, Eb/N0 uniform "
                                     f"{list(wl.ebn0_range)} dB, L={cfg.n_layers} d={cfg.d} h={cfg.heads} "
                                     f"seeded N(0,0.02) weights, T={wl.T}, one packed pass per step",
                         "bins_per_batch": B, "tokens": tokens, "T": wl.T, "remask": wl.remask}
    else:
        res["config"] = {"workload": f"{wl.name}: K={wl.K}, (3,6)-regular binary LDPC n={wl.n}, BPSK sum + AWGN at "
                                     f"Eb/N0 {list(wl.ebn0_db)} dB, denoiser L={cfg.n_layers} d={cfg.d} "
                                     f"h={cfg.heads} seeded N(0,0.02) weights, T={wl.T}, {B} bins per batch"
                                     + (", remasking on" if wl.remask else ""),
                         "bins_per_batch": B, "K": wl.K, "n": wl.n, "T": wl.T, "remask": wl.remask}
    return res, gpu_X, plain_X


def _c2_weights(P, wl):
    import synth
    cfg = wl.model
    blob = synth.make_weights(cfg, wl.weight_seed)
    return cfg, P.Weights(P.make_cfg(cfg.n_layers, cfg.d, cfg.heads, cfg.mlp_mult, cfg.n_max, cfg.q), blob)


def clopper_pearson(k, n, alpha=0.05):
    """Exact two-sided (1 - alpha) interval of a binomial proportion k / n."""
    from scipy.stats import beta
    lo = 0.0 if k == 0 else float(beta.ppf(alpha / 2, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - alpha / 2, k + 1, n - k))
    return lo, hi


def stored_grid_agreement(P, torch, wh, wl):
    """Bit-exact agreement of whole c2 decodes with the FP64 oracle's grids
    stored in tests/golden/c2_oracle_grids.npz (3072 bins, written by a script
    that calls only the oracle): BF16 in the timed configuration (256 bins per
    call, graph replay) and the plain FP32 path (one call per bin, eager)."""
    import synth
    path = os.path.join(ROOT, "tests", "golden", "c2_oracle_grids.npz")
    if wl.name != "c2" or not os.path.exists(path):
        return None
    g = np.load(path)
    shape = tuple(int(v) for v in g["shape"])
    X = np.unpackbits(g["X_packed"], axis=-1, count=shape[-1]).reshape(shape)
    B, K, n = shape
    code = synth.regular_ldpc(wl.n, seed=wl.code_seed)
    bins = synth.make_bins(code, wl.K, B, wl.ebn0_db, wl.bin_seed)
    if float(np.sum(bins.y, dtype=np.float64)) != float(g["y_sum"][0]):
        log("stored grids do not match the generated inputs; agreement not measured")
        return None
    ch = P.Code(code.n, code.m, code.row_ptr, code.col_idx)
    y = torch.from_numpy(bins.y).cuda()
    runs = {}
    out = torch.full((B, K, n), 9, dtype=torch.uint8, device="cuda")
    o = P.cider_opts_default(precision=P.CIDER_BF16, use_graph=1)
    for b0 in range(0, B, 256):
        P.cider_decode_batch([{"y": y[b], "sigma2": float(bins.sigma2[b]), "code": ch, "K": K, "n": n,
                               "out_symbols": out[b]} for b in range(b0, min(B, b0 + 256))], wh, wl.T, o)
    torch.cuda.synchronize()
    runs["bf16_batched"] = out.cpu().numpy()
    # the FP64 mode in the same launch configuration, timed (one warm-up batch first)
    out.fill_(9)
    o = P.cider_opts_default(precision=P.CIDER_FP64, use_graph=1)
    bl = lambda b0: [{"y": y[b], "sigma2": float(bins.sigma2[b]), "code": ch, "K": K, "n": n, "out_symbols": out[b]}
                     for b in range(b0, min(B, b0 + 256))]
    P.cider_decode_batch(bl(0), wh, wl.T, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b0 in range(0, B, 256):
        P.cider_decode_batch(bl(b0), wh, wl.T, o)
    torch.cuda.synchronize()
    fp64_rate = B / (time.perf_counter() - t0)
    runs["fp64_batched"] = out.cpu().numpy()
    log(f"stored-grid agreement: {B} bins BF16 and FP64 ({fp64_rate:.1f} bins/s) batched done; FP32 plain, one "
        f"call per bin")
    out.fill_(9)
    o = P.cider_opts_default(precision=P.CIDER_FP32, use_graph=0)
    for b in range(B):
        P.cider_decode(y[b], float(bins.sigma2[b]), ch, K, n, wh, wl.T, out[b], o)
        if b % 1024 == 1023:
            torch.cuda.synchronize()
            log(f"  fp32 plain {b + 1}/{B}")
    torch.cuda.synchronize()
    runs["fp32_plain"] = out.cpu().numpy()
    res = {"bins": B, "source": "tests/golden/c2_oracle_grids.npz (FP64 oracle, exact grid equality)"}
    for name, got in runs.items():
        same = np.array([np.array_equal(got[b], X[b]) for b in range(B)])
        lo, hi = clopper_pearson(int(same.sum()), B)
        res[name] = {"bin_match": round(float(same.mean()), 5), "ci95": [round(lo, 5), round(hi, 5)],
                     "symbol_match": round(float(np.mean(got == X)), 5)}
    res["fp64_batched"]["bins_per_s"] = round(fp64_rate, 1)
    mg = g["min_rel_gap"]
    res["oracle_min_relative_decision_gap"] = {f"q{q:g}": float(np.quantile(mg, q / 100)) for q in (0.1, 1, 10, 50)}
    return res


def c3_subrecord(args, P, torch):
    """c3 (K=8, n=256, d=256, L=6, T=32, remasking on, 512 bins) timed in the
    same run: bins/s, the dominant kernel against the MFMA peak, rounds."""
    import copy
    import synth
    a = copy.copy(args)
    a.workload, a.steps, a.warmup, a.bins, a.plain_bins, a.qhead = "c3", 2, 1, 0, 0, 0
    r3, _, _ = run_batched(a, synth.workload("c3"), P, torch)
    top = dict(list(r3["kernels"].items())[:4])
    return {"value": r3["value"], "unit": "bins/s", "steps": a.steps, "ms_per_step": r3["ms_per_step"],
            "symbols_per_s": r3["symbols_per_s"], "remask_rounds": r3["remask_rounds"], "roofline": r3["roofline"],
            "kernels": top, "workload": r3["config"]["workload"]}


def run_served(args, wl, P, torch):
    """Served workload (c5): Poisson arrivals through the continuous-batching
    server; latency = completion - submission of each admitted bin."""
    import ctypes as C
    import synth
    cfg = wl.model
    blob = synth.make_weights(cfg, wl.weight_seed)
    wh = P.Weights(P.make_cfg(cfg.n_layers, cfg.d, cfg.heads, cfg.mlp_mult, cfg.n_max, cfg.q), blob)
    codes = {n: synth.regular_ldpc(n, seed=1000 + n) for n in wl.ragged_n}
    handles = {n: P.Code(c.n, c.m, c.row_ptr, c.col_idx) for n, c in codes.items()}
    pool = synth.make_ragged_bins(codes, args.bins or 512, wl.ragged_K, wl.ragged_n, wl.ebn0_range, wl.bin_seed)
    L = P.abi.lib()
    opts = P.cider_opts_default(precision=P.CIDER_BF16, remask=int(wl.remask), remask_thr=wl.remask_thr,
                                remask_max_rounds=wl.remask_max_rounds)

    def make_server():
        sc = P.abi.cider_server_cfg()
        sc.weights = wh.handle
        sc.opts = opts
        sc.steps = wl.T
        sc.max_slots = args.max_slots
        sc.max_queue = 1 << 20
        sc.hbm_budget = int(args.hbm_gib * (1 << 30))
        sc.max_tokens = args.max_tokens
        h = C.c_void_p()
        P.abi.check(L.cider_server_create(C.byref(sc), C.byref(h)), "cider_server_create")
        return h

    def run(rate, duration, burst=0):
        srv = make_server()
        outs = []
        submitted = 0
        t_start = time.perf_counter()
        rng = np.random.default_rng(wl.bin_seed)
        try:
            if burst:
                for i in range(burst):
                    b = pool[i % len(pool)]
                    o = np.zeros((b.K, b.n), np.uint8)
                    rid = C.c_uint64()
                    P.abi.check(L.cider_server_submit(srv, b.y.ctypes.data, b.sigma2, handles[b.n].handle, b.K,
                                                      b.n, o.ctypes.data, C.byref(rid)), "submit")
                    outs.append(o)
                submitted = burst
            else:
                t_next = t_start
                while time.perf_counter() - t_start < duration:
                    t_next += rng.exponential(1.0 / rate)
                    while time.perf_counter() < t_next:
                        time.sleep(min(0.002, max(0.0, t_next - time.perf_counter())))
                    b = pool[submitted % len(pool)]
                    o = np.zeros((b.K, b.n), np.uint8)
                    rid = C.c_uint64()
                    P.abi.check(L.cider_server_submit(srv, b.y.ctypes.data, b.sigma2, handles[b.n].handle, b.K,
                                                      b.n, o.ctypes.data, C.byref(rid)), "submit")
                    outs.append(o)
                    submitted += 1
            P.abi.check(L.cider_server_drain(srv), "drain")
            t_end = time.perf_counter()
            res = (P.abi.cider_result * max(1, submitted))()
            got = C.c_int32()
            P.abi.check(L.cider_server_poll(srv, res, submitted, C.byref(got)), "poll")
        finally:
            L.cider_server_destroy(srv)
        lat = np.array([res[i].t_done - res[i].t_submit for i in range(got.value)])
        wait = np.array([res[i].t_admit - res[i].t_submit for i in range(got.value)])
        return {"offered_rate": rate, "submitted": submitted, "completed": int(got.value),
                "wall_s": round(t_end - t_start, 3), "throughput": round(got.value / (t_end - t_start), 3),
                "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
                "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
                "queue_wait_p50_ms": round(1e3 * float(np.percentile(wait, 50)), 2)}

    log(f"{wl.name}: capacity probe, burst of {args.burst} bins")
    cap = run(0, 0, burst=args.burst)
    capacity = cap["throughput"]
    log(f"capacity {capacity:.2f} bins/s")
    loads = []
    for f in [float(x) for x in args.load.split(",") if x]:
        log(f"Poisson arrivals at {f:.2f} x capacity for {args.duration} s")
        loads.append(dict(run(f * capacity, args.duration), load=f))
    main = loads[-1] if loads else cap
    toks = float(np.mean([b.K * b.n for b in pool]))
    # the dominant kernel of the served model: one profiled packed decode of the
    # first 32 bins of the pool (HIP events around every launch)
    sample = pool[:32]
    so = P.cider_opts_default(precision=P.CIDER_BF16, profile=1, remask=int(wl.remask), remask_thr=wl.remask_thr,
                              remask_max_rounds=wl.remask_max_rounds)
    souts = [torch.zeros(b.K, b.n, dtype=torch.uint8, device="cuda") for b in sample]
    sy = [torch.from_numpy(np.ascontiguousarray(b.y)).cuda() for b in sample]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        P.cider_profile_read(wh, reset=True)
        P.cider_decode_batch([{"y": sy[i], "sigma2": b.sigma2, "code": handles[b.n], "K": b.K, "n": b.n,
                               "out_symbols": souts[i]} for i, b in enumerate(sample)], wh, wl.T, so, stream=stream)
        stream.synchronize()
    prof = P.cider_profile_read(wh, reset=True)
    stoks = sum(b.K * b.n for b in sample)
    roof = roofline(prof, cfg, stoks / sum(b.K for b in sample), stoks / sum(b.n for b in sample), stoks, "bf16",
                    wl.name)
    if roof:
        roof["sample"] = f"one packed decode of the first {len(sample)} bins of the served pool ({stoks} tokens)"
    return {
        "metric": METRIC, "value": main["throughput"], "unit": "bins/s", "n_gpus": 1, "steps": len(loads),
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic", "p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"],
        "symbols_per_s": round(main["throughput"] * toks, 1),
        "config": {"workload": f"{wl.name}: served, Poisson arrivals; K uniform {list(wl.ragged_K)}, n uniform "
                               f"{list(wl.ragged_n)}, Eb/N0 uniform {list(wl.ebn0_range)} dB, L={cfg.n_layers} "
                               f"d={cfg.d} h={cfg.heads}, T={wl.T}, remasking on; offered load as a fraction of "
                               f"the measured capacity (the workload's 20k bins/s is far beyond one GPU)",
                   "max_slots": args.max_slots, "admission": f"HBM budget {args.hbm_gib} GiB (bin state + step "
                                                              f"workspace laid out for the resident mix)"},
        "capacity_probe": cap, "loads": loads, "roofline": roof, "cpu_baseline": None,
        "latency_scope": "per bin: completion minus submission of each admitted request",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32", "fp8", "fp64"])
    ap.add_argument("--bins", type=int, default=0, help="override the batch size")
    ap.add_argument("--cpu-bins", type=int, default=16)
    ap.add_argument("--plain-bins", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="c2: skip the stored-grid agreement and the c3 record")
    ap.add_argument("--qhead", type=int, default=0, help="quality head with this many hidden units as the remask criterion")
    ap.add_argument("--calib-copy", action="store_true", help="end with a 256 MiB device copy (counter calibration)")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="batched workloads: 0 keeps every kernel at its default variant (profiling runs)")
    ap.add_argument("--load", default="0.5,0.9")
    ap.add_argument("--duration", type=float, default=15.0)
    ap.add_argument("--burst", type=int, default=96)
    ap.add_argument("--max-slots", type=int, default=96)
    ap.add_argument("--max-tokens", type=int, default=1 << 40, help="served: cap on resident tokens")
    ap.add_argument("--hbm-gib", type=float, default=16.0, help="served: device memory for bin state + workspace")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              "bins are independent, so N GPUs would each run this engine on a disjoint bin stream.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "amp":
        print(json.dumps(run_amp(args)))
        return
    if args.workload == "gf64":
        print(json.dumps(run_gf64(args)))
        return
    if args.workload == "tiny64":
        print(json.dumps(run_tiny64(args)))
        return

    import synth
    wl = synth.workload(args.workload)
    served = args.workload == "c5"

    # CPU baseline first, before the GPU is initialised (spawned workers)
    cpu, oracle_out = None, {}
    if not args.no_cpu:
        workers = max(1, min(args.cpu_bins, os.cpu_count() or 1, 16))
        if wl.ragged_K is None and wl.name in ("c1", "c2"):
            log(f"oracle cpu baseline: {args.cpu_bins} bins on {workers} workers")
            out, wall = _pool(_oracle_worker, [(wl.name, b) for b in range(args.cpu_bins)], workers)
            for b, X, secs in out:
                oracle_out[b] = X
            cpu = {"value": round(args.cpu_bins / wall, 3), "unit": "bins/s", "cores": workers, "kind": "oracle", "cpu_model": _cpu_model(),
                   "sample": f"first {args.cpu_bins} bins of the {wl.name} batch, FP64 NumPy oracle, full decode, "
                             f"one single-threaded worker process per core, wall {wall:.1f} s, "
                             f"{sum(r[2] for r in out):.1f} s CPU"}
        else:
            K = wl.K if wl.ragged_K is None else int(np.median(wl.ragged_K))
            n = wl.n if wl.ragged_K is None else int(wl.ragged_n[len(wl.ragged_n) // 2])
            code_seed = wl.code_seed if wl.ragged_K is None else 1000 + n
            log(f"oracle cpu baseline: one denoiser forward of a K={K} n={n} bin on {workers} workers")
            out, wall = _pool(_oracle_step_worker, [(K, n, wl.model, wl.weight_seed, code_seed)] * workers, workers)
            per_fwd = float(np.mean(out))
            passes = (wl.T + 1) * (3 if wl.remask else 1)
            cpu = {"value": round(workers / (per_fwd * passes), 5), "unit": "bins/s", "cores": workers,
                   "kind": "oracle", "cpu_model": _cpu_model(),
                   "sample": f"one FP64 oracle denoiser forward of a K={K}, n={n} bin per worker ({per_fwd:.1f} s), "
                             f"scaled by {passes} forwards per bin (T+1{' times 3 passes with remasking' if wl.remask else ''})"}

    import torch
    import paper_2605_26580_amd as P
    torch.cuda.set_device(0)
    if served:
        res = run_served(args, wl, P, torch)
        res["cpu_baseline"] = cpu
    else:
        res, gpu_X, plain_X = run_batched(args, wl, P, torch)
        res["cpu_baseline"] = cpu
        if oracle_out:
            ob = sorted(oracle_out)
            bm = sum(np.array_equal(gpu_X[b], oracle_out[b]) for b in ob)
            sm = float(np.mean([np.mean(gpu_X[b] == oracle_out[b]) for b in ob]))
            pb = [b for b in ob if b < len(plain_X)]
            pbm = sum(np.array_equal(plain_X[b], oracle_out[b]) for b in pb)
            res["oracle_match"] = {"bins": len(ob), "bin_match": round(bm / len(ob), 4), "symbol_match": round(sm, 5),
                                   "fp32_plain_bin_match": round(pbm / len(pb), 4) if pb else None}
        if wl.name == "c2" and not args.bins and not args.no_extra:
            _, wh2 = _c2_weights(P, wl)
            res["stored_grid_agreement"] = stored_grid_agreement(P, torch, wh2, wl)
            res["c3"] = c3_subrecord(args, P, torch)
    if args.calib_copy:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        yb = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            yb.copy_(x)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 256 MiB")
    print(json.dumps(res))


if __name__ == "__main__":
    main()
