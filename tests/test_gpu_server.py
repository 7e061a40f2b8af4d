"""Continuous-batching server through the C ABI: every served bin must equal
the same bin decoded alone, bit for bit, while bins of different sizes
arrive, wait for slots and decode concurrently."""
import ctypes as C
import time

import numpy as np
import pytest

import synth
from gpu_common import code_handle, code_of, lib, say, torch_cuda, weights_handle

pytestmark = pytest.mark.gpu


def _server(P, wh, steps, max_slots, max_tokens, max_queue=64, opts=None):
    cfg = P.abi.cider_server_cfg()
    cfg.weights = wh.handle
    cfg.opts = opts if opts is not None else P.cider_opts_default()
    cfg.steps = steps
    cfg.max_slots = max_slots
    cfg.max_queue = max_queue
    cfg.hbm_budget = 0
    cfg.max_tokens = max_tokens
    h = C.c_void_p()
    P.abi.check(P.abi.lib().cider_server_create(C.byref(cfg), C.byref(h)), "cider_server_create")
    return h


@pytest.mark.parametrize("prec,d,h", [("fp32", 64, 4), ("bf16", 64, 4), ("bf16", 128, 8)])
def test_served_equals_alone(prec, d, h):
    """Requests admitted into a running batch decode exactly as they do alone
    (at d = 128 the BF16 path runs the token-resident kernels, whose tile and
    group tables are rebuilt whenever the resident set changes)."""
    torch = torch_cuda()
    P = lib()
    cfg = synth.ModelCfg(2, d, h, n_max=128)
    wh, _ = weights_handle(cfg, seed=41)
    opts = P.cider_opts_default(precision=P.CIDER_FP32 if prec == "fp32" else P.CIDER_BF16, remask=1)
    rng = np.random.default_rng(7)
    reqs = []
    for i in range(24):
        K = int(rng.integers(1, 7))
        n = int(rng.choice([32, 64, 128]))
        code = code_of(n, 1000 + n)
        b = synth.make_bins(code, K, 1, float(rng.uniform(2, 6)), seed=900 + i)
        reqs.append((K, n, code, np.ascontiguousarray(b.y[0]), float(b.sigma2[0])))
    say(f"server {prec} d={d}: 24 requests, 5 slots")
    srv = _server(P, wh, 8, max_slots=5, max_tokens=5 * 6 * 128, opts=opts)
    L = P.abi.lib()
    outs, ids = [], []
    try:
        for K, n, code, y, s2 in reqs:
            out = np.full((K, n), 7, np.uint8)
            rid = C.c_uint64()
            P.abi.check(L.cider_server_submit(srv, y.ctypes.data, s2, code_handle(code).handle, K, n,
                                              out.ctypes.data, C.byref(rid)), "submit")
            outs.append(out)
            ids.append(rid.value)
            time.sleep(0.001)
        P.abi.check(L.cider_server_drain(srv), "drain")
        res = (P.abi.cider_result * 64)()
        got = C.c_int32()
        P.abi.check(L.cider_server_poll(srv, res, 64, C.byref(got)), "poll")
        assert got.value == len(reqs)
        done = {res[i].id: res[i] for i in range(got.value)}
        assert set(done) == set(ids)
        for r in done.values():
            assert r.status == 0 and r.t_submit <= r.t_admit <= r.t_done
    finally:
        L.cider_server_destroy(srv)
    for (K, n, code, y, s2), out in zip(reqs, outs):
        alone = torch.zeros(K, n, dtype=torch.uint8, device="cuda")
        P.cider_decode_batch([{"y": torch.from_numpy(y).cuda(), "sigma2": s2, "code": code_handle(code), "K": K,
                               "n": n, "out_symbols": alone}], wh, 8, opts)
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), out), (K, n)


def test_queue_backpressure_returns_eagain():
    torch_cuda()
    P = lib()
    cfg = synth.ModelCfg(1, 64, 4, n_max=64)
    wh, _ = weights_handle(cfg, seed=43)
    code = code_of(64, 1064)
    b = synth.make_bins(code, 2, 1, 4.0, seed=1)
    y = np.ascontiguousarray(b.y[0])
    say("server backpressure")
    srv = _server(P, wh, 4, max_slots=1, max_tokens=128, max_queue=2)
    L = P.abi.lib()
    statuses = []
    outs = [np.zeros((2, 64), np.uint8) for _ in range(12)]
    try:
        for i in range(12):
            rid = C.c_uint64()
            statuses.append(L.cider_server_submit(srv, y.ctypes.data, float(b.sigma2[0]), code_handle(code).handle,
                                                  2, 64, outs[i].ctypes.data, C.byref(rid)))
        P.abi.check(L.cider_server_drain(srv), "drain")
    finally:
        L.cider_server_destroy(srv)
    assert P.abi.CIDER_EAGAIN in statuses and statuses[0] == 0
    assert all(s in (0, P.abi.CIDER_EAGAIN) for s in statuses)


def _bins(rng, count, Ks, ns, seed0):
    out = []
    for i in range(count):
        K = int(rng.choice(Ks))
        n = int(rng.choice(ns))
        code = code_of(n, 1000 + n)
        b = synth.make_bins(code, K, 1, float(rng.uniform(2, 6)), seed=seed0 + i)
        out.append((K, n, code, np.ascontiguousarray(b.y[0]), float(b.sigma2[0])))
    return out


def _alone(P, torch, wh, reqs, T, opts):
    res = []
    for K, n, code, y, s2 in reqs:
        a = torch.zeros(K, n, dtype=torch.uint8, device="cuda")
        P.cider_decode_batch([{"y": torch.from_numpy(y).cuda(), "sigma2": s2, "code": code_handle(code), "K": K,
                               "n": n, "out_symbols": a}], wh, T, opts)
        torch.cuda.synchronize()
        res.append(a.cpu().numpy())
    return res


def test_served_equals_alone_at_the_served_model_width():
    """The served workload's model shape (d = 384, 12 heads; two layers) with
    K up to 16 and n up to 1024: each served bin equals the bin decoded alone."""
    torch = torch_cuda()
    P = lib()
    cfg = synth.ModelCfg(2, 384, 12, n_max=1024)
    wh, _ = weights_handle(cfg, seed=15)
    opts = P.cider_opts_default(precision=P.CIDER_BF16, remask=1)
    rng = np.random.default_rng(5)
    reqs = _bins(rng, 1, [16], [1024], 700) + _bins(rng, 5, [2, 9, 16], [128, 512, 1024], 701)
    say(f"server d=384: shapes {[(K, n) for K, n, *_ in reqs]}")
    srv = P.Server(wh, 6, opts, max_slots=4, max_tokens=40000)
    got = []
    try:
        for K, n, code, y, s2 in reqs:
            got.append(srv.submit(y, s2, code_handle(code), K, n)[1])
        srv.drain()
        done = srv.poll()
        assert len(done) == len(reqs) and all(r.status == 0 for r in done)
    finally:
        srv.close()
    for (K, n, *_), g, a in zip(reqs, got, _alone(P, torch, wh, reqs, 6, opts)):
        assert np.array_equal(g, a), (K, n)


def test_hbm_budget_bounds_the_resident_set():
    """At the smallest budget (slot state plus one largest bin's workspace)
    bins of that largest size decode one at a time; a larger budget lets them
    overlap; every result equals the bin decoded alone."""
    torch = torch_cuda()
    P = lib()
    cfg = synth.ModelCfg(1, 64, 4, n_max=64)
    wh, _ = weights_handle(cfg, seed=44)
    opts = P.cider_opts_default(precision=P.CIDER_BF16)
    reqs = _bins(np.random.default_rng(9), 5, [16], [64], 800)
    floor = P.Server.budget_floor(wh, 6, opts, max_slots=4)
    ref = _alone(P, torch, wh, reqs, 6, opts)
    for budget, most in ((floor, 1), (floor * 4, 2)):
        say(f"server hbm_budget={budget} (floor {floor}): 5 bins of K=16 n=64")
        srv = P.Server(wh, 6, opts, max_slots=4, hbm_budget=budget)
        got = []
        try:
            for K, n, code, y, s2 in reqs:
                got.append(srv.submit(y, s2, code_handle(code), K, n)[1])
            srv.drain()
            done = sorted(srv.poll(), key=lambda r: r.id)
        finally:
            srv.close()
        assert len(done) == len(reqs)
        for g, a in zip(got, ref):
            assert np.array_equal(g, a)
        spans = [(r.t_admit, r.t_done) for r in done]
        overlap = max(sum(1 for a2, d2 in spans if a2 < d1 and a1 < d2) for a1, d1 in spans)
        print(f"  most bins resident together: {overlap}")
        if most == 1:
            assert overlap == 1
        else:
            assert overlap >= most
    with pytest.raises(P.CiderError):
        P.Server(wh, 6, opts, max_slots=4, hbm_budget=floor - 1)


def test_frames_served_equal_frames_decoded_in_one_batch():
    """The stochastic-binning front end through the server (each frame's
    decodable bins submitted as the frame arrives) gives the grids the batch
    front end gives (Appendix, protocol-level scalability)."""
    torch = torch_cuda()
    P = lib()
    n, K_max, T = 64, 8, 6
    cfg = synth.ModelCfg(2, 128, 8, n_max=64)
    wh, _ = weights_handle(cfg, seed=46)
    code = code_of(n, 1000 + n)
    ch = code_handle(code)
    frames = synth.make_protocol_frames(code, 3, 30, 6, K_max, (2.0, 6.0), seed=23)
    opts = P.cider_opts_default(precision=P.CIDER_BF16)
    say("frames through the server and through one packed batch")
    host = [{"loads": fr.loads, "payload": {chi: (b.y, b.sigma2) for chi, b in fr.bins}} for fr in frames]
    dev = [{"loads": fr.loads, "payload": {chi: (torch.from_numpy(b.y).cuda(), b.sigma2) for chi, b in fr.bins}}
           for fr in frames]
    srv = P.Server(wh, T, opts, max_slots=6)
    try:
        served = P.serve_frames(srv, host, ch, n, K_max)
    finally:
        srv.close()
    batch = P.decode_frames(dev, ch, n, wh, T, K_max, opts)
    torch.cuda.synchronize()
    for s, b in zip(served, batch):
        assert s["erased"] == b["erased"] and sorted(s["decoded"]) == sorted(b["decoded"])
        for chi, g in s["decoded"].items():
            assert np.array_equal(g, b["decoded"][chi][0].cpu().numpy()), chi
