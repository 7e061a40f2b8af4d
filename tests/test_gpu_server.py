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
