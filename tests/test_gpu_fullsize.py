"""GPU checks at the workloads' full sizes, in the launch configuration the
benchmark times: BF16, the whole batch in one cider_decode_batch call, hipGraph
replay, the workload's own model (L, d, heads), K, n, T and remasking.

At these sizes the FP64 oracle runs on sampled bins only:
- one teacher-forced refinement step of a sampled bin, at the workload's model,
  K and n, against the oracle within the BF16 tolerance (logits and
  intermediate logits relative to max(1, |oracle|));
- the whole batch decoded in one call equals each sampled bin decoded alone,
  bit for bit (symbols, row-valid flags), so the per-bin parity carries over
  to the batch;
- every decoded grid is binary and its row-valid flags equal H x = 0 (mod 2)
  recomputed from the grid.
"""
import numpy as np
import pytest

import synth
from oracle.denoiser import denoise
from oracle.evidence import evidence

from gpu_common import TOL, code_handle, code_of, lib, rel_err, say, torch_cuda, valid_selection, weights_handle

pytestmark = pytest.mark.gpu


_dense = {}


def _syndrome_ok(code, X):
    """1 where row k of X satisfies every parity check of the code."""
    if code.n not in _dense:
        H = np.zeros((code.m, code.n), dtype=np.int64)
        for j in range(code.m):
            H[j, code.col_idx[code.row_ptr[j]:code.row_ptr[j + 1]]] = 1
        _dense[code.n] = H
    return ((_dense[code.n] @ X.T.astype(np.int64)) % 2 == 0).all(axis=0).astype(np.uint8)


def _workload_batch(name):
    """The benchmark's batch for workload `name`: (weights, unpacked weights,
    per-bin (K, n, code, y, sigma2) list)."""
    P = lib()
    wl = synth.workload(name)
    cfg = wl.model
    blob = synth.make_weights(cfg, wl.weight_seed)
    wh = P.Weights(P.make_cfg(cfg.n_layers, cfg.d, cfg.heads, cfg.mlp_mult, cfg.n_max, cfg.q), blob)
    w = synth.unpack_weights(blob, cfg)
    items = []
    if wl.ragged_K is not None:
        codes = {n: synth.regular_ldpc(n, seed=1000 + n) for n in wl.ragged_n}
        for b in synth.make_ragged_bins(codes, wl.batch, wl.ragged_K, wl.ragged_n, wl.ebn0_range, wl.bin_seed):
            items.append((b.K, b.n, codes[b.n], b.y, float(b.sigma2)))
    else:
        code = synth.regular_ldpc(wl.n, seed=wl.code_seed)
        bins = synth.make_bins(code, wl.K, wl.batch, wl.ebn0_db, wl.bin_seed)
        for b in range(wl.batch):
            items.append((wl.K, wl.n, code, bins.y[b], float(bins.sigma2[b])))
    return wl, wh, w, items


@pytest.mark.parametrize("name", ["c2", "c3", "c4"])
def test_full_batch_equals_sampled_bins_alone(name):
    torch = torch_cuda()
    P = lib()
    wl, wh, _, items = _workload_batch(name)
    handles = {}
    for K, n, code, *_ in items:
        if n not in handles:
            handles[n] = P.Code(code.n, code.m, code.row_ptr, code.col_idx)
    ro = dict(remask=int(wl.remask), remask_thr=wl.remask_thr, remask_max_rounds=wl.remask_max_rounds)
    opts = P.cider_opts_default(precision=P.CIDER_BF16, use_graph=1, **ro)
    ys = [torch.from_numpy(np.ascontiguousarray(y)).cuda() for *_, y, _ in items]
    outs = [torch.full((K, n), 9, dtype=torch.uint8, device="cuda") for K, n, *_ in items]
    valid = [torch.zeros(K, dtype=torch.uint8, device="cuda") for K, *_ in items]
    say(f"full batch {name}: {len(items)} bins, BF16, graph replay")
    P.cider_decode_batch([{"y": ys[i], "sigma2": items[i][4], "code": handles[items[i][1]], "K": items[i][0],
                           "n": items[i][1], "out_symbols": outs[i], "out_row_valid": valid[i]}
                          for i in range(len(items))], wh, wl.T, opts)
    torch.cuda.synchronize()
    X = [o.cpu().numpy() for o in outs]
    V = [v.cpu().numpy() for v in valid]
    for i, (K, n, code, *_) in enumerate(items):
        assert X[i].max() <= 1, f"bin {i}: non-binary symbol"
        assert np.array_equal(V[i], _syndrome_ok(code, X[i])), f"bin {i}: row-valid flags"
    sample = sorted({0, len(items) // 2, len(items) - 1})
    for i in sample:
        K, n, code, _, s2 = items[i]
        say(f"  {name} bin {i} (K={K}, n={n}) decoded alone")
        alone = torch.full((K, n), 9, dtype=torch.uint8, device="cuda")
        va = torch.zeros(K, dtype=torch.uint8, device="cuda")
        P.cider_decode_batch([{"y": ys[i], "sigma2": s2, "code": handles[n], "K": K, "n": n, "out_symbols": alone,
                               "out_row_valid": va}], wh, wl.T, opts)
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), X[i]), f"bin {i}: batch and alone differ"
        assert np.array_equal(va.cpu().numpy(), V[i])


@pytest.mark.parametrize("name,prec", [("c2", "bf16"), ("c3", "bf16"), ("c3", "fp8")])
def test_teacher_forced_step_at_workload_size(name, prec):
    """One teacher-forced step of a sampled bin at the workload's model, K and
    n; with FP8 at c3 this runs the token-resident kernels with the e4m3 MLP
    up projection over 2,048 tokens."""
    torch = torch_cuda()
    P = lib()
    wl, wh, w, items = _workload_batch(name)
    cfg = wl.model
    K, n, code, y, s2 = items[len(items) // 2]
    ch = P.Code(code.n, code.m, code.row_ptr, code.col_idx)
    _, p = evidence(y.astype(np.float64), s2, K)
    rng = np.random.default_rng(7)
    opts = P.cider_opts_default(precision={"bf16": P.CIDER_BF16, "fp8": P.CIDER_FP8}[prec])
    tol = TOL[prec]
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    for frac in (1.0, 0.5):
        Xin = rng.integers(0, 2, size=(K, n)).astype(np.uint8)
        Xin[rng.random((K, n)) < frac] = 2
        gamma = float((Xin == 2).mean())
        say(f"teacher-forced {prec} at {name} size: K={K} n={n} L={cfg.n_layers} d={cfg.d} mask={frac}")
        ref = denoise(Xin, p, code, w, cfg.n_layers, cfg.heads, gamma)
        lbar = torch.zeros(K, n, 2, dtype=torch.float32, device="cuda")
        logits = torch.zeros_like(lbar)
        Xo = torch.zeros(K, n, dtype=torch.uint8, device="cuda")
        r = max(1, int((Xin == 2).sum()) // 3)
        P.cider_step_debug(torch.from_numpy(Xin).cuda(), Xo, yd, s2, ch, K, n, wh, gamma, r, 0, opts,
                           out_lbar=lbar, out_logits=logits)
        torch.cuda.synchronize()
        e_lbar = rel_err(lbar.cpu().numpy(), ref["lbar"])
        e_log = rel_err(logits.cpu().numpy(), ref["logits"])
        print(f"  err lbar={e_lbar:.2e} logits={e_log:.2e}")
        assert e_lbar <= tol and e_log <= tol, (e_lbar, e_log)
        valid_selection(Xin, Xo.cpu().numpy(), ref["logits"], r, 0, slack=2 * tol * max(1.0, float(np.abs(ref["logits"]).max())))


# (K, n, workload whose model runs): rows longer than every sublayer-complete
# row kernel (n = 512 at d = 256 takes the QKV projection + LDS-resident row
# attention), and the d = 384, 12-head model of the served workload up to its
# largest bin (16 x 1024 = 16,384 tokens)
LARGE = [(8, 512, "c4"), (4, 512, "c5"), (16, 1024, "c5")]


@pytest.mark.parametrize("K,n,name", LARGE)
def test_teacher_forced_step_at_large_shapes(K, n, name):
    torch = torch_cuda()
    P = lib()
    wl = synth.workload(name)
    cfg = wl.model
    wh, w = weights_handle(cfg, wl.weight_seed)
    code = code_of(n, 1000 + n)
    ch = code_handle(code)
    b = synth.make_bins(code, K, 1, 4.0, seed=K * 1000 + n)
    y, s2 = b.y[0], float(b.sigma2[0])
    _, p = evidence(y.astype(np.float64), s2, K)
    rng = np.random.default_rng(K + n)
    opts = P.cider_opts_default(precision=P.CIDER_BF16)
    tol = TOL["bf16"]
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    for frac, first in ((1.0, 1), (0.5, 0)):
        Xin = rng.integers(0, 2, size=(K, n)).astype(np.uint8)
        Xin[rng.random((K, n)) < frac] = 2
        gamma = float((Xin == 2).mean())
        say(f"teacher-forced BF16 K={K} n={n} L={cfg.n_layers} d={cfg.d} h={cfg.heads} mask={frac} first={first}")
        ref = denoise(Xin, p, code, w, cfg.n_layers, cfg.heads, gamma)
        lbar = torch.zeros(K, n, 2, dtype=torch.float32, device="cuda")
        logits = torch.zeros_like(lbar)
        Xo = torch.zeros(K, n, dtype=torch.uint8, device="cuda")
        ncand = n if first else int((Xin == 2).sum())
        r = max(1, ncand // 3)
        P.cider_step_debug(torch.from_numpy(Xin).cuda(), Xo, yd, s2, ch, K, n, wh, gamma, r, first, opts,
                           out_lbar=lbar, out_logits=logits)
        torch.cuda.synchronize()
        e_lbar = rel_err(lbar.cpu().numpy(), ref["lbar"])
        e_log = rel_err(logits.cpu().numpy(), ref["logits"])
        print(f"  err lbar={e_lbar:.2e} logits={e_log:.2e}")
        assert e_lbar <= tol and e_log <= tol, (e_lbar, e_log)
        valid_selection(Xin, Xo.cpu().numpy(), ref["logits"], r, first,
                        slack=2 * tol * max(1.0, float(np.abs(ref["logits"]).max())))


# bins on both sides of every row-path boundary: n <= 128 (token-resident row
# sublayer at d = 128) beside longer rows, n <= 256 (fused QKV + row attention
# at d = 256) beside n = 512
MIXES = [("c2", [(4, 64), (2, 256), (3, 128), (1, 96)]), ("c4", [(4, 256), (2, 512), (8, 64), (3, 128)])]


@pytest.mark.parametrize("name,shapes", MIXES)
def test_batch_mix_across_row_paths_equals_alone_bitwise(name, shapes):
    """Logits, symbols and row-valid flags of every bin are bit-identical in
    the mixed batch and alone: a bin's kernels depend on its own shape only."""
    torch = torch_cuda()
    P = lib()
    wl = synth.workload(name)
    wh, _ = weights_handle(wl.model, wl.weight_seed)
    items = []
    for i, (K, n) in enumerate(shapes):
        code = code_of(n, 1000 + n)
        b = synth.make_bins(code, K, 1, 3.0 + i, seed=300 + i)
        items.append((K, n, code_handle(code), torch.from_numpy(np.ascontiguousarray(b.y[0])).cuda(),
                      float(b.sigma2[0])))
    opts = P.cider_opts_default(precision=P.CIDER_BF16, use_graph=1)
    T = 8

    def run(sel):
        outs = {i: (torch.full((items[i][0], items[i][1]), 9, dtype=torch.uint8, device="cuda"),
                    torch.zeros(items[i][0], items[i][1], 2, dtype=torch.float32, device="cuda"),
                    torch.zeros(items[i][0], dtype=torch.uint8, device="cuda")) for i in sel}
        P.cider_decode_batch([{"y": items[i][3], "sigma2": items[i][4], "code": items[i][2], "K": items[i][0],
                               "n": items[i][1], "out_symbols": outs[i][0], "out_logits": outs[i][1],
                               "out_row_valid": outs[i][2]} for i in sel], wh, T, opts)
        torch.cuda.synchronize()
        return outs

    say(f"batch mix {name}: shapes {shapes}, BF16, graph replay")
    mixed = run(list(range(len(items))))
    for i, (K, n, *_) in enumerate(items):
        say(f"  {name} bin {i} (K={K}, n={n}) alone")
        alone = run([i])[i]
        for a, m, what in zip(alone, mixed[i], ("symbols", "logits", "row-valid")):
            assert torch.equal(a, m), f"bin {i} (K={K}, n={n}): {what} differ between the mix and alone"


def test_quality_head_control_flow_at_c3_size():
    """The quality head as the remask criterion over c3's whole batch (512
    bins, 1.05 M tokens, the benchmark's launch configuration): a head that
    is always sure equals the decode without remasking, and one that always
    doubts equals the fixed criterion with a threshold above 1, bit for bit."""
    torch = torch_cuda()
    P = lib()
    wl, wh, _, items = _workload_batch("c3")
    code = items[0][2]
    ch = P.Code(code.n, code.m, code.row_ptr, code.col_idx)
    ys = [torch.from_numpy(np.ascontiguousarray(y)).cuda() for *_, y, _ in items]
    H = 16

    def run(opts):
        outs = [torch.full((K, n), 9, dtype=torch.uint8, device="cuda") for K, n, *_ in items]
        valid = [torch.zeros(K, dtype=torch.uint8, device="cuda") for K, *_ in items]
        P.cider_decode_batch([{"y": ys[i], "sigma2": items[i][4], "code": ch, "K": items[i][0], "n": items[i][1],
                               "out_symbols": outs[i], "out_row_valid": valid[i]} for i in range(len(items))],
                             wh, wl.T, opts)
        torch.cuda.synchronize()
        return np.stack([o.cpu().numpy() for o in outs]), np.stack([v.cpu().numpy() for v in valid])

    base = dict(precision=P.CIDER_BF16, use_graph=1)
    for b2, ref_opts in ((30.0, dict(remask=0)), (-30.0, dict(remask=1, remask_thr=2.0, remask_max_rounds=1))):
        psi = torch.from_numpy(synth.make_quality_head(wl.model.d, H, seed=7, b2=b2)).cuda()
        say(f"c3 full batch with the quality head, b2={b2}")
        got = run(P.cider_opts_default(remask=1, qhead=psi, qhead_hidden=H, remask_stages=1, **base))
        ref = run(P.cider_opts_default(**ref_opts, **base))
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), b2
