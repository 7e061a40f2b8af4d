"""Shared helpers of the GPU tests: device setup, handles from synth inputs,
and the comparison rules between the HIP library and the FP64 oracle."""
from __future__ import annotations

import sys
from functools import lru_cache

import numpy as np

import synth

TOL = {"fp32": 1e-5, "bf16": 2e-2, "fp8": 1.5e-1}


def say(msg: str) -> None:
    """Name the case before a GPU step, so a failing run shows what it ran."""
    print(msg, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch


def lib():
    import paper_2605_26580_amd as P
    P.abi.lib()
    return P


def prec_id(name: str) -> int:
    import paper_2605_26580_amd as P
    return {"fp32": P.CIDER_FP32, "bf16": P.CIDER_BF16, "fp8": P.CIDER_FP8}[name]


@lru_cache(maxsize=None)
def code_of(n: int, seed: int):
    return synth.regular_ldpc(n, seed=seed)


_handles = {}


def code_handle(code):
    P = lib()
    key = ("code", code.n, code.seed)
    if key not in _handles:
        _handles[key] = P.Code(code.n, code.m, code.row_ptr, code.col_idx)
    return _handles[key]


def weights_handle(cfg: synth.ModelCfg, seed: int, bias_std=0.0, ln_std=0.0):
    P = lib()
    key = ("w", cfg, seed, bias_std, ln_std)
    if key not in _handles:
        blob = synth.make_weights(cfg, seed, bias_std=bias_std, ln_std=ln_std)
        _handles[key] = (P.Weights(P.make_cfg(cfg.n_layers, cfg.d, cfg.heads, cfg.mlp_mult, cfg.n_max, cfg.q), blob),
                         synth.unpack_weights(blob, cfg))
    return _handles[key]


def rel_err(gpu: np.ndarray, ref: np.ndarray) -> float:
    """max |gpu - ref| / max(1, |ref|)."""
    return float(np.max(np.abs(gpu.astype(np.float64) - ref) / np.maximum(1.0, np.abs(ref))))


def valid_selection(X_in, X_gpu, logits_ref, r, first, slack):
    """Check that the GPU's reveal is a valid outcome for logits within `slack`
    of the oracle's: exactly min(r, #candidates) masked candidates revealed,
    each taking the reference argmax unless the margin is within slack, and no
    unselected candidate beating a selected one by more than 2*slack."""
    MASK = 2
    K, n = X_in.shape
    c = np.abs(logits_ref[..., 0] - logits_ref[..., 1])
    masked = X_in == MASK
    changed = X_gpu != X_in
    assert np.all(masked[changed]), "a revealed site changed"
    if first:
        cand = np.zeros_like(masked)
        for l in range(n):
            ks = np.nonzero(masked[:, l])[0]
            if ks.size:
                best = c[ks, l].max()
                for k in ks:
                    if c[k, l] >= best - 2 * slack:
                        cand[k, l] = True
        assert changed.sum(axis=0).max(initial=0) <= 1, "first-reveal revealed two rows of a slot"
    else:
        cand = masked
    ncand = int(masked.any(axis=0).sum()) if first else int(masked.sum())
    assert changed.sum() == min(r, ncand), (changed.sum(), r, ncand)
    assert np.all(cand[changed]), "revealed a non-candidate"
    if changed.any():
        sel_min = c[changed].min()
        if first:
            # slot-level competition: an unrevealed slot's best row must not beat the cut
            best = np.where(masked, c, -np.inf).max(axis=0)
            open_slots = masked.any(axis=0) & ~changed.any(axis=0)
            if open_slots.any():
                assert best[open_slots].max() <= sel_min + 2 * slack
        else:
            rest = cand & ~changed
            if rest.any():
                assert c[rest].max() <= sel_min + 2 * slack
    for k, l in zip(*np.nonzero(changed)):
        want = 0 if logits_ref[k, l, 0] >= logits_ref[k, l, 1] else 1
        if c[k, l] > slack:
            assert X_gpu[k, l] == want
