"""Protocol-level wrapper over the batched decoder (Appendix, protocol-level
scaling by stochastic binning).

A frame's K_tot users have picked preambles, which split them into zeta
payload bins of loads K_chi.  Each bin with 1 <= K_chi <= K_max is one
decoding instance; a bin above K_max overflows and is erased (not decoded);
an empty bin is skipped.  Every decodable bin of every frame given goes to
the library in ONE cider_decode_batch call (one packed pass per refinement
step, bins of different K side by side), so a frame's decode costs what its
tokens cost, whatever its load mix.

serve_frames feeds the same bins to a continuous-batching server instead:
frames arrive one after another, each decodable bin is submitted as soon as
its frame arrives and joins the bins already on the GPU at its own first
refinement step, and a frame is complete when its last bin is.

Host bookkeeping only: the decode itself runs in the HIP library.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

from . import abi


def decode_frames(frames: Sequence[dict], code: "abi.Code", n: int, w: "abi.Weights", steps: int, K_max: int,
                  opts: Optional["abi.cider_opts"] = None, stream=None) -> List[dict]:
    """frames: dicts with ``loads`` (K_chi per bin, length zeta) and
    ``payload`` {chi: (y, sigma2)} for every bin with 1 <= K_chi <= K_max
    (y a device float32 tensor [n]).  Returns per frame
    {"decoded": {chi: (symbols uint8 [K_chi][n], row_valid uint8 [K_chi])},
     "erased": [chi with K_chi > K_max]}; the outputs are device tensors
    written on ``stream`` (the current torch stream when None)."""
    import torch
    if not 1 <= K_max <= 16:
        raise ValueError("K_max must be 1..16 (the library's largest K)")
    out: List[dict] = []
    batch: List[dict] = []
    dev = None
    for f in frames:
        res = {"decoded": {}, "erased": []}
        for chi, K in enumerate(f["loads"]):
            K = int(K)
            if K == 0:
                continue
            if K > K_max:
                res["erased"].append(chi)
                continue
            y, s2 = f["payload"][chi]
            dev = y.device
            sym = torch.empty(K, n, dtype=torch.uint8, device=dev)
            valid = torch.empty(K, dtype=torch.uint8, device=dev)
            res["decoded"][chi] = (sym, valid)
            batch.append({"y": y, "sigma2": float(s2), "code": code, "K": K, "n": n, "out_symbols": sym,
                          "out_row_valid": valid})
        out.append(res)
    if batch:
        abi.cider_decode_batch(batch, w, steps, opts, stream=stream)
    return out


def serve_frames(server: "abi.Server", frames: Sequence[dict], code: "abi.Code", n: int, K_max: int,
                 drain: bool = True) -> List[dict]:
    """frames: dicts with ``loads`` and ``payload`` {chi: (y, sigma2)} (y a host
    float32 array [n]) for every bin with 1 <= K_chi <= K_max, submitted in
    order.  Returns per frame {"decoded": {chi: host uint8 [K_chi][n]},
    "erased": [chi with K_chi > K_max], "ids": {chi: request id}}; the grids
    are complete once the server has finished their requests (after
    ``server.drain()``, which this call makes unless ``drain`` is False)."""
    if not 1 <= K_max <= 16:
        raise ValueError("K_max must be 1..16 (the library's largest K)")
    out: List[dict] = []
    for f in frames:
        res = {"decoded": {}, "erased": [], "ids": {}}
        for chi, K in enumerate(f["loads"]):
            K = int(K)
            if K == 0:
                continue
            if K > K_max:
                res["erased"].append(chi)
                continue
            y, s2 = f["payload"][chi]
            rid, grid = server.submit(y, float(s2), code, K, n)
            res["decoded"][chi] = grid
            res["ids"][chi] = rid
        out.append(res)
    if drain:
        server.drain()
    return out
