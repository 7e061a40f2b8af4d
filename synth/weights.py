"""Seeded random denoiser weights in one flat float32 blob.

Blob layout (float offsets in this order; every matrix is row-major
[out][in], a linear map is y = x W^T + b):

    E      [3][d]        symbol embedding, row 2 = mask token
    P      [n_max][d]    slot positional embedding
    u      [d]           mask-ratio embedding (added as gamma * u)
    W      [2][d]        symbol projection w_a (intermediate and final logits)
    v      [2][d]        evidence symbol embedding v_a (Module A)
    Wg1    [d][2d], bg1 [d]   gate MLP layer 1, input [Z ; e]
    Wg2    [d][d],  bg2 [d]   gate MLP layer 2
    per layer l = 0..L-1:
      ln1_g [d], ln1_b [d], Wqkv_r [3d][d], bqkv_r [3d], Wo_r [d][d], bo_r [d]
      ln2_g [d], ln2_b [d], Wqkv_u [3d][d], bqkv_u [3d], Wo_u [d][d], bo_u [d]
      ln3_g [d], ln3_b [d], W1 [F][d], b1 [F], W2 [d][F], b2 [d]      (F = mlp_mult*d)
    lnf_g [d], lnf_b [d]

The HIP library computes the same offsets on its own from the model sizes;
this module only draws the numbers.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np


@dataclass(frozen=True)
class ModelCfg:
    n_layers: int
    d: int
    heads: int
    mlp_mult: int = 4
    q: int = 2
    n_max: int = 1024

    @property
    def d_ff(self) -> int:
        return self.mlp_mult * self.d

    @property
    def d_head(self) -> int:
        return self.d // self.heads


# kind: "mat" (N(0, 0.02^2)), "bias" (N(0, bias_std^2)), "ln_g" (1 + N(0, ln_std^2)), "ln_b" (N(0, ln_std^2))
def weight_layout(cfg: ModelCfg) -> List[Tuple[str, Tuple[int, ...], str]]:
    d, F = cfg.d, cfg.d_ff
    ent: List[Tuple[str, Tuple[int, ...], str]] = [
        ("E", (cfg.q + 1, d), "mat"),
        ("P", (cfg.n_max, d), "mat"),
        ("u", (d,), "mat"),
        ("W", (cfg.q, d), "mat"),
        ("v", (cfg.q, d), "mat"),
        ("Wg1", (d, 2 * d), "mat"), ("bg1", (d,), "bias"),
        ("Wg2", (d, d), "mat"), ("bg2", (d,), "bias"),
    ]
    for l in range(cfg.n_layers):
        p = f"l{l}."
        ent += [
            (p + "ln1_g", (d,), "ln_g"), (p + "ln1_b", (d,), "ln_b"),
            (p + "Wqkv_r", (3 * d, d), "mat"), (p + "bqkv_r", (3 * d,), "bias"),
            (p + "Wo_r", (d, d), "mat"), (p + "bo_r", (d,), "bias"),
            (p + "ln2_g", (d,), "ln_g"), (p + "ln2_b", (d,), "ln_b"),
            (p + "Wqkv_u", (3 * d, d), "mat"), (p + "bqkv_u", (3 * d,), "bias"),
            (p + "Wo_u", (d, d), "mat"), (p + "bo_u", (d,), "bias"),
            (p + "ln3_g", (d,), "ln_g"), (p + "ln3_b", (d,), "ln_b"),
            (p + "W1", (F, d), "mat"), (p + "b1", (F,), "bias"),
            (p + "W2", (d, F), "mat"), (p + "b2", (d,), "bias"),
        ]
    ent += [("lnf_g", (d,), "ln_g"), ("lnf_b", (d,), "ln_b")]
    return ent


def blob_size(cfg: ModelCfg) -> int:
    return int(sum(int(np.prod(s)) for _, s, _ in weight_layout(cfg)))


def make_weights(cfg: ModelCfg, seed: int, std: float = 0.02, bias_std: float = 0.0,
                 ln_std: float = 0.0) -> np.ndarray:
    """Flat float32 blob; draws are FP64 normals rounded once to float32."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    parts = []
    for _, shape, kind in weight_layout(cfg):
        cnt = int(np.prod(shape))
        if kind == "mat":
            a = rng.standard_normal(cnt) * std
        elif kind == "bias":
            a = rng.standard_normal(cnt) * bias_std if bias_std > 0 else np.zeros(cnt)
        elif kind == "ln_g":
            a = 1.0 + (rng.standard_normal(cnt) * ln_std if ln_std > 0 else np.zeros(cnt))
        else:
            a = rng.standard_normal(cnt) * ln_std if ln_std > 0 else np.zeros(cnt)
        parts.append(a)
    return np.concatenate(parts).astype(np.float32)


def unpack_weights(blob: np.ndarray, cfg: ModelCfg, dtype=np.float64) -> Dict[str, np.ndarray]:
    """Named views of a blob (copied to ``dtype``)."""
    out: Dict[str, np.ndarray] = {}
    off = 0
    flat = np.asarray(blob)
    if flat.size != blob_size(cfg):
        raise ValueError(f"blob has {flat.size} floats, layout needs {blob_size(cfg)}")
    for name, shape, _ in weight_layout(cfg):
        cnt = int(np.prod(shape))
        out[name] = flat[off:off + cnt].astype(dtype).reshape(shape)
        off += cnt
    return out


def make_quality_head(d: int, H: int, seed: int, std: float = 0.05, b2: float = 2.0) -> np.ndarray:
    """Seeded parameters of a per-token quality head (untrained): flat FP32
    [W1 (H x d), b1 (H), LayerNorm gain (H), LayerNorm bias (H), w2 (H), b2]."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    W1 = rng.standard_normal((H, d)) * std
    b1 = rng.standard_normal(H) * std
    g = 1.0 + rng.standard_normal(H) * std
    b = rng.standard_normal(H) * std
    w2 = rng.standard_normal(H) * 0.5
    return np.concatenate([W1.ravel(), b1, g, b, w2, [b2]]).astype(np.float32)
