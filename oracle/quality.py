"""PRISM-style quality head (Appendix, PRISM-style quality head and
remasking plug-in).  Test infrastructure only: the HIP library never imports
or calls it.

A per-token head reads the refined latent Zhat = LN_f(Z) of the final pass:
omega = sigmoid(g_psi(Zhat)), g_psi a two-layer MLP R^d -> R^H -> R.  The
text lists LayerNorm and GELU between the layers (dropout is off at
inference); the reading here is g(z) = w2 . GELU(LN_H(W1 z + b1)) + b2, the
LayerNorm over the H hidden units with its own gain and bias.  A row's
confidence is the mean of omega over its slots; after pass s the rows with
confidence below phi_s are remasked (multi-stage thresholds).

psi is a flat FP32 vector: W1 [H][d] (row-major), b1 [H], ln gain [H],
ln bias [H], w2 [H], b2 (one value).
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from .denoiser import gelu, layer_norm, sigmoid


def unpack_head(psi, d: int, H: int) -> Dict[str, np.ndarray]:
    psi = np.asarray(psi, dtype=np.float64)
    if psi.size != H * d + 4 * H + 1:
        raise ValueError("quality head size")
    o = 0
    out = {}
    for name, cnt, shape in (("W1", H * d, (H, d)), ("b1", H, (H,)), ("g", H, (H,)), ("b", H, (H,)),
                             ("w2", H, (H,)), ("b2", 1, ())):
        out[name] = psi[o:o + cnt].reshape(shape)
        o += cnt
    return out


def token_quality(Z: np.ndarray, w: Dict[str, np.ndarray], head: Dict[str, np.ndarray]) -> np.ndarray:
    """omega [K][n] from the final residual Z [K][n][d]."""
    zhat = layer_norm(Z, w["lnf_g"], w["lnf_b"])
    h = zhat @ head["W1"].T + head["b1"]
    g = gelu(layer_norm(h, head["g"], head["b"]))
    return sigmoid(g @ head["w2"] + head["b2"])


def row_confidence(Z: np.ndarray, w: Dict[str, np.ndarray], head: Dict[str, np.ndarray]) -> np.ndarray:
    """Mean over slots of the token qualities: [K]."""
    return token_quality(Z, w, head).mean(axis=1)
