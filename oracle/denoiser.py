"""The CIDER denoiser forward in float64 (method section; Appendix, CIDER
architecture and its one-step algorithm).

One call maps the masked grid X (K rows x n slots, symbols {0, 1} and
MASK = 2), the per-slot beliefs p and the mask ratio gamma to logits:

  1. embedding      Z[k,l]   = E[X[k,l]] + P[l] + gamma * u
  2. Module A       intermediate logits Lbar = <Z, w_a>, responsibilities
                    r = softmax over rows k of Lbar / tau, evidence summary
                    e = sum_a r[...,a] p[l,a] v_a, gated blend
                    Z~ = g * Z + (1 - g) * e, g = sigmoid(MLP([Z ; e]))
  3. L layers       pre-LayerNorm residual blocks: multi-head attention of
                    each row over its n slots, multi-head attention of each
                    slot over its K rows, GELU MLP
  4. projection     Lout = <LN_f(Z), w_a>  (the same w_a as in step 2)
  5. Module B       parity messages added as a logit bias (see parity.py)

Rows carry no row embedding, so the map is equivariant under a permutation
of the rows, as the unordered output set requires.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np
from scipy.special import erf

from .parity import module_b

MASK = 2


def layer_norm(x: np.ndarray, g: np.ndarray, b: np.ndarray, eps: float = 1e-5) -> np.ndarray:
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    return (x - mu) / np.sqrt(var + eps) * g + b


def gelu(x: np.ndarray) -> np.ndarray:
    """GELU, exact erf form."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def softmax(x: np.ndarray, axis: int) -> np.ndarray:
    z = x - x.max(axis=axis, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=axis, keepdims=True)


def embed(X: np.ndarray, gamma: float, w: Dict[str, np.ndarray]) -> np.ndarray:
    """Z[k, l] = E[X[k, l]] + P[l] + gamma * u; returns [K][n][d]."""
    K, n = X.shape
    return w["E"][X] + w["P"][:n][None, :, :] + gamma * w["u"][None, None, :]


def module_a(Z: np.ndarray, p: np.ndarray, w: Dict[str, np.ndarray], tau: float = 1.0):
    """Module A (demixing by row competition).  Z [K][n][d], p [n][2].

    Returns (Z~, parts) where parts holds the intermediate logits, the
    responsibilities, the evidence summary e and the gate g.
    """
    lbar = Z @ w["W"].T                               # [K][n][2]
    r = softmax(lbar / tau, axis=0)                   # softmax over the rows k
    e = np.einsum("kla,la,ad->kld", r, p, w["v"])     # sum_a r p_a v_a
    h = gelu(np.concatenate([Z, e], axis=-1) @ w["Wg1"].T + w["bg1"])
    g = sigmoid(h @ w["Wg2"].T + w["bg2"])
    zt = g * Z + (1.0 - g) * e
    return zt, {"lbar": lbar, "r": r, "e": e, "g": g}


def mha(x: np.ndarray, Wqkv: np.ndarray, bqkv: np.ndarray, Wo: np.ndarray, bo: np.ndarray,
        heads: int) -> np.ndarray:
    """Multi-head self-attention over axis -2 of x [B][S][d], no mask.

    q, k, v are the three consecutive d-blocks of x Wqkv^T + bqkv; head h
    uses columns h*dh .. (h+1)*dh - 1 of each; scores are scaled by 1/sqrt(dh).
    """
    B, S, d = x.shape
    dh = d // heads
    qkv = x @ Wqkv.T + bqkv
    q = qkv[..., 0:d].reshape(B, S, heads, dh).transpose(0, 2, 1, 3)
    k = qkv[..., d:2 * d].reshape(B, S, heads, dh).transpose(0, 2, 1, 3)
    v = qkv[..., 2 * d:3 * d].reshape(B, S, heads, dh).transpose(0, 2, 1, 3)
    att = softmax(q @ k.transpose(0, 1, 3, 2) / math.sqrt(dh), axis=-1)
    o = (att @ v).transpose(0, 2, 1, 3).reshape(B, S, d)
    return o @ Wo.T + bo


def layer(Z: np.ndarray, w: Dict[str, np.ndarray], l: int, heads: int) -> np.ndarray:
    """One pre-LN block on Z [K][n][d]: row attention, user attention, MLP."""
    p = f"l{l}."
    Z = Z + mha(layer_norm(Z, w[p + "ln1_g"], w[p + "ln1_b"]),
                w[p + "Wqkv_r"], w[p + "bqkv_r"], w[p + "Wo_r"], w[p + "bo_r"], heads)
    Zt = Z.transpose(1, 0, 2)                          # [n][K][d]: each slot over its rows
    Zt = Zt + mha(layer_norm(Zt, w[p + "ln2_g"], w[p + "ln2_b"]),
                  w[p + "Wqkv_u"], w[p + "bqkv_u"], w[p + "Wo_u"], w[p + "bo_u"], heads)
    Z = Zt.transpose(1, 0, 2)
    h = gelu(layer_norm(Z, w[p + "ln3_g"], w[p + "ln3_b"]) @ w[p + "W1"].T + w[p + "b1"])
    return Z + h @ w[p + "W2"].T + w[p + "b2"]


def project(Z: np.ndarray, w: Dict[str, np.ndarray]) -> np.ndarray:
    """Final logits before Module B: <LN_f(Z), w_a>; returns [K][n][2]."""
    return layer_norm(Z, w["lnf_g"], w["lnf_b"]) @ w["W"].T


def denoise(X: np.ndarray, p: np.ndarray, code, w: Dict[str, np.ndarray], n_layers: int,
            heads: int, gamma: float, tau: float = 1.0, eta: float = 1.0,
            lam_max: float = 20.0, lam_min: float = 1e-6, parity: bool = True) -> Dict[str, np.ndarray]:
    """Full denoiser step; returns {'lbar': pre-Module-B logits, 'logits': final logits, ...}."""
    X = np.asarray(X)
    Z = embed(X, gamma, w)
    Z, parts = module_a(Z, p, w, tau)
    for l in range(n_layers):
        Z = layer(Z, w, l, heads)
    lbar = project(Z, w)
    logits = module_b(lbar, X, code, eta=eta, lam_max=lam_max, lam_min=lam_min) if parity else lbar.copy()
    return {"lbar": lbar, "logits": logits, "z": Z, "module_a": parts}
